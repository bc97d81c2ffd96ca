// Approximate k nearest neighbours on gfx950: the K-NNG construction the
// paper adopts from LargeVis to build P faster (Section 4.3).
//
// 1. Random-projection trees, built level by level for all ranges at once.
//    The points are a permutation; a range [a, b) of more than leaf_size
//    points splits by the hyperplane halfway between two of its points x_a
//    and x_b: a point goes right iff sum_d (x_d - (x_ad + x_bd) / 2)
//    (x_ad - x_bd) > 0, in FP64 with the terms in order of d and every
//    operation rounded on its own.  The split keeps the order inside each
//    side (a global exclusive scan of the side flags gives each point its new
//    place).  If a side would get fewer than k + 1 points, or from level 48
//    on, the range is cut in the middle instead, so every leaf (at most
//    leaf_size >= 2k + 2 points) offers each of its points k candidates.  The
//    two points come from SplitMix64 (Steele, Lea and Flood, 2014) keyed by
//    the seed, the tree, the level and the range's first position.
// 2. Each point's list keeps the best k of its leaf mates over all trees by
//    (squared distance, index), distinct, in FP64 (terms in order of d).
// 3. Rounds of neighbour exploring: each point's new list is the best k of
//    its list and its neighbours' lists, all read from the previous round.
//
// Every decision is taken in FP64 with a fixed operation order, so the result
// is a deterministic function of the data and the seed (the CPU reference
// takes the same steps).
#include "ctx.h"

namespace psne {

namespace {

constexpr int kBlock = 256;
constexpr int kRpMaxLevel = 48;

inline dim3 grid_for(int64_t n) { return dim3((unsigned)ceil_div(n > 0 ? n : 1, kBlock)); }

__device__ __forceinline__ uint64_t rp_draw(uint64_t seed, int tree, int level, int64_t a,
                                            int which) {
    uint64_t x = splitmix64(seed ^ (uint64_t)(uint32_t)tree);
    x = splitmix64(x ^ (uint64_t)(uint32_t)level);
    return splitmix64(x ^ (((uint64_t)a << 1) | (uint64_t)which));
}

__device__ __forceinline__ double as_f64(float v) { return (double)v; }
__device__ __forceinline__ double as_f64(double v) { return v; }
__device__ __forceinline__ double as_f64(uint8_t v) { return (double)v; }

// squared distance of rows i and j, FP64, terms in order of d, no contraction
template <typename X>
__device__ __forceinline__ double sqdist(const X* __restrict__ Xm, int32_t D, int64_t i,
                                         int64_t j) {
#pragma clang fp contract(off)
    const X* a = Xm + i * (int64_t)D;
    const X* b = Xm + j * (int64_t)D;
    double s = 0.0;
    for (int t = 0; t < D; t++) {
        const double e = as_f64(a[t]) - as_f64(b[t]);
        s = s + e * e;
    }
    return s;
}

__device__ __forceinline__ bool knn_less(double da, int32_t ja, double db, int32_t jb) {
    return da < db || (da == db && ja < jb);
}


__global__ __launch_bounds__(kBlock) void k_rp_init(uint32_t* __restrict__ perm,
                                                    uint32_t* __restrict__ sa,
                                                    uint32_t* __restrict__ sb, int64_t n) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    perm[p] = (uint32_t)p;
    sa[p] = 0;
    sb[p] = (uint32_t)n;
}

// side of the hyperplane for every position of a range that splits at this
// level (0 elsewhere); side[n] = 0 closes the scan; *any = 1 if a range splits
template <typename X>
__global__ __launch_bounds__(kBlock) void k_rp_side(const X* __restrict__ Xm, int32_t D,
                                                    const uint32_t* __restrict__ perm,
                                                    const uint32_t* __restrict__ sa,
                                                    const uint32_t* __restrict__ sb, int64_t n,
                                                    int32_t leaf, uint64_t seed, int tree,
                                                    int level, int64_t* __restrict__ side,
                                                    uint32_t* __restrict__ any) {
#pragma clang fp contract(off)
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p > n) return;
    if (p == n) {
        side[n] = 0;
        return;
    }
    const int64_t a = sa[p], m = (int64_t)sb[p] - a;
    int64_t s = 0;
    if (m > leaf) {
        if (p == a) atomicOr(any, 1u);
        if (level < kRpMaxLevel) {
            const int64_t ia = (int64_t)(rp_draw(seed, tree, level, a, 0) % (uint64_t)m);
            int64_t ib = (int64_t)(rp_draw(seed, tree, level, a, 1) % (uint64_t)(m - 1));
            if (ib >= ia) ib++;
            const X* xa = Xm + (int64_t)perm[a + ia] * D;
            const X* xb = Xm + (int64_t)perm[a + ib] * D;
            const X* xi = Xm + (int64_t)perm[p] * D;
            double acc = 0.0;
            for (int d = 0; d < D; d++) {
                const double va = as_f64(xa[d]), vb = as_f64(xb[d]);
                const double mid = (va + vb) * 0.5;
                const double v = va - vb;
                acc = acc + (as_f64(xi[d]) - mid) * v;
            }
            s = acc > 0.0 ? 1 : 0;
        }
    }
    side[p] = s;
}

// new place of every position: the left side keeps its order at the front
// of the range, the right side after it; a range that cannot split well
// (a side under k + 1 points, or level >= 48) is cut in the middle in place
__global__ __launch_bounds__(kBlock) void k_rp_scatter(
    const uint32_t* __restrict__ perm, const uint32_t* __restrict__ sa,
    const uint32_t* __restrict__ sb, const int64_t* __restrict__ side,
    const int64_t* __restrict__ ones, int64_t n, int32_t leaf, int32_t k, int level,
    uint32_t* __restrict__ perm2, uint32_t* __restrict__ sa2, uint32_t* __restrict__ sb2) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    const int64_t a = sa[p], b = sb[p], m = b - a;
    if (m <= leaf) {
        perm2[p] = perm[p];
        sa2[p] = (uint32_t)a;
        sb2[p] = (uint32_t)b;
        return;
    }
    const int64_t right = ones[b] - ones[a];
    const int64_t nl = m - right;
    if (level >= kRpMaxLevel || nl < k + 1 || right < k + 1) {
        const int64_t h = a + m / 2;
        perm2[p] = perm[p];
        sa2[p] = (uint32_t)(p < h ? a : h);
        sb2[p] = (uint32_t)(p < h ? h : b);
        return;
    }
    const int64_t before = ones[p] - ones[a];         // right-side points before p in the range
    int64_t q;
    if (side[p]) {
        q = a + nl + before;
        sa2[q] = (uint32_t)(a + nl);
        sb2[q] = (uint32_t)b;
    } else {
        q = a + (p - a - before);
        sa2[q] = (uint32_t)a;
        sb2[q] = (uint32_t)(a + nl);
    }
    perm2[q] = perm[p];
}

// ---------------------------------------------------------------------------
// List updates, one wavefront per point.  The candidates of a point stream
// through in groups of 64; a hash set in LDS (seeded with the point and its
// current list) drops repeats, so each new candidate's distance is computed
// once: the 64 candidate rows are staged through LDS in slices of kSlice
// dimensions (coalesced loads), and each lane sums its candidate's terms in
// order of d, in FP64.  Candidates that beat the list's k-th entry are then
// inserted by one lane.  The resulting list, the best k of the old list and
// the candidates by (d^2, index), does not depend on the order of insertion.
// ---------------------------------------------------------------------------
constexpr int kWaveBlock = 64;
constexpr int kSlice = 32;
constexpr int kSetBits = 12;
constexpr int kSetSize = 1 << kSetBits;
constexpr int kProbes = 32;
constexpr int kMaxK = 256;

template <typename X> struct TileOf { using type = float; };     // exact for FP32 and uint8
template <> struct TileOf<double> { using type = double; };

template <typename TT>
struct ListLds {
    int32_t set[kSetSize];
    int32_t pend[2 * kWaveBlock];
    double ld[kMaxK];
    int32_t lj[kMaxK];
    double ld2[kMaxK];               // the merged list before it is copied back
    int32_t lj2[kMaxK];
    double gd[kWaveBlock];           // the group, sorted
    int32_t gj[kWaveBlock];
    TT xi[kSlice];
    TT rows[kWaveBlock][kSlice + 1];
    int32_t m, npend;
};

// bitonic sort of one (d, j) pair per lane across the wave, ascending
__device__ __forceinline__ void wave_sort(double& d, int32_t& j) {
    const int lane = lane_id();
#pragma unroll
    for (int size = 2; size <= kWave; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const double od = __shfl_xor(d, stride, kWave);
            const int32_t oj = __shfl_xor(j, stride, kWave);
            const bool up = (lane & size) == 0;          // this block sorts ascending
            const bool low = (lane & stride) == 0;       // this lane holds the lower slot
            const bool other_less = knn_less(od, oj, d, j);
            // the lower slot of an ascending block keeps the smaller pair
            const bool take = (low == up) ? other_less : knn_less(d, j, od, oj);
            if (take) {
                d = od;
                j = oj;
            }
        }
    }
}

// number of entries of a sorted list (ascending (d, j)) below (d, j)
__device__ __forceinline__ int rank_in(const double* ld, const int32_t* lj, int m, double d,
                                       int32_t j) {
    int lo = 0, hi = m;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (knn_less(ld[mid], lj[mid], d, j)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// true if v was not in the set (and is now); a set too full to place v
// reports it as new, which at worst computes a repeat (rejected on insertion)
__device__ __forceinline__ bool set_add(int32_t* set, int32_t v) {
    uint32_t h = ((uint32_t)v * 0x9E3779B1u) >> (32 - kSetBits);
    for (int q = 0; q < kProbes; q++) {
        const int32_t old = atomicCAS(&set[h], -1, v);
        if (old == -1) return true;
        if (old == v) return false;
        h = (h + 1) & (kSetSize - 1);
    }
    return true;
}

// distances of the 64 pending candidates (cand < 0: none) to point i, then
// the insertions that beat the list
template <typename X, typename TT>
__device__ void process_group(const X* __restrict__ Xm, int32_t D, int64_t i, int32_t k,
                              ListLds<TT>& s) {
#pragma clang fp contract(off)
    const int lane = lane_id();
    const int32_t cand = s.pend[lane];
    double acc = 0.0;
    // lane t stages column t % kSlice of rows t / kSlice + kPass q: every load
    // of a slice is issued before the first LDS store
    constexpr int kPass = kWaveBlock / kSlice;
    const int col = lane % kSlice, r0 = lane / kSlice;
    for (int d0 = 0; d0 < D; d0 += kSlice) {
        const int w = D - d0 < kSlice ? D - d0 : kSlice;
        TT v[kWaveBlock / kPass];
        const TT vx = lane < w ? (TT)Xm[i * D + d0 + lane] : TT(0);
#pragma unroll
        for (int q = 0; q < kWaveBlock / kPass; q++) {
            const int32_t c = s.pend[r0 + kPass * q];
            v[q] = (c >= 0 && col < w) ? (TT)Xm[(int64_t)c * D + d0 + col] : TT(0);
        }
        __syncthreads();
        if (lane < kSlice) s.xi[lane] = vx;
#pragma unroll
        for (int q = 0; q < kWaveBlock / kPass; q++) s.rows[r0 + kPass * q][col] = v[q];
        __syncthreads();
        if (cand >= 0)
            for (int d = 0; d < w; d++) {
                const double e = (double)s.xi[d] - (double)s.rows[lane][d];
                acc = acc + e * e;
            }
    }
    // Merge the candidates that may enter into the list, all lanes at once:
    // sort the group, drop repeats (equal pairs: the same index has the same
    // distance), and place every entry of list and group by its rank in the
    // other; the first k form the new list.
    const int32_t m0 = s.m;
    const bool may = cand >= 0 && (m0 < k || knn_less(acc, cand, s.ld[k - 1], s.lj[k - 1]));
    if (!ballot64(may)) return;
    const double kInf = __builtin_inf();
    double d = may ? acc : kInf;
    int32_t j = may ? cand : 0x7FFFFFFF;
    wave_sort(d, j);
    const double pd = __shfl_up(d, 1, kWave);
    const int32_t pj = __shfl_up(j, 1, kWave);
    bool valid = j != 0x7FFFFFFF && !(lane > 0 && pd == d && pj == j);
    const int r_list = valid ? rank_in(s.ld, s.lj, m0, d, j) : 0;
    if (valid && r_list < m0 && s.ld[r_list] == d && s.lj[r_list] == j) valid = false;
    // group entries compacted in order (ranks among the valid ones)
    const uint64_t vb = ballot64(valid);
    const int g_rank = __popcll(vb & lanemask_lt());
    const int ng = __popcll(vb);
    __syncthreads();
    if (valid) {
        s.gd[g_rank] = d;
        s.gj[g_rank] = j;
    }
    __syncthreads();
    const int mn = m0 + ng < k ? m0 + ng : k;
    if (valid && g_rank + r_list < k) {
        s.ld2[g_rank + r_list] = d;
        s.lj2[g_rank + r_list] = j;
    }
    for (int a = lane; a < m0; a += kWaveBlock) {
        const int pos = a + rank_in(s.gd, s.gj, ng, s.ld[a], s.lj[a]);
        if (pos < k) {
            s.ld2[pos] = s.ld[a];
            s.lj2[pos] = s.lj[a];
        }
    }
    __syncthreads();
    for (int a = lane; a < mn; a += kWaveBlock) {
        s.ld[a] = s.ld2[a];
        s.lj[a] = s.lj2[a];
    }
    if (lane == 0) s.m = mn;
    __syncthreads();
}

// Offer candidate v (< 0: none) of this lane: new ones join the pending
// group, and a full group is processed.
template <typename X, typename TT>
__device__ __forceinline__ void offer(const X* __restrict__ Xm, int32_t D, int64_t i, int32_t k,
                                      ListLds<TT>& s, int32_t v) {
    const int lane = lane_id();
    const bool fresh = v >= 0 && set_add(s.set, v);
    const uint64_t b = ballot64(fresh);
    const int32_t base = s.npend;
    if (fresh) s.pend[base + __popcll(b & lanemask_lt())] = v;
    __syncthreads();
    if (lane == 0) s.npend = base + __popcll(b);
    __syncthreads();
    if (s.npend >= kWaveBlock) {
        process_group<X, TT>(Xm, D, i, k, s);
        const int32_t rest = s.npend - kWaveBlock;
        const int32_t carry = lane < rest ? s.pend[kWaveBlock + lane] : -1;
        __syncthreads();
        s.pend[lane] = carry;
        s.pend[kWaveBlock + lane] = -1;
        if (lane == 0) s.npend = rest;
        __syncthreads();
    }
}

// MODE 0: the leaf mates of the point at position blockIdx.x (one tree), the
// list updated in place.  MODE 1: one round of exploring for point
// blockIdx.x: the old lists (ld, lj, lm) of it and its neighbours in, the new
// list (nd, nj, nm) out.
template <typename X, int MODE>
__global__ __launch_bounds__(kWaveBlock) void k_lists_wave(
    const X* __restrict__ Xm, int32_t D, int64_t n, int32_t k, const uint32_t* __restrict__ perm,
    const uint32_t* __restrict__ sa, const uint32_t* __restrict__ sb,
    const double* __restrict__ ld, const int32_t* __restrict__ lj,
    const int32_t* __restrict__ lm, double* __restrict__ nd, int32_t* __restrict__ nj,
    int32_t* __restrict__ nm) {
    using TT = typename TileOf<X>::type;
    __shared__ ListLds<TT> s;
    const int lane = lane_id();
    const int64_t b = blockIdx.x;
    const int64_t i = MODE == 0 ? (int64_t)perm[b] : b;
    for (int q = lane; q < kSetSize; q += kWaveBlock) s.set[q] = -1;
    s.pend[lane] = -1;
    s.pend[kWaveBlock + lane] = -1;
    const int32_t m = lm[i];
    for (int q = lane; q < m; q += kWaveBlock) {
        s.ld[q] = ld[i * k + q];
        s.lj[q] = lj[i * k + q];
    }
    if (lane == 0) {
        s.m = m;
        s.npend = 0;
    }
    __syncthreads();
    // the point itself and its listed neighbours are not candidates
    if (lane == 0) set_add(s.set, (int32_t)i);
    __syncthreads();
    for (int q = lane; q < m; q += kWaveBlock) set_add(s.set, s.lj[q]);
    __syncthreads();
    if (MODE == 0) {
        const int64_t a = sa[b], e = sb[b];
        for (int64_t q0 = a; q0 < e; q0 += kWaveBlock) {
            const int64_t q = q0 + lane;
            offer<X, TT>(Xm, D, i, k, s, q < e ? (int32_t)perm[q] : -1);
        }
    } else {
        // the candidate stream: entry c of the list of neighbour a for
        // x = a k + c (lists are full: every leaf gives each point k
        // candidates), fetched one group ahead of its use
        const int64_t total = (int64_t)m * k;
        auto fetch = [&](int64_t x) -> int32_t {
            if (x >= total) return -1;
            const int64_t j = lj[i * k + x / k];
            const int32_t c = (int32_t)(x % k);
            return c < lm[j] ? lj[j * k + c] : -1;
        };
        int32_t next = fetch(lane);
        for (int64_t x0 = 0; x0 < total; x0 += kWaveBlock) {
            const int32_t v = next;
            next = fetch(x0 + kWaveBlock + lane);
            offer<X, TT>(Xm, D, i, k, s, v);
        }
    }
    if (s.npend > 0) process_group<X, TT>(Xm, D, i, k, s);
    __syncthreads();
    double* od = MODE == 0 ? const_cast<double*>(ld) : nd;
    int32_t* oj = MODE == 0 ? const_cast<int32_t*>(lj) : nj;
    int32_t* om = MODE == 0 ? const_cast<int32_t*>(lm) : nm;
    for (int q = lane; q < s.m; q += kWaveBlock) {
        od[i * k + q] = s.ld[q];
        oj[i * k + q] = s.lj[q];
    }
    if (lane == 0) om[i] = s.m;
}

__global__ __launch_bounds__(kBlock) void k_lists_out(const double* __restrict__ ld,
                                                      const int32_t* __restrict__ lj,
                                                      const int32_t* __restrict__ lm, int64_t n,
                                                      int32_t k, int32_t* __restrict__ idx,
                                                      double* __restrict__ d2,
                                                      uint32_t* __restrict__ short_rows) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= n * (int64_t)k) return;
    const int64_t i = e / k;
    if (e % k == 0 && lm[i] < k) atomicAdd(short_rows, 1u);
    idx[e] = lj[e];
    d2[e] = ld[e];
}

template <typename X>
hipError_t knn_approx_typed(const X* Xm, int64_t n, int32_t D, int32_t k, int32_t trees,
                            int32_t leaf, int32_t explore, uint64_t seed, int32_t* idx,
                            double* d2, hipStream_t s, std::string* err) {
    uint32_t *perm[2] = {nullptr, nullptr}, *sa[2] = {nullptr, nullptr},
             *sb[2] = {nullptr, nullptr}, *flag = nullptr;
    int64_t *side = nullptr, *ones = nullptr, *tmp = nullptr;
    double* ld[2] = {nullptr, nullptr};
    int32_t* lj[2] = {nullptr, nullptr};
    int32_t* lm[2] = {nullptr, nullptr};
    hipError_t e = hipSuccess;
    auto cleanup = [&]() {
        for (int h = 0; h < 2; h++) {
            (void)hipFree(perm[h]); (void)hipFree(sa[h]); (void)hipFree(sb[h]);
            (void)hipFree(ld[h]); (void)hipFree(lj[h]); (void)hipFree(lm[h]);
        }
        (void)hipFree(flag); (void)hipFree(side); (void)hipFree(ones); (void)hipFree(tmp);
    };
    const size_t nk = (size_t)n * k;
    for (int h = 0; h < 2 && e == hipSuccess; h++) {
        e = hipMalloc(&perm[h], 4 * (size_t)n);
        if (e == hipSuccess) e = hipMalloc(&sa[h], 4 * (size_t)n);
        if (e == hipSuccess) e = hipMalloc(&sb[h], 4 * (size_t)n);
        if (e == hipSuccess) e = hipMalloc(&ld[h], 8 * nk);
        if (e == hipSuccess) e = hipMalloc(&lj[h], 4 * nk);
        if (e == hipSuccess) e = hipMalloc(&lm[h], 4 * (size_t)n);
    }
    if (e == hipSuccess) e = hipMalloc(&flag, 8);
    if (e == hipSuccess) e = hipMalloc(&side, 8 * (size_t)(n + 1));
    if (e == hipSuccess) e = hipMalloc(&ones, 8 * (size_t)(n + 1));
    if (e == hipSuccess) e = hipMalloc(&tmp, 8 * (size_t)scan_i64_tmp_len(n + 1));
    if (e == hipSuccess) e = hipMemsetAsync(lm[0], 0, 4 * (size_t)n, s);
    for (int32_t tr = 0; tr < trees && e == hipSuccess; tr++) {
        int cur = 0;
        k_rp_init<<<grid_for(n), kBlock, 0, s>>>(perm[0], sa[0], sb[0], n);
        for (int level = 0; e == hipSuccess; level++) {
            e = hipMemsetAsync(flag, 0, 4, s);
            if (e != hipSuccess) break;
            k_rp_side<X><<<grid_for(n + 1), kBlock, 0, s>>>(Xm, D, perm[cur], sa[cur], sb[cur], n,
                                                            leaf, seed, tr, level, side, flag);
            uint32_t any = 0;
            e = hipMemcpyAsync(&any, flag, 4, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess || !any) break;
            e = scan_i64(side, n + 1, ones, tmp, s);
            if (e != hipSuccess) break;
            k_rp_scatter<<<grid_for(n), kBlock, 0, s>>>(perm[cur], sa[cur], sb[cur], side, ones, n,
                                                        leaf, k, level, perm[cur ^ 1], sa[cur ^ 1],
                                                        sb[cur ^ 1]);
            cur ^= 1;
            e = hipGetLastError();
        }
        if (e == hipSuccess) {
            k_lists_wave<X, 0><<<dim3((unsigned)n), kWaveBlock, 0, s>>>(
                Xm, D, n, k, perm[cur], sa[cur], sb[cur], ld[0], lj[0], lm[0], nullptr, nullptr,
                nullptr);
            e = hipGetLastError();
        }
    }
    int L = 0;
    for (int32_t r = 0; r < explore && e == hipSuccess; r++) {
        k_lists_wave<X, 1><<<dim3((unsigned)n), kWaveBlock, 0, s>>>(
            Xm, D, n, k, nullptr, nullptr, nullptr, ld[L], lj[L], lm[L], ld[L ^ 1], lj[L ^ 1],
            lm[L ^ 1]);
        L ^= 1;
        e = hipGetLastError();
    }
    uint32_t short_rows = 0;
    if (e == hipSuccess) e = hipMemsetAsync(flag, 0, 4, s);
    if (e == hipSuccess) {
        k_lists_out<<<grid_for((int64_t)nk), kBlock, 0, s>>>(ld[L], lj[L], lm[L], n, k, idx, d2,
                                                             flag);
        e = hipMemcpyAsync(&short_rows, flag, 4, hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    cleanup();
    if (e == hipSuccess && short_rows) {
        // every leaf holds at least k + 1 points, so this does not happen
        if (err) *err = "approximate kNN left rows with fewer than k neighbours";
        return hipErrorUnknown;
    }
    return e;
}

}  // namespace

hipError_t knn_approx(const void* X, int64_t n, int32_t D, int32_t x_dtype, int32_t k,
                      int32_t trees, int32_t leaf, int32_t explore, uint64_t seed, int32_t* idx,
                      double* d2, hipStream_t s, std::string* err) {
    switch (x_dtype) {
        case PSNE_X_F32:
            return knn_approx_typed<float>((const float*)X, n, D, k, trees, leaf, explore, seed,
                                           idx, d2, s, err);
        case PSNE_X_F64:
            return knn_approx_typed<double>((const double*)X, n, D, k, trees, leaf, explore, seed,
                                            idx, d2, s, err);
        default:
            return knn_approx_typed<uint8_t>((const uint8_t*)X, n, D, k, trees, leaf, explore,
                                             seed, idx, d2, s, err);
    }
}

}  // namespace psne
