// Per-iteration passes of PixelSNE on gfx950 (wave64).
//
//   snap        pending screen scaling (Section 4.2) + pixel (Eq. 1-2) + Morton key
//   sort        stable LSD radix sort of (key, index), 8-bit digits, LDS ranking
//   tree        P-Quadtree (Section 4.1) as a linear tree: one node per occupied
//               (level, Morton prefix); counts and FP64 coordinate sums (Eq. 8)
//               reduced bottom-up, up to five levels per launch
//   traverse    Barnes-Hut repulsion (Eq. 5, 11, 12): one wavefront walks the
//               union of the interaction lists of 64 Morton-consecutive points,
//               each stack entry carrying the mask of lanes still descending
//   zsum        Z = sum_i Z_i in FP64, fixed order
//   attract     row sums of the sparse attraction over CSR P (Eq. 5), on a
//               second stream beside the traversal and Z (and beside sort and
//               tree too, when the fork-point tuner finds that faster)
//   update      B = alpha A - R / Z, gains/momentum step, new positions and
//               per-block min/max of them
//   finalize    screen scaling factors, scale bookkeeping (Eq. 13), iteration++,
//               the fork-point tuner
#include <math.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "ctx.h"

namespace psne {

namespace {

constexpr int kBlock = 256;
constexpr int kRsItems = 8;
constexpr int kRsTile = kBlock * kRsItems;
constexpr int kAttractBlocksMax = 8192;


// ---------------------------------------------------------------------------
// snap: z = clamp((zh - zmin) * scale, 0, r^-), key = Morton(floor(z))
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_snap(const T* __restrict__ zh, T* __restrict__ z,
                                                 uint32_t* __restrict__ key,
                                                 uint32_t* __restrict__ idx,
                                                 const DevScalars* __restrict__ sc, int64_t n,
                                                 int r) {
    using V = v2_t<T>;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const T top = top_below<T>(r);
    const V p = reinterpret_cast<const V*>(zh)[i];
    T zx = (p.x - (T)sc->zmin[0]) * (T)sc->scale[0];
    T zy = (p.y - (T)sc->zmin[1]) * (T)sc->scale[1];
    zx = zx < T(0) ? T(0) : (zx > top ? top : zx);
    zy = zy < T(0) ? T(0) : (zy > top ? top : zy);
    reinterpret_cast<V*>(z)[i] = V{zx, zy};
    const uint32_t px = (uint32_t)zx, py = (uint32_t)zy;
    key[i] = spread_bits16(px) | (spread_bits16(py) << 1);
    idx[i] = (uint32_t)i;
}

// ---------------------------------------------------------------------------
// radix sort (stable, LSD, 8-bit digits)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_rs_hist(const uint32_t* __restrict__ keys, int64_t n,
                                                    int shift, uint32_t* __restrict__ hist,
                                                    int64_t nblocks) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
#pragma unroll
    for (int j = 0; j < kRsItems; j++) {
        const int64_t p = base + j * kBlock + threadIdx.x;
        if (p < n) atomicAdd(&h[(keys[p] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of each row of a [rows][len] uint32 array in place (one block
// per row; each thread takes 4 consecutive entries of a 1,024-entry piece, so
// long rows need few barrier rounds); the row totals go to tot[row].
constexpr int kScanItems = 4;

__global__ __launch_bounds__(kBlock) void k_rows_scan(uint32_t* __restrict__ a, int64_t len,
                                                      uint32_t* __restrict__ tot) {
    __shared__ uint32_t ws[4];
    const int t = threadIdx.x, w = t >> 6, lane = lane_id();
    uint32_t* row = a + (int64_t)blockIdx.x * len;
    uint32_t carry = 0;
    for (int64_t c0 = 0; c0 < len; c0 += (int64_t)kScanItems * kBlock) {
        const int64_t i0 = c0 + (int64_t)kScanItems * t;
        uint32_t v[kScanItems];
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; k++) {
            v[k] = i0 + k < len ? row[i0 + k] : 0u;
            sum += v[k];
        }
        uint32_t x = sum;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, kWave);
            if (lane >= o) x += y;
        }
        if (lane == kWave - 1) ws[w] = x;
        __syncthreads();
        uint32_t run = carry + x - sum;
        for (int q = 0; q < w; q++) run += ws[q];
#pragma unroll
        for (int k = 0; k < kScanItems; k++) {
            if (i0 + k < len) row[i0 + k] = run;
            run += v[k];
        }
        carry += ws[0] + ws[1] + ws[2] + ws[3];
        __syncthreads();
    }
    if (t == 0) tot[blockIdx.x] = carry;
}

__global__ __launch_bounds__(kBlock) void k_rs_scatter(const uint32_t* __restrict__ kin,
                                                       const uint32_t* __restrict__ vin,
                                                       uint32_t* __restrict__ kout,
                                                       uint32_t* __restrict__ vout, int64_t n,
                                                       int shift,
                                                       const uint32_t* __restrict__ hist,
                                                       const uint32_t* __restrict__ dtot,
                                                       int64_t nblocks) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[4][256];
    const int t = threadIdx.x, w = t >> 6, lane = lane_id();
    {
        // digit bases: exclusive scan of the 256 digit totals
        const uint32_t v = dtot[t];
        uint32_t x = v;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, kWave);
            if (lane >= o) x += y;
        }
        if (lane == kWave - 1) wcnt[0][w] = x;
        __syncthreads();
        uint32_t pre = x - v;
        for (int q = 0; q < w; q++) pre += wcnt[0][q];
        run[t] = pre + hist[(int64_t)t * nblocks + blockIdx.x];
        __syncthreads();
    }
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    // every item's key and value loaded up front, so that the loads overlap
    // instead of waiting behind each round's barriers
    uint32_t keys[kRsItems], vals[kRsItems];
#pragma unroll
    for (int j = 0; j < kRsItems; j++) {
        const int64_t p = base + j * kBlock + t;
        keys[j] = p < n ? kin[p] : 0u;
        vals[j] = p < n ? (vin ? vin[p] : (uint32_t)p) : 0u;
    }
#pragma unroll
    for (int j = 0; j < kRsItems; j++) {
        const int64_t p = base + j * kBlock + t;
        const bool valid = p < n;
        const uint32_t key = keys[j];
        const uint32_t val = vals[j];
        const uint32_t d = (key >> shift) & 255u;
        wcnt[0][t] = 0; wcnt[1][t] = 0; wcnt[2][t] = 0; wcnt[3][t] = 0;
        __syncthreads();
        uint64_t peers = ballot64(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = ballot64(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lanemask_lt());
        if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t off = run[d] + rank;
            for (int q = 0; q < w; q++) off += wcnt[q][d];
            kout[off] = key;
            vout[off] = val;
        }
        __syncthreads();
        run[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
    }
}

// ---------------------------------------------------------------------------
// tree: first level at which sorted position s starts a new cell
// (s = 0 starts a cell at every level; equal keys start none: L + 1)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int first_new_level(const uint32_t* __restrict__ keys, int64_t s,
                                               int L) {
    if (s == 0) return 0;
    const uint32_t x = keys[s] ^ keys[s - 1];
    if (x == 0) return L + 1;
    const int hb = 31 - __clz(x);
    return L - (hb >> 1);
}

__global__ __launch_bounds__(kBlock) void k_tree_count(const uint32_t* __restrict__ keys,
                                                       int64_t n, int L,
                                                       uint32_t* __restrict__ cnt, int64_t nb) {
    __shared__ uint32_t wc[4][kMaxLevels];
    const int t = threadIdx.x, w = t >> 6;
    const int64_t s = (int64_t)blockIdx.x * kBlock + t;
    const int l0 = s < n ? first_new_level(keys, s, L) : L + 1;
    for (int l = 0; l <= L; l++) {
        const uint64_t b = ballot64(l0 <= l);
        if (lane_id() == 0) wc[w][l] = (uint32_t)__popcll(b);
    }
    __syncthreads();
    if (t <= L) cnt[(int64_t)t * nb + blockIdx.x] = wc[0][t] + wc[1][t] + wc[2][t] + wc[3][t];
}

// Number each cell: for every level, the rank of the cell holding sorted
// position s.  Positions that open a cell write its start and first
// child (children of a cell are consecutive in the next level) into dense
// per-cell arrays; the cell record itself is written whole, once, by the
// pass that sums the cell (a part of a record written here would cost a read
// of the rest of its memory line).
// Then the leaf sums, part 1: gather the position into sorted order and run a
// segmented inclusive scan over each wave's 64 positions (segments = leaves,
// fixed shuffle pattern, FP64).  A leaf that starts and ends inside the wave
// gets its sum here; otherwise the wave records the piece of the segment that
// covers its first position (wfirst) and the piece of the segment that covers
// its last position (wlast).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_tree_nodes(
    const uint32_t* __restrict__ keys, int64_t n, int L, const uint32_t* __restrict__ off,
    int64_t nb, const uint32_t* __restrict__ ltot, DevScalars* __restrict__ sc,
    uint32_t* __restrict__ first_child, uint32_t* __restrict__ cell_start,
    uint32_t* __restrict__ leaf_of, const uint32_t* __restrict__ perm, const T* __restrict__ z,
    double2* __restrict__ nsum, T* __restrict__ zs, double2* __restrict__ wfirst,
    double2* __restrict__ wlast) {
    using V = v2_t<T>;
    __shared__ uint32_t wc[4][kMaxLevels];
    __shared__ uint32_t lbase[kMaxLevels + 1];
    const int t = threadIdx.x, w = t >> 6, lane = lane_id();
    if (t == 0) {
        uint32_t b = 0;
        for (int l = 0; l <= L; l++) {
            lbase[l] = b;
            b += ltot[l];
        }
        lbase[L + 1] = b;
        if (blockIdx.x == 0) {
            for (int l = 0; l <= L; l++) {
                sc->level_size[l] = ltot[l];
                sc->level_base[l] = lbase[l];
            }
            sc->level_base[L + 1] = b;
            sc->n_nodes = b;
        }
    }
    const int64_t s = (int64_t)blockIdx.x * kBlock + t;
    const bool valid = s < n;
    V p = V{T(0), T(0)};
    if (valid) p = reinterpret_cast<const V*>(z)[perm[s]];
    const int l0 = valid ? first_new_level(keys, s, L) : L + 1;
    // the next position starts a new leaf (or there is none)
    const bool tail = valid && (s == n - 1 || keys[s + 1] != keys[s]);
    for (int l = 0; l <= L; l++) {
        const uint64_t b = ballot64(l0 <= l);
        if (lane == 0) wc[w][l] = (uint32_t)__popcll(b);
    }
    __syncthreads();
    const uint64_t le = lanemask_lt() | (1ull << lane);
    uint32_t rank[kMaxLevels];
#pragma unroll
    for (int l = 0; l < kMaxLevels; l++) {
        if (l <= L) {
            const uint64_t b = ballot64(l0 <= l);
            uint32_t r = off[(int64_t)l * nb + blockIdx.x] + (uint32_t)__popcll(b & le);
            for (int q = 0; q < w; q++) r += wc[q][l];
            rank[l] = r - 1;
        } else {
            rank[l] = 0;
        }
    }
    const uint32_t lf = lbase[L] + rank[L];
    if (valid) {
        leaf_of[s] = lf;
        reinterpret_cast<V*>(zs)[s] = p;
#pragma unroll
        for (int l = 0; l < kMaxLevels; l++) {
            if (l <= L && l0 <= l) {
                const uint32_t gid = lbase[l] + rank[l];
                cell_start[gid] = (uint32_t)s;
                first_child[gid] = l < L ? lbase[l < L ? l + 1 : L] + rank[l < L ? l + 1 : L] : 0u;
            }
        }
    }
    // leaf sums: a position opens its leaf when its key differs from the
    // previous position's (l0 <= L)
    double vx = (double)p.x, vy = (double)p.y;
    bool f = valid && l0 <= L;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const double ax = __shfl_up(vx, o, kWave), ay = __shfl_up(vy, o, kWave);
        const bool af = __shfl_up((int)f, o, kWave) != 0;
        if (lane >= o) {
            if (!f) {
                vx = ax + vx;
                vy = ay + vy;
            }
            f = f || af;
        }
    }
    const int64_t wv = s / kWave;
    if (tail) {
        if (f) nsum[lf] = double2{vx, vy};
        else wfirst[wv] = double2{vx, vy};
    } else if (valid && lane == kWave - 1) {
        wlast[wv] = double2{vx, vy};
        if (!f) wfirst[wv] = double2{vx, vy};
    }
}

__device__ __forceinline__ void write_node(Node* __restrict__ nodes, CellF* __restrict__ c32,
                                           double2* __restrict__ nsum,
                                           uint32_t g, int level, int L, double sx, double sy,
                                           uint32_t count, uint32_t child, uint32_t start,
                                           uint32_t key0, int com_mode, float rs0, float rs1) {
    double cx, cy;
    if (com_mode == PSNE_COM_CELL_CENTER) {
        const int sh = L - level;
        const uint32_t pre = sh >= 16 ? 0u : (key0 >> (2 * sh));
        const double w = (double)(1u << sh);
        cx = (double)gather_bits16(pre) * w + 0.5 * w;
        cy = (double)gather_bits16(pre >> 1) * w + 0.5 * w;
    } else {
        cx = sx / (double)count;
        cy = sy / (double)count;
    }
    Node nd;
    nd.cx = cx;
    nd.cy = cy;
    nd.count = count;
    nd.child = child;
    nd.start = start;
    nd.level = (uint32_t)level;
    nodes[g] = nd;
    nsum[g] = double2{sx, sy};
    if (c32) c32[g] = CellF{(float)cx * rs0, (float)cy * rs1, (float)count, child};
}

// Leaf sums, part 2 (one thread per leaf): a leaf that spans several waves
// adds its pieces in wave order: the first piece, then the whole-wave pieces,
// then the last piece.  Up to kLeafSerial whole-wave pieces the leaf's own
// thread adds them one after another; a longer leaf (a dense pixel, up to
// thousands of pieces) is summed by the whole wavefront: lane j adds pieces
// j, j + 64, ... in order and the 64 lane sums are combined by a fixed
// butterfly, so the result does not depend on timing either way.  Every leaf
// writes its cell record.
constexpr uint32_t kLeafSerial = 8;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_tree_leaves(
    const uint32_t* __restrict__ keys, int64_t n, int L, int com_mode,
    const DevScalars* __restrict__ sc, const uint32_t* __restrict__ cell_start,
    Node* __restrict__ nodes, CellF* __restrict__ c32,
    double2* __restrict__ nsum, const double2* __restrict__ wfirst,
    const double2* __restrict__ wlast) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = lane_id();
    const uint32_t nleaf = sc->level_size[L];
    // whole waves past the last leaf leave; the others keep every lane for
    // the cooperative sums
    if ((t & ~(int64_t)(kWave - 1)) >= (int64_t)nleaf) return;
    const bool valid = t < (int64_t)nleaf;
    const uint32_t gid = sc->level_base[L] + (uint32_t)(valid ? t : 0);
    const uint32_t start = valid ? cell_start[gid] : 0u;
    const uint32_t end = !valid ? 1u : (t + 1 < nleaf) ? cell_start[gid + 1] : (uint32_t)n;
    const uint32_t wa = start / kWave, wb = (end - 1) / kWave;
    double sx = 0.0, sy = 0.0;
    const bool spans = valid && wa != wb;
    const bool coop = spans && wb - wa - 1 > kLeafSerial;
    if (valid && !spans) {
        const double2 v = nsum[gid];
        sx = v.x;
        sy = v.y;
    } else if (spans && !coop) {
        for (uint32_t w = wa + 1; w < wb; w++) {
            sx += wfirst[w].x;
            sy += wfirst[w].y;
        }
    }
    uint64_t todo = ballot64(coop);
    while (todo) {
        const int src = __ffsll((long long)todo) - 1;
        todo &= todo - 1;
        const uint32_t a = (uint32_t)__shfl((int)wa, src, kWave);
        const uint32_t b = (uint32_t)__shfl((int)wb, src, kWave);
        double px = 0.0, py = 0.0;
        for (uint32_t w = a + 1 + (uint32_t)lane; w < b; w += kWave) {
            px += wfirst[w].x;
            py += wfirst[w].y;
        }
        px = wave_sum(px);
        py = wave_sum(py);
        if (lane == src) {
            sx = px;
            sy = py;
        }
    }
    if (!valid) return;
    if (spans) {
        sx = (wlast[wa].x + sx) + wfirst[wb].x;
        sy = (wlast[wa].y + sy) + wfirst[wb].y;
    }
    write_node(nodes, c32, nsum, gid, L, L, sx, sy, end - start, 0u, start, keys[start], com_mode,
               cell_scale(sc->s[0]), cell_scale(sc->s[1]));
}

// One inner cell: count and sums of its children (consecutive in the next
// level) added in child order.
__device__ __forceinline__ void inner_cell(const uint32_t* __restrict__ keys, int l, int L,
                                           int com_mode, const DevScalars* __restrict__ sc,
                                           const uint32_t* __restrict__ first_child,
                                           const uint32_t* __restrict__ cell_start,
                                           Node* __restrict__ nodes, CellF* __restrict__ c32,
                                           double2* __restrict__ nsum, uint32_t t, uint32_t m,
                                           float rs0, float rs1) {
    const uint32_t g = sc->level_base[l] + t;
    const uint32_t fc = first_child[g];
    const uint32_t lc = (t + 1 < m) ? first_child[g + 1] : sc->level_base[l + 1] + sc->level_size[l + 1];
    double ax = 0.0, ay = 0.0;
    uint32_t c = 0;
    for (uint32_t q = fc; q < lc; q++) {
        const double2 v = nsum[q];
        ax += v.x;
        ay += v.y;
        c += nodes[q].count;
    }
    const uint32_t st = cell_start[g];
    write_node(nodes, c32, nsum, g, l, L, ax, ay, c, fc | ((lc - fc - 1) << 30), st, keys[st],
               com_mode, rs0, rs1);
}

// Up to kGroupLevels consecutive levels of inner cells in one launch.  Block
// b owns the cells [b K, (b + 1) K) of the group's top level and, below
// them, their descendants, which form one contiguous range per level (cells
// are numbered in Morton order within a level, and the children of a cell
// are consecutive): thread 0 follows first_child down to find the ranges,
// then the block sums the levels bottom-up, one level per barrier.  Each cell
// is summed by inner_cell exactly as one launch per level would.
constexpr int kGroupLevels = 5;
constexpr int64_t kGroupBlocks = 4096;

__global__ __launch_bounds__(kBlock) void k_tree_group(const uint32_t* __restrict__ keys,
                                                       int ltop, int lbot, int L, int com_mode,
                                                       uint32_t K,
                                                       const DevScalars* __restrict__ sc,
                                                       const uint32_t* __restrict__ first_child,
                                                       const uint32_t* __restrict__ cell_start,
                                                       Node* __restrict__ nodes,
                                                       CellF* __restrict__ c32,
                                                       double2* __restrict__ nsum) {
    __shared__ uint32_t lo[kGroupLevels], hi[kGroupLevels];
    const int t = threadIdx.x;
    const float rs0 = cell_scale(sc->s[0]), rs1 = cell_scale(sc->s[1]);
    const uint32_t mtop = sc->level_size[ltop];
    const uint32_t a0 = blockIdx.x * K;
    if (a0 >= mtop) return;
    if (t == 0) {
        uint32_t a = a0, e = a0 + K < mtop ? a0 + K : mtop;
        lo[0] = a;
        hi[0] = e;
        for (int l = ltop; l < lbot; l++) {
            // children of the level-l cells [a, e) at level l + 1
            const uint32_t base = sc->level_base[l], nbase = sc->level_base[l + 1];
            const uint32_t m = sc->level_size[l];
            a = first_child[base + a] - nbase;
            e = e < m ? first_child[base + e] - nbase : sc->level_size[l + 1];
            lo[l + 1 - ltop] = a;
            hi[l + 1 - ltop] = e;
        }
    }
    __syncthreads();
    for (int l = lbot; l >= ltop; l--) {
        const uint32_t m = sc->level_size[l];
        for (uint32_t x = lo[l - ltop] + t; x < hi[l - ltop]; x += kBlock)
            inner_cell(keys, l, L, com_mode, sc, first_child, cell_start, nodes, c32, nsum, x, m,
                       rs0, rs1);
        __syncthreads();
    }
}

// Levels top..0 in one block (a level l holds at most 4^l cells, so at most
// kTopThreads for l <= kTopLevel): the block finishes a level before it
// starts the one above.
constexpr int kTopLevel = 5;
constexpr int kTopThreads = 1024;

__global__ __launch_bounds__(kTopThreads) void k_tree_top(const uint32_t* __restrict__ keys,
                                                          int top, int L, int com_mode,
                                                          const DevScalars* __restrict__ sc,
                                                          const uint32_t* __restrict__ first_child,
                                                          const uint32_t* __restrict__ cell_start,
                                                          Node* __restrict__ nodes,
                                                          CellF* __restrict__ c32,
                                                          double2* __restrict__ nsum) {
    const float rs0 = cell_scale(sc->s[0]), rs1 = cell_scale(sc->s[1]);
    for (int l = top; l >= 0; l--) {
        const uint32_t m = sc->level_size[l];
        for (uint32_t t = threadIdx.x; t < m; t += kTopThreads)
            inner_cell(keys, l, L, com_mode, sc, first_child, cell_start, nodes, c32, nsum, t, m,
                       rs0, rs1);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Barnes-Hut traversal
// ---------------------------------------------------------------------------

// one accepted cell: Z_i += m q and R_i += m q^2 (z_i - c), q = 1 / (1 + d^2)
// (Eq. (11), (12)); m in the state type
template <typename T>
__device__ __forceinline__ void bh_term(double d2, double dx, double dy, T m, double& zacc,
                                        T& rx, T& ry);

template <>
__device__ __forceinline__ void bh_term<float>(double d2, double dx, double dy, float m,
                                               double& zacc, float& rx, float& ry) {
    const float q = __builtin_amdgcn_rcpf((float)(1.0 + d2));
    const float mq = m * q;
    zacc += (double)mq;
    const float f = mq * q;
    rx += f * (float)dx;
    ry += f * (float)dy;
}

template <>
__device__ __forceinline__ void bh_term<double>(double d2, double dx, double dy, double m,
                                                double& zacc, double& rx, double& ry) {
    const double q = rcp_nr(1.0 + d2);
    const double mq = m * q;
    zacc += mq;
    rx += mq * q * dx;
    ry += mq * q * dy;
}

// beta-weighted squared distance, evaluated exactly as ((b1*dx)*dx) + ((b2*dy)*dy)
// with every operation rounded separately (no fused multiply-add), so that the
// opening decision is the one the FP64 definition takes
__device__ __forceinline__ double dist2(double b1, double b2, double dx, double dy) {
#pragma clang fp contract(off)
    const double a = (b1 * dx) * dx;
    const double b = (b2 * dy) * dy;
    return a + b;
}
__device__ __forceinline__ double mul_nc(double a, double b) {
#pragma clang fp contract(off)
    return a * b;
}
__device__ __forceinline__ double add_nc(double a, double b) {
#pragma clang fp contract(off)
    return a + b;
}

// the FP32 distance on axis-scaled coordinates (cell_scale): dx*dx + dy*dy,
// each operation rounded separately
__device__ __forceinline__ float dist2s(float dx, float dy) {
#pragma clang fp contract(off)
    const float a = dx * dx;
    const float b = dy * dy;
    return a + b;
}
__device__ __forceinline__ float mulf_nc(float a, float b) {
#pragma clang fp contract(off)
    return a * b;
}

// Write a stack entry (four wave-uniform words, in scalar registers) into
// lane `sel` of the four per-lane stack registers.  With one scalar operand
// per vector instruction the lane select goes through m0 (an input operand:
// the compiler writes it with a scalar move); the s_nop adds two wait states
// before it is read.
__device__ __forceinline__ void push_entry(int& a, int& b, int& c, int& d, int va, int vb,
                                           int vc, int vd, int sel) {
    asm("s_nop 1\n\t"
        "v_writelane_b32 %0, %4, m0\n\t"
        "v_writelane_b32 %1, %5, m0\n\t"
        "v_writelane_b32 %2, %6, m0\n\t"
        "v_writelane_b32 %3, %7, m0"
        : "+v"(a), "+v"(b), "+v"(c), "+v"(d)
        : "s"(va), "s"(vb), "s"(vc), "s"(vd), "{m0}"(sel));
}

// The traversal's stack: entry k (a sibling group: its first cell, size and
// level, and the 64-bit mask of lanes that descend into it) lives in lane k of
// four registers.  A walk pushes at most three pending groups per level plus
// the one it expands next, so 3 (levels) + 1 entries suffice: 52 for the pixel
// tree (at most 17 levels), 100 for the data-driven tree (33 levels), which
// takes a second set of four registers for entries 64..127 (DEEP).
template <bool DEEP>
struct WaveStack {
    int f0 = 0, i0 = 0, lo0 = 0, hi0 = 0;
    int f1 = 0, i1 = 0, lo1 = 0, hi1 = 0;
    __device__ __forceinline__ void push(int sp, int f, int info, int lo, int hi) {
        if (!DEEP || sp < kWave) push_entry(f0, i0, lo0, hi0, f, info, lo, hi, sp);
        else push_entry(f1, i1, lo1, hi1, f, info, lo, hi, sp - kWave);
    }
    __device__ __forceinline__ void read(int sp, uint32_t& first, uint32_t& info,
                                         uint64_t& mask) const {
        if (!DEEP || sp < kWave) {
            first = (uint32_t)__builtin_amdgcn_readlane(f0, sp);
            info = (uint32_t)__builtin_amdgcn_readlane(i0, sp);
            mask = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(hi0, sp) << 32) |
                   (uint64_t)(uint32_t)__builtin_amdgcn_readlane(lo0, sp);
        } else {
            const int k = sp - kWave;
            first = (uint32_t)__builtin_amdgcn_readlane(f1, k);
            info = (uint32_t)__builtin_amdgcn_readlane(i1, k);
            mask = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(hi1, k) << 32) |
                   (uint64_t)(uint32_t)__builtin_amdgcn_readlane(lo1, k);
        }
    }
};

// a sibling group's records, read together
struct alignas(16) CellF4 { CellF c[4]; };
struct alignas(32) Node4 { Node n[4]; };

// F32T (FP32 path only): the opening test and the distances in FP32 on the
// cells' FP32 copies (cells32), whose coordinates are scaled by cell_scale so
// that the beta-weighted squared distance is dx*dx + dy*dy of the scaled
// differences, every operation rounded separately; the force sums run on the
// scaled axes and are scaled back at the end.  Otherwise in FP64 on nodes.
template <typename T, bool COUNT, bool F32T, bool DEEP>
__global__ __launch_bounds__(kBlock) void k_traverse(
    const Node* __restrict__ nodes, const CellF* __restrict__ cells32,
    const double2* __restrict__ nsum, const T* __restrict__ zs,
    const uint32_t* __restrict__ perm, const uint32_t* __restrict__ leaf_of,
    const DevScalars* __restrict__ sc, int64_t n, int L, double th2, int com_mode,
    T* __restrict__ R, double* __restrict__ zpart, const uint32_t* __restrict__ orig,
    double* __restrict__ Zi_out, uint32_t* __restrict__ visits_out,
    uint32_t* __restrict__ used_out) {
    using V = v2_t<T>;
    static_assert(!F32T || sizeof(T) == 4, "the FP32 opening test belongs to the FP32 path");
    __shared__ double wz[4];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool valid = s < n;
    const V zp = valid ? reinterpret_cast<const V*>(zs)[s] : V{T(0), T(0)};
    const double zx = (double)zp.x, zy = (double)zp.y;
    const uint32_t own = valid ? leaf_of[s] : 0xFFFFFFFFu;
    const double s0 = sc->s[0], s1 = sc->s[1];
    const double b1 = mul_nc(s0, s0), b2 = mul_nc(s1, s1), bsum = add_nc(b1, b2);
    // single-precision operands of the FP32 test: beta and theta^2 rounded,
    // the point on the cells' scaled axes
    const float b1f = (float)b1, b2f = (float)b2, th2f = (float)th2;
    const float bsumf = b1f + b2f;
    const float rs0 = cell_scale(s0), rs1 = cell_scale(s1);
    const float xs = (float)zp.x * rs0, ys = (float)zp.y * rs1;

    double zacc = 0.0;
    T rx = T(0), ry = T(0);
    uint32_t nvis = 0, nuse = 0;

    // stack entries: first cell of a sibling group, (group size | level << 8),
    // lane mask (lo, hi)
    WaveStack<DEEP> st;
    int sp = 0;
    const uint64_t m0 = ballot64(valid);
    if (m0) {
        st.push(0, 0, 1, (int)(uint32_t)m0, (int)(uint32_t)(m0 >> 32));
        sp = 1;
    }
    while (sp > 0) {
        sp--;
        uint32_t first, info;
        uint64_t mask;
        st.read(sp, first, info, mask);
        const uint32_t nsib = info & 0xFFu;
        const int level = (int)(info >> 8);
        const bool act = __builtin_amdgcn_inverse_ballot_w64(mask);   // lane in mask
        if constexpr (F32T) {
            // (w w)(b1 + b2) with w = 2^(L - level): a power-of-two scaling, exact in FP32
            const float diag2f = ldexpf(bsumf, 2 * (L - level));
            // the group's four records (children are consecutive; the array
            // has three records of slack at its end) in one 64-byte scalar load
            const CellF4 g4 = *reinterpret_cast<const CellF4*>(cells32 + first);
            const CellF* grp = g4.c;
            float zg = 0.f;
#pragma unroll
            for (uint32_t q = 0; q < 4; q++) {
                if (q >= nsib) break;
                const uint32_t c = first + q;
                const CellF nd = grp[q];
                uint64_t om = 0;
                // per lane: the distance, q = 1 / (1 + d^2), the mass term m q
                // and whether the lane takes the cell; the sums follow below
                float dx, dy, qq, mq;
                bool use;
                if (nd.child != 0u) {
                    dx = xs - nd.cx;
                    dy = ys - nd.cy;
                    const float d2 = dist2s(dx, dy);
                    const uint64_t near = ballot64(!(diag2f < mulf_nc(th2f, d2)));
                    om = near & mask;
                    use = __builtin_amdgcn_inverse_ballot_w64(mask & ~near);
                    qq = __builtin_amdgcn_rcpf(1.0f + d2);
                    mq = qq * nd.mass;
                    if (COUNT) {
                        nuse += use ? 1u : 0u;
                        nvis += act ? 1u : 0u;
                    }
                } else {
                    float cx = nd.cx, cy = nd.cy;
                    float m = nd.mass;
                    use = act;
                    if (c == own) {
                        // the exact count from the FP64 record (its FP32 copy
                        // is rounded above 2^24)
                        const uint32_t others = nodes[c].count - 1u;
                        m = (float)others;
                        if (others > 0u && com_mode != PSNE_COM_CELL_CENTER) {
                            const double2 sm = nsum[c];
                            const double inv = 1.0 / (double)others;
                            cx = (float)((sm.x - zx) * inv) * rs0;
                            cy = (float)((sm.y - zy) * inv) * rs1;
                        }
                        use = act && others > 0u;
                    }
                    dx = xs - cx;
                    dy = ys - cy;
                    qq = __builtin_amdgcn_rcpf(1.0f + dist2s(dx, dy));
                    mq = qq * m;
                    if (COUNT) {
                        nuse += use ? 1u : 0u;
                        nvis += act ? 1u : 0u;
                    }
                }
                // every lane adds the term; a lane that does not take the cell
                // adds zeros, which leaves its sums bit for bit as they were
                mq = use ? mq : 0.f;
                zg += mq;
                const float f = mq * qq;
                rx = fmaf(f, dx, rx);
                ry = fmaf(f, dy, ry);
                if (om) {
                    st.push(sp, (int)(nd.child & 0x3FFFFFFFu),
                            (int)(((nd.child >> 30) + 1u) | ((uint32_t)(level + 1) << 8)),
                            (int)(uint32_t)om, (int)(uint32_t)(om >> 32));
                    sp++;
                }
            }
            zacc += (double)zg;
        } else {
        const double diag2 = ldexp(bsum, 2 * (L - level));
        // the group's records (children are consecutive) in one batch of scalar loads
        const Node4 g4 = *reinterpret_cast<const Node4*>(nodes + first);
        const Node* grp = g4.n;
#pragma unroll
        for (uint32_t q = 0; q < 4; q++) {
            if (q >= nsib) break;
            const uint32_t c = first + q;
            const Node nd = grp[q];
            uint64_t om = 0;   // lanes that open the cell
            // Every lane evaluates the term; lanes that do not take the cell
            // add it with mass 0, which leaves their sums bit for bit as they
            // were and keeps the loop free of divergent branches.
            double dx, dy, d2;
            T m;
            bool use;
            uint64_t take = mask;   // lanes that take the cell
            if (nd.child != 0u) {
                // inner cell: the opening test and, for lanes that accept, the
                // force term share one distance
                dx = zx - nd.cx;
                dy = zy - nd.cy;
                d2 = dist2(b1, b2, dx, dy);
                const uint64_t near = ballot64(!(diag2 < mul_nc(th2, d2)));
                om = near & mask;   // every lane runs this loop
                take = mask & ~near;
                use = __builtin_amdgcn_inverse_ballot_w64(take);
                m = (T)nd.count;
            } else {
                // leaf (one pixel): always used; at its own leaf a point counts
                // the others only, at their centre of mass in mass mode
                double cx = nd.cx, cy = nd.cy;
                m = (T)nd.count;
                use = act;
                if (c == own) {
                    const uint32_t others = nd.count - 1u;
                    m = (T)others;
                    if (others > 0u && com_mode != PSNE_COM_CELL_CENTER) {
                        const double2 sm = nsum[c];
                        cx = (sm.x - zx) / (double)others;
                        cy = (sm.y - zy) / (double)others;
                    }
                    use = act && others > 0u;
                }
                dx = zx - cx;
                dy = zy - cy;
                d2 = dist2(b1, b2, dx, dy);
            }
            // skipped when every lane opens the cell (the FP64 reciprocal is
            // a long sequence; the FP32 path gains nothing from the branch)
            if (take) bh_term<T>(d2, dx, dy, use ? m : T(0), zacc, rx, ry);
            if (COUNT) {
                nuse += use ? 1u : 0u;
                nvis += act ? 1u : 0u;
            }
            if (om) {
                st.push(sp, (int)(nd.child & 0x3FFFFFFFu),
                        (int)(((nd.child >> 30) + 1u) | ((uint32_t)(level + 1) << 8)),
                        (int)(uint32_t)om, (int)(uint32_t)(om >> 32));
                sp++;
            }
        }
        }
    }
    if (valid) {
        const uint32_t i = perm[s];
        if constexpr (F32T) {
            // the FP32 sums ran on the scaled axes: back to pixel units
            reinterpret_cast<V*>(R)[i] = V{rx / rs0, ry / rs1};
        } else {
            reinterpret_cast<V*>(R)[i] = V{rx, ry};
        }
        if (Zi_out) Zi_out[orig[i]] = zacc;
        if (visits_out) visits_out[orig[i]] = nvis;
        if (used_out) used_out[orig[i]] = nuse;
    }
    const double zw = wave_sum(zacc);
    if (lane == 0) wz[w] = zw;
    __syncthreads();
    if (threadIdx.x == 0) zpart[blockIdx.x] = ((wz[0] + wz[1]) + wz[2]) + wz[3];
}

__global__ __launch_bounds__(kBlock) void k_zsum(const double* __restrict__ zpart, int64_t m,
                                                 DevScalars* __restrict__ sc) {
    __shared__ double red[kBlock];
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += kBlock) a += zpart[i];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) sc->Z = red[0];
}

// ---------------------------------------------------------------------------
// attraction + update
// ---------------------------------------------------------------------------
struct StepParams {
    double exaggeration, eta, mom0, mom1, min_gain, alpha_override;
    int32_t exag_iters, mom_switch;
};

template <typename T> __device__ __forceinline__ T rcp_fast(T x);
template <> __device__ __forceinline__ float rcp_fast<float>(float x) {
    return __builtin_amdgcn_rcpf(x);
}
template <> __device__ __forceinline__ double rcp_fast<double>(double x) { return rcp_nr(x); }

template <typename T> __device__ __forceinline__ T sgn(T x) {
    return x > T(0) ? T(1) : (x < T(0) ? T(-1) : T(0));
}

// Lane-shifted copies within a wavefront (DPP).  CTRL selects the pattern:
// row_shr:d moves lane l - d to lane l inside each row of 16 lanes;
// row_bcast:15 / :31 broadcast lane 15 / 31 into the rows that follow.  Lanes
// without a source (the first d of a row, rows outside ROWS) get OLD.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_i(int old, int v) {
    return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_t(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, true));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_t(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = dpp_i<CTRL, ROWS>(0, (int)(uint32_t)b);
    const int hi = dpp_i<CTRL, ROWS>(0, (int)(uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// One step of the segmented scan: add the partial sums of the source lane
// when it carries the same key (a lane without a source sees key -1, which no
// lane carries).  The add is a multiply by 1 or 0, which keeps the step free
// of branches; x + 1 * u and x + 0 * u are exactly x + u and x.
template <int CTRL, int ROWS, typename T>
__device__ __forceinline__ void seg_step(T& x, T& y, int key) {
    const int k = dpp_i<CTRL, ROWS>(-1, key);
    const T ux = dpp_t<CTRL, ROWS>(x), uy = dpp_t<CTRL, ROWS>(y);
    const T m = k == key ? T(1) : T(0);
    x = fma(ux, m, x);
    y = fma(uy, m, y);
}

// Inclusive scan of (x, y) over the lanes of each run of equal keys, for keys
// ascending across the wave (Hillis-Steele: at each step a lane adds the
// partial sum of the lane d below when both carry the same key; keys are
// sorted, so that partial never leaves the run).  The last lane of a run ends
// with the run's total.  CONT has bit l set when lane l continues the run of
// lane l - 1; steps that no run needs are skipped (wave-uniform branches):
// the shift by d only when some run is longer than d, the broadcast of lane
// 15 / 47 or 31 only when a run crosses it.
template <typename T>
__device__ __forceinline__ void seg_scan(T& x, T& y, int key, uint64_t cont) {
    const uint64_t c2 = cont & (cont >> 1), c4 = c2 & (c2 >> 2), c8 = c4 & (c4 >> 4);
    if (cont) seg_step<0x111, 0xF>(x, y, key);
    if (c2) seg_step<0x112, 0xF>(x, y, key);
    if (c4) seg_step<0x114, 0xF>(x, y, key);
    if (c8) seg_step<0x118, 0xF>(x, y, key);
    if (cont & ((1ull << 16) | (1ull << 48))) seg_step<0x142, 0xA>(x, y, key);
    if (cont & (1ull << 32)) seg_step<0x143, 0xC>(x, y, key);
}

// An in-row step of the FP32 scan with the lanes that take a value known in
// scalar registers: a row shift by d moves each lane's value to one lane d
// above, so a source lane whose destination does not take it sends 0 (SRC:
// bit s set when lane s + d takes), and the step is a select and an add
// with the shift folded in, per coordinate.
template <int CTRL>
__device__ __forceinline__ void seg_step_src(float& x, float& y, uint64_t src) {
    const bool send = __builtin_amdgcn_inverse_ballot_w64(src);
    const float sx = send ? x : 0.f, sy = send ? y : 0.f;
    x += dpp_t<CTRL, 0xF>(sx);
    y += dpp_t<CTRL, 0xF>(sy);
}

// Lanes s .. s + w - 1 that continue the run of lane s - 1 without a break:
// the lowest run of set bits of CONT starting at bit s, as a lane mask.
__device__ __forceinline__ uint64_t run_from(uint64_t cont, int s, int w) {
    const uint64_t wmask = (1ull << w) - 1ull;
    const uint64_t x = (cont >> s) & wmask;
    return (((~x & (x + 1ull)) - 1ull) & wmask) << s;   // bits below the lowest clear bit
}

// FP32: lane l takes the value d lanes below when lanes l - d + 1 .. l all
// continue their predecessor's run (A_d, from CONT by doubling).  Across
// rows the same masks decide: rows 1 and 3 take lanes 15 and 47 (one
// broadcast), then rows 2 and 3 take lane 31 (a scalar read), each lane when
// its run reaches back to that lane.  The multiplier 1 or 0 leaves a lane
// that does not take the value exactly as it was.
template <>
__device__ __forceinline__ void seg_scan<float>(float& x, float& y, int, uint64_t cont) {
    const uint64_t a2 = cont & (cont << 1), a4 = a2 & (a2 << 2), a8 = a4 & (a4 << 4);
    if (cont) seg_step_src<0x111>(x, y, cont >> 1);
    if (a2) seg_step_src<0x112>(x, y, a2 >> 2);
    if (a4) seg_step_src<0x114>(x, y, a4 >> 4);
    if (a8) seg_step_src<0x118>(x, y, a8 >> 8);
    const uint64_t ta = run_from(cont, 16, 16) | run_from(cont, 48, 16);
    if (ta) {
        const float m = __builtin_amdgcn_inverse_ballot_w64(ta) ? 1.f : 0.f;
        x = fmaf(dpp_t<0x142, 0xF>(x), m, x);   // row r gets lane 16 r - 1; row 0 gets 0
        y = fmaf(dpp_t<0x142, 0xF>(y), m, y);
    }
    const uint64_t tb = run_from(cont, 32, 32);
    if (tb) {
        const float m = __builtin_amdgcn_inverse_ballot_w64(tb) ? 1.f : 0.f;
        x = fmaf(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 31)), m, x);
        y = fmaf(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(y), 31)), m, y);
    }
}

// The chunk's column words and values are read once per iteration through
// buffer resources over the chunk's range: 32-bit offsets, and the hardware's
// range check returns 0 past the end instead of a per-lane select.  Loads
// carry the non-temporal hint, which keeps the caches for the gathered z_j.
// A chunk holds fewer than 2^27 nonzeros, so offsets in bytes fit in 31 bits.
constexpr int kRawBufferWord3 = 0x00020000;   // descriptor word 3: untyped 32-bit access
template <typename E>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t stream_rsrc(const E* base, int64_t count) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)(count * sizeof(E)),
                                             kRawBufferWord3);
}
constexpr int kStreamPolicy = 2;   // non-temporal
template <typename E> __device__ __forceinline__ E stream_load(__amdgpu_buffer_rsrc_t r, int i);
template <> __device__ __forceinline__ uint32_t stream_load<uint32_t>(__amdgpu_buffer_rsrc_t r,
                                                                      int i) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, i * 4, 0, kStreamPolicy);
}
template <> __device__ __forceinline__ double stream_load<double>(__amdgpu_buffer_rsrc_t r, int i) {
    return __longlong_as_double(
        (long long)__builtin_amdgcn_raw_buffer_load_b64(r, i * 8, 0, kStreamPolicy));
}

// runs of 64 nonzeros per wavefront in flight (measured with the sums on the
// second stream beside the traversal: 8 beats 10, 12, 16, 20 and 24)
template <typename T> constexpr int kBatches = 8;

// One block per row chunk.  MODE 0 (the iteration's row sums, on the second
// stream) and MODE 2 (a helper launched on the main stream once the traversal
// and Z are done) take chunks from one work queue, a counter in DevScalars
// that k_finalize clears for the next iteration: while the main stream is
// busy the second stream's few blocks per CU do the work, and whatever is
// left when it frees the CUs is shared with the helper's blocks.  Which
// block takes a chunk does not change its sums.  MODE 1 walks the chunks
// grid-stride.  Wavefront w takes
// the runs w, w + 4, ... of the chunk's nonzeros (column order, each run of
// 64 ordered by row): loads kBatches runs at once, computes the terms
// p_ij w_ij (z_i - z_j) with z_i from LDS, sums each row's terms across the
// run with a segmented scan, and adds the totals to its own LDS partial sums
// (one writer per address, no atomics).  Thread t < rows of the chunk then
// adds the four waves' partials in a fixed order.  Sums are therefore
// reproducible.  MODE 0 and 2 (the iteration) write the row sums A_i in the
// internal order; MODE 1 (the gradient hook) writes A_i and the full
// gradient B_i = alpha A_i - R_i / Z in the caller's order, after the
// traversal.
template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_attract(
    const uint32_t* __restrict__ ch_row, const int64_t* __restrict__ rp_int,
    const uint32_t* __restrict__ pk, const T* __restrict__ val, const T* __restrict__ z,
    const T* __restrict__ R, DevScalars* __restrict__ sc, double alpha,
    const uint32_t* __restrict__ orig, T* __restrict__ Aout, T* __restrict__ Bout, int early) {
    using V = v2_t<T>;
    if (MODE == 0 && early) {
        // the launch right after the snap pass: it stamps the clock for the
        // fork-point tuner and leaves at once when this iteration forks after
        // the cells (or, EARLY = 2, when the second stream has no blocks)
        if (blockIdx.x == 0 && threadIdx.x == 0) sc->t_begin = wall_clock64();
        if (early > 1 || sc->fork_late) return;
    }
    __shared__ T acc[4][kChunkRows][2];
    __shared__ V zrow[kChunkRows + 1];   // entry kChunkRows: 0 for lanes past the end
    __shared__ uint32_t s_next;
    constexpr bool kQueue = MODE != 1;
    const int t = threadIdx.x, lane = lane_id(), w = t >> 6;
    const double s0 = sc->s[0], s1 = sc->s[1];
    const T b1 = (T)(s0 * s0), b2 = (T)(s1 * s1);
    const int64_t nch = sc->n_chunks;
    constexpr uint32_t kColMask = (1u << kColBits) - 1u;
    int64_t ch = blockIdx.x;
    if (kQueue) {
        if (t == 0) s_next = atomicAdd(&sc->att_next, 1u);
        __syncthreads();
        ch = s_next;
    }
    while (ch < nch) {
        // the next chunk's ticket is taken while this one is summed
        uint32_t ticket = 0;
        if (kQueue && t == 0) ticket = atomicAdd(&sc->att_next, 1u);
        const int64_t ra = ch_row[ch];
        const int nr = (int)((int64_t)ch_row[ch + 1] - ra);
        const int64_t e0 = rp_int[ra], e1 = rp_int[ra + nr];
        if (t <= kChunkRows) zrow[t] = t < nr ? reinterpret_cast<const V*>(z)[ra + t] : V{T(0), T(0)};
        if (t < 4 * kChunkRows) {
            acc[t / kChunkRows][t % kChunkRows][0] = T(0);
            acc[t / kChunkRows][t % kChunkRows][1] = T(0);
        }
        __syncthreads();
        constexpr bool kPair = sizeof(T) == 4;      // FP32: word and value side by side
        const __amdgpu_buffer_rsrc_t rpk =
            kPair ? stream_rsrc(pk + 2 * e0, 2 * (e1 - e0)) : stream_rsrc(pk + e0, e1 - e0);
        const __amdgpu_buffer_rsrc_t rval = kPair ? rpk : stream_rsrc(val + e0, e1 - e0);
        for (int64_t b = e0 + (int64_t)w * kWave; b < e1; b += (int64_t)kBlock * kBatches<T>) {
            uint32_t j[kBatches<T>];
            int r[kBatches<T>];
            T p[kBatches<T>];
#pragma unroll
            for (int q = 0; q < kBatches<T>; q++) {
                const int64_t x = b + q * kBlock + lane;
                const int off = (int)(x - e0);
                uint32_t v;
                if constexpr (kPair) {
                    const auto pv = __builtin_amdgcn_raw_buffer_load_b64(rpk, off * 8, 0,
                                                                         kStreamPolicy);
                    v = pv[0];
                    p[q] = (T)__uint_as_float(pv[1]);
                } else {
                    v = stream_load<uint32_t>(rpk, off);
                    p[q] = stream_load<T>(rval, off);
                }
                j[q] = v & kColMask;
                r[q] = x < e1 ? (int)(v >> kColBits) : kChunkRows;
            }
            V zj[kBatches<T>];
#pragma unroll
            for (int q = 0; q < kBatches<T>; q++) zj[q] = reinterpret_cast<const V*>(z)[j[q]];
#pragma unroll
            for (int q = 0; q < kBatches<T>; q++) {
                const V zi = zrow[r[q]];
                const T dx = zi.x - zj[q].x, dy = zi.y - zj[q].y;
                const T wq = rcp_fast<T>(T(1) + b1 * dx * dx + b2 * dy * dy);
                const T pw = p[q] * wq;
                T sx = pw * dx, sy = pw * dy;
                // lane l continues the run of lane l - 1 when both carry the
                // same row (the row of lane l - 1 by a whole-wave shift; lane 0
                // sees -1); lanes past the chunk's end (row kChunkRows) belong
                // to no run and are never written.  A lane ends its run when
                // the next lane does not continue it.
                const int rprev = __builtin_amdgcn_update_dpp(-1, r[q], 0x138, 0xF, 0xF, false);
                const uint64_t live = ballot64(r[q] < kChunkRows);
                const uint64_t cont = ballot64(rprev == r[q]) & live;
                const uint64_t last = ~(cont >> 1) & live;
                seg_scan<T>(sx, sy, r[q], cont);
                if (__builtin_amdgcn_inverse_ballot_w64(last)) {
                    acc[w][r[q]][0] += sx;
                    acc[w][r[q]][1] += sy;
                }
            }
        }
        __syncthreads();
        if (t < nr) {
            const T mx = ((acc[0][t][0] + acc[1][t][0]) + acc[2][t][0]) + acc[3][t][0];
            const T my = ((acc[0][t][1] + acc[1][t][1]) + acc[2][t][1]) + acc[3][t][1];
            const int64_t i = ra + t;
            if (MODE != 1) {
                reinterpret_cast<V*>(Aout)[i] = V{mx, my};
            } else {
                const double Z = sc->Z;
                const V Ri = reinterpret_cast<const V*>(R)[i];
                const T bx = (T)(alpha * (double)mx - (double)Ri.x / Z);
                const T by = (T)(alpha * (double)my - (double)Ri.y / Z);
                if (Aout) reinterpret_cast<V*>(Aout)[orig[i]] = V{mx, my};
                if (Bout) reinterpret_cast<V*>(Bout)[orig[i]] = V{bx, by};
            }
        }
        if (kQueue && t == 0) s_next = ticket;
        __syncthreads();
        ch = kQueue ? (int64_t)s_next : ch + gridDim.x;
    }
}

// The optimiser step for every point (internal order), after the attraction
// and the traversal: B_i = alpha A_i - R_i / Z, gains and momentum, the new
// positions zh, and the per-block min/max of zh for the screen scaling.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_update(
    const T* __restrict__ A, const T* __restrict__ z, const T* __restrict__ R, T* __restrict__ u,
    T* __restrict__ g, T* __restrict__ zh, DevScalars* __restrict__ sc, StepParams prm, int64_t n,
    double* __restrict__ mm_part) {
    using V = v2_t<T>;
    __shared__ double red[4][4];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const double Z = sc->Z;
    const int it = sc->t;
    const double alpha = it < prm.exag_iters ? prm.exaggeration : 1.0;
    const T mu = (T)(it < prm.mom_switch ? prm.mom0 : prm.mom1);
    const T us0 = (T)sc->uscale[0], us1 = (T)sc->uscale[1];
    const T eta = (T)prm.eta, gmin = (T)prm.min_gain;
    double mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const V a = reinterpret_cast<const V*>(A)[i];
        const V Ri = reinterpret_cast<const V*>(R)[i];
        const T bx = (T)(alpha * (double)a.x - (double)Ri.x / Z);
        const T by = (T)(alpha * (double)a.y - (double)Ri.y / Z);
        const V zi = reinterpret_cast<const V*>(z)[i];
        V ui = reinterpret_cast<V*>(u)[i];
        V gi = reinterpret_cast<V*>(g)[i];
        ui.x *= us0;
        ui.y *= us1;
        T gx = sgn(bx) != sgn(ui.x) ? gi.x + T(0.2) : gi.x * T(0.8);
        T gy = sgn(by) != sgn(ui.y) ? gi.y + T(0.2) : gi.y * T(0.8);
        gx = gx < gmin ? gmin : gx;
        gy = gy < gmin ? gmin : gy;
        ui.x = mu * ui.x - eta * gx * bx;
        ui.y = mu * ui.y - eta * gy * by;
        const T hx = zi.x + ui.x, hy = zi.y + ui.y;
        reinterpret_cast<V*>(u)[i] = ui;
        reinterpret_cast<V*>(g)[i] = V{gx, gy};
        reinterpret_cast<V*>(zh)[i] = V{hx, hy};
        if (!isfinite(hx) || !isfinite(hy)) bad = true;
        mnx = fmin(mnx, (double)hx);
        mny = fmin(mny, (double)hy);
        mxx = fmax(mxx, (double)hx);
        mxy = fmax(mxy, (double)hy);
    }
    if (ballot64(bad) && lane == 0) atomicOr(&sc->nonfinite, 1);
    mnx = wave_min(mnx); mny = wave_min(mny); mxx = wave_max(mxx); mxy = wave_max(mxy);
    if (lane == 0) {
        red[w][0] = mnx; red[w][1] = mny; red[w][2] = mxx; red[w][3] = mxy;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        double v = red[0][k];
        for (int q = 1; q < 4; q++) v = k < 2 ? fmin(v, red[q][k]) : fmax(v, red[q][k]);
        mm_part[(int64_t)blockIdx.x * 4 + k] = v;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_minmax(const T* __restrict__ zh, int64_t n,
                                                   double* __restrict__ mm_part) {
    using V = v2_t<T>;
    __shared__ double red[4][4];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    double mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const V p = reinterpret_cast<const V*>(zh)[i];
        mnx = fmin(mnx, (double)p.x); mny = fmin(mny, (double)p.y);
        mxx = fmax(mxx, (double)p.x); mxy = fmax(mxy, (double)p.y);
    }
    mnx = wave_min(mnx); mny = wave_min(mny); mxx = wave_max(mxx); mxy = wave_max(mxy);
    if (lane == 0) { red[w][0] = mnx; red[w][1] = mny; red[w][2] = mxx; red[w][3] = mxy; }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        double v = red[0][k];
        for (int q = 1; q < 4; q++) v = k < 2 ? fmin(v, red[q][k]) : fmax(v, red[q][k]);
        mm_part[(int64_t)blockIdx.x * 4 + k] = v;
    }
}

// screen-driven scaling: gamma = max - min + eps per axis (Section 4.2)
__global__ __launch_bounds__(kBlock) void k_finalize(const double* __restrict__ mm_part,
                                                     int64_t m, DevScalars* __restrict__ sc,
                                                     int r, double eps, int advance, int fork) {
    __shared__ double red[4][kBlock];
    double mn0 = INFINITY, mn1 = INFINITY, mx0 = -INFINITY, mx1 = -INFINITY;
    for (int64_t i = threadIdx.x; i < m; i += kBlock) {
        mn0 = fmin(mn0, mm_part[4 * i + 0]);
        mn1 = fmin(mn1, mm_part[4 * i + 1]);
        mx0 = fmax(mx0, mm_part[4 * i + 2]);
        mx1 = fmax(mx1, mm_part[4 * i + 3]);
    }
    red[0][threadIdx.x] = mn0; red[1][threadIdx.x] = mn1;
    red[2][threadIdx.x] = mx0; red[3][threadIdx.x] = mx1;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const int a = threadIdx.x, b = threadIdx.x + o;
            red[0][a] = fmin(red[0][a], red[0][b]);
            red[1][a] = fmin(red[1][a], red[1][b]);
            red[2][a] = fmax(red[2][a], red[2][b]);
            red[3][a] = fmax(red[3][a], red[3][b]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int d = 0; d < 2; d++) {
            const double lo = red[d][0], hi = red[2 + d][0];
            const double gamma = hi - lo + eps;
            sc->zmin[d] = lo;
            sc->scale[d] = (double)r / gamma;
            sc->uscale[d] = (double)r / gamma;
            sc->s[d] = sc->s[d] * (gamma / (double)r);
        }
        if (advance) {
            sc->t += 1;
            // The fork-point tuner.  The time from the snap pass to here is
            // the iteration's (the snap pass and the renumbering take the
            // same time at either fork point); it is averaged, as single
            // iterations vary by about as much as the two points differ.
            // Automatic: after fork_gap iterations at one point (whose times
            // feed a moving average), kForkProbeLen run at the other (their
            // plain mean: older probes are out of date), and the next takes
            // the point with the smaller average.  The gap doubles (to
            // kForkGapMax) while the probes confirm the choice and falls back
            // to kForkGapMin when they change it.
            const int cur = sc->fork_late;
            const float ticks = (float)(wall_clock64() - sc->t_begin);
            const float avg = sc->fork_ticks[cur];
            const int k = sc->fork_count + kForkProbeLen;  // sample of this probe
            if (fork == PSNE_FORK_AUTO && sc->fork_count < 0)
                sc->fork_ticks[cur] = k == 0 ? ticks : avg + (ticks - avg) / (float)(k + 1);
            else
                sc->fork_ticks[cur] = avg > 0.f ? avg + kForkWeight * (ticks - avg) : ticks;
            int next = cur;
            if (fork != PSNE_FORK_AUTO) {
                next = fork == PSNE_FORK_CELLS;
            } else if (sc->fork_count < 0) {
                // a probe: go on with it, or take the decision after its last
                if (++sc->fork_count == 0) {
                    next = sc->fork_ticks[1] < sc->fork_ticks[0];
                    sc->fork_gap = next == cur ? kForkGapMin : min(2 * sc->fork_gap, kForkGapMax);
                }
            } else if (++sc->fork_count >= sc->fork_gap) {
                next = 1 - cur;
                sc->fork_count = -kForkProbeLen;
            }
            sc->fork_late = next;
        }
        sc->att_next = 0;
    }
}

// the initial embedding: splitmix64 uniforms through the Box-Muller transform

template <typename T>
__global__ __launch_bounds__(kBlock) void k_init_state(const double* __restrict__ Y, T* __restrict__ zh,
                                                       T* __restrict__ u, T* __restrict__ g,
                                                       int64_t n, uint64_t seed, double sigma) {
    using V = v2_t<T>;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double y0, y1;
    if (Y) {
        y0 = Y[2 * i];
        y1 = Y[2 * i + 1];
    } else {
        const uint64_t a = splitmix64(seed ^ (2ull * (uint64_t)i));
        const uint64_t b = splitmix64(seed ^ (2ull * (uint64_t)i + 1ull));
        const double u1 = ((double)(a >> 11) + 0.5) * 0x1.0p-53;
        const double u2 = ((double)(b >> 11) + 0.5) * 0x1.0p-53;
        const double rad = sqrt(-2.0 * log(u1));
        y0 = sigma * rad * cos(2.0 * M_PI * u2);
        y1 = sigma * rad * sin(2.0 * M_PI * u2);
    }
    reinterpret_cast<V*>(zh)[i] = V{(T)y0, (T)y1};
    reinterpret_cast<V*>(u)[i] = V{T(0), T(0)};
    reinterpret_cast<V*>(g)[i] = V{T(1), T(1)};
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_get_y(const T* __restrict__ zh,
                                                  const DevScalars* __restrict__ sc,
                                                  const uint32_t* __restrict__ orig, int64_t n,
                                                  int r, int frame, void* __restrict__ out) {
    const int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i0 >= n) return;
    const v2_t<T> p = norm_pos<T>(zh, sc, i0, r);
    const int64_t i = orig[i0];
    if (frame == PSNE_FRAME_SCREEN) {
        int px = (int)p.x, py = (int)p.y;
        px = px > r - 1 ? r - 1 : px;
        py = py > r - 1 ? r - 1 : py;
        reinterpret_cast<int2*>(out)[i] = int2{px, py};
    } else if (frame == PSNE_FRAME_Y) {
        reinterpret_cast<double2*>(out)[i] = double2{(double)p.x * sc->s[0], (double)p.y * sc->s[1]};
    } else {
        reinterpret_cast<double2*>(out)[i] = double2{(double)p.x, (double)p.y};
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_get_state(const T* __restrict__ zh, const T* __restrict__ u,
                                                      const T* __restrict__ g,
                                                      const DevScalars* __restrict__ sc,
                                                      const uint32_t* __restrict__ orig, int64_t n,
                                                      int r, T* __restrict__ zo, T* __restrict__ uo,
                                                      T* __restrict__ go) {
    using V = v2_t<T>;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t o = orig[i];
    if (zo) reinterpret_cast<V*>(zo)[o] = norm_pos<T>(zh, sc, i, r);
    if (uo) {
        V v = reinterpret_cast<const V*>(u)[i];
        v.x *= (T)sc->uscale[0];
        v.y *= (T)sc->uscale[1];
        reinterpret_cast<V*>(uo)[o] = v;
    }
    if (go) reinterpret_cast<V*>(go)[o] = reinterpret_cast<const V*>(g)[i];
}

// state from the caller's order (u, g NULL => zeros, ones)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_set_state(const T* __restrict__ zin, const T* __restrict__ uin,
                                                      const T* __restrict__ gin,
                                                      const uint32_t* __restrict__ orig, int64_t n,
                                                      T* __restrict__ zh, T* __restrict__ u,
                                                      T* __restrict__ g) {
    using V = v2_t<T>;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t o = orig[i];
    reinterpret_cast<V*>(zh)[i] = reinterpret_cast<const V*>(zin)[o];
    reinterpret_cast<V*>(u)[i] = uin ? reinterpret_cast<const V*>(uin)[o] : V{T(0), T(0)};
    reinterpret_cast<V*>(g)[i] = gin ? reinterpret_cast<const V*>(gin)[o] : V{T(1), T(1)};
}

__global__ __launch_bounds__(kBlock) void k_export_tree(const Node* __restrict__ nodes,
                                                        const double2* __restrict__ nsum,
                                                        const uint32_t* __restrict__ keys,
                                                        const DevScalars* __restrict__ sc, int L,
                                                        uint32_t* __restrict__ prefix,
                                                        uint32_t* __restrict__ count,
                                                        double* __restrict__ sum) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= sc->n_nodes) return;
    const Node nd = nodes[g];
    const int sh = L - (int)nd.level;
    if (prefix) prefix[g] = sh >= 16 ? 0u : (keys[nd.start] >> (2 * sh));
    if (count) count[g] = nd.count;
    if (sum) {
        sum[2 * g] = nsum[g].x;
        sum[2 * g + 1] = nsum[g].y;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cast_val(const double* __restrict__ a, T* __restrict__ b,
                                                     int64_t m) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < m) b[i] = (T)a[i];
}
// ---------------------------------------------------------------------------
// KL(P || Q) of Eq. (4) with the exact normaliser Z = sum over ordered pairs
// i != j of w_ij (O(n^2) pairs, FP32 terms summed in FP64 per 256-point tile)
// and sum_nnz p (ln p - ln w_ij) in FP64.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_kl_z(const T* __restrict__ zh,
                                                 const DevScalars* __restrict__ sc, int64_t n,
                                                 int r, double* __restrict__ part) {
    __shared__ float2 tile[kBlock];
    __shared__ double red[kBlock];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const double s0 = sc->s[0], s1 = sc->s[1];
    const float b1 = (float)(s0 * s0), b2 = (float)(s1 * s1);
    float2 zi = float2{0.f, 0.f};
    if (i < n) {
        const v2_t<T> p = norm_pos<T>(zh, sc, i, r);
        zi = float2{(float)p.x, (float)p.y};
    }
    double acc = 0.0;
    for (int64_t j0 = 0; j0 < n; j0 += kBlock) {
        __syncthreads();
        const int64_t j = j0 + threadIdx.x;
        if (j < n) {
            const v2_t<T> p = norm_pos<T>(zh, sc, j, r);
            tile[threadIdx.x] = float2{(float)p.x, (float)p.y};
        }
        __syncthreads();
        const int m = n - j0 < kBlock ? (int)(n - j0) : kBlock;
        float sacc = 0.f;
        for (int q = 0; q < m; q++) {
            const float dx = zi.x - tile[q].x, dy = zi.y - tile[q].y;
            const float w = __builtin_amdgcn_rcpf(1.0f + b1 * dx * dx + b2 * dy * dy);
            sacc += (j0 + q == i) ? 0.f : w;
        }
        if (i < n) acc += (double)sacc;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// per row: sum p ln p - p ln w_ij and sum p (one wavefront per row)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_kl_p(const int64_t* __restrict__ rp,
                                                 const uint32_t* __restrict__ col,
                                                 const T* __restrict__ val,
                                                 const uint32_t* __restrict__ inv,
                                                 const T* __restrict__ zh,
                                                 const DevScalars* __restrict__ sc, int64_t n,
                                                 int r, double* __restrict__ part) {
    __shared__ double red[4][2];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int64_t wave = (int64_t)blockIdx.x * 4 + w, nw = (int64_t)gridDim.x * 4;
    const double s0 = sc->s[0], s1 = sc->s[1];
    const double b1 = s0 * s0, b2 = s1 * s1;
    double a = 0.0, ps = 0.0;
    for (int64_t i = wave; i < n; i += nw) {
        const v2_t<T> zi = norm_pos<T>(zh, sc, inv[i], r);
        for (int64_t e = rp[i] + lane; e < rp[i + 1]; e += kWave) {
            const double p = (double)val[e];
            if (!(p > 0.0)) continue;
            const v2_t<T> zj = norm_pos<T>(zh, sc, inv[col[e]], r);
            const double dx = (double)zi.x - (double)zj.x, dy = (double)zi.y - (double)zj.y;
            const double w1 = 1.0 + b1 * dx * dx + b2 * dy * dy;     // 1 / w_ij
            a += p * log(p) + p * log(w1);
            ps += p;
        }
    }
    a = wave_sum(a);
    ps = wave_sum(ps);
    if (lane == 0) { red[w][0] = a; red[w][1] = ps; }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = ((red[0][0] + red[1][0]) + red[2][0]) + red[3][0];
        part[2 * blockIdx.x + 1] = ((red[0][1] + red[1][1]) + red[2][1]) + red[3][1];
    }
}

// The KL's three sums from the block partials, in a fixed order: Z over the
// nz partials of k_kl_z, then sum p (ln p - ln w) and sum p over the np pairs
// of k_kl_p.  Writes out[0..2] = {Z, sum p (ln p - ln w), sum p}.
__global__ __launch_bounds__(kBlock) void k_kl_final(const double* __restrict__ part, int64_t nz,
                                                     int64_t np, double* __restrict__ out) {
    __shared__ double red[3][kBlock];
    double z = 0.0, a = 0.0, ps = 0.0;
    for (int64_t i = threadIdx.x; i < nz; i += kBlock) z += part[i];
    for (int64_t i = threadIdx.x; i < np; i += kBlock) {
        a += part[nz + 2 * i];
        ps += part[nz + 2 * i + 1];
    }
    red[0][threadIdx.x] = z;
    red[1][threadIdx.x] = a;
    red[2][threadIdx.x] = ps;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int q = 0; q < 3; q++) red[q][threadIdx.x] += red[q][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < 3) out[threadIdx.x] = red[threadIdx.x][0];
}

inline dim3 grid_for(int64_t n) { return dim3((unsigned)ceil_div(n > 0 ? n : 1, kBlock)); }

inline int64_t attract_blocks(int64_t n) {
    int64_t b = ceil_div(n, kChunkRows / 2);
    return b < kAttractBlocksMax ? b : kAttractBlocksMax;
}

inline bool fp64(const pixelsne_ctx* c) { return c->prm.precision == PSNE_FP64; }

StepParams step_params(const pixelsne_ctx* c, double alpha) {
    StepParams p;
    p.exaggeration = c->prm.exaggeration;
    p.eta = c->prm.eta;
    p.mom0 = c->prm.mom0;
    p.mom1 = c->prm.mom1;
    p.min_gain = c->prm.min_gain;
    p.alpha_override = alpha;
    p.exag_iters = c->prm.exag_iters;
    p.mom_switch = c->prm.mom_switch;
    return p;
}

}  // namespace

int64_t attract_block_count(int64_t n) { return attract_blocks(n); }

hipError_t run_snap(pixelsne_ctx* c) {
    if (c->prm.tree == PSNE_TREE_DATA) return run_snap_dtree(c);
    if (fp64(c))
        k_snap<double><<<grid_for(c->n), kBlock, 0, c->stream>>>(
            (const double*)c->zh, (double*)c->z, c->tb.key[0], c->tb.idx[0], c->sc, c->n, c->r);
    else
        k_snap<float><<<grid_for(c->n), kBlock, 0, c->stream>>>(
            (const float*)c->zh, (float*)c->z, c->tb.key[0], c->tb.idx[0], c->sc, c->n, c->r);
    return hipGetLastError();
}

hipError_t run_sort(pixelsne_ctx* c) {
    if (c->prm.tree == PSNE_TREE_DATA) return run_sort_dtree(c);
    return run_sort_bits(c, 2 * c->L);
}

hipError_t run_rows_scan(uint32_t* a, int64_t rows, int64_t len, uint32_t* tot, hipStream_t s) {
    k_rows_scan<<<dim3((unsigned)rows), kBlock, 0, s>>>(a, len, tot);
    return hipGetLastError();
}

int64_t sort_blocks_for(int64_t n) { return ceil_div(n, kRsTile); }

hipError_t sort_pairs32(uint32_t* const key[2], uint32_t* const idx[2], int64_t n, int bits,
                        uint32_t* hist, uint32_t* dtot, hipStream_t s, int* sorted) {
    const int64_t nb = sort_blocks_for(n);
    const int passes = (bits + 7) / 8;
    int cur = 0;
    for (int p = 0; p < passes; p++) {
        const int shift = 8 * p;
        k_rs_hist<<<dim3((unsigned)nb), kBlock, 0, s>>>(key[cur], n, shift, hist, nb);
        k_rows_scan<<<256, kBlock, 0, s>>>(hist, nb, dtot);
        // the first pass generates the identity permutation itself
        k_rs_scatter<<<dim3((unsigned)nb), kBlock, 0, s>>>(
            key[cur], p == 0 ? nullptr : idx[cur], key[cur ^ 1], idx[cur ^ 1], n, shift, hist,
            dtot, nb);
        cur ^= 1;
    }
    *sorted = cur;
    return hipGetLastError();
}

hipError_t run_sort_bits(pixelsne_ctx* c, int bits) {
    TreeBufs& tb = c->tb;
    return sort_pairs32(tb.key, tb.idx, c->n, bits, tb.hist, tb.dtot, c->stream, &tb.sorted);
}

hipError_t run_tree(pixelsne_ctx* c) {
    if (c->prm.tree == PSNE_TREE_DATA) return run_tree_dtree(c);
    TreeBufs& tb = c->tb;
    const uint32_t* keys = tb.key[tb.sorted];
    const uint32_t* perm = tb.idx[tb.sorted];
    k_tree_count<<<dim3((unsigned)tb.tree_blocks), kBlock, 0, c->stream>>>(
        keys, c->n, c->L, tb.lvl_cnt, tb.tree_blocks);
    k_rows_scan<<<dim3((unsigned)(c->L + 1)), kBlock, 0, c->stream>>>(tb.lvl_cnt, tb.tree_blocks,
                                                                      tb.ltot);
    if (fp64(c)) {
        k_tree_nodes<double><<<dim3((unsigned)tb.tree_blocks), kBlock, 0, c->stream>>>(
            keys, c->n, c->L, tb.lvl_cnt, tb.tree_blocks, tb.ltot, c->sc, tb.first_child,
            tb.cell_start, tb.leaf_of, perm, (const double*)c->z, tb.nsum, (double*)tb.zs,
            tb.wfirst, tb.wlast);
        k_tree_leaves<double><<<grid_for(c->n), kBlock, 0, c->stream>>>(
            keys, c->n, c->L, c->prm.com_mode, c->sc, tb.cell_start, tb.nodes, tb.cells32,
            tb.nsum, tb.wfirst, tb.wlast);
    } else {
        k_tree_nodes<float><<<dim3((unsigned)tb.tree_blocks), kBlock, 0, c->stream>>>(
            keys, c->n, c->L, tb.lvl_cnt, tb.tree_blocks, tb.ltot, c->sc, tb.first_child,
            tb.cell_start, tb.leaf_of, perm, (const float*)c->z, tb.nsum, (float*)tb.zs,
            tb.wfirst, tb.wlast);
        k_tree_leaves<float><<<grid_for(c->n), kBlock, 0, c->stream>>>(
            keys, c->n, c->L, c->prm.com_mode, c->sc, tb.cell_start, tb.nodes, tb.cells32,
            tb.nsum, tb.wfirst, tb.wlast);
    }
    const int top = c->L - 1 < kTopLevel ? c->L - 1 : kTopLevel;
    for (int lbot = c->L - 1; lbot > top; lbot -= kGroupLevels) {
        const int ltop = lbot - (kGroupLevels - 1) > top ? lbot - (kGroupLevels - 1) : top + 1;
        // the top level holds at most min(4^ltop, n) cells; K of them per block
        const int64_t cap = ltop < 31 ? std::min((int64_t)1 << (2 * ltop), c->n) : c->n;
        const int64_t K = ceil_div(cap, kGroupBlocks);
        k_tree_group<<<dim3((unsigned)ceil_div(cap, K)), kBlock, 0, c->stream>>>(
            keys, ltop, lbot, c->L, c->prm.com_mode, (uint32_t)K, c->sc, tb.first_child,
            tb.cell_start, tb.nodes, tb.cells32, tb.nsum);
    }
    if (top >= 0)
        k_tree_top<<<1, kTopThreads, 0, c->stream>>>(keys, top, c->L, c->prm.com_mode, c->sc,
                                                     tb.first_child, tb.cell_start, tb.nodes,
                                                     tb.cells32, tb.nsum);
    return hipGetLastError();
}

template <typename T, bool COUNT, bool F32T>
void launch_traverse(pixelsne_ctx* c, double th2, uint32_t* visits, uint32_t* used, double* Zi) {
    TreeBufs& tb = c->tb;
    if (c->prm.tree == PSNE_TREE_DATA)
        k_traverse<T, COUNT, F32T, true><<<grid_for(c->n), kBlock, 0, c->stream>>>(
            tb.nodes, tb.cells32, tb.nsum, (const T*)tb.zs, tb.idx[tb.sorted], tb.leaf_of, c->sc,
            c->n, c->L, th2, c->prm.com_mode, (T*)c->R, c->zpart, c->orig, Zi, visits, used);
    else
        k_traverse<T, COUNT, F32T, false><<<grid_for(c->n), kBlock, 0, c->stream>>>(
            tb.nodes, tb.cells32, tb.nsum, (const T*)tb.zs, tb.idx[tb.sorted], tb.leaf_of, c->sc,
            c->n, c->L, th2, c->prm.com_mode, (T*)c->R, c->zpart, c->orig, Zi, visits, used);
}

hipError_t run_traverse(pixelsne_ctx* c, uint32_t* visits, uint32_t* used, double* Zi) {
    const double th2 = c->prm.theta * c->prm.theta;
    // per-point counters only when they are asked for
    const bool count = visits || used;
    const bool f32t = !fp64(c) && !c->prm.opening_fp64;
    if (fp64(c)) {
        if (count) launch_traverse<double, true, false>(c, th2, visits, used, Zi);
        else launch_traverse<double, false, false>(c, th2, visits, used, Zi);
    } else if (f32t) {
        if (count) launch_traverse<float, true, true>(c, th2, visits, used, Zi);
        else launch_traverse<float, false, true>(c, th2, visits, used, Zi);
    } else {
        if (count) launch_traverse<float, true, false>(c, th2, visits, used, Zi);
        else launch_traverse<float, false, false>(c, th2, visits, used, Zi);
    }
    return hipGetLastError();
}

hipError_t run_zsum(pixelsne_ctx* c) {
    k_zsum<<<1, kBlock, 0, c->stream>>>(c->zpart, ceil_div(c->n, kBlock), c->sc);
    return hipGetLastError();
}

// The gradient hook: A and B in the caller's order, on the context's stream
// (after the traversal).
hipError_t run_attract(pixelsne_ctx* c, double alpha, void* A, void* B) {
    const dim3 grid((unsigned)attract_blocks(c->n));
    if (fp64(c))
        k_attract<double, 1><<<grid, kBlock, 0, c->stream>>>(
            c->ch_row, c->rp_int, c->pk, (const double*)c->vch, (const double*)c->z,
            (const double*)c->R, c->sc, alpha, c->orig, (double*)A, (double*)B, 0);
    else
        k_attract<float, 1><<<grid, kBlock, 0, c->stream>>>(
            c->ch_row, c->rp_int, c->pk, (const float*)c->vch, (const float*)c->z,
            (const float*)c->R, c->sc, alpha, c->orig, (float*)A, (float*)B, 0);
    return hipGetLastError();
}

// The iteration's attraction row sums into c->A: MODE 0 on the second
// stream (launched right after the snap pass, EARLY, and again after the
// cells), or (HELP) the MODE 2 helper on the main stream, all taking chunks
// from the same queue.
template <int MODE>
static hipError_t launch_attract_sums(pixelsne_ctx* c, const dim3 grid, hipStream_t s,
                                      int early) {
    if (fp64(c))
        k_attract<double, MODE><<<grid, kBlock, 0, s>>>(
            c->ch_row, c->rp_int, c->pk, (const double*)c->vch, (const double*)c->z, nullptr,
            c->sc, 0.0, c->orig, (double*)c->A, nullptr, early);
    else
        k_attract<float, MODE><<<grid, kBlock, 0, s>>>(
            c->ch_row, c->rp_int, c->pk, (const float*)c->vch, (const float*)c->z, nullptr,
            c->sc, 0.0, c->orig, (float*)c->A, nullptr, early);
    return hipGetLastError();
}

static hipError_t run_attract_sums(pixelsne_ctx* c, bool help, bool early = false) {
    const int64_t blocks = help ? c->help_blocks : c->side_blocks;
    // the early launch always runs: it stamps the tuner's clock
    if (early && blocks == 0) return launch_attract_sums<0>(c, dim3(1), c->side, 2);
    if (blocks == 0) return hipSuccess;
    if (help) return launch_attract_sums<2>(c, dim3((unsigned)blocks), c->stream, 0);
    return launch_attract_sums<0>(c, dim3((unsigned)blocks), c->side, early ? 1 : 0);
}

static hipError_t run_update(pixelsne_ctx* c) {
    const StepParams p = step_params(c, 0.0);
    const dim3 grid((unsigned)attract_blocks(c->n));
    if (fp64(c))
        k_update<double><<<grid, kBlock, 0, c->stream>>>(
            (const double*)c->A, (const double*)c->z, (const double*)c->R, (double*)c->u,
            (double*)c->g, (double*)c->zh, c->sc, p, c->n, c->mm_part);
    else
        k_update<float><<<grid, kBlock, 0, c->stream>>>(
            (const float*)c->A, (const float*)c->z, (const float*)c->R, (float*)c->u,
            (float*)c->g, (float*)c->zh, c->sc, p, c->n, c->mm_part);
    return hipGetLastError();
}

hipError_t run_finalize(pixelsne_ctx* c, int advance) {
    k_finalize<<<1, kBlock, 0, c->stream>>>(c->mm_part, attract_blocks(c->n), c->sc, c->r,
                                            c->prm.eps, advance, c->prm.attract_fork);
    return hipGetLastError();
}

// One iteration.  The attraction's row sums need only the snapped positions
// and P: the second stream takes them up either after the snap pass (beside
// the sort, the tree, the walk and Z) or after the tree (beside the walk and
// Z only), as DevScalars::fork_late says; both points are in every
// iteration's launch sequence, and the launch at the point not chosen leaves
// at once (the early one) or finds the queue empty (the late one).  The
// helper on this stream takes what is left after Z, and the update joins.
// EV, when given, receives the pass boundaries: [0..5] before snap, sort,
// tree, traverse, Z and after Z on this stream, [6] after the join, [7] after
// update and scaling, [8] after a scheduled renumbering, [9] and [10] around
// the second stream's launch after the snap pass, [11] and [12] around its
// launch after the cells.
static hipError_t iteration(pixelsne_ctx* c, hipEvent_t* ev) {
    hipError_t e;
    auto mark = [&](int k, hipStream_t s) {
        return ev ? hipEventRecord(ev[k], s) : hipSuccess;
    };
    auto join_at = [&](hipEvent_t at) {
        hipError_t f;
        if ((f = hipEventRecord(at, c->stream)) != hipSuccess) return f;
        return hipStreamWaitEvent(c->side, at, 0);
    };
    if ((e = mark(0, c->stream)) != hipSuccess) return e;
    if ((e = run_snap(c)) != hipSuccess) return e;
    if ((e = mark(1, c->stream)) != hipSuccess) return e;
    if ((e = join_at(c->ev_fork)) != hipSuccess) return e;
    if ((e = mark(9, c->side)) != hipSuccess) return e;
    if ((e = run_attract_sums(c, false, true)) != hipSuccess) return e;
    if ((e = mark(10, c->side)) != hipSuccess) return e;
    if ((e = run_sort(c)) != hipSuccess) return e;
    if ((e = mark(2, c->stream)) != hipSuccess) return e;
    if ((e = run_tree(c)) != hipSuccess) return e;
    if ((e = mark(3, c->stream)) != hipSuccess) return e;
    if ((e = join_at(c->ev_cells)) != hipSuccess) return e;
    if ((e = mark(11, c->side)) != hipSuccess) return e;
    if ((e = run_attract_sums(c, false)) != hipSuccess) return e;
    if ((e = mark(12, c->side)) != hipSuccess) return e;
    if ((e = hipEventRecord(c->ev_join, c->side)) != hipSuccess) return e;
    if ((e = run_traverse(c, nullptr, nullptr, nullptr)) != hipSuccess) return e;
    if ((e = mark(4, c->stream)) != hipSuccess) return e;
    if ((e = run_zsum(c)) != hipSuccess) return e;
    if ((e = mark(5, c->stream)) != hipSuccess) return e;
    if ((e = run_attract_sums(c, true)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(c->stream, c->ev_join, 0)) != hipSuccess) return e;
    if ((e = mark(6, c->stream)) != hipSuccess) return e;
    if ((e = run_update(c)) != hipSuccess) return e;
    if ((e = run_finalize(c, 1)) != hipSuccess) return e;
    if (!ev) return hipSuccess;
    if ((e = mark(7, c->stream)) != hipSuccess) return e;
    if ((e = run_scheduled_reorder(c)) != hipSuccess) return e;
    return mark(8, c->stream);
}

hipError_t run_iteration_passes(pixelsne_ctx* c) { return iteration(c, nullptr); }

hipError_t run_iteration_timed(pixelsne_ctx* c, hipEvent_t* ev) { return iteration(c, ev); }

hipError_t run_init_state(pixelsne_ctx* c, const double* Y, uint64_t seed, double sigma) {
    DevScalars h{};
    h.s[0] = h.s[1] = 1.0;            // the initial frame is y itself
    h.scale[0] = h.scale[1] = 1.0;
    h.uscale[0] = h.uscale[1] = 1.0;
    reset_fork_tuner(h, c->prm.attract_fork);
    hipError_t e = hipMemcpyAsync(c->sc, &h, sizeof(h), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return e;
    const int64_t nb = attract_blocks(c->n);
    if (fp64(c)) {
        k_init_state<double><<<grid_for(c->n), kBlock, 0, c->stream>>>(
            Y, (double*)c->zh, (double*)c->u, (double*)c->g, c->n, seed, sigma);
        k_minmax<double><<<dim3((unsigned)nb), kBlock, 0, c->stream>>>((const double*)c->zh, c->n,
                                                                         c->mm_part);
    } else {
        k_init_state<float><<<grid_for(c->n), kBlock, 0, c->stream>>>(
            Y, (float*)c->zh, (float*)c->u, (float*)c->g, c->n, seed, sigma);
        k_minmax<float><<<dim3((unsigned)nb), kBlock, 0, c->stream>>>((const float*)c->zh, c->n,
                                                                        c->mm_part);
    }
    return run_finalize(c, 0);
}

hipError_t run_get_y(const pixelsne_ctx* c, void* out, int frame) {
    if (fp64(c))
        k_get_y<double><<<grid_for(c->n), kBlock, 0, c->stream>>>((const double*)c->zh, c->sc,
                                                                   c->orig, c->n, c->r, frame, out);
    else
        k_get_y<float><<<grid_for(c->n), kBlock, 0, c->stream>>>((const float*)c->zh, c->sc,
                                                                  c->orig, c->n, c->r, frame, out);
    return hipGetLastError();
}

hipError_t run_set_state(pixelsne_ctx* c, const void* z, const void* u, const void* g) {
    if (fp64(c))
        k_set_state<double><<<grid_for(c->n), kBlock, 0, c->stream>>>(
            (const double*)z, (const double*)u, (const double*)g, c->orig, c->n, (double*)c->zh,
            (double*)c->u, (double*)c->g);
    else
        k_set_state<float><<<grid_for(c->n), kBlock, 0, c->stream>>>(
            (const float*)z, (const float*)u, (const float*)g, c->orig, c->n, (float*)c->zh,
            (float*)c->u, (float*)c->g);
    return hipGetLastError();
}

hipError_t run_get_state(const pixelsne_ctx* c, void* z, void* u, void* g) {
    if (fp64(c))
        k_get_state<double><<<grid_for(c->n), kBlock, 0, c->stream>>>(
            (const double*)c->zh, (const double*)c->u, (const double*)c->g, c->sc, c->orig, c->n,
            c->r, (double*)z, (double*)u, (double*)g);
    else
        k_get_state<float><<<grid_for(c->n), kBlock, 0, c->stream>>>(
            (const float*)c->zh, (const float*)c->u, (const float*)c->g, c->sc, c->orig, c->n,
            c->r, (float*)z, (float*)u, (float*)g);
    return hipGetLastError();
}

hipError_t run_export_tree(const pixelsne_ctx* c, uint32_t* keys, uint32_t* perm, uint32_t* prefix,
                           uint32_t* count, double* sum) {
    const TreeBufs& tb = c->tb;
    hipError_t e = hipSuccess;
    if (keys)
        e = hipMemcpyAsync(keys, tb.key[tb.sorted], (size_t)c->n * 4, hipMemcpyDeviceToDevice,
                           c->stream);
    if (e == hipSuccess && perm) e = run_map_perm(c, tb.idx[tb.sorted], perm);
    if (e != hipSuccess) return e;
    if (prefix || count || sum)
        k_export_tree<<<grid_for(tb.max_nodes), kBlock, 0, c->stream>>>(
            tb.nodes, tb.nsum, tb.key[tb.sorted], c->sc, c->L, prefix, count, sum);
    return hipGetLastError();
}

// Blocks of the KL's two passes: one per 256 rows for the pair sums, at most
// 4,096 (one wavefront per row, grid-stride) for the sums over P.
static int64_t kl_blocks_z(int64_t n) { return ceil_div(n, kBlock); }
static int64_t kl_blocks_p(int64_t n) { return n / 4 < 4096 ? (n + 3) / 4 : 4096; }

int64_t kl_scratch_doubles(int64_t n) { return kl_blocks_z(n) + 2 * kl_blocks_p(n) + 3; }

// The KL passes with their partial sums in `part` (kl_scratch_doubles(n)
// doubles of device memory); synchronises the context's stream.
static hipError_t run_kl_with(const pixelsne_ctx* c, double* part, double* kl) {
    const int64_t nbz = kl_blocks_z(c->n), nbp = kl_blocks_p(c->n);
    if (fp64(c)) {
        k_kl_z<double><<<dim3((unsigned)nbz), kBlock, 0, c->stream>>>((const double*)c->zh, c->sc,
                                                                     c->n, c->r, part);
        k_kl_p<double><<<dim3((unsigned)nbp), kBlock, 0, c->stream>>>(
            c->row_ptr, c->col, (const double*)c->val, c->inv, (const double*)c->zh, c->sc, c->n, c->r,
            part + nbz);
    } else {
        k_kl_z<float><<<dim3((unsigned)nbz), kBlock, 0, c->stream>>>((const float*)c->zh, c->sc,
                                                                    c->n, c->r, part);
        k_kl_p<float><<<dim3((unsigned)nbp), kBlock, 0, c->stream>>>(
            c->row_ptr, c->col, (const float*)c->val, c->inv, (const float*)c->zh, c->sc, c->n, c->r,
            part + nbz);
    }
    k_kl_final<<<1, kBlock, 0, c->stream>>>(part, nbz, nbp, part + nbz + 2 * nbp);
    double h[3] = {0.0, 0.0, 0.0};
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(h, part + nbz + 2 * nbp, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return e;
    *kl = h[1] + h[2] * log(h[0]);
    return hipSuccess;
}

hipError_t run_kl(const pixelsne_ctx* c, double* kl) {
    double* part = nullptr;
    hipError_t e = hipMalloc((void**)&part, 8 * (size_t)kl_scratch_doubles(c->n));
    if (e != hipSuccess) return e;
    e = run_kl_with(c, part, kl);
    (void)hipFree(part);
    return e;
}

// ---------------------------------------------------------------------------
// The KL without device allocation: its partial sums live in a fixed array
// of the library, one copy per device, held until the process ends.  Host
// code must never pass the array's name to a kernel or a copy (on the host
// it is only a stand-in for the symbol): kl_scratch_address() resolves the
// device address once per device and every use goes through it.  Calls that
// overlap on one device share the array and race.
// ---------------------------------------------------------------------------
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kKlScratchDoubles];
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

hipError_t kl_scratch_address(int device, double** out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;   // resolve with the device current
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = (double*)p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

hipError_t run_kl_static(const pixelsne_ctx* c, double* kl) {
    if (kl_scratch_doubles(c->n) > kKlScratchDoubles) return hipErrorInvalidValue;
    double* part = nullptr;
    hipError_t e = kl_scratch_address(c->device, &part);
    if (e != hipSuccess) return e;
    return run_kl_with(c, part, kl);
}

hipError_t run_convert_val(pixelsne_ctx* c, const double* val64) {
    if (fp64(c))
        return hipMemcpyAsync(c->val, val64, (size_t)c->nnz * 8, hipMemcpyDeviceToDevice,
                              c->stream);
    k_cast_val<float><<<grid_for(c->nnz), kBlock, 0, c->stream>>>(val64, (float*)c->val, c->nnz);
    return hipGetLastError();
}

}  // namespace psne
