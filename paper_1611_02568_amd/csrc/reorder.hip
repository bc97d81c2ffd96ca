// Internal renumbering of the points and conversions to the caller's order.
//
// The sparse attraction gathers z_j for every nonzero of row i.  When points
// are numbered arbitrarily these gathers touch random cache lines of an
// array larger than one XCD's L2.  Every few iterations the library therefore
// renumbers the points by the Morton order of the last sort: P's rows and
// columns and the per-point state are permuted on the device, so that rows
// processed together and their neighbours occupy nearby memory.  The method's
// arithmetic is unchanged; only the order of the per-row summands changes.
#include "ctx.h"

namespace psne {

namespace {

constexpr int kBlock = 256;

inline dim3 grid_for(int64_t n) { return dim3((unsigned)ceil_div(n > 0 ? n : 1, kBlock)); }
inline bool fp64(const pixelsne_ctx* c) { return c->prm.precision == PSNE_FP64; }

// new index of old point perm[s] is s
__global__ __launch_bounds__(kBlock) void k_reorder_index(const uint32_t* __restrict__ perm,
                                                          const uint32_t* __restrict__ orig,
                                                          const int64_t* __restrict__ rp,
                                                          int64_t n, uint32_t* __restrict__ inv,
                                                          uint32_t* __restrict__ orig2,
                                                          int64_t* __restrict__ len2) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s < n) {
        const uint32_t i = perm[s];
        inv[i] = (uint32_t)s;
        orig2[s] = orig[i];
        len2[s] = rp[i + 1] - rp[i];
    } else if (s == n) {
        len2[n] = 0;
    }
}

constexpr int kSortMax = 512;   // rows up to this length get their columns sorted

// One wavefront per new row: the old row's columns are renumbered and, for
// rows of at most kSortMax entries, sorted ascending (bitonic sort of
// (column, position) keys in LDS), so that the attraction's gathers walk
// memory in order.  Longer rows are copied in their old order.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_reorder_csr(
    const int64_t* __restrict__ rp, const uint32_t* __restrict__ col, const T* __restrict__ val,
    const uint32_t* __restrict__ perm, const uint32_t* __restrict__ inv,
    const int64_t* __restrict__ rp2, uint32_t* __restrict__ col2, T* __restrict__ val2,
    int64_t n) {
    __shared__ uint64_t sk[kBlock / kWave][kSortMax];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    uint64_t* key = sk[w];
    const int64_t wave = (int64_t)blockIdx.x * (kBlock / kWave) + w;
    const int64_t nw = (int64_t)gridDim.x * (kBlock / kWave);
    for (int64_t s = wave; s < n; s += nw) {
        const uint32_t i = perm[s];
        const int64_t b = rp[i], m = rp[i + 1] - b, o = rp2[s];
        if (m > kSortMax) {
            for (int64_t e = lane; e < m; e += kWave) {
                col2[o + e] = inv[col[b + e]];
                val2[o + e] = val[b + e];
            }
            continue;
        }
        int P = kWave;
        while (P < m) P <<= 1;
        for (int e = lane; e < P; e += kWave)
            key[e] = e < m ? (((uint64_t)inv[col[b + e]] << 32) | (uint32_t)e) : ~0ull;
        __builtin_amdgcn_wave_barrier();
        for (int k = 2; k <= P; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int t = lane; t < P / 2; t += kWave) {
                    const int a = ((t & ~(j - 1)) << 1) | (t & (j - 1));
                    const int c = a | j;
                    const uint64_t x = key[a], y = key[c];
                    const bool up = (a & k) == 0;
                    if ((x > y) == up) {
                        key[a] = y;
                        key[c] = x;
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        for (int e = lane; e < m; e += kWave) {
            const uint64_t kk = key[e];
            col2[o + e] = (uint32_t)(kk >> 32);
            val2[o + e] = val[b + (uint32_t)kk];
        }
        __builtin_amdgcn_wave_barrier();
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_reorder_state(const uint32_t* __restrict__ perm,
                                                          const T* __restrict__ a0,
                                                          const T* __restrict__ a1,
                                                          const T* __restrict__ a2,
                                                          T* __restrict__ b0, T* __restrict__ b1,
                                                          T* __restrict__ b2, int64_t n) {
    using V = v2_t<T>;
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    const uint32_t i = perm[s];
    reinterpret_cast<V*>(b0)[s] = reinterpret_cast<const V*>(a0)[i];
    reinterpret_cast<V*>(b1)[s] = reinterpret_cast<const V*>(a1)[i];
    reinterpret_cast<V*>(b2)[s] = reinterpret_cast<const V*>(a2)[i];
}

__global__ __launch_bounds__(kBlock) void k_iota(uint32_t* __restrict__ a, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) a[i] = (uint32_t)i;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_to_user_v2(const T* __restrict__ in,
                                                       const uint32_t* __restrict__ orig,
                                                       int64_t n, T* __restrict__ out) {
    using V = v2_t<T>;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) reinterpret_cast<V*>(out)[orig[i]] = reinterpret_cast<const V*>(in)[i];
}

__global__ __launch_bounds__(kBlock) void k_map_perm(const uint32_t* __restrict__ perm,
                                                     const uint32_t* __restrict__ orig, int64_t n,
                                                     uint32_t* __restrict__ out) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s < n) out[s] = orig[perm[s]];
}

// caller row u = internal row inv[u] (inv = inverse of orig)
__global__ __launch_bounds__(kBlock) void k_user_index(const uint32_t* __restrict__ orig,
                                                       const int64_t* __restrict__ rp, int64_t n,
                                                       uint32_t* __restrict__ inv,
                                                       int64_t* __restrict__ len) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        const uint32_t u = orig[i];
        inv[u] = (uint32_t)i;
        len[u] = rp[i + 1] - rp[i];
    } else if (i == n) {
        len[n] = 0;
    }
}

constexpr int kRowLds = 4096;

// One block per caller row: columns renumbered to the caller's indices and
// sorted ascending (rank by counting; rows longer than kRowLds rank from
// global memory), values widened to FP64.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_csr_to_user(
    const int64_t* __restrict__ rp, const uint32_t* __restrict__ col, const T* __restrict__ val,
    const uint32_t* __restrict__ orig, const uint32_t* __restrict__ inv,
    const int64_t* __restrict__ rpu, int32_t* __restrict__ colu, double* __restrict__ valu) {
    __shared__ uint32_t c_in[kRowLds];
    const int64_t u = blockIdx.x;
    const uint32_t i = inv[u];
    const int64_t b = rp[i], m = rp[i + 1] - b, o = rpu[u];
    const bool lds = m <= kRowLds;
    if (lds)
        for (int64_t e = threadIdx.x; e < m; e += kBlock) c_in[e] = orig[col[b + e]];
    __syncthreads();
    for (int64_t e = threadIdx.x; e < m; e += kBlock) {
        const uint32_t ce = lds ? c_in[e] : orig[col[b + e]];
        int64_t r = 0;
        for (int64_t f = 0; f < m; f++) {
            const uint32_t cf = lds ? c_in[f] : orig[col[b + f]];
            r += (cf < ce || (cf == ce && f < e)) ? 1 : 0;
        }
        colu[o + r] = (int32_t)ce;
        valu[o + r] = (double)val[b + e];
    }
}

}  // namespace

hipError_t run_identity_order(pixelsne_ctx* c) {
    k_iota<<<grid_for(c->n), kBlock, 0, c->stream>>>(c->orig, c->n);
    c->since_reorder = 0;
    return hipGetLastError();
}

hipError_t run_reorder(pixelsne_ctx* c) {
    const TreeBufs& tb = c->tb;
    const uint32_t* perm = tb.idx[tb.sorted];
    hipError_t e;
    k_reorder_index<<<grid_for(c->n + 1), kBlock, 0, c->stream>>>(perm, c->orig, c->row_ptr, c->n,
                                                                  c->inv, c->orig2, c->len_tmp);
    if ((e = scan_i64(c->len_tmp, c->n + 1, c->row_ptr2, c->scan_tmp, c->stream)) != hipSuccess)
        return e;
    const int64_t waves = c->n < 32768 ? c->n : 32768;
    const dim3 g((unsigned)ceil_div(waves, kBlock / kWave));
    if (fp64(c)) {
        k_reorder_csr<double><<<g, kBlock, 0, c->stream>>>(
            c->row_ptr, c->col, (const double*)c->val, perm, c->inv, c->row_ptr2, c->col2,
            (double*)c->val2, c->n);
        k_reorder_state<double><<<grid_for(c->n), kBlock, 0, c->stream>>>(
            perm, (const double*)c->zh, (const double*)c->u, (const double*)c->g,
            (double*)c->zh2, (double*)c->u2, (double*)c->g2, c->n);
    } else {
        k_reorder_csr<float><<<g, kBlock, 0, c->stream>>>(
            c->row_ptr, c->col, (const float*)c->val, perm, c->inv, c->row_ptr2, c->col2,
            (float*)c->val2, c->n);
        k_reorder_state<float><<<grid_for(c->n), kBlock, 0, c->stream>>>(
            perm, (const float*)c->zh, (const float*)c->u, (const float*)c->g, (float*)c->zh2,
            (float*)c->u2, (float*)c->g2, c->n);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    std::swap(c->row_ptr, c->row_ptr2);
    std::swap(c->col, c->col2);
    std::swap(c->val, c->val2);
    std::swap(c->zh, c->zh2);
    std::swap(c->u, c->u2);
    std::swap(c->g, c->g2);
    std::swap(c->orig, c->orig2);
    c->since_reorder = 0;
    return hipSuccess;
}

hipError_t run_export_P(const pixelsne_ctx* c, int64_t* row_ptr, int32_t* col, double* val) {
    int64_t* rp = row_ptr ? row_ptr : c->row_ptr2;
    k_user_index<<<grid_for(c->n + 1), kBlock, 0, c->stream>>>(c->orig, c->row_ptr, c->n, c->inv,
                                                               c->len_tmp);
    hipError_t e = scan_i64(c->len_tmp, c->n + 1, rp, c->scan_tmp, c->stream);
    if (e != hipSuccess || (!col && !val)) return e;
    int32_t* cu = col ? col : (int32_t*)c->col2;
    double* vu = val;
    double* vtmp = nullptr;
    if (!vu) {
        if ((e = hipMallocAsync((void**)&vtmp, 8 * (size_t)c->nnz, c->stream)) != hipSuccess) return e;
        vu = vtmp;
    }
    if (fp64(c))
        k_csr_to_user<double><<<dim3((unsigned)c->n), kBlock, 0, c->stream>>>(
            c->row_ptr, c->col, (const double*)c->val, c->orig, c->inv, rp, cu, vu);
    else
        k_csr_to_user<float><<<dim3((unsigned)c->n), kBlock, 0, c->stream>>>(
            c->row_ptr, c->col, (const float*)c->val, c->orig, c->inv, rp, cu, vu);
    e = hipGetLastError();
    if (vtmp) (void)hipFreeAsync(vtmp, c->stream);
    return e;
}

hipError_t run_to_user_v2(const pixelsne_ctx* c, const void* in, void* out) {
    if (fp64(c))
        k_to_user_v2<double><<<grid_for(c->n), kBlock, 0, c->stream>>>((const double*)in, c->orig,
                                                                        c->n, (double*)out);
    else
        k_to_user_v2<float><<<grid_for(c->n), kBlock, 0, c->stream>>>((const float*)in, c->orig,
                                                                       c->n, (float*)out);
    return hipGetLastError();
}

hipError_t run_map_perm(const pixelsne_ctx* c, const uint32_t* perm, uint32_t* out) {
    k_map_perm<<<grid_for(c->n), kBlock, 0, c->stream>>>(perm, c->orig, c->n, out);
    return hipGetLastError();
}

}  // namespace psne
