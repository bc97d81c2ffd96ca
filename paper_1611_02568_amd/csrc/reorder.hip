// Internal renumbering of the points and the attraction pass's copy of P.
//
// The sparse attraction gathers z_j for every nonzero of row i.  When points
// are numbered arbitrarily these gathers touch random cache lines of an
// array larger than one XCD's L2.  The library therefore renumbers the points
// by the Morton order of a recent sort (after the first iteration or the early
// exaggeration, then after intervals of params.reorder_every iterations that
// grow by params.reorder_growth): the per-point state is permuted, and P,
// kept in the caller's numbering, is copied into the attraction's layout for
// the new numbering.  That layout cuts the internal rows into chunks of up to
// kChunkRows consecutive rows and orders each chunk's nonzeros by column, so
// that the 64 gathers of one wavefront instruction fall on few cache lines;
// each run of 64 is then ordered by row, which lets the attraction kernel sum
// a row's terms with a segmented scan across the wave.  The method's
// arithmetic is unchanged; only the order of the per-row summands changes.
#include <cmath>

#include "ctx.h"

namespace psne {

namespace {

constexpr int kBlock = 256;
constexpr int64_t kChunkHalf = kChunkMaxNnz / 2;
constexpr int kBuildBlocksMax = 4096;

inline dim3 grid_for(int64_t n) { return dim3((unsigned)ceil_div(n > 0 ? n : 1, kBlock)); }
inline bool fp64(const pixelsne_ctx* c) { return c->prm.precision == PSNE_FP64; }

// new internal index of old internal point perm[s] is s
__global__ __launch_bounds__(kBlock) void k_reorder_index(const uint32_t* __restrict__ perm,
                                                          const uint32_t* __restrict__ orig,
                                                          int64_t n, uint32_t* __restrict__ inv,
                                                          uint32_t* __restrict__ orig2) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s < n) {
        const uint32_t u = orig[perm[s]];
        orig2[s] = u;
        inv[u] = (uint32_t)s;
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

__global__ __launch_bounds__(kBlock) void k_iota2(uint32_t* __restrict__ a, uint32_t* __restrict__ b,
                                                  int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        a[i] = (uint32_t)i;
        b[i] = (uint32_t)i;
    }
}

// row lengths in internal order (entry n is 0, so that an exclusive scan of
// n + 1 entries gives the offsets and the total)
__global__ __launch_bounds__(kBlock) void k_int_len(const uint32_t* __restrict__ orig,
                                                    const int64_t* __restrict__ rp, int64_t n,
                                                    int64_t* __restrict__ len) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s < n) {
        const uint32_t u = orig[s];
        len[s] = rp[u + 1] - rp[u];
    } else if (s == n) {
        len[n] = 0;
    }
}

// Chunks are the groups of kChunkRows consecutive rows.  A group with
// kChunkMaxNnz nonzeros or more is cut further: a chunk starts where the row
// offset (from the group's start) enters a new window of kChunkHalf nonzeros,
// and around every row longer than kChunkHalf.  So a chunk of several rows
// holds fewer than kChunkMaxNnz nonzeros (one window plus one row of at most
// kChunkHalf).  Full groups keep the attraction's per-chunk work (prologue,
// barriers, the last partly filled batch) small against its streaming.
__device__ __forceinline__ bool chunk_start(const int64_t* __restrict__ rp, int64_t n, int64_t s) {
    if (s % kChunkRows == 0) return true;
    const int64_t g0 = s - s % kChunkRows, g1 = g0 + kChunkRows < n ? g0 + kChunkRows : n;
    const int64_t base = rp[g0];
    if (rp[g1] - base < kChunkMaxNnz) return false;
    const int64_t a = rp[s - 1] - base, b = rp[s] - base, c = rp[s + 1] - base;
    return (a / kChunkHalf) != (b / kChunkHalf) || c - b > kChunkHalf || b - a > kChunkHalf;
}

__global__ __launch_bounds__(kBlock) void k_chunk_flags(const int64_t* __restrict__ rp, int64_t n,
                                                        int64_t* __restrict__ flag) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s < n) flag[s] = chunk_start(rp, n, s) ? 1 : 0;
    else if (s == n) flag[n] = 0;
}

__global__ __launch_bounds__(kBlock) void k_chunk_rows(const int64_t* __restrict__ rp, int64_t n,
                                                       const int64_t* __restrict__ cid,
                                                       uint32_t* __restrict__ ch_row,
                                                       DevScalars* __restrict__ sc) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s < n) {
        if (chunk_start(rp, n, s)) ch_row[cid[s]] = (uint32_t)s;
    } else if (s == n) {
        ch_row[cid[n]] = (uint32_t)n;
        sc->n_chunks = cid[n];
    }
}

constexpr int kBuildThreads = 1024;

// One block per chunk (grid-stride).  A chunk of one row is copied as it is.
// For several rows (fewer than kChunkMaxNnz nonzeros), the keys
// column << 5 | row (unique: a row holds a column once) are sorted in LDS
// (bitonic), then every aligned run of 64 is sorted again by (row, column).
// A value is found in its caller row by binary search for the caller's column
// (rows of the caller's P are ascending).
// One nonzero of the chunked copy.  FP32: the column word and the value side
// by side in pk ([nnz][2] words, one 64-bit load in the attraction); FP64:
// column words in pk, values in vch.
__device__ __forceinline__ void put_nz(uint32_t* __restrict__ pk, float* __restrict__,
                                       int64_t e, uint32_t key, float v) {
    reinterpret_cast<uint2*>(pk)[e] = uint2{key, __float_as_uint(v)};
}
__device__ __forceinline__ void put_nz(uint32_t* __restrict__ pk, double* __restrict__ vch,
                                       int64_t e, uint32_t key, double v) {
    pk[e] = key;
    vch[e] = v;
}

template <typename T>
__global__ __launch_bounds__(kBuildThreads) void k_chunk_build(
    const int64_t* __restrict__ rp_c, const uint32_t* __restrict__ col_c,
    const T* __restrict__ val_c, const uint32_t* __restrict__ orig,
    const uint32_t* __restrict__ inv, const int64_t* __restrict__ rp_int,
    const uint32_t* __restrict__ ch_row, const DevScalars* __restrict__ sc,
    uint32_t* __restrict__ pk, T* __restrict__ vch) {
    __shared__ uint32_t key[kChunkMaxNnz];
    __shared__ int64_t off[kChunkRows + 1];
    __shared__ int64_t src[kChunkRows];
    constexpr uint32_t kColMask = (1u << kColBits) - 1u;
    const int t = threadIdx.x;
    const int64_t nch = sc->n_chunks;
    for (int64_t ch = blockIdx.x; ch < nch; ch += gridDim.x) {
        const int64_t ra = ch_row[ch], nr = (int64_t)ch_row[ch + 1] - ra;
        const int64_t e0 = rp_int[ra], m = rp_int[ra + nr] - e0;
        if (nr == 1 || m >= kChunkMaxNnz) {
            // one row (any length), or a chunk the sort cannot hold (not made by
            // the chunking rule): rows in order, each run of 64 is then ordered by row
            for (int64_t lr = 0; lr < nr; lr++) {
                const int64_t s0 = rp_c[orig[ra + lr]], o = rp_int[ra + lr];
                const int64_t len = rp_int[ra + lr + 1] - o;
                for (int64_t e = t; e < len; e += kBuildThreads)
                    put_nz(pk, vch, o + e, inv[col_c[s0 + e]] | ((uint32_t)lr << kColBits),
                           val_c[s0 + e]);
            }
            continue;
        }
        if (t <= nr) off[t] = rp_int[ra + t] - e0;
        if (t < nr) src[t] = rp_c[orig[ra + t]];
        __syncthreads();
        int P = 64;
        while (P < m) P <<= 1;
        for (int e = t; e < P; e += kBuildThreads) {
            uint32_t k = ~0u;
            if (e < m) {
                int lo = 0, hi = (int)nr;            // off[lo] <= e < off[hi]
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (off[mid] <= e) lo = mid;
                    else hi = mid;
                }
                k = (inv[col_c[src[lo] + (e - off[lo])]] << 5) | (uint32_t)lo;
            }
            key[e] = k;
        }
        __syncthreads();
        for (int k = 2; k <= P; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int q = t; q < P / 2; q += kBuildThreads) {
                    const int a = ((q & ~(j - 1)) << 1) | (q & (j - 1));
                    const int b = a | j;
                    const uint32_t x = key[a], y = key[b];
                    if ((x > y) == ((a & k) == 0)) {
                        key[a] = y;
                        key[b] = x;
                    }
                }
                __syncthreads();
            }
        }
        // re-key to row << 27 | column and order each run of 64
        for (int p = t; p < m; p += kBuildThreads) {
            const uint32_t k = key[p];
            key[p] = ((k & 31u) << kColBits) | (k >> 5);
        }
        __syncthreads();
        for (int k = 2; k <= 64; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int q = t; q < P / 2; q += kBuildThreads) {
                    const int a = ((q & ~(j - 1)) << 1) | (q & (j - 1));
                    const int b = a | j;
                    const uint32_t x = key[a], y = key[b];
                    const bool up = k == 64 || (a & k) == 0;
                    if ((x > y) == up) {
                        key[a] = y;
                        key[b] = x;
                    }
                }
                __syncthreads();
            }
        }
        for (int p = t; p < m; p += kBuildThreads) {
            const uint32_t k = key[p];
            const uint32_t lr = k >> kColBits, cn = k & kColMask;
            const uint32_t cu = orig[cn];
            int64_t lo = src[lr], hi = src[lr] + (off[lr + 1] - off[lr]);   // col_c[pos] == cu
            while (hi - lo > 1) {
                const int64_t mid = (lo + hi) >> 1;
                if (col_c[mid] <= cu) lo = mid;
                else hi = mid;
            }
            put_nz(pk, vch, e0 + p, k, val_c[lo]);         // column | row << 27
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_check_csr(const int64_t* __restrict__ rp,
                                                      const uint32_t* __restrict__ col, int64_t n,
                                                      int64_t nnz,
                                                      unsigned long long* __restrict__ bad) {
    unsigned long long b = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const int64_t a = rp[i], e = rp[i + 1];
        if (i == 0 && a != 0) b++;
        if (i == n - 1 && e != nnz) b++;
        if (e < a || a < 0 || e > nnz) { b++; continue; }
        for (int64_t q = a; q < e; q++) {
            const uint32_t j = col[q];
            if (j >= (uint64_t)n || j == (uint64_t)i || (q > a && j <= col[q - 1])) b++;
        }
    }
    if (b) atomicAdd(bad, b);
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

__global__ __launch_bounds__(kBlock) void k_widen(const float* __restrict__ a, int64_t m,
                                                  double* __restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < m) b[i] = (double)a[i];
}

hipError_t build_chunks(pixelsne_ctx* c) {
    hipError_t e;
    k_int_len<<<grid_for(c->n + 1), kBlock, 0, c->stream>>>(c->orig, c->row_ptr, c->n, c->len_tmp);
    if ((e = scan_i64(c->len_tmp, c->n + 1, c->rp_int, c->scan_tmp, c->stream)) != hipSuccess) return e;
    k_chunk_flags<<<grid_for(c->n + 1), kBlock, 0, c->stream>>>(c->rp_int, c->n, c->len_tmp);
    if ((e = scan_i64(c->len_tmp, c->n + 1, c->ch_tmp, c->scan_tmp, c->stream)) != hipSuccess) return e;
    k_chunk_rows<<<grid_for(c->n + 1), kBlock, 0, c->stream>>>(c->rp_int, c->n, c->ch_tmp, c->ch_row,
                                                              c->sc);
    const int64_t nb = c->n < kBuildBlocksMax ? c->n : kBuildBlocksMax;
    if (fp64(c))
        k_chunk_build<double><<<dim3((unsigned)nb), kBuildThreads, 0, c->stream>>>(
            c->row_ptr, c->col, (const double*)c->val, c->orig, c->inv, c->rp_int, c->ch_row, c->sc,
            c->pk, (double*)c->vch);
    else
        k_chunk_build<float><<<dim3((unsigned)nb), kBuildThreads, 0, c->stream>>>(
            c->row_ptr, c->col, (const float*)c->val, c->orig, c->inv, c->rp_int, c->ch_row, c->sc,
            c->pk, (float*)c->vch);
    return hipGetLastError();
}

}  // namespace

hipError_t run_identity_order(pixelsne_ctx* c) {
    k_iota2<<<grid_for(c->n), kBlock, 0, c->stream>>>(c->orig, c->inv, c->n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the first renumbering follows the first iteration
    c->reorder_interval = c->prm.reorder_every;
    c->since_reorder = c->prm.reorder_every > 0 ? c->prm.reorder_every - 1 : 0;
    c->since_reorder0 = c->since_reorder;
    return build_chunks(c);
}

hipError_t run_data_order(pixelsne_ctx* c, const void* X, int32_t D, int32_t x_dtype) {
    hipError_t e = projection_keys(X, c->n, D, x_dtype, c->tb.key[0], c->stream);
    if (e == hipSuccess) e = run_sort_bits(c, 30);
    if (e == hipSuccess) e = run_reorder(c);
    if (e != hipSuccess) return e;
    // the embedding's own order is worth following once the early exaggeration
    // has formed its clusters
    c->reorder_interval = c->prm.reorder_every;
    if (c->prm.reorder_every > 0) {
        const int32_t first = c->prm.exag_iters > 1 ? c->prm.exag_iters : 1;
        c->since_reorder = c->prm.reorder_every - first;
    }
    c->since_reorder0 = c->since_reorder;
    return hipSuccess;
}

void reset_reorder_schedule(pixelsne_ctx* c, int32_t t) {
    c->reorder_interval = c->prm.reorder_every;
    c->since_reorder = c->since_reorder0;
    c->scheduled_reorders = 0;
    if (c->prm.reorder_every <= 0) return;
    for (int32_t it = 0; it < t; it++) {
        if (++c->since_reorder < c->reorder_interval) continue;
        c->since_reorder = 0;
        if (c->scheduled_reorders++ > 0) {
            const double next = std::ceil((double)c->reorder_interval * c->prm.reorder_growth);
            c->reorder_interval = next < 2147483647.0 ? (int64_t)next : 2147483647;
        }
    }
}

// After an iteration: renumber when the schedule says so.  The interval after
// the first scheduled renumbering is reorder_every; after each later one it
// grows by reorder_growth.
hipError_t run_scheduled_reorder(pixelsne_ctx* c) {
    if (c->prm.reorder_every <= 0 || ++c->since_reorder < c->reorder_interval) return hipSuccess;
    const hipError_t e = run_reorder(c);
    if (c->scheduled_reorders++ > 0) {
        const double next = std::ceil((double)c->reorder_interval * c->prm.reorder_growth);
        c->reorder_interval = next < 2147483647.0 ? (int64_t)next : 2147483647;
    }
    return e;
}

hipError_t run_reorder(pixelsne_ctx* c) {
    const TreeBufs& tb = c->tb;
    const uint32_t* perm = tb.idx[tb.sorted];
    k_reorder_index<<<grid_for(c->n), kBlock, 0, c->stream>>>(perm, c->orig, c->n, c->inv, c->orig2);
    if (fp64(c))
        k_reorder_state<double><<<grid_for(c->n), kBlock, 0, c->stream>>>(
            perm, (const double*)c->zh, (const double*)c->u, (const double*)c->g,
            (double*)c->zh2, (double*)c->u2, (double*)c->g2, c->n);
    else
        k_reorder_state<float><<<grid_for(c->n), kBlock, 0, c->stream>>>(
            perm, (const float*)c->zh, (const float*)c->u, (const float*)c->g, (float*)c->zh2,
            (float*)c->u2, (float*)c->g2, c->n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    std::swap(c->zh, c->zh2);
    std::swap(c->u, c->u2);
    std::swap(c->g, c->g2);
    std::swap(c->orig, c->orig2);
    c->parity ^= 1;
    c->since_reorder = 0;
    return build_chunks(c);
}

hipError_t run_export_P(const pixelsne_ctx* c, int64_t* row_ptr, int32_t* col, double* val) {
    hipError_t e = hipSuccess;
    if (row_ptr)
        e = hipMemcpyAsync(row_ptr, c->row_ptr, 8 * (size_t)(c->n + 1), hipMemcpyDeviceToDevice,
                           c->stream);
    if (e == hipSuccess && col)
        e = hipMemcpyAsync(col, c->col, 4 * (size_t)c->nnz, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess && val) {
        if (fp64(c)) {
            e = hipMemcpyAsync(val, c->val, 8 * (size_t)c->nnz, hipMemcpyDeviceToDevice, c->stream);
        } else {
            k_widen<<<grid_for(c->nnz), kBlock, 0, c->stream>>>((const float*)c->val, c->nnz, val);
            e = hipGetLastError();
        }
    }
    return e;
}

hipError_t check_csr(const int64_t* row_ptr, const uint32_t* col, int64_t n, int64_t nnz,
                     hipStream_t s, int64_t* bad) {
    unsigned long long* d = nullptr;
    hipError_t e = hipMalloc((void**)&d, sizeof(unsigned long long));
    if (e != hipSuccess) return e;
    unsigned long long h = 0;
    e = hipMemcpyAsync(d, &h, sizeof(h), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        const int64_t nb = ceil_div(n, kBlock) < 4096 ? ceil_div(n, kBlock) : 4096;
        k_check_csr<<<dim3((unsigned)nb), kBlock, 0, s>>>(row_ptr, col, n, nnz, d);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d);
    *bad = (int64_t)h;
    return e;
}

hipError_t run_check_csr(const pixelsne_ctx* c, int64_t* bad) {
    return check_csr(c->row_ptr, c->col, c->n, c->nnz, c->stream, bad);
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
