// One-time setup on gfx950: the sparse affinity matrix P (paper Section 3.2-3.3).
//
//   knn          brute-force k nearest neighbours.  Distance tiles come from
//                FP32 MFMA (v_mfma_f32_32x32x2f32): d = |x|^2 + |y|^2 - 2 x.y,
//                or, for uint8 rows, exactly from INT8 MFMA on x - 128;
//                each row keeps a candidate list (global memory, per-row
//                threshold in LDS) that is compacted to the K' = k + 32 best
//                by a block-wide bitonic sort whenever it fills up.  The K'
//                survivors are re-ranked with exact FP64 distances and ties go
//                to the smaller index.
//   perplexity   per-row bisection on the Gaussian precision (FP64)
//   symmetrize   p_ij = (p_{j|i} + p_{i|j}) / 2n on the union pattern -> CSR
#include <math.h>

#include <string>
#include <type_traits>

#include "ctx.h"

namespace psne {

namespace {


constexpr int kQB = 128;       // query rows per block
constexpr int kCB = 128;       // candidate columns per tile
constexpr int kKC = 32;        // reduction chunk staged in LDS (2 threads x 16 per row)
constexpr int kCap = 512;      // candidate list capacity per row
constexpr int kMargin = 32;    // extra candidates kept for the exact re-rank

template <typename X> __device__ __forceinline__ float to_f32(X v) { return (float)v; }

template <typename X>
__device__ __forceinline__ double to_f64(X v) { return (double)v; }

template <typename X>
__global__ __launch_bounds__(256) void k_row_norms(const X* __restrict__ Xm, int64_t n, int D,
                                                   float* __restrict__ nrm) {
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = lane_id();
    if (i >= n) return;
    double a = 0.0;
    for (int d = lane; d < D; d += 64) {
        const float v = to_f32(Xm[i * D + d]);
        a += (double)v * (double)v;
    }
    a = wave_sum(a);
    if (lane == 0) nrm[i] = (float)a;
}

// block-wide bitonic sort of 512 uint64 keys in LDS (256 threads)
__device__ void bitonic512(uint64_t* s) {
    const int t = threadIdx.x;
    for (int k = 2; k <= 512; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            // thread t handles the pair whose lower index has bit j clear
            const int i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
            const int l = i | j;
            const uint64_t a = s[i], b = s[l];
            const bool up = (i & k) == 0;
            if ((a > b) == up) {
                s[i] = b;
                s[l] = a;
            }
            __syncthreads();
        }
    }
}

__device__ __forceinline__ uint64_t cand_key(float d, uint32_t j) {
    const float c = d > 0.0f ? d : 0.0f;
    return ((uint64_t)__float_as_uint(c) << 32) | (uint64_t)j;
}

// A candidate key is (distance bits << 32 | column): the bits of a
// non-negative float, or an exact integer distance, both ordered as unsigned
// integers.  A row's threshold is the distance bits of its kp-th best key
// (kNoThr while the list is not full).
constexpr uint32_t kNoThr = 0xFFFFFFFFu;

// Compact the candidate list of local row q to its kp best (sorted).
__device__ void compact_row(int q, int64_t grow, uint32_t* cnt, uint32_t* thr, uint64_t* cand,
                            uint64_t* sbuf, int kp) {
    const int t = threadIdx.x;
    const int m = (int)cnt[q];
    uint64_t* lst = cand + grow * kCap;
    for (int e = t; e < 512; e += 256) sbuf[e] = e < m ? lst[e] : ~0ull;
    __syncthreads();
    bitonic512(sbuf);
    const int keep = m < kp ? m : kp;
    for (int e = t; e < keep; e += 256) lst[e] = sbuf[e];
    __syncthreads();
    if (t == 0) {
        cnt[q] = (uint32_t)keep;
        thr[q] = keep == kp ? (uint32_t)(sbuf[kp - 1] >> 32) : kNoThr;
    }
    __syncthreads();
}

// After a tile: compact the rows whose lists could overflow during the next
// one.  Threads 0..kQB-1 test their row and the waves' ballots go through LDS,
// so the block walks only the rows that need it (usually none).
__device__ void compact_full_rows(int64_t q0, uint32_t* cnt, uint32_t* thr, uint64_t* cand,
                                  uint64_t* sbuf, uint64_t* need, int kp) {
    static_assert(kQB == 2 * 64, "two waves test the rows");
    const int t = threadIdx.x;
    if (t < kQB) {
        const uint64_t b = ballot64(cnt[t] > (uint32_t)(kCap - kCB));
        if (lane_id() == 0) need[t >> 6] = b;
    }
    __syncthreads();
    // need[] is next written after the next tile's barriers
    const uint64_t m0 = need[0], m1 = need[1];
    for (int h = 0; h < 2; h++) {
        uint64_t m = h ? m1 : m0;
        while (m) {
            const int q = 64 * h + __ffsll((long long)m) - 1;
            m &= m - 1;
            compact_row(q, q0 + q, cnt, thr, cand, sbuf, kp);
        }
    }
}

// Candidate generation.  One block (four waves) per kQB query rows sweeps all
// candidate columns in tiles of kCB; the 128 x 128 distance tile comes from
// FP32 MFMA (v_mfma_f32_32x32x2f32), each wave owning a 64 x 64 quarter as
// 2 x 2 MFMA tiles.  X is staged through LDS in chunks of kKC dimensions,
// k-major so that a fragment read is 32 consecutive words, with the next
// chunk's global loads in flight while the current one is multiplied.
typedef float v16f __attribute__((ext_vector_type(16)));

template <typename X, bool VEC>
__global__ __launch_bounds__(256) void k_knn_candidates(const X* __restrict__ Xm, int64_t n,
                                                        int D, const float* __restrict__ nrm,
                                                        int kp, uint64_t* __restrict__ cand,
                                                        uint32_t* __restrict__ cand_cnt,
                                                        uint32_t* __restrict__ cand_thr) {
    static_assert(!VEC || std::is_same<X, float>::value, "16-byte loads of FP32 rows");
    // [buffer][k][row]: rows 0..127 queries, 128..255 candidates
    __shared__ float S[2][kKC][2 * kQB + 4];
    __shared__ uint32_t cnt[kQB];
    __shared__ uint32_t thr[kQB];
    __shared__ float nq[kQB];
    __shared__ float nc[kCB];
    __shared__ uint64_t sbuf[512];
    __shared__ uint64_t need[2];

    const int t = threadIdx.x, w = t >> 6, lane = lane_id();
    const int wr = 64 * (w >> 1), wc = 64 * (w & 1);
    const int64_t q0 = (int64_t)blockIdx.x * kQB;
    if (t < kQB) {
        cnt[t] = 0;
        thr[t] = kNoThr;
        nq[t] = q0 + t < n ? nrm[q0 + t] : 0.0f;
    }
    const int nk = (D + kKC - 1) / kKC;

    for (int64_t c0 = 0; c0 < n; c0 += kCB) {
        v16f acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < 2; b++)
#pragma unroll
                for (int v = 0; v < 16; v++) acc[a][b][v] = 0.0f;
        if (t < kCB) nc[t] = c0 + t < n ? nrm[c0 + t] : 0.0f;
        // query rows q0.. as staging rows 0..127, candidates c0.. as 128..255:
        // thread t loads row t / 2 of the queries (h = 0) and of the candidates (h = 1)
        float g[kKC];                           // kKC / 2 query and kKC / 2 candidate values
        const int64_t rq = q0 + (t >> 1), rc = c0 + (t >> 1);
        const bool okq = rq < n, okc = rc < n;
        constexpr int kH = kKC / 2;                     // dimensions per thread and row
        const X* pq = Xm + (okq ? rq : 0) * (int64_t)D + kH * (t & 1);
        const X* pc = Xm + (okc ? rc : 0) * (int64_t)D + kH * (t & 1);
        auto fetch = [&](int k0) {
            if constexpr (VEC) {
                // FP32 rows, D a multiple of 4, 16-byte aligned: 16-byte loads;
                // a group of four past the row's end reads the row's first four
                // (D >= 4), a row past n reads row 0, and both are zeroed
                const int lim = D - k0 - kH * (t & 1);          // elements left in the row
#pragma unroll
                for (int u = 0; u < kH; u += 4) {
                    const bool in = u < lim;                    // lim is a multiple of 4
                    const int off = in ? k0 + u : -kH * (t & 1);   // else the row's start
                    const float4 a = *reinterpret_cast<const float4*>(pq + off);
                    const float4 c = *reinterpret_cast<const float4*>(pc + off);
                    const bool iq = okq && in, ic = okc && in;
                    g[u] = iq ? a.x : 0.0f;
                    g[u + 1] = iq ? a.y : 0.0f;
                    g[u + 2] = iq ? a.z : 0.0f;
                    g[u + 3] = iq ? a.w : 0.0f;
                    g[kH + u] = ic ? c.x : 0.0f;
                    g[kH + u + 1] = ic ? c.y : 0.0f;
                    g[kH + u + 2] = ic ? c.z : 0.0f;
                    g[kH + u + 3] = ic ? c.w : 0.0f;
                }
            } else {
                const int lim = D - k0 - kH * (t & 1);          // elements left in the row
#pragma unroll
                for (int e = 0; e < kH; e++) {
                    g[e] = (okq && e < lim) ? to_f32(pq[k0 + e]) : 0.0f;
                    g[kH + e] = (okc && e < lim) ? to_f32(pc[k0 + e]) : 0.0f;
                }
            }
        };
        auto store = [&](int buf) {
            const int row = t >> 1, kb = kH * (t & 1);
#pragma unroll
            for (int e = 0; e < kH; e++) {
                S[buf][kb + e][row] = g[e];
                S[buf][kb + e][kQB + row] = g[kH + e];
            }
        };
        __syncthreads();                       // previous tile's readers are done
        fetch(0);
        store(0);
        __syncthreads();
        for (int kc = 0; kc < nk; kc++) {
            const int buf = kc & 1;
            if (kc + 1 < nk) fetch((kc + 1) * kKC);
#pragma unroll
            for (int kk = 0; kk < kKC; kk += 2) {
                const int k = kk + (lane >> 5);
                const float a0 = S[buf][k][wr + (lane & 31)];
                const float a1 = S[buf][k][wr + 32 + (lane & 31)];
                const float b0 = S[buf][k][kQB + wc + (lane & 31)];
                const float b1 = S[buf][k][kQB + wc + 32 + (lane & 31)];
                acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
            }
            if (kc + 1 < nk) store(buf ^ 1);
            __syncthreads();
        }
        // filter, one 32 x 32 MFMA tile at a time through a wave-private LDS
        // tile (the staging buffer is free after the last chunk): element v of
        // tile (a, b) is row 8(v / 4) + 4(lane / 32) + v % 4, column lane % 32
        float* T = &S[0][0][0] + w * (32 * 33);
        const int cj = lane & 31;
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < 2; b++) {
#pragma unroll
                for (int v = 0; v < 16; v++)
                    T[(8 * (v >> 2) + 4 * (lane >> 5) + (v & 3)) * 33 + cj] = acc[a][b][v];
                const int cl = wc + 32 * b + cj;
                const int64_t gc = c0 + cl;
                const float ncv = nc[cl];
#pragma unroll 2
                for (int m = 0; m < 16; m++) {
                    const int i = 2 * m + (lane >> 5);
                    const int rl = wr + 32 * a + i;
                    const int64_t gr = q0 + rl;
                    const float d = nq[rl] + ncv - 2.0f * T[i * 33 + cj];
                    const uint64_t key = cand_key(d, (uint32_t)gc);
                    if (gr < n && gc < n && gc != gr && (uint32_t)(key >> 32) <= thr[rl]) {
                        const uint32_t pos = atomicAdd(&cnt[rl], 1u);
                        cand[gr * kCap + pos] = key;
                    }
                }
            }
        __syncthreads();
        compact_full_rows(q0, cnt, thr, cand, sbuf, need, kp);
    }
    for (int q = 0; q < kQB; q++) {
        if (q0 + q < n) compact_row(q, q0 + q, cnt, thr, cand, sbuf, kp);
    }
    if (t < kQB && q0 + t < n) {
        cand_cnt[q0 + t] = cnt[t];
        cand_thr[q0 + t] = thr[t];
    }
}

// Exact candidates for uint8 rows: x' = x - 128 as int8 through
// v_mfma_i32_32x32x16_i8, so that every distance |x'|^2 + |y'|^2 - 2 x'.y'
// is an exact int32 (|x'| <= 128, D <= 32768).  Same blocking as the FP32
// kernel: 128 x 128 tile per block, a 64 x 64 quarter per wave; X staged in
// LDS row-major, kKB bytes of each row per chunk.
typedef int v16i __attribute__((ext_vector_type(16)));
constexpr int kKB = 64;

__global__ __launch_bounds__(256) void k_row_norms_i8(const uint8_t* __restrict__ Xm, int64_t n,
                                                      int D, int32_t* __restrict__ nrm) {
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = lane_id();
    if (i >= n) return;
    int a = 0;
    for (int d = lane; d < D; d += 64) {
        const int v = (int)Xm[i * D + d] - 128;
        a += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    if (lane == 0) nrm[i] = a;
}

__global__ __launch_bounds__(256) void k_knn_candidates_i8(const uint8_t* __restrict__ Xm,
                                                           int64_t n, int D,
                                                           const int32_t* __restrict__ nrm,
                                                           int kp, uint64_t* __restrict__ cand,
                                                           uint32_t* __restrict__ cand_cnt,
                                                           uint32_t* __restrict__ cand_thr) {
    // [buffer][row][k]: rows 0..127 queries, 128..255 candidates; 16 bytes pad
    __shared__ __attribute__((aligned(16))) int8_t S[2][2 * kQB][kKB + 16];
    __shared__ int32_t T[4][32][33];
    __shared__ uint32_t cnt[kQB];
    __shared__ uint32_t thr[kQB];
    __shared__ int32_t nq[kQB];
    __shared__ int32_t nc[kCB];
    __shared__ uint64_t sbuf[512];
    __shared__ uint64_t need[2];

    const int t = threadIdx.x, w = t >> 6, lane = lane_id();
    const int wr = 64 * (w >> 1), wc = 64 * (w & 1);
    const int64_t q0 = (int64_t)blockIdx.x * kQB;
    if (t < kQB) {
        cnt[t] = 0;
        thr[t] = kNoThr;
        nq[t] = q0 + t < n ? nrm[q0 + t] : 0;
    }
    const int nk = (D + kKB - 1) / kKB;
    const int seg = 16 * (t & 3);                  // this thread's 16 bytes of a row

    for (int64_t c0 = 0; c0 < n; c0 += kCB) {
        v16i acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < 2; b++)
#pragma unroll
                for (int v = 0; v < 16; v++) acc[a][b][v] = 0;
        if (t < kCB) nc[t] = c0 + t < n ? nrm[c0 + t] : 0;
        // thread t stages staging rows t / 4 + 64 h (h = 0..3), bytes seg..seg+15
        uint4 g[4];
        auto fetch = [&](int k0) {
#pragma unroll
            for (int h = 0; h < 4; h++) {
                const int row = (t >> 2) + 64 * h;
                const int64_t gr = row < kQB ? q0 + row : c0 + (row - kQB);
                const int kb = k0 + seg;
                union {
                    uint4 q;
                    uint8_t b[16];
                } v;
                const uint8_t* src = Xm + (gr < n ? gr : 0) * (int64_t)D + kb;
                if (gr < n && kb + 16 <= D && ((reinterpret_cast<uintptr_t>(src) & 15u) == 0)) {
                    v.q = *reinterpret_cast<const uint4*>(src);
                } else {
#pragma unroll
                    for (int e = 0; e < 16; e++)
                        v.b[e] = (gr < n && kb + e < D) ? src[e] : (uint8_t)128;   // x' = 0
                }
                // centre: x - 128 as int8 is the byte with its top bit flipped
                v.q.x ^= 0x80808080u;
                v.q.y ^= 0x80808080u;
                v.q.z ^= 0x80808080u;
                v.q.w ^= 0x80808080u;
                g[h] = v.q;
            }
        };
        auto store = [&](int buf) {
#pragma unroll
            for (int h = 0; h < 4; h++)
                *reinterpret_cast<uint4*>(&S[buf][(t >> 2) + 64 * h][seg]) = g[h];
        };
        __syncthreads();                       // previous tile's readers are done
        fetch(0);
        store(0);
        __syncthreads();
        for (int kc = 0; kc < nk; kc++) {
            const int buf = kc & 1;
            if (kc + 1 < nk) fetch((kc + 1) * kKB);
#pragma unroll
            for (int kk = 0; kk < kKB; kk += 16) {
                const int kb = kk + 8 * (lane >> 5);
                const long a0 = *reinterpret_cast<const long*>(&S[buf][wr + (lane & 31)][kb]);
                const long a1 = *reinterpret_cast<const long*>(&S[buf][wr + 32 + (lane & 31)][kb]);
                const long b0 = *reinterpret_cast<const long*>(&S[buf][kQB + wc + (lane & 31)][kb]);
                const long b1 =
                    *reinterpret_cast<const long*>(&S[buf][kQB + wc + 32 + (lane & 31)][kb]);
                acc[0][0] = __builtin_amdgcn_mfma_i32_32x32x16_i8(a0, b0, acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_i32_32x32x16_i8(a0, b1, acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_i32_32x32x16_i8(a1, b0, acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_i32_32x32x16_i8(a1, b1, acc[1][1], 0, 0, 0);
            }
            if (kc + 1 < nk) store(buf ^ 1);
            __syncthreads();
        }
        // filter through a wave-private LDS tile, as in the FP32 kernel
        const int cj = lane & 31;
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < 2; b++) {
#pragma unroll
                for (int v = 0; v < 16; v++)
                    T[w][8 * (v >> 2) + 4 * (lane >> 5) + (v & 3)][cj] = acc[a][b][v];
                const int cl = wc + 32 * b + cj;
                const int64_t gc = c0 + cl;
                const int32_t ncv = nc[cl];
#pragma unroll 2
                for (int m = 0; m < 16; m++) {
                    const int i = 2 * m + (lane >> 5);
                    const int rl = wr + 32 * a + i;
                    const int64_t gr = q0 + rl;
                    const int32_t d = nq[rl] + ncv - 2 * T[w][i][cj];
                    if (gr < n && gc < n && gc != gr && (uint32_t)d <= thr[rl]) {
                        const uint32_t pos = atomicAdd(&cnt[rl], 1u);
                        cand[gr * kCap + pos] = ((uint64_t)(uint32_t)d << 32) | (uint64_t)gc;
                    }
                }
            }
        __syncthreads();
        compact_full_rows(q0, cnt, thr, cand, sbuf, need, kp);
    }
    for (int q = 0; q < kQB; q++) {
        if (q0 + q < n) compact_row(q, q0 + q, cnt, thr, cand, sbuf, kp);
    }
    if (t < kQB && q0 + t < n) {
        cand_cnt[q0 + t] = cnt[t];
        cand_thr[q0 + t] = thr[t];
    }
}

// Exact re-rank: FP64 distances of the candidates, sorted by (d, j); emits
// the first k.  flag[i] = 1 when the error bound of the FP32 pre-selection
// does not prove that the k best are among the candidates.
template <typename X>
__global__ __launch_bounds__(256) void k_knn_rerank(const X* __restrict__ Xm, int D,
                                                    int k, const uint64_t* __restrict__ cand,
                                                    const uint32_t* __restrict__ cand_cnt,
                                                    const uint32_t* __restrict__ cand_thr,
                                                    const float* __restrict__ nrm, float nrm_max,
                                                    int exact_keys,
                                                    int32_t* __restrict__ idx,
                                                    double* __restrict__ d2,
                                                    uint32_t* __restrict__ flag) {
    __shared__ double dv[512];
    __shared__ uint32_t jv[512];
    const int64_t i = blockIdx.x;
    const int t = threadIdx.x;
    const int m = (int)cand_cnt[i];
    const uint64_t* lst = cand + i * kCap;
    for (int e = t; e < 512; e += 256) {
        if (e < m) {
            const uint32_t j = (uint32_t)(lst[e] & 0xFFFFFFFFu);
            double a = 0.0;
            for (int d = 0; d < D; d++) {
                const double v = to_f64(Xm[i * D + d]) - to_f64(Xm[(int64_t)j * D + d]);
                a += v * v;
            }
            dv[e] = a;
            jv[e] = j;
        } else {
            dv[e] = INFINITY;
            jv[e] = 0xFFFFFFFFu;
        }
    }
    __syncthreads();
    for (int kk = 2; kk <= 512; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            const int a = ((t & ~(j - 1)) << 1) | (t & (j - 1));
            const int b = a | j;
            const double da = dv[a], db = dv[b];
            const uint32_t ja = jv[a], jb = jv[b];
            const bool gt = da > db || (da == db && ja > jb);
            const bool up = (a & kk) == 0;
            if (gt == up) {
                dv[a] = db; dv[b] = da;
                jv[a] = jb; jv[b] = ja;
            }
            __syncthreads();
        }
    }
    for (int e = t; e < k; e += 256) {
        idx[i * k + e] = (int32_t)jv[e];
        d2[i * k + e] = dv[e];
    }
    if (t == 0) {
        const uint32_t tb = cand_thr[i];
        if (tb == kNoThr) {
            flag[i] = 0u;                        // every candidate was kept
        } else if (exact_keys) {
            // exact integer distances: only a tie at the threshold is unproven
            flag[i] = dv[k - 1] < (double)tb ? 0u : 1u;
        } else {
            // |fp32(d) - d| <= (D + 4) 2^-24 (|x| + |y|)^2  (conservative)
            const double tau = (double)__uint_as_float(tb);
            const double sx = sqrt((double)nrm[i]), sy = sqrt((double)nrm_max);
            const double err = (double)(D + 4) * 0x1.0p-24 * (sx + sy) * (sx + sy) * 1.01;
            flag[i] = dv[k - 1] < tau - err ? 0u : 1u;
        }
    }
}

// Exact fallback for rows the bound could not certify: block per row,
// FP64 over all n, keeps a sorted top-k in LDS by repeated block passes.
template <typename X>
__global__ __launch_bounds__(256) void k_knn_exact_row(const X* __restrict__ Xm, int64_t n, int D,
                                                       int k, const uint32_t* __restrict__ rows,
                                                       int32_t* __restrict__ idx,
                                                       double* __restrict__ d2) {
    __shared__ double bd[256];
    __shared__ uint32_t bj[256];
    const int64_t i = rows[blockIdx.x];
    const int t = threadIdx.x;
    double last_d = -1.0;
    uint32_t last_j = 0;
    for (int r = 0; r < k; r++) {
        // smallest (d, j) strictly greater than (last_d, last_j)
        double bdv = INFINITY;
        uint32_t bjv = 0xFFFFFFFFu;
        for (int64_t j = t; j < n; j += 256) {
            if (j == i) continue;
            double a = 0.0;
            for (int d = 0; d < D; d++) {
                const double v = to_f64(Xm[i * D + d]) - to_f64(Xm[j * D + d]);
                a += v * v;
            }
            const bool after = a > last_d || (a == last_d && (uint32_t)j > last_j);
            const bool better = a < bdv || (a == bdv && (uint32_t)j < bjv);
            if (after && better) { bdv = a; bjv = (uint32_t)j; }
        }
        bd[t] = bdv; bj[t] = bjv;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (t < o) {
                const bool better = bd[t + o] < bd[t] || (bd[t + o] == bd[t] && bj[t + o] < bj[t]);
                if (better) { bd[t] = bd[t + o]; bj[t] = bj[t + o]; }
            }
            __syncthreads();
        }
        last_d = bd[0];
        last_j = bj[0];
        if (t == 0) {
            idx[i * k + r] = (int32_t)last_j;
            d2[i * k + r] = last_d;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// perplexity calibration, one thread per row (FP64)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_perplexity(const double* __restrict__ d2, int64_t n,
                                                    int k, double target, double tol,
                                                    int max_iter, double* __restrict__ P,
                                                    double* __restrict__ beta_out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double* d = d2 + i * k;
    double* p = P + i * k;
    double dmin = d[0];
    for (int j = 1; j < k; j++) dmin = fmin(dmin, d[j]);
    double b = 1.0, lo = 0.0, hi = 0.0, S = 0.0;
    bool have_lo = false, have_hi = false;
    for (int it = 0; it < max_iter; it++) {
        S = 0.0;
        double SD = 0.0;
        for (int j = 0; j < k; j++) {
            const double dj = d[j] - dmin;
            const double e = exp(-b * dj);
            p[j] = e;
            S += e;
            SD += dj * e;
        }
        const double H = log(S) + b * SD / S;
        if (fabs(H - target) < tol || it == max_iter - 1) break;
        if (H > target) {
            lo = b; have_lo = true;
            b = have_hi ? 0.5 * (b + hi) : 2.0 * b;
        } else {
            hi = b; have_hi = true;
            b = have_lo ? 0.5 * (b + lo) : 0.5 * b;
        }
    }
    for (int j = 0; j < k; j++) p[j] /= S;
    if (beta_out) beta_out[i] = b;
}

// ---------------------------------------------------------------------------
// symmetrisation
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_indeg(const int32_t* __restrict__ idx, int64_t m,
                                               uint32_t* __restrict__ indeg) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < m) atomicAdd(&indeg[idx[e]], 1u);
}

__global__ __launch_bounds__(256) void k_row_caps(const uint32_t* __restrict__ indeg, int64_t n,
                                                  int k, int64_t* __restrict__ cap) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) cap[i] = (int64_t)k + indeg[i];
    if (i == n) cap[n] = 0;
}

// exclusive scan of int64, three phases (block size 1024 elements)
__global__ __launch_bounds__(256) void k_scan64_reduce(const int64_t* __restrict__ a, int64_t m,
                                                       int64_t* __restrict__ bsum) {
    __shared__ int64_t red[256];
    const int64_t base = (int64_t)blockIdx.x * 1024;
    int64_t s = 0;
    for (int e = threadIdx.x; e < 1024; e += 256)
        if (base + e < m) s += a[base + e];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(1024) void k_scan64_top(int64_t* __restrict__ bsum, int64_t nb) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (nb + 1023) / 1024;
    const int64_t b = t * per, e = b + per < nb ? b + per : nb;
    int64_t s = 0;
    for (int64_t i = b; i < e; i++) s += bsum[i];
    part[t] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        int64_t v = t >= o ? part[t - o] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = t ? part[t - 1] : 0;
    for (int64_t i = b; i < e; i++) {
        int64_t v = bsum[i];
        bsum[i] = run;
        run += v;
    }
}

__global__ __launch_bounds__(256) void k_scan64_apply(const int64_t* __restrict__ a, int64_t m,
                                                      const int64_t* __restrict__ bsum,
                                                      int64_t* __restrict__ out) {
    __shared__ int64_t s[1024];
    const int64_t base = (int64_t)blockIdx.x * 1024;
    for (int e = threadIdx.x; e < 1024; e += 256) s[e] = base + e < m ? a[base + e] : 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = bsum[blockIdx.x];
        for (int e = 0; e < 1024; e++) {
            const int64_t v = s[e];
            s[e] = run;
            run += v;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 1024; e += 256)
        if (base + e < m) out[base + e] = s[e];
}

__global__ __launch_bounds__(256) void k_sym_fill(const int32_t* __restrict__ idx,
                                                  const double* __restrict__ Pc, int64_t n, int k,
                                                  const int64_t* __restrict__ off,
                                                  uint32_t* __restrict__ fill,
                                                  uint32_t* __restrict__ tcol,
                                                  double* __restrict__ tval) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n * (int64_t)k) return;
    const int64_t i = e / k;
    const int t = (int)(e - i * k);
    const int32_t j = idx[e];
    const double v = Pc[e];
    tcol[off[i] + t] = (uint32_t)j;
    tval[off[i] + t] = v;
    const uint32_t slot = atomicAdd(&fill[j], 1u);
    tcol[off[j] + k + slot] = (uint32_t)i;
    tval[off[j] + k + slot] = v;
}

constexpr int kRowMax = 4096;

// Sort one row by column (rank by counting, ties by position) into scol/sval
// at the same offsets, merge the (at most two) summands of each column, write
// the unique entries at the row start of tcol/tval and their number.  Rows
// up to kRowMax entries are ranked from LDS, longer rows from global memory.
__global__ __launch_bounds__(256) void k_sym_row(const int64_t* __restrict__ off,
                                                 uint32_t* __restrict__ tcol,
                                                 double* __restrict__ tval,
                                                 uint32_t* __restrict__ scol,
                                                 double* __restrict__ sval,
                                                 int64_t* __restrict__ ucnt) {
    __shared__ uint32_t c_in[kRowMax];
    __shared__ uint32_t wsum[4];
    const int64_t i = blockIdx.x;
    const int t = threadIdx.x;
    const int64_t b = off[i];
    const int64_t len = off[i + 1] - b;
    const bool in_lds = len <= kRowMax;
    if (in_lds)
        for (int64_t e = t; e < len; e += 256) c_in[e] = tcol[b + e];
    __syncthreads();
    for (int64_t e = t; e < len; e += 256) {
        const uint32_t ce = in_lds ? c_in[e] : tcol[b + e];
        int64_t r = 0;
        if (in_lds) {
            for (int64_t f = 0; f < len; f++) {
                const uint32_t cf = c_in[f];
                r += (cf < ce || (cf == ce && f < e)) ? 1 : 0;
            }
        } else {
            for (int64_t f = 0; f < len; f++) {
                const uint32_t cf = tcol[b + f];
                r += (cf < ce || (cf == ce && f < e)) ? 1 : 0;
            }
        }
        scol[b + r] = ce;
        sval[b + r] = tval[b + e];
    }
    __threadfence_block();
    __syncthreads();
    // unique flags and their exclusive prefix, 256 entries at a time
    int64_t base = 0;
    for (int64_t c0 = 0; c0 < len; c0 += 256) {
        const int64_t e = c0 + t;
        const bool u = e < len && (e == 0 || scol[b + e] != scol[b + e - 1]);
        const uint64_t bal = ballot64(u);
        if (lane_id() == 0) wsum[t >> 6] = (uint32_t)__popcll(bal);
        __syncthreads();
        int64_t pre = base + (int64_t)__popcll(bal & lanemask_lt());
        for (int q = 0; q < (t >> 6); q++) pre += wsum[q];
        if (u) {
            double v = sval[b + e];
            if (e + 1 < len && scol[b + e + 1] == scol[b + e]) v = v + sval[b + e + 1];
            tcol[b + pre] = scol[b + e];
            tval[b + pre] = v;
        }
        const int64_t tot = (int64_t)wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
        base += tot;
    }
    if (t == 0) ucnt[i] = base;
}

__global__ __launch_bounds__(256) void k_sym_write(const int64_t* __restrict__ off,
                                                   const int64_t* __restrict__ rp,
                                                   const uint32_t* __restrict__ tcol,
                                                   const double* __restrict__ tval,
                                                   uint32_t* __restrict__ col,
                                                   double* __restrict__ val, double inv2n) {
    const int64_t i = blockIdx.x;
    const int64_t b = off[i], o = rp[i], m = rp[i + 1] - rp[i];
    for (int64_t e = threadIdx.x; e < m; e += 256) {
        col[o + e] = tcol[b + e];
        val[o + e] = tval[b + e] * inv2n;
    }
}

hipError_t scan_i64_local(const int64_t* a, int64_t m, int64_t* out, int64_t* tmp, hipStream_t s) {
    const int64_t nb = ceil_div(m, 1024);
    k_scan64_reduce<<<dim3((unsigned)nb), 256, 0, s>>>(a, m, tmp);
    k_scan64_top<<<1, 1024, 0, s>>>(tmp, nb);
    k_scan64_apply<<<dim3((unsigned)nb), 256, 0, s>>>(a, m, tmp, out);
    return hipGetLastError();
}

template <typename X>
hipError_t knn_typed(const X* Xm, int64_t n, int32_t D, int32_t k, int32_t* idx, double* d2,
                     hipStream_t s, std::string* err) {
    const int kp = (int)((int64_t)(k + kMargin) < n - 1 ? (k + kMargin) : (n - 1));
    float* nrm = nullptr;
    uint64_t* cand = nullptr;
    uint32_t *ccnt = nullptr, *flag = nullptr, *cthr = nullptr;
    int32_t* nrm_i = nullptr;
    hipError_t e = hipSuccess;
    auto fail = [&](hipError_t x) {
        (void)hipFree(nrm); (void)hipFree(cand); (void)hipFree(ccnt); (void)hipFree(flag);
        (void)hipFree(cthr); (void)hipFree(nrm_i);
        return x;
    };
    if ((e = hipMalloc(&nrm, sizeof(float) * n)) != hipSuccess) return fail(e);
    if ((e = hipMalloc(&cand, sizeof(uint64_t) * kCap * n)) != hipSuccess) return fail(e);
    if ((e = hipMalloc(&ccnt, sizeof(uint32_t) * n)) != hipSuccess) return fail(e);
    if ((e = hipMalloc(&cthr, sizeof(uint32_t) * n)) != hipSuccess) return fail(e);
    if ((e = hipMalloc(&flag, sizeof(uint32_t) * n)) != hipSuccess) return fail(e);
    k_row_norms<X><<<dim3((unsigned)ceil_div(n, 4)), 256, 0, s>>>(Xm, n, D, nrm);
    std::vector<float> hn(n);
    if ((e = hipMemcpyAsync(hn.data(), nrm, sizeof(float) * n, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return fail(e);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e);
    float nmax = 0.0f;
    for (float v : hn) {
        if (!isfinite(v)) {
            if (err) *err = "X contains non-finite values";
            return fail(hipErrorInvalidValue);
        }
        nmax = v > nmax ? v : nmax;
    }
    // exact while 256^2 D fits an int32
    const bool kExact = std::is_same<X, uint8_t>::value && D <= 32768;
    if (kExact) {
        // uint8 rows: exact integer distances from INT8 MFMA
        if ((e = hipMalloc(&nrm_i, sizeof(int32_t) * n)) != hipSuccess) return fail(e);
        k_row_norms_i8<<<dim3((unsigned)ceil_div(n, 4)), 256, 0, s>>>(
            (const uint8_t*)Xm, n, D, nrm_i);
        k_knn_candidates_i8<<<dim3((unsigned)ceil_div(n, kQB)), 256, 0, s>>>(
            (const uint8_t*)Xm, n, D, nrm_i, kp, cand, ccnt, cthr);
    } else {
        bool vec = false;
        if constexpr (std::is_same<X, float>::value)
            vec = D % 4 == 0 && ((uintptr_t)Xm & 15) == 0;
        if (vec)
            k_knn_candidates<float, true><<<dim3((unsigned)ceil_div(n, kQB)), 256, 0, s>>>(
                (const float*)Xm, n, D, nrm, kp, cand, ccnt, cthr);
        else
            k_knn_candidates<X, false><<<dim3((unsigned)ceil_div(n, kQB)), 256, 0, s>>>(
                Xm, n, D, nrm, kp, cand, ccnt, cthr);
    }
    k_knn_rerank<X><<<dim3((unsigned)n), 256, 0, s>>>(Xm, D, k, cand, ccnt, cthr, nrm, nmax,
                                                      kExact ? 1 : 0, idx, d2, flag);
    if ((e = hipGetLastError()) != hipSuccess) return fail(e);
    std::vector<uint32_t> hf(n);
    if ((e = hipMemcpyAsync(hf.data(), flag, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return fail(e);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e);
    std::vector<uint32_t> rows;
    for (int64_t i = 0; i < n; i++)
        if (hf[i]) rows.push_back((uint32_t)i);
    if (!rows.empty()) {
        // exact FP64 fallback for rows the FP32 bound did not certify
        if ((e = hipMemcpyAsync(flag, rows.data(), sizeof(uint32_t) * rows.size(),
                                hipMemcpyHostToDevice, s)) != hipSuccess)
            return fail(e);
        k_knn_exact_row<X><<<dim3((unsigned)rows.size()), 256, 0, s>>>(Xm, n, D, k, flag, idx, d2);
        if ((e = hipGetLastError()) != hipSuccess) return fail(e);
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e);
    }
    (void)err;
    return fail(hipSuccess);
}

// ---------------------------------------------------------------------------
// initial numbering: three random +-1 projections of each row, quantised and
// interleaved into a Morton code (points close in X get close codes)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float rademacher(int axis, int d) {
    uint32_t h = (uint32_t)d * 0x9E3779B1u ^ (uint32_t)(axis + 1) * 0x85EBCA77u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    return (h & 1u) ? 1.0f : -1.0f;
}

// one wavefront per row; proj [n][3]; per-block min/max of each axis
template <typename X>
__global__ __launch_bounds__(256) void k_project(const X* __restrict__ Xm, int64_t n, int D,
                                                 float* __restrict__ proj,
                                                 float* __restrict__ part) {
    __shared__ float red[4][6];
    const int w = threadIdx.x >> 6, lane = lane_id();
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * 4 + w; i < n; i += (int64_t)gridDim.x * 4) {
        float a[3] = {0.f, 0.f, 0.f};
        for (int d = lane; d < D; d += 64) {
            const float v = to_f32(Xm[i * D + d]);
#pragma unroll
            for (int q = 0; q < 3; q++) a[q] += rademacher(q, d) * v;
        }
#pragma unroll
        for (int q = 0; q < 3; q++) {
            a[q] = wave_sum(a[q]);
            mn[q] = fminf(mn[q], a[q]);
            mx[q] = fmaxf(mx[q], a[q]);
        }
        if (lane == 0) {
            proj[3 * i + 0] = a[0];
            proj[3 * i + 1] = a[1];
            proj[3 * i + 2] = a[2];
        }
    }
    if (lane == 0)
        for (int q = 0; q < 3; q++) {
            red[w][q] = mn[q];
            red[w][3 + q] = mx[q];
        }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int q = threadIdx.x;
        float v = red[0][q];
        for (int k = 1; k < 4; k++) v = q < 3 ? fminf(v, red[k][q]) : fmaxf(v, red[k][q]);
        part[6 * blockIdx.x + q] = v;
    }
}

__device__ __forceinline__ uint32_t spread3(uint32_t v) {     // 10 bits -> every third bit
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__global__ __launch_bounds__(256) void k_project_keys(const float* __restrict__ proj, int64_t n,
                                                      const float* __restrict__ part, int nb,
                                                      uint32_t* __restrict__ keys) {
    __shared__ float lo[3], hi[3];
    if (threadIdx.x < 3) {
        float a = INFINITY, b = -INFINITY;
        for (int k = 0; k < nb; k++) {
            a = fminf(a, part[6 * k + threadIdx.x]);
            b = fmaxf(b, part[6 * k + 3 + threadIdx.x]);
        }
        lo[threadIdx.x] = a;
        hi[threadIdx.x] = b;
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    uint32_t code = 0;
#pragma unroll
    for (int q = 0; q < 3; q++) {
        const float span = hi[q] - lo[q];
        float f = span > 0.f ? (proj[3 * i + q] - lo[q]) / span * 1024.f : 0.f;
        f = f < 0.f ? 0.f : (f > 1023.f ? 1023.f : f);
        code |= spread3((uint32_t)f) << q;
    }
    keys[i] = code;
}

}  // namespace

hipError_t projection_keys(const void* X, int64_t n, int32_t D, int32_t x_dtype, uint32_t* keys,
                           hipStream_t s) {
    const int nb = (int)(ceil_div(n, 4) < 1024 ? ceil_div(n, 4) : 1024);
    float *proj = nullptr, *part = nullptr;
    hipError_t e = hipMalloc(&proj, sizeof(float) * 3 * (size_t)n);
    if (e == hipSuccess) e = hipMalloc(&part, sizeof(float) * 6 * (size_t)nb);
    if (e == hipSuccess) {
        switch (x_dtype) {
            case PSNE_X_F32:
                k_project<float><<<nb, 256, 0, s>>>((const float*)X, n, D, proj, part);
                break;
            case PSNE_X_F64:
                k_project<double><<<nb, 256, 0, s>>>((const double*)X, n, D, proj, part);
                break;
            default:
                k_project<uint8_t><<<nb, 256, 0, s>>>((const uint8_t*)X, n, D, proj, part);
                break;
        }
        k_project_keys<<<dim3((unsigned)ceil_div(n, 256)), 256, 0, s>>>(proj, n, part, nb, keys);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(proj);
    (void)hipFree(part);
    return e;
}

hipError_t scan_i64(const int64_t* a, int64_t m, int64_t* out, int64_t* tmp, hipStream_t s) {
    return scan_i64_local(a, m, out, tmp, s);
}

int64_t scan_i64_tmp_len(int64_t m) { return ceil_div(m, 1024) + 1; }

hipError_t knn(const void* X, int64_t n, int32_t D, int32_t x_dtype, int32_t k, int32_t* idx,
               double* d2, hipStream_t s, std::string* err) {
    switch (x_dtype) {
        case PSNE_X_F32: return knn_typed<float>((const float*)X, n, D, k, idx, d2, s, err);
        case PSNE_X_F64: return knn_typed<double>((const double*)X, n, D, k, idx, d2, s, err);
        case PSNE_X_U8: return knn_typed<uint8_t>((const uint8_t*)X, n, D, k, idx, d2, s, err);
        default: return hipErrorInvalidValue;
    }
}

hipError_t perplexity(const double* d2, int64_t n, int32_t k, double u, double* P, double* beta,
                      hipStream_t s) {
    k_perplexity<<<dim3((unsigned)ceil_div(n, 256)), 256, 0, s>>>(d2, n, k, log(u), 1e-5, 200, P,
                                                                  beta);
    return hipGetLastError();
}

hipError_t symmetrize(const int32_t* idx, const double* Pc, int64_t n, int32_t k,
                      int64_t** row_ptr_out, uint32_t** col_out, double** val_out, int64_t* nnz_out,
                      hipStream_t s) {
    const int64_t m = n * (int64_t)k;
    uint32_t *indeg = nullptr, *fill = nullptr, *tcol = nullptr, *scol = nullptr;
    int64_t *cap = nullptr, *off = nullptr, *tmp = nullptr, *ucnt = nullptr, *rp = nullptr;
    double *tval = nullptr, *sval = nullptr;
    uint32_t* col = nullptr;
    double* val = nullptr;
    hipError_t e = hipSuccess;
    auto cleanup = [&]() {
        for (void* q : {(void*)indeg, (void*)fill, (void*)tcol, (void*)scol, (void*)cap,
                        (void*)off, (void*)tmp, (void*)ucnt, (void*)tval, (void*)sval})
            (void)hipFree(q);
    };
    auto fail = [&](hipError_t x) {
        cleanup();
        (void)hipFree(rp); (void)hipFree(col); (void)hipFree(val);
        return x;
    };
    const int64_t nb = ceil_div(n + 1, 1024);
    if ((e = hipMalloc(&indeg, 4 * n)) != hipSuccess) return fail(e);
    if ((e = hipMalloc(&fill, 4 * n)) != hipSuccess) return fail(e);
    if ((e = hipMalloc(&cap, 8 * (n + 1))) != hipSuccess) return fail(e);
    if ((e = hipMalloc(&off, 8 * (n + 1))) != hipSuccess) return fail(e);
    if ((e = hipMalloc(&tmp, 8 * (nb + 1))) != hipSuccess) return fail(e);
    if ((e = hipMalloc(&ucnt, 8 * (n + 1))) != hipSuccess) return fail(e);
    if ((e = hipMalloc(&rp, 8 * (n + 1))) != hipSuccess) return fail(e);
    if ((e = hipMalloc(&tcol, 4 * 2 * m)) != hipSuccess) return fail(e);
    if ((e = hipMalloc(&tval, 8 * 2 * m)) != hipSuccess) return fail(e);
    if ((e = hipMalloc(&scol, 4 * 2 * m)) != hipSuccess) return fail(e);
    if ((e = hipMalloc(&sval, 8 * 2 * m)) != hipSuccess) return fail(e);
    if ((e = hipMemsetAsync(indeg, 0, 4 * n, s)) != hipSuccess) return fail(e);
    if ((e = hipMemsetAsync(fill, 0, 4 * n, s)) != hipSuccess) return fail(e);
    k_indeg<<<dim3((unsigned)ceil_div(m, 256)), 256, 0, s>>>(idx, m, indeg);
    k_row_caps<<<dim3((unsigned)ceil_div(n + 1, 256)), 256, 0, s>>>(indeg, n, k, cap);
    if ((e = scan_i64_local(cap, n + 1, off, tmp, s)) != hipSuccess) return fail(e);
    k_sym_fill<<<dim3((unsigned)ceil_div(m, 256)), 256, 0, s>>>(idx, Pc, n, k, off, fill, tcol, tval);
    k_sym_row<<<dim3((unsigned)n), 256, 0, s>>>(off, tcol, tval, scol, sval, ucnt);
    if ((e = hipMemsetAsync(ucnt + n, 0, 8, s)) != hipSuccess) return fail(e);
    if ((e = scan_i64_local(ucnt, n + 1, rp, tmp, s)) != hipSuccess) return fail(e);
    int64_t nnz = 0;
    if ((e = hipMemcpyAsync(&nnz, rp + n, 8, hipMemcpyDeviceToHost, s)) != hipSuccess) return fail(e);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e);
    if ((e = hipMalloc(&col, 4 * (nnz > 0 ? nnz : 1))) != hipSuccess) return fail(e);
    if ((e = hipMalloc(&val, 8 * (nnz > 0 ? nnz : 1))) != hipSuccess) return fail(e);
    k_sym_write<<<dim3((unsigned)n), 256, 0, s>>>(off, rp, tcol, tval, col, val,
                                                  1.0 / (2.0 * (double)n));
    if ((e = hipGetLastError()) != hipSuccess) return fail(e);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e);
    cleanup();
    *row_ptr_out = rp;
    *col_out = col;
    *val_out = val;
    *nnz_out = nnz;
    return hipSuccess;
}

}  // namespace psne
