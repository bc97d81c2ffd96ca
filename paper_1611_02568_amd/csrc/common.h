// Shared device-side definitions of the gfx950 PixelSNE library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pixelsne.h"

namespace psne {

constexpr int kWave = 64;
constexpr int kMaxLevels = 17;          // L <= 16 (r <= 65536): levels 0..16
// The data-driven tree (Barnes-Hut-SNE's D-Quadtree) splits down to single
// points on a 2^32 x 2^32 grid over the screen: levels 0..32, 64-bit keys.
constexpr int kDLevels = 32;
constexpr int kMaxLevelsAll = kDLevels + 1;

// Row chunks of the attraction pass: at most kChunkRows rows; a chunk of more
// than one row holds fewer than kChunkMaxNnz nonzeros.  Columns are packed
// with the row-in-chunk into one word, so n < 2^kColBits.
constexpr int kChunkRows = 32;
constexpr int kChunkMaxNnz = 16384;
constexpr int kColBits = 27;

// Scalars that live on the device so that an iteration needs no host round
// trip.  All FP64.
struct DevScalars {
    double s[2];        // y units per pixel of the current (normalised) frame
    double zmin[2];     // pending screen scaling: z = (zh - zmin) * scale
    double scale[2];    // r / gamma of the pending scaling
    double uscale[2];   // factor applied to the stored velocity before its next use
    double Z;           // Barnes-Hut normaliser of the last gradient
    int32_t t;          // iterations done
    int32_t nonfinite;  // set when a non-finite position appears
    int64_t n_nodes;    // occupied cells of the last tree
    int64_t n_chunks;   // row chunks of the attraction's copy of P
    uint32_t att_next;  // the attraction's work queue: next row chunk to take
    int32_t fork_late;  // this iteration's row sums start after the cells (else after snap)
    uint64_t t_begin;   // wall clock (device ticks) when the second stream's first launch starts
    float fork_ticks[2]; // moving average of the iteration time with each fork point
                         // (ticks); 0: not measured yet
    int32_t fork_count; // iterations since the last probe; < 0: probing (-left)
    int32_t fork_gap;   // iterations from one probe to the next
    uint32_t level_size[kMaxLevelsAll];
    uint32_t level_base[kMaxLevelsAll + 1];
};

// The fork-point tuner (PSNE_FORK_AUTO): iterations between two probes of
// the other fork point (the bounds of the gap), iterations per probe, and the
// weight of a new time in a fork point's moving average.
constexpr int kForkGapMin = 16;
constexpr int kForkGapMax = 64;
constexpr int kForkProbeLen = 2;
constexpr float kForkWeight = 0.25f;

// The fork-point tuner's starting state: the automatic choice starts after
// the cells, the better point while the layout is compressed.
inline void reset_fork_tuner(DevScalars& h, int32_t fork) {
    h.fork_late = fork != PSNE_FORK_SNAP;
    h.fork_ticks[0] = h.fork_ticks[1] = 0.f;
    h.fork_count = 0;
    h.fork_gap = kForkGapMin;
    h.t_begin = 0;
}

// One quadtree cell as the traversal reads it (32 bytes, one scalar load).
// child: index of the first child cell | (number of children - 1) << 30.
struct alignas(32) Node {
    double cx, cy;      // representative point: centre of mass or cell centre
    uint32_t count;     // points in the cell
    uint32_t child;
    uint32_t start;     // first sorted position of the cell
    uint32_t level;
};

// The traversal's copy of a cell for the FP32 path (16 bytes): the
// representative point rounded to FP32 and multiplied by the axis scale of
// cell_scale (so that the beta-weighted squared distance is a plain sum of
// squares), the point count rounded to FP32 (the mass the FP32 force terms
// use), and child as in Node.
struct alignas(16) CellF {
    float cx, cy;
    float mass;
    uint32_t child;
};

// The FP32 traversal's scale of axis d: sqrt(beta_d) rounded to FP32, with
// beta_d = s_d^2 the Eq. (12) metric weight of the current frame.
__device__ __forceinline__ float cell_scale(double s) { return (float)sqrt(s * s); }

template <typename T> struct V2;
template <> struct V2<float> { using type = float2; };
template <> struct V2<double> { using type = double2; };
template <typename T> using v2_t = typename V2<T>::type;

__device__ __forceinline__ uint32_t spread_bits16(uint32_t x) {
    x &= 0xFFFFu;
    x = (x | (x << 8)) & 0x00FF00FFu;
    x = (x | (x << 4)) & 0x0F0F0F0Fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}

__device__ __forceinline__ uint32_t gather_bits16(uint32_t x) {
    x &= 0x55555555u;
    x = (x | (x >> 1)) & 0x33333333u;
    x = (x | (x >> 2)) & 0x0F0F0F0Fu;
    x = (x | (x >> 4)) & 0x00FF00FFu;
    x = (x | (x >> 8)) & 0x0000FFFFu;
    return x;
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ uint64_t ballot64(bool p) { return __builtin_amdgcn_ballot_w64(p); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) { T w = __shfl_xor(v, o, kWave); v = w < v ? w : v; }
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) { T w = __shfl_xor(v, o, kWave); v = w > v ? w : v; }
    return v;
}

// largest value of T below r (positions are kept in [0, r))
template <typename T> __device__ __forceinline__ T top_below(int r);
template <> __device__ __forceinline__ float top_below<float>(int r) {
    return __int_as_float(__float_as_int((float)r) - 1);
}
template <> __device__ __forceinline__ double top_below<double>(int r) {
    return __longlong_as_double(__double_as_longlong((double)r) - 1);
}

// normalised position of point i: the pending screen scaling applied to zh
// (same arithmetic as the snap pass)
template <typename T>
__device__ __forceinline__ v2_t<T> norm_pos(const T* __restrict__ zh,
                                            const DevScalars* __restrict__ sc, int64_t i, int r) {
    using V = v2_t<T>;
    const T top = top_below<T>(r);
    const V p = reinterpret_cast<const V*>(zh)[i];
    T zx = (p.x - (T)sc->zmin[0]) * (T)sc->scale[0];
    T zy = (p.y - (T)sc->zmin[1]) * (T)sc->scale[1];
    zx = zx < T(0) ? T(0) : (zx > top ? top : zx);
    zy = zy < T(0) ? T(0) : (zy > top ? top : zy);
    return V{zx, zy};
}

// 1 / x for x >= 1: the hardware estimate refined by two Newton-Raphson steps
// r <- r + r (1 - x r), each roughly squaring the relative error, which ends
// within an ulp or two of the correctly rounded quotient
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// SplitMix64 (Steele, Lea & Flood 2014): the counter-based generator of the
// generated initial embeddings
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace psne
