// Learned placement network on gfx950: Linear-GELU-Linear-GELU-Linear(2),
// trained with the mean squared error against screen positions z / r of a
// converged embedding.  Matrix products use bfloat16 operands on the MFMA
// units (v_mfma_f32_16x16x32_bf16) with FP32 accumulation; master weights and
// Adam moments are FP32.  The 2-wide output layer runs on the vector units.
//
// Cast points (operands rounded to bfloat16, round to nearest even):
//   forward   X^, W1 | H1, W2 | H2, W3
//   backward  dA2, H1, W2 (dW2, dH1) and dA1, X^ (dW1); the head uses H2, W3.
#include <math.h>
#include <string.h>

#include <random>
#include <string>
#include <vector>

#include "ctx.h"

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

struct pixelsne_mlp {
    int32_t d = 0, h1 = 0, h2 = 0;
    int64_t n_params = 0;
    hipStream_t stream = nullptr;
    uint64_t seed = 0;
    int64_t step = 0;                   // Adam step count
    int64_t cap_batch = 0;              // rows the work buffers hold
    float* theta = nullptr;             // FP32 master parameters (flat)
    float* grad = nullptr;              // FP32 gradient (flat, same layout)
    float* m1 = nullptr;                // Adam first moment
    float* m2 = nullptr;                // Adam second moment
    uint16_t* w1b = nullptr;            // bfloat16 copies of W1, W2, W3
    uint16_t* w2b = nullptr;
    uint16_t* w3b = nullptr;
    float* mean = nullptr;              // input standardisation
    float* inv_std = nullptr;
    // per-batch work buffers
    uint16_t* xb = nullptr;             // X^ [B][d] bf16
    float* yb = nullptr;                // targets [B][2]
    float* a1 = nullptr;                // pre-activations [B][h1], [B][h2]
    float* a2 = nullptr;
    uint16_t* h1b = nullptr;            // activations (bf16) [B][h1], [B][h2]
    uint16_t* h2b = nullptr;
    float* out = nullptr;               // [B][2]
    float* dout = nullptr;              // [B][2]
    float* da2 = nullptr;               // [B][h2]
    uint16_t* da2b = nullptr;
    float* da1 = nullptr;               // [B][h1]
    uint16_t* da1b = nullptr;
    float* splitk = nullptr;            // split-K partials
    int64_t splitk_len = 0;
    float* part = nullptr;              // row-slice partial sums of the batch reductions
    double* lossbuf = nullptr;          // per-block loss partials
    int64_t lossbuf_len = 0;
    uint32_t* order = nullptr;          // batch row order (device)
    int64_t order_len = 0;
    std::vector<void*> allocs;
};

namespace psne {
namespace {

constexpr int kT = 256;

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) +
           x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

enum { EPI_F32 = 0, EPI_BIAS_GELU = 1, EPI_GELU_GRAD = 2 };

// Stage rows r0..r0+63, k0..k0+31 of an operand into S[row][k] (k < ke, row
// < R zero-filled beyond).  kmaj: stored [row][ld] with k contiguous;
// otherwise stored [k][ld] with rows contiguous.  Thread t moves 8 elements,
// with one 16-byte load when the run is inside the matrix and aligned.
__device__ __forceinline__ void load_tile(const uint16_t* __restrict__ G, int ld, int kmaj,
                                          int r0, int R, int k0, int ke, int t,
                                          uint16_t (*S)[40]) {
    union {
        uint4 q;
        uint16_t h[8];
    } v;
    if (kmaj) {
        const int r = t >> 2, c = (t & 3) * 8;                 // row r, k c..c+7
        const int gr = r0 + r, gk = k0 + c;
        const uint16_t* p = G + (int64_t)gr * ld + gk;
        if (gr < R && gk + 8 <= ke && ((reinterpret_cast<uintptr_t>(p) & 15u) == 0)) {
            v.q = *reinterpret_cast<const uint4*>(p);
        } else {
#pragma unroll
            for (int e = 0; e < 8; e++) v.h[e] = (gr < R && gk + e < ke) ? p[e] : (uint16_t)0;
        }
        *reinterpret_cast<uint4*>(&S[r][c]) = v.q;
    } else {
        const int k = t >> 3, c = (t & 7) * 8;                 // k, rows c..c+7
        const int gk = k0 + k, gr = r0 + c;
        const uint16_t* p = G + (int64_t)gk * ld + gr;
        if (gk < ke && gr + 8 <= R && ((reinterpret_cast<uintptr_t>(p) & 15u) == 0)) {
            v.q = *reinterpret_cast<const uint4*>(p);
        } else {
#pragma unroll
            for (int e = 0; e < 8; e++) v.h[e] = (gk < ke && gr + e < R) ? p[e] : (uint16_t)0;
        }
#pragma unroll
        for (int e = 0; e < 8; e++) S[c + e][k] = v.h[e];
    }
}

// C[M,N] = op(A)[M,K] * op(B)[K,N], bfloat16 operands, FP32 accumulate.
// ta: A stored [K][lda] (transposed); tb: B stored [N][ldb] (transposed).
// 64 x 64 tile per block, four wavefronts of 32 x 32 (2 x 2 MFMA tiles),
// K in steps of 32 staged through LDS as [row][k].  With gridDim.z > 1 each
// z-slice reduces its own K range into C + z*M*N (split-K, FP32 only).
template <int EPI>
__global__ __launch_bounds__(kT) void k_gemm_bf16(const uint16_t* __restrict__ A, int lda, int ta,
                                                  const uint16_t* __restrict__ B, int ldb, int tb,
                                                  int M, int N, int K, int kchunk,
                                                  float* __restrict__ C, int ldc,
                                                  const float* __restrict__ bias,
                                                  const float* __restrict__ pre,
                                                  uint16_t* __restrict__ Cb) {
    __shared__ uint16_t As[64][40];
    __shared__ uint16_t Bs[64][40];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int kb = blockIdx.z * kchunk;
    const int ke = kb + kchunk < K ? kb + kchunk : K;
    v4f acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int k0 = kb; k0 < ke; k0 += 32) {
        __syncthreads();
        // 64 x 32 elements per operand and step: one run of 8 consecutive
        // elements (16 bytes) per thread, along k for an operand stored with k
        // contiguous and along m (n) for a transposed one
        load_tile(A, lda, !ta, m0, M, k0, ke, t, As);
        load_tile(B, ldb, tb, n0, N, k0, ke, t, Bs);
        __syncthreads();
        v8bf af[2], bfr[2];
#pragma unroll
        for (int i = 0; i < 2; i++)
            af[i] = *reinterpret_cast<const v8bf*>(&As[32 * wm + 16 * i + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
        for (int j = 0; j < 2; j++)
            bfr[j] = *reinterpret_cast<const v8bf*>(&Bs[32 * wn + 16 * j + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
            for (int j = 0; j < 2; j++)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }
    float* Cz = C + (int64_t)blockIdx.z * M * ldc;
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int row = m0 + 32 * wm + 16 * i + 4 * (lane >> 4) + e;
                const int col = n0 + 32 * wn + 16 * j + (lane & 15);
                if (row >= M || col >= N) continue;
                const float v = acc[i][j][e];
                const int64_t o = (int64_t)row * ldc + col;
                if (EPI == EPI_F32) {
                    Cz[o] = v;
                } else if (EPI == EPI_BIAS_GELU) {
                    const float a = v + bias[col];
                    C[o] = a;
                    Cb[o] = f2bf(gelu_f(a));
                } else {
                    const float d = v * gelu_grad_f(pre[o]);
                    C[o] = d;
                    Cb[o] = f2bf(d);
                }
            }
}

// sum the split-K slices in slice order
__global__ __launch_bounds__(kT) void k_splitk_sum(const float* __restrict__ part, int64_t mn,
                                                   int S, float* __restrict__ C) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= mn) return;
    float a = 0.f;
    for (int z = 0; z < S; z++) a += part[(int64_t)z * mn + i];
    C[i] = a;
}

// X^ rows of a batch: gather by order, standardise, round to bfloat16
__global__ __launch_bounds__(kT) void k_stage_x(const float* __restrict__ X, int d,
                                                const uint32_t* __restrict__ order, int64_t b0,
                                                int Bn, const float* __restrict__ mean,
                                                const float* __restrict__ inv_std,
                                                uint16_t* __restrict__ xb,
                                                const float* __restrict__ Y, float* __restrict__ yb) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= (int64_t)Bn * d) return;
    const int64_t r = i / d;
    const int c = (int)(i - r * d);
    const int64_t src = order ? order[b0 + r] : b0 + r;
    xb[i] = f2bf((X[src * d + c] - mean[c]) * inv_std[c]);
    if (Y && c == 0) {
        yb[r * 2] = Y[src * 2];
        yb[r * 2 + 1] = Y[src * 2 + 1];
    }
}

// head: out = H2 W3 + b3 (one wavefront per row), then dout and the loss
__global__ __launch_bounds__(kT) void k_head_fwd(const uint16_t* __restrict__ h2b, int h2,
                                                 const uint16_t* __restrict__ w3b,
                                                 const float* __restrict__ b3, int Bn,
                                                 float* __restrict__ out,
                                                 const float* __restrict__ yb,
                                                 float* __restrict__ dout,
                                                 double* __restrict__ lossp) {
    __shared__ double red[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = blockIdx.x * 4 + w;
    double l = 0.0;
    if (r < Bn) {
        float s0 = 0.f, s1 = 0.f;
        for (int j = lane; j < h2; j += 64) {
            const float h = bf2f(h2b[(int64_t)r * h2 + j]);
            s0 += h * bf2f(w3b[2 * j]);
            s1 += h * bf2f(w3b[2 * j + 1]);
        }
        s0 = psne::wave_sum(s0);
        s1 = psne::wave_sum(s1);
        if (lane == 0) {
            const float o0 = s0 + b3[0], o1 = s1 + b3[1];
            out[2 * r] = o0;
            out[2 * r + 1] = o1;
            if (yb) {
                const float e0 = o0 - yb[2 * r], e1 = o1 - yb[2 * r + 1];
                dout[2 * r] = 2.f * e0 / (float)Bn;
                dout[2 * r + 1] = 2.f * e1 / (float)Bn;
                l = (double)e0 * e0 + (double)e1 * e1;
            }
        }
    }
    if (lane == 0) red[w] = l;
    __syncthreads();
    if (threadIdx.x == 0 && lossp) lossp[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// dW3[j][d] = sum_b H2[b][j] dout[b][d];  db3[d] = sum_b dout[b][d]
// Batch reductions are split into kSlices row slices: block (x, z) sums its
// slice for 64 columns (4 row phases x 64 columns, then the phases in order)
// into part[z][...]; k_sum_slices adds the slices in slice order.
constexpr int kSlices = 32;

// dW3[j][c] = sum_b H2[b][j] dout[b][c]; columns j < h2 give 2 outputs each,
// and block x == 0 also sums dout itself (db3) into part[z][2 h2 + c]
__global__ __launch_bounds__(kT) void k_head_wgrad_part(const uint16_t* __restrict__ h2b, int h2,
                                                        const float* __restrict__ dout, int Bn,
                                                        float* __restrict__ part) {
    __shared__ float red[4][64][3];
    const int t = threadIdx.x, cj = t & 63, ph = t >> 6;
    const int j = blockIdx.x * 64 + cj;
    const int per = (Bn + kSlices - 1) / kSlices;
    const int b0 = blockIdx.z * per, b1 = b0 + per < Bn ? b0 + per : Bn;
    float s0 = 0.f, s1 = 0.f, d0 = 0.f, d1 = 0.f;
    for (int b = b0 + ph; b < b1; b += 4) {
        const float o0 = dout[2 * b], o1 = dout[2 * b + 1];
        if (j < h2) {
            const float h = bf2f(h2b[(int64_t)b * h2 + j]);
            s0 += h * o0;
            s1 += h * o1;
        }
        d0 += o0;
        d1 += o1;
    }
    red[ph][cj][0] = s0;
    red[ph][cj][1] = s1;
    red[ph][cj][2] = cj == 0 ? d0 : (cj == 1 ? d1 : 0.f);
    __syncthreads();
    if (ph == 0) {
        const float a0 = ((red[0][cj][0] + red[1][cj][0]) + red[2][cj][0]) + red[3][cj][0];
        const float a1 = ((red[0][cj][1] + red[1][cj][1]) + red[2][cj][1]) + red[3][cj][1];
        float* p = part + (int64_t)blockIdx.z * (2 * h2 + 2);
        if (j < h2) {
            p[2 * j] = a0;
            p[2 * j + 1] = a1;
        }
        if (blockIdx.x == 0 && cj < 2)
            p[2 * h2 + cj] = ((red[0][cj][2] + red[1][cj][2]) + red[2][cj][2]) + red[3][cj][2];
    }
}

// dA2 = (dout W3^T) * GELU'(A2)
__global__ __launch_bounds__(kT) void k_head_bgrad(const float* __restrict__ dout,
                                                   const uint16_t* __restrict__ w3b,
                                                   const float* __restrict__ a2, int h2, int Bn,
                                                   float* __restrict__ da2,
                                                   uint16_t* __restrict__ da2b) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= (int64_t)Bn * h2) return;
    const int64_t b = i / h2;
    const int j = (int)(i - b * h2);
    const float g = dout[2 * b] * bf2f(w3b[2 * j]) + dout[2 * b + 1] * bf2f(w3b[2 * j + 1]);
    const float d = g * gelu_grad_f(a2[i]);
    da2[i] = d;
    da2b[i] = f2bf(d);
}

// column sums over the batch (bias gradients), per row slice
__global__ __launch_bounds__(kT) void k_colsum_part(const float* __restrict__ a, int rows, int cols,
                                                    float* __restrict__ part) {
    __shared__ float red[4][64];
    const int t = threadIdx.x, cj = t & 63, ph = t >> 6;
    const int j = blockIdx.x * 64 + cj;
    const int per = (rows + kSlices - 1) / kSlices;
    const int b0 = blockIdx.z * per, b1 = b0 + per < rows ? b0 + per : rows;
    float s = 0.f;
    if (j < cols)
        for (int b = b0 + ph; b < b1; b += 4) s += a[(int64_t)b * cols + j];
    red[ph][cj] = s;
    __syncthreads();
    if (ph == 0 && j < cols)
        part[(int64_t)blockIdx.z * cols + j] = ((red[0][cj] + red[1][cj]) + red[2][cj]) + red[3][cj];
}

__global__ __launch_bounds__(kT) void k_sum_slices(const float* __restrict__ part, int m,
                                                   float* __restrict__ out) {
    const int i = blockIdx.x * kT + threadIdx.x;
    if (i >= m) return;
    float s = 0.f;
    for (int z = 0; z < kSlices; z++) s += part[(int64_t)z * m + i];
    out[i] = s;
}

__global__ __launch_bounds__(kT) void k_adam(float* __restrict__ th, const float* __restrict__ g,
                                             float* __restrict__ m1, float* __restrict__ m2,
                                             int64_t np, float lr, float b1, float b2, float eps,
                                             float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= np) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = v;
    th[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

__global__ __launch_bounds__(kT) void k_to_bf16(const float* __restrict__ a, int64_t m,
                                                uint16_t* __restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < m) b[i] = f2bf(a[i]);
}

// per-feature mean and 1/std over n rows, FP64 accumulation (one block per feature)
__global__ __launch_bounds__(kT) void k_feature_stats(const float* __restrict__ X, int64_t n, int d,
                                                      float* __restrict__ mean,
                                                      float* __restrict__ inv_std) {
    __shared__ double r1[kT], r2[kT];
    const int c = blockIdx.x;
    double s = 0.0, q = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kT) {
        const double v = X[i * d + c];
        s += v;
        q += v * v;
    }
    r1[threadIdx.x] = s;
    r2[threadIdx.x] = q;
    __syncthreads();
    for (int o = kT / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            r1[threadIdx.x] += r1[threadIdx.x + o];
            r2[threadIdx.x] += r2[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mu = r1[0] / (double)n;
        double var = r2[0] / (double)n - mu * mu;
        if (!(var > 0.0)) var = 1.0;
        mean[c] = (float)mu;
        inv_std[c] = (float)(1.0 / sqrt(var));
    }
}

// placed embedding: y = clamp(out, 0, 1 - 2^-24) * r * s  (double [n][2])
__global__ __launch_bounds__(kT) void k_place(const float* __restrict__ out, int64_t n, double r,
                                              double sx, double sy, double* __restrict__ Y) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    const double top = 1.0 - 0x1.0p-24;
    double a = (double)out[2 * i], b = (double)out[2 * i + 1];
    a = a < 0.0 ? 0.0 : (a > top ? top : a);
    b = b < 0.0 ? 0.0 : (b > top ? top : b);
    Y[2 * i] = a * r * sx;
    Y[2 * i + 1] = b * r * sy;
}

inline dim3 g1(int64_t n) { return dim3((unsigned)ceil_div(n > 0 ? n : 1, kT)); }

template <typename P>
hipError_t mal(pixelsne_mlp* m, P** p, size_t bytes) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, bytes ? bytes : 1);
    if (e != hipSuccess) return e;
    m->allocs.push_back(q);
    *p = (P*)q;
    return hipSuccess;
}

int64_t off_W1(const pixelsne_mlp*) { return 0; }
int64_t off_b1(const pixelsne_mlp* m) { return (int64_t)m->d * m->h1; }
int64_t off_W2(const pixelsne_mlp* m) { return off_b1(m) + m->h1; }
int64_t off_b2(const pixelsne_mlp* m) { return off_W2(m) + (int64_t)m->h1 * m->h2; }
int64_t off_W3(const pixelsne_mlp* m) { return off_b2(m) + m->h2; }
int64_t off_b3(const pixelsne_mlp* m) { return off_W3(m) + (int64_t)m->h2 * 2; }

hipError_t ensure_batch(pixelsne_mlp* m, int64_t B) {
    if (B <= m->cap_batch) return hipSuccess;
    hipError_t e;
    const int64_t h = m->h1 > m->h2 ? m->h1 : m->h2;
    if ((e = mal(m, &m->xb, 2 * B * m->d)) != hipSuccess) return e;
    if ((e = mal(m, &m->yb, 4 * B * 2)) != hipSuccess) return e;
    if ((e = mal(m, &m->a1, 4 * B * m->h1)) != hipSuccess) return e;
    if ((e = mal(m, &m->a2, 4 * B * m->h2)) != hipSuccess) return e;
    if ((e = mal(m, &m->h1b, 2 * B * m->h1)) != hipSuccess) return e;
    if ((e = mal(m, &m->h2b, 2 * B * m->h2)) != hipSuccess) return e;
    if ((e = mal(m, &m->out, 4 * B * 2)) != hipSuccess) return e;
    if ((e = mal(m, &m->dout, 4 * B * 2)) != hipSuccess) return e;
    if ((e = mal(m, &m->da2, 4 * B * m->h2)) != hipSuccess) return e;
    if ((e = mal(m, &m->da2b, 2 * B * m->h2)) != hipSuccess) return e;
    if ((e = mal(m, &m->da1, 4 * B * m->h1)) != hipSuccess) return e;
    if ((e = mal(m, &m->da1b, 2 * B * m->h1)) != hipSuccess) return e;
    m->lossbuf_len = ceil_div(B, 4);
    if ((e = mal(m, &m->lossbuf, 8 * m->lossbuf_len)) != hipSuccess) return e;
    if (!m->part && (e = mal(m, &m->part, 4 * (size_t)kSlices * (2 * h + 2))) != hipSuccess) return e;
    m->cap_batch = B;
    return hipSuccess;
}

int splits_for(int64_t K) {
    int s = (int)(K / 512);
    return s < 1 ? 1 : (s > 16 ? 16 : s);
}

hipError_t gemm(pixelsne_mlp* m, int epi, const uint16_t* A, int lda, int ta, const uint16_t* B,
                int ldb, int tb, int M, int N, int K, float* C, const float* bias,
                const float* pre, uint16_t* Cb) {
    dim3 grid((unsigned)ceil_div(N, 64), (unsigned)ceil_div(M, 64), 1);
    if (epi == EPI_F32) {
        const int S = splits_for(K);
        if (S > 1) {
            const int64_t need = (int64_t)S * M * N;
            if (need > m->splitk_len) {
                hipError_t e = mal(m, &m->splitk, 4 * need);
                if (e != hipSuccess) return e;
                m->splitk_len = need;
            }
            const int kc = (int)ceil_div(ceil_div(K, S), 32) * 32;
            grid.z = (unsigned)ceil_div(K, kc);
            k_gemm_bf16<EPI_F32><<<grid, kT, 0, m->stream>>>(A, lda, ta, B, ldb, tb, M, N, K, kc,
                                                             m->splitk, N, nullptr, nullptr,
                                                             nullptr);
            k_splitk_sum<<<g1((int64_t)M * N), kT, 0, m->stream>>>(m->splitk, (int64_t)M * N,
                                                                  (int)grid.z, C);
            return hipGetLastError();
        }
        k_gemm_bf16<EPI_F32><<<grid, kT, 0, m->stream>>>(A, lda, ta, B, ldb, tb, M, N, K, K, C, N,
                                                         nullptr, nullptr, nullptr);
    } else if (epi == EPI_BIAS_GELU) {
        k_gemm_bf16<EPI_BIAS_GELU><<<grid, kT, 0, m->stream>>>(A, lda, ta, B, ldb, tb, M, N, K, K,
                                                               C, N, bias, nullptr, Cb);
    } else {
        k_gemm_bf16<EPI_GELU_GRAD><<<grid, kT, 0, m->stream>>>(A, lda, ta, B, ldb, tb, M, N, K, K,
                                                               C, N, nullptr, pre, Cb);
    }
    return hipGetLastError();
}

// forward of staged rows xb[0..Bn) -> out (and, with targets, dout + loss partials)
hipError_t forward_batch(pixelsne_mlp* m, int Bn, bool with_targets) {
    hipError_t e;
    if ((e = gemm(m, EPI_BIAS_GELU, m->xb, m->d, 0, m->w1b, m->h1, 0, Bn, m->h1, m->d, m->a1,
                  m->theta + off_b1(m), nullptr, m->h1b)) != hipSuccess)
        return e;
    if ((e = gemm(m, EPI_BIAS_GELU, m->h1b, m->h1, 0, m->w2b, m->h2, 0, Bn, m->h2, m->h1, m->a2,
                  m->theta + off_b2(m), nullptr, m->h2b)) != hipSuccess)
        return e;
    k_head_fwd<<<dim3((unsigned)ceil_div(Bn, 4)), kT, 0, m->stream>>>(
        m->h2b, m->h2, m->w3b, m->theta + off_b3(m), Bn, m->out, with_targets ? m->yb : nullptr,
        m->dout, with_targets ? m->lossbuf : nullptr);
    return hipGetLastError();
}

hipError_t backward_batch(pixelsne_mlp* m, int Bn) {
    hipError_t e;
    float* g = m->grad;
    // dW3 and db3 are adjacent in the flat gradient: 2 h2 + 2 values
    k_head_wgrad_part<<<dim3((unsigned)ceil_div(m->h2, 64), 1, kSlices), kT, 0, m->stream>>>(
        m->h2b, m->h2, m->dout, Bn, m->part);
    k_sum_slices<<<g1(2 * m->h2 + 2), kT, 0, m->stream>>>(m->part, 2 * m->h2 + 2, g + off_W3(m));
    k_head_bgrad<<<g1((int64_t)Bn * m->h2), kT, 0, m->stream>>>(m->dout, m->w3b, m->a2, m->h2, Bn,
                                                               m->da2, m->da2b);
    k_colsum_part<<<dim3((unsigned)ceil_div(m->h2, 64), 1, kSlices), kT, 0, m->stream>>>(
        m->da2, Bn, m->h2, m->part);
    k_sum_slices<<<g1(m->h2), kT, 0, m->stream>>>(m->part, m->h2, g + off_b2(m));
    // dW2 = H1^T dA2 : A = H1 stored [B][h1] (transposed), B = dA2 [B][h2]
    if ((e = gemm(m, EPI_F32, m->h1b, m->h1, 1, m->da2b, m->h2, 0, m->h1, m->h2, Bn,
                  g + off_W2(m), nullptr, nullptr, nullptr)) != hipSuccess)
        return e;
    // dA1 = (dA2 W2^T) * GELU'(A1) : B = W2 stored [h1][h2] = [N][K] (transposed)
    if ((e = gemm(m, EPI_GELU_GRAD, m->da2b, m->h2, 0, m->w2b, m->h2, 1, Bn, m->h1, m->h2, m->da1,
                  nullptr, m->a1, m->da1b)) != hipSuccess)
        return e;
    k_colsum_part<<<dim3((unsigned)ceil_div(m->h1, 64), 1, kSlices), kT, 0, m->stream>>>(
        m->da1, Bn, m->h1, m->part);
    k_sum_slices<<<g1(m->h1), kT, 0, m->stream>>>(m->part, m->h1, g + off_b1(m));
    // dW1 = X^T dA1
    return gemm(m, EPI_F32, m->xb, m->d, 1, m->da1b, m->h1, 0, m->d, m->h1, Bn, g + off_W1(m),
                nullptr, nullptr, nullptr);
}

hipError_t refresh_bf16(pixelsne_mlp* m) {
    k_to_bf16<<<g1((int64_t)m->d * m->h1), kT, 0, m->stream>>>(m->theta + off_W1(m),
                                                              (int64_t)m->d * m->h1, m->w1b);
    k_to_bf16<<<g1((int64_t)m->h1 * m->h2), kT, 0, m->stream>>>(m->theta + off_W2(m),
                                                               (int64_t)m->h1 * m->h2, m->w2b);
    k_to_bf16<<<g1((int64_t)m->h2 * 2), kT, 0, m->stream>>>(m->theta + off_W3(m),
                                                           (int64_t)m->h2 * 2, m->w3b);
    return hipGetLastError();
}

// One Adam step (Kingma & Ba, 2015; beta 0.9 / 0.999, eps 1e-8, bias-corrected)
// on the master weights with gradient g, then the bfloat16 weight copies.
hipError_t adam_update(pixelsne_mlp* m, const float* g, float lr) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    m->step++;
    const float c1 = 1.f - powf(b1, (float)m->step), c2 = 1.f - powf(b2, (float)m->step);
    k_adam<<<g1(m->n_params), kT, 0, m->stream>>>(m->theta, g, m->m1, m->m2, m->n_params, lr, b1,
                                                 b2, eps, c1, c2);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? refresh_bf16(m) : e;
}

psne_status mlp_error(hipError_t e, const char* where) {
    set_error(std::string(where) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? PSNE_E_NOMEM : PSNE_E_DEVICE;
}

bool dev_ptr(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

}  // namespace
}  // namespace psne

using namespace psne;

extern "C" {

psne_status pixelsne_mlp_forward(pixelsne_mlp* m, const float* X, int64_t n, float* Y01_out);

pixelsne_mlp* pixelsne_mlp_create(int32_t d_in, int32_t h1, int32_t h2, uint64_t seed,
                                  void* stream) {
    if (d_in < 1 || h1 < 1 || h2 < 1 || d_in > 65536 || h1 > 65536 || h2 > 65536) {
        set_error("MLP sizes must be in [1, 65536]");
        return nullptr;
    }
    pixelsne_mlp* m = new pixelsne_mlp();
    m->d = d_in;
    m->h1 = h1;
    m->h2 = h2;
    m->seed = seed;
    m->stream = (hipStream_t)stream;
    m->n_params = (int64_t)d_in * h1 + h1 + (int64_t)h1 * h2 + h2 + (int64_t)h2 * 2 + 2;
    hipError_t e = mal(m, &m->theta, 4 * m->n_params);
    if (e == hipSuccess) e = mal(m, &m->grad, 4 * m->n_params);
    if (e == hipSuccess) e = mal(m, &m->m1, 4 * m->n_params);
    if (e == hipSuccess) e = mal(m, &m->m2, 4 * m->n_params);
    if (e == hipSuccess) e = mal(m, &m->w1b, 2 * (size_t)d_in * h1);
    if (e == hipSuccess) e = mal(m, &m->w2b, 2 * (size_t)h1 * h2);
    if (e == hipSuccess) e = mal(m, &m->w3b, 2 * (size_t)h2 * 2);
    if (e == hipSuccess) e = mal(m, &m->mean, 4 * (size_t)d_in);
    if (e == hipSuccess) e = mal(m, &m->inv_std, 4 * (size_t)d_in);
    if (e != hipSuccess) {
        mlp_error(e, "mlp_create");
        pixelsne_mlp_destroy(m);
        return nullptr;
    }
    // He-style initialisation from a seeded host generator, zero biases
    std::vector<float> th(m->n_params, 0.f);
    std::mt19937_64 rng(seed);
    std::normal_distribution<float> nd(0.f, 1.f);
    auto fill = [&](int64_t off, int64_t rows, int64_t cols) {
        const float sc = sqrtf(2.f / (float)rows);
        for (int64_t i = 0; i < rows * cols; i++) th[off + i] = nd(rng) * sc;
    };
    fill(off_W1(m), d_in, h1);
    fill(off_W2(m), h1, h2);
    fill(off_W3(m), h2, 2);
    std::vector<float> ones(d_in, 1.f), zeros(d_in, 0.f);
    e = hipMemcpyAsync(m->theta, th.data(), 4 * m->n_params, hipMemcpyHostToDevice, m->stream);
    if (e == hipSuccess) e = hipMemsetAsync(m->m1, 0, 4 * m->n_params, m->stream);
    if (e == hipSuccess) e = hipMemsetAsync(m->m2, 0, 4 * m->n_params, m->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(m->mean, zeros.data(), 4 * d_in, hipMemcpyHostToDevice, m->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(m->inv_std, ones.data(), 4 * d_in, hipMemcpyHostToDevice, m->stream);
    if (e == hipSuccess) e = refresh_bf16(m);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) {
        mlp_error(e, "mlp_create");
        pixelsne_mlp_destroy(m);
        return nullptr;
    }
    return m;
}

void pixelsne_mlp_destroy(pixelsne_mlp* m) {
    if (!m) return;
    (void)hipStreamSynchronize(m->stream);
    for (void* p : m->allocs) (void)hipFree(p);
    delete m;
}

int64_t pixelsne_mlp_num_params(const pixelsne_mlp* m) { return m ? m->n_params : -1; }

psne_status pixelsne_mlp_set_params(pixelsne_mlp* m, const float* theta) {
    if (!m || !dev_ptr(theta)) { set_error("mlp_set_params: null mlp or non-device theta"); return PSNE_E_INVAL; }
    hipError_t e = hipMemcpyAsync(m->theta, theta, 4 * m->n_params, hipMemcpyDeviceToDevice, m->stream);
    if (e == hipSuccess) e = refresh_bf16(m);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    return e == hipSuccess ? PSNE_OK : mlp_error(e, "mlp_set_params");
}

psne_status pixelsne_mlp_get_params(const pixelsne_mlp* m, float* theta) {
    if (!m || !dev_ptr(theta)) { set_error("mlp_get_params: null mlp or non-device theta"); return PSNE_E_INVAL; }
    hipError_t e = hipMemcpyAsync(theta, m->theta, 4 * m->n_params, hipMemcpyDeviceToDevice, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    return e == hipSuccess ? PSNE_OK : mlp_error(e, "mlp_get_params");
}

psne_status pixelsne_mlp_set_norm(pixelsne_mlp* m, const float* mean, const float* inv_std) {
    if (!m || !dev_ptr(mean) || !dev_ptr(inv_std)) { set_error("mlp_set_norm: bad arguments"); return PSNE_E_INVAL; }
    hipError_t e = hipMemcpyAsync(m->mean, mean, 4 * (size_t)m->d, hipMemcpyDeviceToDevice, m->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(m->inv_std, inv_std, 4 * (size_t)m->d, hipMemcpyDeviceToDevice, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    return e == hipSuccess ? PSNE_OK : mlp_error(e, "mlp_set_norm");
}

psne_status pixelsne_mlp_fit_norm(pixelsne_mlp* m, const float* X, int64_t n) {
    if (!m || !dev_ptr(X) || n < 1) { set_error("mlp_fit_norm: bad arguments"); return PSNE_E_INVAL; }
    k_feature_stats<<<dim3((unsigned)m->d), kT, 0, m->stream>>>(X, n, m->d, m->mean, m->inv_std);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    return e == hipSuccess ? PSNE_OK : mlp_error(e, "mlp_fit_norm");
}

psne_status pixelsne_mlp_grad(pixelsne_mlp* m, const float* X, const float* Y01, int64_t n,
                              float* grads_out, double* loss) {
    if (!m || !dev_ptr(X) || !dev_ptr(Y01) || n < 1 || n > (1 << 20)) {
        set_error("mlp_grad: bad arguments (n must be in [1, 2^20])");
        return PSNE_E_INVAL;
    }
    if (grads_out && !dev_ptr(grads_out)) { set_error("mlp_grad: grads_out must be a device pointer"); return PSNE_E_INVAL; }
    hipError_t e = ensure_batch(m, n);
    if (e != hipSuccess) return mlp_error(e, "mlp_grad");
    k_stage_x<<<g1(n * m->d), kT, 0, m->stream>>>(X, m->d, nullptr, 0, (int)n, m->mean, m->inv_std,
                                                  m->xb, Y01, m->yb);
    if ((e = forward_batch(m, (int)n, true)) == hipSuccess) e = backward_batch(m, (int)n);
    std::vector<double> lp(m->lossbuf_len);
    if (e == hipSuccess && grads_out)
        e = hipMemcpyAsync(grads_out, m->grad, 4 * m->n_params, hipMemcpyDeviceToDevice, m->stream);
    const int64_t nb = ceil_div(n, 4);
    if (e == hipSuccess)
        e = hipMemcpyAsync(lp.data(), m->lossbuf, 8 * nb, hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) return mlp_error(e, "mlp_grad");
    if (loss) {
        double s = 0.0;
        for (int64_t i = 0; i < nb; i++) s += lp[i];
        *loss = s / (double)n;
    }
    return PSNE_OK;
}

psne_status pixelsne_mlp_train(pixelsne_mlp* m, const float* X, const float* Y01, int64_t n,
                               int32_t epochs, int32_t batch, float lr, double* last_epoch_loss) {
    if (!m || !dev_ptr(X) || !dev_ptr(Y01) || n < 1 || epochs < 0 || batch < 1 ||
        batch > (1 << 20) || !(lr > 0.f)) {
        set_error("mlp_train: bad arguments");
        return PSNE_E_INVAL;
    }
    const int64_t B = batch < n ? batch : n;
    hipError_t e = ensure_batch(m, B);
    if (e == hipSuccess && m->order_len < n) {
        e = mal(m, &m->order, 4 * (size_t)n);
        m->order_len = n;
    }
    if (e != hipSuccess) return mlp_error(e, "mlp_train");
    std::vector<uint32_t> ord(n);
    for (int64_t i = 0; i < n; i++) ord[i] = (uint32_t)i;
    std::mt19937_64 rng(m->seed ^ 0x5DEECE66DULL);
    double epoch_loss = 0.0;
    for (int32_t ep = 0; ep < epochs; ep++) {
        std::shuffle(ord.begin(), ord.end(), rng);
        e = hipMemcpyAsync(m->order, ord.data(), 4 * (size_t)n, hipMemcpyHostToDevice, m->stream);
        if (e != hipSuccess) return mlp_error(e, "mlp_train");
        std::vector<double> lsum;
        const int64_t nbatch = n / B;            // full batches only
        std::vector<double> lp(m->lossbuf_len);
        double acc = 0.0;
        for (int64_t bi = 0; bi < nbatch && e == hipSuccess; bi++) {
            k_stage_x<<<g1(B * m->d), kT, 0, m->stream>>>(X, m->d, m->order, bi * B, (int)B,
                                                          m->mean, m->inv_std, m->xb, Y01, m->yb);
            e = forward_batch(m, (int)B, true);
            if (e == hipSuccess) e = backward_batch(m, (int)B);
            if (e == hipSuccess) e = adam_update(m, m->grad, lr);
            if (e == hipSuccess && ep == epochs - 1) {
                e = hipMemcpyAsync(lp.data(), m->lossbuf, 8 * ceil_div(B, 4), hipMemcpyDeviceToHost,
                                   m->stream);
                if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
                for (int64_t i = 0; i < ceil_div(B, 4); i++) acc += lp[i];
            }
        }
        if (ep == epochs - 1 && nbatch > 0) epoch_loss = acc / (double)(nbatch * B);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) return mlp_error(e, "mlp_train");
    if (last_epoch_loss) *last_epoch_loss = epoch_loss;
    return PSNE_OK;
}

psne_status pixelsne_mlp_adam_step(pixelsne_mlp* m, const float* grad, float lr) {
    if (!m || !dev_ptr(grad) || !(lr > 0.f)) {
        set_error("mlp_adam_step: bad arguments");
        return PSNE_E_INVAL;
    }
    hipError_t e = adam_update(m, grad, lr);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    return e == hipSuccess ? PSNE_OK : mlp_error(e, "mlp_adam_step");
}

psne_status pixelsne_mlp_place(pixelsne_mlp* m, const float* X, int64_t n, int32_t screen,
                               const double* s, double* Y_out) {
    if (!m || !dev_ptr(X) || !dev_ptr(Y_out) || n < 1 || screen < 2 || !s || !(s[0] > 0.0) ||
        !(s[1] > 0.0)) {
        set_error("mlp_place: bad arguments");
        return PSNE_E_INVAL;
    }
    float* tmp = nullptr;
    hipError_t e = hipMalloc(&tmp, 8 * (size_t)n);
    if (e != hipSuccess) return mlp_error(e, "mlp_place");
    psne_status st = pixelsne_mlp_forward(m, X, n, tmp);
    if (st == PSNE_OK) {
        k_place<<<g1(n), kT, 0, m->stream>>>(tmp, n, (double)screen, s[0], s[1], Y_out);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
        if (e != hipSuccess) st = mlp_error(e, "mlp_place");
    }
    (void)hipFree(tmp);
    return st;
}

psne_status pixelsne_mlp_forward(pixelsne_mlp* m, const float* X, int64_t n, float* Y01_out) {
    if (!m || !dev_ptr(X) || !dev_ptr(Y01_out) || n < 1) {
        set_error("mlp_forward: bad arguments");
        return PSNE_E_INVAL;
    }
    const int64_t B = n < 8192 ? n : 8192;
    hipError_t e = ensure_batch(m, B);
    for (int64_t b0 = 0; b0 < n && e == hipSuccess; b0 += B) {
        const int Bn = (int)(n - b0 < B ? n - b0 : B);
        k_stage_x<<<g1((int64_t)Bn * m->d), kT, 0, m->stream>>>(X, m->d, nullptr, b0, Bn, m->mean,
                                                                m->inv_std, m->xb, nullptr, nullptr);
        e = forward_batch(m, Bn, false);
        if (e == hipSuccess)
            e = hipMemcpyAsync(Y01_out + 2 * b0, m->out, 8 * (size_t)Bn, hipMemcpyDeviceToDevice,
                               m->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    return e == hipSuccess ? PSNE_OK : mlp_error(e, "mlp_forward");
}

}  // extern "C"
