// Embedding quality: the k nearest neighbours of every point in the 2-D
// embedding and the neighbourhood precision of Eq. (14),
//   (1 / kN) sum_i |N_D^(k)(i) intersect N_d^(k)(i)|,
// with N_D the high-dimensional neighbours (an input) and N_d the 2-D ones.
#include <string>
#include <vector>

#include "ctx.h"

namespace psne {

namespace {

constexpr int kB = 256;
constexpr int kK2 = 32;      // 2-D neighbours kept per point

__device__ __forceinline__ bool closer(double d, uint32_t j, double e, uint32_t k) {
    return d < e || (d == e && j < k);
}

// Brute-force 2-D kNN in the embedding metric d^2 = b1 dx^2 + b2 dy^2 (FP64,
// pixel frame), ties to the smaller caller index; writes the kK2 nearest as
// caller indices at the caller's row.
template <typename T>
__global__ __launch_bounds__(kB) void k_knn2d(const T* __restrict__ zh,
                                              const DevScalars* __restrict__ sc,
                                              const uint32_t* __restrict__ orig, int64_t n, int r,
                                              int32_t* __restrict__ out) {
    __shared__ double tx[kB], ty[kB];
    __shared__ uint32_t tu[kB];
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    const double s0 = sc->s[0], s1 = sc->s[1];
    const double b1 = s0 * s0, b2 = s1 * s1;
    double zx = 0.0, zy = 0.0;
    if (i < n) {
        const v2_t<T> p = norm_pos<T>(zh, sc, i, r);
        zx = (double)p.x;
        zy = (double)p.y;
    }
    double bd[kK2];
    uint32_t bj[kK2];
#pragma unroll
    for (int q = 0; q < kK2; q++) {
        bd[q] = INFINITY;
        bj[q] = 0xFFFFFFFFu;
    }
    for (int64_t j0 = 0; j0 < n; j0 += kB) {
        __syncthreads();
        const int64_t j = j0 + threadIdx.x;
        if (j < n) {
            const v2_t<T> p = norm_pos<T>(zh, sc, j, r);
            tx[threadIdx.x] = (double)p.x;
            ty[threadIdx.x] = (double)p.y;
            tu[threadIdx.x] = orig[j];
        }
        __syncthreads();
        const int m = n - j0 < kB ? (int)(n - j0) : kB;
        for (int q = 0; q < m; q++) {
            if (j0 + q == i) continue;
            const double dx = zx - tx[q], dy = zy - ty[q];
            const double d = b1 * dx * dx + b2 * dy * dy;
            const uint32_t u = tu[q];
            if (closer(d, u, bd[kK2 - 1], bj[kK2 - 1])) {
                bd[kK2 - 1] = d;
                bj[kK2 - 1] = u;
#pragma unroll
                for (int t = kK2 - 1; t > 0; t--) {
                    if (closer(bd[t], bj[t], bd[t - 1], bj[t - 1])) {
                        const double a = bd[t]; bd[t] = bd[t - 1]; bd[t - 1] = a;
                        const uint32_t b = bj[t]; bj[t] = bj[t - 1]; bj[t - 1] = b;
                    }
                }
            }
        }
    }
    if (i < n) {
        const int64_t o = (int64_t)orig[i] * kK2;
#pragma unroll
        for (int q = 0; q < kK2; q++) out[o + q] = (int32_t)bj[q];
    }
}

// per-point overlap counts for each requested k, summed per block
__global__ __launch_bounds__(kB) void k_overlap(const int32_t* __restrict__ hi, int k_hi,
                                                const int32_t* __restrict__ lo, int64_t n,
                                                const int32_t* __restrict__ ks, int nk,
                                                unsigned long long* __restrict__ part) {
    __shared__ unsigned long long red[kB];
    const int64_t u = (int64_t)blockIdx.x * kB + threadIdx.x;
    for (int q = 0; q < nk; q++) {
        const int k = ks[q];
        unsigned long long c = 0;
        if (u < n) {
            for (int a = 0; a < k; a++) {
                const int32_t h = hi[u * k_hi + a];
                for (int b = 0; b < k; b++) c += (lo[u * kK2 + b] == h) ? 1ull : 0ull;
            }
        }
        red[threadIdx.x] = c;
        __syncthreads();
        for (int o = kB / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[(int64_t)blockIdx.x * nk + q] = red[0];
        __syncthreads();
    }
}

hipError_t knn2d(const pixelsne_ctx* c, int32_t* out) {
    const dim3 g((unsigned)ceil_div(c->n, kB));
    if (c->prm.precision == PSNE_FP64)
        k_knn2d<double><<<g, kB, 0, c->stream>>>((const double*)c->zh, c->sc, c->orig, c->n, c->r,
                                                 out);
    else
        k_knn2d<float><<<g, kB, 0, c->stream>>>((const float*)c->zh, c->sc, c->orig, c->n, c->r,
                                                out);
    return hipGetLastError();
}

}  // namespace
}  // namespace psne

using namespace psne;

extern "C" {

psne_status pixelsne_knn2d(const pixelsne_ctx* c, int32_t* idx) {
    if (!c || !is_device_ptr(idx)) { set_error("knn2d: null context or non-device output"); return PSNE_E_INVAL; }
    if (c->n - 1 < kK2) { set_error("knn2d needs n > 32"); return PSNE_E_UNSUPPORTED; }
    hipError_t e = knn2d(c, idx);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_error(const_cast<pixelsne_ctx*>(c), e, "knn2d");
    return PSNE_OK;
}

psne_status pixelsne_neighborhood_precision(const pixelsne_ctx* c, const int32_t* hi_knn,
                                            int32_t k_hi, const int32_t* ks, int32_t nk,
                                            double* out) {
    if (!c || !is_device_ptr(hi_knn) || !ks || !out || nk < 1 || nk > 64 || k_hi < 1) {
        set_error("neighborhood_precision: bad arguments");
        return PSNE_E_INVAL;
    }
    for (int q = 0; q < nk; q++)
        if (ks[q] < 1 || ks[q] > k_hi || ks[q] > kK2) {
            set_error("neighborhood_precision: every k must be in [1, min(k_hi, 32)]");
            return PSNE_E_INVAL;
        }
    if (c->n - 1 < kK2) { set_error("neighborhood_precision needs n > 32"); return PSNE_E_UNSUPPORTED; }
    const int64_t nb = ceil_div(c->n, kB);
    int32_t *lo = nullptr, *kd = nullptr;
    unsigned long long* part = nullptr;
    hipError_t e = hipMalloc(&lo, sizeof(int32_t) * (size_t)c->n * kK2);
    if (e == hipSuccess) e = hipMalloc(&kd, sizeof(int32_t) * nk);
    if (e == hipSuccess) e = hipMalloc(&part, sizeof(unsigned long long) * (size_t)nb * nk);
    if (e == hipSuccess) e = hipMemcpyAsync(kd, ks, sizeof(int32_t) * nk, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = knn2d(c, lo);
    if (e == hipSuccess) {
        k_overlap<<<dim3((unsigned)nb), kB, 0, c->stream>>>(hi_knn, k_hi, lo, c->n, kd, nk, part);
        e = hipGetLastError();
    }
    std::vector<unsigned long long> h((size_t)nb * nk);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h.data(), part, h.size() * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(lo); (void)hipFree(kd); (void)hipFree(part);
    if (e != hipSuccess) return device_error(const_cast<pixelsne_ctx*>(c), e, "neighborhood_precision");
    for (int q = 0; q < nk; q++) {
        unsigned long long s = 0;
        for (int64_t b = 0; b < nb; b++) s += h[(size_t)b * nk + q];
        out[q] = (double)s / ((double)ks[q] * (double)c->n);
    }
    return PSNE_OK;
}

}  // extern "C"
