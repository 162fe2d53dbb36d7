// Colour transfer by NNS-EMD (Sec. IV-D): k-means palettes of two 8-bit RGB
// images, NNS-EMD from the reference palette to the source palette, and the
// source recoloured through the per-consumer barycentric map of the plan.
//
// The palette reduction is Lloyd iteration with every step made exactly
// reproducible, so its result does not depend on thread order:
//   start      centroid k = colour of pixel floor(k P / K)
//   assign     argmin_k sum_c (p_c - C_kc)^2 in FP64, channels in order, no
//              fused multiply-add, ties to the smallest k (centroids staged
//              in LDS, one thread per pixel)
//   accumulate integer channel sums and counts per cluster: 64-bit integer
//              atomics, first into a per-workgroup LDS table, then one
//              global add per cluster and workgroup -- integer sums are the
//              same in any order
//   update     C_kc = S_kc / n_k (FP64, correctly rounded); an empty cluster
//              keeps its centroid
// The palettes become colour histograms: bin colour C / 255 and mass
// n_k / P, both rounded once from FP64 to FP32.  Recolouring writes
// round-half-even(255 T) clamped to 0..255 for each channel of the pixel's
// bin, or keeps the pixel when its bin received no flow.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "internal.hpp"

namespace nnsemd {
namespace {

constexpr int kKmThreads = 256;

__global__ __launch_bounds__(kKmThreads) void km_init(const uint8_t* __restrict__ px, int64_t P, int K,
                                                      double* __restrict__ C, unsigned long long* __restrict__ S) {
    const int k = blockIdx.x * kKmThreads + threadIdx.x;
    if (k >= K) return;
    const int64_t src = (int64_t)k * P / K;
#pragma unroll
    for (int c = 0; c < 3; ++c) C[k * 3 + c] = (double)px[src * 3 + c];
#pragma unroll
    for (int c = 0; c < 4; ++c) S[k * 4 + c] = 0ull;
}

// One assignment step: every pixel to its nearest centroid; the cluster
// sums and counts of this assignment are accumulated into S (zero on entry).
__global__ __launch_bounds__(kKmThreads) void km_assign(const uint8_t* __restrict__ px, int64_t P, int K,
                                                        const double* __restrict__ C,
                                                        unsigned long long* __restrict__ S,
                                                        int32_t* __restrict__ assign) {
#pragma clang fp contract(off)
    extern __shared__ __align__(16) char km_lds[];
    double* cs = reinterpret_cast<double*>(km_lds);                                       // K x 3
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(km_lds + 24 * (size_t)K);  // K x 4
    const int tid = threadIdx.x;
    for (int e = tid; e < 3 * K; e += kKmThreads) cs[e] = C[e];
    for (int e = tid; e < 4 * K; e += kKmThreads) acc[e] = 0ull;
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * kKmThreads + tid;
    if (p < P) {
        const double r = (double)px[p * 3], g = (double)px[p * 3 + 1], b = (double)px[p * 3 + 2];
        int best = 0;
        double bd = INFINITY;
        for (int k = 0; k < K; ++k) {
            const double t0 = r - cs[3 * k], t1 = g - cs[3 * k + 1], t2 = b - cs[3 * k + 2];
            double d = 0.0;
            d = d + t0 * t0;
            d = d + t1 * t1;
            d = d + t2 * t2;
            if (d < bd) {
                bd = d;
                best = k;
            }
        }
        assign[p] = best;
        atomicAdd(&acc[4 * best], (unsigned long long)px[p * 3]);
        atomicAdd(&acc[4 * best + 1], (unsigned long long)px[p * 3 + 1]);
        atomicAdd(&acc[4 * best + 2], (unsigned long long)px[p * 3 + 2]);
        atomicAdd(&acc[4 * best + 3], 1ull);
    }
    __syncthreads();
    for (int e = tid; e < 4 * K; e += kKmThreads)
        if (acc[e] != 0ull) atomicAdd(&S[e], acc[e]);
}

// Update from the sums of the last assignment, then clear them for the next.
__global__ __launch_bounds__(kKmThreads) void km_update(int K, double* __restrict__ C,
                                                        unsigned long long* __restrict__ S) {
    const int k = blockIdx.x * kKmThreads + threadIdx.x;
    if (k >= K) return;
    const unsigned long long n = S[k * 4 + 3];
    if (n > 0ull) {
#pragma unroll
        for (int c = 0; c < 3; ++c) C[k * 3 + c] = (double)S[k * 4 + c] / (double)n;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) S[k * 4 + c] = 0ull;
}

// Palette histogram from the final assignment's counts.
__global__ __launch_bounds__(kKmThreads) void km_palette(int K, int64_t P, const double* __restrict__ C,
                                                         const unsigned long long* __restrict__ S,
                                                         float* __restrict__ pts, float* __restrict__ mass) {
    const int k = blockIdx.x * kKmThreads + threadIdx.x;
    if (k >= K) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) pts[k * 3 + c] = (float)(C[k * 3 + c] / 255.0);
    mass[k] = (float)((double)S[k * 4 + 3] / (double)P);
}

__global__ __launch_bounds__(kKmThreads) void recolour_kernel(const uint8_t* __restrict__ px,
                                                              const int32_t* __restrict__ assign, int64_t P,
                                                              const double* __restrict__ T,
                                                              uint8_t* __restrict__ out) {
    const int64_t p = (int64_t)blockIdx.x * kKmThreads + threadIdx.x;
    if (p >= P) return;
    const double* t = T + (int64_t)assign[p] * 3;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (isnan(t[c])) {
            out[p * 3 + c] = px[p * 3 + c];
            continue;
        }
        double v = rint(255.0 * t[c]);
        v = v < 0.0 ? 0.0 : (v > 255.0 ? 255.0 : v);
        out[p * 3 + c] = (uint8_t)v;
    }
}

}  // namespace

size_t kmeans_lds_bytes(int K) { return 24 * (size_t)K + 32 * (size_t)K; }

int launch_kmeans(const uint8_t* px, int64_t P, int K, int iters, double* C, unsigned long long* S,
                  int32_t* assign, float* pts, float* mass, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    const unsigned kb = (unsigned)((K + kKmThreads - 1) / kKmThreads);
    const unsigned pb = (unsigned)((P + kKmThreads - 1) / kKmThreads);
    const size_t lds = kmeans_lds_bytes(K);
    if (lds > 48 * 1024) {
        const hipError_t e = hipFuncSetAttribute((const void*)km_assign, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds);
        if (e != hipSuccess) return (int)e;
    }
    hipLaunchKernelGGL(km_init, dim3(kb), dim3(kKmThreads), 0, st, px, P, K, C, S);
    for (int it = 0; it <= iters; ++it) {
        hipLaunchKernelGGL(km_assign, dim3(pb), dim3(kKmThreads), lds, st, px, P, K, C, S, assign);
        if (it < iters) hipLaunchKernelGGL(km_update, dim3(kb), dim3(kKmThreads), 0, st, K, C, S);
    }
    hipLaunchKernelGGL(km_palette, dim3(kb), dim3(kKmThreads), 0, st, K, P, C, S, pts, mass);
    return (int)hipGetLastError();
}

int launch_recolour(const uint8_t* px, const int32_t* assign, int64_t P, const double* T, uint8_t* out,
                    void* stream) {
    const unsigned pb = (unsigned)((P + kKmThreads - 1) / kKmThreads);
    hipLaunchKernelGGL(recolour_kernel, dim3(pb), dim3(kKmThreads), 0, (hipStream_t)stream, px, assign, P, T, out);
    return (int)hipGetLastError();
}

}  // namespace nnsemd
