// Barycentric transport map of a plan (colour transfer, Sec. IV-D).
//
// For the supplier side every supplier i gets T_i = sum_j F_ij y_j / sum_j F_ij,
// for the consumer side every consumer j gets T_j = sum_i F_ij x_i / sum_i F_ij.
// The definition sums each row in plan order, so the kernels keep that order
// (a plain FP64 accumulation in any other order would differ in the last
// bits):
//   map_zero     row counters to zero (a kernel, not a memset, so the
//                sequence can be captured in a graph)
//   map_count    entries per row
//   map_scan     exclusive scan into row starts (one workgroup)
//   map_scatter  entry indices into their rows' buckets (any order)
//   map_rows     one thread per row: the row's entries in ascending plan
//                position, each found by a scan of the bucket for the
//                smallest position above the last one (rows of up to
//                kMapThreadRow entries; longer rows go to a list)
//   map_big      one wavefront per listed row: the same selection with a
//                wavefront-wide minimum
// Both row kernels accumulate sum f and sum f p_k in FP64 without fused
// multiply-add and divide at the end (NaN for a row without flow).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "internal.hpp"

namespace nnsemd {
namespace {

constexpr int kMapThreads = 256;
constexpr int kMapScanThreads = 1024;
constexpr int kMapThreadRow = 16;  // rows longer than this take a wavefront

struct MapArgs {
    const int32_t* src;
    const int32_t* dst;
    const double* flow;
    int64_t cap;           // plan entries available
    const int64_t* nnz;    // device count of entries used, or null (cap)
    const float* P;        // p_rows x d points of the other side
    int64_t p_rows;
    int32_t d;
    int32_t side;          // 0: rows are suppliers, 1: rows are consumers
    int64_t rows;
    double* map;           // rows x d
    MapWork w;
};

__device__ inline int64_t map_nnz(const MapArgs& A) {
    if (A.nnz == nullptr) return A.cap;
    const int64_t k = *A.nnz;
    return k < 0 ? 0 : (k > A.cap ? A.cap : k);
}

// Row and other-side index of entry e; false when either is out of range.
__device__ inline bool map_entry(const MapArgs& A, int64_t e, int& r, int& o) {
    const int s = A.src[e], t = A.dst[e];
    r = A.side == 0 ? s : t;
    o = A.side == 0 ? t : s;
    return r >= 0 && (int64_t)r < A.rows && o >= 0 && (int64_t)o < A.p_rows;
}

__global__ __launch_bounds__(kMapThreads) void map_zero(MapArgs A) {
    const int64_t r = (int64_t)blockIdx.x * kMapThreads + threadIdx.x;
    if (r < A.rows) A.w.cnt[r] = 0;
    if (r == 0) *A.w.nbig = 0;
}

__global__ __launch_bounds__(kMapThreads) void map_count(MapArgs A) {
    const int64_t e = (int64_t)blockIdx.x * kMapThreads + threadIdx.x;
    if (e >= map_nnz(A)) return;
    int r, o;
    if (map_entry(A, e, r, o)) atomicAdd(&A.w.cnt[r], 1);
}

// Exclusive scan of cnt into start and cursor; each thread owns a run.
__global__ __launch_bounds__(kMapScanThreads) void map_scan(MapArgs A) {
    __shared__ int64_t part[kMapScanThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid / 64;
    const int64_t cs = (A.rows + kMapScanThreads - 1) / kMapScanThreads;
    const int64_t lo = tid * cs < A.rows ? tid * cs : A.rows;
    const int64_t hi = lo + cs < A.rows ? lo + cs : A.rows;
    int64_t sum = 0;
    for (int64_t r = lo; r < hi; ++r) sum += A.w.cnt[r];
    int64_t x = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) part[w] = x;
    __syncthreads();
    int64_t run = x - sum;
    for (int k = 0; k < w; ++k) run += part[k];
    for (int64_t r = lo; r < hi; ++r) {
        A.w.start[r] = (int32_t)run;
        A.w.cursor[r] = (int32_t)run;
        run += A.w.cnt[r];
    }
}

__global__ __launch_bounds__(kMapThreads) void map_scatter(MapArgs A) {
    const int64_t e = (int64_t)blockIdx.x * kMapThreads + threadIdx.x;
    if (e >= map_nnz(A)) return;
    int r, o;
    if (map_entry(A, e, r, o)) A.w.ent[atomicAdd(&A.w.cursor[r], 1)] = (int32_t)e;
}

// The row's sums in plan order: w = sum f, acc_k = sum f p_k (FP64, no FMA).
template <int D>
__device__ inline void map_store(const MapArgs& A, int64_t r, double w, const double (&acc)[D]) {
#pragma clang fp contract(off)
#pragma unroll
    for (int k = 0; k < D; ++k) A.map[r * D + k] = w > 0.0 ? acc[k] / w : NAN;
}

template <int D>
__global__ __launch_bounds__(kMapThreads) void map_rows(MapArgs A) {
#pragma clang fp contract(off)
    const int64_t r = (int64_t)blockIdx.x * kMapThreads + threadIdx.x;
    if (r >= A.rows) return;
    const int c = A.w.cnt[r];
    if (c > kMapThreadRow) {
        A.w.big[atomicAdd(A.w.nbig, 1)] = (int32_t)r;
        return;
    }
    const int s0 = A.w.start[r];
    double w = 0.0, acc[D];
#pragma unroll
    for (int k = 0; k < D; ++k) acc[k] = 0.0;
    int last = -1;
    for (int step = 0; step < c; ++step) {
        int e = 0x7fffffff;
        for (int q = s0; q < s0 + c; ++q) {
            const int x = A.w.ent[q];
            e = (x > last && x < e) ? x : e;
        }
        last = e;
        const double f = A.flow[e];
        const int o = A.side == 0 ? A.dst[e] : A.src[e];
        w = w + f;
#pragma unroll
        for (int k = 0; k < D; ++k) acc[k] = acc[k] + f * (double)A.P[(int64_t)o * D + k];
    }
    map_store<D>(A, r, w, acc);
}

template <int D>
__global__ __launch_bounds__(kMapThreads) void map_big(MapArgs A) {
#pragma clang fp contract(off)
    const int lane = threadIdx.x & 63;
    const int64_t slot = (int64_t)blockIdx.x * (kMapThreads / 64) + threadIdx.x / 64;
    if (slot >= *A.w.nbig) return;  // whole wavefronts
    const int64_t r = A.w.big[slot];
    const int c = A.w.cnt[r], s0 = A.w.start[r];
    double w = 0.0, acc[D];
#pragma unroll
    for (int k = 0; k < D; ++k) acc[k] = 0.0;
    int last = -1;
    for (int step = 0; step < c; ++step) {
        int e = 0x7fffffff;
        for (int q = s0 + lane; q < s0 + c; q += 64) {
            const int x = A.w.ent[q];
            e = (x > last && x < e) ? x : e;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) e = min(e, __shfl_xor(e, o));
        last = e;
        const double f = A.flow[e];
        const int o = A.side == 0 ? A.dst[e] : A.src[e];
        w = w + f;
#pragma unroll
        for (int k = 0; k < D; ++k) acc[k] = acc[k] + f * (double)A.P[(int64_t)o * D + k];
    }
    if (lane == 0) map_store<D>(A, r, w, acc);
}

template <int D>
int launch_typed(const MapArgs& A, hipStream_t st) {
    const int64_t eb = (A.cap + kMapThreads - 1) / kMapThreads;
    const int64_t rb = (A.rows + kMapThreads - 1) / kMapThreads;
    if (rb == 0) return 0;
    hipLaunchKernelGGL(map_zero, dim3((unsigned)rb), dim3(kMapThreads), 0, st, A);
    if (eb > 0) hipLaunchKernelGGL(map_count, dim3((unsigned)eb), dim3(kMapThreads), 0, st, A);
    hipLaunchKernelGGL(map_scan, dim3(1), dim3(kMapScanThreads), 0, st, A);
    if (eb > 0) hipLaunchKernelGGL(map_scatter, dim3((unsigned)eb), dim3(kMapThreads), 0, st, A);
    hipLaunchKernelGGL(map_rows<D>, dim3((unsigned)rb), dim3(kMapThreads), 0, st, A);
    // every row could be long only when the plan holds > 16 entries per row;
    // the wavefront kernel's grid covers the largest possible list
    const int64_t maxbig = A.cap / (kMapThreadRow + 1) < A.rows ? A.cap / (kMapThreadRow + 1) : A.rows;
    if (maxbig > 0) {
        const int64_t bb = (maxbig + kMapThreads / 64 - 1) / (kMapThreads / 64);
        hipLaunchKernelGGL(map_big<D>, dim3((unsigned)bb), dim3(kMapThreads), 0, st, A);
    }
    return (int)hipGetLastError();
}

}  // namespace

size_t map_ws_bytes(int64_t rows, int64_t cap) {
    return align_up(4 * (size_t)rows, 256) * 4 + align_up(4 * (size_t)(cap > 0 ? cap : 1), 256) + 256;
}

MapWork map_ws_carve(char* base, int64_t rows, int64_t cap) {
    const size_t rb = align_up(4 * (size_t)rows, 256);
    MapWork w;
    w.cnt = reinterpret_cast<int32_t*>(base);
    w.start = reinterpret_cast<int32_t*>(base + rb);
    w.cursor = reinterpret_cast<int32_t*>(base + 2 * rb);
    w.big = reinterpret_cast<int32_t*>(base + 3 * rb);
    w.ent = reinterpret_cast<int32_t*>(base + 4 * rb);
    w.nbig = reinterpret_cast<int32_t*>(base + 4 * rb + align_up(4 * (size_t)(cap > 0 ? cap : 1), 256));
    return w;
}

int launch_barycentric_map(const int32_t* src, const int32_t* dst, const double* flow, int64_t cap,
                           const int64_t* nnz, const float* P, int64_t p_rows, int d, int side, int64_t rows,
                           double* map, const MapWork& w, void* stream) {
    MapArgs A;
    A.src = src;
    A.dst = dst;
    A.flow = flow;
    A.cap = cap;
    A.nnz = nnz;
    A.P = P;
    A.p_rows = p_rows;
    A.d = d;
    A.side = side;
    A.rows = rows;
    A.map = map;
    A.w = w;
    hipStream_t st = (hipStream_t)stream;
    switch (d) {
        case 1: return launch_typed<1>(A, st);
        case 2: return launch_typed<2>(A, st);
        case 3: return launch_typed<3>(A, st);
        case 4: return launch_typed<4>(A, st);
        case 5: return launch_typed<5>(A, st);
        case 6: return launch_typed<6>(A, st);
        case 7: return launch_typed<7>(A, st);
        case 8: return launch_typed<8>(A, st);
        default: return (int)hipErrorInvalidValue;
    }
}

}  // namespace nnsemd
