// Per-pair workgroup solver of NNS-EMD for low-dimensional FP32 points.
//
// One workgroup owns one pair at a time and keeps everything about it in
// LDS: the compacted active suppliers (search records), per-point FP64
// masses, the consumers' current picks and the claimant buckets.  The rounds
// of Algorithm 1 (Sec. III-A) run as barrier-separated phases without ever
// leaving the chip:
//   1. NNS (Alg. 1 NNS step): every active consumer scans the active
//      supplier records in FP32.  For the Euclidean metrics the record is
//      (-2 x^, ||x^||^2) with x^ = x - centre, so one key costs d FMAs and
//      equals ||x^ - y^||^2 - ||y^||^2 up to a rounding bound E_q; best and
//      second-best keys are tracked and a consumer whose two keys are within
//      that bound is re-scored in FP64 by a whole wavefront, so every pick
//      equals the FP64 argmin with ties going to the smallest index.
//   2. Claimant sets a_i: LDS-atomic counting sort of consumers by pick.
//   3. Flow & cost (greedy or random protocol): one lane per claimed
//      supplier selects its claimants in (D_ij, j) order (or the random
//      protocol's key order) and serves f = min(s_i, c_j) in FP64 with the
//      same operations as the definition, so flows are bit-identical to it.
//   4. Weights update: plan entries and the surviving suppliers/consumers
//      are compacted with one block-wide prefix scan (ballot-free: per-lane
//      contiguous chunks, wavefront shuffles, one LDS hop).
// One launch covers any number of ragged pairs, one workgroup each (the
// batching of Sec. III-D without padding).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "internal.hpp"
#include "round_common.hpp"
#include "point_search.hpp"

namespace nnsemd {
namespace {

using namespace rc;
using namespace ps;

// CL: the pair's coordinates are copied into LDS at ingest (L.xl, L.yl) and
// every later read takes them from there; otherwise from HBM.
template <int D, int T, int CSMAX, bool L1, bool CL>
__device__ void solve_pair(const PairSolverArgs& A, int64_t p, const Lds16& L, SharedCore& sh) {
    constexpr int RS = record_stride(D);
    constexpr int NW = T / kWave;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;

    NNSEMD_PH_DECL
    if (tid == 0) {  // the ingest's block reductions order these before any use
        sh.tie_nn = 0ull;
        sh.tie_order = 0ull;
    }
    // ---------------------------------------------------------- pair geometry
    int64_t x0 = 0, y0 = 0, m = A.single_m, n = A.single_n;
    int status = NNSEMD_OK;
    if (A.x_off != nullptr) {
        int64_t px = A.pair_x ? (int64_t)A.pair_x[p] : p;
        int64_t py = A.pair_y ? (int64_t)A.pair_y[p] : p;
        if (px < 0 || px >= A.num_x_sets || py < 0 || py >= A.num_y_sets) {
            status = NNSEMD_ERR_INVALID_ARG;
            m = n = 0;
        } else {
            x0 = A.x_off[px];
            m = A.x_off[px + 1] - x0;
            y0 = A.y_off[py];
            n = A.y_off[py + 1] - y0;
        }
    }
    if (status == NNSEMD_OK && (m < 0 || n < 0 || m > A.max_m || n > A.max_n)) {
        status = NNSEMD_ERR_INVALID_ARG;
        m = n = 0;
    }
    int64_t plan_base = 0, plan_cap = 0;
    const bool want_plan = A.plan_src != nullptr;
    if (want_plan) {
        if (A.plan_off != nullptr) {
            plan_base = A.plan_off[p];
            plan_cap = A.plan_off[p + 1] - plan_base;
        } else {
            plan_cap = A.single_plan_cap;
        }
        if (status == NNSEMD_OK && m + n > 0 && plan_cap < m + n - 1) {
            status = NNSEMD_ERR_CAPACITY;
            m = n = 0;
        }
    }
    const float* __restrict__ Xg = A.X + x0 * D;
    const float* __restrict__ Yg = A.Y + y0 * D;
    const int mi = (int)m, ni = (int)n;
    // coordinates for the rounds (LDS copies in the CL variant, filled below)
    const float* __restrict__ X = CL ? L.xl : Xg;
    const float* __restrict__ Y = CL ? L.yl : Yg;

    // ------------------------------------- ingest: masses, checks, bounding box
    double red[3 + 2 * D];
    int rop[3 + 2 * D];
    red[0] = 0.0; rop[0] = 0;  // sum a
    red[1] = 0.0; rop[1] = 0;  // sum b
    red[2] = 0.0; rop[2] = 2;  // bad value seen
#pragma unroll
    for (int t = 0; t < D; ++t) {
        red[3 + t] = INFINITY;      rop[3 + t] = 1;
        red[3 + D + t] = -INFINITY; rop[3 + D + t] = 2;
    }
    for (int i = tid; i < mi; i += T) {
        float av = A.a[x0 + i];
        if (!(av >= 0.f) || !isfinite(av)) red[2] = 1.0;
        L.smass[i] = (double)av;
        red[0] += (double)av;
#pragma unroll
        for (int t = 0; t < D; ++t) {
            float xv = Xg[(size_t)i * D + t];
            if constexpr (CL) L.xl[(size_t)i * D + t] = xv;
            if (!isfinite(xv)) red[2] = 1.0;
            red[3 + t] = fmin(red[3 + t], (double)xv);
            red[3 + D + t] = fmax(red[3 + D + t], (double)xv);
        }
    }
    for (int j = tid; j < ni; j += T) {
        float bv = A.b[y0 + j];
        if (!(bv >= 0.f) || !isfinite(bv)) red[2] = 1.0;
        L.cmass[j] = (double)bv;
        red[1] += (double)bv;
#pragma unroll
        for (int t = 0; t < D; ++t) {
            const float yv = Yg[(size_t)j * D + t];
            if constexpr (CL) L.yl[(size_t)j * D + t] = yv;
            if (!isfinite(yv)) red[2] = 1.0;
        }
    }
    block_reduce<T, 3 + 2 * D>(red, rop, L.ckey);  // the key array is free outside the rounds
    if (status == NNSEMD_OK && red[2] != 0.0) status = NNSEMD_ERR_INVALID_ARG;
    if (status == NNSEMD_OK) {
        double big = fmax(red[0], red[1]);
        if (fabs(red[0] - red[1]) > 1e-5 * big) status = NNSEMD_ERR_MASS_MISMATCH;
    }
    float centre[D];
#pragma unroll
    for (int t = 0; t < D; ++t)
        centre[t] = (L1 || mi == 0) ? 0.f : 0.5f * ((float)red[3 + t] + (float)red[3 + D + t]);

    // ------------------- initial active sets (zero-mass points never enter)
    // Supplier state is kept by active slot from here on: records, local
    // index, mass, claimant count and bucket offset are compacted together.
    int mact = 0, nact = 0;
    float rhat = 0.f;
    bool exact = false;  // every FP32 key is exact (keys_exact)
    if (status == NNSEMD_OK) {
        const int cs = (mi + T - 1) / T;
        const int cc = (ni + T - 1) / T;
        const int slo = min(tid * cs, mi), shi = min(slo + cs, mi);
        const int clo = min(tid * cc, ni), chi = min(clo + cc, ni);
        double mv[CSMAX];
        int ks = 0, kc = 0;
#pragma unroll
        for (int u = 0; u < CSMAX; ++u) {
            const int i = slo + u;
            mv[u] = (u < cs && i < shi) ? L.smass[i] : 0.0;
            ks += mv[u] > 0.0;
        }
        for (int j = clo; j < chi; ++j) kc += L.cmass[j] > 0.0;
        unsigned long long tot;
        unsigned long long pre = block_scan_u64<T>((unsigned long long)ks | ((unsigned long long)kc << 32), &tot, sh);
        int ps = (int)(pre & 0xffffffffu), pc = (int)(pre >> 32);
        mact = (int)(tot & 0xffffffffu);
        nact = (int)(tot >> 32);
        float rmax = 0.f;
        int fq = 0;        // fractional bits of the (centred) coordinates
        float amax = 0.f;  // their largest magnitude
#pragma unroll
        for (int u = 0; u < CSMAX; ++u) {
            if (!(mv[u] > 0.0)) continue;
            const int i = slo + u;
            float r[RS];
#pragma unroll
            for (int q = 0; q < RS; ++q) r[q] = 0.f;
            if (L1) {
#pragma unroll
                for (int t = 0; t < D; ++t) {
                    r[t] = X[(size_t)i * D + t];
                    fq = max(fq, frac_bits(r[t]));
                    amax = fmaxf(amax, fabsf(r[t]));
                }
            } else {
                float h = 0.f;
#pragma unroll
                for (int t = 0; t < D; ++t) {
                    float xc = X[(size_t)i * D + t] - centre[t];
                    r[t] = -2.f * xc;
                    h = fmaf(xc, xc, h);
                    fq = max(fq, frac_bits(xc));
                    amax = fmaxf(amax, fabsf(xc));
                }
                r[D] = h;
                rmax = fmaxf(rmax, sqrtf(h));
            }
            store_rec<RS>(L.srec, ps, r);
            L.sidx[ps] = i;
            L.smass[ps] = mv[u];
            L.scnt[ps] = 0;
            ++ps;
        }
        for (int j = clo; j < chi; ++j) {
            if (L.cmass[j] > 0.0) {
                L.cact[pc++] = j;
#pragma unroll
                for (int t = 0; t < D; ++t) {
                    const float yc = L1 ? Y[(size_t)j * D + t] : Y[(size_t)j * D + t] - centre[t];
                    fq = max(fq, frac_bits(yc));
                    amax = fmaxf(amax, fabsf(yc));
                }
            }
        }
        double rr[3] = {(double)rmax, (double)fq, (double)amax};
        const int ro[3] = {2, 2, 2};
        block_reduce<T, 3>(rr, ro, L.ckey);  // also orders the writes above
        rhat = (float)rr[0] * (1.f + 1e-6f);
        exact = keys_exact<D, L1>(rr[1], rr[2]);
        if (tid == 0) sh.nflag = 0;
        __syncthreads();
    }
    NNSEMD_PH(0)

    // ------------------------------------------------------------- rounds
    const int64_t max_rounds = A.max_rounds > 0 ? A.max_rounds : (int64_t)mi + ni;
    int rounds = 0;
    int64_t work = 0, nnz = 0, near = 0;
    double cost = 0.0;  // this thread's part of R
    while (status == NNSEMD_OK && mact > 0 && nact > 0) {
        if (rounds >= max_rounds) {
            status = NNSEMD_ERR_NOT_CONVERGED;
            break;
        }
        work += (int64_t)mact * nact;

        // ---- 1. NNS: FP32 scan, best + second best, near ties deferred
        // and re-scored in FP64; each pick counted into its bucket.
        near += ps::search_round<D, T, CSMAX, L1>(L, sh, X, Y, centre, rhat, mact, nact, A.split, exact,
                                                   A.metric);
        NNSEMD_PH(1)
        NNSEMD_PH(2)

        // ---- 2. claimant sets a_i
        round_buckets<T>(L, sh, mact, nact);
        NNSEMD_PH(3)
        // ---- 3. flow & cost: claimant order, then the serve walk
        round_rank<T, CSMAX>(L, nact, A.protocol, A.seed, rounds, A.metric,
                             A.protocol == NNSEMD_GREEDY ? &sh.tie_order : nullptr);
        NNSEMD_PH(5)
        round_walk<T, true, true>(L, mact, A.metric, cost);
        NNSEMD_PH(6)
        // ---- 4. weights update: plan append + compaction
        round_compact<T, CSMAX, RS, true>(L, sh, mact, nact, nnz, want_plan ? A.plan_src : nullptr, A.plan_dst,
                                    A.plan_flow, plan_base);
        NNSEMD_PH(7)
        ++rounds;
    }

    // ---------------------------------------------------------- results
    double fin[3] = {cost, 0.0, 0.0};
    const int fop[3] = {0, 0, 0};
    if (status == NNSEMD_OK || status == NNSEMD_ERR_NOT_CONVERGED) {
        for (int s = tid; s < mact; s += T) fin[1] += L.smass[s];
        for (int q = tid; q < nact; q += T) fin[2] += L.cmass[L.cact[q]];
    }
    block_reduce<T, 3>(fin, fop, L.ckey);  // its barriers also order the counters' atomics
    NNSEMD_PH(8)
    NNSEMD_PH_FLUSH(A.phase_cycles)
    if (tid == 0) {
        A.costs[p] = status == NNSEMD_OK ? fin[0] : NAN;
        if (A.stats != nullptr) {
            nnsemd_stats_t st;
            st.status = status;
            st.rounds = rounds;
            st.nnz = nnz;
            st.work = work;
            st.rescored = near;
            st.residual_src = fin[1];
            st.residual_dst = fin[2];
            st.near_ties_nn = (int64_t)sh.tie_nn;
            st.near_ties_order = (int64_t)sh.tie_order;
            A.stats[p] = st;
        }
    }
}

// One workgroup per pair: the hardware dispatcher hands out workgroups as
// earlier ones retire, which balances ragged pairs without a software queue.
// (A persistent loop whose head is a thread-0-only queue fetch must not be
// used here: its back-edge merges with the thread-0-only result write, and
// the structurized code lets lanes 1-63 of wave 0 pass the following
// barrier without the fetch, re-solving the same pair forever.)
// Register budget, up to four claimants per thread, chosen so that no
// variant spills: 128 VGPRs for d <= 3 (four waves per SIMD, so small
// pairs keep four workgroups per CU), 168 for d = 4, 5 and 256 for d = 6, 7,
// whose larger LDS records hold a 1024-point pair to two or three
// workgroups per CU anyway.
template <int D, int T, int CSMAX, bool L1, bool CL>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(CSMAX <= 2 && D <= 3 ? 6 : (CSMAX <= 4 ? (D <= 3 ? 4 : (D <= 5 ? 3 : 2)) : 1))))
void pair_solver_kernel(PairSolverArgs A) {
    extern __shared__ __align__(16) char lds_dyn[];
    __shared__ SharedCore sh;
    const Lds16 L = carve16(lds_dyn, A.max_m, A.max_n, record_stride(D), CL ? D : 0, A.share_order != 0);
    const int64_t p = A.order != nullptr ? (int64_t)A.order[blockIdx.x] : (int64_t)blockIdx.x;
    solve_pair<D, T, CSMAX, L1, CL>(A, p, L, sh);
}

// Longest-first schedule: order[] lists the pairs by decreasing m * n (in
// quarter-octave buckets; order inside a bucket is arbitrary and does not
// affect any result), so the largest pairs start first and the short ones
// fill the tail of the launch.  One workgroup of 1024 threads.
constexpr int kOrderBuckets = 256;
__global__ __launch_bounds__(1024) void order_kernel(const int64_t* __restrict__ x_off,
                                                     const int64_t* __restrict__ y_off,
                                                     const int32_t* __restrict__ pair_x,
                                                     const int32_t* __restrict__ pair_y, int64_t num_pairs,
                                                     int64_t num_x_sets, int64_t num_y_sets,
                                                     int32_t* __restrict__ order) {
    __shared__ int hist[kOrderBuckets];
    __shared__ int cursor[kOrderBuckets];
    const int tid = threadIdx.x;
    for (int b = tid; b < kOrderBuckets; b += blockDim.x) hist[b] = 0;
    __syncthreads();
    auto bucket_of = [&](int64_t p) -> int {
        const int64_t px = pair_x ? (int64_t)pair_x[p] : p;
        const int64_t py = pair_y ? (int64_t)pair_y[p] : p;
        if (px < 0 || px >= num_x_sets || py < 0 || py >= num_y_sets) return 0;
        const int64_t m = x_off[px + 1] - x_off[px];
        const int64_t n = y_off[py + 1] - y_off[py];
        if (m <= 0 || n <= 0) return 0;
        const unsigned long long w = (unsigned long long)m * (unsigned long long)n;
        const int lg = 63 - __clzll(w);
        const int frac = lg >= 2 ? (int)((w >> (lg - 2)) & 3ull) : 0;
        const int b = 1 + 4 * lg + frac;
        return b < kOrderBuckets ? b : kOrderBuckets - 1;
    };
    for (int64_t p = tid; p < num_pairs; p += blockDim.x) atomicAdd(&hist[bucket_of(p)], 1);
    __syncthreads();
    if (tid == 0) {
        int run = 0;
        for (int b = kOrderBuckets - 1; b >= 0; --b) {
            cursor[b] = run;
            run += hist[b];
        }
    }
    __syncthreads();
    for (int64_t p = tid; p < num_pairs; p += blockDim.x) {
        const int pos = atomicAdd(&cursor[bucket_of(p)], 1);
        order[pos] = (int32_t)p;
    }
}

template <int D, int T, int CSMAX, bool L1, bool CL>
int launch_typed(const PairSolverArgs& A, size_t lds, int grid, hipStream_t st) {
    if (lds > 48 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)pair_solver_kernel<D, T, CSMAX, L1, CL>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return (int)e;
    }
    hipLaunchKernelGGL((pair_solver_kernel<D, T, CSMAX, L1, CL>), dim3(grid), dim3(T), lds, st, A);
    return (int)hipGetLastError();
}

template <int D, int T, int CSMAX, bool L1, bool CL>
int occupancy_typed(size_t lds, int* blocks) {
    if (lds > 48 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)pair_solver_kernel<D, T, CSMAX, L1, CL>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return (int)e;
    }
    return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, pair_solver_kernel<D, T, CSMAX, L1, CL>, T,
                                                             lds);
}

// Dispatch over (D, metric class) for one workgroup size, chunk class and
// coordinate placement.
template <int T, int CSMAX, bool CL>
int dispatch(bool run, const PairSolverArgs& A, int d, size_t lds, int grid, hipStream_t st,
             int* blocks) {
    const bool l1 = A.metric == NNSEMD_L1;
#define NNSEMD_CASE(DD)                                                                      \
    case DD:                                                                                 \
        if (run)                                                                             \
            return l1 ? launch_typed<DD, T, CSMAX, true, CL>(A, lds, grid, st)               \
                      : launch_typed<DD, T, CSMAX, false, CL>(A, lds, grid, st);             \
        return l1 ? occupancy_typed<DD, T, CSMAX, true, CL>(lds, blocks)                     \
                  : occupancy_typed<DD, T, CSMAX, false, CL>(lds, blocks);
    switch (d) {
        NNSEMD_CASE(1)
        NNSEMD_CASE(2)
        NNSEMD_CASE(3)
        NNSEMD_CASE(4)
        NNSEMD_CASE(5)
        NNSEMD_CASE(6)
        NNSEMD_CASE(7)
        default:
            return (int)hipErrorInvalidValue;
    }
#undef NNSEMD_CASE
}

template <bool CL>
int dispatch_cl(bool run, const PairSolverArgs& A, int d, int threads, int chunk_max, size_t lds, int grid,
                hipStream_t st, int* blocks) {
    if (threads == 256) {
        if (chunk_max <= 4) return dispatch<256, 4, CL>(run, A, d, lds, grid, st, blocks);
        if (chunk_max <= 16) return dispatch<256, 16, CL>(run, A, d, lds, grid, st, blocks);
    } else if (threads == 512) {
        if (chunk_max <= 2) return dispatch<512, 2, CL>(run, A, d, lds, grid, st, blocks);
        if (chunk_max <= 8) return dispatch<512, 8, CL>(run, A, d, lds, grid, st, blocks);
    }
    return (int)hipErrorInvalidValue;
}

int dispatch_all(bool run, const PairSolverArgs& A, int d, int threads, int chunk_max, size_t lds,
                 int grid, hipStream_t st, int* blocks, bool coords) {
    return coords ? dispatch_cl<true>(run, A, d, threads, chunk_max, lds, grid, st, blocks)
                  : dispatch_cl<false>(run, A, d, threads, chunk_max, lds, grid, st, blocks);
}

}  // namespace

int launch_pair_solver(const PairSolverArgs& args, int d, int threads, int chunk_max, bool coords, size_t lds_bytes,
                       int grid, void* stream) {
    return dispatch_all(true, args, d, threads, chunk_max, lds_bytes, grid, (hipStream_t)stream, nullptr, coords);
}

int launch_order(const int64_t* x_off, const int64_t* y_off, const int32_t* pair_x, const int32_t* pair_y,
                 int64_t num_pairs, int64_t num_x_sets, int64_t num_y_sets, int32_t* order, void* stream) {
    hipLaunchKernelGGL(order_kernel, dim3(1), dim3(1024), 0, (hipStream_t)stream, x_off, y_off, pair_x, pair_y,
                       num_pairs, num_x_sets, num_y_sets, order);
    return (int)hipGetLastError();
}

int pair_solver_blocks_per_cu(int d, int metric, int threads, int chunk_max, size_t lds_bytes, int* blocks,
                              bool coords) {
    PairSolverArgs A{};
    A.metric = metric;
    return dispatch_all(false, A, d, threads, chunk_max, lds_bytes, 0, nullptr, blocks, coords);
}


}  // namespace nnsemd
