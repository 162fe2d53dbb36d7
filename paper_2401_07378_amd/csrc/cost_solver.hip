// NNS-EMD on a given ground-distance matrix: Algorithm 1 (Sec. III-A) takes
// D itself as its input (NNS-EMD(S, C, D)), and the method accepts any valid
// D (Sec. IV-F), so this form needs no point coordinates at all.
//
// One workgroup per pair, everything but D in LDS (compact 16-bit layout of
// the point path without search records).  D (FP32 or FP64, row-major m x n,
// caller-owned) stays in HBM and is read where the search needs it: consumer
// j of an active supplier slot s reads D[sidx[s] * n + j], so lanes holding
// neighbouring consumers read neighbouring addresses of one row.  The keys
// are the entries themselves, compared exactly (ties to the smallest
// supplier index), so there is no rounding bound and no re-score; the best
// and second-best entry of every consumer also give the near-tie count
// exactly.  The round phases after the search are the shared ones
// (round_common.hpp).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "internal.hpp"
#include "round_common.hpp"

namespace nnsemd {
namespace {

using namespace rc;

template <typename TD>
__device__ inline bool bad_entry(TD v) {
    return !(v >= (TD)0) || !isfinite(v);
}

template <typename TD, int T, int CSMAX>
__device__ void solve_cost_pair(const CostArgs& A, int64_t p, const Lds16& L, SharedCore& sh) {
    const int tid = threadIdx.x;
    if (tid == 0) sh.tie_order = 0ull;  // ordered before use by the ingest's reductions
    int64_t m = A.single_m, n = A.single_n, a0 = 0, b0 = 0, d0 = 0;
    int status = NNSEMD_OK;
    if (A.a_off != nullptr) {
        const int64_t px = A.pair_x ? (int64_t)A.pair_x[p] : p;
        const int64_t py = A.pair_y ? (int64_t)A.pair_y[p] : p;
        if (px < 0 || px >= A.num_a_sets || py < 0 || py >= A.num_b_sets) {
            status = NNSEMD_ERR_INVALID_ARG;
            m = n = 0;
        } else {
            a0 = A.a_off[px];
            m = A.a_off[px + 1] - a0;
            b0 = A.b_off[py];
            n = A.b_off[py + 1] - b0;
            if (A.d_off != nullptr) {
                d0 = A.d_off[p];
                if (A.d_off[p + 1] - d0 != m * n) status = NNSEMD_ERR_INVALID_ARG;
            } else {
                d0 = (p - A.pair_base) * A.d_stride;
            }
            if (m < 0 || n < 0) status = NNSEMD_ERR_INVALID_ARG;
            if (status != NNSEMD_OK) m = n = 0;
        }
    }
    if (status == NNSEMD_OK && (m > A.max_m || n > A.max_n)) {
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
    const TD* __restrict__ D = reinterpret_cast<const TD*>(A.D) + d0;
    const int mi = (int)m, ni = (int)n;

    // ---- ingest: masses, every entry of D checked (finite, >= 0)
    double red[3] = {0.0, 0.0, 0.0};
    const int rop[3] = {0, 0, 2};
    for (int i = tid; i < mi; i += T) {
        const float av = A.a[a0 + i];
        if (!(av >= 0.f) || !isfinite(av)) red[2] = 1.0;
        L.smass[i] = (double)av;
        red[0] += (double)av;
    }
    for (int j = tid; j < ni; j += T) {
        const float bv = A.b[b0 + j];
        if (!(bv >= 0.f) || !isfinite(bv)) red[2] = 1.0;
        L.cmass[j] = (double)bv;
        red[1] += (double)bv;
    }
    {
        const int64_t tot = (int64_t)mi * ni;
        bool bad = false;
        for (int64_t e = tid; e < tot; e += T) bad |= bad_entry(D[e]);
        if (bad) red[2] = 1.0;
    }
    block_reduce<T, 3>(red, rop, L.ckey);
    if (status == NNSEMD_OK && red[2] != 0.0) status = NNSEMD_ERR_INVALID_ARG;
    if (status == NNSEMD_OK) {
        const double big = fmax(red[0], red[1]);
        if (fabs(red[0] - red[1]) > 1e-5 * big) status = NNSEMD_ERR_MASS_MISMATCH;
    }

    // ---- initial active sets (zero-mass points never enter)
    int mact = 0, nact = 0;
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
        const unsigned long long pre =
            block_scan_u64<T>((unsigned long long)ks | ((unsigned long long)kc << 32), &tot, sh);
        int ps = (int)(pre & 0xffffffffu), pc = (int)(pre >> 32);
        mact = (int)(tot & 0xffffffffu);
        nact = (int)(tot >> 32);
#pragma unroll
        for (int u = 0; u < CSMAX; ++u) {
            if (!(mv[u] > 0.0)) continue;
            L.sidx[ps] = slo + u;
            L.smass[ps] = mv[u];
            L.scnt[ps] = 0;
            ++ps;
        }
        for (int j = clo; j < chi; ++j)
            if (L.cmass[j] > 0.0) L.cact[pc++] = j;
        if (tid == 0) sh.nflag = 0;
        __syncthreads();
    }

    // ---- rounds
    const int64_t max_rounds = A.max_rounds > 0 ? A.max_rounds : (int64_t)mi + ni;
    int rounds = 0;
    int64_t work = 0, nnz = 0, ties_nn = 0;
    double cost = 0.0;
    while (status == NNSEMD_OK && mact > 0 && nact > 0) {
        if (rounds >= max_rounds) {
            status = NNSEMD_ERR_NOT_CONVERGED;
            break;
        }
        work += (int64_t)mact * nact;
        // NNS: S lanes per consumer while consumers are few (each scans every
        // S-th active supplier), one lane per consumer otherwise; the best
        // entry (smallest slot among equals) and the second-best value.
        int S = 1;
        while (S < kWave && nact * S * 2 <= T) S <<= 1;
        while (S > 1 && S > mact) S >>= 1;
        const int r = tid & (S - 1);
        const int G = T / S;
        for (int q0 = 0; q0 < nact; q0 += G) {
            const int q = q0 + tid / S;
            const bool valid = q < nact;
            const int j = L.cact[valid ? q : 0];
            TD b1 = (TD)INFINITY, b2 = (TD)INFINITY;
            int bs = 0x7fffffff;
            constexpr int U = 4;
            const int stride = S * U;
            const int full = (mact / stride) * stride;
            for (int s0 = r; s0 < full; s0 += stride) {
                TD k[U];
#pragma unroll
                for (int u = 0; u < U; ++u) k[u] = D[(int64_t)L.sidx[s0 + u * S] * ni + j];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const bool lt = k[u] < b1;
                    bs = lt ? s0 + u * S : bs;
                    b2 = lt ? b1 : (k[u] < b2 ? k[u] : b2);
                    b1 = lt ? k[u] : b1;
                }
            }
            for (int s = full + r; s < mact; s += S) {
                const TD k = D[(int64_t)L.sidx[s] * ni + j];
                const bool lt = k < b1;
                bs = lt ? s : bs;
                b2 = lt ? b1 : (k < b2 ? k : b2);
                b1 = lt ? k : b1;
            }
            for (int o = 1; o < S; o <<= 1) {
                const TD c1 = __shfl_xor(b1, o);
                const TD c2 = __shfl_xor(b2, o);
                const int cs2 = __shfl_xor(bs, o);
                const TD hi1 = b1 < c1 ? c1 : b1;
                const TD lo2 = b2 < c2 ? b2 : c2;
                const TD n2 = hi1 < lo2 ? hi1 : lo2;
                const bool take = (c1 < b1) || (c1 == b1 && cs2 < bs);
                b1 = take ? c1 : b1;
                bs = take ? cs2 : bs;
                b2 = n2;
            }
            if (valid && r == 0) {
                L.cnn[j] = bs;
                L.ckey[j] = (double)b1;
                cnt_add(L.scnt, bs);
                if (mact > 1 && near_tie_dist((double)b1, (double)b2)) ++ties_nn;
            }
        }
        __syncthreads();
        round_buckets<T>(L, sh, mact, nact);
        // keys are the distances themselves (metric code SQEUCLIDEAN: D = key)
        round_rank<T, CSMAX>(L, nact, A.protocol, A.seed, rounds, NNSEMD_SQEUCLIDEAN,
                             A.protocol == NNSEMD_GREEDY ? &sh.tie_order : nullptr);
        round_walk<T, true, true>(L, mact, NNSEMD_SQEUCLIDEAN, cost);
        round_compact<T, CSMAX, 0, true>(L, sh, mact, nact, nnz, want_plan ? A.plan_src : nullptr, A.plan_dst,
                                   A.plan_flow, plan_base);
        ++rounds;
    }

    double fin[4] = {cost, 0.0, 0.0, (double)ties_nn};
    const int fop[4] = {0, 0, 0, 0};
    if (status == NNSEMD_OK || status == NNSEMD_ERR_NOT_CONVERGED) {
        for (int s = tid; s < mact; s += T) fin[1] += L.smass[s];
        for (int q = tid; q < nact; q += T) fin[2] += L.cmass[L.cact[q]];
    }
    block_reduce<T, 4>(fin, fop, L.ckey);  // its barriers also order the order-tie atomics
    if (tid == 0) {
        A.costs[p] = status == NNSEMD_OK ? fin[0] : NAN;
        if (A.stats != nullptr) {
            nnsemd_stats_t st;
            st.status = status;
            st.rounds = rounds;
            st.nnz = nnz;
            st.work = work;
            st.rescored = 0;
            st.residual_src = fin[1];
            st.residual_dst = fin[2];
            st.near_ties_nn = (int64_t)fin[3];
            st.near_ties_order = (int64_t)sh.tie_order;
            A.stats[p] = st;
        }
    }
}

template <typename TD, int T, int CSMAX>
__global__ __launch_bounds__(T) void cost_pair_kernel(CostArgs A) {
    extern __shared__ __align__(16) char lds_dyn[];
    __shared__ SharedCore sh;
    const Lds16 L = carve16(lds_dyn, A.max_m, A.max_n, 0, 0, true);
    const int64_t p = A.order != nullptr ? (int64_t)A.order[blockIdx.x] : A.pair_base + (int64_t)blockIdx.x;
    solve_cost_pair<TD, T, CSMAX>(A, p, L, sh);
}

// ---------------------------------------------------------------------
// Exact L1 distance matrices of high-dimensional pairs.  The L1 key is not a
// contraction (no matrix-core form); it is summed in FP64 in dimension order
// with the definition's operations (subtract, absolute value, add), which
// are the same on every machine, so each entry equals the FP64 definition's
// bit for bit and the given-D solver then needs no rounding bound at all.
// One workgroup per pair: 32 x 32 output blocks, 2 x 2 entries per thread,
// the rows of the block staged in LDS 32 coordinates at a time (as FP64;
// BF16 and FP32 values convert exactly); each thread carries its four sums
// across the stages, so the summation order is the dimension order.
constexpr int kL1Block = 32;
constexpr int kL1K = 32;

__device__ inline double l1_in(const uint16_t* p, int64_t k) { return (double)__uint_as_float((uint32_t)p[k] << 16); }
__device__ inline double l1_in(const float* p, int64_t k) { return (double)p[k]; }

template <typename TIn>
__global__ __launch_bounds__(256) void l1_tile_kernel(DocArgs A, double* __restrict__ tiles, int64_t stride) {
#pragma clang fp contract(off)
    __shared__ double xs[kL1Block][kL1K + 1];
    __shared__ double ys[kL1Block][kL1K + 1];
    const int64_t p = A.pair_base + blockIdx.x;
    int64_t x0 = 0, y0 = 0, m = A.single_m, n = A.single_n;
    if (A.x_off != nullptr) {
        const int64_t px = A.pair_x ? (int64_t)A.pair_x[p] : p;
        const int64_t py = A.pair_y ? (int64_t)A.pair_y[p] : p;
        if (px < 0 || px >= A.num_x_sets || py < 0 || py >= A.num_y_sets) return;  // the solver reports it
        x0 = A.x_off[px];
        m = A.x_off[px + 1] - x0;
        y0 = A.y_off[py];
        n = A.y_off[py + 1] - y0;
    }
    if (m <= 0 || n <= 0 || m > A.max_m || n > A.max_n) return;
    const int d = A.d;
    const TIn* __restrict__ X = reinterpret_cast<const TIn*>(A.X) + x0 * d;
    const TIn* __restrict__ Y = reinterpret_cast<const TIn*>(A.Y) + y0 * d;
    double* __restrict__ T = tiles + (int64_t)blockIdx.x * stride;
    const int tid = threadIdx.x;
    const int ti = tid / 16, tj = tid % 16;
    for (int64_t i0 = 0; i0 < m; i0 += kL1Block) {
        for (int64_t j0 = 0; j0 < n; j0 += kL1Block) {
            double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
            for (int k0 = 0; k0 < d; k0 += kL1K) {
                const int kc = min(kL1K, d - k0);
                for (int e = tid; e < kL1Block * kL1K; e += 256) {
                    const int r = e / kL1K, k = e % kL1K;
                    const bool kin = k < kc;
                    xs[r][k] = (kin && i0 + r < m) ? l1_in(X, (i0 + r) * d + k0 + k) : 0.0;
                    ys[r][k] = (kin && j0 + r < n) ? l1_in(Y, (j0 + r) * d + k0 + k) : 0.0;
                }
                __syncthreads();
                for (int k = 0; k < kc; ++k) {
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int b = 0; b < 2; ++b)
                            acc[a][b] = acc[a][b] + fabs(xs[2 * ti + a][k] - ys[2 * tj + b][k]);
                }
                __syncthreads();
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const int64_t i = i0 + 2 * ti + a, j = j0 + 2 * tj + b;
                    if (i < m && j < n) T[i * n + j] = acc[a][b];
                }
        }
    }
}

template <typename TD, int T, int CSMAX>
int launch_typed(const CostArgs& A, size_t lds, int grid, hipStream_t st, int* blocks) {
    if (lds > 48 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)cost_pair_kernel<TD, T, CSMAX>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return (int)e;
    }
    if (blocks != nullptr)
        return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, cost_pair_kernel<TD, T, CSMAX>, T, lds);
    hipLaunchKernelGGL((cost_pair_kernel<TD, T, CSMAX>), dim3(grid), dim3(T), lds, st, A);
    return (int)hipGetLastError();
}

}  // namespace

int launch_l1_tiles(const DocArgs& A, bool bf16, double* tiles, int64_t tile_stride, int grid, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    if (grid <= 0) return 0;
    if (bf16)
        hipLaunchKernelGGL(l1_tile_kernel<uint16_t>, dim3(grid), dim3(256), 0, st, A, tiles, tile_stride);
    else
        hipLaunchKernelGGL(l1_tile_kernel<float>, dim3(grid), dim3(256), 0, st, A, tiles, tile_stride);
    return (int)hipGetLastError();
}

int launch_cost_solver(const CostArgs& A, bool f64, int chunk_max, size_t lds, int grid, void* stream, int* blocks) {
    hipStream_t st = (hipStream_t)stream;
    if (chunk_max <= 4)
        return f64 ? launch_typed<double, 256, 4>(A, lds, grid, st, blocks)
                   : launch_typed<float, 256, 4>(A, lds, grid, st, blocks);
    if (chunk_max <= 16)
        return f64 ? launch_typed<double, 256, 16>(A, lds, grid, st, blocks)
                   : launch_typed<float, 256, 16>(A, lds, grid, st, blocks);
    return (int)hipErrorInvalidValue;
}

}  // namespace nnsemd
