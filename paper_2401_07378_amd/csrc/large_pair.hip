// Multi-workgroup NNS-EMD for one pair of any size (low-dimensional FP32
// points), and the per-supplier barycentric transport map of its plan.
//
// Each round of Algorithm 1 (Sec. III-A) is a fixed sequence of kernels over
// the whole device; the round state (active sizes, counters, the index of the
// live ping-pong buffer) lives in a device struct, so the host enqueues
// rounds without reading anything back and only synchronises every few
// rounds to shrink the grids.
//   search   consumer blocks x supplier chunks; supplier records staged in
//            LDS tiles; FP32 best / second-best per (chunk, consumer)
//   decide   merge the chunk partials; near ties (FP32 rounding bound) go to
//            the FP64 re-score list, others store pick + exact FP64 key and
//            count themselves into the pick's bucket
//   rescore  FP64 argmin of near-tie consumers, one workgroup each: FP32
//            keys filter the suppliers, FP64 keys decide among the rest
//   offsets  exclusive scan of the bucket counts (one workgroup)
//   scatter  claimants into buckets
//   serve    one wavefront per claimed supplier selects its claimants in
//            (D, j) (or random-key) order while it holds mass and serves
//            them in FP64: only the served prefix of the order is formed
//   compact  plan append + surviving suppliers / consumers: per-block counts,
//            stable writes at the blocks' offsets, one-thread commit
// Cost and map are accumulated per supplier (local index) in serve order, so
// results are deterministic and the map equals the definition bit for bit.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "internal.hpp"
#include "point_search.hpp"
#include "round_common.hpp"

namespace nnsemd {
namespace {

constexpr int kWave = 64;
constexpr int kLpThreads = 256;
constexpr int kLpScanThreads = 1024;
constexpr int kLpTile = 1024;   // supplier records per LDS tile in the search
constexpr int kLpUnroll = 8;

// The round kernels run while the pair is unfinished and the
// single-workgroup finish has not taken over.
__device__ inline bool lp_live(const LPState* st) { return st->status == NNSEMD_OK && !st->done && !st->tail; }

template <int D, bool L1>
__device__ inline double lp_key64(const float* __restrict__ x, const float* __restrict__ y) {
#pragma clang fp contract(off)
    double acc = 0.0;
#pragma unroll
    for (int t = 0; t < D; ++t) {
        double diff = (double)x[t] - (double)y[t];
        if (L1)
            acc = acc + fabs(diff);
        else
            acc = acc + diff * diff;
    }
    return acc;
}

// Search gap bound of the FP32 keys, as in the one-workgroup path: one key
// of a consumer is within B = (2D + 2) u e^2 (e = rhat + ||y^||) of
// ||x - y||^2 - ||y^||^2 -- D roundings of the record's norm, D of the FMA
// chain, 2u e^2 from centring both points -- so a wrong FP32 argmin needs a
// second key within 2B of the best; the threshold 4B = 8 (D + 1) u e^2 leaves
// a factor 2.  L1 keys: relative error D u each, threshold 4 (D + 1) u b1.
template <int D>
__device__ inline float lp_gap_bound(float rhat, float yn2) {
    const float e = rhat + sqrtf(yn2);
    return 8.f * (float)(D + 1) * kU32 * e * e + 1e-30f;
}

template <int D>
__device__ inline float lp_gap_bound_l1(float b1) {
    return 4.f * (float)(D + 1) * kU32 * b1 + 1e-30f;
}

// Near tie: two distances whose gap is at most 1e-6 relative (1e-12 at 0).
__device__ inline bool lp_near_tie(double d1, double d2) {
    const double gap = d2 - d1;
    return d1 == 0.0 ? gap <= 1e-12 : gap <= 1e-6 * d1;
}

// Key-space width past the bound in which a near tie may hide (squared keys:
// a 1e-6 distance gap is at most (2e-6 + 1e-12) of the squared distance).
__device__ inline float lp_near_window(float kmax, bool l1) {
    return (l1 ? 1.1e-6f : 2.2e-6f) * fmaxf(kmax, 0.f) + 1e-12f;
}

__device__ inline double lp_dist(double key, int metric) { return metric == NNSEMD_L2 ? sqrt(key) : key; }

__device__ inline uint64_t lp_rp_key(uint64_t seed, int64_t round, int32_t j) {
    uint64_t ctr = ((uint64_t)round << 32) ^ (uint64_t)(uint32_t)j;
    uint64_t z = seed + (ctr + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Exclusive scan of one 64-bit value per thread over a workgroup of T.
template <int T>
__device__ inline unsigned long long lp_block_scan(unsigned long long v, unsigned long long* total,
                                                   unsigned long long* scratch) {
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    unsigned long long x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        unsigned long long y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) scratch[w] = x;
    __syncthreads();
    unsigned long long off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < T / kWave; ++k) {
        unsigned long long s = scratch[k];
        off += (k < w) ? s : 0ull;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + x - v;
}

template <int T>
__device__ inline double lp_block_sum(double v, double* scratch) {
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) scratch[w] = v;
    __syncthreads();
    double r = scratch[0];
#pragma unroll
    for (int k = 1; k < T / kWave; ++k) r += scratch[k];
    __syncthreads();
    return r;
}

// Adds one to cnt[t] for every active lane of the wavefront and returns the
// lane's rank among the adds to its target.  Lanes with equal targets are
// combined behind one atomic (up to kLpAggPasses targets per wavefront, the
// rest add alone), so thousands of consumers picking one supplier do not
// serialise on its counter.  Call with the whole wavefront.
constexpr int kLpAggPasses = 4;

__device__ inline int lp_count_rank(int* cnt, int t, bool active) {
    const int lane = threadIdx.x & (kWave - 1);
    bool todo = active;
    int rank = 0;
#pragma unroll 1
    for (int pass = 0; pass < kLpAggPasses; ++pass) {
        const unsigned long long m = __ballot(todo);
        if (m == 0ull) return rank;
        const int leader = __builtin_ctzll(m);
        const int lt = __shfl(t, leader);
        const bool mine = todo && t == lt;
        const unsigned long long same = __ballot(mine);
        int base = 0;
        if (lane == leader) base = atomicAdd(&cnt[lt], __popcll(same));
        base = __shfl(base, leader);
        if (mine) {
            rank = base + __popcll(same & ((1ull << lane) - 1ull));
            todo = false;
        }
    }
    if (todo) rank = atomicAdd(&cnt[t], 1);
    return rank;
}

// ---------------------------------------------------------------- ingest
// Per block: masses to FP64, validity, sums, bounding box partials.
template <int D>
__global__ __launch_bounds__(kLpThreads) void lp_ingest(LPArgs A) {
    __shared__ double scratch[kLpThreads / kWave][3 + 2 * D];
    const int tid = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * kLpThreads + tid;
    double v[3 + 2 * D];
    v[0] = 0.0;
    v[1] = 0.0;
    v[2] = 0.0;
#pragma unroll
    for (int t = 0; t < D; ++t) {
        v[3 + t] = INFINITY;
        v[3 + D + t] = -INFINITY;
    }
    if (i < A.m) {
        const float av = A.a[i];
        if (!(av >= 0.f) || !isfinite(av)) v[2] = 1.0;
        v[0] = (double)av;
        A.w.smass[0][i] = (double)av;
#pragma unroll
        for (int t = 0; t < D; ++t) {
            const float xv = A.X[i * D + t];
            if (!isfinite(xv)) v[2] = 1.0;
            v[3 + t] = (double)xv;
            v[3 + D + t] = (double)xv;
        }
        A.w.costacc[i] = 0.0;
        if (A.w.wsum != nullptr) {
            A.w.wsum[i] = 0.0;
#pragma unroll
            for (int t = 0; t < D; ++t) A.w.bsum[i * D + t] = 0.0;
        }
    }
    if (i < A.n) {
        A.w.thead[i] = -1;  // bin tables of the near-tie count start empty
        const float bv = A.b[i];
        if (!(bv >= 0.f) || !isfinite(bv)) v[2] = 1.0;
        v[1] = (double)bv;
        A.w.cmass[i] = (double)bv;
#pragma unroll
        for (int t = 0; t < D; ++t)
            if (!isfinite(A.Y[i * D + t])) v[2] = 1.0;
    }
    const int lane = tid & (kWave - 1), w = tid / kWave;
#pragma unroll
    for (int k = 0; k < 3 + 2 * D; ++k) {
        double x = v[k];
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) {
            const double y = __shfl_xor(x, o);
            x = (k < 2) ? x + y : (k < 3 + D && k >= 3) ? fmin(x, y) : fmax(x, y);
        }
        if (lane == 0) scratch[w][k] = x;
    }
    __syncthreads();
    if (tid < 3 + 2 * D) {
        const int k = tid;
        double x = scratch[0][k];
        for (int q = 1; q < kLpThreads / kWave; ++q) {
            const double y = scratch[q][k];
            x = (k < 2) ? x + y : (k < 3 + D && k >= 3) ? fmin(x, y) : fmax(x, y);
        }
        A.w.red[(size_t)blockIdx.x * (3 + 2 * D) + k] = x;
    }
}

// ----------------------------------------------------------------- setup
// One workgroup: reduce the ingest partials, check, centre, build the first
// active sets (in buffer 1; buffer 0 holds the masses by local index) and the
// radius that enters the FP32 rounding bound.
template <int D, bool L1>
__global__ __launch_bounds__(kLpScanThreads) void lp_setup(LPArgs A, int nblocks) {
    constexpr int RS = record_stride(D);
    constexpr int K = 3 + 2 * D;
    __shared__ double red[K];
    __shared__ unsigned long long scan_scratch[kLpScanThreads / kWave];
    __shared__ double sum_scratch[kLpScanThreads / kWave];
    const int tid = threadIdx.x;
    LPState* st = A.w.st;
    if (tid < K) {
        const int k = tid;
        double x = (k < 2) ? 0.0 : (k == 2 ? 0.0 : (k < 3 + D ? INFINITY : -INFINITY));
        for (int b = 0; b < nblocks; ++b) {
            const double y = A.w.red[(size_t)b * K + k];
            x = (k < 2) ? x + y : (k == 2 ? fmax(x, y) : (k < 3 + D ? fmin(x, y) : fmax(x, y)));
        }
        red[k] = x;
    }
    __syncthreads();
    int status = NNSEMD_OK;
    if (red[2] != 0.0) status = NNSEMD_ERR_INVALID_ARG;
    if (status == NNSEMD_OK) {
        const double big = fmax(red[0], red[1]);
        if (fabs(red[0] - red[1]) > 1e-5 * big) status = NNSEMD_ERR_MASS_MISMATCH;
    }
    float centre[D];
#pragma unroll
    for (int t = 0; t < D; ++t)
        centre[t] = (L1 || A.m == 0) ? 0.f : 0.5f * ((float)red[3 + t] + (float)red[3 + D + t]);
    const int m = (int)A.m, n = (int)A.n;
    // initial compaction (zero masses never enter), chunked per thread
    const int cs = (m + kLpScanThreads - 1) / kLpScanThreads;
    const int cc = (n + kLpScanThreads - 1) / kLpScanThreads;
    const int slo = min(tid * cs, m), shi = min(slo + cs, m);
    const int clo = min(tid * cc, n), chi = min(clo + cc, n);
    int ks = 0, kc = 0;
    if (status == NNSEMD_OK) {
        for (int i = slo; i < shi; ++i) ks += A.w.smass[0][i] > 0.0;
        for (int j = clo; j < chi; ++j) kc += A.w.cmass[j] > 0.0;
    }
    unsigned long long tot;
    const unsigned long long pre =
        lp_block_scan<kLpScanThreads>((unsigned long long)ks | ((unsigned long long)kc << 32), &tot, scan_scratch);
    int ps = (int)(pre & 0xffffffffu), pc = (int)(pre >> 32);
    float rmax = 0.f;
    if (status == NNSEMD_OK) {
        // Records are written to buffer 1 first (buffer 0 still holds the
        // masses by local index), then the masses follow.
        for (int i = slo; i < shi; ++i) {
            const double mv = A.w.smass[0][i];
            if (!(mv > 0.0)) continue;
            float r[RS];
#pragma unroll
            for (int q = 0; q < RS; ++q) r[q] = 0.f;
            if (L1) {
#pragma unroll
                for (int t = 0; t < D; ++t) r[t] = A.X[(int64_t)i * D + t];
            } else {
                float h = 0.f;
#pragma unroll
                for (int t = 0; t < D; ++t) {
                    const float xc = A.X[(int64_t)i * D + t] - centre[t];
                    r[t] = -2.f * xc;
                    h = fmaf(xc, xc, h);
                }
                r[D] = h;
                rmax = fmaxf(rmax, sqrtf(h));
            }
            float4* dst = reinterpret_cast<float4*>(A.w.srec[1] + (size_t)ps * RS);
#pragma unroll
            for (int q = 0; q < RS / 4; ++q) dst[q] = make_float4(r[4 * q], r[4 * q + 1], r[4 * q + 2], r[4 * q + 3]);
            A.w.sidx[1][ps] = i;
            A.w.smass[1][ps] = mv;
            A.w.scnt[ps] = 0;
            ++ps;
        }
        for (int j = clo; j < chi; ++j)
            if (A.w.cmass[j] > 0.0) A.w.cact[1][pc++] = j;
    }
    // max radius (positive floats order like their bit patterns)
    __shared__ unsigned int rbits;
    if (tid == 0) rbits = 0u;
    __syncthreads();
    atomicMax(&rbits, __float_as_uint(rmax));
    (void)sum_scratch;
    __syncthreads();
    if (tid == 0) {
        st->status = status;
        st->mact = status == NNSEMD_OK ? (int)(tot & 0xffffffffu) : 0;
        st->nact = status == NNSEMD_OK ? (int)(tot >> 32) : 0;
        st->nflag = 0;
        st->nnz = 0;
        st->work = 0;
        st->near = 0;
        st->ties_nn = 0;
        st->ties_order = 0;
        st->rounds = 0;
        st->ticket = 0;
        st->parity = 1;
        st->done = (st->mact == 0 || st->nact == 0) ? 1 : 0;
        st->tail = (!st->done && st->mact <= A.tail_cap && st->nact <= A.tail_cap) ? 1 : 0;
        st->rhat = __uint_as_float(rbits) * (1.f + 1e-6f);
#pragma unroll
        for (int t = 0; t < D; ++t) st->centre[t] = centre[t];
        st->sum_a = red[0];
        st->sum_b = red[1];
    }
}

// ---------------------------------------------------------------- search
// FP32 search key of one record: L1 sums |x_t - y_t| in dimension order;
// the Euclidean metrics run the FMA chain ||x^||^2 + sum_t (-2 x^_t) y^_t.
template <int D, int RS, bool L1>
__device__ inline float lp_key(const float (&rec)[RS], const float (&y)[D]) {
    float key;
    if (L1) {
        key = 0.f;
#pragma unroll
        for (int t = 0; t < D; ++t) key += fabsf(rec[t] - y[t]);
    } else {
        key = rec[D];
#pragma unroll
        for (int t = D - 1; t >= 0; --t) key = fmaf(rec[t], y[t], key);
    }
    return key;
}

template <int D, bool L1, int KC>
__global__ __launch_bounds__(kLpThreads) void lp_search(LPArgs A, int split) {
    constexpr int RS = record_stride(D);
    __shared__ __align__(16) float tile[kLpTile * RS];
    const LPState* st = A.w.st;
    if (!lp_live(st)) return;
    const int mact = st->mact, nact = st->nact, par = st->parity;
    const int tid = threadIdx.x;
    const int base = blockIdx.x * kLpThreads * KC;
    if (base >= nact) return;
    const int chunk = (mact + split - 1) / split;
    const int s_lo = min((int)blockIdx.y * chunk, mact), s_hi = min(s_lo + chunk, mact);
    const float* __restrict__ srec = A.w.srec[par];
    const int* __restrict__ cact = A.w.cact[par];
    float y[KC][D];
    float b1[KC], b2[KC];
    int bs[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        const int q = base + tid + k * kLpThreads;
        const int j = cact[q < nact ? q : 0];
#pragma unroll
        for (int t = 0; t < D; ++t) y[k][t] = L1 ? A.Y[(int64_t)j * D + t] : A.Y[(int64_t)j * D + t] - st->centre[t];
        b1[k] = INFINITY;
        b2[k] = INFINITY;
        bs[k] = 0x7fffffff;
    }
    // Blocks of kLpUnroll records: two keys at a time update (b1, b2) as
    // b2 <- min(b2, med3(b1, ka, kb)), b1 <- min(b1, ka, kb) (the two smallest
    // of the multiset); only the block in which b1 last fell strictly is
    // remembered, and its records are scanned again at the end (from the
    // global records, the same FP32 values) for the first slot holding b1.
    // Records past the last full block (the chunk's tail) keep their slot
    // directly; they come after every block, so a fall there is the last.
    int blk[KC], bsr[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        blk[k] = -1;
        bsr[k] = -1;
    }
    for (int t0 = s_lo; t0 < s_hi; t0 += kLpTile) {
        const int cnt = min(kLpTile, s_hi - t0);
        const float4* src = reinterpret_cast<const float4*>(srec + (size_t)t0 * RS);
        float4* dst = reinterpret_cast<float4*>(tile);
        for (int e = tid; e < cnt * (RS / 4); e += kLpThreads) dst[e] = src[e];
        __syncthreads();
        const int full = (cnt / kLpUnroll) * kLpUnroll;
        for (int s0 = 0; s0 < full; s0 += kLpUnroll) {
            float rec[kLpUnroll][RS];
#pragma unroll
            for (int u = 0; u < kLpUnroll; ++u) {
                const float4* p = reinterpret_cast<const float4*>(tile + (size_t)(s0 + u) * RS);
#pragma unroll
                for (int q = 0; q < RS / 4; ++q) {
                    const float4 v = p[q];
                    rec[u][4 * q] = v.x;
                    rec[u][4 * q + 1] = v.y;
                    rec[u][4 * q + 2] = v.z;
                    rec[u][4 * q + 3] = v.w;
                }
            }
            float b1o[KC];
#pragma unroll
            for (int k = 0; k < KC; ++k) b1o[k] = b1[k];
#pragma unroll
            for (int u = 0; u < kLpUnroll; u += 2) {
#pragma unroll
                for (int k = 0; k < KC; ++k) {
                    const float ka = lp_key<D, RS, L1>(rec[u], y[k]);
                    const float kb = lp_key<D, RS, L1>(rec[u + 1], y[k]);
                    b2[k] = fminf(b2[k], __builtin_amdgcn_fmed3f(b1[k], ka, kb));
                    b1[k] = fminf(b1[k], fminf(ka, kb));
                }
            }
#pragma unroll
            for (int k = 0; k < KC; ++k) blk[k] = b1[k] < b1o[k] ? t0 + s0 : blk[k];
        }
        for (int s = full; s < cnt; ++s) {
            float rec[RS];
#pragma unroll
            for (int q = 0; q < RS; ++q) rec[q] = tile[(size_t)s * RS + q];
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                const float key = lp_key<D, RS, L1>(rec, y[k]);
                const bool lt = key < b1[k];
                bsr[k] = lt ? t0 + s : bsr[k];
                b2[k] = __builtin_amdgcn_fmed3f(b1[k], key, b2[k]);
                b1[k] = fminf(b1[k], key);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        bs[k] = bsr[k];
        if (bsr[k] < 0 && blk[k] >= 0) {
            int u = kLpUnroll - 1;
#pragma unroll
            for (int v = kLpUnroll - 2; v >= 0; --v) {
                float rv[RS];
                const float4* p = reinterpret_cast<const float4*>(srec + (size_t)(blk[k] + v) * RS);
#pragma unroll
                for (int q = 0; q < RS / 4; ++q) {
                    const float4 w = p[q];
                    rv[4 * q] = w.x;
                    rv[4 * q + 1] = w.y;
                    rv[4 * q + 2] = w.z;
                    rv[4 * q + 3] = w.w;
                }
                u = lp_key<D, RS, L1>(rv, y[k]) == b1[k] ? v : u;
            }
            bs[k] = blk[k] + u;
        } else if (bsr[k] < 0) {
            bs[k] = 0x7fffffff;
        }
    }
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        const int q = base + tid + k * kLpThreads;
        if (q < nact)
            A.w.part[(size_t)blockIdx.y * A.w.ncap + q] = make_float4(b1[k], b2[k], __int_as_float(bs[k]), 0.f);
    }
}

// ---------------------------------------------------------------- decide
// Best / second-best merge of two FP32 partials; equal keys keep the smaller
// slot, so the result does not depend on the merge order.
__device__ inline void lp_merge2(float& b1, float& b2, int& bs, float x1, float x2, int xs) {
    const float n2 = fminf(fmaxf(b1, x1), fminf(b2, x2));
    const bool take = (x1 < b1) || (x1 == b1 && xs < bs);
    b1 = take ? x1 : b1;
    bs = take ? xs : bs;
    b2 = n2;
}

// kLpDecideSub lanes per consumer merge the supplier chunks' partials (four
// loads in flight each), then combine by shuffles; the first lane decides.
constexpr int kLpDecideSub = 8;
constexpr int kLpDecideBatch = 4;

template <int D, bool L1>
__global__ __launch_bounds__(kLpThreads) void lp_decide(LPArgs A, int split) {
    LPState* st = A.w.st;
    if (!lp_live(st)) return;
    const int nact = st->nact, par = st->parity;
    const int sub = threadIdx.x & (kLpDecideSub - 1);
    const int q = blockIdx.x * (kLpThreads / kLpDecideSub) + threadIdx.x / kLpDecideSub;
    const bool valid = q < nact;  // the whole wavefront stays for the shuffles and counting
    float b1 = INFINITY, b2 = INFINITY;
    int bs = 0x7fffffff;
    if (valid) {
        for (int c0 = sub; c0 < split; c0 += kLpDecideBatch * kLpDecideSub) {
            float4 v[kLpDecideBatch];
#pragma unroll
            for (int u = 0; u < kLpDecideBatch; ++u) {
                const int c = c0 + u * kLpDecideSub;
                v[u] = c < split ? A.w.part[(size_t)c * A.w.ncap + q]
                                 : make_float4(INFINITY, INFINITY, __int_as_float(0x7fffffff), 0.f);
            }
#pragma unroll
            for (int u = 0; u < kLpDecideBatch; ++u) lp_merge2(b1, b2, bs, v[u].x, v[u].y, __float_as_int(v[u].z));
        }
    }
#pragma unroll
    for (int o = 1; o < kLpDecideSub; o <<= 1) {
        const float x1 = __shfl_xor(b1, o), x2 = __shfl_xor(b2, o);
        const int xs = __shfl_xor(bs, o);
        lp_merge2(b1, b2, bs, x1, x2, xs);
    }
    const bool live = valid && sub == 0;
    const int j = live ? A.w.cact[par][q] : 0;
    // Gap threshold: the proven per-key bound B taken twice, with a factor 2
    // of margin (derivation at lp_gap_bound), plus the near-tie window.
    float win;
    if (L1) {
        win = lp_gap_bound_l1<D>(b1) + lp_near_window(b1, true);
    } else {
        float yn2 = 0.f;
#pragma unroll
        for (int t = 0; t < D; ++t) {
            const float yv = A.Y[(int64_t)j * D + t] - st->centre[t];
            yn2 = fmaf(yv, yv, yn2);
        }
        const float thr = lp_gap_bound<D>(st->rhat, yn2);
        win = thr + lp_near_window(b1 + yn2 + thr, false);
    }
    const bool near = live && !(b2 - b1 > win);
    const bool pick = live && !near;
    // The FP64 argmin's FP32 key lies within 2B of b1 (half the bound part of
    // win), and a supplier that is a near tie with it within 2B + the window,
    // so b1 + win bounds every candidate the re-score must see.
    const int f = lp_count_rank(&st->nflag, 0, near);
    if (near) {
        A.w.flagged[f] = j;
        A.w.ckey[j] = (double)(b1 + win);
    }
    // rank within the pick's bucket (sorted is free until the serve)
    const int r = lp_count_rank(A.w.scnt, pick ? bs : 0, pick);
    if (pick) {
        const int i = A.w.sidx[par][bs];
        A.w.cnn[j] = bs;
        A.w.ckey[j] = lp_key64<D, L1>(A.X + (int64_t)i * D, A.Y + (int64_t)j * D);
        A.w.sorted[j] = r;
    }
}

// --------------------------------------------------------------- rescore
// One workgroup per near-tie consumer: every active supplier's FP32 key is
// formed again from the slot records (contiguous, as in the search); only
// those at or below the cutoff that decide stored (a NaN key or cutoff lets
// every supplier through) are re-scored in FP64 from the original points.
// The argmin over (FP64 key, slot) is order-free, hence deterministic.
constexpr int kLpRescoreThreads = 1024;
constexpr int kLpRescoreUnroll = 4;

template <int D, bool L1>
__global__ __launch_bounds__(kLpRescoreThreads) void lp_rescore(LPArgs A) {
    constexpr int RS = record_stride(D);
    constexpr int NW = kLpRescoreThreads / kWave;
    __shared__ double sk[NW];
    __shared__ double s2[NW];
    __shared__ int ss[NW];
    LPState* st = A.w.st;
    if (!lp_live(st)) return;
    const int nf = st->nflag, mact = st->mact, par = st->parity;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    const float* __restrict__ srec = A.w.srec[par];
    const int* __restrict__ sidx = A.w.sidx[par];
    for (int f = blockIdx.x; f < nf; f += gridDim.x) {
        const int j = A.w.flagged[f];
        const float* yp = A.Y + (int64_t)j * D;
        const float cut = (float)A.w.ckey[j];
        float y[D];
#pragma unroll
        for (int t = 0; t < D; ++t) y[t] = L1 ? yp[t] : yp[t] - st->centre[t];
        double best = INFINITY, sec = INFINITY;
        int bsl = 0x7fffffff;
        for (int s0 = tid; s0 < mact; s0 += kLpRescoreThreads * kLpRescoreUnroll) {
            float key[kLpRescoreUnroll];
#pragma unroll
            for (int u = 0; u < kLpRescoreUnroll; ++u) {
                const int s = s0 + u * kLpRescoreThreads;
                float rec[RS];
                const float4* p = reinterpret_cast<const float4*>(srec + (size_t)(s < mact ? s : 0) * RS);
#pragma unroll
                for (int q = 0; q < RS / 4; ++q) {
                    const float4 v = p[q];
                    rec[4 * q] = v.x;
                    rec[4 * q + 1] = v.y;
                    rec[4 * q + 2] = v.z;
                    rec[4 * q + 3] = v.w;
                }
                float kv;
                if (L1) {
                    kv = 0.f;
#pragma unroll
                    for (int t = 0; t < D; ++t) kv += fabsf(rec[t] - y[t]);
                } else {
                    kv = rec[D];
#pragma unroll
                    for (int t = D - 1; t >= 0; --t) kv = fmaf(rec[t], y[t], kv);
                }
                key[u] = kv;
            }
#pragma unroll
            for (int u = 0; u < kLpRescoreUnroll; ++u) {
                const int s = s0 + u * kLpRescoreThreads;
                if (s < mact && !(key[u] > cut)) {
                    const double k = lp_key64<D, L1>(A.X + (int64_t)sidx[s] * D, yp);
                    if (k < best) {  // slots rise along the thread's walk: ties keep the first
                        sec = best;
                        best = k;
                        bsl = s;
                    } else if (k < sec) {
                        sec = k;
                    }
                }
            }
        }
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) {
            const double cb = __shfl_xor(best, o);
            const double c2 = __shfl_xor(sec, o);
            const int cs = __shfl_xor(bsl, o);
            sec = fmin(fmax(best, cb), fmin(sec, c2));
            if (cb < best || (cb == best && cs < bsl)) {
                best = cb;
                bsl = cs;
            }
        }
        if (lane == 0) {
            sk[w] = best;
            ss[w] = bsl;
            s2[w] = sec;
        }
        __syncthreads();
        if (tid == 0) {
#pragma unroll
            for (int k = 1; k < NW; ++k) {
                sec = fmin(fmax(best, sk[k]), fmin(sec, s2[k]));
                if (sk[k] < best || (sk[k] == best && ss[k] < bsl)) {
                    best = sk[k];
                    bsl = ss[k];
                }
            }
            A.w.cnn[j] = bsl;
            A.w.ckey[j] = best;
            A.w.sorted[j] = atomicAdd(&A.w.scnt[bsl], 1);
            // The second-nearest supplier is among the survivors of the cut
            // whenever it is a near tie with the nearest one.
            if (mact > 1 && lp_near_tie(lp_dist(best, A.metric), lp_dist(sec, A.metric)))
                atomicAdd((unsigned long long*)&st->ties_nn, 1ull);
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------- offsets
// Exclusive scan of the bucket counts into bucket starts.  Each thread owns
// a run of counts starting at a multiple of four (16-byte loads and stores);
// runs of up to 4 kLpOffRegs counts (up to 65536 suppliers) are loaded all at
// once and kept in registers.
constexpr int kLpOffRegs = 16;

__global__ __launch_bounds__(kLpScanThreads) void lp_offsets(LPArgs A) {
    __shared__ unsigned long long scratch[kLpScanThreads / kWave];
    LPState* st = A.w.st;
    if (!lp_live(st)) return;
    const int mact = st->mact;
    const int tid = threadIdx.x;
    const int cs = (((mact + kLpScanThreads - 1) / kLpScanThreads) + 3) & ~3;
    const int lo = min(tid * cs, mact), hi = min(lo + cs, mact);
    const int hq = lo + ((hi - lo) & ~3);
    const int* __restrict__ cnt = A.w.scnt;
    if (cs <= 4 * kLpOffRegs) {
        int4 v[kLpOffRegs];
        int sum = 0;
#pragma unroll
        for (int u = 0; u < kLpOffRegs; ++u) {
            const int s = lo + 4 * u;
            v[u] = s < hq ? *reinterpret_cast<const int4*>(cnt + s) : make_int4(0, 0, 0, 0);
        }
        int tail[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) tail[k] = hq + k < hi ? cnt[hq + k] : 0;
#pragma unroll
        for (int u = 0; u < kLpOffRegs; ++u) sum += (v[u].x + v[u].y) + (v[u].z + v[u].w);
        sum += tail[0] + tail[1] + tail[2];
        unsigned long long tot;
        int run = (int)lp_block_scan<kLpScanThreads>((unsigned long long)sum, &tot, scratch);
#pragma unroll
        for (int u = 0; u < kLpOffRegs; ++u) {
            const int s = lo + 4 * u;
            if (s < hq) {
                int4 o;
                o.x = run;
                o.y = o.x + v[u].x;
                o.z = o.y + v[u].y;
                o.w = o.z + v[u].z;
                run = o.w + v[u].w;
                *reinterpret_cast<int4*>(A.w.soff + s) = o;
            }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (hq + k < hi) {
                A.w.soff[hq + k] = run;
                run += tail[k];
            }
        }
        return;
    }
    int sum = 0;
#pragma unroll 4
    for (int s = lo; s < hq; s += 4) {
        const int4 v = *reinterpret_cast<const int4*>(cnt + s);
        sum += (v.x + v.y) + (v.z + v.w);
    }
    for (int s = hq; s < hi; ++s) sum += cnt[s];
    unsigned long long tot;
    int run = (int)lp_block_scan<kLpScanThreads>((unsigned long long)sum, &tot, scratch);
#pragma unroll 4
    for (int s = lo; s < hq; s += 4) {
        const int4 v = *reinterpret_cast<const int4*>(cnt + s);
        int4 o;
        o.x = run;
        o.y = o.x + v.x;
        o.z = o.y + v.y;
        o.w = o.z + v.z;
        run = o.w + v.w;
        *reinterpret_cast<int4*>(A.w.soff + s) = o;
    }
    for (int s = hq; s < hi; ++s) {
        A.w.soff[s] = run;
        run += cnt[s];
    }
}

// ------------------------------------------------------------------ ties
// Greedy protocol: near ties of neighbouring claimants in each supplier's
// serve order, over the whole bucket (served or not), on the exact FP64 keys
// the decide / re-score stored.  The count over a bucket depends only on its
// sorted keys, so any total order that sorts by key will do; (key, bucket
// position) is used.  A claimant counts when its predecessor in that order
// -- the largest member below it -- is a near tie of it.
//
// No sort: keys fall into bins of relative width 2^-18 .. 2^-17 (the FP64
// bit pattern shifted right by 35; every key below 2^-30 in bin 0), wider
// than any near-tie gap (2.1e-6 relative in squared keys, 1e-6 in distances,
// and 1e-12 at distance zero lies inside bin 0).  So if the predecessor is a
// near tie it lies in the claimant's bin or the one below, and the largest
// member below the claimant within those two bins is then the predecessor
// itself; if the two bins hold no member below it, the predecessor is at
// least a whole bin away and not a near tie.  Each bucket keeps a chained
// hash table of its members by bin, in its own span of bucket positions:
// heads (thead, all -1 between rounds), links (tnext) and the keys by
// position (tkey).  The scatter inserts, lp_ties queries, the serve clears
// the heads of its bucket for the next round.
constexpr double kLpTieBinFloor = 0x1p-30;

__device__ inline uint64_t lp_tie_bin(double k) {
    const uint64_t f = (uint64_t)__double_as_longlong(kLpTieBinFloor);
    return k < kLpTieBinFloor ? 0ull : (((uint64_t)__double_as_longlong(k) - f) >> 35) + 1ull;
}

__device__ inline int lp_tie_slot(uint64_t bin, int c) {
    const uint64_t h = (bin * 0x9E3779B97F4A7C15ull) >> 32;  // Fibonacci hashing
    return (int)((h * (uint64_t)c) >> 32);
}

// Near tie of two keys (L2: of their square roots).  The key-space test
// rejects every pair whose distances are more than (2e-6 + 1e-12) apart
// relative, so the square roots are taken only for candidates.
__device__ inline bool lp_keys_near(double k1, double k2, int metric) {
    if (metric == NNSEMD_L2 && k2 - k1 > 2.1e-6 * k1 + 1e-24) return false;
    return lp_near_tie(lp_dist(k1, metric), lp_dist(k2, metric));
}

// --------------------------------------------------------------- scatter
// Claimants into their buckets at the ranks the counting handed out; under
// the greedy protocol each member of a bucket of two or more also enters
// its bucket's bin table.
__global__ __launch_bounds__(kLpThreads) void lp_scatter(LPArgs A) {
    const LPState* st = A.w.st;
    if (!lp_live(st)) return;
    const int q = blockIdx.x * kLpThreads + threadIdx.x;
    if (q >= st->nact) return;
    const int j = A.w.cact[st->parity][q];
    const int s = A.w.cnn[j];
    const int start = A.w.soff[s];
    const int e = start + A.w.sorted[j];
    A.w.list[e] = j;
    const int c = A.w.scnt[s];
    if (A.protocol == NNSEMD_GREEDY && c > 1) {
        const double k = A.w.ckey[j];
        A.w.tkey[e] = k;
        A.w.tnext[e] = atomicExch(&A.w.thead[start + lp_tie_slot(lp_tie_bin(k), c)], e);
    }
}

// One thread per claimant: the largest member below it in its own bin and
// the bin below (an equal key at a smaller position ends the search: the
// predecessor then has the claimant's key), then the near-tie test.
__global__ __launch_bounds__(kLpThreads) void lp_ties(LPArgs A) {
    LPState* st = A.w.st;
    if (!lp_live(st)) return;
    const int q = blockIdx.x * kLpThreads + threadIdx.x;
    int hit = 0;
    if (q < st->nact) {
        const int j = A.w.cact[st->parity][q];
        const int s = A.w.cnn[j];
        const int c = A.w.scnt[s];
        if (c > 1) {
            const int start = A.w.soff[s];
            const int e = start + A.w.sorted[j];
            const double x = A.w.tkey[e];
            const uint64_t bx = lp_tie_bin(x);
            double pk = -1.0;  // keys are >= +0: -1 = no member below
            for (int db = 0; db < 2 && pk != x; ++db) {
                if (db == 1 && bx == 0ull) break;
                const uint64_t bb = bx - (uint64_t)db;
                for (int f = A.w.thead[start + lp_tie_slot(bb, c)]; f >= 0; f = A.w.tnext[f]) {
                    const double y = A.w.tkey[f];
                    if (f == e || lp_tie_bin(y) != bb) continue;
                    if (y < x || (y == x && f < e)) {
                        pk = fmax(pk, y);
                        if (pk == x) break;
                    }
                }
            }
            hit = pk >= 0.0 && lp_keys_near(pk, x, A.metric);
        }
    }
    const unsigned long long m = __ballot(hit != 0);
    if ((threadIdx.x & (kWave - 1)) == 0 && m != 0ull)
        atomicAdd((unsigned long long*)&st->ties_order, (unsigned long long)__popcll(m));
}

// ----------------------------------------------------------------- serve
// Claimant order and serve fused, one wavefront per claimed supplier.  The
// greedy protocol serves claimants in (key, j) order (the random one in
// (random key, j) order) while the supplier holds mass, so only that prefix
// of the order is needed: each step selects, by a wavefront-wide argmin,
// the smallest claimant above the previous one, and the supplier serves it
// with the definition's FP64 operations in the definition's order (one lane
// does the arithmetic).  Served claimants go to the bucket's head in serve
// order, unserved ones after them; flows replace keys after the walk (the
// selection compares keys until then); flowtmp is free scratch indexed by
// consumer.  Work O(served x bucket / 64) instead of O(bucket^2).
constexpr int kLpServeBatch = 4;  // bucket entries in flight per lane

template <int D>
__global__ __launch_bounds__(kLpThreads) void lp_serve(LPArgs A) {
#pragma clang fp contract(off)
    const LPState* st = A.w.st;
    if (!lp_live(st)) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int s = blockIdx.x * (kLpThreads / kWave) + threadIdx.x / kWave;
    const int par = st->parity;
    if (s >= st->mact) return;  // whole wavefronts
    const int c = A.w.scnt[s];
    if (c == 0) return;
    const int start = A.w.soff[s];
    const int end = start + c;
    const int isup = A.w.sidx[par][s];
    const bool greedy = A.protocol == NNSEMD_GREEDY;
    const uint64_t seed = A.seed;
    const int64_t rnd = st->rounds;
    double* flowtmp = reinterpret_cast<double*>(A.w.part);
    auto okey = [&](int j) -> uint64_t {
        // keys are >= +0, so their bit patterns order like the values
        return greedy ? (uint64_t)__double_as_longlong(A.w.ckey[j]) : lp_rp_key(seed, rnd, j);
    };
    double sm = A.w.smass[par][s];
    double acc = A.w.costacc[isup];
    uint64_t lk = 0;   // last served (key, j); nothing served yet
    int lj = -1;
    int served = 0;
    while (served < c && sm > 0.0) {
        uint64_t bk = ~0ull;
        int bj = 0x7fffffff;
        for (int e0 = start + lane; e0 < end; e0 += kLpServeBatch * kWave) {
            int jj[kLpServeBatch];
            uint64_t kk[kLpServeBatch];
#pragma unroll
            for (int u = 0; u < kLpServeBatch; ++u) {
                const int e = e0 + u * kWave;
                jj[u] = e < end ? A.w.list[e] : -1;
            }
#pragma unroll
            for (int u = 0; u < kLpServeBatch; ++u) kk[u] = jj[u] >= 0 ? okey(jj[u]) : 0ull;
#pragma unroll
            for (int u = 0; u < kLpServeBatch; ++u) {
                const int j = jj[u];
                const uint64_t k = kk[u];
                const bool above = lj < 0 || k > lk || (k == lk && j > lj);
                if (j >= 0 && above && (k < bk || (k == bk && j < bj))) {
                    bk = k;
                    bj = j;
                }
            }
        }
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) {
            const uint64_t ck = __shfl_xor(bk, o);
            const int cj = __shfl_xor(bj, o);
            if (ck < bk || (ck == bk && cj < bj)) {
                bk = ck;
                bj = cj;
            }
        }
        const double cm = A.w.cmass[bj];
        const double f = sm < cm ? sm : cm;
        sm = sm - f;
        if (lane == 0) {
            A.w.cmass[bj] = cm - f;
            const double key = A.w.ckey[bj];
            acc = acc + f * (A.metric == NNSEMD_L2 ? sqrt(key) : key);
            if (A.w.wsum != nullptr) {
                A.w.wsum[isup] = A.w.wsum[isup] + f;
#pragma unroll
                for (int t = 0; t < D; ++t)
                    A.w.bsum[(int64_t)isup * D + t] =
                        A.w.bsum[(int64_t)isup * D + t] + f * (double)A.Y[(int64_t)bj * D + t];
            }
            flowtmp[bj] = f;
            A.w.cnn[bj] = isup;
            A.w.sorted[start + served] = bj;
        }
        lk = bk;
        lj = bj;
        ++served;
    }
    // Unserved claimants (above the last served one, by their keys, which
    // nobody has changed yet) go after the served ones with flow 0; then lane
    // 0 replaces the served claimants' keys by their flows.
    int pos = start + served;
    for (int e0 = start + lane; e0 < end + lane; e0 += kLpServeBatch * kWave) {
        int jj[kLpServeBatch];
        uint64_t kk[kLpServeBatch];
#pragma unroll
        for (int u = 0; u < kLpServeBatch; ++u) {
            const int e = e0 + u * kWave;
            jj[u] = e < end ? A.w.list[e] : -1;
        }
#pragma unroll
        for (int u = 0; u < kLpServeBatch; ++u) kk[u] = jj[u] >= 0 ? okey(jj[u]) : 0ull;
#pragma unroll
        for (int u = 0; u < kLpServeBatch; ++u) {
            const int j = jj[u];
            const uint64_t k = kk[u];
            const bool un = j >= 0 && (lj < 0 || k > lk || (k == lk && j > lj));
            const uint64_t m = __ballot(un);
            if (un) {
                A.w.sorted[pos + __popcll(m & ((1ull << lane) - 1ull))] = j;
                A.w.ckey[j] = 0.0;
            }
            pos += __popcll(m);
        }
    }
    if (greedy && c > 1)  // the bin table of this bucket, empty again for the next round
        for (int e = start + lane; e < end; e += kWave) A.w.thead[e] = -1;
    if (lane == 0) {
        for (int q = start; q < start + served; ++q) {
            const int j = A.w.sorted[q];
            A.w.ckey[j] = flowtmp[j];
        }
        A.w.smass[par][s] = sm;
        A.w.costacc[isup] = acc;
    }
}

// --------------------------------------------------------------- compact
// Stable compaction of three streams in one pass structure: plan entries
// (claimants in serve order with a positive flow), surviving suppliers
// (records, index, mass; into the other buffer) and surviving consumers.
// count: per-block counts; write: each block derives its offsets from the
// counts of the blocks before it; commit: one thread updates the round state.
constexpr int kLpCompactPer = 4;  // elements per thread and stream
constexpr int kLpCompactBlock = kLpThreads * kLpCompactPer;

__device__ inline void lp_flags(const LPArgs& A, int par, int mact, int nact, int e, bool& fp, bool& fs, bool& fc) {
    fp = e < nact && A.w.ckey[A.w.sorted[e]] > 0.0;
    fs = e < mact && A.w.smass[par][e] > 0.0;
    fc = e < nact && A.w.cmass[A.w.cact[par][e]] > 0.0;
}

__global__ __launch_bounds__(kLpThreads) void lp_ccount(LPArgs A) {
    __shared__ unsigned long long scratch[kLpThreads / kWave];
    const LPState* st = A.w.st;
    if (!lp_live(st)) return;
    const int mact = st->mact, nact = st->nact, par = st->parity;
    const int e0 = blockIdx.x * kLpCompactBlock + threadIdx.x * kLpCompactPer;
    int kp = 0, ks = 0, kc = 0;
#pragma unroll
    for (int u = 0; u < kLpCompactPer; ++u) {
        bool fp, fs, fc;
        lp_flags(A, par, mact, nact, e0 + u, fp, fs, fc);
        kp += fp;
        ks += fs;
        kc += fc;
    }
    unsigned long long tot;
    (void)lp_block_scan<kLpThreads>((unsigned long long)kp | ((unsigned long long)ks << 21) |
                                        ((unsigned long long)kc << 42), &tot, scratch);
    if (threadIdx.x == 0) A.w.blkcnt[blockIdx.x] = tot;
}

// Ends the round: packed totals of the three compaction streams (the one
// block's own total, or the per-block counts of lp_ccount), new active
// sizes, plan length, statistics, termination.  Run by one whole block;
// reads only data that no block of the running kernel writes.
__device__ void lp_commit_round(const LPArgs& A, int nblocks, bool single, unsigned long long own,
                                unsigned long long* red) {
    LPState* st = A.w.st;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    unsigned long long tot = 0;
    if (!single) {
        for (int b = threadIdx.x; b < nblocks; b += kLpThreads) tot += A.w.blkcnt[b];
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) tot += __shfl_xor(tot, o);
        if (lane == 0) red[w] = tot;
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    if (single) {
        tot = own;
    } else {
        tot = 0;
#pragma unroll
        for (int k = 0; k < kLpThreads / kWave; ++k) tot += red[k];
    }
    const unsigned long long mask = (1ull << 21) - 1;
    const int m2 = (int)((tot >> 21) & mask), n2 = (int)(tot >> 42);
    st->nnz += (int64_t)(tot & mask);
    st->work += (int64_t)st->mact * st->nact;
    st->near += st->nflag;
    st->nflag = 0;
    st->rounds += 1;
    st->mact = m2;
    st->nact = n2;
    st->parity = 1 - st->parity;
    st->ticket = 0;
    if (m2 == 0 || n2 == 0) {
        st->done = 1;
    } else if (A.max_rounds > 0 && st->rounds >= A.max_rounds) {
        st->status = NNSEMD_ERR_NOT_CONVERGED;
        st->done = 1;
    } else if (m2 <= A.tail_cap && n2 <= A.tail_cap) {
        st->tail = 1;
    }
}

// Compaction writes of the round and, in the block that takes the last
// ticket, the round's commit.  With several blocks the packed per-block
// counts come from lp_ccount; a single block (at most kLpCompactBlock
// elements per stream) counts its own and no counting kernel runs.  Every
// block has used the round state it read before it takes its ticket, so the
// last block may update it; the compaction outputs are read only by later
// kernels.
template <int D>
__global__ __launch_bounds__(kLpThreads) void lp_cwrite(LPArgs A) {
    constexpr int RS = record_stride(D);
    __shared__ unsigned long long scratch[kLpThreads / kWave];
    __shared__ unsigned long long base_sh;
    __shared__ int last_sh;
    const LPState* st = A.w.st;
    if (!lp_live(st)) return;
    const int mact = st->mact, nact = st->nact, par = st->parity;
    const int tid = threadIdx.x;
    // offsets of this block: sum of the packed counts of earlier blocks
    unsigned long long part = 0;
    for (int b = tid; b < (int)blockIdx.x; b += kLpThreads) part += A.w.blkcnt[b];
    unsigned long long btot;
    (void)lp_block_scan<kLpThreads>(part, &btot, scratch);
    if (tid == 0) base_sh = btot;
    __syncthreads();
    const unsigned long long base = base_sh;
    const int e0 = blockIdx.x * kLpCompactBlock + tid * kLpCompactPer;
    bool fp[kLpCompactPer], fs[kLpCompactPer], fc[kLpCompactPer];
    int kp = 0, ks = 0, kc = 0;
#pragma unroll
    for (int u = 0; u < kLpCompactPer; ++u) {
        lp_flags(A, par, mact, nact, e0 + u, fp[u], fs[u], fc[u]);
        kp += fp[u];
        ks += fs[u];
        kc += fc[u];
    }
    unsigned long long tot;
    const unsigned long long pre = base + lp_block_scan<kLpThreads>(
        (unsigned long long)kp | ((unsigned long long)ks << 21) | ((unsigned long long)kc << 42), &tot, scratch);
    const unsigned long long mask = (1ull << 21) - 1;
    int wp = (int)(pre & mask), ws = (int)((pre >> 21) & mask), wc = (int)(pre >> 42);
    const int64_t nnz0 = st->nnz;
    const int np = 1 - par;
#pragma unroll
    for (int u = 0; u < kLpCompactPer; ++u) {
        const int e = e0 + u;
        if (fp[u] && A.plan_src != nullptr) {
            const int j = A.w.sorted[e];
            const int64_t o = nnz0 + wp;
            A.plan_src[o] = A.w.cnn[j];
            A.plan_dst[o] = j;
            A.plan_flow[o] = A.w.ckey[j];
        }
        wp += fp[u];
        if (fs[u]) {
            const float4* src = reinterpret_cast<const float4*>(A.w.srec[par] + (size_t)e * RS);
            float4* dst = reinterpret_cast<float4*>(A.w.srec[np] + (size_t)ws * RS);
#pragma unroll
            for (int q = 0; q < RS / 4; ++q) dst[q] = src[q];
            A.w.sidx[np][ws] = A.w.sidx[par][e];
            A.w.smass[np][ws] = A.w.smass[par][e];
            A.w.scnt[ws] = 0;
            ++ws;
        }
        if (fc[u]) A.w.cact[np][wc++] = A.w.cact[par][e];
    }
    __syncthreads();
    if (tid == 0) last_sh = gridDim.x == 1 || atomicAdd(&A.w.st->ticket, 1) == (int)gridDim.x - 1;
    __syncthreads();
    if (last_sh) lp_commit_round(A, (int)gridDim.x, gridDim.x == 1, tot, scratch);
}

// ---------------------------------------------------------------- finish
template <int D>
__global__ __launch_bounds__(kLpScanThreads) void lp_finish(LPArgs A) {
    __shared__ double scratch[kLpScanThreads / kWave];
    LPState* st = A.w.st;
    const int tid = threadIdx.x;
    const int m = (int)A.m;
    const bool ok = st->status == NNSEMD_OK || st->status == NNSEMD_ERR_NOT_CONVERGED;
    const int cs = (m + kLpScanThreads - 1) / kLpScanThreads;
    const int lo = min(tid * cs, m), hi = min(lo + cs, m);
    double c = 0.0;
    if (ok)
        for (int i = lo; i < hi; ++i) c += A.w.costacc[i];
    const double cost = lp_block_sum<kLpScanThreads>(c, scratch);
    const int par = st->parity;
    double rs = 0.0, rc = 0.0;
    if (ok) {
        for (int s = tid; s < st->mact; s += kLpScanThreads) rs += A.w.smass[par][s];
        for (int q = tid; q < st->nact; q += kLpScanThreads) rc += A.w.cmass[A.w.cact[par][q]];
    }
    rs = lp_block_sum<kLpScanThreads>(rs, scratch);
    rc = lp_block_sum<kLpScanThreads>(rc, scratch);
    if (A.map != nullptr) {
#pragma clang fp contract(off)
        for (int64_t e = tid; e < (int64_t)m * D; e += kLpScanThreads) {
            const int64_t i = e / D;
            const double w = (ok && A.w.wsum != nullptr) ? A.w.wsum[i] : 0.0;
            A.map[e] = w > 0.0 ? A.w.bsum[e] / w : NAN;
        }
    }
    if (tid == 0) {
        A.cost[0] = st->status == NNSEMD_OK ? cost : NAN;
        if (A.stats != nullptr) {
            nnsemd_stats_t out;
            out.status = st->status;
            out.rounds = st->rounds;
            out.nnz = st->nnz;
            out.work = st->work;
            out.rescored = st->near;
            out.residual_src = rs;
            out.residual_dst = rc;
            out.near_ties_nn = st->ties_nn;
            out.near_ties_order = st->ties_order;
            A.stats[0] = out;
        }
    }
}

// ----------------------------------------------------------------- tail
// Single-workgroup finish.  Once both active sets fit (tail_cap points per
// side), the remaining rounds run in one workgroup with the pair in LDS, as
// on the one-workgroup path, instead of nine grid-wide launches per round.
// The suppliers keep their slots (ascending supplier index, so ties still go
// to the smallest index) and records; the consumers are renumbered 0..nact-1
// in ascending index order (the greedy order's tie rule is unchanged) and
// mapped back to the caller's indices for the random order, the plan and the
// map.  Costs and the map sums go to the same per-supplier accumulators, in
// the same serve order, as on the grid-wide rounds.
constexpr int kLpTailThreads = 512;
constexpr int kLpTailChunk = 4;  // points per thread and side: capacity 2048

__host__ __device__ inline size_t lp_tail_lds(int cap, int rs) {
    return align_up(pair_lds_layout(cap, cap, rs, 0, false, false).total, 16) + sizeof(int32_t) * (size_t)cap;
}

template <int D, bool L1>
__global__ __launch_bounds__(kLpTailThreads) void lp_tail(LPArgs A) {
#pragma clang fp contract(off)
    constexpr int RS = record_stride(D);
    constexpr int T = kLpTailThreads;
    extern __shared__ __align__(16) char lds_dyn[];
    __shared__ rc::SharedCore sh;
    LPState* st = A.w.st;
    if (!(st->status == NNSEMD_OK && !st->done && st->tail)) return;  // uniform
    const int cap = A.tail_cap;
    rc::Lds L = rc::carve(lds_dyn, cap, cap, RS);
    int32_t* jmap = reinterpret_cast<int32_t*>(lds_dyn + align_up(pair_lds_layout(cap, cap, RS, 0, false, false).total, 16));
    L.jmap = jmap;
    const int tid = threadIdx.x;
    const int par = st->parity;
    const int nact0 = st->nact;
    int mact = st->mact, nact = nact0;
    float centre[D];
#pragma unroll
    for (int t = 0; t < D; ++t) centre[t] = st->centre[t];
    const float rhat = st->rhat;
    // consumer coordinates gathered by tail-local index (the partial-result
    // buffer is free from here on)
    float* Yt = reinterpret_cast<float*>(A.w.part);
    if (tid == 0) {
        sh.tie_nn = 0ull;
        sh.tie_order = 0ull;
        sh.nflag = 0;
    }
    for (int s = tid; s < mact; s += T) {
        const float4* src = reinterpret_cast<const float4*>(A.w.srec[par] + (size_t)s * RS);
        float4* dst = reinterpret_cast<float4*>(L.srec + (size_t)s * RS);
#pragma unroll
        for (int q = 0; q < RS / 4; ++q) dst[q] = src[q];
        L.sidx[s] = A.w.sidx[par][s];
        L.smass[s] = A.w.smass[par][s];
        L.scnt[s] = 0;
    }
    for (int q = tid; q < nact; q += T) {
        const int j = A.w.cact[par][q];
        jmap[q] = j;
        L.cact[q] = q;
        L.cmass[q] = A.w.cmass[j];
#pragma unroll
        for (int t = 0; t < D; ++t) Yt[(size_t)q * D + t] = A.Y[(int64_t)j * D + t];
    }
    __syncthreads();
    const int64_t max_rounds = A.max_rounds;
    int status = NNSEMD_OK;
    int64_t rounds = st->rounds;
    int64_t work = 0, nnz = 0, near = 0;
    const int64_t plan_base = st->nnz;
    while (mact > 0 && nact > 0) {
        if (max_rounds > 0 && rounds >= max_rounds) {
            status = NNSEMD_ERR_NOT_CONVERGED;
            break;
        }
        work += (int64_t)mact * nact;
        near += ps::search_round<D, T, kLpTailChunk, L1>(L, sh, A.X, Yt, centre, rhat, mact, nact, 1, false,
                                                          A.metric);
        rc::round_buckets<T>(L, sh, mact, nact);
        rc::round_rank<T, kLpTailChunk>(L, nact, A.protocol, A.seed, (int)rounds, A.metric,
                                        A.protocol == NNSEMD_GREEDY ? &sh.tie_order : nullptr);
        // serve walk (the grid-wide rounds' operations and accumulators)
        for (int s = tid; s < mact; s += T) {
            const int c = L.scnt[s];
            if (c == 0) continue;
            const int end = L.soff[s];
            const int isup = L.sidx[s];
            int pos = end - c;
            double sm = L.smass[s];
            double acc = A.w.costacc[isup];
            while (pos < end && sm > 0.0) {
                const int q = L.sorted[pos];
                const double cm = L.cmass[q];
                const double f = sm < cm ? sm : cm;
                sm = sm - f;
                L.cmass[q] = cm - f;
                const double key = L.ckey[q];
                acc = acc + f * (A.metric == NNSEMD_L2 ? sqrt(key) : key);
                if (A.w.wsum != nullptr) {
                    A.w.wsum[isup] = A.w.wsum[isup] + f;
#pragma unroll
                    for (int t = 0; t < D; ++t)
                        A.w.bsum[(int64_t)isup * D + t] =
                            A.w.bsum[(int64_t)isup * D + t] + f * (double)Yt[(size_t)q * D + t];
                }
                L.ckey[q] = -f;  // negated flow: unserved claimants keep their keys
                L.cnn[q] = isup;
                ++pos;
            }
            L.smass[s] = sm;
            A.w.costacc[isup] = acc;
        }
        __syncthreads();
        rc::round_compact<T, kLpTailChunk, RS, true>(L, sh, mact, nact, nnz, A.plan_src, A.plan_dst, A.plan_flow,
                                               plan_base);
        ++rounds;
    }
    // hand the state back to the finish: survivors in slots 0.. of the
    // current buffers, consumer masses by the caller's index
    for (int s = tid; s < mact; s += T) {
        A.w.sidx[par][s] = L.sidx[s];
        A.w.smass[par][s] = L.smass[s];
    }
    for (int q = tid; q < nact; q += T) A.w.cact[par][q] = jmap[L.cact[q]];
    for (int q = tid; q < nact0; q += T) A.w.cmass[jmap[q]] = L.cmass[q];
    __syncthreads();
    if (tid == 0) {
        st->status = status;
        st->rounds = (int32_t)rounds;
        st->nnz += nnz;
        st->work += work;
        st->near += near;
        st->ties_nn += (int64_t)sh.tie_nn;
        st->ties_order += (int64_t)sh.tie_order;
        st->mact = mact;
        st->nact = nact;
        st->done = 1;
    }
}

#define NNSEMD_LP_DISPATCH(D_, EXPR)                   \
    switch (D_) {                                      \
        case 1: { constexpr int DD = 1; EXPR; } break; \
        case 2: { constexpr int DD = 2; EXPR; } break; \
        case 3: { constexpr int DD = 3; EXPR; } break; \
        case 4: { constexpr int DD = 4; EXPR; } break; \
        case 5: { constexpr int DD = 5; EXPR; } break; \
        case 6: { constexpr int DD = 6; EXPR; } break; \
        case 7: { constexpr int DD = 7; EXPR; } break; \
        default: return (int)hipErrorInvalidValue;     \
    }

}  // namespace

int lp_launch_init(const LPArgs& A, int d, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    const int64_t pts = A.m > A.n ? A.m : A.n;
    const int nblocks = (int)((pts + kLpThreads - 1) / kLpThreads);
    const bool l1 = A.metric == NNSEMD_L1;
    NNSEMD_LP_DISPATCH(d, {
        if (nblocks > 0) hipLaunchKernelGGL(lp_ingest<DD>, dim3(nblocks), dim3(kLpThreads), 0, st, A);
        if (l1)
            hipLaunchKernelGGL((lp_setup<DD, true>), dim3(1), dim3(kLpScanThreads), 0, st, A, nblocks);
        else
            hipLaunchKernelGGL((lp_setup<DD, false>), dim3(1), dim3(kLpScanThreads), 0, st, A, nblocks);
    })
    return (int)hipGetLastError();
}

int lp_launch_round(const LPArgs& A, int d, int mact_ub, int nact_ub, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    const bool l1 = A.metric == NNSEMD_L1;
    const int kc = nact_ub > 4 * kLpThreads ? 4 : 1;
    const int cblocks = (nact_ub + kLpThreads * kc - 1) / (kLpThreads * kc);
    int split = (2048 + cblocks - 1) / cblocks;
    const int max_split_by_work = mact_ub / 64 > 1 ? mact_ub / 64 : 1;
    if (split > max_split_by_work) split = max_split_by_work;
    if ((int64_t)split * A.w.ncap > A.w.part_cap) split = (int)(A.w.part_cap / A.w.ncap);
    if (split < 1) split = 1;
    const int qblocks = (nact_ub + kLpThreads - 1) / kLpThreads;
    const int dblocks = (nact_ub + kLpThreads / kLpDecideSub - 1) / (kLpThreads / kLpDecideSub);
    const int wblocks = (mact_ub + kLpThreads / kWave - 1) / (kLpThreads / kWave);  // one wavefront per supplier
    const int cmax = mact_ub > nact_ub ? mact_ub : nact_ub;
    const int cmblocks = (cmax + kLpCompactBlock - 1) / kLpCompactBlock;
    if (qblocks == 0 || wblocks == 0) return 0;
    if (cmblocks > A.w.blkcnt_cap) return (int)hipErrorInvalidValue;
    NNSEMD_LP_DISPATCH(d, {
        if (kc == 4) {
            if (l1) hipLaunchKernelGGL((lp_search<DD, true, 4>), dim3(cblocks, split), dim3(kLpThreads), 0, st, A, split);
            else hipLaunchKernelGGL((lp_search<DD, false, 4>), dim3(cblocks, split), dim3(kLpThreads), 0, st, A, split);
        } else {
            if (l1) hipLaunchKernelGGL((lp_search<DD, true, 1>), dim3(cblocks, split), dim3(kLpThreads), 0, st, A, split);
            else hipLaunchKernelGGL((lp_search<DD, false, 1>), dim3(cblocks, split), dim3(kLpThreads), 0, st, A, split);
        }
        if (l1) {
            hipLaunchKernelGGL((lp_decide<DD, true>), dim3(dblocks), dim3(kLpThreads), 0, st, A, split);
            hipLaunchKernelGGL((lp_rescore<DD, true>), dim3(512), dim3(kLpRescoreThreads), 0, st, A);
        } else {
            hipLaunchKernelGGL((lp_decide<DD, false>), dim3(dblocks), dim3(kLpThreads), 0, st, A, split);
            hipLaunchKernelGGL((lp_rescore<DD, false>), dim3(512), dim3(kLpRescoreThreads), 0, st, A);
        }
        hipLaunchKernelGGL(lp_offsets, dim3(1), dim3(kLpScanThreads), 0, st, A);
        hipLaunchKernelGGL(lp_scatter, dim3(qblocks), dim3(kLpThreads), 0, st, A);
        if (A.protocol == NNSEMD_GREEDY) hipLaunchKernelGGL(lp_ties, dim3(qblocks), dim3(kLpThreads), 0, st, A);
        hipLaunchKernelGGL(lp_serve<DD>, dim3(wblocks), dim3(kLpThreads), 0, st, A);
        if (cmblocks > 1) hipLaunchKernelGGL(lp_ccount, dim3(cmblocks), dim3(kLpThreads), 0, st, A);
        hipLaunchKernelGGL(lp_cwrite<DD>, dim3(cmblocks), dim3(kLpThreads), 0, st, A);
    })
    return (int)hipGetLastError();
}

template <int D, bool L1>
int launch_tail_typed(const LPArgs& A, size_t lds, hipStream_t st) {
    hipError_t e = hipFuncSetAttribute((const void*)lp_tail<D, L1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return (int)e;
    hipLaunchKernelGGL((lp_tail<D, L1>), dim3(1), dim3(kLpTailThreads), lds, st, A);
    return (int)hipGetLastError();
}

template <int D>
int launch_tail_metric(const LPArgs& A, bool l1, size_t lds, hipStream_t st) {
    return l1 ? launch_tail_typed<D, true>(A, lds, st) : launch_tail_typed<D, false>(A, lds, st);
}

// Hand-over point: both active sets at most 512 points.  The workgroup
// could hold 2048 a side, but the on-chip claimant order costs O(c) per
// claimant of a bucket of c, and the colour-transfer pair's late rounds
// have buckets of hundreds to thousands of claimants (one supplier left
// among many consumers): handing over at 2048 took that pair from 63.0 to
// 68.1 ms, at 1024 to 62.0 ms, at 512 to 61.0 ms.
constexpr int kLpTailHandOver = 512;

int lp_tail_capacity(int d, size_t max_lds) {
    const int rs = record_stride(d);
    for (int cap = kLpTailHandOver; cap >= 64; cap /= 2)
        if (lp_tail_lds(cap, rs) + 8192 <= max_lds) return cap;
    return 0;
}

int lp_launch_tail(const LPArgs& A, int d, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    const bool l1 = A.metric == NNSEMD_L1;
    const size_t lds = lp_tail_lds(A.tail_cap, record_stride(d));
    NNSEMD_LP_DISPATCH(d, { return launch_tail_metric<DD>(A, l1, lds, st); })
    return (int)hipGetLastError();
}

int lp_launch_finish(const LPArgs& A, int d, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    NNSEMD_LP_DISPATCH(d, { hipLaunchKernelGGL(lp_finish<DD>, dim3(1), dim3(kLpScanThreads), 0, st, A); })
    return (int)hipGetLastError();
}

}  // namespace nnsemd
