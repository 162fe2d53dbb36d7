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

namespace nnsemd {
namespace {

using namespace rc;

// supplier records in flight per step of the search: 8, or 4 for the
// 512-thread kernels held to 80 VGPRs (six wavefronts per SIMD)
template <int CSMAX>
constexpr int search_unroll() { return CSMAX <= 2 ? 4 : 8; }

// Exact FP64 key in the definition's operation order (dimension order, no
// fused multiply-add): squared Euclidean, or L1.
template <int D, bool L1>
__device__ inline double key64(const float* __restrict__ x, const float* __restrict__ y) {
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

// Search gap bound (Euclidean metrics).  With x^ = fl(x - c), y^ = fl(y - c)
// (c the FP32 centre of the supplier box), the record (-2 x^, fl(||x^||^2))
// and the FMA chain key = ||x^||^2 + sum_t (-2 x^_t) y^_t, one key differs
// from ||x - y||^2 - ||y^||^2 by at most B = (2D + 2) u e^2 to first order,
// e = ||x^|| + ||y^|| <= rhat + ||y^|| (u = 2^-24): D roundings in the norm
// (<= D u ||x^||^2), D in the chain (<= D u (||x^||^2 + 2 ||x^|| ||y^||)) and
// 2u e^2 from the two centring subtractions.  If the FP32 argmin were not
// the FP64 one, some other key would lie within 2B of the best, so the
// threshold 2 x 2B = 8 (D + 1) u e^2 leaves a factor 2 for second-order
// terms, the FP64 reference's own rounding and the rounding of e.
template <int D>
__device__ inline float search_gap_bound(float rhat, float yn2) {
    const float e = rhat + sqrtf(yn2);
    return 8.f * (float)(D + 1) * kU32 * e * e + 1e-30f;
}

// L1 keys sum D rounded |x_t - y_t| terms (no centring): relative error at
// most D u of the key, so two keys of one consumer can disagree with their
// FP64 order only within 2 D u b1; 4 (D + 1) u b1 leaves a factor 2.
template <int D>
__device__ inline float search_gap_bound_l1(float b1) {
    return 4.f * (float)(D + 1) * kU32 * b1 + 1e-30f;
}

// Fractional bits of a finite FP32 value: the smallest q >= 0 with v a
// multiple of 2^-q (0 for 0; a large value for subnormals, which never
// qualify for the exact-key test below).
__device__ inline int frac_bits(float v) {
    const uint32_t u = __float_as_uint(v) & 0x7fffffffu;
    if (u == 0u) return 0;
    const int e = (int)(u >> 23);
    if (e == 0) return 200;
    const int tz = __builtin_ctz((u & 0x7fffffu) | 0x800000u);
    const int q = 23 - tz - (e - 127);
    return q > 0 ? q : 0;
}

// Exact-key test.  If every centred coordinate is a multiple of 2^-q with
// magnitude <= R, every term of a Euclidean key (x^_t^2, 2 x^_t y^_t) is a
// multiple of 2^-2q and every partial sum is at most 3 D R^2 in magnitude, so
// all of them are FP32 numbers when 3 D R^2 4^q < 2^24: each FMA of the key
// chain is then exact, the FP32 keys equal the exact ones (shifted by the
// exact ||y^||^2), and the FP32 argmin with its smallest-slot tie rule is the
// FP64 definition's.  L1 (uncentred): terms |x_t - y_t| <= 2R, sums <= 2DR,
// exact when 2 D R 2^q < 2^24.  Integer-lattice inputs (pixel grids) pass.
template <int D, bool L1>
__device__ inline bool keys_exact(double q, double R) {
    if (q > 40.0) return false;
    const double s = exp2(q);
    return L1 ? 2.0 * D * R * s < 16777216.0 : 3.0 * D * R * R * s * s < 16777216.0;
}

template <int D, int RS, bool L1>
__device__ inline float key32(const float* __restrict__ rec, const float (&y)[D]) {
    if (L1) {
        float k = 0.f;
#pragma unroll
        for (int t = 0; t < D; ++t) k += fabsf(rec[t] - y[t]);
        return k;
    } else {
        float k = rec[D];
#pragma unroll
        for (int t = D - 1; t >= 0; --t) k = fmaf(rec[t], y[t], k);
        return k;
    }
}

// One pass of the search for the consumers q = qa + k*G (k < KC) of this
// lane; S lanes share each consumer and scan every S-th active supplier.
// Per consumer: FP32 best and second-best keys; if they are closer than the
// rounding bound the consumer is queued for the FP64 re-score, otherwise its
// pick and the exact FP64 key of the pick are stored.
template <int D, int RS, bool L1, int KC, int UN>
__device__ inline void nns_pass(const Lds16& L, SharedCore& sh, const float* __restrict__ X,
                                const float* __restrict__ Y, const float (&centre)[D], float rhat,
                                int mact, int nact, int S, int qa, int G, int r, bool exact, int metric) {
    int jj[KC];
    bool valid[KC];
    float y[KC][D];
    float yn2[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        const int q = qa + k * G;
        valid[k] = q < nact;
        jj[k] = L.cact[valid[k] ? q : 0];
    }
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        yn2[k] = 0.f;
#pragma unroll
        for (int t = 0; t < D; ++t) {
            const float yv = L1 ? Y[(size_t)jj[k] * D + t] : Y[(size_t)jj[k] * D + t] - centre[t];
            y[k][t] = yv;
            yn2[k] = fmaf(yv, yv, yn2[k]);
        }
    }
    float b1[KC], b2[KC];
    int bs[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        b1[k] = INFINITY;
        b2[k] = INFINITY;
        bs[k] = 0x7fffffff;
    }
    // Full blocks of UN records.  Two keys at a time update the pair
    // (b1, b2): b2 <- min(b2, med3(b1, ka, kb)) and b1 <- min(b1, ka, kb)
    // give the two smallest of {b1, b2, ka, kb} (as a multiset, so equal
    // keys leave b2 = b1).  Only the block in which b1 last fell strictly
    // is remembered; its records are scanned again afterwards for the first
    // slot holding b1, which is the smallest slot with the smallest key.
    const int stride = S * UN;
    const int full = (mact / stride) * stride;
    int blk[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) blk[k] = -1;
    for (int s0 = r; s0 < full; s0 += stride) {
        float rec[UN][RS];
#pragma unroll
        for (int u = 0; u < UN; ++u) load_rec<RS>(L.srec, s0 + u * S, rec[u]);
        float b1o[KC];
#pragma unroll
        for (int k = 0; k < KC; ++k) b1o[k] = b1[k];
#pragma unroll
        for (int u = 0; u < UN; u += 2) {
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                const float ka = key32<D, RS, L1>(rec[u], y[k]);
                const float kb = key32<D, RS, L1>(rec[u + 1], y[k]);
                b2[k] = fminf(b2[k], __builtin_amdgcn_fmed3f(b1[k], ka, kb));
                b1[k] = fminf(b1[k], fminf(ka, kb));
            }
        }
#pragma unroll
        for (int k = 0; k < KC; ++k) blk[k] = b1[k] < b1o[k] ? s0 : blk[k];
    }
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        if (blk[k] >= 0) {
            int u = UN - 1;
#pragma unroll
            for (int v = UN - 2; v >= 0; --v) {
                float rv[RS];
                load_rec<RS>(L.srec, blk[k] + v * S, rv);
                u = key32<D, RS, L1>(rv, y[k]) == b1[k] ? v : u;
            }
            bs[k] = blk[k] + u * S;
        }
    }
    for (int s = full + r; s < mact; s += S) {
        float rec[RS];
        load_rec<RS>(L.srec, s, rec);
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            const float key = key32<D, RS, L1>(rec, y[k]);
            const bool lt = key < b1[k];
            bs[k] = lt ? s : bs[k];
            b2[k] = __builtin_amdgcn_fmed3f(b1[k], key, b2[k]);
            b1[k] = fminf(b1[k], key);
        }
    }
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        for (int o = 1; o < S; o <<= 1) {
            const float c1 = __shfl_xor(b1[k], o);
            const float c2 = __shfl_xor(b2[k], o);
            const int cs2 = __shfl_xor(bs[k], o);
            const float n2 = fminf(fmaxf(b1[k], c1), fminf(b2[k], c2));
            const bool take = (c1 < b1[k]) || (c1 == b1[k] && cs2 < bs[k]);
            b1[k] = take ? c1 : b1[k];
            bs[k] = take ? cs2 : bs[k];
            b2[k] = n2;
        }
    }
    if (r != 0) return;
    bool flag[KC];
    int pick[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        if (exact) {
            // exact keys: the pick stands; the two nearest distances are
            // b + ||y^||^2 exactly (FP64 holds the sum exactly)
            flag[k] = false;
            pick[k] = bs[k];
            if (valid[k] && mact > 1) {
                const double k1 = L1 ? (double)b1[k] : (double)b1[k] + (double)yn2[k];
                const double k2 = L1 ? (double)b2[k] : (double)b2[k] + (double)yn2[k];
                if (near_tie_dist(dist_of_key(k1, metric), dist_of_key(k2, metric))) atomicAdd(&sh.tie_nn, 1ull);
            }
            continue;
        }
        // win: the proven search bound (see search_gap_bound) plus the window
        // in which the two nearest suppliers may still be a near tie.
        float win;
        if (L1) {
            const float thr = search_gap_bound_l1<D>(b1[k]);
            win = thr + near_window(b1[k], true);
        } else {
            const float thr = search_gap_bound<D>(rhat, yn2[k]);
            win = thr + near_window(b1[k] + yn2[k] + thr, false);
        }
        flag[k] = !(b2[k] - b1[k] > win);
        pick[k] = flag[k] ? 0 : bs[k];
    }
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        if (!valid[k]) continue;
        if (flag[k]) {
            const int f = atomicAdd(&sh.nflag, 1);
            L.list[f] = jj[k];
        } else {
            L.cnn[jj[k]] = pick[k];
            L.ckey[jj[k]] = key64<D, L1>(X + (size_t)L.sidx[pick[k]] * D, Y + (size_t)jj[k] * D);
            cnt_add(L.scnt, pick[k]);
        }
    }
}

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

        // ---- 1. NNS: FP32 scan, best + second best, near ties deferred;
        // each decided consumer also counts itself into its pick's bucket.
        // S lanes share one consumer (each scans every S-th supplier) when
        // there are too few consumers to fill the workgroup.  Otherwise the
        // active consumers are cut into 64-consumer slots and the slots
        // dealt to the wavefronts as evenly as possible; a wavefront with k
        // slots scans the records once with k consumers per lane (one record
        // load feeds k key chains), so only the last slot has idle lanes.
        // S is the largest power of two (at most 64 and at most mact) with
        // nact * S * split <= T, so every active consumer gets its S lanes.
        constexpr int UN = search_unroll<CSMAX>();
        int S = 1;
        while ((S << 1) <= kWave && (S << 1) <= mact && nact * (S << 1) * A.split <= T) S <<= 1;
        if (S > 1) {
            nns_pass<D, RS, L1, 1, UN>(L, sh, X, Y, centre, rhat, mact, nact, S, tid / S, T / S, tid & (S - 1), exact, A.metric);
        } else {
            const int nslots = (nact + kWave - 1) / kWave;
            const int lo = wave * nslots / NW, hi = (wave + 1) * nslots / NW;
            // a wavefront holds at most CSMAX slots (nact <= CSMAX * T)
            constexpr int KMAX = CSMAX < 4 ? CSMAX : 4;
            for (int u0 = lo; u0 < hi; u0 += KMAX) {
                const int k = min(KMAX, hi - u0);  // wavefront-uniform
                const int qa = u0 * kWave + lane;
                if (KMAX >= 4 && k == 4)
                    nns_pass<D, RS, L1, KMAX, UN>(L, sh, X, Y, centre, rhat, mact, nact, 1, qa, kWave, 0, exact, A.metric);
                else if (KMAX >= 3 && k == 3)
                    nns_pass<D, RS, L1, KMAX >= 3 ? 3 : 1, UN>(L, sh, X, Y, centre, rhat, mact, nact, 1, qa, kWave, 0, exact, A.metric);
                else if (KMAX >= 2 && k == 2)
                    nns_pass<D, RS, L1, KMAX >= 2 ? 2 : 1, UN>(L, sh, X, Y, centre, rhat, mact, nact, 1, qa, kWave, 0, exact, A.metric);
                else
                    nns_pass<D, RS, L1, 1, UN>(L, sh, X, Y, centre, rhat, mact, nact, 1, qa, kWave, 0, exact, A.metric);
            }
        }
        __syncthreads();
        NNSEMD_PH(1)
        const int nf = sh.nflag;
        if (nf > 0) {
            // FP64 re-score of the flagged consumers, one wavefront per
            // consumer: the argmin (ties to the smallest slot) and the
            // second-smallest key decide the pick and the near-tie count.
            for (int f = wave; f < nf; f += NW) {
                const int j = L.list[f];
                const float* yp = Y + (size_t)j * D;
                double best = INFINITY, sec = INFINITY;
                int bsl = 0x7fffffff;
                for (int s = lane; s < mact; s += kWave) {
                    const double k = key64<D, L1>(X + (size_t)L.sidx[s] * D, yp);
                    if (k < best) {
                        sec = best;
                        best = k;
                        bsl = s;
                    } else if (k < sec) {
                        sec = k;
                    }
                }
#pragma unroll
                for (int o = kWave / 2; o > 0; o >>= 1) {
                    const double cb = __shfl_xor(best, o);
                    const double c2 = __shfl_xor(sec, o);
                    const int cs2 = __shfl_xor(bsl, o);
                    sec = fmin(fmax(best, cb), fmin(sec, c2));
                    if (cb < best || (cb == best && cs2 < bsl)) {
                        best = cb;
                        bsl = cs2;
                    }
                }
                if (lane == 0) {
                    L.cnn[j] = bsl;
                    L.ckey[j] = best;
                    cnt_add(L.scnt, bsl);
                    if (mact > 1 && near_tie_dist(dist_of_key(best, A.metric), dist_of_key(sec, A.metric)))
                        atomicAdd(&sh.tie_nn, 1ull);
                }
            }
            near += nf;
            __syncthreads();
        }
        NNSEMD_PH(2)

        // ---- 2. claimant sets a_i
        round_buckets<T>(L, sh, mact, nact);
        NNSEMD_PH(3)
        // ---- 3. flow & cost: claimant order, then the serve walk
        round_rank<T, CSMAX>(L, nact, A.protocol, A.seed, rounds, A.metric,
                             A.protocol == NNSEMD_GREEDY ? &sh.tie_order : nullptr);
        NNSEMD_PH(5)
        round_walk<T>(L, mact, A.metric, cost);
        NNSEMD_PH(6)
        // ---- 4. weights update: plan append + compaction
        round_compact<T, CSMAX, RS>(L, sh, mact, nact, nnz, want_plan ? A.plan_src : nullptr, A.plan_dst,
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
