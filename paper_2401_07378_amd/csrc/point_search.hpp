// FP32 nearest-supplier search of one round (the NNS step of Algorithm 1,
// Sec. III-A) for a pair whose active suppliers sit in LDS as search
// records, shared by the one-workgroup pair solver and the single-workgroup
// finish of the multi-workgroup path.  Every pick is the FP64 argmin (ties
// to the smallest slot, and slots are in ascending supplier order); the
// consumers whose two nearest FP32 keys are closer than the rounding bound
// plus the near-tie window are re-scored in FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "internal.hpp"
#include "round_common.hpp"

namespace nnsemd {
namespace ps {

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
template <int D, int RS, bool L1, int KC, int UN, typename LT>
__device__ inline void nns_pass(const LT& L, SharedCore& sh, const float* __restrict__ X,
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


// One round's search: every active consumer's pick (active slot in cnn[j],
// exact FP64 key in ckey[j]) counted into scnt; returns the number of
// consumers re-scored in FP64.  Ends with a workgroup barrier.
// S lanes share one consumer (each scans every S-th supplier) when there
// are too few consumers to fill the workgroup.  Otherwise the active
// consumers are cut into 64-consumer slots and the slots dealt to the
// wavefronts as evenly as possible; a wavefront with k slots scans the
// records once with k consumers per lane (one record load feeds k key
// chains), so only the last slot has idle lanes.  S is the largest power of
// two (at most 64 and at most mact) with nact * S * split <= T, so every
// active consumer gets its S lanes.
template <int D, int T, int CSMAX, bool L1, typename LT>
__device__ inline int search_round(const LT& L, SharedCore& sh, const float* __restrict__ X,
                                   const float* __restrict__ Y, const float (&centre)[D], float rhat, int mact,
                                   int nact, int split, bool exact, int metric) {
    constexpr int RS = record_stride(D);
    constexpr int NW = T / kWave;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    int near = 0;
        constexpr int UN = search_unroll<CSMAX>();
    int S = 1;
    while ((S << 1) <= kWave && (S << 1) <= mact && nact * (S << 1) * split <= T) S <<= 1;
    if (S > 1) {
        nns_pass<D, RS, L1, 1, UN>(L, sh, X, Y, centre, rhat, mact, nact, S, tid / S, T / S, tid & (S - 1), exact, metric);
    } else {
        const int nslots = (nact + kWave - 1) / kWave;
        const int lo = wave * nslots / NW, hi = (wave + 1) * nslots / NW;
        // a wavefront holds at most CSMAX slots (nact <= CSMAX * T)
        constexpr int KMAX = CSMAX < 4 ? CSMAX : 4;
        for (int u0 = lo; u0 < hi; u0 += KMAX) {
            const int k = min(KMAX, hi - u0);  // wavefront-uniform
            const int qa = u0 * kWave + lane;
            if (KMAX >= 4 && k == 4)
                nns_pass<D, RS, L1, KMAX, UN>(L, sh, X, Y, centre, rhat, mact, nact, 1, qa, kWave, 0, exact, metric);
            else if (KMAX >= 3 && k == 3)
                nns_pass<D, RS, L1, KMAX >= 3 ? 3 : 1, UN>(L, sh, X, Y, centre, rhat, mact, nact, 1, qa, kWave, 0, exact, metric);
            else if (KMAX >= 2 && k == 2)
                nns_pass<D, RS, L1, KMAX >= 2 ? 2 : 1, UN>(L, sh, X, Y, centre, rhat, mact, nact, 1, qa, kWave, 0, exact, metric);
            else
                nns_pass<D, RS, L1, 1, UN>(L, sh, X, Y, centre, rhat, mact, nact, 1, qa, kWave, 0, exact, metric);
        }
    }
    __syncthreads();
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
                if (mact > 1 && near_tie_dist(dist_of_key(best, metric), dist_of_key(sec, metric)))
                    atomicAdd(&sh.tie_nn, 1ull);
            }
        }
        near += nf;
        __syncthreads();
    }
    return near;
}

}  // namespace ps
}  // namespace nnsemd
