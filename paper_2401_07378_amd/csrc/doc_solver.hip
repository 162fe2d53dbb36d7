// NNS-EMD for high-dimensional point sets (word-embedding documents): one
// workgroup per pair, the distance keys of the whole pair computed once.
//
// Keys: key(i, j) = ||x_i||^2 - 2 x_i . y_j (the consumer's ||y_j||^2 is the
// same for every supplier and drops out of the search).  With BF16 inputs the
// m x n dot products run on the matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulation; each wavefront computes 32 x 32 output tiles from 2 x 2
// MFMA blocks); with FP32 inputs they run on the vector ALUs.  The tile goes
// to a per-workgroup global scratch slot that the rounds read.
//
// Exactness.  Products of BF16 (and the FP32 products fused into FMAs) are
// exact; every addition is taken to round with error at most 2u (u = 2^-24),
// whatever the order.  Bound on |key - exact| written t = tscale (R + ||y||)^2
// with R = max ||x|| (R ||y|| <= (R + ||y||)^2 / 4):
//   unsplit form (FP32 norms, FP32 accumulation over all d products):
//     tscale = 4 (d + 2) u;
//   split form (BF16, d <= 320): every MFMA sums 32 products from a zero
//     accumulator (at most 31 roundings, each at most 2u of the chunk's sum
//     of |x_k y_k|), and the 10 chunk results are added in FP32 in K order
//     (9 roundings of at most u sum |x_k y_k|), so the dot product is within
//     71u ||x|| ||y|| and -2 x.y within 142u R ||y|| <= 35.5u (R + ||y||)^2;
//     the key fma(-2, dot, fl(||x||^2)) adds two roundings (<= 2u (R +
//     ||y||)^2) and the full key fl(key + fl(||y||^2)) two more: 39.5u,
//     tscale = 44u.
//  * Search: a consumer whose two best FP32 keys are closer than 2t (twice
//    the worst disagreement of two keys) is re-scored in FP64 on the
//    suppliers whose FP32 key lies within 2t of the best, in the
//    definition's operation order.  Every pick is therefore the FP64 argmin,
//    ties to the smallest index.
//  * Serve order (greedy protocol): claimants of one supplier are ordered by
//    their full FP32 keys (tile + ||y||^2), each within t_j; two claimants
//    closer than t_a + t_b get exact FP64 keys and are compared on those.
//  * Cost: R = sum f * D over the plan.  The split form takes D from the
//    pick's exact key, or from its FP32 key when the bound makes that term
//    accurate to 1e-5 relative (else every D of the pair is recomputed in
//    FP64); the other forms recompute every D in FP64 after the rounds.
// The plan is thus the one of the FP64 definition, and R agrees with the
// sequential FP64 sum up to the summation order (split form: within 1e-5).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "internal.hpp"
#include "round_common.hpp"

namespace nnsemd {
namespace {

using namespace rc;

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ inline float to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ inline float to_f32(float v) { return v; }
__device__ inline bool finite_in(uint16_t b) { return (b & 0x7F80u) != 0x7F80u; }
__device__ inline bool finite_in(float v) { return isfinite(v); }

__device__ inline float bf_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ inline float bf_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
__device__ inline bool finite_pair(uint32_t w) {
    return (w & 0x7F80u) != 0x7F80u && (w & 0x7F800000u) != 0x7F800000u;
}

// Exact FP64 squared Euclidean key of two points: the sum of the squared
// coordinate differences in dimension order, no fused multiply-add.  Loads
// are 8 or 16 bytes wide when both rows allow it (the arithmetic order is
// the same either way).
template <typename TIn>
__device__ inline double dkey64(const TIn* __restrict__ x, const TIn* __restrict__ y, int d) {
#pragma clang fp contract(off)
    double acc = 0.0;
    int k = 0;
    const uintptr_t al = reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y);
    if constexpr (sizeof(TIn) == 2) {
        if ((al & 7u) == 0) {
            const int d4 = d & ~3;
#pragma unroll 4
            for (; k < d4; k += 4) {
                const uint2 xv = *reinterpret_cast<const uint2*>(x + k);
                const uint2 yv = *reinterpret_cast<const uint2*>(y + k);
                double t;
                t = (double)bf_lo(xv.x) - (double)bf_lo(yv.x);
                acc = acc + t * t;
                t = (double)bf_hi(xv.x) - (double)bf_hi(yv.x);
                acc = acc + t * t;
                t = (double)bf_lo(xv.y) - (double)bf_lo(yv.y);
                acc = acc + t * t;
                t = (double)bf_hi(xv.y) - (double)bf_hi(yv.y);
                acc = acc + t * t;
            }
        }
    } else {
        if ((al & 15u) == 0) {
            const int d4 = d & ~3;
#pragma unroll 2
            for (; k < d4; k += 4) {
                const float4 xv = *reinterpret_cast<const float4*>(x + k);
                const float4 yv = *reinterpret_cast<const float4*>(y + k);
                double t;
                t = (double)xv.x - (double)yv.x;
                acc = acc + t * t;
                t = (double)xv.y - (double)yv.y;
                acc = acc + t * t;
                t = (double)xv.z - (double)yv.z;
                acc = acc + t * t;
                t = (double)xv.w - (double)yv.w;
                acc = acc + t * t;
            }
        }
    }
    for (; k < d; ++k) {
        const double t = (double)to_f32(x[k]) - (double)to_f32(y[k]);
        acc = acc + t * t;
    }
    return acc;
}

// FP64 squared Euclidean distances of E row pairs (x[e], y[e]), each shared
// by G lanes (lane gl of them): each lane sums the squared differences of
// its coordinate groups, the partial sums meet in a shuffle tree and every
// lane returns the totals.  BF16 rows of d <= 4 G kGroupLoads with 8-byte
// alignment issue all their loads at once (E pairs in flight); otherwise a
// plain strided loop.  Any summation order: for the cost only, never for a
// decision.
constexpr int kGroupLoads = 8;

template <int G, int E, typename TIn>
__device__ inline void dkey64_group(const TIn* const (&x)[E], const TIn* const (&y)[E], const bool (&on)[E], int d,
                                    int gl, double (&out)[E]) {
    double acc[E][2];
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e][0] = acc[e][1] = 0.0;
    bool fast = sizeof(TIn) == 2 && (d & 3) == 0 && d <= 4 * G * kGroupLoads;
#pragma unroll
    for (int e = 0; e < E; ++e)
        fast = fast && ((reinterpret_cast<uintptr_t>(x[e]) | reinterpret_cast<uintptr_t>(y[e])) & 7u) == 0;
    if constexpr (sizeof(TIn) == 2) {
        if (fast) {
            uint2 xv[E][kGroupLoads], yv[E][kGroupLoads];
#pragma unroll
            for (int e = 0; e < E; ++e)
#pragma unroll
                for (int u = 0; u < kGroupLoads; ++u) {
                    const int k = 4 * (gl + G * u);
                    const bool in = on[e] && k < d;
                    xv[e][u] = in ? *reinterpret_cast<const uint2*>(x[e] + k) : make_uint2(0u, 0u);
                    yv[e][u] = in ? *reinterpret_cast<const uint2*>(y[e] + k) : make_uint2(0u, 0u);
                }
#pragma unroll
            for (int e = 0; e < E; ++e)
#pragma unroll
                for (int u = 0; u < kGroupLoads; ++u) {
                    const double t0 = (double)bf_lo(xv[e][u].x) - (double)bf_lo(yv[e][u].x);
                    const double t1 = (double)bf_hi(xv[e][u].x) - (double)bf_hi(yv[e][u].x);
                    const double t2 = (double)bf_lo(xv[e][u].y) - (double)bf_lo(yv[e][u].y);
                    const double t3 = (double)bf_hi(xv[e][u].y) - (double)bf_hi(yv[e][u].y);
                    acc[e][0] = fma(t0, t0, acc[e][0]);
                    acc[e][1] = fma(t1, t1, acc[e][1]);
                    acc[e][0] = fma(t2, t2, acc[e][0]);
                    acc[e][1] = fma(t3, t3, acc[e][1]);
                }
        }
    }
    if (!fast) {
#pragma unroll
        for (int e = 0; e < E; ++e)
            for (int k = gl; on[e] && k < d; k += G) {
                const double t = (double)to_f32(x[e][k]) - (double)to_f32(y[e][k]);
                acc[e][0] = fma(t, t, acc[e][0]);
            }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        double a = acc[e][0] + acc[e][1];
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) a += __shfl_xor(a, o);
        out[e] = a;
    }
}

// This lane's part (lane gl of G sharing the row) of the FP32 squared norm
// of one row, and whether any coordinate is not finite.  Any summation
// order is covered by the error bounds above.
template <int G, typename TIn>
__device__ inline float norm2_part(const TIn* __restrict__ row, int d, int gl, bool& bad) {
    float s2 = 0.f;
    int k0 = 0;
    if constexpr (sizeof(TIn) == 2) {
        if (((d & 3) == 0) && ((reinterpret_cast<uintptr_t>(row) & 7u) == 0)) {
            for (int c = gl; c < d / 4; c += G) {
                const uint2 v = *reinterpret_cast<const uint2*>(row + 4 * c);
                bad |= !finite_pair(v.x) || !finite_pair(v.y);
                const float f0 = bf_lo(v.x), f1 = bf_hi(v.x), f2 = bf_lo(v.y), f3 = bf_hi(v.y);
                s2 = fmaf(f0, f0, s2);
                s2 = fmaf(f1, f1, s2);
                s2 = fmaf(f2, f2, s2);
                s2 = fmaf(f3, f3, s2);
            }
            k0 = d;
        }
    } else {
        if (((d & 3) == 0) && ((reinterpret_cast<uintptr_t>(row) & 15u) == 0)) {
            for (int c = gl; c < d / 4; c += G) {
                const float4 v = *reinterpret_cast<const float4*>(row + 4 * c);
                bad |= !isfinite(v.x) || !isfinite(v.y) || !isfinite(v.z) || !isfinite(v.w);
                s2 = fmaf(v.x, v.x, s2);
                s2 = fmaf(v.y, v.y, s2);
                s2 = fmaf(v.z, v.z, s2);
                s2 = fmaf(v.w, v.w, s2);
            }
            k0 = d;
        }
    }
    for (int k = k0 + gl; k < d; k += G) {
        const TIn v = row[k];
        bad |= !finite_in(v);
        const float f = to_f32(v);
        s2 = fmaf(f, f, s2);
    }
    return s2;
}

// 8 consecutive BF16 values of row r starting at column k0 (zeros beyond d
// or for rows >= rows), as an MFMA fragment.
__device__ inline bf16x8 frag8(const uint16_t* __restrict__ base, int r, int rows, int k0, int d) {
    union {
        uint2 w[2];
        uint32_t s[4];
        bf16x8 v;
    } u;
    if (r < rows && k0 + 8 <= d) {
        const uint16_t* p = base + (size_t)r * d + k0;
        if ((reinterpret_cast<uintptr_t>(p) & 7u) == 0) {
            u.w[0] = reinterpret_cast<const uint2*>(p)[0];
            u.w[1] = reinterpret_cast<const uint2*>(p)[1];
            return u.v;
        }
    }
    uint16_t h[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) h[e] = (r < rows && k0 + e < d) ? base[(size_t)r * d + k0 + e] : (uint16_t)0;
#pragma unroll
    for (int e = 0; e < 4; ++e) u.s[e] = (uint32_t)h[2 * e] | ((uint32_t)h[2 * e + 1] << 16);
    return u.v;
}

// Key tile with matrix cores: each wavefront owns 32 x 32 output tiles; the
// fragments of the next K step are loaded while the current one multiplies.
// MFMA 16x16x32 lane layout (checked on gfx950): A lane l holds row l%16,
// k = 8(l/16)..+8; B lane l holds column l%16, the same k; C lane l
// register r is row 4(l/16)+r, column l%16.
template <int T>
__device__ void key_tile_mfma(const uint16_t* __restrict__ X, const uint16_t* __restrict__ Y, int m, int n, int ld,
                              int d, const float* __restrict__ xx, float* __restrict__ tile) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x / 64;
    const int tm = (m + 31) / 32, tn = (n + 31) / 32;
    const int ksteps = (d + 31) / 32;
    const int r16 = lane & 15, kq = 8 * (lane >> 4);
    for (int t = wave; t < tm * tn; t += T / 64) {
        const int i0 = (t / tn) * 32, j0 = (t % tn) * 32;
        f32x4 acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
        bf16x8 a0 = frag8(X, i0 + r16, m, kq, d);
        bf16x8 a1 = frag8(X, i0 + 16 + r16, m, kq, d);
        bf16x8 b0 = frag8(Y, j0 + r16, n, kq, d);
        bf16x8 b1 = frag8(Y, j0 + 16 + r16, n, kq, d);
        for (int ks = 0; ks < ksteps; ++ks) {
            bf16x8 na0 = a0, na1 = a1, nb0 = b0, nb1 = b1;
            if (ks + 1 < ksteps) {
                const int k1 = (ks + 1) * 32 + kq;
                na0 = frag8(X, i0 + r16, m, k1, d);
                na1 = frag8(X, i0 + 16 + r16, m, k1, d);
                nb0 = frag8(Y, j0 + r16, n, k1, d);
                nb1 = frag8(Y, j0 + 16 + r16, n, k1, d);
            }
            acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[1][1], 0, 0, 0);
            a0 = na0;
            a1 = na1;
            b0 = nb0;
            b1 = nb1;
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = i0 + 16 * a + 4 * (lane >> 4) + r;
                    const int j = j0 + 16 * b + r16;
                    if (i < m && j < n) tile[(size_t)i * ld + j] = xx[i] - 2.f * acc[a][b][r];
                }
    }
}

// K steps of 32 whose consumer fragments stay in registers in
// key_tile_mfma_stripes (d <= 320); larger d takes key_tile_mfma.
constexpr int kStripeKSteps = 10;

// Stripe epilogue shared by both split-form tile passes.  The MFMAs of a
// stripe run transposed (C^T = Y X^T: the consumers' fragments are the A
// operand), so lane l holds consumers jg .. jg + 3 (jg = j0 + 4 (l / 16))
// against supplier i0 + l % 16 (first block half) and i0 + 16 + l % 16
// (second half).  Each half is one 16-byte store of four consecutive keys
// of tile row i (rows padded to a multiple of 16 columns), and the running
// best / second-best / best-index of the four consumers take the suppliers
// in ascending order.
struct StripeTop {
    float b1[4], b2[4];
    int bs[4];
};

__device__ inline void stripe_top_init(StripeTop& tp) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        tp.b1[r] = INFINITY;
        tp.b2[r] = INFINITY;
        tp.bs[r] = 0x7fffffff;
    }
}

__device__ inline void stripe_block_epilogue(const float (&dot0)[4], const float (&dot1)[4], int i0, int m, int jg,
                                             int n, int ld, const double* __restrict__ xx,
                                             const float* __restrict__ amass, float* __restrict__ tile,
                                             StripeTop& tp) {
    const int r16 = threadIdx.x & 15;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int i = i0 + 16 * h + r16;
        if (i < m) {
            const float xf = (float)xx[i];
            float v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = fmaf(-2.f, h == 0 ? dot0[r] : dot1[r], xf);
            if (jg < n) *reinterpret_cast<float4*>(tile + (size_t)i * ld + jg) = make_float4(v[0], v[1], v[2], v[3]);
            if (amass[i] > 0.f) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const bool lt = v[r] < tp.b1[r];
                    tp.bs[r] = lt ? i : tp.bs[r];
                    tp.b2[r] = __builtin_amdgcn_fmed3f(tp.b1[r], v[r], tp.b2[r]);
                    tp.b1[r] = fminf(tp.b1[r], v[r]);
                }
            }
        }
    }
}

// Merge of the 16 lanes that hold the same four consumers (smallest key,
// ties to the smallest index; the second-best of the multiset); lane
// 16 g then writes consumers jg .. jg + 3.
__device__ inline void stripe_top_finish(StripeTop& tp, int jg, int n, float* __restrict__ b1,
                                         float* __restrict__ b2, int32_t* __restrict__ bs) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            const float c1 = __shfl_xor(tp.b1[r], o);
            const float c2 = __shfl_xor(tp.b2[r], o);
            const int cs2 = __shfl_xor(tp.bs[r], o);
            const float n2 = fminf(fmaxf(tp.b1[r], c1), fminf(tp.b2[r], c2));
            const bool take = (c1 < tp.b1[r]) || (c1 == tp.b1[r] && cs2 < tp.bs[r]);
            tp.b1[r] = take ? c1 : tp.b1[r];
            tp.bs[r] = take ? cs2 : tp.bs[r];
            tp.b2[r] = n2;
        }
    }
    if ((threadIdx.x & 15) == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (jg + r < n) {
                b1[jg + r] = tp.b1[r];
                b2[jg + r] = tp.b2[r];
                bs[jg + r] = tp.bs[r];
            }
    }
}

// Key tile with matrix cores for the split form, consumer-stationary: the
// four wavefronts each own a stripe of 16 consumers (their BF16 fragments
// for all of K loaded once into registers: the only read of the candidate
// rows), while the workgroup stages the supplier rows 32 at a time in LDS
// (zero-padded to whole K steps) and every wavefront multiplies its stripe
// with them.  ||y||^2 and the finiteness of every coordinate come from the
// consumers' fragments.  It also takes the first round's search from the
// keys in registers: for every consumer the best and second-best key over
// the suppliers of positive mass and the smallest local index holding the
// best, with the same update and merge rules as the search over the stored
// tile.  Lane layout as in key_tile_mfma.  xs: LDS, 32 x kStripeLdx BF16.
constexpr int kStripeLdx = kStripeKSteps * 32 + 8;

template <int T>
__device__ void key_tile_mfma_stripes(const uint16_t* __restrict__ X, const uint16_t* __restrict__ Y, int m, int n,
                                      int ld, int d, const double* __restrict__ xx, float* __restrict__ tile,
                                      float* __restrict__ yy, bool& bad, const float* __restrict__ amass,
                                      float* __restrict__ r1b1, float* __restrict__ r1b2, int32_t* __restrict__ r1bs,
                                      uint16_t* __restrict__ xs
#ifdef NNSEMD_PHASE_TILE
                                      , uint64_t (&ph)[9], uint64_t& ph_t
#endif
) {
    constexpr int KS = kStripeKSteps;
    constexpr int NW = T / 64;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid / 64;
    const int tm = (m + 31) / 32, tn = (n + 15) / 16;
    const int ksteps = (d + 31) / 32;
    const int kp = ksteps * 32;
    const int r16 = lane & 15, kq = 8 * (lane >> 4);
    const bool rows8 = (d & 3) == 0 && (reinterpret_cast<uintptr_t>(X) & 7u) == 0;
    // Double buffering (8-byte rows): the next supplier block is loaded into
    // registers while the current one is multiplied.
    constexpr int PRE = (32 * (KS * 32 / 4) + T - 1) / T;
    const int nq = 32 * (kp / 4);
    uint2 pre[PRE];
    auto fetch = [&](int ib) {
        const int i0 = ib * 32;
#pragma unroll
        for (int u = 0; u < PRE; ++u) {
            const int e = tid + u * T;
            pre[u] = make_uint2(0u, 0u);
            if (e < nq) {
                const int r = e / (kp / 4), k = 4 * (e % (kp / 4));
                if (i0 + r < m && k < d) pre[u] = *reinterpret_cast<const uint2*>(X + (size_t)(i0 + r) * d + k);
            }
        }
    };
    if (rows8 && tm > 0) fetch(0);
    for (int sg = 0; sg < (tn + NW - 1) / NW; ++sg) {
        const int cs = sg * NW + wave;
        const bool mine = cs < tn;
        const int j0 = cs * 16;
        bf16x8 yb[KS];
        StripeTop tp;
        stripe_top_init(tp);
        if (mine) {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
                if (ks < ksteps) yb[ks] = frag8(Y, j0 + r16, n, ks * 32 + kq, d);
            double ss = 0.0;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                if (ks < ksteps) {
                    union {
                        bf16x8 v;
                        uint32_t w[4];
                    } u;
                    u.v = yb[ks];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        bad |= !finite_pair(u.w[e]);
                        const double f0 = bf_lo(u.w[e]), f1 = bf_hi(u.w[e]);
                        ss = fma(f0, f0, ss);
                        ss = fma(f1, f1, ss);
                    }
                }
            }
            ss += __shfl_xor(ss, 16);
            ss += __shfl_xor(ss, 32);
            if (lane < 16 && j0 + r16 < n) yy[j0 + r16] = (float)ss;
        }
#ifdef NNSEMD_PHASE_TILE
        NNSEMD_PH(1)
#endif
        for (int ib = 0; ib < tm; ++ib) {
            const int i0 = ib * 32;
            __syncthreads();  // the previous block's fragments have been read
            if (rows8) {
#pragma unroll
                for (int u = 0; u < PRE; ++u) {
                    const int e = tid + u * T;
                    if (e < nq) {
                        const int r = e / (kp / 4), k = 4 * (e % (kp / 4));
                        *reinterpret_cast<uint2*>(&xs[r * kStripeLdx + k]) = pre[u];
                    }
                }
            } else {
                for (int e = tid; e < 32 * kp; e += T) {
                    const int r = e / kp, k = e % kp;
                    xs[r * kStripeLdx + k] = (i0 + r < m && k < d) ? X[(size_t)(i0 + r) * d + k] : (uint16_t)0;
                }
            }
            __syncthreads();
            if (rows8) fetch(ib + 1 < tm ? ib + 1 : 0);  // next block (the first again for the next stripes)
#ifdef NNSEMD_PHASE_TILE
            NNSEMD_PH(2)
#endif
            if (!mine) continue;
            // each K step from a zero accumulator (at most 31 roundings),
            // the chunk results added in FP32 in K order
            float dot0[4] = {0.f, 0.f, 0.f, 0.f}, dot1[4] = {0.f, 0.f, 0.f, 0.f};
            const f32x4 zero = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                if (ks < ksteps) {
                    union {
                        uint4 u;
                        bf16x8 v;
                    } f0, f1;
                    f0.u = *reinterpret_cast<const uint4*>(&xs[r16 * kStripeLdx + ks * 32 + kq]);
                    f1.u = *reinterpret_cast<const uint4*>(&xs[(16 + r16) * kStripeLdx + ks * 32 + kq]);
                    const f32x4 c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yb[ks], f0.v, zero, 0, 0, 0);
                    const f32x4 c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yb[ks], f1.v, zero, 0, 0, 0);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        dot0[r] += c0[r];
                        dot1[r] += c1[r];
                    }
                }
            }
#ifdef NNSEMD_PHASE_TILE
            NNSEMD_PH(3)
#endif
            stripe_block_epilogue(dot0, dot1, i0, m, j0 + 4 * (lane >> 4), n, ld, xx, amass, tile, tp);
#ifdef NNSEMD_PHASE_TILE
            NNSEMD_PH(4)
#endif
        }
        if (mine) stripe_top_finish(tp, j0 + 4 * (lane >> 4), n, r1b1, r1b2, r1bs);
    }
}

// Key tile on the vector ALUs (FP32 inputs) for launches of few pairs: each
// lane owns a 4 x 4 block of (i, j) and walks the d products with 16-byte
// loads from global memory when rows allow it, with no barrier (a pair that
// has a CU to itself is bound by latency, not by the L2).
template <int T>
__device__ void key_tile_valu_direct(const float* __restrict__ X, const float* __restrict__ Y, int m, int n, int ld, int d,
                              const float* __restrict__ xx, float* __restrict__ tile) {
    const int bm = (m + 3) / 4, bn = (n + 3) / 4;
    const bool vec = (d & 3) == 0 && ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Y)) & 15u) == 0;
    for (int e = threadIdx.x; e < bm * bn; e += T) {
        const int i0 = (e / bn) * 4, j0 = (e % bn) * 4;
        const float* xr[4];
        const float* yr[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            xr[u] = X + (size_t)min(i0 + u, m - 1) * d;  // clamped rows are computed, not stored
            yr[u] = Y + (size_t)min(j0 + u, n - 1) * d;
        }
        float acc[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = 0.f;
        int k = 0;
        if (vec) {
            for (; k < d; k += 4) {
                float4 xv[4], yv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    xv[u] = *reinterpret_cast<const float4*>(xr[u] + k);
                    yv[u] = *reinterpret_cast<const float4*>(yr[u] + k);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        acc[u][v] = fmaf(xv[u].x, yv[v].x, acc[u][v]);
                        acc[u][v] = fmaf(xv[u].y, yv[v].y, acc[u][v]);
                        acc[u][v] = fmaf(xv[u].z, yv[v].z, acc[u][v]);
                        acc[u][v] = fmaf(xv[u].w, yv[v].w, acc[u][v]);
                    }
            }
        }
        for (; k < d; ++k) {
            float xs[4], ys[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                xs[u] = xr[u][k];
                ys[u] = yr[u][k];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = fmaf(xs[u], ys[v], acc[u][v]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                if (i0 + u < m && j0 + v < n) tile[(size_t)(i0 + u) * ld + j0 + v] = xx[i0 + u] - 2.f * acc[u][v];
    }
}

// Key tile on the vector ALUs (FP32 inputs) for batches, blocked through LDS
// (the direct form re-reads every operand through the L2, which the whole
// chip then contends for): the workgroup computes 64 x 64 blocks of (i, j);
// each K chunk of 16 of both
// row panels is staged in LDS (transposed, zero-padded), and each thread
// accumulates a 4 x 4 block with FMAs.  Any accumulation order is covered by
// the FP32 bound of the unsplit form.  stage: LDS, 2 x 16 x kValuLd floats,
// 16-byte aligned.
constexpr int kValuBK = 16;
constexpr int kValuLd = 68;  // 64 rows + padding (keeps the float4 reads aligned)
constexpr size_t kValuStageBytes = sizeof(float) * 2 * kValuBK * kValuLd;
constexpr unsigned kValuBlockedMinPairs = 256;  // launches of at least one pair per CU

template <int T>
__device__ void key_tile_valu(const float* __restrict__ X, const float* __restrict__ Y, int m, int n, int ld, int d,
                              const float* __restrict__ xx, float* __restrict__ tile, float* __restrict__ stage) {
    static_assert(T == 256, "16 x 16 threads of 4 x 4 outputs");
    float* xs = stage;                      // [kValuBK][kValuLd]: X panel, k-major
    float* ys = stage + kValuBK * kValuLd;  // [kValuBK][kValuLd]: Y panel
    const int tid = threadIdx.x;
    const int ty = tid / 16, tx = tid % 16;
    const int bm = (m + 63) / 64, bn = (n + 63) / 64;
    for (int blk = 0; blk < bm * bn; ++blk) {
        const int i0 = (blk / bn) * 64, j0 = (blk % bn) * 64;
        float acc[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = 0.f;
        for (int k0 = 0; k0 < d; k0 += kValuBK) {
            __syncthreads();  // the previous chunk has been read
#pragma unroll
            for (int q = 0; q < 64 * kValuBK / T; ++q) {
                const int e = tid + q * T;
                const int r = e / kValuBK, k = e % kValuBK;
                const bool kin = k0 + k < d;
                xs[k * kValuLd + r] = (i0 + r < m && kin) ? X[(size_t)(i0 + r) * d + k0 + k] : 0.f;
                ys[k * kValuLd + r] = (j0 + r < n && kin) ? Y[(size_t)(j0 + r) * d + k0 + k] : 0.f;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kValuBK; ++k) {
                const float4 a = *reinterpret_cast<const float4*>(&xs[k * kValuLd + 4 * ty]);
                const float4 b = *reinterpret_cast<const float4*>(&ys[k * kValuLd + 4 * tx]);
                const float av[4] = {a.x, a.y, a.z, a.w}, bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[u][v] = fmaf(av[u], bv[v], acc[u][v]);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + 4 * ty + u;
            if (i >= m) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int j = j0 + 4 * tx + v;
                if (j < n) tile[(size_t)i * ld + j] = xx[i] - 2.f * acc[u][v];
            }
        }
    }
}

// Greedy serve order of the claimants (see the file comment): rank of each
// claimant in its bucket from the full FP32 keys; claimants with an
// undecided comparison get exact keys and are ranked again.
// Comparisons closer than the two keys' bounds plus the near-tie window are
// settled on exact keys, so every pair of neighbours in the final order that
// may be a near tie carries exact keys, and the near ties of neighbouring
// claimants are counted on those (ties_order).
template <int T, typename TIn>
__device__ inline void rank_greedy_doc(const Lds16& L, Shared& sh, int nact, const float* __restrict__ kap,
                                       const float* __restrict__ yn, float rhat, float tscale,
                                       int32_t* __restrict__ amb, const TIn* __restrict__ X,
                                       const TIn* __restrict__ Y, int d, int metric, int64_t& near,
                                       int64_t& ties_order) {
    for (int pass = 0; pass < 2; ++pass) {
        const int cnt = pass == 0 ? nact : sh.namb;
        for (int q = threadIdx.x; q < cnt; q += T) {
            const int j = pass == 0 ? L.cact[q] : amb[q];
            const int sl = L.cnn[j];
            const int c = L.scnt[sl];
            const int end = L.soff[sl];
            const int start = end - c;
            int rank = 0;
            bool undecided = false;
            if (c > 1) {
                const float a = kap[j];
                const float ea = rhat + yn[j];
                const float ta = tscale * ea * ea;
                const double ka = L.ckey[j];
#pragma unroll 4
                for (int e = start; e < end; ++e) {
                    const int j2 = L.list[e];
                    if (j2 == j) continue;
                    const float b = kap[j2];
                    const float eb = rhat + yn[j2];
                    const float tb = ta + tscale * eb * eb;
                    const float tol = tb + near_window(fmaxf(a, b) + tb, false);
                    if (b < a - tol) {
                        ++rank;
                    } else if (!(b > a + tol)) {
                        const double kb = L.ckey[j2];
                        if (ka >= 0.0 && kb >= 0.0)
                            rank += (kb < ka) || (kb == ka && j2 < j);
                        else
                            undecided = true;
                    }
                }
            }
            // (No comparison is undecided in the second pass: both sides of
            // each undecided one now carry exact keys.)
            if (undecided && pass == 0)
                amb[atomicAdd(&sh.namb, 1)] = j;
            else
                L.sorted[start + rank] = j;
        }
        __syncthreads();
        const int na = sh.namb;
        if (pass == 1 || na == 0) break;
        // Undecided comparisons are symmetric, so both claimants of each one
        // are listed; their exact keys decide the second pass.
        for (int f = threadIdx.x; f < na; f += T) {
            const int j = amb[f];
            L.ckey[j] = dkey64<TIn>(X + (size_t)L.sidx[L.cnn[j]] * d, Y + (size_t)j * d, d);
        }
        near += na;
        __syncthreads();
    }
    __syncthreads();
    // neighbours in serve order: a near tie needs both exact keys (above)
    for (int e = threadIdx.x; e < nact; e += T) {
        const int j = L.sorted[e];
        const int sl = L.cnn[j];
        if (e > L.soff[sl] - L.scnt[sl]) {
            const double kp = L.ckey[L.sorted[e - 1]], kj = L.ckey[j];
            if (kp >= 0.0 && kj >= 0.0 && keys_near(kp, kj, metric)) ++ties_order;
        }
    }
    if (threadIdx.x == 0) sh.namb = 0;
    __syncthreads();  // the serve walk overwrites the keys and picks read above
}

// Relative accuracy of the served distances in the split form's cost: a
// term is taken from the FP32 key when its bound guarantees this, else the
// whole cost is taken from exact FP64 distances.
constexpr double kKeyCostTau = 1e-5;

// Distances of this round's picks for the split form's cost, taken before
// the serve walk (one thread per active consumer, in place of the pick's
// key, which the walk then replaces by the flow; round_walk is called with
// the squared-Euclidean rule so that it uses these values as they are).  D
// comes from the pick's exact FP64 key where the round computed one, else
// from the FP32 full key kap (|kap - D^2| <= t = tscale (R + ||y||)^2): when
// kap >= t (1 + 1/tau), D^2 >= kap - t > 0 and the term's relative error is
// at most t / (kap - t) <= tau (for L2, |sqrt(kap) - D| / D <= t / D^2).  A
// pick that fails the test sets the LDS flag loose_flag, and the caller
// then recomputes every distance exactly instead.
template <int T, typename LT>
__device__ inline void doc_pick_distances(const LT& L, int& loose_flag, int nact, int metric,
                                          const float* __restrict__ kap, const float* __restrict__ yn, float rhat,
                                          float tscale) {
    bool loose = false;
    for (int q = threadIdx.x; q < nact; q += T) {
        const int j = L.cact[q];
        const double ek = L.ckey[j];
        double key = ek;
        if (!(ek >= 0.0)) {
            key = (double)kap[j];
            const double e = (double)rhat + (double)yn[j];
            const double t = (double)tscale * e * e * (1.0 + 1e-6);
            loose |= !(key >= t * (1.0 + 1.0 / kKeyCostTau));
        }
        L.ckey[j] = dist_of_key(key, metric);
    }
    if (loose) loose_flag = 1;
    __syncthreads();
}

// Row ranges of pair p (status INVALID_ARG and empty sides if the tables or
// sizes are out of range).
__device__ inline int resolve_pair(const DocArgs& A, int64_t p, int64_t& x0, int64_t& m, int64_t& y0, int64_t& n) {
    x0 = 0;
    y0 = 0;
    m = A.single_m;
    n = A.single_n;
    int status = NNSEMD_OK;
    if (A.x_off != nullptr) {
        const int64_t px = A.pair_x ? (int64_t)A.pair_x[p] : p;
        const int64_t py = A.pair_y ? (int64_t)A.pair_y[p] : p;
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
    return status;
}

// SPLIT: the key tile, the norms, the coordinates' finiteness and the first
// round's search were done by doc_tile_kernel into this workgroup's slot.
template <typename TIn, bool MFMA, int T, int CSMAX, bool SPLIT>
__device__ void solve_doc_pair(const DocArgs& A, int64_t p, char* __restrict__ slot, const Lds16& L,
                               float* __restrict__ xx, float* __restrict__ yy, float* __restrict__ yn,
                               float* __restrict__ kap, int32_t* __restrict__ amb, Shared& sh, int& kloose,
                               float* __restrict__ vstage) {
    constexpr int NW = T / 64;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid / 64;
    const int d = A.d;
    NNSEMD_PH_DECL

    int64_t x0, y0, m, n;
    int status = resolve_pair(A, p, x0, m, y0, n);
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
    // Plan destination: the caller's arrays, or the scratch slot (the cost
    // pass reads the plan back either way).
    float* __restrict__ tile = reinterpret_cast<float*>(slot);
    int32_t* psrc = A.plan_src;
    int32_t* pdst = A.plan_dst;
    double* pflow = A.plan_flow;
    if (!want_plan) {
        const size_t tb = doc_tile_bytes(A.max_m, A.max_n);
        const int64_t cap = (int64_t)A.max_m + A.max_n;
        pflow = reinterpret_cast<double*>(slot + tb);
        psrc = reinterpret_cast<int32_t*>(pflow + cap);
        pdst = psrc + cap;
        plan_base = 0;
    }
    const TIn* __restrict__ X = reinterpret_cast<const TIn*>(A.X) + x0 * d;
    const TIn* __restrict__ Y = reinterpret_cast<const TIn*>(A.Y) + y0 * d;
    const int mi = (int)m, ni = (int)n;
    const int ldt = doc_tile_ld(ni);  // tile row stride (columns padded to a multiple of 16)

    // ---- ingest: masses, validity, norms (16 lanes per row)
    double red[4] = {0.0, 0.0, 0.0, 0.0};  // sum a, sum b, bad, max ||x||^2
    const int rop[4] = {0, 0, 2, 2};
    for (int i = tid; i < mi; i += T) {
        const float av = A.a[x0 + i];
        if (!(av >= 0.f) || !isfinite(av)) red[2] = 1.0;
        L.smass[i] = (double)av;
        red[0] += (double)av;
    }
    for (int j = tid; j < ni; j += T) {
        const float bv = A.b[y0 + j];
        if (!(bv >= 0.f) || !isfinite(bv)) red[2] = 1.0;
        L.cmass[j] = (double)bv;
        red[1] += (double)bv;
    }
    const float infl = 1.f + (float)(d + 2) * kU32;  // covers the FP32 norms' own rounding
    // In the split form the tile kernel took the norms, the finiteness and
    // the first round's search; otherwise the norms are taken here.
    const bool stripes = SPLIT;
    const int nrows = SPLIT ? 0 : mi + ni;
    if constexpr (SPLIT) {
        const char* aux = slot + doc_aux_offset(A.max_m, A.max_n);
        const float* axx = reinterpret_cast<const float*>(aux);
        const float* ayy = axx + A.max_m;
        const float* ab1 = ayy + A.max_n;
        const float* ab2 = ab1 + A.max_n;
        const int32_t* abs_ = reinterpret_cast<const int32_t*>(ab2 + A.max_n);
        const int32_t* aflag = abs_ + A.max_n;
        for (int i = tid; i < mi; i += T) {
            xx[i] = axx[i];
            red[3] = fmax(red[3], (double)axx[i]);
        }
        for (int j = tid; j < ni; j += T) {
            const float s2 = ayy[j];
            yy[j] = s2;
            yn[j] = sqrtf(s2) * infl;
            kap[j] = ab1[j];
            L.ckey[j] = (double)ab2[j];
            L.cnn[j] = abs_[j];
        }
        if (tid == 0 && mi + ni > 0 && *aflag != 0) red[2] = 1.0;
    }
    {
        constexpr int G = 16;
        const int gl = tid & (G - 1);
        for (int r0 = 0; r0 < nrows; r0 += T / G) {
            const int row = r0 + tid / G;
            bool bad = false;
            float s2 = 0.f;
            if (row < nrows) {
                const TIn* pr = row < mi ? X + (size_t)row * d : Y + (size_t)(row - mi) * d;
                s2 = norm2_part<G, TIn>(pr, d, gl, bad);
            }
            int bi = bad ? 1 : 0;
#pragma unroll
            for (int o = G / 2; o > 0; o >>= 1) {
                s2 += __shfl_xor(s2, o);
                bi |= __shfl_xor(bi, o);
            }
            if (gl == 0 && row < nrows) {
                if (bi) red[2] = 1.0;
                if (row < mi) {
                    xx[row] = s2;
                    red[3] = fmax(red[3], (double)s2);
                } else {
                    yy[row - mi] = s2;
                    yn[row - mi] = sqrtf(s2) * infl;
                }
            }
        }
    }
    block_reduce<T, 4>(red, rop, &sh.red[0][0]);
    if (status == NNSEMD_OK && red[2] != 0.0) status = NNSEMD_ERR_INVALID_ARG;
    if (status == NNSEMD_OK) {
        const double big = fmax(red[0], red[1]);
        if (fabs(red[0] - red[1]) > 1e-5 * big) status = NNSEMD_ERR_MASS_MISMATCH;
    }
    const float rhat = sqrtf((float)red[3]) * infl;
    // Key error bound t = tscale (R + ||y||)^2; the search gap threshold is 2t.
    const float tscale = SPLIT ? 44.f * kU32 : 4.f * (float)(d + 2) * kU32;

    NNSEMD_PH(0)
    // ---- key tile
    if (!SPLIT && status == NNSEMD_OK) {
        if constexpr (MFMA) {
            key_tile_mfma<T>(reinterpret_cast<const uint16_t*>(X), reinterpret_cast<const uint16_t*>(Y), mi, ni, ldt, d, xx,
                             tile);
        } else {
            if (gridDim.x >= kValuBlockedMinPairs)
                key_tile_valu<T>(reinterpret_cast<const float*>(X), reinterpret_cast<const float*>(Y), mi, ni, ldt, d,
                                 xx, tile, vstage);
            else
                key_tile_valu_direct<T>(reinterpret_cast<const float*>(X), reinterpret_cast<const float*>(Y), mi, ni,
                                        ldt, d, xx, tile);
        }
    }
    __syncthreads();
    NNSEMD_PH(1)

    // ---- initial active sets (zero-mass points never enter)
    int mact = 0, nact = 0;
    if (status == NNSEMD_OK) {
        const int cs = (mi + T - 1) / T;
        const int cc = (ni + T - 1) / T;
        const int slo = min(tid * cs, mi);
        const int clo = min(tid * cc, ni), chi = min(clo + cc, ni);
        double mv[CSMAX];
        int ks = 0, kc = 0;
#pragma unroll
        for (int u = 0; u < CSMAX; ++u) {
            const int i = slo + u;
            mv[u] = (u < cs && i < mi) ? L.smass[i] : 0.0;
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
            L.soff[slo + u] = ps;  // slot of a local index, for the first round
            L.smass[ps] = mv[u];
            L.scnt[ps] = 0;
            ++ps;
        }
        for (int j = clo; j < chi; ++j)
            if (L.cmass[j] > 0.0) L.cact[pc++] = j;
        if (tid == 0) {
            sh.nflag = 0;
            sh.namb = 0;
            kloose = 0;
        }
        __syncthreads();
    }

    // ---- rounds
    const int64_t max_rounds = A.max_rounds > 0 ? A.max_rounds : (int64_t)mi + ni;
    int rounds = 0;
    int64_t work = 0, nnz = 0, near = 0;
    int64_t ties_nn = 0, ties_order = 0;  // this thread's near-tie counts
    double wcost = 0.0;                    // split form: this thread's part of R from the walk
    float* flag_b1 = reinterpret_cast<float*>(amb);  // re-score cutoff of each flagged consumer (amb is free until the order)
    while (status == NNSEMD_OK && mact > 0 && nact > 0) {
        if (rounds >= max_rounds) {
            status = NNSEMD_ERR_NOT_CONVERGED;
            break;
        }
        work += (int64_t)mact * nact;
        if (rounds == 0 && stripes) {
            // First round: the tile pass already found every consumer's best
            // and second-best key (all suppliers of positive mass are active).
            for (int q = tid; q < nact; q += T) {
                const int j = L.cact[q];
                const float b1 = kap[j], b2 = (float)L.ckey[j];
                const int bl = L.cnn[j];
                const float e = rhat + yn[j];
                const float thr = 2.f * tscale * e * e + 1e-30f;
                const float win = thr + near_window(b1 + yy[j] + thr, false);
                if (!(b2 - b1 > win)) {
                    const int f = atomicAdd(&sh.nflag, 1);
                    L.list[f] = j;
                    flag_b1[f] = b1 + win;
                } else {
                    const int bs = L.soff[bl];
                    L.cnn[j] = bs;
                    kap[j] = b1 + yy[j];
                    L.ckey[j] = -1.0;  // exact key not known
                    cnt_add(L.scnt, bs);
                }
            }
        } else {
        // NNS over the key tile: S lanes per consumer when consumers are few.
        int S = 1;
        while (S < 64 && nact * S * 2 <= T) S <<= 1;
        while (S > 1 && S > mact) S >>= 1;
        const int r = tid & (S - 1);
        const int g = tid / S;
        const int G = T / S;
        for (int q0 = 0; q0 < nact; q0 += G) {
            const int q = q0 + g;
            const bool valid = q < nact;
            const int j = L.cact[valid ? q : 0];
            float b1 = INFINITY, b2 = INFINITY;
            int bs = 0x7fffffff;
            constexpr int U = 16;
            const int stride = S * U;
            const int full = (mact / stride) * stride;
            for (int s0 = r; s0 < full; s0 += stride) {
                float kk[U];
#pragma unroll
                for (int u = 0; u < U; ++u) kk[u] = tile[(size_t)L.sidx[s0 + u * S] * ldt + j];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const bool lt = kk[u] < b1;
                    bs = lt ? s0 + u * S : bs;
                    b2 = __builtin_amdgcn_fmed3f(b1, kk[u], b2);
                    b1 = fminf(b1, kk[u]);
                }
            }
            for (int s = full + r; s < mact; s += S) {
                const float k = tile[(size_t)L.sidx[s] * ldt + j];
                const bool lt = k < b1;
                bs = lt ? s : bs;
                b2 = __builtin_amdgcn_fmed3f(b1, k, b2);
                b1 = fminf(b1, k);
            }
            for (int o = 1; o < S; o <<= 1) {
                const float c1 = __shfl_xor(b1, o);
                const float c2 = __shfl_xor(b2, o);
                const int cs2 = __shfl_xor(bs, o);
                const float n2 = fminf(fmaxf(b1, c1), fminf(b2, c2));
                const bool take = (c1 < b1) || (c1 == b1 && cs2 < bs);
                b1 = take ? c1 : b1;
                bs = take ? cs2 : bs;
                b2 = n2;
            }
            if (valid && r == 0) {
                const float e = rhat + yn[j];
                const float thr = 2.f * tscale * e * e + 1e-30f;
                const float win = thr + near_window(b1 + yy[j] + thr, false);
                if (!(b2 - b1 > win)) {
                    const int f = atomicAdd(&sh.nflag, 1);
                    L.list[f] = j;
                    flag_b1[f] = b1 + win;
                } else {
                    L.cnn[j] = bs;
                    kap[j] = b1 + yy[j];
                    L.ckey[j] = -1.0;  // exact key not known
                    cnt_add(L.scnt, bs);
                }
            }
        }
        }
        __syncthreads();
        NNSEMD_PH(2)
        const int nf = sh.nflag;
        if (nf > 0) {
            // Flagged consumers: the FP64 argmin, and any supplier that is a
            // near tie with it, lie among the suppliers whose FP32 key is at
            // most the stored cutoff (best + bound + near-tie window); only
            // those are re-scored.
            for (int f = wave; f < nf; f += NW) {
                const int j = L.list[f];
                const float lim = flag_b1[f];
                double best = INFINITY, sec = INFINITY;
                int bsl = 0x7fffffff;
                for (int s = lane; s < mact; s += 64) {
                    const int i = L.sidx[s];
                    if (tile[(size_t)i * ldt + j] > lim) continue;
                    const double k = dkey64<TIn>(X + (size_t)i * d, Y + (size_t)j * d, d);
                    if (k < best) {
                        sec = best;
                        best = k;
                        bsl = s;
                    } else if (k < sec) {
                        sec = k;
                    }
                }
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
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
                    kap[j] = tile[(size_t)L.sidx[bsl] * ldt + j] + yy[j];
                    cnt_add(L.scnt, bsl);
                    if (mact > 1 && near_tie_dist(dist_of_key(best, A.metric), dist_of_key(sec, A.metric)))
                        ++ties_nn;
                }
            }
            near += nf;
            __syncthreads();
        }
        NNSEMD_PH(3)
        round_buckets<T>(L, sh, mact, nact);
        if (A.protocol == NNSEMD_GREEDY)
            rank_greedy_doc<T, TIn>(L, sh, nact, kap, yn, rhat, tscale, amb, X, Y, d, A.metric, near, ties_order);
        else
            round_rank<T>(L, nact, A.protocol, A.seed, rounds);
        NNSEMD_PH(4)
        if constexpr (SPLIT) {
            doc_pick_distances<T>(L, kloose, nact, A.metric, kap, yn, rhat, tscale);
            round_walk<T, true>(L, mact, NNSEMD_SQEUCLIDEAN, wcost);
        } else {
            double unused = 0.0;
            round_walk<T, false>(L, mact, A.metric, unused);
        }
        NNSEMD_PH(5)
        round_compact<T, CSMAX, 0>(L, sh, mact, nact, nnz, psrc, pdst, pflow, plan_base);
        NNSEMD_PH(6)
        ++rounds;
    }

    double fin[5] = {0.0, 0.0, 0.0, (double)ties_nn, (double)ties_order};
    const int fop[5] = {0, 0, 0, 0, 0};
    if (status == NNSEMD_OK || status == NNSEMD_ERR_NOT_CONVERGED) {
        for (int s = tid; s < mact; s += T) fin[1] += L.smass[s];
        for (int q = tid; q < nact; q += T) fin[2] += L.cmass[L.cact[q]];
    }
    // ---- R = sum f * D.  The split form took every term in its walk unless
    // one failed the key bound (kloose, read after the last round's
    // barriers, the same in every thread).
    const bool exact_cost = !SPLIT || kloose != 0;
    if (status == NNSEMD_OK && !exact_cost) fin[0] = wcost;
    // ---- R = sum f * D over the plan, D from exact FP64 keys.  Entries are
    // sorted by consumer (counting sort in LDS) and dealt to lanes in that
    // order, so neighbouring lanes share a consumer row (one fetch) and heavy
    // consumers are spread over many lanes; each entry's f * D goes to its
    // own slot and the slots are summed in a fixed order, so R does not
    // depend on the sort's order.
    if (status == NNSEMD_OK && exact_cost) {
        __syncthreads();  // residuals read; the LDS below is reused
        int32_t* cnt = reinterpret_cast<int32_t*>(L.ckey);  // [N]
        int32_t* off = cnt + A.max_n;                       // [N]
        int32_t* ent = reinterpret_cast<int32_t*>(L.sidx);  // [m + n] (sidx .. sorted are contiguous)
        double* contrib = L.smass;                          // [m + n] (smass, cmass are contiguous)
        const int ne = (int)nnz;
        for (int j = tid; j < ni; j += T) cnt[j] = 0;
        __syncthreads();
        for (int e = tid; e < ne; e += T) atomicAdd(&cnt[pdst[plan_base + e]], 1);
        __syncthreads();
        {
            const int cs = (ni + T - 1) / T;
            const int lo = min(tid * cs, ni), hi = min(lo + cs, ni);
            int sum = 0;
            for (int j = lo; j < hi; ++j) sum += cnt[j];
            unsigned long long tot;
            int run = (int)block_scan_u64<T>((unsigned long long)sum, &tot, sh);
            for (int j = lo; j < hi; ++j) {
                off[j] = run;
                run += cnt[j];
            }
        }
        __syncthreads();
        for (int e = tid; e < ne; e += T) ent[atomicAdd(&off[pdst[plan_base + e]], 1)] = e;
        __syncthreads();
        // 16 lanes per entry, each taking every 16th group of coordinates;
        // the FP64 partial sums meet in a shuffle tree.  (The cost only needs
        // D to FP64 accuracy, not in the definition's operation order: 300
        // terms in any order stay within 1e-13 relative.)
        {
            constexpr int G = 16, E = SPLIT ? 1 : 2, NG = T / G;  // (split form: rare, kept light)
            const int gl = tid & (G - 1);
            for (int q0 = tid / G; q0 < ne; q0 += E * NG) {
                const TIn* xr[E];
                const TIn* yr[E];
                bool on[E];
                int ee[E];
#pragma unroll
                for (int u = 0; u < E; ++u) {
                    const int q = q0 + u * NG;
                    on[u] = q < ne;
                    ee[u] = on[u] ? ent[q] : 0;
                    const int i = on[u] ? psrc[plan_base + ee[u]] : 0, j = on[u] ? pdst[plan_base + ee[u]] : 0;
                    xr[u] = X + (size_t)i * d;
                    yr[u] = Y + (size_t)j * d;
                }
                double key[E];
                dkey64_group<G, E, TIn>(xr, yr, on, d, gl, key);
#pragma unroll
                for (int u = 0; u < E; ++u)
                    if (gl == 0 && on[u]) contrib[ee[u]] = pflow[plan_base + ee[u]] * dist_of_key(key[u], A.metric);
            }
        }
        __syncthreads();
        for (int e = tid; e < ne; e += T) fin[0] += contrib[e];
    }
    NNSEMD_PH(7)
    block_reduce<T, 5>(fin, fop, &sh.red[0][0]);
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
            st.near_ties_nn = (int64_t)fin[3];
            st.near_ties_order = (int64_t)fin[4];
            A.stats[p] = st;
        }
    }
    NNSEMD_PH(8)
#ifndef NNSEMD_PHASE_TILE
    NNSEMD_PH_FLUSH(A.phase_cycles)
#endif
}

// FP64 squared norm of one BF16 row shared by G lanes (lane gl of them), and
// whether any coordinate is not finite; every lane returns both.
template <int G>
__device__ inline double row_norm_bf16(const uint16_t* __restrict__ pr, int d, int gl, bool& bad) {
    bool rb = false;
    double s2 = 0.0;
    int k0 = 0;
    if ((d & 3) == 0 && (reinterpret_cast<uintptr_t>(pr) & 7u) == 0) {
#pragma unroll 4
        for (int c = gl; c < d / 4; c += G) {
            const uint2 v = *reinterpret_cast<const uint2*>(pr + 4 * c);
            rb |= !finite_pair(v.x) || !finite_pair(v.y);
            const double f0 = bf_lo(v.x), f1 = bf_hi(v.x), f2 = bf_lo(v.y), f3 = bf_hi(v.y);
            s2 = fma(f0, f0, s2);
            s2 = fma(f1, f1, s2);
            s2 = fma(f2, f2, s2);
            s2 = fma(f3, f3, s2);
        }
        k0 = d;
    }
    for (int k = k0 + gl; k < d; k += G) {
        rb |= !finite_in(pr[k]);
        const double f = to_f32(pr[k]);
        s2 = fma(f, f, s2);
    }
    int bi = rb ? 1 : 0;
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
        s2 += __shfl_xor(s2, o);
        bi |= __shfl_xor(bi, o);
    }
    bad = bi != 0;
    return s2;
}

// Tile kernel of the split form (BF16, K steps <= kStripeKSteps, sides <=
// 1024): one workgroup per pair, the same pair <-> slot mapping as
// doc_pair_kernel.  Supplier norms (16 lanes per row), the stripes tile with
// the consumers' norms and the first round's search, and the finiteness of
// every coordinate, into the slot.
template <int T>
__device__ void doc_tile_pair(const DocArgs& A, int64_t p, char* __restrict__ slot, double* __restrict__ xx,
                              float* __restrict__ am, uint16_t* __restrict__ xs, Shared& sh) {
    const int tid = threadIdx.x;
    const int d = A.d;
#ifdef NNSEMD_PHASE_TILE
    NNSEMD_PH_DECL
#endif
    int64_t x0, y0, m, n;
    const int status = resolve_pair(A, p, x0, m, y0, n);
    const int mi = status == NNSEMD_OK ? (int)m : 0, ni = status == NNSEMD_OK ? (int)n : 0;
    const uint16_t* X = reinterpret_cast<const uint16_t*>(A.X) + x0 * d;
    const uint16_t* Y = reinterpret_cast<const uint16_t*>(A.Y) + y0 * d;
    char* aux = slot + doc_aux_offset(A.max_m, A.max_n);
    float* axx = reinterpret_cast<float*>(aux);
    float* ayy = axx + A.max_m;
    float* ab1 = ayy + A.max_n;
    float* ab2 = ab1 + A.max_n;
    int32_t* abs_ = reinterpret_cast<int32_t*>(ab2 + A.max_n);
    int32_t* aflag = abs_ + A.max_n;
    bool bad = false;
    for (int i = tid; i < mi; i += T) am[i] = A.a[x0 + i];
    // supplier norms from the set pass (NaN marks a non-finite row)
    const int64_t px = A.x_off != nullptr ? (A.pair_x ? (int64_t)A.pair_x[p] : p) : 0;
    for (int i = tid; i < mi; i += T) {
        const double s2 = A.xnorm[px * A.max_m + i];
        bad |= s2 != s2;
        xx[i] = s2;
        axx[i] = (float)s2;
    }
    __syncthreads();
#ifdef NNSEMD_PHASE_TILE
    NNSEMD_PH(0)
    key_tile_mfma_stripes<T>(X, Y, mi, ni, doc_tile_ld(ni), d, xx, reinterpret_cast<float*>(slot), ayy, bad, am, ab1,
                             ab2, abs_, xs,
                             ph, ph_t);
#else
    key_tile_mfma_stripes<T>(X, Y, mi, ni, doc_tile_ld(ni), d, xx, reinterpret_cast<float*>(slot), ayy, bad, am, ab1,
                             ab2, abs_, xs);
#endif
    double bd[1] = {bad ? 1.0 : 0.0};
    const int bop[1] = {2};
    block_reduce<T, 1>(bd, bop, &sh.red[0][0]);
    if (tid == 0) *aflag = bd[0] != 0.0 ? 1 : 0;
#ifdef NNSEMD_PHASE_TILE
    NNSEMD_PH(8)
    NNSEMD_PH_FLUSH(A.phase_cycles)
#endif
}

// Norm pass of the split form: every row (up to max_m) of every supplier
// set, 16 lanes per row; blockIdx.x = set * chunks + chunk.  The suppliers
// are shared by many pairs (one query against candidates), so their norms
// are taken once here instead of once per pair.
template <int T>
__global__ __launch_bounds__(T) void doc_xnorm_kernel(DocArgs A, int chunks) {
    constexpr int G = 16;
    const int64_t set = blockIdx.x / chunks;
    const int row = (int)(blockIdx.x % chunks) * (T / G) + (int)threadIdx.x / G;
    const int gl = threadIdx.x & (G - 1);
    int64_t x0 = 0, m = A.single_m;
    if (A.x_off != nullptr) {
        x0 = A.x_off[set];
        m = A.x_off[set + 1] - x0;
    }
    if (m > A.max_m) m = A.max_m;  // such pairs are rejected; their rows are not needed
    if (row >= m) return;          // whole 16-lane groups
    bool bad;
    const double s2 = row_norm_bf16<G>(reinterpret_cast<const uint16_t*>(A.X) + (x0 + row) * A.d, A.d, gl, bad);
    if (gl == 0) A.xnorm[set * A.max_m + row] = bad ? (double)NAN : s2;
}

template <int T>
__global__ __launch_bounds__(T) void doc_tile_kernel(DocArgs A) {
    extern __shared__ __align__(16) char lds_dyn[];
    __shared__ Shared sh;
    __shared__ __align__(16) uint16_t xs[32 * kStripeLdx];
    double* xx = reinterpret_cast<double*>(lds_dyn);
    float* am = reinterpret_cast<float*>(xx + A.max_m);
    const int64_t b = A.pair_base + (int64_t)blockIdx.x;
    const int64_t p = A.order != nullptr ? (int64_t)A.order[b] : b;
    char* slot = A.scratch + (size_t)blockIdx.x * (size_t)A.slot_bytes;
    doc_tile_pair<T>(A, p, slot, xx, am, xs, sh);
}

// ---- Tile pass when every pair searches the same supplier set (one query
// against many candidates).  The query's rows are staged in LDS once per
// workgroup for the whole launch, and each wavefront then computes 16-consumer
// stripes on its own, with no barrier after the staging: wavefront w of W
// takes stripes w, w + W, w + 2W, ... of the list below (the stripes of the
// largest pairs first; every stripe costs the same, 16 consumers against all
// suppliers).  A stripe computes exactly what key_tile_mfma_stripes computes
// for it: the same MFMA blocks, the same FP32 chunk sums in K order, the same
// top-2 updates in ascending supplier order and the same merge, so the tiles
// and the first round's results are bit-identical to the per-pair tile pass.

// Stripe list of one launch: one 16-byte record per pair of 16-consumer
// stripes, (local pair position << 6 | stripe pair, consumers of the pair or
// -1 for a pair that fails its checks, first consumer row as int64); n <=
// 1024 per side so a pair has at most 32 records, and every pair gets at
// least one (its first record also writes the pair's supplier norms).  The
// order of the list does not matter (every record is nearly the same work:
// 32 consumers against all suppliers).  The list kernel also clears each
// pair's non-finite flag, which the stripes raise with atomic ORs.
constexpr int kStripeShift = 6;
constexpr int kSharedTileThreads = 768;  // 12 wavefronts: up to 170 VGPRs each

__device__ inline int32_t* doc_aux_flag(const DocArgs& A, char* slot) {
    char* aux = slot + doc_aux_offset(A.max_m, A.max_n);
    return reinterpret_cast<int32_t*>(reinterpret_cast<float*>(aux) + A.max_m + 3 * (size_t)A.max_n) + A.max_n;
}

__global__ void doc_stripe_reset_kernel(DocArgs A) {
    if (threadIdx.x == 0) *A.stripe_total = 0;
}

// One thread per pair: its stripe count, a workgroup scan, one atomic for the
// workgroup's place in the list (list order is free), then the records.
template <int T>
__global__ __launch_bounds__(T) void doc_stripe_list_kernel(DocArgs A, int npairs) {
    __shared__ int wsum[T / 64];
    __shared__ int base;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid / 64;
    const int b = (int)blockIdx.x * T + tid;
    int n = 0;
    int64_t y0 = 0;
    if (b < npairs) {
        const int64_t q = A.pair_base + b;
        const int64_t p = A.order != nullptr ? (int64_t)A.order[q] : q;
        int64_t x0, m, nn;
        const int status = resolve_pair(A, p, x0, m, y0, nn);
        n = status == NNSEMD_OK ? (int)nn : -1;
    }
    const int k = b < npairs ? (n > 0 ? (n + 31) / 32 : 1) : 0;
    int v = k;  // inclusive scan over the wavefront
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int w = __shfl_up(v, o);
        if (lane >= o) v += w;
    }
    if (lane == 63) wsum[wave] = v;
    __syncthreads();
    if (tid == 0) {
        int tot = 0;
        for (int w = 0; w < T / 64; ++w) tot += wsum[w];
        base = atomicAdd(A.stripe_total, tot);
    }
    __syncthreads();
    int off = base + v - k;
    for (int w = 0; w < wave; ++w) off += wsum[w];
    for (int s = 0; s < k; ++s)
        A.stripes[off + s] = make_int4((b << kStripeShift) | s, n, (int)(uint32_t)(uint64_t)y0,
                                       (int)(uint32_t)((uint64_t)y0 >> 32));
    if (b < npairs) *doc_aux_flag(A, A.scratch + (size_t)b * (size_t)A.slot_bytes) = 0;
}

// LDS of doc_tile_shared_kernel: the query rows (zero-padded to whole
// 32-row blocks and K steps), their FP64 norms and their masses.
__host__ __device__ inline size_t doc_shared_rows(int max_m) { return (size_t)((max_m + 31) & ~31); }
__host__ __device__ inline size_t doc_shared_lds(int max_m) {
    return doc_shared_rows(max_m) * (sizeof(uint16_t) * kStripeLdx + sizeof(double) + sizeof(float));
}

// Record s of a pair: its stripes 2 s and 2 s + 1, the consumers
// 32 s .. 32 s + 31 of the pair's consumer set.
struct StripeRec {
    int b, s, n;       // local pair position, stripe pair, consumers (-1: the pair failed its checks)
    const uint16_t* Y;  // the pair's first consumer row
};

__device__ inline StripeRec stripe_rec(const DocArgs& A, int t, int total) {
    StripeRec r{0, 0, 0, nullptr};
    if (t < total) {
        // the list from its end: the pairs scheduled first have their tiles
        // written last, so the rounds kernel finds more of them in the caches
        const int4 e = A.stripes[total - 1 - t];
        r.b = e.x >> kStripeShift;
        r.s = e.x & ((1 << kStripeShift) - 1);
        r.n = e.y;
        const int64_t y0 = (int64_t)(((uint64_t)(uint32_t)e.w << 32) | (uint64_t)(uint32_t)e.z);
        r.Y = reinterpret_cast<const uint16_t*>(A.Y) + y0 * A.d;
    }
    return r;
}

template <int T>
__global__ __launch_bounds__(T) void doc_tile_shared_kernel(DocArgs A) {
    constexpr int KS = kStripeKSteps;
    extern __shared__ __align__(16) char lds_dyn[];
    const int mrows = (int)doc_shared_rows(A.max_m);
    uint16_t* xs = reinterpret_cast<uint16_t*>(lds_dyn);
    double* xx = reinterpret_cast<double*>(lds_dyn + sizeof(uint16_t) * kStripeLdx * (size_t)mrows);
    float* am = reinterpret_cast<float*>(xx + mrows);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int d = A.d;
    const int ksteps = (d + 31) / 32;
    const int kp = ksteps * 32;
    const int64_t qx0 = A.x_off != nullptr ? A.x_off[0] : 0;
    const int mq = (int)min<int64_t>(A.x_off != nullptr ? A.x_off[1] - qx0 : A.single_m, (int64_t)A.max_m);
    const uint16_t* Xq = reinterpret_cast<const uint16_t*>(A.X) + qx0 * d;
    // ---- stage the query once (rows >= mq and columns >= d are zero)
    const bool rows8 = (d & 3) == 0 && (reinterpret_cast<uintptr_t>(Xq) & 7u) == 0;
    for (int e = tid; e < mrows * (kp / 4); e += T) {
        const int r = e / (kp / 4), k = 4 * (e % (kp / 4));
        uint2 v = make_uint2(0u, 0u);
        if (r < mq && k < d) {
            if (rows8) {
                v = *reinterpret_cast<const uint2*>(Xq + (size_t)r * d + k);
            } else {
                uint16_t h[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) h[u] = k + u < d ? Xq[(size_t)r * d + k + u] : (uint16_t)0;
                v = make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16));
            }
        }
        *reinterpret_cast<uint2*>(&xs[r * kStripeLdx + k]) = v;
    }
    for (int i = tid; i < mrows; i += T) {
        xx[i] = i < mq ? A.xnorm[i] : 0.0;
        am[i] = i < mq ? A.a[qx0 + i] : 0.f;
    }
    __syncthreads();  // the only barrier: every thread reaches it once

    const int r16 = lane & 15, kq = 8 * (lane >> 4);
    const int W = (int)gridDim.x * (T / 64);
    const int total = *A.stripe_total;
    // A record covers the stripes 2 sp and 2 sp + 1 of a pair (consumers
    // 32 sp .. 32 sp + 31): both take the same supplier fragments from LDS,
    // and their 64-byte row segments are the two halves of one 128-byte
    // block.  A second stripe beyond the pair's consumers multiplies zero
    // fragments and stores nothing.
    auto load_frags = [&](const StripeRec& r, int h, bf16x8 (&yb)[KS]) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
            if (ks < ksteps) yb[ks] = frag8(r.Y, r.s * 32 + 16 * h + r16, max(r.n, 0), ks * 32 + kq, d);
    };
    auto norm_of = [&](const bf16x8 (&yb)[KS], bool& bad) {
        double ss = 0.0;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            if (ks < ksteps) {
                union {
                    bf16x8 v;
                    uint32_t w[4];
                } u;
                u.v = yb[ks];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    bad |= !finite_pair(u.w[e]);
                    const double f0 = bf_lo(u.w[e]), f1 = bf_hi(u.w[e]);
                    ss = fma(f0, f0, ss);
                    ss = fma(f1, f1, ss);
                }
            }
        }
        ss += __shfl_xor(ss, 16);
        ss += __shfl_xor(ss, 32);
        return ss;
    };
    // The record of the stripe pair after next is loaded while this one
    // multiplies.
    int t = (int)blockIdx.x * (T / 64) + tid / 64;
    StripeRec cur = stripe_rec(A, t, total);
    StripeRec nxt = stripe_rec(A, t + W, total);
    for (; t < total; t += W) {
        const StripeRec nn = stripe_rec(A, t + 2 * W, total);
        const int mi = cur.n >= 0 ? mq : 0, ni = max(cur.n, 0);
        char* slot = A.scratch + (size_t)cur.b * (size_t)A.slot_bytes;
        char* aux = slot + doc_aux_offset(A.max_m, A.max_n);
        float* axx = reinterpret_cast<float*>(aux);
        float* ayy = axx + A.max_m;
        float* ab1 = ayy + A.max_n;
        float* ab2 = ab1 + A.max_n;
        int32_t* abs_ = reinterpret_cast<int32_t*>(ab2 + A.max_n);
        float* tile = reinterpret_cast<float*>(slot);
        bool bad = false;
        if (cur.s == 0) {
            for (int i = lane; i < mi; i += 64) {
                const double s2 = xx[i];
                bad |= s2 != s2;
                axx[i] = (float)s2;
            }
        }
        const int j0 = cur.s * 32;
        if (j0 < ni) {
            bf16x8 ya[KS], yb[KS];
            load_frags(cur, 0, ya);
            load_frags(cur, 1, yb);
            const double ssa = norm_of(ya, bad), ssb = norm_of(yb, bad);
            if (lane < 16 && j0 + r16 < ni) ayy[j0 + r16] = (float)ssa;
            if (lane < 16 && j0 + 16 + r16 < ni) ayy[j0 + 16 + r16] = (float)ssb;
            StripeTop ta, tb;
            stripe_top_init(ta);
            stripe_top_init(tb);
            const int jg = j0 + 4 * (lane >> 4);
            const int ldt = doc_tile_ld(ni);
            const f32x4 zero = (f32x4){0.f, 0.f, 0.f, 0.f};
            for (int i0 = 0; i0 < mi; i0 += 32) {
                float a0[4] = {0.f, 0.f, 0.f, 0.f}, a1[4] = {0.f, 0.f, 0.f, 0.f};
                float b0[4] = {0.f, 0.f, 0.f, 0.f}, b1[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    if (ks < ksteps) {
                        union {
                            uint4 u;
                            bf16x8 v;
                        } f0, f1;
                        f0.u = *reinterpret_cast<const uint4*>(&xs[(i0 + r16) * kStripeLdx + ks * 32 + kq]);
                        f1.u = *reinterpret_cast<const uint4*>(&xs[(i0 + 16 + r16) * kStripeLdx + ks * 32 + kq]);
                        const f32x4 ca0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ya[ks], f0.v, zero, 0, 0, 0);
                        const f32x4 ca1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ya[ks], f1.v, zero, 0, 0, 0);
                        const f32x4 cb0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yb[ks], f0.v, zero, 0, 0, 0);
                        const f32x4 cb1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yb[ks], f1.v, zero, 0, 0, 0);
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            a0[r] += ca0[r];
                            a1[r] += ca1[r];
                            b0[r] += cb0[r];
                            b1[r] += cb1[r];
                        }
                    }
                }
                stripe_block_epilogue(a0, a1, i0, mi, jg, ni, ldt, xx, am, tile, ta);
                stripe_block_epilogue(b0, b1, i0, mi, jg + 16, ni, ldt, xx, am, tile, tb);
            }
            stripe_top_finish(ta, jg, ni, ab1, ab2, abs_);
            stripe_top_finish(tb, jg + 16, ni, ab1, ab2, abs_);
        }
        if (__ballot(bad) != 0 && lane == 0) atomicOr(doc_aux_flag(A, slot), 1);
        cur = nxt;
        nxt = nn;
    }
}

// The split form runs at five wavefronts per SIMD (94 VGPRs, no spills; at
// six the 80-VGPR limit spills 30 registers, whose scratch traffic costs as
// much as the extra wavefront gains).  Its compact LDS layout (16-bit
// indices) fits five 162 x 500 pairs per CU.
template <typename TIn, bool MFMA, int T, int CSMAX, bool SPLIT>
__global__ __launch_bounds__(T, SPLIT ? 5 : 1) void doc_pair_kernel(DocArgs A) {
    extern __shared__ __align__(16) char lds_dyn[];
    __shared__ Shared sh;
    __shared__ int kloose;  // split form: a served distance needs its exact FP64 value
    const PairLdsLayout lay = pair_lds_layout(A.max_m, A.max_n, 0, 0, true, false);
    const Lds16 L = carve16(lds_dyn, A.max_m, A.max_n, 0, 0, false);
    float* xx = reinterpret_cast<float*>(lds_dyn + lay.total);
    float* yy = xx + A.max_m;
    float* yn = yy + A.max_n;
    float* kap = yn + A.max_n;
    int32_t* amb = reinterpret_cast<int32_t*>(kap + A.max_n);
    // FP32 vector tile: its LDS staging panels after the pair's arrays
    float* vstage = reinterpret_cast<float*>(align_up(reinterpret_cast<uintptr_t>(amb + A.max_n), 16));
    const int64_t b = A.pair_base + (int64_t)blockIdx.x;
    const int64_t p = A.order != nullptr ? (int64_t)A.order[b] : b;
    char* slot = A.scratch + (size_t)blockIdx.x * (size_t)A.slot_bytes;
    solve_doc_pair<TIn, MFMA, T, CSMAX, SPLIT>(A, p, slot, L, xx, yy, yn, kap, amb, sh, kloose, vstage);
}

template <typename TIn, bool MFMA, int CSMAX, bool SPLIT>
int doc_launch_typed(const DocArgs& A, size_t lds, int grid, hipStream_t st, bool run, int* blocks) {
    auto k = doc_pair_kernel<TIn, MFMA, 256, CSMAX, SPLIT>;
    if (lds > 48 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return (int)e;
    }
    if (!run) return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k, 256, lds);
    if constexpr (SPLIT) {
        if (A.stripes != nullptr) {
            // the records' pair positions and stripe-pair numbers must fit
            // their packed fields (the split form caps each side at 1024)
            if ((A.max_n + 31) / 32 > (1 << kStripeShift) || grid > (1 << (31 - kStripeShift)) ||
                A.tile_grid < 1)
                return (int)hipErrorInvalidValue;
            hipLaunchKernelGGL(doc_stripe_reset_kernel, dim3(1), dim3(64), 0, st, A);
            hipLaunchKernelGGL(doc_stripe_list_kernel<256>, dim3((grid + 255) / 256), dim3(256), 0, st, A, grid);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return (int)e;
            const size_t tl = doc_shared_lds(A.max_m);
            e = hipFuncSetAttribute((const void*)doc_tile_shared_kernel<kSharedTileThreads>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)tl);
            if (e != hipSuccess) return (int)e;
            hipLaunchKernelGGL(doc_tile_shared_kernel<kSharedTileThreads>, dim3(A.tile_grid), dim3(kSharedTileThreads),
                               tl, st, A);
        } else {
            const size_t tl = (sizeof(double) + sizeof(float)) * (size_t)A.max_m;
            hipLaunchKernelGGL(doc_tile_kernel<256>, dim3(grid), dim3(256), tl, st, A);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return (int)e;
    }
    hipLaunchKernelGGL(k, dim3(grid), dim3(256), lds, st, A);
    return (int)hipGetLastError();
}


}  // namespace

// Compact pair layout (16-bit indices, no records, its own serve-order
// array) + xx[M], yy[N], yn[N], kap[N] (float), amb[N] (int32), and for FP32
// points the staging panels of the vector tile (16-byte aligned).
size_t doc_lds_bytes(int max_m, int max_n, bool fp32_points) {
    return pair_lds_layout(max_m, max_n, 0, 0, true, false).total +
           sizeof(float) * ((size_t)max_m + 4 * (size_t)max_n) + (fp32_points ? kValuStageBytes + 16 : 0);
}

size_t doc_shared_tile_lds(int max_m) { return doc_shared_lds(max_m); }

int doc_shared_tile_threads() { return kSharedTileThreads; }

int doc_shared_tile_occupancy(int max_m) {
    const size_t tl = doc_shared_lds(max_m);
    const void* k = (const void*)doc_tile_shared_kernel<kSharedTileThreads>;
    if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)tl) != hipSuccess) return 0;
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, doc_tile_shared_kernel<kSharedTileThreads>,
                                                     kSharedTileThreads, tl) != hipSuccess)
        return 0;
    return blocks;
}

bool doc_split_form(int d, bool bf16_mfma, int chunk_max) {
    return bf16_mfma && chunk_max <= 4 && (d + 31) / 32 <= kStripeKSteps;
}

int launch_doc_xnorm(const DocArgs& A, void* stream) {
    constexpr int T = 256;
    const int chunks = (A.max_m + T / 16 - 1) / (T / 16);
    const int64_t sets = A.x_off != nullptr ? A.num_x_sets : 1;
    const int64_t grid = sets * chunks;
    if (grid <= 0) return 0;
    if (grid > 0x7fffffffll) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(doc_xnorm_kernel<T>, dim3((unsigned)grid), dim3(T), 0, (hipStream_t)stream, A, chunks);
    return (int)hipGetLastError();
}

int launch_doc_solver(const DocArgs& A, bool bf16_mfma, int chunk_max, size_t lds, int grid, void* stream,
                      int* blocks, bool allow_split) {
    const bool run = blocks == nullptr;
    hipStream_t st = (hipStream_t)stream;
    const bool split = allow_split && doc_split_form(A.d, bf16_mfma, chunk_max);
    if (bf16_mfma) {
        if (chunk_max <= 4 && split) return doc_launch_typed<uint16_t, true, 4, true>(A, lds, grid, st, run, blocks);
        if (chunk_max <= 4) return doc_launch_typed<uint16_t, true, 4, false>(A, lds, grid, st, run, blocks);
        if (chunk_max <= 16) return doc_launch_typed<uint16_t, true, 16, false>(A, lds, grid, st, run, blocks);
    } else {
        if (chunk_max <= 4) return doc_launch_typed<float, false, 4, false>(A, lds, grid, st, run, blocks);
        if (chunk_max <= 16) return doc_launch_typed<float, false, 16, false>(A, lds, grid, st, run, blocks);
    }
    return (int)hipErrorInvalidValue;
}

}  // namespace nnsemd
