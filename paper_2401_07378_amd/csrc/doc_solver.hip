// NNS-EMD for high-dimensional point sets (word-embedding documents): one
// workgroup per pair, the distance keys of the whole pair computed once.
//
// Keys: key(i, j) = ||x_i||^2 - 2 x_i . y_j (the consumer's ||y_j||^2 is the
// same for every supplier and drops out of the search).  With BF16 inputs the
// m x n dot products run on the matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulation; each wavefront computes 32 x 32 output tiles from 2 x 2
// MFMA blocks); with FP32 inputs they run on the vector ALUs.  The tile goes
// to a per-workgroup global scratch area (it stays in L2 / MALL while the
// workgroup runs its rounds).
//
// Exactness: an FP32 key differs from the exact one by at most
// E = 2 (d + 1) u (||x|| + ||y||)^2 (u = 2^-24) for any accumulation order of
// the d products, even if every addition rounded with error 2u; a consumer
// whose best and second-best keys are closer than 4E (twice the worst
// disagreement of two keys, with R = max ||x|| in place of ||x||) is re-scored
// over all active suppliers in FP64 from the inputs, in the definition's
// operation order.  Every pick is then
// the exact argmin (ties to the smallest index) and carries its exact FP64
// key, so the plan equals the FP64 definition's.  After the search the
// round continues with the phases shared with the point path.
#ifndef NNSEMD_CPU_EMULATION
#include <hip/hip_runtime.h>
#endif
#include <math.h>
#include <stdint.h>

#include "internal.hpp"
#include "round_common.hpp"

namespace nnsemd {
namespace {

using namespace rc;

#ifndef NNSEMD_CPU_EMULATION
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
#else
typedef emu_bf16x8 bf16x8;
typedef emu_f32x4 f32x4;
#endif

__device__ inline float to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ inline float to_f32(float v) { return v; }
__device__ inline bool finite_in(uint16_t b) { return (b & 0x7F80u) != 0x7F80u; }
__device__ inline bool finite_in(float v) { return isfinite(v); }

__device__ inline float bf_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ inline float bf_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

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

// 8 consecutive BF16 values of row r starting at column k0 (zeros beyond d
// or for rows >= rows), as an MFMA fragment.
__device__ inline bf16x8 frag8(const uint16_t* __restrict__ base, int r, int rows, int k0, int d) {
    union {
        uint32_t w[4];
        bf16x8 v;
    } u;
    if (r < rows && k0 + 8 <= d) {
        const uint32_t* p = reinterpret_cast<const uint32_t*>(base + (size_t)r * d + k0);
        if (((uintptr_t)p & 3u) == 0) {
            u.w[0] = p[0];
            u.w[1] = p[1];
            u.w[2] = p[2];
            u.w[3] = p[3];
            return u.v;
        }
    }
    uint16_t h[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) h[e] = (r < rows && k0 + e < d) ? base[(size_t)r * d + k0 + e] : (uint16_t)0;
#pragma unroll
    for (int e = 0; e < 4; ++e) u.w[e] = (uint32_t)h[2 * e] | ((uint32_t)h[2 * e + 1] << 16);
    return u.v;
}

// Key tile with matrix cores: each wavefront owns 32 x 32 output tiles.
// MFMA 16x16x32 lane layout (checked on gfx950): A lane l holds row l%16,
// k = 8(l/16)..+8; B lane l holds column l%16, the same k; C lane l
// register r is row 4(l/16)+r, column l%16.
template <int T>
__device__ void key_tile_mfma(const uint16_t* __restrict__ X, const uint16_t* __restrict__ Y, int m, int n, int d,
                              const float* __restrict__ xx, float* __restrict__ tile) {
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
        for (int ks = 0; ks < ksteps; ++ks) {
            const int k0 = ks * 32 + kq;
            const bf16x8 a0 = frag8(X, i0 + r16, m, k0, d);
            const bf16x8 a1 = frag8(X, i0 + 16 + r16, m, k0, d);
            const bf16x8 b0 = frag8(Y, j0 + r16, n, k0, d);
            const bf16x8 b1 = frag8(Y, j0 + 16 + r16, n, k0, d);
            acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[1][1], 0, 0, 0);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = i0 + 16 * a + 4 * (lane >> 4) + r;
                    const int j = j0 + 16 * b + r16;
                    if (i < m && j < n) tile[(size_t)i * n + j] = xx[i] - 2.f * acc[a][b][r];
                }
    }
}

// Key tile on the vector ALUs (FP32 inputs): each lane owns a 4 x 4 block
// of (i, j) and walks the d products with 16-byte loads when rows allow it.
template <int T>
__device__ void key_tile_valu(const float* __restrict__ X, const float* __restrict__ Y, int m, int n, int d,
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
                if (i0 + u < m && j0 + v < n) tile[(size_t)(i0 + u) * n + j0 + v] = xx[i0 + u] - 2.f * acc[u][v];
    }
}

template <typename TIn, bool MFMA, int T, int CSMAX>
__device__ void solve_doc_pair(const DocArgs& A, int64_t p, float* __restrict__ tile, const Lds& L,
                               float* __restrict__ xx, float* __restrict__ yn, Shared& sh) {
    constexpr int NW = T / 64;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid / 64;
    const int d = A.d;

    int64_t x0 = 0, y0 = 0, m = A.single_m, n = A.single_n;
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
    const TIn* __restrict__ X = reinterpret_cast<const TIn*>(A.X) + x0 * d;
    const TIn* __restrict__ Y = reinterpret_cast<const TIn*>(A.Y) + y0 * d;
    const int mi = (int)m, ni = (int)n;

    // ---- ingest: masses, validity, norms
    double red[4] = {0.0, 0.0, 0.0, 0.0};  // sum a, sum b, bad, max ||x||^2
    const int rop[4] = {0, 0, 2, 2};
    for (int i = tid; i < mi; i += T) {
        const float av = A.a[x0 + i];
        if (!(av >= 0.f) || !isfinite(av)) red[2] = 1.0;
        L.smass[i] = (double)av;
        red[0] += (double)av;
        float s2 = 0.f;
        for (int k = 0; k < d; ++k) {
            const TIn v = X[(size_t)i * d + k];
            if (!finite_in(v)) red[2] = 1.0;
            const float f = to_f32(v);
            s2 = fmaf(f, f, s2);
        }
        xx[i] = s2;
        red[3] = fmax(red[3], (double)s2);
    }
    for (int j = tid; j < ni; j += T) {
        const float bv = A.b[y0 + j];
        if (!(bv >= 0.f) || !isfinite(bv)) red[2] = 1.0;
        L.cmass[j] = (double)bv;
        red[1] += (double)bv;
        float s2 = 0.f;
        for (int k = 0; k < d; ++k) {
            const TIn v = Y[(size_t)j * d + k];
            if (!finite_in(v)) red[2] = 1.0;
            const float f = to_f32(v);
            s2 = fmaf(f, f, s2);
        }
        yn[j] = sqrtf(s2);
    }
    block_reduce<T, 4>(red, rop, sh);
    if (status == NNSEMD_OK && red[2] != 0.0) status = NNSEMD_ERR_INVALID_ARG;
    if (status == NNSEMD_OK) {
        const double big = fmax(red[0], red[1]);
        if (fabs(red[0] - red[1]) > 1e-5 * big) status = NNSEMD_ERR_MASS_MISMATCH;
    }
    // R >= max ||x|| despite the FP32 norms' own rounding; gap threshold
    // 8 (d + 2) u (R + ||y||)^2.
    const float rhat = sqrtf((float)red[3]) * (1.f + (float)(d + 2) * kU32);
    const float thr_scale = 8.f * (float)(d + 2) * kU32;

    // ---- key tile
    if (status == NNSEMD_OK) {
        if constexpr (MFMA)
            key_tile_mfma<T>(reinterpret_cast<const uint16_t*>(X), reinterpret_cast<const uint16_t*>(Y), mi, ni, d, xx,
                             tile);
        else
            key_tile_valu<T>(reinterpret_cast<const float*>(X), reinterpret_cast<const float*>(Y), mi, ni, d, xx,
                             tile);
    }
    __syncthreads();

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
    int64_t work = 0, nnz = 0, near = 0;
    double cost = 0.0;
    float* flag_b1 = reinterpret_cast<float*>(L.sorted);  // best FP32 key of each flagged consumer
    while (status == NNSEMD_OK && mact > 0 && nact > 0) {
        if (rounds >= max_rounds) {
            status = NNSEMD_ERR_NOT_CONVERGED;
            break;
        }
        work += (int64_t)mact * nact;
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
            constexpr int U = 8;
            const int stride = S * U;
            const int full = (mact / stride) * stride;
            for (int s0 = r; s0 < full; s0 += stride) {
                float kk[U];
#pragma unroll
                for (int u = 0; u < U; ++u) kk[u] = tile[(size_t)L.sidx[s0 + u * S] * ni + j];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const bool lt = kk[u] < b1;
                    bs = lt ? s0 + u * S : bs;
                    b2 = __builtin_amdgcn_fmed3f(b1, kk[u], b2);
                    b1 = fminf(b1, kk[u]);
                }
            }
            for (int s = full + r; s < mact; s += S) {
                const float k = tile[(size_t)L.sidx[s] * ni + j];
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
                const float thr = thr_scale * e * e + 1e-30f;
                if (!(b2 - b1 > thr)) {
                    const int f = atomicAdd(&sh.nflag, 1);
                    L.list[f] = j;
                    flag_b1[f] = b1;
                    L.ckey[j] = 0.0;  // set by the re-scoring wave; skipped by the pass below
                } else {
                    L.cnn[j] = bs;
                    L.ckey[j] = -1.0;  // exact key computed below
                    atomicAdd(&L.scnt[bs], 1);
                }
            }
        }
        __syncthreads();
        const int nf = sh.nflag;
        if (nf > 0) {
            // Near ties: the FP64 argmin is among the suppliers whose FP32
            // key is within the threshold of the best one; only those are
            // re-scored.
            for (int f = wave; f < nf; f += NW) {
                const int j = L.list[f];
                const float e = rhat + yn[j];
                const float lim = flag_b1[f] + (thr_scale * e * e + 1e-30f);
                double best = INFINITY;
                int bsl = 0x7fffffff;
                for (int s = lane; s < mact; s += 64) {
                    const int i = L.sidx[s];
                    if (tile[(size_t)i * ni + j] > lim) continue;
                    const double k = dkey64<TIn>(X + (size_t)i * d, Y + (size_t)j * d, d);
                    if (k < best) {
                        best = k;
                        bsl = s;
                    }
                }
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    const double cb = __shfl_xor(best, o);
                    const int cs2 = __shfl_xor(bsl, o);
                    if (cb < best || (cb == best && cs2 < bsl)) {
                        best = cb;
                        bsl = cs2;
                    }
                }
                if (lane == 0) {
                    L.cnn[j] = bsl;
                    L.ckey[j] = best;
                    atomicAdd(&L.scnt[bsl], 1);
                }
            }
            near += nf;
        }
        // Exact FP64 key of every other pick (for the serve order and R).
        for (int q = tid; q < nact; q += T) {
            const int j = L.cact[q];
            if (L.ckey[j] < 0.0) L.ckey[j] = dkey64<TIn>(X + (size_t)L.sidx[L.cnn[j]] * d, Y + (size_t)j * d, d);
        }
        __syncthreads();
        round_buckets<T>(L, sh, mact, nact);
        round_rank<T>(L, nact, A.protocol, A.seed, rounds);
        round_walk<T>(L, mact, A.metric, cost);
        round_compact<T, CSMAX, 0>(L, sh, mact, nact, nnz, want_plan ? A.plan_src : nullptr, A.plan_dst,
                                   A.plan_flow, plan_base);
        ++rounds;
    }

    double fin[3] = {cost, 0.0, 0.0};
    const int fop[3] = {0, 0, 0};
    if (status == NNSEMD_OK || status == NNSEMD_ERR_NOT_CONVERGED) {
        for (int s = tid; s < mact; s += T) fin[1] += L.smass[s];
        for (int q = tid; q < nact; q += T) fin[2] += L.cmass[L.cact[q]];
    }
    block_reduce<T, 3>(fin, fop, sh);
    if (tid == 0) {
        A.costs[p] = status == NNSEMD_OK ? fin[0] : NAN;
        if (A.stats != nullptr) {
            nnsemd_stats_t st;
            st.status = status;
            st.rounds = rounds;
            st.nnz = nnz;
            st.work = work;
            st.near_ties = near;
            st.residual_src = fin[1];
            st.residual_dst = fin[2];
            A.stats[p] = st;
        }
    }
}

#ifndef NNSEMD_CPU_EMULATION
template <typename TIn, bool MFMA, int T, int CSMAX>
__global__ __launch_bounds__(T) void doc_pair_kernel(DocArgs A) {
    extern __shared__ __align__(16) char lds_dyn[];
    __shared__ Shared sh;
    const PairLdsLayout lay = pair_lds_layout(A.max_m, A.max_n, 0);
    const Lds L = carve(lds_dyn, A.max_m, A.max_n, 0);
    float* xx = reinterpret_cast<float*>(lds_dyn + lay.total);
    float* yn = xx + A.max_m;
    const int64_t b = A.pair_base + (int64_t)blockIdx.x;
    const int64_t p = A.order != nullptr ? (int64_t)A.order[b] : b;
    float* tile = A.tiles + (size_t)blockIdx.x * (size_t)A.tile_stride;
    solve_doc_pair<TIn, MFMA, T, CSMAX>(A, p, tile, L, xx, yn, sh);
}

template <typename TIn, bool MFMA, int CSMAX>
int doc_launch_typed(const DocArgs& A, size_t lds, int grid, hipStream_t st, bool run, int* blocks) {
    auto k = doc_pair_kernel<TIn, MFMA, 256, CSMAX>;
    if (lds > 48 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return (int)e;
    }
    if (!run) return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k, 256, lds);
    hipLaunchKernelGGL(k, dim3(grid), dim3(256), lds, st, A);
    return (int)hipGetLastError();
}

#endif  // NNSEMD_CPU_EMULATION

}  // namespace

size_t doc_lds_bytes(int max_m, int max_n) {
    return pair_lds_layout(max_m, max_n, 0).total + sizeof(float) * ((size_t)max_m + (size_t)max_n);
}

#ifndef NNSEMD_CPU_EMULATION
int launch_doc_solver(const DocArgs& A, bool bf16_mfma, int chunk_max, size_t lds, int grid, void* stream,
                      int* blocks) {
    const bool run = blocks == nullptr;
    hipStream_t st = (hipStream_t)stream;
    if (bf16_mfma) {
        if (chunk_max <= 4) return doc_launch_typed<uint16_t, true, 4>(A, lds, grid, st, run, blocks);
        if (chunk_max <= 16) return doc_launch_typed<uint16_t, true, 16>(A, lds, grid, st, run, blocks);
    } else {
        if (chunk_max <= 4) return doc_launch_typed<float, false, 4>(A, lds, grid, st, run, blocks);
        if (chunk_max <= 16) return doc_launch_typed<float, false, 16>(A, lds, grid, st, run, blocks);
    }
    return (int)hipErrorInvalidValue;
}
#endif  // NNSEMD_CPU_EMULATION

}  // namespace nnsemd
