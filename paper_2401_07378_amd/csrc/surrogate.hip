// Deep-sets EMD surrogate: kernels and their host launchers.
//
// The surrogate is a learned pre-filter for retrieval (not part of the
// paper, whose method it serves): NNS-EMD re-ranks what it keeps.
//   phi(x)  = relu(W2 relu(W1 x + b1) + b2)          per point, 3 -> 256 -> 256
//   E(X, a) = sum_i a_i phi(x_i)                      mass-weighted pooling
//   z       = [E_q, E_c, |E_q - E_c|]                 768
//   pred    = softplus(w4 . relu(W3 z + b3) + b4)
//   loss    = mean_b (log pred_b - log y_b)^2
// Weights are used rounded to BF16 (FP32 master copies are optimised); the
// operands of the matrix-core products (layer-1 activations, pair features,
// back-propagated layer-2 and head gradients) are BF16; accumulation, biases,
// activations, pooling and the optimiser are FP32.
//
// Kernels: a generic BF16 "NT" GEMM on v_mfma_f32_16x16x32_bf16 (C = A B^T,
// both operands K-contiguous, optional split-K), a fused phi + pooling
// kernel for inference (one workgroup per set, no workspace), unfused layer
// kernels for training, LDS transposes, deterministic column sums, Adam, and
// a radix top-k.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "internal.hpp"

namespace nnsemd {
namespace sg {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int H = kSgHidden;

__device__ inline uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ inline float bfround(float f) { return bf2f(f2bf(f)); }

__device__ inline float softplusf(float t) { return t > 20.f ? t : log1pf(expf(t)); }
// ReLU that keeps NaN (fmaxf would return 0 for it).
__device__ inline float relu_nan(float v) { return v != v ? v : fmaxf(v, 0.f); }
__device__ inline float sigmoidf(float t) { return 1.f / (1.f + expf(-t)); }

// 16-byte fragment of 8 consecutive BF16 values (zeros outside the matrix).
__device__ inline bf16x8 frag16(const uint16_t* __restrict__ base, int64_t ld, int r, int rows, int k) {
    union {
        uint4 q;
        bf16x8 v;
    } u;
    if (r < rows) {
        u.q = *reinterpret_cast<const uint4*>(base + (int64_t)r * ld + k);
    } else {
        u.q = make_uint4(0u, 0u, 0u, 0u);
    }
    return u.v;
}

// ---------------------------------------------------------------- weights
__global__ void prepare_kernel(const float* __restrict__ theta, SgQuant q) {
    const int64_t n = (int64_t)H * H + (int64_t)H * 3 * H + H * 3 + H;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        if (e < (int64_t)H * H) {
            const int o = (int)(e / H), i = (int)(e % H);
            const uint16_t b = f2bf(theta[kSgW2 + e]);
            q.W2[(int64_t)o * H + i] = b;
            q.W2T[(int64_t)i * H + o] = b;
            continue;
        }
        int64_t f = e - (int64_t)H * H;
        if (f < (int64_t)H * 3 * H) {
            const int o = (int)(f / (3 * H)), i = (int)(f % (3 * H));
            const uint16_t b = f2bf(theta[kSgW3 + f]);
            q.W3[(int64_t)o * 3 * H + i] = b;
            q.W3T[(int64_t)i * H + o] = b;
            continue;
        }
        f -= (int64_t)H * 3 * H;
        if (f < H * 3) {
            q.W1[f] = bfround(theta[kSgW1 + f]);
            continue;
        }
        f -= H * 3;
        q.w4[f] = bfround(theta[kSgW4 + f]);
    }
}

// ---------------------------------------------------------------- GEMM
// C[M x N] (+ split z * c_split) = A[M x K] B[N x K]^T over K range of split z.
// Workgroup tile 64 x 64, four wavefronts of 32 x 32 (2 x 2 MFMA blocks).
// Requires lda, ldb multiples of 8, K multiple of 32, 16-byte aligned bases.
__global__ __launch_bounds__(256) void gemm_nt_kernel(const uint16_t* __restrict__ A, int64_t lda,
                                                      const uint16_t* __restrict__ B, int64_t ldb,
                                                      float* __restrict__ C, int64_t ldc, int M, int N, int K,
                                                      int kchunk, int64_t c_split) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int m0 = blockIdx.x * 64 + (wave >> 1) * 32;
    const int n0 = blockIdx.y * 64 + (wave & 1) * 32;
    const int kb = blockIdx.z * kchunk;
    const int ke = min(K, kb + kchunk);
    const int r16 = lane & 15, kq = 8 * (lane >> 4);
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
    if (kb < ke) {
        bf16x8 a0 = frag16(A, lda, m0 + r16, M, kb + kq);
        bf16x8 a1 = frag16(A, lda, m0 + 16 + r16, M, kb + kq);
        bf16x8 b0 = frag16(B, ldb, n0 + r16, N, kb + kq);
        bf16x8 b1 = frag16(B, ldb, n0 + 16 + r16, N, kb + kq);
        for (int k = kb; k < ke; k += 32) {
            bf16x8 na0 = a0, na1 = a1, nb0 = b0, nb1 = b1;
            if (k + 32 < ke) {
                na0 = frag16(A, lda, m0 + r16, M, k + 32 + kq);
                na1 = frag16(A, lda, m0 + 16 + r16, M, k + 32 + kq);
                nb0 = frag16(B, ldb, n0 + r16, N, k + 32 + kq);
                nb1 = frag16(B, ldb, n0 + 16 + r16, N, k + 32 + kq);
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
    }
    float* Cz = C + (int64_t)blockIdx.z * c_split;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = m0 + 16 * a + 4 * (lane >> 4) + r;
                const int j = n0 + 16 * b + r16;
                if (i < M && j < N) Cz[(int64_t)i * ldc + j] = acc[a][b][r];
            }
}

// out[i] = sum_z parts[z * stride + i], z ascending.
__global__ void sum_splits_kernel(const float* __restrict__ parts, int splits, int64_t stride, float* __restrict__ out,
                                  int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int z = 0; z < splits; ++z) s += parts[(int64_t)z * stride + i];
        out[i] = s;
    }
}

// out[j] (+)= sum over rows r of in[r * ld + j] (j < cols): 16 row slices
// per column (rows r = slice mod 16, ascending), then the slices in order.
constexpr int kColsumThreads = 1024;
__global__ __launch_bounds__(kColsumThreads) void colsum_kernel(const float* __restrict__ in, int64_t rows, int64_t ld,
                                                                int cols, float* __restrict__ out, int accumulate) {
    __shared__ float part[16][64];
    const int c = threadIdx.x & 63, slice = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + c;
    float s = 0.f;
    if (j < cols)
        for (int64_t r = slice; r < rows; r += 16) s += in[r * ld + j];
    part[slice][c] = s;
    __syncthreads();
    if (slice == 0 && j < cols) {
        float t = 0.f;
#pragma unroll
        for (int q = 0; q < 16; ++q) t += part[q][c];
        out[j] = accumulate ? out[j] + t : t;
    }
}

// out[c * ldo + r] = in[r * ldi + c] for r < R (zeros for R <= r < Rpad), c < C.
__global__ __launch_bounds__(256) void transpose_kernel(const uint16_t* __restrict__ in, int64_t ldi, int R, int Rpad,
                                                        int Cc, uint16_t* __restrict__ out, int64_t ldo) {
    __shared__ uint16_t t[64][66];
    const int r0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int rr = e / 64, cc = e % 64;
        const int r = r0 + rr, c = c0 + cc;
        t[rr][cc] = (r < R && c < Cc) ? in[(int64_t)r * ldi + c] : (uint16_t)0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int cc = e / 64, rr = e % 64;
        const int r = r0 + rr, c = c0 + cc;
        if (r < Rpad && c < Cc) out[(int64_t)c * ldo + r] = t[rr][cc];
    }
}

// ---------------------------------------------------------------- phi
__device__ inline float layer1_pre(const float* __restrict__ x, const float* __restrict__ W1q,
                                   const float* __restrict__ b1, int j) {
    return fmaf(x[2], W1q[3 * j + 2], fmaf(x[1], W1q[3 * j + 1], fmaf(x[0], W1q[3 * j], b1[j])));
}

// H1q[p][j] = bf16(relu(W1 x_p + b1)) for p < P, zero rows up to Ppad.
__global__ __launch_bounds__(256) void layer1_kernel(const float* __restrict__ X, int64_t P, int64_t Ppad,
                                                     const float* __restrict__ W1q, const float* __restrict__ b1,
                                                     uint16_t* __restrict__ H1q) {
    const int j = threadIdx.x;
    for (int64_t p = blockIdx.x; p < Ppad; p += gridDim.x) {
        float h = 0.f;
        if (p < P) h = fmaxf(layer1_pre(X + 3 * p, W1q, b1, j), 0.f);
        H1q[p * H + j] = f2bf(h);
    }
}

// Point range of set s clamped to [0, P) (offsets are caller data; bad
// offsets make the loss NaN, never an access outside the buffers).
__device__ inline void set_range(const int64_t* __restrict__ off, int64_t s, int64_t P, int64_t& lo, int64_t& hi) {
    lo = min<int64_t>(max<int64_t>(off[s], 0), P);
    hi = min<int64_t>(max<int64_t>(off[s + 1], lo), P);
}

// flag = 1 unless off[0] == 0, off is non-decreasing and off[S] == P.
__global__ void check_offsets_kernel(const int64_t* __restrict__ off, int64_t S, int64_t P, int* __restrict__ flag) {
    __shared__ int bad;
    if (threadIdx.x == 0) bad = (off[0] != 0 || off[S] != P) ? 1 : 0;
    __syncthreads();
    for (int64_t s = threadIdx.x; s < S; s += blockDim.x)
        if (off[s + 1] < off[s]) bad = 1;
    __syncthreads();
    if (threadIdx.x == 0) *flag = bad;
}

// E[s][j] = sum_{p in s} a_p relu(PRE2[p][j] + b2[j]), p ascending.
__global__ __launch_bounds__(256) void pool_kernel(const float* __restrict__ PRE2, const float* __restrict__ b2,
                                                   const float* __restrict__ a, const int64_t* __restrict__ off,
                                                   int64_t P, float* __restrict__ E) {
    const int s = blockIdx.x, j = threadIdx.x;
    const float bj = b2[j];
    int64_t lo, hi;
    set_range(off, s, P, lo, hi);
    float acc = 0.f;
    for (int64_t p = lo; p < hi; ++p) acc = fmaf(a[p], fmaxf(PRE2[p * H + j] + bj, 0.f), acc);
    E[(int64_t)s * H + j] = acc;
}

// Fused inference: one workgroup per set, 64 points at a time: layer 1 into
// LDS (BF16), layer 2 on the matrix cores (each wavefront 64 points x 64
// outputs), bias + ReLU + mass weighting, column sums kept in registers.
// Global loads are issued ahead of their use (the next chunk's points and
// masses, the next K step's W2 fragments); three waves per SIMD are asked
// for, which the compiler meets without spilling.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void embed_fused_kernel(const float* __restrict__ X, const float* __restrict__ a,
                                                          const int64_t* __restrict__ off, int64_t P, SgQuant q,
                                                          const float* __restrict__ theta, float* __restrict__ E) {
    constexpr int LD = H + 8;  // padded row (elements) against bank conflicts
    __shared__ __align__(16) uint16_t h1[64 * LD];
    __shared__ float am[64];
    __shared__ float xs[64 * 3];
    const int s = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, kq = 8 * (lane >> 4);
    const float* b1 = theta + kSgB1;
    const float* b2 = theta + kSgB2;
    int64_t lo, hi;
    set_range(off, s, P, lo, hi);
    float colsum[4] = {0.f, 0.f, 0.f, 0.f};  // column 64 wave + 16 b + r16, after the lane reduction
    static_assert(H == 256, "layer 1: one hidden unit per thread");
    // this thread's hidden unit of layer 1 (same operation order as layer1_pre)
    const int j1 = tid;
    const float w10 = q.W1[3 * j1], w11 = q.W1[3 * j1 + 1], w12 = q.W1[3 * j1 + 2], b1j = b1[j1];
    // The next 64 points' coordinates (threads 0..191) and masses (192..255)
    // are loaded one chunk ahead, so their latency overlaps the products.
    float pre = 0.f;
    auto fetch = [&](int64_t pn) {
        const int64_t npn = min<int64_t>(64, hi - pn);
        if (tid < 192)
            pre = tid < 3 * npn ? X[3 * pn + tid] : 0.f;
        else
            pre = tid - 192 < npn ? a[pn + tid - 192] : 0.f;
    };
    fetch(lo);
    for (int64_t p0 = lo; p0 < hi; p0 += 64) {
        const int np = (int)min<int64_t>(64, hi - p0);
        if (tid < 192)
            xs[tid] = pre;
        else
            am[tid - 192] = pre;
        // first K step of this wavefront's W2 fragments, in flight during layer 1
        bf16x8 bfr[4], bnx[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) bfr[b] = frag16(q.W2, H, wave * 64 + 16 * b + r16, H, kq);
        __syncthreads();
        if (p0 + 64 < hi) fetch(p0 + 64);
#pragma unroll 8
        for (int pr = 0; pr < 64; ++pr) {
            float h = 0.f;
            if (pr < np) h = fmaxf(fmaf(xs[3 * pr + 2], w12, fmaf(xs[3 * pr + 1], w11, fmaf(xs[3 * pr], w10, b1j))), 0.f);
            h1[pr * LD + j1] = f2bf(h);
        }
        __syncthreads();
        f32x4 acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[i][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k0 = 0; k0 < H; k0 += 32) {
            if (k0 + 32 < H) {
#pragma unroll
                for (int b = 0; b < 4; ++b) bnx[b] = frag16(q.W2, H, wave * 64 + 16 * b + r16, H, k0 + 32 + kq);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                union {
                    uint4 u;
                    bf16x8 v;
                } af;
                af.u = *reinterpret_cast<const uint4*>(&h1[(16 * i + r16) * LD + k0 + kq]);
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[i][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af.v, bfr[b], acc[i][b], 0, 0, 0);
            }
            if (k0 + 32 < H) {
#pragma unroll
                for (int b = 0; b < 4; ++b) bfr[b] = bnx[b];
            }
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const float bj = b2[wave * 64 + 16 * b + r16];
            float part = 0.f;
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int pr = 16 * i + 4 * (lane >> 4) + r;
                    part = fmaf(am[pr], fmaxf(acc[i][b][r] + bj, 0.f), part);
                }
            part += __shfl_xor(part, 16);
            part += __shfl_xor(part, 32);
            colsum[b] += part;
        }
        __syncthreads();
    }
    if (lane < 16) {
#pragma unroll
        for (int b = 0; b < 4; ++b) E[(int64_t)s * H + wave * 64 + 16 * b + lane] = colsum[b];
    }
}

// ---------------------------------------------------------------- head
// Zq[b] = bf16([Eq, Ec, |Eq - Ec|]) for b < B, zero rows up to Bpad.
// Rows outside the tables (nq, nc rows) give NaN features, hence NaN pred.
__global__ __launch_bounds__(256) void build_z_kernel(const float* __restrict__ Eq_tab, const float* __restrict__ Ec_tab,
                                                      const int32_t* __restrict__ qi, const int32_t* __restrict__ ci,
                                                      int64_t nq, int64_t nc, int train_layout, int64_t B,
                                                      int64_t Bpad, uint16_t* __restrict__ Z) {
    const int j = threadIdx.x;
    for (int64_t b = blockIdx.x; b < Bpad; b += gridDim.x) {
        float vq = 0.f, vc = 0.f;
        if (b < B) {
            const int64_t sq = train_layout ? 2 * b : (qi ? (int64_t)qi[b] : 0);
            const int64_t sc = train_layout ? 2 * b + 1 : (ci ? (int64_t)ci[b] : b);
            vq = (sq >= 0 && sq < nq) ? Eq_tab[sq * H + j] : NAN;
            vc = (sc >= 0 && sc < nc) ? Ec_tab[sc * H + j] : NAN;
        }
        uint16_t* zr = Z + b * 3 * H;
        zr[j] = f2bf(vq);
        zr[H + j] = f2bf(vc);
        zr[2 * H + j] = f2bf(fabsf(vq - vc));
    }
}

// Fused inference head: one workgroup per 64 pairs.  The pair features
// [Eq, Ec, |Eq - Ec|] are built into LDS as BF16 one 64-wide column block at
// a time, all three parts together, so every embedding row is read once
// (each thread one row's 16 features, 16-byte loads issued one block ahead,
// so they overlap the products), each
// wavefront multiplies them with 64 rows of W3 on the matrix cores (K = 768,
// each 64-deep block's W3 fragments loaded during the previous block),
// and the epilogue applies b3, ReLU and w4, sums the four wavefronts' parts
// in order and writes softplus(t + b4).  Rows outside the tables give NaN.
__global__ __launch_bounds__(256) void rho_fused_kernel(const float* __restrict__ Eq_tab, int64_t nq,
                                                        const float* __restrict__ Ec_tab, int64_t nc,
                                                        const int32_t* __restrict__ qi,
                                                        const int32_t* __restrict__ ci, int64_t B, SgQuant q,
                                                        const float* __restrict__ theta, float* __restrict__ pred) {
    constexpr int LD = 64 + 8;
    constexpr int NCB = H / 64;  // 64-wide column blocks of an embedding
    __shared__ __align__(16) uint16_t zt[3][64 * LD];
    __shared__ float red[4][64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, kq = 8 * (lane >> 4);
    const int64_t b0 = (int64_t)blockIdx.x * 64;
    // Staging: thread -> (row, 16 consecutive features) of a 64 x 64 block.
    const int srow = tid >> 2, sseg = (tid & 3) * 16;
    int64_t sq = -2, sc = -2;  // -2: padding row, -1: index outside the table
    {
        const int64_t b = b0 + srow;
        if (b < B) {
            sq = qi ? (int64_t)qi[b] : 0;
            sc = ci ? (int64_t)ci[b] : b;
            if (sq < 0 || sq >= nq) sq = -1;
            if (sc < 0 || sc >= nc) sc = -1;
        }
    }
    const bool rvalid = sq >= 0 && sc >= 0, rbad = sq == -1 || sc == -1;
    float4 fq[4], fc[4];
    auto load_feats = [&](int cb) {
        const int col = cb * 64 + sseg;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            fq[v] = make_float4(0.f, 0.f, 0.f, 0.f);
            fc[v] = fq[v];
        }
        if (rvalid) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                fq[v] = *reinterpret_cast<const float4*>(Eq_tab + sq * H + col + 4 * v);
                fc[v] = *reinterpret_cast<const float4*>(Ec_tab + sc * H + col + 4 * v);
            }
        }
    };
    // W3 fragments of one 64-deep K block (part p, column block cb: K offset
    // p * H + cb * 64), both 32-deep steps (L2-resident: every block reads W3).
    bf16x8 w3[2][4], w3n[2][4];
    auto load_w3 = [&](bf16x8 (&w)[2][4], int kb) {
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int b = 0; b < 4; ++b) w[ks][b] = frag16(q.W3, 3 * H, wave * 64 + 16 * b + r16, H, kb * 64 + ks * 32 + kq);
    };
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[i][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
    load_feats(0);
    load_w3(w3, 0);  // K block (part 0, column block 0)
    for (int cb = 0; cb < NCB; ++cb) {
        __syncthreads();  // the previous column block's fragments have been read
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            uint32_t wv[8];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float a[4] = {fq[v].x, fq[v].y, fq[v].z, fq[v].w};
                const float c[4] = {fc[v].x, fc[v].y, fc[v].z, fc[v].w};
                float z[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) z[e] = rbad ? NAN : (p == 0 ? a[e] : (p == 1 ? c[e] : fabsf(a[e] - c[e])));
                wv[2 * v] = (uint32_t)f2bf(z[0]) | ((uint32_t)f2bf(z[1]) << 16);
                wv[2 * v + 1] = (uint32_t)f2bf(z[2]) | ((uint32_t)f2bf(z[3]) << 16);
            }
            uint4* dst = reinterpret_cast<uint4*>(&zt[p][srow * LD + sseg]);
            dst[0] = make_uint4(wv[0], wv[1], wv[2], wv[3]);
            dst[1] = make_uint4(wv[4], wv[5], wv[6], wv[7]);
        }
        __syncthreads();
        if (cb + 1 < NCB) load_feats(cb + 1);  // in flight during the products
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            // the next K block's W3 fragments, in flight during these products
            const bool more = p < 2 || cb + 1 < NCB;
            if (more) load_w3(w3n, p < 2 ? (p + 1) * NCB + cb : cb + 1);
            const auto& wc = w3;
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    union {
                        uint4 u;
                        bf16x8 v;
                    } af;
                    af.u = *reinterpret_cast<const uint4*>(&zt[p][(16 * i + r16) * LD + ks * 32 + kq]);
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        acc[i][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af.v, wc[ks][b], acc[i][b], 0, 0, 0);
                }
            }
            if (more) {
#pragma unroll
                for (int ks = 0; ks < 2; ++ks)
#pragma unroll
                    for (int b = 0; b < 4; ++b) w3[ks][b] = w3n[ks][b];
            }
        }
    }
    const float* b3 = theta + kSgB3;
    // per-row partial over this wavefront's 64 columns
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float sum = 0.f;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int col = wave * 64 + 16 * b + r16;
                sum = fmaf(relu_nan(acc[i][b][r] + b3[col]), q.w4[col], sum);
            }
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) sum += __shfl_xor(sum, o);
            if (r16 == 0) red[wave][16 * i + 4 * (lane >> 4) + r] = sum;
        }
    __syncthreads();
    if (tid < 64 && b0 + tid < B) {
        const float t = ((red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid])) + theta[kSgB4];
        pred[b0 + tid] = softplusf(t);
    }
}

// One wavefront per pair: t = w4 . relu(PRE3 + b3) + b4, pred = softplus(t).
__global__ __launch_bounds__(256) void head_fwd_kernel(const float* __restrict__ PRE3, const float* __restrict__ theta,
                                                       const float* __restrict__ w4q, int64_t B,
                                                       float* __restrict__ t_out, float* __restrict__ pred) {
    const int lane = threadIdx.x & 63;
    const int64_t b = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= B) return;
    const float* b3 = theta + kSgB3;
    float s = 0.f;
#pragma unroll
    for (int u = 0; u < H / 64; ++u) {
        const int j = lane + 64 * u;
        s = fmaf(relu_nan(PRE3[b * H + j] + b3[j]), w4q[j], s);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) {
        const float t = s + theta[kSgB4];
        if (t_out) t_out[b] = t;
        pred[b] = softplusf(t);
    }
}

// Head backward, one wavefront per pair.  Row b of HB (ld kSgHbCols):
// [dg (H) | dt * g (H) | dt | r^2 / B]; dGq[b] = bf16(dg).
__global__ __launch_bounds__(256) void head_bwd_kernel(const float* __restrict__ PRE3, const float* __restrict__ theta,
                                                       const float* __restrict__ w4q, const float* __restrict__ t_in,
                                                       const float* __restrict__ pred, const float* __restrict__ y,
                                                       int64_t B, float* __restrict__ HB, uint16_t* __restrict__ dGq) {
    const int lane = threadIdx.x & 63;
    const int64_t b = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= B) return;
    const float* b3 = theta + kSgB3;
    const float pv = pred[b];
    const float r = logf(pv) - logf(y[b]);
    const float dpred = 2.f * r / ((float)B * pv);
    const float dt = dpred * sigmoidf(t_in[b]);
    float* row = HB + b * kSgHbCols;
#pragma unroll
    for (int u = 0; u < H / 64; ++u) {
        const int j = lane + 64 * u;
        const float pre = PRE3[b * H + j] + b3[j];
        const float g = relu_nan(pre);
        const float dg = pre > 0.f ? dt * w4q[j] : 0.f;
        row[j] = dg;
        row[H + j] = dt * g;
        dGq[b * H + j] = f2bf(dg);
    }
    if (lane == 0) {
        row[2 * H] = dt;
        row[2 * H + 1] = r * r / (float)B;
    }
}

// dE of the two sets of pair b from dZ (B x 3H).
__global__ void dz_to_de_kernel(const float* __restrict__ dZ, const float* __restrict__ E, int64_t B,
                                float* __restrict__ dE) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < B * H; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = e / H;
        const int j = (int)(e % H);
        const float q = E[2 * b * H + j], c = E[(2 * b + 1) * H + j];
        const float sg = (float)((q > c) - (q < c));
        const float* dz = dZ + b * 3 * H;
        dE[2 * b * H + j] = fmaf(dz[2 * H + j], sg, dz[j]);
        dE[(2 * b + 1) * H + j] = dz[H + j] - dz[2 * H + j] * sg;
    }
}

// dPRE2[p][j] = a_p dE[s][j] where PRE2 + b2 > 0 (BF16), and the per-set
// column sums (FP32, p ascending) for db2.
__global__ __launch_bounds__(256) void pool_bwd_kernel(const float* __restrict__ PRE2, const float* __restrict__ b2,
                                                       const float* __restrict__ a, const int64_t* __restrict__ off,
                                                       int64_t P, const float* __restrict__ dE,
                                                       uint16_t* __restrict__ dP2q, float* __restrict__ db2_part) {
    const int s = blockIdx.x, j = threadIdx.x;
    const float bj = b2[j];
    const float de = dE[(int64_t)s * H + j];
    int64_t lo, hi;
    set_range(off, s, P, lo, hi);
    float acc = 0.f;
    for (int64_t p = lo; p < hi; ++p) {
        const float v = PRE2[p * H + j] + bj > 0.f ? a[p] * de : 0.f;
        acc += v;
        dP2q[p * H + j] = f2bf(v);
    }
    db2_part[(int64_t)s * H + j] = acc;
}

// Partial sums over a chunk of points of dpre1 * [x, 1] (dW1, db1).
__global__ __launch_bounds__(256) void layer1_bwd_kernel(const float* __restrict__ dH1, const float* __restrict__ X,
                                                         const float* __restrict__ W1q, const float* __restrict__ b1,
                                                         int64_t P, int64_t chunk, float* __restrict__ part) {
    const int j = threadIdx.x;
    const int64_t lo = blockIdx.x * chunk, hi = min<int64_t>(P, lo + chunk);
    float gw0 = 0.f, gw1 = 0.f, gw2 = 0.f, gb = 0.f;
    for (int64_t p = lo; p < hi; ++p) {
        const float* x = X + 3 * p;
        if (layer1_pre(x, W1q, b1, j) > 0.f) {
            const float g = dH1[p * H + j];
            gb += g;
            gw0 = fmaf(g, x[0], gw0);
            gw1 = fmaf(g, x[1], gw1);
            gw2 = fmaf(g, x[2], gw2);
        }
    }
    float* o = part + (int64_t)blockIdx.x * 4 * H;
    o[3 * j] = gw0;
    o[3 * j + 1] = gw1;
    o[3 * j + 2] = gw2;
    o[3 * H + j] = gb;
}

// Scatter of the head column sums into the flat gradient.
__global__ void head_grad_scatter_kernel(const float* __restrict__ hsum, const int* __restrict__ bad,
                                         float* __restrict__ grad, float* __restrict__ loss) {
    const int j = threadIdx.x;
    grad[kSgB3 + j] = hsum[j];
    grad[kSgW4 + j] = hsum[H + j];
    if (j == 0) {
        grad[kSgB4] = hsum[2 * H];
        if (loss) *loss = *bad ? NAN : hsum[2 * H + 1];
    }
}

__global__ void layer1_grad_scatter_kernel(const float* __restrict__ s, float* __restrict__ grad) {
    const int j = threadIdx.x;
    grad[kSgW1 + 3 * j] = s[3 * j];
    grad[kSgW1 + 3 * j + 1] = s[3 * j + 1];
    grad[kSgW1 + 3 * j + 2] = s[3 * j + 2];
    grad[kSgB1 + j] = s[3 * H + j];
}

// Adam with host-rounded coefficients (beta, 1 - beta each rounded once).
__global__ void adam_kernel(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, int64_t n, float lr, float beta1, float omb1, float beta2,
                            float omb2, float eps, float bc1, float bc2) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = beta1 * m[i] + omb1 * gi;
        const float vi = beta2 * v[i] + omb2 * gi * gi;
        m[i] = mi;
        v[i] = vi;
        theta[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    }
}

// ---------------------------------------------------------------- top-k
// Order-preserving unsigned keys: -0 == +0, NaN after everything.
__device__ inline uint32_t ord_key(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0xffffffffu;
    if ((u & 0x7fffffffu) == 0u) u = 0u;
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline uint64_t ord_key(double f) {
    uint64_t u = (uint64_t)__double_as_longlong(f);
    if ((u & 0x7fffffffffffffffull) > 0x7ff0000000000000ull) return ~0ull;
    if ((u & 0x7fffffffffffffffull) == 0ull) u = 0ull;
    return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}

constexpr int kTopkThreads = 1024;

constexpr int kTopkCap = 2 * kSgTopkMax;  // sort buffer
constexpr int kTopkSample = 4096;         // sampled keys of the threshold pass
constexpr int kTopkBuf = 16384;           // candidate buffer behind the threshold

// Ascending bitonic sort of T * E (key, index) pairs held in registers:
// element e = s * T + threadIdx.x sits in slot s.  Partners at strides of T
// and above are in the same thread (register swap), below 64 in the same
// wavefront (shuffles); only strides 64 .. T/2 go through LDS (xk, xi: T * E
// entries each), with barriers.  Order: key, then index (WITH_IDX), so the
// result is unique; without indices equal keys are interchangeable.
template <typename K, int T, int E, bool WITH_IDX>
__device__ inline void bitonic_regs(K (&k)[E], int32_t (&ix)[E], K* xk, int32_t* xi) {
    const int tid = threadIdx.x;
    constexpr int N = T * E;
    auto greater = [](K a, int32_t ia, K b, int32_t ib) { return a > b || (WITH_IDX && a == b && ia > ib); };
    for (int size = 2; size <= N; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            if (stride >= T) {
                const int ds = stride / T;
#pragma unroll
                for (int s = 0; s < E; ++s) {
                    if (s & ds) continue;
                    const int ps = s | ds;
                    const bool up = ((s * T + tid) & size) == 0;
                    if (greater(k[s], ix[s], k[ps], ix[ps]) == up) {
                        const K tk = k[s];
                        k[s] = k[ps];
                        k[ps] = tk;
                        const int32_t ti = ix[s];
                        ix[s] = ix[ps];
                        ix[ps] = ti;
                    }
                }
                continue;
            }
            K pk[E];
            int32_t pi[E];
            if (stride >= 64) {
                __syncthreads();  // earlier readers of xk / xi are done
#pragma unroll
                for (int s = 0; s < E; ++s) {
                    xk[s * T + tid] = k[s];
                    if (WITH_IDX) xi[s * T + tid] = ix[s];
                }
                __syncthreads();
#pragma unroll
                for (int s = 0; s < E; ++s) {
                    pk[s] = xk[(s * T + tid) ^ stride];
                    pi[s] = WITH_IDX ? xi[(s * T + tid) ^ stride] : 0;
                }
            } else {
#pragma unroll
                for (int s = 0; s < E; ++s) {
                    pk[s] = __shfl_xor(k[s], stride);
                    pi[s] = WITH_IDX ? __shfl_xor(ix[s], stride) : 0;
                }
            }
#pragma unroll
            for (int s = 0; s < E; ++s) {
                const int e = s * T + tid;
                const bool keep_min = ((e & stride) == 0) == ((e & size) == 0);
                const bool take = keep_min ? greater(k[s], ix[s], pk[s], pi[s]) : greater(pk[s], pi[s], k[s], ix[s]);
                if (take) {
                    k[s] = pk[s];
                    ix[s] = pi[s];
                }
            }
        }
    }
}

// The k smallest of n values, ascending by (value, index), in one workgroup.
// 1. Radix select of the k-th key, 8-bit digits, coalesced passes; a
//    wavefront whose active lanes share one digit adds them with one atomic
//    (the leading digits of similar values would otherwise serialise).
// 2. Collection: all keys below it, and the keys equal to it, into an LDS
//    buffer (unordered); if the equal keys overflow the buffer they are
//    collected again in index order instead, as many as needed.
// 3. Bitonic sort of the buffer by (key, index); the first k are the answer.
// When all n values fit the buffer, steps 1 and 2 are skipped.
// BUF: the values were first narrowed to the candidates at or below a
// sampled threshold (bkey / bidx, *count of them, original indices); those
// are used when they hold at least k and fit, and the direct pass over all
// values runs otherwise, or when the equal keys would need the index-order
// collection (the buffer is in arrival order).  Either way the answer is the
// exact (key, index) order of all n values.
template <typename V, typename K, bool BUF>
__global__ __launch_bounds__(kTopkThreads) void topk_kernel(const V* __restrict__ vals, int64_t n, int k,
                                                            int32_t* __restrict__ out, const K* __restrict__ bkey,
                                                            const int32_t* __restrict__ bidx,
                                                            const unsigned int* __restrict__ count) {
    constexpr int T = kTopkThreads;
    constexpr int NB = (int)sizeof(K) * 8;
    __shared__ unsigned int hist[256];
    __shared__ K skey[kTopkCap];
    __shared__ int32_t sidx[kTopkCap];
    __shared__ int64_t scan[T];
    __shared__ K s_prefix;
    __shared__ int64_t s_need;
    __shared__ int cnt_less, cnt_eq;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    bool use_buf = false;
    int64_t nn = n;
    if constexpr (BUF) {
        const unsigned int c = *count;
        use_buf = c >= (unsigned int)k && c <= (unsigned int)kTopkBuf;
        if (use_buf) nn = c;
    }
    auto key_at = [&](int64_t i) -> K { return use_buf ? bkey[i] : ord_key(vals[i]); };
    auto idx_at = [&](int64_t i) -> int32_t { return use_buf ? bidx[i] : (int32_t)i; };
    int64_t filled = 0;
    for (int attempt = 0; attempt < 2; ++attempt) {  // the second only when the buffer cannot serve
    K prefix = 0, mask = 0;
    int64_t need = k;
    filled = 0;
    bool redo = false;
    if (nn <= kTopkCap) {
        // Everything fits the sort buffer: no selection needed.
        for (int64_t i = tid; i < nn; i += T) {
            skey[i] = key_at(i);
            sidx[i] = idx_at(i);
        }
        filled = nn;
    } else {
    for (int shift = NB - 8; shift >= 0; shift -= 8) {
        for (int b = tid; b < 256; b += T) hist[b] = 0u;
        __syncthreads();
        for (int64_t i = tid; i < nn; i += T) {
            const K key = key_at(i);
            const int bin = (key & mask) == prefix ? (int)((key >> shift) & 0xff) : -1;
            const uint64_t active = __ballot(1);
            const int b0 = __builtin_amdgcn_readfirstlane(bin);
            const uint64_t same = __ballot(bin == b0);
            if (same == active) {
                if (b0 >= 0 && lane == __ffsll((unsigned long long)active) - 1)
                    atomicAdd(&hist[b0], (unsigned int)__popcll(active));
            } else if (bin >= 0) {
                atomicAdd(&hist[bin], 1u);
            }
        }
        __syncthreads();
        if (tid == 0) {
            int64_t c = 0;
            int b = 0;
            for (; b < 255; ++b) {
                if (c + (int64_t)hist[b] >= need) break;
                c += hist[b];
            }
            s_prefix = prefix | ((K)b << shift);
            s_need = need - c;
            cnt_less = 0;
            cnt_eq = 0;
        }
        __syncthreads();
        prefix = s_prefix;
        need = s_need;
        mask |= (K)0xff << shift;
        __syncthreads();
    }
    // prefix = key of the k-th smallest; need = how many of that key to take.
    const int64_t nless = k - need;
    for (int64_t i = tid; i < nn; i += T) {
        const K key = key_at(i);
        if (key < prefix) {
            const int p = atomicAdd(&cnt_less, 1);
            skey[p] = key;
            sidx[p] = idx_at(i);
        } else if (key == prefix) {
            const int64_t q = nless + atomicAdd(&cnt_eq, 1);
            if (q < kTopkCap) {
                skey[q] = key;
                sidx[q] = idx_at(i);
            }
        }
    }
    __syncthreads();
    filled = nless + cnt_eq;
    if (filled > kTopkCap && use_buf) {
        redo = true;  // index order is not the buffer's order: take all values
    } else if (filled > kTopkCap) {
        // Too many equal keys: take the first `need` of them in index order.
        const int64_t per = (nn + T - 1) / T;
        const int64_t lo = min<int64_t>(nn, tid * per), hi = min<int64_t>(nn, lo + per);
        int64_t ce = 0;
        for (int64_t i = lo; i < hi; ++i) ce += key_at(i) == prefix;
        scan[tid] = ce;
        __syncthreads();
        if (tid == 0) {
            int64_t run = 0;
            for (int t = 0; t < T; ++t) {
                const int64_t v = scan[t];
                scan[t] = run;
                run += v;
            }
        }
        __syncthreads();
        int64_t we = scan[tid];
        for (int64_t i = lo; i < hi && we < need; ++i) {
            if (key_at(i) == prefix) {
                skey[nless + we] = prefix;
                sidx[nless + we] = idx_at(i);
                ++we;
            }
        }
        filled = k;
    }
    }  // nn > kTopkCap
    if (!redo) break;
    use_buf = false;  // workgroup-uniform
    nn = n;
    __syncthreads();
    }
    for (int64_t e = filled + tid; e < kTopkCap; e += T) {
        skey[e] = ~(K)0;
        sidx[e] = 0x7fffffff;
    }
    __syncthreads();
    constexpr int E = kTopkCap / T;
    K rk[E];
    int32_t ri[E];
#pragma unroll
    for (int s = 0; s < E; ++s) {
        rk[s] = skey[s * T + tid];
        ri[s] = sidx[s * T + tid];
    }
    bitonic_regs<K, T, E, true>(rk, ri, skey, sidx);
#pragma unroll
    for (int s = 0; s < E; ++s)
        if (s * T + tid < k) out[s * T + tid] = ri[s];
}

// Threshold for the candidate pass: kTopkSample evenly spaced keys, sorted;
// the key 1.5 k / n of the way up plus 16 ranks (about four standard
// deviations of the sample quantile above rank k at 10^5 values), so that at
// least k values lie at or below it unless the sample misleads -- then the
// selection falls back to all values.  Also clears the candidate count.
template <typename V, typename K>
__global__ __launch_bounds__(kTopkThreads) void topk_sample_kernel(const V* __restrict__ vals, int64_t n, int k,
                                                                   K* __restrict__ thr, unsigned int* __restrict__ count) {
    constexpr int T = kTopkThreads, S = kTopkSample;
    __shared__ K sk[S];
    const int tid = threadIdx.x;
    constexpr int E = S / T;
    K rk[E];
    int32_t ri[E];
#pragma unroll
    for (int s = 0; s < E; ++s) {
        rk[s] = ord_key(vals[(int64_t)(s * T + tid) * n / S]);
        ri[s] = 0;
    }
    bitonic_regs<K, T, E, false>(rk, ri, sk, nullptr);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < E; ++s) sk[s * T + tid] = rk[s];
    __syncthreads();
    if (tid == 0) {
        const double frac = 1.5 * (double)k / (double)n;
        int r = (int)(frac * S) + 16;
        if (r > S - 1) r = S - 1;
        *thr = sk[r];
        *count = 0u;
    }
}

// Every value whose key is at or below the threshold, appended (key,
// index) in arrival order; the count keeps rising past the buffer so the
// selection can tell an overflow.
template <typename V, typename K>
__global__ __launch_bounds__(256) void topk_collect_kernel(const V* __restrict__ vals, int64_t n,
                                                           const K* __restrict__ thr, unsigned int* __restrict__ count,
                                                           K* __restrict__ bkey, int32_t* __restrict__ bidx) {
    const K t = *thr;
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < n; i0 += stride) {  // uniform per wavefront
        const int64_t i = i0 + threadIdx.x;
        K key = 0;
        bool take = false;
        if (i < n) {
            key = ord_key(vals[i]);
            take = key <= t;
        }
        const unsigned long long m = __ballot(take);
        if (m == 0ull) continue;
        const int leader = __builtin_ctzll(m);
        unsigned int base = 0u;
        if (lane == leader) base = atomicAdd(count, (unsigned int)__popcll(m));
        base = __shfl(base, leader);
        if (take) {
            const unsigned int pos = base + (unsigned int)__popcll(m & ((1ull << lane) - 1ull));
            if (pos < (unsigned int)kTopkBuf) {
                bkey[pos] = key;
                bidx[pos] = (int32_t)i;
            }
        }
    }
}

// out_idx[r] = sel[pos[r]], out_val[r] = vals[pos[r]].
__global__ void gather_ranked_kernel(const int32_t* __restrict__ pos, const int32_t* __restrict__ sel,
                                     const double* __restrict__ vals, int k, int32_t* __restrict__ out_idx,
                                     double* __restrict__ out_val) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= k) return;
    const int p = pos[r];
    out_idx[r] = sel[p];
    if (out_val) out_val[r] = vals[p];
}

__global__ void fill_i32_kernel(int32_t* __restrict__ p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void two_offsets_kernel(int64_t* __restrict__ off, int64_t m) {
    if (threadIdx.x == 0) {
        off[0] = 0;
        off[1] = m;
    }
}

inline int grid_for(int64_t n, int per_block = 256, int cap = 65536) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + per_block - 1) / per_block, cap));
}

inline int gemm_nt(const uint16_t* A, int64_t lda, const uint16_t* B, int64_t ldb, float* C, int64_t ldc, int M,
                   int N, int K, int splits, int64_t c_split, hipStream_t st) {
    const int kchunk = ((K / splits + 31) / 32) * 32;
    dim3 grid((M + 63) / 64, (N + 63) / 64, splits);
    hipLaunchKernelGGL(gemm_nt_kernel, grid, dim3(256), 0, st, A, lda, B, ldb, C, ldc, M, N, K, kchunk, c_split);
    return (int)hipGetLastError();
}

inline int transpose(const uint16_t* in, int64_t ldi, int R, int Rpad, int C, uint16_t* out, int64_t ldo,
                     hipStream_t st) {
    dim3 grid((Rpad + 63) / 64, (C + 63) / 64);
    hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, st, in, ldi, R, Rpad, C, out, ldo);
    return (int)hipGetLastError();
}

}  // namespace

// ---------------------------------------------------------------- launchers
int launch_prepare(const float* theta, const SgQuant& q, void* stream) {
    hipLaunchKernelGGL(prepare_kernel, dim3(512), dim3(256), 0, (hipStream_t)stream, theta, q);
    return (int)hipGetLastError();
}

int launch_embed(const float* theta, const SgQuant& q, const float* X, const float* a, const int64_t* set_off,
                 int64_t num_sets, int64_t num_points, float* E, void* stream) {
    if (num_sets == 0) return 0;
    hipLaunchKernelGGL(embed_fused_kernel, dim3((unsigned)num_sets), dim3(256), 0, (hipStream_t)stream, X, a, set_off,
                       num_points, q, theta, E);
    return (int)hipGetLastError();
}

int launch_predict(const float* theta, const SgQuant& q, const float* Eq, int64_t nq, const float* Ec, int64_t nc,
                   const int32_t* qi, const int32_t* ci, int train_layout, int64_t B, const SgPredictWork& w,
                   float* t_out, float* pred, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    if (B == 0) return 0;
    const int64_t Bpad = (B + 63) / 64 * 64;
    // The fused kernel reads embedding rows with 16-byte loads.
    const bool aligned = ((reinterpret_cast<uintptr_t>(Eq) | reinterpret_cast<uintptr_t>(Ec)) & 15u) == 0;
    if (!train_layout && t_out == nullptr && aligned) {
        hipLaunchKernelGGL(rho_fused_kernel, dim3((unsigned)(Bpad / 64)), dim3(256), 0, st, Eq, nq, Ec, nc, qi, ci, B,
                           q, theta, pred);
        return (int)hipGetLastError();
    }
    hipLaunchKernelGGL(build_z_kernel, dim3(grid_for(Bpad, 1)), dim3(256), 0, st, Eq, Ec, qi, ci, nq, nc, train_layout,
                       B, Bpad, w.Z);
    int err = (int)hipGetLastError();
    if (err) return err;
    err = gemm_nt(w.Z, 3 * H, q.W3, 3 * H, w.PRE3, H, (int)B, H, 3 * H, 1, 0, st);
    if (err) return err;
    hipLaunchKernelGGL(head_fwd_kernel, dim3((unsigned)((B + 3) / 4)), dim3(256), 0, st, w.PRE3, theta, q.w4, B, t_out,
                       pred);
    return (int)hipGetLastError();
}

int launch_loss_grad(const float* theta, const SgQuant& q, const float* X, const float* a, const int64_t* set_off,
                     int64_t B, int64_t P, const float* labels, const SgTrainWork& w, float* loss, float* grad,
                     void* stream) {
    hipStream_t st = (hipStream_t)stream;
    const int64_t S = 2 * B;
    const int64_t Ppad = (P + 63) / 64 * 64;
    const int64_t Bpad = (B + 63) / 64 * 64;
    int err;
    hipLaunchKernelGGL(check_offsets_kernel, dim3(1), dim3(256), 0, st, set_off, S, P, w.bad);
    // forward
    hipLaunchKernelGGL(layer1_kernel, dim3(grid_for(Ppad, 1)), dim3(256), 0, st, X, P, Ppad, q.W1, theta + kSgB1,
                       w.H1q);
    if ((err = (int)hipGetLastError())) return err;
    if ((err = gemm_nt(w.H1q, H, q.W2, H, w.PRE2, H, (int)P, H, H, 1, 0, st))) return err;
    hipLaunchKernelGGL(pool_kernel, dim3((unsigned)S), dim3(256), 0, st, w.PRE2, theta + kSgB2, a, set_off, P, w.E);
    if ((err = (int)hipGetLastError())) return err;
    SgPredictWork pw{w.Z, w.PRE3};
    if ((err = launch_predict(theta, q, w.E, S, w.E, S, nullptr, nullptr, 1, B, pw, w.t, w.pred, stream))) return err;
    // head backward
    hipLaunchKernelGGL(head_bwd_kernel, dim3((unsigned)((B + 3) / 4)), dim3(256), 0, st, w.PRE3, theta, q.w4, w.t,
                       w.pred, labels, B, w.HB, w.dGq);
    if ((err = (int)hipGetLastError())) return err;
    hipLaunchKernelGGL(colsum_kernel, dim3((kSgHbCols + 63) / 64), dim3(kColsumThreads), 0, st, w.HB, B,
                       (int64_t)kSgHbCols, kSgHbCols, w.hsum, 0);
    hipLaunchKernelGGL(head_grad_scatter_kernel, dim3(1), dim3(256), 0, st, w.hsum, w.bad, grad, loss);
    // dW3 = dG^T Z: both transposed to K = pair index
    if ((err = transpose(w.dGq, H, (int)B, (int)Bpad, H, w.dGqT, Bpad, st))) return err;
    if ((err = transpose(w.Z, 3 * H, (int)B, (int)Bpad, 3 * H, w.ZT, Bpad, st))) return err;
    if ((err = gemm_nt(w.dGqT, Bpad, w.ZT, Bpad, grad + kSgW3, 3 * H, H, 3 * H, (int)Bpad, 1, 0, st))) return err;
    // dZ = dG W3
    if ((err = gemm_nt(w.dGq, H, q.W3T, H, w.dZ, 3 * H, (int)B, 3 * H, H, 1, 0, st))) return err;
    hipLaunchKernelGGL(dz_to_de_kernel, dim3(grid_for(B * H)), dim3(256), 0, st, w.dZ, w.E, B, w.dE);
    if ((err = (int)hipGetLastError())) return err;
    // pooling and layer-2 backward
    hipLaunchKernelGGL(pool_bwd_kernel, dim3((unsigned)S), dim3(256), 0, st, w.PRE2, theta + kSgB2, a, set_off, P,
                       w.dE, w.dP2q, w.db2p);
    if ((err = (int)hipGetLastError())) return err;
    hipLaunchKernelGGL(colsum_kernel, dim3(H / 64), dim3(kColsumThreads), 0, st, w.db2p, S, (int64_t)H, H,
                       grad + kSgB2, 0);
    if ((err = transpose(w.dP2q, H, (int)P, (int)Ppad, H, w.dP2qT, Ppad, st))) return err;
    if ((err = transpose(w.H1q, H, (int)P, (int)Ppad, H, w.H1qT, Ppad, st))) return err;
    const int splits = (int)std::max<int64_t>(1, std::min<int64_t>(64, Ppad / 2048));
    if ((err = gemm_nt(w.dP2qT, Ppad, w.H1qT, Ppad, w.split, H, H, H, (int)Ppad, splits, (int64_t)H * H, st)))
        return err;
    hipLaunchKernelGGL(sum_splits_kernel, dim3(grid_for((int64_t)H * H)), dim3(256), 0, st, w.split, splits,
                       (int64_t)H * H, grad + kSgW2, (int64_t)H * H);
    // dH1 = dP2 W2
    if ((err = gemm_nt(w.dP2q, H, q.W2T, H, w.dH1, H, (int)P, H, H, 1, 0, st))) return err;
    const int64_t chunk = 512;
    const int64_t nblk = std::max<int64_t>(1, (P + chunk - 1) / chunk);
    hipLaunchKernelGGL(layer1_bwd_kernel, dim3((unsigned)nblk), dim3(256), 0, st, w.dH1, X, q.W1, theta + kSgB1, P,
                       chunk, w.l1p);
    if ((err = (int)hipGetLastError())) return err;
    hipLaunchKernelGGL(colsum_kernel, dim3(4 * H / 64), dim3(kColsumThreads), 0, st, w.l1p, nblk, (int64_t)4 * H,
                       4 * H, w.l1s, 0);
    hipLaunchKernelGGL(layer1_grad_scatter_kernel, dim3(1), dim3(256), 0, st, w.l1s, grad);
    return (int)hipGetLastError();
}

int launch_adam(float* theta, float* m, float* v, const float* grad, float lr, double beta1, double beta2, float eps,
                float bc1, float bc2, void* stream) {
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(kSgParams)), dim3(256), 0, (hipStream_t)stream, theta, m, v, grad,
                       (int64_t)kSgParams, lr, (float)beta1, (float)(1.0 - beta1), (float)beta2, (float)(1.0 - beta2),
                       eps, bc1, bc2);
    return (int)hipGetLastError();
}

size_t topk_ws_bytes() { return 256 + (size_t)kTopkBuf * (sizeof(uint64_t) + sizeof(int32_t)); }

template <typename V, typename K>
int launch_topk(const V* vals, int64_t n, int k, int32_t* out, void* ws, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    // Large inputs: sampled threshold and a grid-wide candidate pass first.
    if (ws != nullptr && n > 2 * (int64_t)kTopkBuf) {
        char* b = static_cast<char*>(ws);
        K* thr = reinterpret_cast<K*>(b);
        unsigned int* count = reinterpret_cast<unsigned int*>(b + 64);
        K* bkey = reinterpret_cast<K*>(b + 256);
        int32_t* bidx = reinterpret_cast<int32_t*>(b + 256 + (size_t)kTopkBuf * sizeof(K));
        hipLaunchKernelGGL((topk_sample_kernel<V, K>), dim3(1), dim3(kTopkThreads), 0, st, vals, n, k, thr, count);
        const int64_t blocks = std::min<int64_t>((n + 255) / 256, 2048);
        hipLaunchKernelGGL((topk_collect_kernel<V, K>), dim3((unsigned)blocks), dim3(256), 0, st, vals, n, thr, count,
                           bkey, bidx);
        hipLaunchKernelGGL((topk_kernel<V, K, true>), dim3(1), dim3(kTopkThreads), 0, st, vals, n, k, out, bkey, bidx,
                           count);
        return (int)hipGetLastError();
    }
    hipLaunchKernelGGL((topk_kernel<V, K, false>), dim3(1), dim3(kTopkThreads), 0, st, vals, n, k, out, nullptr,
                       nullptr, nullptr);
    return (int)hipGetLastError();
}

int launch_topk_f32(const float* vals, int64_t n, int k, int32_t* out, void* ws, void* stream) {
    return launch_topk<float, uint32_t>(vals, n, k, out, ws, stream);
}

int launch_topk_f64(const double* vals, int64_t n, int k, int32_t* out, void* ws, void* stream) {
    return launch_topk<double, uint64_t>(vals, n, k, out, ws, stream);
}

int launch_gather_ranked(const int32_t* pos, const int32_t* sel, const double* vals, int k, int32_t* out_idx,
                         double* out_val, void* stream) {
    hipLaunchKernelGGL(gather_ranked_kernel, dim3((k + 255) / 256), dim3(256), 0, (hipStream_t)stream, pos, sel, vals, k,
                       out_idx, out_val);
    return (int)hipGetLastError();
}

int launch_fill_i32(int32_t* p, int64_t n, int32_t v, void* stream) {
    hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, p, n, v);
    return (int)hipGetLastError();
}

int launch_two_offsets(int64_t* off, int64_t m, void* stream) {
    hipLaunchKernelGGL(two_offsets_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, off, m);
    return (int)hipGetLastError();
}

}  // namespace sg
}  // namespace nnsemd
