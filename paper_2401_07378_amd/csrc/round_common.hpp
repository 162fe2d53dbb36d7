// Pieces shared by the one-workgroup-per-pair solvers (point path and the
// BF16 document path): LDS layout of a pair, workgroup scans and reductions,
// and the generic phases of one round of Algorithm 1 (Sec. III-A) that run
// after the search has stored every active consumer's pick (active supplier
// slot in cnn[j], exact FP64 key in ckey[j]) and counted it into scnt[slot]:
//   round_buckets  claimant sets a_i: scan of the counts, scatter
//   round_rank     each claimant's place in its bucket: (D_ij, j) order for
//                  the greedy protocol, (random key, j) for the random one
//   round_walk     one lane per claimed supplier serves in that order (FP64)
//   round_compact  plan append + surviving suppliers / consumers
// Every function ends with a workgroup barrier; all of them must be called
// by every thread of the workgroup with block-uniform arguments.
#pragma once

#include <stdint.h>

#include "internal.hpp"

// Optional per-phase cycle accounting for profiling builds only
// (-DNNSEMD_PHASE_TIMING).  Every thread reads the clock (no divergent code);
// thread 0 adds its totals to the phase buffer once, at the end of the pair.
#ifdef NNSEMD_PHASE_TIMING
#define NNSEMD_PH_DECL uint64_t ph[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}; uint64_t ph_t = clock64();
#define NNSEMD_PH(k) { const uint64_t ph_n = clock64(); ph[k] += ph_n - ph_t; ph_t = ph_n; }
#define NNSEMD_PH_FLUSH(buf)                                                              \
    if (threadIdx.x == 0 && (buf) != nullptr)                                             \
        for (int k = 0; k < 9; ++k) atomicAdd(&(buf)[k], (unsigned long long)ph[k]);
#else
#define NNSEMD_PH_DECL
#define NNSEMD_PH(k)
#define NNSEMD_PH_FLUSH(buf)
#endif

namespace nnsemd {
namespace rc {

constexpr int kWave = 64;

// LDS arrays of one pair; I is the index type (int32_t, or uint16_t in the
// compact layout of the point path, where sorted and list share storage).
template <typename I>
struct LdsT {
    double* smass;  // [M] supplier mass (by local index while loading, then by active slot)
    double* cmass;  // [N] consumer mass by local index
    double* ckey;   // [N] FP64 key of (pick, j); after the serve: flow (0 = unserved)
    float* srec;    // [M * RS] active supplier records, compacted
    I* sidx;        // [M] local index of active supplier slot
    I* scnt;        // [M] claimant count by active slot
    I* soff;        // [M] bucket start, then bucket end, by active slot
    I* cact;        // [N] active consumers, compacted, ascending
    I* cnn;         // [N] pick (active slot) by consumer; after the serve: supplier local index
    I* list;        // [N] near-tie consumers during the search; claimant buckets after
    I* sorted;      // [N] claimant buckets in serve order (the list's storage when compact)
    float* xl;      // [M * cd] supplier coordinates by local index (coordinate variant only)
    float* yl;      // [N * cd] consumer coordinates by local index (coordinate variant only)
    const int32_t* jmap;  // [N] caller's consumer index of each local one (null: the same)
};
using Lds = LdsT<int32_t>;
using Lds16 = LdsT<uint16_t>;

constexpr int kMaxWaves = 8;    // workgroups of up to 512 threads
constexpr int kMaxReduce = 17;  // values per block reduction (3 + 2d, d <= 7)
static_assert(sizeof(double) * kMaxWaves * kMaxReduce == kPairRedBytes, "reduction scratch size");

// Static LDS of a workgroup: scan scratch and counters.  The block
// reductions' scratch (kMaxWaves x kMaxReduce doubles) is passed separately:
// Shared carries one, the compact point path lends its FP64 key array.
struct SharedCore {
    unsigned long long scan[kMaxWaves];
    unsigned long long tie_nn;     // near-tie counters of the pair (LDS atomics: hits are rare,
    unsigned long long tie_order;  // and no register is held across the rounds for them)
    int32_t nflag;  // near-tie consumers of the search
    int32_t namb;   // claimants whose serve order needs exact keys (high-dimensional path)
};
struct Shared : SharedCore {
    double red[kMaxWaves][kMaxReduce];
};

template <typename I>
__device__ inline LdsT<I> carve_t(char* base, const PairLdsLayout& L) {
    LdsT<I> s;
    s.smass = reinterpret_cast<double*>(base + L.smass);
    s.cmass = reinterpret_cast<double*>(base + L.cmass);
    s.ckey = reinterpret_cast<double*>(base + L.ckey);
    s.srec = reinterpret_cast<float*>(base + L.srec);
    s.sidx = reinterpret_cast<I*>(base + L.sidx);
    s.scnt = reinterpret_cast<I*>(base + L.scnt);
    s.soff = reinterpret_cast<I*>(base + L.soff);
    s.cact = reinterpret_cast<I*>(base + L.cact);
    s.cnn = reinterpret_cast<I*>(base + L.cnn);
    s.list = reinterpret_cast<I*>(base + L.list);
    s.sorted = reinterpret_cast<I*>(base + L.sorted);
    s.xl = reinterpret_cast<float*>(base + L.xl);
    s.yl = reinterpret_cast<float*>(base + L.yl);
    s.jmap = nullptr;
    return s;
}

__device__ inline Lds carve(char* base, int M, int N, int rs, int cd = 0) {
    return carve_t<int32_t>(base, pair_lds_layout(M, N, rs, cd));
}

__device__ inline Lds16 carve16(char* base, int M, int N, int rs, int cd, bool share) {
    return carve_t<uint16_t>(base, pair_lds_layout(M, N, rs, cd, true, share));
}

// Claimant counter increment; returns the count before it.  16-bit counters
// take a 32-bit atomic on their word (counts stay below 2^16, so nothing
// carries into the neighbouring counter).
__device__ inline int cnt_add(int32_t* a, int s) { return atomicAdd(&a[s], 1); }
__device__ inline int cnt_add(uint16_t* a, int s) {
    unsigned* w = reinterpret_cast<unsigned*>(a) + (s >> 1);
    const int sh = (s & 1) * 16;
    return (int)((atomicAdd(w, 1u << sh) >> sh) & 0xffffu);
}

__device__ inline double dist_of_key(double key, int metric) {
    return metric == NNSEMD_L2 ? sqrt(key) : key;
}

// Near tie of two distances d1 <= d2 (FP64): a gap of at most 1e-6 relative,
// or at most 1e-12 when d1 is 0.
__device__ inline bool near_tie_dist(double d1, double d2) {
    const double gap = d2 - d1;
    return d1 == 0.0 ? gap <= 1e-12 : gap <= 1e-6 * d1;
}

// Near tie of two keys k1 <= k2 (L2: of their square roots).  For L2 the
// key-space test first rejects every pair whose distances are more than
// (2e-6 + 1e-12) apart relative, so square roots are taken only for the few
// candidates; the decision itself is always the one on distances.
__device__ inline bool keys_near(double k1, double k2, int metric) {
    if (metric == NNSEMD_L2 && k2 - k1 > 2.1e-6 * k1 + 1e-24) return false;
    return near_tie_dist(dist_of_key(k1, metric), dist_of_key(k2, metric));
}

// Width, in FP32 key units, of the window past the proven search bound in
// which two keys may still be a near tie.  Squared keys: the distances'
// relative gap 1e-6 is a key gap of at most (2e-6 + 1e-12) of the smaller
// squared distance (2.2e-6 bounds it with room for the FP32 roundings); L1
// keys are distances (1.1e-6).  kmax bounds the larger true key; the 1e-12
// covers the absolute rule at zero distance.
__device__ inline float near_window(float kmax, bool l1) {
    return (l1 ? 1.1e-6f : 2.2e-6f) * fmaxf(kmax, 0.f) + 1e-12f;
}

// SplitMix64 output function of the counter (seed, round, consumer): the
// random protocol's serve order key.
__device__ inline uint64_t rp_key(uint64_t seed, int64_t round, int32_t j) {
    uint64_t ctr = ((uint64_t)round << 32) ^ (uint64_t)(uint32_t)j;
    uint64_t z = seed + (ctr + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// One DPP move of a 64-bit value (both halves); lanes without a source, or
// in rows the row mask leaves out, read 0.
template <int CTRL, int ROWS>
__device__ inline unsigned long long dpp_u64(unsigned long long x) {
    const int lo = (int)(unsigned)(x & 0xffffffffull), hi = (int)(unsigned)(x >> 32);
    const unsigned rlo = (unsigned)__builtin_amdgcn_update_dpp(0, lo, CTRL, ROWS, 0xf, false);
    const unsigned rhi = (unsigned)__builtin_amdgcn_update_dpp(0, hi, CTRL, ROWS, 0xf, false);
    return ((unsigned long long)rhi << 32) | rlo;
}

// Inclusive scan over the 64 lanes of a wavefront with DPP moves: shifts by
// 1, 2, 4, 8 within 16-lane rows, then lane 15's total added to rows 1 and
// 3 and lane 31's to rows 2 and 3.  No LDS traffic (a shuffle is an LDS
// permute).  Every lane of the wavefront must be active.
__device__ inline unsigned long long wave_incl_scan_u64(unsigned long long x) {
    x += dpp_u64<0x111, 0xf>(x);  // row_shr:1
    x += dpp_u64<0x112, 0xf>(x);  // row_shr:2
    x += dpp_u64<0x114, 0xf>(x);  // row_shr:4
    x += dpp_u64<0x118, 0xf>(x);  // row_shr:8
    x += dpp_u64<0x142, 0xa>(x);  // row_bcast:15
    x += dpp_u64<0x143, 0xc>(x);  // row_bcast:31
    return x;
}

// Exclusive block scan of one 64-bit value per thread; *total = block sum.
template <int T>
__device__ inline unsigned long long block_scan_u64(unsigned long long v, unsigned long long* total,
                                                    SharedCore& sh) {
    static_assert(T / kWave <= kMaxWaves, "workgroup too large for the scan scratch");
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    unsigned long long x = wave_incl_scan_u64(v);
    if (lane == kWave - 1) sh.scan[w] = x;
    __syncthreads();
    unsigned long long off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < T / kWave; ++k) {
        unsigned long long s = sh.scan[k];
        off += (k < w) ? s : 0ull;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + x - v;
}

// Block-wide reduction of K values per thread (op 0 = sum, 1 = min, 2 = max),
// deterministic (fixed butterfly + fixed wave order).  Results in out[].
template <int T, int K>
__device__ inline void block_reduce(double (&v)[K], const int (&op)[K], double* scratch) {
    double(*red)[kMaxReduce] = reinterpret_cast<double(*)[kMaxReduce]>(scratch);
    static_assert(T / kWave <= kMaxWaves && K <= kMaxReduce, "reduction scratch too small");
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) {
            double y = __shfl_xor(v[k], o);
            v[k] = op[k] == 0 ? v[k] + y : (op[k] == 1 ? fmin(v[k], y) : fmax(v[k], y));
        }
        if (lane == 0) red[w][k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double r = red[0][k];
#pragma unroll
        for (int q = 1; q < T / kWave; ++q) {
            double y = red[q][k];
            r = op[k] == 0 ? r + y : (op[k] == 1 ? fmin(r, y) : fmax(r, y));
        }
        v[k] = r;
    }
    __syncthreads();
}

// FP32 search key of record `rec` for consumer y (see file comment).
template <int RS>
__device__ inline void load_rec(const float* __restrict__ base, int s, float (&r)[RS]) {
    const float4* p = reinterpret_cast<const float4*>(base + (size_t)s * RS);
#pragma unroll
    for (int q = 0; q < RS / 4; ++q) {
        float4 v = p[q];
        r[4 * q + 0] = v.x;
        r[4 * q + 1] = v.y;
        r[4 * q + 2] = v.z;
        r[4 * q + 3] = v.w;
    }
}

template <int RS>
__device__ inline void store_rec(float* __restrict__ base, int s, const float (&r)[RS]) {
    float4* p = reinterpret_cast<float4*>(base + (size_t)s * RS);
#pragma unroll
    for (int q = 0; q < RS / 4; ++q)
        p[q] = make_float4(r[4 * q + 0], r[4 * q + 1], r[4 * q + 2], r[4 * q + 3]);
}


// ---- claimant sets a_i: scan the counts, scatter the claimants
template <int T, typename LT>
__device__ inline void round_buckets(const LT& L, SharedCore& sh, int mact, int nact) {
    const int tid = threadIdx.x;
    {
        const int cs = (mact + T - 1) / T;
        const int lo = min(tid * cs, mact), hi = min(lo + cs, mact);
        int sum = 0;
        for (int s = lo; s < hi; ++s) sum += L.scnt[s];
        unsigned long long tot;
        int run = (int)block_scan_u64<T>((unsigned long long)sum, &tot, sh);
        for (int s = lo; s < hi; ++s) {
            L.soff[s] = run;
            run += L.scnt[s];
        }
    }
    __syncthreads();
    for (int q = tid; q < nact; q += T) {
        const int j = L.cact[q];
        const int pos = cnt_add(L.soff, L.cnn[j]);
        L.list[pos] = j;
    }
    __syncthreads();
}

// ---- claimant order: each claimant counts the bucket members that precede
// it and writes itself to that rank; no dependent chains.  When the serve
// order shares the buckets' storage (compact layout), every rank is taken
// first (at most CS claimants per thread, kept in registers) and written
// after a barrier.  With `ties_order` (greedy order, exact FP64 keys) the
// same scan keeps the largest key below the claimant's -- its neighbour's
// in the serve order over the whole bucket -- and counts the pair when the
// two distances are a near tie.
template <typename LT>
__device__ inline int claimant_place(const LT& L, int j, int protocol, uint64_t seed, int rounds, int metric,
                                     unsigned long long* ties_order) {
    const int sl = L.cnn[j];
    const int c = L.scnt[sl];
    const int end = L.soff[sl];
    const int start = end - c;
    int rank = 0;
    if (c > 1) {
        if (protocol == NNSEMD_GREEDY) {
            const double k = L.ckey[j];
            double pk = -1.0;  // keys are >= +0: -1 = no predecessor
#pragma unroll 4
            for (int e = start; e < end; ++e) {
                const int j2 = L.list[e];
                const double k2 = L.ckey[j2];
                const bool below = (k2 < k) || (k2 == k && j2 < j);
                rank += below;
                if (below && k2 > pk) pk = k2;
            }
            if (ties_order != nullptr && pk >= 0.0 && keys_near(pk, k, metric)) atomicAdd(ties_order, 1ull);
        } else {
            // the random order is drawn for the caller's consumer indices
            const uint64_t k = rp_key(seed, rounds, L.jmap != nullptr ? L.jmap[j] : j);
#pragma unroll 4
            for (int e = start; e < end; ++e) {
                const int j2 = L.list[e];
                const uint64_t k2 = rp_key(seed, rounds, L.jmap != nullptr ? L.jmap[j2] : j2);
                rank += (k2 < k) || (k2 == k && j2 < j);
            }
        }
    }
    return start + rank;
}

template <int T, int CS = 1, typename LT>
__device__ inline void round_rank(const LT& L, int nact, int protocol, uint64_t seed, int rounds, int metric = 0,
                                  unsigned long long* ties_order = nullptr) {
    if (L.sorted == L.list) {
        int pos[CS], jv[CS];
#pragma unroll
        for (int u = 0; u < CS; ++u) {
            const int q = threadIdx.x + u * T;
            pos[u] = -1;
            jv[u] = 0;
            if (q < nact) {
                jv[u] = L.cact[q];
                pos[u] = claimant_place(L, jv[u], protocol, seed, rounds, metric, ties_order);
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < CS; ++u)
            if (pos[u] >= 0) L.sorted[pos[u]] = jv[u];
    } else {
        for (int q = threadIdx.x; q < nact; q += T) {
            const int j = L.cact[q];
            L.sorted[claimant_place(L, j, protocol, seed, rounds, metric, ties_order)] = j;
        }
    }
    __syncthreads();
}

// ---- flow & cost: one lane per claimed supplier walks its ordered
// claimants while it still holds mass.  A served claimant records the local
// index of its supplier (for the plan) and its flow in place of its key; an
// unserved one gets flow 0.  With NEGF (every key is >= +0 when the walk
// starts) the flow is stored negated and unserved claimants keep their keys,
// so the walk never visits the unserved part of a bucket (one serve can
// exhaust a supplier with thousands of claimants); round_compact must then be
// told the same.  With COST (the keys are the exact FP64 keys), `cost`
// accumulates this thread's part of R; without it, R is left to the caller.
template <int T, bool COST = true, bool NEGF = false, typename LT>
__device__ inline void round_walk(const LT& L, int mact, int metric, double& cost) {
    for (int s = threadIdx.x; s < mact; s += T) {
        const int c = L.scnt[s];
        if (c == 0) continue;
        const int end = L.soff[s];
        const int start = end - c;
        const int isup = L.sidx[s];
        int pos = start;
        double sm = L.smass[s];
        while (pos < end && sm > 0.0) {
            const int j = L.sorted[pos];
            const double cm = L.cmass[j];
            const double f = sm < cm ? sm : cm;
            sm = sm - f;
            L.cmass[j] = cm - f;
            if constexpr (COST) cost = cost + f * dist_of_key(L.ckey[j], metric);
            L.ckey[j] = NEGF ? -f : f;
            L.cnn[j] = isup;
            ++pos;
        }
        if constexpr (!NEGF)
            for (int e = pos; e < end; ++e) L.ckey[L.sorted[e]] = 0.0;
        L.smass[s] = sm;
    }
    __syncthreads();
}

// ---- weights update: plan append + compaction of the active sets (and of
// the RS-float search records when RS > 0), one scan for all three streams.
template <int T, int CSMAX, int RS, bool NEGF = false, typename LT>
__device__ inline void round_compact(const LT& L, SharedCore& sh, int& mact, int& nact, int64_t& nnz,
                                     int32_t* plan_src, int32_t* plan_dst, double* plan_flow, int64_t plan_base) {
    constexpr int RSA = RS > 0 ? RS : 4;
    const int tid = threadIdx.x;
    const int pc = (nact + T - 1) / T;
    const int plo = min(tid * pc, nact), phi = min(plo + pc, nact);
    // this thread's claimants in serve order and their flows (pc <= CSMAX),
    // read once for the count and the plan append (kept in registers for up
    // to four per thread)
    constexpr int PK = CSMAX <= 4 ? CSMAX : 1;
    int pj[PK];
    double pf[PK];
    int kp = 0;
    if constexpr (CSMAX <= 4) {
#pragma unroll
        for (int u = 0; u < CSMAX; ++u) {
            const int k = plo + u;
            pj[u] = k < phi ? (int)L.sorted[k] : 0;
            pf[u] = k < phi ? L.ckey[pj[u]] : 0.0;
            if constexpr (NEGF) pf[u] = pf[u] < 0.0 ? -pf[u] : 0.0;
            kp += pf[u] > 0.0;
        }
    } else {
        for (int k = plo; k < phi; ++k) kp += NEGF ? L.ckey[L.sorted[k]] < 0.0 : L.ckey[L.sorted[k]] > 0.0;
    }
    const int cs = (mact + T - 1) / T;
    const int slo = min(tid * cs, mact);
    float rec[CSMAX][RSA];
    double smv[CSMAX];
    int sid[CSMAX], cid[CSMAX];
    int ks = 0, kc2 = 0;
#pragma unroll
    for (int u = 0; u < CSMAX; ++u) {
        const int s = slo + u;
        sid[u] = -1;
        smv[u] = 0.0;
        if (u < cs && s < mact) {
            smv[u] = L.smass[s];
            if (smv[u] > 0.0) {
                sid[u] = L.sidx[s];
                if constexpr (RS > 0) load_rec<RS>(L.srec, s, rec[u]);
                ++ks;
            }
        }
        const int q = plo + u;
        cid[u] = -1;
        if (u < pc && q < nact) {
            const int j = L.cact[q];
            if (L.cmass[j] > 0.0) {
                cid[u] = j;
                ++kc2;
            }
        }
    }
    unsigned long long tot;
    const unsigned long long pre = block_scan_u64<T>(
        (unsigned long long)kp | ((unsigned long long)ks << 21) | ((unsigned long long)kc2 << 42), &tot, sh);
    const unsigned long long mask = (1ull << 21) - 1;
    int wp = (int)(pre & mask), ws = (int)((pre >> 21) & mask), wc = (int)(pre >> 42);
    if (plan_src != nullptr) {
        if constexpr (CSMAX <= 4) {
#pragma unroll
            for (int u = 0; u < CSMAX; ++u) {
                if (pf[u] > 0.0) {
                    const int j = pj[u];
                    const int64_t e = plan_base + nnz + wp;
                    plan_src[e] = L.cnn[j];
                    plan_dst[e] = L.jmap != nullptr ? L.jmap[j] : j;
                    plan_flow[e] = pf[u];
                    ++wp;
                }
            }
        } else {
            for (int k = plo; k < phi; ++k) {
                const int j = L.sorted[k];
                const double f = NEGF ? -L.ckey[j] : L.ckey[j];
                if (f > 0.0) {
                    const int64_t e = plan_base + nnz + wp;
                    plan_src[e] = L.cnn[j];
                    plan_dst[e] = L.jmap != nullptr ? L.jmap[j] : j;
                    plan_flow[e] = f;
                    ++wp;
                }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < CSMAX; ++u) {
        if (sid[u] >= 0) {
            if constexpr (RS > 0) store_rec<RS>(L.srec, ws, rec[u]);
            L.sidx[ws] = sid[u];
            L.smass[ws] = smv[u];
            L.scnt[ws] = 0;
            ++ws;
        }
        if (cid[u] >= 0) L.cact[wc++] = cid[u];
    }
    nnz += (int64_t)(tot & mask);
    mact = (int)((tot >> 21) & mask);
    nact = (int)(tot >> 42);
    if (tid == 0) sh.nflag = 0;
    __syncthreads();
}

}  // namespace rc
}  // namespace nnsemd
