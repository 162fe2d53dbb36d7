// Internal declarations shared by the host runtime and the kernels of the
// NNS-EMD library.  Not part of the public ABI (include/nnsemd.h is).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "nnsemd.h"

namespace nnsemd {

// Unit roundoff of FP32 (2^-24).
constexpr float kU32 = 5.9604644775390625e-08f;

// Record stride (floats) of one active supplier in LDS for dimension d:
// Euclidean metrics store (-2 x_0 .. -2 x_{d-1}, ||x||^2), L1 stores x.
__host__ __device__ constexpr int record_stride(int d) { return d + 1 <= 4 ? 4 : 8; }

// Arguments of the per-pair workgroup solver (low-dimensional FP32 points).
struct PairSolverArgs {
    int64_t num_pairs;
    const float* X;
    const float* a;
    const int64_t* x_off;  // nullptr: single pair of single_m rows
    int64_t num_x_sets;
    const float* Y;
    const float* b;
    const int64_t* y_off;
    int64_t num_y_sets;
    const int32_t* pair_x;
    const int32_t* pair_y;
    int64_t single_m;
    int64_t single_n;
    int32_t max_m;  // LDS capacity of this launch
    int32_t max_n;
    int32_t metric;
    int32_t protocol;
    uint64_t seed;
    int64_t max_rounds;  // <= 0: m + n
    double* costs;
    int32_t* plan_src;
    int32_t* plan_dst;
    double* plan_flow;
    const int64_t* plan_off;  // nullptr with a plan: single pair, capacity below
    int64_t single_plan_cap;
    nnsemd_stats_t* stats;
    const int32_t* order;  // nullable: workgroup b solves pair order[b]
    unsigned long long* phase_cycles;  // profiling builds only: 9 per-phase cycle totals
};

// Byte layout of the dynamic LDS of one workgroup (one pair at a time).
struct PairLdsLayout {
    size_t smass, cmass, ckey, srec, sidx, scnt, soff, cact, cnn, list, sorted, total;
};

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

__host__ __device__ inline PairLdsLayout pair_lds_layout(int M, int N, int rs) {
    PairLdsLayout L;
    size_t o = 0;
    L.smass = o; o += sizeof(double) * (size_t)M;
    L.cmass = o; o += sizeof(double) * (size_t)N;
    L.ckey = o;  o += sizeof(double) * (size_t)N;
    o = align_up(o, 16);
    L.srec = o;  o += sizeof(float) * (size_t)rs * (size_t)M;
    L.sidx = o;  o += sizeof(int32_t) * (size_t)M;
    L.scnt = o;  o += sizeof(int32_t) * (size_t)M;
    L.soff = o;  o += sizeof(int32_t) * (size_t)M;
    L.cact = o;  o += sizeof(int32_t) * (size_t)N;
    L.cnn = o;   o += sizeof(int32_t) * (size_t)N;
    L.list = o;  o += sizeof(int32_t) * (size_t)N;
    L.sorted = o; o += sizeof(int32_t) * (size_t)N;
    L.total = align_up(o, 16);
    return L;
}

// ---------------------------------------------------------------------
// Multi-workgroup path for one pair of any size (large_pair.hip).
struct LPState {
    int32_t status, mact, nact, nflag;
    int64_t nnz, work, near;
    int32_t rounds, done, parity, pad0;
    float centre[8];
    float rhat, pad1;
    double sum_a, sum_b;
};

struct LPWork {
    float* srec[2];      // active supplier records by slot (ping-pong)
    int32_t* sidx[2];    // slot -> local supplier index
    double* smass[2];    // slot -> FP64 mass
    int32_t* scnt;       // claimant count by slot
    int32_t* soff;       // bucket start / end by slot
    int32_t* cact[2];    // active consumers (ping-pong)
    double* cmass;       // consumer FP64 mass by local index
    int32_t* cnn;        // pick slot (then supplier local index after the serve)
    double* ckey;        // FP64 key of the pick (then the flow)
    int32_t* list;       // claimant buckets
    int32_t* sorted;     // claimant buckets in serve order
    int32_t* flagged;    // near-tie consumers of the round
    float4* part;        // per (supplier chunk, consumer) FP32 best/second/slot
    int64_t ncap;        // consumer capacity (row stride of part)
    int64_t part_cap;    // entries of part
    unsigned long long* blkcnt;  // per-block packed compaction counts
    int32_t blkcnt_cap;
    int32_t pad;
    double* costacc;     // per supplier (local index) cost, serve order
    double* wsum;        // per supplier outgoing flow (map only; may be null)
    double* bsum;        // per supplier sum f * y (map only)
    double* red;         // ingest partials
    LPState* st;
};

struct LPArgs {
    int64_t m, n;
    const float* X;
    const float* a;
    const float* Y;
    const float* b;
    int32_t metric, protocol;
    uint64_t seed;
    int64_t max_rounds;
    double* cost;
    int32_t* plan_src;
    int32_t* plan_dst;
    double* plan_flow;
    nnsemd_stats_t* stats;
    double* map;  // m x d FP64 barycentric map, or null
    LPWork w;
};

int lp_launch_init(const LPArgs& A, int d, void* stream);
int lp_launch_round(const LPArgs& A, int d, int mact_ub, int nact_ub, void* stream);
int lp_launch_finish(const LPArgs& A, int d, void* stream);

// ---------------------------------------------------------------------
// High-dimensional path (doc_solver.hip): one workgroup per pair, the key
// tile of the pair in a per-workgroup global scratch slot.
struct DocArgs {
    int64_t num_pairs;
    const void* X;  // BF16 bits (uint16) or FP32, row-major, d per point
    const float* a;
    const int64_t* x_off;  // nullptr: single pair of single_m rows
    int64_t num_x_sets;
    const void* Y;
    const float* b;
    const int64_t* y_off;
    int64_t num_y_sets;
    const int32_t* pair_x;
    const int32_t* pair_y;
    int64_t single_m;
    int64_t single_n;
    int32_t max_m;
    int32_t max_n;
    int32_t d;
    int32_t metric;
    int32_t protocol;
    int32_t pad;
    uint64_t seed;
    int64_t max_rounds;
    double* costs;
    int32_t* plan_src;
    int32_t* plan_dst;
    double* plan_flow;
    const int64_t* plan_off;
    int64_t single_plan_cap;
    nnsemd_stats_t* stats;
    const int32_t* order;  // nullable: workgroup b solves pair order[pair_base + b]
    int64_t pair_base;     // first schedule position of this launch
    char* scratch;         // grid * slot_bytes: per-workgroup key tile, then the plan when none is requested
    int64_t slot_bytes;    // doc_slot_bytes(max_m, max_n)
    unsigned long long* phase_cycles;  // profiling builds only: 9 per-phase cycle totals
};

size_t doc_lds_bytes(int max_m, int max_n);
// Scratch slot of one workgroup: the m x n FP32 key tile (256-byte aligned)
// followed by m + n plan entries (int32 src, int32 dst, double flow).
__host__ __device__ inline size_t doc_tile_bytes(int max_m, int max_n) {
    return align_up(sizeof(float) * (size_t)max_m * (size_t)max_n, 256);
}
__host__ __device__ inline size_t doc_slot_bytes(int max_m, int max_n) {
    return doc_tile_bytes(max_m, max_n) + align_up(16 * ((size_t)max_m + (size_t)max_n), 256);
}
// blocks == nullptr: launch; else query resident workgroups per CU.
int launch_doc_solver(const DocArgs& A, bool bf16_mfma, int chunk_max, size_t lds, int grid, void* stream,
                      int* blocks);

// Launch entry points (defined in pair_solver.hip).
// Returns hipSuccess-compatible int (0 on success).
int launch_pair_solver(const PairSolverArgs& args, int d, int threads, int chunk_max,
                       size_t lds_bytes, int grid, void* stream);
int launch_order(const int64_t* x_off, const int64_t* y_off, const int32_t* pair_x, const int32_t* pair_y,
                 int64_t num_pairs, int64_t num_x_sets, int64_t num_y_sets, int32_t* order, void* stream);
int pair_solver_blocks_per_cu(int d, int metric, int threads, int chunk_max, size_t lds_bytes,
                              int* blocks);

}  // namespace nnsemd
