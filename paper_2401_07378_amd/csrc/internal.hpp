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
    int32_t split;         // search: lanes per consumer = largest power of two with nact * lanes * split <= threads
    int32_t share_order;   // LDS layout: the serve order written over the claimant buckets
};

// Byte layout of the dynamic LDS of one workgroup (one pair at a time).
struct PairLdsLayout {
    size_t smass, cmass, ckey, srec, sidx, scnt, soff, cact, cnn, list, sorted, xl, yl, total;
};

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// cd > 0: also the pair's coordinates, cd floats per point (suppliers then
// consumers, by local index), so the rounds never read them from HBM.
// compact (point path): 16-bit index arrays (even lengths, 4-byte aligned,
// so a packed 32-bit counter atomic stays inside its array) and the FP64 key
// array at least kPairRedBytes long: it is the block reductions' scratch
// outside the rounds.  share (compact only): the serve order is written over
// the claimant buckets (one more barrier per round, 2 bytes less per
// consumer).
constexpr size_t kPairRedBytes = 8 * 17 * 8;
__host__ __device__ inline PairLdsLayout pair_lds_layout(int M, int N, int rs, int cd = 0, bool compact = false,
                                                         bool share = true) {
    PairLdsLayout L;
    const size_t isz = compact ? 2 : 4;
    const size_t Me = compact ? (size_t)((M + 1) & ~1) : (size_t)M;
    const size_t Ne = compact ? (size_t)((N + 1) & ~1) : (size_t)N;
    size_t o = 0;
    L.smass = o; o += sizeof(double) * (size_t)M;
    L.cmass = o; o += sizeof(double) * (size_t)N;
    L.ckey = o;  o += compact && sizeof(double) * (size_t)N < kPairRedBytes ? kPairRedBytes : sizeof(double) * (size_t)N;
    o = align_up(o, 16);
    L.srec = o;  o += sizeof(float) * (size_t)rs * (size_t)M;
    o = align_up(o, 4);
    L.sidx = o;  o += isz * Me;
    L.scnt = o;  o += isz * Me;
    L.soff = o;  o += isz * Me;
    L.cact = o;  o += isz * Ne;
    L.cnn = o;   o += isz * Ne;
    L.list = o;  o += isz * Ne;
    if (compact && share) {
        L.sorted = L.list;
    } else {
        L.sorted = o; o += isz * Ne;
    }
    o = align_up(o, 16);
    L.xl = o;    o += sizeof(float) * (size_t)cd * (size_t)M;
    L.yl = o;    o += sizeof(float) * (size_t)cd * (size_t)N;
    L.total = align_up(o, 16);
    return L;
}

// ---------------------------------------------------------------------
// Multi-workgroup path for one pair of any size (large_pair.hip).
struct LPState {
    int32_t status, mact, nact, nflag;
    int64_t nnz, work, near;
    int64_t ties_nn, ties_order;  // near-tie counters (see nnsemd_stats_t)
    int32_t rounds, done, parity, ticket;  // ticket: blocks of the round's last kernel that have finished
    int32_t tail, pad2;  // tail: both active sets fit the single-workgroup finish
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
    double* tkey;        // near-tie bin tables, by bucket position: FP64 key,
    int32_t* thead;      //   chain heads (-1 = empty; all -1 between rounds)
    int32_t* tnext;      //   and chain links
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
    int32_t tail_cap;  // active points per side at which the single-workgroup finish takes over (0: never)
    int32_t tail_pad;
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
// The single-workgroup finish: its largest capacity per side that fits
// max_lds bytes of LDS (0 if none), and its launch.
int lp_tail_capacity(int d, size_t max_lds);
int lp_launch_tail(const LPArgs& A, int d, void* stream);

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
    double* xnorm;         // split form: FP64 squared norms of the supplier sets' rows,
                           // [set * max_m + i], NaN for a row with a non-finite coordinate
    int4* stripes;         // split form, one supplier set for every pair: the launch's stripe
                           // records (nullptr: the per-pair tile kernel runs instead)
    int32_t* stripe_total; // its length (written by the list kernel)
    int32_t tile_grid;     // workgroups of the shared-query tile kernel
    int32_t pad2;
};

size_t doc_lds_bytes(int max_m, int max_n, bool fp32_points);
// Whether a launch takes the split form (tile kernel + rounds kernel), and
// the supplier-set norm pass it needs first (A.xnorm: num_x_sets * max_m).
bool doc_split_form(int d, bool bf16_mfma, int chunk_max);
int launch_doc_xnorm(const DocArgs& A, void* stream);
// LDS bytes of the shared-query tile kernel (the query staged whole), and
// its resident workgroups per CU (0 if it does not fit).
size_t doc_shared_tile_lds(int max_m);
int doc_shared_tile_occupancy(int max_m);
int doc_shared_tile_threads();
// Scratch slot of one workgroup: the m x n FP32 key tile (256-byte aligned,
// rows of doc_tile_ld(n) columns)
// followed by m + n plan entries (int32 src, int32 dst, double flow).
// Tile row stride: the columns padded to a multiple of 16, so that the
// 64-byte row segment of one 16-consumer stripe is one aligned 64-byte block.
__host__ __device__ inline int doc_tile_ld(int n) { return (n + 15) & ~15; }
__host__ __device__ inline size_t doc_tile_bytes(int max_m, int max_n) {
    return align_up(sizeof(float) * (size_t)max_m * (size_t)doc_tile_ld(max_n), 256);
}
// After the plan area, the results of the separate tile kernel: xx[M],
// yy[N], first-round best b1[N], second best b2[N] (FP32), best local index
// bs[N] (int32), and a flag (non-finite coordinate seen).
__host__ __device__ inline size_t doc_aux_offset(int max_m, int max_n) {
    return doc_tile_bytes(max_m, max_n) + align_up(16 * ((size_t)max_m + (size_t)max_n), 256);
}
__host__ __device__ inline size_t doc_slot_bytes(int max_m, int max_n) {
    return doc_aux_offset(max_m, max_n) + align_up(4 * ((size_t)max_m + 4 * (size_t)max_n) + 16, 256);
}
// blocks == nullptr: launch; else query resident workgroups per CU.
// allow_split = false takes the fused form even where the split one exists.
int launch_doc_solver(const DocArgs& A, bool bf16_mfma, int chunk_max, size_t lds, int grid, void* stream,
                      int* blocks, bool allow_split = true);

// ---------------------------------------------------------------------
// Deep-sets EMD surrogate (surrogate.hip).  Flat FP32 parameter layout:
// W1 (H x 3), b1 (H), W2 (H x H), b2 (H), W3 (H x 3H), b3 (H), w4 (H), b4.
constexpr int kSgHidden = 256;
constexpr int64_t kSgW1 = 0;
constexpr int64_t kSgB1 = kSgW1 + 3 * kSgHidden;
constexpr int64_t kSgW2 = kSgB1 + kSgHidden;
constexpr int64_t kSgB2 = kSgW2 + (int64_t)kSgHidden * kSgHidden;
constexpr int64_t kSgW3 = kSgB2 + kSgHidden;
constexpr int64_t kSgB3 = kSgW3 + (int64_t)kSgHidden * 3 * kSgHidden;
constexpr int64_t kSgW4 = kSgB3 + kSgHidden;
constexpr int64_t kSgB4 = kSgW4 + kSgHidden;
constexpr int64_t kSgParams = kSgB4 + 1;
constexpr int kSgHbCols = 2 * kSgHidden + 8;  // head-backward row: dg | dt*g | dt | r^2/B | pad
constexpr int kSgTopkMax = 1024;

namespace sg {
// BF16 (and BF16-rounded FP32) copies of the weights used by the kernels.
struct SgQuant {
    float* W1;      // H x 3, rounded
    float* w4;      // H, rounded
    uint16_t* W2;   // H x H   [out][in]
    uint16_t* W2T;  // H x H   [in][out]
    uint16_t* W3;   // H x 3H  [out][in]
    uint16_t* W3T;  // 3H x H  [in][out]
};
struct SgPredictWork {
    uint16_t* Z;  // Bpad x 3H
    float* PRE3;  // B x H
};
struct SgTrainWork {
    uint16_t *H1q, *H1qT, *dP2q, *dP2qT;  // Ppad x H and H x Ppad
    float *PRE2, *dH1;                    // P x H
    float *E, *dE;                        // 2B x H
    uint16_t *Z, *ZT, *dGq, *dGqT;        // Bpad x 3H, 3H x Bpad, Bpad x H, H x Bpad
    float *PRE3, *dZ, *HB, *hsum, *t, *pred, *db2p, *split, *l1p, *l1s;
    int* bad;  // offsets check
};
int launch_prepare(const float* theta, const SgQuant& q, void* stream);
int launch_embed(const float* theta, const SgQuant& q, const float* X, const float* a, const int64_t* set_off,
                 int64_t num_sets, int64_t num_points, float* E, void* stream);
int launch_predict(const float* theta, const SgQuant& q, const float* Eq, int64_t nq, const float* Ec, int64_t nc,
                   const int32_t* qi, const int32_t* ci, int train_layout, int64_t B, const SgPredictWork& w,
                   float* t_out, float* pred, void* stream);
int launch_loss_grad(const float* theta, const SgQuant& q, const float* X, const float* a, const int64_t* set_off,
                     int64_t B, int64_t P, const float* labels, const SgTrainWork& w, float* loss, float* grad,
                     void* stream);
int launch_adam(float* theta, float* m, float* v, const float* grad, float lr, double beta1, double beta2, float eps,
                float bc1, float bc2, void* stream);
// ws: topk_ws_bytes() of device scratch (nullable: single-workgroup scan only).
size_t topk_ws_bytes();
int launch_topk_f32(const float* vals, int64_t n, int k, int32_t* out, void* ws, void* stream);
int launch_topk_f64(const double* vals, int64_t n, int k, int32_t* out, void* ws, void* stream);
int launch_gather_ranked(const int32_t* pos, const int32_t* sel, const double* vals, int k, int32_t* out_idx,
                         double* out_val, void* stream);
int launch_fill_i32(int32_t* p, int64_t n, int32_t v, void* stream);
int launch_two_offsets(int64_t* off, int64_t m, void* stream);
}  // namespace sg

// ---------------------------------------------------------------------
// Given ground-distance matrices (cost_solver.hip): one workgroup per pair.
struct CostArgs {
    int64_t num_pairs;
    const void* D;          // FP32 or FP64 entries, pair p row-major m_p x n_p
    const int64_t* d_off;   // num_pairs + 1 entry offsets; nullptr: single pair, or
                            // pair p at (p - pair_base) * d_stride when d_stride > 0
    int64_t d_stride;
    int64_t pair_base;      // workgroup b solves pair pair_base + b (no order table)
    const float* a;
    const int64_t* a_off;   // supplier set offsets, or nullptr (single pair)
    const float* b;
    const int64_t* b_off;   // consumer set offsets, or nullptr
    const int32_t* pair_x;  // nullable: pair p uses supplier set pair_x[p] (else p)
    const int32_t* pair_y;  // nullable: consumer set pair_y[p] (else p)
    int64_t num_a_sets;
    int64_t num_b_sets;
    int64_t single_m;
    int64_t single_n;
    int32_t max_m;          // LDS capacity of this launch
    int32_t max_n;
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
    const int32_t* order;   // nullable: workgroup b solves pair order[b]
};
// blocks != nullptr: occupancy query only.
int launch_cost_solver(const CostArgs& A, bool f64, int chunk_max, size_t lds, int grid, void* stream, int* blocks);
// Exact FP64 L1 distance matrices of high-dimensional pairs (BF16 or FP32
// points), in dimension order: pair pair_base + b of the doc arguments into
// tiles + b * tile_stride (FP64, row-major m x n).
int launch_l1_tiles(const DocArgs& A, bool bf16, double* tiles, int64_t tile_stride, int grid, void* stream);

// ---------------------------------------------------------------------
// Barycentric map of a plan (transport_map.hip): per-row buckets of plan
// positions, so every row is summed in plan order.
struct MapWork {
    int32_t* cnt;     // [rows] entries per row
    int32_t* start;   // [rows] bucket start
    int32_t* cursor;  // [rows] scatter cursor
    int32_t* big;     // [rows] rows handled by a wavefront
    int32_t* ent;     // [cap] plan positions by row
    int32_t* nbig;    // [1]
};
size_t map_ws_bytes(int64_t rows, int64_t cap);
MapWork map_ws_carve(char* base, int64_t rows, int64_t cap);
// side 0: rows are suppliers (P = consumer points), 1: rows are consumers.
int launch_barycentric_map(const int32_t* src, const int32_t* dst, const double* flow, int64_t cap,
                           const int64_t* nnz, const float* P, int64_t p_rows, int d, int side, int64_t rows,
                           double* map, const MapWork& w, void* stream);

// ---------------------------------------------------------------------
// Colour transfer application (colour_transfer.hip).
size_t kmeans_lds_bytes(int K);
// K-means palette of P 8-bit RGB pixels (iters update steps, then the final
// assignment): centroids C (K x 3, FP64), sums/counts S (K x 4), assignment,
// palette points (K x 3 FP32) and masses (K FP32).
int launch_kmeans(const uint8_t* px, int64_t P, int K, int iters, double* C, unsigned long long* S,
                  int32_t* assign, float* pts, float* mass, void* stream);
int launch_recolour(const uint8_t* px, const int32_t* assign, int64_t P, const double* T, uint8_t* out,
                    void* stream);

// Launch entry points (defined in pair_solver.hip).
// Returns hipSuccess-compatible int (0 on success).
int launch_pair_solver(const PairSolverArgs& args, int d, int threads, int chunk_max, bool coords,
                       size_t lds_bytes, int grid, void* stream);
int launch_order(const int64_t* x_off, const int64_t* y_off, const int32_t* pair_x, const int32_t* pair_y,
                 int64_t num_pairs, int64_t num_x_sets, int64_t num_y_sets, int32_t* order, void* stream);
// coords: the variant that keeps the pair's coordinates in LDS.
int pair_solver_blocks_per_cu(int d, int metric, int threads, int chunk_max, size_t lds_bytes, int* blocks,
                              bool coords = false);

}  // namespace nnsemd
