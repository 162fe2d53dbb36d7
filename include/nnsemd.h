/*
 * nnsemd.h -- C ABI of the MI355X (gfx950) NNS-EMD library.
 *
 * NNS-EMD approximates the Earth Mover's Distance (the transport LP of the
 * paper's Eqs. (1)-(3)) by iterated nearest-neighbour search, Algorithm 1
 * of the paper (Sec. III-A): in every round each active consumer (a point
 * of C = (Y, b)) picks its nearest active supplier (a point of S = (X, a));
 * every supplier serves its claimants nearest-first with
 * f = min(s_i, c_j), adds f * D_ij to the cost R and records F_ij += f;
 * points whose mass reached zero leave the active sets; the rounds repeat
 * until one side is empty.  The method is not symmetric: X/a are always the
 * suppliers that are searched, Y/b the consumers that search.
 *
 * Conventions shared by every call:
 *  - Pointers marked "device" must be device memory of the handle's GPU
 *    (any allocator: hipMalloc, torch, ...); "host" pointers are read during
 *    the call only.  The library never frees caller memory.
 *  - Point sets are row-major (rows x d), FP32 unless a call says
 *    otherwise; masses are FP32 and are promoted exactly to FP64, in which
 *    all mass arithmetic and the cost sum run.
 *  - Calls enqueue work on `stream` (a hipStream_t; NULL = the default
 *    stream) and return at once.  Argument checks that need no device data
 *    happen before anything is enqueued and return a negative status.
 *    Checks of the data itself (non-finite coordinates, negative or
 *    non-finite masses, total masses that differ by more than 1e-5
 *    relative, a plan buffer below m+n-1 entries, a round cap reached) are
 *    reported per pair in nnsemd_stats_t.status once the stream has run;
 *    such a pair's cost is NaN.
 *  - Zero masses are allowed: those points never become active.
 *  - Results are deterministic: identical inputs give bit-identical costs
 *    and plans.  The search runs in FP32 with a proven error bound; any
 *    consumer whose best and second-best FP32 keys are closer than that
 *    bound is re-scored in FP64, so every nearest-neighbour decision and
 *    the whole plan equal those of the FP64 definition (ties: smallest
 *    supplier index; greedy order: (D_ij, j) ascending).
 *  - A handle owns its workspace and must not be used by two host threads
 *    at once; calls on one handle must be ordered on one stream.
 *  - No C++ exception crosses this interface.
 */
#ifndef NNSEMD_H
#define NNSEMD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nnsemd_handle* nnsemd_handle_t;

typedef enum {
    NNSEMD_OK = 0,
    NNSEMD_ERR_INVALID_ARG = -1,   /* bad pointer, size, enum or data value */
    NNSEMD_ERR_MASS_MISMATCH = -2, /* |sum a - sum b| > 1e-5 max(sum a, sum b) */
    NNSEMD_ERR_CAPACITY = -3,      /* plan buffer smaller than m + n - 1 */
    NNSEMD_ERR_OUT_OF_MEMORY = -4, /* workspace allocation failed */
    NNSEMD_ERR_DEVICE = -5,        /* a HIP runtime call failed */
    NNSEMD_ERR_NOT_CONVERGED = -6, /* the round cap was reached */
    NNSEMD_ERR_UNSUPPORTED = -7    /* combination not implemented */
} nnsemd_status_t;

/* Ground distance D_ij (Sec. II-A uses L1 and L2; Table 8b compares them). */
typedef enum {
    NNSEMD_L2 = 0,          /* D = ||x - y||_2; search and order by ||x - y||^2 */
    NNSEMD_SQEUCLIDEAN = 1, /* D = ||x - y||_2^2 */
    NNSEMD_L1 = 2           /* D = ||x - y||_1 */
} nnsemd_metric_t;

/* Element type of points (F32, BF16) or of a given distance matrix (F32, F64). */
typedef enum { NNSEMD_F32 = 0, NNSEMD_BF16 = 1, NNSEMD_F64 = 2 } nnsemd_dtype_t;

/* Flow protocol of Sec. III-A: greedy serves claimants nearest-first (ties
 * by consumer index); random serves them in the order of the SplitMix64
 * output of the counter (seed, round, consumer), see nnsemd_options_t. */
typedef enum { NNSEMD_GREEDY = 0, NNSEMD_RANDOM = 1 } nnsemd_protocol_t;

/* Arithmetic of the distance search.  FP32 (FP32 points): FP32 keys on the
 * vector ALUs.  BF16_MFMA_REFINE (BF16 points): the key tile
 * ||x||^2 - 2 x.y of a pair from BF16 matrix-core products with FP32
 * accumulation.  In both modes a consumer whose two best FP32 keys are
 * closer than the proven FP32 error bound is re-scored in FP64 from the
 * inputs, so every argmin and every serve order is the one of the FP64
 * definition (ties to the smallest index) and the cost is summed in FP64.
 * Cost terms: FP32 mode recomputes every served distance in FP64.
 * BF16_MFMA_REFINE with d <= 320 and sides <= 1024 takes a served distance
 * from its key when the key's error bound makes the term accurate to 1e-5
 * relative.  Where that fails for any term of a pair, it recomputes every
 * distance of the pair in FP64.  The cost is then within 1e-5 relative of
 * the definition's (Sec. III-A: R sums flow times distance), inside the
 * 1e-3 allowed for this mode. */
typedef enum { NNSEMD_MODE_FP32 = 0, NNSEMD_MODE_BF16_MFMA_REFINE = 1 } nnsemd_mode_t;

/* Order in which a batched call starts its pairs (results do not depend on
 * it): longest first by m * n, or as given. */
typedef enum { NNSEMD_SCHEDULE_LONGEST_FIRST = 0, NNSEMD_SCHEDULE_AS_GIVEN = 1 } nnsemd_schedule_t;

/* Which implementation solves a single pair: automatic (on-chip whenever the
 * pair fits one workgroup's LDS), the on-chip one-workgroup path, or the
 * multi-workgroup path (any size; its host thread waits for the result).
 * The multi-workgroup path hands the last rounds, once both active sets fit
 * one workgroup's LDS, to a single-workgroup finish; MULTI_NO_TAIL runs
 * every round grid-wide (same results; for tests and comparisons). */
typedef enum {
    NNSEMD_PATH_AUTO = 0,
    NNSEMD_PATH_ON_CHIP = 1,
    NNSEMD_PATH_MULTI = 2,
    NNSEMD_PATH_MULTI_NO_TAIL = 3
} nnsemd_path_t;

typedef struct {
    int32_t protocol;   /* nnsemd_protocol_t, default NNSEMD_GREEDY */
    int32_t mode;       /* nnsemd_mode_t, default NNSEMD_MODE_FP32 */
    int64_t max_rounds; /* <= 0: m + n (never reached by valid input) */
    uint64_t seed;      /* random protocol only */
    int32_t threads;    /* workgroup size override (0 = tuned choice) */
    int32_t schedule;   /* nnsemd_schedule_t, default longest first */
    int32_t path;       /* nnsemd_path_t (single pairs), default automatic */
    int32_t reserved;   /* must be 0 */
} nnsemd_options_t;

/* Per-pair results, written by the device (64 bytes).
 * A near tie is a gap of at most 1e-6 relative between two distances D
 * (second - first <= 1e-6 * first, or <= 1e-12 when first is 0), evaluated
 * in FP64 on the exact keys.  Both counters are those of a plain FP64 run
 * of Algorithm 1 on the same inputs, whatever the search precision. */
typedef struct {
    int32_t status;          /* nnsemd_status_t of this pair */
    int32_t rounds;          /* NNS iterations t */
    int64_t nnz;             /* plan entries (serves), <= m + n - 1 */
    int64_t work;            /* sum over rounds of |active S| * |active C| */
    int64_t rescored;        /* consumer searches settled by an FP64 re-score
                                (the FP32 keys were closer than their proven
                                error bound or a near-tie window) */
    double residual_src;     /* supplier mass left when the rounds stopped */
    double residual_dst;     /* consumer mass left when the rounds stopped */
    int64_t near_ties_nn;    /* NNS step: active consumers (with >= 2 active
                                suppliers) whose nearest and second-nearest
                                suppliers are a near tie, summed over rounds */
    int64_t near_ties_order; /* greedy protocol: neighbouring claimants of a
                                supplier, in serve order, that are a near tie,
                                summed over suppliers and rounds (0 under the
                                random protocol) */
} nnsemd_stats_t;

/* Create a handle on HIP device `device` (its workspace grows on demand).
 * Returns INVALID_ARG for a NULL `out` or a bad device index. */
nnsemd_status_t nnsemd_create(nnsemd_handle_t* out, int32_t device);

/* Free the handle and its workspace (waits for the device to be idle). */
nnsemd_status_t nnsemd_destroy(nnsemd_handle_t h);

/* Static description of a status code. */
const char* nnsemd_status_string(nnsemd_status_t s);

/* Text of the last host-side error on this handle ("" if none). */
const char* nnsemd_last_error(nnsemd_handle_t h);

/*
 * emd_approx -- NNS-EMD of one pair (Algorithm 1; problem statement Sec. II-A).
 *   X: device, m x d suppliers; a: device, m masses.
 *   Y: device, n x d consumers; b: device, n masses.
 *   dtype: F32 (points are float) with mode FP32, or BF16 (points are
 *      bfloat16 bit patterns, uint16 per coordinate) with mode
 *      BF16_MFMA_REFINE.
 *   d: F32 with 1 <= d <= 7 takes the low-dimensional point path (any m, n;
 *      pairs beyond one workgroup's LDS run on the multi-workgroup path);
 *      BF16 with any d, or F32 with d > 7, takes the high-dimensional path
 *      (d <= 65536, m, n <= 4096, metrics L2 and SQEUCLIDEAN; the pair's
 *      m x n FP32 key tile is kept in library-owned device scratch).
 *   opts: host, nullable (defaults above).
 *   cost: device, 1 double: R = sum f * D_ij.
 *   plan_src/plan_dst/plan_flow: device, nullable together; when given they
 *      receive the plan F* as (supplier, consumer, flow) triples in
 *      (round, supplier, serve) order; plan_capacity >= m + n - 1 entries.
 *   stats: device, nullable; one nnsemd_stats_t.
 * Errors: INVALID_ARG (NULL handle/pointers, negative sizes, bad enums),
 * UNSUPPORTED (d or size beyond the implemented paths), OUT_OF_MEMORY,
 * DEVICE.  Data errors go to stats->status.
 */
nnsemd_status_t emd_approx(nnsemd_handle_t h,
                           const void* X, const float* a, int64_t m,
                           const void* Y, const float* b, int64_t n,
                           int32_t d, nnsemd_dtype_t dtype, nnsemd_metric_t metric,
                           const nnsemd_options_t* opts,
                           double* cost,
                           int32_t* plan_src, int32_t* plan_dst, double* plan_flow,
                           int64_t plan_capacity,
                           nnsemd_stats_t* stats,
                           void* stream);

/*
 * emd_approx_map -- emd_approx plus the per-supplier barycentric transport
 * map of the plan (colour transfer, Sec. IV-D): map[i*d + k] =
 * sum_j F*_ij y_jk / sum_j F*_ij, accumulated in FP64 in plan order; rows of
 * suppliers that sent nothing are NaN.  map: device, m x d doubles.  FP32
 * points with 1 <= d <= 7 only (else UNSUPPORTED).  The path is chosen as in
 * emd_approx: a pair that fits one workgroup is solved on chip and its map
 * taken by the kernels of emd_barycentric_map (asynchronous); a larger pair
 * (or opts->path = MULTI) runs on the multi-workgroup path, which forms the
 * map while it serves.  Plan arrays and stats may be NULL as in emd_approx
 * (library workspace then holds the plan).
 */
nnsemd_status_t emd_approx_map(nnsemd_handle_t h,
                               const void* X, const float* a, int64_t m,
                               const void* Y, const float* b, int64_t n,
                               int32_t d, nnsemd_dtype_t dtype, nnsemd_metric_t metric,
                               const nnsemd_options_t* opts,
                               double* cost, double* map,
                               int32_t* plan_src, int32_t* plan_dst, double* plan_flow,
                               int64_t plan_capacity,
                               nnsemd_stats_t* stats,
                               void* stream);

/*
 * emd_approx_cost -- NNS-EMD of one pair whose ground distances are given:
 * Algorithm 1 (Sec. III-A) takes the m x n matrix D as its input, and the
 * method works with any valid D (Sec. IV-F), so no coordinates are needed.
 *   D: device, m x n row-major (D[i * n + j] = D_ij between supplier i and
 *      consumer j), dtype F32 or F64, every entry finite and >= 0 (else the
 *      pair's status is INVALID_ARG); caller-owned, read in place.
 *   a: device, m FP32 supplier masses; b: device, n FP32 consumer masses.
 *   Each consumer picks argmin_i D_ij over the active suppliers (entries
 *   compared exactly, ties to the smallest i); the greedy order is by
 *   (D_ij, j); R = sum f * D_ij in FP64.  Options, cost, plan and stats as
 *   in emd_approx (opts->mode, metric-related and path fields are ignored).
 *   One workgroup per pair on chip: 1 <= m, n <= 4096 (else UNSUPPORTED).
 * Errors: INVALID_ARG, CAPACITY, UNSUPPORTED, OUT_OF_MEMORY, DEVICE.
 */
nnsemd_status_t emd_approx_cost(nnsemd_handle_t h,
                                const void* D, nnsemd_dtype_t dtype,
                                const float* a, int64_t m, const float* b, int64_t n,
                                const nnsemd_options_t* opts,
                                double* cost,
                                int32_t* plan_src, int32_t* plan_dst, double* plan_flow,
                                int64_t plan_capacity,
                                nnsemd_stats_t* stats,
                                void* stream);

/*
 * emd_approx_cost_batched -- many independent pairs of given distance
 * matrices in one launch (one workgroup per pair, longest first unless
 * opts->schedule says otherwise), each solved exactly as by emd_approx_cost.
 *   Dcat: device, the matrices back to back; d_off: device, num_pairs + 1
 *      int64 entry offsets (pair p's m_p x n_p matrix at
 *      [d_off[p], d_off[p+1]), which must hold m_p * n_p entries).
 *   acat / a_off, bcat / b_off: device masses and num_pairs + 1 int64
 *      offsets (m_p = a_off[p+1] - a_off[p], n_p likewise).
 *   max_m, max_n: host bounds on every m_p, n_p (<= 4096).
 *   costs, plan arrays, plan_off, stats: as in emd_approx_batched.
 */
nnsemd_status_t emd_approx_cost_batched(nnsemd_handle_t h, int64_t num_pairs,
                                        const void* Dcat, const int64_t* d_off, nnsemd_dtype_t dtype,
                                        const float* acat, const int64_t* a_off,
                                        const float* bcat, const int64_t* b_off,
                                        int64_t max_m, int64_t max_n,
                                        const nnsemd_options_t* opts,
                                        double* costs,
                                        int32_t* plan_src, int32_t* plan_dst, double* plan_flow,
                                        const int64_t* plan_off,
                                        nnsemd_stats_t* stats,
                                        void* stream);

/* Which side of a plan a barycentric map is taken for. */
typedef enum { NNSEMD_MAP_SUPPLIERS = 0, NNSEMD_MAP_CONSUMERS = 1 } nnsemd_map_side_t;

/*
 * emd_barycentric_map -- barycentric transport map of a given plan (colour
 * transfer, Sec. IV-D: each colour moves to the F*-weighted mean of the
 * colours it is transported to).
 *   side SUPPLIERS: rows = m suppliers, P = Y (the consumers, p_rows = n):
 *     map[i*d + k] = sum_j F_ij y_jk / sum_j F_ij;
 *   side CONSUMERS: rows = n consumers, P = X (the suppliers, p_rows = m):
 *     map[j*d + k] = sum_i F_ij x_ik / sum_i F_ij (recolouring the side
 *     that consumes).
 * Each row is summed in FP64 in plan order, so the map of a plan is the same
 * bit for bit whichever path produced the plan; rows without flow are NaN.
 *   plan_src, plan_dst, plan_flow: device, plan_capacity entries (a plan
 *     written by emd_approx, emd_approx_map or emd_approx_batched, or any
 *     list of (supplier, consumer, flow) entries).
 *   plan_nnz: device, nullable: the number of entries in use, e.g.
 *     &stats->nnz of the call that wrote the plan, so no host round trip is
 *     needed; NULL uses all plan_capacity entries.
 *   P: device, p_rows x d FP32; map: device, rows x d doubles.
 * Entries with a supplier or consumer index outside the sizes are skipped.
 * Asynchronous on stream; the handle's workspace grows on the first call
 * for a size.  1 <= d <= 8; rows, p_rows, plan_capacity < 2^31.
 * Errors: INVALID_ARG (NULL arrays, sizes, side), UNSUPPORTED (d),
 * OUT_OF_MEMORY, DEVICE.
 */
nnsemd_status_t emd_barycentric_map(nnsemd_handle_t h,
                                    const int32_t* plan_src, const int32_t* plan_dst, const double* plan_flow,
                                    int64_t plan_capacity, const int64_t* plan_nnz,
                                    const float* P, int64_t p_rows, int32_t d,
                                    int64_t rows, nnsemd_map_side_t side, double* map,
                                    void* stream);

/*
 * emd_approx_batched -- NNS-EMD of many independent ragged pairs in one
 * launch (the batching of Sec. III-D without padding): one workgroup per
 * pair, started longest-first unless opts->schedule says otherwise; each
 * pair is solved exactly as by emd_approx.
 *   Xcat: device, sum_k |X_k| x d rows; acat: device masses; x_off: device,
 *      num_x_sets + 1 int64 row offsets (set k = rows [x_off[k], x_off[k+1])).
 *   Ycat, bcat, y_off, num_y_sets: the same for consumer sets.
 *   pair_x, pair_y: device, num_pairs int32 set indices each, nullable
 *      (NULL: pair p uses set p; one query against many candidates passes
 *      pair_x = all zeros).
 *   max_m, max_n: host upper bounds on any pair's set sizes (they size the
 *      on-chip workspace); a pair above them fails with INVALID_ARG.
 *   costs: device, num_pairs doubles.
 *   plan_src/plan_dst/plan_flow: device, nullable together; pair p writes
 *      at [plan_off[p], plan_off[p+1]) which must hold m_p + n_p - 1
 *      entries (else that pair's status is CAPACITY); plan_off: device,
 *      num_pairs + 1 int64, required with a plan.
 *   stats: device, nullable; num_pairs entries.
 * Errors as emd_approx.
 */
nnsemd_status_t emd_approx_batched(nnsemd_handle_t h, int64_t num_pairs,
                                   const void* Xcat, const float* acat,
                                   const int64_t* x_off, int64_t num_x_sets,
                                   const void* Ycat, const float* bcat,
                                   const int64_t* y_off, int64_t num_y_sets,
                                   const int32_t* pair_x, const int32_t* pair_y,
                                   int64_t max_m, int64_t max_n,
                                   int32_t d, nnsemd_dtype_t dtype, nnsemd_metric_t metric,
                                   const nnsemd_options_t* opts,
                                   double* costs,
                                   int32_t* plan_src, int32_t* plan_dst, double* plan_flow,
                                   const int64_t* plan_off,
                                   nnsemd_stats_t* stats,
                                   void* stream);

/*
 * nnsemd_colour_transfer -- colour transfer by NNS-EMD (Sec. IV-D).  The
 * colours of each 8-bit RGB image are reduced to a palette by k-means (the
 * reference to k_ref bins, the source to k_src bins: Lloyd iteration with
 * `iters` update steps, started from the colours of pixels floor(k P / K),
 * FP64 distances in channel order with ties to the smallest bin, integer
 * cluster sums, so the palettes are reproducible bit for bit); each palette
 * is a colour histogram (bin colour / 255 in [0,1]^3, mass = share of
 * pixels, both FP32).  NNS-EMD (`metric`, opts as in emd_approx) moves the
 * reference palette (suppliers) onto the source palette (consumers), and
 * every source pixel takes the per-consumer barycentric colour of its bin,
 * T_j = sum_i F_ij c_i / sum_i F_ij (as emd_barycentric_map with side
 * CONSUMERS), written as round-half-even(255 T) clamped to 0..255 (a bin
 * that received no flow keeps its pixels' colours).
 *   ref_rgb: device, ref_pixels x 3 uint8; src_rgb: device, src_pixels x 3.
 *   out_rgb: device, src_pixels x 3 uint8, the recoloured source.
 *   ref_palette / src_palette (k x 3 FP32), ref_mass / src_mass (k FP32),
 *   src_assign (src_pixels int32, the bin of each source pixel), cost (1
 *   double) and stats (one record of the NNS-EMD solve): device, nullable.
 * 1 <= k_ref, k_src <= 1024, 0 <= iters <= 1000, 1 <= pixels < 2^31.
 * Asynchronous; the handle's workspace holds the palettes and the plan.
 * Errors: INVALID_ARG, UNSUPPORTED, OUT_OF_MEMORY, DEVICE.
 */
nnsemd_status_t nnsemd_colour_transfer(nnsemd_handle_t h,
                                       const uint8_t* ref_rgb, int64_t ref_pixels,
                                       const uint8_t* src_rgb, int64_t src_pixels,
                                       int32_t k_ref, int32_t k_src, int32_t iters,
                                       nnsemd_metric_t metric, const nnsemd_options_t* opts,
                                       uint8_t* out_rgb,
                                       float* ref_palette, float* ref_mass,
                                       float* src_palette, float* src_mass, int32_t* src_assign,
                                       double* cost, nnsemd_stats_t* stats,
                                       void* stream);

/*
 * emd_approx_batched_noalloc -- emd_approx_batched for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments and results as
 * emd_approx_batched on the low-dimensional point path; its one scratch
 * buffer, the longest-first schedule (one int32 per pair), lives in a fixed
 * device array of 65536 entries (256 KiB on every GPU the library runs on,
 * held until the process ends) instead of handle workspace, so the call
 * allocates nothing.
 * Limits: FP32 points with 1 <= d <= 7 (else UNSUPPORTED), num_pairs <=
 * 65536 (else INVALID_ARG); other errors as emd_approx_batched.
 * All calls on one GPU share that array (the schedule is rewritten in full
 * by every call, nothing needs clearing): calls that overlap in time on the
 * same GPU -- from other streams or host threads -- race on it and must be
 * ordered by the caller.
 */
nnsemd_status_t emd_approx_batched_noalloc(nnsemd_handle_t h, int64_t num_pairs,
                                           const void* Xcat, const float* acat,
                                           const int64_t* x_off, int64_t num_x_sets,
                                           const void* Ycat, const float* bcat,
                                           const int64_t* y_off, int64_t num_y_sets,
                                           const int32_t* pair_x, const int32_t* pair_y,
                                           int64_t max_m, int64_t max_n,
                                           int32_t d, nnsemd_dtype_t dtype, nnsemd_metric_t metric,
                                           const nnsemd_options_t* opts,
                                           double* costs,
                                           int32_t* plan_src, int32_t* plan_dst, double* plan_flow,
                                           const int64_t* plan_off,
                                           nnsemd_stats_t* stats,
                                           void* stream);

/* ------------------------------------------------------------------------
 * Autotuning of the batched point path (FP32, 1 <= d <= 7).  The launch
 * configuration -- workgroup size (256 or 512) and the search split factor
 * (each active consumer gets the largest power-of-two number of lanes, at
 * most 64, with active consumers x lanes x split <= workgroup size, i.e. how
 * early the search spreads one consumer over several lanes as the active
 * sets shrink; split 1 fills the workgroup) -- is timed with HIP events on synthetic ragged
 * pairs shaped like the caller's (sides uniform in [max/8, max], uniform
 * coordinates, exponential masses) and the fastest is recorded in the handle
 * for (d, metric, size class of max(max_m, max_n)).  Later calls with
 * opts->threads == 0 use it; results never depend on the configuration.
 * The call synchronises stream.  1 <= max_m, max_n <= 4096,
 * 1 <= num_pairs <= 65536. */
typedef struct {
    int32_t threads;  /* chosen workgroup size */
    int32_t split;    /* chosen search split factor (1, 2 or 4) */
    float ms_best;    /* its time per launch on the synthetic batch */
    float ms_default; /* time of the default (256, 1) */
} nnsemd_tuning_t;

nnsemd_status_t nnsemd_autotune(nnsemd_handle_t h, int32_t d, nnsemd_metric_t metric, int64_t max_m, int64_t max_n,
                                int64_t num_pairs, nnsemd_tuning_t* result, void* stream);

/* The handle's tuning table as text ("nnsemd-tuning 2", then one line
 * "d metric class threads split ms" per entry), and back. */
nnsemd_status_t nnsemd_tuning_save(nnsemd_handle_t h, const char* path);
nnsemd_status_t nnsemd_tuning_load(nnsemd_handle_t h, const char* path);
/* Forget every recorded configuration (both tables): later calls use the
 * defaults. */
nnsemd_status_t nnsemd_tuning_clear(nnsemd_handle_t h);

/* Autotuning of the high-dimensional BF16 matrix-core path (Sec. III-D
 * batching with the distance tile of the blueprint's matrix-core form).
 * Two launch forms compute the same plans and costs: the split form (a key
 * tile kernel with 16-consumer stripes whose BF16 fragments stay in
 * registers, then the rounds kernel) and the fused form (32 x 32 blocked
 * tiles computed by the rounds kernel itself).  The split form exists for
 * d <= 320 and sides <= 1024.  Both are timed with HIP events on synthetic
 * ragged BF16 pairs shaped like the caller's (sides uniform in
 * [max/8, max], N(0, 1/d) coordinates, exponential masses) and the faster
 * is recorded for (d class: <= 64, <= 128, <= 320, larger; size class of
 * max(max_m, max_n)).  Later BF16 calls use it.  The call synchronises
 * stream.  1 <= d <= 4096, 1 <= max_m, max_n <= 4096,
 * 1 <= num_pairs <= 65536. */
typedef struct {
    int32_t split;    /* 1: split form chosen, 0: fused form */
    float ms_split;   /* split form per launch on the synthetic batch (-1: not available) */
    float ms_fused;   /* fused form per launch */
} nnsemd_doc_tuning_t;

nnsemd_status_t nnsemd_autotune_docs(nnsemd_handle_t h, int32_t d, int64_t max_m, int64_t max_n, int64_t num_pairs,
                                     nnsemd_doc_tuning_t* result, void* stream);
/* Record a launch form by hand for the (d class, size class of max_side)
 * entry: split 1 = split form where it exists (its tile pass stages a supplier
 * set shared by every pair once per workgroup and runs stripe by stripe, else
 * one workgroup per pair), 2 = split form with the per-pair tile pass always,
 * 0 = fused form.  All three give the same plans and costs. */
nnsemd_status_t nnsemd_tuning_set_docs(nnsemd_handle_t h, int32_t d, int64_t max_side, int32_t split);

/* ------------------------------------------------------------------------
 * Learned surrogate for retrieval (not part of the paper, which treats
 * NNS-EMD as a non-differentiable procedure): a deep-sets network predicts
 * the EMD of two 3-D point sets from pooled per-point features, a retrieval
 * keeps the candidates it ranks best, and NNS-EMD (Algorithm 1) re-ranks
 * them.  It never replaces an NNS-EMD value in a result.
 *
 *   phi(x)  = relu(W2 relu(W1 x + b1) + b2)            3 -> 256 -> 256
 *   E(X, a) = sum_i a_i phi(x_i)                        (mass-weighted pooling)
 *   pred    = softplus(w4 . relu(W3 [E_q, E_c, |E_q - E_c|] + b3) + b4)
 *   loss    = mean_b (log pred_b - log y_b)^2           (labels y_b > 0)
 *
 * theta: device, nnsemd_sg_num_params() FP32 master parameters, in the order
 * W1 (256 x 3), b1 (256), W2 (256 x 256), b2 (256), W3 (256 x 768), b3 (256),
 * w4 (256), b4 (1), matrices row-major [out][in].  The kernels use the
 * weights rounded to BF16, with FP32 accumulation; every call re-derives the
 * BF16 copies from theta.  Point sets are concatenated FP32 rows (x, y, z)
 * with masses and int64 offsets (set s = rows [off[s], off[s+1])).  All
 * arrays are caller-owned device memory; calls are asynchronous on stream.
 * ------------------------------------------------------------------------ */
int64_t nnsemd_sg_num_params(void);

/* Pooled embeddings E (num_sets x 256 FP32) of point sets.  num_points: the
 * rows of X (offsets are clamped to it; bad offsets never read outside X). */
nnsemd_status_t nnsemd_sg_embed(nnsemd_handle_t h, const float* theta, const float* X, const float* a,
                                const int64_t* set_off, int64_t num_sets, int64_t num_points, float* E,
                                void* stream);

/* pred[b] for pairs (Eq[q_idx[b]], Ec[c_idx[b]]); q_idx NULL = row 0 for all,
 * c_idx NULL = row b.  num_q / num_c: rows of the tables; an index outside
 * them gives pred NaN. */
nnsemd_status_t nnsemd_sg_predict(nnsemd_handle_t h, const float* theta, const float* Eq, int64_t num_q,
                                  const float* Ec, int64_t num_c, const int32_t* q_idx, const int32_t* c_idx,
                                  int64_t num_pairs, float* pred, void* stream);

/* Loss (1 float) and gradient (nnsemd_sg_num_params floats, master layout;
 * the gradient of each rounded weight is that of its master value) of one
 * training batch: pair b compares set 2b with set 2b+1 (set_off has
 * 2 num_pairs + 1 entries, set_off[2 num_pairs] = num_points); labels: the
 * NNS-EMD values, > 0.  Offsets that are not a partition of the points make
 * the loss NaN.  1 <= num_pairs <= 2^20, 1 <= num_points <= 2^26. */
nnsemd_status_t nnsemd_sg_loss_grad(nnsemd_handle_t h, const float* theta, const float* X, const float* a,
                                    const int64_t* set_off, int64_t num_pairs, int64_t num_points,
                                    const float* labels, float* loss, float* grad, void* stream);

/* nnsemd_sg_loss_grad, then one Adam step on theta (beta1 0.9, beta2 0.999,
 * eps 1e-8, bias-corrected with step >= 1; adam_m / adam_v: device FP32
 * moments, zero before step 1).  grad: device output, or NULL for library
 * workspace. */
nnsemd_status_t nnsemd_sg_train_step(nnsemd_handle_t h, float* theta, float* adam_m, float* adam_v, int64_t step,
                                     float lr, const float* X, const float* a, const int64_t* set_off,
                                     int64_t num_pairs, int64_t num_points, const float* labels, float* loss,
                                     float* grad, void* stream);

/* Indices of the k smallest of n values, ascending by (value, index), NaN
 * last; 1 <= k <= min(n, 1024). */
nnsemd_status_t nnsemd_topk_smallest_f32(nnsemd_handle_t h, const float* values, int64_t n, int32_t k,
                                         int32_t* idx, void* stream);
nnsemd_status_t nnsemd_topk_smallest_f64(nnsemd_handle_t h, const double* values, int64_t n, int32_t k,
                                         int32_t* idx, void* stream);

/* Surrogate-pruned retrieval of one query (Xq, aq: mq points, suppliers)
 * among num_candidates candidate sets (Ycat, bcat, y_off: consumers; their
 * embeddings index_E from nnsemd_sg_embed): the keep candidates of smallest
 * pred are re-ranked by NNS-EMD (greedy, L2, exactly as emd_approx_batched);
 * out_idx / out_cost receive the top of them by NNS-EMD (ascending, ties by
 * index).  kept_idx (keep int32) and kept_stats (keep records), nullable,
 * receive the kept candidates and their NNS-EMD stats.  max_n: host bound
 * on the candidate sizes.  1 <= top <= keep <= min(num_candidates, 1024). */
nnsemd_status_t nnsemd_sg_retrieve(nnsemd_handle_t h, const float* theta, const float* index_E,
                                   int64_t num_candidates, const float* Xq, const float* aq, int64_t mq,
                                   const float* Ycat, const float* bcat, const int64_t* y_off, int64_t max_n,
                                   int32_t keep, int32_t top, int32_t* out_idx, double* out_cost,
                                   int32_t* kept_idx, nnsemd_stats_t* kept_stats, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* NNSEMD_H */
