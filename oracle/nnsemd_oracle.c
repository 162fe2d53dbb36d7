/*
 * Plain FP64 CPU oracle for NNS-EMD -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the checker, not the product.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or helper with the GPU library.
 *
 * What it computes: Algorithm 1 of the paper (NNS-EMD with the Greedy
 * Protocol, Sec. III-A "NNS-EMD Algorithm"), taken step by step:
 *   - active index sets m^(t) = {i : s_i > 0}, n^(t) = {j : c_j > 0};
 *   - NNS: every active consumer j picks argmin_{i in m^(t)} D_ij;
 *   - flow & cost: every active supplier i serves the consumers that picked
 *     it, nearest first, f = min(s_i, c_j), s_i -= f, c_j -= f, R += f D_ij,
 *     F*_ij += f, while s_i > 0;
 *   - weights update: points whose weight reached zero leave the active sets.
 * The Random Protocol of the same section (serve claimants in a random
 * order) is selectable; its random order comes from a counter-based
 * generator (SplitMix64, Steele, Lea & Flood, OOPSLA 2014) keyed by
 * (seed, round, consumer), so any implementation can reproduce it.
 *
 * Readings taken where the paper is silent or garbled:
 *   - the inner serve loop visits every claimant while s_i > 0 (the printed
 *     bound on l skips the last claimant, which cannot terminate when each
 *     supplier has one claimant);
 *   - argmin ties go to the smallest supplier index; the greedy claimant
 *     order is by (D_ij, j) ascending;
 *   - the outer loop runs while BOTH sides still hold mass (floating-point
 *     marginals need not empty together); leftover mass is reported;
 *   - D_ij = d(x_i, y_j): squared Euclidean key for the search and the sort
 *     for both L2 and squared-Euclidean metrics (same order), L1 key for L1;
 *     the cost uses sqrt(key) for L2 and the key itself otherwise;
 *   - masses are used as given (no renormalisation); the total masses must
 *     agree to 1e-5 relative.
 * D is never stored: each entry is recomputed from the coordinates, in
 * dimension order, in FP64, without fused multiply-add (build with
 * -ffp-contract=off).  Algorithm 1 itself takes D as its input; that form
 * (nnsemd_oracle_solve_cost) runs the same steps on a given m x n matrix.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR_INVALID_ARG -1
#define ORC_ERR_MASS_MISMATCH -2
#define ORC_ERR_CAPACITY -3
#define ORC_ERR_OUT_OF_MEMORY -4
#define ORC_ERR_NOT_CONVERGED -6

#define ORC_METRIC_L2 0
#define ORC_METRIC_SQEUCLIDEAN 1
#define ORC_METRIC_L1 2
#define ORC_METRIC_GIVEN 3 /* D is given: key = distance = D_ij */

#define ORC_PROTOCOL_GREEDY 0
#define ORC_PROTOCOL_RANDOM 1

typedef struct {
    double cost;          /* R */
    int64_t rounds;       /* number of NNS iterations t */
    int64_t nnz;          /* plan entries (one per serve) */
    int64_t work;         /* sum_t |m^(t)| * |n^(t)| distance evaluations */
    int64_t near_ties_nn; /* consumers whose best/second-best gap <= 1e-6 rel */
    int64_t near_ties_order; /* adjacent claimants with gap <= 1e-6 rel */
    double residual_src;  /* sum of s_i left when the loop ends */
    double residual_dst;  /* sum of c_j left when the loop ends */
    int32_t status;
    int32_t pad;
} oracle_stats;

/* Key used by the search and by the greedy order. */
static double key_of(const double* x, const double* y, int d, int metric) {
    double acc = 0.0;
    if (metric == ORC_METRIC_L1) {
        for (int k = 0; k < d; ++k) acc += fabs(x[k] - y[k]);
    } else {
        for (int k = 0; k < d; ++k) {
            double t = x[k] - y[k];
            acc += t * t;
        }
    }
    return acc;
}

/* Ground distance D_ij used in the cost (a given matrix: the entry itself). */
static double dist_of_key(double key, int metric) {
    return metric == ORC_METRIC_L2 ? sqrt(key) : key;
}

/* Where the keys come from: two point sets and a metric, or the m x n
 * ground-distance matrix D itself (Algorithm 1 takes D as its input). */
typedef struct {
    const double* X; /* m x d suppliers (points mode) */
    const double* Y; /* n x d consumers (points mode) */
    int d;
    int metric;      /* ORC_METRIC_*, ORC_METRIC_GIVEN for a matrix */
    const double* D; /* m x n row-major, or NULL (points mode) */
    int64_t n;
} ground_t;

static double ground_key(const ground_t* g, int64_t i, int64_t j) {
    if (g->D != NULL) return g->D[i * g->n + j];
    return key_of(g->X + i * g->d, g->Y + j * g->d, g->d, g->metric);
}

static int near_tie(double d1, double d2) {
    double gap = d2 - d1;
    if (d1 == 0.0) return gap <= 1e-12;
    return gap <= 1e-6 * d1;
}

/* SplitMix64 output function applied to a counter built from
 * (seed, round, consumer): the random protocol's serve order key. */
uint64_t nnsemd_oracle_rp_key(uint64_t seed, int64_t round, int64_t j) {
    uint64_t ctr = ((uint64_t)round << 32) ^ (uint64_t)(uint32_t)j;
    uint64_t z = seed + (ctr + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

typedef struct {
    double key;
    uint64_t rk; /* random-protocol rank key */
    int32_t j;
} claimant;

static int cmp_greedy(const void* pa, const void* pb) {
    const claimant* a = (const claimant*)pa;
    const claimant* b = (const claimant*)pb;
    if (a->key < b->key) return -1;
    if (a->key > b->key) return 1;
    return (a->j > b->j) - (a->j < b->j);
}

static int cmp_random(const void* pa, const void* pb) {
    const claimant* a = (const claimant*)pa;
    const claimant* b = (const claimant*)pb;
    if (a->rk < b->rk) return -1;
    if (a->rk > b->rk) return 1;
    return (a->j > b->j) - (a->j < b->j);
}

/*
 * One pair on a ground (points or a given matrix); see nnsemd_oracle_solve.
 */
static int solve_ground(const ground_t* G, const double* a, int64_t m,
                        const double* b, int64_t n, int32_t protocol,
                        uint64_t seed, int64_t max_rounds,
                        int32_t* plan_src, int32_t* plan_dst,
                        double* plan_flow, int64_t plan_capacity,
                        oracle_stats* st) {
    const int metric = G->metric;
    memset(st, 0, sizeof(*st));
    if (m < 0 || n < 0 || (G->D == NULL && G->d < 1) ||
        (protocol != ORC_PROTOCOL_GREEDY && protocol != ORC_PROTOCOL_RANDOM)) {
        st->status = ORC_ERR_INVALID_ARG;
        return st->status;
    }
    if (plan_src != NULL && m + n > 0 && plan_capacity < m + n - 1) {
        st->status = ORC_ERR_CAPACITY;
        return st->status;
    }
    /* Input checks: finite coordinates (or finite, non-negative entries of a
     * given D), finite non-negative masses. */
    double sum_a = 0.0, sum_b = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        if (!isfinite(a[i]) || a[i] < 0.0) { st->status = ORC_ERR_INVALID_ARG; return st->status; }
        if (G->D == NULL) {
            for (int k = 0; k < G->d; ++k)
                if (!isfinite(G->X[i * G->d + k])) { st->status = ORC_ERR_INVALID_ARG; return st->status; }
        } else {
            for (int64_t j = 0; j < n; ++j)
                if (!isfinite(G->D[i * n + j]) || G->D[i * n + j] < 0.0) {
                    st->status = ORC_ERR_INVALID_ARG;
                    return st->status;
                }
        }
        sum_a += a[i];
    }
    for (int64_t j = 0; j < n; ++j) {
        if (!isfinite(b[j]) || b[j] < 0.0) { st->status = ORC_ERR_INVALID_ARG; return st->status; }
        if (G->D == NULL)
            for (int k = 0; k < G->d; ++k)
                if (!isfinite(G->Y[j * G->d + k])) { st->status = ORC_ERR_INVALID_ARG; return st->status; }
        sum_b += b[j];
    }
    double big = sum_a > sum_b ? sum_a : sum_b;
    if (fabs(sum_a - sum_b) > 1e-5 * big) { st->status = ORC_ERR_MASS_MISMATCH; return st->status; }
    if (max_rounds <= 0) max_rounds = m + n;

    double* s = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    double* c = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int64_t* M = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    int64_t* N = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t* nn = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t* bucket_start = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m + 1));
    int64_t* bucket_fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    claimant* cl = (claimant*)malloc(sizeof(claimant) * (size_t)(n > 0 ? n : 1));
    if (!s || !c || !M || !N || !nn || !bucket_start || !bucket_fill || !cl) {
        free(s); free(c); free(M); free(N); free(nn); free(bucket_start); free(bucket_fill); free(cl);
        st->status = ORC_ERR_OUT_OF_MEMORY;
        return st->status;
    }
    for (int64_t i = 0; i < m; ++i) s[i] = a[i];
    for (int64_t j = 0; j < n; ++j) c[j] = b[j];

    double R = 0.0;
    int64_t nnz = 0, t = 0;
    int status = ORC_OK;
    for (;;) {
        /* Active index sets (ascending). */
        int64_t mm = 0, nc = 0;
        for (int64_t i = 0; i < m; ++i) if (s[i] > 0.0) M[mm++] = i;
        for (int64_t j = 0; j < n; ++j) if (c[j] > 0.0) N[nc++] = j;
        if (mm == 0 || nc == 0) break;
        if (t >= max_rounds) { status = ORC_ERR_NOT_CONVERGED; break; }
        st->work += mm * nc;

        /* NNS: each active consumer picks its nearest active supplier;
         * the first (smallest index) of equal minima wins. */
        for (int64_t q = 0; q < nc; ++q) {
            int64_t j = N[q];
            double best = INFINITY, second = INFINITY;
            int64_t arg = -1;
            for (int64_t p = 0; p < mm; ++p) {
                int64_t i = M[p];
                double k = ground_key(G, i, j);
                if (k < best) { second = best; best = k; arg = i; }
                else if (k < second) { second = k; }
            }
            nn[j] = arg;
            if (mm > 1 && near_tie(dist_of_key(best, metric), dist_of_key(second, metric)))
                st->near_ties_nn++;
        }

        /* Claimant sets a_i: bucket the active consumers by their pick. */
        for (int64_t i = 0; i <= m; ++i) bucket_start[i] = 0;
        for (int64_t q = 0; q < nc; ++q) bucket_start[nn[N[q]] + 1]++;
        for (int64_t i = 0; i < m; ++i) bucket_start[i + 1] += bucket_start[i];
        for (int64_t i = 0; i < m; ++i) bucket_fill[i] = bucket_start[i];
        for (int64_t q = 0; q < nc; ++q) {
            int64_t j = N[q];
            int64_t i = nn[j];
            claimant* e = &cl[bucket_fill[i]++];
            e->j = (int32_t)j;
            e->key = ground_key(G, i, j);
            e->rk = nnsemd_oracle_rp_key(seed, t, j);
        }

        /* Flow & cost: suppliers in ascending index, claimants in protocol
         * order, while the supplier still holds mass. */
        for (int64_t p = 0; p < mm; ++p) {
            int64_t i = M[p];
            int64_t lo = bucket_start[i], hi = bucket_start[i + 1];
            if (hi == lo) continue;
            qsort(cl + lo, (size_t)(hi - lo), sizeof(claimant),
                  protocol == ORC_PROTOCOL_GREEDY ? cmp_greedy : cmp_random);
            if (protocol == ORC_PROTOCOL_GREEDY) {
                for (int64_t e = lo + 1; e < hi; ++e)
                    if (near_tie(dist_of_key(cl[e - 1].key, metric), dist_of_key(cl[e].key, metric)))
                        st->near_ties_order++;
            }
            for (int64_t e = lo; e < hi; ++e) {
                if (!(s[i] > 0.0)) break;
                int64_t j = cl[e].j;
                double f = s[i] < c[j] ? s[i] : c[j];
                s[i] = s[i] - f;
                c[j] = c[j] - f;
                R = R + f * dist_of_key(cl[e].key, metric);
                if (plan_src != NULL) {
                    plan_src[nnz] = (int32_t)i;
                    plan_dst[nnz] = (int32_t)j;
                    plan_flow[nnz] = f;
                }
                nnz++;
            }
        }
        t++;
    }
    double rs = 0.0, rc = 0.0;
    for (int64_t i = 0; i < m; ++i) rs += s[i];
    for (int64_t j = 0; j < n; ++j) rc += c[j];
    st->cost = R;
    st->rounds = t;
    st->nnz = nnz;
    st->residual_src = rs;
    st->residual_dst = rc;
    st->status = status;
    free(s); free(c); free(M); free(N); free(nn); free(bucket_start); free(bucket_fill); free(cl);
    return status;
}

/*
 * Solve one pair.  X: m x d row-major suppliers, a: m masses; Y: n x d
 * consumers, b: n masses.  Plan arrays may be NULL (plan_capacity ignored);
 * otherwise they must hold m + n - 1 entries.  max_rounds <= 0 means m + n.
 */
int nnsemd_oracle_solve(const double* X, const double* a, int64_t m,
                        const double* Y, const double* b, int64_t n,
                        int32_t d, int32_t metric, int32_t protocol,
                        uint64_t seed, int64_t max_rounds,
                        int32_t* plan_src, int32_t* plan_dst,
                        double* plan_flow, int64_t plan_capacity,
                        oracle_stats* st) {
    if (metric < 0 || metric > 2) {
        memset(st, 0, sizeof(*st));
        st->status = ORC_ERR_INVALID_ARG;
        return st->status;
    }
    ground_t G = {X, Y, d, metric, NULL, n};
    return solve_ground(&G, a, m, b, n, protocol, seed, max_rounds, plan_src, plan_dst,
                        plan_flow, plan_capacity, st);
}

/*
 * Solve one pair whose ground distances are given (Algorithm 1's input D):
 * D is m x n row-major, D[i * n + j] = D_ij, finite and non-negative; the
 * search, the greedy order and the cost all use D_ij itself.
 */
int nnsemd_oracle_solve_cost(const double* D, const double* a, int64_t m,
                             const double* b, int64_t n, int32_t protocol,
                             uint64_t seed, int64_t max_rounds,
                             int32_t* plan_src, int32_t* plan_dst,
                             double* plan_flow, int64_t plan_capacity,
                             oracle_stats* st) {
    ground_t G = {NULL, NULL, 1, ORC_METRIC_GIVEN, D, n};
    if (D == NULL && m > 0 && n > 0) {
        memset(st, 0, sizeof(*st));
        st->status = ORC_ERR_INVALID_ARG;
        return st->status;
    }
    return solve_ground(&G, a, m, b, n, protocol, seed, max_rounds, plan_src, plan_dst,
                        plan_flow, plan_capacity, st);
}

/*
 * Many independent pairs (the batched workload of Sec. III-D, "Batch
 * Processing"): pair p uses rows [x_off[px], x_off[px+1]) of X and
 * [y_off[py], y_off[py+1]) of Y, with px = pair_x ? pair_x[p] : p and
 * likewise for py.  Pairs run in parallel over OpenMP threads when the
 * library is built with -fopenmp; each pair is solved exactly as above.
 * Plans are not returned.  Returns the number of threads used.
 */
int nnsemd_oracle_solve_batched(int64_t num_pairs,
                                const double* X, const double* a, const int64_t* x_off,
                                const double* Y, const double* b, const int64_t* y_off,
                                const int32_t* pair_x, const int32_t* pair_y,
                                int32_t d, int32_t metric, int32_t protocol, uint64_t seed,
                                oracle_stats* stats) {
    int threads = 1;
#ifdef _OPENMP
#pragma omp parallel
    {
#pragma omp single
        threads = omp_get_num_threads();
    }
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t p = 0; p < num_pairs; ++p) {
        int64_t px = pair_x ? pair_x[p] : p;
        int64_t py = pair_y ? pair_y[p] : p;
        int64_t x0 = x_off[px], x1 = x_off[px + 1];
        int64_t y0 = y_off[py], y1 = y_off[py + 1];
        nnsemd_oracle_solve(X + x0 * d, a + x0, x1 - x0, Y + y0 * d, b + y0, y1 - y0,
                            d, metric, protocol, seed, 0, NULL, NULL, NULL, 0, &stats[p]);
    }
    return threads;
}

/*
 * Barycentric transport map of a plan (colour transfer, Sec. IV-D): for every
 * supplier i, T_i = sum_j F_ij y_j / sum_j F_ij; rows with no outgoing flow
 * are NaN.  `out` is m x d.
 */
void nnsemd_oracle_barycentric(const int32_t* plan_src, const int32_t* plan_dst,
                               const double* plan_flow, int64_t nnz,
                               const double* Y, int64_t m, int32_t d, double* out) {
    double* w = (double*)calloc((size_t)(m > 0 ? m : 1), sizeof(double));
    for (int64_t i = 0; i < m * d; ++i) out[i] = 0.0;
    for (int64_t e = 0; e < nnz; ++e) {
        int64_t i = plan_src[e], j = plan_dst[e];
        w[i] += plan_flow[e];
        for (int k = 0; k < d; ++k) out[i * d + k] += plan_flow[e] * Y[j * d + k];
    }
    for (int64_t i = 0; i < m; ++i)
        for (int k = 0; k < d; ++k)
            out[i * d + k] = w[i] > 0.0 ? out[i * d + k] / w[i] : NAN;
    free(w);
}

/*
 * The other direction (recolouring the source of a colour transfer, where
 * the source palette consumes): for every consumer j,
 * T_j = sum_i F_ij x_i / sum_i F_ij, NaN for consumers that received
 * nothing.  `out` is n x d; sums run in plan order.
 */
void nnsemd_oracle_barycentric_dst(const int32_t* plan_src, const int32_t* plan_dst,
                                   const double* plan_flow, int64_t nnz,
                                   const double* X, int64_t n, int32_t d, double* out) {
    double* w = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    for (int64_t j = 0; j < n * d; ++j) out[j] = 0.0;
    for (int64_t e = 0; e < nnz; ++e) {
        int64_t i = plan_src[e], j = plan_dst[e];
        w[j] += plan_flow[e];
        for (int k = 0; k < d; ++k) out[j * d + k] += plan_flow[e] * X[i * d + k];
    }
    for (int64_t j = 0; j < n; ++j)
        for (int k = 0; k < d; ++k)
            out[j * d + k] = w[j] > 0.0 ? out[j * d + k] / w[j] : NAN;
    free(w);
}


/*
 * Colour transfer application (Sec. IV-D): k-means palette reduction of an
 * 8-bit RGB image, and the recolouring of an image through a per-bin colour
 * map.  The paper reduces the reference image's colours with k-means before
 * transporting them; it gives no further detail, so this is plain Lloyd
 * iteration with every step fixed so that any implementation reproduces it:
 *   - start: centroid k = the colour of pixel floor(k * P / K);
 *   - assignment: argmin_k sum_c (p_c - C_kc)^2 in FP64, channels in order,
 *     no fused multiply-add, ties to the smallest k;
 *   - update: integer sums of the assigned pixels' channels and counts, then
 *     C_kc = S_kc / n_k (FP64, correctly rounded); an empty cluster keeps its
 *     centroid;
 *   - `iters` assignment + update steps, then one final assignment.
 * Outputs: centroids (K x 3, FP64, 0..255 scale), counts (K), assignment (P).
 */
static int nearest_centroid(const uint8_t* px, const double* C, int32_t K) {
    int best = 0;
    double bd = INFINITY;
    for (int k = 0; k < K; ++k) {
        double acc = 0.0;
        for (int c = 0; c < 3; ++c) {
            double t = (double)px[c] - C[k * 3 + c];
            acc = acc + t * t;
        }
        if (acc < bd) { bd = acc; best = k; }
    }
    return best;
}

void nnsemd_oracle_kmeans(const uint8_t* pixels, int64_t P, int32_t K, int32_t iters,
                          double* centroids, int64_t* counts, int32_t* assign) {
    int64_t* S = (int64_t*)calloc((size_t)K * 3, sizeof(int64_t));
    for (int k = 0; k < K; ++k) {
        int64_t src = (int64_t)k * P / K;
        for (int c = 0; c < 3; ++c) centroids[k * 3 + c] = (double)pixels[src * 3 + c];
    }
    for (int it = 0; it <= iters; ++it) {
        for (int64_t p = 0; p < P; ++p) assign[p] = nearest_centroid(pixels + p * 3, centroids, K);
        for (int k = 0; k < K; ++k) counts[k] = 0;
        for (int64_t k = 0; k < (int64_t)K * 3; ++k) S[k] = 0;
        for (int64_t p = 0; p < P; ++p) {
            counts[assign[p]]++;
            for (int c = 0; c < 3; ++c) S[assign[p] * 3 + c] += pixels[p * 3 + c];
        }
        if (it == iters) break;  /* the final assignment is not followed by an update */
        for (int k = 0; k < K; ++k)
            if (counts[k] > 0)
                for (int c = 0; c < 3; ++c) centroids[k * 3 + c] = (double)S[k * 3 + c] / (double)counts[k];
    }
    free(S);
}

/*
 * Recolour: pixel p takes the colour map[assign[p]] (a colour in [0,1]^3),
 * written as round-half-even of 255 * value clamped to 0..255; a bin whose
 * map row is NaN (it received no flow) keeps the pixel's own colour.
 */
void nnsemd_oracle_recolour(const uint8_t* pixels, const int32_t* assign, int64_t P,
                            const double* map, uint8_t* out) {
    for (int64_t p = 0; p < P; ++p) {
        const double* T = map + (int64_t)assign[p] * 3;
        for (int c = 0; c < 3; ++c) {
            if (isnan(T[c])) { out[p * 3 + c] = pixels[p * 3 + c]; continue; }
            double v = nearbyint(255.0 * T[c]);
            v = v < 0.0 ? 0.0 : (v > 255.0 ? 255.0 : v);
            out[p * 3 + c] = (uint8_t)v;
        }
    }
}
