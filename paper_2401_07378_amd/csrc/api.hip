// Host runtime of the NNS-EMD library: handles, argument checks, workspace
// and dispatch to the kernels.  Implements include/nnsemd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"

// Fixed device scratch of emd_approx_batched_noalloc: the longest-first
// schedule (one int32 per pair) for callers that cannot allocate.  Each GPU
// holds its own copy until the process ends.  Host code never uses this name
// as an address: the device address of each GPU's copy is taken once per
// device (nnsemd_create) and kept in g_scratch_dev.
constexpr int kNoAllocMaxPairs = 65536;
static __device__ __align__(256) int32_t scratch[kNoAllocMaxPairs];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int32_t* g_scratch_dev[kMaxDevices] = {};
}  // namespace

constexpr int nnsemd_tune_classes = 6;  // max side <= 128, 256, 512, 1024, 2048, 4096

struct nnsemd_handle {
    int device = 0;
    int num_cus = 0;
    size_t max_lds = 0;
    std::string last_error;
    unsigned long long* phase_cycles = nullptr;  // profiling builds only
    int32_t* order = nullptr;                    // longest-first pair schedule (device)
    int64_t order_cap = 0;
    void* lp_base = nullptr;                     // multi-workgroup path workspace (device)
    size_t lp_bytes = 0;
    nnsemd::LPState* lp_host = nullptr;          // pinned copy of the round state
    char* doc_tiles = nullptr;                   // key-tile scratch of the high-dimensional path
    size_t doc_bytes = 0;
    char* topk_ws = nullptr;                     // top-k threshold, count and candidate buffer
    double* doc_xnorm = nullptr;                 // supplier-set norms of the split document form
    size_t doc_xnorm_bytes = 0;
    int32_t* doc_stripes = nullptr;              // stripe list of the shared-query tile kernel, then its length
    size_t doc_stripes_bytes = 0;
    // Autotuned launch configuration of the batched point path, by
    // dimension (1..7), metric and size class of max(max_m, max_n).
    struct Tune {
        int32_t valid = 0, threads = 256, split = 1;
        float ms = 0.f;
    } tune[8][3][nnsemd_tune_classes];
    char* sg_quant = nullptr;                    // BF16 weight copies of the surrogate
    char* sg_ws = nullptr;                       // surrogate workspace
    size_t sg_bytes = 0;
    char* map_ws = nullptr;                      // barycentric map: row buckets
    size_t map_bytes = 0;
    char* map_plan = nullptr;                    // emd_approx_map: plan and stats when the caller keeps none
    size_t map_plan_bytes = 0;
    char* ct_ws = nullptr;                       // colour transfer: palettes, assignments, plan, map
    size_t ct_bytes = 0;
    int32_t* fixed_order = nullptr;              // this device's copy of `scratch` (no-alloc schedule)
    // Autotuned launch form of the BF16 high-dimensional path, by d class
    // (<= 64, <= 128, <= 320, larger) and size class of max(max_m, max_n).
    struct DocTune {
        int32_t valid = 0, split = 1;
        float ms_split = -1.f, ms_fused = -1.f;
    } doc_tune[4][nnsemd_tune_classes];
};

namespace {

using namespace nnsemd;

nnsemd_status_t fail(nnsemd_handle_t h, nnsemd_status_t s, const char* msg) {
    if (h) h->last_error = msg;
    return s;
}

nnsemd_status_t device_fail(nnsemd_handle_t h, int err, const char* where) {
    if (h) {
        char buf[256];
        std::snprintf(buf, sizeof(buf), "%s: %s", where, hipGetErrorString((hipError_t)err));
        h->last_error = buf;
    }
    return NNSEMD_ERR_DEVICE;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

nnsemd_options_t default_options() {
    nnsemd_options_t o;
    std::memset(&o, 0, sizeof(o));
    o.protocol = NNSEMD_GREEDY;
    o.mode = NNSEMD_MODE_FP32;
    return o;
}

// Longest-first schedule of a batch into h->order (device).
nnsemd_status_t schedule(nnsemd_handle_t h, const int64_t* x_off, const int64_t* y_off, const int32_t* pair_x,
                         const int32_t* pair_y, int64_t num_pairs, int64_t num_x_sets, int64_t num_y_sets,
                         void* stream) {
    if (h->order_cap < num_pairs) {
        if (h->order) (void)hipFree(h->order);
        h->order = nullptr;
        h->order_cap = 0;
        if (hipMalloc((void**)&h->order, sizeof(int32_t) * (size_t)num_pairs) != hipSuccess)
            return fail(h, NNSEMD_ERR_OUT_OF_MEMORY, "schedule workspace");
        h->order_cap = num_pairs;
    }
    int err = launch_order(x_off, y_off, pair_x, pair_y, num_pairs, num_x_sets, num_y_sets, h->order, stream);
    if (err != 0) return device_fail(h, err, "schedule launch");
    return NNSEMD_OK;
}

int tune_class(int64_t maxp) {
    int c = 0;
    for (int64_t lim = 128; c < nnsemd_tune_classes - 1 && maxp > lim; lim <<= 1) ++c;
    return c;
}

// Common entry for one or many pairs of low-dimensional FP32 points.
// forced_threads / forced_split > 0 bypass the options and the tuning table.
// fixed_order != nullptr: the schedule goes there (no handle workspace).
nnsemd_status_t run_pairs(nnsemd_handle_t h, PairSolverArgs& A, int d, int64_t max_m, int64_t max_n,
                          const nnsemd_options_t& o, void* stream, int forced_threads = 0, int forced_split = 0,
                          int32_t* fixed_order = nullptr) {
    if (d < 1 || d > 7) return fail(h, NNSEMD_ERR_UNSUPPORTED, "point path supports 1 <= d <= 7");
    int threads = o.threads > 0 ? o.threads : 256;
    int split = 1;
    const auto& tn = h->tune[d][A.metric][tune_class(std::max<int64_t>(max_m, max_n))];
    if (o.threads == 0 && tn.valid) {
        threads = tn.threads;
        split = tn.split;
    }
    if (forced_threads > 0) threads = forced_threads;
    if (forced_split > 0) split = forced_split;
    A.split = split;
    if (threads != 256 && threads != 512)
        return fail(h, NNSEMD_ERR_UNSUPPORTED, "workgroup size must be 256 or 512");
    const int64_t maxp = std::max<int64_t>({max_m, max_n, 1});
    const int chunk = (int)((maxp + threads - 1) / threads);
    const int chunk_cap = threads == 256 ? 16 : 8;
    if (chunk > chunk_cap) return fail(h, NNSEMD_ERR_UNSUPPORTED, "set too large for the on-chip pair path");
    const int mcap = (int)std::max<int64_t>(max_m, 1), ncap = (int)std::max<int64_t>(max_n, 1);
    A.max_m = mcap;
    A.max_n = ncap;
    A.protocol = o.protocol;
    A.seed = o.seed;
    A.max_rounds = o.max_rounds;
    A.phase_cycles = h->phase_cycles;
    // LDS layout: the serve order gets its own array unless sharing the
    // bucket array's storage adds a resident workgroup; the coordinates are
    // copied into LDS (no HBM reads inside the rounds) whenever that costs no
    // resident workgroup.
    int blocks = 0, err = 0;
    bool share = false, coords = false;
    size_t lds_bytes = 0;
    for (int c = 0; c < 2; ++c) {
        for (int sh = 0; sh < 2; ++sh) {
            const PairLdsLayout lay = pair_lds_layout(mcap, ncap, record_stride(d), c ? d : 0, true, sh != 0);
            if (lay.total + 8192 > h->max_lds) continue;
            int b = 0;
            if ((err = pair_solver_blocks_per_cu(d, A.metric, threads, chunk, lay.total, &b, c != 0)) != 0)
                return device_fail(h, err, "occupancy query");
            // more resident workgroups first; then the separate order, then the coordinates
            if (b > blocks || (b == blocks && b > 0 && ((share && !sh) || (!share == !sh && c)))) {
                blocks = b;
                share = sh != 0;
                coords = c != 0;
                lds_bytes = lay.total;
            }
        }
    }
    if (blocks < 1) return fail(h, NNSEMD_ERR_UNSUPPORTED, "pair workgroup does not fit on a compute unit");
    A.share_order = share ? 1 : 0;
    const int64_t grid = A.num_pairs;
    if (A.x_off != nullptr && A.num_pairs > 1 && o.schedule == NNSEMD_SCHEDULE_LONGEST_FIRST) {
        if (fixed_order != nullptr) {
            err = launch_order(A.x_off, A.y_off, A.pair_x, A.pair_y, A.num_pairs, A.num_x_sets, A.num_y_sets,
                               fixed_order, stream);
            if (err != 0) return device_fail(h, err, "schedule launch");
            A.order = fixed_order;
        } else {
            nnsemd_status_t s = schedule(h, A.x_off, A.y_off, A.pair_x, A.pair_y, A.num_pairs, A.num_x_sets,
                                         A.num_y_sets, stream);
            if (s != NNSEMD_OK) return s;
            A.order = h->order;
        }
    }
    err = launch_pair_solver(A, d, threads, chunk, coords, lds_bytes, (int)grid, stream);
    if (err != 0) return device_fail(h, err, "solver launch");
    return NNSEMD_OK;
}

// Given distance matrices: one workgroup per pair (on chip, sides <= 4096).
constexpr int kCostMaxSide = 4096;

nnsemd_status_t run_cost(nnsemd_handle_t h, CostArgs& A, int64_t max_m, int64_t max_n, bool f64,
                         const nnsemd_options_t& o, void* stream) {
    if (max_m > kCostMaxSide || max_n > kCostMaxSide)
        return fail(h, NNSEMD_ERR_UNSUPPORTED, "given-D path supports up to 4096 points per side");
    const int mcap = (int)std::max<int64_t>(max_m, 1), ncap = (int)std::max<int64_t>(max_n, 1);
    const int chunk = (std::max(mcap, ncap) + 255) / 256;
    const PairLdsLayout lay = pair_lds_layout(mcap, ncap, 0, 0, true, true);
    if (lay.total + 8192 > h->max_lds) return fail(h, NNSEMD_ERR_UNSUPPORTED, "pair does not fit in LDS");
    A.max_m = mcap;
    A.max_n = ncap;
    A.protocol = o.protocol;
    A.seed = o.seed;
    A.max_rounds = o.max_rounds;
    int blocks = 0;
    int err = launch_cost_solver(A, f64, chunk, lay.total, 0, stream, &blocks);
    if (err != 0) return device_fail(h, err, "occupancy query");
    if (blocks < 1) return fail(h, NNSEMD_ERR_UNSUPPORTED, "pair workgroup does not fit on a compute unit");
    if (A.a_off != nullptr && A.num_pairs > 1 && o.schedule == NNSEMD_SCHEDULE_LONGEST_FIRST) {
        nnsemd_status_t s = schedule(h, A.a_off, A.b_off, nullptr, nullptr, A.num_pairs, A.num_pairs, A.num_pairs,
                                     stream);
        if (s != NNSEMD_OK) return s;
        A.order = h->order;
    }
    err = launch_cost_solver(A, f64, chunk, lay.total, (int)A.num_pairs, stream, nullptr);
    if (err != 0) return device_fail(h, err, "given-D solver launch");
    return NNSEMD_OK;
}

// Option checks of the given-D calls (no metric, points dtype or mode).
nnsemd_status_t check_cost_options(nnsemd_handle_t h, nnsemd_dtype_t dtype, const nnsemd_options_t& o) {
    if (dtype != NNSEMD_F32 && dtype != NNSEMD_F64) return fail(h, NNSEMD_ERR_INVALID_ARG, "D must be F32 or F64");
    if (o.protocol != NNSEMD_GREEDY && o.protocol != NNSEMD_RANDOM)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "bad protocol");
    if (o.schedule != NNSEMD_SCHEDULE_LONGEST_FIRST && o.schedule != NNSEMD_SCHEDULE_AS_GIVEN)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "bad schedule");
    if (o.threads != 0 && o.threads != 256) return fail(h, NNSEMD_ERR_UNSUPPORTED, "given-D path runs 256 threads");
    if (o.reserved != 0) return fail(h, NNSEMD_ERR_INVALID_ARG, "reserved option field must be 0");
    return NNSEMD_OK;
}

// Multi-workgroup path for one pair (any size).  Carves one device
// allocation into the round state and per-point arrays, enqueues rounds and
// reads the round state back every kChunk rounds to shrink the grids.
nnsemd_status_t run_large(nnsemd_handle_t h, LPArgs& A, int d, void* stream) {
    if (d < 1 || d > 7) return fail(h, NNSEMD_ERR_UNSUPPORTED, "point path supports 1 <= d <= 7");
    if (A.m > (1ll << 20) || A.n > (1ll << 20))
        return fail(h, NNSEMD_ERR_UNSUPPORTED, "multi-workgroup path supports up to 2^20 points per side");
    const int rs = record_stride(d);
    const int64_t mcap = std::max<int64_t>(A.m, 1), ncap = std::max<int64_t>(A.n, 1);
    const int K = 3 + 2 * d;
    const int64_t nb = (std::max(mcap, ncap) + 255) / 256;
    const int64_t part_cap = std::max<int64_t>(ncap * 8, (int64_t)1 << 22);
    const int64_t blk_cap = (std::max(mcap, ncap) + 1023) / 1024 + 1;
    const bool want_map = A.map != nullptr;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = align_up(off, 256); off = o + bytes; return o; };
    const size_t o_srec0 = take(sizeof(float) * rs * mcap), o_srec1 = take(sizeof(float) * rs * mcap);
    const size_t o_sidx0 = take(4 * mcap), o_sidx1 = take(4 * mcap);
    const size_t o_smass0 = take(8 * mcap), o_smass1 = take(8 * mcap);
    const size_t o_scnt = take(4 * mcap), o_soff = take(4 * mcap);
    const size_t o_cact0 = take(4 * ncap), o_cact1 = take(4 * ncap);
    const size_t o_cmass = take(8 * ncap), o_cnn = take(4 * ncap), o_ckey = take(8 * ncap);
    const size_t o_list = take(4 * ncap), o_sorted = take(4 * ncap), o_flag = take(4 * ncap);
    const size_t o_tkey = take(8 * ncap), o_thead = take(4 * ncap), o_tnext = take(4 * ncap);
    const size_t o_part = take(16 * part_cap), o_blk = take(8 * blk_cap);
    const size_t o_cost = take(8 * mcap);
    const size_t o_wsum = want_map ? take(8 * mcap) : 0, o_bsum = want_map ? take(8 * mcap * d) : 0;
    const size_t o_red = take(8 * nb * K), o_st = take(sizeof(LPState));
    const size_t total = align_up(off, 256);
    if (h->lp_bytes < total) {
        if (h->lp_base) (void)hipFree(h->lp_base);
        h->lp_base = nullptr;
        h->lp_bytes = 0;
        if (hipMalloc(&h->lp_base, total) != hipSuccess) return fail(h, NNSEMD_ERR_OUT_OF_MEMORY, "workspace");
        h->lp_bytes = total;
    }
    if (h->lp_host == nullptr && hipHostMalloc((void**)&h->lp_host, sizeof(LPState)) != hipSuccess) {
        h->lp_host = nullptr;
        return fail(h, NNSEMD_ERR_OUT_OF_MEMORY, "pinned round state");
    }
    char* base = static_cast<char*>(h->lp_base);
    LPWork& w = A.w;
    w.srec[0] = reinterpret_cast<float*>(base + o_srec0);
    w.srec[1] = reinterpret_cast<float*>(base + o_srec1);
    w.sidx[0] = reinterpret_cast<int32_t*>(base + o_sidx0);
    w.sidx[1] = reinterpret_cast<int32_t*>(base + o_sidx1);
    w.smass[0] = reinterpret_cast<double*>(base + o_smass0);
    w.smass[1] = reinterpret_cast<double*>(base + o_smass1);
    w.scnt = reinterpret_cast<int32_t*>(base + o_scnt);
    w.soff = reinterpret_cast<int32_t*>(base + o_soff);
    w.cact[0] = reinterpret_cast<int32_t*>(base + o_cact0);
    w.cact[1] = reinterpret_cast<int32_t*>(base + o_cact1);
    w.cmass = reinterpret_cast<double*>(base + o_cmass);
    w.cnn = reinterpret_cast<int32_t*>(base + o_cnn);
    w.ckey = reinterpret_cast<double*>(base + o_ckey);
    w.list = reinterpret_cast<int32_t*>(base + o_list);
    w.sorted = reinterpret_cast<int32_t*>(base + o_sorted);
    w.flagged = reinterpret_cast<int32_t*>(base + o_flag);
    w.tkey = reinterpret_cast<double*>(base + o_tkey);
    w.thead = reinterpret_cast<int32_t*>(base + o_thead);
    w.tnext = reinterpret_cast<int32_t*>(base + o_tnext);
    w.part = reinterpret_cast<float4*>(base + o_part);
    w.ncap = ncap;
    w.part_cap = part_cap;
    w.blkcnt = reinterpret_cast<unsigned long long*>(base + o_blk);
    w.blkcnt_cap = (int32_t)blk_cap;
    w.costacc = reinterpret_cast<double*>(base + o_cost);
    w.wsum = want_map ? reinterpret_cast<double*>(base + o_wsum) : nullptr;
    w.bsum = want_map ? reinterpret_cast<double*>(base + o_bsum) : nullptr;
    w.red = reinterpret_cast<double*>(base + o_red);
    w.st = reinterpret_cast<LPState*>(base + o_st);
    if (A.max_rounds <= 0) A.max_rounds = A.m + A.n;
    int err = lp_launch_init(A, d, stream);
    if (err != 0) return device_fail(h, err, "multi-workgroup init");
    constexpr int kChunk = 16;
    int mact_ub = (int)A.m, nact_ub = (int)A.n;
    int64_t launched = 0;
    for (;;) {
        hipError_t e = hipMemcpyAsync(h->lp_host, w.st, sizeof(LPState), hipMemcpyDeviceToHost, (hipStream_t)stream);
        if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
        if (e != hipSuccess) return device_fail(h, (int)e, "round state readback");
        if (h->lp_host->done || h->lp_host->status != NNSEMD_OK) break;
        if (h->lp_host->tail) {  // both active sets fit one workgroup: it runs the rest
            err = lp_launch_tail(A, d, stream);
            if (err != 0) return device_fail(h, err, "single-workgroup finish");
            break;
        }
        if (launched > A.max_rounds + kChunk) break;  // unreachable: the device caps the rounds
        mact_ub = h->lp_host->mact;
        nact_ub = h->lp_host->nact;
        for (int r = 0; r < kChunk; ++r) {
            err = lp_launch_round(A, d, mact_ub, nact_ub, stream);
            if (err != 0) return device_fail(h, err, "multi-workgroup round");
            ++launched;
        }
    }
    err = lp_launch_finish(A, d, stream);
    if (err != 0) return device_fail(h, err, "multi-workgroup finish");
    return NNSEMD_OK;
}

// High-dimensional path: BF16 points on the matrix cores, or FP32 points
// with d > 7 on the vector ALUs.  Pairs are launched in chunks whose key
// tiles fit the scratch budget.
constexpr size_t kDocTileBudget = (size_t)4 << 30;
constexpr int kDocMaxSide = 4096;
constexpr int kDocMaxDim = 65536;

// High-dimensional L1: the exact FP64 distance matrix of each pair (dimension
// order, the definition's operations), then the given-D solver on it, in
// chunks whose matrices fit the scratch budget.
nnsemd_status_t run_docs_l1(nnsemd_handle_t h, DocArgs& A, int64_t max_m, int64_t max_n, nnsemd_dtype_t dtype,
                            const nnsemd_options_t& o, void* stream);

int doc_dim_class(int64_t d) { return d <= 64 ? 0 : (d <= 128 ? 1 : (d <= 320 ? 2 : 3)); }

// force_split: -1 = the tuned (or default split) form, 0 = fused, 1 = split where it exists.
nnsemd_status_t run_docs(nnsemd_handle_t h, DocArgs& A, int64_t max_m, int64_t max_n, nnsemd_dtype_t dtype,
                         const nnsemd_options_t& o, void* stream, int force_split = -1) {
    if (A.metric == NNSEMD_L1) return run_docs_l1(h, A, max_m, max_n, dtype, o, stream);
    if (A.d > kDocMaxDim) return fail(h, NNSEMD_ERR_UNSUPPORTED, "d above 65536");
    if (o.threads != 0 && o.threads != 256)
        return fail(h, NNSEMD_ERR_UNSUPPORTED, "high-dimensional path runs 256-thread workgroups");
    if (max_m > kDocMaxSide || max_n > kDocMaxSide)
        return fail(h, NNSEMD_ERR_UNSUPPORTED, "high-dimensional path supports up to 4096 points per side");
    const int mcap = (int)std::max<int64_t>(max_m, 1), ncap = (int)std::max<int64_t>(max_n, 1);
    const int chunk = (std::max(mcap, ncap) + 255) / 256;
    const size_t lds = doc_lds_bytes(mcap, ncap, dtype != NNSEMD_BF16);
    if (lds + 8192 > h->max_lds) return fail(h, NNSEMD_ERR_UNSUPPORTED, "pair does not fit in LDS");
    A.max_m = mcap;
    A.max_n = ncap;
    A.protocol = o.protocol;
    A.seed = o.seed;
    A.max_rounds = o.max_rounds;
    const bool mfma = dtype == NNSEMD_BF16;
    bool split = doc_split_form(A.d, mfma, chunk);
    bool per_pair_tile = false;
    if (force_split == 0) {
        split = false;
    } else if (force_split < 0 && split) {
        const auto& dt = h->doc_tune[doc_dim_class(A.d)][tune_class(std::max<int64_t>(max_m, max_n))];
        if (dt.valid && dt.split == 0) split = false;
        if (dt.valid && dt.split == 2) per_pair_tile = true;
    }
    int blocks = 0;
    int err = launch_doc_solver(A, mfma, chunk, lds, 0, stream, &blocks, split);
    if (err != 0) return device_fail(h, err, "occupancy query");
    if (blocks < 1) return fail(h, NNSEMD_ERR_UNSUPPORTED, "pair workgroup does not fit on a compute unit");
    const int64_t slot = (int64_t)doc_slot_bytes(mcap, ncap);
    // (at most 2^24 pairs per launch: the stripe records pack the pair position in 25 bits)
    const int64_t per_launch = std::max<int64_t>(
        1, std::min<int64_t>({A.num_pairs, (int64_t)(kDocTileBudget / (size_t)slot), (int64_t)1 << 24}));
    const size_t need = (size_t)slot * (size_t)per_launch;
    if (h->doc_bytes < need) {
        if (h->doc_tiles) (void)hipFree(h->doc_tiles);
        h->doc_tiles = nullptr;
        h->doc_bytes = 0;
        if (hipMalloc((void**)&h->doc_tiles, need) != hipSuccess)
            return fail(h, NNSEMD_ERR_OUT_OF_MEMORY, "key-tile scratch");
        h->doc_bytes = need;
    }
    A.scratch = h->doc_tiles;
    A.slot_bytes = slot;
    A.phase_cycles = h->phase_cycles;
    if (A.x_off != nullptr && A.num_pairs > 1 && o.schedule == NNSEMD_SCHEDULE_LONGEST_FIRST) {
        nnsemd_status_t s = schedule(h, A.x_off, A.y_off, A.pair_x, A.pair_y, A.num_pairs, A.num_x_sets,
                                     A.num_y_sets, stream);
        if (s != NNSEMD_OK) return s;
        A.order = h->order;
    }
    A.xnorm = nullptr;
    if (split && A.num_pairs > 0) {
        const int64_t sets = A.x_off != nullptr ? A.num_x_sets : 1;
        const size_t xb = sizeof(double) * (size_t)std::max<int64_t>(sets, 1) * (size_t)mcap;
        if (h->doc_xnorm_bytes < xb) {
            if (h->doc_xnorm) (void)hipFree(h->doc_xnorm);
            h->doc_xnorm = nullptr;
            h->doc_xnorm_bytes = 0;
            if (hipMalloc((void**)&h->doc_xnorm, xb) != hipSuccess)
                return fail(h, NNSEMD_ERR_OUT_OF_MEMORY, "supplier norm scratch");
            h->doc_xnorm_bytes = xb;
        }
        A.xnorm = h->doc_xnorm;
        err = launch_doc_xnorm(A, stream);
        if (err != 0) return device_fail(h, err, "supplier norm launch");
    }
    // One supplier set for every pair (one query against many candidates):
    // the tile pass stages it once per workgroup and runs stripe by stripe.
    A.stripes = nullptr;
    A.stripe_total = nullptr;
    A.tile_grid = 0;
    if (split && !per_pair_tile && A.x_off != nullptr && A.num_x_sets == 1 && A.num_pairs > 0 &&
        doc_shared_tile_lds(mcap) <= h->max_lds) {
        const int occ = doc_shared_tile_occupancy(mcap);
        if (occ >= 1) {
            // one 16-byte record per 32 consumers of a pair (at least one)
            const int64_t rmax = (ncap + 31) / 32;
            const size_t sb = 16 * ((size_t)per_launch * (size_t)rmax) + 256;
            if (h->doc_stripes_bytes < sb) {
                if (h->doc_stripes) (void)hipFree(h->doc_stripes);
                h->doc_stripes = nullptr;
                h->doc_stripes_bytes = 0;
                if (hipMalloc((void**)&h->doc_stripes, sb) != hipSuccess)
                    return fail(h, NNSEMD_ERR_OUT_OF_MEMORY, "stripe list");
                h->doc_stripes_bytes = sb;
            }
            A.stripe_total = h->doc_stripes;
            A.stripes = reinterpret_cast<int4*>(h->doc_stripes + 64);
            // a wavefront for every record of the launch, at most the
            // resident workgroups of the whole chip
            const int64_t wpg = doc_shared_tile_threads() / 64;
            const int64_t want = (std::min<int64_t>(per_launch, A.num_pairs) * rmax + wpg - 1) / wpg;
            A.tile_grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)occ * h->num_cus));
        }
    }
    for (int64_t base = 0; base < A.num_pairs; base += per_launch) {
        A.pair_base = base;
        const int grid = (int)std::min<int64_t>(per_launch, A.num_pairs - base);
        err = launch_doc_solver(A, mfma, chunk, lds, grid, stream, nullptr, split);
        if (err != 0) return device_fail(h, err, "high-dimensional solver launch");
    }
    return NNSEMD_OK;
}

// Whether one pair of FP32 points fits the one-workgroup path.
bool fits_on_chip(nnsemd_handle_t h, int64_t m, int64_t n, int32_t d, int32_t threads_opt) {
    const int threads = threads_opt > 0 ? threads_opt : 256;
    const int64_t maxp = std::max<int64_t>({m, n, 1});
    const int chunk_cap = threads == 256 ? 16 : 8;
    const PairLdsLayout lay = pair_lds_layout((int)std::min<int64_t>(std::max<int64_t>(m, 1), 1 << 20),
                                              (int)std::min<int64_t>(std::max<int64_t>(n, 1), 1 << 20),
                                              record_stride(std::max(1, std::min(d, 7))), 0, true);
    return (maxp + threads - 1) / threads <= chunk_cap && lay.total + 8192 <= h->max_lds;
}

nnsemd_status_t run_docs_l1(nnsemd_handle_t h, DocArgs& A, int64_t max_m, int64_t max_n, nnsemd_dtype_t dtype,
                            const nnsemd_options_t& o, void* stream) {
    if (A.d > kDocMaxDim) return fail(h, NNSEMD_ERR_UNSUPPORTED, "d above 65536");
    if (max_m > kCostMaxSide || max_n > kCostMaxSide)
        return fail(h, NNSEMD_ERR_UNSUPPORTED, "high-dimensional L1 supports up to 4096 points per side");
    if (o.threads != 0 && o.threads != 256)
        return fail(h, NNSEMD_ERR_UNSUPPORTED, "high-dimensional path runs 256-thread workgroups");
    const int64_t mcap = std::max<int64_t>(max_m, 1), ncap = std::max<int64_t>(max_n, 1);
    A.max_m = (int32_t)mcap;
    A.max_n = (int32_t)ncap;
    const int64_t stride = mcap * ncap;  // FP64 entries per pair
    const int64_t per_launch =
        std::max<int64_t>(1, std::min<int64_t>(A.num_pairs, (int64_t)(kDocTileBudget / (8 * (size_t)stride))));
    const size_t need = 8 * (size_t)stride * (size_t)per_launch;
    if (h->doc_bytes < need) {
        if (h->doc_tiles) (void)hipFree(h->doc_tiles);
        h->doc_tiles = nullptr;
        h->doc_bytes = 0;
        if (hipMalloc((void**)&h->doc_tiles, need) != hipSuccess)
            return fail(h, NNSEMD_ERR_OUT_OF_MEMORY, "L1 distance scratch");
        h->doc_bytes = need;
    }
    double* tiles = reinterpret_cast<double*>(h->doc_tiles);
    CostArgs C{};
    C.num_pairs = A.num_pairs;
    C.D = tiles;
    C.d_stride = stride;
    C.a = A.a;
    C.b = A.b;
    C.single_m = A.single_m;
    C.single_n = A.single_n;
    if (A.x_off != nullptr) {
        C.a_off = A.x_off;
        C.b_off = A.y_off;
        C.pair_x = A.pair_x;
        C.pair_y = A.pair_y;
        C.num_a_sets = A.num_x_sets;
        C.num_b_sets = A.num_y_sets;
    }
    C.costs = A.costs;
    C.plan_src = A.plan_src;
    C.plan_dst = A.plan_dst;
    C.plan_flow = A.plan_flow;
    C.plan_off = A.plan_off;
    C.single_plan_cap = A.single_plan_cap;
    C.stats = A.stats;
    nnsemd_options_t oc = o;
    oc.schedule = NNSEMD_SCHEDULE_AS_GIVEN;  // chunks run in the given order
    for (int64_t base = 0; base < A.num_pairs; base += per_launch) {
        const int grid = (int)std::min<int64_t>(per_launch, A.num_pairs - base);
        A.pair_base = base;
        const int err = launch_l1_tiles(A, dtype == NNSEMD_BF16, tiles, stride, grid, stream);
        if (err != 0) return device_fail(h, err, "L1 distance launch");
        CostArgs Cc = C;
        Cc.pair_base = base;
        Cc.num_pairs = grid;
        nnsemd_status_t s = run_cost(h, Cc, max_m, max_n, true, oc, stream);
        if (s != NNSEMD_OK) return s;
    }
    return NNSEMD_OK;
}

// FP32 points with d <= 7 take the point path; BF16 points (matrix-core
// mode) and FP32 points with d > 7 take the high-dimensional path.
bool use_doc_path(int32_t d, nnsemd_dtype_t dtype) { return dtype == NNSEMD_BF16 || d > 7; }

// ---- surrogate helpers
struct Carver {
    size_t off = 0;
    size_t take(size_t bytes) {
        const size_t o = align_up(off, 256);
        off = o + bytes;
        return o;
    }
};

nnsemd_status_t sg_workspace(nnsemd_handle_t h, size_t bytes) {
    if (h->sg_bytes >= bytes) return NNSEMD_OK;
    if (h->sg_ws) (void)hipFree(h->sg_ws);
    h->sg_ws = nullptr;
    h->sg_bytes = 0;
    if (hipMalloc((void**)&h->sg_ws, bytes) != hipSuccess) return fail(h, NNSEMD_ERR_OUT_OF_MEMORY, "surrogate workspace");
    h->sg_bytes = bytes;
    return NNSEMD_OK;
}

// BF16 weight copies from the FP32 master parameters (enqueued on stream).
nnsemd_status_t sg_quantize(nnsemd_handle_t h, const float* theta, sg::SgQuant& q, void* stream) {
    constexpr int64_t Hd = kSgHidden;
    Carver c;
    const size_t oW1 = c.take(sizeof(float) * 3 * Hd), ow4 = c.take(sizeof(float) * Hd);
    const size_t oW2 = c.take(2 * Hd * Hd), oW2T = c.take(2 * Hd * Hd);
    const size_t oW3 = c.take(2 * Hd * 3 * Hd), oW3T = c.take(2 * Hd * 3 * Hd);
    if (h->sg_quant == nullptr && hipMalloc((void**)&h->sg_quant, align_up(c.off, 256)) != hipSuccess) {
        h->sg_quant = nullptr;
        return fail(h, NNSEMD_ERR_OUT_OF_MEMORY, "surrogate weights");
    }
    char* b = h->sg_quant;
    q.W1 = reinterpret_cast<float*>(b + oW1);
    q.w4 = reinterpret_cast<float*>(b + ow4);
    q.W2 = reinterpret_cast<uint16_t*>(b + oW2);
    q.W2T = reinterpret_cast<uint16_t*>(b + oW2T);
    q.W3 = reinterpret_cast<uint16_t*>(b + oW3);
    q.W3T = reinterpret_cast<uint16_t*>(b + oW3T);
    const int err = sg::launch_prepare(theta, q, stream);
    if (err != 0) return device_fail(h, err, "surrogate weight conversion");
    return NNSEMD_OK;
}

size_t sg_predict_bytes(int64_t B) {
    const int64_t Bpad = (B + 63) / 64 * 64;
    return align_up(2 * (size_t)Bpad * 3 * kSgHidden, 256) + align_up(4 * (size_t)Bpad * kSgHidden, 256) + 256;
}

sg::SgPredictWork sg_predict_carve(char* base, int64_t B) {
    const int64_t Bpad = (B + 63) / 64 * 64;
    Carver c;
    const size_t oZ = c.take(2 * (size_t)Bpad * 3 * kSgHidden), oP = c.take(4 * (size_t)Bpad * kSgHidden);
    return sg::SgPredictWork{reinterpret_cast<uint16_t*>(base + oZ), reinterpret_cast<float*>(base + oP)};
}

constexpr int64_t kSgMaxRows = (int64_t)1 << 30;

// Grow-on-demand device buffer of the handle (contents are not kept).
nnsemd_status_t grow(nnsemd_handle_t h, char** buf, size_t* cap, size_t bytes, const char* what) {
    if (*cap >= bytes) return NNSEMD_OK;
    if (*buf) (void)hipFree(*buf);
    *buf = nullptr;
    *cap = 0;
    if (hipMalloc((void**)buf, bytes) != hipSuccess) {
        *buf = nullptr;
        return fail(h, NNSEMD_ERR_OUT_OF_MEMORY, what);
    }
    *cap = bytes;
    return NNSEMD_OK;
}

// Barycentric map of a device plan; rows and the plan capacity are host
// values, the number of entries used may be a device count.
nnsemd_status_t run_map(nnsemd_handle_t h, const int32_t* src, const int32_t* dst, const double* flow, int64_t cap,
                        const int64_t* nnz, const float* P, int64_t p_rows, int d, int side, int64_t rows,
                        double* map, void* stream) {
    if (rows == 0) return NNSEMD_OK;
    nnsemd_status_t s = grow(h, &h->map_ws, &h->map_bytes, map_ws_bytes(rows, cap), "map workspace");
    if (s != NNSEMD_OK) return s;
    const MapWork w = map_ws_carve(h->map_ws, rows, cap);
    const int err = launch_barycentric_map(src, dst, flow, cap, nnz, P, p_rows, d, side, rows, map, w, stream);
    if (err != 0) return device_fail(h, err, "barycentric map launch");
    return NNSEMD_OK;
}

nnsemd_status_t check_common(nnsemd_handle_t h, int32_t d, nnsemd_dtype_t dtype, nnsemd_metric_t metric,
                             const nnsemd_options_t& o) {
    if (d < 1) return fail(h, NNSEMD_ERR_INVALID_ARG, "d must be >= 1");
    if (dtype != NNSEMD_F32 && dtype != NNSEMD_BF16) return fail(h, NNSEMD_ERR_INVALID_ARG, "bad dtype");
    if (metric != NNSEMD_L2 && metric != NNSEMD_SQEUCLIDEAN && metric != NNSEMD_L1)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "bad metric");
    if (o.protocol != NNSEMD_GREEDY && o.protocol != NNSEMD_RANDOM)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "bad protocol");
    if (o.schedule != NNSEMD_SCHEDULE_LONGEST_FIRST && o.schedule != NNSEMD_SCHEDULE_AS_GIVEN)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "bad schedule");
    if (o.path != NNSEMD_PATH_AUTO && o.path != NNSEMD_PATH_ON_CHIP && o.path != NNSEMD_PATH_MULTI &&
        o.path != NNSEMD_PATH_MULTI_NO_TAIL)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "bad path");
    if (o.reserved != 0) return fail(h, NNSEMD_ERR_INVALID_ARG, "reserved option field must be 0");
    if (o.mode != NNSEMD_MODE_FP32 && o.mode != NNSEMD_MODE_BF16_MFMA_REFINE)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "bad mode");
    if (o.mode == NNSEMD_MODE_FP32 && dtype != NNSEMD_F32)
        return fail(h, NNSEMD_ERR_UNSUPPORTED, "FP32 mode takes FP32 points");
    if (o.mode == NNSEMD_MODE_BF16_MFMA_REFINE && dtype != NNSEMD_BF16)
        return fail(h, NNSEMD_ERR_UNSUPPORTED, "BF16 matrix-core mode takes BF16 points");
    return NNSEMD_OK;
}

}  // namespace

extern "C" {

nnsemd_status_t nnsemd_create(nnsemd_handle_t* out, int32_t device) {
    if (out == nullptr) return NNSEMD_ERR_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return NNSEMD_ERR_INVALID_ARG;
    nnsemd_handle* h = new (std::nothrow) nnsemd_handle();
    if (h == nullptr) return NNSEMD_ERR_OUT_OF_MEMORY;
    h->device = device;
    DeviceGuard g(device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete h;
        return NNSEMD_ERR_DEVICE;
    }
    {
        // the device address of this GPU's fixed scratch, taken once per device
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (device < kMaxDevices && g_scratch_dev[device] == nullptr) {
            void* ptr = nullptr;
            if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) {
                delete h;
                return NNSEMD_ERR_DEVICE;
            }
            g_scratch_dev[device] = static_cast<int32_t*>(ptr);
        }
        h->fixed_order = device < kMaxDevices ? g_scratch_dev[device] : nullptr;
    }
    h->num_cus = prop.multiProcessorCount;
    h->max_lds = prop.sharedMemPerBlock;
    int optin = 0;
    if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, device) == hipSuccess &&
        optin > 0)
        h->max_lds = std::max<size_t>(h->max_lds, (size_t)optin);
    *out = h;
    return NNSEMD_OK;
}

nnsemd_status_t nnsemd_destroy(nnsemd_handle_t h) {
    if (h == nullptr) return NNSEMD_ERR_INVALID_ARG;
    {
        DeviceGuard g(h->device);
        (void)hipDeviceSynchronize();
        if (h->order) (void)hipFree(h->order);
        if (h->lp_base) (void)hipFree(h->lp_base);
        if (h->lp_host) (void)hipHostFree(h->lp_host);
        if (h->topk_ws) (void)hipFree(h->topk_ws);
        if (h->doc_xnorm) (void)hipFree(h->doc_xnorm);
        if (h->doc_stripes) (void)hipFree(h->doc_stripes);
        if (h->doc_tiles) (void)hipFree(h->doc_tiles);
        if (h->sg_quant) (void)hipFree(h->sg_quant);
        if (h->sg_ws) (void)hipFree(h->sg_ws);
        if (h->map_ws) (void)hipFree(h->map_ws);
        if (h->ct_ws) (void)hipFree(h->ct_ws);
        if (h->map_plan) (void)hipFree(h->map_plan);
    }
    delete h;
    return NNSEMD_OK;
}

const char* nnsemd_status_string(nnsemd_status_t s) {
    switch (s) {
        case NNSEMD_OK: return "ok";
        case NNSEMD_ERR_INVALID_ARG: return "invalid argument";
        case NNSEMD_ERR_MASS_MISMATCH: return "total masses differ by more than 1e-5 relative";
        case NNSEMD_ERR_CAPACITY: return "plan buffer smaller than m + n - 1";
        case NNSEMD_ERR_OUT_OF_MEMORY: return "out of memory";
        case NNSEMD_ERR_DEVICE: return "device error";
        case NNSEMD_ERR_NOT_CONVERGED: return "round cap reached";
        case NNSEMD_ERR_UNSUPPORTED: return "unsupported combination";
    }
    return "unknown status";
}

const char* nnsemd_last_error(nnsemd_handle_t h) { return h ? h->last_error.c_str() : ""; }

nnsemd_status_t emd_approx(nnsemd_handle_t h, const void* X, const float* a, int64_t m, const void* Y,
                           const float* b, int64_t n, int32_t d, nnsemd_dtype_t dtype,
                           nnsemd_metric_t metric, const nnsemd_options_t* opts, double* cost,
                           int32_t* plan_src, int32_t* plan_dst, double* plan_flow, int64_t plan_capacity,
                           nnsemd_stats_t* stats, void* stream) {
    if (h == nullptr) return NNSEMD_ERR_INVALID_ARG;
    h->last_error.clear();
    const nnsemd_options_t o = opts ? *opts : default_options();
    nnsemd_status_t s = check_common(h, d, dtype, metric, o);
    if (s != NNSEMD_OK) return s;
    if (m < 0 || n < 0) return fail(h, NNSEMD_ERR_INVALID_ARG, "negative size");
    if (cost == nullptr) return fail(h, NNSEMD_ERR_INVALID_ARG, "cost must not be NULL");
    if ((m > 0 && (X == nullptr || a == nullptr)) || (n > 0 && (Y == nullptr || b == nullptr)))
        return fail(h, NNSEMD_ERR_INVALID_ARG, "NULL point or mass array");
    const bool plan = plan_src != nullptr || plan_dst != nullptr || plan_flow != nullptr;
    if (plan && (plan_src == nullptr || plan_dst == nullptr || plan_flow == nullptr))
        return fail(h, NNSEMD_ERR_INVALID_ARG, "plan arrays must be all given or all NULL");
    if (plan && m + n > 0 && plan_capacity < m + n - 1)
        return fail(h, NNSEMD_ERR_CAPACITY, "plan capacity below m + n - 1");
    DeviceGuard g(h->device);
    if (use_doc_path(d, dtype)) {
        if (o.path == NNSEMD_PATH_MULTI || o.path == NNSEMD_PATH_MULTI_NO_TAIL)
            return fail(h, NNSEMD_ERR_UNSUPPORTED, "multi-workgroup path supports FP32 points with d <= 7");
        DocArgs A{};
        A.num_pairs = 1;
        A.X = X;
        A.a = a;
        A.Y = Y;
        A.b = b;
        A.single_m = m;
        A.single_n = n;
        A.d = d;
        A.metric = metric;
        A.costs = cost;
        A.plan_src = plan ? plan_src : nullptr;
        A.plan_dst = plan ? plan_dst : nullptr;
        A.plan_flow = plan ? plan_flow : nullptr;
        A.single_plan_cap = plan_capacity;
        A.stats = stats;
        return run_docs(h, A, m, n, dtype, o, stream);
    }
    const bool multi = o.path == NNSEMD_PATH_MULTI || o.path == NNSEMD_PATH_MULTI_NO_TAIL ||
                       (o.path == NNSEMD_PATH_AUTO && !fits_on_chip(h, m, n, d, o.threads));
    if (multi) {
        LPArgs L{};
        L.m = m;
        L.n = n;
        L.X = static_cast<const float*>(X);
        L.a = a;
        L.Y = static_cast<const float*>(Y);
        L.b = b;
        L.metric = metric;
        L.protocol = o.protocol;
        L.seed = o.seed;
        L.max_rounds = o.max_rounds;
        L.cost = cost;
        L.plan_src = plan ? plan_src : nullptr;
        L.plan_dst = plan ? plan_dst : nullptr;
        L.plan_flow = plan ? plan_flow : nullptr;
        L.stats = stats;
        L.tail_cap = o.path == NNSEMD_PATH_MULTI_NO_TAIL ? 0 : lp_tail_capacity(d, h->max_lds);
        return run_large(h, L, d, stream);
    }
    PairSolverArgs A{};
    A.num_pairs = 1;
    A.X = static_cast<const float*>(X);
    A.a = a;
    A.Y = static_cast<const float*>(Y);
    A.b = b;
    A.single_m = m;
    A.single_n = n;
    A.metric = metric;
    A.costs = cost;
    A.plan_src = plan ? plan_src : nullptr;
    A.plan_dst = plan ? plan_dst : nullptr;
    A.plan_flow = plan ? plan_flow : nullptr;
    A.single_plan_cap = plan_capacity;
    A.stats = stats;
    return run_pairs(h, A, d, m, n, o, stream);
}

nnsemd_status_t emd_approx_map(nnsemd_handle_t h, const void* X, const float* a, int64_t m, const void* Y,
                               const float* b, int64_t n, int32_t d, nnsemd_dtype_t dtype, nnsemd_metric_t metric,
                               const nnsemd_options_t* opts, double* cost, double* map, int32_t* plan_src,
                               int32_t* plan_dst, double* plan_flow, int64_t plan_capacity, nnsemd_stats_t* stats,
                               void* stream) {
    if (h == nullptr) return NNSEMD_ERR_INVALID_ARG;
    h->last_error.clear();
    const nnsemd_options_t o = opts ? *opts : default_options();
    nnsemd_status_t s = check_common(h, d, dtype, metric, o);
    if (s != NNSEMD_OK) return s;
    if (m < 0 || n < 0) return fail(h, NNSEMD_ERR_INVALID_ARG, "negative size");
    if (cost == nullptr || (map == nullptr && m > 0)) return fail(h, NNSEMD_ERR_INVALID_ARG, "cost and map must not be NULL");
    if ((m > 0 && (X == nullptr || a == nullptr)) || (n > 0 && (Y == nullptr || b == nullptr)))
        return fail(h, NNSEMD_ERR_INVALID_ARG, "NULL point or mass array");
    const bool plan = plan_src != nullptr || plan_dst != nullptr || plan_flow != nullptr;
    if (plan && (plan_src == nullptr || plan_dst == nullptr || plan_flow == nullptr))
        return fail(h, NNSEMD_ERR_INVALID_ARG, "plan arrays must be all given or all NULL");
    if (plan && m + n > 0 && plan_capacity < m + n - 1)
        return fail(h, NNSEMD_ERR_CAPACITY, "plan capacity below m + n - 1");
    if (use_doc_path(d, dtype))
        return fail(h, NNSEMD_ERR_UNSUPPORTED, "the transport map is computed for FP32 points with d <= 7");
    DeviceGuard g(h->device);
    if (o.path == NNSEMD_PATH_MULTI || o.path == NNSEMD_PATH_MULTI_NO_TAIL ||
        (o.path == NNSEMD_PATH_AUTO && !fits_on_chip(h, m, n, d, o.threads))) {
        // the multi-workgroup path accumulates the map while it serves
        LPArgs L{};
        L.m = m;
        L.n = n;
        L.X = static_cast<const float*>(X);
        L.a = a;
        L.Y = static_cast<const float*>(Y);
        L.b = b;
        L.metric = metric;
        L.protocol = o.protocol;
        L.seed = o.seed;
        L.max_rounds = o.max_rounds;
        L.cost = cost;
        L.plan_src = plan ? plan_src : nullptr;
        L.plan_dst = plan ? plan_dst : nullptr;
        L.plan_flow = plan ? plan_flow : nullptr;
        L.stats = stats;
        L.map = map;
        L.tail_cap = o.path == NNSEMD_PATH_MULTI_NO_TAIL ? 0 : lp_tail_capacity(d, h->max_lds);
        return run_large(h, L, d, stream);
    }
    // On-chip solve into the caller's plan (or the handle's), then the map of
    // that plan; the entry count is read on the device from the stats.
    const int64_t cap = std::max<int64_t>(m + n - 1, 1);
    int32_t* ps = plan_src;
    int32_t* pd = plan_dst;
    double* pf = plan_flow;
    nnsemd_stats_t* st = stats;
    int64_t pcap = plan ? plan_capacity : cap;
    if (!plan || stats == nullptr) {
        const size_t need = align_up(sizeof(nnsemd_stats_t), 256) + (plan ? 0 : align_up(16 * (size_t)cap, 256));
        if ((s = grow(h, &h->map_plan, &h->map_plan_bytes, need, "map plan scratch")) != NNSEMD_OK) return s;
        char* base = h->map_plan;
        if (stats == nullptr) st = reinterpret_cast<nnsemd_stats_t*>(base);
        if (!plan) {
            char* pb = base + align_up(sizeof(nnsemd_stats_t), 256);
            pf = reinterpret_cast<double*>(pb);
            ps = reinterpret_cast<int32_t*>(pb + 8 * (size_t)cap);
            pd = ps + cap;
        }
    }
    nnsemd_options_t oc = o;
    oc.path = NNSEMD_PATH_ON_CHIP;
    PairSolverArgs A{};
    A.num_pairs = 1;
    A.X = static_cast<const float*>(X);
    A.a = a;
    A.Y = static_cast<const float*>(Y);
    A.b = b;
    A.single_m = m;
    A.single_n = n;
    A.metric = metric;
    A.costs = cost;
    A.plan_src = ps;
    A.plan_dst = pd;
    A.plan_flow = pf;
    A.single_plan_cap = pcap;
    A.stats = st;
    if ((s = run_pairs(h, A, d, m, n, oc, stream)) != NNSEMD_OK) return s;
    return run_map(h, ps, pd, pf, pcap, &st->nnz, static_cast<const float*>(Y), n, d, NNSEMD_MAP_SUPPLIERS, m, map,
                   stream);
}

nnsemd_status_t emd_approx_cost(nnsemd_handle_t h, const void* D, nnsemd_dtype_t dtype, const float* a, int64_t m,
                                const float* b, int64_t n, const nnsemd_options_t* opts, double* cost,
                                int32_t* plan_src, int32_t* plan_dst, double* plan_flow, int64_t plan_capacity,
                                nnsemd_stats_t* stats, void* stream) {
    if (h == nullptr) return NNSEMD_ERR_INVALID_ARG;
    h->last_error.clear();
    const nnsemd_options_t o = opts ? *opts : default_options();
    nnsemd_status_t s = check_cost_options(h, dtype, o);
    if (s != NNSEMD_OK) return s;
    if (m < 0 || n < 0) return fail(h, NNSEMD_ERR_INVALID_ARG, "negative size");
    if (cost == nullptr) return fail(h, NNSEMD_ERR_INVALID_ARG, "cost must not be NULL");
    if ((m > 0 && a == nullptr) || (n > 0 && b == nullptr) || (m > 0 && n > 0 && D == nullptr))
        return fail(h, NNSEMD_ERR_INVALID_ARG, "NULL matrix or mass array");
    const bool plan = plan_src != nullptr || plan_dst != nullptr || plan_flow != nullptr;
    if (plan && (plan_src == nullptr || plan_dst == nullptr || plan_flow == nullptr))
        return fail(h, NNSEMD_ERR_INVALID_ARG, "plan arrays must be all given or all NULL");
    if (plan && m + n > 0 && plan_capacity < m + n - 1)
        return fail(h, NNSEMD_ERR_CAPACITY, "plan capacity below m + n - 1");
    DeviceGuard g(h->device);
    CostArgs A{};
    A.num_pairs = 1;
    A.D = D;
    A.a = a;
    A.b = b;
    A.single_m = m;
    A.single_n = n;
    A.costs = cost;
    A.plan_src = plan ? plan_src : nullptr;
    A.plan_dst = plan ? plan_dst : nullptr;
    A.plan_flow = plan ? plan_flow : nullptr;
    A.single_plan_cap = plan_capacity;
    A.stats = stats;
    return run_cost(h, A, m, n, dtype == NNSEMD_F64, o, stream);
}

nnsemd_status_t emd_approx_cost_batched(nnsemd_handle_t h, int64_t num_pairs, const void* Dcat, const int64_t* d_off,
                                        nnsemd_dtype_t dtype, const float* acat, const int64_t* a_off,
                                        const float* bcat, const int64_t* b_off, int64_t max_m, int64_t max_n,
                                        const nnsemd_options_t* opts, double* costs, int32_t* plan_src,
                                        int32_t* plan_dst, double* plan_flow, const int64_t* plan_off,
                                        nnsemd_stats_t* stats, void* stream) {
    if (h == nullptr) return NNSEMD_ERR_INVALID_ARG;
    h->last_error.clear();
    const nnsemd_options_t o = opts ? *opts : default_options();
    nnsemd_status_t s = check_cost_options(h, dtype, o);
    if (s != NNSEMD_OK) return s;
    if (num_pairs < 0 || max_m < 0 || max_n < 0) return fail(h, NNSEMD_ERR_INVALID_ARG, "negative count");
    if (num_pairs == 0) return NNSEMD_OK;
    if (num_pairs > 0x7fffffffLL - (1LL << 20)) return fail(h, NNSEMD_ERR_UNSUPPORTED, "too many pairs for one call");
    if (costs == nullptr || Dcat == nullptr || d_off == nullptr || acat == nullptr || a_off == nullptr ||
        bcat == nullptr || b_off == nullptr)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "NULL required array");
    const bool plan = plan_src != nullptr || plan_dst != nullptr || plan_flow != nullptr;
    if (plan && (plan_src == nullptr || plan_dst == nullptr || plan_flow == nullptr || plan_off == nullptr))
        return fail(h, NNSEMD_ERR_INVALID_ARG, "plan arrays and plan_off must be all given or all NULL");
    DeviceGuard g(h->device);
    CostArgs A{};
    A.num_pairs = num_pairs;
    A.D = Dcat;
    A.d_off = d_off;
    A.a = acat;
    A.a_off = a_off;
    A.b = bcat;
    A.b_off = b_off;
    A.costs = costs;
    A.plan_src = plan ? plan_src : nullptr;
    A.plan_dst = plan ? plan_dst : nullptr;
    A.plan_flow = plan ? plan_flow : nullptr;
    A.plan_off = plan ? plan_off : nullptr;
    A.stats = stats;
    A.num_a_sets = num_pairs;
    A.num_b_sets = num_pairs;
    return run_cost(h, A, max_m, max_n, dtype == NNSEMD_F64, o, stream);
}

nnsemd_status_t nnsemd_colour_transfer(nnsemd_handle_t h, const uint8_t* ref_rgb, int64_t ref_pixels,
                                       const uint8_t* src_rgb, int64_t src_pixels, int32_t k_ref, int32_t k_src,
                                       int32_t iters, nnsemd_metric_t metric, const nnsemd_options_t* opts,
                                       uint8_t* out_rgb, float* ref_palette, float* ref_mass, float* src_palette,
                                       float* src_mass, int32_t* src_assign, double* cost, nnsemd_stats_t* stats,
                                       void* stream) {
    if (h == nullptr) return NNSEMD_ERR_INVALID_ARG;
    h->last_error.clear();
    const nnsemd_options_t o = opts ? *opts : default_options();
    nnsemd_status_t s = check_common(h, 3, NNSEMD_F32, metric, o);
    if (s != NNSEMD_OK) return s;
    if (ref_rgb == nullptr || src_rgb == nullptr || out_rgb == nullptr)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "NULL image");
    if (ref_pixels < 1 || src_pixels < 1 || ref_pixels > 0x7fffffffLL || src_pixels > 0x7fffffffLL)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "pixel counts must be in [1, 2^31)");
    if (k_ref < 1 || k_src < 1 || k_ref > 1024 || k_src > 1024 || iters < 0 || iters > 1000)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "need 1 <= k <= 1024 and 0 <= iters <= 1000");
    if (kmeans_lds_bytes(std::max(k_ref, k_src)) + 8192 > h->max_lds)
        return fail(h, NNSEMD_ERR_UNSUPPORTED, "palette does not fit in LDS");
    DeviceGuard g(h->device);
    // workspace: both clusterings, both palettes, plan, stats, map
    Carver c;
    const size_t oCr = c.take(24 * (size_t)k_ref), oSr = c.take(32 * (size_t)k_ref);
    const size_t oAr = c.take(4 * (size_t)ref_pixels);
    const size_t oCs = c.take(24 * (size_t)k_src), oSs = c.take(32 * (size_t)k_src);
    const size_t oAs = c.take(4 * (size_t)src_pixels);
    const size_t oXr = c.take(12 * (size_t)k_ref), oar = c.take(4 * (size_t)k_ref);
    const size_t oYs = c.take(12 * (size_t)k_src), obs = c.take(4 * (size_t)k_src);
    const int64_t cap = (int64_t)k_ref + k_src - 1;
    const size_t opf = c.take(8 * (size_t)cap), ops = c.take(4 * (size_t)cap), opd = c.take(4 * (size_t)cap);
    const size_t ost = c.take(sizeof(nnsemd_stats_t)), ocost = c.take(8), omap = c.take(24 * (size_t)k_src);
    if ((s = grow(h, &h->ct_ws, &h->ct_bytes, align_up(c.off, 256), "colour transfer workspace")) != NNSEMD_OK)
        return s;
    char* b = h->ct_ws;
    double* Cr = reinterpret_cast<double*>(b + oCr);
    double* Cs = reinterpret_cast<double*>(b + oCs);
    auto* Sr = reinterpret_cast<unsigned long long*>(b + oSr);
    auto* Ss = reinterpret_cast<unsigned long long*>(b + oSs);
    int32_t* Ar = reinterpret_cast<int32_t*>(b + oAr);
    int32_t* As = src_assign ? src_assign : reinterpret_cast<int32_t*>(b + oAs);
    float* Xr = ref_palette ? ref_palette : reinterpret_cast<float*>(b + oXr);
    float* ar = ref_mass ? ref_mass : reinterpret_cast<float*>(b + oar);
    float* Ys = src_palette ? src_palette : reinterpret_cast<float*>(b + oYs);
    float* bs = src_mass ? src_mass : reinterpret_cast<float*>(b + obs);
    double* pf = reinterpret_cast<double*>(b + opf);
    int32_t* ps = reinterpret_cast<int32_t*>(b + ops);
    int32_t* pd = reinterpret_cast<int32_t*>(b + opd);
    nnsemd_stats_t* st = stats ? stats : reinterpret_cast<nnsemd_stats_t*>(b + ost);
    double* cst = cost ? cost : reinterpret_cast<double*>(b + ocost);
    double* T = reinterpret_cast<double*>(b + omap);
    int err = launch_kmeans(ref_rgb, ref_pixels, k_ref, iters, Cr, Sr, Ar, Xr, ar, stream);
    if (err == 0) err = launch_kmeans(src_rgb, src_pixels, k_src, iters, Cs, Ss, As, Ys, bs, stream);
    if (err != 0) return device_fail(h, err, "palette reduction");
    nnsemd_options_t oc = o;
    oc.path = NNSEMD_PATH_ON_CHIP;
    PairSolverArgs A{};
    A.num_pairs = 1;
    A.X = Xr;
    A.a = ar;
    A.Y = Ys;
    A.b = bs;
    A.single_m = k_ref;
    A.single_n = k_src;
    A.metric = metric;
    A.costs = cst;
    A.plan_src = ps;
    A.plan_dst = pd;
    A.plan_flow = pf;
    A.single_plan_cap = cap;
    A.stats = st;
    if ((s = run_pairs(h, A, 3, k_ref, k_src, oc, stream)) != NNSEMD_OK) return s;
    if ((s = run_map(h, ps, pd, pf, cap, &st->nnz, Xr, k_ref, 3, NNSEMD_MAP_CONSUMERS, k_src, T, stream)) != NNSEMD_OK)
        return s;
    err = launch_recolour(src_rgb, As, src_pixels, T, out_rgb, stream);
    if (err != 0) return device_fail(h, err, "recolour");
    return NNSEMD_OK;
}

nnsemd_status_t emd_barycentric_map(nnsemd_handle_t h, const int32_t* plan_src, const int32_t* plan_dst,
                                    const double* plan_flow, int64_t plan_capacity, const int64_t* plan_nnz,
                                    const float* P, int64_t p_rows, int32_t d, int64_t rows, nnsemd_map_side_t side,
                                    double* map, void* stream) {
    if (h == nullptr) return NNSEMD_ERR_INVALID_ARG;
    h->last_error.clear();
    if (side != NNSEMD_MAP_SUPPLIERS && side != NNSEMD_MAP_CONSUMERS)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "bad map side");
    if (d < 1 || d > 8) return fail(h, NNSEMD_ERR_UNSUPPORTED, "the map supports 1 <= d <= 8");
    if (plan_capacity < 0 || p_rows < 0 || rows < 0 || rows > 0x7fffffffLL || p_rows > 0x7fffffffLL ||
        plan_capacity > 0x7fffffffLL)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "sizes must be in [0, 2^31)");
    if (rows > 0 && map == nullptr) return fail(h, NNSEMD_ERR_INVALID_ARG, "map must not be NULL");
    if (plan_capacity > 0 && (plan_src == nullptr || plan_dst == nullptr || plan_flow == nullptr || P == nullptr))
        return fail(h, NNSEMD_ERR_INVALID_ARG, "NULL plan or point array");
    DeviceGuard g(h->device);
    return run_map(h, plan_src, plan_dst, plan_flow, plan_capacity, plan_nnz, P, p_rows, d, (int)side, rows, map,
                   stream);
}

nnsemd_status_t emd_approx_batched(nnsemd_handle_t h, int64_t num_pairs, const void* Xcat, const float* acat,
                                   const int64_t* x_off, int64_t num_x_sets, const void* Ycat,
                                   const float* bcat, const int64_t* y_off, int64_t num_y_sets,
                                   const int32_t* pair_x, const int32_t* pair_y, int64_t max_m, int64_t max_n,
                                   int32_t d, nnsemd_dtype_t dtype, nnsemd_metric_t metric,
                                   const nnsemd_options_t* opts, double* costs, int32_t* plan_src,
                                   int32_t* plan_dst, double* plan_flow, const int64_t* plan_off,
                                   nnsemd_stats_t* stats, void* stream) {
    if (h == nullptr) return NNSEMD_ERR_INVALID_ARG;
    h->last_error.clear();
    const nnsemd_options_t o = opts ? *opts : default_options();
    nnsemd_status_t s = check_common(h, d, dtype, metric, o);
    if (s != NNSEMD_OK) return s;
    if (num_pairs < 0 || num_x_sets < 0 || num_y_sets < 0 || max_m < 0 || max_n < 0)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "negative count");
    if (num_pairs == 0) return NNSEMD_OK;
    if (costs == nullptr || x_off == nullptr || y_off == nullptr || Xcat == nullptr || Ycat == nullptr ||
        acat == nullptr || bcat == nullptr)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "NULL required array");
    if (num_x_sets == 0 || num_y_sets == 0) return fail(h, NNSEMD_ERR_INVALID_ARG, "no point sets");
    if ((pair_x == nullptr && num_x_sets < num_pairs) || (pair_y == nullptr && num_y_sets < num_pairs))
        return fail(h, NNSEMD_ERR_INVALID_ARG, "fewer sets than pairs without a pair table");
    const bool plan = plan_src != nullptr || plan_dst != nullptr || plan_flow != nullptr;
    if (plan && (plan_src == nullptr || plan_dst == nullptr || plan_flow == nullptr || plan_off == nullptr))
        return fail(h, NNSEMD_ERR_INVALID_ARG, "plan arrays and plan_off must be all given or all NULL");
    if (num_pairs > 0x7fffffffLL - (1LL << 20))
        return fail(h, NNSEMD_ERR_UNSUPPORTED, "too many pairs for one call");
    DeviceGuard g(h->device);
    if (use_doc_path(d, dtype)) {
        DocArgs A{};
        A.num_pairs = num_pairs;
        A.X = Xcat;
        A.a = acat;
        A.x_off = x_off;
        A.num_x_sets = num_x_sets;
        A.Y = Ycat;
        A.b = bcat;
        A.y_off = y_off;
        A.num_y_sets = num_y_sets;
        A.pair_x = pair_x;
        A.pair_y = pair_y;
        A.d = d;
        A.metric = metric;
        A.costs = costs;
        A.plan_src = plan ? plan_src : nullptr;
        A.plan_dst = plan ? plan_dst : nullptr;
        A.plan_flow = plan ? plan_flow : nullptr;
        A.plan_off = plan ? plan_off : nullptr;
        A.stats = stats;
        return run_docs(h, A, max_m, max_n, dtype, o, stream);
    }
    PairSolverArgs A{};
    A.num_pairs = num_pairs;
    A.X = static_cast<const float*>(Xcat);
    A.a = acat;
    A.x_off = x_off;
    A.num_x_sets = num_x_sets;
    A.Y = static_cast<const float*>(Ycat);
    A.b = bcat;
    A.y_off = y_off;
    A.num_y_sets = num_y_sets;
    A.pair_x = pair_x;
    A.pair_y = pair_y;
    A.metric = metric;
    A.costs = costs;
    A.plan_src = plan ? plan_src : nullptr;
    A.plan_dst = plan ? plan_dst : nullptr;
    A.plan_flow = plan ? plan_flow : nullptr;
    A.plan_off = plan ? plan_off : nullptr;
    A.stats = stats;
    return run_pairs(h, A, d, max_m, max_n, o, stream);
}

nnsemd_status_t emd_approx_batched_noalloc(nnsemd_handle_t h, int64_t num_pairs, const void* Xcat,
                                           const float* acat, const int64_t* x_off, int64_t num_x_sets,
                                           const void* Ycat, const float* bcat, const int64_t* y_off,
                                           int64_t num_y_sets, const int32_t* pair_x, const int32_t* pair_y,
                                           int64_t max_m, int64_t max_n, int32_t d, nnsemd_dtype_t dtype,
                                           nnsemd_metric_t metric, const nnsemd_options_t* opts, double* costs,
                                           int32_t* plan_src, int32_t* plan_dst, double* plan_flow,
                                           const int64_t* plan_off, nnsemd_stats_t* stats, void* stream) {
    if (h == nullptr) return NNSEMD_ERR_INVALID_ARG;
    h->last_error.clear();
    const nnsemd_options_t o = opts ? *opts : default_options();
    nnsemd_status_t s = check_common(h, d, dtype, metric, o);
    if (s != NNSEMD_OK) return s;
    if (use_doc_path(d, dtype))
        return fail(h, NNSEMD_ERR_UNSUPPORTED, "the no-allocation call covers FP32 points with 1 <= d <= 7");
    if (num_pairs < 0 || num_x_sets < 0 || num_y_sets < 0 || max_m < 0 || max_n < 0)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "negative count");
    if (num_pairs > kNoAllocMaxPairs)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "the no-allocation call takes at most 65536 pairs");
    if (num_pairs == 0) return NNSEMD_OK;
    if (costs == nullptr || x_off == nullptr || y_off == nullptr || Xcat == nullptr || Ycat == nullptr ||
        acat == nullptr || bcat == nullptr)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "NULL required array");
    if (num_x_sets == 0 || num_y_sets == 0) return fail(h, NNSEMD_ERR_INVALID_ARG, "no point sets");
    if ((pair_x == nullptr && num_x_sets < num_pairs) || (pair_y == nullptr && num_y_sets < num_pairs))
        return fail(h, NNSEMD_ERR_INVALID_ARG, "fewer sets than pairs without a pair table");
    const bool plan = plan_src != nullptr || plan_dst != nullptr || plan_flow != nullptr;
    if (plan && (plan_src == nullptr || plan_dst == nullptr || plan_flow == nullptr || plan_off == nullptr))
        return fail(h, NNSEMD_ERR_INVALID_ARG, "plan arrays and plan_off must be all given or all NULL");
    if (h->fixed_order == nullptr) return fail(h, NNSEMD_ERR_DEVICE, "fixed scratch not available on this device");
    DeviceGuard g(h->device);
    PairSolverArgs A{};
    A.num_pairs = num_pairs;
    A.X = static_cast<const float*>(Xcat);
    A.a = acat;
    A.x_off = x_off;
    A.num_x_sets = num_x_sets;
    A.Y = static_cast<const float*>(Ycat);
    A.b = bcat;
    A.y_off = y_off;
    A.num_y_sets = num_y_sets;
    A.pair_x = pair_x;
    A.pair_y = pair_y;
    A.metric = metric;
    A.costs = costs;
    A.plan_src = plan ? plan_src : nullptr;
    A.plan_dst = plan ? plan_dst : nullptr;
    A.plan_flow = plan ? plan_flow : nullptr;
    A.plan_off = plan ? plan_off : nullptr;
    A.stats = stats;
    return run_pairs(h, A, d, max_m, max_n, o, stream, 0, 0, h->fixed_order);
}

nnsemd_status_t nnsemd_autotune(nnsemd_handle_t h, int32_t d, nnsemd_metric_t metric, int64_t max_m, int64_t max_n,
                                int64_t num_pairs, nnsemd_tuning_t* result, void* stream) {
    if (h == nullptr) return NNSEMD_ERR_INVALID_ARG;
    h->last_error.clear();
    if (d < 1 || d > 7) return fail(h, NNSEMD_ERR_UNSUPPORTED, "autotuning covers the point path, 1 <= d <= 7");
    if (metric != NNSEMD_L2 && metric != NNSEMD_SQEUCLIDEAN && metric != NNSEMD_L1)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "bad metric");
    if (max_m < 1 || max_n < 1 || max_m > 4096 || max_n > 4096 || num_pairs < 1 || num_pairs > 65536)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "need 1 <= max_m, max_n <= 4096 and 1 <= num_pairs <= 65536");
    DeviceGuard g(h->device);
    hipStream_t st = (hipStream_t)stream;
    // Synthetic pairs shaped like the caller's: sides uniform in
    // [max/8, max], coordinates uniform in [0,1)^d, normalised exponential masses.
    std::vector<int64_t> xo(num_pairs + 1, 0), yo(num_pairs + 1, 0);
    uint64_t rs = 0x9E3779B97F4A7C15ull ^ (uint64_t)(d * 131 + metric * 7 + max_m * 3 + max_n);
    auto next = [&rs]() {
        rs += 0x9E3779B97F4A7C15ull;
        uint64_t z = rs;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    auto unif = [&next]() { return (double)(next() >> 11) * 0x1.0p-53; };
    for (int64_t p = 0; p < num_pairs; ++p) {
        const int64_t lm = std::max<int64_t>(1, max_m / 8), ln = std::max<int64_t>(1, max_n / 8);
        xo[p + 1] = xo[p] + lm + (int64_t)(unif() * (double)(max_m - lm + 1));
        yo[p + 1] = yo[p] + ln + (int64_t)(unif() * (double)(max_n - ln + 1));
    }
    auto points = [&](const std::vector<int64_t>& off, std::vector<float>& P, std::vector<float>& w) {
        P.resize((size_t)off.back() * d);
        w.resize((size_t)off.back());
        for (auto& v : P) v = (float)unif();
        for (size_t s = 0; s + 1 < off.size(); ++s) {
            double sum = 0.0;
            for (int64_t i = off[s]; i < off[s + 1]; ++i) sum += (w[i] = (float)-std::log(1.0 - unif()));
            for (int64_t i = off[s]; i < off[s + 1]; ++i) w[i] = (float)(w[i] / sum);
        }
    };
    std::vector<float> X, a, Y, b;
    points(xo, X, a);
    points(yo, Y, b);
    Carver c;
    const size_t oX = c.take(4 * X.size()), oa = c.take(4 * a.size()), oY = c.take(4 * Y.size()),
                 ob = c.take(4 * b.size()), oxo = c.take(8 * xo.size()), oyo = c.take(8 * yo.size()),
                 oc = c.take(8 * (size_t)num_pairs);
    char* base = nullptr;
    if (hipMalloc((void**)&base, align_up(c.off, 256)) != hipSuccess)
        return fail(h, NNSEMD_ERR_OUT_OF_MEMORY, "autotuning inputs");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    nnsemd_status_t status = NNSEMD_OK;
    float best_ms = -1.f, default_ms = -1.f;
    int best_t = 256, best_s = 1;
    bool ok = hipMemcpyAsync(base + oX, X.data(), 4 * X.size(), hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(base + oa, a.data(), 4 * a.size(), hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(base + oY, Y.data(), 4 * Y.size(), hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(base + ob, b.data(), 4 * b.size(), hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(base + oxo, xo.data(), 8 * xo.size(), hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(base + oyo, yo.data(), 8 * yo.size(), hipMemcpyHostToDevice, st) == hipSuccess &&
              hipStreamSynchronize(st) == hipSuccess && hipEventCreate(&e0) == hipSuccess &&
              hipEventCreate(&e1) == hipSuccess;
    if (!ok) status = fail(h, NNSEMD_ERR_DEVICE, "autotuning set-up");
    const int threads_c[2] = {256, 512}, split_c[3] = {1, 2, 4};
    for (int ti = 0; ti < 2 && status == NNSEMD_OK; ++ti) {
        for (int si = 0; si < 3 && status == NNSEMD_OK; ++si) {
            PairSolverArgs A{};
            A.num_pairs = num_pairs;
            A.X = reinterpret_cast<const float*>(base + oX);
            A.a = reinterpret_cast<const float*>(base + oa);
            A.x_off = reinterpret_cast<const int64_t*>(base + oxo);
            A.num_x_sets = num_pairs;
            A.Y = reinterpret_cast<const float*>(base + oY);
            A.b = reinterpret_cast<const float*>(base + ob);
            A.y_off = reinterpret_cast<const int64_t*>(base + oyo);
            A.num_y_sets = num_pairs;
            A.metric = metric;
            A.costs = reinterpret_cast<double*>(base + oc);
            const nnsemd_options_t o = default_options();
            nnsemd_status_t s = run_pairs(h, A, d, max_m, max_n, o, stream, threads_c[ti], split_c[si]);
            if (s == NNSEMD_ERR_UNSUPPORTED) {
                h->last_error.clear();
                continue;  // this configuration does not fit
            }
            if (s != NNSEMD_OK) {
                status = s;
                break;
            }
            float ms = 0.f;
            bool good = hipEventRecord(e0, st) == hipSuccess;
            for (int r = 0; r < 3 && good; ++r)
                good = run_pairs(h, A, d, max_m, max_n, o, stream, threads_c[ti], split_c[si]) == NNSEMD_OK;
            good = good && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                   hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
            if (!good) {
                status = fail(h, NNSEMD_ERR_DEVICE, "autotuning launch");
                break;
            }
            ms /= 3.f;
            if (threads_c[ti] == 256 && split_c[si] == 1) default_ms = ms;
            if (best_ms < 0.f || ms < best_ms) {
                best_ms = ms;
                best_t = threads_c[ti];
                best_s = split_c[si];
            }
        }
    }
    (void)hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(base);
    if (status != NNSEMD_OK) return status;
    if (best_ms < 0.f) return fail(h, NNSEMD_ERR_UNSUPPORTED, "no launch configuration fits these sizes");
    auto& tn = h->tune[d][metric][tune_class(std::max(max_m, max_n))];
    tn.valid = 1;
    tn.threads = best_t;
    tn.split = best_s;
    tn.ms = best_ms;
    if (result) {
        result->threads = best_t;
        result->split = best_s;
        result->ms_best = best_ms;
        result->ms_default = default_ms;
    }
    return NNSEMD_OK;
}

nnsemd_status_t nnsemd_tuning_save(nnsemd_handle_t h, const char* path) {
    if (h == nullptr || path == nullptr) return NNSEMD_ERR_INVALID_ARG;
    FILE* f = std::fopen(path, "w");
    if (f == nullptr) return fail(h, NNSEMD_ERR_INVALID_ARG, "cannot open the tuning file for writing");
    std::fprintf(f, "nnsemd-tuning 2\n");
    for (int d = 1; d <= 7; ++d)
        for (int m = 0; m < 3; ++m)
            for (int c = 0; c < nnsemd_tune_classes; ++c) {
                const auto& t = h->tune[d][m][c];
                if (t.valid) std::fprintf(f, "%d %d %d %d %d %.6f\n", d, m, c, t.threads, t.split, (double)t.ms);
            }
    const bool ok = std::fclose(f) == 0;
    return ok ? NNSEMD_OK : fail(h, NNSEMD_ERR_INVALID_ARG, "writing the tuning file failed");
}

nnsemd_status_t nnsemd_tuning_clear(nnsemd_handle_t h) {
    if (h == nullptr) return NNSEMD_ERR_INVALID_ARG;
    for (auto& per_d : h->tune)
        for (auto& per_metric : per_d)
            for (auto& tn : per_metric) tn.valid = 0;
    for (auto& per_d : h->doc_tune)
        for (auto& dt : per_d) dt.valid = 0;
    return NNSEMD_OK;
}

nnsemd_status_t nnsemd_tuning_set_docs(nnsemd_handle_t h, int32_t d, int64_t max_side, int32_t split) {
    if (h == nullptr) return NNSEMD_ERR_INVALID_ARG;
    h->last_error.clear();
    if (d < 1 || max_side < 1 || split < 0 || split > 2)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "need d >= 1, max_side >= 1 and split 0, 1 or 2");
    auto& dt = h->doc_tune[doc_dim_class(d)][tune_class(max_side)];
    dt.valid = 1;
    dt.split = split;
    dt.ms_split = dt.ms_fused = -1.f;
    return NNSEMD_OK;
}

nnsemd_status_t nnsemd_autotune_docs(nnsemd_handle_t h, int32_t d, int64_t max_m, int64_t max_n, int64_t num_pairs,
                                     nnsemd_doc_tuning_t* result, void* stream) {
    if (h == nullptr) return NNSEMD_ERR_INVALID_ARG;
    h->last_error.clear();
    if (d < 1 || d > 4096) return fail(h, NNSEMD_ERR_INVALID_ARG, "need 1 <= d <= 4096");
    if (max_m < 1 || max_n < 1 || max_m > 4096 || max_n > 4096 || num_pairs < 1 || num_pairs > 65536)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "need 1 <= max_m, max_n <= 4096 and 1 <= num_pairs <= 65536");
    DeviceGuard g(h->device);
    hipStream_t st = (hipStream_t)stream;
    // Synthetic BF16 pairs shaped like the caller's: sides uniform in
    // [max/8, max], N(0, 1/d) coordinates rounded to BF16, normalised
    // exponential masses.
    std::vector<int64_t> xo(num_pairs + 1, 0), yo(num_pairs + 1, 0);
    uint64_t rs = 0xD1B54A32D192ED03ull ^ (uint64_t)(d * 977 + max_m * 3 + max_n);
    auto next = [&rs]() {
        rs += 0x9E3779B97F4A7C15ull;
        uint64_t z = rs;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    auto unif = [&next]() { return ((double)(next() >> 11) + 0.5) * 0x1.0p-53; };
    for (int64_t p = 0; p < num_pairs; ++p) {
        const int64_t lm = std::max<int64_t>(1, max_m / 8), ln = std::max<int64_t>(1, max_n / 8);
        xo[p + 1] = xo[p] + lm + (int64_t)(unif() * (double)(max_m - lm + 1));
        yo[p + 1] = yo[p] + ln + (int64_t)(unif() * (double)(max_n - ln + 1));
    }
    const double sd = 1.0 / std::sqrt((double)d);
    auto points = [&](const std::vector<int64_t>& off, std::vector<uint16_t>& P, std::vector<float>& w) {
        P.resize((size_t)off.back() * d);
        w.resize((size_t)off.back());
        for (auto& v : P) {  // Box-Muller, then round to nearest even BF16
            const double g = std::sqrt(-2.0 * std::log(unif())) * std::cos(6.283185307179586 * unif());
            const float f = (float)(g * sd);
            uint32_t u;
            std::memcpy(&u, &f, 4);
            u += 0x7fffu + ((u >> 16) & 1u);
            v = (uint16_t)(u >> 16);
        }
        for (size_t s = 0; s + 1 < off.size(); ++s) {
            double sum = 0.0;
            for (int64_t i = off[s]; i < off[s + 1]; ++i) sum += (w[i] = (float)-std::log(unif()));
            for (int64_t i = off[s]; i < off[s + 1]; ++i) w[i] = (float)(w[i] / sum);
        }
    };
    std::vector<uint16_t> X, Y;
    std::vector<float> a, b;
    points(xo, X, a);
    points(yo, Y, b);
    Carver c;
    const size_t oX = c.take(2 * X.size()), oa = c.take(4 * a.size()), oY = c.take(2 * Y.size()),
                 ob = c.take(4 * b.size()), oxo = c.take(8 * xo.size()), oyo = c.take(8 * yo.size()),
                 oc = c.take(8 * (size_t)num_pairs);
    char* base = nullptr;
    if (hipMalloc((void**)&base, align_up(c.off, 256)) != hipSuccess)
        return fail(h, NNSEMD_ERR_OUT_OF_MEMORY, "autotuning inputs");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    nnsemd_status_t status = NNSEMD_OK;
    bool ok = hipMemcpyAsync(base + oX, X.data(), 2 * X.size(), hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(base + oa, a.data(), 4 * a.size(), hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(base + oY, Y.data(), 2 * Y.size(), hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(base + ob, b.data(), 4 * b.size(), hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(base + oxo, xo.data(), 8 * xo.size(), hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(base + oyo, yo.data(), 8 * yo.size(), hipMemcpyHostToDevice, st) == hipSuccess &&
              hipStreamSynchronize(st) == hipSuccess && hipEventCreate(&e0) == hipSuccess &&
              hipEventCreate(&e1) == hipSuccess;
    if (!ok) status = fail(h, NNSEMD_ERR_DEVICE, "autotuning set-up");
    float ms_form[2] = {-1.f, -1.f};  // fused, split
    const int mcap = (int)max_m, ncap = (int)max_n;
    const int chunk = (std::max(mcap, ncap) + 255) / 256;
    const bool split_exists = doc_split_form(d, true, chunk);
    for (int form = 0; form < 2 && status == NNSEMD_OK; ++form) {
        if (form == 1 && !split_exists) break;
        DocArgs A{};
        A.num_pairs = num_pairs;
        A.X = base + oX;
        A.a = reinterpret_cast<const float*>(base + oa);
        A.x_off = reinterpret_cast<const int64_t*>(base + oxo);
        A.num_x_sets = num_pairs;
        A.Y = base + oY;
        A.b = reinterpret_cast<const float*>(base + ob);
        A.y_off = reinterpret_cast<const int64_t*>(base + oyo);
        A.num_y_sets = num_pairs;
        A.d = d;
        A.metric = NNSEMD_L2;
        A.costs = reinterpret_cast<double*>(base + oc);
        const nnsemd_options_t o = default_options();
        DocArgs Aw = A;
        nnsemd_status_t s = run_docs(h, Aw, max_m, max_n, NNSEMD_BF16, o, stream, form);
        if (s != NNSEMD_OK) {
            status = s;
            break;
        }
        float ms = 0.f;
        bool good = hipEventRecord(e0, st) == hipSuccess;
        for (int r = 0; r < 3 && good; ++r) {
            DocArgs Ar = A;
            good = run_docs(h, Ar, max_m, max_n, NNSEMD_BF16, o, stream, form) == NNSEMD_OK;
        }
        good = good && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
               hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        if (!good) {
            status = fail(h, NNSEMD_ERR_DEVICE, "autotuning launch");
            break;
        }
        ms_form[form] = ms / 3.f;
    }
    (void)hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(base);
    if (status != NNSEMD_OK) return status;
    auto& dt = h->doc_tune[doc_dim_class(d)][tune_class(std::max(max_m, max_n))];
    dt.valid = 1;
    dt.split = ms_form[1] >= 0.f && ms_form[1] <= ms_form[0] ? 1 : 0;
    dt.ms_split = ms_form[1];
    dt.ms_fused = ms_form[0];
    if (result != nullptr) {
        result->split = dt.split;
        result->ms_split = dt.ms_split;
        result->ms_fused = dt.ms_fused;
    }
    return NNSEMD_OK;
}

nnsemd_status_t nnsemd_tuning_load(nnsemd_handle_t h, const char* path) {
    if (h == nullptr || path == nullptr) return NNSEMD_ERR_INVALID_ARG;
    FILE* f = std::fopen(path, "r");
    if (f == nullptr) return fail(h, NNSEMD_ERR_INVALID_ARG, "cannot open the tuning file");
    int version = 0;
    nnsemd_status_t s = NNSEMD_OK;
    if (std::fscanf(f, "nnsemd-tuning %d", &version) != 1 || version != 2) {
        s = fail(h, NNSEMD_ERR_INVALID_ARG, "not a tuning file (version 2)");
    } else {
        int d, m, c, t, sp;
        double ms;
        int n;
        while ((n = std::fscanf(f, "%d %d %d %d %d %lf", &d, &m, &c, &t, &sp, &ms)) == 6) {
            if (d < 1 || d > 7 || m < 0 || m > 2 || c < 0 || c >= nnsemd_tune_classes || (t != 256 && t != 512) ||
                (sp != 1 && sp != 2 && sp != 4)) {
                s = fail(h, NNSEMD_ERR_INVALID_ARG, "bad entry in the tuning file");
                break;
            }
            auto& tn = h->tune[d][m][c];
            tn.valid = 1;
            tn.threads = t;
            tn.split = sp;
            tn.ms = (float)ms;
        }
        if (s == NNSEMD_OK && n != EOF) s = fail(h, NNSEMD_ERR_INVALID_ARG, "malformed tuning file");
    }
    std::fclose(f);
    return s;
}

int64_t nnsemd_sg_num_params(void) { return kSgParams; }

nnsemd_status_t nnsemd_sg_embed(nnsemd_handle_t h, const float* theta, const float* X, const float* a,
                                const int64_t* set_off, int64_t num_sets, int64_t num_points, float* E,
                                void* stream) {
    if (h == nullptr) return NNSEMD_ERR_INVALID_ARG;
    h->last_error.clear();
    if (num_sets < 0 || num_points < 0 || num_sets > 0x7fffffffLL || num_points > kSgMaxRows)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "bad set or point count");
    if (num_sets == 0) return NNSEMD_OK;
    if (theta == nullptr || set_off == nullptr || E == nullptr || (num_points > 0 && (X == nullptr || a == nullptr)))
        return fail(h, NNSEMD_ERR_INVALID_ARG, "NULL array");
    DeviceGuard g(h->device);
    sg::SgQuant q;
    nnsemd_status_t s = sg_quantize(h, theta, q, stream);
    if (s != NNSEMD_OK) return s;
    const int err = sg::launch_embed(theta, q, X, a, set_off, num_sets, num_points, E, stream);
    if (err != 0) return device_fail(h, err, "surrogate embedding");
    return NNSEMD_OK;
}

nnsemd_status_t nnsemd_sg_predict(nnsemd_handle_t h, const float* theta, const float* Eq, int64_t num_q,
                                  const float* Ec, int64_t num_c, const int32_t* q_idx, const int32_t* c_idx,
                                  int64_t num_pairs, float* pred, void* stream) {
    if (h == nullptr) return NNSEMD_ERR_INVALID_ARG;
    h->last_error.clear();
    if (num_pairs < 0 || num_pairs > kSgMaxRows) return fail(h, NNSEMD_ERR_INVALID_ARG, "bad pair count");
    if (num_q < 1 || num_c < 1) return fail(h, NNSEMD_ERR_INVALID_ARG, "empty embedding table");
    if (q_idx == nullptr && c_idx == nullptr && num_c < num_pairs)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "fewer candidate rows than pairs without an index table");
    if (num_pairs == 0) return NNSEMD_OK;
    if (theta == nullptr || Eq == nullptr || Ec == nullptr || pred == nullptr)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "NULL array");
    DeviceGuard g(h->device);
    sg::SgQuant q;
    nnsemd_status_t s = sg_quantize(h, theta, q, stream);
    if (s != NNSEMD_OK) return s;
    if ((s = sg_workspace(h, sg_predict_bytes(num_pairs))) != NNSEMD_OK) return s;
    const sg::SgPredictWork w = sg_predict_carve(h->sg_ws, num_pairs);
    const int err =
        sg::launch_predict(theta, q, Eq, num_q, Ec, num_c, q_idx, c_idx, 0, num_pairs, w, nullptr, pred, stream);
    if (err != 0) return device_fail(h, err, "surrogate prediction");
    return NNSEMD_OK;
}

namespace {
// Carve the training workspace for B pairs and P points; returns bytes
// needed (base == nullptr: size only).
static size_t sg_train_carve(char* base, int64_t B, int64_t P, bool own_grad, sg::SgTrainWork& w, float** grad) {
    constexpr int64_t Hd = kSgHidden;
    const int64_t Ppad = (P + 63) / 64 * 64, Bpad = (B + 63) / 64 * 64, S = 2 * B;
    const int64_t nblk = std::max<int64_t>(1, (P + 511) / 512);
    Carver c;
    const size_t oH1 = c.take(2 * Ppad * Hd), oH1T = c.take(2 * Ppad * Hd);
    const size_t odP = c.take(2 * Ppad * Hd), odPT = c.take(2 * Ppad * Hd);
    const size_t oPRE2 = c.take(4 * Ppad * Hd), odH1 = c.take(4 * Ppad * Hd);
    const size_t oE = c.take(4 * S * Hd), odE = c.take(4 * S * Hd);
    const size_t oZ = c.take(2 * Bpad * 3 * Hd), oZT = c.take(2 * Bpad * 3 * Hd);
    const size_t odG = c.take(2 * Bpad * Hd), odGT = c.take(2 * Bpad * Hd);
    const size_t oPRE3 = c.take(4 * Bpad * Hd), odZ = c.take(4 * Bpad * 3 * Hd);
    const size_t oHB = c.take(4 * Bpad * kSgHbCols), ohs = c.take(4 * kSgHbCols);
    const size_t ot = c.take(4 * Bpad), opred = c.take(4 * Bpad), odb2 = c.take(4 * S * Hd);
    const size_t osplit = c.take(4 * 64 * Hd * Hd), ol1p = c.take(4 * nblk * 4 * Hd), ol1s = c.take(4 * 4 * Hd);
    const size_t obad = c.take(64);
    const size_t ograd = own_grad ? c.take(4 * kSgParams) : 0;
    if (base != nullptr) {
        auto F = [&](size_t o) { return reinterpret_cast<float*>(base + o); };
        auto U = [&](size_t o) { return reinterpret_cast<uint16_t*>(base + o); };
        w.H1q = U(oH1);
        w.H1qT = U(oH1T);
        w.dP2q = U(odP);
        w.dP2qT = U(odPT);
        w.PRE2 = F(oPRE2);
        w.dH1 = F(odH1);
        w.E = F(oE);
        w.dE = F(odE);
        w.Z = U(oZ);
        w.ZT = U(oZT);
        w.dGq = U(odG);
        w.dGqT = U(odGT);
        w.PRE3 = F(oPRE3);
        w.dZ = F(odZ);
        w.HB = F(oHB);
        w.hsum = F(ohs);
        w.t = F(ot);
        w.pred = F(opred);
        w.db2p = F(odb2);
        w.split = F(osplit);
        w.l1p = F(ol1p);
        w.l1s = F(ol1s);
        w.bad = reinterpret_cast<int*>(base + obad);
        if (own_grad) *grad = F(ograd);
    }
    return align_up(c.off, 256);
}

static nnsemd_status_t sg_loss_grad_common(nnsemd_handle_t h, const float* theta, const float* X, const float* a,
                                    const int64_t* set_off, int64_t num_pairs, int64_t num_points,
                                    const float* labels, float* loss, float** grad, sg::SgQuant& q, void* stream) {
    if (num_pairs < 1 || num_pairs > (1 << 20) || num_points < 1 || num_points > (int64_t)1 << 26)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "training batch: 1 <= pairs <= 2^20, 1 <= points <= 2^26");
    if (theta == nullptr || X == nullptr || a == nullptr || set_off == nullptr || labels == nullptr)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "NULL array");
    nnsemd_status_t s = sg_quantize(h, theta, q, stream);
    if (s != NNSEMD_OK) return s;
    sg::SgTrainWork w;
    const bool own = *grad == nullptr;
    const size_t need = sg_train_carve(nullptr, num_pairs, num_points, own, w, grad);
    if ((s = sg_workspace(h, need)) != NNSEMD_OK) return s;
    sg_train_carve(h->sg_ws, num_pairs, num_points, own, w, grad);
    const int err = sg::launch_loss_grad(theta, q, X, a, set_off, num_pairs, num_points, labels, w, loss, *grad, stream);
    if (err != 0) return device_fail(h, err, "surrogate backward");
    return NNSEMD_OK;
}
}  // namespace

nnsemd_status_t nnsemd_sg_loss_grad(nnsemd_handle_t h, const float* theta, const float* X, const float* a,
                                    const int64_t* set_off, int64_t num_pairs, int64_t num_points,
                                    const float* labels, float* loss, float* grad, void* stream) {
    if (h == nullptr) return NNSEMD_ERR_INVALID_ARG;
    h->last_error.clear();
    if (grad == nullptr) return fail(h, NNSEMD_ERR_INVALID_ARG, "grad must not be NULL");
    DeviceGuard g(h->device);
    sg::SgQuant q;
    return sg_loss_grad_common(h, theta, X, a, set_off, num_pairs, num_points, labels, loss, &grad, q, stream);
}

nnsemd_status_t nnsemd_sg_train_step(nnsemd_handle_t h, float* theta, float* adam_m, float* adam_v, int64_t step,
                                     float lr, const float* X, const float* a, const int64_t* set_off,
                                     int64_t num_pairs, int64_t num_points, const float* labels, float* loss,
                                     float* grad, void* stream) {
    if (h == nullptr) return NNSEMD_ERR_INVALID_ARG;
    h->last_error.clear();
    if (adam_m == nullptr || adam_v == nullptr || step < 1 || !(lr > 0.f))
        return fail(h, NNSEMD_ERR_INVALID_ARG, "Adam state, step >= 1 and lr > 0 required");
    DeviceGuard g(h->device);
    sg::SgQuant q;
    nnsemd_status_t s =
        sg_loss_grad_common(h, theta, X, a, set_off, num_pairs, num_points, labels, loss, &grad, q, stream);
    if (s != NNSEMD_OK) return s;
    const double beta1 = 0.9, beta2 = 0.999;
    const float bc1 = (float)(1.0 - std::pow(beta1, (double)step));
    const float bc2 = (float)(1.0 - std::pow(beta2, (double)step));
    const int err = sg::launch_adam(theta, adam_m, adam_v, grad, lr, beta1, beta2, 1e-8f, bc1, bc2, stream);
    if (err != 0) return device_fail(h, err, "Adam update");
    return NNSEMD_OK;
}

// Top-k scratch of the handle (allocated once).
static nnsemd_status_t topk_workspace(nnsemd_handle_t h) {
    if (h->topk_ws) return NNSEMD_OK;
    if (hipMalloc((void**)&h->topk_ws, sg::topk_ws_bytes()) != hipSuccess) {
        h->topk_ws = nullptr;
        return fail(h, NNSEMD_ERR_OUT_OF_MEMORY, "top-k scratch");
    }
    return NNSEMD_OK;
}

nnsemd_status_t nnsemd_topk_smallest_f32(nnsemd_handle_t h, const float* values, int64_t n, int32_t k, int32_t* idx,
                                         void* stream) {
    if (h == nullptr) return NNSEMD_ERR_INVALID_ARG;
    h->last_error.clear();
    if (values == nullptr || idx == nullptr || k < 1 || k > kSgTopkMax || n < k || n > 0x7fffffffLL)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "top-k needs 1 <= k <= min(n, 1024), n < 2^31");
    DeviceGuard g(h->device);
    nnsemd_status_t s = topk_workspace(h);
    if (s != NNSEMD_OK) return s;
    const int err = sg::launch_topk_f32(values, n, k, idx, h->topk_ws, stream);
    if (err != 0) return device_fail(h, err, "top-k");
    return NNSEMD_OK;
}

nnsemd_status_t nnsemd_topk_smallest_f64(nnsemd_handle_t h, const double* values, int64_t n, int32_t k, int32_t* idx,
                                         void* stream) {
    if (h == nullptr) return NNSEMD_ERR_INVALID_ARG;
    h->last_error.clear();
    if (values == nullptr || idx == nullptr || k < 1 || k > kSgTopkMax || n < k || n > 0x7fffffffLL)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "top-k needs 1 <= k <= min(n, 1024), n < 2^31");
    DeviceGuard g(h->device);
    nnsemd_status_t s = topk_workspace(h);
    if (s != NNSEMD_OK) return s;
    const int err = sg::launch_topk_f64(values, n, k, idx, h->topk_ws, stream);
    if (err != 0) return device_fail(h, err, "top-k");
    return NNSEMD_OK;
}

nnsemd_status_t nnsemd_sg_retrieve(nnsemd_handle_t h, const float* theta, const float* index_E, int64_t num_candidates,
                                   const float* Xq, const float* aq, int64_t mq, const float* Ycat, const float* bcat,
                                   const int64_t* y_off, int64_t max_n, int32_t keep, int32_t top, int32_t* out_idx,
                                   double* out_cost, int32_t* kept_idx, nnsemd_stats_t* kept_stats, void* stream) {
    if (h == nullptr) return NNSEMD_ERR_INVALID_ARG;
    h->last_error.clear();
    if (theta == nullptr || index_E == nullptr || Xq == nullptr || aq == nullptr || Ycat == nullptr ||
        bcat == nullptr || y_off == nullptr || out_idx == nullptr || out_cost == nullptr)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "NULL array");
    if (num_candidates < 1 || num_candidates > kSgMaxRows || mq < 1 || max_n < 1 || keep < 1 ||
        keep > kSgTopkMax || keep > num_candidates || top < 1 || top > keep)
        return fail(h, NNSEMD_ERR_INVALID_ARG, "need 1 <= top <= keep <= min(candidates, 1024), mq, max_n >= 1");
    DeviceGuard g(h->device);
    sg::SgQuant q;
    nnsemd_status_t s = sg_quantize(h, theta, q, stream);
    if (s != NNSEMD_OK) return s;
    if ((s = topk_workspace(h)) != NNSEMD_OK) return s;
    Carver c;
    const size_t oEq = c.take(4 * kSgHidden), oqoff = c.take(2 * 8), opred = c.take(4 * (size_t)num_candidates);
    const size_t osel = c.take(4 * (size_t)keep), ozero = c.take(4 * (size_t)keep), oxoff = c.take(16);
    const size_t ocost = c.take(8 * (size_t)keep), opos = c.take(4 * (size_t)top);
    const size_t ostats = c.take(sizeof(nnsemd_stats_t) * (size_t)keep);
    const size_t opw = c.take(sg_predict_bytes(num_candidates));
    if ((s = sg_workspace(h, align_up(c.off, 256))) != NNSEMD_OK) return s;
    char* b = h->sg_ws;
    float* Eq = reinterpret_cast<float*>(b + oEq);
    int64_t* qoff = reinterpret_cast<int64_t*>(b + oqoff);
    float* pred = reinterpret_cast<float*>(b + opred);
    int32_t* sel = kept_idx ? kept_idx : reinterpret_cast<int32_t*>(b + osel);
    int32_t* zeros = reinterpret_cast<int32_t*>(b + ozero);
    int64_t* xoff = reinterpret_cast<int64_t*>(b + oxoff);
    double* costs = reinterpret_cast<double*>(b + ocost);
    int32_t* pos = reinterpret_cast<int32_t*>(b + opos);
    nnsemd_stats_t* st = kept_stats ? kept_stats : reinterpret_cast<nnsemd_stats_t*>(b + ostats);
    const sg::SgPredictWork pw = sg_predict_carve(b + opw, num_candidates);
    int err = sg::launch_two_offsets(qoff, mq, stream);
    if (err == 0) err = sg::launch_embed(theta, q, Xq, aq, qoff, 1, mq, Eq, stream);
    if (err == 0)
        err = sg::launch_predict(theta, q, Eq, 1, index_E, num_candidates, nullptr, nullptr, 0, num_candidates, pw,
                                 nullptr, pred, stream);
    if (err == 0) err = sg::launch_topk_f32(pred, num_candidates, keep, sel, h->topk_ws, stream);
    if (err == 0) err = sg::launch_fill_i32(zeros, keep, 0, stream);
    if (err == 0) err = sg::launch_two_offsets(xoff, mq, stream);
    if (err != 0) return device_fail(h, err, "surrogate retrieval");
    PairSolverArgs A{};
    A.num_pairs = keep;
    A.X = Xq;
    A.a = aq;
    A.x_off = xoff;
    A.num_x_sets = 1;
    A.Y = Ycat;
    A.b = bcat;
    A.y_off = y_off;
    A.num_y_sets = num_candidates;
    A.pair_x = zeros;
    A.pair_y = sel;
    A.metric = NNSEMD_L2;
    A.costs = costs;
    A.stats = st;
    const nnsemd_options_t o = default_options();
    if ((s = run_pairs(h, A, 3, mq, max_n, o, stream)) != NNSEMD_OK) return s;
    err = sg::launch_topk_f64(costs, keep, top, pos, h->topk_ws, stream);
    if (err == 0) err = sg::launch_gather_ranked(pos, sel, costs, top, out_idx, out_cost, stream);
    if (err != 0) return device_fail(h, err, "re-rank selection");
    return NNSEMD_OK;
}

#ifdef NNSEMD_PHASE_TIMING
// Profiling builds only: device buffer of 9 unsigned 64-bit per-phase cycle
// totals that every later launch on this handle adds to.
nnsemd_status_t nnsemd_debug_phase_buffer(nnsemd_handle_t h, unsigned long long* cycles) {
    if (h == nullptr) return NNSEMD_ERR_INVALID_ARG;
    h->phase_cycles = cycles;
    return NNSEMD_OK;
}
#endif

}  // extern "C"
