// MTTKRP launch plans: strategy resolution, LDS sizing and the counting pass
// that fixes every workgroup's record offsets for the TABLE strategy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "spt_internal.h"

namespace spt {

namespace {

// Dynamic LDS available to one table/privatised workgroup (160 KB per CU on
// gfx950, minus the kernel's static LDS and a margin).
constexpr size_t kLdsBudget = 160 * 1024 - 512;

int next_pow2_bits(int v) {
    int b = 0;
    while ((1 << b) < v) ++b;
    return b;
}

// Largest accumulator that fits LDS for the TABLE strategy; cap >= sub-tile size.
bool table_params(int nmodes, int R, int *ts, int *cap, int *hbits, int *stride) {
    const int st = R + 1;
    for (int t : {512, 256}) {
        int best = 0, best_h = 0;
        for (int c = 16; c <= 8192; c += 16) {
            const int hb = next_pow2_bits(2 * c);
            if (table_lds_needed(nmodes, t, c, hb, st, false, true) > kLdsBudget) break;
            best = c;
            best_h = hb;
        }
        if (best >= t) {
            *ts = t;
            *cap = best;
            *hbits = best_h;
            *stride = st;
            return true;
        }
    }
    return false;
}

// Column passes for PRIV: the smallest pass count whose slice fits LDS.
bool priv_params(int nmodes, int64_t rows, int R, int max_pass, int *npass, int *rs, int *stride) {
    if (rows > 65535) return false;
    for (int p = 1; p <= max_pass; p *= 2) {
        int w = (R + p - 1) / p;
        if ((R & 3) == 0) w = (w + 3) & ~3;
        if ((int64_t)(p - 1) * w >= R) break;
        const int st = w + 1;
        if (table_lds_needed(nmodes, 512, (int)rows, 0, st, true, true) <= kLdsBudget) {
            *npass = (R + w - 1) / w;
            *rs = w;
            *stride = st;
            return true;
        }
    }
    return false;
}

}  // namespace

// PRIV fits this mode with at most 2 column passes
bool priv_feasible(const Tensor *t, int mode, int rank) {
    int npass = 1, rs = rank, stride = rank + 1;
    return priv_params(t->nmodes, t->dims[mode], rank, 2, &npass, &rs, &stride);
}

int device_cus() {
    static int cus[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cus[dev] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        cus[dev] = v;
    }
    return cus[dev];
}

void release_mode_plan(Tensor *t, int n, hipStream_t s) {
    ModePlan &p = t->mplan[n];
    for (void *q : {(void *)p.rec_off, (void *)p.pl_pos, (void *)p.pl_off, (void *)p.pl_piece})
        dev_free(q, s);
    p = ModePlan{};
}

void release_batch_plan(Tensor *t, int n, hipStream_t s) {
    ModePlan &p = t->bplan[n];
    for (void *q : {(void *)p.pl_pos, (void *)p.pl_off, (void *)p.pl_desc, (void *)p.pl_row, (void *)p.pl_dest})
        dev_free(q, s);
    p = ModePlan{};
}

void release_dict(Tensor *t, hipStream_t s) {
    for (int k = 0; k < kMaxModes; ++k) {
        for (void *q : {(void *)t->dict_slot[k], (void *)t->dict_row[k], (void *)t->dict_off[k]}) dev_free(q, s);
        t->dict_slot[k] = nullptr;
        t->dict_row[k] = nullptr;
        t->dict_off[k] = nullptr;
    }
    t->dict_state = 0;
}

void release_plans(Tensor *t, hipStream_t s) {
    for (int n = 0; n < kMaxModes; ++n) {
        release_mode_plan(t, n, s);
        release_batch_plan(t, n, s);
    }
    release_dict(t, s);
}

// Tile dictionaries (per mode, once per encoding).  They are an
// optimisation: a tensor that cannot have them (more than 4 modes, a mode of
// 2^31 rows or more) or whose build fails (no memory) is marked, and the
// uncached kernel runs.
static bool dict_eligible(const Tensor *t) {
    if (t->dict_state < 0 || t->nmodes < 2 || t->nmodes > 4 || t->nnz == 0 || !seg_tile_ok(kDictTile, t->nmodes))
        return false;
    for (int k = 0; k < t->nmodes; ++k)
        if (t->dims[k] >= (int64_t)kDictMiss) return false;
    return true;
}

// Mode k's dictionary.  pairs: per tile of kDictTile nonzeros, the exclusive
// prefix of its distinct mode-k rows (ntiles + 1 entries) when a counting
// pass already produced it (the mode-k SEGMENT plan's), else null (the pass
// runs here and synchronises s).  Asynchronous otherwise.
static spt_status build_dict_mode(Tensor *t, int k, hipStream_t s, const int64_t *pairs) {
    if (t->dict_slot[k] || !dict_eligible(t)) return SPT_OK;
    const int64_t ntiles = (t->nnz + kDictTile - 1) / kDictTile;
    std::vector<int64_t> h;
    const MttkrpArgs a = make_args(t, nullptr, 1, k, nullptr, kDictTile);
    t->dict_off[k] = (int64_t *)dev_alloc(sizeof(int64_t) * (ntiles + 1), s);
    bool ok = t->dict_off[k] != nullptr;
    if (ok && !pairs) {
        h.assign(ntiles + 1, 0);
        ok = launch_count_pieces(a, t->dict_off[k], s) == SPT_OK &&
             hipMemcpyAsync(h.data(), t->dict_off[k], sizeof(int64_t) * ntiles, hipMemcpyDeviceToHost, s) ==
                 hipSuccess &&
             hipStreamSynchronize(s) == hipSuccess;
        int64_t run = 0;
        for (int64_t i = 0; ok && i < ntiles; ++i) {
            const int64_t c = h[i] >> 32;  // distinct mode-k rows of the tile
            h[i] = run;
            run += c;
        }
        if (ok) h[ntiles] = run;
        pairs = h.data();
    }
    if (ok) {
        t->dict_slot[k] = (uint16_t *)dev_alloc(sizeof(uint16_t) * t->nnz, s);
        t->dict_row[k] = (uint32_t *)dev_alloc(sizeof(uint32_t) * std::max<int64_t>(pairs[ntiles], 1), s);
    }
    ok = ok && t->dict_slot[k] && t->dict_row[k] &&
         hipMemcpyAsync(t->dict_off[k], pairs, sizeof(int64_t) * (ntiles + 1), hipMemcpyHostToDevice, s) ==
             hipSuccess &&
         launch_emit_dict(a, t->dict_off[k], t->dict_row[k], t->dict_slot[k], s) == SPT_OK;
    // the host prefix must outlive the copy
    ok = hipStreamSynchronize(s) == hipSuccess && ok;
    if (!ok) {
        (void)hipGetLastError();
        release_dict(t, s);
        t->dict_state = -1;
    }
    return SPT_OK;
}

// SEGMENT tile: the plan's tile if it is one the kernel serves and it fits
// LDS, else the largest that fits (4096 up to 5 modes, 2048 beyond)
int segment_tile(const Tensor *t, int mode) {
    const int want = t->plan.tile[mode];
    if (want >= 1024 && seg_tile_ok(want, t->nmodes)) return want;
    return seg_tile_ok(4096, t->nmodes) ? 4096 : (seg_tile_ok(2048, t->nmodes) ? 2048 : 1024);
}

// SEGMENT plan (once per tensor and mode; synchronises s once).  A tile's
// records are its pieces (runs of at most L nonzeros of one row).
//  1. a counting pass gives every tile's pieces and distinct rows;
//  2. the emission pass (same regrouping) writes every nonzero's position in
//     its tile's row-grouped order, every piece's start, length and row, and
//     every distinct (tile, row) pair with its piece count, tile-major;
//  3. a stable sort of the pairs by row (tile order kept within a row) and an
//     exclusive scan of their piece counts give each pair its first record,
//     so the records of one row are contiguous; each piece's record follows.
// Calls then stage a tile with one scatter and write records in row order.
spt_status build_segment_plan(Tensor *t, int mode, int rank, hipStream_t s, ModePlan &p) {
    p.ts = segment_tile(t, mode);
    const int64_t ntiles = (t->nnz + p.ts - 1) / p.ts;
    std::vector<int64_t> h(ntiles + 1, 0), hq(ntiles + 1, 0);
    p.pl_off = (int64_t *)dev_alloc(sizeof(int64_t) * (ntiles + 1), s);
    if (!p.pl_off) return fail(SPT_E_OOM, "plan: offsets");
    if (ntiles > 0) {
        spt_status st = launch_count_pieces(make_args(t, nullptr, rank, mode, nullptr, p.ts), p.pl_off, s);
        if (st != SPT_OK) return st;
        SPT_HIP(hipMemcpyAsync(h.data(), p.pl_off, sizeof(int64_t) * ntiles, hipMemcpyDeviceToHost, s));
        SPT_HIP(hipStreamSynchronize(s));
    }
    int64_t pieces = 0, pairs = 0;
    for (int64_t i = 0; i < ntiles; ++i) {
        const int64_t c = h[i];
        h[i] = pieces;
        hq[i] = pairs;
        pieces += c & 0xFFFFFFFFll;
        pairs += c >> 32;
    }
    h[ntiles] = pieces;
    hq[ntiles] = pairs;
    p.records = pieces;
    if (pieces >= (int64_t(1) << 32)) return fail(SPT_E_INVALID_ARG, "plan: more than 2^32 records");
    SPT_HIP(hipMemcpyAsync(p.pl_off, h.data(), sizeof(int64_t) * (ntiles + 1), hipMemcpyHostToDevice, s));
    const size_t n1 = (size_t)std::max<int64_t>(t->nnz, 1), k1 = (size_t)std::max<int64_t>(pieces, 1),
                 q1 = (size_t)std::max<int64_t>(pairs, 1);
    p.pl_pos = (uint16_t *)dev_alloc(sizeof(uint16_t) * n1, s);
    p.pl_piece = (uint32_t *)dev_alloc(sizeof(uint32_t) * 4 * k1, s);
    if (!p.pl_pos || !p.pl_piece) {
        (void)hipStreamSynchronize(s);  // the host offsets must outlive their copy
        return fail(SPT_E_OOM, "plan: arrays");
    }
    if (pieces == 0) {
        SPT_HIP(hipStreamSynchronize(s));
        return SPT_OK;
    }
    int64_t *pair_off = (int64_t *)dev_alloc(sizeof(int64_t) * (ntiles + 1), s);
    uint32_t *desc = (uint32_t *)dev_alloc(sizeof(uint32_t) * k1, s);
    uint32_t *prow = (uint32_t *)dev_alloc(sizeof(uint32_t) * k1, s);
    uint32_t *ppair = (uint32_t *)dev_alloc(sizeof(uint32_t) * k1, s);
    uint32_t *psub = (uint32_t *)dev_alloc(sizeof(uint32_t) * k1, s);
    uint64_t *keys = (uint64_t *)dev_alloc(sizeof(uint64_t) * q1, s);
    uint64_t *keys2 = (uint64_t *)dev_alloc(sizeof(uint64_t) * q1, s);
    uint32_t *np = (uint32_t *)dev_alloc(sizeof(uint32_t) * q1, s);
    uint32_t *ia = (uint32_t *)dev_alloc(sizeof(uint32_t) * q1, s);
    uint32_t *ib = (uint32_t *)dev_alloc(sizeof(uint32_t) * q1, s);
    uint32_t *cnt = (uint32_t *)dev_alloc(sizeof(uint32_t) * std::max(sort_ws_counts(pairs), exclusive_scan_ws(pairs)), s);
    spt_status st = (pair_off && desc && prow && ppair && psub && keys && keys2 && np && ia && ib && cnt)
                        ? SPT_OK
                        : fail(SPT_E_OOM, "plan: workspace");
    if (st == SPT_OK &&
        hipMemcpyAsync(pair_off, hq.data(), sizeof(int64_t) * (ntiles + 1), hipMemcpyHostToDevice, s) != hipSuccess)
        st = hip_fail(hipGetLastError(), "plan: pair offsets");
    MttkrpArgs a = make_args(t, nullptr, rank, mode, nullptr, p.ts);
    a.pl_off = p.pl_off;
    PlanOut o{pair_off, p.pl_pos, desc, prow, ppair, psub, keys, np};
    if (st == SPT_OK) st = launch_emit_plan(a, o, s);
    uint64_t *sk = nullptr;
    uint32_t *sidx = nullptr;
    if (st == SPT_OK) st = sort_u64_keys_ws(keys, keys2, ia, ib, cnt, pairs, t->lbits[mode], &sk, &sidx, s);
    // pair pieces in row order -> exclusive prefix -> first record of each pair (emission order)
    uint32_t *np_sorted = (sidx == ia) ? ib : ia;
    uint32_t *tmp = (uint32_t *)((sk == keys2) ? keys : keys2);  // the unsorted key buffer is free now
    uint32_t *pair_first = tmp + q1;                               // second half of that buffer
    if (st == SPT_OK) st = launch_gather_u32(np, sidx, np_sorted, pairs, s);
    if (st == SPT_OK) st = launch_exclusive_scan_u32(np_sorted, tmp, pairs, cnt, s);
    if (st == SPT_OK) st = launch_scatter_u32(tmp, sidx, pair_first, pairs, s);
    if (st == SPT_OK) st = launch_piece_pack(ppair, psub, pair_first, desc, prow, p.pl_piece, pieces, s);
    if (st == SPT_OK && hipStreamSynchronize(s) != hipSuccess) st = hip_fail(hipGetLastError(), "plan: build");
    for (void *q : {(void *)pair_off, (void *)desc, (void *)prow, (void *)ppair, (void *)psub, (void *)keys,
                    (void *)keys2, (void *)np, (void *)ia, (void *)ib, (void *)cnt})
        dev_free(q, s);
    // the counting pass gave this mode's distinct rows per tile: its tile
    // dictionary costs one more pass
    if (st == SPT_OK && p.ts == kDictTile) st = build_dict_mode(t, mode, s, hq.data());
    return st;
}

// The plan of `mode` for `rank` under the tensor's strategy.  SEGMENT and
// TABLE plans come from a pass over the nonzeros that synchronises s; they
// are built only with `build` (spt_tensor_prepare), so an MTTKRP call never
// synchronises.  The SEGMENT plan holds for every rank; PRIV, DIRECT and
// REGROUP need only host arithmetic.
spt_status resolve_plan(Tensor *t, int mode, int rank, hipStream_t s, ModePlan **out, bool build) {
    ModePlan &p = t->mplan[mode];
    int want = t->plan.strategy[mode];
    const int64_t rows = t->dims[mode];
    int npass = 1, rs = rank, stride = rank + 1;
    if (want == SPT_STRATEGY_AUTO) want = SPT_STRATEGY_SEGMENT;  // measured fastest for every mode size
    const bool rank_free = want == SPT_STRATEGY_SEGMENT || want == SPT_STRATEGY_DIRECT || want == SPT_STRATEGY_REGROUP;
    const bool tile_same = want == SPT_STRATEGY_SEGMENT ? p.ts == segment_tile(t, mode)
                           : (want == SPT_STRATEGY_DIRECT || want == SPT_STRATEGY_REGROUP) ? p.ts == t->plan.tile[mode]
                                                                                         : true;
    if (p.valid && p.strategy == want && tile_same && (rank_free || p.rank == rank)) {
        *out = &p;
        return SPT_OK;
    }
    const bool device_pass = want == SPT_STRATEGY_SEGMENT || want == SPT_STRATEGY_TABLE;
    if (device_pass && !build)
        return fail(SPT_E_INVALID_ARG, "mttkrp: tensor not prepared for mode " + std::to_string(mode) +
                                           " at rank " + std::to_string(rank) + " (call spt_tensor_prepare)");
    release_mode_plan(t, mode, s);  // stream-ordered: earlier calls on s still see the old arrays
    p.rank = rank;
    p.strategy = want;
    if (want == SPT_STRATEGY_PRIV) {
        if (!priv_params(t->nmodes, rows, rank, 64, &npass, &rs, &stride))
            return fail(SPT_E_INVALID_ARG, "PRIV strategy: mode " + std::to_string(mode) + " output does not fit LDS");
        const int64_t nsub = (t->nnz + 511) / 512;
        p.ts = 512;
        p.cap = (int)rows;
        p.npass = npass;
        p.rs = rs;
        p.stride = stride;
        p.nwg = (int)std::max<int64_t>(1, std::min<int64_t>(device_cus(), nsub));
        p.sub_per_wg = (nsub + p.nwg - 1) / p.nwg;
        p.nwg = (int)std::max<int64_t>(1, (nsub + p.sub_per_wg - 1) / std::max<int64_t>(p.sub_per_wg, 1));
    } else if (want == SPT_STRATEGY_TABLE) {
        if (!table_params(t->nmodes, rank, &p.ts, &p.cap, &p.hbits, &p.stride))
            return fail(SPT_E_INVALID_ARG, "TABLE strategy: rank too large for the LDS accumulator");
        const int64_t nsub = (t->nnz + p.ts - 1) / p.ts;
        p.nwg = (int)std::max<int64_t>(1, std::min<int64_t>(device_cus(), nsub));
        p.sub_per_wg = std::max<int64_t>(1, (nsub + p.nwg - 1) / p.nwg);
        p.nwg = (int)std::max<int64_t>(1, (nsub + p.sub_per_wg - 1) / p.sub_per_wg);
        // counting pass: the same flush decisions as the real kernel, records only counted
        int64_t *cnt = (int64_t *)dev_alloc(sizeof(int64_t) * p.nwg, s);
        if (!cnt) return fail(SPT_E_OOM, "plan: record counts");
        TableArgs ta{};
        ta.a = make_args(t, nullptr, rank, mode, nullptr, 0);
        ta.cap = p.cap;
        ta.hbits = p.hbits;
        ta.stride = p.stride;
        ta.rs = rank;
        ta.ts = p.ts;
        ta.sub_per_wg = p.sub_per_wg;
        ta.rec_cnt = cnt;
        spt_status st = t->nnz > 0 ? launch_table_count(ta, p.nwg, s) : SPT_OK;
        std::vector<int64_t> h(p.nwg, 0);
        if (st == SPT_OK && t->nnz > 0) {
            if (hipMemcpyAsync(h.data(), cnt, sizeof(int64_t) * p.nwg, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                st = hip_fail(hipGetLastError(), "plan: record counts");
        }
        if (st != SPT_OK) {
            dev_free(cnt, s);
            p = ModePlan{};
            return st;
        }
        int64_t run = 0;
        for (int w = 0; w < p.nwg; ++w) {
            const int64_t c = h[w];
            h[w] = run;
            run += c;
        }
        p.records = run;
        if (hipMemcpyAsync(cnt, h.data(), sizeof(int64_t) * p.nwg, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            dev_free(cnt, s);
            p = ModePlan{};
            return hip_fail(hipGetLastError(), "plan: record offsets");
        }
        p.rec_off = cnt;
    } else if (want == SPT_STRATEGY_SEGMENT) {
        spt_status st = build_segment_plan(t, mode, rank, s, p);
        if (st != SPT_OK) {
            release_mode_plan(t, mode, s);
            return st;
        }
    } else {
        p.ts = t->plan.tile[mode];
    }
    p.valid = 1;
    *out = &p;
    return SPT_OK;
}

// Every mode's plan for `rank`, and the tile dictionaries when a mode runs
// the row-cached kernel.
spt_status prepare_single(Tensor *t, int rank, hipStream_t s) {
    bool want_dict = false;
    for (int n = 0; n < t->nmodes; ++n) {
        ModePlan *p = nullptr;
        spt_status st = resolve_plan(t, n, rank, s, &p, true);
        if (st != SPT_OK) return st;
        want_dict = want_dict || (p->strategy == SPT_STRATEGY_SEGMENT && p->ts == kDictTile);
    }
    if (want_dict && t->plan.row_cache != 0)
        for (int k = 0; k < t->nmodes; ++k) {
            spt_status st = build_dict_mode(t, k, s, nullptr);
            if (st != SPT_OK) return st;
        }
    return SPT_OK;
}

// ---------------------------------------------------------------- instrumentation
// When enabled, every MTTKRP call (all of its kernels) is bracketed by two HIP
// events on the call's stream; spt_profile_read sums their elapsed times.
namespace {
struct ProfEvent {
    int mode;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfEvent> g_prof;

void prof_clear_locked() {
    for (auto &e : g_prof) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    g_prof.clear();
}
}  // namespace

spt_status run_mttkrp_impl(Tensor *t, const float *const *factors, int rank, int mode, float *out, hipStream_t s,
                           const RecordWs *ws);

spt_status run_mttkrp(Tensor *t, const float *const *factors, int rank, int mode, float *out, hipStream_t s,
                      const RecordWs *ws) {
    bool on;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        on = g_prof_on;
    }
    if (!on) return run_mttkrp_impl(t, factors, rank, mode, out, s, ws);
    ProfEvent e{mode, nullptr, nullptr};
    SPT_HIP(hipEventCreate(&e.a));
    SPT_HIP(hipEventCreate(&e.b));
    SPT_HIP(hipEventRecord(e.a, s));
    spt_status st = run_mttkrp_impl(t, factors, rank, mode, out, s, ws);
    SPT_HIP(hipEventRecord(e.b, s));
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof.push_back(e);
    return st;
}

spt_status profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_clear_locked();
    g_prof_on = on != 0;
    return SPT_OK;
}

spt_status profile_read(double *ms, int64_t *launches) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (int n = 0; n < kMaxModes; ++n) {
        ms[n] = 0.0;
        launches[n] = 0;
    }
    for (auto &e : g_prof) {
        SPT_HIP(hipEventSynchronize(e.b));
        float v = 0.f;
        SPT_HIP(hipEventElapsedTime(&v, e.a, e.b));
        ms[e.mode] += v;
        launches[e.mode] += 1;
    }
    return SPT_OK;
}

// Records path shared by SEGMENT and TABLE: the main kernel writes P
// records (row, R floats) and the reducer sums them per row into out.
// SEGMENT records come out grouped by row (the plan laid them out); TABLE
// records are radix-sorted by row first.  The record buffers belong to the
// call (taken and released in stream order on s).
spt_status reduce_via_records(Tensor *t, MttkrpArgs &a, int64_t P, int rank, int64_t rows, float *out, hipStream_t s,
                              bool segment, TableArgs *ta = nullptr, int nwg = 0, const RecordWs *ws = nullptr) {
    const size_t n1 = (size_t)std::max<int64_t>(P, 1);
    // SEGMENT records go to the caller's workspace when they fit
    const bool own = !(segment && ws && ws->row && ws->val && (int64_t)n1 <= ws->records &&
                       (int64_t)n1 * rank <= ws->val_floats);
    uint64_t *rrow = own ? (uint64_t *)dev_alloc(sizeof(uint64_t) * n1, s) : ws->row;
    float *rval = own ? (float *)dev_alloc(sizeof(float) * n1 * rank, s) : ws->val;
    uint64_t *keys2 = nullptr;
    uint32_t *ia = nullptr, *ib = nullptr, *cnt = nullptr;
    auto release = [&]() {
        if (own) {
            dev_free(rrow, s);
            dev_free(rval, s);
        }
        dev_free(keys2, s); dev_free(ia, s); dev_free(ib, s); dev_free(cnt, s);
    };
    if (!rrow || !rval) {
        release();
        return fail(SPT_E_OOM, "mttkrp: record workspace allocation failed");
    }
    spt_status st;
    if (segment) {
        a.rec_row = rrow;
        a.rec_val = rval;
        st = launch_mttkrp_seg(a, s);
        if (st == SPT_OK) st = launch_fill_zero(out, rows * (int64_t)rank, s);
        if (st == SPT_OK) st = launch_reduce_records(rrow, nullptr, rval, P, rank, rows, out, s);
        release();
        return st;
    }
    keys2 = (uint64_t *)dev_alloc(sizeof(uint64_t) * n1, s);
    ia = (uint32_t *)dev_alloc(sizeof(uint32_t) * n1, s);
    ib = (uint32_t *)dev_alloc(sizeof(uint32_t) * n1, s);
    cnt = (uint32_t *)dev_alloc(sizeof(uint32_t) * sort_ws_counts((int64_t)n1), s);
    if (!keys2 || !ia || !ib || !cnt) {
        release();
        return fail(SPT_E_OOM, "mttkrp: record workspace allocation failed");
    }
    ta->rec_row = rrow;
    ta->rec_val = rval;
    st = launch_table(*ta, nwg, s);
    uint64_t *srow = nullptr;
    uint32_t *sidx = nullptr;
    if (st == SPT_OK) st = sort_u64_keys_ws(rrow, keys2, ia, ib, cnt, P, t->lbits[a.mode], &srow, &sidx, s);
    if (st == SPT_OK) st = launch_fill_zero(out, rows * (int64_t)rank, s);
    if (st == SPT_OK) st = launch_reduce_records(srow, sidx, rval, P, rank, rows, out, s);
    release();
    return st;
}

int64_t max_plan_records(const Tensor *t) {
    int64_t m = 0;
    for (int n = 0; n < t->nmodes; ++n)
        if (t->mplan[n].valid) m = std::max<int64_t>(m, t->mplan[n].records);
    return m;
}

spt_status run_mttkrp_impl(Tensor *t, const float *const *factors, int rank, int mode, float *out, hipStream_t s,
                           const RecordWs *ws) {
    ModePlan *p = nullptr;
    spt_status st = resolve_plan(t, mode, rank, s, &p, false);
    if (st != SPT_OK) return st;
    const int64_t rows = t->dims[mode];
    if (p->strategy == SPT_STRATEGY_SEGMENT && t->nnz > 0) {
        MttkrpArgs a = make_args(t, factors, rank, mode, out, p->ts);
        a.pl_pos = p->pl_pos;
        a.pl_off = p->pl_off;
        a.pl_piece = p->pl_piece;
        a.rec_cap = p->records;
        // row cache: 4096-nonzero tiles, when the cache holds enough rows and
        // every non-output mode has its tile dictionary (spt_tensor_prepare)
        const int cap = p->ts == kDictTile ? dict_cap(t->nmodes, rank) : 0;
        if (cap > 0 && t->plan.row_cache != 0) {
            bool all = true;
            for (int k = 0; k < t->nmodes; ++k)
                if (k != mode) all = all && t->dict_slot[k] != nullptr;
            if (all) {
                for (int o = 0, k = 0; k < t->nmodes; ++k) {
                    if (k == mode) continue;
                    a.d_slot[o] = t->dict_slot[k];
                    a.d_row[o] = t->dict_row[k];
                    a.d_off[o] = t->dict_off[k];
                    ++o;
                }
                a.d_cap = cap;
            }
        }
        return reduce_via_records(t, a, p->records, rank, rows, out, s, /*segment=*/true, nullptr, 0, ws);
    }
    if (t->nnz == 0 || p->strategy == SPT_STRATEGY_SEGMENT || p->strategy == SPT_STRATEGY_DIRECT ||
        p->strategy == SPT_STRATEGY_REGROUP) {
        st = launch_fill_zero(out, rows * (int64_t)rank, s);
        if (st != SPT_OK || t->nnz == 0) return st;
        return launch_mttkrp(make_args(t, factors, rank, mode, out, std::min(t->plan.tile[mode], 1024)), p->strategy, s);
    }
    TableArgs ta{};
    ta.a = make_args(t, factors, rank, mode, out, 0);
    ta.cap = p->cap;
    ta.hbits = p->hbits;
    ta.stride = p->stride;
    ta.rs = p->rs;
    ta.ts = p->ts;
    ta.sub_per_wg = p->sub_per_wg;
    if (p->strategy == SPT_STRATEGY_PRIV) {
        float *part = (float *)dev_alloc(sizeof(float) * (size_t)p->nwg * rows * rank, s);
        if (!part) return fail(SPT_E_OOM, "mttkrp: partials allocation failed");
        ta.rec_val = part;
        st = launch_priv(ta, p->nwg, p->npass, s);
        if (st == SPT_OK) st = launch_reduce_priv(part, p->nwg, rows, rank, out, s);
        dev_free(part, s);
        return st;
    }
    // TABLE
    ta.rec_off = p->rec_off;
    MttkrpArgs a = ta.a;
    a.rec_off = p->rec_off;
    return reduce_via_records(t, a, p->records, rank, rows, out, s, /*segment=*/false, &ta, p->nwg);
}

}  // namespace spt

namespace spt {
// FP64 MTTKRP over the tensor's SEGMENT plan with call-owned FP64 records.
spt_status run_mttkrp_f64(Tensor *t, const double *const *factors, int rank, int mode, double *out, hipStream_t s) {
    if (!t->vals64 && t->nnz > 0) return fail(SPT_E_INVALID_ARG, "mttkrp_f64: no FP64 values (spt_tensor_attach_f64)");
    ModePlan *p = nullptr;
    spt_status st = resolve_plan(t, mode, rank, s, &p, false);
    if (st != SPT_OK) return st;
    if (p->strategy != SPT_STRATEGY_SEGMENT)
        return fail(SPT_E_INVALID_ARG, "mttkrp_f64: runs the SEGMENT plan (strategy SEGMENT or AUTO)");
    const int64_t rows = t->dims[mode];
    if (t->nnz == 0) return launch_fill_zero((float *)out, 2 * rows * (int64_t)rank, s);  // FP64 zeros: zero bits
    if (!f64_tile_ok(p->ts, t->nmodes)) return fail(SPT_E_INVALID_ARG, "mttkrp_f64: the plan's tile does not fit LDS");
    MttkrpArgs a = make_args(t, nullptr, rank, mode, nullptr, p->ts);
    a.pl_pos = p->pl_pos;
    a.pl_off = p->pl_off;
    a.pl_piece = p->pl_piece;
    a.rec_cap = p->records;
    const size_t n1 = (size_t)std::max<int64_t>(p->records, 1);
    uint64_t *rrow = (uint64_t *)dev_alloc(sizeof(uint64_t) * n1, s);
    double *rval = (double *)dev_alloc(sizeof(double) * n1 * rank, s);
    if (!rrow || !rval) {
        dev_free(rrow, s);
        dev_free(rval, s);
        return fail(SPT_E_OOM, "mttkrp_f64: record workspace");
    }
    a.rec_row = rrow;
    st = launch_mttkrp_seg_f64(a, t->vals64, factors, rval, s);
    if (st == SPT_OK) st = launch_fill_zero((float *)out, 2 * rows * (int64_t)rank, s);
    if (st == SPT_OK) st = launch_reduce_records_f64(rrow, rval, p->records, rank, rows, out, s);
    dev_free(rrow, s);
    dev_free(rval, s);
    return st;
}
}  // namespace spt

// ---------------------------------------------------------------- no-allocation MTTKRP
// For callers that cannot allocate device memory (code under graph capture,
// tight serving loops): the record workspace of the SEGMENT strategy lives in
// a fixed device array.  Host code never passes `scratch` itself to a kernel
// (its name is a host-side stand-in); it uses the device address taken once
// per device with hipGetSymbolAddress.  Every call on one GPU shares that
// array, so calls that overlap on one GPU race.
namespace spt {
namespace {
constexpr size_t kScratchBytes = SPT_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

spt_status scratch_ptr(void **out) {
    int dev = 0;
    SPT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SPT_E_DEVICE, "mttkrp_noalloc: device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "mttkrp_noalloc: scratch address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SPT_OK;
}
}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

// The SEGMENT (and DIRECT/REGROUP) paths of run_mttkrp_impl with the records
// in the fixed array instead of call-owned buffers.  Nothing here allocates.
spt_status run_mttkrp_noalloc(Tensor *t, const float *const *factors, int rank, int mode, float *out, hipStream_t s) {
    ModePlan *p = nullptr;
    spt_status st = resolve_plan(t, mode, rank, s, &p, false);
    if (st != SPT_OK) return st;
    const int64_t rows = t->dims[mode];
    if (t->nnz == 0 || p->strategy == SPT_STRATEGY_DIRECT || p->strategy == SPT_STRATEGY_REGROUP) {
        st = launch_fill_zero(out, rows * (int64_t)rank, s);
        if (st != SPT_OK || t->nnz == 0) return st;
        return launch_mttkrp(make_args(t, factors, rank, mode, out, std::min(t->plan.tile[mode], 1024)), p->strategy, s);
    }
    if (p->strategy != SPT_STRATEGY_SEGMENT)
        return fail(SPT_E_INVALID_ARG, "mttkrp_noalloc: only the SEGMENT, DIRECT and REGROUP strategies run without allocation");
    const int64_t P = p->records;
    const size_t row_bytes = ((sizeof(uint64_t) * (size_t)std::max<int64_t>(P, 1)) + 255) & ~size_t(255);
    const size_t need = row_bytes + sizeof(float) * (size_t)std::max<int64_t>(P, 1) * rank;
    if (need > kScratchBytes)
        return fail(SPT_E_INVALID_ARG, "mttkrp_noalloc: " + std::to_string(P) + " records of rank " + std::to_string(rank) +
                                           " need " + std::to_string(need) + " bytes of scratch, above the " +
                                           std::to_string(kScratchBytes) + "-byte maximum");
    void *base = nullptr;
    st = scratch_ptr(&base);
    if (st != SPT_OK) return st;
    MttkrpArgs a = make_args(t, factors, rank, mode, out, p->ts);
    a.pl_pos = p->pl_pos;
    a.pl_off = p->pl_off;
    a.pl_piece = p->pl_piece;
    a.rec_cap = P;
    const int cap = p->ts == kDictTile ? dict_cap(t->nmodes, rank) : 0;
    if (cap > 0 && t->plan.row_cache != 0) {
        bool all = true;
        for (int k = 0; k < t->nmodes; ++k)
            if (k != mode) all = all && t->dict_slot[k] != nullptr;
        if (all) {
            for (int o = 0, k = 0; k < t->nmodes; ++k) {
                if (k == mode) continue;
                a.d_slot[o] = t->dict_slot[k];
                a.d_row[o] = t->dict_row[k];
                a.d_off[o] = t->dict_off[k];
                ++o;
            }
            a.d_cap = cap;
        }
    }
    // every record the plan lays out is written by the main kernel before the
    // reduction reads it, so the array needs no clearing between calls
    a.rec_row = (uint64_t *)base;
    a.rec_val = (float *)((char *)base + row_bytes);
    st = launch_mttkrp_seg(a, s);
    if (st == SPT_OK) st = launch_fill_zero(out, rows * (int64_t)rank, s);
    if (st == SPT_OK) st = launch_reduce_records(a.rec_row, nullptr, a.rec_val, P, rank, rows, out, s);
    return st;
}

}  // namespace spt
