// Lock-step CP-ALS of many independent tensors (many decompositions run side
// by side, as in the paper's workflow of repeated decompositions, Section
// IV-D) and the batched MTTKRP behind it.
//
// Per mode index n, every member tensor with more than n modes takes part in
// ONE launch of each step:
//   * SEGMENT MTTKRP over all members' tiles in one persistent launch (one
//     tile size per launch: the batched tile of the first member);
//     records carry rows of a concatenated output M_all (member b's rows start
//     at row_base[b], leading dimension ld = the largest rank of the mode),
//     one radix sort of all records by row, one segmented reduction into M_all;
//   * Gram of every member's block of M_all, the FP64 normal-equation solve,
//     the apply (factor = M S, rounded to FP32, fit inner product on the last
//     mode), and the Gram of the new factor, each one workgroup per member
//     (apply: a grid over all members' row blocks).
// One FP64 fit kernel for all members and one host readback close the
// iteration; members leave the active set when they converge.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "spt_internal.h"

namespace spt {

spt_status check_factors(const Tensor *t, const float *const *factors, int rank, int skip_mode);

namespace {

int bit_len(int64_t x) {  // bits to hold values 0..x-1
    int b = 0;
    while ((int64_t(1) << b) < x) ++b;
    return b;
}

// give every Gram item its row slices in the launch; returns the total
int64_t assign_slices(std::vector<GramItem> &v) {
    int64_t run = 0;
    for (GramItem &g : v) {
        g.first_slice = run;
        g.nslices = gram_slices(g.rows);
        run += g.nslices;
    }
    return run;
}

void set_batch_plan_args(MttkrpArgs &a, const ModePlan &p) {
    a.pl_off = p.pl_off;
    a.pl_pos = p.pl_pos;
    a.pl_desc = p.pl_desc;
    a.pl_row = p.pl_row;
    a.pl_dest = p.pl_dest;
    a.rec_cap = p.records;
}

}  // namespace

// Builds the batched SEGMENT plan of `mode` for every tensor that lacks it,
// for all of them at once: one counting launch and readback, one emission
// launch, one sort of all distinct (tile, row) pairs by row of the
// concatenated output (tensors in order, tile order kept within a row), one
// scan of their piece counts.  Each tensor's records come out grouped by row,
// numbered from 0 within the tensor.
int batch_tile_of(const Tensor *t) {
    const int b = t->plan.batch_tile;
    return (b == 1024 || b == 2048 || b == 4096) ? b : kBatchTileDefault;
}

spt_status ensure_batch_plans(const std::vector<Tensor *> &ts, int mode, int tile, hipStream_t s) {
    std::vector<Tensor *> need;
    for (Tensor *t : ts) {
        if (t->nmodes <= mode) continue;
        if (t->bplan[mode].pl_off && t->bplan[mode].ts != tile) release_batch_plan(t, mode, s);  // stream-ordered
        if (!t->bplan[mode].pl_off) need.push_back(t);
    }
    if (need.empty()) return SPT_OK;
    const int n = (int)need.size();
    int nmax = 0;
    std::vector<SegItem> items(n);
    int64_t tiles = 0, rows = 0;
    for (int i = 0; i < n; ++i) {
        items[i] = SegItem{};
        items[i].a = make_args(need[i], nullptr, 1, mode, nullptr, tile);
        items[i].first_tile = tiles;
        items[i].row_base = rows;
        tiles += (need[i]->nnz + tile - 1) / tile;
        rows += need[i]->dims[mode];
        nmax = std::max(nmax, need[i]->nmodes);
    }
    if (!seg_batch_fits(nmax, tile)) return fail(SPT_E_INVALID_ARG, "batch: too many modes for the batched tile");
    if (tiles == 0) return SPT_OK;
    DevBuf d_items, d_cnt;
    std::vector<int64_t> h(tiles, 0);
    if (!d_items.get(sizeof(SegItem) * n, s) || !d_cnt.get(sizeof(int64_t) * tiles, s)) {
        d_items.release(s);
        d_cnt.release(s);
        return fail(SPT_E_OOM, "batch plan: counts");
    }
    SPT_HIP(hipMemcpyAsync(d_items.p, items.data(), sizeof(SegItem) * n, hipMemcpyHostToDevice, s));
    spt_status st = launch_count_pieces_batched((SegItem *)d_items.p, n, tiles, nmax, tile, (int64_t *)d_cnt.p, s);
    if (st == SPT_OK && (hipMemcpyAsync(h.data(), d_cnt.p, sizeof(int64_t) * tiles, hipMemcpyDeviceToHost, s) != hipSuccess ||
                         hipStreamSynchronize(s) != hipSuccess))
        st = hip_fail(hipGetLastError(), "batch plan: counts");
    if (st != SPT_OK) {
        d_items.release(s);
        d_cnt.release(s);
        return st;
    }
    // offsets: per tensor (local pieces per tile) and batch-wide (pieces, pairs)
    std::vector<std::vector<int64_t>> loff(n);
    std::vector<int64_t> gpiece(tiles), gpair(tiles), piece_base(n + 1, 0);
    int64_t G = 0, Q = 0;
    for (int i = 0; i < n; ++i) {
        const int64_t nt = (need[i]->nnz + tile - 1) / tile;
        loff[i].assign(nt + 1, 0);
        piece_base[i] = G;
        int64_t local = 0;
        for (int64_t k = 0; k < nt; ++k) {
            const int64_t it = items[i].first_tile + k, c = h[it];
            loff[i][k] = local;
            gpiece[it] = G + local;
            gpair[it] = Q;
            local += c & 0xFFFFFFFFll;
            Q += c >> 32;
        }
        loff[i][nt] = local;
        G += local;
    }
    piece_base[n] = G;
    if (G >= (int64_t(1) << 32)) {
        d_items.release(s);
        d_cnt.release(s);
        return fail(SPT_E_INVALID_ARG, "batch plan: more than 2^32 records");
    }
    // the tensors' plan arrays (stream-ordered: released without a device-wide sync)
    for (int i = 0; i < n; ++i) {
        Tensor *t = need[i];
        ModePlan &p = t->bplan[mode];
        const int64_t nt = (int64_t)loff[i].size() - 1, P = loff[i][nt];
        p.pl_off = (int64_t *)dev_alloc(sizeof(int64_t) * (nt + 1), s);
        p.pl_pos = (uint16_t *)dev_alloc(sizeof(uint16_t) * std::max<int64_t>(t->nnz, 1), s);
        p.pl_desc = (uint32_t *)dev_alloc(sizeof(uint32_t) * std::max<int64_t>(P, 1), s);
        p.pl_row = (uint32_t *)dev_alloc(sizeof(uint32_t) * std::max<int64_t>(P, 1), s);
        p.pl_dest = (uint32_t *)dev_alloc(sizeof(uint32_t) * std::max<int64_t>(P, 1), s);
        if (!p.pl_off || !p.pl_pos || !p.pl_desc || !p.pl_row || !p.pl_dest) {
            (void)hipStreamSynchronize(s);  // copies from host vectors may be in flight
            for (int k = 0; k <= i; ++k) release_batch_plan(need[k], mode, s);
            d_items.release(s);
            d_cnt.release(s);
            return fail(SPT_E_OOM, "batch plan: arrays");
        }
        SPT_HIP(hipMemcpyAsync(p.pl_off, loff[i].data(), sizeof(int64_t) * (nt + 1), hipMemcpyHostToDevice, s));
        p.ts = tile;
        p.records = P;
        p.strategy = SPT_STRATEGY_SEGMENT;
        p.valid = 1;
        SegItem &it = items[i];
        it.a.pl_off = p.pl_off;
        it.a.pl_pos = p.pl_pos;
        it.a.pl_desc = p.pl_desc;
        it.a.pl_row = p.pl_row;
        it.a.pl_dest = p.pl_dest;
        it.a.rec_cap = P;
    }
    SPT_HIP(hipMemcpyAsync(d_items.p, items.data(), sizeof(SegItem) * n, hipMemcpyHostToDevice, s));
    const size_t g1 = (size_t)std::max<int64_t>(G, 1), q1 = (size_t)std::max<int64_t>(Q, 1);
    DevBuf d_gpiece, d_gpair, d_base, ppair, psub, keys, keys2, np, ia, ib, cnt;
    if (!d_gpiece.get(sizeof(int64_t) * tiles, s) || !d_gpair.get(sizeof(int64_t) * tiles, s) ||
        !d_base.get(sizeof(int64_t) * (n + 1), s) || !ppair.get(sizeof(uint32_t) * g1, s) ||
        !psub.get(sizeof(uint32_t) * g1, s) || !keys.get(sizeof(uint64_t) * q1, s) ||
        !keys2.get(sizeof(uint64_t) * q1, s) || !np.get(sizeof(uint32_t) * q1, s) || !ia.get(sizeof(uint32_t) * q1, s) ||
        !ib.get(sizeof(uint32_t) * q1, s) ||
        !cnt.get(sizeof(uint32_t) * std::max(sort_ws_counts(Q), exclusive_scan_ws(Q)), s)) {
        (void)hipStreamSynchronize(s);
        for (Tensor *t : need) release_batch_plan(t, mode, s);
        for (DevBuf *b : {&d_items, &d_cnt, &d_gpiece, &d_gpair, &d_base, &ppair, &psub, &keys, &keys2, &np, &ia, &ib, &cnt})
            b->release(s);
        return fail(SPT_E_OOM, "batch plan: workspace");
    }
    SPT_HIP(hipMemcpyAsync(d_gpiece.p, gpiece.data(), sizeof(int64_t) * tiles, hipMemcpyHostToDevice, s));
    SPT_HIP(hipMemcpyAsync(d_gpair.p, gpair.data(), sizeof(int64_t) * tiles, hipMemcpyHostToDevice, s));
    SPT_HIP(hipMemcpyAsync(d_base.p, piece_base.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s));
    st = launch_emit_plan_batched((SegItem *)d_items.p, n, tiles, nmax, tile, (int64_t *)d_gpiece.p, (int64_t *)d_gpair.p,
                                  (uint32_t *)ppair.p, (uint32_t *)psub.p, (uint64_t *)keys.p, (uint32_t *)np.p, s);
    uint64_t *sk = nullptr;
    uint32_t *sidx = nullptr;
    if (st == SPT_OK)
        st = sort_u64_keys_ws((uint64_t *)keys.p, (uint64_t *)keys2.p, (uint32_t *)ia.p, (uint32_t *)ib.p,
                              (uint32_t *)cnt.p, Q, bit_len(rows), &sk, &sidx, s);
    uint32_t *np_sorted = (sidx == (uint32_t *)ia.p) ? (uint32_t *)ib.p : (uint32_t *)ia.p;
    uint32_t *tmp = (uint32_t *)((sk == (uint64_t *)keys2.p) ? keys.p : keys2.p);  // free after the sort
    uint32_t *pair_first = tmp + q1;
    if (st == SPT_OK) st = launch_gather_u32((uint32_t *)np.p, sidx, np_sorted, Q, s);
    if (st == SPT_OK) st = launch_exclusive_scan_u32(np_sorted, tmp, Q, (uint32_t *)cnt.p, s);
    if (st == SPT_OK) st = launch_scatter_u32(tmp, sidx, pair_first, Q, s);
    if (st == SPT_OK)
        st = launch_piece_dest_batched((SegItem *)d_items.p, n, (int64_t *)d_base.p, (uint32_t *)ppair.p,
                                       (uint32_t *)psub.p, pair_first, G, s);
    if (st == SPT_OK && hipStreamSynchronize(s) != hipSuccess) st = hip_fail(hipGetLastError(), "batch plan: build");
    if (st != SPT_OK) {
        (void)hipStreamSynchronize(s);
        for (Tensor *t : need) release_batch_plan(t, mode, s);
    }
    for (DevBuf *b : {&d_items, &d_cnt, &d_gpiece, &d_gpair, &d_base, &ppair, &psub, &keys, &keys2, &np, &ia, &ib, &cnt})
        b->release(s);
    return st;
}

spt_status prepare_batched(Tensor *t, hipStream_t s) {
    std::vector<Tensor *> one{t};
    for (int n = 0; n < t->nmodes; ++n) {
        spt_status st = ensure_batch_plans(one, n, batch_tile_of(t), s);
        if (st != SPT_OK) return st;
    }
    return SPT_OK;
}

// The batched MTTKRP pipeline of one mode into M_all (rows x ld, overwritten).
spt_status run_mttkrp_batched_mode(const SegItem *d_items, int count, int64_t total_tiles, int nmodes_min, int nmodes_max,
                                   int tile, int64_t records, int64_t rows, int ld, bool vec4, float *M_all,
                                   BatchMttkrpWs &ws, hipStream_t s) {
    if (rows == 0) return SPT_OK;
    if (records == 0 || total_tiles == 0) return launch_fill_zero(M_all, rows * (int64_t)ld, s);
    if (records >= (int64_t(1) << 32)) return fail(SPT_E_INVALID_ARG, "batch: more than 2^32 records");
    const size_t n1 = (size_t)records;
    uint64_t *rrow = (uint64_t *)ws.rec_row.get(sizeof(uint64_t) * n1, s);
    float *rval = (float *)ws.rec_val.get(sizeof(float) * n1 * ld, s);
    unsigned long long *counter = (unsigned long long *)ws.counter.get(256, s);
    if (!rrow || !rval || !counter) return fail(SPT_E_OOM, "batch: record workspace");
    // the batch's records come out grouped by row: no sort
    spt_status st = launch_mttkrp_seg_batched(d_items, count, total_tiles, nmodes_min, nmodes_max, tile, ld, vec4, rrow,
                                              rval, counter, s);
    if (st == SPT_OK) st = launch_fill_zero(M_all, rows * (int64_t)ld, s);
    if (st == SPT_OK) st = launch_reduce_records(rrow, nullptr, rval, records, ld, rows, M_all, s);
    return st;
}

// ---------------------------------------------------------------- staged uploads
// Host-to-device copies of per-call item tables go through a ring of pinned
// host slots, each guarded by an event: a copy from pinned memory is truly
// asynchronous, and a slot is reused only once its previous copy has run
// (the host waits only when every slot's copy is still queued).
namespace {
struct PinnedSlot {
    void *host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
};
constexpr int kPinnedSlots = 8;
std::mutex g_pin_mu;
PinnedSlot g_pin[kPinnedSlots];
int g_pin_next = 0;
}  // namespace

spt_status upload_staged(void *dst, const void *src, size_t bytes, hipStream_t s) {
    if (bytes == 0) return SPT_OK;
    std::lock_guard<std::mutex> lk(g_pin_mu);
    PinnedSlot &p = g_pin[g_pin_next];
    g_pin_next = (g_pin_next + 1) % kPinnedSlots;
    if (p.done) SPT_HIP(hipEventSynchronize(p.done));  // the slot's previous copy
    else SPT_HIP(hipEventCreateWithFlags(&p.done, hipEventDisableTiming));
    if (p.bytes < bytes) {
        if (p.host) SPT_HIP(hipHostFree(p.host));
        p.host = nullptr;
        p.bytes = 0;
        const size_t want = std::max<size_t>(bytes, 64 * 1024);
        SPT_HIP(hipHostMalloc(&p.host, want, hipHostMallocDefault));
        p.bytes = want;
    }
    std::memcpy(p.host, src, bytes);
    SPT_HIP(hipMemcpyAsync(dst, p.host, bytes, hipMemcpyHostToDevice, s));
    SPT_HIP(hipEventRecord(p.done, s));
    return SPT_OK;
}

// ---------------------------------------------------------------- engine
BatchEngine::BatchEngine(hipStream_t s) : s_(s) {}

// Every engine buffer is released in stream order on the engine's stream:
// work already queued keeps its memory until it has run.
BatchEngine::~BatchEngine() {
    for (Member *m : members_) free_member_state(m);
    release_buffers();
}

void BatchEngine::release_buffers() {
    for (DevBuf *b : {&items_buf_, &M_buf_, &fit_buf_, &status_buf_, &inner_buf_, &resid_buf_, &resid_items_buf_, &gram_ws_})
        b->release(s_);
    d_items_ = nullptr;
    M_all_ = nullptr;
    fit_all_ = nullptr;
    status_all_ = nullptr;
    inner_all_ = nullptr;
    resid_ = nullptr;
    ws_.release(s_);
}

void BatchEngine::free_member_state(Member *m) {
    dev_free(m->state, s_);  // stream-ordered after the member's last kernels
    m->state = nullptr;
}

spt_status BatchEngine::add(Member *m) {
    Tensor *t = m->t;
    if (!t || m->R < 1 || m->R > SPT_MAX_ALS_RANK) return fail(SPT_E_INVALID_ARG, "batch: rank must be 1..64");
    if (!(t->norm_x2 > 0.0)) return fail(SPT_E_INVALID_ARG, "batch: tensor norm is zero");
    spt_status st = check_factors(t, (const float *const *)m->F, m->R, -1);
    if (st != SPT_OK) return st;
    const int N = t->nmodes, R = m->R;
    const size_t bytes = sizeof(double) * ((size_t)N * R * R + 2 * (size_t)R * R);
    m->state = dev_alloc(bytes, s_);
    if (!m->state) return fail(SPT_E_OOM, "batch: member state");
    m->grams = (double *)m->state;
    m->gram_m = m->grams + (size_t)N * R * R;
    m->S = m->gram_m + (size_t)R * R;
    m->fit = m->fit_prev = 0.0;
    m->iters = 0;
    m->done = false;
    m->err = SPT_OK;
    m->fresh = true;
    members_.push_back(m);
    dirty_ = true;
    return SPT_OK;
}

void BatchEngine::remove(Member *m) {
    auto it = std::find(members_.begin(), members_.end(), m);
    if (it == members_.end()) return;
    free_member_state(m);
    members_.erase(it);
    dirty_ = true;
}

// Per-mode item arrays and workspace sizes for the current members.
spt_status BatchEngine::rebuild() {
    std::vector<Member *> act;
    for (Member *m : members_)
        if (!m->done) act.push_back(m);
    active_ = act;
    nmodes_max_ = 0;
    nmodes_min_ = kMaxModes;
    for (Member *m : act) {
        nmodes_max_ = std::max(nmodes_max_, m->t->nmodes);
        nmodes_min_ = std::min(nmodes_min_, m->t->nmodes);
    }
    // one tile size for the whole batch: the first member's batched tile
    tile_ = act.empty() ? kBatchTileDefault : batch_tile_of(act[0]->t);
    if (!act.empty() && !seg_batch_fits(nmodes_max_, tile_)) return fail(SPT_E_INVALID_ARG, "batch: too many modes");
    std::vector<Tensor *> ts;
    for (Member *m : act) ts.push_back(m->t);
    for (int n = 0; n < nmodes_max_; ++n) {
        spt_status st = ensure_batch_plans(ts, n, tile_, s_);
        if (st != SPT_OK) return st;
    }
    // host images of every item array, packed into one upload
    std::vector<char> blob;
    blob.reserve(blob_.capacity());
    auto put = [&blob](const void *p, size_t bytes) {
        const size_t off = (blob.size() + 255) & ~size_t(255);
        blob.resize(off + bytes);
        if (bytes) std::memcpy(blob.data() + off, p, bytes);
        return off;
    };
    const int A = (int)act.size();
    // inner-product partials: one range per member for its last mode
    std::vector<int64_t> inner_base(A, 0), inner_n(A, 0);
    int64_t inner_total = 0;
    modes_.assign(nmodes_max_, ModeItems{});
    size_t M_need = 0, gram_need = 0;
    int64_t max_records = 0;
    for (int n = 0; n < nmodes_max_; ++n) {
        ModeItems &mi = modes_[n];
        std::vector<SegItem> seg;
        std::vector<GramItem> gm;
        std::vector<SolveItem> sv;
        std::vector<ApplyItem> ap;
        int rmax = 0;
        bool vec4 = true;
        for (Member *m : act)
            if (m->t->nmodes > n) {
                rmax = std::max(rmax, m->R);
                vec4 = vec4 && (m->R % 4 == 0);
            }
        const int ld = rmax;
        const int rw = rmax > 0 ? apply_rows_per_launch_block(rmax) : 1;
        int64_t tiles = 0, recs = 0, rows = 0, blocks = 0;
        for (int i = 0; i < A; ++i) {
            Member *m = act[i];
            Tensor *t = m->t;
            if (t->nmodes <= n) continue;
            const int R = m->R;
            SegItem si{};
            si.a = make_args(t, (const float *const *)m->F, R, n, nullptr, tile_);
            set_batch_plan_args(si.a, t->bplan[n]);
            si.first_tile = tiles;
            si.rec_base = recs;
            si.row_base = rows;
            seg.push_back(si);
            const int64_t In = t->dims[n];
            // M_all block of this member: filled in below once M_all exists (offset only here)
            GramItem g1{};
            g1.C = reinterpret_cast<const float *>((uintptr_t)(rows * ld));  // element offset, rebased later
            g1.rows = In;
            g1.ld = ld;
            g1.rank = R;
            g1.G = m->gram_m;
            gm.push_back(g1);
            SolveItem so{};
            so.grams = m->grams;
            so.gram_m = m->gram_m;
            so.S = m->S;
            so.lambda = m->lambda;
            so.status = nullptr;  // rebased below (status_all + 8 i)
            so.gram_new = m->grams + (size_t)n * R * R;  // the solve forms the new factor's Gram
            so.nmodes = t->nmodes;
            so.rank = R;
            sv.push_back(so);
            ApplyItem ai{};
            ai.M = reinterpret_cast<const float *>((uintptr_t)(rows * ld));
            ai.S = m->S;
            ai.C = m->F[n];
            ai.lambda = m->lambda;
            const int64_t nb = std::max<int64_t>(1, (In + rw - 1) / rw);
            if (n == t->nmodes - 1) {
                inner_base[i] = inner_total;
                inner_n[i] = nb;
                inner_total += nb;
                ai.inner = reinterpret_cast<double *>((uintptr_t)(inner_base[i] + 1));  // marker, rebased below
            }
            ai.rows = In;
            ai.first_block = blocks;
            ai.ldm = ld;
            ai.rank = R;
            ap.push_back(ai);
            mi.member_idx.push_back(i);
            tiles += (t->nnz + tile_ - 1) / tile_;
            recs += t->bplan[n].records;
            rows += In;
            blocks += nb;
        }
        mi.count = (int)seg.size();
        mi.tiles = tiles;
        mi.records = recs;
        mi.rows = rows;
        mi.blocks = blocks;
        mi.ld = ld;
        mi.rmax = rmax;
        mi.vec4 = vec4;
        M_need = std::max(M_need, sizeof(float) * (size_t)rows * std::max(ld, 1));
        max_records = std::max(max_records, recs);
        mi.seg_v = std::move(seg);
        mi.gm_slices = assign_slices(gm);
        gram_need = std::max(gram_need, gram_batched_ws_bytes(mi.gm_slices, rmax));
        mi.gm_v = std::move(gm);
        mi.sv_v = std::move(sv);
        mi.ap_v = std::move(ap);
    }
    (void)max_records;
    // device buffers that item pointers refer to (replaced in stream order)
    M_all_ = (float *)M_buf_.get(std::max<size_t>(M_need, 256), s_);
    fit_all_ = (double *)fit_buf_.get(sizeof(double) * 4 * std::max(A, 1), s_);
    status_all_ = (int *)status_buf_.get(sizeof(int) * kMaxModes * std::max(A, 1), s_);
    inner_all_ = (double *)inner_buf_.get(sizeof(double) * std::max<int64_t>(inner_total, 1), s_);
    if (!M_all_ || !fit_all_ || !status_all_ || !inner_all_) return fail(SPT_E_OOM, "batch: engine buffers");
    // rebase offsets into real pointers and pack
    std::vector<FitItem> fit(A);
    for (int i = 0; i < A; ++i) {
        Member *m = act[i];
        FitItem f{};
        f.grams = m->grams;
        f.lambda = m->lambda;
        f.inner = inner_all_ + inner_base[i];
        f.nparts = (int)inner_n[i];
        f.out = fit_all_ + 4 * i;
        f.norm_x2 = m->t->norm_x2;
        f.nmodes = m->t->nmodes;
        f.rank = m->R;
        fit[i] = f;
    }
    for (int n = 0; n < nmodes_max_; ++n) {
        ModeItems &mi = modes_[n];
        for (size_t k = 0; k < mi.gm_v.size(); ++k) {
            mi.gm_v[k].C = M_all_ + (uintptr_t)mi.gm_v[k].C;
            mi.ap_v[k].M = M_all_ + (uintptr_t)mi.ap_v[k].M;
            if (mi.ap_v[k].inner) mi.ap_v[k].inner = inner_all_ + ((uintptr_t)mi.ap_v[k].inner - 1);
            mi.sv_v[k].status = status_all_ + kMaxModes * mi.member_idx[k];
        }
        mi.seg_off = put(mi.seg_v.data(), sizeof(SegItem) * mi.seg_v.size());
        mi.gm_off = put(mi.gm_v.data(), sizeof(GramItem) * mi.gm_v.size());
        mi.sv_off = put(mi.sv_v.data(), sizeof(SolveItem) * mi.sv_v.size());
        mi.ap_off = put(mi.ap_v.data(), sizeof(ApplyItem) * mi.ap_v.size());
    }
    fit_off_ = put(fit.data(), sizeof(FitItem) * fit.size());
    // initial Grams of the new members' factors
    std::vector<GramItem> init;
    int init_rmax = 0;
    for (Member *m : act)
        if (m->fresh) {
            for (int k = 0; k < m->t->nmodes; ++k) {
                GramItem g{};
                g.C = m->F[k];
                g.rows = m->t->dims[k];
                g.ld = m->R;
                g.rank = m->R;
                g.G = m->grams + (size_t)k * m->R * m->R;
                init.push_back(g);
            }
            init_rmax = std::max(init_rmax, m->R);
            m->fresh = false;
        }
    init_slices_ = assign_slices(init);
    gram_need = std::max(gram_need, gram_batched_ws_bytes(init_slices_, std::max(init_rmax, 1)));
    if (!gram_ws_.get(gram_need, s_)) return fail(SPT_E_OOM, "batch: Gram workspace");
    init_off_ = put(init.data(), sizeof(GramItem) * init.size());
    init_count_ = (int)init.size();
    init_rmax_ = init_rmax;
    // the host image lives in the engine until the next rebuild, which comes
    // after a step's synchronisation: the asynchronous upload has run by then
    blob_.swap(blob);
    d_items_ = (char *)items_buf_.get(std::max<size_t>(blob_.size(), 256), s_);
    if (!d_items_) return fail(SPT_E_OOM, "batch: item arrays");
    if (!blob_.empty()) SPT_HIP(hipMemcpyAsync(d_items_, blob_.data(), blob_.size(), hipMemcpyHostToDevice, s_));
    if (init_count_ > 0) {
        spt_status st = launch_gram_batched((const GramItem *)(d_items_ + init_off_), init_count_, init_slices_,
                                            init_rmax_, (double *)gram_ws_.p, s_);
        if (st != SPT_OK) return st;
    }
    dirty_ = false;
    return SPT_OK;
}

void BatchEngine::drop_done() { dirty_ = true; }

spt_status BatchEngine::step(bool *before_kernels) {
    if (before_kernels) *before_kernels = false;
    if (dirty_) {
        spt_status st = rebuild();
        if (st != SPT_OK) {
            if (before_kernels) *before_kernels = true;
            return st;
        }
    }
    const int A = (int)active_.size();
    if (A == 0) return SPT_OK;
    for (int n = 0; n < nmodes_max_; ++n) {
        const ModeItems &mi = modes_[n];
        if (mi.count == 0) continue;
        spt_status st = run_mttkrp_batched_mode((const SegItem *)(d_items_ + mi.seg_off), mi.count, mi.tiles, nmodes_min_,
                                                nmodes_max_, tile_, mi.records, mi.rows, mi.ld, mi.vec4, M_all_, ws_, s_);
        if (st == SPT_OK)
            st = launch_gram_batched((const GramItem *)(d_items_ + mi.gm_off), mi.count, mi.gm_slices, mi.rmax,
                                     (double *)gram_ws_.p, s_);
        if (st == SPT_OK) st = launch_solve_prep_batched((const SolveItem *)(d_items_ + mi.sv_off), mi.count, n, s_);
        if (st == SPT_OK)
            st = launch_apply_batched((const ApplyItem *)(d_items_ + mi.ap_off), mi.count, mi.blocks, mi.rmax, s_);
        if (st != SPT_OK) return st;
    }
    spt_status st = launch_fit_batched((const FitItem *)(d_items_ + fit_off_), A, s_);
    if (st != SPT_OK) return st;
    hfit_.resize(4 * (size_t)A);
    hstat_.resize((size_t)kMaxModes * A);
    if (hipMemcpyAsync(hfit_.data(), fit_all_, sizeof(double) * 4 * A, hipMemcpyDeviceToHost, s_) != hipSuccess ||
        hipMemcpyAsync(hstat_.data(), status_all_, sizeof(int) * kMaxModes * A, hipMemcpyDeviceToHost, s_) != hipSuccess ||
        hipStreamSynchronize(s_) != hipSuccess)
        return hip_fail(hipGetLastError(), "batch: fit readback");
    // direct FP64 residual near convergence, as in the single-tensor driver
    std::vector<int> direct;
    for (int i = 0; i < A; ++i) {
        Member *m = active_[i];
        for (int n = 0; n < m->t->nmodes; ++n)
            if (hstat_[(size_t)kMaxModes * i + n] < 0) {
                m->err = fail(SPT_E_NOT_SPD, "cp_als: normal equations of mode " + std::to_string(n) +
                                                 " not positive definite after ridge retries");
                m->done = true;
                dirty_ = true;
            }
        if (!m->done && 1.0 - hfit_[4 * i] < 1e-2 && m->t->nnz > 0) direct.push_back(i);
    }
    if (!direct.empty()) {
        // one residual launch over every member that takes the direct fit,
        // then one fit launch (a workgroup per member)
        std::vector<ResidItem> ri;
        std::vector<FitDirectItem> fi;
        int64_t tiles = 0;
        int rmax = 0, nmax = 0;
        bool vec4 = true;
        for (int i : direct) {
            Member *m = active_[i];
            ResidItem r{};
            r.a = make_args(m->t, (const float *const *)m->F, m->R, -1, nullptr, kResidTile);
            r.lambda = m->lambda;
            r.first_tile = tiles;  // partials rebased below
            ri.push_back(r);
            FitDirectItem f{};
            f.nparts = (m->t->nnz + kResidTile - 1) / kResidTile;
            f.norm_x2 = m->t->norm_x2;
            f.out = fit_all_ + 4 * i;
            fi.push_back(f);
            tiles += f.nparts;
            rmax = std::max(rmax, m->R);
            nmax = std::max(nmax, m->t->nmodes);
            vec4 = vec4 && m->R % 4 == 0;
        }
        resid_ = (double *)resid_buf_.get(sizeof(double) * 2 * std::max<int64_t>(tiles, 1), s_);
        char *d_ri = (char *)resid_items_buf_.get(sizeof(ResidItem) * ri.size() + 256 + sizeof(FitDirectItem) * fi.size(), s_);
        if (!resid_ || !d_ri) return fail(SPT_E_OOM, "batch: residual partials");
        for (size_t k = 0; k < ri.size(); ++k) {
            ri[k].partials = resid_ + 2 * ri[k].first_tile;
            fi[k].parts = ri[k].partials;
        }
        const size_t fi_off = (sizeof(ResidItem) * ri.size() + 255) & ~size_t(255);
        st = upload_staged(d_ri, ri.data(), sizeof(ResidItem) * ri.size(), s_);
        if (st == SPT_OK) st = upload_staged(d_ri + fi_off, fi.data(), sizeof(FitDirectItem) * fi.size(), s_);
        if (st == SPT_OK)
            st = launch_resid_batched((const ResidItem *)d_ri, (int)ri.size(), tiles, nmax, rmax, vec4, s_);
        if (st == SPT_OK) st = launch_fit_direct_batched((const FitDirectItem *)(d_ri + fi_off), (int)fi.size(), s_);
        if (st != SPT_OK) return st;
        if (hipMemcpyAsync(hfit_.data(), fit_all_, sizeof(double) * 4 * A, hipMemcpyDeviceToHost, s_) != hipSuccess ||
            hipStreamSynchronize(s_) != hipSuccess)
            return hip_fail(hipGetLastError(), "batch: direct fit readback");
    }
    for (int i = 0; i < A; ++i) {
        Member *m = active_[i];
        if (m->done) continue;
        m->fit = hfit_[4 * i];
        ++m->iters;
        const bool conv = m->tol > 0.0 && std::fabs(m->fit - m->fit_prev) < m->tol;
        m->fit_prev = m->fit;
        if (conv || m->iters >= m->max_iters) {
            m->done = true;
            dirty_ = true;
        }
    }
    return SPT_OK;
}

bool BatchEngine::any_active() const {
    for (Member *m : members_)
        if (!m->done) return true;
    return false;
}

}  // namespace spt

using namespace spt;

extern "C" {

spt_status spt_mttkrp_batched(const spt_tensor *ts, int count, const float *const *const *factors, const int *ranks,
                              int mode, float *const *outs, void *stream) {
    if (count < 0 || (count > 0 && (!ts || !factors || !ranks || !outs)))
        return fail(SPT_E_INVALID_ARG, "mttkrp_batched: NULL argument");
    if (mode < 0 || mode >= kMaxModes) return fail(SPT_E_INVALID_ARG, "mttkrp_batched: mode out of range");
    hipStream_t s = (hipStream_t)stream;
    std::vector<Tensor *> tv;
    std::vector<int> idx;
    int rmax = 0, nmax = 0, nmin = kMaxModes, tile = 0;
    bool vec4 = true;
    for (int b = 0; b < count; ++b) {
        Tensor *t = ts[b];
        if (!t) return fail(SPT_E_INVALID_ARG, "mttkrp_batched: NULL tensor " + std::to_string(b));
        if (t->nmodes <= mode) continue;
        if (ranks[b] < 1 || ranks[b] > 64) return fail(SPT_E_INVALID_ARG, "mttkrp_batched: rank must be 1..64");
        if (!outs[b]) return fail(SPT_E_INVALID_ARG, "mttkrp_batched: NULL output " + std::to_string(b));
        if (tile == 0) tile = batch_tile_of(t);  // one tile size per launch: the first member's
        if (!t->bplan[mode].pl_off || t->bplan[mode].ts != tile)
            return fail(SPT_E_INVALID_ARG, "mttkrp_batched: tensor " + std::to_string(b) +
                                               " not prepared for the batched launch at the batch's tile of " +
                                               std::to_string(tile) + " (spt_tensor_prepare, plan batch_tile)");
        spt_status st = check_factors(t, factors[b], ranks[b], mode);
        if (st != SPT_OK) return st;
        tv.push_back(t);
        idx.push_back(b);
        rmax = std::max(rmax, ranks[b]);
        nmax = std::max(nmax, t->nmodes);
        nmin = std::min(nmin, t->nmodes);
        vec4 = vec4 && ranks[b] % 4 == 0;
    }
    if (tv.empty()) return SPT_OK;
    if (!seg_batch_fits(nmax, tile)) return fail(SPT_E_INVALID_ARG, "mttkrp_batched: too many modes");
    const int ld = rmax;
    std::vector<SegItem> items(tv.size());
    int64_t tiles = 0, recs = 0, rows = 0;
    std::vector<int64_t> row_base(tv.size());
    for (size_t i = 0; i < tv.size(); ++i) {
        Tensor *t = tv[i];
        const int b = idx[i];
        items[i] = SegItem{};
        items[i].a = make_args(t, factors[b], ranks[b], mode, nullptr, tile);
        set_batch_plan_args(items[i].a, t->bplan[mode]);
        items[i].first_tile = tiles;
        items[i].rec_base = recs;
        items[i].row_base = rows;
        row_base[i] = rows;
        tiles += (t->nnz + tile - 1) / tile;
        recs += t->bplan[mode].records;
        rows += t->dims[mode];
    }
    SegItem *d_items = (SegItem *)dev_alloc(sizeof(SegItem) * items.size(), s);
    float *M = (float *)dev_alloc(sizeof(float) * std::max<int64_t>(rows * ld, 1), s);
    if (!d_items || !M) {
        dev_free(d_items, s);
        dev_free(M, s);
        return fail(SPT_E_OOM, "mttkrp_batched: workspace");
    }
    spt_status st = upload_staged(d_items, items.data(), sizeof(SegItem) * items.size(), s);
    BatchMttkrpWs ws;
    if (st == SPT_OK)
        st = run_mttkrp_batched_mode(d_items, (int)items.size(), tiles, nmin, nmax, tile, recs, rows, ld, vec4, M, ws, s);
    for (size_t i = 0; st == SPT_OK && i < tv.size(); ++i) {
        const int b = idx[i];
        const int64_t In = tv[i]->dims[mode];
        if (In == 0) continue;
        if (hipMemcpy2DAsync(outs[b], sizeof(float) * ranks[b], M + row_base[i] * ld, sizeof(float) * ld,
                             sizeof(float) * ranks[b], In, hipMemcpyDeviceToDevice, s) != hipSuccess)
            st = hip_fail(hipGetLastError(), "mttkrp_batched: output copy");
    }
    // released in stream order after the kernels above: no synchronisation
    ws.release(s);
    dev_free(d_items, s);
    dev_free(M, s);
    return st;
}

spt_status spt_cp_als_batched(const spt_tensor *ts, int count, const int *ranks, int max_iters, double tol,
                              float *const *const *factors, double *const *lambdas, double *fits, int *iters,
                              void *stream) {
    if (count < 0 || (count > 0 && (!ts || !ranks || !factors || !lambdas || !fits || !iters)))
        return fail(SPT_E_INVALID_ARG, "cp_als_batched: NULL argument");
    if (max_iters < 0) return fail(SPT_E_INVALID_ARG, "cp_als_batched: max_iters < 0");
    hipStream_t s = (hipStream_t)stream;
    std::vector<Member> mem(count);
    // the iterations run on copies of the factors and lambdas: the caller's
    // buffers are written only when every member succeeded
    std::vector<void *> owned;
    auto release_owned = [&]() {
        for (void *p : owned) dev_free(p, s);
        owned.clear();
    };
    spt_status st = SPT_OK;
    {
        BatchEngine eng(s);
        for (int b = 0; b < count && st == SPT_OK; ++b) {
            Member &m = mem[b];
            if (!ts[b] || !factors[b] || !lambdas[b]) {
                st = fail(SPT_E_INVALID_ARG, "cp_als_batched: NULL member " + std::to_string(b));
                break;
            }
            m.t = ts[b];
            m.R = ranks[b];
            if (m.R < 1 || m.R > SPT_MAX_ALS_RANK) {
                st = fail(SPT_E_INVALID_ARG, "cp_als_batched: rank must be 1..64");
                break;
            }
            st = check_factors(m.t, (const float *const *)factors[b], m.R, -1);
            for (int k = 0; k < m.t->nmodes && st == SPT_OK; ++k) {
                const size_t bytes = sizeof(float) * (size_t)m.t->dims[k] * m.R;
                m.F[k] = (float *)dev_alloc(bytes, s);
                if (!m.F[k]) st = fail(SPT_E_OOM, "cp_als_batched: factor copies");
                else {
                    owned.push_back(m.F[k]);
                    if (hipMemcpyAsync(m.F[k], factors[b][k], bytes, hipMemcpyDeviceToDevice, s) != hipSuccess)
                        st = hip_fail(hipGetLastError(), "cp_als_batched: factor copy");
                }
            }
            if (st != SPT_OK) break;
            m.lambda = (double *)dev_alloc(sizeof(double) * m.R, s);
            if (!m.lambda) {
                st = fail(SPT_E_OOM, "cp_als_batched: lambda");
                break;
            }
            owned.push_back(m.lambda);
            m.max_iters = max_iters;
            m.tol = tol;
            st = eng.add(&m);
            if (st == SPT_OK && max_iters == 0) m.done = true;
        }
        while (st == SPT_OK && eng.any_active()) {
            st = eng.step();
            for (int b = 0; st == SPT_OK && b < count; ++b)
                if (mem[b].err != SPT_OK) st = mem[b].err;
        }
        for (int b = 0; st == SPT_OK && b < count; ++b) {
            for (int k = 0; k < mem[b].t->nmodes && st == SPT_OK; ++k)
                if (hipMemcpyAsync(factors[b][k], mem[b].F[k], sizeof(float) * (size_t)mem[b].t->dims[k] * mem[b].R,
                                   hipMemcpyDeviceToDevice, s) != hipSuccess)
                    st = hip_fail(hipGetLastError(), "cp_als_batched: factor copy back");
            if (st == SPT_OK && max_iters > 0 &&
                hipMemcpyAsync(lambdas[b], mem[b].lambda, sizeof(double) * mem[b].R, hipMemcpyDeviceToDevice, s) !=
                    hipSuccess)
                st = hip_fail(hipGetLastError(), "cp_als_batched: lambda copy back");
        }
    }  // the engine releases its buffers in stream order here
    release_owned();
    if (st != SPT_OK) return st;
    for (int b = 0; b < count; ++b) {
        fits[b] = mem[b].fit;
        iters[b] = mem[b].iters;
    }
    return SPT_OK;
}

}  // extern "C"
