// Autotuner: a measured search over the encoding of one tensor and the
// per-mode MTTKRP plan.
//
// The search space is the paper's (Section III-C, Eq. (1)): one bit layout per
// tensor, i.e. an interleaving in which mode n fills exactly l(n) key bits,
// low bits of each coordinate first; Eq. (1) counts these interleavings as the
// multinomial coefficient l(p)! / prod_n l(n)!.  The reward is the paper's:
// the all-mode MTTKRP time of a layout relative to the default (ALTO)
// interleaving (Section III-C, reward function).  The paper learns the layout
// with a reinforcement-learning agent; here the agent is replaced by a
// measured search:
//   1. the layout the tensor has, and the ALTO layout (the reward baseline);
//   2. seeded uniform samples of the interleaving space (a uniformly shuffled
//      multiset of mode ids, which gives every distinct interleaving the same
//      probability);
//   3. a hill climb from the best layout so far: a move exchanges two
//      adjacent key bits of different modes, which keeps every mode's bit
//      count, so every candidate is a valid interleaving.
// A layout is measured with each mode at its best plan (strategy and tile).
// Measurements are cached per (mode lengths, nnz, rank, layout, content
// fingerprint), the fingerprint taken from the encoded tensor's first and last
// keys and values and its norm.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "spt_internal.h"

namespace spt {

spt_status check_factors(const Tensor *t, const float *const *factors, int rank, int skip_mode);

namespace {

struct CacheKey {
    std::vector<int64_t> dims;
    int64_t nnz;
    int rank;
    std::vector<uint8_t> layout;
    uint64_t fingerprint;
    bool operator<(const CacheKey &o) const {
        return std::tie(dims, nnz, rank, layout, fingerprint) <
               std::tie(o.dims, o.nnz, o.rank, o.layout, o.fingerprint);
    }
};

struct CacheEntry {
    spt_plan plan;
    double ms;
};

std::mutex g_cache_mu;
std::map<CacheKey, CacheEntry> g_cache;

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

uint64_t fnv1a(uint64_t h, const void *p, size_t n) {
    const unsigned char *b = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

// Content fingerprint of an encoded tensor: its first and last (up to) 512
// keys and values and its norm.  Two tensors of one shape and nnz but other
// nonzeros differ here with overwhelming probability.  Synchronises s.
spt_status fingerprint(const Tensor *t, hipStream_t s, uint64_t *out) {
    uint64_t h = 0xcbf29ce484222325ull;
    h = fnv1a(h, &t->norm_x2, sizeof(double));
    const int64_t k = std::min<int64_t>(t->nnz, 512);
    if (k > 0) {
        std::vector<uint64_t> keys(2 * k);
        std::vector<float> vals(2 * k);
        SPT_HIP(hipMemcpyAsync(keys.data(), t->lo, sizeof(uint64_t) * k, hipMemcpyDeviceToHost, s));
        SPT_HIP(hipMemcpyAsync(keys.data() + k, t->lo + (t->nnz - k), sizeof(uint64_t) * k, hipMemcpyDeviceToHost, s));
        SPT_HIP(hipMemcpyAsync(vals.data(), t->vals, sizeof(float) * k, hipMemcpyDeviceToHost, s));
        SPT_HIP(hipMemcpyAsync(vals.data() + k, t->vals + (t->nnz - k), sizeof(float) * k, hipMemcpyDeviceToHost, s));
        SPT_HIP(hipStreamSynchronize(s));
        h = fnv1a(h, keys.data(), sizeof(uint64_t) * keys.size());
        h = fnv1a(h, vals.data(), sizeof(float) * vals.size());
    }
    *out = h;
    return SPT_OK;
}

// ms per call of mode-`mode` MTTKRP under the tensor's current (prepared)
// plan: one warm-up call, then `reps` calls between two events.
spt_status time_mode(Tensor *t, const float *const *F, int R, int mode, float *out, int reps, hipStream_t s,
                     double *ms) {
    spt_status st = run_mttkrp(t, F, R, mode, out, s);
    if (st != SPT_OK) return st;
    hipEvent_t e0, e1;
    SPT_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(hipGetLastError(), "autotune: event");
    }
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps && st == SPT_OK; ++r) st = run_mttkrp(t, F, R, mode, out, s);
    (void)hipEventRecord(e1, s);
    float el = 0.f;
    if (st == SPT_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&el, e0, e1) != hipSuccess))
        st = hip_fail(hipGetLastError(), "autotune: timing");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = (double)el / reps;
    return st;
}

// Best plan of every mode for the tensor's current layout; returns the
// all-mode time.  Leaves t->plan at the winner (prepared).
spt_status tune_plan(Tensor *t, const float *const *F, int R, float *out, hipStream_t s, spt_plan *best_plan,
                     double *best_ms, bool *cached) {
    CacheKey key;
    key.dims.assign(t->dims, t->dims + t->nmodes);
    key.nnz = t->nnz;
    key.rank = R;
    key.layout.assign(t->layout, t->layout + t->lp);
    spt_status st = fingerprint(t, s, &key.fingerprint);
    if (st != SPT_OK) return st;
    *cached = false;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            *best_plan = it->second.plan;
            *best_ms = it->second.ms;
            *cached = true;
        }
    }
    if (*cached) {
        for (int n = 0; n < kMaxModes; ++n) release_mode_plan(t, n, s);
        t->plan = *best_plan;
        return prepare_single(t, R, s);
    }
    const int reps = t->nnz > 20'000'000 ? 3 : 5;
    // tile dictionaries for the row-cached candidates (built once per encoding)
    for (int n = 0; n < t->nmodes; ++n) {
        t->plan.strategy[n] = SPT_STRATEGY_SEGMENT;
        t->plan.tile[n] = 4096;
    }
    for (int n = 0; n < kMaxModes; ++n) release_mode_plan(t, n, s);
    st = prepare_single(t, R, s);
    if (st != SPT_OK) return st;
    spt_plan plan = t->plan;
    double total = 0.0;
    for (int n = 0; n < t->nmodes; ++n) {
        struct Cand {
            int strategy, tile;
        };
        std::vector<Cand> cands;
        for (int tile : {4096, 2048, 1024})
            if (seg_tile_ok(tile, t->nmodes)) cands.push_back({SPT_STRATEGY_SEGMENT, tile});
        if (priv_feasible(t, n, R)) cands.push_back({SPT_STRATEGY_PRIV, 2048});
        double best = 1e300;
        Cand win = cands.front();
        for (const Cand &c : cands) {
            t->plan.strategy[n] = c.strategy;
            t->plan.tile[n] = c.tile;
            ModePlan *p = nullptr;
            st = resolve_plan(t, n, R, s, &p, true);
            double ms = 0.0;
            if (st == SPT_OK) st = time_mode(t, F, R, n, out, reps, s, &ms);
            if (st != SPT_OK) return st;
            if (ms < best) {
                best = ms;
                win = c;
            }
        }
        plan.strategy[n] = win.strategy;
        plan.tile[n] = win.tile;
        t->plan.strategy[n] = win.strategy;
        t->plan.tile[n] = win.tile;
        ModePlan *p = nullptr;
        st = resolve_plan(t, n, R, s, &p, true);
        if (st != SPT_OK) return st;
        total += best;
    }
    *best_plan = plan;
    *best_ms = total;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache[key] = CacheEntry{plan, total};
    return SPT_OK;
}

}  // namespace

}  // namespace spt

using namespace spt;

extern "C" {

spt_status spt_autotune(spt_tensor *tp, const float *const *factors, int rank, double budget_ms, int random_samples,
                        uint64_t seed, spt_tune_result *res, void *stream) {
    if (!tp || !*tp || !res) return fail(SPT_E_INVALID_ARG, "autotune: NULL argument");
    Tensor *t = *tp;
    if (rank < 1 || rank > SPT_MAX_RANK) return fail(SPT_E_INVALID_ARG, "autotune: rank out of range");
    if (random_samples < 0) return fail(SPT_E_INVALID_ARG, "autotune: random_samples < 0");
    spt_status st = check_factors(t, factors, rank, -1);
    if (st != SPT_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const double t_start = now_ms();
    int64_t maxI = 1;
    for (int n = 0; n < t->nmodes; ++n) maxI = std::max(maxI, t->dims[n]);
    const int lp = t->lp;
    float *out = (float *)dev_alloc(sizeof(float) * maxI * rank, s);
    uint32_t *coords = nullptr;
    auto cleanup = [&]() {
        dev_free(out, s);
        dev_free(coords, s);
    };
    if (!out) return fail(SPT_E_OOM, "autotune: output buffer");
    spt_tune_result r{};
    // candidates other than the tensor's own layout are encoded from its
    // decoded coordinates (key order) and its values
    auto measure = [&](const std::vector<uint8_t> &lay, spt_plan *plan, double *ms) -> spt_status {
        bool cached = false;
        if (std::memcmp(lay.data(), t->layout, lp) == 0) {
            st = tune_plan(t, factors, rank, out, s, plan, ms, &cached);
        } else {
            if (!coords) {
                coords = (uint32_t *)dev_alloc(sizeof(uint32_t) * (size_t)t->nmodes * std::max<int64_t>(t->nnz, 1), s);
                if (!coords) return fail(SPT_E_OOM, "autotune: coordinate buffer");
                spt_status d = launch_decode(t, coords, s);
                if (d != SPT_OK) return d;
            }
            spt_tensor c = nullptr;
            st = spt_encode(t->dims, t->nmodes, coords, t->vals, t->nnz, lay.data(), lp, s, &c);
            if (st != SPT_OK) return st;
            st = tune_plan(c, factors, rank, out, s, plan, ms, &cached);
            tensor_release(c, s);
        }
        ++r.candidates;
        r.cache_hits += cached ? 1 : 0;
        return st;
    };
    std::vector<uint8_t> start(t->layout, t->layout + lp), alto(lp);
    default_layout(t->nmodes, t->lbits, alto.data());
    spt_plan best_plan{}, p{};
    double best = 0.0, ms = 0.0;
    st = measure(start, &best_plan, &best);
    if (st != SPT_OK) {
        cleanup();
        return st;
    }
    std::vector<uint8_t> best_layout = start;
    r.start_ms = best;
    r.alto_ms = best;
    auto consider = [&](const std::vector<uint8_t> &lay) -> spt_status {
        spt_status e = measure(lay, &p, &ms);
        if (e != SPT_OK) return e;
        if (ms < best) {
            best = ms;
            best_layout = lay;
            best_plan = p;
        }
        return SPT_OK;
    };
    if (alto != start) {
        st = measure(alto, &p, &ms);
        if (st == SPT_OK) {
            r.alto_ms = ms;
            if (ms < best) {
                best = ms;
                best_layout = alto;
                best_plan = p;
            }
        }
    }
    const bool moves = lp >= 2 && t->nnz > 0 && t->nmodes >= 2;
    std::mt19937_64 rng(seed);
    // uniform samples of the interleaving space
    for (int i = 0; st == SPT_OK && moves && i < random_samples && now_ms() - t_start < budget_ms; ++i) {
        std::vector<uint8_t> lay = start;
        std::shuffle(lay.begin(), lay.end(), rng);
        ++r.random_samples;
        st = consider(lay);
    }
    // hill climb from the best layout so far
    int stale = 0;
    std::vector<uint8_t> cur = best_layout;
    while (st == SPT_OK && moves && now_ms() - t_start < budget_ms && stale < 3) {
        std::vector<int> pos;
        for (int i = 0; i + 1 < lp; ++i)
            if (cur[i] != cur[i + 1]) pos.push_back(i);
        if (pos.empty()) break;
        std::shuffle(pos.begin(), pos.end(), rng);
        pos.resize(std::min<size_t>(pos.size(), 4));
        const double before = best;
        for (int i : pos) {
            if (now_ms() - t_start >= budget_ms) break;
            std::vector<uint8_t> cand = cur;
            std::swap(cand[i], cand[i + 1]);
            st = consider(cand);
            if (st != SPT_OK) break;
        }
        if (best < 0.99 * before) {
            cur = best_layout;
            stale = 0;
        } else {
            ++stale;
        }
    }
    if (st == SPT_OK && std::memcmp(best_layout.data(), t->layout, lp) != 0) {
        // re-encode in place with the winning layout; perm keeps naming the
        // caller's input order: perm_new = perm_old[perm_rel]
        spt_tensor c = nullptr;
        st = spt_encode(t->dims, t->nmodes, coords, t->vals, t->nnz, best_layout.data(), lp, s, &c);
        uint32_t *perm = nullptr;
        if (st == SPT_OK && !(perm = (uint32_t *)dev_alloc(sizeof(uint32_t) * std::max<int64_t>(t->nnz, 1), s)))
            st = fail(SPT_E_OOM, "autotune: perm");
        // FP64 values follow the new key order (c->perm is still relative to t's order)
        if (st == SPT_OK && t->vals64) {
            c->vals64 = (double *)dev_alloc(sizeof(double) * std::max<int64_t>(t->nnz, 1), s);
            st = c->vals64 ? launch_gather_f64(t->vals64, c->perm, c->vals64, t->nnz, s)
                           : fail(SPT_E_OOM, "autotune: FP64 values");
        }
        if (st == SPT_OK) st = launch_gather_u32(t->perm, c->perm, perm, t->nnz, s);
        if (st == SPT_OK && hipMemcpyAsync(c->perm, perm, sizeof(uint32_t) * t->nnz, hipMemcpyDeviceToDevice, s) != hipSuccess)
            st = hip_fail(hipGetLastError(), "autotune: perm copy");
        dev_free(perm, s);
        if (st == SPT_OK) {
            std::swap(*static_cast<Tensor *>(t), *static_cast<Tensor *>(c));
            tensor_release(c, s);  // the old encoding, after the copies above
        } else if (c) {
            tensor_release(c, s);
        }
    }
    if (st == SPT_OK) {
        for (int n = 0; n < kMaxModes; ++n) release_mode_plan(t, n, s);
        t->plan = best_plan;
        st = prepare_single(t, rank, s);  // the winner is left prepared
    }
    cleanup();
    if (st != SPT_OK) return st;
    r.best_ms = best;
    *res = r;
    return SPT_OK;
}

// Batches: the members' layouts (each by the search above, with its own
// factors and rank, under the same reward) and then the batch's tile, by
// timing the all-mode batched MTTKRP at every tile that fits.
spt_status spt_autotune_batched(spt_tensor *ts, int count, const float *const *const *factors, const int *ranks,
                                double layout_budget_ms, int random_samples, uint64_t seed,
                                spt_batch_tune_result *result, void *stream) {
    if (count < 1 || !ts || !factors || !ranks || !result) return fail(SPT_E_INVALID_ARG, "autotune_batched: NULL argument");
    const hipStream_t s = (hipStream_t)stream;
    int nmax = 0;
    for (int b = 0; b < count; ++b) {
        if (!ts[b] || !factors[b]) return fail(SPT_E_INVALID_ARG, "autotune_batched: NULL member " + std::to_string(b));
        if (ranks[b] < 1 || ranks[b] > 64) return fail(SPT_E_INVALID_ARG, "autotune_batched: rank must be 1..64");
        spt_status st = check_factors(ts[b], factors[b], ranks[b], -1);
        if (st != SPT_OK) return st;
        nmax = std::max(nmax, ts[b]->nmodes);
    }
    spt_batch_tune_result r{};
    double log_gain = 0.0;
    if (layout_budget_ms > 0.0) {
        for (int b = 0; b < count; ++b) {
            spt_tune_result tr{};
            spt_status st = spt_autotune(&ts[b], factors[b], ranks[b], layout_budget_ms, random_samples, seed + (uint64_t)b,
                                         &tr, stream);
            if (st != SPT_OK) return st;
            ++r.layouts_tuned;
            if (tr.best_ms > 0.0 && tr.start_ms > 0.0) log_gain += std::log(tr.start_ms / tr.best_ms);
        }
    }
    r.layout_speedup = r.layouts_tuned ? std::exp(log_gain / r.layouts_tuned) : 1.0;
    // one output buffer per member, as large as its largest mode
    std::vector<float *> outs(count, nullptr);
    spt_status st = SPT_OK;
    for (int b = 0; b < count && st == SPT_OK; ++b) {
        int64_t rows = 1;
        for (int n = 0; n < ts[b]->nmodes; ++n) rows = std::max(rows, ts[b]->dims[n]);
        outs[b] = (float *)dev_alloc(sizeof(float) * (size_t)rows * ranks[b], s);
        if (!outs[b]) st = fail(SPT_E_OOM, "autotune_batched: outputs");
    }
    std::vector<Tensor *> tv(ts, ts + count);
    const int tiles[3] = {1024, 2048, 4096};
    auto all_modes = [&]() -> spt_status {
        for (int n = 0; n < nmax; ++n) {
            spt_status e = spt_mttkrp_batched(ts, count, factors, ranks, n, outs.data(), stream);
            if (e != SPT_OK) return e;
        }
        return SPT_OK;
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (st == SPT_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        st = hip_fail(hipGetLastError(), "autotune_batched: events");
    double best = 0.0;
    int best_tile = 0;
    for (int i = 0; i < 3 && st == SPT_OK; ++i) {
        const int T = tiles[i];
        r.ms[i] = 0.0;
        if (!seg_batch_fits(nmax, T)) continue;
        for (Tensor *t : tv) t->plan.batch_tile = T;
        for (int n = 0; n < nmax && st == SPT_OK; ++n) st = ensure_batch_plans(tv, n, T, s);
        if (st == SPT_OK) st = all_modes();  // warm-up
        constexpr int kReps = 3;
        if (st == SPT_OK && hipEventRecord(e0, s) != hipSuccess) st = hip_fail(hipGetLastError(), "autotune_batched: event");
        for (int k = 0; k < kReps && st == SPT_OK; ++k) st = all_modes();
        float el = 0.f;
        if (st == SPT_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&el, e0, e1) != hipSuccess))
            st = hip_fail(hipGetLastError(), "autotune_batched: timing");
        if (st != SPT_OK) break;
        r.ms[i] = el / kReps;
        if (best_tile == 0 || r.ms[i] < best) {
            best = r.ms[i];
            best_tile = T;
        }
    }
    if (st == SPT_OK && best_tile == 0) st = fail(SPT_E_INVALID_ARG, "autotune_batched: no batched tile fits");
    if (st == SPT_OK) {
        for (Tensor *t : tv) t->plan.batch_tile = best_tile;
        for (int n = 0; n < nmax && st == SPT_OK; ++n) st = ensure_batch_plans(tv, n, best_tile, s);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    for (float *o : outs) dev_free(o, s);
    if (st != SPT_OK) return st;
    r.best_tile = best_tile;
    *result = r;
    return SPT_OK;
}

}  // extern "C"
