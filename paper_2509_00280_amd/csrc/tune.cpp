// Autotuner: a measured search over the encoding of one tensor and the
// per-mode MTTKRP plan.
//
// The search space is the paper's (Section III-C, Eq. (1)): one bit layout per
// tensor, i.e. an interleaving in which mode n fills exactly l(n) key bits,
// low bits of each coordinate first.  The paper learns the layout with a
// reinforcement-learning agent; here a hill climb seeded at the default
// (ALTO) interleaving replaces the agent: a move exchanges two adjacent key
// bits that come from different modes, which keeps every mode's bit count, so
// every candidate is a valid interleaving.  The objective is the measured
// all-mode MTTKRP time, each mode at its best plan (strategy and tile).
// Measurements are cached per (mode lengths, nnz, rank, layout).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
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
    bool operator<(const CacheKey &o) const {
        return std::tie(dims, nnz, rank, layout) < std::tie(o.dims, o.nnz, o.rank, o.layout);
    }
};

struct CacheEntry {
    spt_plan plan;
    double ms;
};

std::mutex g_cache_mu;
std::map<CacheKey, CacheEntry> g_cache;

CacheKey key_of(const Tensor *t, int rank) {
    CacheKey k;
    k.dims.assign(t->dims, t->dims + t->nmodes);
    k.nnz = t->nnz;
    k.rank = rank;
    k.layout.assign(t->layout, t->layout + t->lp);
    return k;
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ms per call of mode-`mode` MTTKRP under the tensor's current plan: one call
// to plan and warm up, then `reps` calls between two events.
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
// all-mode time.  Leaves t->plan at the winner.
spt_status tune_plan(Tensor *t, const float *const *F, int R, float *out, hipStream_t s, spt_plan *best_plan,
                     double *best_ms) {
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_cache.find(key_of(t, R));
        if (it != g_cache.end()) {
            *best_plan = it->second.plan;
            *best_ms = it->second.ms;
            t->plan = *best_plan;
            release_plans(t);
            return SPT_OK;
        }
    }
    const int reps = t->nnz > 20'000'000 ? 2 : 4;
    spt_plan plan = t->plan;
    double total = 0.0;
    for (int n = 0; n < t->nmodes; ++n) {
        struct Cand {
            int strategy, tile;
        };
        std::vector<Cand> cands;
        for (int tile : {1024, 2048, 4096})
            if (seg_tile_ok(tile, t->nmodes)) cands.push_back({SPT_STRATEGY_SEGMENT, tile});
        if (priv_feasible(t, n, R)) cands.push_back({SPT_STRATEGY_PRIV, 2048});
        double best = 1e300;
        Cand win = cands.front();
        for (const Cand &c : cands) {
            t->plan.strategy[n] = c.strategy;
            t->plan.tile[n] = c.tile;
            release_mode_plan(t, n);
            double ms = 0.0;
            spt_status st = time_mode(t, F, R, n, out, reps, s, &ms);
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
        release_mode_plan(t, n);
        total += best;
    }
    *best_plan = plan;
    *best_ms = total;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache[key_of(t, R)] = CacheEntry{plan, total};
    return SPT_OK;
}

}  // namespace

}  // namespace spt

using namespace spt;

extern "C" {

spt_status spt_autotune(spt_tensor *tp, const float *const *factors, int rank, double budget_ms, double *best_ms_out,
                        void *stream) {
    if (!tp || !*tp || !best_ms_out) return fail(SPT_E_INVALID_ARG, "autotune: NULL argument");
    Tensor *t = *tp;
    if (rank < 1 || rank > SPT_MAX_RANK) return fail(SPT_E_INVALID_ARG, "autotune: rank out of range");
    spt_status st = check_factors(t, factors, rank, -1);
    if (st != SPT_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const double t_start = now_ms();
    int64_t maxI = 1;
    for (int n = 0; n < t->nmodes; ++n) maxI = std::max(maxI, t->dims[n]);
    float *out = nullptr;
    SPT_HIP(hipMalloc(&out, sizeof(float) * maxI * rank));
    uint32_t *coords = nullptr;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(s);
        if (out) (void)hipFree(out);
        if (coords) (void)hipFree(coords);
    };
    spt_plan best_plan{};
    double best = 0.0;
    st = tune_plan(t, factors, rank, out, s, &best_plan, &best);
    if (st != SPT_OK) {
        cleanup();
        return st;
    }
    std::vector<uint8_t> best_layout(t->layout, t->layout + t->lp);
    const int lp = t->lp;
    // layout moves need the coordinates: decode once (key order; the values are t->vals)
    bool moves = lp >= 2 && t->nnz > 0 && t->nmodes >= 2;
    if (moves && now_ms() - t_start < budget_ms) {
        if (hipMalloc(&coords, sizeof(uint32_t) * (size_t)t->nmodes * t->nnz) != hipSuccess) {
            (void)hipGetLastError();
            cleanup();
            return fail(SPT_E_OOM, "autotune: coordinate buffer");
        }
        st = launch_decode(t, coords, s);
        if (st != SPT_OK) {
            cleanup();
            return st;
        }
        std::mt19937_64 rng(0x5eed ^ (uint64_t)t->nnz ^ ((uint64_t)lp << 40));
        std::vector<uint8_t> cur = best_layout;
        int stale = 0;
        while (now_ms() - t_start < budget_ms && stale < 3) {
            // up to four distinct adjacent exchanges of the current layout
            std::vector<int> pos;
            for (int i = 0; i + 1 < lp; ++i)
                if (cur[i] != cur[i + 1]) pos.push_back(i);
            if (pos.empty()) break;
            std::shuffle(pos.begin(), pos.end(), rng);
            pos.resize(std::min<size_t>(pos.size(), 4));
            bool improved = false;
            std::vector<uint8_t> round_best;
            double round_ms = best;
            spt_plan round_plan{};
            for (int i : pos) {
                if (now_ms() - t_start >= budget_ms) break;
                std::vector<uint8_t> cand = cur;
                std::swap(cand[i], cand[i + 1]);
                spt_tensor c = nullptr;
                st = spt_encode(t->dims, t->nmodes, coords, t->vals, t->nnz, cand.data(), lp, s, &c);
                if (st != SPT_OK) {
                    cleanup();
                    return st;
                }
                spt_plan p{};
                double ms = 0.0;
                st = tune_plan(c, factors, rank, out, s, &p, &ms);
                spt_tensor_free(c);
                if (st != SPT_OK) {
                    cleanup();
                    return st;
                }
                if (ms < round_ms) {
                    round_ms = ms;
                    round_best = cand;
                    round_plan = p;
                }
            }
            if (!round_best.empty() && round_ms < 0.99 * best) {
                best = round_ms;
                best_layout = round_best;
                best_plan = round_plan;
                cur = round_best;
                improved = true;
            }
            stale = improved ? 0 : stale + 1;
        }
    }
    if (std::memcmp(best_layout.data(), t->layout, lp) != 0) {
        // re-encode in place with the winning layout; perm keeps naming the
        // caller's input order: perm_new = perm_old[perm_rel]
        spt_tensor c = nullptr;
        st = spt_encode(t->dims, t->nmodes, coords, t->vals, t->nnz, best_layout.data(), lp, s, &c);
        uint32_t *perm = nullptr;
        if (st == SPT_OK && hipMalloc(&perm, sizeof(uint32_t) * std::max<int64_t>(t->nnz, 1)) != hipSuccess) {
            (void)hipGetLastError();
            st = fail(SPT_E_OOM, "autotune: perm");
        }
        if (st == SPT_OK) st = launch_gather_u32(t->perm, c->perm, perm, t->nnz, s);
        if (st == SPT_OK && hipMemcpyAsync(c->perm, perm, sizeof(uint32_t) * t->nnz, hipMemcpyDeviceToDevice, s) != hipSuccess)
            st = hip_fail(hipGetLastError(), "autotune: perm copy");
        if (st == SPT_OK && hipStreamSynchronize(s) != hipSuccess) st = hip_fail(hipGetLastError(), "autotune: sync");
        if (perm) (void)hipFree(perm);
        if (st != SPT_OK) {
            if (c) spt_tensor_free(c);
            cleanup();
            return st;
        }
        release_plans(t);
        release_ws(t);
        std::swap(*static_cast<Tensor *>(t), *static_cast<Tensor *>(c));
        spt_tensor_free(c);  // the old encoding
    }
    t->plan = best_plan;
    release_plans(t);
    cleanup();
    *best_ms_out = best;
    return SPT_OK;
}

}  // extern "C"
