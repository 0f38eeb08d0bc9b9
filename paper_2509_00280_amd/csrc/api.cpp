// Host runtime of the C-ABI: argument checks, the coordinate<->key codec, the
// encoded-tensor handle, MTTKRP dispatch and the CP-ALS driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "spt_internal.h"

namespace spt {

// ---------------------------------------------------------------- errors
static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

spt_status fail(spt_status st, const std::string &msg) {
    set_error(msg);
    return st;
}

spt_status hip_fail(hipError_t e, const char *what) {
    const spt_status st = (e == hipErrorOutOfMemory) ? SPT_E_OOM : SPT_E_DEVICE;
    return fail(st, std::string("HIP error ") + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ") in " + what);
}

// ---------------------------------------------------------------- device memory
// Every device buffer the library owns comes from dev_alloc and goes back
// through dev_free on a stream, in stream order: a buffer released on stream
// s may be reused by work ordered after that point of s, so releasing never
// waits for the device.  spt_set_allocator can replace the source, e.g. with
// PyTorch's caching allocator; the default is the block cache below.
static std::atomic<spt_alloc_fn> g_alloc{nullptr};
static std::atomic<spt_release_fn> g_release{nullptr};
static std::atomic<void *> g_alloc_ctx{nullptr};

// Buffers taken from a hook remember the hook that releases them, so
// changing the hook never sends a buffer to the wrong allocator.
struct HookOwner {
    spt_release_fn release;
    void *ctx;
};
static std::mutex g_owner_mu;
static std::unordered_map<void *, HookOwner> g_owner;

// Default source: a cache of device blocks per device.  A block comes from
// hipMalloc once and stays with the library after release.  A block released
// on stream s serves a later request on s at once (stream order makes that
// safe); a request on another stream takes it only once the event recorded
// at its release has completed.  hipMalloc runs only when no idle block fits;
// when it fails, the idle blocks of that device are returned to the driver
// (after their release events) and the request is tried once more.  The
// runtime's stream-ordered pool is not used: once many different sizes had
// passed through it (a layout search), single hipMallocAsync and hipFreeAsync
// calls were measured holding the host for 0.15 s to 2.7 s with the GPU idle.
namespace {
constexpr size_t kLargeGrain = size_t(1) << 21;  // 2 MiB: large requests round up to this
constexpr int kMaxDevices = 64;
constexpr int kMaxProbe = 32;  // idle blocks examined per request

struct Block {
    size_t bytes = 0;
    int dev = 0;
    hipStream_t stream = nullptr;  // stream of the last release
    hipEvent_t ev = nullptr;       // recorded at the last release; nullptr: no work pending
};

struct BlockCache {
    std::mutex mu;
    std::unordered_map<void *, Block> live;
    std::multimap<size_t, std::pair<void *, Block>> idle[kMaxDevices];
    int64_t bytes_live = 0, bytes_idle = 0, device_allocs = 0, reuses = 0;
};

// Never destroyed: blocks may still be released while the process exits.
BlockCache &cache() {
    static BlockCache *c = new BlockCache;
    return *c;
}

size_t cache_size(size_t bytes) {
    if (bytes >= kLargeGrain) return (bytes + kLargeGrain - 1) & ~(kLargeGrain - 1);
    size_t b = 512;
    while (b < bytes) b <<= 1;
    return b;
}

// Largest idle block a request of `need` bytes may take.
size_t cache_limit(size_t need) { return need < kLargeGrain ? need : need + need / 8 + kLargeGrain; }

// Returns the idle blocks of `dev` to the driver (caller holds the lock).
void release_idle(BlockCache &c, int dev) {
    for (auto &kv : c.idle[dev]) {
        Block &b = kv.second.second;
        if (b.ev) {
            (void)hipEventSynchronize(b.ev);
            (void)hipEventDestroy(b.ev);
        }
        (void)hipFree(kv.second.first);
        c.bytes_idle -= (int64_t)b.bytes;
    }
    c.idle[dev].clear();
}

void *cache_alloc(size_t bytes, hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return nullptr;
    }
    const size_t need = cache_size(bytes);
    BlockCache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto &idle = c.idle[dev];
    int probed = 0;
    for (auto it = idle.lower_bound(need); it != idle.end() && it->first <= cache_limit(need) && probed < kMaxProbe;
         ++it, ++probed) {
        Block &b = it->second.second;
        bool ready = b.ev == nullptr || b.stream == s;
        if (!ready) {
            const hipError_t q = hipEventQuery(b.ev);
            if (q != hipSuccess && q != hipErrorNotReady) (void)hipGetLastError();
            ready = q == hipSuccess;
        }
        if (!ready) continue;
        void *p = it->second.first;
        Block blk = b;
        idle.erase(it);
        c.bytes_idle -= (int64_t)blk.bytes;
        c.bytes_live += (int64_t)blk.bytes;
        ++c.reuses;
        c.live[p] = blk;
        return p;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, need);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        release_idle(c, dev);
        e = hipMalloc(&p, need);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    Block blk;
    blk.bytes = need;
    blk.dev = dev;
    c.live[p] = blk;
    c.bytes_live += (int64_t)need;
    ++c.device_allocs;
    return p;
}

bool cache_free(void *p, hipStream_t s) {
    BlockCache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.live.find(p);
    if (it == c.live.end()) return false;
    Block b = it->second;
    c.live.erase(it);
    b.stream = s;
    int cur = -1;
    (void)hipGetDevice(&cur);
    bool recorded = false;
    if (cur == b.dev) {
        if (!b.ev && hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) != hipSuccess) b.ev = nullptr;
        recorded = b.ev && hipEventRecord(b.ev, s) == hipSuccess;
    }
    if (!recorded) {  // no event: wait here so that every stream may take the block
        (void)hipGetLastError();
        (void)hipStreamSynchronize(s);
        if (b.ev) (void)hipEventDestroy(b.ev);
        b.ev = nullptr;
    }
    c.bytes_live -= (int64_t)b.bytes;
    c.bytes_idle += (int64_t)b.bytes;
    c.idle[b.dev].emplace(b.bytes, std::make_pair(p, b));
    return true;
}
}  // namespace

void *dev_alloc(size_t bytes, hipStream_t s) {
    if (bytes == 0) bytes = 16;
    bytes = (bytes + 255) & ~size_t(255);
    if (spt_alloc_fn f = g_alloc.load()) {
        void *ctx = g_alloc_ctx.load();
        const spt_release_fn rel = g_release.load();
        void *p = f(bytes, (void *)s, ctx);
        if (!p) return nullptr;
        if ((uintptr_t)p & 255u) {  // the kernels assume 256-byte alignment
            rel(p, (void *)s, ctx);
            return nullptr;
        }
        std::lock_guard<std::mutex> lk(g_owner_mu);
        g_owner[p] = HookOwner{rel, ctx};
        return p;
    }
    return cache_alloc(bytes, s);
}

void dev_free(void *p, hipStream_t s) {
    if (!p) return;
    HookOwner o{nullptr, nullptr};
    {
        std::lock_guard<std::mutex> lk(g_owner_mu);
        auto it = g_owner.find(p);
        if (it != g_owner.end()) {
            o = it->second;
            g_owner.erase(it);
        }
    }
    if (o.release) {
        o.release(p, (void *)s, o.ctx);
        return;
    }
    (void)cache_free(p, s);
}

spt_status memory_stats(int64_t *stats) {
    BlockCache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    stats[0] = c.bytes_live;
    stats[1] = c.bytes_idle;
    stats[2] = c.device_allocs;
    stats[3] = c.reuses;
    return SPT_OK;
}

spt_status empty_cache() {
    BlockCache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return hip_fail(hipGetLastError(), "empty_cache");
    for (int d = 0; d < kMaxDevices; ++d) {
        if (c.idle[d].empty()) continue;
        if (hipSetDevice(d) != hipSuccess) return hip_fail(hipGetLastError(), "empty_cache: set device");
        release_idle(c, d);
    }
    if (hipSetDevice(cur) != hipSuccess) return hip_fail(hipGetLastError(), "empty_cache: restore device");
    return SPT_OK;
}

// ---------------------------------------------------------------- codec
void make_codec(int nmodes, const int *lbits, const uint8_t *layout, int lp, Codec *c) {
    std::memset(c, 0, sizeof(*c));
    c->nmodes = nmodes;
    c->key_words = lp > 64 ? 2 : 1;
    int nr = 0;
    for (int n = 0; n < nmodes; ++n) {
        std::vector<int> pos;  // pos[j] = key bit that holds coordinate bit j
        for (int t = 0; t < lp; ++t)
            if (layout[t] == n) pos.push_back(t);
        const int start = nr;
        int j = 0;
        while (j < (int)pos.size()) {
            const int kp = pos[j];
            int len = 1;
            while (len < 31 && j + len < (int)pos.size() && pos[j + len] == kp + len && (kp + len) / 32 == kp / 32)
                ++len;
            c->run[nr++] = pack_run(kp / 32, kp % 32, j, len);
            j += len;
        }
        const int end = nr;
        for (int w = 0; w <= 4; ++w) {
            int r = start;
            while (r < end && (int)(c->run[r] & 0xFFu) < w) ++r;
            c->rb[n][w] = (uint8_t)(w == 4 ? end : r);
        }
        (void)lbits;
    }
    for (int n = nmodes; n < kMaxModes; ++n)
        for (int w = 0; w <= 4; ++w) c->rb[n][w] = (uint8_t)nr;
    c->nruns = nr;
}

static int bit_length(int64_t d) {  // ceil(log2 d) for d >= 1
    int b = 0;
    while ((int64_t(1) << b) < d) ++b;
    return b;
}

// The default (ALTO) interleaving: level by level, modes of shorter bit
// length first, equal lengths in mode order (Section III-C: partitioning the
// longest mode first is interleaving from the shortest mode).
void default_layout(int nmodes, const int *lbits, uint8_t *layout) {
    int order[kMaxModes];
    for (int n = 0; n < nmodes; ++n) order[n] = n;
    std::stable_sort(order, order + nmodes, [&](int a, int b) { return lbits[a] < lbits[b]; });
    int maxb = 0;
    for (int n = 0; n < nmodes; ++n) maxb = std::max(maxb, lbits[n]);
    int pos = 0;
    for (int j = 0; j < maxb; ++j)
        for (int i = 0; i < nmodes; ++i)
            if (j < lbits[order[i]]) layout[pos++] = (uint8_t)order[i];
}

static void default_plan(const Tensor *t, spt_plan *p) {
    for (int n = 0; n < kMaxModes; ++n) {
        p->tile[n] = 4096;
        p->strategy[n] = SPT_STRATEGY_AUTO;
    }
    p->row_cache = 1;
    p->batch_tile = kBatchTileDefault;
    (void)t;
}

static bool plan_ok(const spt_plan *p, int nmodes) {
    for (int n = 0; n < nmodes; ++n) {
        const int T = p->tile[n];
        if (T != 256 && T != 512 && T != 1024 && T != 2048 && T != 4096) return false;
        if (p->strategy[n] < SPT_STRATEGY_DIRECT || p->strategy[n] > SPT_STRATEGY_SEGMENT) return false;
    }
    const int b = p->batch_tile;
    if (b != 0 && b != 1024 && b != 2048 && b != 4096) return false;
    return p->row_cache == 0 || p->row_cache == 1;
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

MttkrpArgs make_args(const Tensor *t, const float *const *factors, int rank, int mode, float *out, int tile) {
    MttkrpArgs a{};
    a.lo = t->lo;
    a.hi = t->hi;
    a.vals = t->vals;
    a.nnz = t->nnz;
    a.nmodes = t->nmodes;
    a.mode = mode;
    a.rank = rank;
    a.tile = tile;
    for (int k = 0; k < t->nmodes; ++k) {
        a.f[k] = factors ? factors[k] : nullptr;
        a.frows[k] = (uint32_t)std::min<int64_t>(t->dims[k], 0xFFFFFFFFll);
    }
    a.out = out;
    a.codec = t->codec;
    return a;
}

spt_status check_factors(const Tensor *t, const float *const *factors, int rank, int skip_mode) {
    if (!factors) return fail(SPT_E_INVALID_ARG, "factors is NULL");
    for (int k = 0; k < t->nmodes; ++k) {
        if (k == skip_mode) continue;
        if (!factors[k]) return fail(SPT_E_INVALID_ARG, "factor " + std::to_string(k) + " is NULL");
        if (!aligned16(factors[k])) return fail(SPT_E_INVALID_ARG, "factor " + std::to_string(k) + " not 16-byte aligned");
    }
    (void)rank;
    return SPT_OK;
}

}  // namespace spt

using namespace spt;

extern "C" {

const char *spt_last_error(void) { return g_last_error.c_str(); }

const char *spt_version(void) { return "spt-gfx950 0.1"; }

spt_status spt_set_allocator(spt_alloc_fn alloc, spt_release_fn release, void *ctx) {
    if ((alloc == nullptr) != (release == nullptr)) return fail(SPT_E_INVALID_ARG, "set_allocator: give both hooks or neither");
    g_alloc_ctx.store(ctx);
    g_release.store(release);
    g_alloc.store(alloc);
    return SPT_OK;
}

spt_status spt_memory_stats(int64_t *stats) {
    if (!stats) return fail(SPT_E_INVALID_ARG, "memory_stats: NULL output");
    return memory_stats(stats);
}

spt_status spt_empty_cache(void) { return empty_cache(); }

spt_status spt_profile_enable(int on) { return profile_enable(on); }

spt_status spt_profile_read(double *ms, int64_t *launches) {
    if (!ms || !launches) return fail(SPT_E_INVALID_ARG, "NULL output");
    return profile_read(ms, launches);
}

spt_status spt_encode(const int64_t *dims, int nmodes, const uint32_t *coords, const float *vals, int64_t nnz,
                      const uint8_t *layout, int layout_len, void *stream, spt_tensor *out) {
    if (!dims || !out) return fail(SPT_E_INVALID_ARG, "dims/out is NULL");
    if (nmodes < 1 || nmodes > kMaxModes) return fail(SPT_E_INVALID_ARG, "nmodes must be in 1..8");
    if (nnz < 0 || nnz >= (int64_t(1) << 32)) return fail(SPT_E_INVALID_ARG, "nnz must be in [0, 2^32)");
    if (nnz > 0 && (!coords || !vals)) return fail(SPT_E_INVALID_ARG, "coords/vals is NULL");
    hipStream_t s = (hipStream_t)stream;
    spt_tensor_s *t = new (std::nothrow) spt_tensor_s();
    if (!t) return fail(SPT_E_OOM, "host allocation failed");
    t->nmodes = nmodes;
    t->nnz = nnz;
    int lp = 0;
    for (int n = 0; n < nmodes; ++n) {
        if (dims[n] < 1 || dims[n] > 0xFFFFFFFELL) {
            delete t;
            return fail(SPT_E_INVALID_ARG, "mode length must be in 1..2^32-2");
        }
        t->dims[n] = dims[n];
        t->lbits[n] = bit_length(dims[n]);
        lp += t->lbits[n];
    }
    if (lp > SPT_MAX_KEY_BITS) {
        delete t;
        return fail(SPT_E_TOO_MANY_BITS, "l(p) = " + std::to_string(lp) + " exceeds 128 bits");
    }
    t->lp = lp;
    t->key_words = lp > 64 ? 2 : 1;
    if (layout) {
        if (layout_len != lp) {
            delete t;
            return fail(SPT_E_BAD_LAYOUT, "layout length " + std::to_string(layout_len) + " != l(p) " + std::to_string(lp));
        }
        int cnt[kMaxModes] = {};
        for (int i = 0; i < lp; ++i) {
            if (layout[i] >= nmodes) {
                delete t;
                return fail(SPT_E_BAD_LAYOUT, "layout names a mode out of range");
            }
            ++cnt[layout[i]];
        }
        for (int n = 0; n < nmodes; ++n)
            if (cnt[n] != t->lbits[n]) {
                delete t;
                return fail(SPT_E_BAD_LAYOUT, "mode " + std::to_string(n) + " appears " + std::to_string(cnt[n]) +
                                                  " times, needs " + std::to_string(t->lbits[n]));
            }
        std::memcpy(t->layout, layout, lp);
    } else {
        default_layout(nmodes, t->lbits, t->layout);
    }
    make_codec(nmodes, t->lbits, t->layout, lp, &t->codec);
    default_plan(t, &t->plan);
    spt_status st = launch_encode(t, coords, vals, s);
    if (st != SPT_OK) {
        delete t;
        return st;
    }
    *out = t;
    return SPT_OK;
}

spt_status spt_tensor_get_info(spt_tensor t, spt_tensor_info *info) {
    if (!t || !info) return fail(SPT_E_INVALID_ARG, "NULL argument");
    std::memset(info, 0, sizeof(*info));
    info->nnz = t->nnz;
    info->nmodes = t->nmodes;
    info->lp = t->lp;
    info->key_words = t->key_words;
    for (int n = 0; n < t->nmodes; ++n) {
        info->dims[n] = t->dims[n];
        info->lbits[n] = t->lbits[n];
    }
    std::memcpy(info->layout, t->layout, t->lp);
    info->encoded_bytes = (size_t)t->nnz * (8 * t->key_words + 4);
    info->norm_x2 = t->norm_x2;
    return SPT_OK;
}

spt_status spt_tensor_export(spt_tensor t, uint64_t *keys, float *vals, uint32_t *perm, void *stream) {
    if (!t) return fail(SPT_E_INVALID_ARG, "NULL tensor");
    hipStream_t s = (hipStream_t)stream;
    if (t->nnz == 0) return SPT_OK;
    if (keys) {
        spt_status st = launch_export(t, keys, s);
        if (st != SPT_OK) return st;
    }
    if (vals) SPT_HIP(hipMemcpyAsync(vals, t->vals, sizeof(float) * t->nnz, hipMemcpyDeviceToDevice, s));
    if (perm) SPT_HIP(hipMemcpyAsync(perm, t->perm, sizeof(uint32_t) * t->nnz, hipMemcpyDeviceToDevice, s));
    return SPT_OK;
}

spt_status spt_tensor_decode(spt_tensor t, uint32_t *coords, void *stream) {
    if (!t || (!coords && t->nnz)) return fail(SPT_E_INVALID_ARG, "NULL argument");
    return launch_decode(t, coords, (hipStream_t)stream);
}

spt_status spt_tensor_get_plan(spt_tensor t, spt_plan *plan) {
    if (!t || !plan) return fail(SPT_E_INVALID_ARG, "NULL argument");
    *plan = t->plan;
    return SPT_OK;
}

spt_status spt_tensor_set_plan(spt_tensor t, const spt_plan *plan, void *stream) {
    if (!t || !plan) return fail(SPT_E_INVALID_ARG, "NULL argument");
    if (!plan_ok(plan, t->nmodes)) return fail(SPT_E_INVALID_ARG, "plan: tile must be 256..4096 (power of two), strategy 0..5, row_cache 0 or 1, batch_tile 0, 1024, 2048 or 4096");
    // the old plans may still be read by queued work: released in stream order
    const hipStream_t s = (hipStream_t)stream;
    for (int n = 0; n < kMaxModes; ++n) release_mode_plan(t, n, s);
    if (plan->row_cache != t->plan.row_cache) release_dict(t, s);
    t->plan = *plan;
    return SPT_OK;
}

spt_status spt_tensor_prepare(spt_tensor t, int rank, int what, void *stream) {
    if (!t) return fail(SPT_E_INVALID_ARG, "NULL tensor");
    if (rank < 1 || rank > SPT_MAX_RANK) return fail(SPT_E_INVALID_ARG, "rank must be in 1..256");
    if (what & ~(SPT_PREPARE_SINGLE | SPT_PREPARE_BATCHED)) return fail(SPT_E_INVALID_ARG, "prepare: unknown flags");
    const hipStream_t s = (hipStream_t)stream;
    if (what & SPT_PREPARE_SINGLE) {
        spt_status st = prepare_single(t, rank, s);
        if (st != SPT_OK) return st;
    }
    if (what & SPT_PREPARE_BATCHED) {
        spt_status st = prepare_batched(t, s);
        if (st != SPT_OK) return st;
    }
    return SPT_OK;
}

}  // extern "C"

namespace spt {
// Release a handle after its last use on stream s: every buffer is freed in
// stream order, so nothing waits for the device.
void tensor_release(Tensor *t, hipStream_t s) {
    if (!t) return;
    release_plans(t, s);
    dev_free(t->lo, s);
    dev_free(t->hi, s);
    dev_free(t->vals, s);
    dev_free(t->vals64, s);
    dev_free(t->perm, s);
    delete static_cast<spt_tensor_s *>(t);
}
}  // namespace spt

extern "C" {

void spt_tensor_free(spt_tensor t, void *stream) { tensor_release(t, (hipStream_t)stream); }

spt_status spt_mttkrp(spt_tensor t, const float *const *factors, int rank, int mode, float *out, void *stream) {
    if (!t) return fail(SPT_E_INVALID_ARG, "NULL tensor");
    if (mode < 0 || mode >= t->nmodes) return fail(SPT_E_INVALID_ARG, "mode out of range");
    if (rank < 1 || rank > SPT_MAX_RANK) return fail(SPT_E_INVALID_ARG, "rank must be in 1..256");
    if (!out) return fail(SPT_E_INVALID_ARG, "out is NULL");
    if (!aligned16(out)) return fail(SPT_E_INVALID_ARG, "out not 16-byte aligned");
    spt_status st = check_factors(t, factors, rank, mode);
    if (st != SPT_OK) return st;
    return run_mttkrp(t, factors, rank, mode, out, (hipStream_t)stream);
}

spt_status spt_tensor_attach_f64(spt_tensor t, const double *vals, void *stream) {
    if (!t || (t->nnz > 0 && !vals)) return fail(SPT_E_INVALID_ARG, "attach_f64: NULL argument");
    if (t->nnz == 0) return SPT_OK;
    hipStream_t s = (hipStream_t)stream;
    double *v = (double *)dev_alloc(sizeof(double) * t->nnz, s);
    if (!v) return fail(SPT_E_OOM, "attach_f64: values");
    // key order: element j is the input element perm[j]
    spt_status st = launch_gather_f64(vals, t->perm, v, t->nnz, s);
    if (st != SPT_OK) {
        dev_free(v, s);
        return st;
    }
    dev_free(t->vals64, s);
    t->vals64 = v;
    return SPT_OK;
}

spt_status spt_mttkrp_f64(spt_tensor t, const double *const *factors, int rank, int mode, double *out, void *stream) {
    if (!t) return fail(SPT_E_INVALID_ARG, "NULL tensor");
    if (mode < 0 || mode >= t->nmodes) return fail(SPT_E_INVALID_ARG, "mode out of range");
    if (rank < 1 || rank > SPT_MAX_RANK) return fail(SPT_E_INVALID_ARG, "rank must be in 1..256");
    if (!out || !aligned16(out)) return fail(SPT_E_INVALID_ARG, "out is NULL or not 16-byte aligned");
    spt_status st = check_factors(t, (const float *const *)factors, rank, mode);
    if (st != SPT_OK) return st;
    return run_mttkrp_f64(t, factors, rank, mode, out, (hipStream_t)stream);
}

spt_status spt_mttkrp_noalloc(spt_tensor t, const float *const *factors, int rank, int mode, float *out,
                              void *stream) {
    if (!t) return fail(SPT_E_INVALID_ARG, "NULL tensor");
    if (mode < 0 || mode >= t->nmodes) return fail(SPT_E_INVALID_ARG, "mode out of range");
    if (rank < 1 || rank > SPT_MAX_RANK) return fail(SPT_E_INVALID_ARG, "rank must be in 1..256");
    if (!out) return fail(SPT_E_INVALID_ARG, "out is NULL");
    if (!aligned16(out)) return fail(SPT_E_INVALID_ARG, "out not 16-byte aligned");
    spt_status st = check_factors(t, factors, rank, mode);
    if (st != SPT_OK) return st;
    return run_mttkrp_noalloc(t, factors, rank, mode, out, (hipStream_t)stream);
}

spt_status spt_cp_als(spt_tensor t, int rank, int max_iters, double tol, float *const *factors, double *lambda,
                      double *fit_out, int *iters_out, void *stream) {
    if (!t) return fail(SPT_E_INVALID_ARG, "NULL tensor");
    if (rank < 1 || rank > SPT_MAX_ALS_RANK) return fail(SPT_E_INVALID_ARG, "rank must be in 1..64");
    if (max_iters < 0) return fail(SPT_E_INVALID_ARG, "max_iters < 0");
    if (!lambda || !fit_out || !iters_out) return fail(SPT_E_INVALID_ARG, "NULL output");
    if (!(t->norm_x2 > 0.0)) return fail(SPT_E_INVALID_ARG, "tensor norm is zero");
    spt_status st = check_factors(t, (const float *const *)factors, rank, -1);
    if (st != SPT_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    st = prepare_single(t, rank, s);
    if (st != SPT_OK) return st;
    const int N = t->nmodes;
    const int R = rank;
    int64_t maxI = 0;
    size_t gw = 0;
    for (int n = 0; n < N; ++n) {
        maxI = std::max(maxI, t->dims[n]);
        gw = std::max(gw, gram_work_bytes(t->dims[n], R));
    }
    const int inner_parts = apply_blocks(t->dims[N - 1], R);
    const int64_t resid_tiles = (t->nnz + 1023) / 1024;
    float *M = (float *)dev_alloc(sizeof(float) * maxI * R, s);
    double *grams = (double *)dev_alloc(sizeof(double) * N * R * R, s);
    double *gram_m = (double *)dev_alloc(sizeof(double) * R * R, s);
    double *S = (double *)dev_alloc(sizeof(double) * R * R, s);
    double *gwork = (double *)dev_alloc(gw, s);
    double *inner = (double *)dev_alloc(sizeof(double) * inner_parts, s);
    double *resid = (double *)dev_alloc(sizeof(double) * 2 * std::max<int64_t>(resid_tiles, 1), s);
    double *fitd = (double *)dev_alloc(sizeof(double) * 4 + sizeof(int) * kMaxModes, s);
    double *lam = (double *)dev_alloc(sizeof(double) * R, s);
    // one record workspace for every mode's MTTKRP (the largest plan's records)
    RecordWs ws;
    ws.records = std::max<int64_t>(max_plan_records(t), 1);
    ws.val_floats = ws.records * R;
    ws.row = (uint64_t *)dev_alloc(sizeof(uint64_t) * ws.records, s);
    ws.val = (float *)dev_alloc(sizeof(float) * ws.val_floats, s);
    // the iterations run on copies: the caller's factors and lambda are
    // written only when the call succeeds
    float *F[kMaxModes] = {};
    bool fok = true;
    for (int k = 0; k < N; ++k) fok = fok && (F[k] = (float *)dev_alloc(sizeof(float) * t->dims[k] * R, s)) != nullptr;
    auto cleanup = [&]() {
        dev_free(M, s); dev_free(grams, s); dev_free(gram_m, s); dev_free(S, s); dev_free(gwork, s);
        dev_free(inner, s); dev_free(resid, s); dev_free(fitd, s); dev_free(lam, s);
        dev_free(ws.row, s); dev_free(ws.val, s);
        for (int k = 0; k < N; ++k) dev_free(F[k], s);
    };
    if (!M || !grams || !gram_m || !S || !gwork || !inner || !resid || !fitd || !lam || !ws.row || !ws.val || !fok) {
        cleanup();
        return fail(SPT_E_OOM, "cp_als: workspace allocation failed");
    }
    for (int k = 0; k < N; ++k)
        if (hipMemcpyAsync(F[k], factors[k], sizeof(float) * t->dims[k] * R, hipMemcpyDeviceToDevice, s) != hipSuccess) {
            cleanup();
            return hip_fail(hipGetLastError(), "cp_als: factor copy");
        }
    int *status = (int *)(fitd + 4);
#define CK(x)                    \
    do {                         \
        spt_status st__ = (x);   \
        if (st__ != SPT_OK) {    \
            cleanup();           \
            return st__;         \
        }                        \
    } while (0)
    for (int k = 0; k < N; ++k) CK(launch_gram(F[k], t->dims[k], R, grams + (size_t)k * R * R, gwork, gw, s));
    double fit = 0.0, fit_prev = 0.0;
    int it = 0;
    while (it < max_iters) {
        for (int n = 0; n < N; ++n) {
            const int64_t In = t->dims[n];
            CK(run_mttkrp(t, (const float *const *)F, R, n, M, s, &ws));
            CK(launch_gram(M, In, R, gram_m, gwork, gw, s));
            CK(launch_solve_prep(grams, N, n, R, gram_m, S, lam, status + n, grams + (size_t)n * R * R, s));
            CK(launch_apply(M, In, R, S, F[n], lam, n == N - 1 ? inner : nullptr, nullptr, s));
        }
        CK(launch_fit(grams, N, R, lam, inner, inner_parts, t->norm_x2, fitd, s));
        double hf[4];
        int hs[kMaxModes];
        if (hipMemcpyAsync(hf, fitd, sizeof(hf), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(hs, status, sizeof(int) * N, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            cleanup();
            return hip_fail(hipGetLastError(), "cp_als: fit readback");
        }
        for (int n = 0; n < N; ++n)
            if (hs[n] < 0) {
                cleanup();
                return fail(SPT_E_NOT_SPD, "cp_als: normal equations of mode " + std::to_string(n) +
                                               " not positive definite after ridge retries");
            }
        fit = hf[0];
        if (1.0 - fit < 1e-2 && t->nnz > 0) {
            // near convergence the Gram shortcut loses accuracy (FP32 MTTKRP); take the
            // residual directly over the nonzeros in FP64
            MttkrpArgs a = make_args(t, (const float *const *)F, R, -1, nullptr, 1024);
            CK(launch_resid(a, lam, resid, (int)resid_tiles, s));
            CK(launch_fit_direct(resid, (int)resid_tiles, t->norm_x2, fitd, s));
            if (hipMemcpyAsync(hf, fitd, sizeof(hf), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                cleanup();
                return hip_fail(hipGetLastError(), "cp_als: direct fit readback");
            }
            fit = hf[0];
        }
        ++it;
        if (tol > 0.0 && std::fabs(fit - fit_prev) < tol) break;
        fit_prev = fit;
    }
    for (int k = 0; k < N; ++k)
        if (hipMemcpyAsync(factors[k], F[k], sizeof(float) * t->dims[k] * R, hipMemcpyDeviceToDevice, s) != hipSuccess) {
            cleanup();
            return hip_fail(hipGetLastError(), "cp_als: factor copy back");
        }
    if (it > 0 && hipMemcpyAsync(lambda, lam, sizeof(double) * R, hipMemcpyDeviceToDevice, s) != hipSuccess) {
        cleanup();
        return hip_fail(hipGetLastError(), "cp_als: lambda copy back");
    }
#undef CK
    cleanup();
    *fit_out = fit;
    *iters_out = it;
    return SPT_OK;
}

}  // extern "C"

extern "C" {

spt_status spt_als_update(const double *grams, int nmodes, int mode, int rank, const float *M, int64_t rows,
                          float *C, double *lambda, int *retries_out, void *stream) {
    if (!grams || !lambda || !retries_out || (rows > 0 && (!M || !C)))
        return fail(SPT_E_INVALID_ARG, "als_update: NULL argument");
    if (nmodes < 1 || nmodes > kMaxModes || mode < 0 || mode >= nmodes)
        return fail(SPT_E_INVALID_ARG, "als_update: mode out of range");
    if (rank < 1 || rank > SPT_MAX_ALS_RANK) return fail(SPT_E_INVALID_ARG, "als_update: rank must be in 1..64");
    if (rows < 0) return fail(SPT_E_INVALID_ARG, "als_update: rows < 0");
    if ((M && !aligned16(M)) || (C && !aligned16(C))) return fail(SPT_E_INVALID_ARG, "als_update: M/C not 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    const int R = rank;
    const size_t gw = gram_work_bytes(rows, R);
    double *gram_m = (double *)dev_alloc(sizeof(double) * R * R, s);
    double *S = (double *)dev_alloc(sizeof(double) * R * R, s);
    double *gwork = (double *)dev_alloc(gw, s);
    double *lam = (double *)dev_alloc(sizeof(double) * R, s);
    int *status = (int *)dev_alloc(sizeof(int), s);
    auto cleanup = [&]() {
        dev_free(gram_m, s); dev_free(S, s); dev_free(gwork, s); dev_free(lam, s); dev_free(status, s);
    };
    if (!gram_m || !S || !gwork || !lam || !status) {
        cleanup();
        return fail(SPT_E_OOM, "als_update: workspace allocation failed");
    }
    spt_status st = SPT_OK;
    if (rows > 0) st = launch_gram(M, rows, R, gram_m, gwork, gw, s);
    else st = launch_fill_zero((float *)gram_m, 2 * (int64_t)R * R, s);  // FP64 zeros are all-zero bits
    if (st == SPT_OK) st = launch_solve_prep(grams, nmodes, mode, R, gram_m, S, lam, status, nullptr, s);
    int hs = 0;
    if (st == SPT_OK && (hipMemcpyAsync(&hs, status, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
                         hipStreamSynchronize(s) != hipSuccess))
        st = hip_fail(hipGetLastError(), "als_update: status readback");
    if (st == SPT_OK && hs < 0)
        st = fail(SPT_E_NOT_SPD, "als_update: normal-equation matrix not positive definite after ridge retries");
    // outputs are written only once the solve is known to have succeeded
    if (st == SPT_OK && rows > 0) st = launch_apply(M, rows, R, S, C, lam, nullptr, nullptr, s);
    if (st == SPT_OK &&
        hipMemcpyAsync(lambda, lam, sizeof(double) * R, hipMemcpyDeviceToDevice, s) != hipSuccess)
        st = hip_fail(hipGetLastError(), "als_update: lambda copy");
    cleanup();
    if (st == SPT_OK) *retries_out = hs;
    return st;
}

}  // extern "C"
