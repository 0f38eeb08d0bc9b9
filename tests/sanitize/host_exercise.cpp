// Exercise the library's host code under AddressSanitizer and
// UndefinedBehaviorSanitizer (host instrumentation only: the kernels are
// built as usual).  Test infrastructure: it checks statuses and the
// consistency of results between entry points, not numerics against the
// oracle (the parity tests do that).
//
//   host_exercise cpu   host-only paths: admission simulation over random
//                       arrival streams, argument checks of every entry point
//   host_exercise gpu   the whole C-ABI on a small tensor on device 0:
//                       encode, prepare, MTTKRP (allocating, allocation-free,
//                       FP64), CP-ALS, batched calls, the autotuner, plan
//                       changes, the allocator hook and the server
//
// Exit status 0 when every check holds; a sanitizer report aborts the run.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "spt.h"

namespace {

int g_fail = 0;

void check(bool ok, const char *what) {
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s (%s)\n", what, spt_last_error());
        ++g_fail;
    }
}

void check_ok(spt_status st, const char *what) {
    if (st != SPT_OK) {
        std::fprintf(stderr, "FAILED: %s -> status %d (%s)\n", what, (int)st, spt_last_error());
        ++g_fail;
    }
}

// splitmix64: seeded test inputs
struct Rng {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
    uint32_t below(uint64_t n) { return (uint32_t)(next() % n); }
};

// ------------------------------------------------------------------ cpu
void run_cpu() {
    check(std::strlen(spt_version()) > 0, "version string");
    Rng rng{1};
    for (int trial = 0; trial < 300; ++trial) {
        const int count = 1 + (int)rng.below(200);
        const int slots = 1 + (int)rng.below(8);
        const size_t budget = 1000 + rng.below(100000);
        std::vector<size_t> bytes(count);
        std::vector<double> arrive(count), service(count), admit(count), done(count);
        std::vector<int> status(count);
        double t = 0.0;
        for (int i = 0; i < count; ++i) {
            t += rng.uniform() * 0.01;
            arrive[i] = t;
            service[i] = 0.001 + rng.uniform() * 0.05;
            bytes[i] = 1 + rng.below(budget + budget / 8);  // some above the whole budget
        }
        check_ok(spt_server_simulate(budget, slots, count, bytes.data(), arrive.data(), service.data(), admit.data(),
                                     done.data(), status.data()),
                 "simulate");
        for (int i = 0; i < count; ++i) {
            if (bytes[i] > budget) {
                check(status[i] == SPT_E_OOM, "simulate: over-budget request rejected");
            } else {
                check(status[i] == SPT_OK, "simulate: request served");
                check(admit[i] >= arrive[i] && done[i] >= admit[i] + service[i] - 1e-12, "simulate: times ordered");
            }
        }
    }
    // argument checks: every call below must fail on the host
    const int64_t dims[3] = {4, 4, 4};
    spt_tensor t = nullptr;
    check(spt_encode(nullptr, 3, nullptr, nullptr, 1, nullptr, 0, nullptr, &t) != SPT_OK, "encode: null dims");
    check(spt_encode(dims, 0, nullptr, nullptr, 1, nullptr, 0, nullptr, &t) != SPT_OK, "encode: no modes");
    check(spt_encode(dims, SPT_MAX_MODES + 1, nullptr, nullptr, 1, nullptr, 0, nullptr, &t) != SPT_OK,
          "encode: too many modes");
    check(t == nullptr, "encode: no handle on failure");
    check(std::strlen(spt_last_error()) > 0, "last error message");
    spt_tensor_info info;
    check(spt_tensor_get_info(nullptr, &info) != SPT_OK, "info: null tensor");
    check(spt_tensor_prepare(nullptr, 4, SPT_PREPARE_SINGLE, nullptr) != SPT_OK, "prepare: null tensor");
    check(spt_mttkrp(nullptr, nullptr, 4, 0, nullptr, nullptr) != SPT_OK, "mttkrp: null tensor");
    check(spt_mttkrp_noalloc(nullptr, nullptr, 4, 0, nullptr, nullptr) != SPT_OK, "mttkrp_noalloc: null tensor");
    check(spt_cp_als(nullptr, 4, 1, 0.0, nullptr, nullptr, nullptr, nullptr, nullptr) != SPT_OK, "cp_als: null");
    check(spt_mttkrp_batched(nullptr, 1, nullptr, nullptr, 0, nullptr, nullptr) != SPT_OK, "batched: null");
    check(spt_cp_als_batched(nullptr, 1, nullptr, 1, 0.0, nullptr, nullptr, nullptr, nullptr, nullptr) != SPT_OK,
          "cp_als_batched: null");
    check(spt_als_update(nullptr, 3, 0, 4, nullptr, 4, nullptr, nullptr, nullptr, nullptr) != SPT_OK,
          "als_update: null");
    check(spt_set_allocator(reinterpret_cast<spt_alloc_fn>(&std::malloc), nullptr, nullptr) != SPT_OK,
          "allocator: one hook");
    check(spt_server_simulate(100, 1, -1, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) != SPT_OK,
          "simulate: negative count");
    check(spt_server_submit(nullptr, nullptr, nullptr) != SPT_OK, "submit: null server");
    spt_tensor_free(nullptr, nullptr);
}

// ------------------------------------------------------------------ gpu
struct Dev {
    std::vector<void *> ptrs;
    template <class T>
    T *alloc(size_t n) {
        void *p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
            std::fprintf(stderr, "hipMalloc failed\n");
            std::exit(2);
        }
        ptrs.push_back(p);
        return (T *)p;
    }
    template <class T>
    T *upload(const std::vector<T> &h) {
        T *p = alloc<T>(h.size());
        (void)hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
        return p;
    }
    ~Dev() {
        for (void *p : ptrs) (void)hipFree(p);
    }
};

struct HostTensor {
    std::vector<int64_t> dims;
    std::vector<uint32_t> coords;  // SoA
    std::vector<float> vals;
    int64_t nnz;
};

HostTensor make_tensor(std::vector<int64_t> dims, int64_t nnz, uint64_t seed) {
    HostTensor h{dims, {}, {}, nnz};
    Rng rng{seed};
    h.coords.resize(dims.size() * nnz);
    h.vals.resize(nnz);
    for (size_t n = 0; n < dims.size(); ++n)
        for (int64_t j = 0; j < nnz; ++j) h.coords[n * nnz + j] = rng.below((uint64_t)dims[n]);
    for (int64_t j = 0; j < nnz; ++j) h.vals[j] = (float)rng.uniform();
    return h;
}

std::vector<float> random_factor(int64_t rows, int rank, Rng &rng) {
    std::vector<float> f((size_t)rows * rank);
    for (float &x : f) x = (float)(rng.uniform() - 0.5);
    return f;
}

std::vector<float> download(const float *p, size_t n) {
    std::vector<float> h(n);
    (void)hipMemcpy(h.data(), p, n * sizeof(float), hipMemcpyDeviceToHost);
    return h;
}

double max_rel_diff(const std::vector<float> &a, const std::vector<float> &b) {
    double m = 0.0, s = 1e-30;
    for (size_t i = 0; i < a.size(); ++i) {
        m = std::max(m, (double)std::fabs(a[i] - b[i]));
        s = std::max(s, (double)std::fabs(b[i]));
    }
    return m / s;
}

int64_t g_hook_allocs = 0, g_hook_frees = 0;
void *hook_alloc(size_t bytes, void *, void *) {
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    ++g_hook_allocs;
    return p;
}
void hook_release(void *p, void *stream, void *) {
    (void)hipStreamSynchronize((hipStream_t)stream);
    (void)hipFree(p);
    ++g_hook_frees;
}

void run_gpu() {
    check(hipSetDevice(0) == hipSuccess, "device 0");
    Dev dev;
    const int R = 16;
    HostTensor a = make_tensor({40, 30, 20, 6}, 3000, 7);
    HostTensor b = make_tensor({25, 50, 12}, 2000, 8);
    spt_tensor ta = nullptr, tb = nullptr;
    check_ok(spt_encode(a.dims.data(), 4, dev.upload(a.coords), dev.upload(a.vals), a.nnz, nullptr, 0, nullptr, &ta),
             "encode a");
    check_ok(spt_encode(b.dims.data(), 3, dev.upload(b.coords), dev.upload(b.vals), b.nnz, nullptr, 0, nullptr, &tb),
             "encode b");
    if (!ta || !tb) return;
    spt_tensor_info info;
    check_ok(spt_tensor_get_info(ta, &info), "info");
    check(info.nnz == a.nnz && info.nmodes == 4, "info fields");
    uint32_t *dec = dev.alloc<uint32_t>(4 * a.nnz);
    check_ok(spt_tensor_decode(ta, dec, nullptr), "decode");
    check_ok(spt_tensor_prepare(ta, R, SPT_PREPARE_SINGLE | SPT_PREPARE_BATCHED, nullptr), "prepare a");
    check_ok(spt_tensor_prepare(tb, R, SPT_PREPARE_SINGLE | SPT_PREPARE_BATCHED, nullptr), "prepare b");

    Rng rng{9};
    std::vector<float *> fa, fb;
    for (int64_t d : a.dims) fa.push_back(dev.upload(random_factor(d, R, rng)));
    for (int64_t d : b.dims) fb.push_back(dev.upload(random_factor(d, R, rng)));
    std::vector<float *> oa, ob;
    for (int64_t d : a.dims) oa.push_back(dev.alloc<float>((size_t)d * R));
    for (int64_t d : b.dims) ob.push_back(dev.alloc<float>((size_t)d * R));
    for (int n = 0; n < 4; ++n) check_ok(spt_mttkrp(ta, fa.data(), R, n, oa[n], nullptr), "mttkrp a");
    float *na = dev.alloc<float>((size_t)a.dims[0] * R);
    check_ok(spt_mttkrp_noalloc(ta, fa.data(), R, 0, na, nullptr), "mttkrp_noalloc");
    check(hipDeviceSynchronize() == hipSuccess, "sync");
    check(max_rel_diff(download(na, a.dims[0] * R), download(oa[0], a.dims[0] * R)) <= 1e-6,
          "noalloc matches mttkrp");

    // FP64 values and factors
    std::vector<double> v64(a.vals.begin(), a.vals.end());
    check_ok(spt_tensor_attach_f64(ta, dev.upload(std::vector<double>(v64)), nullptr), "attach f64");
    std::vector<double *> fa64;
    for (int64_t d : a.dims) {
        std::vector<double> f((size_t)d * R);
        for (double &x : f) x = rng.uniform() - 0.5;
        fa64.push_back(dev.upload(f));
    }
    double *o64 = dev.alloc<double>((size_t)a.dims[1] * R);
    check_ok(spt_mttkrp_f64(ta, fa64.data(), R, 1, o64, nullptr), "mttkrp_f64");

    // batched MTTKRP against the single-tensor call
    spt_tensor ts[2] = {ta, tb};
    const float *const *fs[2] = {fa.data(), fb.data()};
    const int ranks[2] = {R, R};
    float *bo[2] = {dev.alloc<float>((size_t)a.dims[2] * R), dev.alloc<float>((size_t)b.dims[2] * R)};
    check_ok(spt_mttkrp_batched(ts, 2, fs, ranks, 2, bo, nullptr), "mttkrp_batched");
    check_ok(spt_mttkrp(tb, fb.data(), R, 2, ob[2], nullptr), "mttkrp b");
    check(hipDeviceSynchronize() == hipSuccess, "sync");
    const double da = max_rel_diff(download(bo[0], a.dims[2] * R), download(oa[2], a.dims[2] * R));
    const double db = max_rel_diff(download(bo[1], b.dims[2] * R), download(ob[2], b.dims[2] * R));
    if (da > 1e-5 || db > 1e-5) std::fprintf(stderr, "batched vs single: %.3e %.3e\n", da, db);
    check(da <= 1e-5, "batched a");
    check(db <= 1e-5, "batched b");

    // CP-ALS, single and batched
    double *lam = dev.alloc<double>(R);
    double fit = 0.0;
    int its = 0;
    check_ok(spt_cp_als(ta, R, 4, 0.0, fa.data(), lam, &fit, &its, nullptr), "cp_als");
    check(its == 4 && fit > -1.0 && fit <= 1.0, "cp_als fit");
    float *const *fsm[2] = {fa.data(), fb.data()};
    double *lams[2] = {dev.alloc<double>(R), dev.alloc<double>(R)};
    double fits[2] = {0, 0};
    int iters[2] = {0, 0};
    check_ok(spt_cp_als_batched(ts, 2, ranks, 3, 0.0, fsm, lams, fits, iters, nullptr), "cp_als_batched");

    // allocator hook: a counting hook, then back to the default
    check_ok(spt_set_allocator(hook_alloc, hook_release, nullptr), "set allocator");
    for (int n = 0; n < 4; ++n) check_ok(spt_mttkrp(ta, fa.data(), R, n, oa[n], nullptr), "mttkrp under hook");
    check_ok(spt_set_allocator(nullptr, nullptr, nullptr), "default allocator");
    check(hipDeviceSynchronize() == hipSuccess, "sync");
    check(g_hook_allocs > 0 && g_hook_allocs == g_hook_frees, "hook allocations returned");

    // plan change, then the autotuner (re-encodes in place)
    spt_plan plan;
    check_ok(spt_tensor_get_plan(tb, &plan), "get plan");
    for (int n = 0; n < 3; ++n) plan.tile[n] = 1024;
    check_ok(spt_tensor_set_plan(tb, &plan, nullptr), "set plan");
    check_ok(spt_tensor_prepare(tb, R, SPT_PREPARE_SINGLE, nullptr), "prepare after plan change");
    check_ok(spt_mttkrp(tb, fb.data(), R, 0, ob[0], nullptr), "mttkrp after plan change");
    spt_tune_result tr;
    check_ok(spt_autotune(&tb, fb.data(), R, 300.0, 2, 11, &tr, nullptr), "autotune");
    check(tr.best_ms > 0.0 && tr.alto_ms > 0.0 && tr.candidates >= 2, "autotune result");
    check_ok(spt_mttkrp(tb, fb.data(), R, 1, ob[1], nullptr), "mttkrp after autotune");
    check(hipDeviceSynchronize() == hipSuccess, "sync");

    // server: good requests, one with an out-of-range coordinate
    spt_server srv = nullptr;
    check_ok(spt_server_create((size_t)1 << 30, 3, &srv), "server create");
    if (srv) {
        std::vector<HostTensor> reqs;
        for (int i = 0; i < 5; ++i) reqs.push_back(make_tensor({30, 20, 10}, 800 + 100 * i, 100 + i));
        reqs[3].coords[5] = 99;  // mode 0 has 30 rows
        std::vector<std::vector<float>> init;
        for (int i = 0; i < 3; ++i) init.push_back(random_factor(reqs[0].dims[i], 8, rng));
        const float *initp[3] = {init[0].data(), init[1].data(), init[2].data()};
        std::vector<uint64_t> tickets;
        for (auto &h : reqs) {
            spt_request q{};
            q.nmodes = 3;
            for (int n = 0; n < 3; ++n) q.dims[n] = h.dims[n];
            q.nnz = h.nnz;
            q.coords = h.coords.data();
            q.vals = h.vals.data();
            q.init = initp;
            q.rank = 8;
            q.max_iters = 5;
            q.tol = 0.0;
            uint64_t tk = 0;
            check_ok(spt_server_submit(srv, &q, &tk), "submit");
            tickets.push_back(tk);
        }
        for (size_t i = 0; i < tickets.size(); ++i) {
            spt_result res;
            check_ok(spt_server_wait(srv, tickets[i], 120.0, &res, nullptr, nullptr), "wait");
            if (i == 3) check(res.status == SPT_E_INDEX_RANGE, "bad request retired alone");
            else check(res.status == SPT_OK && res.iters == 5, "request served");
        }
        spt_server_destroy(srv);
    }
    spt_tensor_free(ta, nullptr);
    spt_tensor_free(tb, nullptr);
    check(hipDeviceSynchronize() == hipSuccess, "final sync");
}

}  // namespace

int main(int argc, char **argv) {
    const char *mode = argc > 1 ? argv[1] : "cpu";
    if (std::strcmp(mode, "cpu") == 0) run_cpu();
    else if (std::strcmp(mode, "gpu") == 0) run_gpu();
    else {
        std::fprintf(stderr, "usage: host_exercise cpu|gpu\n");
        return 2;
    }
    std::printf("host_exercise %s: %s\n", mode, g_fail ? "FAILED" : "ok");
    return g_fail ? 1 : 0;
}
