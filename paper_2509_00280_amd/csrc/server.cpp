// Serving loop: continuous batching of CP-ALS requests on one GPU.
//
// Two host threads share a server:
//   * admission: takes submitted requests in arrival order, admits one while
//     its estimated device bytes fit the HBM budget and a slot is free,
//     uploads it and builds its linearized encoding on a side stream, and
//     hands the ready request to the worker;
//   * worker: at every iteration boundary adds the ready requests to the
//     lock-step batch (the batched CP-ALS engine), runs one iteration of all
//     active requests on the compute stream, and retires the converged ones
//     (results copied to host, device memory released, waiters woken).
// Requests that arrive while others run therefore share the GPU from their
// next iteration on.  Timestamps (arrive, admit, done) are on one monotonic
// clock for latency accounting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <utility>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "spt_internal.h"

namespace spt {
namespace {

struct Job {
    uint64_t ticket = 0;
    spt_request req{};
    std::vector<uint32_t> coords;
    std::vector<float> vals;
    std::vector<std::vector<float>> init;
    size_t bytes = 0;  // admission estimate
    // device side (after admission)
    spt_tensor t = nullptr;
    std::vector<float *> F;
    double *lambda = nullptr;
    Member m;
    // result
    spt_result res{};
    std::vector<std::vector<float>> factors_out;
    std::vector<double> lambda_out;
    bool finished = false;
};

size_t estimate_bytes(const spt_request &r) {
    int lp = 0;
    for (int n = 0; n < r.nmodes; ++n) {
        int b = 0;
        while ((int64_t(1) << b) < r.dims[n]) ++b;
        lp += b;
    }
    const size_t kw = lp > 64 ? 2 : 1;
    size_t b = (size_t)r.nnz * (8 * kw + 4 + 4);  // keys, values, perm
    int64_t maxI = 0;
    for (int n = 0; n < r.nmodes; ++n) {
        b += (size_t)r.dims[n] * r.rank * 4;  // factors
        maxI = std::max<int64_t>(maxI, r.dims[n]);
    }
    b += (size_t)maxI * r.rank * 4;                                // its block of the MTTKRP output
    b += (size_t)(r.nmodes + 2) * r.rank * r.rank * 8;             // Grams, solve matrix
    b += (size_t)r.nnz * (size_t)(4 * r.rank + 24);                // record and sort share (pieces <= nnz)
    return b;
}

// Admission by HBM budget and free slots, in arrival order: the head request
// is admitted when a slot is free and its bytes fit the unused budget,
// rejected at once when it exceeds the whole budget, and otherwise waits
// (later requests wait behind it).  Shared by the server and by
// spt_server_simulate, which drives it with a modelled executor.
struct AdmissionPolicy {
    size_t budget = 0;
    int max_slots = 1;
    size_t used = 0;
    int slots = 0;
    enum Decision { WAIT, ADMIT, REJECT };
    Decision decide(size_t bytes) const {
        if (bytes > budget) return REJECT;
        return (slots < max_slots && used + bytes <= budget) ? ADMIT : WAIT;
    }
    void admit(size_t bytes) {
        used += bytes;
        ++slots;
    }
    void release(size_t bytes) {
        used -= bytes;
        --slots;
    }
};

}  // namespace
}  // namespace spt

using namespace spt;

struct spt_server_s {
    AdmissionPolicy policy;
    hipStream_t compute = nullptr, side = nullptr;
    int device = 0;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_admit, cv_work, cv_done;
    std::deque<std::shared_ptr<Job>> pending, ready;
    std::map<uint64_t, std::shared_ptr<Job>> jobs;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread admit_thr, work_thr;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    void finish(const std::shared_ptr<Job> &j, spt_status st) {
        std::lock_guard<std::mutex> lk(mu);
        j->res.status = st;
        j->res.t_done = now();
        j->finished = true;
        cv_done.notify_all();
    }

    // stream-ordered frees after the job's last use on stream s (no device-wide sync)
    void release_device(Job &j, hipStream_t s) {
        tensor_release(j.t, s);
        j.t = nullptr;
        for (float *p : j.F) dev_free(p, s);
        j.F.clear();
        dev_free(j.lambda, s);
        j.lambda = nullptr;
    }

    spt_status stage(Job &j) {
        const spt_request &r = j.req;
        uint32_t *dc = nullptr;
        float *dv = nullptr;
        const size_t nnz = (size_t)r.nnz;
        spt_status st = SPT_OK;
        if (nnz > 0) {
            dc = (uint32_t *)dev_alloc(sizeof(uint32_t) * nnz * r.nmodes, side);
            dv = (float *)dev_alloc(sizeof(float) * nnz, side);
            if (!dc || !dv) st = fail(SPT_E_OOM, "server: staging buffers");
            if (st == SPT_OK &&
                (hipMemcpyAsync(dc, j.coords.data(), sizeof(uint32_t) * nnz * r.nmodes, hipMemcpyHostToDevice, side) != hipSuccess ||
                 hipMemcpyAsync(dv, j.vals.data(), sizeof(float) * nnz, hipMemcpyHostToDevice, side) != hipSuccess))
                st = hip_fail(hipGetLastError(), "server: upload");
        }
        if (st == SPT_OK) st = spt_encode(r.dims, r.nmodes, dc, dv, r.nnz, nullptr, 0, side, &j.t);
        dev_free(dc, side);
        dev_free(dv, side);
        if (st != SPT_OK) return st;
        j.F.assign(r.nmodes, nullptr);
        for (int n = 0; n < r.nmodes && st == SPT_OK; ++n) {
            const size_t e = (size_t)r.dims[n] * r.rank;
            j.F[n] = (float *)dev_alloc(sizeof(float) * e, side);
            if (!j.F[n]) {
                st = fail(SPT_E_OOM, "server: factors");
                break;
            }
            if (hipMemcpyAsync(j.F[n], j.init[n].data(), sizeof(float) * e, hipMemcpyHostToDevice, side) != hipSuccess)
                st = hip_fail(hipGetLastError(), "server: factor upload");
        }
        if (st == SPT_OK && !(j.lambda = (double *)dev_alloc(sizeof(double) * r.rank, side)))
            st = fail(SPT_E_OOM, "server: lambda");
        if (st == SPT_OK && hipStreamSynchronize(side) != hipSuccess) st = hip_fail(hipGetLastError(), "server: stage sync");
        // the host copies are no longer needed
        std::vector<uint32_t>().swap(j.coords);
        std::vector<float>().swap(j.vals);
        return st;
    }

    void admission_loop() {
        (void)hipSetDevice(device);
        for (;;) {
            std::shared_ptr<Job> j;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_admit.wait(lk, [&] {
                    if (stop && pending.empty()) return true;
                    if (pending.empty()) return false;
                    return policy.decide(pending.front()->bytes) != AdmissionPolicy::WAIT;
                });
                if (pending.empty()) return;  // stopping
                j = pending.front();
                pending.pop_front();
                if (policy.decide(j->bytes) == AdmissionPolicy::ADMIT) policy.admit(j->bytes);
            }
            if (j->bytes > policy.budget) {
                set_error("server: request exceeds the HBM budget");
                finish(j, SPT_E_OOM);
                continue;
            }
            j->res.t_admit = now();
            spt_status st = stage(*j);
            if (st != SPT_OK) {
                (void)hipStreamSynchronize(side);
                release_device(*j, side);
                {
                    std::lock_guard<std::mutex> lk(mu);
                    policy.release(j->bytes);
                }
                cv_admit.notify_all();
                finish(j, st);
                continue;
            }
            {
                std::lock_guard<std::mutex> lk(mu);
                ready.push_back(j);
            }
            cv_work.notify_all();
        }
    }

    void work_loop() {
        (void)hipSetDevice(device);
        BatchEngine eng(compute);
        std::vector<std::shared_ptr<Job>> active;
        for (;;) {
            std::vector<std::shared_ptr<Job>> joining;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] { return !ready.empty() || !active.empty() || (stop && pending.empty() && policy.slots == 0); });
                if (ready.empty() && active.empty()) return;  // stopping, nothing left
                while (!ready.empty()) {
                    joining.push_back(ready.front());
                    ready.pop_front();
                }
            }
            for (auto &j : joining) {
                Member &m = j->m;
                m = Member{};
                m.t = j->t;
                m.R = j->req.rank;
                for (int n = 0; n < j->req.nmodes; ++n) m.F[n] = j->F[n];
                m.lambda = j->lambda;
                m.max_iters = j->req.max_iters;
                m.tol = j->req.tol;
                spt_status st = eng.add(&m);
                if (st != SPT_OK) {
                    retire(*j, st);
                    continue;
                }
                if (m.max_iters == 0) m.done = true;
                active.push_back(j);
            }
            if (eng.any_active()) {
                bool before_kernels = false;
                spt_status st = eng.step(&before_kernels);
                if (st != SPT_OK && before_kernels && !joining.empty()) {
                    // the step failed while re-planning for the requests that just
                    // joined (e.g. their workspace does not fit): those requests
                    // retire with the error, the others run the step without them
                    for (auto &j : joining) {
                        if (j->m.done) continue;
                        j->m.done = true;
                        j->m.err = st;
                    }
                    eng.drop_done();
                    st = eng.step(&before_kernels);
                }
                if (st != SPT_OK)
                    for (auto &j : active) {
                        if (j->m.done) continue;
                        j->m.done = true;
                        j->m.err = st;
                    }
            }
            std::vector<std::shared_ptr<Job>> still;
            for (auto &j : active) {
                if (!j->m.done) {
                    still.push_back(j);
                    continue;
                }
                eng.remove(&j->m);
                retire(*j, j->m.err);
            }
            active.swap(still);
        }
    }

    void retire(Job &j, spt_status st) {
        const spt_request &r = j.req;
        if (st == SPT_OK) {
            j.factors_out.resize(r.nmodes);
            for (int n = 0; n < r.nmodes && st == SPT_OK; ++n) {
                j.factors_out[n].resize((size_t)r.dims[n] * r.rank);
                if (hipMemcpy(j.factors_out[n].data(), j.F[n], sizeof(float) * j.factors_out[n].size(),
                              hipMemcpyDeviceToHost) != hipSuccess)
                    st = hip_fail(hipGetLastError(), "server: result copy");
            }
            j.lambda_out.resize(r.rank);
            if (st == SPT_OK &&
                hipMemcpy(j.lambda_out.data(), j.lambda, sizeof(double) * r.rank, hipMemcpyDeviceToHost) != hipSuccess)
                st = hip_fail(hipGetLastError(), "server: lambda copy");
            j.res.fit = j.m.fit;
            j.res.iters = j.m.iters;
        }
        release_device(j, compute);
        {
            std::lock_guard<std::mutex> lk(mu);
            policy.release(j.bytes);
            j.res.status = st;
            j.res.t_done = now();
            j.finished = true;
        }
        cv_done.notify_all();
        cv_admit.notify_all();
        cv_work.notify_all();
    }
};

extern "C" {

spt_status spt_server_create(size_t hbm_budget_bytes, int max_slots, spt_server *out) {
    if (!out || max_slots < 1 || hbm_budget_bytes == 0) return fail(SPT_E_INVALID_ARG, "server: bad arguments");
    auto *s = new (std::nothrow) spt_server_s();
    if (!s) return fail(SPT_E_OOM, "server: host allocation");
    s->policy.budget = hbm_budget_bytes;
    s->policy.max_slots = max_slots;
    s->t0 = std::chrono::steady_clock::now();
    if (hipGetDevice(&s->device) != hipSuccess ||
        hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking) != hipSuccess) {
        spt_status st = hip_fail(hipGetLastError(), "server: streams");
        if (s->compute) (void)hipStreamDestroy(s->compute);
        delete s;
        return st;
    }
    s->admit_thr = std::thread([s] { s->admission_loop(); });
    s->work_thr = std::thread([s] { s->work_loop(); });
    *out = s;
    return SPT_OK;
}

spt_status spt_server_submit(spt_server s, const spt_request *req, uint64_t *ticket) {
    if (!s || !req || !ticket) return fail(SPT_E_INVALID_ARG, "server: NULL argument");
    const spt_request &r = *req;
    if (r.nmodes < 2 || r.nmodes > kMaxModes) return fail(SPT_E_INVALID_ARG, "server: nmodes must be 2..8");
    if (r.rank < 1 || r.rank > SPT_MAX_ALS_RANK) return fail(SPT_E_INVALID_ARG, "server: rank must be 1..64");
    if (r.nnz < 0 || (r.nnz > 0 && (!r.coords || !r.vals)) || !r.init || r.max_iters < 0)
        return fail(SPT_E_INVALID_ARG, "server: bad request");
    auto j = std::make_shared<Job>();
    j->req = r;
    const size_t nnz = (size_t)r.nnz;
    j->coords.assign(r.coords, r.coords + nnz * r.nmodes);
    j->vals.assign(r.vals, r.vals + nnz);
    j->init.resize(r.nmodes);
    for (int n = 0; n < r.nmodes; ++n) {
        if (!r.init[n] || r.dims[n] < 1) return fail(SPT_E_INVALID_ARG, "server: bad initial factor");
        j->init[n].assign(r.init[n], r.init[n] + (size_t)r.dims[n] * r.rank);
    }
    j->req.coords = nullptr;
    j->req.vals = nullptr;
    j->req.init = nullptr;
    j->bytes = estimate_bytes(r);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return fail(SPT_E_INVALID_ARG, "server: stopping");
        j->ticket = s->next_ticket++;
        j->res.t_arrive = s->now();
        s->jobs[j->ticket] = j;
        s->pending.push_back(j);
        *ticket = j->ticket;
    }
    s->cv_admit.notify_all();
    return SPT_OK;
}

spt_status spt_server_wait(spt_server s, uint64_t ticket, double timeout_s, spt_result *res, float *const *factors_out,
                           double *lambda) {
    if (!s || !res) return fail(SPT_E_INVALID_ARG, "server: NULL argument");
    std::shared_ptr<Job> j;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->jobs.find(ticket);
        if (it == s->jobs.end()) return fail(SPT_E_NOT_FOUND, "server: unknown ticket");
        j = it->second;
        auto done = [&] { return j->finished; };
        if (timeout_s < 0) s->cv_done.wait(lk, done);
        else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done))
            return fail(SPT_E_BUSY, "server: timed out");
        s->jobs.erase(it);
    }
    *res = j->res;
    if (j->res.status == SPT_OK) {
        if (factors_out)
            for (int n = 0; n < j->req.nmodes; ++n)
                if (factors_out[n]) std::memcpy(factors_out[n], j->factors_out[n].data(), sizeof(float) * j->factors_out[n].size());
        if (lambda) std::memcpy(lambda, j->lambda_out.data(), sizeof(double) * j->lambda_out.size());
    }
    return SPT_OK;
}

double spt_server_now(spt_server s) { return s ? s->now() : 0.0; }

spt_status spt_server_simulate(size_t hbm_budget_bytes, int max_slots, int count, const size_t *bytes,
                               const double *arrive, const double *service, double *admit_out, double *done_out,
                               int *status_out) {
    if (max_slots < 1 || hbm_budget_bytes == 0 || count < 0 ||
        (count > 0 && (!bytes || !arrive || !service || !admit_out || !done_out || !status_out)))
        return fail(SPT_E_INVALID_ARG, "server_simulate: bad arguments");
    for (int i = 1; i < count; ++i)
        if (arrive[i] < arrive[i - 1]) return fail(SPT_E_INVALID_ARG, "server_simulate: arrivals must be sorted");
    AdmissionPolicy pol;
    pol.budget = hbm_budget_bytes;
    pol.max_slots = max_slots;
    // the modelled executor: an admitted request finishes `service` seconds later
    std::multimap<double, int> running;  // done time -> request
    std::deque<int> queue;
    int next = 0;
    double now = 0.0;
    std::vector<double> admit(count, 0.0), done(count, 0.0);
    std::vector<int> status(count, SPT_OK);
    while (next < count || !queue.empty() || !running.empty()) {
        // admit from the queue head while the policy allows at the current time
        while (!queue.empty()) {
            const int h = queue.front();
            const auto d = pol.decide(bytes[h]);
            if (d == AdmissionPolicy::WAIT) break;
            queue.pop_front();
            admit[h] = now;
            if (d == AdmissionPolicy::REJECT) {
                status[h] = SPT_E_OOM;
                done[h] = now;
                continue;
            }
            pol.admit(bytes[h]);
            running.emplace(now + service[h], h);
        }
        // next event: an arrival or a completion (completions first at equal times)
        const double ta = next < count ? arrive[next] : 1e300;
        const double tc = running.empty() ? 1e300 : running.begin()->first;
        if (tc <= ta) {
            now = tc;
            const int r = running.begin()->second;
            running.erase(running.begin());
            done[r] = now;
            pol.release(bytes[r]);
        } else {
            now = ta;
            queue.push_back(next++);
        }
    }
    for (int i = 0; i < count; ++i) {
        admit_out[i] = admit[i];
        done_out[i] = done[i];
        status_out[i] = status[i];
    }
    return SPT_OK;
}

void spt_server_destroy(spt_server s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_admit.notify_all();
    s->cv_work.notify_all();
    if (s->admit_thr.joinable()) s->admit_thr.join();
    s->cv_work.notify_all();
    if (s->work_thr.joinable()) s->work_thr.join();
    (void)hipStreamSynchronize(s->compute);
    (void)hipStreamDestroy(s->compute);
    (void)hipStreamDestroy(s->side);
    delete s;
}

}  // extern "C"
