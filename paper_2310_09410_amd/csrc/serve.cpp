// Serving runtime: OPF solve requests of differing feeder sizes, admitted by
// device memory and compute capacity, solved concurrently on the GPU.
//
// A request is assembled and decomposed on the caller's thread at submit
// (errors come back at once), then queued. A scheduler thread owns every HIP
// call: it admits queued requests first-fit in arrival order as soon as
// (a) a stream slot is free, (b) the request's device bytes fit the HBM
// budget next to the requests in flight, and (c) its sweep's workgroups fit
// the chip next to the sweeps running — counted per XCD, ceil(P/8) of the 32
// CUs of each, one CU per workgroup, so that concurrently running persistent
// sweeps can always be resident together. An admitted request gets its
// operators precomputed and its solve launched on its slot's stream; its
// state stays resident on the device until it finishes, when the results are
// copied to host memory and its device memory and slot are released. The
// sweeps are launched as ordinary (not cooperative) launches, because
// cooperative launches share one hardware queue and would run one after
// another: the admission by compute units is what keeps every workgroup of
// every running sweep resident, so the sweeps of different requests run side
// by side. A request whose real plan needs more units than were admitted for
// it (a rank-deficient subsystem changes the plan) is launched cooperatively.
// Latency = completion - submit.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "host_util.h"
#include "internal.h"
#include "problem.h"

namespace ldopf {
namespace {

using Clock = std::chrono::steady_clock;

constexpr int32_t kUnitsPerChip = 32;  // CUs per XCD on a 256-CU part; units are per-XCD CU counts

struct Request {
    int64_t id = 0;
    ConsensusLP lp;
    ldopf_options opts{};
    int64_t bytes = 0;
    int32_t units = 0;
    int32_t state = LDOPF_REQ_QUEUED;
    int32_t skipped = 0;
    Clock::time_point t_submit, t_done;
    int slot = -1;
    ldopf_problem* prob = nullptr;
    ldopf_status status{};
    int32_t code = LDOPF_OK;
    std::string detail;
    std::vector<double> x, xs, lam;
};

}  // namespace
}  // namespace ldopf

using namespace ldopf;

struct ldopf_server {
    int64_t budget = 0;
    int32_t n_slots = 0;
    std::vector<hipStream_t> streams;
    SweepStatus* pinned = nullptr;  // one pinned status word per slot
    std::vector<int64_t> slot_req;  // request id per slot, -1 free
    int dev = 0;
    int32_t units_per_xcd = kUnitsPerChip;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::map<int64_t, std::unique_ptr<Request>> reqs;
    std::deque<int64_t> queue;
    int64_t next_id = 1;
    bool stop = false;
    std::thread worker;

    // accounting (scheduler thread writes under mu)
    int64_t bytes_in_use = 0, peak_bytes = 0;
    int32_t units_in_use = 0, running = 0, peak_running = 0;
    int64_t submitted = 0, completed = 0, failed = 0;
    std::vector<double> latencies_ms;
    Clock::time_point t_first{}, t_last{};
    bool any = false;
    std::string worker_error;

    void run();
};

namespace {

void finish_request(ldopf_server& srv, Request& r) {
    // Everything slow happens first, outside the lock and into locals: wait
    // for the solve, copy the results to the host, free the device memory.
    // The request stays RUNNING meanwhile, so no client can release it.
    ldopf_problem* p = r.prob;
    ldopf_status status{};
    int32_t code = LDOPF_OK;
    std::string detail;
    std::vector<double> x, xs, lam;
    try {
        code = problem_finish(*p, &status);
        const int64_t n = p->lp.n, nl = int64_t(p->lp.gidx.size());
        x.resize(n);
        xs.resize(nl);
        lam.resize(nl);
        hip_check(hipMemcpyAsync(x.data(), p->x.p, n * 8, hipMemcpyDeviceToHost, p->stream), "download x");
        hip_check(hipMemcpyAsync(xs.data(), p->xs.p, nl * 8, hipMemcpyDeviceToHost, p->stream), "download x_s");
        hip_check(hipMemcpyAsync(lam.data(), p->lam.p, nl * 8, hipMemcpyDeviceToHost, p->stream), "download lambda");
        hip_check(hipStreamSynchronize(p->stream), "download results");
    } catch (const Error& e) {
        code = e.code;
        detail = e.detail;
    }
    delete p;
    const bool ok = code == LDOPF_OK || code == LDOPF_NOT_CONVERGED;
    const Clock::time_point t_done = Clock::now();
    ConsensusLP lp_drop;  // the host LP is freed after the lock is released
    {
        // One critical section publishes the request: results, status and
        // the server's bookkeeping, and the state last. A client can see
        // DONE (and release the request) only after this section, and the
        // scheduler touches the request no more after it.
        std::lock_guard<std::mutex> lk(srv.mu);
        r.prob = nullptr;
        r.status = status;
        r.code = code;
        r.detail = std::move(detail);
        r.x = std::move(x);
        r.xs = std::move(xs);
        r.lam = std::move(lam);
        r.t_done = t_done;
        lp_drop = std::move(r.lp);
        srv.slot_req[r.slot] = -1;
        srv.bytes_in_use -= r.bytes;
        srv.units_in_use -= r.units;
        srv.running--;
        if (ok) {
            srv.completed++;
            srv.latencies_ms.push_back(std::chrono::duration<double, std::milli>(t_done - r.t_submit).count());
            srv.t_last = t_done;
        } else {
            srv.failed++;
        }
        r.state = ok ? LDOPF_REQ_DONE : LDOPF_REQ_FAILED;
        srv.cv_done.notify_all();
    }
}

}  // namespace

void ldopf_server::run() {
    (void)hipSetDevice(dev);
    for (;;) {
        // 1. completions
        std::vector<Request*> ready;
        {
            std::lock_guard<std::mutex> lk(mu);
            for (int s = 0; s < n_slots; ++s) {
                if (slot_req[s] < 0) continue;
                Request& r = *reqs[slot_req[s]];
                if (r.state == LDOPF_REQ_RUNNING && r.prob && problem_ready(*r.prob)) ready.push_back(&r);
            }
        }
        for (Request* r : ready) finish_request(*this, *r);
        // 2. admission, first fit in arrival order
        Request* admit = nullptr;
        int slot = -1;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (stop && queue.empty() && running == 0) return;
            for (int s = 0; s < n_slots && slot < 0; ++s)
                if (slot_req[s] < 0) slot = s;
            if (slot >= 0) {
                for (auto it = queue.begin(); it != queue.end(); ++it) {
                    Request& r = *reqs[*it];
                    if (r.state != LDOPF_REQ_QUEUED) continue;
                    const bool fits = bytes_in_use + r.bytes <= budget && units_in_use + r.units <= units_per_xcd;
                    if (fits) {
                        admit = &r;
                        queue.erase(it);
                        break;
                    }
                    // the oldest request may not be overtaken forever
                    if (it == queue.begin() && ++r.skipped > 64) break;
                }
            }
            if (admit) {
                slot_req[slot] = admit->id;
                admit->slot = slot;
                admit->state = LDOPF_REQ_RUNNING;
                bytes_in_use += admit->bytes;
                peak_bytes = std::max(peak_bytes, bytes_in_use);
                units_in_use += admit->units;
                running++;
                peak_running = std::max(peak_running, running);
            } else if (ready.empty()) {
                // nothing to start: sleep until a submit, or poll completions soon
                cv_work.wait_for(lk, std::chrono::microseconds(running > 0 ? 50 : 2000));
                continue;
            }
        }
        if (!admit) continue;
        try {
            ConsensusLP lp = admit->lp;
            admit->prob = problem_create(std::move(lp), admit->opts, streams[slot], true, pinned + slot);
            const int32_t units = (admit->prob->plan.n_parts + 7) / 8;
            problem_launch(*admit->prob, nullptr, units > admit->units);
        } catch (const Error& e) {
            std::lock_guard<std::mutex> lk(mu);
            admit->code = e.code;
            admit->detail = e.detail;
            admit->state = LDOPF_REQ_FAILED;
            delete admit->prob;
            admit->prob = nullptr;
            slot_req[slot] = -1;
            bytes_in_use -= admit->bytes;
            units_in_use -= admit->units;
            running--;
            failed++;
            cv_done.notify_all();
        }
    }
}

extern "C" {

int ldopf_server_create(int64_t hbm_budget_bytes, int32_t max_slots, ldopf_server** out) {
    return guard([&] {
        need(out, "out");
        *out = nullptr;
        if (max_slots < 1 || max_slots > 64) fail(LDOPF_INVALID_ARGUMENT, "max_slots must be in [1, 64]");
        auto* srv = new ldopf_server();
        try {
            hip_check(hipGetDevice(&srv->dev), "hipGetDevice");
            int cus = 256;
            hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, srv->dev), "device attribute");
            srv->units_per_xcd = std::max(1, cus / 8);
            if (hbm_budget_bytes <= 0) {
                size_t free_b = 0, total_b = 0;
                hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
                hbm_budget_bytes = int64_t(free_b / 10 * 8);
            }
            srv->budget = hbm_budget_bytes;
            srv->n_slots = max_slots;
            srv->slot_req.assign(max_slots, -1);
            for (int i = 0; i < max_slots; ++i) {
                hipStream_t s;
                hip_check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "stream");
                srv->streams.push_back(s);
            }
            hip_check(hipHostMalloc(reinterpret_cast<void**>(&srv->pinned), sizeof(SweepStatus) * size_t(max_slots),
                                    hipHostMallocDefault),
                      "pinned status words");
            srv->worker = std::thread([srv] { srv->run(); });
        } catch (...) {
            for (hipStream_t s : srv->streams) (void)hipStreamDestroy(s);
            if (srv->pinned) (void)hipHostFree(srv->pinned);
            delete srv;
            throw;
        }
        *out = srv;
    });
}

int ldopf_server_submit(ldopf_server* srv, const ldopf_network* net, const ldopf_options* opts, int64_t* req_id) {
    return guard([&] {
        need(srv, "server");
        need(net, "net");
        need(req_id, "req_id");
        ldopf_options o;
        ldopf_default_options(&o);
        if (opts) o = *opts;
        check_options(o);
        if (o.sweep_path == LDOPF_PATH_STREAMED)
            fail(LDOPF_UNSUPPORTED, "served requests run on the persistent sweep (admitted by compute units)");
        o.sweep_path = LDOPF_PATH_PERSISTENT;  // a request too large for it fails at admission
        o.history = 0;  // results only; no per-sweep history on the server
        auto r = std::make_unique<Request>();
        r->lp = assemble_network(*net);
        r->opts = o;
        r->bytes = problem_device_bytes(r->lp, o);
        const int32_t parts = problem_parts_estimate(r->lp, o);
        r->units = (parts + 7) / 8;
        if (r->bytes > srv->budget)
            fail(LDOPF_OUT_OF_MEMORY, "request needs " + std::to_string(r->bytes) + " device bytes, above the server budget");
        if (r->units > srv->units_per_xcd) fail(LDOPF_UNSUPPORTED, "request needs more workgroups than the chip holds");
        r->t_submit = Clock::now();
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop) fail(LDOPF_INVALID_ARGUMENT, "server is shutting down");
        r->id = srv->next_id++;
        *req_id = r->id;
        if (!srv->any) {
            srv->t_first = r->t_submit;
            srv->any = true;
        }
        srv->submitted++;
        srv->queue.push_back(r->id);
        srv->reqs[r->id] = std::move(r);
        srv->cv_work.notify_all();
    });
}

int ldopf_request_estimate(const ldopf_network* net, const ldopf_options* opts, int64_t* bytes, int32_t* workgroups) {
    return guard([&] {
        need(net, "net");
        ldopf_options o;
        ldopf_default_options(&o);
        if (opts) o = *opts;
        check_options(o);
        o.history = 0;
        const ConsensusLP lp = assemble_network(*net);
        if (bytes) *bytes = problem_device_bytes(lp, o);
        if (workgroups) *workgroups = problem_parts_estimate(lp, o);
    });
}

int ldopf_server_poll(ldopf_server* srv, int64_t req_id, int32_t* state, ldopf_status* status) {
    return guard([&] {
        need(srv, "server");
        need(state, "state");
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->reqs.find(req_id);
        if (it == srv->reqs.end()) fail(LDOPF_INVALID_ARGUMENT, "unknown request id");
        *state = it->second->state;
        if (status) *status = it->second->status;
    });
}

int ldopf_server_wait(ldopf_server* srv, int64_t req_id, double timeout_s, int32_t* state, ldopf_status* status) {
    return guard([&] {
        need(srv, "server");
        std::unique_lock<std::mutex> lk(srv->mu);
        if (srv->reqs.find(req_id) == srv->reqs.end()) fail(LDOPF_INVALID_ARGUMENT, "unknown request id");
        const auto until = Clock::now() + std::chrono::duration<double>(timeout_s < 0 ? 1e9 : timeout_s);
        // the request is looked up again after every wake-up: another thread
        // may have released it meanwhile
        auto finished = [&] {
            auto it = srv->reqs.find(req_id);
            return it == srv->reqs.end() || it->second->state == LDOPF_REQ_DONE ||
                   it->second->state == LDOPF_REQ_FAILED;
        };
        srv->cv_done.wait_until(lk, until, finished);
        auto it = srv->reqs.find(req_id);
        if (it == srv->reqs.end()) fail(LDOPF_INVALID_ARGUMENT, "request released while waiting");
        const Request& r = *it->second;
        if (state) *state = r.state;
        if (status) *status = r.status;
        if (r.state == LDOPF_REQ_FAILED) fail(r.code, "request failed: " + r.detail);
    });
}

int ldopf_server_cancel(ldopf_server* srv, int64_t req_id) {
    return guard([&] {
        need(srv, "server");
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->reqs.find(req_id);
        if (it == srv->reqs.end()) fail(LDOPF_INVALID_ARGUMENT, "unknown request id");
        Request& r = *it->second;
        if (r.state != LDOPF_REQ_QUEUED) fail(LDOPF_INVALID_ARGUMENT, "only a queued request can be cancelled");
        srv->queue.erase(std::find(srv->queue.begin(), srv->queue.end(), req_id));
        r.state = LDOPF_REQ_FAILED;
        r.code = LDOPF_INVALID_ARGUMENT;
        r.detail = "cancelled";
        srv->failed++;
        srv->cv_done.notify_all();
    });
}

int ldopf_server_fetch(ldopf_server* srv, int64_t req_id, double* x, int64_t cap_x, double* xs, double* lam,
                       int64_t cap_local, int64_t sizes[2]) {
    return guard([&] {
        need(srv, "server");
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->reqs.find(req_id);
        if (it == srv->reqs.end()) fail(LDOPF_INVALID_ARGUMENT, "unknown request id");
        Request& r = *it->second;
        if (r.state != LDOPF_REQ_DONE) fail(LDOPF_INVALID_ARGUMENT, "request has no results");
        const int64_t n = int64_t(r.x.size()), nl = int64_t(r.xs.size());
        if (sizes) {
            sizes[0] = n;
            sizes[1] = nl;
        }
        if (x) {
            if (cap_x < n) fail(LDOPF_BUFFER_TOO_SMALL, "x needs n entries");
            std::memcpy(x, r.x.data(), n * 8);
        }
        if (xs || lam) {
            if (cap_local < nl) fail(LDOPF_BUFFER_TOO_SMALL, "x_s and lambda need N_loc entries");
            if (xs) std::memcpy(xs, r.xs.data(), nl * 8);
            if (lam) std::memcpy(lam, r.lam.data(), nl * 8);
        }
    });
}

int ldopf_server_release(ldopf_server* srv, int64_t req_id) {
    return guard([&] {
        need(srv, "server");
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->reqs.find(req_id);
        if (it == srv->reqs.end()) fail(LDOPF_INVALID_ARGUMENT, "unknown request id");
        if (it->second->state != LDOPF_REQ_DONE && it->second->state != LDOPF_REQ_FAILED)
            fail(LDOPF_INVALID_ARGUMENT, "request still queued or running");
        srv->reqs.erase(it);
    });
}

int ldopf_server_get_stats(ldopf_server* srv, ldopf_server_stats* st) {
    return guard([&] {
        need(srv, "server");
        need(st, "stats");
        std::lock_guard<std::mutex> lk(srv->mu);
        std::memset(st, 0, sizeof(*st));
        st->submitted = srv->submitted;
        st->completed = srv->completed;
        st->failed = srv->failed;
        st->queued = int64_t(srv->queue.size());
        st->running = srv->running;
        st->peak_running = srv->peak_running;
        st->bytes_in_use = srv->bytes_in_use;
        st->peak_bytes_in_use = srv->peak_bytes;
        st->budget_bytes = srv->budget;
        std::vector<double> lat = srv->latencies_ms;
        if (!lat.empty()) {
            std::sort(lat.begin(), lat.end());
            auto pct = [&](double p) {
                // nearest-rank percentile
                const size_t k = size_t(std::max(1.0, std::ceil(p / 100.0 * double(lat.size()))));
                return lat[std::min(lat.size(), k) - 1];
            };
            st->p50_ms = pct(50.0);
            st->p99_ms = pct(99.0);
            double sum = 0.0;
            for (double v : lat) sum += v;
            st->mean_ms = sum / double(lat.size());
            st->max_ms = lat.back();
            st->wall_s = std::chrono::duration<double>(srv->t_last - srv->t_first).count();
            st->solves_per_s = st->wall_s > 0 ? double(srv->completed) / st->wall_s : 0.0;
        }
    });
}

int ldopf_server_destroy(ldopf_server* srv) {
    return guard([&] {
        if (!srv) return;
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->stop = true;
            // queued requests are dropped; running ones finish
            for (int64_t id : srv->queue) {
                Request& r = *srv->reqs[id];
                r.code = LDOPF_INVALID_ARGUMENT;
                r.detail = "dropped at shutdown";
                r.state = LDOPF_REQ_FAILED;
                srv->failed++;
            }
            srv->queue.clear();
            srv->cv_work.notify_all();
            srv->cv_done.notify_all();
        }
        if (srv->worker.joinable()) srv->worker.join();
        for (hipStream_t s : srv->streams) (void)hipStreamDestroy(s);
        if (srv->pinned) (void)hipHostFree(srv->pinned);
        delete srv;
    });
}

}  // extern "C"
