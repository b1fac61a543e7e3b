// C ABI of libldopf: validation, ownership, device buffers and the calls of
// include/ldopf.h. The arithmetic of the method runs in device.hip.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <new>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "device.h"
#include "host_util.h"
#include "internal.h"
#include "problem.h"

namespace ldopf {

namespace {
thread_local std::string g_detail;
}

void fail(int code, const std::string& detail) { throw Error{code, detail}; }
void record_error_detail(const std::string& detail) { g_detail = detail; }

void check_options(const ldopf_options& o) {
    if (!(o.rho > 0.0) || !std::isfinite(o.rho)) fail(LDOPF_INVALID_ARGUMENT, "rho must be positive and finite");
    if (!(o.eps_rel >= 0.0) || !std::isfinite(o.eps_rel)) fail(LDOPF_INVALID_ARGUMENT, "eps_rel must be >= 0");
    if (!(o.eps_abs >= 0.0) || !std::isfinite(o.eps_abs)) fail(LDOPF_INVALID_ARGUMENT, "eps_abs must be >= 0");
    if (o.max_iter < 0) fail(LDOPF_INVALID_ARGUMENT, "max_iter must be >= 0");
    if (o.precision != LDOPF_FP64 && o.precision != LDOPF_FP32_MIXED) fail(LDOPF_INVALID_ARGUMENT, "unknown precision");
    if (o.residual_form != LDOPF_RESIDUAL_PAPER && o.residual_form != LDOPF_RESIDUAL_AGGREGATED)
        fail(LDOPF_INVALID_ARGUMENT, "unknown residual form");
    if (o.rho_update != LDOPF_RHO_FIXED && o.rho_update != LDOPF_RHO_BALANCE) fail(LDOPF_INVALID_ARGUMENT, "unknown rho_update");
    if (o.rho_update == LDOPF_RHO_BALANCE) {
        if (o.rho_period < kRhoLag) fail(LDOPF_INVALID_ARGUMENT, "rho_period must be >= 4 (a change takes effect 4 sweeps later)");
        if (o.rho_max_changes < 0 || o.rho_max_changes > kMaxRhoChanges)
            fail(LDOPF_INVALID_ARGUMENT, "rho_max_changes must be in [0, 1024]");
        if (!(o.rho_mu > 1.0) || !std::isfinite(o.rho_mu)) fail(LDOPF_INVALID_ARGUMENT, "rho_mu must be > 1 and finite");
        if (!(o.rho_tau > 1.0) || !std::isfinite(o.rho_tau)) fail(LDOPF_INVALID_ARGUMENT, "rho_tau must be > 1 and finite");
    }
    if (o.check_termination != 0 && o.check_termination != 1) fail(LDOPF_INVALID_ARGUMENT, "check_termination must be 0 or 1");
    if (o.history != 0 && o.history != 1) fail(LDOPF_INVALID_ARGUMENT, "history must be 0 or 1");
    if (o.profile != 0 && o.profile != 1) fail(LDOPF_INVALID_ARGUMENT, "profile must be 0 or 1");
    if (o.rows_per_part < 0) fail(LDOPF_INVALID_ARGUMENT, "rows_per_part must be >= 0");
    if (o.block_threads != 0 && (o.block_threads < 128 || o.block_threads > 1024 || o.block_threads % 64))
        fail(LDOPF_INVALID_ARGUMENT, "block_threads must be 0 or a multiple of 64 in [128, 1024]");
    if (o.sweep_path != LDOPF_PATH_AUTO && o.sweep_path != LDOPF_PATH_PERSISTENT && o.sweep_path != LDOPF_PATH_STREAMED)
        fail(LDOPF_INVALID_ARGUMENT, "unknown sweep_path");
    if (o.reserved != 0) fail(LDOPF_INVALID_ARGUMENT, "reserved option fields must be zero");
}

void check_batch_options(const ldopf_options& o) {
    if (o.residual_form != LDOPF_RESIDUAL_PAPER)
        fail(LDOPF_UNSUPPORTED, "batched scenarios use the literal residual form of Section III-C");
    if (o.rho_update != LDOPF_RHO_FIXED) fail(LDOPF_UNSUPPORTED, "batched scenarios keep rho fixed");
}

}  // namespace ldopf

using namespace ldopf;

namespace {

void init_state(ldopf_problem& h) {
    const ConsensusLP& lp = h.lp;
    std::vector<double> xs(lp.gidx.size()), lam(lp.gidx.size(), 0.0), x(lp.n, NAN);
    for (size_t k = 0; k < lp.gidx.size(); ++k) xs[k] = lp.x_init[lp.gidx[k]];
    hip_check(hipMemcpyAsync(h.xs.p, xs.data(), xs.size() * 8, hipMemcpyHostToDevice, h.stream), "upload x_s");
    hip_check(hipMemcpyAsync(h.lam.p, lam.data(), lam.size() * 8, hipMemcpyHostToDevice, h.stream), "upload lambda");
    hip_check(hipMemcpyAsync(h.x.p, x.data(), x.size() * 8, hipMemcpyHostToDevice, h.stream), "upload x");
    hip_check(hipStreamSynchronize(h.stream), "initial state");
    h.have_x = false;
    h.hist_len = 0;
}

// Global data (cost, bounds, copy counts) and the state buffers, for both
// sweep paths.
void c_upload_globals(ldopf_problem& h) {
    const ConsensusLP& lp = h.lp;
    hipStream_t s = h.stream;
    std::vector<double> cnt(lp.n, 0.0);
    for (int64_t g : lp.gidx) cnt[g] += 1.0;
    h.c.upload(lp.c, s, "upload c");
    h.lo.upload(lp.lo, s, "upload lo");
    h.hi.upload(lp.hi, s, "upload hi");
    h.cnt.upload(cnt, s, "upload counts");
    h.xs.alloc(lp.gidx.size(), "x_s");
    h.lam.alloc(lp.gidx.size(), "lambda");
    h.x.alloc(lp.n, "x");
    h.st.alloc(1, "status");
}

// Everything after the host LP exists: device precompute, plan, buffers.
void build_device(ldopf_problem& h) {
    ConsensusLP& lp = h.lp;
    hipStream_t s = h.stream;
    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    h.device = dev;
    int cus = 0, coop = 0, lds_optin = 0, clock_khz = 0;
    hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "device attribute");
    hip_check(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev), "device attribute");
    hip_check(hipDeviceGetAttribute(&lds_optin, hipDeviceAttributeSharedMemPerBlockOptin, dev), "device attribute");
    hip_check(hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev), "device attribute");
    if (!coop) fail(LDOPF_UNSUPPORTED, "the device does not support cooperative launches");
    if (lds_optin <= 0) hip_check(hipDeviceGetAttribute(&lds_optin, hipDeviceAttributeMaxSharedMemoryPerBlock, dev), "device attribute");
    // a barrier wait longer than 5 s means the launch is broken
    h.spin_limit = uint64_t(std::max(clock_khz, 1000)) * 1000ull * 5ull;
    h.tick_ms = 1.0 / double(std::max(clock_khz, 1));

    int32_t max_n = 1;
    for (int32_t n : lp.ns) max_n = std::max(max_n, n);
    if (max_n > kMaxSubsystemVars)
        fail(LDOPF_UNSUPPORTED, "subsystems with more than " + std::to_string(kMaxSubsystemVars) +
                                    " variables are not supported on the device");
    const int64_t S = lp.S;
    std::vector<int64_t> boff(S + 1, 0);
    for (int64_t i = 0; i < S; ++i) boff[i + 1] = boff[i] + int64_t(lp.ns[i]) * lp.ns[i];

    h.A.upload(lp.A, s, "upload A");
    h.b.upload(lp.b, s, "upload b");
    h.ns.upload(lp.ns, s, "upload n_s");
    h.ms.upload(lp.ms, s, "upload m_s");
    h.a_off.upload(lp.a_off, s, "upload offsets");
    h.row_off.upload(lp.row_off, s, "upload offsets");
    h.loc_off.upload(lp.loc_off, s, "upload offsets");
    h.basis_off.upload(boff, s, "upload offsets");
    h.basis.alloc(boff[S], "basis");
    h.abar.alloc(boff[S], "abar");
    h.bbar.alloc(lp.gidx.size(), "bbar");
    h.rank_d.alloc(S, "rank");
    h.flags.alloc(S, "flags");

    PrecomputeArgs pa{};
    pa.S = S;
    pa.ns = h.ns.p;
    pa.ms = h.ms.p;
    pa.a_off = h.a_off.p;
    pa.row_off = h.row_off.p;
    pa.loc_off = h.loc_off.p;
    pa.basis_off = h.basis_off.p;
    pa.A = h.A.p;
    pa.b = h.b.p;
    pa.basis = h.basis.p;
    pa.abar = h.abar.p;
    pa.bbar = h.bbar.p;
    pa.rank = h.rank_d.p;
    pa.flags = h.flags.p;
    pa.tol_dep = 1e-10;
    pa.tol_rhs = 1e-9;
    pa.max_n = max_n;
    hip_check(hipEventRecord(h.ev0, s), "event");
    hip_check(launch_precompute(pa, s), "precompute launch");
    hip_check(hipEventRecord(h.ev1, s), "event");
    h.rank.resize(S);
    std::vector<int32_t> flags(S);
    hip_check(hipMemcpyAsync(h.rank.data(), h.rank_d.p, S * 4, hipMemcpyDeviceToHost, s), "download ranks");
    hip_check(hipMemcpyAsync(flags.data(), h.flags.p, S * 4, hipMemcpyDeviceToHost, s), "download flags");
    hip_check(hipStreamSynchronize(s), "precompute");
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, h.ev0, h.ev1), "event time");
    h.precompute_ms = ms;
    for (int64_t i = 0; i < S; ++i)
        if (flags[i]) fail(LDOPF_INCONSISTENT_SUBSYSTEM, "subsystem " + std::to_string(i) + ": dependent rows with inconsistent right-hand side");
    // the rows of A_s are no longer needed on the device
    h.A.release();
    h.b.release();

    // the persistent sweep if the problem fits it, else (or on request) the
    // streamed sweep, which takes FP64, the literal residual form and fixed rho
    const int32_t path = h.opts.sweep_path;
    const bool stream_ok = !h.fp32 && h.opts.residual_form == LDOPF_RESIDUAL_PAPER && h.opts.rho_update == LDOPF_RHO_FIXED;
    auto streamed = [&] {
        c_upload_globals(h);
        stream_prepare(h);
        init_state(h);
    };
    if (path == LDOPF_PATH_STREAMED) {
        if (!stream_ok)
            fail(LDOPF_UNSUPPORTED, "the streamed sweep runs in FP64 with the literal residual form and fixed rho");
        streamed();
        return;
    }
    try {
        h.plan = make_plan(lp, h.rank, h.fp32, h.opts.rows_per_part, h.opts.block_threads, cus, lds_optin);
        const Plan& pl = h.plan;
        if (pl.n_parts > kMaxParts) fail(LDOPF_UNSUPPORTED, "more than " + std::to_string(kMaxParts) + " sweep workgroups");
        hip_check(prepare_sweep(h.fp32, size_t(pl.lds_bytes)), "sweep LDS attribute");
        int per_cu = 0;
        hip_check(sweep_occupancy(h.fp32, pl.block_threads, size_t(pl.lds_bytes), &per_cu), "sweep occupancy");
        if (int64_t(per_cu) * cus < pl.n_parts)
            fail(LDOPF_UNSUPPORTED, "the sweep's " + std::to_string(pl.n_parts) + " workgroups cannot be co-resident (" +
                                        std::to_string(per_cu) + " per CU, " + std::to_string(cus) + " CUs)");
    } catch (const Error& e) {
        if (e.code != LDOPF_UNSUPPORTED || path != LDOPF_PATH_AUTO || !stream_ok) throw;
        streamed();
        return;
    }
    const Plan& pl = h.plan;

    h.parts.upload(pl.parts, s, "upload plan");
    h.subs.upload(pl.subs, s, "upload plan");
    h.row_canon.upload(pl.row_canon, s, "upload plan");
    h.row_lvar.upload(pl.row_lvar, s, "upload plan");
    h.row_sub.upload(pl.row_sub, s, "upload plan");
    h.var_gid.upload(pl.var_gid, s, "upload plan");
    h.var_slot.upload(pl.var_slot, s, "upload plan");
    h.var_slot_lo.upload(pl.var_slot_lo, s, "upload plan");
    h.var_slot_hi.upload(pl.var_slot_hi, s, "upload plan");
    h.var_writer.upload(pl.var_writer, s, "upload plan");
    h.var_copy_off.upload(pl.var_copy_off, s, "upload plan");
    h.var_copy_rows.upload(pl.var_copy_rows, s, "upload plan");
    h.tk_sub.upload(pl.tk_sub, s, "upload plan");

    c_upload_globals(h);
    h.bpart.alloc(size_t(2) * std::max(pl.n_slots, 1) * (h.fp32 ? 4 : 8), "boundary slots");
    h.rpart.alloc(size_t(kRing) * pl.n_parts * 8, "residual slots");
    h.gpart.alloc(size_t(kRing) * 8 * kGroup, "residual group slots");
    h.rholog.alloc(size_t(2) * kMaxRhoChanges, "rho log");
    h.prof.alloc(size_t(8) * std::max(pl.n_parts, 1), "phase times");
    init_state(h);
}

template <typename T>
SweepArgs<T> sweep_args(ldopf_problem& h) {
    SweepArgs<T> a{};
    a.parts = h.parts.p;
    a.subs = h.subs.p;
    a.row_canon = h.row_canon.p;
    a.row_lvar = h.row_lvar.p;
    a.row_sub = h.row_sub.p;
    a.var_gid = h.var_gid.p;
    a.var_slot = h.var_slot.p;
    a.var_slot_lo = h.var_slot_lo.p;
    a.var_slot_hi = h.var_slot_hi.p;
    a.var_writer = h.var_writer.p;
    a.var_copy_off = h.var_copy_off.p;
    a.var_copy_rows = h.var_copy_rows.p;
    a.tk_sub = h.tk_sub.p;
    a.basis = h.basis.p;
    a.bbar = h.bbar.p;
    a.c = h.c.p;
    a.lo = h.lo.p;
    a.hi = h.hi.p;
    a.cnt = h.cnt.p;
    a.xs = h.xs.p;
    a.lam = h.lam.p;
    a.x = h.x.p;
    a.bpart = reinterpret_cast<T*>(h.bpart.p);
    a.rpart = h.rpart.p;
    a.gpart = h.gpart.p;
    a.hist = h.hist.p;
    a.hist_cap = h.opts.history ? int64_t(h.hist.count / 4) : 0;
    a.st = h.st.p;
    a.rho = h.opts.rho;
    a.eps_rel = h.opts.eps_rel;
    a.eps_abs = h.opts.eps_abs;
    a.max_iter = h.opts.max_iter;
    a.nloc = int64_t(h.lp.gidx.size());
    a.n = h.lp.n;
    a.rho_update = h.opts.rho_update;
    a.rho_period = std::max(h.opts.rho_period, 1);
    a.rho_max_changes = h.opts.rho_update ? h.opts.rho_max_changes : 0;
    a.rho_mu = h.opts.rho_mu;
    a.rho_tau = h.opts.rho_tau;
    a.rho_log = h.rholog.p;
    a.bagg = h.opts.residual_form == LDOPF_RESIDUAL_AGGREGATED ? h.bagg.p : nullptr;
    a.n_slots = h.plan.n_slots;
    a.check = h.opts.check_termination;
    a.P = h.plan.n_parts;
    a.block = h.plan.block_threads;
    a.spin_limit = h.spin_limit;
    a.prof = h.opts.profile ? h.prof.p : nullptr;
    return a;
}

ldopf_problem* new_problem(const ldopf_options* opts, void* stream, SweepStatus* pinned_status = nullptr) {
    ldopf_options o;
    ldopf_default_options(&o);
    if (opts) o = *opts;
    check_options(o);
    auto* h = new ldopf_problem();
    h->opts = o;
    h->fp32 = o.precision == LDOPF_FP32_MIXED;
    try {
        if (stream) {
            h->stream = static_cast<hipStream_t>(stream);
        } else {
            hip_check(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking), "stream");
            h->own_stream = true;
        }
        hip_check(hipEventCreate(&h->ev0), "event");
        hip_check(hipEventCreate(&h->ev1), "event");
        hip_check(hipEventCreateWithFlags(&h->done, hipEventDisableTiming), "event");
        if (pinned_status) {
            h->last_pinned = pinned_status;
        } else {
            hip_check(hipHostMalloc(reinterpret_cast<void**>(&h->last_pinned), sizeof(SweepStatus), hipHostMallocDefault),
                      "pinned status");
            h->own_pinned = true;
        }
    } catch (...) {
        delete h;
        throw;
    }
    return h;
}

}  // namespace

namespace ldopf {

ldopf_problem* problem_create(ConsensusLP&& lp, const ldopf_options& opts, hipStream_t stream, bool ordered_memory,
                              SweepStatus* pinned_status) {
    ldopf_problem* h = new_problem(&opts, stream, pinned_status);
    if (ordered_memory) h->use_stream_ordered_memory(h->stream);
    try {
        h->lp = std::move(lp);
        build_device(*h);
    } catch (...) {
        delete h;
        throw;
    }
    return h;
}

static_assert(sizeof(SweepStatus) <= 256, "the status word sits in the first 256 bytes of the scratch");

namespace {
size_t agg_words(const ldopf_problem& h) {
    return h.opts.residual_form == LDOPF_RESIDUAL_AGGREGATED ? size_t(4) * size_t(std::max(h.plan.n_slots, 1)) : 0;
}
}  // namespace

size_t problem_sync_bytes(const ldopf_problem& h) {
    const size_t w = h.fp32 ? 4 : 8;
    const size_t nb = (size_t(2) * size_t(std::max(h.plan.n_slots, 1)) * w + 255) & ~size_t(255);
    // status word, group sums, every part's sums, boundary words (each
    // 256-aligned), then the aggregated form's boundary words
    return 256 + size_t(kRing) * 8 * kGroup * 8 + size_t(kRing) * size_t(std::max(h.plan.n_parts, 1)) * 64 + nb +
           agg_words(h) * 8;
}

void problem_launch(ldopf_problem& h, const SyncWords* sw, bool cooperative) {
    if (h.in_flight) fail(LDOPF_INVALID_ARGUMENT, "a solve is already in flight on this handle");
    if (h.streamed) {
        // the whole solve runs here (the host replays the sweep's graph until
        // the test holds); the status is then read like the persistent one's
        if (sw) fail(LDOPF_UNSUPPORTED, "the streamed sweep allocates its own words (no allocation-free solve)");
        if (h.opts.residual_form != LDOPF_RESIDUAL_PAPER || h.opts.rho_update != LDOPF_RHO_FIXED || h.opts.profile)
            fail(LDOPF_UNSUPPORTED, "the streamed sweep takes the literal residual form, fixed rho and no profile");
        const int64_t want = h.opts.history ? std::min<int64_t>(std::max<int64_t>(h.opts.max_iter, 1), int64_t(1) << 22) : 1;
        if (int64_t(h.hist.count) < want * 4) h.hist.alloc(size_t(want) * 4, "history");
        hip_check(hipEventRecord(h.ev0, h.stream), "event");
        stream_solve(h);
        hip_check(hipEventRecord(h.ev1, h.stream), "event");
        hip_check(hipMemcpyAsync(h.last_pinned, h.st.p, sizeof(SweepStatus), hipMemcpyDeviceToHost, h.stream),
                  "download status");
        hip_check(hipEventRecord(h.done, h.stream), "event");
        h.in_flight = true;
        return;
    }
    if (!sw) {
        const int64_t want = h.opts.history ? std::min<int64_t>(std::max<int64_t>(h.opts.max_iter, 1), int64_t(1) << 22) : 1;
        if (int64_t(h.hist.count) < want * 4) h.hist.alloc(size_t(want) * 4, "history");
        if (h.bagg.count < agg_words(h)) h.bagg.alloc(agg_words(h), "aggregated residual words");
    }
    hipError_t e;
    hip_check(hipEventRecord(h.ev0, h.stream), "event");
    auto launch = [&](auto args) {
        using T = std::remove_pointer_t<decltype(args.bpart)>;
        if (sw) {
            args.bpart = static_cast<T*>(sw->bpart);
            args.rpart = sw->rpart;
            args.gpart = sw->gpart;
            args.bagg = sw->bagg;
            args.st = sw->st;
        }
        return launch_sweep(args, h.plan.n_parts, h.plan.block_threads, size_t(h.plan.lds_bytes), h.stream, cooperative);
    };
    e = h.fp32 ? launch(sweep_args<float>(h)) : launch(sweep_args<double>(h));
    hip_check(e, "sweep launch");
    hip_check(hipEventRecord(h.ev1, h.stream), "event");
    hip_check(hipMemcpyAsync(h.last_pinned, sw ? sw->st : h.st.p, sizeof(SweepStatus), hipMemcpyDeviceToHost, h.stream),
              "download status");
    hip_check(hipEventRecord(h.done, h.stream), "event");
    h.in_flight = true;
}

bool problem_ready(const ldopf_problem& h) {
    if (!h.in_flight) return true;
    return hipEventQuery(h.done) == hipSuccess;
}

int problem_finish(ldopf_problem& h, ldopf_status* status) {
    if (!h.in_flight) fail(LDOPF_INVALID_ARGUMENT, "no solve in flight on this handle");
    h.in_flight = false;
    hip_check(hipEventSynchronize(h.done), "sweep");
    h.last = *h.last_pinned;
    const SweepStatus st = h.last;
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, h.ev0, h.ev1), "event time");
    h.last_sweep_ms = ms;
    h.phase_ms.assign(size_t(8) * std::max(h.plan.n_parts, 1), 0.0);
    if (h.opts.profile) {
        hip_check(hipMemcpy(h.phase_ms.data(), h.prof.p, h.phase_ms.size() * 8, hipMemcpyDeviceToHost),
                  "download phase times");
        for (double& t : h.phase_ms) t *= h.tick_ms;
    }
    h.hist_len = h.opts.history ? std::min<int64_t>(st.iters, int64_t(h.hist.count / 4)) : 0;
    if (st.iters > 0) h.have_x = true;
    if (st.flags & 1) fail(LDOPF_DEVICE_ERROR, "a cross-workgroup wait timed out in the sweep kernel");
    int code = LDOPF_OK;
    if (st.flags & 2) {
        code = LDOPF_NUMERICAL;
        record_error_detail("non-finite residual sums");
    } else if (h.opts.check_termination && !st.converged) {
        code = LDOPF_NOT_CONVERGED;
    }
    if (status) {
        status->iterations = st.iters;
        status->converged = st.converged;
        status->pres = st.pres;
        status->dres = st.dres;
        status->eps_prim = st.eps_p;
        status->eps_dual = st.eps_d;
        status->sweep_ms = ms;
        status->precompute_ms = h.precompute_ms;
        status->sweeps_computed = st.computed;
        status->rho = st.rho;
        status->rho_changes = st.rho_changes;
        status->code = code;
    }
    return code;
}

int64_t problem_device_bytes(const ConsensusLP& lp, const ldopf_options& o) {
    const int64_t S = lp.S, n = lp.n, nloc = int64_t(lp.gidx.size());
    int64_t nn = 0;
    for (int32_t v : lp.ns) nn += int64_t(v) * v;
    const int64_t hist = o.history ? std::min<int64_t>(std::max<int64_t>(o.max_iter, 1), int64_t(1) << 22) * 32 : 32;
    int64_t bytes = 8 * int64_t(lp.A.size() + lp.b.size()) + 8 * 2 * nn + 8 * nloc * 3 + 8 * n * 5 +
                    S * (4 * 4 + 8 * 4 + 32) + nloc * (4 + 2 * 4 + 4 * 4 + 1) + 2 * 8 * nloc * 4 +
                    int64_t(kRing) * kMaxParts * 64 + hist;
    return bytes + 48 * 4096;  // allocation granularity of about 48 buffers
}

int32_t problem_parts_estimate(const ConsensusLP& lp, const ldopf_options& o) {
    int dev = 0, cus = 256, lds = 163840;
    if (hipGetDevice(&dev) == hipSuccess) {
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipDeviceGetAttribute(&lds, hipDeviceAttributeSharedMemPerBlockOptin, dev);
    }
    std::vector<int32_t> rank(lp.S);
    for (int64_t s = 0; s < lp.S; ++s) rank[s] = std::min(lp.ms[s], lp.ns[s]);
    const Plan pl = make_plan(lp, rank, o.precision == LDOPF_FP32_MIXED, o.rows_per_part, o.block_threads, cus, lds);
    return pl.n_parts;
}

}  // namespace ldopf

extern "C" {

const char* ldopf_error_string(int code) {
    switch (code) {
        case LDOPF_OK: return "ok";
        case LDOPF_NOT_CONVERGED: return "not converged within max_iter";
        case LDOPF_INVALID_ARGUMENT: return "invalid argument";
        case LDOPF_INVALID_NETWORK: return "invalid network";
        case LDOPF_INFEASIBLE_BOUNDS: return "infeasible bounds";
        case LDOPF_INCONSISTENT_SUBSYSTEM: return "inconsistent subsystem";
        case LDOPF_OUT_OF_MEMORY: return "out of memory";
        case LDOPF_DEVICE_ERROR: return "device error";
        case LDOPF_NUMERICAL: return "numerical failure (NaN or Inf)";
        case LDOPF_BUFFER_TOO_SMALL: return "buffer too small";
        case LDOPF_UNSUPPORTED: return "unsupported";
        default: return "unknown code";
    }
}

const char* ldopf_last_error_detail(void) { return g_detail.c_str(); }

void ldopf_default_options(ldopf_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->rho = 100.0;
    o->eps_rel = 1e-4;
    o->eps_abs = 0.0;
    o->max_iter = 1000000;
    o->precision = LDOPF_FP64;
    o->residual_form = LDOPF_RESIDUAL_PAPER;
    o->check_termination = 1;
    o->history = 1;
    o->rho_update = LDOPF_RHO_FIXED;
    o->rho_period = 100;
    o->rho_max_changes = 16;
    o->rho_mu = 10.0;
    o->rho_tau = 2.0;
}

int ldopf_describe_network(const ldopf_network* net, int64_t sizes[5], double* c, double* lo, double* hi,
                           double* x_init, int32_t* n_s, int32_t* m_s, double* A, double* b, int64_t* gidx) {
    return guard([&] {
        need(net, "net");
        need(sizes, "sizes");
        ConsensusLP lp = assemble_network(*net);
        sizes[0] = lp.n;
        sizes[1] = lp.S;
        sizes[2] = int64_t(lp.gidx.size());
        sizes[3] = int64_t(lp.A.size());
        sizes[4] = int64_t(lp.b.size());
        auto put = [](auto* dst, const auto& v) {
            if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(v[0]));
        };
        put(c, lp.c);
        put(lo, lp.lo);
        put(hi, lp.hi);
        put(x_init, lp.x_init);
        put(n_s, lp.ns);
        put(m_s, lp.ms);
        put(A, lp.A);
        put(b, lp.b);
        put(gidx, lp.gidx);
    });
}

int ldopf_create(const ldopf_network* net, const ldopf_options* opts, void* stream, ldopf_problem** out) {
    return guard([&] {
        need(net, "net");
        need(out, "out");
        *out = nullptr;
        ConsensusLP lp = assemble_network(*net);
        ldopf_problem* h = new_problem(opts, stream);
        try {
            h->lp = std::move(lp);
            build_device(*h);
        } catch (...) {
            delete h;
            throw;
        }
        *out = h;
    });
}

int ldopf_create_lp(int64_t n, const double* c, const double* lo, const double* hi, const double* x_init,
                    int64_t n_sub, const int32_t* n_s, const int32_t* m_s, const double* A, const double* b,
                    const int64_t* gidx, const ldopf_options* opts, void* stream, ldopf_problem** out) {
    return guard([&] {
        need(out, "out");
        *out = nullptr;
        if (n < 1 || n_sub < 1) fail(LDOPF_INVALID_ARGUMENT, "n and n_sub must be >= 1");
        need(c, "c");
        need(lo, "lo");
        need(hi, "hi");
        need(n_s, "n_s");
        need(m_s, "m_s");
        need(gidx, "gidx");
        ConsensusLP lp;
        lp.n = n;
        lp.c.assign(c, c + n);
        lp.lo.assign(lo, lo + n);
        lp.hi.assign(hi, hi + n);
        if (x_init) lp.x_init.assign(x_init, x_init + n);
        lp.S = n_sub;
        lp.ns.assign(n_s, n_s + n_sub);
        lp.ms.assign(m_s, m_s + n_sub);
        int64_t nloc = 0, words = 0, rows = 0;
        for (int64_t s = 0; s < n_sub; ++s) {
            if (n_s[s] < 1 || m_s[s] < 0) fail(LDOPF_INVALID_ARGUMENT, "n_s must be >= 1 and m_s >= 0");
            nloc += n_s[s];
            rows += m_s[s];
            words += int64_t(n_s[s]) * m_s[s];
        }
        if (words > 0) need(A, "A");
        if (rows > 0) need(b, "b");
        if (words > 0) lp.A.assign(A, A + words);
        if (rows > 0) lp.b.assign(b, b + rows);
        lp.gidx.assign(gidx, gidx + nloc);
        finish_lp(lp);
        ldopf_problem* h = new_problem(opts, stream);
        try {
            h->lp = std::move(lp);
            build_device(*h);
        } catch (...) {
            delete h;
            throw;
        }
        *out = h;
    });
}

int ldopf_destroy(ldopf_problem* h) {
    return guard([&] { delete h; });
}

int ldopf_get_sizes(const ldopf_problem* h, ldopf_sizes* o) {
    return guard([&] {
        need(h, "handle");
        need(o, "out");
        std::memset(o, 0, sizeof(*o));
        o->n = h->lp.n;
        o->n_sub = h->lp.S;
        o->n_local = int64_t(h->lp.gidx.size());
        o->sum_m = int64_t(h->lp.b.size());
        int64_t ow = 0;
        int32_t mn = 0, mm = 0;
        for (int64_t s = 0; s < h->lp.S; ++s) {
            ow += int64_t(h->lp.ns[s]) * h->lp.ns[s];
            mn = std::max(mn, h->lp.ns[s]);
            mm = std::max(mm, h->lp.ms[s]);
        }
        o->op_words = ow;
        o->rank_words = h->plan.rank_words;
        o->max_n = mn;
        o->max_m = mm;
        o->n_parts = h->plan.n_parts;
        o->block_threads = h->plan.block_threads;
        o->lds_bytes = h->plan.lds_bytes;
        o->sync_bytes = h->streamed ? 0 : int64_t(problem_sync_bytes(*h));
        o->sweep_path = h->streamed ? LDOPF_PATH_STREAMED : LDOPF_PATH_PERSISTENT;
    });
}

int ldopf_set_options(ldopf_problem* h, const ldopf_options* opts) {
    return guard([&] {
        need(h, "handle");
        need(opts, "opts");
        check_options(*opts);
        if (opts->precision != h->opts.precision || opts->rows_per_part != h->opts.rows_per_part ||
            opts->block_threads != h->opts.block_threads || opts->sweep_path != h->opts.sweep_path)
            fail(LDOPF_INVALID_ARGUMENT, "precision, sweep path and tuning fields are fixed at creation");
        h->opts = *opts;
    });
}

int ldopf_solve(ldopf_problem* h, ldopf_status* status) {
    int code = LDOPF_OK;
    const int rc = guard([&] {
        need(h, "handle");
        problem_launch(*h);
        code = problem_finish(*h, status);
    });
    if (rc != LDOPF_OK && status) status->code = rc;
    return rc != LDOPF_OK ? rc : code;
}

namespace {
// One allocation-free solve at a time per GPU: they share its static array.
std::mutex g_noalloc_mu[kMaxDevices];

// Makes `dev` current for the scope of one call and restores the caller's.
struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev) {
        int cur = 0;
        hip_check(hipGetDevice(&cur), "hipGetDevice");
        if (cur != dev) {
            hip_check(hipSetDevice(dev), "hipSetDevice");
            prev = cur;
        }
    }
    ~DeviceScope() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
    DeviceScope(const DeviceScope&) = delete;
    DeviceScope& operator=(const DeviceScope&) = delete;
};
}  // namespace

int ldopf_solve_noalloc(ldopf_problem* h, ldopf_status* status) {
    int code = LDOPF_OK;
    const int rc = guard([&] {
        need(h, "handle");
        const size_t bytes = problem_sync_bytes(*h);
        if (bytes > kStaticScratchBytes)
            fail(LDOPF_OUT_OF_MEMORY, "the sweep needs " + std::to_string(bytes) + " bytes of synchronisation words; the static scratch holds " +
                                          std::to_string(kStaticScratchBytes));
        if (h->device < 0 || h->device >= kMaxDevices) fail(LDOPF_UNSUPPORTED, "device index out of range");
        DeviceScope scope(h->device);
        std::lock_guard<std::mutex> lock(g_noalloc_mu[h->device]);
        void* base = nullptr;
        hip_check(static_scratch(&base), "address of the static scratch");
        unsigned char* p = static_cast<unsigned char*>(base);
        const size_t P = size_t(std::max(h->plan.n_parts, 1));
        SyncWords sw{};
        sw.st = reinterpret_cast<SweepStatus*>(p);
        sw.gpart = reinterpret_cast<double*>(p + 256);
        sw.rpart = reinterpret_cast<double*>(p + 256 + size_t(kRing) * 8 * kGroup * 8);
        sw.bpart = p + 256 + size_t(kRing) * 8 * kGroup * 8 + size_t(kRing) * P * 64;
        const size_t w = h->fp32 ? 4 : 8;
        const size_t nb = (size_t(2) * size_t(std::max(h->plan.n_slots, 1)) * w + 255) & ~size_t(255);
        sw.bagg = agg_words(*h) ? reinterpret_cast<double*>(static_cast<unsigned char*>(sw.bpart) + nb) : nullptr;
        problem_launch(*h, &sw);
        code = problem_finish(*h, status);
    });
    if (rc != LDOPF_OK && status) status->code = rc;
    return rc != LDOPF_OK ? rc : code;
}

}  // extern "C"

namespace {

// One persistent launch for several problems (see ldopf_solve_many).
template <typename T>
void launch_many(const std::vector<ldopf_problem*>& hs, int block, size_t lds, hipStream_t stream) {
    std::vector<SweepArgs<T>> args;
    std::vector<int32_t> first{0};
    for (ldopf_problem* h : hs) {
        args.push_back(sweep_args<T>(*h));
        first.push_back(first.back() + h->plan.n_parts);
    }
    DevBuf<SweepArgs<T>> d_args;
    DevBuf<int32_t> d_first;
    d_args.upload(args, stream, "upload problems");
    d_first.upload(first, stream, "upload problems");
    for (ldopf_problem* h : hs) hip_check(hipEventRecord(h->ev0, stream), "event");
    hip_check(launch_sweep_many(args, d_args.p, d_first.p, first.back(), block, lds, stream), "sweep launch");
    for (ldopf_problem* h : hs) {
        hip_check(hipEventRecord(h->ev1, stream), "event");
        hip_check(hipMemcpyAsync(h->last_pinned, h->st.p, sizeof(SweepStatus), hipMemcpyDeviceToHost, stream),
                  "download status");
        hip_check(hipEventRecord(h->done, stream), "event");
        h->in_flight = true;
    }
    // the argument buffers are freed when they go out of scope: wait first
    hip_check(hipStreamSynchronize(stream), "sweep");
}

}  // namespace

extern "C" {

int ldopf_solve_many(ldopf_problem* const* hs, int32_t count, ldopf_status* statuses) {
    int worst = LDOPF_OK;
    const int rc = guard([&] {
        need(hs, "problems");
        if (count < 1 || count > 1024) fail(LDOPF_INVALID_ARGUMENT, "count must be in [1, 1024]");
        std::vector<ldopf_problem*> v(hs, hs + count);
        for (int32_t i = 0; i < count; ++i) {
            need(v[i], "problem");
            for (int32_t j = 0; j < i; ++j)
                if (v[j] == v[i]) fail(LDOPF_INVALID_ARGUMENT, "a problem appears twice");
            if (v[i]->in_flight) fail(LDOPF_INVALID_ARGUMENT, "a solve is already in flight on a problem");
            if (v[i]->streamed) fail(LDOPF_UNSUPPORTED, "a problem on the streamed sweep cannot share a launch");
            if (v[i]->fp32 != v[0]->fp32 || v[i]->opts.residual_form != v[0]->opts.residual_form ||
                v[i]->opts.profile != v[0]->opts.profile || v[i]->device != v[0]->device)
                fail(LDOPF_INVALID_ARGUMENT, "the problems must share precision, residual form, profiling and device");
        }
        DeviceScope scope(v[0]->device);
        // one launch size for all: the largest workgroup and LDS of any
        // problem; each problem's workgroups run with their own size
        int block = 0;
        int64_t blocks = 0;
        size_t lds = 0;
        for (ldopf_problem* h : v) {
            block = std::max(block, h->plan.block_threads);
            blocks += h->plan.n_parts;
            lds = std::max<size_t>(lds, size_t(h->plan.lds_bytes));
        }
        int lds_optin = 0, cus = 0;
        hip_check(hipDeviceGetAttribute(&lds_optin, hipDeviceAttributeSharedMemPerBlockOptin, v[0]->device), "device attribute");
        hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, v[0]->device), "device attribute");
        if (lds > size_t(lds_optin)) fail(LDOPF_UNSUPPORTED, "the problems' workgroups need more LDS together than a workgroup has");
        hip_check(prepare_sweep(v[0]->fp32, lds), "sweep LDS attribute");
        int per_cu = 0;
        hip_check(sweep_many_occupancy(v[0]->fp32, block, lds, &per_cu), "sweep occupancy");
        if (int64_t(per_cu) * cus < blocks)
            fail(LDOPF_UNSUPPORTED, "the problems' " + std::to_string(blocks) + " workgroups cannot be resident together (" +
                                        std::to_string(per_cu) + " per CU); solve them in smaller groups");
        for (ldopf_problem* h : v) {
            hip_check(hipStreamSynchronize(h->stream), "earlier work of a problem");
            const int64_t want = h->opts.history ? std::min<int64_t>(std::max<int64_t>(h->opts.max_iter, 1), int64_t(1) << 22) : 1;
            if (int64_t(h->hist.count) < want * 4) h->hist.alloc(size_t(want) * 4, "history");
            if (h->bagg.count < agg_words(*h)) h->bagg.alloc(agg_words(*h), "aggregated residual words");
        }
        if (v[0]->fp32)
            launch_many<float>(v, block, lds, v[0]->stream);
        else
            launch_many<double>(v, block, lds, v[0]->stream);
        for (int32_t i = 0; i < count; ++i) {
            const int code = problem_finish(*v[i], statuses ? &statuses[i] : nullptr);
            if (code < 0 && (worst >= 0 || code < worst)) worst = code;
            if (code > 0 && worst == LDOPF_OK) worst = code;
        }
    });
    return rc != LDOPF_OK ? rc : worst;
}

int ldopf_reset(ldopf_problem* h) {
    return guard([&] {
        need(h, "handle");
        init_state(*h);
    });
}

int ldopf_warm_start(ldopf_problem* h, const double* xs, const double* lam, int64_t n_local) {
    return guard([&] {
        need(h, "handle");
        need(xs, "xs");
        need(lam, "lam");
        if (n_local != int64_t(h->lp.gidx.size())) fail(LDOPF_INVALID_ARGUMENT, "n_local does not match the problem");
        for (int64_t k = 0; k < n_local; ++k)
            if (!std::isfinite(xs[k]) || !std::isfinite(lam[k]))
                fail(LDOPF_NUMERICAL, "non-finite warm-start value at local copy " + std::to_string(k));
        hip_check(hipMemcpyAsync(h->xs.p, xs, n_local * 8, hipMemcpyHostToDevice, h->stream), "upload x_s");
        hip_check(hipMemcpyAsync(h->lam.p, lam, n_local * 8, hipMemcpyHostToDevice, h->stream), "upload lambda");
        hip_check(hipStreamSynchronize(h->stream), "warm start");
        h->hist_len = 0;
    });
}

int ldopf_get_global(const ldopf_problem* h, double* x, int64_t cap) {
    return guard([&] {
        need(h, "handle");
        need(x, "x");
        if (cap < h->lp.n) fail(LDOPF_BUFFER_TOO_SMALL, "x needs n entries");
        hip_check(hipMemcpyAsync(x, h->x.p, h->lp.n * 8, hipMemcpyDeviceToHost, h->stream), "download x");
        hip_check(hipStreamSynchronize(h->stream), "download x");
    });
}

int ldopf_get_local(const ldopf_problem* h, double* xs, double* lam, int64_t cap) {
    return guard([&] {
        need(h, "handle");
        const int64_t nl = int64_t(h->lp.gidx.size());
        if (cap < nl) fail(LDOPF_BUFFER_TOO_SMALL, "x_s and lambda need N_loc entries");
        if (xs) hip_check(hipMemcpyAsync(xs, h->xs.p, nl * 8, hipMemcpyDeviceToHost, h->stream), "download x_s");
        if (lam) hip_check(hipMemcpyAsync(lam, h->lam.p, nl * 8, hipMemcpyDeviceToHost, h->stream), "download lambda");
        hip_check(hipStreamSynchronize(h->stream), "download state");
    });
}

int ldopf_get_structure(const ldopf_problem* h, int64_t* gidx, int64_t cap_local, int64_t* sub_off, int64_t cap_sub) {
    return guard([&] {
        need(h, "handle");
        if (gidx) {
            if (cap_local < int64_t(h->lp.gidx.size())) fail(LDOPF_BUFFER_TOO_SMALL, "gidx needs N_loc entries");
            std::memcpy(gidx, h->lp.gidx.data(), h->lp.gidx.size() * 8);
        }
        if (sub_off) {
            if (cap_sub < h->lp.S + 1) fail(LDOPF_BUFFER_TOO_SMALL, "sub_off needs S + 1 entries");
            std::memcpy(sub_off, h->lp.loc_off.data(), (h->lp.S + 1) * 8);
        }
    });
}

int ldopf_get_history(const ldopf_problem* h, double* hist, int64_t cap_rows, int64_t* len) {
    return guard([&] {
        need(h, "handle");
        need(len, "len");
        *len = h->hist_len;
        if (!hist) return;
        if (cap_rows < h->hist_len) fail(LDOPF_BUFFER_TOO_SMALL, "history needs len rows");
        if (h->hist_len > 0) {
            hip_check(hipMemcpyAsync(hist, h->hist.p, h->hist_len * 4 * 8, hipMemcpyDeviceToHost, h->stream), "download history");
            hip_check(hipStreamSynchronize(h->stream), "download history");
        }
    });
}

int ldopf_get_operators(const ldopf_problem* h, double* abar, int64_t cap_abar, double* bbar, int64_t cap_bbar,
                        int32_t* rank, int64_t cap_rank) {
    return guard([&] {
        need(h, "handle");
        const int64_t words = int64_t(h->abar.count);
        const int64_t nl = int64_t(h->lp.gidx.size());
        if (abar) {
            if (cap_abar < words) fail(LDOPF_BUFFER_TOO_SMALL, "abar needs op_words entries");
            hip_check(hipMemcpyAsync(abar, h->abar.p, words * 8, hipMemcpyDeviceToHost, h->stream), "download abar");
        }
        if (bbar) {
            if (cap_bbar < nl) fail(LDOPF_BUFFER_TOO_SMALL, "bbar needs N_loc entries");
            hip_check(hipMemcpyAsync(bbar, h->bbar.p, nl * 8, hipMemcpyDeviceToHost, h->stream), "download bbar");
        }
        if (rank) {
            if (cap_rank < h->lp.S) fail(LDOPF_BUFFER_TOO_SMALL, "rank needs S entries");
            std::memcpy(rank, h->rank.data(), h->lp.S * 4);
        }
        hip_check(hipStreamSynchronize(h->stream), "download operators");
    });
}

int ldopf_get_rho_log(const ldopf_problem* h, int64_t* sweeps, double* rhos, int64_t cap, int64_t* len) {
    return guard([&] {
        need(h, "handle");
        need(len, "len");
        const int64_t n = std::min<int64_t>(h->last.rho_changes, kMaxRhoChanges);
        *len = n;
        const int64_t k = std::min(n, std::max<int64_t>(cap, 0));
        if (k == 0 || (!sweeps && !rhos)) return;
        std::vector<double> log(size_t(2) * k);
        hip_check(hipMemcpyAsync(log.data(), h->rholog.p, log.size() * 8, hipMemcpyDeviceToHost, h->stream), "download rho log");
        hip_check(hipStreamSynchronize(h->stream), "download rho log");
        for (int64_t i = 0; i < k; ++i) {
            if (sweeps) sweeps[i] = int64_t(log[2 * i]);
            if (rhos) rhos[i] = log[2 * i + 1];
        }
    });
}

int ldopf_get_phase_times(const ldopf_problem* h, double* ms) {
    return ldopf_get_phase_times_part(h, 0, ms);
}

int ldopf_get_phase_times_part(const ldopf_problem* h, int32_t part, double* ms) {
    return guard([&] {
        need(h, "handle");
        need(ms, "ms");
        if (part < 0 || part >= std::max(h->plan.n_parts, 1)) fail(LDOPF_INVALID_ARGUMENT, "part out of range");
        for (int i = 0; i < 8; ++i)
            ms[i] = size_t(part) * 8 + i < h->phase_ms.size() ? h->phase_ms[size_t(part) * 8 + i] : 0.0;
    });
}

int ldopf_objective(const ldopf_problem* h, double* f) {
    return guard([&] {
        need(h, "handle");
        need(f, "f");
        std::vector<double> x(h->lp.n);
        hip_check(hipMemcpyAsync(x.data(), h->x.p, h->lp.n * 8, hipMemcpyDeviceToHost, h->stream), "download x");
        hip_check(hipStreamSynchronize(h->stream), "download x");
        double acc = 0.0;
        for (int64_t g = 0; g < h->lp.n; ++g) acc += h->lp.c[g] * x[g];
        *f = acc;
    });
}

int ldopf_get_global_device(const ldopf_problem* h, double* x_device, int64_t cap) {
    return guard([&] {
        need(h, "handle");
        need(x_device, "x_device");
        if (cap < h->lp.n) fail(LDOPF_BUFFER_TOO_SMALL, "x needs n entries");
        hip_check(hipMemcpyAsync(x_device, h->x.p, h->lp.n * 8, hipMemcpyDeviceToDevice, h->stream), "copy x");
    });
}

int ldopf_get_local_device(const ldopf_problem* h, double* xs_device, double* lam_device, int64_t cap) {
    return guard([&] {
        need(h, "handle");
        const int64_t nl = int64_t(h->lp.gidx.size());
        if (cap < nl) fail(LDOPF_BUFFER_TOO_SMALL, "x_s and lambda need N_loc entries");
        if (xs_device) hip_check(hipMemcpyAsync(xs_device, h->xs.p, nl * 8, hipMemcpyDeviceToDevice, h->stream), "copy x_s");
        if (lam_device) hip_check(hipMemcpyAsync(lam_device, h->lam.p, nl * 8, hipMemcpyDeviceToDevice, h->stream), "copy lambda");
    });
}

}  // extern "C"
