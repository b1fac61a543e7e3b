// The problem handle of the plain solver and the internal calls the serving
// runtime shares with the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "device.h"
#include "host_util.h"
#include "internal.h"

// The C ABI names its handle at global scope; its members are library types.
using ldopf::ConsensusLP;
using ldopf::DevBuf;
using ldopf::PartInfo;
using ldopf::Plan;
using ldopf::SubMeta;
using ldopf::SweepStatus;

struct ldopf_problem {
    SweepStatus last{};  // status read back by the last finished solve
    // pinned host word the solve's status is copied into: a copy into
    // pageable memory would block the launching thread until the sweep ends
    SweepStatus* last_pinned = nullptr;
    bool own_pinned = false;
    bool in_flight = false;
    ConsensusLP lp;
    ldopf_options opts{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;  // the GPU the handle's buffers live on
    hipEvent_t ev0 = nullptr, ev1 = nullptr, done = nullptr;
    bool fp32 = false;
    Plan plan;
    std::vector<int32_t> rank;
    double precompute_ms = 0.0;
    double last_sweep_ms = 0.0;
    int64_t hist_len = 0;
    bool have_x = false;
    uint64_t spin_limit = 0;

    DevBuf<double> A, b, basis, abar, bbar, c, lo, hi, cnt, xs, lam, x, hist, rpart, gpart, prof;
    DevBuf<double> rholog;  // [kMaxRhoChanges][2] residual-balancing changes of the last solve
    DevBuf<double> bagg;    // aggregated residual form: boundary words (allocated at the first such solve)
    std::vector<double> phase_ms;  // [parts][8] per-phase ms of the last profiled solve
    double tick_ms = 1e-5;  // wall-clock tick in ms
    DevBuf<int32_t> ns, ms, rank_d, flags;
    DevBuf<int64_t> a_off, row_off, loc_off, basis_off;
    DevBuf<PartInfo> parts;
    DevBuf<SubMeta> subs;
    DevBuf<int32_t> row_canon, var_gid, var_slot, var_slot_lo, var_slot_hi;
    DevBuf<uint16_t> row_lvar, row_sub, var_copy_off, var_copy_rows, tk_sub;
    DevBuf<uint8_t> var_writer;
    DevBuf<unsigned char> bpart;
    DevBuf<SweepStatus> st;
    // streamed sweep (a problem too large for the persistent sweep's LDS):
    // groups of subsystems with their words, copies as 32-bit indices, the
    // copies of each variable (CSR, and the first four padded), the blocks'
    // residual rows, control words, the graph
    bool streamed = false;
    int32_t s_nq = 1;
    int64_t s_n_groups = 0;
    DevBuf<int64_t> s_ctrl;
    DevBuf<int32_t> s_gidx, s_var_off, s_var_copy, s_groups;
    DevBuf<int4> s_ell;  // the first four copies of each variable
    DevBuf<double4> s_vconst;  // each variable's c, bounds and copy count
    DevBuf<double> s_part, s_x2, s_u2, s_lam2;
    hipGraph_t s_graph = nullptr;
    hipGraphExec_t s_exec = nullptr;
    int64_t* s_hctrl = nullptr;                 // pinned: the control words after two graphs
    hipEvent_t s_evc[2] = {nullptr, nullptr};  // recorded after each of those reads

    // every device buffer allocated and released in order on `s` (the
    // serving runtime's slot streams, which outlive their problems)
    void use_stream_ordered_memory(hipStream_t s) {
        for (DevBuf<double>* q : {&A, &b, &basis, &abar, &bbar, &c, &lo, &hi, &cnt, &xs, &lam, &x, &hist, &rpart, &gpart,
                                  &prof, &rholog, &bagg, &s_part, &s_x2, &s_u2, &s_lam2})
            q->ordered = s;
        for (DevBuf<int32_t>* q : {&ns, &ms, &rank_d, &flags, &row_canon, &var_gid, &var_slot, &var_slot_lo, &var_slot_hi,
                                   &s_gidx, &s_var_off, &s_var_copy, &s_groups})
            q->ordered = s;
        for (DevBuf<int64_t>* q : {&a_off, &row_off, &loc_off, &basis_off, &s_ctrl}) q->ordered = s;
        for (DevBuf<uint16_t>* q : {&row_lvar, &row_sub, &var_copy_off, &var_copy_rows, &tk_sub}) q->ordered = s;
        parts.ordered = s;
        subs.ordered = s;
        s_ell.ordered = s;
        s_vconst.ordered = s;
        var_writer.ordered = s;
        bpart.ordered = s;
        st.ordered = s;
    }

    ~ldopf_problem() {
        if (stream) (void)hipStreamSynchronize(stream);
        if (s_exec) (void)hipGraphExecDestroy(s_exec);
        if (s_graph) (void)hipGraphDestroy(s_graph);
        if (s_hctrl) (void)hipHostFree(s_hctrl);
        for (hipEvent_t e : s_evc)
            if (e) (void)hipEventDestroy(e);
        if (own_pinned && last_pinned) (void)hipHostFree(last_pinned);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        if (done) (void)hipEventDestroy(done);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};


namespace ldopf {

// Host LP -> handle with operators precomputed on the device (throws). With
// ordered_memory, every device buffer is allocated and freed in order on
// `stream`, which must outlive the handle.
ldopf_problem* problem_create(ConsensusLP&& lp, const ldopf_options& opts, hipStream_t stream,
                              bool ordered_memory = false, SweepStatus* pinned_status = nullptr);
// Where the sweep's synchronisation words live: the handle's own buffers,
// or (allocation-free solve) carved from the static scratch array.
struct SyncWords {
    void* bpart;
    double* rpart;
    double* gpart;
    double* bagg;  // null unless the aggregated residual form is selected
    SweepStatus* st;
};
// Device bytes of the synchronisation words of the handle's sweep.
size_t problem_sync_bytes(const ldopf_problem& h);
// Enqueue one solve (from the current state) on the handle's stream. With
// sw, the sweep uses those words and nothing is allocated (the history goes
// only into the buffer the handle already holds). cooperative = false only
// where the caller's admission keeps every workgroup resident (serving).
void problem_launch(ldopf_problem& h, const SyncWords* sw = nullptr, bool cooperative = true);
// True when the enqueued solve has finished on the device.
bool problem_ready(const ldopf_problem& h);
// Wait for the enqueued solve, read its status; returns the ldopf_code.
int problem_finish(ldopf_problem& h, ldopf_status* status);
// Streamed sweep: device tables of a problem whose precompute is done
// (switches the handle to that path), and one whole solve, enqueued and
// waited for on the handle's stream (throws).
void stream_prepare(ldopf_problem& h);
void stream_solve(ldopf_problem& h);
// Device bytes a problem allocates at its peak (creation plus one solve).
int64_t problem_device_bytes(const ConsensusLP& lp, const ldopf_options& opts);
// Workgroups of its sweep, planned on the host assuming full row rank.
int32_t problem_parts_estimate(const ConsensusLP& lp, const ldopf_options& opts);

}  // namespace ldopf
