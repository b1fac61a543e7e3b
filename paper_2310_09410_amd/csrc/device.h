// Argument blocks and launchers of the device kernels (see device.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "internal.h"

namespace ldopf {

struct PrecomputeArgs {
    int64_t S;
    const int32_t* ns;
    const int32_t* ms;
    const int64_t* a_off;      // words of A before subsystem s
    const int64_t* row_off;    // rows (entries of b) before s
    const int64_t* loc_off;    // copies before s
    const int64_t* basis_off;  // n_s * n_s words before s
    const double* A;
    const double* b;
    double* basis;  // out: n_s x n_s orthonormal rows, row space first
    double* abar;   // out: dense Abar_s, row-major
    double* bbar;   // out: per copy
    int32_t* rank;  // out
    int32_t* flags; // out: 1 = inconsistent dependent row
    double tol_dep; // a row is dependent when its residual norm is below tol_dep * its norm
    double tol_rhs; // ... and then its right-hand side must be below tol_rhs * (1 + max |b_s|)
    int32_t max_n;  // largest n_s (selects the kernel's columns per lane)
};

// Residual sums of the last kRing sweeps: every part's ([kRing][8][P]
// doubles, quantity-major), emptied by its group leader once read, and the
// sums of each group of kGroup consecutive parts ([kRing][8][kGroup]),
// emptied by the leader once every part has read them.
constexpr int kRing = 8;
constexpr int kGroup = 16;
// Parts the sweep can run: kGroup groups of kGroup parts.
constexpr int kMaxParts = kGroup * kGroup;

// Residual balancing: a change of rho decided from the test of sweep t is
// used from sweep t + kRhoLag on (the test of sweep t is read during sweep
// t + 3, and the partial sums published in that sweep already feed sweep
// t + 4's global update).
constexpr int kRhoLag = 4;
constexpr int kMaxRhoChanges = 1024;

struct SweepStatus {
    int64_t iters;     // sweep whose state is returned
    int64_t computed;  // sweeps computed (the test of a sweep is read during the next one)
    int32_t converged;
    int32_t flags;  // 1: an exchange wait timed out, 2: non-finite residuals
    double pres, dres, eps_p, eps_d;
    double rho;           // rho of the returned sweep
    int64_t rho_changes;  // changes made by residual balancing
};

template <typename T>
struct SweepArgs {
    const PartInfo* parts;
    const SubMeta* subs;
    const int32_t* row_canon;
    const uint16_t* row_lvar;
    const uint16_t* row_sub;
    const int32_t* var_gid;
    const int32_t* var_slot;
    const int32_t* var_slot_lo;
    const int32_t* var_slot_hi;
    const uint8_t* var_writer;
    const uint16_t* var_copy_off;
    const uint16_t* var_copy_rows;
    const uint16_t* tk_sub;
    const double* basis;
    const double* bbar;  // per copy, canonical order
    const double* c;
    const double* lo;
    const double* hi;
    const double* cnt;   // copies per global variable
    double* xs;          // state in and out, canonical copy order
    double* lam;
    double* x;           // global x out
    T* bpart;            // [2][n_slots] boundary partial sums, one word per (var, writer, reader)
    double* rpart;       // [kRing][8][P] residual partial sums
    double* gpart;       // [kRing][8][kGroup] residual sums per group of parts
    double* hist;        // [hist_cap][4]
    int64_t hist_cap;
    SweepStatus* st;
    double rho, eps_rel, eps_abs;
    int64_t max_iter;
    int64_t nloc;
    int64_t n;           // global variables (dimension of the aggregated dual residual)
    int64_t n_slots;
    int32_t check;
    int32_t P;
    int32_t block;       // threads of the problem's workgroups (a multiple of 64, at most the launch's)
    uint64_t spin_limit; // wall-clock ticks an exchange wait may take
    double* prof;        // nullable: per-phase wall-clock ticks of every workgroup ([P][8])
    // residual balancing of rho (rho_update != 0)
    int32_t rho_update, rho_period, rho_max_changes;
    double rho_mu, rho_tau;
    double* rho_log;     // [rho_max_changes][2]: first sweep, rho (written by workgroup 0)
    // aggregated residual form: boundary variables' per-owner sums of
    // rho (x_s - x_s_prev) and of lambda over their copies, sent to owner 0
    // ([2 parities][2 quantities][n_slots] doubles); null in the paper form
    double* bagg;
};

// Device memory of the allocation-free solve: the sweep's exchange words,
// residual rings and status word come from one static array per GPU instead
// of buffers of the handle. static_scratch gives its address on the current
// device (looked up once per device, then remembered).
constexpr size_t kStaticScratchBytes = size_t(4) << 20;
constexpr int kMaxDevices = 64;
hipError_t static_scratch(void** ptr);

hipError_t launch_precompute(const PrecomputeArgs& a, hipStream_t stream);
hipError_t prepare_sweep(bool fp32, size_t lds_bytes);
hipError_t sweep_occupancy(bool fp32, int block, size_t lds_bytes, int* blocks_per_cu);
// cooperative: the runtime guarantees that every workgroup is resident at
// once (cooperative launches share one hardware queue, so they run one after
// another); otherwise the caller guarantees it by admission (the serving
// runtime counts compute units per XCD), and the sweeps of several problems
// can run side by side. Either way a wait that cannot end is cut by the
// bounded exchange waits (LDOPF_DEVICE_ERROR), not left to hang.
hipError_t launch_sweep(const SweepArgs<double>& a, int grid, int block, size_t lds, hipStream_t stream,
                        bool cooperative);
hipError_t launch_sweep(const SweepArgs<float>& a, int grid, int block, size_t lds, hipStream_t stream,
                        bool cooperative);
// Several problems in one cooperative launch (sweep_many_kernel): host
// copies of their arguments (for the per-problem resets), the same in device
// memory, and the first block of each problem plus the total (count + 1).
hipError_t sweep_many_occupancy(bool fp32, int block, size_t lds_bytes, int* blocks_per_cu);
hipError_t launch_sweep_many(const std::vector<SweepArgs<double>>& a, const SweepArgs<double>* dev_args,
                             const int32_t* dev_first, int total_blocks, int block, size_t lds, hipStream_t stream);
hipError_t launch_sweep_many(const std::vector<SweepArgs<float>>& a, const SweepArgs<float>* dev_args,
                             const int32_t* dev_first, int total_blocks, int block, size_t lds, hipStream_t stream);

}  // namespace ldopf
