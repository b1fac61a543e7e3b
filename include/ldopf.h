/*
 * ldopf.h - C ABI of the MI355X (gfx950) closed-form ADMM solver for
 * linearized multi-phase unbalanced optimal power flow.
 *
 * The method (Ryu, Byeon, Kim, "A GPU-based Distributed Algorithm for
 * Linearized Optimal Power Flow in Distribution Systems", PSCC 2024):
 *   - Section II-A builds the LP  min c'x  s.t.  A x = b,  lo <= x <= hi
 *     (LP_model) from the network: operational bounds, power balance, the
 *     voltage-dependent load model, the linearized power flow and the
 *     objective "sum of generator real power".
 *   - Section III-A rewrites it as the consensus model OurModel: every
 *     subsystem s keeps its rows A_s x_s = b_s, a 0-1 matrix B_s selects its
 *     copies x_s = B_s x of the global variables, and the bounds act only on
 *     the global vector x.
 *   - Section III-B gives both ADMM blocks in closed form: the global update
 *     closed_1 (a clipped average of the copies), the local update closed_2
 *     (x_s = (1/rho) Abar_s d_s + bbar_s with Abar_s, bbar_s precomputed
 *     once), and the dual update ADMM-3.
 *   - Section III-C is the termination test; Algorithm 1 is the whole loop;
 *     Section V-A gives the decomposition (one subsystem per line and per
 *     bus, each leaf bus merged into its line), the defaults rho = 100 and
 *     the initial point.
 *
 * Conventions for every call:
 *   - Host pointers unless a name ends in _device. Inputs are read during the
 *     call and copied; the library never keeps a caller pointer.
 *   - Output buffers are caller-allocated; each getter takes a capacity and
 *     fails with LDOPF_BUFFER_TOO_SMALL (writing nothing) when it is short.
 *     Sizes come from ldopf_get_sizes.
 *   - Return value: an ldopf_code. ldopf_last_error_detail() gives a message
 *     for the most recent failure on the calling thread.
 *   - A problem handle is used by one host thread at a time.
 *   - All device work of a handle runs on the HIP stream given at creation
 *     (NULL: a stream the library creates at default priority).
 *
 * Orderings shared by inputs and outputs:
 *   - Global variables x follow the block order of LP_model: generators
 *     (p^g, q^g per phase), squared voltages w (per bus, per phase), loads
 *     (p^b, q^b, p^d, q^d per phase), line flows (p_ij, q_ij, p_ji, q_ji per
 *     phase); components in input order, phases ascending (a, b, c).
 *   - Subsystems: one per line in line order (a leaf end bus merged into it),
 *     then one per non-leaf bus in bus order. A leaf is a non-root bus with
 *     exactly one incident line.
 *   - Local copies: subsystem by subsystem, each subsystem's copies sorted by
 *     global index (gidx ascending).
 *   - Rows of a line subsystem: per line phase, the two loss rows and the
 *     voltage-drop row; then, per merged leaf bus, its balance rows (real,
 *     reactive per phase) and its loads' rows. A bus subsystem: its balance
 *     rows, then its loads' rows. Wye load rows per phase: p^d model, q^d
 *     model, p^b = p^d, q^b = q^d. Delta load rows: the three p^d model rows,
 *     the three q^d model rows, the two sum rows, the four coupling rows.
 */
#ifndef LDOPF_H
#define LDOPF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LDOPF_API __attribute__((visibility("default")))

typedef enum ldopf_code {
    LDOPF_OK = 0,
    LDOPF_NOT_CONVERGED = 1,           /* max_iter reached; results are valid */
    LDOPF_INVALID_ARGUMENT = -1,       /* null pointer, bad size or option */
    LDOPF_INVALID_NETWORK = -2,        /* index out of range, bad phase set, NaN data */
    LDOPF_INFEASIBLE_BOUNDS = -3,      /* a lower bound above its upper bound */
    LDOPF_INCONSISTENT_SUBSYSTEM = -4, /* rank-deficient A_s with b_s outside its range */
    LDOPF_OUT_OF_MEMORY = -5,          /* device allocation failed */
    LDOPF_DEVICE_ERROR = -6,           /* a HIP call or kernel failed */
    LDOPF_NUMERICAL = -7,              /* NaN or Inf in the iterate or residuals */
    LDOPF_BUFFER_TOO_SMALL = -8,       /* output capacity below the needed size */
    LDOPF_UNSUPPORTED = -9             /* valid request this library does not run */
} ldopf_code;

typedef enum ldopf_precision {
    /* every step in FP64 */
    LDOPF_FP64 = 0,
    /* global, local and dual updates in FP32 on FP32 copies of the operators;
     * operator precompute, residual norms and the termination test in FP64 */
    LDOPF_FP32_MIXED = 1
} ldopf_precision;

typedef enum ldopf_residual_form {
    /* Section III-C taken literally: dres = rho * ||x_s - x_s_prev|| and
     * eps_dual = eps_rel * ||lambda|| over all local copies */
    LDOPF_RESIDUAL_PAPER = 0,
    /* textbook form with sum_s B_s' applied before the norm: per global
     * variable the sums over its copies, dres = rho * ||sum_s B_s' (x_s -
     * x_s_prev)||, eps_dual = eps_rel * ||sum_s B_s' lambda_s|| (and
     * sqrt(n) * eps_abs instead of sqrt(N_loc) * eps_abs) */
    LDOPF_RESIDUAL_AGGREGATED = 1
} ldopf_residual_form;

typedef enum ldopf_rho_update {
    /* rho fixed for the whole solve (Algorithm 1) */
    LDOPF_RHO_FIXED = 0,
    /* residual balancing (one of the acceleration schemes Section III-D
     * names; rule of He et al. 2000 / Boyd et al. 2011 on relative
     * residuals as in Wohlberg 2017): after every sweep t that is a multiple
     * of rho_period, with r = pres / eps_prim and s = dres / eps_dual,
     * rho is multiplied by rho_tau if r > rho_mu * s and divided by it if
     * s > rho_mu * r; the new rho is used from sweep t + 4 on; at most
     * rho_max_changes changes. lambda (unscaled) is kept; Abar_s and bbar_s
     * do not depend on rho, so nothing is recomputed. */
    LDOPF_RHO_BALANCE = 1
} ldopf_rho_update;

typedef enum ldopf_sweep_path {
    /* the persistent sweep when its workgroups (one per CU) hold the
     * problem's operators and state in LDS, else the streamed sweep */
    LDOPF_PATH_AUTO = 0,
    /* the persistent sweep only: one cooperative launch per solve, operators
     * and state in LDS for the whole solve; LDOPF_UNSUPPORTED if they do not
     * fit */
    LDOPF_PATH_PERSISTENT = 1,
    /* the streamed sweep: the same steps of Algorithm 1 with the operators
     * and state in HBM, one launch per sweep (global, local and dual update
     * with the residual sums of each block, and beside them the test of the
     * previous sweep on those sums in a fixed order), captured in HIP graphs
     * and replayed by the host until the test holds. It keeps lambda and
     * x_s - lambda / rho per copy; the x_s it returns is formed from the two
     * (a warm start from it reproduces the state up to one rounding). FP64 only, literal residual form and fixed rho;
     * not for ldopf_solve_noalloc, ldopf_solve_many or the server (those
     * calls return LDOPF_UNSUPPORTED for such a problem) */
    LDOPF_PATH_STREAMED = 2
} ldopf_sweep_path;

/*
 * Network data (nomenclature table of Section II). Structure of arrays,
 * caller-owned, copied by ldopf_create. Per-phase arrays are [count x 3]
 * row-major with columns a, b, c; 3x3 matrices are [count x 9] row-major.
 * Phase sets are bitmasks a=1, b=2, c=4. Entries for phases a component does
 * not carry are ignored. Pointers marked "nullable" take the stated default.
 */
typedef struct ldopf_network {
    int32_t n_bus, n_line, n_load, n_gen;
    int32_t root;                 /* substation bus (never a leaf) */
    const uint8_t* bus_phases;    /* [n_bus] */
    const double* bus_wlo;        /* [n_bus x 3] squared-voltage bounds; nullable: -inf */
    const double* bus_whi;        /* nullable: +inf */
    const double* bus_gsh;        /* shunt conductance g^sh; nullable: 0 */
    const double* bus_bsh;        /* shunt susceptance b^sh; nullable: 0 */
    const int32_t* line_from;     /* [n_line] bus i of line (e, i, j) */
    const int32_t* line_to;       /* [n_line] bus j */
    const uint8_t* line_phases;   /* [n_line], subset of both end buses' phases */
    const double* line_r;         /* [n_line x 9] series resistance, per unit */
    const double* line_x;         /* [n_line x 9] series reactance, per unit */
    const double* line_gs_from;   /* [n_line x 3] g^s at the i end; nullable: 0 */
    const double* line_bs_from;   /* b^s at the i end; nullable: 0 */
    const double* line_gs_to;     /* g^s at the j end; nullable: 0 */
    const double* line_bs_to;     /* b^s at the j end; nullable: 0 */
    const double* line_tau;       /* [n_line x 3] tap ratio; nullable: 1 */
    const double* line_plo;       /* [n_line x 3] bounds on p at both ends; nullable: -inf */
    const double* line_phi;       /* nullable: +inf */
    const double* line_qlo;       /* bounds on q at both ends; nullable: -inf */
    const double* line_qhi;       /* nullable: +inf */
    const int32_t* load_bus;      /* [n_load] */
    const uint8_t* load_phases;   /* [n_load], subset of the bus's phases */
    const uint8_t* load_conn;     /* [n_load] 0 wye, 1 delta (three-phase only); nullable: wye */
    const double* load_a;         /* [n_load x 3] reference real power a */
    const double* load_b;         /* reference reactive power b */
    const double* load_alpha;     /* load-type exponent alpha; nullable: 0 */
    const double* load_beta;      /* load-type exponent beta; nullable: 0 */
    const int32_t* gen_bus;       /* [n_gen] */
    const uint8_t* gen_phases;    /* [n_gen], subset of the bus's phases */
    const double* gen_plo;        /* [n_gen x 3]; nullable: -inf */
    const double* gen_phi;        /* nullable: +inf */
    const double* gen_qlo;        /* nullable: -inf */
    const double* gen_qhi;        /* nullable: +inf */
    const double* gen_cost_p;     /* objective coefficient of p^g; nullable: 1 */
    const double* gen_cost_q;     /* objective coefficient of q^g; nullable: 0 */
} ldopf_network;

typedef struct ldopf_options {
    double rho;              /* penalty of the augmented Lagrangian; default 100 (Section V-A) */
    double eps_rel;          /* relative tolerance of the termination test; default 1e-4 */
    double eps_abs;          /* absolute term sqrt(dim) * eps_abs added to both tolerances; default 0 */
    int64_t max_iter;        /* sweep limit; default 1e6 */
    int32_t precision;       /* ldopf_precision; default LDOPF_FP64 */
    int32_t residual_form;   /* ldopf_residual_form; default LDOPF_RESIDUAL_PAPER */
    int32_t check_termination; /* 1 (default): stop at the test; 0: run exactly max_iter sweeps */
    int32_t history;         /* 1 (default): record pres, dres, eps_prim, eps_dual per sweep */
    int32_t rows_per_part;   /* tuning: local copies per workgroup; 0 = automatic */
    int32_t block_threads;   /* tuning: threads per workgroup (128..1024, multiple of 64: row waves plus the
                                wave that runs the termination test); 0 = automatic */
    int32_t profile;         /* 1: record per-phase device time of the sweep (ldopf_get_phase_times); default 0 */
    int32_t rho_update;      /* ldopf_rho_update; default LDOPF_RHO_FIXED */
    int32_t rho_period;      /* residual balancing: sweeps between evaluations of the rule (>= 4); default 100 */
    int32_t rho_max_changes; /* residual balancing: changes at most (0..1024); default 16 */
    int32_t sweep_path;      /* ldopf_sweep_path; default LDOPF_PATH_AUTO */
    int32_t reserved;        /* must be zero */
    double rho_mu;           /* residual balancing: imbalance that triggers a change (> 1); default 10 */
    double rho_tau;          /* residual balancing: factor of a change (> 1); default 2 */
} ldopf_options;

typedef struct ldopf_sizes {
    int64_t n;          /* global variables */
    int64_t n_sub;      /* subsystems S */
    int64_t n_local;    /* local copies, sum of n_s */
    int64_t sum_m;      /* sum of m_s */
    int64_t op_words;   /* sum of n_s * n_s (dense operators, ldopf_get_operators) */
    int64_t rank_words; /* sum of n_s * K_s, K_s = min(rank_s, n_s - rank_s): the sweep's operator */
    int32_t max_n, max_m;
    int32_t n_parts;    /* workgroups of the persistent sweep */
    int32_t block_threads;
    int64_t lds_bytes;  /* LDS per workgroup of the sweep */
    int64_t sync_bytes; /* device bytes of the sweep's exchange words, residual sums and status
                           (what ldopf_solve_noalloc takes from its static array) */
    int32_t sweep_path; /* the path the problem runs on: LDOPF_PATH_PERSISTENT or LDOPF_PATH_STREAMED
                           (n_parts, lds_bytes and sync_bytes are 0 on the streamed path) */
    int32_t reserved;
} ldopf_sizes;

typedef struct ldopf_status {
    int64_t iterations;   /* completed sweeps of this solve call */
    int32_t converged;    /* termination test met */
    int32_t code;         /* ldopf_code of the solve */
    double pres, dres, eps_prim, eps_dual; /* last sweep */
    double sweep_ms;      /* device time of the sweep kernel (HIP events on the handle's stream) */
    double precompute_ms; /* device time of the operator precompute at creation */
    int64_t sweeps_computed; /* sweeps the kernel ran: the test of a sweep is evaluated while the
                                next one runs, so a converged solve computes one sweep more than
                                it returns */
    double rho;           /* rho of the returned sweep */
    int64_t rho_changes;  /* changes of rho made by residual balancing in this solve */
} ldopf_status;

typedef struct ldopf_problem ldopf_problem;

LDOPF_API const char* ldopf_error_string(int code);
LDOPF_API const char* ldopf_last_error_detail(void);
LDOPF_API void ldopf_default_options(ldopf_options* opts);

/*
 * Host-only: assemble and decompose a network without touching the GPU.
 * Writes the consensus LP of OurModel: c, lo, hi and the starting value of
 * each global variable [n]; per subsystem n_s, m_s [S]; A (all A_s blocks,
 * row-major, concatenated), b (concatenated), gidx (all copies, concatenated).
 * Call with every output pointer NULL to get the sizes only:
 *   sizes[0] = n, [1] = S, [2] = N_loc, [3] = total A words, [4] = total rows.
 */
LDOPF_API int ldopf_describe_network(const ldopf_network* net, int64_t sizes[5],
                                     double* c, double* lo, double* hi, double* x_init,
                                     int32_t* n_s, int32_t* m_s, double* A, double* b,
                                     int64_t* gidx);

/*
 * Assemble, decompose, upload and precompute Abar_s, bbar_s in FP64 on the
 * device (Algorithm 1 precomputation; Section III-B). The problem starts at
 * the initial point of Section V-A (lambda = 0; copies of a squared voltage
 * at 1, of a variable with two finite bounds at their midpoint, others at 0
 * clipped into the box). stream: a hipStream_t or NULL.
 */
LDOPF_API int ldopf_create(const ldopf_network* net, const ldopf_options* opts, void* stream,
                           ldopf_problem** out);

/*
 * The same from the consensus LP directly (OurModel): n globals with c, lo,
 * hi; x_init [n] nullable (then: midpoint of finite boxes, else 0 clipped);
 * S subsystems with sizes n_s, m_s; A: the row-major m_s x n_s blocks
 * concatenated; b: concatenated; gidx: each subsystem's global indices,
 * strictly ascending within a subsystem (B_s has row sums 1 and column sums
 * <= 1). Every global variable needs at least one copy.
 */
LDOPF_API int ldopf_create_lp(int64_t n, const double* c, const double* lo, const double* hi,
                              const double* x_init, int64_t n_sub, const int32_t* n_s,
                              const int32_t* m_s, const double* A, const double* b,
                              const int64_t* gidx, const ldopf_options* opts, void* stream,
                              ldopf_problem** out);

LDOPF_API int ldopf_destroy(ldopf_problem* h);
LDOPF_API int ldopf_get_sizes(const ldopf_problem* h, ldopf_sizes* out);

/* Replace rho, eps_rel, eps_abs, max_iter, check_termination, history for
 * later solves. Abar_s, bbar_s do not depend on rho, so nothing is
 * recomputed. precision, sweep_path and tuning fields must equal the
 * creation values (else LDOPF_INVALID_ARGUMENT). */
LDOPF_API int ldopf_set_options(ldopf_problem* h, const ldopf_options* opts);

/*
 * Run ADMM sweeps (Algorithm 1: global update closed_1, local update
 * closed_2, dual update ADMM-3, termination test of Section III-C) from the
 * handle's current state until the test holds or max_iter sweeps ran; the
 * state then holds the last sweep's x, x_s, lambda. Blocks until done.
 * Runs on the path the handle was created for (ldopf_sizes.sweep_path); on
 * the streamed sweep the options must keep the literal residual form, fixed
 * rho and no profile (else LDOPF_UNSUPPORTED).
 * Returns LDOPF_OK, LDOPF_NOT_CONVERGED, LDOPF_NUMERICAL or an error.
 */
LDOPF_API int ldopf_solve(ldopf_problem* h, ldopf_status* status);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as ldopf_solve, from a handle created beforehand, with the sweep's
 * synchronisation words (exchange words between workgroups, residual sums,
 * status) taken from a static device array of 4 MiB that every GPU the
 * library runs on holds until the process ends, instead of the handle's
 * buffers. Calls no hipMalloc or hipFree and allocates no device memory.
 * The residual history is recorded only into the buffer an earlier
 * ldopf_solve on this handle allocated (rows beyond it are not recorded;
 * none without one). Results equal ldopf_solve's bit for bit.
 * Limit: ldopf_sizes.sync_bytes <= 4 MiB, else LDOPF_OUT_OF_MEMORY with
 * nothing run. Every call on one GPU uses that GPU's one array, so calls
 * that overlap on a GPU would race: this library serializes them (a second
 * caller waits for the first to return). Runs on the handle's device and
 * stream; blocks until done. Returns as ldopf_solve; LDOPF_UNSUPPORTED for a
 * handle on the streamed sweep (which allocates its own words).
 */
LDOPF_API int ldopf_solve_noalloc(ldopf_problem* h, ldopf_status* status);

/*
 * Several problems (different feeders, or one feeder with different data)
 * solved together in one persistent launch: each runs Algorithm 1 on its
 * own -- its global, local and dual updates, its exchange words, its
 * termination test (Section III-C) and its stop -- while their workgroups
 * share the GPU. Results equal ldopf_solve's on each problem bit for bit.
 * problems[count]: created on one device with the same precision, residual
 * form and profiling option, none repeated; together their workgroups must
 * fit on the device at once (else LDOPF_UNSUPPORTED and nothing runs: solve
 * them in smaller groups). statuses[count] (nullable) receives each
 * problem's status as ldopf_solve reports it; status.sweep_ms is the time of
 * the shared launch. Runs on the first problem's stream after every
 * problem's earlier work; blocks until done. Returns LDOPF_OK when every
 * problem did, else the most severe code among them (an error before
 * LDOPF_NOT_CONVERGED). A problem on the streamed sweep cannot share the
 * launch (LDOPF_UNSUPPORTED).
 */
LDOPF_API int ldopf_solve_many(ldopf_problem* const* problems, int32_t count, ldopf_status* statuses);

/* Back to the initial point of Section V-A. */
LDOPF_API int ldopf_reset(ldopf_problem* h);

/* Continue from a given state: x_s and lambda [N_loc] in local-copy order.
 * A following ldopf_solve resumes exactly as if the sweeps had not stopped.
 * A NaN or Inf entry is refused with LDOPF_NUMERICAL (nothing is uploaded). */
LDOPF_API int ldopf_warm_start(ldopf_problem* h, const double* xs, const double* lam, int64_t n_local);

/* Global x [n] of the last sweep (NaN before the first sweep). */
LDOPF_API int ldopf_get_global(const ldopf_problem* h, double* x, int64_t cap);
/* Local copies x_s and duals lambda [N_loc]; either pointer may be NULL. */
LDOPF_API int ldopf_get_local(const ldopf_problem* h, double* xs, double* lam, int64_t cap);
/* gidx [N_loc] and subsystem offsets [S+1] of the local-copy order. */
LDOPF_API int ldopf_get_structure(const ldopf_problem* h, int64_t* gidx, int64_t cap_local,
                                  int64_t* sub_off, int64_t cap_sub);
/* Residual history of the last solve: [len x 4] = pres, dres, eps_prim, eps_dual. */
LDOPF_API int ldopf_get_history(const ldopf_problem* h, double* hist, int64_t cap_rows, int64_t* len);
/* Precomputed operators in FP64: dense Abar_s blocks [op_words] row-major,
 * bbar [N_loc], numerical rank of each A_s [S]; any pointer may be NULL. */
LDOPF_API int ldopf_get_operators(const ldopf_problem* h, double* abar, int64_t cap_abar,
                                  double* bbar, int64_t cap_bbar, int32_t* rank, int64_t cap_rank);
/* The changes of rho residual balancing made in the last solve: the first
 * sweep that used each new value and the value; *len = the number of
 * changes; writes min(len, cap) entries (either array may be NULL). */
LDOPF_API int ldopf_get_rho_log(const ldopf_problem* h, int64_t* sweeps, double* rhos, int64_t cap, int64_t* len);
/* Per-phase device time of the last solve with options.profile = 1, in ms,
 * measured by workgroup 0 with the wall clock: [0] global update, with the
 * wait for the neighbours' partial sums, [1] gather of B_s x + lambda/rho,
 * [2] t = W v, alongside the termination test of an earlier sweep, [3] local
 * and dual update with residual row sums, [4] partial sums and publication,
 * [5] end of the sweep; [6] the reader wave's termination test (the grid
 * totals from the group sums, inside [2]), [7] the workgroup's own global
 * update before its barrier (inside [0]). Zeros when profiling was off. */
LDOPF_API int ldopf_get_phase_times(const ldopf_problem* h, double ms[8]);
/* The same for workgroup `part` (0 <= part < ldopf_sizes.n_parts). */
LDOPF_API int ldopf_get_phase_times_part(const ldopf_problem* h, int32_t part, double ms[8]);

/* c'x at the last sweep's global x. */
LDOPF_API int ldopf_objective(const ldopf_problem* h, double* f);

/* Device-pointer getters for caller-allocated device buffers (for example
 * torch tensors); enqueued on the handle's stream, which the caller then
 * orders against its own work. */
LDOPF_API int ldopf_get_global_device(const ldopf_problem* h, double* x_device, int64_t cap);
LDOPF_API int ldopf_get_local_device(const ldopf_problem* h, double* xs_device, double* lam_device,
                                     int64_t cap);

/* ------------------------------------------------------------------------
 * Batched scenarios: one network, B load scenarios solved together.
 *
 * Scenario k multiplies the reference powers a, b of every load l by
 * load_scale[k * n_load + l]. For a voltage-dependent load that also scales
 * the squared-voltage coefficient of its model rows (VDLM-1, VDLM-2), so only
 * subsystems without such loads share one operator Abar_s across scenarios;
 * their local update (closed_2) for all scenarios is one small GEMM on the
 * matrix cores. Every scenario runs Algorithm 1 on its own: its own global
 * update, dual update and termination test (Section III-C), and it keeps the
 * state of its first sweep that passes the test while the others continue.
 * Sweeps run in the FP32-mixed form: operators are precomputed in FP64 and
 * stored in FP32; residual sums and the test are FP64. */
typedef struct ldopf_batch ldopf_batch;

typedef struct ldopf_batch_status {
    int64_t sweeps;       /* sweeps the batch ran: its slowest scenario's count, or max_iter */
    int32_t n_scen;
    int32_t n_converged;
    int32_t n_numerical;  /* scenarios stopped by NaN or Inf */
    int32_t code;         /* LDOPF_OK, LDOPF_NOT_CONVERGED or LDOPF_NUMERICAL */
    double solve_ms;      /* device time of the solve (HIP events on the batch's stream) */
    double precompute_ms; /* device time of the operator precompute of all scenarios */
} ldopf_batch_status;

typedef struct ldopf_batch_sizes {
    int64_t n, n_sub, n_local;
    int32_t n_scen, n_scen_padded;          /* scenarios, padded to a multiple of 64 */
    int64_t n_mfma_subsystems;              /* shared operator, GEMM on matrix cores */
    int64_t n_vector_subsystems;            /* per-scenario operator, rank form */
    int64_t scenario_operator_words;        /* FP32 words of per-scenario operators */
    int64_t shared_operator_words;          /* FP32 words of shared operators */
    int32_t rows_per_chunk, blocks_per_tile; /* tuning of the local update */
    int32_t graph_sweeps;                   /* sweeps per captured HIP graph */
    int32_t pad;
} ldopf_batch_sizes;

/* Assemble the network, precompute every (subsystem, scenario) operator on
 * the device and set every scenario to the initial point of Section V-A.
 * load_scale: [n_scen x n_load] row-major host array (finite; nullable when
 * n_load = 0). 1 <= n_scen <= 1024. opts->precision must be
 * LDOPF_FP32_MIXED (else LDOPF_UNSUPPORTED); rho is fixed at creation;
 * rows_per_part sets the rows per chunk of the local update (0: 64). The
 * batch runs on a stream of its own, ordered after the caller's stream. */
LDOPF_API int ldopf_batch_create(const ldopf_network* net, int32_t n_scen, const double* load_scale,
                                 const ldopf_options* opts, void* stream, ldopf_batch** out);
LDOPF_API int ldopf_batch_destroy(ldopf_batch* h);
/* Replace eps_rel, eps_abs, max_iter, check_termination (rho and precision fixed). */
LDOPF_API int ldopf_batch_set_options(ldopf_batch* h, const ldopf_options* opts);
/* Every scenario back to the initial point. */
LDOPF_API int ldopf_batch_reset(ldopf_batch* h);
/* Run until every scenario stopped or max_iter sweeps; blocks until done. */
LDOPF_API int ldopf_batch_solve(ldopf_batch* h, ldopf_batch_status* status);
/* One scenario's iterations (its stopping sweep), converged flag and last residuals. */
LDOPF_API int ldopf_batch_get_scenario(const ldopf_batch* h, int32_t scen, ldopf_status* status);
/* One scenario's global x [n] and local x_s, lambda [N_loc] (either nullable), as FP64,
 * of its returned sweep. The batch keeps lambda and x_s - lambda / rho per copy in FP32;
 * x_s is formed from the two as the sweep forms it. */
LDOPF_API int ldopf_batch_get_global(const ldopf_batch* h, int32_t scen, double* x, int64_t cap);
LDOPF_API int ldopf_batch_get_local(const ldopf_batch* h, int32_t scen, double* xs, double* lam, int64_t cap);
LDOPF_API int ldopf_batch_get_sizes(const ldopf_batch* h, ldopf_batch_sizes* out);
/* Autotuner: time short runs of the local update over rows per chunk and
 * blocks per 64-scenario tile, keep the fastest, and remember it in a text cache
 * file keyed by device, network shape and batch size (cache_path nullable:
 * no cache). Resets the batch. Results do not depend on the choice except
 * for the summation order of the residual sums. */
LDOPF_API int ldopf_batch_tune(ldopf_batch* h, const char* cache_path, int32_t* rows_per_chunk,
                               int32_t* blocks_per_tile);

/* ------------------------------------------------------------------------
 * Serving: a request loop for OPF solves of differing feeders.
 *
 * Requests are assembled at submit (network errors are returned at once) and
 * queued. A scheduler thread admits queued requests first-fit in arrival
 * order when a stream slot is free, the request's device bytes fit the HBM
 * budget beside the requests in flight, and its sweep's workgroups fit the
 * chip beside the sweeps running; the oldest request is not overtaken more
 * than 64 times. Admitted requests have their operators precomputed and their
 * solve (Algorithm 1 to the termination test) launched on their slot's
 * stream; their state stays resident until they finish, and several run on
 * the device at once. Results are copied to host memory at completion and the
 * device memory is released. Latency = completion - submit. Every call is
 * thread-safe. A result does not depend on what else runs beside it. */
typedef struct ldopf_server ldopf_server;

typedef enum ldopf_request_state {
    LDOPF_REQ_QUEUED = 0,
    LDOPF_REQ_RUNNING = 1,
    LDOPF_REQ_DONE = 2,   /* solved (converged or max_iter reached); results available */
    LDOPF_REQ_FAILED = 3  /* error, cancelled, or dropped at shutdown */
} ldopf_request_state;

typedef struct ldopf_server_stats {
    int64_t submitted, completed, failed, queued, running;
    int64_t peak_running;
    int64_t bytes_in_use, peak_bytes_in_use, budget_bytes;
    double p50_ms, p99_ms, mean_ms, max_ms; /* latency of completed requests (nearest rank) */
    double wall_s;        /* first submit to last completion */
    double solves_per_s;  /* completed / wall_s */
} ldopf_server_stats;

/* Host-only: the device bytes a request would hold at its peak and the
 * workgroups of its sweep (planned assuming full row rank), as the server's
 * admission counts them. */
LDOPF_API int ldopf_request_estimate(const ldopf_network* net, const ldopf_options* opts, int64_t* bytes,
                                     int32_t* workgroups);

/* hbm_budget_bytes <= 0: 80% of the free device memory. 1 <= max_slots <= 64
 * streams (requests in flight at once). */
LDOPF_API int ldopf_server_create(int64_t hbm_budget_bytes, int32_t max_slots, ldopf_server** out);
/* Copy and queue one request; LDOPF_OUT_OF_MEMORY when it alone exceeds the
 * budget. opts: as for ldopf_create (history is not recorded); requests run
 * on the persistent sweep only (sweep_path LDOPF_PATH_STREAMED is refused
 * with LDOPF_UNSUPPORTED, and a request too large for it fails at admission). */
LDOPF_API int ldopf_server_submit(ldopf_server* srv, const ldopf_network* net, const ldopf_options* opts,
                                  int64_t* req_id);
/* Current state (ldopf_request_state) and, once done, the solve status. */
LDOPF_API int ldopf_server_poll(ldopf_server* srv, int64_t req_id, int32_t* state, ldopf_status* status);
/* Block until the request is done or failed or timeout_s passed (< 0: no
 * limit); returns the request's error code when it failed. */
LDOPF_API int ldopf_server_wait(ldopf_server* srv, int64_t req_id, double timeout_s, int32_t* state,
                                ldopf_status* status);
/* Remove a queued request (it becomes FAILED with LDOPF_INVALID_ARGUMENT). */
LDOPF_API int ldopf_server_cancel(ldopf_server* srv, int64_t req_id);
/* Results of a done request: x [n], x_s and lambda [N_loc] (each nullable);
 * sizes (nullable) receives n and N_loc. */
LDOPF_API int ldopf_server_fetch(ldopf_server* srv, int64_t req_id, double* x, int64_t cap_x, double* xs,
                                 double* lam, int64_t cap_local, int64_t sizes[2]);
/* Forget a finished request and its host-side results. */
LDOPF_API int ldopf_server_release(ldopf_server* srv, int64_t req_id);
LDOPF_API int ldopf_server_get_stats(ldopf_server* srv, ldopf_server_stats* stats);
/* Drop queued requests, wait for running ones, stop the scheduler. */
LDOPF_API int ldopf_server_destroy(ldopf_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* LDOPF_H */
