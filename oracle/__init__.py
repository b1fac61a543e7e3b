"""Plain FP64 CPU oracle for the closed-form ADMM of linearized multi-phase OPF.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports this package:
only the tests, the smoke check and the benchmark's CPU-baseline leg do. It
shares no code with the GPU library; both only read the seeded inputs of the
``synth`` package.

Modules
-------
model      network -> LP rows (Section II-A: operational bounds, power balance,
           voltage-dependent load model, linearized power flow, objective),
           canonical variable order of the abstract LP, and the component-wise
           decomposition with leaf merging (Sections III-A and V-A, Table 3).
admm       operator precompute (Section III-B, closed_2), initialization
           (Section V-A), the ADMM iteration of Algorithm 1 (closed_1, closed_2,
           ADMM-3) and the termination test (Section III-C).
central    the centralized LP (LP_model) solved by HiGHS, and a KKT certificate
           built from ADMM's own duals; used to pin the oracle's fixed point.

Parity status: every function here is pinned by a test under ``tests/``
against brute force, closed forms, a worked example, the LinDistFlow sweep,
HiGHS, or invariants; the delta-load rows are pinned by a balanced phasor
check. The paper's Table 5 iteration counts cannot be pinned (the IEEE
feeder data are absent).
"""
