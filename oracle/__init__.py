"""FP64 CPU oracle for the adjoint FDTD hot path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import it; the GPU library never does, and the two share
no code (only the seeded inputs of ``workloads``).

Modules:
  fdtd     FP64 Yee/CPML/source/DFT time stepping in C (fdtd.c) and the
           least-squares amplitude/phase extraction;
  chain    C -> rho -> eps -> kappa and its VJP, explicit dense operators;
  ports    Appendix A mode sources, monitor weights, modal coefficient;
  adjoint  forward + adjoint runs and the Eq. (1) gradient.

Parity status: every function is pinned by tests in tests/test_oracle_*.py
(closed forms, conservation laws, reciprocity, brute-force finite
differences, dot-product identities).  Values the paper itself prints for a
worked example do not exist for this path, so none are used.
"""
