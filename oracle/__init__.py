"""Plain FP64 CPU oracle for BDDC-SO (test infrastructure only).

This package is the reference the GPU path is checked against.  It is slow
and written to be read against the paper: numpy/scipy in float64, one
subdomain at a time, assembled sparse matrices, direct local and coarse
solves.  It shares no code with the HIP path and imports nothing from it; the
only common module is ``workloads`` (seeded inputs, no method arithmetic).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import it.  The product path never calls it.

Modules
-------
q1            Q1 element matrices and global assembly (Section 2, Remark 4).
classify      interface nodes, subobjects, coarse numbering, weights
              (Section 3: the fine partition, Remark 2 on classification,
              eq. (W), Remark 4).
bddc          BDDC-SO setup and the preconditioner application, following the
              multispace definition (Definition 1) with V1 = U_I, V2 = W~,
              Q1 = I, Q2 = (I-P)E (Section 3).
pcg           preconditioned conjugate gradients and the Lanczos estimate of
              the condition number (Section 5 stopping rule, Theorem 3).
definitional  the preconditioner assembled densely from its definition on
              tiny meshes (Definition 1, Section 3), used to pin ``bddc``.
adjoint       the gradient of a least-squares loss with respect to the
              element log-coefficients (direct solves).

Parity status: every function is pinned by a CPU test against something other
than itself (closed forms, the paper's Figure 1 and Table 1 counts, brute
force, the definitional preconditioner, Theorem 3's lower bound, direct
solves, finite differences).  See the test modules ``tests/test_oracle_*.py``.
"""
