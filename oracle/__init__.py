"""Plain FP64 CPU oracle of the hybrid-snapshot adaptive ROM (Zucatti & Zahr,
"An adaptive, training-free reduced-order model for convection-dominated
problems based on hybrid snapshots", arXiv 2301.01718).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or execute anything here.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark use it.

The oracle is written from the paper, step by step, in numpy/scipy double
precision, with no blocking, fusion or reordering beyond what the paper's
definitions state.  It shares no code with the GPU path; the only common
dependency is :mod:`workloads`, which draws inputs and holds none of the
method's arithmetic.

Modules
-------
``fv``        finite-volume residual of the backward-Euler HDM, its Jacobian,
              and the Newton solve (Sec. 2.2, eq. hdm; Sec. 3.1, eq. euler).
``sampling``  reconstruction-error indicator, error ordering, G, the sampled
              set and its neighbours (Sec. 2.3.3, eq. rre; Alg. 1 set ops).
``pod``       window mean and the POD basis (Sec. 2.3.1, eq. pod, eq. mean).
``hybrid``    partial HDM, gappy-POD fit, subiterations, reconstruction and
              the residual-gated Shapiro filter (Sec. 2.3, 2.3.1, 2.3.2, 2.3.4).
``arom``      Algorithm 1 (the full/hybrid schedule) and the error and
              sampling statistics of Sec. 3.1.
``adjoint``   the discrete adjoint of the hybrid trajectory with decisions
              frozen at their forward values.

Readings of points the paper leaves open are listed in each module header.
"""
