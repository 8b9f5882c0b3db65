"""FP64 CPU oracle for the diagonalized waveform-relaxation (WR) sweep of
Wu & Zhou, "A parallel-in-time algorithm for high-order BDF methods for
diffusion and subdiffusion equations" (arXiv 2007.13125).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package; only
the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the GPU path: the two meet only
through the seeded input generators, which hold none of the method's
arithmetic.

Modules
-------
bdf          BDF-k weights (Sec. 2.1, eq. bdf-gen) and the starting-step
             corrections a_n, b_{l,n} (Sec. 2.1, eq. BDF, Table 1).
cq           CQ-BDF-k weights, power-series coefficients of delta_k^alpha
             (Sec. 3.1, eqs. CQ and delta).
grid         finite-difference Dirichlet Laplacian A_h on a box, its sine
             eigenvalues, the discrete L2 norm.
sequential   O1: the plain time stepper of the corrected BDF-k / CQ-BDF-k
             scheme (Sec. 2.1 eq. BDF, Sec. 3.1 eq. BDF-frac, Sec. 3.2 cost
             paragraph); the fixed point every WR sweep must converge to.
sweep        O2: one WR sweep by diagonalization in time with dense DFT
             matrices (Algorithms 1 and 2), direct and residual forms.
bruteforce   O3: the same sweep as one dense space-time linear solve of the
             kappa-circulant all-at-once system (eqs. BDF-k-matrix,
             BDF-k-matrix-frac).
contraction  spectral radius of the WR error-propagation matrix for one
             spatial mode (Sec. 2.4 Lemma conv-heat, Sec. 3.3 Lemma conv-frac).
exact        exact semi-discrete single-mode solutions used to pin the order
             of the corrected schemes (Lemmas 2.2 and 3.2).
fem          P1 finite elements in 1D (Sec. 4's discretisation): the scaled
             mass matrix, O1 and O2 with the mass on the time derivative.
nonlinear    the semilinear scheme stepped in time and Algorithm 3.
windows      consecutive time windows, each solved by O1.

Parity pins for every function live in ``tests/test_oracle_*.py``; the only
result without an external pin is listed as "parity unpinned" in the module
that computes it.
"""
