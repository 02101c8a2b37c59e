"""FP64 CPU oracle for the visibility / likelihood / HMC hot path.

TEST INFRASTRUCTURE ONLY.  This package is the independent checker of the
HIP library: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with
the GPU path; the only common module is the seeded input generator
``paper_2504_07090_amd.workload``, which holds no forward-model arithmetic.

Everything here is the plain definition written out in float64 with NumPy
(a matrix product, an ``exp`` or a Gauss-Legendre rule from NumPy/SciPy may
serve as a step).  Each function cites the passage of Kern (2025),
"A Differentiable, End-to-End Forward Model for 21 cm Cosmology", that it
follows.  Modules:

``array``      baselines and redundant (unique) baselines            Sec. 2.1, 3.1
``sky``        equal-area grid, real spherical harmonics, I = Y a     Sec. 2.1, 3.2, App. A
``rime``       directions, Gaussian power beam, direct-sum RIME       Sec. 2.1 (eq. rime_discrete)
``model``      gains, residual, chi^2 and its analytic gradient       Sec. 2.3 (eq. likelihood)
``filter``     delay filter and the filtered chi^2                   Sec. 2.1 (eq. rime_filter, gpr), 3.5
``hmc``        leapfrog / Hamiltonian, diagonal or block-dense mass  Sec. 4.2, App. B
``nuts``       No-U-Turn sampler, biased progressive sampling        Sec. 4.2 (Hoffman & Gelman 2014,
               Betancourt 2017)
``mapmaking``  diagonally normalised dirty map                        Sec. 4.3
``philox``     Philox-4x32-10 counter-based generator (Salmon et al. 2011)

Parity status: every function is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_*.py`` against a closed form, an invariant, a library
routine or a value printed in the paper; none is "parity unpinned".
"""
