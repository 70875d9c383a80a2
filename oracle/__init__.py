"""Plain FP64 CPU oracle for the pairwise line-of-sight P_ell / xi_ell estimators
of Philcox & Slepian, "Beyond Yamamoto" (arXiv:2102.08384).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything under ``oracle/``.  The
product (``paper_2102_08384_amd`` + ``libpw``) never imports, links or calls it,
and the oracle imports nothing from the product: the two share no code.

Modules
-------
coeffs      coupling coefficients (Appendices A-F): Wigner 3j, Gaunt, A, c~,
            Gegenbauer, phi, omega, Omega, Phi, f, h, F, B.
ylm         complex spherical harmonics (Condon-Shortley, orthonormal).
mesh        painting, DFT conventions, assignment window, k / r grids.
estimators  midpoint / bisector / Yamamoto P_ell and xi_ell, FFT-based.
brute       O(N^2) pair sums, truncated-series and exact line of sight.

Every estimator follows the paper's boxed equations step by step, on full
complex grids, summing over every m and M (no Hermitian shortcuts).
"""
