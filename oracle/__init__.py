"""FP64 CPU oracle for the staggered-grid real P_N system (Koerner, Portsmouth
& Jakob, "P_N-Method for Multiple Scattering in Participating Media", EGSR 2018).

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain, obviously-correct
reference that the HIP solver is checked against.  Only ``tests/``
(with the reference-solution script ``tests/golden/make_references.py``),
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it (``__graft_entry__.build()`` compiles its C part).  The product path (``paper_1807_00410_amd``) never imports, calls or
links anything in here, and this package never imports the product path; the
two share only the seeded input generators in ``synth/``.

Contents (each function cites the passage of the paper it follows):

* ``sh``          real spherical-harmonics basis (appendix, real basis equation)
* ``couplings``   transport couplings  A_d[k,k'] = int omega_d Y_k Y_k' by
                  quadrature; phase-function moments (appendix, phase function)
* ``closed_form`` the printed closed-form couplings (a..f, beta), with the
                  three corrections stated in that module -- used only as a pin
* ``stagger``     staggered coefficient classes, extents and vector layout;
                  boundary types per axis (vacuum/Dirichlet, periodic, Neumann)
* ``medium``      sigma_t threshold and interpolation of the RTE parameters to
                  the staggered locations
* ``assemble``    sparse FP64 assembly of A (row by row, SciPy CSR)
* ``apply``       matrix-free FP64 apply of A / A^T (NumPy) and ``rows_of``
                  (single rows from the row equation, for grids too large to
                  assemble), both pinned to the CSR
* ``solve``       direct (SuperLU) solve and FP64 CGLS on the normal equations
* ``ref``         the same operator (A, A^T) and CGLS in plain C with OpenMP
                  (``pn_ref.c``, compiled with gcc on first use) for systems too
                  large for the assembled matrix; pinned to the CSR and SuperLU

Every function here is pinned by a ``-m "not gpu"`` test in ``tests/`` except
the ones whose docstring says "parity unpinned".
"""
