"""Plain CPU FP64 oracle for the scattering solve of Cosicova, Dvorak & Cizek,
"Vibronic dynamics in electron continuum - iterative solvers" (arXiv:2307.13483).

THIS PACKAGE IS TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it. The product path
(``paper_2307_13483_amd``) never imports, calls or links anything here, and
nothing here imports the product path. The two share no code; the seeded input
generators (parameter draws, job lists) live in a module of their own that
holds none of the method's arithmetic, and the oracle takes their output as
plain arguments.

Everything is written for clarity, not speed: explicit matrix assembly from
matrix elements, library LU solves, a textbook restarted GMRES.

Modules
-------
levelshift   widths, the level-shift integral transform, Eqs. (19), (20), (22)
model2d      the generalized two-state, two-mode model of Sec. II.C assembled
             as an explicit sparse matrix, Eqs. (18), (23), (25), (28)
solvers      sparse/dense LU and a textbook GMRES(m) of Sec. III.A
precond      block-diagonal sections of A as preconditioners, Sec. III.B
observables  T-matrix and cross sections, Eqs. (15), (16), (24)
adjoint      d(loss)/d(parameters) by explicit derivative matrices and LU
poly         the CO2-like three-state, four-mode polynomial model (Sec. III.C)
             assembled the same way, and its bend-block preconditioner
terms        any model of the class given by polynomial term lists (D states,
             M modes, P partial waves), assembled the same way
polar        the 2D bend of the CO2-like model in the polar (circular) basis
             of the isotropic oscillator, with H_0 + U in it

Parity status: every function is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_*.py``; none is "parity unpinned".
"""
