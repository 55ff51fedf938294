"""FP64 CPU oracle for the 3+1D Glasma colored-particle-in-cell (CPIC) method.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
HIP library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code
with ``paper_2009_02044_amd`` (neither imports the other); the only module both
sides use is ``synth``, which draws seeded random numbers and holds none of the
method's arithmetic.

Everything is NumPy float64 / complex128, vectorised over lattice sites, with
fields stored as full N x N matrices so that each formula can be read against
the paper (Ipp & Mueller, "Progress on 3+1D Glasma simulations", arXiv:2009.02044):

* ``su``           -- SU(N) algebra: generators, P(X), exp, log, transport
* ``lattice``      -- plaquettes, force, leapfrog step (Sec. 3, eqs. lattice_1/2,
                      plaquette) and the CPIC hop + current (Sec. 3, eq. continuity)
* ``init_mv``      -- MV initial conditions (Sec. 2, eqs. for W[rho], the Poisson
                      solution; Sec. 3, eqs. single_sheet, 3d_colorfield_1/2)
* ``observables``  -- T^{mu nu} slices, energy, Gauss residual (Sec. 3 eq. gauss,
                      Sec. 4 eqs. for <T^{mu nu}> and pT_eL)
* ``semi_implicit``-- the improved (time-averaged plaquette) scheme (Sec. 3,
                      fig. wilson and the text after eq. gauss)
* ``components``   -- conversion between matrices and the real component layout
                      used at the C-ABI (host-side marshalling for tests)

Parity status of each function is stated in its docstring ("pinned by ..." or
"parity unpinned").
"""
