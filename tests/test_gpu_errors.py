"""Error behaviour of the C-ABI on a GPU context, as include/glasma.h states it: argument
errors, calls before a state exists, a semi-implicit solve that reaches max_iter, and
non-finite fields reported by the semi-implicit solve and by the observables.  Every
condition is set from the host (arguments, iteration limits, a NaN in the uploaded state):
the kernels run to completion on valid memory."""
import sys
import numpy as np
import pytest

import synth
from oracle import init_mv
from oracle import semi_implicit as si
from _gpu import gpu, lattice_or_skip, to_comp, mv_setup

pytestmark = gpu

E_ARG, E_NONFINITE, E_NOCONV, E_STATE = -1, -3, -5, -6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def code_of(fn):
    from paper_2009_02044_amd import GlasmaError
    with pytest.raises(GlasmaError) as e:
        fn()
    return e.value.code


def small_state(nc=3, nz=8, nt=4, seed=910):
    w = synth.Workload(f"su{nc}-{nz}x{nt}", nc=nc, nz=nz, nt=nt, dt=0.5, mu=0.5, sigma=1.0, seed=seed)
    p, mv = mv_setup(w)
    rA, rB = synth.mv_charges(w.seed, nc, nt, w.mu, w.a_T)
    st, _ = init_mv.initial_state(rA, rB, nz, p, mv)
    return w, st


def test_argument_and_state_errors():
    pkg = lattice_or_skip()
    say("case: argument and state errors")
    assert code_of(lambda: pkg.Lattice(nc=4, nz=8, nt=4)) == E_ARG
    assert code_of(lambda: pkg.Lattice(nc=3, nz=1, nt=4)) == E_ARG
    assert code_of(lambda: pkg.Lattice(nc=3, nz=8, nt=4, fp=16)) == E_ARG
    assert code_of(lambda: pkg.Lattice(nc=3, nz=8, nt=4, dt=-0.5)) == E_ARG
    assert code_of(lambda: pkg.Lattice(nc=3, nz=8, nt=4, scheme=1, tol=0.0)) == E_ARG
    lat = pkg.Lattice(nc=3, nz=8, nt=4)
    # no state yet
    assert code_of(lambda: lat.step(1)) == E_STATE
    assert code_of(lambda: lat.observables()) == E_STATE
    w, st = small_state()
    lat.init_state(*to_comp(st), step0=0)
    assert code_of(lambda: lat.step(-1)) == E_ARG
    buf = lat.obs_buffer()
    assert code_of(lambda: lat.step_observe(0, buf)) == E_ARG
    rA, rB = synth.mv_charges(w.seed, 3, w.nt, w.mu, w.a_T)
    empty = np.zeros((0,) + rA.shape)
    assert code_of(lambda: lat.init_mv(empty, empty)) == E_ARG
    assert code_of(lambda: lat.init_mv(rA, rB, m_ir=0.0)) == E_ARG
    # the context is still usable after each error
    lat.step(3)
    o = lat.observables()                  # raises on a non-finite field
    assert o["gauss_rel"] < 1e-12


def test_semi_implicit_reaching_max_iter():
    pkg = lattice_or_skip()
    say("case: semi-implicit max_iter")
    w, st = small_state()
    st = si.charges_for_scheme(st)
    lat = pkg.Lattice(nc=3, nz=w.nz, nt=w.nt, a_T=w.a_T, a_L=w.a_L, dt=1.0, scheme=1, max_iter=1, tol=1e-15)
    lat.init_state(*to_comp(st), step0=0)
    before = lat.get_state()
    # at dt = a_L every step hops: the failed solve must not have moved the charges
    assert code_of(lambda: lat.step(1)) == E_NOCONV
    assert lat.last_iterations == 1
    after = lat.get_state()
    assert after["step"] == before["step"] == 0
    for k in ("U", "E", "rhoA", "rhoB"):
        assert np.array_equal(after[k], before[k]), k


@pytest.mark.parametrize("scheme", [0, 1])
def test_non_finite_fields_are_reported(scheme):
    """A NaN in one E component of the uploaded state: the semi-implicit solve stops with
    GLASMA_E_NONFINITE; the leapfrog (asynchronous, unchecked) carries it, and the
    observables report it."""
    pkg = lattice_or_skip()
    say("case: non-finite field, scheme", scheme)
    w, st = small_state()
    if scheme == 1:
        st = si.charges_for_scheme(st)
    U, E, rA, rB = to_comp(st)
    E = E.copy()
    E[1, 2, 37] = np.nan
    lat = pkg.Lattice(nc=3, nz=w.nz, nt=w.nt, a_T=w.a_T, a_L=w.a_L, dt=0.5, scheme=scheme,
                      max_iter=50, tol=1e-12 if scheme == 1 else 0.0)
    lat.init_state(U, E, rA, rB, step0=0)
    if scheme == 1:
        before = lat.get_state()
        assert code_of(lambda: lat.step(1)) == E_NONFINITE
        after = lat.get_state()
        assert after["step"] == 0
        for k in ("U", "rhoA", "rhoB"):
            assert np.array_equal(after[k], before[k]), k
    else:
        lat.step(2)
        assert code_of(lambda: lat.observables()) == E_NONFINITE


def test_batch_observe_and_cotangent_errors():
    """glasma_batch_observe refuses events without a state and an n_grid outside
    [1, smallest N_z]; glasma_adjoint_backward_cotangent refuses a call without its forward
    pass, a work buffer smaller than the layout and a context stepped since the forward pass.
    Each context stays usable after the error."""
    pkg = lattice_or_skip()
    say("case: batch observe and cotangent reverse-pass errors")
    shapes = [(16, 4), (24, 4)]
    b = pkg.Batch(3, shapes, fp=64, reunit_every=0)
    assert code_of(lambda: b.observe(8)) == E_STATE
    for (nz, nt), lat in zip(shapes, b.events):
        w, st = small_state(nz=nz, nt=nt)
        lat.init_state(*to_comp(st), step0=0)
    assert code_of(lambda: b.observe(0)) == E_ARG
    assert code_of(lambda: b.observe(17)) == E_ARG          # above the smallest N_z
    r = b.observe(16)
    assert r["grid"].shape == (4, 16) and bool(r["grid"].isfinite().all())

    lat = pkg.Lattice(nc=3, nz=8, nt=4, fp=64)
    w, st = small_state()
    lat.init_state(*to_comp(st), step0=0)
    work = lat.adjoint_work(4, 2)
    assert code_of(lambda: lat.adjoint_backward_cotangent(work)) == E_STATE   # no forward pass
    lat.adjoint_forward(4, 2, work)
    assert code_of(lambda: lat.adjoint_backward_cotangent(work[:256])) == E_ARG
    g = lat.adjoint_backward_cotangent(work)                                  # zero cotangent
    assert float(g["dE0"].abs().max()) == 0.0 and float(g["dU0"].abs().max()) == 0.0
    lat.step(1)
    assert code_of(lambda: lat.adjoint_backward_cotangent(work)) == E_STATE   # stepped since
