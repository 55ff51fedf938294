"""GPU parity of the multi-sheet initial conditions (glasma_init_mv_sheets: nuclei with
colour structure along the beam axis) against the FP64 oracle, and the evolution of
such a state; per-component bar 1e-10 as for the single sheet."""
import sys
import numpy as np
import pytest

import synth
from oracle import lattice, init_mv
from _gpu import gpu, lattice_or_skip, to_comp, state_errs, mv_setup, new_lattice

pytestmark = gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = [
    (synth.Workload("su2-64x8x8-sheets", nc=2, nz=64, nt=8, mu=1.0, sigma=4.0, seed=1101), 5),
    (synth.Workload("su3-40x6x6-sheets", nc=3, nz=40, nt=6, mu=0.5, sigma=3.0, seed=1177), 4),
]


@pytest.mark.parametrize("w,ns", CASES, ids=[c[0].name for c in CASES])
def test_init_mv_sheets_matches_oracle_and_evolves(w, ns):
    pkg = lattice_or_skip()
    say("case:", w.name, "ns", ns)
    p, mv = mv_setup(w)
    rA, rB = synth.mv_sheet_charges(w.seed, w.nc, w.nt, w.mu, w.a_T, ns)
    st, _ = init_mv.initial_state(rA, rB, w.nz, p, mv)
    lat = new_lattice(pkg, w)
    lat.init_mv(rA, rB, m_ir=w.m_ir, uv_cut=w.uv_cut, sigma=w.sigma, zA=w.zA, zB=w.zB)
    errs = state_errs(lat.get_state(), st)
    say("init errs", errs)
    assert max(errs.values()) < 1e-10, errs
    o = lat.observables()
    assert o["gauss_rel"] < 1e-13 and o["unitarity"] < 1e-13
    worst = 0.0
    for s in range(20):
        st = lattice.leapfrog_step(st)
        lat.step(1)
        e = state_errs(lat.get_state(), st)
        worst = max(worst, max(e.values()))
        assert max(e.values()) < 1e-10, (s, e)
    say("per-component worst over 20 steps", worst)


@pytest.mark.parametrize("fp", [64, 32])
def test_identical_sheets_equal_one_sheet(fp):
    """rho_k = rho / ns for every sheet: the same state as the single sheet rho."""
    pkg = lattice_or_skip()
    w = synth.Workload("su3-32x8x8", nc=3, nz=32, nt=8, mu=0.5, sigma=2.0, seed=1203)
    ns = 3
    rA, rB = synth.mv_charges(w.seed, w.nc, w.nt, w.mu, w.a_T)
    one = new_lattice(pkg, w, fp=fp)
    one.init_mv(rA, rB, m_ir=w.m_ir, sigma=w.sigma)
    many = new_lattice(pkg, w, fp=fp)
    many.init_mv(np.repeat(rA[None] / ns, ns, 0), np.repeat(rB[None] / ns, ns, 0), m_ir=w.m_ir, sigma=w.sigma)
    a, b = one.get_state(), many.get_state()
    tol = 1e-12 if fp == 64 else 2e-6
    for k in ("U", "E", "rhoA", "rhoB"):
        ref = np.asarray(a[k])
        d = np.abs(np.asarray(b[k]) - ref).max() / max(np.abs(ref).max(), 1e-300)
        say(fp, k, d)
        assert d < tol, (k, d)


def test_sheet_arguments_are_checked():
    pkg = lattice_or_skip()
    w = synth.Workload("su3-4x8x8", nc=3, nz=4, nt=8, mu=0.5, sigma=1.0, seed=5)
    lat = new_lattice(pkg, w, fp=32)
    # second link buffer: 3 * 12 * 256 floats = 36864 bytes holds 4 sheets of 2 * 8 * 64 doubles
    rA, rB = synth.mv_sheet_charges(w.seed, 3, 8, 0.5, w.a_T, 4)
    lat.init_mv(rA, rB, sigma=1.0)
    rA, rB = synth.mv_sheet_charges(w.seed, 3, 8, 0.5, w.a_T, 5)
    with pytest.raises(pkg.GlasmaError, match="too many sheets"):
        lat.init_mv(rA, rB, sigma=1.0)
    with pytest.raises(ValueError):
        lat.init_mv(rA, rB[:2], sigma=1.0)
