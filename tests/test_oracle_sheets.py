"""Pins of the oracle's multi-sheet initial conditions: nuclei whose colour structure
varies along the beam axis (Sec. 3 after eq. single_sheet; Sec. 5, a stack of
uncorrelated colour sheets; Sec. 2, path-ordered Wilson lines)."""
import numpy as np
import pytest
from scipy.linalg import expm

import synth
from oracle import su, lattice, init_mv, observables


def setup(nc=2, nz=32, nt=4, ns=3, seed=11, mu=1.0, sigma=2.0, dt=0.5, a_T=4.0):
    p = lattice.Params(nc=nc, a_T=a_T, a_L=1.0, dt=dt)
    mv = init_mv.MVParams(m_ir=0.2, uv_cut=0.0, sigma=sigma, zA=0.75 * nz, zB=0.25 * nz)
    rA, rB = synth.mv_sheet_charges(seed, nc, nt, mu, a_T, ns)
    return p, mv, rA, rB


def test_sheet_weights_partition_the_profile():
    prof = np.linspace(0.0, 1.0, 37)
    lam = init_mv.sheet_weights(prof, 4)
    np.testing.assert_allclose(lam.sum(0), 4 * prof, atol=1e-15)
    # sheet k fills only once the sheets before it are complete
    for k in range(1, 4):
        assert np.all(lam[k][lam[k - 1] < 1.0] == 0.0)


@pytest.mark.parametrize("nc", [2, 3])
def test_identical_sheets_reduce_to_one_sheet(nc):
    """rho_k = rho / ns for every k: the sheets commute and add up to the single sheet."""
    ns, nz = 3, 32
    p, mv, rA, rB = setup(nc=nc, nz=nz, ns=1)
    one, U1a = init_mv.initial_state(rA[0], rB[0], nz, p, mv)
    many, U1b = init_mv.initial_state(np.repeat(rA / ns, ns, 0), np.repeat(rB / ns, ns, 0), nz, p, mv)
    np.testing.assert_allclose(many.U, one.U, atol=1e-13)
    np.testing.assert_allclose(U1b, U1a, atol=1e-13)
    np.testing.assert_allclose(many.E, one.E, atol=1e-12)
    np.testing.assert_allclose(many.rhoA, one.rhoA, atol=1e-12)
    np.testing.assert_allclose(many.rhoB, one.rhoB, atol=1e-12)


@pytest.mark.parametrize("nc", [2, 3])
def test_wilson_line_is_the_ordered_product(nc):
    """Behind the nucleus V = e^{-i phi_0} e^{-i phi_1} e^{-i phi_2}; inside sheet 1 the
    partial factor e^{-i s phi_1} stands right of the complete e^{-i phi_0}.  Matrix
    exponentials from scipy; the reversed order differs (the sheets do not commute)."""
    ns = 3
    p, mv, rA, _ = setup(nc=nc, ns=ns, mu=2.0)
    phi = init_mv.sheet_fields(rA, p, mv)
    s = 0.4
    prof = np.array([1.0, (1.0 + s) / ns, 0.0])
    V = init_mv.wilson_lines(phi, prof)
    for y in range(phi.shape[1]):
        for x in range(phi.shape[2]):
            e = [expm(-1j * phi[k, y, x]) for k in range(ns)]
            np.testing.assert_allclose(V[0, y, x], e[0] @ e[1] @ e[2], atol=1e-12)
            np.testing.assert_allclose(V[1, y, x], e[0] @ expm(-1j * s * phi[1, y, x]), atol=1e-12)
            np.testing.assert_allclose(V[2, y, x], np.eye(nc), atol=1e-15)
    e = [expm(-1j * phi[k, 0, 0]) for k in range(ns)]
    assert np.abs(V[0, 0, 0] - e[2] @ e[1] @ e[0]).max() > 1e-3


@pytest.mark.parametrize("nc", [2, 3])
def test_multi_sheet_state_structure(nc):
    nz = 48
    p, mv, rA, rB = setup(nc=nc, nz=nz, ns=4)
    st, U1 = init_mv.initial_state(rA, rB, nz, p, mv)
    a = p.a
    for i in range(3):
        np.testing.assert_allclose(su.expi(a[i] * p.dt * st.E[i]) @ U1[i], st.U[i], atol=1e-13)
    assert lattice.gauss_residual(st)[0] < 1e-14
    P_xy = lattice.plaquette(st.U, 0, 1)
    np.testing.assert_allclose(P_xy, np.broadcast_to(np.eye(nc), P_xy.shape), atol=1e-12)


def test_abelian_sheets_reproduce_their_sources():
    """One colour component (abelian, exact): rho_B(x) = sum_k (dlambda_k(z)/dt)
    (m^2 phi_k - rho_k)(x_T), each sheet sourcing only where it is crossed."""
    nc, nz, ns = 2, 64, 3
    p, mv, rA, rB = setup(nc=nc, nz=nz, ns=ns, mu=0.05)
    rA[:, :2] = 0
    rB[:, :2] = 0
    st, _ = init_mv.initial_state(rA, rB, nz, p, mv)
    z = np.arange(nz) * p.a_L
    half = nz // 2
    for rho_tr, prof, stq, sel in ((rB, init_mv.profile_B, st.rhoB, slice(0, half)),
                                   (rA, init_mv.profile_A, st.rhoA, slice(half, nz))):
        lam0 = init_mv.sheet_weights(prof(z, 0.0, mv), ns)
        lam1 = init_mv.sheet_weights(prof(z, -p.dt, mv), ns)
        expect = np.zeros((nz,) + rho_tr.shape[-2:])
        for k in range(ns):
            phi = init_mv.poisson(rho_tr[k], p.a_T, mv.m_ir, mv.uv_cut)
            expect += ((lam0[k] - lam1[k]) / p.dt)[:, None, None] * (mv.m_ir ** 2 * phi[2] - rho_tr[k, 2])[None]
        got = su.to_components(stq)[..., 2]
        np.testing.assert_allclose(got[sel], expect[sel], rtol=1e-10, atol=1e-13)
    # each sheet's source is confined to its own stretch of the nucleus
    lamB = init_mv.sheet_weights(init_mv.profile_B(z, 0.0, mv), ns)
    # sheet k is half crossed at the last layer with lambda_k > 1/2: sheet 0 leads (largest z)
    assert np.all(np.diff((lamB > 0.5).sum(axis=1)) < 0)


@pytest.mark.parametrize("nc", [2, 3])
def test_field_energy_is_the_sum_over_sheets(nc):
    """Gauge covariance: inside piece k the field strength is that of sheet k alone,
    rotated by the completed sheets, so the E^2 of a multi-sheet nucleus equals the sum
    of the E^2 of nuclei made of one of its sheets each (exact on layers where a single
    sheet changes over the step that defines E; the rest is the overlap of neighbouring
    pieces).  A wrong factor order adds commutators with phi itself: many times more."""
    nz, ns = 64, 4
    p, mv, rA, rB = setup(nc=nc, nz=nz, nt=6, ns=ns, sigma=4.0, mu=1.0)
    rA[:] = 0.0
    st, _ = init_mv.initial_state(rA, rB, nz, p, mv)
    e2 = lambda s: su.algebra_norm2(s.E[:2]).sum(axis=(0, 2, 3))
    full = e2(st)
    parts = np.zeros(nz)
    for k in range(ns):
        rk = np.zeros_like(rB)
        rk[k] = rB[k]
        sk, _ = init_mv.initial_state(rA, rk, nz, p, mv)
        parts += e2(sk)
    assert abs(full.sum() - parts.sum()) < 0.03 * parts.sum(), (full.sum(), parts.sum())


def test_multi_sheet_nucleus_is_light_like():
    """A nucleus with longitudinal colour structure still carries purely transverse,
    equal E and B (p_T ~ 0, p_L ~ eps, |S_L| ~ eps)."""
    nz = 96
    p, mv, rA, rB = setup(nc=3, nz=nz, nt=6, ns=4, sigma=4.0, mu=0.3)
    st, _ = init_mv.initial_state(rA, rB, nz, p, mv)
    eps, pL, pT, SL = observables.tmunu_slices(st)[0]
    for s, sgn in ((slice(0, 48), +1), (slice(48, 96), -1)):
        e = eps[s].sum()
        assert abs(pT[s].sum()) < 0.02 * e
        assert abs(pL[s].sum() - e) < 0.05 * e
        assert abs(sgn * SL[s].sum() - e) < 0.15 * e
