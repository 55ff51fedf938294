"""Pins of the oracle's MV initial conditions (Sec. 2 and Sec. 3) and observables (Sec. 4)."""
import numpy as np
import pytest

import synth
from oracle import su, lattice, init_mv, observables


def setup(nc=2, nz=32, nt=6, seed=7, mu=1.0, sigma=2.0, dt=0.5, a_T=4.0, m=0.2, uv=0.0,
          zA=None, zB=None):
    p = lattice.Params(nc=nc, a_T=a_T, a_L=1.0, dt=dt)
    mv = init_mv.MVParams(m_ir=m, uv_cut=uv, sigma=sigma,
                          zA=0.75 * nz if zA is None else zA, zB=0.25 * nz if zB is None else zB)
    rA, rB = synth.mv_charges(seed, nc, nt, mu, a_T)
    return p, mv, rA, rB


def test_poisson_inverts_screened_lattice_laplacian():
    _, mv, rA, _ = setup(nc=3, nt=8)
    phi = init_mv.poisson(rA, 4.0, 0.2, 0.0)
    lhs = -init_mv.lattice_laplacian_T(phi, 4.0) + 0.2 ** 2 * phi
    np.testing.assert_allclose(lhs, rA, atol=1e-13)


def test_uv_cut_is_noop_below_max_ktilde_and_active_above():
    _, _, rA, _ = setup(nc=3, nt=8)
    a_T = 4.0
    kmax = np.sqrt(init_mv.ktilde2(8, a_T).max())
    assert kmax == pytest.approx(2 * np.sqrt(2) / a_T)
    full = init_mv.poisson(rA, a_T, 0.2, 0.0)
    np.testing.assert_array_equal(init_mv.poisson(rA, a_T, 0.2, 2.5), full)
    cut = init_mv.poisson(rA, a_T, 0.2, 0.3)
    assert np.abs(cut - full).max() > 1e-3
    # a cut removes exactly the modes above it
    k = np.sqrt(init_mv.ktilde2(8, a_T))
    ft = np.fft.fft2(cut, axes=(-2, -1))
    assert np.abs(ft[:, k > 0.3]).max() < 1e-12


@pytest.mark.parametrize("nc", [2, 3])
def test_initial_state_structure(nc):
    p, mv, rA, rB = setup(nc=nc, nz=48, nt=4, sigma=2.0)
    st, U1 = init_mv.initial_state(rA, rB, 48, p, mv)
    a = p.a
    # eq. lattice_2 maps U(t0 - dt) onto U(t0) with E(t0 - dt/2)
    for i in range(3):
        np.testing.assert_allclose(su.expi(a[i] * p.dt * st.E[i]) @ U1[i], st.U[i], atol=1e-13)
    # Gauss law exact at t0
    assert lattice.gauss_residual(st)[0] < 1e-14
    # transverse plaquettes are trivial (pure gauge per layer) except where both
    # nuclei overlap; the nuclei are 24 cells = 12 sigma apart
    P_xy = lattice.plaquette(st.U, 0, 1)
    np.testing.assert_allclose(P_xy, np.broadcast_to(np.eye(nc), P_xy.shape), atol=1e-12)
    # the seam (z-link between the last and first layers) gives trivial (x,z), (y,z) plaquettes
    for i in range(2):
        P = lattice.plaquette(st.U, i, 2)[-1]
        np.testing.assert_allclose(P, np.broadcast_to(np.eye(nc), P.shape), atol=1e-12)
    # fields vanish between the nuclei (Sec. 3, before eq. 3d_colorfield_2)
    sl, _ = observables.tmunu_slices(st)
    eps = sl[0]
    assert eps[22:26].max() < 1e-10 * eps.max()
    # charges live inside each nucleus
    cA = np.sqrt(su.algebra_norm2(st.rhoA).sum(axis=(1, 2)))
    cB = np.sqrt(su.algebra_norm2(st.rhoB).sum(axis=(1, 2)))
    assert np.argmax(cA) in (35, 36, 37) and np.argmax(cB) in (11, 12, 13)


def test_single_nucleus_is_light_like():
    """Before the collision each nucleus carries purely transverse E and B of equal
    magnitude (Sec. 2): p_T ~ 0, p_L ~ eps, S_L ~ +eps for B (+z) and -eps for A (-z)."""
    for sig in (2.0, 4.0):
        p, mv, rA, rB = setup(nc=3, nz=96, nt=6, sigma=sig, mu=0.3)
        st, _ = init_mv.initial_state(rA, rB, 96, p, mv)
        sl, _ = observables.tmunu_slices(st)
        eps, pL, pT, SL = sl
        B = slice(0, 48)
        A = slice(48, 96)
        tot = lambda x, s: x[s].sum()
        for s, sgn in ((B, +1), (A, -1)):
            assert abs(tot(pT, s)) < 0.02 * tot(eps, s)
            assert abs(tot(pL, s) - tot(eps, s)) < 0.05 * tot(eps, s)
            assert abs(sgn * tot(SL, s) - tot(eps, s)) < 0.15 * tot(eps, s)


def test_single_colour_charge_reproduces_the_source():
    """With one colour component (abelian, exact): rho_B(x) = (dLambda_B(z)/dt)
    * Delta_T phi_B(x_T) = (dLambda_B/dt) (m^2 phi_B - rho_T,B), dLambda the profile
    difference over one time step.  Fixes the profile, Poisson, links, Log and Gauss."""
    nc, nz, nt = 2, 64, 6          # nuclei 8 sigma from the seam
    p, mv, rA, rB = setup(nc=nc, nz=nz, nt=nt, sigma=2.0, mu=0.05)
    rA[:2] = 0
    rB[:2] = 0
    st, _ = init_mv.initial_state(rA, rB, nz, p, mv)
    z = np.arange(nz) * p.a_L
    for rho_tr, prof, stq in ((rB, init_mv.profile_B, st.rhoB), (rA, init_mv.profile_A, st.rhoA)):
        phi = init_mv.poisson(rho_tr, p.a_T, mv.m_ir, mv.uv_cut)
        dlam = (prof(z, 0.0, mv) - prof(z, -p.dt, mv)) / p.dt
        expect = dlam[:, None, None] * (mv.m_ir ** 2 * phi[2] - rho_tr[2])[None]
        got = su.to_components(stq)[..., 2]
        half = nz // 2
        sel = slice(0, half) if stq is st.rhoB else slice(half, nz)
        np.testing.assert_allclose(got[sel], expect[sel], rtol=1e-10, atol=1e-13)
        assert np.abs(su.to_components(stq)[..., :2]).max() < 1e-16


def test_observables_closed_forms():
    """eps of a pure E field is |E|^2/2 (no force when all links are 1); eps of a
    static single-colour magnetic field is (2/a^4) 2 (1 - cos(Theta/2)) per SU(2)
    xy-plaquette with angle Theta."""
    nc = 2
    dims = (3, 4, 4)
    p = lattice.Params(nc=nc, a_T=2.0, a_L=1.0, dt=0.5)
    ec = synth.normal(90, (3,) + dims + (3,), 0.4)
    E = su.from_components(ec, nc)
    U = su.eye_like(E)
    z = np.zeros(dims + (2, 2), complex)
    st = lattice.State(U, E, z, z.copy(), 0, p)
    sl, H = observables.tmunu_slices(st)
    e2 = (ec ** 2).sum(-1)
    np.testing.assert_allclose(sl[0], 0.5 * e2.sum(0).mean(axis=(1, 2)), rtol=1e-14)
    np.testing.assert_allclose(sl[2], 0.5 * e2[2].mean(axis=(1, 2)), rtol=1e-14)
    assert H == pytest.approx(2.0 * 2.0 * 1.0 * 0.5 * e2.sum(), rel=1e-14)
    # magnetic: U_x(x) = exp(i b n_y t^3): xy-plaquette angle Theta = -b everywhere except the wrap row
    b = 0.3
    ny = np.arange(dims[1])[None, :, None]
    alg = np.zeros((3,) + dims + (3,))
    alg[0, ..., 2] = b * ny
    U = su.expi(su.from_components(alg, nc))
    st = lattice.State(U, np.zeros_like(U), z, z.copy(), 0, p)
    # E_new = dt * F is non-zero; use E_new = 0 explicitly to isolate the magnetic part
    sl, _ = observables.tmunu_slices(st, E_new=np.zeros_like(U))
    a = 2.0
    per = 0.5 * 4.0 / a ** 4 * 2 * (1 - np.cos(b / 2))
    Theta_wrap = b * (dims[1] - 1)
    per_wrap = 0.5 * 4.0 / a ** 4 * 2 * (1 - np.cos(Theta_wrap / 2))
    expect = (per * (dims[1] - 1) + per_wrap) / dims[1]
    np.testing.assert_allclose(sl[0], expect, rtol=1e-13)
    np.testing.assert_allclose(sl[2], expect, rtol=1e-13)       # B_L only -> p_T = eps
    np.testing.assert_allclose(sl[1], -expect, rtol=1e-13)      # p_L = -B_L^2/2
