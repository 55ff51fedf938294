"""Pins of the oracle's semi-implicit scheme against the properties the paper names
(time-averaged plaquette terms, iterative solve, dispersion-free propagation along
the beam axis, conserved constraint from gauge invariance) and against finite
differences of its own action."""
import numpy as np
import pytest

import synth
from oracle import su, lattice, init_mv, semi_implicit as si


def rand_links(nc, dims, seed, scale=0.7):
    return su.expi(su.from_components(synth.normal(seed, (3,) + dims + (nc * nc - 1,), scale), nc))


@pytest.mark.parametrize("nc", [2, 3])
def test_forces_match_finite_differences(nc):
    dims = (3, 3, 3)
    a = (2.0, 2.0, 1.0)
    U0 = rand_links(nc, dims, 10 + nc)
    U1 = rand_links(nc, dims, 20 + nc)
    t = su.generators(nc)
    g = {0: si.grad(U0, U1, a, 0), 1: si.grad(U0, U1, a, 1)}
    rng = synth.rng(5)
    eps = 1e-5
    for _ in range(12):
        which = int(rng.integers(2))
        d = int(rng.integers(3))
        site = tuple(int(rng.integers(n)) for n in dims)
        b = int(rng.integers(nc * nc - 1))
        vals = []
        for sgn in (1, -1):
            Uv = (U0 if which == 0 else U1).copy()
            Uv[d][site] = su.expi(sgn * eps * t[b]) @ Uv[d][site]
            vals.append(si.potential(Uv, U1, a) if which == 0 else si.potential(U0, Uv, a))
        fd = (vals[0] - vals[1]) / (2 * eps)
        an = 2.0 * np.real(np.trace(t[b] @ g[which][d][site]))
        assert abs(fd - an) < 1e-8 * max(1.0, abs(an)), (which, d, site, b, fd, an)


@pytest.mark.parametrize("nc", [2, 3])
def test_potential_gauge_invariant_and_static_limit(nc):
    dims = (3, 4, 3)
    a = (4.0, 4.0, 1.0)
    U0 = rand_links(nc, dims, 30)
    U1 = rand_links(nc, dims, 31)
    Om = su.expi(su.from_components(synth.normal(32, dims + (nc * nc - 1,), 2.0), nc))
    p = lattice.Params(nc, a[0], a[2], 0.5)

    def gt(U):
        z = np.zeros(dims + (nc, nc), complex)
        return lattice.gauge_transform(lattice.State(U, np.zeros_like(U), z, z, 0, p), Om).U

    v = si.potential(U0, U1, a)
    assert abs(si.potential(gt(U0), gt(U1), a) - v) < 1e-12 * abs(v)
    # slices equal: the action reduces to sum P.P/(a_i a_j)^2 / 2 over all planes
    Us = rand_links(nc, dims, 33, 0.05)
    ref = 0.0
    for (i, j) in ((0, 1), (1, 2), (2, 0)):
        P = su.proj(lattice.plaquette(Us, i, j))
        ref += 0.5 * np.sum(su.algebra_norm2(P)) / (a[i] * a[j]) ** 2
    assert abs(si.potential(Us, Us, a) - ref) < 1e-12 * ref


@pytest.mark.parametrize("nc,dt", [(2, 0.5), (3, 1.0)])
def test_modified_gauss_law_conserved_through_hops(nc, dt):
    nz, nt = 16, 4
    p = lattice.Params(nc=nc, a_T=4.0, a_L=1.0, dt=dt)
    mv = init_mv.MVParams(m_ir=0.2, sigma=1.5, zA=12.0, zB=4.0)
    rA, rB = synth.mv_charges(40 + nc, nc, nt, 0.5, 4.0)
    st, _ = init_mv.initial_state(rA, rB, nz, p, mv)
    st = si.charges_for_scheme(st)
    assert si.gauss_mod_residual(st) < 1e-14
    std0 = lattice.gauss_residual(st)[0]
    for _ in range(6):
        st, it = si.semi_implicit_step(st, tol=1e-15, return_iters=True)
        assert it < 60
        assert si.gauss_mod_residual(st) < 1e-12
    # the standard Gauss law is not the conserved one, but stays close (O(dt^2) terms)
    assert lattice.gauss_residual(st)[0] < 0.25
    assert std0 > 1e-6


def _plane_wave(nc, dims, a, k, pol, amp=1e-6):
    nx = np.arange(dims[2])[None, None, :]
    nz = np.arange(dims[0])[:, None, None]
    phase = 2 * np.pi * (k[0] * nx / dims[2] + k[2] * nz / dims[0])
    alg = np.zeros((3,) + dims + (nc * nc - 1,))
    alg[pol, ..., 2] = a[pol] * amp * np.cos(phase)
    return su.expi(su.from_components(alg, nc))


@pytest.mark.parametrize("k,dt", [((0, 0, 3), 1.0), ((0, 0, 7), 1.0), ((2, 0, 5), 1.0), ((3, 0, 6), 0.5)])
def test_abelian_dispersion_closed_form(k, dt):
    """y-polarised single-colour wave with k = (k_x, 0, k_z): the scheme's linearised
    recurrence is A(t+dt) + A(t-dt) = 2 cos(w dt) A(t) with
        cos(w dt) = (1 - dt^2 K_z / 2) / (1 + dt^2 K_x / 2),  K_i = (2/a_i)^2 sin^2(k_i a_i / 2),
    which at k_x = 0 and dt = a_L gives w = k_z exactly (no dispersion along z)."""
    nc = 2
    dims = (16, 2, 8)
    a = (4.0, 4.0, 1.0)
    p = lattice.Params(nc=nc, a_T=4.0, a_L=1.0, dt=dt)
    U = _plane_wave(nc, dims, a, k, pol=1)
    z = np.zeros(dims + (2, 2), complex)
    st = lattice.State(U, np.zeros_like(U), z, z.copy(), 0, p)
    A = []
    for _ in range(4):
        A.append(su.to_components(su.logi(st.U[1]))[..., 2])
        st = si.semi_implicit_step(st, tol=1e-15)
    A = np.array(A)
    kx = 2 * np.pi * k[0] / dims[2]
    kz = 2 * np.pi * k[2] / dims[0]
    Kx = (2 / a[0]) ** 2 * np.sin(kx / 2) ** 2
    Kz = (2 / a[2]) ** 2 * np.sin(kz / 2) ** 2
    expect = (1 - dt ** 2 * Kz / 2) / (1 + dt ** 2 * Kx / 2)
    for n in (1, 2):
        msk = np.abs(A[n]) > 0.3 * np.abs(A[n]).max()
        got = ((A[n + 1] + A[n - 1]) / (2 * A[n]))[msk]
        np.testing.assert_allclose(got, expect, rtol=1e-7, atol=1e-8)
    if k[0] == 0 and dt == 1.0:
        assert abs(np.arccos(expect) - kz) < 1e-12


def test_stable_where_leapfrog_is_not():
    """dt = a_L with a_T = 4 a_L: the leapfrog violates its CFL bound and a mode near the
    z Brillouin-zone edge with transverse momentum grows; the semi-implicit scheme keeps it
    bounded."""
    nc = 2
    dims = (8, 2, 4)
    a = (4.0, 4.0, 1.0)
    p = lattice.Params(nc=nc, a_T=4.0, a_L=1.0, dt=1.0)
    U = _plane_wave(nc, dims, a, (2, 0, 4), pol=1)     # k_x = pi/a_x, k_z = pi
    z = np.zeros(dims + (2, 2), complex)
    s0 = lattice.State(U, np.zeros_like(U), z, z.copy(), 0, p)

    def amp(st):
        return np.abs(su.to_components(su.logi(st.U[1]))).max()

    a0 = amp(s0)
    lf, sm = s0, s0
    hist = []
    for _ in range(30):
        lf = lattice.leapfrog_step(lf)
        sm = si.semi_implicit_step(sm, tol=1e-14)
        hist.append(amp(sm))
    assert amp(lf) > 100 * a0
    # bounded oscillation: the start (E = 0) excites amplitude a0 / cos(w dt / 2), no growth after
    assert max(hist[15:]) < 1.02 * max(hist[:15]) and max(hist) < 6 * a0


def test_potential_symmetric_in_the_two_slices():
    """v(m, m+1) is symmetric under exchange of the slices, so the force on the later
    slice's links is the force on the earlier slice's links with the arguments swapped."""
    nc, dims = 3, (3, 3, 3)
    a = (4.0, 4.0, 1.0)
    U0 = rand_links(nc, dims, 60)
    U1 = rand_links(nc, dims, 61)
    assert abs(si.potential(U0, U1, a) - si.potential(U1, U0, a)) < 1e-12 * abs(si.potential(U0, U1, a))
    f1, f2 = si.f_forces(U0, U1, a)
    g1, _ = si.f_forces(U1, U0, a)
    np.testing.assert_allclose(f2, g1, atol=1e-13)
