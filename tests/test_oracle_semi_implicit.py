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


def _wave_state(nc, dims, a, k_int, vec, amp, c, dt):
    """Small-amplitude single-colour plane wave A_i(x) = amp Re[vec_i exp(i k.x)] on the links
    (base-site convention), in a cos(w t) phase: A(t - dt) = c A(t), so E(t - dt/2) =
    (1 - c) A(t) / dt.  k_int: integer wave numbers over the lattice (n_x, n_y, n_z)."""
    nz, ny, nx = dims
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    phase = 2 * np.pi * (k_int[0] * xx / nx + k_int[1] * yy / ny + k_int[2] * zz / nz)
    A = np.stack([amp * np.real(vec[i] * np.exp(1j * phase)) for i in range(3)])
    ng = nc * nc - 1
    alg = np.zeros((3,) + dims + (ng,))
    alg[..., ng - 1] = A
    U = su.expi(su.from_components(alg * np.array(a)[:, None, None, None, None], nc))
    E = su.from_components(alg * (1.0 - c) / dt, nc)
    p = lattice.Params(nc=nc, a_T=a[0], a_L=a[2], dt=dt)
    z = np.zeros(dims + (nc, nc), complex)
    return lattice.State(U, E, z, z.copy(), 0, p), A


def _recurrence_c(A):
    """c of A(n + 1) + A(n - 1) = 2 c A(n), least squares over the steps and sites of a
    field history A[n] (well conditioned also where one A(n) nearly vanishes)."""
    num = sum(np.sum((A[n + 1] + A[n - 1]) * A[n]) for n in range(1, len(A) - 1))
    den = sum(2 * np.sum(A[n] * A[n]) for n in range(1, len(A) - 1))
    return num / den


def _link_fields(st, a, nc):
    return np.stack([su.to_components(su.logi(st.U[i]))[..., nc * nc - 2] / a[i] for i in range(3)])


@pytest.mark.parametrize("k_int,dt", [((1, 2, 3), 1.0), ((1, 1, 5), 0.5), ((2, 1, 2), 1.0), ((1, 0, 0), 1.0)])
def test_full_linear_symbol_general_k(k_int, dt):
    """Every polarisation of a general wave vector, including the A_z-polarised wave of the
    E_L equation with its time-averaged transverse Laplacian: the oracle's semi-implicit step
    propagates each physical eigenmode of the hand-derived symbol (tests/_symbol.py) with
    A(t + dt) + A(t - dt) = 2 c A(t), c its generalized eigenvalue."""
    from _symbol import modes
    nc = 2
    dims = (12, 4, 6)
    a = (4.0, 4.0, 1.0)
    k = tuple(2 * np.pi * k_int[i] / (dims[2 - i] * a[i]) for i in range(3))
    cs, vs = modes(k, a, dt)
    checked = 0
    for m in range(3):
        c, v = cs[m], vs[:, m]
        if abs(c - 1.0) < 1e-9:         # the static gauge mode
            continue
        st, A0 = _wave_state(nc, dims, a, k_int, v / np.abs(v).max(), 1e-6, c, dt)
        A = [A0]
        for _ in range(4):
            st = si.semi_implicit_step(st, tol=1e-15)
            A.append(_link_fields(st, a, nc))
        assert abs(_recurrence_c(np.array(A)) - c) < 1e-6, (m, c, _recurrence_c(np.array(A)))
        checked += 1
    assert checked == 2
    if k_int == (1, 0, 0):
        # pure A_z wave along x: c = 1 / (1 + dt^2 K_x / 2)
        Kx = (2 / a[0]) ** 2 * np.sin(k[0] * a[0] / 2) ** 2
        assert np.isclose(cs[np.argmin(np.abs(cs - 1 / (1 + dt ** 2 * Kx / 2)))], 1 / (1 + dt ** 2 * Kx / 2),
                          rtol=1e-12)


def test_symbol_stability_boundary_at_dt_equal_a_L():
    """The symbol has |c| <= 1 for every k of a 7^3 grid over the Brillouin zone at dt = a_L
    (a_T = 4 a_L and a_T = a_L) and |c| > 1 for some k just above it, so the scheme is stable
    exactly up to dt = a_L (the method itself needs dt <= a_L: a charge hops at most one cell
    per step, so the oracle cannot be run beyond it).  The mode at the corner of the zone,
    the first to go unstable, reaches c = -1 at dt = a_L: the oracle follows its symbol at
    dt = 0.98 a_L and keeps it bounded at dt = a_L."""
    from _symbol import modes
    for aT in (4.0, 1.0):
        a = (aT, aT, 1.0)
        for dt, stable in ((1.0, True), (1.05, False)):
            worst = 0.0
            for nx in range(7):
                for ny in range(7):
                    for nzk in range(7):
                        k = (np.pi * nx / 6 / a[0], np.pi * ny / 6 / a[1], np.pi * nzk / 6)
                        worst = max(worst, np.abs(modes(k, a, dt)[0]).max())
            assert (worst <= 1 + 1e-12) == stable, (aT, dt, worst)
    nc, dims, a = 2, (2, 2, 2), (4.0, 4.0, 1.0)
    k_int = (1, 1, 1)
    k = (np.pi / a[0], np.pi / a[1], np.pi)
    for dt in (0.98, 1.0):
        cs, vs = modes(k, a, dt)
        m = int(np.argmin(cs))
        c = cs[m]
        st, A0 = _wave_state(nc, dims, a, k_int, vs[:, m] / np.abs(vs[:, m]).max(), 1e-8, c, dt)
        A = [A0]
        for _ in range(12):
            st = si.semi_implicit_step(st, tol=1e-15)
            A.append(_link_fields(st, a, nc))
        A = np.array(A)
        amp = np.abs(A).reshape(len(A), -1).max(axis=1)
        if dt < 1:
            assert -1 < c < -0.9 and abs(_recurrence_c(A) - c) < 1e-6
        else:
            # c = -1: the cos(w t) start stays an alternating pattern of constant amplitude
            assert abs(c + 1) < 1e-12 and max(amp) < 1.01 * amp[0]


def test_cherenkov_lone_nucleus():
    """Numerical Cherenkov radiation (Sec. 3; Sec. 5): a lone nucleus (dilute MV charges,
    sigma = 2 a_L, moving +z at the speed of light) leaves energy behind it under the
    leapfrog at dt = a_L/2, growing with time along with the total field energy (the moving
    source feeds the lattice modes slower than light); under the semi-implicit scheme at
    dt = a_L, dispersion-free along z, the energy behind it stays orders of magnitude smaller
    and the total stays put.  Energy behind = the eps slices over the 20 layers ending
    5 sigma behind the nucleus centre, as a fraction of the total."""
    nc, nz, nt, sigma, mu, zB = 2, 48, 4, 2.0, 0.05, 8.0
    rA, rB = synth.mv_charges(77, nc, nt, mu, 4.0)
    rA = np.zeros_like(rA)
    from oracle import observables
    curves, Hs = {}, {}
    for scheme, dt in ((0, 0.5), (1, 1.0)):
        p = lattice.Params(nc=nc, a_T=4.0, a_L=1.0, dt=dt)
        mv = init_mv.MVParams(m_ir=0.2, uv_cut=0.0, sigma=sigma, zA=0.75 * nz, zB=zB)
        st, _ = init_mv.initial_state(rA, rB, nz, p, mv)
        if scheme == 1:
            st = si.charges_for_scheme(st)
        z = np.arange(nz)
        frac, H = [], []
        n = int(round(28 / dt))
        for k in range(n + 1):
            nxt = si.semi_implicit_step(st, tol=1e-12) if scheme else lattice.leapfrog_step(st)
            if k % int(round(4 / dt)) == 0:
                sl, h = observables.tmunu_slices(st, E_new=nxt.E)
                zc = zB + k * dt
                win = (z > zc - 5 * sigma - 20) & (z < zc - 5 * sigma)
                frac.append(sl[0][win].sum() / sl[0].sum())
                H.append(h)
            st = nxt
        curves[scheme], Hs[scheme] = np.array(frac), np.array(H)
    lf, sm = curves[0], curves[1]
    # leapfrog: the trailing energy grows from t = 8 on and the total grows
    assert np.all(np.diff(lf[2:]) > 0) and lf[-1] > 3e-3
    assert Hs[0][-1] / Hs[0][0] > 1.03
    # semi-implicit: trailing energy below 3% of the leapfrog's at every t >= 8, total within 1e-3
    assert np.all(sm[2:] < 0.03 * lf[2:]) and sm.max() < 2e-4
    assert abs(Hs[1][-1] / Hs[1][0] - 1) < 1e-3
