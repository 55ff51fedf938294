"""Pins of the oracle's leapfrog + CPIC evolution (Sec. 3) against invariants and
closed forms that the paper and the mathematics fix."""
import numpy as np
import pytest

import synth
from oracle import su, lattice, init_mv, observables


def mv_state(nc=2, nz=16, nt=4, seed=5, mu=1.0, sigma=1.5, dt=0.5, a_T=4.0):
    p = lattice.Params(nc=nc, a_T=a_T, a_L=1.0, dt=dt)
    mv = init_mv.MVParams(m_ir=0.2, uv_cut=0.0, sigma=sigma, zA=0.75 * nz, zB=0.25 * nz)
    rA, rB = synth.mv_charges(seed, nc, nt, mu, a_T)
    st, _ = init_mv.initial_state(rA, rB, nz, p, mv)
    return st


def random_state(nc, dims, seed, uscale=0.8, escale=0.3, dt=0.5, a_T=4.0, a_L=1.0):
    p = lattice.Params(nc=nc, a_T=a_T, a_L=a_L, dt=dt)
    ng = nc * nc - 1
    Ua = synth.normal(seed, (3,) + dims + (ng,), uscale)
    Ea = synth.normal(seed + 1, (3,) + dims + (ng,), escale)
    return init_mv.state_from_algebra(Ua, Ea, p)


def test_hop_schedule_one_cell_every_two_steps():
    p = lattice.Params(nc=2, a_T=4.0, a_L=1.0, dt=0.5)
    hops = [s for s in range(0, 12) if lattice.is_hop_step(s, p)]
    assert hops == [1, 3, 5, 7, 9, 11]
    p1 = lattice.Params(nc=2, a_T=4.0, a_L=1.0, dt=1.0)
    assert all(lattice.is_hop_step(s, p1) for s in range(10))
    # over n steps a charge advances n dt / a_L cells (speed of light)
    assert lattice.hop_count(99, p) - lattice.hop_count(-1, p) == 50
    p3 = lattice.Params(nc=2, a_T=4.0, a_L=1.0, dt=0.25)
    assert lattice.hop_count(399, p3) - lattice.hop_count(-1, p3) == 100


@pytest.mark.parametrize("nc", [2, 3])
def test_gauss_law_exact_through_hops(nc):
    st = mv_state(nc=nc, nz=16, nt=4, seed=21 + nc)
    g0, _ = lattice.gauss_residual(st)
    assert g0 < 1e-14
    for _ in range(12):
        st = lattice.leapfrog_step(st)
        g, gmax = lattice.gauss_residual(st)
        assert g < 1e-13 and gmax < 1e-13
    # charges did move: six hops at dt = a_L / 2
    assert lattice.hop_count(11, st.params) - lattice.hop_count(-1, st.params) == 6


def test_gauss_law_detects_a_broken_current():
    # a planted mistake in the current (wrong sign) must break the Gauss law
    st = mv_state(nc=2, nz=16, nt=4, seed=3)
    p = st.params
    st = lattice.leapfrog_step(st)            # step 0: no hop
    rhoA, rhoB, j = lattice.cpic_hop(st.U, st.rhoA, st.rhoB, p)
    E_bad = st.E + p.dt * (lattice.force(st.U, p.a) - j)
    bad = lattice.State(st.U, E_bad, rhoA, rhoB, st.step + 1, p)
    assert lattice.gauss_residual(bad)[0] > 1e-3


@pytest.mark.parametrize("nc", [2, 3])
def test_unitarity_preserved(nc):
    st = random_state(nc, (4, 3, 3), seed=30 + nc)
    st = lattice.evolve(st, 40)
    # exact in exact arithmetic; rounding grows at most linearly in the number of steps
    assert lattice.unitarity_violation(st.U) < 40 * 1e-14


@pytest.mark.parametrize("nc", [2, 3])
def test_gauge_covariance(nc):
    st = mv_state(nc=nc, nz=12, nt=3, seed=40 + nc, sigma=1.2)
    dims = st.U.shape[1:4]
    Om = su.expi(su.from_components(synth.normal(50 + nc, dims + (nc * nc - 1,), 2.0), nc))
    a = lattice.evolve(lattice.gauge_transform(st, Om), 6)
    b = lattice.gauge_transform(lattice.evolve(st, 6), Om)
    for x, y in ((a.U, b.U), (a.E, b.E), (a.rhoA, b.rhoA), (a.rhoB, b.rhoB)):
        np.testing.assert_allclose(x, y, atol=1e-12)
    oa = observables.observables(a)
    ob = observables.observables(lattice.evolve(st, 6))
    np.testing.assert_allclose(oa["tmunu_z"], ob["tmunu_z"], atol=1e-12, rtol=1e-10)
    assert abs(oa["energy"] - ob["energy"]) < 1e-10 * abs(ob["energy"])


def _free_energy_series(dt, nsteps_time, nc=2):
    # free evolution, rho = 0: small random links, E = 0 (Gauss trivially satisfied)
    p = lattice.Params(nc=nc, a_T=1.0, a_L=1.0, dt=dt)
    dims = (4, 4, 4)
    Ua = synth.normal(60, (3,) + dims + (nc * nc - 1,), 0.3)
    U = su.expi(su.from_components(Ua, nc))
    E = np.zeros_like(U)
    z = np.zeros_like(U[0])
    st = lattice.State(U, E, z, z.copy(), 0, p)
    H = []
    n = int(round(nsteps_time / dt))
    for _ in range(n):
        H.append(observables.tmunu_slices(st)[1])
        st = lattice.leapfrog_step(st)
    return np.array(H)


def test_free_energy_conservation_dt2_scaling():
    T = 8.0
    H1 = _free_energy_series(0.1, T)
    H2 = _free_energy_series(0.05, T)
    f1 = H1.max() - H1.min()
    f2 = H2.max() - H2.min()
    # bounded, no secular drift, fluctuation ~ dt^2
    assert f1 / H1.mean() < 0.05
    assert 3.8 < f1 / f2 < 4.2
    n = len(H2) // 2
    assert abs(H2[:n].mean() - H2[n:].mean()) < 0.5 * f2


@pytest.mark.parametrize("a_T,dt,k", [(1.0, 0.2, (0, 1, 2)), (4.0, 0.5, (0, 2, 3)),
                                      (4.0, 0.25, (0, 1, 5))])
def test_leapfrog_dispersion_relation(a_T, dt, k):
    """Small single-colour plane wave A_x ~ cos(k.x): the linearised leapfrog obeys
    A(t+dt) + A(t-dt) = 2 cos(w dt) A(t) with (2/dt)^2 sin^2(w dt/2) = sum_i (2/a_i)^2 sin^2(k_i a_i/2)."""
    nc = 2
    dims = (16, 8, 8)          # (nz, ny, nx)
    a = (a_T, a_T, 1.0)
    p = lattice.Params(nc=nc, a_T=a_T, a_L=1.0, dt=dt)
    nx = np.arange(dims[2])[None, None, :]
    ny = np.arange(dims[1])[None, :, None]
    nz = np.arange(dims[0])[:, None, None]
    kv = [2 * np.pi * k[0] / dims[2], 2 * np.pi * k[1] / dims[1], 2 * np.pi * k[2] / dims[0]]
    phase = kv[0] * nx + kv[1] * ny + kv[2] * nz
    amp = 1e-6
    alg = np.zeros((3,) + dims + (3,))
    alg[0, ..., 2] = a[0] * amp * np.cos(phase)         # polarisation x, k has no x part
    st = lattice.State(su.expi(su.from_components(alg, nc)), np.zeros((3,) + dims + (2, 2), complex),
                       np.zeros(dims + (2, 2), complex), np.zeros(dims + (2, 2), complex), 0, p)
    A = []
    for _ in range(4):
        A.append(su.to_components(su.logi(st.U[0]))[..., 2])
        st = lattice.leapfrog_step(st)
    A = np.array(A)
    msk = np.abs(A[1]) > 0.3 * np.abs(A[1]).max()
    cos_w = ((A[2] + A[0]) / (2 * A[1]))[msk]
    Om2 = sum((2 / a[i]) ** 2 * np.sin(kv[i] / 2) ** 2 for i in range(3))
    expect = 1 - dt ** 2 * Om2 / 2
    np.testing.assert_allclose(cos_w, expect, rtol=1e-8, atol=1e-9)


def test_time_reversibility_free():
    nc = 3
    st0 = random_state(nc, (4, 3, 3), seed=70, escale=0.2)
    st0 = lattice.State(st0.U, st0.E, np.zeros_like(st0.rhoA), np.zeros_like(st0.rhoB), 0, st0.params)
    # without charges the Gauss law needs D.E = 0; use E = 0 so it holds trivially
    st0.E[:] = 0
    n = 10
    st = lattice.evolve(st0, n)
    p = st.params
    a = p.a
    # undo the last link update, flip E, run n-1 steps: arrive at (U_0, -E_{1/2})
    Ub = np.stack([su.expi(-a[i] * p.dt * st.E[i]) @ st.U[i] for i in range(3)])
    rev = lattice.State(Ub, -st.E, st.rhoA, st.rhoB, 0, p)
    rev = lattice.evolve(rev, n - 1)
    fwd1 = lattice.leapfrog_step(st0)
    np.testing.assert_allclose(rev.U, st0.U, atol=1e-12)
    np.testing.assert_allclose(rev.E, -fwd1.E, atol=1e-12)


def test_abelian_reduction_to_compact_u1():
    """All fields along t^3 of SU(2): the evolution is compact U(1) lattice
    electrodynamics; compare with an independent angle-variable update."""
    nc = 2
    dims = (5, 4, 4)
    a = (2.0, 2.0, 1.0)
    dt = 0.4
    p = lattice.Params(nc=nc, a_T=2.0, a_L=1.0, dt=dt)
    th = synth.normal(80, (3,) + dims, 0.7)          # link angles: U_i = exp(i th_i t^3)
    e = synth.normal(81, (3,) + dims, 0.2)           # E^3 components
    alg_U = np.zeros((3,) + dims + (3,))
    alg_U[..., 2] = th
    alg_E = np.zeros((3,) + dims + (3,))
    alg_E[..., 2] = e
    zero = np.zeros(dims + (2, 2), complex)
    st = lattice.State(su.expi(su.from_components(alg_U, nc)), su.from_components(alg_E, nc),
                       zero, zero.copy(), 0, p)

    def sh(x, i, d):
        return np.roll(x, -d, axis={0: 2, 1: 1, 2: 0}[i])

    for _ in range(15):
        # independent U(1): plaquette angle, force 2 sin(Theta/2) per plaquette
        f = np.zeros_like(th)
        for i in range(3):
            for j in range(3):
                if i == j:
                    continue
                Tp = th[i] + sh(th[j], i, 1) - sh(th[i], j, 1) - th[j]
                tj_m = sh(th[j], j, -1)
                Tm = th[i] - sh(tj_m, i, 1) - sh(th[i], j, -1) + tj_m
                f[i] += 2 * (np.sin(Tp / 2) + np.sin(Tm / 2)) / a[j] ** 2
            f[i] *= -1 / a[i]
        e = e + dt * f
        th = th + np.array(a)[:, None, None, None] * dt * e
        st = lattice.leapfrog_step(st)
    got_e = su.to_components(st.E)[..., 2]
    np.testing.assert_allclose(got_e, e, atol=1e-13)
    expect_U = su.expi(su.from_components(np.concatenate(
        [np.zeros((3,) + dims + (2,)), th[..., None]], axis=-1), nc))
    np.testing.assert_allclose(st.U, expect_U, atol=1e-12)
