"""Pins of the oracle's differentiation-form reference (tangent-linear leapfrog and the
slab-energy loss) against a library routine, closed forms, finite differences and gauge
invariance."""
import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import su, lattice, init_mv, adjoint


def mv_state(nc, nz=12, nt=4, seed=11, mu=1.0, sigma=1.2, dt=0.5, a_T=4.0):
    p = lattice.Params(nc=nc, a_T=a_T, a_L=1.0, dt=dt)
    mv = init_mv.MVParams(m_ir=0.2, uv_cut=0.0, sigma=sigma, zA=0.75 * nz, zB=0.25 * nz)
    rA, rB = synth.mv_charges(seed, nc, nt, mu, a_T)
    st, _ = init_mv.initial_state(rA, rB, nz, p, mv)
    return st


def random_state(nc, dims, seed, uscale=0.8, escale=0.3, dt=0.5, a_T=4.0, rscale=0.2):
    p = lattice.Params(nc=nc, a_T=a_T, a_L=1.0, dt=dt)
    ng = nc * nc - 1
    st = init_mv.state_from_algebra(synth.normal(seed, (3,) + dims + (ng,), uscale),
                                    synth.normal(seed + 1, (3,) + dims + (ng,), escale), p)
    st.rhoA = su.from_components(synth.normal(seed + 2, dims + (ng,), rscale), nc)
    st.rhoB = su.from_components(synth.normal(seed + 3, dims + (ng,), rscale), nc)
    return st


def random_tangent(st, seed, parts="UEAB"):
    nc = st.params.nc
    ng = nc * nc - 1
    dims = st.U.shape[1:4]
    return adjoint.tangent_from_components(
        st,
        synth.normal(seed, (3,) + dims + (ng,), 1.0) if "U" in parts else None,
        synth.normal(seed + 1, (3,) + dims + (ng,), 1.0) if "E" in parts else None,
        synth.normal(seed + 2, dims + (ng,), 1.0) if "A" in parts else None,
        synth.normal(seed + 3, dims + (ng,), 1.0) if "B" in parts else None)


@pytest.mark.parametrize("nc", [2, 3])
def test_exponential_derivative_matches_expm_frechet(nc):
    ng = nc * nc - 1
    for seed, c in ((1, 0.3), (2, 2.0), (3, 5.0)):
        H = su.from_components(synth.normal(seed, (ng,), 1.0), nc)
        dH = su.from_components(synth.normal(seed + 10, (ng,), 1.0), nc)
        expA, L = scipy.linalg.expm_frechet(1j * c * H, 1j * c * dH)
        xi = adjoint.dexpi_left(H, dH, c)
        assert np.abs(-1j * L @ su.dag(expA) - xi).max() < 1e-13 * max(1.0, c)
        # the left derivative is hermitian traceless
        assert np.abs(xi - su.dag(xi)).max() < 1e-14 * max(1.0, c)
    # degenerate spectrum (H = 0): the derivative is c dH
    assert np.abs(adjoint.dexpi_left(np.zeros((nc, nc), complex), dH, 0.7) - 0.7 * dH).max() < 1e-15


def test_slab_loss_closed_forms():
    # unit links: only the electric term, a^3 * 1/2 |E|^2 per site of the slab
    p = lattice.Params(nc=3, a_T=2.0, a_L=0.5, dt=0.25)
    dims = (6, 3, 3)
    e = np.array([0.1, -0.2, 0.3, 0.0, 0.5, -0.1, 0.2, 0.4])
    Ea = np.broadcast_to(e, (3,) + dims + (8,))
    st = init_mv.state_from_algebra(np.zeros((3,) + dims + (8,)), Ea, p)
    L = adjoint.slab_loss(st, 2, 5)
    assert L == pytest.approx(2.0 * 2.0 * 0.5 * 3 * 9 * 0.5 * 3 * np.sum(e * e), rel=1e-14)
    # abelian field along t^3 with a uniform flux phi in the xy plane: U_x(x, y) =
    # exp(i phi y t^3), U_y = U_z = 1, phi = 4 pi / n_t so that the wrap-around row closes
    # the flux (exp(i theta t^3) has period 4 pi).  Every xy plaquette is exp(-i phi t^3)
    # with Re Tr = 2 cos(phi/2) + 1; the xz and yz plaquettes are 1.
    nt = 6
    phi = 4 * np.pi / nt
    dims = (6, nt, nt)
    Ua = np.zeros((3,) + dims + (8,))
    Ua[0, :, :, :, 2] = (phi * np.arange(nt))[None, :, None]
    st = init_mv.state_from_algebra(Ua, np.zeros((3,) + dims + (8,)), p)
    P = lattice.plaquette(st.U, 0, 1)
    assert np.allclose(np.real(su.trace(P)), 2 * np.cos(phi / 2) + 1, atol=1e-14)
    L = adjoint.slab_loss(st, 1, 4)
    expect = (2.0 * 2.0 * 0.5) * 3 * nt * nt * 2.0 / (2.0 * 2.0) ** 2 * (3 - 2 * np.cos(phi / 2) - 1)
    assert L == pytest.approx(expect, rel=1e-13)


def test_zero_steps_gradient_in_E_is_a3_E_on_the_slab():
    st = random_state(3, (6, 3, 3), seed=40)
    a = st.params.a
    tan = random_tangent(st, 50, parts="E")
    _, d = adjoint.jvp(st, tan, 0, 2, 4)
    expect = a[0] * a[1] * a[2] * np.sum(su.to_components(st.E[:, 2:4]) * su.to_components(tan[1][:, 2:4]))
    assert d == pytest.approx(expect, rel=1e-13)


@pytest.mark.parametrize("nc", [2, 3])
def test_tangent_linear_matches_central_differences(nc):
    # MV initial state: the charges hop on odd steps, so 5 steps cover both kinds
    st = mv_state(nc)
    st.E = st.E + su.from_components(synth.normal(70, st.E.shape[:-2] + (nc * nc - 1,), 0.05), nc)
    for seed, parts in ((80, "UEAB"), (90, "E"), (100, "AB")):
        tan = random_tangent(st, seed, parts)
        L, d = adjoint.jvp(st, tan, 5, 4, 8)
        fd1 = adjoint.fd_directional(st, tan, 5, 4, 8, h=1e-4)
        fd2 = adjoint.fd_directional(st, tan, 5, 4, 8, h=5e-5)
        assert abs(d) > 1e-3
        # central differences approach the derivative as h^2 (ratio 4 per halving) ...
        assert abs(d - fd1) <= 1e-5 * abs(d), (parts, d, fd1)
        assert 3.5 < abs(fd1 - d) / abs(fd2 - d) < 4.5, (parts, d, fd1, fd2)
        # ... and their Richardson extrapolation (error O(h^4)) agrees to 1e-8
        assert abs(d - (4 * fd2 - fd1) / 3) <= 1e-8 * abs(d), (parts, d, fd1, fd2)


def test_tangent_linear_detects_a_dropped_term():
    # a planted mistake in the oracle: the hop's link term in the rho_A tangent left out
    st = mv_state(2)
    tan = random_tangent(st, 120, "U")
    st1 = lattice.leapfrog_step(st)            # step 0: no hop; step 1 hops
    _, tan1 = adjoint.tangent_step(st, tan)
    good = adjoint.jvp(st1, tan1, 2, 2, 10)[1]
    saved = adjoint.comm
    try:
        calls = []

        def comm_dropping_hop(A, B):
            calls.append(1)
            return 0 * A if len(calls) == 1 else saved(A, B)
        adjoint.comm = comm_dropping_hop
        bad = adjoint.jvp(st1, tan1, 2, 2, 10)[1]
    finally:
        adjoint.comm = saved
    fd = adjoint.fd_directional(st1, tan1, 2, 2, 10, h=1e-4)
    assert abs(good - fd) < 1e-6 * abs(fd)
    assert abs(bad - fd) > 1e-4 * abs(fd)


@pytest.mark.parametrize("nc", [2, 3])
def test_derivative_along_gauge_transformations_vanishes(nc):
    st = mv_state(nc)
    omega = su.from_components(synth.normal(130, st.rhoA.shape[:-2] + (nc * nc - 1,), 1.0), nc)
    tan = adjoint.gauge_tangent(st, omega)
    L, d = adjoint.jvp(st, tan, 4, 3, 9)
    other = adjoint.jvp(st, random_tangent(st, 140), 4, 3, 9)[1]
    assert abs(d) < 1e-12 * max(abs(other), abs(L))
