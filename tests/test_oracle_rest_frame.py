"""Pins of the oracle's local rest frame (Sec. 4: eps_loc from diagonalising T^{mu nu}) and of
the Milne coordinates, independent of its closed form."""
import numpy as np

import synth
from oracle import observables, init_mv, lattice


def _slices(eps, pL, pT, SL):
    return np.stack([np.atleast_1d(np.asarray(x, dtype=np.float64)) for x in (eps, pL, pT, SL)])


def test_eigenvalue_problem_of_the_mixed_tensor():
    """eps_loc and v are the timelike eigenpair of T^mu_nu = [[eps, -S], [S, -p_L]]: compare
    with numpy's general eigensolver on random physical tensors (eps > |S|, eps + p_L > 2|S|)."""
    g = np.random.default_rng(7)
    eps = g.uniform(1.0, 2.0, 200)
    pL = g.uniform(-0.2, 1.0, 200) * eps
    SL = g.uniform(-0.45, 0.45, 200) * (eps + pL)
    el, v = observables.local_rest_frame(_slices(eps, pL, 0 * eps, SL))
    for k in range(200):
        M = np.array([[eps[k], -SL[k]], [SL[k], -pL[k]]])
        w, vec = np.linalg.eig(M)
        # timelike eigenvector: |u^0| > |u^z|
        j = int(np.argmax(np.abs(vec[0]) - np.abs(vec[1])))
        assert abs(w[j].real - el[k]) < 1e-12 * eps[k]
        assert abs(vec[1, j].real / vec[0, j].real - v[k]) < 1e-12


def test_boosted_perfect_fluid():
    """T^{mu nu} = (e + p) u^mu u^nu - p g^{mu nu} with u = gamma (1, v): the rest frame gives
    back e and v exactly (to rounding) for any v in (-1, 1)."""
    for e, p in [(1.0, 1.0 / 3.0), (2.0, 0.0), (1.0, 0.9)]:
        for v in (-0.95, -0.3, 0.0, 0.5, 0.99):
            g2 = 1.0 / (1.0 - v * v)
            T00 = (e + p) * g2 - p
            T0z = (e + p) * g2 * v
            Tzz = (e + p) * g2 * v * v + p
            el, vv = observables.local_rest_frame(_slices(T00, Tzz, p, T0z))
            assert abs(el[0] - e) < 1e-12 * max(1.0, e) * g2, (e, p, v, el[0])
            assert abs(vv[0] - v) < 1e-12 * g2, (e, p, v, vv[0])


def test_light_like_single_nucleus_has_no_rest_frame_energy():
    """A lone nucleus before the collision is a light-like field (eps = p_L = S_L up to lattice
    artefacts of order (a_L / sigma)^2), so eps_loc / eps vanishes like their square root,
    ~ 1 / sigma, and the frame velocity tends to +1 as the nucleus gets smoother."""
    ratio, vel = [], []
    for sig in (3.0, 6.0, 12.0):
        w = synth.Workload("su2-128x8x8-single", nc=2, nz=128, nt=8, mu=1.0, sigma=sig, seed=77)
        p = lattice.Params(nc=2, a_T=w.a_T, a_L=w.a_L, dt=w.dt)
        mv = init_mv.MVParams(m_ir=w.m_ir, uv_cut=w.uv_cut, sigma=w.sigma, zA=w.zA, zB=w.zB)
        rA, rB = synth.mv_charges(w.seed, 2, w.nt, w.mu, w.a_T)
        st, _ = init_mv.initial_state(0 * rA, rB, w.nz, p, mv)
        sl, _ = observables.tmunu_slices(st)
        el, v = observables.local_rest_frame(sl)
        ratio.append(el.sum() / sl[0].sum())
        vel.append((sl[0] * v).sum() / sl[0].sum())
    for k in range(2):
        assert 0.4 < ratio[k + 1] / ratio[k] < 0.65, ratio
        assert vel[k + 1] > vel[k], vel
    assert ratio[-1] < 0.07 and vel[-1] > 0.95


def test_milne_coordinates():
    tau, eta = observables.milne(np.array([5.0, 5.0, 5.0, 2.0]), np.array([3.0, 0.0, -3.0, 4.0]), 0.0, 0.0)
    assert np.allclose(tau[:3], [4.0, 5.0, 4.0]) and np.isnan(tau[3])
    assert np.allclose(eta[:3], [0.5 * np.log(8.0 / 2.0), 0.0, -0.5 * np.log(8.0 / 2.0)])
