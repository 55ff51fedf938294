"""GPU parity of the semi-implicit scheme against the oracle: per field component over
several steps with CPIC hops, the initial charges of the modified Gauss law, and its
conservation on the GPU states (evaluated by the oracle)."""
import sys
import numpy as np
import pytest

import synth
from oracle import lattice, init_mv, observables, semi_implicit as si
from _gpu import gpu, lattice_or_skip, to_comp, from_comp, state_errs, mv_setup, new_lattice

pytestmark = gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("nc,nz,nt,dt", [(2, 16, 4, 1.0), (3, 24, 6, 0.5), (3, 16, 5, 1.0)])
def test_semi_implicit_parity(nc, nz, nt, dt):
    pkg = lattice_or_skip()
    w = synth.Workload(f"su{nc}-{nz}x{nt}", nc=nc, nz=nz, nt=nt, dt=dt, mu=0.5, sigma=1.5, seed=300 + nz)
    say("case: semi-implicit", w.name, "dt", dt)
    p, mv = mv_setup(w)
    rA, rB = synth.mv_charges(w.seed, nc, nt, w.mu, w.a_T)
    st, _ = init_mv.initial_state(rA, rB, nz, p, mv)
    st = si.charges_for_scheme(st)
    lat = new_lattice(pkg, w, scheme=1, max_iter=100, tol=1e-15)
    lat.init_state(*to_comp(st), step0=0)
    for s in range(5):
        st = si.semi_implicit_step(st, tol=1e-15)
        lat.step(1)
        errs = state_errs(lat.get_state(), st)
        say(" step", s + 1, "iters", lat.last_iterations, {k: f"{v:.1e}" for k, v in errs.items()})
        assert max(errs.values()) < 1e-10, (s, errs)
    gst = from_comp(lat.get_state(), nc, (nz, nt, nt), p)
    assert si.gauss_mod_residual(gst) < 1e-12
    # observables at integer time with E averaged over the two half steps (the definition
    # the leapfrog uses): E(t + dt/2) from the oracle's own solve of the next step
    st_next = si.semi_implicit_step(st, tol=1e-15)
    oo = observables.observables(st, E_new=st_next.E)
    go = lat.observables()
    sl = oo["tmunu_z"]
    err = np.max(np.abs(go["tmunu_z"] - sl) / np.abs(sl).max(axis=1, keepdims=True))
    say(" T^{mu nu} slices (averaged time level)", err, "H", abs(go["energy"] - oo["energy"]) / oo["energy"])
    assert err < 1e-9
    assert abs(go["energy"] - oo["energy"]) < 1e-10 * abs(oo["energy"])
    # the one-sided level (E(t - dt/2) for both halves) differs by O(dt): the test sees it
    one_sided = observables.observables(st, E_new=st.E)["tmunu_z"]
    assert np.max(np.abs(one_sided - sl) / np.abs(sl).max(axis=1, keepdims=True)) > 1e-6
    # observing step: the same numbers from the solve that the step itself commits
    obs = lat.obs_buffer()
    lat.step_observe(1, obs)
    o2 = pkg.Lattice.unpack_obs(obs, nz)
    assert np.max(np.abs(o2["tmunu_z"] - sl) / np.abs(sl).max(axis=1, keepdims=True)) < 1e-9
    errs = state_errs(lat.get_state(), st_next)
    assert max(errs.values()) < 1e-10, errs


def test_semi_implicit_init_mv_charges():
    pkg = lattice_or_skip()
    w = synth.Workload("su3-32x6", nc=3, nz=32, nt=6, dt=1.0, mu=0.5, sigma=2.0, seed=330)
    p, mv = mv_setup(w)
    rA, rB = synth.mv_charges(w.seed, 3, w.nt, w.mu, w.a_T)
    st, _ = init_mv.initial_state(rA, rB, w.nz, p, mv)
    st = si.charges_for_scheme(st)
    lat = new_lattice(pkg, w, scheme=1, max_iter=100, tol=1e-14)
    lat.init_mv(rA, rB, m_ir=w.m_ir, sigma=w.sigma, zA=w.zA, zB=w.zB)
    errs = state_errs(lat.get_state(), st)
    assert max(errs.values()) < 1e-10, errs
    lat.step(8)
    gst = from_comp(lat.get_state(), 3, (w.nz, w.nt, w.nt), p)
    assert si.gauss_mod_residual(gst) < 1e-12


@pytest.mark.parametrize("nc", [2, 3])
def test_semi_implicit_fp32_against_fp64_oracle(nc):
    """The semi-implicit scheme in FP32 storage and arithmetic (fixed point iterated to
    1e-6, about the FP32 resolution) stays within FP32 rounding of the FP64 oracle over 6
    steps with hops; observables within 1e-4."""
    pkg = lattice_or_skip()
    nz, nt, dt = 24, 6, 1.0
    w = synth.Workload(f"su{nc}-{nz}x{nt}-fp32", nc=nc, nz=nz, nt=nt, dt=dt, mu=0.5, sigma=1.5, seed=370 + nc)
    say("case: semi-implicit fp32", w.name)
    p, mv = mv_setup(w)
    rA, rB = synth.mv_charges(w.seed, nc, nt, w.mu, w.a_T)
    st, _ = init_mv.initial_state(rA, rB, nz, p, mv)
    st = si.charges_for_scheme(st)
    lat = new_lattice(pkg, w, fp=32, scheme=1, max_iter=100, tol=1e-6)
    lat.init_state(*to_comp(st), step0=0)
    worst = 0.0
    for s in range(6):
        st = si.semi_implicit_step(st, tol=1e-15)
        lat.step(1)
        errs = state_errs(lat.get_state(), st)
        worst = max(worst, max(errs.values()))
        assert max(errs.values()) < 1e-4, (s, errs)
    say(" worst per-component error over 6 steps", worst)
    go = lat.observables()
    oo = observables.observables(st, E_new=si.semi_implicit_step(st, tol=1e-15).E)
    sl = oo["tmunu_z"]
    err = np.max(np.abs(go["tmunu_z"] - sl) / np.abs(sl).max(axis=1, keepdims=True))
    say(" T^{mu nu} slices", err)
    assert err < 1e-4


@pytest.mark.parametrize("k,dt", [((0, 0, 3), 1.0), ((0, 0, 7), 1.0), ((2, 0, 5), 1.0), ((3, 0, 6), 0.5)])
def test_semi_implicit_dispersion_on_the_gpu(k, dt):
    """A small y-polarised single-colour wave with k = (k_x, 0, k_z) under the GPU's
    semi-implicit scheme: A(t+dt) + A(t-dt) = 2 cos(w dt) A(t) with the closed form
    cos(w dt) = (1 - dt^2 K_z / 2) / (1 + dt^2 K_x / 2), K_i = (2/a_i)^2 sin^2(k_i a_i / 2);
    at k_x = 0 and dt = a_L, w = k_z: no dispersion along the beam axis."""
    pkg = lattice_or_skip()
    from oracle import su
    nc, nz, nt = 2, 16, 8
    say(f"case: semi-implicit dispersion k {k} dt {dt}")
    dims = (nz, nt, nt)
    a = (4.0, 4.0, 1.0)
    p = lattice.Params(nc=nc, a_T=4.0, a_L=1.0, dt=dt)
    nx = np.arange(nt)[None, None, :]
    nzv = np.arange(nz)[:, None, None]
    phase = 2 * np.pi * (k[0] * nx / nt + k[2] * nzv / nz) + np.zeros(dims)
    alg = np.zeros((3,) + dims + (3,))
    alg[1, ..., 2] = a[1] * 1e-6 * np.cos(phase)
    U = su.expi(su.from_components(alg, nc))
    z = np.zeros(dims + (2, 2), complex)
    st = lattice.State(U, np.zeros_like(U), z, z.copy(), 0, p)
    lat = pkg.Lattice(nc=nc, nz=nz, nt=nt, a_T=4.0, a_L=1.0, dt=dt, fp=64, scheme=1, max_iter=100, tol=1e-15)
    lat.init_state(*to_comp(st), step0=0)
    A = []
    for _ in range(4):
        g = from_comp(lat.get_state(), nc, dims, p)
        A.append(su.to_components(su.logi(g.U[1]))[..., 2])
        lat.step(1)
    A = np.array(A)
    kx, kz = 2 * np.pi * k[0] / nt, 2 * np.pi * k[2] / nz
    Kx = (2 / a[0]) ** 2 * np.sin(kx / 2) ** 2
    Kz = (2 / a[2]) ** 2 * np.sin(kz / 2) ** 2
    expect = (1 - dt ** 2 * Kz / 2) / (1 + dt ** 2 * Kx / 2)
    for n in (1, 2):
        msk = np.abs(A[n]) > 0.3 * np.abs(A[n]).max()
        got = ((A[n + 1] + A[n - 1]) / (2 * A[n]))[msk]
        say(f"  n {n}: cos(w dt) {float(np.mean(got)):.12f} closed form {expect:.12f}")
        np.testing.assert_allclose(got, expect, rtol=1e-7, atol=1e-8)
    if k[0] == 0 and dt == 1.0:
        assert abs(np.arccos(expect) - kz) < 1e-12
