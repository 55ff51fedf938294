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


# nt = 4, 5, 6: the per-link kernels; nt = 8, 16: the marching pass (x rows in wavefronts),
# with nz below, equal to and across its 16-layer chunks
@pytest.mark.parametrize("nc,nz,nt,dt", [(2, 16, 4, 1.0), (3, 24, 6, 0.5), (3, 16, 5, 1.0), (3, 16, 8, 1.0),
                                         (3, 20, 8, 0.5), (2, 12, 16, 1.0), (2, 40, 8, 0.5)])
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


@pytest.mark.parametrize("nc,nt", [(2, 6), (3, 6), (3, 8)])
def test_semi_implicit_fp32_against_fp64_oracle(nc, nt):
    """The semi-implicit scheme in FP32 storage and arithmetic (fixed point iterated to
    1e-6, about the FP32 resolution) stays within FP32 rounding of the FP64 oracle over 6
    steps with hops; observables within 1e-4 (nt = 8: the marching pass)."""
    pkg = lattice_or_skip()
    nz, dt = 24, 1.0
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
        # the FP32 bar needs the reference to ~1e-8 only; 1e-15 sits at FP64 round-off,
        # which the oracle's plain iteration need not reach on larger lattices
        st = si.semi_implicit_step(st, tol=1e-13)
        lat.step(1)
        errs = state_errs(lat.get_state(), st)
        worst = max(worst, max(errs.values()))
        assert max(errs.values()) < 1e-4, (s, errs)
    say(" worst per-component error over 6 steps", worst)
    go = lat.observables()
    oo = observables.observables(st, E_new=si.semi_implicit_step(st, tol=1e-13).E)
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


@pytest.mark.parametrize("k_int,dt,nt", [((1, 2, 3), 1.0, 6), ((2, 1, 5), 0.5, 6), ((1, 1, 0), 1.0, 6),
                                         ((1, 3, 3), 1.0, 8), ((3, 1, 5), 0.5, 8)])
def test_full_linear_symbol_on_the_gpu(k_int, dt, nt):
    """Every physical polarisation of a general wave vector (the A_z-polarised wave of the
    E_L equation included) propagates under the GPU's semi-implicit step with the cos(w dt)
    of the hand-derived symbol (tests/_symbol.py); nt = 6: the per-link kernels, nt = 8: the
    marching pass."""
    pkg = lattice_or_skip()
    from _symbol import modes
    from test_oracle_semi_implicit import _wave_state, _link_fields, _recurrence_c
    nc, dims, a = 2, (12, nt, nt), (4.0, 4.0, 1.0)   # the library's lattices are nt x nt transverse
    say(f"case: semi-implicit symbol k {k_int} dt {dt}")
    k = tuple(2 * np.pi * k_int[i] / (dims[2 - i] * a[i]) for i in range(3))
    cs, vs = modes(k, a, dt)
    p = lattice.Params(nc=nc, a_T=a[0], a_L=a[2], dt=dt)
    checked = 0
    for m in range(3):
        c, v = cs[m], vs[:, m]
        if abs(c - 1.0) < 1e-9:
            continue
        st, A0 = _wave_state(nc, dims, a, k_int, v / np.abs(v).max(), 1e-6, c, dt)
        lat = pkg.Lattice(nc=nc, nz=dims[0], nt=dims[1], a_T=a[0], a_L=a[2], dt=dt, fp=64, scheme=1,
                          max_iter=100, tol=1e-15)
        lat.init_state(*to_comp(st), step0=0)
        A = [A0]
        for _ in range(4):
            lat.step(1)
            A.append(_link_fields(from_comp(lat.get_state(), nc, dims, p), a, nc))
        got = _recurrence_c(np.array(A))
        say(f"  mode {m}: c {c:.10f} GPU {got:.10f}")
        assert abs(got - c) < 1e-6
        checked += 1
    assert checked == 2


def test_cherenkov_lone_nucleus_on_the_gpu():
    """Numerical Cherenkov radiation on a 256 x 16 x 16 SU(3) lattice: one nucleus (dilute MV
    charges, sigma = 2 a_L) moving +z at the speed of light.  Leapfrog at dt = a_L/2: the
    energy in the 64 layers that end 5 sigma behind the nucleus grows with t and the total
    grows.  Semi-implicit at dt = a_L: the same fraction stays orders of magnitude smaller
    and the total stays put.  Semi-implicit at dt = a_L/2 is dispersive along z like the
    leapfrog and radiates like it."""
    pkg = lattice_or_skip()
    nc, nz, nt, aT, sigma, mu, zB = 3, 256, 16, 4.0, 2.0, 0.05, 32.0
    rA, rB = synth.mv_charges(77, nc, nt, mu, aT)
    rA = np.zeros_like(rA)
    z = np.arange(nz)
    res = {}
    for scheme, dt in ((0, 0.5), (1, 1.0), (1, 0.5)):
        say(f"case: lone nucleus scheme {scheme} dt {dt}")
        lat = pkg.Lattice(nc=nc, nz=nz, nt=nt, a_T=aT, a_L=1.0, dt=dt, fp=64, scheme=scheme, max_iter=300,
                          tol=1e-12)
        lat.init_mv(rA, rB, m_ir=0.2, uv_cut=0.0, sigma=sigma, zA=0.75 * nz, zB=zB)
        per = int(round(16 / dt))
        frac, H = [], []
        for k in range(11):
            o = lat.observables()
            eps = o["tmunu_z"][0]
            zc = zB + 16 * k
            win = (z > zc - 5 * sigma - 64) & (z < zc - 5 * sigma)
            frac.append(eps[win].sum() / eps.sum())
            H.append(o["energy"])
            if k < 10:
                lat.step(per)
        res[(scheme, dt)] = (np.array(frac), np.array(H))
        say("  behind/total at t = 64..160:", " ".join(f"{f:.1e}" for f in frac[4:]),
            f" H(t)/H(0) {H[-1] / H[0]:.5f}")
    lf, Hl = res[(0, 0.5)]
    sm, Hs = res[(1, 1.0)]
    s5, _ = res[(1, 0.5)]
    assert np.all(np.diff(lf[4:]) > 0) and lf[-1] > 2e-2 and Hl[-1] / Hl[0] > 1.05
    assert np.all(sm[4:] < 1e-3 * lf[4:]) and abs(Hs[-1] / Hs[0] - 1) < 3e-3
    assert np.all(s5[4:] > 0.5 * lf[4:])


def _patch_links(Udev, nc, dims, center, half=2):
    """Links U[i] on the periodic (2 half + 1)^3 patch around center, from a device array in
    the C-ABI plain layout (3, r_U, V): oracle matrices (3, n, n, n, N, N), the center at
    (half, half, half)."""
    import torch
    from oracle import components
    nz, ny, nx = dims
    z0, y0, x0 = center
    r = torch.arange(-half, half + 1, device=Udev.device)
    zz = (z0 + r) % nz
    yy = (y0 + r) % ny
    xx = (x0 + r) % nx
    idx = ((zz[:, None, None] * ny + yy[None, :, None]) * nx + xx[None, None, :]).reshape(-1)
    n = 2 * half + 1
    sub = Udev[:, :, idx].cpu().numpy()
    return components.comp_to_links(sub, nc, (n, n, n))


@pytest.mark.parametrize("hop", [False, True])
def test_full_size_semi_implicit_sampled(hop):
    """The semi-implicit scheme at the benchmark's full size and launch configuration (SU(3)
    FP64, 512 x 64 x 64, dt = a_L/2, MV initial state, the marching pass): after a step, at
    sampled sites, the GPU's E(t + dt/2) satisfies the scheme's update
        E(t + dt/2) = E(t - dt/2) + dt [f2(U(t - dt), U(t)) + f1(U(t), U(t + dt))] + dt j
    with the slice forces evaluated by the oracle (semi_implicit.f_forces) on a periodic
    5^3 patch around each site (the loops of a link reach one site from it), U(t - dt) from
    the oracle's links_prev, U(t + dt) the GPU's new links, and on the hop step the oracle's
    hop current; and U(t + dt) = exp(i a dt E(t + dt/2)) U(t) (solver tolerance 1e-12)."""
    import torch
    pkg = lattice_or_skip()
    from oracle import su
    w = synth.PLAIN_SU3
    say("case: full-size semi-implicit 512x64x64, hop", hop)
    rA, rB = synth.mv_charges(w.seed, 3, w.nt, w.mu, w.a_T)
    lat = pkg.Lattice(nc=3, nz=w.nz, nt=w.nt, a_T=w.a_T, a_L=w.a_L, dt=w.dt, fp=64, scheme=1, max_iter=200,
                      tol=1e-12)
    lat.init_mv(rA, rB, m_ir=w.m_ir, uv_cut=w.uv_cut, sigma=w.sigma)
    lat.step(3 if hop else 2)
    p = lattice.Params(3, w.a_T, w.a_L, w.dt)
    assert lattice.is_hop_step(lat.step_count, p) == hop
    s0 = lat.get_state_device()
    lat.step(1)
    s1 = lat.get_state_device()
    torch.cuda.synchronize()
    dims = (w.nz, w.nt, w.nt)
    g = synth.rng(21)
    sites = [(int(g.integers(w.nz)), int(g.integers(w.nt)), int(g.integers(w.nt))) for _ in range(10)]
    sites += [(w.nz // 4 + 2, 5, 63), (3 * w.nz // 4 - 1, 0, 17), (0, 63, 0), (w.nz - 1, 31, 32)]
    a = p.a
    E_scale = float(s1["E"].abs().max())
    worst = 0.0
    for (z, y, x) in sites:
        U0 = _patch_links(s0["U"], 3, dims, (z, y, x))
        U1 = _patch_links(s1["U"], 3, dims, (z, y, x))
        from oracle import components
        s = (z * w.nt + y) * w.nt + x
        # E(t - dt/2) on the patch (plain layout (3, n_g, V))
        n = 5
        r = torch.arange(-2, 3, device=s0["E"].device)
        idx = ((((z + r) % w.nz)[:, None, None] * w.nt + ((y + r) % w.nt)[None, :, None]) * w.nt
               + ((x + r) % w.nt)[None, None, :]).reshape(-1)
        Eo = components.comp_to_alg(s0["E"][:, :, idx].cpu().numpy(), 3, (n, n, n), lead=(3,))
        Up = si.links_prev(U0, Eo, p)
        _, f2 = si.f_forces(Up, U0, a)
        f1, _ = si.f_forces(U0, U1, a)
        rhs = Eo[:, 2, 2, 2] + p.dt * (f2[:, 2, 2, 2] + f1[:, 2, 2, 2])
        if hop:
            from test_gpu_parity import _hop_at_site
            rA_at = lambda q: su.from_components(s0["rhoA"][:, (q[0] * w.nt + q[1]) * w.nt + q[2]].cpu().numpy(), 3)
            rB_at = lambda q: su.from_components(s0["rhoB"][:, (q[0] * w.nt + q[1]) * w.nt + q[2]].cpu().numpy(), 3)
            Ufull = lambda i, q: _patch_links(s0["U"], 3, dims, q, half=0)[i, 0, 0, 0]
            jz, _, _ = _hop_at_site(Ufull, rA_at, rB_at, (z, y, x), dims, p)
            rhs[2] = rhs[2] + p.dt * jz
        E_new = su.from_components(s1["E"][:, :, s].cpu().numpy(), 3)
        err = np.abs(E_new - rhs).max() / E_scale
        worst = max(worst, err)
        assert err < 1e-10, ((z, y, x), err)
        # the new links are the exponential update of U(t) with E(t + dt/2)
        for i in range(3):
            ref = su.expi(a[i] * p.dt * E_new[i]) @ U0[i, 2, 2, 2]
            assert np.abs(U1[i, 2, 2, 2] - ref).max() < 1e-12
    say("worst sampled E residual (relative to max |E|)", worst)
