"""GPU tests of the differentiation form (reverse mode of the leapfrog step, checkpointed).

Parity: the HIP gradients dL/dE0, dL/drho0, dL/damp against the oracle's tangent-linear
derivatives (forward mode, an independent algorithm) on the same seeded states, along
random dense directions and along sampled single components; FP64 on both sides, bar
1e-10 relative.  At the full differentiation workload (SU(3) 256 x 32 x 32, 256 steps,
checkpoint every 32) the gradients are checked against central finite differences of the
GPU's own FP64 forward pass along 50 random directions."""
import sys
import numpy as np
import pytest

import synth
from oracle import lattice, init_mv, adjoint
from _gpu import gpu, lattice_or_skip, to_comp, mv_setup, new_lattice

pytestmark = gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small_state(nc, nz, nt, seed):
    p = lattice.Params(nc=nc, a_T=4.0, a_L=1.0, dt=0.5)
    mv = init_mv.MVParams(m_ir=0.2, uv_cut=0.0, sigma=max(1.0, nz / 10), zA=0.75 * nz, zB=0.25 * nz)
    rA, rB = synth.mv_charges(seed, nc, nt, 1.0, 4.0)
    st, _ = init_mv.initial_state(rA, rB, nz, p, mv)
    ng = nc * nc - 1
    # a generic transverse + longitudinal field on top of the MV state
    from oracle import su
    st.E = st.E + su.from_components(synth.normal(seed + 1, (3, nz, nt, nt, ng), 0.05), nc)
    return st


def to_oracle_alg(c, nz, nt, lead):
    """C-ABI components (lead..., n_g, V) -> oracle component layout (lead..., nz, ny, nx, n_g)."""
    ng = c.shape[-2]
    return np.swapaxes(c, -1, -2).reshape(lead + (nz, nt, nt, ng))


def gpu_grad(pkg, st, nz, nt, steps, every, z0, z1, fp=64):
    import torch
    nc = st.params.nc
    lat = pkg.Lattice(nc=nc, nz=nz, nt=nt, a_T=4.0, a_L=1.0, dt=0.5, fp=fp)
    lat.init_state(*to_comp(st), step0=st.step)
    work = lat.adjoint_work(steps, every)
    lat.adjoint_forward(steps, every, work)
    g = lat.adjoint_backward(z0, z1, work)
    torch.cuda.synchronize()
    out = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in g.items()}
    return lat, out


def oracle_dir(st, vE, vA, vB, steps, z0, z1):
    nz, nt = st.E.shape[1], st.E.shape[2]
    tan = adjoint.tangent_from_components(
        st, None, to_oracle_alg(vE, nz, nt, (3,)) if vE is not None else None,
        to_oracle_alg(vA, nz, nt, ()) if vA is not None else None,
        to_oracle_alg(vB, nz, nt, ()) if vB is not None else None)
    return adjoint.jvp(st, tan, steps, z0, z1)


@pytest.mark.parametrize("nc", [2, 3])
def test_gradient_matches_oracle_along_random_directions(nc):
    """nz=14, nt=5 (V = 350: a ragged last record), 9 steps in checkpoint segments 4, 4, 1
    (hop and non-hop steps), slab [5, 9); 12 dense random directions over E0, rho_A, rho_B
    and 4 over the per-cell amplitudes."""
    pkg = lattice_or_skip()
    nz, nt, steps, every, z0, z1 = 14, 5, 9, 4, 5, 9
    say(f"case: adjoint nc={nc} {nz}x{nt}x{nt} steps={steps} every={every}")
    st = small_state(nc, nz, nt, seed=300 + nc)
    ng, V = nc * nc - 1, nz * nt * nt
    _, g = gpu_grad(pkg, st, nz, nt, steps, every, z0, z1)
    L_ref = adjoint.slab_loss(lattice.evolve(st, steps), z0, z1)
    assert abs(g["L"] - L_ref) <= 1e-12 * abs(L_ref), (g["L"], L_ref)
    worst = 0.0
    for k in range(12):
        vE = synth.normal(400 + 10 * k, (3, ng, V), 1.0)
        vA = synth.normal(401 + 10 * k, (ng, V), 1.0) if k % 3 != 1 else None
        vB = synth.normal(402 + 10 * k, (ng, V), 1.0) if k % 3 != 2 else None
        got = np.sum(g["dE0"] * vE) + (np.sum(g["drhoA0"] * vA) if vA is not None else 0.0) \
            + (np.sum(g["drhoB0"] * vB) if vB is not None else 0.0)
        ref = oracle_dir(st, vE, vA, vB, steps, z0, z1)[1]
        err = abs(got - ref) / abs(ref)
        worst = max(worst, err)
        assert err < 1e-10, (k, got, ref)
    # per-cell charge amplitudes: rho(x) -> (1 + h alpha(x)) rho(x)
    rA_c, rB_c = to_comp(st)[2], to_comp(st)[3]
    for k in range(4):
        al = synth.normal(500 + k, (V,), 1.0)
        be = synth.normal(510 + k, (V,), 1.0)
        got = np.sum(g["dampA"] * al) + np.sum(g["dampB"] * be)
        ref = oracle_dir(st, None, rA_c * al, rB_c * be, steps, z0, z1)[1]
        err = abs(got - ref) / abs(ref)
        worst = max(worst, err)
        assert err < 1e-10, (k, got, ref)
    say("worst relative difference", worst)


@pytest.mark.parametrize("nc", [2, 3])
def test_gradient_matches_oracle_element_by_element(nc):
    """nz=4, nt=3, 5 steps (checkpoint every 2): 120 sampled single components of dL/dE0,
    dL/drho_A, dL/drho_B against the oracle's derivative along that component."""
    pkg = lattice_or_skip()
    nz, nt, steps, every, z0, z1 = 4, 3, 5, 2, 1, 3
    say(f"case: adjoint elementwise nc={nc} {nz}x{nt}x{nt}")
    st = small_state(nc, nz, nt, seed=600 + nc)
    ng, V = nc * nc - 1, nz * nt * nt
    _, g = gpu_grad(pkg, st, nz, nt, steps, every, z0, z1)
    gen = synth.rng(700 + nc)
    scale = max(np.abs(g["dE0"]).max(), np.abs(g["drhoA0"]).max(), np.abs(g["drhoB0"]).max())
    worst = 0.0
    for k in range(120):
        part = k % 3
        if part == 0:
            i, a, s = gen.integers(3), gen.integers(ng), gen.integers(V)
            v = np.zeros((3, ng, V)); v[i, a, s] = 1.0
            got, ref = g["dE0"][i, a, s], oracle_dir(st, v, None, None, steps, z0, z1)[1]
        else:
            a, s = gen.integers(ng), gen.integers(V)
            v = np.zeros((ng, V)); v[a, s] = 1.0
            if part == 1:
                got, ref = g["drhoA0"][a, s], oracle_dir(st, None, v, None, steps, z0, z1)[1]
            else:
                got, ref = g["drhoB0"][a, s], oracle_dir(st, None, None, v, steps, z0, z1)[1]
        err = abs(got - ref) / max(abs(ref), 1e-3 * scale)
        worst = max(worst, err)
        assert err < 1e-10, (k, part, got, ref)
    say("worst", worst)


def test_checkpoint_interval_and_rerun_are_bitwise_invariant():
    pkg = lattice_or_skip()
    nz, nt, steps, z0, z1 = 12, 4, 11, 4, 8
    say("case: adjoint checkpoint invariance su3 12x4x4")
    st = small_state(3, nz, nt, seed=800)
    ref = gpu_grad(pkg, st, nz, nt, steps, steps, z0, z1)[1]
    for every in (1, 3, 4, 11, 50):
        g = gpu_grad(pkg, st, nz, nt, steps, every, z0, z1)[1]
        for k in ("dE0", "drhoA0", "drhoB0", "dampA", "dampB", "L"):
            assert np.array_equal(np.asarray(g[k]), np.asarray(ref[k])), (every, k)


def test_zero_steps_gradient_is_the_loss_derivative():
    """steps = 0: dL/dE = a^3 E on the slab, zero elsewhere; no charge dependence."""
    pkg = lattice_or_skip()
    nz, nt, z0, z1 = 8, 4, 2, 5
    st = small_state(3, nz, nt, seed=900)
    _, g = gpu_grad(pkg, st, nz, nt, 0, 4, z0, z1)
    E = to_comp(st)[1].reshape(3, 8, nz, nt * nt)
    expect = np.zeros_like(E)
    expect[:, :, z0:z1] = 4.0 * 4.0 * 1.0 * E[:, :, z0:z1]
    assert np.abs(g["dE0"].reshape(E.shape) - expect).max() <= 1e-14 * np.abs(expect).max()
    assert np.abs(g["drhoA0"]).max() == 0 and np.abs(g["drhoB0"]).max() == 0
    assert g["L"] == pytest.approx(adjoint.slab_loss(st, z0, z1), rel=1e-13)


def test_call_order_and_argument_errors():
    pkg = lattice_or_skip()
    import torch
    st = small_state(2, 8, 4, seed=950)
    lat = pkg.Lattice(nc=2, nz=8, nt=4, fp=64)
    lat.init_state(*to_comp(st))
    work = lat.adjoint_work(4, 2)
    with pytest.raises(pkg.GlasmaError, match="E_STATE"):
        lat.adjoint_backward(2, 4, work)
    lat.adjoint_forward(4, 2, work)
    with pytest.raises(pkg.GlasmaError, match="E_ARG"):
        lat.adjoint_backward(4, 4, work)
    lat.step(1)
    with pytest.raises(pkg.GlasmaError, match="E_STATE"):
        lat.adjoint_backward(2, 4, work)
    with pytest.raises(pkg.GlasmaError, match="E_ARG"):
        lat.adjoint_forward(4, 2, work[: work.numel() // 2])
    semi = pkg.Lattice(nc=2, nz=8, nt=4, fp=64, scheme=1, tol=1e-10)
    semi.init_state(*to_comp(st))
    with pytest.raises(pkg.GlasmaError, match="E_ARG"):
        semi.adjoint_forward(4, 2, work)
    torch.cuda.synchronize()


def test_autograd_function_matches_the_c_abi():
    pkg = lattice_or_skip()
    import torch
    nz, nt, steps, every, z0, z1 = 12, 4, 7, 3, 4, 8
    st = small_state(3, nz, nt, seed=960)
    dev = torch.device("cuda")
    U0, E0, rA, rB = [torch.tensor(x, device=dev) for x in to_comp(st)]
    lat = pkg.Lattice(nc=3, nz=nz, nt=nt, fp=64)
    E = E0.clone().requires_grad_(True)
    aA = torch.ones(nz * nt * nt, dtype=torch.float64, device=dev, requires_grad=True)
    aB = torch.ones(nz * nt * nt, dtype=torch.float64, device=dev, requires_grad=True)
    L = pkg.SlabEnergy.apply(E, aA, aB, lat, U0, rA, rB, steps, every, z0, z1)
    (2.0 * L).backward()
    _, g = gpu_grad(pkg, st, nz, nt, steps, every, z0, z1)
    assert float(L.detach()) == pytest.approx(g["L"], rel=1e-14)
    assert np.array_equal(E.grad.cpu().numpy(), 2.0 * g["dE0"])
    assert np.array_equal(aA.grad.cpu().numpy(), 2.0 * g["dampA"])
    assert np.array_equal(aB.grad.cpu().numpy(), 2.0 * g["dampB"])


def _config5(pkg, fp, reunit):
    import torch
    w = synth.ADJOINT_SU3
    p, mv = mv_setup(w)
    rA, rB = synth.mv_charges(w.seed, w.nc, w.nt, w.mu, w.a_T)
    lat = new_lattice(pkg, w, fp=64)
    lat.init_mv(rA, rB, m_ir=w.m_ir, uv_cut=w.uv_cut, sigma=w.sigma, zA=w.zA, zB=w.zB)
    s0 = lat.get_state_device()
    run = new_lattice(pkg, w, fp=fp, reunit_every=reunit) if fp != 64 else lat
    torch.cuda.synchronize()
    return w, s0, lat, run


_FULL = {}


def _full_workload_gradient(pkg, fp):
    """Adjoint gradient at the full differentiation workload, forward in precision fp."""
    import torch
    w, s0, lat64, run = _config5(pkg, fp, 4 if fp == 32 else 0)
    steps, every, z0, z1 = w.steps, 32, w.nz // 2 - 8, w.nz // 2 + 8
    run.set_state_device(s0["U"], s0["E"], s0["rhoA"], s0["rhoB"])
    work = run.adjoint_work(steps, every)
    run.adjoint_forward(steps, every, work)
    g = run.adjoint_backward(z0, z1, work)
    del work
    torch.cuda.synchronize()
    return w, s0, lat64, g, (steps, z0, z1)


@pytest.mark.parametrize("fp", [64, 32])
def test_full_workload_gradient_against_finite_differences(fp):
    """SU(3) 256 x 32 x 32, MV nuclei (sigma 8, z_B = 64, z_A = 192), 256 steps with a
    checkpoint every 32, loss = energy of the central 16 layers.  50 random directions v of
    unit 2-norm over (E0, per-cell amplitudes of both nuclei); central differences of the
    FP64 GPU forward pass with h = 5e-3 and 2.5e-3, Richardson-extrapolated (with unit-norm
    directions a step of 1e-4 moves the loss by a few 1e-7 of itself, where the rounding of
    256 chaotic steps already shows; 5e-3 keeps the truncation error, O(h^4), far below it).
    FP64 forward: the adjoint is exact to rounding, so the bar (1e-7 of the largest
    directional derivative) is set by the differences' own truncation and rounding.
    FP32 forward (reunitarised every 4 steps): the gradient is that of the FP32 trajectory,
    which differs from the FP64 one by the trajectory's FP32 error grown over 256 chaotic
    steps (measured 2.4e-5, median 7.2e-6, above the 1e-5 aimed for: the FP32 trajectory's
    own rounding, not the FP64 reverse pass; 4.0e-5 with reunitarisation every 8 steps); bar
    5e-5 of the largest directional derivative."""
    pkg = lattice_or_skip()
    import torch
    w, s0, lat64, g, (steps, z0, z1) = _full_workload_gradient(pkg, fp)
    say(f"case: full-workload adjoint fp={fp}, {w.nz}x{w.nt}x{w.nt}, {steps} steps, L={g['L']}")
    V, dev = w.nz * w.nt * w.nt, s0["E"].device
    one = torch.ones(V, dtype=torch.float64, device=dev)

    def loss(vE, vA, vB, h):
        lat64.set_state_device(s0["U"], s0["E"] + h * vE, s0["rhoA"], s0["rhoB"], one + h * vA, one + h * vB)
        lat64.step(steps)
        return lat64.slab_energy(z0, z1)

    gen = torch.Generator(device=dev).manual_seed(5001)
    dots, fds = [], []
    for k in range(50):
        vE = torch.randn(s0["E"].shape, generator=gen, dtype=torch.float64, device=dev)
        vA = torch.randn(V, generator=gen, dtype=torch.float64, device=dev)
        vB = torch.randn(V, generator=gen, dtype=torch.float64, device=dev)
        n = float(torch.sqrt((vE * vE).sum() + (vA * vA).sum() + (vB * vB).sum()))
        vE, vA, vB = vE / n, vA / n, vB / n
        dot = float((g["dE0"] * vE).sum() + (g["dampA"] * vA).sum() + (g["dampB"] * vB).sum())
        f1 = (loss(vE, vA, vB, 5e-3) - loss(vE, vA, vB, -5e-3)) / 1e-2
        f2 = (loss(vE, vA, vB, 2.5e-3) - loss(vE, vA, vB, -2.5e-3)) / 5e-3
        dots.append(dot)
        fds.append((4 * f2 - f1) / 3)
        if k % 10 == 0:
            say(k, dot, fds[-1], f1, f2)
    dots, fds = np.array(dots), np.array(fds)
    scale = np.abs(fds).max()
    rel = np.abs(dots - fds) / scale
    say("max |adjoint - FD| / max |FD|", rel.max(), "median", np.median(rel))
    assert rel.max() < (1e-7 if fp == 64 else 5e-5)


def test_full_workload_fp32_forward_gradient_against_fp64_forward():
    """The whole gradient (every component of dL/dE0, dL/damp_A, dL/damp_B) with the FP32
    forward pass against the FP64 forward pass: relative 2-norm of the difference (measured
    2.7e-5; bar 6e-5)."""
    pkg = lattice_or_skip()
    g64 = _full_workload_gradient(pkg, 64)[3]
    g32 = _full_workload_gradient(pkg, 32)[3]
    out = {}
    for k in ("dE0", "dampA", "dampB"):
        d = float((g32[k] - g64[k]).norm() / g64[k].norm())
        out[k] = d
    say("relative 2-norm differences FP32 vs FP64 forward", out, "L", g32["L"], g64["L"])
    assert abs(g32["L"] - g64["L"]) < 1e-4 * abs(g64["L"])
    assert max(out.values()) < 6e-5, out


def _final_tangent(st, tan, steps):
    for _ in range(steps):
        st, tan = adjoint.tangent_step(st, tan)
    return st, tan


def _comp_of(X, nc, lead):
    """oracle matrices (lead..., nz, ny, nx, N, N) -> C-ABI components (lead..., n_g, V)."""
    from oracle import su
    c = su.to_components(X)                       # (lead..., nz, ny, nx, n_g)
    ng = c.shape[-1]
    c = c.reshape(lead + (-1, ng))
    return np.ascontiguousarray(np.swapaxes(c, -1, -2))


@pytest.mark.parametrize("nc", [2, 3])
def test_general_cotangent_against_oracle_jvp(nc):
    """glasma_adjoint_backward_cotangent: for a random cotangent c of the final state (links,
    E, both charge populations) and random directions v of the starting state (links, E,
    charges), <J^T c, v> from the GPU's reverse pass equals <c, J v> with J v the oracle's
    tangent-linear propagation (nz = 12, nt = 4, 7 steps in checkpoint segments 3, 3, 1 with
    hops); and for a second observable, L2 = sum_x w(x) |E_z(x)|^2 of the final state
    (cotangent 2 w E_z), its gradient along v equals the oracle's JVP of L2.  FP64, 1e-10."""
    import torch
    pkg = lattice_or_skip()
    nz, nt, steps, every = 12, 4, 7, 3
    say(f"case: general cotangent nc={nc}")
    st = small_state(nc, nz, nt, seed=700 + nc)
    ng, V = nc * nc - 1, nz * nt * nt
    lat = pkg.Lattice(nc=nc, nz=nz, nt=nt, a_T=4.0, a_L=1.0, dt=0.5, fp=64)
    lat.init_state(*to_comp(st), step0=st.step)
    work = lat.adjoint_work(steps, every)
    lat.adjoint_forward(steps, every, work)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=lat.device)
    cU = synth.normal(710, (3, ng, V), 1.0)
    cE = synth.normal(711, (3, ng, V), 1.0)
    cA = synth.normal(712, (ng, V), 1.0)
    cB = synth.normal(713, (ng, V), 1.0)
    g = lat.adjoint_backward_cotangent(work, dev(cU), dev(cE), dev(cA), dev(cB))
    g = {k: v.cpu().numpy() for k, v in g.items()}
    worst = 0.0
    for k in range(4):
        vU = synth.normal(720 + k, (3, ng, V), 1.0)
        vE = synth.normal(730 + k, (3, ng, V), 1.0)
        vA = synth.normal(740 + k, (ng, V), 1.0)
        vB = synth.normal(750 + k, (ng, V), 1.0)
        tan = adjoint.tangent_from_components(st, to_oracle_alg(vU, nz, nt, (3,)), to_oracle_alg(vE, nz, nt, (3,)),
                                              to_oracle_alg(vA, nz, nt, ()), to_oracle_alg(vB, nz, nt, ()))
        _, tf = _final_tangent(st, tan, steps)
        rhs = (np.sum(cU * _comp_of(tf[0], nc, (3,))) + np.sum(cE * _comp_of(tf[1], nc, (3,)))
               + np.sum(cA * _comp_of(tf[2], nc, ())) + np.sum(cB * _comp_of(tf[3], nc, ())))
        lhs = np.sum(g["dU0"] * vU) + np.sum(g["dE0"] * vE) + np.sum(g["drhoA0"] * vA) + np.sum(g["drhoB0"] * vB)
        err = abs(lhs - rhs) / abs(rhs)
        worst = max(worst, err)
        say(f"  direction {k}: <J^T c, v> {lhs:.12e}  <c, J v> {rhs:.12e}  rel {err:.1e}")
        assert err < 1e-10
    # a second observable: L2 = sum_x w(x) |E_z(x)|^2 of the final state
    fin = lattice.evolve(st, steps)
    Ez = _comp_of(fin.E, nc, (3,))[2]                      # (n_g, V)
    wgt = synth.uniform(760, (V,), 0.0, 1.0)
    cE2 = np.zeros((3, ng, V))
    cE2[2] = 2.0 * wgt[None, :] * Ez
    g2 = lat.adjoint_backward_cotangent(work, None, dev(cE2), None, None)
    g2 = {k: v.cpu().numpy() for k, v in g2.items()}
    vE = synth.normal(770, (3, ng, V), 1.0)
    vA = synth.normal(771, (ng, V), 1.0)
    tan = adjoint.tangent_from_components(st, None, to_oracle_alg(vE, nz, nt, (3,)), to_oracle_alg(vA, nz, nt, ()),
                                          None)
    fst, tf = _final_tangent(st, tan, steps)
    from oracle import su
    dEz = su.to_components(tf[1][2])                       # (nz, ny, nx, n_g)
    Ezf = su.to_components(fst.E[2])
    jvp = np.sum(2.0 * wgt.reshape(nz, nt, nt)[..., None] * Ezf * dEz)
    lhs = np.sum(g2["dE0"] * vE) + np.sum(g2["drhoA0"] * vA)
    say(f"  second observable: GPU {lhs:.12e} oracle JVP {jvp:.12e}")
    assert abs(lhs - jvp) <= 1e-10 * abs(jvp)
    assert np.all(g2["dU0"] == g2["dU0"])                  # finite output
