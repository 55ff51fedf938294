"""GPU checks of the batched form: several events of different lattice sizes advanced
together (one launch per step, HIP-graph replay) give the states of the same events
run one by one (to a few units in the last place: the two kernels are compiled
separately and may contract floating-point operations differently), bitwise the same
states for every tiling, and match the FP64 oracle."""
import sys
import numpy as np
import pytest

import synth
from oracle import lattice, init_mv
from _gpu import gpu, lattice_or_skip, state_errs, mv_setup

pytestmark = gpu

# nt = 4, 8: rows inside wavefronts (x neighbours from adjacent lanes); nt = 5, 6, 48: rows
# straddle wavefronts (x neighbours from memory), 48 as in the benchmark's event mix
SHAPES = [(16, 4), (24, 6), (20, 5), (32, 8), (6, 48)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _events(nc):
    out = []
    for e, (nz, nt) in enumerate(SHAPES):
        w = synth.Workload(f"ev{e}", nc=nc, nz=nz, nt=nt, mu=0.3 + 0.1 * e, sigma=1.5 + 0.5 * e, seed=4100 + e)
        out.append((w, synth.mv_charges(w.seed, nc, nt, w.mu, w.a_T)))
    return out


def _init(lat, w, rho):
    lat.init_mv(rho[0], rho[1], m_ir=w.m_ir, sigma=w.sigma, zA=w.zA, zB=w.zB)


@pytest.mark.parametrize("nc,fp,reunit", [(3, 64, 0), (3, 32, 8), (2, 64, 0)])
def test_batched_equals_one_by_one(nc, fp, reunit):
    pkg = lattice_or_skip()
    evs = _events(nc)
    say("case: batched", nc, fp, reunit)
    n = 13
    singles = []
    for w, rho in evs:
        lat = pkg.Lattice(nc=nc, nz=w.nz, nt=w.nt, a_T=w.a_T, a_L=w.a_L, dt=w.dt, fp=fp, reunit_every=reunit)
        _init(lat, w, rho)
        lat.step(n)
        singles.append(lat.get_state())
    tol = 1e-13 if fp == 64 else 2e-5
    first = None
    for tiling in [(256, 0), (64, 1024), (128, 8)]:
        b = pkg.Batch(nc, SHAPES, fp=fp, reunit_every=reunit)
        b.set_tiling(*tiling)
        for (w, rho), lat in zip(evs, b.events):
            _init(lat, w, rho)
        b.run(5, graph_chunk=2)      # two graph replays and one direct step
        b.run(n - 5, graph_chunk=0)
        states = [lat.get_state() for lat in b.events]
        for e, got in enumerate(states):
            assert got["step"] == n
            for k in ("U", "E", "rhoA", "rhoB"):
                ref = singles[e][k]
                d = np.abs(got[k] - ref).max()
                assert d <= tol * max(1.0, np.abs(ref).max()), (tiling, e, k, d)
                if first is not None:
                    assert np.array_equal(got[k], first[e][k]), (tiling, e, k)
        first = states


def test_batched_event_matches_oracle():
    pkg = lattice_or_skip()
    evs = _events(3)
    b = pkg.Batch(3, SHAPES, fp=64, reunit_every=0)
    for (w, rho), lat in zip(evs, b.events):
        _init(lat, w, rho)
    refs = {}
    for e in (1, 4):
        w, rho = evs[e]
        p, mv = mv_setup(w)
        refs[e] = init_mv.initial_state(rho[0], rho[1], w.nz, p, mv)[0]
    for k in range(4):
        b.run(2, graph_chunk=2)
        for e in refs:
            refs[e] = lattice.evolve(refs[e], 2)
            errs = state_errs(b.events[e].get_state(), refs[e])
            assert max(errs.values()) < 1e-10, (k, e, errs)


def test_autotune_reports_candidates():
    pkg = lattice_or_skip()
    b = pkg.Batch(3, SHAPES, fp=32, reunit_every=8)
    for (w, rho), lat in zip(_events(3), b.events):
        _init(lat, w, rho)
    rep = b.autotune(steps=1)
    assert len(rep["candidates"]) == 12
    assert rep["chosen"]["sites_per_item"] in (64, 128, 256)
    say("autotune", rep["chosen"])
    o = b.events[0].observables()
    assert o["gauss_rel"] < 1e-4 and o["unitarity"] < 1e-5


def test_graph_replays_match_direct_launches():
    """The captured chunk replayed several times, with the program's own eager work and
    synchronisations between the replays (observables of every event, a torch reduction),
    against a batch advanced by direct launches: bitwise equal after every replay (the same
    kernels; the step counter lives in device memory, so each replay advances it).  Ten steps
    with reunitarisation every 8 put a reunitarising step inside a replay."""
    pkg = lattice_or_skip()
    import torch
    evs = _events(3)
    g = pkg.Batch(3, SHAPES, fp=32, reunit_every=8)
    d = pkg.Batch(3, SHAPES, fp=32, reunit_every=8)
    for bb in (g, d):
        bb.set_tiling(128, 0)
        for (w, rho), lat in zip(evs, bb.events):
            _init(lat, w, rho)
    say("case: graph replays against direct launches")
    for rep in range(5):
        g.run(2, graph_chunk=2)
        d.run(2, graph_chunk=0)
        for lat in g.events:
            o = lat.observables()
            assert o["unitarity"] < 1e-5
        torch.cuda.synchronize()
        assert torch.ones(1 << 20, device="cuda").sum().item() == float(1 << 20)
        for e, (a, b) in enumerate(zip(g.events, d.events)):
            sa, sb = a.get_state(), b.get_state()
            assert sa["step"] == sb["step"] == 2 * (rep + 1)
            for k in ("U", "E", "rhoA", "rhoB"):
                assert np.array_equal(sa[k], sb[k]), (rep, e, k)


def test_batch_event_average_on_the_device():
    """glasma_batch_observe: the per-N_z-class averages and the common z / N_z grid equal the
    mean of the events' own observables (glasma_observables, one by one), and each
    per-event buffer equals that event's observables."""
    pkg = lattice_or_skip()
    shapes = [(16, 4), (24, 6), (16, 5), (32, 4), (24, 4)]
    say("case: batch event average", shapes)
    evs = []
    for e, (nz, nt) in enumerate(shapes):
        w = synth.Workload(f"ev{e}", nc=3, nz=nz, nt=nt, mu=0.4, sigma=1.5, seed=4300 + e)
        evs.append((w, synth.mv_charges(w.seed, 3, nt, w.mu, w.a_T)))
    b = pkg.Batch(3, shapes, fp=64, reunit_every=0)
    for (w, rho), lat in zip(evs, b.events):
        _init(lat, w, rho)
    b.run(7, graph_chunk=0)
    n_grid = 8
    r = b.observe(n_grid, per_event=True)
    b.stream.synchronize()
    ones = [lat.observables()["tmunu_z"] for lat in b.events]
    assert [c for c, _ in b.classes()] == [16, 24, 32]
    assert dict(b.classes()) == {16: 2, 24: 2, 32: 1}
    for nz, got in r["class"].items():
        ref = np.mean([o for o, (w, _) in zip(ones, evs) if w.nz == nz], axis=0)
        np.testing.assert_allclose(got.cpu().numpy(), ref, rtol=1e-12, atol=1e-15 * np.abs(ref).max())
    grid = np.zeros((4, n_grid))
    for o in ones:
        nz = o.shape[1]
        bins = (np.arange(nz) * n_grid) // nz
        grid += np.stack([np.bincount(bins, weights=o[q], minlength=n_grid) / np.bincount(bins) for q in range(4)])
    grid /= len(ones)
    np.testing.assert_allclose(r["grid"].cpu().numpy(), grid, rtol=1e-12, atol=1e-15 * np.abs(grid).max())
    pe = r["per_event"].cpu().numpy()
    off = 0
    for o in ones:
        nz = o.shape[1]
        np.testing.assert_allclose(pe[off:off + 4 * nz].reshape(4, nz), o, rtol=1e-13, atol=1e-300)
        off += 4 * nz + 8
    from paper_2009_02044_amd import GlasmaError
    with pytest.raises(GlasmaError):
        b.observe(17)       # more bins than the smallest N_z


@pytest.mark.parametrize("fp", [32, 64])
def test_event_step_observe_without_parked_projections(fp):
    """An event of a batch has no room in its work region for the projections the observing
    step parks: its glasma_step_observe takes the standalone observables pass, then the plain
    step.  Against glasma_step, glasma_observe, glasma_step on a second, identical batch: the
    same observables and final state, bitwise (the same kernels in the same order)."""
    pkg = lattice_or_skip()
    import torch
    say(f"case: batch event step_observe fp{fp}")
    evs = _events(3)
    shapes = [(w.nz, w.nt) for w, _ in evs]
    ba = pkg.Batch(3, shapes, fp=fp, reunit_every=8 if fp == 32 else 0)
    bb = pkg.Batch(3, shapes, fp=fp, reunit_every=8 if fp == 32 else 0)
    for b in (ba, bb):
        for (w, rho), lat in zip(evs, b.events):
            _init(lat, w, rho)
    for e in (0, 4):   # nt = 4 and nt = 48
        nz = shapes[e][0]
        a, b = ba.events[e], bb.events[e]
        oa, ob = a.obs_buffer(), b.obs_buffer()
        a.step_observe(3, oa)
        b.step(2)
        b.observe(ob)
        b.step(1)
        ba.stream.synchronize()
        bb.stream.synchronize()
        torch.cuda.synchronize()
        assert torch.equal(oa, ob), e
        sa, sb = a.get_state(), b.get_state()
        for k in ("U", "E", "rhoA", "rhoB"):
            assert np.array_equal(sa[k], sb[k]), (e, k)
        assert pkg.Lattice.unpack_obs(oa, nz)["nonfinite"] == 0
