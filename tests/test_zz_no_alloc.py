"""The allocation-free observables call (glasma_observe_noalloc) against glasma_observe on
the same states: bitwise equal, on two calls in a row with a smaller lattice second (the
static partial-sum array keeps the first call's contents beyond what the second writes),
in double and single precision, and the documented refusals (scheme 1, a lattice whose
partial sums exceed the array)."""
import ctypes as C
import sys
import numpy as np
import pytest

import synth
from _gpu import gpu, lattice_or_skip

pytestmark = gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _event(pkg, nc, nz, nt, fp, seed):
    w = synth.Workload(f"su{nc}-{nz}x{nt}", nc=nc, nz=nz, nt=nt, mu=0.5, sigma=3.0, uv_cut=2.5, seed=seed)
    lat = pkg.Lattice(nc=nc, nz=nz, nt=nt, a_T=w.a_T, a_L=w.a_L, dt=w.dt, fp=fp,
                      reunit_every=8 if fp == 32 else 0)
    rA, rB = synth.mv_charges(w.seed, nc, nt, w.mu, w.a_T)
    lat.init_mv(rA, rB, m_ir=w.m_ir, uv_cut=w.uv_cut, sigma=w.sigma)
    lat.step(5)
    return lat


@pytest.mark.parametrize("fp", [64, 32])
def test_observe_noalloc_matches_observe(fp):
    import torch
    pkg = lattice_or_skip()
    # first the larger lattice (fills more of the static array), then a smaller one
    for nz, nt, seed in ((256, 64, 8101), (24, 12, 8102)):
        say(f"case: observe_noalloc su3 {nz}x{nt}x{nt} fp{fp}")
        lat = _event(pkg, 3, nz, nt, fp, seed)
        a, b = lat.obs_buffer(), lat.obs_buffer()
        a.fill_(np.nan)
        b.fill_(-1.0)
        lat.observe(a)
        lat.observe_noalloc(b)
        torch.cuda.synchronize()
        ha, hb = a.cpu().numpy(), b.cpu().numpy()
        assert np.all(np.isfinite(hb))
        assert np.array_equal(ha, hb), np.abs(ha - hb).max()
        del lat


def test_observe_noalloc_refusals():
    pkg = lattice_or_skip()
    from paper_2009_02044_amd import GlasmaError
    say("case: observe_noalloc refusals")
    # the semi-implicit scheme
    lat = pkg.Lattice(nc=2, nz=8, nt=4, scheme=1, max_iter=50, tol=1e-12)
    U = np.zeros((3, 4, 8 * 16))
    U[:, 0] = 1.0
    z = np.zeros((3, 3, 8 * 16))
    lat.init_state(U, z, z[0], z[0], step0=0)
    with pytest.raises(GlasmaError) as e:
        lat.observe_noalloc(lat.obs_buffer())
    assert e.value.code == -1
    # partial sums beyond the array: 1024 x 192^2 needs 1024 * 144 * 9 = 1327104 doubles
    big = pkg.Lattice(nc=2, nz=1024, nt=192)
    U = np.zeros((3, 4, 1024 * 192 * 192))
    U[:, 0] = 1.0
    z = np.zeros((3, 3, 1024 * 192 * 192))
    big.init_state(U, z, z[0], z[0], step0=0)
    with pytest.raises(GlasmaError) as e:
        big.observe_noalloc(big.obs_buffer())
    assert e.value.code == -1 and "too large" in str(e.value)
