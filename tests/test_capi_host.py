"""CPU checks of the C-ABI library: it loads, exports every function the header
declares, validates arguments, and its device group algebra (evaluated on the host
through glasma_host_group_op) matches SciPy / closed forms."""
import ctypes as C
import os
import re

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import su, components

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2009_02044_amd import _lib
    return _lib


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "glasma.h")).read()
    names = set(re.findall(r"^\s*(?:int|const char\*)\s+(glasma_\w+)\s*\(", hdr, flags=re.M))
    assert len(names) >= 15
    so = C.CDLL(_lib().LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(so, n)]
    assert not missing, missing


def test_layout_sizes_and_argument_errors():
    L = _lib()
    p = L.Params(3, 16, 8, 4.0, 1.0, 0.5, 64, 0, 0, 50, 0.0)
    sizes = (C.c_size_t * 6)()
    assert L.lib.glasma_layout(C.byref(p), sizes) == 0
    V = 16 * 8 * 8
    # SU(3) links are stored by rows 0 and 1 (12 reals); V = 1024 is a multiple of 64
    assert sizes[0] == 3 * 12 * V * 8 and sizes[1] == sizes[0]
    assert sizes[2] == 3 * 8 * V * 8 and sizes[3] == 8 * V * 8 == sizes[4]
    p32 = L.Params(2, 16, 8, 4.0, 1.0, 0.5, 32, 0, 0, 50, 0.0)
    assert L.lib.glasma_layout(C.byref(p32), sizes) == 0
    assert sizes[0] == 3 * 4 * V * 4 and sizes[2] == 3 * 3 * V * 4
    for bad in (L.Params(4, 16, 8, 4.0, 1.0, 0.5, 64, 0, 0, 50, 0.0),
                L.Params(3, 1, 8, 4.0, 1.0, 0.5, 64, 0, 0, 50, 0.0),
                L.Params(3, 16, 8, 4.0, 1.0, 0.5, 16, 0, 0, 50, 0.0),
                L.Params(3, 16, 8, 4.0, 1.0, 1.5, 64, 0, 0, 50, 0.0),      # dt > a_L
                L.Params(3, 16, 8, 4.0, 1.0, 0.5 + 1e-9, 64, 0, 0, 50, 0.0)):  # irrational ratio
        assert L.lib.glasma_layout(C.byref(bad), sizes) == -1
        assert L.lib.glasma_last_error(None)
    # create rejects NULL buffers without touching the GPU
    ctx = C.c_void_p()
    b = L.Buffers(None, None, None, None, None, None)
    assert L.lib.glasma_create(C.byref(p), C.byref(b), None, C.byref(ctx)) == -1
    assert L.lib.glasma_host_group_op(5, 64, 0, 0, None, None) == -1


def _links(nc, n, seed, scale=1.0):
    c = synth.normal(seed, (n, nc * nc - 1), scale)
    U = su.expi(su.from_components(c, nc))
    return U, c


def _link_reals(U):
    n = U.shape[0]
    U3 = np.broadcast_to(U.reshape((1, n, 1, 1) + U.shape[1:]), (3, n, 1, 1) + U.shape[1:])
    return components.links_to_comp(np.ascontiguousarray(U3))[0].T.copy()     # (n, r_U)


def _reals_link(r, nc):
    n = r.shape[0]
    return components.comp_to_links(np.broadcast_to(r.T, (3,) + r.T.shape).copy(), nc, (n, 1, 1))[0].reshape(n, nc, nc)


@pytest.mark.parametrize("nc", [2, 3])
@pytest.mark.parametrize("fp,tol", [(64, 2e-14), (32, 3e-6)])
def test_device_exp_matches_expm(nc, fp, tol):
    from paper_2009_02044_amd import host_group_op
    ng = nc * nc - 1
    rng_c = np.concatenate([synth.normal(3, (60, ng), 1.5), synth.normal(4, (20, ng), 1e-4),
                            np.zeros((1, ng)), synth.normal(5, (20, ng), 3.0)])
    # degenerate spectra: single generator directions
    degen = np.zeros((2 * ng, ng))
    for k in range(ng):
        degen[k, k] = 0.9
        degen[ng + k, k] = -2.1
    rng_c = np.concatenate([rng_c, degen])
    s = np.linspace(-1.3, 1.7, len(rng_c))[:, None]
    out = host_group_op(nc, fp, 0, np.concatenate([s, rng_c], axis=1), 4 if nc == 2 else 18)
    W = _reals_link(out, nc)
    H = su.from_components(rng_c * s, nc)
    ref = np.stack([sla.expm(1j * h) for h in H])
    np.testing.assert_allclose(W, ref, atol=tol)


@pytest.mark.parametrize("nc", [2, 3])
def test_device_log_proj_transport_reunit(nc):
    from paper_2009_02044_amd import host_group_op
    ng = nc * nc - 1
    r = 4 if nc == 2 else 18
    U, c = _links(nc, 40, 21, 0.5)           # eigen-angles well inside (-pi/2, pi/2)
    lg = host_group_op(nc, 64, 1, _link_reals(U), ng)
    np.testing.assert_allclose(lg, su.to_components(su.logi(U)), atol=1e-13)
    M = synth.normal(22, (40, nc, nc)) + 1j * synth.normal(23, (40, nc, nc))
    if nc == 2:   # the SU(2) type is the real span of SU(2): project onto quaternion form
        M = _reals_link(_link_reals(M), 2)
    pr = host_group_op(nc, 64, 2, _link_reals(M), ng)
    np.testing.assert_allclose(pr, su.to_components(su.proj(M)), atol=1e-14)
    X = synth.normal(24, (40, ng))
    tr = host_group_op(nc, 64, 3, np.concatenate([_link_reals(U), X], axis=1), ng)
    np.testing.assert_allclose(tr, su.to_components(su.transport(U, su.from_components(X, nc))), atol=1e-13)
    noisy = _link_reals(U) + synth.normal(25, (40, r), 1e-5)
    ru = host_group_op(nc, 64, 4, noisy, r)
    W = _reals_link(ru, nc)
    np.testing.assert_allclose(su.dag(W) @ W, np.broadcast_to(np.eye(nc), W.shape), atol=1e-14)
    np.testing.assert_allclose(np.linalg.det(W), 1.0, atol=1e-14)
    np.testing.assert_allclose(W, U, atol=1e-4)
    uv = host_group_op(nc, 64, 5, _link_reals(U), 1)
    assert uv.max() < 1e-14
    prod = host_group_op(nc, 64, 6, np.concatenate([_link_reals(U), _link_reals(U[::-1])], axis=1), r)
    np.testing.assert_allclose(_reals_link(prod, nc), U @ U[::-1], atol=1e-14)


@pytest.mark.parametrize("nc", [2, 3])
def test_device_exp_derivative_transpose_matches_expm_frechet(nc):
    """op 7 (the reverse-mode kernel's exponential step): T(L)^b = <L, xi(t^b)> with the
    left derivative xi(Y) = -i D exp(i c X)[i c Y] exp(-i c X) from scipy's expm_frechet."""
    from paper_2009_02044_amd import host_group_op
    ng = nc * nc - 1
    t = su.generators(nc)
    # norms from zero through the range where the series shortens (7-13 terms) to the
    # doubling range, where it keeps all 14
    cases = [(0.3, 0.5), (2.0, 1.0), (4.0, 2.5), (1.0, 0.0), (0.5, 1e-5), (2.0, 0.004), (0.5, 0.05),
             (2.0, 0.02), (2.0, 0.05), (0.5, 0.4)]
    for k, (c, amp) in enumerate(cases):
        X = synth.normal(30 + k, (ng,), amp)
        Lm = synth.normal(40 + k, (ng,), 1.0)
        got = host_group_op(nc, 64, 7, np.concatenate([[c], X, Lm])[None, :], ng)[0]
        A = 1j * c * su.from_components(X, nc)
        W = sla.expm(A)
        ref = np.empty(ng)
        for b in range(ng):
            _, D = sla.expm_frechet(A, 1j * c * t[b])
            xi = -1j * D @ W.conj().T
            ref[b] = np.sum(Lm * su.to_components(xi))
        assert np.abs(got - ref).max() <= 1e-13 * max(1.0, c), (c, amp, got, ref)


@pytest.mark.timeout(60)
@pytest.mark.parametrize("nc", [2, 3])
@pytest.mark.parametrize("fp", [64, 32])
def test_device_exp_ends_on_non_finite_input(nc, fp):
    """The SU(3) exponential halves its argument until its spectral bound is below 1/2; the
    number of halvings is capped at what the largest finite value needs, so an infinite or
    NaN argument gives a non-finite matrix instead of an endless loop (the same source runs on
    the device, where that loop would hang the step kernel)."""
    from paper_2009_02044_amd import host_group_op
    ng = nc * nc - 1
    x = np.zeros((3, 1 + ng))
    x[:, 0] = 1.0
    x[0, 1] = np.inf
    x[1, 1] = np.nan
    x[2, 1] = 0.5                          # a finite row next to them is unaffected
    out = host_group_op(nc, fp, 0, x, 4 if nc == 2 else 18)
    assert not np.isfinite(out[0]).all() and not np.isfinite(out[1]).all()
    assert np.isfinite(out[2]).all()
