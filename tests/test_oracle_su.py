"""Pins of the oracle's SU(N) algebra against textbook facts and SciPy."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import su, components


@pytest.mark.parametrize("nc", [2, 3])
def test_generators_normalisation(nc):
    t = su.generators(nc)
    ng = nc * nc - 1
    assert t.shape == (ng, nc, nc)
    np.testing.assert_allclose(t, su.dag(t), atol=0)
    np.testing.assert_allclose(su.trace(t), 0, atol=1e-15)
    gram = np.einsum("aij,bji->ab", t, t)
    np.testing.assert_allclose(gram, 0.5 * np.eye(ng), atol=1e-15)


def test_su3_structure_constants():
    # textbook values: f^{123} = 1, f^{147} = 1/2, f^{458} = f^{678} = sqrt(3)/2
    t = su.generators(3)

    def f(a, b, c):
        comm = t[a] @ t[b] - t[b] @ t[a]
        return np.real(-2j * np.trace(comm @ t[c]))

    assert f(0, 1, 2) == pytest.approx(1.0, abs=1e-15)
    assert f(0, 3, 6) == pytest.approx(0.5, abs=1e-15)
    assert f(3, 4, 7) == pytest.approx(np.sqrt(3) / 2, abs=1e-15)
    assert f(5, 6, 7) == pytest.approx(np.sqrt(3) / 2, abs=1e-15)
    assert f(0, 1, 7) == pytest.approx(0.0, abs=1e-15)


@pytest.mark.parametrize("nc", [2, 3])
def test_expi_matches_expm_and_is_special_unitary(nc):
    c = synth.normal(11, (50, nc * nc - 1), 1.3)
    H = su.from_components(c, nc)
    W = su.expi(H)
    ref = np.stack([sla.expm(1j * h) for h in H])
    np.testing.assert_allclose(W, ref, atol=1e-13)
    np.testing.assert_allclose(su.dag(W) @ W, np.broadcast_to(np.eye(nc), W.shape), atol=1e-14)
    np.testing.assert_allclose(np.linalg.det(W), 1.0, atol=1e-14)


@pytest.mark.parametrize("nc", [2, 3])
def test_logi_inverts_expi_and_matches_logm(nc):
    c = synth.normal(12, (50, nc * nc - 1), 0.4)
    H = su.from_components(c, nc)
    W = su.expi(H)
    np.testing.assert_allclose(su.logi(W), H, atol=1e-13)
    ref = np.stack([sla.logm(w) / 1j for w in W])
    np.testing.assert_allclose(su.logi(W), ref, atol=1e-12)


@pytest.mark.parametrize("nc", [2, 3])
def test_proj_properties(nc):
    c = synth.normal(13, (20, nc * nc - 1))
    H = su.from_components(c, nc)
    # proj(i H) = H for hermitian traceless H; proj(1) = 0; result hermitian traceless
    np.testing.assert_allclose(su.proj(1j * H), H, atol=1e-15)
    np.testing.assert_allclose(su.proj(np.eye(nc) + 0 * H), 0, atol=0)
    M = synth.normal(14, (20, nc, nc)) + 1j * synth.normal(15, (20, nc, nc))
    P = su.proj(M)
    np.testing.assert_allclose(P, su.dag(P), atol=1e-15)
    np.testing.assert_allclose(su.trace(P), 0, atol=1e-14)
    # [M]_ah = i proj(M): the anti-hermitian traceless part
    ah = (M - su.dag(M)) / 2 - (su.trace(M - su.dag(M)) / (2 * nc))[:, None, None] * np.eye(nc)
    np.testing.assert_allclose(1j * P, ah, atol=1e-15)


def test_su2_closed_forms():
    # exp(i theta n.sigma/2) = cos(theta/2) + i sin(theta/2) n.sigma
    th = 0.7
    n = np.array([0.6, 0.0, 0.8])
    H = su.from_components(th * n, 2)
    W = su.expi(H)
    sig = su.generators(2) * 2
    ref = np.cos(th / 2) * np.eye(2) + 1j * np.sin(th / 2) * np.tensordot(n, sig, 1)
    np.testing.assert_allclose(W, ref, atol=1e-15)


@pytest.mark.parametrize("nc", [2, 3])
def test_component_roundtrip(nc):
    dims = (2, 3, 3)
    c = synth.normal(16, (3,) + dims + (nc * nc - 1,), 0.9)
    U = su.expi(su.from_components(c, nc))
    back = components.comp_to_links(components.links_to_comp(U), nc, dims)
    np.testing.assert_allclose(back, U, atol=1e-15)
    X = su.from_components(c, nc)
    xc = components.alg_to_comp(X)
    assert xc.shape == (3, nc * nc - 1, 18)
    np.testing.assert_allclose(components.comp_to_alg(xc, nc, dims, lead=(3,)), X, atol=1e-15)
    if nc == 2:
        q = components.links_to_comp(U)
        np.testing.assert_allclose(np.sum(q ** 2, axis=1), 1.0, atol=1e-14)
