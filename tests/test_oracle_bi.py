"""Pins of the boost-invariant tau = 0+ fields (Sec. 2, eqs. glasma_ic1/2, LC_gauge1)."""
import numpy as np
import pytest
from scipy.linalg import expm

import synth
from oracle import su, lattice, init_mv, glasma_bi as bi


def const(nc, comp, scale, shape=(4, 5)):
    c = np.zeros(shape + (nc * nc - 1,))
    c[..., comp] = scale
    return su.from_components(c, nc)


def test_constant_su2_fields_closed_forms():
    """SU(2), T^a = sigma^a / 2, [T^1, T^2] = i T^3: alpha_A^x = a T^1 with alpha_B^x = b T^2
    gives E_z = a b T^3 and B_z = 0; with alpha_B^y = b T^2 instead, E_z = 0 and
    B_z = a b T^3; |X|^2 = sum_a (X^a)^2."""
    a, b = 0.7, -1.3
    z = const(2, 0, 0.0)
    Ez, Bz = bi.bi_fields((const(2, 0, a), z), (const(2, 1, b), z))
    np.testing.assert_allclose(su.to_components(Ez), np.broadcast_to([0, 0, a * b], Ez.shape[:2] + (3,)), atol=1e-15)
    assert np.abs(Bz).max() < 1e-15
    Ez, Bz = bi.bi_fields((const(2, 0, a), z), (z, const(2, 1, b)))
    assert np.abs(Ez).max() < 1e-15
    np.testing.assert_allclose(su.to_components(Bz), np.broadcast_to([0, 0, a * b], Bz.shape[:2] + (3,)), atol=1e-15)
    # alpha_A^y with alpha_B^x enters B_z with the opposite sign (epsilon^{yx} = -1)
    Ez, Bz = bi.bi_fields((z, const(2, 0, a)), (const(2, 1, b), z))
    np.testing.assert_allclose(su.to_components(Bz), np.broadcast_to([0, 0, -a * b], Bz.shape[:2] + (3,)), atol=1e-15)
    e0, e, bb = bi.bi_energy((const(2, 0, a), const(2, 0, a)), (const(2, 1, b), const(2, 1, b)))
    # E_z = 2 a b T^3 (both directions), B_z = a b T^3 - a b T^3 = 0
    assert e == pytest.approx(0.5 * (2 * a * b) ** 2, rel=1e-14) and bb < 1e-30


@pytest.mark.parametrize("nc", [2, 3])
def test_commuting_fields_give_nothing_and_rotations_leave_eps0(nc):
    p = lattice.Params(nc=nc, a_T=4.0, a_L=1.0, dt=0.5)
    mv = init_mv.MVParams(m_ir=0.2, sigma=2.0, zA=24.0, zB=8.0)
    rA, rB = synth.mv_charges(31, nc, 6, 0.5, 4.0)
    # one colour component for both nuclei: abelian, every commutator vanishes
    r1A, r1B = np.zeros_like(rA), np.zeros_like(rB)
    r1A[0], r1B[0] = rA[0], rB[0]
    assert bi.bi_eps0(r1A, r1B, p, mv)[0] < 1e-30
    e0 = bi.bi_eps0(rA, rB, p, mv)
    assert e0[0] > 0
    # a global colour rotation R (same for both nuclei) rotates alpha, not eps_0
    aA = bi.transverse_alpha(bi.wilson_behind(rA, p, mv), p.a_T)
    aB = bi.transverse_alpha(bi.wilson_behind(rB, p, mv), p.a_T)
    R = expm(1j * su.from_components(synth.normal(5, (nc * nc - 1,), 1.0), nc))
    rot = lambda al: tuple(R @ x @ su.dag(R) for x in al)
    np.testing.assert_allclose(bi.bi_energy(rot(aA), rot(aB)), e0, rtol=1e-12)
    # A <-> B flips E_z (one commutator) and keeps B_z (commutator times epsilon^{ij})
    EzAB, BzAB = bi.bi_fields(aA, aB)
    EzBA, BzBA = bi.bi_fields(aB, aA)
    np.testing.assert_allclose(EzBA, -EzAB, atol=1e-15)
    np.testing.assert_allclose(BzBA, BzAB, atol=1e-15)


def test_alpha_is_the_lattice_gradient_in_the_weak_field_limit():
    """V = exp(-i eps phi): alpha^i = P(V(x) V^dag(x+i)) / a_T = eps (phi(x+i) - phi(x)) / a_T
    + O(eps^2)."""
    nc, a_T = 3, 4.0
    phi = su.from_components(synth.normal(8, (5, 6, 8), 1.0), nc)
    for eps in (1e-3, 1e-4):
        ax, ay = bi.transverse_alpha(su.expi(-eps * phi), a_T)
        gx = eps * (np.roll(phi, -1, axis=1) - phi) / a_T
        gy = eps * (np.roll(phi, -1, axis=0) - phi) / a_T
        assert np.abs(ax - gx).max() < 10 * eps ** 2 and np.abs(ay - gy).max() < 10 * eps ** 2


def _smooth_phi(nc, seed, X, Y, L):
    """A smooth periodic algebra field phi(x, y) = sum_m c_m^a t^a cos(2 pi (k_m . x) / L + d_m)
    with O(1) components along non-commuting generators."""
    rng = np.random.default_rng(seed)
    ng = nc * nc - 1
    out = np.zeros(X.shape + (ng,))
    for (kx, ky) in ((1, 0), (0, 1), (1, 1), (2, -1)):
        c = rng.normal(0.0, 0.6, ng)
        d = rng.uniform(0, 2 * np.pi)
        out += np.cos(2 * np.pi * (kx * X + ky * Y) / L + d)[..., None] * c
    return su.from_components(out, nc)


def _continuum_fields(nc, seeds, X, Y, L, h=1e-5):
    """The paper's continuum tau = 0+ fields at points (X, Y) for V_N = exp(-i phi_N):
    alpha^i = -i V d_i V^dag (pure gauge), E_z = -i sum_i [alpha_A^i, alpha_B^i],
    B_z = -i ([alpha_A^x, alpha_B^y] - [alpha_A^y, alpha_B^x]); d_i by central differences."""
    al = []
    for sd in seeds:
        V = su.expi(-_smooth_phi(nc, sd, X, Y, L))
        dx = (su.expi(_smooth_phi(nc, sd, X + h, Y, L)) - su.expi(_smooth_phi(nc, sd, X - h, Y, L))) / (2 * h)
        dy = (su.expi(_smooth_phi(nc, sd, X, Y + h, L)) - su.expi(_smooth_phi(nc, sd, X, Y - h, L))) / (2 * h)
        al.append((-1j * V @ dx, -1j * V @ dy))
    (axA, ayA), (axB, ayB) = al
    Ez = bi._com(axA, axB) + bi._com(ayA, ayB)
    Bz = bi._com(axA, ayB) - bi._com(ayA, axB)
    return Ez, Bz


@pytest.mark.parametrize("nc", [2, 3])
def test_lattice_fields_converge_to_the_continuum_formula(nc):
    """The lattice reading of the tau = 0+ fields (alpha on the transverse links, E_z at the
    sites, B_z at the plaquette centres) against the paper's continuum formula (Sec. 2, eqs.
    glasma_ic1/2) for smooth, strongly non-abelian Wilson lines on a periodic square of side L:
    the error falls by ~4 per halving of the spacing (second order)."""
    L = 12.0
    errs = []
    for n in (32, 64, 128):
        a = L / n
        j = np.arange(n) * a
        X, Y = np.meshgrid(j, j)                      # [y, x]
        alA = bi.transverse_alpha(su.expi(-_smooth_phi(nc, 1, X, Y, L)), a)
        alB = bi.transverse_alpha(su.expi(-_smooth_phi(nc, 2, X, Y, L)), a)
        Ez, Bz = bi.bi_fields(alA, alB)
        Ez_c, _ = _continuum_fields(nc, (1, 2), X, Y, L)
        _, Bz_c = _continuum_fields(nc, (1, 2), X + a / 2, Y + a / 2, L)
        assert np.abs(Ez_c).max() > 0.1 and np.abs(Bz_c).max() > 0.1     # genuinely non-abelian
        errs.append((np.abs(Ez - Ez_c).max() / np.abs(Ez_c).max(), np.abs(Bz - Bz_c).max() / np.abs(Bz_c).max()))
    for q in (0, 1):
        r1, r2 = errs[0][q] / errs[1][q], errs[1][q] / errs[2][q]
        assert 3.5 < r1 < 4.5 and 3.7 < r2 < 4.3, (q, errs)
    assert errs[2][0] < 1e-2 and errs[2][1] < 1e-2, errs
