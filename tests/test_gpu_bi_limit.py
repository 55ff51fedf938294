"""Boost-invariant Glasma (Sec. 2, eqs. glasma_ic1/2, LC_gauge1).

glasma_bi_fields against the oracle's tau = 0+ fields, element by element.

Boost-invariant limit: at mid-rapidity, shortly after thin
nuclei have passed through each other, the 3+1D Glasma carries the longitudinal fields of
the tau = 0+ boost-invariant initial condition of the same nuclei (oracle.glasma_bi):
p_T = eps_0 and p_L < 0 (flux tubes).  The nuclei must be resolved by the longitudinal
lattice and thin against 1/Q_s, so the lattice is fine along z: a_T = 16 a_L, dilute MV
charges (mu a_T = 1.4, m a_T = 0.8), sigma = 8, 4, 2 a_L.  The whole GPU pipeline (initial
conditions, CPIC, semi-implicit scheme at dt = a_L, observables, boost-invariant fields);
expected: p_T(z_c)/eps_0 rises towards 1 as sigma shrinks and p_L turns negative."""
import sys
import numpy as np
import pytest

import synth
from oracle import su, lattice, init_mv, glasma_bi
from _gpu import gpu, lattice_or_skip

pytestmark = gpu


@pytest.mark.parametrize("nc,nt,ns", [(2, 12, 1), (3, 10, 1), (3, 16, 3)])
def test_bi_fields_match_oracle(nc, nt, ns):
    pkg = lattice_or_skip()
    print("case: boost-invariant fields nc", nc, "nt", nt, "sheets", ns, flush=True)
    a_T, m = 4.0, 0.2
    if ns == 1:
        rA, rB = synth.mv_charges(91, nc, nt, 0.6, a_T)
    else:
        rA, rB = synth.mv_sheet_charges(91, nc, nt, 0.6, a_T, ns)
    p = lattice.Params(nc=nc, a_T=a_T, a_L=1.0, dt=0.5)
    mv = init_mv.MVParams(m_ir=m, uv_cut=0.0)
    aA = glasma_bi.transverse_alpha(glasma_bi.wilson_behind(rA, p, mv), a_T)
    aB = glasma_bi.transverse_alpha(glasma_bi.wilson_behind(rB, p, mv), a_T)
    Ez, Bz = glasma_bi.bi_fields(aA, aB)
    e0 = glasma_bi.bi_energy(aA, aB)
    got = pkg.boost_invariant_fields(nc, nt, rA, rB, a_T=a_T, m_ir=m)
    for name, ref in (("Ez", Ez), ("Bz", Bz)):
        r = np.moveaxis(su.to_components(ref), -1, 0)
        g = got[name].cpu().numpy()
        err = np.abs(g - r).max() / np.abs(r).max()
        print(" ", name, "max rel err", err, flush=True)
        assert err < 1e-11, (name, err)
    np.testing.assert_allclose([got["eps0"], got["EL2_half"], got["BL2_half"]], e0, rtol=1e-11)


def scan(pkg, sigma, scheme=1, dt=1.0):
    nc, nt, nz, aT = 3, 32, 96, 16.0
    m, mu, zA, zB = 0.8 / aT, 1.4 / aT, 72.0, 24.0
    rA, rB = synth.mv_charges(77, nc, nt, mu, aT)
    e0 = pkg.boost_invariant_fields(nc, nt, rA, rB, a_T=aT, m_ir=m)["eps0"]
    lat = pkg.Lattice(nc=nc, nz=nz, nt=nt, a_T=aT, a_L=1.0, dt=dt, fp=64, scheme=scheme, max_iter=300,
                      tol=1e-12)
    lat.init_mv(rA, rB, m_ir=m, uv_cut=0.0, sigma=sigma, zA=zA, zB=zB)
    t_c, z_c = 0.5 * (zA - zB), int(0.5 * (zA + zB))
    s_c = int(round(t_c / dt))
    per = int(round(2 / dt))
    lat.step(s_c)
    pt, pl = [], []
    for _ in range(10):
        lat.step(per)
        sl = lat.observables()["tmunu_z"]
        pt.append(sl[2][z_c] / e0)
        pl.append(sl[1][z_c] / sl[0][z_c])
    return np.array(pt), np.array(pl)


def test_thin_nuclei_approach_the_boost_invariant_glasma():
    pkg = lattice_or_skip()
    peaks, mins = [], []
    for sig in (8.0, 4.0, 2.0):
        print("case: boost-invariant limit, sigma", sig, flush=True)
        pt, pl = scan(pkg, sig)
        print("  p_T/eps_0", np.round(pt, 3), "p_L/eps", np.round(pl, 3), flush=True)
        peaks.append(pt.max())
        mins.append(pl.min())
    assert peaks[0] < peaks[1] < peaks[2], peaks
    assert abs(peaks[2] - 1.0) < 0.15, peaks
    assert mins[0] > 0.0 and mins[2] < -0.5, mins
