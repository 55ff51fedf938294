"""Physical-unit front end on the GPU (Sec. 4): the RHIC 200 GeV set-up on a lattice of half
the paper's resolution (1024 x 96^2 cells for the (6 fm)^3 box), two MV events per IR
regulator m.  The paper finds rapidity profiles of eps_loc that narrow as m grows
(sigma_eta = 2.34, 1.66, 1.28 for m = 0.2, 0.4, 0.8 GeV over 15 events); the ordering must
hold here, with widths of that order."""
import numpy as np

import synth
from _gpu import gpu, lattice_or_skip

pytestmark = gpu


def test_rapidity_width_narrows_with_the_ir_regulator():
    pkg = lattice_or_skip()
    from paper_2009_02044_amd import physunits as pu
    widths = []
    for m in (0.2, 0.4, 0.8):
        print("case: RHIC 200 GeV profile, 1024 x 96^2, m", m, flush=True)
        s = pu.rhic_setup(m_GeV=m, nz=1024, nt=96)
        ev = [synth.mv_charges(6000 + 100 * e, 2, s.nt, s.mu, s.a_T) for e in range(2)]
        r = pu.rapidity_profile(s, ev, T_fm=2.6)
        print("  sigma_eta", r["sigma_eta"], "Gauss", r["gauss_rel_max"], flush=True)
        assert r["gauss_rel_max"] < 1e-10
        widths.append(r["sigma_eta"])
    assert widths[0] > widths[1] > widths[2], widths
    assert 0.8 < widths[2] < 2.5 and widths[1] < 4.0, widths
