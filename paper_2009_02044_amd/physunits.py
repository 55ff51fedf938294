"""Physical-unit front end (Sec. 4): the collision energy and the MV-model parameters in
GeV and fm mapped onto lattice inputs in units of the longitudinal spacing a_L = 1.

Sec. 4 fixes: Gaussian longitudinal profile of width L = m_N R / sqrt(s_NN), m_N ~ 1 GeV;
Q_s^2 ~ (sqrt(s_NN))^0.25 GeV^2; 0.75 g^2 mu ~ Q_s with g ~ 2; UV regulator
Lambda = 10 GeV; IR regulator m in 0.2 .. 0.8 GeV; SU(2); a 2048 x 192^2 lattice for a
(6 fm)^3 box; profiles read at tau_0 = 1 fm/c; the Landau width sqrt(ln gamma).
The nuclear radius R is not given; it defaults to the textbook 1.2 A^(1/3) fm of gold
(A = 197).  The fields absorb the coupling (g A -> A), so the charges' MV scale on the
lattice is g^2 mu (per-site standard deviation g^2 mu / a_T)."""
from dataclasses import dataclass
import math

HBARC_GEV_FM = 0.1973269804


@dataclass
class LatticeSetup:
    nz: int
    nt: int
    a_T: float        # transverse spacing in units of a_L
    a_L_fm: float     # a_L in fm
    sigma: float      # longitudinal width L / a_L
    mu: float         # g^2 mu in units of 1/a_L
    m_ir: float       # m in units of 1/a_L
    uv_cut: float     # Lambda in units of 1/a_L
    tau0: float       # 1 fm/c in units of a_L
    tau_fs: float     # 0.3 fm/c (onset of free streaming) in units of a_L
    gamma: float      # Lorentz factor sqrt(s_NN) / (2 m_N)
    sigma_landau: float
    L_fm: float
    Qs_GeV: float


def nuclear_radius_fm(A=197):
    return 1.2 * A ** (1.0 / 3.0)


def rhic_setup(sqrt_s_GeV=200.0, m_GeV=0.2, R_fm=None, box_fm=6.0, nz=2048, nt=192, g=2.0,
               Lambda_GeV=10.0, mN_GeV=1.0):
    """Lattice inputs for a collision at sqrt(s_NN) (defaults: the RHIC set-up of Sec. 4)."""
    R = nuclear_radius_fm() if R_fm is None else R_fm
    a_L_fm = box_fm / nz
    a_T_fm = box_fm / nt
    to_lat = a_L_fm / HBARC_GEV_FM          # GeV -> 1/a_L
    L_fm = mN_GeV * R / sqrt_s_GeV
    Qs = math.sqrt(sqrt_s_GeV ** 0.25)
    g2mu = Qs / 0.75
    gamma = sqrt_s_GeV / (2.0 * mN_GeV)
    return LatticeSetup(nz=nz, nt=nt, a_T=a_T_fm / a_L_fm, a_L_fm=a_L_fm, sigma=L_fm / a_L_fm,
                        mu=g2mu * to_lat, m_ir=m_GeV * to_lat, uv_cut=Lambda_GeV * to_lat,
                        tau0=1.0 / a_L_fm, tau_fs=0.3 / a_L_fm, gamma=gamma,
                        sigma_landau=math.sqrt(math.log(gamma)), L_fm=L_fm, Qs_GeV=Qs)


def gaussian_width(eta, f):
    """Width sigma_eta of the Gaussian A exp(-eta^2 / (2 sigma^2)) that fits f(eta) > 0 best
    in the least-squares sense of log f (a parabola in eta, symmetric about 0)."""
    import numpy as np
    eta = np.asarray(eta, dtype=np.float64)
    y = np.log(np.asarray(f, dtype=np.float64))
    M = np.stack([np.ones_like(eta), eta ** 2], axis=1)
    (c0, c2), *_ = np.linalg.lstsq(M, y, rcond=None)
    return math.sqrt(-1.0 / (2.0 * c2)) if c2 < 0 else float("inf")


def rapidity_profile(setup, charges, T_fm=2.6, nc=2, progress=None):
    """eps_loc tau against eta_s for the MV events whose transverse charges `charges` lists
    ((rhoT_A, rhoT_B) per event, drawn with setup.mu and setup.a_T) in the set-up:
    T^{mu nu} slices averaged over the events at lab
    time T_fm after the collision and diagonalised per layer on the GPU
    (glasma_rest_frame).  Under free streaming eps_loc tau depends on eta_s only, so the
    profile is read at one lab time: layers with tau >= 0.3 fm, clear of the receding
    nuclei and their wakes (|z - z_c| < T - 8 sigma).  Returns eta, eps_loc tau, the fitted
    Gaussian width and bookkeeping."""
    import numpy as np
    import torch
    from .glasma import Lattice
    nz, nt = setup.nz, setup.nt
    z_c = nz // 2
    t_c = int(round(6 * setup.sigma))
    T = int(round(T_fm / setup.a_L_fm))
    if T + 4 * setup.sigma >= z_c:
        raise ValueError("the nuclei leave the box before the lab time T_fm")
    acc, last, gauss = None, None, []
    events = len(charges)
    for e, (rA, rB) in enumerate(charges):
        lat = Lattice(nc=nc, nz=nz, nt=nt, a_T=setup.a_T, a_L=1.0, dt=0.5, fp=64)
        lat.init_mv(rA, rB, m_ir=setup.m_ir, uv_cut=setup.uv_cut, sigma=setup.sigma, zA=z_c + t_c, zB=z_c - t_c)
        lat.step(2 * (t_c + T))
        obs = lat.obs_buffer()
        lat.observe(obs)
        acc = obs.clone() if acc is None else acc + obs
        gauss.append(Lattice.unpack_obs(obs, nz)["gauss_rel"])
        if progress:
            progress(e, gauss[-1])
        if e == events - 1:
            last = lat
        del lat
    rf = last.rest_frame(acc / events).cpu().numpy()
    torch.cuda.synchronize()
    dz = np.arange(nz) - z_c
    tau = np.sqrt(np.maximum(T ** 2 - dz ** 2, 0.0))
    sel = (np.abs(dz) < T - 8 * setup.sigma) & (tau >= setup.tau_fs)
    eta = np.arctanh(dz[sel] / T)
    f = rf[0][sel] * tau[sel]
    return {"eta": eta, "eps_loc_tau": f, "sigma_eta": gaussian_width(eta, f), "steps": 2 * (t_c + T),
            "gauss_rel_max": max(gauss)}
