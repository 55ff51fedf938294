"""Observables at integer time t = t0 + s dt (Sec. 4: <T^{mu nu}> and eq. pT_eL).

From the state at step s (U(t), E(t - dt/2), rho(t - dt/2)) the oracle takes the E
update of that step without applying it, so that E(t + dt/2) is known, and forms
    E_i^2     = ( |E_i(t-dt/2)|^2 + |E_i(t+dt/2)|^2 ) / 2,  |X|^2 = sum_a X^a X^a,
    B_{ij}^2  = 4 / (a_i a_j)^2 * Re Tr(1 - U_{i,j}),      (magnetic energy density
                 B^2/2 of the Wilson action in the normalisation Tr t^a t^b = delta/2)
    E_L^2 = E_z^2, E_T^2 = E_x^2 + E_y^2, B_L^2 = B_xy^2, B_T^2 = B_yz^2 + B_zx^2,
    eps = (E^2 + B^2)/2,  p_T = (E_L^2 + B_L^2)/2,  p_L = (E_T^2 + B_T^2 - E_L^2 - B_L^2)/2,
    S_L = -sum_a ( Ebar_x^a B_y^a - Ebar_y^a B_x^a ),  Ebar = (E(t-dt/2) + E(t+dt/2))/2,
    B_x^a = F_yz^a, B_y^a = F_zx^a, F_ij^a = 2 Tr(t^a proj(U_{i,j})) / (a_i a_j).
E = d_t A is minus the physical electric field, hence the overall sign of S_L, which
makes a +z mover carry S_L > 0 (checked on a single nucleus).  All quantities sit at
the base site x of their link / plaquette.  Slices are transverse means at each n_z.

Pinned by tests/test_oracle_lattice.py and tests/test_oracle_init.py: energy conservation in free evolution,
gauge invariance, a single nucleus before the collision (p_T ~ 0, p_L ~ eps,
S_L ~ +/- eps), and an abelian plane wave with closed-form energy density.
"""
import numpy as np

from . import su
from .lattice import (plaquette, force, is_hop_step, cpic_hop, gauss_residual,
                      unitarity_violation)


def half_step_fields(st, stepper_E=None):
    """E(t + dt/2) of the step that starts from st, without changing st."""
    p = st.params
    if stepper_E is not None:
        return stepper_E(st)
    if is_hop_step(st.step, p):
        _, _, j = cpic_hop(st.U, st.rhoA, st.rhoB, p)
    else:
        j = 0.0
    return st.E + p.dt * (force(st.U, p.a) + j)


def tmunu_slices(st, E_new=None):
    """Per-z transverse means: array (4, Nz) = [eps, p_L, p_T, S_L]; and the energy H."""
    p = st.params
    a = p.a
    if E_new is None:
        E_new = half_step_fields(st)
    E_old = st.E
    e2 = [0.5 * (su.algebra_norm2(E_old[i]) + su.algebra_norm2(E_new[i])) for i in range(3)]
    plaq = {(0, 1): plaquette(st.U, 0, 1), (1, 2): plaquette(st.U, 1, 2),
            (2, 0): plaquette(st.U, 2, 0)}
    b2 = {k: 4.0 / (a[k[0]] * a[k[1]]) ** 2 * np.real(su.trace(np.eye(p.nc) - P))
          for k, P in plaq.items()}
    EL2, ET2 = e2[2], e2[0] + e2[1]
    BL2, BT2 = b2[(0, 1)], b2[(1, 2)] + b2[(2, 0)]
    eps = 0.5 * (EL2 + ET2 + BL2 + BT2)
    pT = 0.5 * (EL2 + BL2)
    pL = 0.5 * (ET2 + BT2 - EL2 - BL2)
    Bx = su.to_components(su.proj(plaq[(1, 2)])) / (a[1] * a[2])
    By = su.to_components(su.proj(plaq[(2, 0)])) / (a[2] * a[0])
    Ebar = 0.5 * (E_old + E_new)
    Ex = su.to_components(Ebar[0])
    Ey = su.to_components(Ebar[1])
    SL = -np.sum(Ex * By - Ey * Bx, axis=-1)
    slices = np.stack([f.mean(axis=(1, 2)) for f in (eps, pL, pT, SL)])
    H = a[0] * a[1] * a[2] * eps.sum()
    return slices, H


def observables(st, E_new=None):
    """Everything the C-ABI's observables call reports, as a dict."""
    slices, H = tmunu_slices(st, E_new)
    g_rel, g_max = gauss_residual(st)
    return {"tmunu_z": slices, "energy": H, "gauss_rel": g_rel, "gauss_max": g_max,
            "unitarity": unitarity_violation(st.U)}


def local_rest_frame(slices):
    """Local rest frame energy density and flow velocity per z slice (Sec. 4: diagonalising
    the energy-momentum tensor gives eps_loc).

    From the transverse means T^00 = eps, T^0z = T^z0 = S_L (momentum density along +z) and
    T^zz = p_L the (t, z) block of T^mu_nu = T^{mu rho} g_{rho nu}, g = diag(1, -1), is
    [[eps, -S_L], [S_L, -p_L]].  Its timelike eigenvector u = gamma (1, v) solves
    S_L v^2 - (eps + p_L) v + S_L = 0, the root with |v| < 1 being
        v = 2 S_L / ((eps + p_L) + sqrt((eps + p_L)^2 - 4 S_L^2)),
    and the eigenvalue eps_loc = eps - S_L v = ((eps - p_L) + sqrt((eps + p_L)^2 - 4 S_L^2)) / 2.
    (The transverse block is already diagonal after the transverse average.)
    slices: (4, Nz) = [eps, p_L, p_T, S_L].  Returns (eps_loc, v), each (Nz,)."""
    eps, pL, _, SL = (np.asarray(slices[k], dtype=np.float64) for k in range(4))
    s = eps + pL
    root = np.sqrt(np.maximum(s * s - 4.0 * SL * SL, 0.0))
    den = s + root
    v = np.where(den > 0, 2.0 * SL / np.where(den > 0, den, 1.0), 0.0)
    return eps - SL * v, v


def milne(t, z, t_c, z_c):
    """Proper time and space-time rapidity of (t, z) relative to the collision point
    (t_c, z_c): tau = sqrt(dt^2 - dz^2), eta_s = atanh(dz / dt) for |dz| < dt (Sec. 4)."""
    dt, dz = np.asarray(t, dtype=np.float64) - t_c, np.asarray(z, dtype=np.float64) - z_c
    inside = np.abs(dz) < dt
    tau = np.where(inside, np.sqrt(np.where(inside, dt * dt - dz * dz, 0.0)), np.nan)
    eta = np.where(inside, np.arctanh(np.where(inside, dz / np.where(dt != 0, dt, 1.0), 0.0)), np.nan)
    return tau, eta
