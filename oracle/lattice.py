"""Leapfrog evolution with CPIC charges (Sec. 3: eqs. lattice_1, lattice_2, plaquette,
continuity and the nearest-grid-point hop with parallel transport).

Field layout: U, E have shape (3, Nz, Ny, Nx, N, N) (direction i = 0:x, 1:y, 2:z);
charges rho_A, rho_B have shape (Nz, Ny, Nx, N, N).  All three directions are periodic.

Variables (the reading of the paper's mixed factors of a^i): E_i and j_i are the
physical (continuum-normalised) fields; the paper's E and j in eqs. lattice_1/2 are
a^i E_i and a^i j_i.  With that identification
    E_i(t + dt/2) = E_i(t - dt/2) + dt [ F_i(x) + j_i(x) ],
    F_i(x)        = -(1/a_i) sum_{j != i} a_j^{-2} proj(U_{i,j}(x) + U_{i,-j}(x)),
    U_i(t + dt)   = exp(i a_i dt E_i(t + dt/2)) U_i(t)
is eq. lattice_1/2 term by term, and the Gauss law (eq. gauss) and the continuity
equation (eq. continuity) read
    G(x) = sum_i [E_i(x) - U_i^dag(x-i) E_i(x-i) U_i(x-i)] / a_i - rho(x) = 0,
    [rho(t+dt/2) - rho(t-dt/2)] / dt = sum_i [j_i(x) - U_i^dag(x-i) j_i(x-i) U_i(x-i)] / a_i.

Pinned by tests/test_oracle_lattice.py: Gauss law to round-off through hops, unitarity,
gauge covariance, energy conservation with O(dt^2) fluctuations, the textbook
leapfrog dispersion relation, time reversibility and reduction to compact U(1).
"""
from dataclasses import dataclass, field
from fractions import Fraction
import numpy as np

from . import su

# array axis (within Nz, Ny, Nx) of lattice direction i
AXIS = {0: 2, 1: 1, 2: 0}


def shift(X, i, d):
    """Value at x + d * e_i (periodic) for a per-site array of shape (Nz, Ny, Nx, ...)."""
    return np.roll(X, -d, axis=AXIS[i])


@dataclass
class Params:
    nc: int
    a_T: float
    a_L: float
    dt: float

    @property
    def a(self):
        return (self.a_T, self.a_T, self.a_L)


@dataclass
class State:
    U: np.ndarray
    E: np.ndarray
    rhoA: np.ndarray
    rhoB: np.ndarray
    step: int = 0
    params: Params = None

    def copy(self):
        return State(self.U.copy(), self.E.copy(), self.rhoA.copy(), self.rhoB.copy(),
                     self.step, self.params)


def plaquette(U, i, j):
    """U_{i,j}(x) = U_i(x) U_j(x+i) U_i^dag(x+j) U_j^dag(x)  (eq. plaquette)."""
    return su.mul(U[i], shift(U[j], i, 1), su.dag(shift(U[i], j, 1)), su.dag(U[j]))


def plaquette_neg(U, i, j):
    """U_{i,-j}(x) = U_i(x) U_j^dag(x+i-j) U_i^dag(x-j) U_j(x-j): the plaquette in the
    (i, -j) plane, i.e. eq. plaquette with the link U_{-j}(y) = U_j^dag(y-j)."""
    Uj_m = shift(U[j], j, -1)
    return su.mul(U[i], su.dag(shift(Uj_m, i, 1)), su.dag(shift(U[i], j, -1)), Uj_m)


def force(U, a):
    """F_i(x) = -(1/a_i) sum_{j != i} a_j^{-2} proj(U_{i,j} + U_{i,-j})  (eq. lattice_1)."""
    F = np.zeros_like(U)
    for i in range(3):
        acc = np.zeros_like(U[i])
        for j in range(3):
            if j == i:
                continue
            acc += su.proj(plaquette(U, i, j) + plaquette_neg(U, i, j)) / a[j] ** 2
        F[i] = -acc / a[i]
    return F


def dt_ratio(params):
    """dt / a_L as an exact fraction (the hop schedule is integer arithmetic)."""
    r = Fraction(params.dt / params.a_L).limit_denominator(4096)
    if abs(float(r) - params.dt / params.a_L) > 1e-12 or r > 1 or r <= 0:
        raise ValueError("dt/a_L must be a rational number in (0, 1]")
    return r


def hop_count(s, params):
    """Number of cells a charge has advanced by time t0 + (s + 1/2) dt.

    The particles move at the speed of light (Sec. 2, eq. JA; recoil-less trajectories,
    Sec. 3); the nearest grid point of a particle that started on a site at t0 - dt/2
    changes when (s + 1/2) dt / a_L crosses a half-integer.  A tie is broken in the
    direction of motion.  S(s) = floor((s + 1/2) r + 1/2), r = dt/a_L.
    """
    r = dt_ratio(params)
    return int(np.floor((Fraction(2 * s + 1, 2)) * r + Fraction(1, 2)))


def is_hop_step(s, params):
    return hop_count(s, params) > hop_count(s - 1, params)


def cpic_hop(U, rhoA, rhoB, params):
    """One nearest-grid-point hop of every particle, with parallel transport and the
    current that satisfies eq. continuity exactly.

    Nucleus B moves along +z: a charge Q at x goes to x+z as U_z^dag(x) Q U_z(x)
    and leaves j_z(x) = -(a_L/dt) Q.  Nucleus A moves along -z: a charge Q at x goes
    to x-z as U_z(x-z) Q U_z^dag(x-z) and leaves j_z(x-z) = +(a_L/dt) Q', Q' the
    transported charge.  Substituting into eq. continuity at the source and the
    destination site gives an identity, so the Gauss law stays exact.
    Returns (rhoA_new, rhoB_new, j) with j of shape (3, Nz, Ny, Nx, N, N).
    """
    Uz = U[2]
    rhoB_moved = su.transport(Uz, rhoB)          # value that arrives at x+z
    rhoB_new = shift(rhoB_moved, 2, -1)           # new value at x comes from x-z
    rhoA_new = su.mul(Uz, shift(rhoA, 2, 1), su.dag(Uz))   # new A at x comes from x+z
    j = np.zeros((3,) + rhoA.shape, dtype=np.complex128)
    j[2] = (params.a_L / params.dt) * (rhoA_new - rhoB)
    return rhoA_new, rhoB_new, j


def leapfrog_step(st):
    """One step of eqs. lattice_1/2 with the CPIC hop on hop steps; returns a new State.

    State at step s: U(t), E(t - dt/2), rho(t - dt/2), t = t0 + s dt.
    """
    p = st.params
    a = p.a
    U, E = st.U, st.E
    if is_hop_step(st.step, p):
        rhoA, rhoB, j = cpic_hop(U, st.rhoA, st.rhoB, p)
    else:
        rhoA, rhoB, j = st.rhoA, st.rhoB, 0.0
    F = force(U, a)
    E_new = E + p.dt * (F + j)
    U_new = np.empty_like(U)
    for i in range(3):
        U_new[i] = su.expi(a[i] * p.dt * E_new[i]) @ U[i]
    return State(U_new, E_new, rhoA, rhoB, st.step + 1, p)


def evolve(st, n, stepper=None):
    stepper = stepper or leapfrog_step
    for _ in range(n):
        st = stepper(st)
    return st


def gauss(U, E, rho, a):
    """G(x) = sum_i [E_i(x) - U_i^dag(x-i) E_i(x-i) U_i(x-i)] / a_i - rho(x)  (eq. gauss)."""
    G = -rho.copy()
    for i in range(3):
        Um = shift(U[i], i, -1)
        Em = shift(E[i], i, -1)
        G += (E[i] - su.transport(Um, Em)) / a[i]
    return G


def gauss_residual(st):
    """(||G||_2 / ||rho||_2, max_a |G^a|) at the stored time level."""
    rho = st.rhoA + st.rhoB
    G = gauss(st.U, st.E, rho, st.params.a)
    g2 = np.sqrt(np.sum(su.algebra_norm2(G)))
    r2 = np.sqrt(np.sum(su.algebra_norm2(rho)))
    gmax = np.max(np.abs(su.to_components(G))) if G.size else 0.0
    return (g2 / r2 if r2 > 0 else g2), gmax


def unitarity_violation(U):
    n = U.shape[-1]
    dev = np.abs(su.dag(U) @ U - np.eye(n)).max()
    ddet = np.abs(np.linalg.det(U) - 1).max()
    return max(dev, ddet)


def gauge_transform(st, Omega):
    """U_i(x) -> Omega(x) U_i(x) Omega^dag(x+i); E, rho -> Omega E Omega^dag."""
    U = np.empty_like(st.U)
    E = np.empty_like(st.E)
    for i in range(3):
        U[i] = su.mul(Omega, st.U[i], su.dag(shift(Omega, i, 1)))
        E[i] = su.mul(Omega, st.E[i], su.dag(Omega))
    rA = su.mul(Omega, st.rhoA, su.dag(Omega))
    rB = su.mul(Omega, st.rhoB, su.dag(Omega))
    return State(U, E, rA, rB, st.step, st.params)


def force_at_site(U, a, site):
    """F_i at one site (z, y, x) by direct indexing: the same formula as force(),
    evaluated for a single site so that full-size lattices can be sampled."""
    nz, ny, nx = U.shape[1:4]

    def at(i, pos):
        z, y, x = pos
        return U[i, z % nz, y % ny, x % nx]

    def sh(pos, i, d):
        z, y, x = pos
        if i == 0:
            return (z, y, x + d)
        if i == 1:
            return (z, y + d, x)
        return (z + d, y, x)

    out = []
    for i in range(3):
        acc = 0
        for j in range(3):
            if j == i:
                continue
            xpi = sh(site, i, 1)
            up = at(i, site) @ at(j, xpi) @ su.dag(at(i, sh(site, j, 1))) @ su.dag(at(j, site))
            xmj = sh(site, j, -1)
            dn = at(i, site) @ su.dag(at(j, sh(xpi, j, -1))) @ su.dag(at(i, xmj)) @ at(j, xmj)
            acc = acc + su.proj(up + dn) / a[j] ** 2
        out.append(-acc / a[i])
    return np.stack(out)
