"""Reference for the differentiation form (test infrastructure only): a loss of the final
state, its directional derivative by the tangent-linear (forward-mode) leapfrog, and
central finite differences.

Loss (reading of "integrated final energy density in a mid-rapidity slab", Sec. 4):
with the stored fields of the final state (U(t_N), E(t_N - dt/2)),
    L = a_x a_y a_z sum_{x: z0 <= z < z1} [ 1/2 sum_i |E_i(x)|^2
                                            + sum_{i<j} 2/(a_i a_j)^2 Re Tr(1 - U_{i,j}(x)) ],
the electric and Wilson magnetic energy of layers [z0, z1) (E at the stored half step,
no time averaging, so that the loss is a function of one state).

Tangents: a perturbation of the state is (xi, dE, drhoA, drhoB) with hermitian traceless
xi_i(x) (links move as U_i -> exp(i h xi_i) U_i, i.e. dU_i = i xi_i U_i), and hermitian
traceless dE, drho.  tangent_step() differentiates one leapfrog step (eqs. lattice_1/2,
plaquette, the CPIC hop) term by term with the product rule; the derivative of the
link update uses the Daleckii-Krein form of the derivative of the matrix exponential
in the eigenbasis of E.

Pinned by tests/test_oracle_adjoint.py: the exponential derivative against
scipy.linalg.expm_frechet; the loss in closed form; the tangent-linear result against
central finite differences through hop and non-hop steps; vanishing derivative along
infinitesimal gauge transformations (gauge invariance of the loss and covariance of
the dynamics).
"""
import numpy as np

from . import su
from .lattice import State, plaquette, plaquette_neg, shift, is_hop_step, cpic_hop, leapfrog_step, evolve

PLANES = ((0, 1), (1, 2), (2, 0))


def slab_loss(st, z0, z1):
    p = st.params
    a = p.a
    e2 = 0.5 * np.sum(su.algebra_norm2(st.E[:, z0:z1]))
    b = 0.0
    for (i, j) in PLANES:
        P = plaquette(st.U, i, j)[z0:z1]
        b += 2.0 / (a[i] * a[j]) ** 2 * np.sum(np.real(su.trace(np.eye(p.nc) - P)))
    return a[0] * a[1] * a[2] * (e2 + b)


def dexpi_left(H, dH, c):
    """xi with d/dh exp(i c (H + h dH)) = i xi exp(i c H), for hermitian H, dH.

    xi = c int_0^1 exp(i s c H) dH exp(-i s c H) ds; in the eigenbasis H = V diag(l) V^dag
    the integral multiplies entry (k, l) of V^dag dH V by phi(i c (l_k - l_l)),
    phi(z) = (e^z - 1)/z, phi(0) = 1."""
    w, V = np.linalg.eigh(H)
    D = su.dag(V) @ dH @ V
    z = 1j * c * (w[..., :, None] - w[..., None, :])
    small = np.abs(z) < 1e-8
    zs = np.where(small, 1.0, z)
    phi = np.where(small, 1.0 + z / 2 + z * z / 6, np.expm1(zs) / zs)
    return c * (V @ (D * phi) @ su.dag(V))


def dplaquette(U, dU, i, j):
    """Derivative of U_{i,j}(x) = U_i(x) U_j(x+i) U_i^dag(x+j) U_j^dag(x) for link
    derivatives dU (product rule)."""
    f = (U[i], shift(U[j], i, 1), su.dag(shift(U[i], j, 1)), su.dag(U[j]))
    d = (dU[i], shift(dU[j], i, 1), su.dag(shift(dU[i], j, 1)), su.dag(dU[j]))
    return _product_rule(f, d)


def dplaquette_neg(U, dU, i, j):
    """Derivative of U_{i,-j}(x) = U_i(x) U_j^dag(x+i-j) U_i^dag(x-j) U_j(x-j)."""
    Uj_m, dUj_m = shift(U[j], j, -1), shift(dU[j], j, -1)
    f = (U[i], su.dag(shift(Uj_m, i, 1)), su.dag(shift(U[i], j, -1)), Uj_m)
    d = (dU[i], su.dag(shift(dUj_m, i, 1)), su.dag(shift(dU[i], j, -1)), dUj_m)
    return _product_rule(f, d)


def _product_rule(f, d):
    out = 0
    for k in range(len(f)):
        out = out + su.mul(*[d[m] if m == k else f[m] for m in range(len(f))])
    return out


def comm(A, B):
    return A @ B - B @ A


def tangent_step(st, tan):
    """One leapfrog step of the state and of its tangent (xi, dE, drhoA, drhoB)."""
    p = st.params
    a = p.a
    U = st.U
    xi, dE, drA, drB = tan
    dU = 1j * (xi @ U)
    if is_hop_step(st.step, p):
        rA_new, _, _ = cpic_hop(U, st.rhoA, st.rhoB, p)
        Uz, xz = U[2], xi[2]
        # rho_A'(x) = U_z(x) rho_A(x+z) U_z^dag(x)
        drA_new = 1j * comm(xz, rA_new) + su.mul(Uz, shift(drA, 2, 1), su.dag(Uz))
        # rho_B'(x+z) = U_z^dag(x) rho_B(x) U_z(x)
        drB_new = shift(su.transport(Uz, drB - 1j * comm(xz, st.rhoB)), 2, -1)
        dj = np.zeros_like(dE)
        dj[2] = (p.a_L / p.dt) * (drA_new - drB)
    else:
        drA_new, drB_new, dj = drA, drB, 0.0
    dF = np.zeros_like(dE)
    for i in range(3):
        acc = 0
        for j in range(3):
            if j == i:
                continue
            acc = acc + su.proj(dplaquette(U, dU, i, j) + dplaquette_neg(U, dU, i, j)) / a[j] ** 2
        dF[i] = -acc / a[i]
    dE_new = dE + p.dt * (dF + dj)
    new = leapfrog_step(st)
    xi_new = np.empty_like(xi)
    for i in range(3):
        c = a[i] * p.dt
        W = su.expi(c * new.E[i])
        xi_new[i] = dexpi_left(new.E[i], dE_new[i], c) + su.mul(W, xi[i], su.dag(W))
    return new, (xi_new, dE_new, drA_new, drB_new)


def dloss(st, tan, z0, z1):
    """Derivative of slab_loss along the tangent."""
    p = st.params
    a = p.a
    xi, dE = tan[0], tan[1]
    dU = 1j * (xi @ st.U)
    de = np.sum(2.0 * np.real(su.trace(st.E[:, z0:z1] @ dE[:, z0:z1])))
    db = 0.0
    for (i, j) in PLANES:
        dP = dplaquette(st.U, dU, i, j)[z0:z1]
        db -= 2.0 / (a[i] * a[j]) ** 2 * np.sum(np.real(su.trace(dP)))
    return a[0] * a[1] * a[2] * (de + db)


def jvp(st, tan, steps, z0, z1):
    """(L, dL) after `steps` leapfrog steps from st along the initial tangent."""
    for _ in range(steps):
        st, tan = tangent_step(st, tan)
    return slab_loss(st, z0, z1), dloss(st, tan, z0, z1)


def zero_tangent(st):
    return (np.zeros_like(st.U), np.zeros_like(st.E), np.zeros_like(st.rhoA), np.zeros_like(st.rhoB))


def tangent_from_components(st, cU=None, cE=None, cA=None, cB=None):
    """Tangent from algebra components ((3, nz, ny, nx, n_g) for xi and dE, (nz, ny, nx, n_g)
    for the charges); missing parts are zero."""
    nc = st.params.nc
    z = zero_tangent(st)
    return tuple(z[k] if c is None else su.from_components(c, nc)
                 for k, c in enumerate((cU, cE, cA, cB)))


def perturbed(st, tan, h):
    """The state moved by h along the tangent (links by exp(i h xi))."""
    xi, dE, drA, drB = tan
    return State(su.expi(h * xi) @ st.U, st.E + h * dE, st.rhoA + h * drA, st.rhoB + h * drB,
                 st.step, st.params)


def fd_directional(st, tan, steps, z0, z1, h=1e-4):
    """(L(x0 + h v) - L(x0 - h v)) / (2 h) after `steps` leapfrog steps."""
    lp = slab_loss(evolve(perturbed(st, tan, h), steps), z0, z1)
    lm = slab_loss(evolve(perturbed(st, tan, -h), steps), z0, z1)
    return (lp - lm) / (2 * h)


def gauge_tangent(st, omega):
    """Tangent of the gauge transformation Omega = exp(i h omega(x)) at h = 0:
    U_i(x) -> Omega(x) U_i(x) Omega^dag(x+i), E, rho -> Omega E Omega^dag."""
    U = st.U
    xi = np.empty_like(U)
    dE = np.empty_like(st.E)
    for i in range(3):
        xi[i] = omega - su.mul(U[i], shift(omega, i, 1), su.dag(U[i]))
        dE[i] = 1j * comm(omega, st.E[i])
    return (xi, dE, 1j * comm(omega, st.rhoA), 1j * comm(omega, st.rhoB))
