"""Linear (abelian, small-amplitude) symbol of the semi-implicit scheme, derived by hand
from the potential between two time slices that the scheme reads the improved action as
(Sec. 3, fig. wilson), for checking the oracle's and the GPU's evolution of plane waves.

Abelian limit: U_i = exp(i a_i A_i t^b) along one generator, plaquette fluxes
Phi_ij = a_i a_j F_ij with the lattice field strength F_ij = D_i A_j - D_j A_i,
D_j f(x) = (f(x + j) - f(x)) / a_j -> d_j = (exp(i k_j a_j) - 1) / a_j in Fourier space,
K_j = |d_j|^2 = (2/a_j)^2 sin^2(k_j a_j / 2).  In the (i, z) planes the flux splits into the
part of the transverse links, T = -a_i a_z D_z A_i, and of the longitudinal links,
L = a_i a_z D_i A_z.  Differentiating the slice potential
    k_xy Phi_xy^m Phi_xy^{m+1} + k_iz [(T^m + L^m)(T^m + L^{m+1}) + (T^{m+1} + L^{m+1})(T^{m+1} + L^m)]
with respect to the fields of slice t (both slice pairs (t - dt, t) and (t, t + dt)) gives,
with the time shift S (S A(t) = A(t + dt)), u = (S + S^-1)/2 and w = (S^-1 + 2 + S)/4:
  * the (x, y) plane: the Wilson force of F_xy averaged with u;
  * the (i, z) planes, equation of A_i: -K_z A_i(t) (explicit) + conj(d_z) d_i w A_z;
  * the (i, z) planes, equation of A_z: -K_i u A_z + conj(d_i) d_z w A_i.
For a mode A(t) ~ exp(-i w t), u -> c = cos(w dt), w -> (1 + c)/2, and the update
(A(t + dt) - 2 A(t) + A(t - dt)) / dt^2 = force reads lambda A = N(c) A with
lambda = 2 (1 - c) / dt^2 and N(c) = N0 + c N1 hermitian 3 x 3.  Both sides are linear in c:
    (2/dt^2 - N0) A = c (N1 + 2/dt^2) A,
a generalized hermitian eigenproblem whose eigenvalues are the cos(w dt) of the three
polarisations (one of them c = 1: the static gauge mode A ~ d).  Special cases: the
y-polarised wave with k_y = 0 gives c = (1 - dt^2 K_z/2) / (1 + dt^2 K_x/2); the A_z wave
with k_z = 0 gives c = 1 / (1 + dt^2 (K_x + K_y)/2).
"""
import numpy as np
import scipy.linalg as sla


def pencil(k, a, dt):
    """(P, Q) with P A = c Q A for the wave vector k = (k_x, k_y, k_z) (physical units)."""
    d = np.array([(np.exp(1j * k[i] * a[i]) - 1.0) / a[i] for i in range(3)])
    K = np.abs(d) ** 2
    N0 = np.zeros((3, 3), complex)
    N1 = np.zeros((3, 3), complex)
    N0[0, 0] = K[2]
    N1[0, 0] = K[1]
    N0[1, 1] = K[2]
    N1[1, 1] = K[0]
    N1[2, 2] = K[0] + K[1]
    N1[0, 1] = -np.conj(d[1]) * d[0]
    N1[1, 0] = np.conj(N1[0, 1])
    for i in (0, 1):
        v = -0.5 * np.conj(d[2]) * d[i]
        N0[i, 2] = N1[i, 2] = v
        N0[2, i] = N1[2, i] = np.conj(v)
    I = np.eye(3)
    return 2.0 / dt ** 2 * I - N0, N1 + 2.0 / dt ** 2 * I


def modes(k, a, dt):
    """Eigenvalues c = cos(w dt) (ascending) and eigenvectors (columns) of the pencil."""
    P, Q = pencil(k, a, dt)
    c, v = sla.eigh(P, Q)
    return c, v
