"""Boost-invariant Glasma at tau = 0+ (Sec. 2, eqs. glasma_ic1, glasma_ic2 and LC_gauge1):
the reference that thin nuclei must approach at mid-rapidity.

Test infrastructure (oracle): used by tests and the benchmark's physics legs only.

In the boost-invariant limit the nuclei are infinitely thin and the field at the
boundary of the forward light cone is fixed by the two pure-gauge LC fields alpha^i_A,
alpha^i_B (eq. LC_gauge1): A^i = alpha_A^i + alpha_B^i and A^eta = (ig/2)[alpha_A^i,
alpha_B^i].  With E^eta = (1/tau) d_tau A_eta and A_eta = tau^2 A^eta this gives purely
longitudinal fields (g = 1, hermitian algebra elements, sum over i = x, y):
    E_z = -i [alpha_A^i, alpha_B^i],
    B_z = -i ([alpha_A^x, alpha_B^y] - [alpha_A^y, alpha_B^x]),
and the energy density eps_0 = (E_z^2 + B_z^2) / 2 = p_T, p_L = -eps_0.

Lattice reading (the paper gives the continuum formula only; the reading is pinned against
it by its convergence, below): alpha^i_N lives on the transverse link (x, x + i) of the
lattice, alpha^i_N = P(V_N(x) V_N^dag(x + i)) / a_T with P the hermitian traceless part
of (W - W^dag)/(2i) (the nucleus' own transverse link U_i^N = exp(i a_T alpha^i_N) to
first order); E_z is taken at the site, averaging each commutator over the two links
of direction i that meet there; B_z at the centre of the xy plaquette, averaging
alpha^x over the plaquette's two x links and alpha^y over its two y links.  The
Wilson lines V_N are those behind the nucleus (all of its profile passed):
V_N = exp(-i phi_N) for one sheet, the ordered product over the sheets otherwise.

Pinned by tests/test_oracle_bi.py: closed forms for constant SU(2) fields (E_z and B_z
from a single commutator of generators), zero for commuting fields, invariance under
global colour rotations, E_z odd and B_z even under A <-> B, the weak-field limit of
alpha against the lattice derivative of phi, and convergence to the continuum formula:
for smooth, strongly non-abelian Wilson lines on a periodic square, E_z at the sites and
B_z at the plaquette centres approach the continuum commutators of alpha^i = -i V d_i V^dag
at second order in the spacing.
"""
import numpy as np

from . import su
from . import init_mv


def _com(X, Y):
    """-i [X, Y]: hermitian for hermitian X, Y."""
    return -1j * (X @ Y - Y @ X)


def transverse_alpha(V, a_T):
    """alpha^x, alpha^y on the links (x, x + i) from Wilson lines V (ny, nx, N, N)."""
    ax = su.proj(V @ su.dag(np.roll(V, -1, axis=1))) / a_T
    ay = su.proj(V @ su.dag(np.roll(V, -1, axis=0))) / a_T
    return ax, ay


def bi_fields(alpha_A, alpha_B):
    """(E_z at sites, B_z at plaquette centres) from (alpha^x, alpha^y) of each nucleus."""
    (axA, ayA), (axB, ayB) = alpha_A, alpha_B
    cx = _com(axA, axB)
    cy = _com(ayA, ayB)
    Ez = 0.5 * (cx + np.roll(cx, 1, axis=1)) + 0.5 * (cy + np.roll(cy, 1, axis=0))
    axA_p = 0.5 * (axA + np.roll(axA, -1, axis=0))
    axB_p = 0.5 * (axB + np.roll(axB, -1, axis=0))
    ayA_p = 0.5 * (ayA + np.roll(ayA, -1, axis=1))
    ayB_p = 0.5 * (ayB + np.roll(ayB, -1, axis=1))
    Bz = _com(axA_p, ayB_p) - _com(ayA_p, axB_p)
    return Ez, Bz


def bi_energy(alpha_A, alpha_B):
    """Transverse means (eps_0, E_z^2 / 2, B_z^2 / 2)."""
    Ez, Bz = bi_fields(alpha_A, alpha_B)
    e = 0.5 * su.algebra_norm2(Ez).mean()
    b = 0.5 * su.algebra_norm2(Bz).mean()
    return e + b, e, b


def wilson_behind(rhoT, p, mv):
    """V_N behind a nucleus from its transverse charges (one sheet or (ns, ...) sheets)."""
    phi = init_mv.sheet_fields(rhoT, p, mv)
    V = su.expi(-phi[0])
    for k in range(1, phi.shape[0]):
        V = V @ su.expi(-phi[k])
    return V


def bi_eps0(rhoT_A, rhoT_B, p, mv):
    """(eps_0, E_z^2/2, B_z^2/2) of the boost-invariant Glasma of these two nuclei."""
    aA = transverse_alpha(wilson_behind(rhoT_A, p, mv), p.a_T)
    aB = transverse_alpha(wilson_behind(rhoT_B, p, mv), p.a_T)
    return bi_energy(aA, aB)
