"""Initial conditions: two MV nuclei with finite longitudinal extent at t0.

Steps, in the paper's order:
1. MV colour charges rho^a_N(x_T) (Sec. 2, Gaussian W[rho]).  They are random draws
   and arrive as an input (``synth.mv_charges``); this module holds no RNG.
2. Transverse Poisson equation -Delta_T phi = rho with IR regulator m and UV cutoff
   Lambda (Sec. 2, the Fourier solution of the covariant-gauge field):
       phi^a(k) = rho^a(k) Theta(Lambda - |k~|) / (k~^2 + m^2),
       k~^2 = sum_{i=x,y} (2/a_T)^2 sin^2(k_i a_T / 2)   (lattice Laplacian symbol).
3. Single-sheet longitudinal profile (Sec. 3, eq. single_sheet; Sec. 4: a Gaussian of
   width L along z).  The colour structure does not depend on z, so the path-ordered
   Wilson line (Sec. 2) is an ordinary exponential of the cumulative profile:
       V_N(x, t) = exp(-i Lambda_N(z, t) phi_N(x_T)),
       Lambda_B = erfc((z - z_B - (t - t0)) / (sqrt(2) sigma)) / 2   (B moves along +z),
       Lambda_A = erfc(-(z - z_A + (t - t0)) / (sqrt(2) sigma)) / 2  (A moves along -z),
   so V = 1 ahead of a nucleus and exp(-i phi) behind it.
4. Pure-gauge LC fields of each nucleus (Sec. 3, eq. 3d_colorfield_1):
   U_i^N(x) = V_N(x) V_N^dag(x+i) for i = x, y and U_z^N = 1; the two nuclei are
   superposed (eq. 3d_colorfield_2) as U_i = U_i^A U_i^B, which equals the algebra
   sum wherever the nuclei do not overlap.
   Periodic z uses a seam link U_z(x_T, Nz-1) = V_A(x_T, Nz-1) V_B^dag(x_T, 0) that
   makes the plaquettes across the boundary trivial.
3'. Several sheets (longitudinal colour structure; Sec. 3 notes that charge densities
   rho(x^+-, x_T) more general than eq. single_sheet are allowed, and Sec. 5 names the
   stack of uncorrelated colour sheets).  The MV functional of Sec. 2 makes charges at
   different x^+- independent, so the nucleus is cut into ns pieces of equal weight of
   the profile, piece k carrying its own transverse charges rho_k (drawn with mu^2 / ns
   each, so that the total charge has the single-sheet variance).  Piece k is crossed
   while ns Lambda runs through [k, k + 1], with cumulative weight
       lambda_k(z, t) = clip(ns Lambda(z, t) - k, 0, 1),
   and within it the colour structure is that of rho_k, so the Wilson line is the
   ordered product
       V_N = exp(-i lambda_0 phi_{N,0}) exp(-i lambda_1 phi_{N,1}) ... exp(-i lambda_{ns-1} phi_{N,ns-1}),
   the factor of the piece the path crosses later on the right (sheet 0 is the leading
   edge: B's largest z, A's smallest z).  Sec. 2 defines V^dag as the path-ordered
   exponential of the field integrated up to x^+-; with later points to the left in
   V^dag, they stand to the right in V.  The same order follows from the form
   A_i = V d_i V^dag / (ig) of eq. 3d_colorfield_1: inside piece k, V = W e_k with W the
   completed pieces, so d_z A_i = W d_z(e_k d_i e_k^dag) W^dag and the field strength there
   is that of sheet k alone, rotated by W, as gauge covariance of the covariant-gauge
   field d_i phi_k demands (with e_k on the left it would pick up commutators of phi_k
   with the earlier sheets' pure gauge).  ns = 1 is step 3.  Identical sheets
   (rho_k = rho / ns) commute and give the single sheet with rho.
5. The links are built at t0 and t0 - dt; E(t0 - dt/2) = Log(U(t0) U^dag(t0 - dt)) /
   (i a_i dt) with the principal Log, so that eq. lattice_2 maps U(t0 - dt) onto U(t0).
6. The CPIC particles (Sec. 3) carry the charge that the lattice Gauss law (eq. gauss)
   assigns to the initial fields, one particle per site and nucleus: rho_B on
   n_z < Nz/2, rho_A on n_z >= Nz/2.  G = 0 to round-off at t0.

Pinned by tests/test_oracle_init.py: Poisson solve against the lattice Laplacian
applied back, Lambda cut as a no-op below max |k~|, trivial seam and transverse
plaquettes, exact reproduction of U(t0 - dt), Gauss law at t0, and a single nucleus
carrying the light-like field of Sec. 2 (p_T ~ 0, p_L ~ eps).  Sheets: identical sheets
reduce to one sheet, the Wilson line behind a nucleus equals the ordered product of
matrix exponentials of the sheets' fields (scipy's expm), the field energy of a
multi-sheet nucleus is the sum of those of its sheets taken alone (gauge covariance),
Gauss law and trivial transverse plaquettes at t0, and a single multi-sheet nucleus
stays light-like.
"""
from dataclasses import dataclass
import numpy as np
from scipy.special import erfc

from . import su
from .lattice import Params, State, shift, gauss


@dataclass
class MVParams:
    m_ir: float = 0.2
    uv_cut: float = 0.0      # Lambda; <= 0 means no cut
    sigma: float = 4.0       # longitudinal width L (in units of a_L)
    zA: float = 48.0         # centre of nucleus A (moves along -z)
    zB: float = 16.0         # centre of nucleus B (moves along +z)


def ktilde2(nt, a_T):
    """Lattice Laplacian symbol on the nt x nt transverse torus, shape (nt, nt) [ky, kx]."""
    n = np.arange(nt)
    s2 = (2.0 / a_T) ** 2 * np.sin(np.pi * n / nt) ** 2
    return s2[:, None] + s2[None, :]


def poisson(rhoT, a_T, m_ir, uv_cut):
    """phi^a = DFT^-1[ rho~^a Theta(Lambda - |k~|) / (k~^2 + m^2) ], rhoT shape (ng, ny, nx)."""
    nt = rhoT.shape[-1]
    k2 = ktilde2(nt, a_T)
    filt = 1.0 / (k2 + m_ir ** 2)
    if uv_cut > 0:
        filt = filt * (np.sqrt(k2) <= uv_cut)
    return np.real(np.fft.ifft2(np.fft.fft2(rhoT, axes=(-2, -1)) * filt, axes=(-2, -1)))


def lattice_laplacian_T(phi, a_T):
    """Delta_T phi on the transverse torus (used by the Poisson pin)."""
    out = -4.0 * phi
    for ax in (-1, -2):
        out = out + np.roll(phi, 1, axis=ax) + np.roll(phi, -1, axis=ax)
    return out / a_T ** 2


def profile_B(z, tau, mv):
    return 0.5 * erfc((z - mv.zB - tau) / (np.sqrt(2.0) * mv.sigma))


def profile_A(z, tau, mv):
    return 0.5 * erfc(-(z - mv.zA + tau) / (np.sqrt(2.0) * mv.sigma))


def sheet_weights(prof, ns):
    """lambda_k(z) = clip(ns Lambda(z) - k, 0, 1) for k = 0..ns-1, shape (ns, nz)."""
    k = np.arange(ns)[:, None]
    return np.clip(ns * prof[None, :] - k, 0.0, 1.0)


def wilson_lines(phi_mats, prof):
    """V(z, x_T) = prod_k exp(-i lambda_k(z) phi_k(x_T)), later sheets to the right.
    phi_mats (ns, ny, nx, N, N), prof (nz,)."""
    lam = sheet_weights(prof, phi_mats.shape[0])
    V = su.expi(-lam[0][:, None, None, None, None] * phi_mats[0][None])
    for k in range(1, phi_mats.shape[0]):
        V = V @ su.expi(-lam[k][:, None, None, None, None] * phi_mats[k][None])
    return V


def links_at(phiA, phiB, nz, tau, p, mv):
    """Links U (3, nz, ny, nx, N, N) of the superposed nuclei at t0 + tau; phiA, phiB
    (ns, ny, nx, N, N)."""
    z = np.arange(nz) * p.a_L
    VA = wilson_lines(phiA, profile_A(z, tau, mv))
    VB = wilson_lines(phiB, profile_B(z, tau, mv))
    U = np.empty((3,) + VA.shape, dtype=np.complex128)
    for i in range(2):
        UA = VA @ su.dag(shift(VA, i, 1))
        UB = VB @ su.dag(shift(VB, i, 1))
        U[i] = UA @ UB
    U[2] = su.eye_like(VA)
    U[2][nz - 1] = VA[nz - 1] @ su.dag(VB[0])
    return U


def sheet_fields(rhoT, p, mv):
    """phi of every sheet as matrices (ns, ny, nx, N, N); rhoT (ng, nt, nt) for one
    sheet or (ns, ng, nt, nt)."""
    r = np.asarray(rhoT, dtype=np.float64)
    if r.ndim == 3:
        r = r[None]
    return np.stack([su.from_components(np.moveaxis(poisson(rk, p.a_T, mv.m_ir, mv.uv_cut), 0, -1), p.nc)
                     for rk in r])


def initial_state(rhoT_A, rhoT_B, nz, p, mv):
    """State at step 0 from the transverse charges: components of shape (ng, nt, nt)
    (one sheet) or (ns, ng, nt, nt) (ns sheets, sheet 0 the leading edge)."""
    phiA = sheet_fields(rhoT_A, p, mv)
    phiB = sheet_fields(rhoT_B, p, mv)
    U0 = links_at(phiA, phiB, nz, 0.0, p, mv)
    U1 = links_at(phiA, phiB, nz, -p.dt, p, mv)
    a = p.a
    E = np.empty_like(U0)
    for i in range(3):
        E[i] = su.logi(U0[i] @ su.dag(U1[i])) / (a[i] * p.dt)
    rho = gauss(U0, E, np.zeros_like(U0[0]), a)
    half = nz // 2
    rhoB = rho.copy()
    rhoB[half:] = 0
    rhoA = rho.copy()
    rhoA[:half] = 0
    return State(U0, E, rhoA, rhoB, 0, p), U1


def state_from_algebra(Ualg, Ealg, p, split=True):
    """A general state from algebra components: U_i = exp(i Ualg_i), E_i = Ealg_i, and
    charges from the Gauss law (so that G = 0), split at Nz/2 between the nuclei.
    Ualg, Ealg: (3, nz, ny, nx, ng).  Used by tests to build arbitrary states."""
    nc = p.nc
    U = su.expi(su.from_components(Ualg, nc))
    E = su.from_components(Ealg, nc)
    rho = gauss(U, E, np.zeros_like(U[0]), p.a)
    nz = U.shape[1]
    half = nz // 2
    rhoB = rho.copy()
    rhoA = rho.copy()
    if split:
        rhoB[half:] = 0
        rhoA[:half] = 0
    else:
        rhoA[:] = 0
    return State(U, E, rhoA, rhoB, 0, p)
