"""Real component layout used at the C-ABI boundary (host-side, FP64), for tests.

Site index s = (n_z * Nt + n_y) * Nt + n_x (x fastest).
* links   U[i][c][s]: SU(2) c = 0..3 with U = u0 + i (u1 s1 + u2 s2 + u3 s3) (unit
  quaternion); SU(3) c = 2 (3 r + k) + {0: Re, 1: Im} for the entry (r, k).
* E field E[i][a][s] and charges rho[a][s]: algebra components X^a = 2 Tr(t^a X).
"""
import numpy as np

from . import su


def links_to_comp(U):
    """(3, nz, ny, nx, N, N) complex -> (3, r_U, V) float64."""
    nc = U.shape[-1]
    V = int(np.prod(U.shape[1:4]))
    M = U.reshape(3, V, nc, nc)
    if nc == 2:
        q = np.empty((3, 4, V))
        q[:, 0] = np.real(M[..., 0, 0] + M[..., 1, 1]) / 2
        q[:, 1] = np.imag(M[..., 0, 1] + M[..., 1, 0]) / 2
        q[:, 2] = np.real(M[..., 0, 1] - M[..., 1, 0]) / 2
        q[:, 3] = np.imag(M[..., 0, 0] - M[..., 1, 1]) / 2
        return q
    out = np.empty((3, 18, V))
    flat = M.reshape(3, V, 9)
    out[:, 0::2] = np.real(flat).transpose(0, 2, 1)
    out[:, 1::2] = np.imag(flat).transpose(0, 2, 1)
    return out


def comp_to_links(c, nc, dims):
    """Inverse of links_to_comp; dims = (nz, ny, nx)."""
    c = np.asarray(c, dtype=np.float64)
    V = int(np.prod(dims))
    c = c.reshape(3, -1, V)
    if nc == 2:
        u0, u1, u2, u3 = c[:, 0], c[:, 1], c[:, 2], c[:, 3]
        M = np.empty((3, V, 2, 2), dtype=np.complex128)
        M[..., 0, 0] = u0 + 1j * u3
        M[..., 0, 1] = u2 + 1j * u1
        M[..., 1, 0] = -u2 + 1j * u1
        M[..., 1, 1] = u0 - 1j * u3
    else:
        z = c[:, 0::2] + 1j * c[:, 1::2]          # (3, 9, V)
        M = z.transpose(0, 2, 1).reshape(3, V, 3, 3)
    return M.reshape((3,) + tuple(dims) + (nc, nc))


def alg_to_comp(X):
    """(..., nz, ny, nx, N, N) hermitian -> (..., ng, V)."""
    c = su.to_components(X)                       # (..., nz, ny, nx, ng)
    lead = c.shape[:-4]
    V = int(np.prod(c.shape[-4:-1]))
    c = c.reshape(lead + (V, c.shape[-1]))
    return np.swapaxes(c, -1, -2).copy()


def comp_to_alg(c, nc, dims, lead=()):
    c = np.asarray(c, dtype=np.float64)
    ng = nc * nc - 1
    V = int(np.prod(dims))
    c = c.reshape(lead + (ng, V))
    c = np.swapaxes(c, -1, -2).reshape(lead + tuple(dims) + (ng,))
    return su.from_components(c, nc)
