"""SU(N) algebra for the oracle (N = 2, 3), matrices in the last two axes.

Conventions (Sec. 2: the generators t^a are traceless and hermitian):
* t^a = sigma^a / 2 (SU(2)) or lambda^a / 2 (SU(3), Gell-Mann), Tr t^a t^b = delta^ab / 2.
* A Lie-algebra field is a hermitian traceless matrix X = X^a t^a, X^a = 2 Tr(t^a X).
* ``proj(X)`` is the hermitian traceless part of (X - X^dag)/(2i).  The paper's
  anti-hermitian traceless part [X]_ah (Sec. 3, after eq. lattice_2) equals
  i * proj(X); the leapfrog update is written with proj so that E stays hermitian.

Pinned by tests/test_oracle_su.py against scipy.linalg.expm / logm and closed forms.
"""
import numpy as np

_SIGMA = np.array([[[0, 1], [1, 0]],
                   [[0, -1j], [1j, 0]],
                   [[1, 0], [0, -1]]], dtype=np.complex128)

_GELLMANN = np.zeros((8, 3, 3), dtype=np.complex128)
_GELLMANN[0][0, 1] = _GELLMANN[0][1, 0] = 1
_GELLMANN[1][0, 1], _GELLMANN[1][1, 0] = -1j, 1j
_GELLMANN[2][0, 0], _GELLMANN[2][1, 1] = 1, -1
_GELLMANN[3][0, 2] = _GELLMANN[3][2, 0] = 1
_GELLMANN[4][0, 2], _GELLMANN[4][2, 0] = -1j, 1j
_GELLMANN[5][1, 2] = _GELLMANN[5][2, 1] = 1
_GELLMANN[6][1, 2], _GELLMANN[6][2, 1] = -1j, 1j
_GELLMANN[7] = np.diag([1, 1, -2]) / np.sqrt(3)


def generators(nc):
    """t^a, shape (N^2-1, N, N)."""
    if nc == 2:
        return _SIGMA / 2
    if nc == 3:
        return _GELLMANN / 2
    raise ValueError("nc must be 2 or 3")


def ngen(nc):
    return nc * nc - 1


def dag(X):
    return np.conj(np.swapaxes(X, -1, -2))


def mul(*Ms):
    out = Ms[0]
    for M in Ms[1:]:
        out = out @ M
    return out


def trace(X):
    return np.trace(X, axis1=-2, axis2=-1)


def eye_like(X):
    n = X.shape[-1]
    return np.broadcast_to(np.eye(n, dtype=np.complex128), X.shape).copy()


def from_components(c, nc):
    """X = X^a t^a from components of shape (..., N^2-1)."""
    return np.tensordot(np.asarray(c, dtype=np.float64), generators(nc), axes=([-1], [0]))


def to_components(X):
    """X^a = 2 Re Tr(t^a X), shape (..., N^2-1)."""
    nc = X.shape[-1]
    t = generators(nc)
    return 2.0 * np.real(np.einsum("aij,...ji->...a", t, X))


def proj(X):
    """Hermitian traceless part of (X - X^dag)/(2i); [X]_ah = i proj(X)."""
    nc = X.shape[-1]
    Y = (X - dag(X)) / 2j
    return Y - (trace(Y)[..., None, None] / nc) * np.eye(nc)


def expi(H):
    """exp(i H) for hermitian H, through the spectral decomposition (eigh)."""
    w, V = np.linalg.eigh(H)
    return (V * np.exp(1j * w)[..., None, :]) @ dag(V)


def logi(W):
    """Principal Log with W = exp(i H): returns hermitian H with eigenvalues in (-pi/2, pi/2).

    W is unitary, hence normal; its eigenvectors are those of the hermitian matrix
    (W - W^dag)/(2i) = sin(H), which determines them uniquely while every eigen-angle
    lies in (-pi/2, pi/2).  The angles are then read off the diagonal of V^dag W V.
    Raises if an angle leaves that range (the initial conditions never get there).
    """
    K = (W - dag(W)) / 2j
    _, V = np.linalg.eigh(K)
    d = np.einsum("...ji,...jk,...ki->...i", np.conj(V), W, V)
    ang = np.angle(d)
    if np.any(np.abs(ang) >= np.pi / 2):
        raise ValueError("logi: eigen-angle outside (-pi/2, pi/2)")
    return (V * ang[..., None, :]) @ dag(V)


def transport(U, X):
    """U^dag X U: parallel transport of an adjoint quantity (Sec. 3, eq. gauss / CPIC)."""
    return dag(U) @ X @ U


def algebra_norm2(X):
    """|X|^2 = sum_a X^a X^a = 2 Tr X^2 for hermitian traceless X."""
    return 2.0 * np.real(trace(X @ X))


def reunitarize(U):
    """Nearest special-unitary matrix by polar decomposition (used only in tests)."""
    u, _, vh = np.linalg.svd(U)
    W = u @ vh
    det = np.linalg.det(W)
    nc = U.shape[-1]
    return W / (det ** (1.0 / nc))[..., None, None]
