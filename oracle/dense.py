"""Dense and Krylov solves of the discretised vector Helmholtz system.
TEST INFRASTRUCTURE ONLY.

CBS converges to the solution of one linear system, A E_s = S with
A = L - K I_3 (the fixed point of the iteration: multiply E = G(V E + S) by
(L - kt2) and the shift cancels).  This module writes that system out with no
FFT at all: the 3D DFT is the Kronecker product of explicit 1D DFT matrices
built from cos/sin of exactly reduced angles, and the solve is LU
(numpy.linalg.solve).  It is the plain definition the iteration must reach.

``gmres_solve`` solves the same system matrix-free (FFT curl-curl, scipy GMRES)
for grids too large for dense LU.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse.linalg as spla

from . import cbs as _cbs


def dft_matrix(n: int) -> np.ndarray:
    """F[m, j] = exp(-2 pi i m j / n), angle reduced exactly mod n."""
    m = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    r = (m * j) % n
    ang = 2.0 * math.pi * r / n
    return np.cos(ang) - 1j * np.sin(ang)


def _freq_1d(n: int, d: float):
    """2 pi m/(n d) with m in FFT order (m = k for k < (n+1)//2, else k - n),
    and the same vector with its Nyquist entry zeroed for even n."""
    k = np.arange(n)
    m = np.where(k < (n + 1) // 2, k, k - n).astype(np.float64)
    p = 2.0 * math.pi * m / (n * d)
    pt = p.copy()
    if n % 2 == 0:
        pt[n // 2] = 0.0
    return p, pt


def curl_curl_dense(g: "_cbs.Grid") -> np.ndarray:
    """L (3N x 3N): L_ab = F3^-1 diag(|p|^2 delta_ab - pt_a pt_b) F3 with
    F3 = Fz (x) Fy (x) Fx acting on a [nz, ny, nx] volume flattened x-fastest."""
    N = g.n_vox
    F3 = np.kron(dft_matrix(g.nz), np.kron(dft_matrix(g.ny), dft_matrix(g.nx)))
    F3inv = F3.conj().T / N
    px, ptx = _freq_1d(g.nx, g.pitch)
    py, pty = _freq_1d(g.ny, g.pitch)
    pz, ptz = _freq_1d(g.nz, g.pitch)
    # per-mode vectors over the flattened (kz, ky, kx) index
    PX = np.tile(px, g.ny * g.nz)
    PY = np.tile(np.repeat(py, g.nx), g.nz)
    PZ = np.repeat(pz, g.nx * g.ny)
    TX = np.tile(ptx, g.ny * g.nz)
    TY = np.tile(np.repeat(pty, g.nx), g.nz)
    TZ = np.repeat(ptz, g.nx * g.ny)
    p2 = PX ** 2 + PY ** 2 + PZ ** 2
    T = (TX, TY, TZ)
    L = np.zeros((3 * N, 3 * N), dtype=np.complex128)
    for a in range(3):
        for b in range(3):
            diag = -T[a] * T[b]
            if a == b:
                diag = diag + p2
            L[a * N:(a + 1) * N, b * N:(b + 1) * N] = F3inv @ (diag[:, None] * F3)
    return L


def operator_dense(g: "_cbs.Grid", eps_r: np.ndarray) -> np.ndarray:
    """A = L - diag(K) (x) I_3, K = k0^2 eps_r + i kb^2 sigma."""
    L = curl_curl_dense(g)
    K = (g.k0 ** 2 * np.asarray(eps_r).astype(np.complex128)
         + 1j * g.kb ** 2 * _cbs.absorber_sigma(g)).reshape(-1)
    A = L.copy()
    idx = np.arange(3 * g.n_vox)
    A[idx, idx] -= np.tile(K, 3)
    return A


def dense_solve(g: "_cbs.Grid", eps_r: np.ndarray, S: np.ndarray) -> np.ndarray:
    """E_s = A^-1 S by LU, returned as [3, nz, ny, nx]."""
    A = operator_dense(g, eps_r)
    x = np.linalg.solve(A, np.asarray(S, dtype=np.complex128).reshape(-1))
    return x.reshape((3,) + g.vshape)


def gmres_solve(g: "_cbs.Grid", eps_r: np.ndarray, S: np.ndarray, rtol: float = 1e-12,
                maxiter: int = 20000, restart: int = 200) -> np.ndarray:
    """E_s = A^-1 S with FP64 GMRES and the matrix-free operator L - K."""
    N3 = 3 * g.n_vox
    K = (g.k0 ** 2 * np.asarray(eps_r).astype(np.complex128)
         + 1j * g.kb ** 2 * _cbs.absorber_sigma(g))
    shp = (3,) + g.vshape

    def mv(v):
        E = np.asarray(v).reshape(shp)
        return (_cbs.curl_curl_apply(g, E) - K[None] * E).reshape(-1)

    A = spla.LinearOperator((N3, N3), matvec=mv, dtype=np.complex128)
    b = np.asarray(S, dtype=np.complex128).reshape(-1)
    x, info = spla.gmres(A, b, rtol=rtol, atol=0.0, restart=restart, maxiter=maxiter)
    if info != 0:
        raise RuntimeError(f"GMRES did not converge (info={info})")
    return x.reshape(shp)


def cbs_gmres_solve(g: "_cbs.Grid", eps_r: np.ndarray, S: np.ndarray, rtol: float = 1e-10,
                    restart: int = 20, maxiter: int = 2000, x0: np.ndarray | None = None,
                    callback=None, require_convergence: bool = True) -> np.ndarray:
    """E_s = A^-1 S by FP64 GMRES on the preconditioned system of the CBS
    iteration (references [25], [26]).  The CBS step E <- E + gamma (G (V E + S) - E)
    has the fixed point of

        gamma (I - G V) E = gamma G S,

    which is A E = S multiplied by gamma G (G = (L - kb^2 - i eps)^-1, V = K -
    kb^2 - i eps, so (L - kb^2 - i eps)(I - G V) = L - K = A); GMRES on it reaches
    the same solution as the iteration without its slow tail.  rtol is the
    relative residual of this preconditioned system; x0 is an initial E_s (for
    instance a CBS iterate).  callback(k, residual) is called every inner step.
    With require_convergence=False the iterate after maxiter restart cycles is
    returned even if rtol was not met."""
    pot = _cbs.potentials(g, eps_r)
    shp = (3,) + g.vshape
    N3 = 3 * g.n_vox
    gam = pot.gamma[None]
    V = pot.V[None]

    def mv(v):
        E = np.asarray(v).reshape(shp)
        return (gam * (E - _cbs.green_apply(g, V * E, pot.kt2))).reshape(-1)

    M = spla.LinearOperator((N3, N3), matvec=mv, dtype=np.complex128)
    b = (gam * _cbs.green_apply(g, np.asarray(S, dtype=np.complex128), pot.kt2)).reshape(-1)
    steps = [0]

    def cb(r):
        steps[0] += 1
        if callback is not None:
            callback(steps[0], float(r))

    x, info = spla.gmres(M, b, x0=None if x0 is None else np.asarray(x0).reshape(-1),
                         rtol=rtol, atol=0.0, restart=restart, maxiter=maxiter,
                         callback=cb, callback_type="pr_norm")
    if info != 0 and require_convergence:
        raise RuntimeError(f"GMRES did not converge (info={info})")
    return x.reshape(shp)
