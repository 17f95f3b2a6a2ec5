"""Closed forms the CBS iteration must reproduce.  TEST INFRASTRUCTURE ONLY.

uniform_medium
    With K constant (no absorbing layer) every Fourier mode p evolves
    independently.  One CBS step is the affine 3x3 map
        E^ <- (1 - gamma) E^ + gamma G(p) (V E^ + S^),
    with G(p) = inv(M(p) - kt2 I) formed by explicit 3x3 inversion (not the
    Sherman-Morrison expression of the solver), and the limit is
    (M(p) - K I)^-1 S^.  This costs two FFTs on the host at any grid size, so
    it checks the iteration at full size.

slab_1d
    eps_r varying only along z, absorbing layer only along z and a source
    uniform in x and y: the field is uniform in x, y, only the px = py = 0
    modes are excited and M = pz^2 I - pt pt^T acts on the x component as pz^2.
    The x component then solves the 1D scalar spectral Helmholtz equation
        (D2 - K(z)) e = s,  D2 = F1^-1 diag(pz^2) F1,
    a dense nz x nz system built from an explicit DFT matrix (scalar CBS of
    reference [25] is exactly this reduction).
"""

from __future__ import annotations

import math

import numpy as np

from . import cbs as _cbs
from . import dense as _dense


def _mode_matrices(g, kt_or_K):
    """Stack of M(p) - c I over the [nz, ny, nx] grid -> [nz, ny, nx, 3, 3]."""
    (pz, py, px), (ptz, pty, ptx) = _cbs.fourier_grid(g)
    shp = g.vshape
    P = [np.broadcast_to(a, shp) for a in (px, py, pz)]
    T = [np.broadcast_to(a, shp) for a in (ptx, pty, ptz)]
    p2 = P[0] ** 2 + P[1] ** 2 + P[2] ** 2
    M = np.empty(shp + (3, 3), dtype=np.complex128)
    for a in range(3):
        for b in range(3):
            M[..., a, b] = -T[a] * T[b] + (p2 - kt_or_K if a == b else 0.0)
    return M


def uniform_medium(g, eps_const: complex, S: np.ndarray, iterations: int):
    """(E_s after `iterations` CBS steps, converged E_s) for a uniform medium.

    g must have no absorbing layer (sigma = 0 everywhere)."""
    assert tuple(g.pml) == (0, 0, 0)
    k0sq = g.k0 ** 2
    kb2 = g.kb ** 2
    V0 = k0sq * (complex(eps_const) - g.n_bg ** 2)
    eps = g.shift_factor * max(abs(V0), 1e-3 * kb2)
    V = V0 - 1j * eps
    gamma = 1j * V / eps
    kt2 = kb2 + 1j * eps
    Sh = _cbs.fftn3(np.asarray(S, dtype=np.complex128))          # [3, nz, ny, nx]
    Sv = np.moveaxis(Sh, 0, -1)                                   # [..., 3]
    Gm = np.linalg.inv(_mode_matrices(g, kt2))                    # explicit inverse
    E = np.zeros_like(Sv)
    for _ in range(iterations):
        GW = np.einsum("...ab,...b->...a", Gm, V * E + Sv)
        E = (1 - gamma) * E + gamma * GW
    Kc = k0sq * complex(eps_const)
    Einf = np.linalg.solve(_mode_matrices(g, Kc), Sv[..., None])[..., 0]
    Ek = _cbs.ifftn3(np.moveaxis(E, -1, 0))
    Ei = _cbs.ifftn3(np.moveaxis(Einf, -1, 0))
    return Ek, Ei


def slab_1d(nz: int, pitch: float, lambda0: float, n_bg: float, pml_z: int,
            eps_z: np.ndarray, s_z: np.ndarray, pml_order: int = 2,
            sigma_max: float = 1.0) -> np.ndarray:
    """Dense solve of (D2 - K(z)) e = s for the 1D reduction (see module doc).

    The absorbing profile along z is restated here from its definition:
    u = (p - k)/p on the low side, (k - (nz - p - 1))/p on the high side,
    sigma = sigma_max * min(1, u^m)."""
    k0 = 2.0 * math.pi / lambda0
    kb2 = (k0 * n_bg) ** 2
    sig = np.zeros(nz)
    for k in range(nz):
        if pml_z > 0 and k < pml_z:
            u = (pml_z - k) / pml_z
        elif pml_z > 0 and k >= nz - pml_z:
            u = (k - (nz - pml_z - 1)) / pml_z
        else:
            u = 0.0
        sig[k] = sigma_max * min(1.0, u ** pml_order)
    K = k0 ** 2 * np.asarray(eps_z, dtype=np.complex128) + 1j * kb2 * sig
    F = _dense.dft_matrix(nz)
    kk = np.arange(nz)
    m = np.where(kk < (nz + 1) // 2, kk, kk - nz)
    pz = 2.0 * math.pi * m / (nz * pitch)
    D2 = (F.conj().T / nz) @ ((pz ** 2)[:, None] * F)
    A = D2 - np.diag(K)
    return np.linalg.solve(A, np.asarray(s_z, dtype=np.complex128))


def uniform_medium_modes(g, eps_const: complex, modes, iterations: int):
    """Closed form for a source made of single Fourier modes in a uniform medium.

    modes: list of ((kx, ky, kz) FFT indices, s (3 complex)) with the source
    S(r) = sum_m s_m exp(i p_m . r).  Each mode stays a single mode:
    E_k(r) = sum_m exp(i p_m . r) e_m^(k), where e^(k) follows the 3x3 affine
    map e <- (1 - gamma) e + gamma inv(M(p) - kt2 I) (V e + s), e^(0) = 0, with
    the matrix inverted explicitly.  Returns [(p_m (x, y, z), e_m^(k))] with p
    in rad/m; evaluating at any voxel costs O(#modes), so this checks the
    iteration at any grid size."""
    k0sq = g.k0 ** 2
    kb2 = g.kb ** 2
    V0 = k0sq * (complex(eps_const) - g.n_bg ** 2)
    eps = g.shift_factor * max(abs(V0), 1e-3 * kb2)
    V = V0 - 1j * eps
    gamma = 1j * V / eps
    kt2 = kb2 + 1j * eps
    out = []
    for (kx, ky, kz), s in modes:
        p = []
        pt = []
        for k, n in ((kx, g.nx), (ky, g.ny), (kz, g.nz)):
            m = k if k < (n + 1) // 2 else k - n
            pa = 2.0 * math.pi * m / (n * g.pitch)
            p.append(pa)
            pt.append(0.0 if (n % 2 == 0 and 2 * k == n) else pa)
        p = np.array(p)
        pt = np.array(pt)
        M = np.dot(p, p) * np.eye(3) - np.outer(pt, pt)
        G = np.linalg.inv(M - kt2 * np.eye(3))
        s = np.asarray(s, dtype=np.complex128)
        e = np.zeros(3, dtype=np.complex128)
        for _ in range(iterations):
            e = (1 - gamma) * e + gamma * (G @ (V * e + s))
        out.append((p, e))
    return out
