"""Stretched-coordinate PML (reference [31]) for the spectral vector Helmholtz
operator.  TEST INFRASTRUCTURE ONLY.

The paper's simulation volume is bounded by an absorbing layer, lambda thick
on the lateral axes and 6 lambda along z in total, of the perfectly matched kind
compared by its reference [31] (setup paragraph).  A stretched-coordinate PML replaces
every derivative d/da by (1/s_a(a)) d/da, with s_a = 1 + i alpha_a(a) inside the
layer of axis a and 1 elsewhere, so an outgoing wave exp(i k a) continues as
exp(i k a - k integral alpha) and decays without (in the continuum) reflecting.

Discretised with the spectral derivatives of the solver's operator: D_a =
F^-1 diag(i p_a) F (p with its Nyquist entry) and T_a = F^-1 diag(i pt_a) F (pt
zero at the Nyquist bin of an even axis), S_a = diag(s_a), and

    (L_s E)_c = - sum_{b != c} S_b^-1 D_b S_b^-1 D_b E_c
                + sum_{b != c} S_c^-1 S_b^-1 T_c T_b E_b   +   (N E)_c,

the stretched curl-curl (s_b depends on b only, so the mixed derivatives
commute with the other axes' stretch), plus N_c = F^-1 diag(p_c^2 - pt_c^2) F,
nonzero only at the Nyquist frequency of an even axis c, which makes L_s equal
the solver's L = F^-1 (|p|^2 I - pt pt^T) F exactly when alpha = 0.  The system
is (L_s - k0^2 eps_r) E_s = S with the scattered-field source S = k0^2 (eps_r -
n_bg^2) E_inc, which vanishes in the layer; there is no absorbing potential.

Profile (reading: the paper gives none): alpha(u) = alpha_max u^m with u the
depth into the layer in units of its thickness, the same u as the graded
potential's (outermost voxel u = 1).  In the continuum the round-trip
attenuation of a normally incident wave is exp(-2 k d alpha_max / (m + 1)) for
a layer of thickness d.

The CBS iteration needs a multiplicative potential V with |V| <= eps; the
stretched derivatives are differential operators with unbounded symbols, so
this operator is solved here by dense LU (the plain definition) and, for the
reflection of the 1D reduction, by a dense 1D solve.
"""

from __future__ import annotations

import math

import numpy as np

from . import cbs as _cbs
from . import dense as _dense


def stretch_1d(n: int, p: int, alpha_max: float, order: int) -> np.ndarray:
    """s(i) = 1 + i alpha_max u(i)^order over one axis (u as in the graded layer)."""
    u = _cbs._depth_1d(n, p)
    return 1.0 + 1j * alpha_max * u ** order


def _deriv_matrices(n: int, d: float):
    """Dense D (i p, Nyquist kept), T (i pt, Nyquist zeroed) and the Nyquist
    correction N = F^-1 diag(p^2 - pt^2) F of one axis."""
    F = _dense.dft_matrix(n)
    Fi = F.conj().T / n
    p, pt = _dense._freq_1d(n, d)
    D = Fi @ ((1j * p)[:, None] * F)
    T = Fi @ ((1j * pt)[:, None] * F)
    N = Fi @ ((p * p - pt * pt)[:, None] * F)
    return D, T, N


def operator_dense(g: "_cbs.Grid", eps_r: np.ndarray, alpha_max: float, order: int = 2):
    """A_s = L_s - k0^2 eps_r (3N x 3N) on the [nz, ny, nx] grid flattened x fastest."""
    dims = (g.nx, g.ny, g.nz)
    I = [np.eye(n) for n in dims]
    D, T, N, Si = [], [], [], []
    for a in range(3):
        Da, Ta, Na = _deriv_matrices(dims[a], g.pitch)
        D.append(Da)
        T.append(Ta)
        N.append(Na)
        Si.append(np.diag(1.0 / stretch_1d(dims[a], g.pml[a], alpha_max, order)))

    def lift(mats):
        """Kronecker lift of per-axis matrices (x, y, z) to the flattened volume."""
        return np.kron(mats[2], np.kron(mats[1], mats[0]))

    def on_axis(a, M):
        mats = list(I)
        mats[a] = M
        return lift(mats)

    def on_two(a, Ma, b, Mb):
        mats = list(I)
        mats[a] = Ma
        mats[b] = Mb
        return lift(mats)

    n = g.n_vox
    A = np.zeros((3 * n, 3 * n), dtype=np.complex128)
    for c in range(3):
        blk = on_axis(c, N[c]).astype(np.complex128)
        for b in range(3):
            if b == c:
                continue
            blk -= on_axis(b, Si[b] @ D[b] @ Si[b] @ D[b])
            A[c * n:(c + 1) * n, b * n:(b + 1) * n] += on_two(c, Si[c] @ T[c], b, Si[b] @ T[b])
        A[c * n:(c + 1) * n, c * n:(c + 1) * n] += blk
    K = g.k0 ** 2 * np.asarray(eps_r, dtype=np.complex128).reshape(-1)
    idx = np.arange(3 * n)
    A[idx, idx] -= np.tile(K, 3)
    return A


def solve_dense(g: "_cbs.Grid", eps_r: np.ndarray, S: np.ndarray, alpha_max: float,
                order: int = 2) -> np.ndarray:
    """E_s = A_s^-1 S by LU, [3, nz, ny, nx]."""
    A = operator_dense(g, eps_r, alpha_max, order)
    x = np.linalg.solve(A, np.asarray(S, dtype=np.complex128).reshape(-1))
    return x.reshape((3,) + g.vshape)


def slab_1d(nz: int, pitch: float, lambda0: float, n_bg: float, pml_z: int,
            eps_z: np.ndarray, s_z: np.ndarray, alpha_max: float, order: int = 2,
            kt: float = 0.0, component: str = "s") -> np.ndarray:
    """The 1D reduction along z of a field exp(i kt x) f(z) polarised along y
    ('s', kt a grid frequency, no x or y layer): -S^-1 D S^-1 D f + kt^2 f -
    k0^2 eps f = s (the y component has no z-Nyquist correction term).  With
    kt = 0 it is the normal-incidence reduction of either polarisation."""
    if component != "s":
        raise ValueError("only the s-polarised reduction is written out")
    k0 = 2.0 * math.pi / lambda0
    D, T, N = _deriv_matrices(nz, pitch)
    Si = np.diag(1.0 / stretch_1d(nz, pml_z, alpha_max, order))
    A = -Si @ D @ Si @ D + (kt * kt) * np.eye(nz) \
        - np.diag(k0 ** 2 * np.asarray(eps_z, dtype=np.complex128))
    return np.linalg.solve(A, np.asarray(s_z, dtype=np.complex128))


def reflection_normal(n: int, pitch: float, lambda0: float, pml: int, alpha_max: float,
                      order: int = 2, n_bg: float = 1.0):
    """R of the stretched layer at normal incidence (same sheet source and fit
    as the graded potential's ``absorber.reflection_normal``)."""
    from . import absorber as _ab
    k = 2.0 * math.pi * n_bg / lambda0
    src = pml + 6
    s = np.zeros(n, dtype=np.complex128)
    s[src] = 1.0
    e = slab_1d(n, pitch, lambda0, n_bg, pml, np.full(n, n_bg ** 2), s, alpha_max, order)
    lo, hi = _ab.fit_window(n, pml, src)
    z = np.arange(n) * pitch
    a, b, res = _ab.fit_counterpropagating(e[lo:hi], z[lo:hi], k)
    return abs(b / a) ** 2, res


# ---------------------------------------------------------------------------
# The stretched operator applied with FFTs, and its solve by GMRES on the CBS
# preconditioned system (grids too large for dense LU)
# ---------------------------------------------------------------------------
def _deriv_axis(f: np.ndarray, axis: int, symbol: np.ndarray) -> np.ndarray:
    """F^-1 diag(symbol) F along one numpy axis of f."""
    shape = [1] * f.ndim
    shape[axis] = symbol.size
    return np.fft.ifft(symbol.reshape(shape) * np.fft.fft(f, axis=axis), axis=axis)


def stretched_apply(g: "_cbs.Grid", E: np.ndarray, alpha_max: float, order: int = 2) -> np.ndarray:
    """L_s E for a field [3, nz, ny, nx], term by term as in the module notes:

        (L_s E)_c = - sum_{b != c} S_b^-1 D_b S_b^-1 D_b E_c
                    + sum_{b != c} S_c^-1 T_c S_b^-1 T_b E_b  +  N_c E_c

    with every 1D operator applied by FFT along its axis (the same operator
    as ``operator_dense``, which forms it as a matrix)."""
    E = np.asarray(E, dtype=np.complex128)
    dims = (g.nx, g.ny, g.nz)
    np_axis = (3, 2, 1)   # numpy axis of x, y, z in a [3, nz, ny, nx] array
    D, T, N, Si = [], [], [], []
    for a in range(3):
        p, pt = _dense._freq_1d(dims[a], g.pitch)
        D.append(1j * p)
        T.append(1j * pt)
        N.append(p * p - pt * pt)
        shape = [1, 1, 1, 1]
        shape[np_axis[a]] = dims[a]
        Si.append((1.0 / stretch_1d(dims[a], g.pml[a], alpha_max, order)).reshape(shape))

    def dS(f, a, sym):   # S_a^-1 (derivative with symbol sym along a) f
        return Si[a] * _deriv_axis(f, np_axis[a], sym[a])

    out = np.zeros_like(E)
    for c in range(3):
        Ec = E[c:c + 1]
        acc = _deriv_axis(Ec, np_axis[c], N[c].astype(np.complex128))
        for b in range(3):
            if b == c:
                continue
            acc = acc - dS(dS(Ec, b, D), b, D)
            acc = acc + dS(dS(E[b:b + 1], b, T), c, T)
        out[c] = acc[0]
    return out


def delta_apply(g: "_cbs.Grid", E: np.ndarray, alpha_max: float, order: int = 2) -> np.ndarray:
    """(L_s - L) E: what the stretched layer adds to the solver's operator."""
    return stretched_apply(g, E, alpha_max, order) - _cbs.curl_curl_apply(g, E)


def gmres_solve(g: "_cbs.Grid", eps_r: np.ndarray, S: np.ndarray, alpha_max: float,
                order: int = 2, rtol: float = 1e-10, restart: int = 20, maxiter: int = 200,
                callback=None, require_convergence: bool = True):
    """E_s = A_s^-1 S by FP64 GMRES, A_s = L_s - k0^2 eps_r (no absorbing
    potential: the grid must have sigma_max = 0).

    The CBS splitting (references [25], [26]) with G = (L - kb^2 - i eps)^-1,
    V = k0^2 eps_r - kb^2 - i eps and gamma = 1 + i V0/eps turns A_s E = S into

        gamma [E - G (V E - (L_s - L) E)] = gamma G S

    (multiply A_s = (L - kb^2 - i eps) - V + (L_s - L) by gamma G).  The CBS
    step with the source S - (L_s - L) E is E + (right side - left side), so
    this is the CBS iteration's own preconditioned system with the stretched
    derivatives added; GMRES solves it where the fixed-point iteration cannot
    (G (L_s - L) is not a contraction).  Restarted GMRES(restart) from E = 0;
    maxiter counts restart cycles; rtol is the relative residual of this
    system.  Returns (E_s [3, nz, ny, nx], relative residual)."""
    import scipy.sparse.linalg as spla
    if g.sigma_max != 0.0:
        raise ValueError("the stretched layer replaces the graded potential: sigma_max must be 0")
    pot = _cbs.potentials(g, eps_r)
    shp = (3,) + g.vshape
    N3 = 3 * g.n_vox
    gam = pot.gamma[None]
    V = pot.V[None]

    def mv(v):
        E = np.asarray(v).reshape(shp)
        W = V * E - delta_apply(g, E, alpha_max, order)
        return (gam * (E - _cbs.green_apply(g, W, pot.kt2))).reshape(-1)

    M = spla.LinearOperator((N3, N3), matvec=mv, dtype=np.complex128)
    b = (gam * _cbs.green_apply(g, np.asarray(S, dtype=np.complex128), pot.kt2)).reshape(-1)
    steps = [0]

    def cb(r):
        steps[0] += 1
        if callback is not None:
            callback(steps[0], float(r))

    x, info = spla.gmres(M, b, rtol=rtol, atol=0.0, restart=restart, maxiter=maxiter,
                         callback=cb, callback_type="pr_norm")
    res = float(np.linalg.norm(b - mv(x)) / np.linalg.norm(b))
    if info != 0 and require_convergence:
        raise RuntimeError(f"GMRES did not converge (info={info}, residual {res:.3e})")
    return x.reshape(shp), res
