"""Plain FP64 vector convergent Born series (CBS).  TEST INFRASTRUCTURE ONLY.

What is computed
----------------
The paper (arXiv 2506.15411) solves the 3D vector Helmholtz/Maxwell problem
with the convergent Born series of its references [25] (scalar CBS, Osnabrugge
et al. 2016) and [26] (vector CBS, Krueger et al. 2017), with an absorbing layer
of thickness [lambda, lambda, 6 lambda] (simulation-setup paragraph, reference
[31]) and an x-polarised plane wave at normal incidence (design paragraph).
The paper prints none of the CBS equations; this module restates them:

    A E_s = S,  A = L - K I_3,  L = F^-1 diag(M(p)) F,  M(p) = |p|^2 I - pt pt^T
    K(r)  = k0^2 eps_r(r) + i kb^2 sigma(r)          (sigma: absorbing profile)
    V0    = K - kb^2,  eps = kappa max|V0|,  V = V0 - i eps,  gamma = (i/eps) V
    G^(p) = (M(p) - (kb^2 + i eps) I)^-1                (dyadic Green's tensor)
    iteration:  E_s <- E_s + gamma (F^-1 G^ F (V E_s + S) - E_s),  E_s^(0) = 0

Readings taken where the paper is silent (each also listed in the design notes):
  * time convention exp(-i w t); Im eps_r >= 0 is passive/absorbing;
  * eps = kappa * max|V0| over the grid (floor 1e-3 kb^2 on max|V0|), with
    kappa >= 1 (default 1.1).  The convergence condition of [25] is on the
    unshifted potential, eps >= max|V0| ("eps >= max|V|" with the shifted V is
    impossible since |V0 - i eps| >= eps).  Any admissible eps gives the same
    converged field; kappa = 1 leaves the local factor |1 - gamma| = |V0|/eps
    at 1 in the strongest-contrast voxels, where high spatial frequencies then
    barely decay, and makes gamma = 0 (voxels never updated) wherever the
    absorbing potential alone attains the bound;
  * Nyquist bins of even axes: pt (the vector in the dyadic term only) is zero
    there, which makes A exactly complex-symmetric (A^T = A);
  * scattered-field formulation: S = k0^2 (eps_r - n_bg^2) E_inc with
    E_inc = pol * exp(i kb z), phase zero at grid index z = 0, unit amplitude;
    the absorbing potential acts on the scattered field only;
  * absorbing layer thickness: per-side voxel counts pml = (px, py, pz) given by
    the caller; profile sigma = sigma_max * min(1, sum_a u_a^m) with u_a the
    depth into the layer in units of its thickness (m = 2, sigma_max = 1 by
    default, fixed per plan so that sigma does not depend on eps_r);
  * stopping rule: eta_k = ||E^(k+1) - E^(k)|| / ||E^(k+1)|| <= tol (FP64 norms
    over all voxels and components) or k = max_iter.

Arrays use the device layout: scalar volumes are [nz, ny, nx] (x fastest),
vector fields are [3, nz, ny, nx]; component 0 is x.  Lengths are in metres.
"""

from __future__ import annotations

import dataclasses
import math
import os

import numpy as np
import scipy.fft as sfft

_WORKERS = max(1, int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1))


# ---------------------------------------------------------------------------
# Problem description
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Grid:
    """Voxel grid with one isotropic pitch (simulation-setup paragraph).

    shape is (nx, ny, nz); pml is the per-side absorbing-layer thickness in
    voxels along x, y, z.  Voxel (i, j, k) has its centre at (i d, j d, k d).
    """

    nx: int
    ny: int
    nz: int
    pitch: float
    lambda0: float = 1.064e-6
    n_bg: float = 1.0
    pml: tuple = (0, 0, 0)
    pml_order: int = 2
    sigma_max: float = 1.0
    shift_factor: float = 1.1

    @property
    def k0(self) -> float:
        return 2.0 * math.pi / self.lambda0

    @property
    def kb(self) -> float:
        return self.k0 * self.n_bg

    @property
    def n_vox(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def vshape(self):
        return (self.nz, self.ny, self.nx)


# ---------------------------------------------------------------------------
# Absorbing layer (simulation-setup paragraph, reference [31]; reading above)
# ---------------------------------------------------------------------------
def _depth_1d(n: int, p: int) -> np.ndarray:
    """u in (0, 1] inside a layer of p voxels on each side of an axis, else 0.

    Low side: voxel i < p has u = (p - i)/p; high side: voxel i >= n - p has
    u = (i - (n - p - 1))/p.  The outermost voxel gets u = 1 and the first
    layer voxel next to the interior gets 1/p; mirror-symmetric in i -> n-1-i.
    """
    u = np.zeros(n, dtype=np.float64)
    if p <= 0:
        return u
    i = np.arange(n)
    lo = i < p
    hi = i >= n - p
    u[lo] = (p - i[lo]) / p
    u[hi] = (i[hi] - (n - p - 1)) / p
    return u


def absorber_sigma(g: Grid) -> np.ndarray:
    """sigma(r) = sigma_max * min(1, sum_a u_a(r)^m), zero in the interior."""
    ux = _depth_1d(g.nx, g.pml[0]) ** g.pml_order
    uy = _depth_1d(g.ny, g.pml[1]) ** g.pml_order
    uz = _depth_1d(g.nz, g.pml[2]) ** g.pml_order
    s = uz[:, None, None] + uy[None, :, None] + ux[None, None, :]
    return g.sigma_max * np.minimum(1.0, s)


def interior_mask(g: Grid) -> np.ndarray:
    """True for voxels outside the absorbing layer."""
    def m1(n, p):
        i = np.arange(n)
        return (i >= p) & (i < n - p)
    return (m1(g.nz, g.pml[2])[:, None, None]
            & m1(g.ny, g.pml[1])[None, :, None]
            & m1(g.nx, g.pml[0])[None, None, :])


def validate(g: Grid, eps_r: np.ndarray) -> None:
    """Input checks of a passive medium: finite, Im eps_r >= 0, and
    eps_r == n_bg^2 inside the absorbing layer (compared at float32, the
    precision in which permittivities are supplied)."""
    eps_r = np.asarray(eps_r)
    if eps_r.shape != g.vshape:
        raise ValueError(f"eps_r shape {eps_r.shape} != {g.vshape}")
    if not np.all(np.isfinite(eps_r)):
        raise ValueError("eps_r has non-finite values")
    if np.any(np.imag(eps_r) < 0):
        raise ValueError("gain medium (Im eps_r < 0) is not admissible")
    nb2 = np.float32(g.n_bg * g.n_bg)
    layer = ~interior_mask(g)
    if np.any(eps_r[layer] != nb2):
        raise ValueError("eps_r must equal n_bg^2 inside the absorbing layer")


# ---------------------------------------------------------------------------
# Potentials (vector CBS, references [25], [26])
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Potentials:
    K: np.ndarray        # k0^2 eps_r + i kb^2 sigma           [nz,ny,nx] complex128
    V0: np.ndarray       # K - kb^2                             unshifted potential
    eps: float           # shift, kappa * max|V0| (floor 1e-3 kb^2)
    V: np.ndarray        # V0 - i eps                           shifted potential
    gamma: np.ndarray    # (i/eps) V = 1 + i V0/eps             preconditioner
    kt2: complex         # kb^2 + i eps                         Green's denominator


def potentials(g: Grid, eps_r: np.ndarray, eps_shift: float | None = None) -> Potentials:
    """K, V0, eps, V, gamma exactly as defined for CBS in [25]/[26]
    (eps = shift_factor * max|V0|, see the module notes).

    V0 is formed as k0^2 (eps_r - n_bg^2) + i kb^2 sigma, which equals
    K - kb^2 without the cancellation of subtracting two large numbers.
    ``eps_shift`` overrides eps (used by the eps-independence pin).
    """
    eps_r = np.asarray(eps_r).astype(np.complex128)
    sigma = absorber_sigma(g)
    k0sq = g.k0 ** 2
    kb2 = g.kb ** 2
    V0 = k0sq * (eps_r - g.n_bg ** 2) + 1j * kb2 * sigma
    K = V0 + kb2
    if eps_shift is None:
        eps = g.shift_factor * max(float(np.max(np.abs(V0))) if V0.size else 0.0, 1e-3 * kb2)
    else:
        eps = float(eps_shift)
    V = V0 - 1j * eps
    gamma = (1j / eps) * V
    return Potentials(K=K, V0=V0, eps=eps, V=V, gamma=gamma, kt2=kb2 + 1j * eps)


# ---------------------------------------------------------------------------
# Fourier grid and dyadic Green's tensor
# ---------------------------------------------------------------------------
def frequencies(n: int, d: float):
    """p = 2 pi m/(n d) with m in FFT order; pt equals p except that it is 0
    at the Nyquist index m = -n/2 of an even axis (reading of the dyadic term
    that keeps the discrete operator complex-symmetric)."""
    m = np.fft.fftfreq(n) * n          # exact integers in FFT order
    p = 2.0 * math.pi * m / (n * d)
    pt = p.copy()
    if n % 2 == 0:
        pt[n // 2] = 0.0
    return p, pt


def fourier_grid(g: Grid):
    """Broadcastable (pz, py, px) and (ptz, pty, ptx) over [nz, ny, nx]."""
    px, ptx = frequencies(g.nx, g.pitch)
    py, pty = frequencies(g.ny, g.pitch)
    pz, ptz = frequencies(g.nz, g.pitch)
    P = (pz[:, None, None], py[None, :, None], px[None, None, :])
    Pt = (ptz[:, None, None], pty[None, :, None], ptx[None, None, :])
    return P, Pt


def green_tensor(p: np.ndarray, pt: np.ndarray, kt2: complex) -> np.ndarray:
    """G^(p) = (M(p) - kt2 I)^-1 with M = |p|^2 I - pt pt^T, written in
    Sherman-Morrison form:  [I + pt pt^T / (|p|^2 - |pt|^2 - kt2)] / (|p|^2 - kt2).
    Where pt = p this is (I - p p^T / kt2) / (|p|^2 - kt2), the dyadic Green's
    function of vector CBS [26].  p, pt: [..., 3] (x, y, z); returns [..., 3, 3].
    """
    p = np.asarray(p, dtype=np.float64)
    pt = np.asarray(pt, dtype=np.float64)
    p2 = np.sum(p * p, axis=-1)
    pt2 = np.sum(pt * pt, axis=-1)
    a = 1.0 / (p2 - kt2)
    b = 1.0 / (p2 - pt2 - kt2)
    eye = np.eye(3)
    outer = pt[..., :, None] * pt[..., None, :]
    return a[..., None, None] * (eye + b[..., None, None] * outer)


def fftn3(f: np.ndarray) -> np.ndarray:
    """Unnormalised forward DFT (kernel exp(-i p.r)) of each component."""
    return sfft.fftn(f, axes=(-3, -2, -1), workers=_WORKERS)


def ifftn3(f: np.ndarray) -> np.ndarray:
    """Inverse DFT with the 1/N factor."""
    return sfft.ifftn(f, axes=(-3, -2, -1), workers=_WORKERS)


def green_factors(g: Grid, kt2: complex):
    """The mode-wise scalars of the Sherman-Morrison form of G^(p) on the
    broadcast grid: pt, a = 1 / (p^2 - kt2) and b = 1 / (p^2 - |pt|^2 - kt2).
    They depend on the grid and kt2 only, so a solve forms them once."""
    (pz, py, px), (ptz, pty, ptx) = fourier_grid(g)
    p2 = px * px + py * py + pz * pz
    pt2 = ptx * ptx + pty * pty + ptz * ptz
    a = 1.0 / (p2 - kt2)
    b = 1.0 / (p2 - pt2 - kt2)
    return (ptz, pty, ptx), a, b


def green_apply(g: Grid, W: np.ndarray, kt2: complex, factors=None) -> np.ndarray:
    """G W = F^-1 [G^(p) . F W]  for a vector field W [3, nz, ny, nx].

    Applies the 3x3 Sherman-Morrison tensor mode by mode (same formula as
    ``green_tensor``, written out on the broadcast grid).  factors is
    green_factors(g, kt2), formed here when not given."""
    (ptz, pty, ptx), a, b = factors if factors is not None else green_factors(g, kt2)
    Wh = fftn3(W)
    s = ptx * Wh[0] + pty * Wh[1] + ptz * Wh[2]      # pt . W^
    bs = b * s
    out = np.empty_like(Wh)
    out[0] = a * (Wh[0] + ptx * bs)
    out[1] = a * (Wh[1] + pty * bs)
    out[2] = a * (Wh[2] + ptz * bs)
    return ifftn3(out)


def curl_curl_apply(g: Grid, E: np.ndarray) -> np.ndarray:
    """L E = F^-1 M(p) F E (spectral curl-curl with the same Nyquist reading)."""
    (pz, py, px), (ptz, pty, ptx) = fourier_grid(g)
    p2 = px * px + py * py + pz * pz
    Eh = fftn3(E)
    s = ptx * Eh[0] + pty * Eh[1] + ptz * Eh[2]
    out = np.empty_like(Eh)
    out[0] = p2 * Eh[0] - ptx * s
    out[1] = p2 * Eh[1] - pty * s
    out[2] = p2 * Eh[2] - ptz * s
    return ifftn3(out)


# ---------------------------------------------------------------------------
# Sources (design paragraph: x-polarised plane wave, normal incidence;
# Fig. 2 caption and optimisation paragraph: adjoint source at r0)
# ---------------------------------------------------------------------------
def wave_vector(g: Grid, direction=(0.0, 0.0)):
    """(kx, ky, kz) of a plane wave travelling towards +z with transverse
    direction cosines direction = (kx/kb, ky/kb); (0, 0) is normal incidence."""
    sx, sy = (float(v) for v in direction)
    c2 = 1.0 - sx * sx - sy * sy
    if not c2 > 0.0:
        raise ValueError("direction cosines must satisfy sx^2 + sy^2 < 1")
    return g.kb * sx, g.kb * sy, g.kb * math.sqrt(c2)


def plane_wave(g: Grid, pol=(1.0, 0.0, 0.0), direction=(0.0, 0.0)) -> np.ndarray:
    """E_inc = pol * exp(i k.r), r = (i, j, k) d, phase 0 at the voxel (0, 0, 0),
    k from ``wave_vector`` (normal incidence: exp(i kb z) along +z)."""
    kx, ky, kz = wave_vector(g, direction)
    ph = (np.exp(1j * kz * np.arange(g.nz) * g.pitch)[:, None, None]
          * np.exp(1j * ky * np.arange(g.ny) * g.pitch)[None, :, None]
          * np.exp(1j * kx * np.arange(g.nx) * g.pitch)[None, None, :])
    E = np.zeros((3,) + g.vshape, dtype=np.complex128)
    for c in range(3):
        if pol[c] != 0:
            E[c] = complex(pol[c]) * ph
    return E


def plane_wave_source(g: Grid, eps_r: np.ndarray, pol=(1.0, 0.0, 0.0),
                      direction=(0.0, 0.0)) -> np.ndarray:
    """Scattered-field source S = k0^2 (eps_r - n_bg^2) E_inc."""
    contrast = g.k0 ** 2 * (np.asarray(eps_r).astype(np.complex128) - g.n_bg ** 2)
    return contrast[None] * plane_wave(g, pol, direction)


def box_mask(g: Grid, lo, hi) -> np.ndarray:
    """Indicator of the half-open voxel box [lo, hi) (x, y, z) over [nz, ny, nx]."""
    m = np.zeros(g.vshape, dtype=bool)
    m[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = True
    return m


def tfsf_source(g: Grid, lo, hi, pol=(1.0, 0.0, 0.0), direction=(0.0, 0.0)) -> np.ndarray:
    """Total-field / scattered-field source of a plane wave for the box [lo, hi):
    S = (L - K_bg)(chi E_inc),  K_bg = kb^2 + i kb^2 sigma,  chi the box indicator.

    In the background medium (L - K_bg) E = S is solved exactly by E = chi E_inc:
    the incident wave inside the box and nothing outside.  With material inside
    the box, E - chi E_inc solves the scattered-field problem, so the solution
    is the total field inside the box and the scattered field outside.  L is the
    same spectral curl-curl as the solver's operator (``curl_curl_apply``)."""
    U = box_mask(g, lo, hi)[None] * plane_wave(g, pol, direction)
    Kbg = g.kb ** 2 * (1.0 + 1j * absorber_sigma(g))
    return curl_curl_apply(g, U) - Kbg[None] * U


def point_source(g: Grid, r0, amp) -> np.ndarray:
    """Vector source amp (3 complex) at voxel r0 = (ix, iy, iz), zero elsewhere."""
    S = np.zeros((3,) + g.vshape, dtype=np.complex128)
    ix, iy, iz = r0
    S[:, iz, iy, ix] = np.asarray(amp, dtype=np.complex128)
    return S


# ---------------------------------------------------------------------------
# The CBS iteration
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class CBSResult:
    E_s: np.ndarray          # scattered field (or adjoint field) [3, nz, ny, nx]
    iterations: int          # number of updates applied
    eta: float               # last relative update norm
    eps: float               # shift used
    history: list            # eta per iteration


def cbs(g: Grid, eps_r: np.ndarray, S: np.ndarray, tol: float = 1e-6,
        max_iter: int = 20000, E0: np.ndarray | None = None,
        eps_shift: float | None = None) -> CBSResult:
    """Vector CBS (references [25], [26]) in FP64, step by step:

        W    = V E_s + S
        GW   = F^-1 G^ F W
        dE   = gamma (GW - E_s)
        E_s += dE
        eta  = ||dE|| / ||E_s||      stop when eta <= tol or k = max_iter
    """
    pot = potentials(g, eps_r, eps_shift)
    E = np.zeros((3,) + g.vshape, dtype=np.complex128) if E0 is None else np.array(E0, dtype=np.complex128)
    S = np.asarray(S, dtype=np.complex128)
    hist = []
    eta = float("inf")
    k = 0
    gf = green_factors(g, pot.kt2)
    for k in range(1, max_iter + 1):
        W = pot.V[None] * E + S
        GW = green_apply(g, W, pot.kt2, gf)
        dE = pot.gamma[None] * (GW - E)
        E = E + dE
        nd = math.sqrt(float(np.sum(dE.real ** 2 + dE.imag ** 2)))
        ne = math.sqrt(float(np.sum(E.real ** 2 + E.imag ** 2)))
        eta = nd / ne if ne > 0 else (0.0 if nd == 0 else float("inf"))
        hist.append(eta)
        if not math.isfinite(eta):
            raise FloatingPointError("CBS diverged (non-finite residual)")
        if eta <= tol:
            break
    return CBSResult(E_s=E, iterations=k, eta=eta, eps=pot.eps, history=hist)


def solve_forward(g: Grid, eps_r: np.ndarray, tol: float = 1e-6, max_iter: int = 20000,
                  pol=(1.0, 0.0, 0.0), eps_shift: float | None = None, direction=(0.0, 0.0)):
    """Total field E = E_inc + E_s for plane-wave illumination.

    Returns (E_total, CBSResult)."""
    validate(g, eps_r)
    S = plane_wave_source(g, eps_r, pol, direction)
    res = cbs(g, eps_r, S, tol, max_iter, eps_shift=eps_shift)
    return plane_wave(g, pol, direction) + res.E_s, res


# ---------------------------------------------------------------------------
# Objective, adjoint solve and gradient (Fig. 2 caption; optimisation paragraph)
# ---------------------------------------------------------------------------
def focal_objective(E: np.ndarray, r0) -> float:
    """L = |E(r0)|^2 = sum_c |E_c(r0)|^2 at voxel r0 = (ix, iy, iz)."""
    ix, iy, iz = r0
    v = E[:, iz, iy, ix]
    return float(np.sum(np.abs(v) ** 2))


def adjoint_point_source(g: Grid, E: np.ndarray, r0) -> np.ndarray:
    """g = conj(E(r0)) delta_{r0}: the source whose solution E_adj = A^-1 g
    turns dL = 2 Re(conj(E(r0))^T dE(r0)) into a voxel-local product
    (A is complex-symmetric, so g^T A^-1 = (A^-1 g)^T)."""
    ix, iy, iz = r0
    return point_source(g, r0, np.conj(E[:, iz, iy, ix]))


def solve_adjoint(g: Grid, eps_r: np.ndarray, src: np.ndarray, tol: float = 1e-6,
                  max_iter: int = 20000, eps_shift: float | None = None) -> CBSResult:
    """E_adj = A^-1 src with the same operator and iteration (A^T = A)."""
    validate(g, eps_r)
    return cbs(g, eps_r, src, tol, max_iter, eps_shift=eps_shift)


def gradient(g: Grid, E: np.ndarray, E_adj: np.ndarray, box_lo=None, box_hi=None,
             scale: float = 2.0) -> np.ndarray:
    """dL/d eps_r(r) = scale * k0^2 * Re(sum_c E_adj,c(r) E_c(r)) over a box.

    scale = 2 with the adjoint source conj(E(r0)) gives the gradient of
    L = |E(r0)|^2 (perturbing eps_r by h changes K and S by k0^2 h, so
    A dE = k0^2 h E with E the total field).  box_lo/box_hi are (x, y, z),
    half-open; the result is [z, y, x] over the box."""
    if box_lo is None:
        box_lo = (0, 0, 0)
    if box_hi is None:
        box_hi = (g.nx, g.ny, g.nz)
    x0, y0, z0 = box_lo
    x1, y1, z1 = box_hi
    sl = (slice(None), slice(z0, z1), slice(y0, y1), slice(x0, x1))
    prod = np.sum(E_adj[sl] * E[sl], axis=0)
    return scale * g.k0 ** 2 * prod.real


def objective_of_eps(g: Grid, eps_r: np.ndarray, r0, tol: float, max_iter: int,
                     E0_s: np.ndarray | None = None):
    """L(eps_r) and the scattered field, used by finite-difference pins."""
    S = plane_wave_source(g, eps_r)
    res = cbs(g, eps_r, S, tol, max_iter, E0=E0_s)
    E = plane_wave(g) + res.E_s
    return focal_objective(E, r0), res
