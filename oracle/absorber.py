"""Reflection of the absorbing layer.  TEST INFRASTRUCTURE ONLY.

The paper surrounds its CBS volume with an absorbing layer of thickness
[lambda, lambda, 6 lambda] (simulation-setup paragraph, reference [31]) but
states neither its profile nor how well it absorbs.  The layer used here is
the graded imaginary potential of ``cbs.absorber_sigma``; these functions
measure how much of a plane wave it reflects, so the profile can be chosen
and its reflection reported.

Method.  A source sheet in the homogeneous interior launches plane waves of
transverse wavenumber kt towards the layer of one axis (the "normal" axis).
Between the sheet and the layer the field along that axis is, up to the
spectral operator's small non-locality, a e^{i kn s} + b e^{-i kn s} with
kn = sqrt(kb^2 - kt^2): the outgoing wave and the wave the layer sends back.
A least-squares fit of a and b over a window well inside the interior gives
the amplitude reflection |b / a| (the far layer's reflection of the backward
wave re-enters as part of a, not of b).  R = |b / a|^2.

reflection_normal
    Normal incidence from the exact 1D reduction (``closed.slab_1d``): a field
    uniform in the transverse plane reduces the vector problem to the scalar
    1D spectral Helmholtz equation along the normal axis.
reflection_oblique
    Oblique incidence on the z layer from the full 3D FP64 CBS solve on a grid
    periodic in x and y (no layer there), driven by a current sheet
    J e^{i kx x} at one z: one transverse Fourier mode, so the field is that
    mode times a function of z.  Polarisation 's' drives E_y, 'p' drives E_x
    (field in the plane of incidence); the fit uses that component.
fit_counterpropagating
    The least-squares split itself, pinned against Fresnel reflection at an
    index step (tests).
"""

from __future__ import annotations

import math

import numpy as np

from . import cbs as _cbs
from . import closed as _closed


def fit_counterpropagating(f: np.ndarray, s: np.ndarray, kn: float):
    """(a, b, relative residual) of f(s) ~ a e^{i kn s} + b e^{-i kn s}."""
    A = np.stack([np.exp(1j * kn * s), np.exp(-1j * kn * s)], axis=1)
    c, *_ = np.linalg.lstsq(A, f, rcond=None)
    res = float(np.linalg.norm(A @ c - f) / np.linalg.norm(f))
    return complex(c[0]), complex(c[1]), res


def fit_window(n: int, pml: int, src: int, margin_src: int = 12, margin_layer: int = 6):
    """Window (lo, hi) of grid indices between the sheet and the far layer."""
    lo, hi = src + margin_src, n - pml - margin_layer
    if hi - lo < 16:
        raise ValueError("interior too short for a reflection fit")
    return lo, hi


def reflection_normal(n: int, pitch: float, lambda0: float, pml: int, order: int = 2,
                      sigma_max: float = 1.0, n_bg: float = 1.0, eps_profile=None):
    """R at normal incidence on a layer of `pml` voxels along an axis of n voxels.

    eps_profile (optional, length n) replaces the homogeneous background, e.g.
    an index step for the Fresnel pin; the sheet sits 6 voxels inside the
    near layer.  Returns (R, fit residual)."""
    k = 2.0 * math.pi * n_bg / lambda0
    eps = np.full(n, n_bg ** 2, dtype=np.complex128) if eps_profile is None else \
        np.asarray(eps_profile, dtype=np.complex128)
    src = pml + 6
    s = np.zeros(n, dtype=np.complex128)
    s[src] = 1.0
    e = _closed.slab_1d(n, pitch, lambda0, n_bg, pml, eps, s, order, sigma_max)
    lo, hi = fit_window(n, pml, src)
    z = np.arange(n) * pitch
    a, b, res = fit_counterpropagating(e[lo:hi], z[lo:hi], k)
    return abs(b / a) ** 2, res


def oblique_mode(g: _cbs.Grid, mx: int):
    """kx of FFT index mx along x and the matching kz in the background."""
    kx = 2.0 * math.pi * mx / (g.nx * g.pitch)
    kz2 = g.kb ** 2 - kx ** 2
    if kz2 <= 0:
        raise ValueError("evanescent mode")
    return kx, math.sqrt(kz2)


def oblique_source(g: _cbs.Grid, mx: int, pol: str, z_src: int, amp: float = 1.0):
    """Current sheet amp e^{i kx x} at z = z_src: component y ('s') or x ('p')."""
    kx, _ = oblique_mode(g, mx)
    x = np.arange(g.nx) * g.pitch
    S = np.zeros((3,) + g.vshape, dtype=np.complex128)
    c = 1 if pol == "s" else 0
    S[c, z_src] = amp * np.exp(1j * kx * x)[None, :]
    return S


def reflection_from_field(g: _cbs.Grid, E: np.ndarray, mx: int, pol: str, z_src: int):
    """R from a solved field of ``oblique_source``: the fit of the driven
    component's x-mode amplitude along z."""
    kx, kz = oblique_mode(g, mx)
    c = 1 if pol == "s" else 0
    x = np.arange(g.nx) * g.pitch
    # project every z plane on the driven transverse mode (uniform in y)
    f = np.einsum("zyx,x->z", E[c], np.exp(-1j * kx * x)) / (g.nx * g.ny)
    lo, hi = fit_window(g.nz, g.pml[2], z_src)
    z = np.arange(g.nz) * g.pitch
    a, b, res = fit_counterpropagating(f[lo:hi], z[lo:hi], kz)
    return abs(b / a) ** 2, res


def reflection_oblique(g: _cbs.Grid, mx: int, pol: str, tol: float = 1e-10):
    """R of the z layer for the plane waves of transverse index mx (angle
    asin(kx / kb)) from the FP64 CBS solve; g must have no x or y layer.
    Returns (R, fit residual, angle in degrees)."""
    if g.pml[0] or g.pml[1]:
        raise ValueError("the oblique measurement needs a grid periodic in x and y")
    z_src = g.pml[2] + 6
    S = oblique_source(g, mx, pol, z_src, amp=g.k0 ** 2)
    eps = np.full(g.vshape, g.n_bg ** 2, dtype=np.float64)
    res = _cbs.cbs(g, eps, S, tol=tol, max_iter=200000)
    R, fr = reflection_from_field(g, res.E_s, mx, pol, z_src)
    kx, _ = oblique_mode(g, mx)
    return R, fr, math.degrees(math.asin(kx / g.kb))
