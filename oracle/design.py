"""Thickness-map lens design: eps_r(h) and the chain rule dL/dh.  TEST INFRASTRUCTURE ONLY.

Optimisation paragraph (Fig. 2a): the design variable is the lens thickness
map h(x, y); mirror symmetry h(x, y) = h(+-x, +-y) is imposed, optionally a
Gaussian smoothing of standard deviation 355 nm, then the profile becomes the
3D shape function of the lens (n = 1.54) and CBS gives E, the figure of merit
L = |E(r0)|^2 and, through one adjoint solve, dL/d eps_r; dL/dh follows by the
chain rule.  Readings where the paper is silent:

R1  symmetry: the mean of the four mirror images about the lateral centre
    ((n - 1) / 2), i.e. the orthogonal projection onto mirror-symmetric maps;
R2  smoothing: 2D convolution with the normalised Gaussian of standard
    deviation sigma = 355 nm / d voxels, truncated at 4 sigma, zero outside
    the grid;
R3  aperture: h is zero outside the lens diameter D and outside the lateral
    interior (eps_r must equal n_bg^2 in the absorbing layer);
R4  shape function (printed garbled; read Theta(h - (z - z_b))) with the
    subpixel axial fill of the lens conventions: voxel z holds
    fill = clip(h - (z - z_b), 0, 1) and eps_r = n_bg^2 + fill (n^2 - n_bg^2);
    its derivative is taken one-sided from above, d fill / dh = 1 on
    0 <= h - (z - z_b) < 1, so a zero thickness can grow;
R5  units: h in voxel pitches; the Adam step size 0.3 is in those units and h
    is clipped to [0, h_max] after every step.

The map p -> h is linear (projection, convolution, mask), so its adjoint is
written out: mask, correlation with the same kernel, projection.
"""

from __future__ import annotations

import math

import numpy as np
from scipy import signal


def symmetrize(p: np.ndarray) -> np.ndarray:
    """R1: mean of p and its mirror images in x, y and both."""
    return 0.25 * (p + p[:, ::-1] + p[::-1, :] + p[::-1, ::-1])


def gaussian_kernel(sigma: float) -> np.ndarray:
    """R2: normalised 2D Gaussian, truncated at 4 sigma."""
    r = int(math.ceil(4.0 * sigma))
    x = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-x * x / (2.0 * sigma * sigma))
    g /= g.sum()
    return np.outer(g, g)


def smooth(h: np.ndarray, sigma: float) -> np.ndarray:
    return signal.convolve2d(h, gaussian_kernel(sigma), mode="same", boundary="fill", fillvalue=0.0)


def smooth_adjoint(g: np.ndarray, sigma: float) -> np.ndarray:
    """Adjoint of `smooth`: correlation with the same kernel (zero fill)."""
    return signal.correlate2d(g, gaussian_kernel(sigma), mode="same", boundary="fill", fillvalue=0.0)


def thickness(p: np.ndarray, d, smoothing: bool = True) -> np.ndarray:
    """h = aperture * smooth(symmetrize(p)) (voxels) for a scenes.LensDesign d."""
    h = symmetrize(np.asarray(p, dtype=np.float64))
    if smoothing:
        h = smooth(h, d.sigma_vox)
    return h * d.aperture


def fill(h: np.ndarray, d) -> np.ndarray:
    """R4: axial fill of the slab voxels z in [z0, z1): [z1 - z0, ny, nx]."""
    z0, z1 = d.slab
    dz = (np.arange(z0, z1) - d.z_base).astype(np.float64)
    return np.clip(h[None] - dz[:, None, None], 0.0, 1.0)


def eps_of(p: np.ndarray, d, smoothing: bool = True) -> np.ndarray:
    """eps_r [nz, ny, nx] of the design p."""
    nx, ny, nz = d.shape
    eps = np.full((nz, ny, nx), d.n_bg ** 2, dtype=np.float64)
    z0, z1 = d.slab
    eps[z0:z1] += fill(thickness(p, d, smoothing), d) * (d.n_lens ** 2 - d.n_bg ** 2)
    return eps


def grad_p(grad_eps_slab: np.ndarray, p: np.ndarray, d, smoothing: bool = True) -> np.ndarray:
    """dL/dp from dL/d eps_r over the slab voxels [z1 - z0, ny, nx] (FP64 z-sum)."""
    h = thickness(p, d, smoothing)
    z0, z1 = d.slab
    dz = (np.arange(z0, z1) - d.z_base).astype(np.float64)
    u = h[None] - dz[:, None, None]
    dfill = ((u >= 0.0) & (u < 1.0)).astype(np.float64)
    gh = (d.n_lens ** 2 - d.n_bg ** 2) * np.sum(np.asarray(grad_eps_slab, np.float64) * dfill, axis=0)
    gh = gh * d.aperture
    if smoothing:
        gh = smooth_adjoint(gh, d.sigma_vox)
    return symmetrize(gh)


def adam_step(p, g, m, v, t, lr=0.3, b1=0.9, b2=0.999, eps=1e-6, h_max=None):
    """One Adam ascent step on the figure of merit (Adam paragraph: step 0.3,
    decay rates 0.9 / 0.999, 1e-6), t counted from 1; returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    p = p + lr * mh / (np.sqrt(vh) + eps)
    if h_max is not None:
        p = np.clip(p, 0.0, h_max)
    return p, m, v
