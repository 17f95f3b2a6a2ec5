"""Lens figures of a field: focus, FWHM, focusing efficiency.  TEST INFRASTRUCTURE ONLY.

Focusing-efficiency paragraph: eta_f is the power inside a disc of diameter
three times the lateral full width at half maximum at the focal plane, divided
by the incident power (after the paper's reference [18]).  Readings (the paper
and the solver fix no more):

*  the intensity that locates the focus and sets the widths is |E|^2 summed
   over the three components;
*  the focal point is the voxel of maximum |E|^2 inside a search box (ties:
   the smaller linear index z, y, x);
*  widths come from the profiles along x and y in the focal plane and along z
   through the focus, with the half-maximum crossings interpolated linearly
   between voxel centres; the lateral FWHM is the mean of the x and y widths;
*  the power through the disc (centred on the focal voxel, voxel centres within
   the radius) is the flux of the Poynting vector S_z = Re(Ex conj(Hy) -
   Ey conj(Hx)) of the focal plane's propagating angular spectrum: per plane
   wave (kx, ky, kz = sqrt(k^2 - kx^2 - ky^2)) Ez follows from k . E = 0 and
   H = k x E / k (units where a plane wave carries |E|^2); evanescent
   components carry no flux and are dropped;
*  the incident power is |e0|^2 pi (D/2)^2, a plane wave of amplitude e0 on
   the lens aperture D in the same medium.
"""

from __future__ import annotations

import math

import numpy as np


def intensity(E: np.ndarray) -> np.ndarray:
    """|E|^2 summed over components, [nz, ny, nx] in FP64."""
    E = np.asarray(E)
    return np.sum(E.real.astype(np.float64) ** 2 + E.imag.astype(np.float64) ** 2, axis=0)


def focus(I: np.ndarray, lo, hi):
    """(x, y, z) of the maximum of I inside [lo, hi) (first in z, y, x order)."""
    sub = I[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
    k = int(np.argmax(sub))
    z, y, x = np.unravel_index(k, sub.shape)
    return (lo[0] + int(x), lo[1] + int(y), lo[2] + int(z))


def fwhm(v: np.ndarray, i0: int, pitch: float) -> float:
    """Width at half of v[i0] around i0 with linear interpolation; NaN if the
    profile does not drop below half on both sides."""
    half = 0.5 * v[i0]
    left = None
    for i in range(i0, 0, -1):
        if v[i - 1] < half:
            left = (i - 1) + (half - v[i - 1]) / (v[i] - v[i - 1])
            break
    right = None
    for i in range(i0, len(v) - 1):
        if v[i + 1] < half:
            right = i + (v[i] - half) / (v[i] - v[i + 1])
            break
    if left is None or right is None:
        return math.nan
    return (right - left) * pitch


def plane_flux(Ex: np.ndarray, Ey: np.ndarray, pitch: float, k: float) -> np.ndarray:
    """S_z [ny, nx] of the propagating angular spectrum of (Ex, Ey) in a plane."""
    ny, nx = Ex.shape
    kx = 2 * math.pi * np.fft.fftfreq(nx, pitch)[None, :]
    ky = 2 * math.pi * np.fft.fftfreq(ny, pitch)[:, None]
    kz2 = k * k - kx * kx - ky * ky
    prop = kz2 > 0
    kz = np.sqrt(np.where(prop, kz2, 1.0))
    ax = np.fft.fft2(Ex) * prop
    ay = np.fft.fft2(Ey) * prop
    az = -(kx * ax + ky * ay) / kz
    hx = np.fft.ifft2((ky * az - kz * ay) / k)
    hy = np.fft.ifft2((kz * ax - kx * az) / k)
    ex, ey = np.fft.ifft2(ax), np.fft.ifft2(ay)
    return np.real(ex * np.conj(hy) - ey * np.conj(hx))


def lens_figures(E: np.ndarray, pitch: float, lo, hi, aperture: float, k: float,
                 disc_factor: float = 3.0, e0: float = 1.0) -> dict:
    """Focus, FWHM (x, y, z) and eta_f of a field E [3, nz, ny, nx]; k is the
    background wavenumber 2 pi n_bg / lambda0."""
    I = intensity(E)
    fx, fy, fz = focus(I, lo, hi)
    w = (fwhm(I[fz, fy, :], fx, pitch), fwhm(I[fz, :, fx], fy, pitch), fwhm(I[:, fy, fx], fz, pitch))
    out = {"focus": (fx, fy, fz), "peak": float(I[fz, fy, fx]), "fwhm": w,
           "disc_flux": math.nan, "eta_f": math.nan}
    if math.isfinite(w[0]) and math.isfinite(w[1]):
        r = 0.5 * disc_factor * 0.5 * (w[0] + w[1]) / pitch
        ny, nx = I.shape[1:]
        yy, xx = np.meshgrid(np.arange(ny) - fy, np.arange(nx) - fx, indexing="ij")
        disc = (xx * xx + yy * yy) <= r * r
        Sz = plane_flux(np.asarray(E[0, fz], np.complex128), np.asarray(E[1, fz], np.complex128),
                        pitch, k)
        out["disc_flux"] = float(np.sum(Sz[disc])) * pitch * pitch
        out["eta_f"] = out["disc_flux"] / (e0 * e0 * math.pi * (aperture / 2.0) ** 2)
    return out
