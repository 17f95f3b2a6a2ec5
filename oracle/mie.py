"""Mie series for a homogeneous sphere in a plane wave.  TEST INFRASTRUCTURE ONLY.

The continuum closed form against which the discrete CBS field of a dielectric
sphere is compared (the check the method's validation names for a sphere; the
paper's benchmark scene of its setup paragraph is a sphere of this kind).
Written from the textbook expansion of Bohren and Huffman, "Absorption and
Scattering of Light by Small Particles" (Wiley, 1983), chapter 4, in their
conventions, which match the solver's: time dependence exp(-i w t), incident
field E0 x^ exp(i k z) travelling along +z, outgoing waves exp(+i k r).

    incident   E_i = sum_n E_n (M^(1)_o1n - i N^(1)_e1n)
    scattered  E_s = sum_n E_n (i a_n N^(3)_e1n - b_n M^(3)_o1n)
    E_n = i^n E0 (2n + 1) / (n (n + 1))

M and N are the vector spherical harmonics built from the radial function z_n
(spherical Bessel j_n for (1), spherical Hankel h_n^(1) = j_n + i y_n for (3))
and the angular functions pi_n = P_n^1(cos t) / sin t, tau_n = d P_n^1 / d t
from their upward recurrences.  The coefficients a_n, b_n follow from the
Riccati-Bessel functions psi_n(r) = r j_n(r), xi_n(r) = r h_n^(1)(r) with
relative index m and size parameter x = k a; the series is cut after
n_max = x + 4 x^(1/3) + 2 terms (Wiscombe's criterion).

Pinned by: the (1) expansion reproducing the plane wave itself, extinction
equal to scattering for a lossless sphere (optical theorem), the Rayleigh
limit of a_1, and the book's sample calculation (m = 1.55, x = 5.213).
"""

from __future__ import annotations

import math

import numpy as np
from scipy import special


def n_terms(x: float) -> int:
    """Series length for size parameter x (Wiscombe's criterion)."""
    return int(round(x + 4.0 * x ** (1.0 / 3.0) + 2.0))


def _psi(n, r, derivative=False):
    """Riccati-Bessel psi_n(r) = r j_n(r) (or its derivative)."""
    j = special.spherical_jn(n, r)
    if not derivative:
        return r * j
    return j + r * special.spherical_jn(n, r, derivative=True)


def _xi(n, r, derivative=False):
    """Riccati-Bessel xi_n(r) = r h_n^(1)(r) (or its derivative), real r."""
    j = special.spherical_jn(n, r)
    y = special.spherical_yn(n, r)
    if not derivative:
        return r * (j + 1j * y)
    jd = special.spherical_jn(n, r, derivative=True)
    yd = special.spherical_yn(n, r, derivative=True)
    return (j + 1j * y) + r * (jd + 1j * yd)


def coefficients(m: complex, x: float, nmax: int | None = None):
    """Scattering coefficients a_n, b_n, n = 1..nmax (non-magnetic sphere)."""
    if nmax is None:
        nmax = n_terms(x)
    n = np.arange(1, nmax + 1)
    mx = m * x
    pm, pmd = _psi(n, mx), _psi(n, mx, True)
    px, pxd = _psi(n, x), _psi(n, x, True)
    xx, xxd = _xi(n, x), _xi(n, x, True)
    a = (m * pm * pxd - px * pmd) / (m * pm * xxd - xx * pmd)
    b = (pm * pxd - m * px * pmd) / (pm * xxd - m * xx * pmd)
    return a, b


def efficiencies(m: complex, x: float):
    """(Q_ext, Q_sca, Q_back) from the coefficients."""
    a, b = coefficients(m, x)
    n = np.arange(1, a.size + 1)
    qext = 2.0 / x ** 2 * float(np.sum((2 * n + 1) * (a + b).real))
    qsca = 2.0 / x ** 2 * float(np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2)))
    qback = float(np.abs(np.sum((2 * n + 1) * (-1.0) ** n * (a - b))) ** 2) / x ** 2
    return qext, qsca, qback


def _angular(nmax: int, mu: np.ndarray):
    """pi_n(mu), tau_n(mu) for n = 1..nmax; arrays [nmax, ...]."""
    pi = np.zeros((nmax + 1,) + mu.shape)
    tau = np.zeros((nmax + 1,) + mu.shape)
    pi[1] = 1.0
    tau[1] = mu
    for n in range(2, nmax + 1):
        pi[n] = (2 * n - 1) / (n - 1) * mu * pi[n - 1] - n / (n - 1) * pi[n - 2]
        tau[n] = n * mu * pi[n] - (n + 1) * pi[n - 1]
    return pi[1:], tau[1:]


def _harmonics(nmax, rho, mu, phi, kind):
    """Cartesian components of M_o1n and N_e1n, n = 1..nmax, at the points.

    kind 1: z_n = j_n; kind 3: z_n = h_n^(1).  Returns (M, N) as complex
    arrays [nmax, 3, npts]."""
    n = np.arange(1, nmax + 1)[:, None]
    if kind == 1:
        z = special.spherical_jn(n, rho[None])
        zm1 = special.spherical_jn(n - 1, rho[None])
    else:
        z = special.spherical_jn(n, rho[None]) + 1j * special.spherical_yn(n, rho[None])
        zm1 = (special.spherical_jn(n - 1, rho[None])
               + 1j * special.spherical_yn(n - 1, rho[None]))
    dz = (rho[None] * zm1 - n * z) / rho[None]          # [rho z_n]' / rho
    pi, tau = _angular(nmax, mu)
    st = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    cp, sp = np.cos(phi), np.sin(phi)
    # spherical unit vectors in Cartesian components
    er = np.stack([st * cp, st * sp, mu])
    et = np.stack([mu * cp, mu * sp, -st])
    ef = np.stack([-sp, cp, np.zeros_like(cp)])
    # M_o1n = cos(phi) pi z e_t - sin(phi) tau z e_f
    M = (cp * pi * z)[:, None] * et[None] - (sp * tau * z)[:, None] * ef[None]
    # N_e1n = cos(phi) n(n+1) sin(t) pi z/rho e_r + cos(phi) tau dz e_t - sin(phi) pi dz e_f
    N = ((cp * n * (n + 1) * st * pi * z / rho[None])[:, None] * er[None]
         + (cp * tau * dz)[:, None] * et[None]
         - (sp * pi * dz)[:, None] * ef[None])
    return M, N


def _spherical(points, center):
    d = np.asarray(points, dtype=np.float64) - np.asarray(center, dtype=np.float64)[:, None]
    r = np.sqrt(np.sum(d * d, axis=0))
    mu = np.where(r > 0, d[2] / np.where(r > 0, r, 1.0), 1.0)
    phi = np.arctan2(d[1], d[0])
    return r, mu, phi


def incident_expansion(k: float, points, center, nmax: int):
    """x^ exp(i k (z - z_c)) from its (1) expansion, truncated at nmax: [3, npts]."""
    r, mu, phi = _spherical(points, center)
    M, N = _harmonics(nmax, k * r, mu, phi, 1)
    n = np.arange(1, nmax + 1)
    En = (1j ** n) * (2 * n + 1) / (n * (n + 1))
    return np.einsum("n,nck->ck", En, M - 1j * N)


def scattered_field(k: float, radius: float, m: complex, points, center, E0: complex = 1.0):
    """Scattered field E_s at points outside the sphere: [3, npts] complex.

    points [3, npts] (x, y, z) in metres, center (x, y, z); the incident wave
    is E0 x^ exp(i k (z - z_c)), i.e. phase zero at the sphere centre."""
    r, mu, phi = _spherical(points, center)
    if np.any(r <= radius):
        raise ValueError("scattered_field is evaluated outside the sphere only")
    x = k * radius
    a, b = coefficients(m, x)
    nmax = a.size
    M, N = _harmonics(nmax, k * r, mu, phi, 3)
    n = np.arange(1, nmax + 1)
    En = E0 * (1j ** n) * (2 * n + 1) / (n * (n + 1))
    return np.einsum("n,nck->ck", En * 1j * a, N) - np.einsum("n,nck->ck", En * b, M)
