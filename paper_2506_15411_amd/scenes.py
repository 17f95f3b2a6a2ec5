"""Seeded synthetic scenes: permittivity volumes, focal voxels and random fields.

This module is the only code shared by the HIP path and the FP64 oracle.  It
holds geometry and random-number generation only -- none of the solver's
arithmetic (no potentials, absorbing profile, Green's tensor or iteration).

Geometry follows the paper (arXiv 2506.15411):
  * wavelength 1064 nm, background index 1, lens index 1.45 in the workloads
    used here (the design paragraph uses 1.54 for the polymerised resist);
  * focal point r0 = (0, 0, f_eff) with asin(NA) = atan(D / (2 f_eff))
    (Fig. 2 caption, objective paragraph);
  * subpixel averaging of the permittivity at material boundaries
    (simulation-setup paragraph, reference [30]) -- here the isotropic
    volume-fraction variant eps = n_bg^2 + f (n^2 - n_bg^2);
  * absorbing layer [lambda, lambda, 6 lambda] read as the total per axis,
    split evenly over the two sides and rounded to whole voxels with a lateral
    floor of 8 voxels.

Arrays are [nz, ny, nx] float32 (x fastest); vector fields [3, nz, ny, nx]
complex64.  Voxel (i, j, k) is centred at (i d, j d, k d).
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

LAMBDA0 = 1.064e-6


@dataclasses.dataclass
class Scene:
    """A complete solver input: grid, absorbing layer, permittivity, focus."""

    name: str
    shape: tuple              # (nx, ny, nz)
    pitch: float              # metres
    pml: tuple                # per-side voxels (px, py, pz)
    eps_r: np.ndarray         # [nz, ny, nx] float32
    lambda0: float = LAMBDA0
    n_bg: float = 1.0
    r0: tuple | None = None   # focal voxel (ix, iy, iz)
    design_box: tuple | None = None   # ((x0, y0, z0), (x1, y1, z1)) half-open
    info: dict = dataclasses.field(default_factory=dict)

    @property
    def n_vox(self) -> int:
        nx, ny, nz = self.shape
        return nx * ny * nz


def pml_voxels(pitch: float, lambda0: float = LAMBDA0, lateral_floor: int = 8):
    """Per-side layer thickness for [lambda, lambda, 6 lambda] total per axis."""
    lat = max(lateral_floor, int(round(0.5 * lambda0 / pitch)))
    ax = int(round(3.0 * lambda0 / pitch))
    return (lat, lat, ax)


def focal_length(D: float, NA: float) -> float:
    """f_eff from asin(NA) = atan(D / (2 f_eff))  (Fig. 2 caption)."""
    return D / (2.0 * math.tan(math.asin(NA)))


# ---------------------------------------------------------------------------
# Sphere (plain CBS benchmark at 64^3)
# ---------------------------------------------------------------------------
def sphere_fraction(shape, pitch, radius, center=None, supersample: int = 8) -> np.ndarray:
    """Volume fraction of a sphere in each voxel by supersample^3 point tests.

    Voxels whose centre is farther than sqrt(3)/2 d from the surface are
    classified from the centre alone; the rest are supersampled at offsets
    ((s + 1/2)/S - 1/2) d."""
    nx, ny, nz = shape
    if center is None:
        center = ((nx - 1) / 2 * pitch, (ny - 1) / 2 * pitch, (nz - 1) / 2 * pitch)
    cx, cy, cz = center
    z = np.arange(nz)[:, None, None] * pitch - cz
    y = np.arange(ny)[None, :, None] * pitch - cy
    x = np.arange(nx)[None, None, :] * pitch - cx
    r = np.sqrt(x * x + y * y + z * z)
    frac = (r <= radius).astype(np.float64)
    band = np.abs(r - radius) <= 0.5 * math.sqrt(3.0) * pitch + 1e-15
    kz, ky, kx = np.nonzero(band)
    if kz.size:
        off = ((np.arange(supersample) + 0.5) / supersample - 0.5) * pitch
        ox, oy, oz = np.meshgrid(off, off, off, indexing="ij")
        ox, oy, oz = ox.ravel(), oy.ravel(), oz.ravel()
        xs = (kx * pitch - cx)[:, None] + ox[None]
        ys = (ky * pitch - cy)[:, None] + oy[None]
        zs = (kz * pitch - cz)[:, None] + oz[None]
        inside = (xs * xs + ys * ys + zs * zs) <= radius * radius
        frac[kz, ky, kx] = inside.mean(axis=1)
    return frac


def sphere_scene(n: int = 64, pitch: float = LAMBDA0 / 6, radius: float = 1.2e-6,
                 n_sphere: float = 1.45, n_bg: float = 1.0, pml=(8, 8, 16),
                 supersample: int = 8, name: str = "sphere64") -> Scene:
    """Dielectric sphere centred at ((n-1)/2) d on each axis."""
    shape = (n, n, n) if isinstance(n, int) else tuple(n)
    f = sphere_fraction(shape, pitch, radius, supersample=supersample)
    eps = (n_bg ** 2 + f * (n_sphere ** 2 - n_bg ** 2)).astype(np.float32)
    _clear_layer(eps, pml, n_bg)
    return Scene(name=name, shape=shape, pitch=pitch, pml=tuple(pml), eps_r=eps, n_bg=n_bg,
                 info=dict(radius=radius, n_sphere=n_sphere))


# ---------------------------------------------------------------------------
# Binary zone plate (Fresnel zone-plate lens; configs at 16 um and 100 um)
# ---------------------------------------------------------------------------
def zone_radii(D: float, f: float, lambda0: float = LAMBDA0):
    """Zone boundaries r_m = sqrt(m lambda f + (m lambda / 2)^2) inside D/2."""
    out = []
    m = 1
    while True:
        r = math.sqrt(m * lambda0 * f + (m * lambda0 / 2.0) ** 2)
        if r >= D / 2.0:
            break
        out.append(r)
        m += 1
    return out


def _clear_layer(eps: np.ndarray, pml, n_bg: float) -> None:
    """Force eps_r = n_bg^2 (at float32) inside the absorbing layer."""
    px, py, pz = pml
    nb2 = np.float32(n_bg * n_bg)
    nz, ny, nx = eps.shape
    if pz:
        eps[:pz] = nb2
        eps[nz - pz:] = nb2
    if py:
        eps[:, :py] = nb2
        eps[:, ny - py:] = nb2
    if px:
        eps[:, :, :px] = nb2
        eps[:, :, nx - px:] = nb2


def zone_plate_scene(shape, pitch, D: float, NA: float = 0.84, n_lens: float = 1.45,
                     n_bg: float = 1.0, lambda0: float = LAMBDA0, pml=None,
                     supersample: int = 8, name: str = "zoneplate") -> Scene:
    """Free-standing binary zone plate, centre disc filled, alternating zones.

    Thickness t = lambda0 / (2 (n - 1)) (a pi phase step).  The lower face
    sits on the lower face of voxel z_b = pz + ceil(lambda0 / (2 d)).  The
    lateral fill fraction comes from supersample^2 point tests per voxel and
    the axial one from the exact overlap of each voxel with [z_lo, z_lo + t].
    The focal voxel is r0 = (floor((nx-1)/2), floor((ny-1)/2),
    round((z_lo + t + f_eff) / d)) in voxel-centre coordinates."""
    nx, ny, nz = shape
    if pml is None:
        pml = pml_voxels(pitch, lambda0)
    f = focal_length(D, NA)
    t = lambda0 / (2.0 * (n_lens - 1.0))
    radii = zone_radii(D, f, lambda0)
    bounds = [0.0] + radii + [D / 2.0]
    cx = (nx - 1) / 2.0 * pitch
    cy = (ny - 1) / 2.0 * pitch
    off = ((np.arange(supersample) + 0.5) / supersample - 0.5) * pitch
    ys = (np.arange(ny) * pitch - cy)[:, None] + off[None, :]          # [ny, S]
    xs = (np.arange(nx) * pitch - cx)[:, None] + off[None, :]          # [nx, S]
    r = np.sqrt(ys[:, None, :, None] ** 2 + xs[None, :, None, :] ** 2)  # [ny, nx, S, S]
    zone = np.searchsorted(np.asarray(bounds), r, side="right") - 1     # zone index
    filled = (zone % 2 == 0) & (r < D / 2.0)
    lat = filled.reshape(ny, nx, -1).mean(axis=2)
    z_b = pml[2] + int(math.ceil(lambda0 / (2.0 * pitch)))
    z_lo = (z_b - 0.5) * pitch
    z_hi = z_lo + t
    kz = np.arange(nz)
    ax = np.clip(np.minimum((kz + 0.5) * pitch, z_hi) - np.maximum((kz - 0.5) * pitch, z_lo),
                 0.0, None) / pitch
    frac = ax[:, None, None] * lat[None, :, :]
    eps = (n_bg ** 2 + frac * (n_lens ** 2 - n_bg ** 2)).astype(np.float32)
    _clear_layer(eps, pml, n_bg)
    r0 = ((nx - 1) // 2, (ny - 1) // 2, int(math.floor((z_hi + f) / pitch + 0.5)))
    return Scene(name=name, shape=tuple(shape), pitch=pitch, pml=tuple(pml), eps_r=eps,
                 lambda0=lambda0, n_bg=n_bg, r0=r0,
                 info=dict(D=D, NA=NA, n_lens=n_lens, f_eff=f, thickness=t, z_base=z_b,
                           zones=len(radii)))


# ---------------------------------------------------------------------------
# Thickness-map lens design (optimisation paragraph, Fig. 2a)
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class LensDesign:
    """Inputs of the thickness-map inverse design: the grid, where the lens
    sits, the starting thickness map and the focus.  Thicknesses are in units
    of the voxel pitch d; the lens occupies z in [z_lo, z_lo + h(x, y) d] with
    z_lo = (z_base - 1/2) d (the lower face of voxel z_base)."""

    name: str
    shape: tuple              # (nx, ny, nz)
    pitch: float
    pml: tuple
    z_base: int
    h_max: float              # thickness bound (voxels): one 2 pi wrap, lambda0 / (n - n_bg)
    n_lens: float
    n_bg: float
    D: float
    NA: float
    f_eff: float
    r0: tuple                 # focal voxel (x, y, z)
    aperture: np.ndarray      # [ny, nx] float32, 1 inside D/2 and the lateral interior
    h_init: np.ndarray        # [ny, nx] float64, kinoform start (voxels)
    sigma_vox: float          # Gaussian smoothing width (voxels)
    lambda0: float = LAMBDA0

    @property
    def slab(self):
        """z range [z0, z1) the lens can occupy."""
        return self.z_base, self.z_base + int(math.ceil(self.h_max)) + 1


def kinoform_design(shape, pitch, D: float, NA: float = 0.84, n_lens: float = 1.54,
                    n_bg: float = 1.0, lambda0: float = LAMBDA0, pml=None,
                    smoothing: float = 355e-9, name: str = "lens") -> LensDesign:
    """A Fresnel (kinoform) lens of diameter D as the starting thickness map:
    h = h_max (1 - frac(s)), s = (sqrt(r^2 + f^2) - f) / (lambda0 / n_bg), so
    the optical path (n - n_bg) h + n_bg sqrt(r^2 + f^2) is constant modulo
    lambda0, thickest at the centre, maximum thickness one wrap
    lambda0 / (n - n_bg) (2.0 um at n = 1.54, the paper's starting lens).
    r is measured from the lateral centre ((n - 1) / 2) d at voxel centres; the
    base plane and focus follow the zone-plate conventions (exit face at the
    maximum thickness)."""
    nx, ny, nz = shape
    if pml is None:
        pml = pml_voxels(pitch, lambda0)
    f = focal_length(D, NA)
    hmax_m = lambda0 / (n_lens - n_bg)
    y = (np.arange(ny) - (ny - 1) / 2.0) * pitch
    x = (np.arange(nx) - (nx - 1) / 2.0) * pitch
    r = np.sqrt(y[:, None] ** 2 + x[None, :] ** 2)
    lat = np.zeros((ny, nx), dtype=bool)
    lat[pml[1]:ny - pml[1], pml[0]:nx - pml[0]] = True
    aperture = (r < D / 2.0) & lat
    s = (np.sqrt(r * r + f * f) - f) / (lambda0 / n_bg)
    h = np.where(aperture, hmax_m * (1.0 - (s - np.floor(s))), 0.0) / pitch
    z_b = pml[2] + int(math.ceil(lambda0 / (2.0 * pitch)))
    z_lo = (z_b - 0.5) * pitch
    r0 = ((nx - 1) // 2, (ny - 1) // 2, int(math.floor((z_lo + hmax_m + f) / pitch + 0.5)))
    return LensDesign(name=name, shape=tuple(shape), pitch=pitch, pml=tuple(pml), z_base=z_b,
                      h_max=hmax_m / pitch, n_lens=n_lens, n_bg=n_bg, D=D, NA=NA, f_eff=f,
                      r0=r0, aperture=aperture.astype(np.float32), h_init=h,
                      sigma_vox=smoothing / pitch, lambda0=lambda0)


def lens32_design() -> LensDesign:
    """The optimisation benchmark: D = 32 um, NA 0.84, n = 1.54 on the
    189 x 189 x 121 grid at 177 nm (benchmark paragraph)."""
    return kinoform_design((189, 189, 121), 177e-9, 32e-6, name="lens32")


def lens_design_small(n: int = 48, nz: int = 64, D: float = 5e-6) -> LensDesign:
    """A small kinoform (n x n x nz at lambda/6) for parity tests of the design loop."""
    return kinoform_design((n, n, nz), LAMBDA0 / 6, D, name=f"lens{n}")


def design_slab(scene: Scene, thickness: float = 2.0e-6, seed: int = 0,
                amp: float = 0.25, lo: float = 1.0, hi: float = 2.1) -> Scene:
    """Seed-random eps_r perturbation in a design slab above the lens base.

    The slab is z in [z_b, z_b + round(thickness / d)) over the lateral
    interior; eps_r <- clip(eps_r + U(-amp, amp), lo, hi) with
    numpy.random.default_rng(seed)."""
    px, py, pz = scene.pml
    nx, ny, nz = scene.shape
    z_b = scene.info["z_base"]
    nzs = int(round(thickness / scene.pitch))
    lo_c = (px, py, z_b)
    hi_c = (nx - px, ny - py, z_b + nzs)
    eps = scene.eps_r.copy()
    rng = np.random.default_rng(seed)
    sl = (slice(lo_c[2], hi_c[2]), slice(lo_c[1], hi_c[1]), slice(lo_c[0], hi_c[0]))
    block = eps[sl].astype(np.float64)
    block = np.clip(block + rng.uniform(-amp, amp, size=block.shape), lo, hi)
    eps[sl] = block.astype(np.float32)
    return dataclasses.replace(scene, eps_r=eps, design_box=(lo_c, hi_c),
                               name=scene.name + "+slab")


# ---------------------------------------------------------------------------
# The workloads
# ---------------------------------------------------------------------------
def sphere64() -> Scene:
    """64^3 at lambda/6, layer 8/8/16 per side, n = 1.45 sphere of radius 1.2 um."""
    return sphere_scene(64, LAMBDA0 / 6, 1.2e-6, 1.45, 1.0, (8, 8, 16), name="sphere64")


def zoneplate16() -> Scene:
    """275 x 275 x 315 at lambda/16, D = 16 um, NA 0.84, n = 1.45."""
    pitch = LAMBDA0 / 16
    return zone_plate_scene((275, 275, 315), pitch, 16e-6, 0.84, 1.45,
                            pml=pml_voxels(pitch), name="zoneplate16")


def zoneplate16_design(seed: int = 0) -> Scene:
    """The 16 um lens with a 2 um seed-random design slab (adjoint gradient)."""
    return design_slab(zoneplate16(), 2.0e-6, seed)


def zoneplate100() -> Scene:
    """621 x 621 x 261 at 177 nm, D = 100 um, NA 0.84, n = 1.45."""
    pitch = 177e-9
    return zone_plate_scene((621, 621, 261), pitch, 100e-6, 0.84, 1.45,
                            pml=pml_voxels(pitch), name="zoneplate100")


def zoneplate100_design(seed: int = 0) -> Scene:
    return design_slab(zoneplate100(), 2.0e-6, seed)


# ---------------------------------------------------------------------------
# Generic random inputs for parity tests
# ---------------------------------------------------------------------------
def random_passive_eps(shape, pml, seed: int, n_bg: float = 1.0, lo: float = 1.0,
                       hi: float = 2.1, loss: float = 0.0) -> np.ndarray:
    """Random eps_r in [lo, hi] (+ i U[0, loss]) with n_bg^2 in the layer.

    Returned as float32 if loss == 0 else complex64."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    re = rng.uniform(lo, hi, size=(nz, ny, nx))
    if loss > 0:
        eps = (re + 1j * rng.uniform(0.0, loss, size=(nz, ny, nx))).astype(np.complex64)
    else:
        eps = re.astype(np.float32)
    px, py, pz = pml
    nb2 = np.float32(n_bg * n_bg)
    if pz:
        eps[:pz] = nb2
        eps[nz - pz:] = nb2
    if py:
        eps[:, :py] = nb2
        eps[:, ny - py:] = nb2
    if px:
        eps[:, :, :px] = nb2
        eps[:, :, nx - px:] = nb2
    return eps


def random_field(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """Complex64 vector field [3, nz, ny, nx] with N(0, scale^2) parts."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((2, 3, nz, ny, nx)) * scale
    return (f[0] + 1j * f[1]).astype(np.complex64)


# ---------------------------------------------------------------------------
# Served batch: a seeded stream of mixed-size forward / adjoint requests
# ---------------------------------------------------------------------------
SERVED_GRIDS = (
    ((64, 64, 64), LAMBDA0 / 6),
    ((128, 128, 128), LAMBDA0 / 6),
    ((192, 192, 256), LAMBDA0 / 12),
    ((275, 275, 315), LAMBDA0 / 16),
)


@dataclasses.dataclass
class ServedRequest:
    """One request of a served trace: a scene, its kind and its arrival time."""

    rid: int
    kind: str            # "forward" or "adjoint" (forward + adjoint + gradient)
    scene: Scene
    arrival: float       # seconds after the start of the trace


def served_scene(rng: np.random.Generator, grid=None, name="served") -> Scene:
    """Random sphere or zone plate, n ~ U[1.3, 1.6], on one of the served grids."""
    if grid is None:
        grid = SERVED_GRIDS[int(rng.integers(len(SERVED_GRIDS)))]
    shape, pitch = grid
    nx, ny, nz = shape
    pml = pml_voxels(pitch)
    n_obj = float(rng.uniform(1.3, 1.6))
    ix, iy, iz = nx - 2 * pml[0], ny - 2 * pml[1], nz - 2 * pml[2]
    if rng.random() < 0.5:
        rmax = 0.35 * min(ix, iy, iz) * pitch
        radius = float(rng.uniform(0.5e-6, max(0.5e-6, rmax)))
        jit = rng.uniform(-1.0, 1.0, size=3) * pitch
        c = ((nx - 1) / 2 * pitch + jit[0], (ny - 1) / 2 * pitch + jit[1], (nz - 1) / 2 * pitch + jit[2])
        f = sphere_fraction(shape, pitch, radius, center=c, supersample=4)
        eps = (1.0 + f * (n_obj ** 2 - 1.0)).astype(np.float32)
        _clear_layer(eps, pml, 1.0)
        zf = int(round((c[2] + radius + 1e-6) / pitch))
        r0 = ((nx - 1) // 2, (ny - 1) // 2, min(zf, nz - pml[2] - 1))
        sc = Scene(name=name, shape=shape, pitch=pitch, pml=pml, eps_r=eps, r0=r0,
                   info=dict(kind="sphere", radius=radius, n=n_obj))
        lo = (pml[0], pml[1], pml[2])
        hi = (nx - pml[0], ny - pml[1], nz - pml[2])
    else:
        D = min(16e-6, 0.9 * min(ix, iy) * pitch)
        sc = zone_plate_scene(shape, pitch, D, 0.84, n_obj, pml=pml, supersample=4, name=name)
        zb = sc.info["z_base"]
        lo = (pml[0], pml[1], zb)
        hi = (nx - pml[0], ny - pml[1], zb + max(1, int(round(2e-6 / pitch))))
        sc.info["kind"] = "zoneplate"
    return dataclasses.replace(sc, design_box=(lo, hi))


def served_trace(n_requests: int = 200, rate_hz: float = 5.0, seed: int = 0, grids=None):
    """Poisson arrivals (numpy default_rng(seed)) of forward/adjoint requests
    at 50/50, grids uniform over `grids` (default: the four served grids)."""
    rng = np.random.default_rng(seed)
    grids = SERVED_GRIDS if grids is None else grids
    t = 0.0
    out = []
    for i in range(n_requests):
        t += float(rng.exponential(1.0 / rate_hz))
        grid = grids[int(rng.integers(len(grids)))]
        kind = "forward" if rng.random() < 0.5 else "adjoint"
        out.append(ServedRequest(i, kind, served_scene(rng, grid, name=f"req{i}"), t))
    return out
