"""Pins of the oracle's lens-design map (thickness map -> eps_r) and its chain
rule, CPU only: projection and adjoint identities checked on explicit
matrices, directional finite differences of the map and of the figure of
merit through the FP64 CBS solve, and the Adam step against torch's Adam."""

import math

import numpy as np
import pytest

from oracle import cbs as oc
from oracle import design as od
from paper_2506_15411_amd import scenes

LAM = scenes.LAMBDA0


def tiny_design():
    """A kinoform on a 20 x 20 x 32 grid at lambda/6 with a thin layer."""
    return scenes.kinoform_design((20, 20, 32), LAM / 6, 2.5e-6, pml=(2, 2, 3), name="lens20")


def test_symmetrize_is_an_orthogonal_projection():
    rng = np.random.default_rng(0)
    a, b = rng.normal(size=(2, 9, 11))
    s = od.symmetrize(a)
    assert np.allclose(s, s[:, ::-1]) and np.allclose(s, s[::-1, :])
    assert np.allclose(od.symmetrize(s), s)
    assert np.sum(od.symmetrize(a) * b) == pytest.approx(np.sum(a * od.symmetrize(b)), rel=1e-12)


def test_smoothing_adjoint_on_explicit_matrices():
    """Build the matrix of `smooth` column by column and compare its transpose
    with the matrix of `smooth_adjoint`; the kernel sums to one and a
    constant far from the edges stays constant."""
    sigma, shape = 1.3, (9, 11)
    n = shape[0] * shape[1]
    A = np.zeros((n, n))
    B = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        A[:, k] = od.smooth(e.reshape(shape), sigma).ravel()
        B[:, k] = od.smooth_adjoint(e.reshape(shape), sigma).ravel()
    assert np.allclose(A.T, B, atol=1e-15)
    K = od.gaussian_kernel(2.0)
    assert K.sum() == pytest.approx(1.0, abs=1e-14)
    c = od.smooth(np.ones((40, 40)), 2.0)
    assert np.allclose(c[12:-12, 12:-12], 1.0, atol=1e-13)


def test_kinoform_start():
    d = scenes.lens32_design()
    h = d.h_init
    assert h.min() >= 0.0 and h.max() <= d.h_max + 1e-12
    assert np.allclose(h, h[:, ::-1]) and np.allclose(h, h[::-1, :])
    cy, cx = (d.shape[1] - 1) // 2, (d.shape[0] - 1) // 2
    assert h[cy, cx] == pytest.approx(d.h_max, rel=1e-6)        # thickest at the centre
    assert d.h_max * d.pitch == pytest.approx(LAM / 0.54, rel=1e-12)   # one wrap: 1.97 um
    assert np.all(h[d.aperture == 0] == 0.0)
    z0, z1 = d.slab
    assert z0 >= d.pml[2] and z1 <= d.shape[2] - d.pml[2] and d.r0[2] < d.shape[2] - d.pml[2]


@pytest.mark.parametrize("smoothing", [False, True])
def test_design_map_directional_derivative(smoothing):
    """<w, eps(p + t v)> by central differences against <grad_p(w), v>; the
    map is piecewise linear, so a small step is exact unless it crosses a
    voxel face (the random p keeps every column away from one)."""
    d = tiny_design()
    rng = np.random.default_rng(1)
    ny, nx = d.aperture.shape
    p = d.h_init + rng.uniform(-0.3, 0.3, size=(ny, nx))
    v = rng.normal(size=(ny, nx))
    z0, z1 = d.slab
    w = rng.normal(size=(z1 - z0, ny, nx))
    t = 1e-6

    def F(q):
        return float(np.sum(w * od.eps_of(q, d, smoothing)[z0:z1]))

    fd = (F(p + t * v) - F(p - t * v)) / (2 * t)
    an = float(np.sum(od.grad_p(w, p, d, smoothing) * v))
    assert fd == pytest.approx(an, rel=1e-6)


def test_figure_of_merit_gradient_by_finite_differences():
    """L(p) = |E(r0)|^2 through the FP64 CBS solve: central differences along
    a random direction against the chain rule from the adjoint gradient."""
    d = tiny_design()
    g = oc.Grid(*d.shape, d.pitch, LAM, d.n_bg, d.pml)
    rng = np.random.default_rng(2)
    ny, nx = d.aperture.shape
    p = d.h_init + rng.uniform(-0.3, 0.3, size=(ny, nx))
    z0, z1 = d.slab

    def L(q):
        E, _ = oc.solve_forward(g, od.eps_of(q, d), tol=1e-13, max_iter=40000)
        ix, iy, iz = d.r0
        return float(np.sum(np.abs(E[:, iz, iy, ix]) ** 2)), E

    L0, E = L(p)
    ga = oc.solve_adjoint(g, od.eps_of(p, d), oc.adjoint_point_source(g, E, d.r0),
                          tol=1e-13, max_iter=40000)
    geps = oc.gradient(g, E, ga.E_s, (0, 0, z0), (nx, ny, z1), scale=2.0)
    gp = od.grad_p(geps, p, d)
    v = rng.normal(size=(ny, nx))
    t = 1e-5
    fd = (L(p + t * v)[0] - L(p - t * v)[0]) / (2 * t)
    assert fd == pytest.approx(float(np.sum(gp * v)), rel=1e-5)


def test_adam_step_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(4)
    p0 = rng.uniform(0.0, 5.0, size=(6, 7))
    grads = [rng.normal(size=(6, 7)) for _ in range(4)]
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for t, gr in enumerate(grads, start=1):
        p, m, v = od.adam_step(p, gr, m, v, t)
    q = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([q], lr=0.3, betas=(0.9, 0.999), eps=1e-6, maximize=True)
    for gr in grads:
        opt.zero_grad()
        q.grad = torch.tensor(gr)
        opt.step()
    assert np.allclose(p, q.detach().numpy(), rtol=0, atol=1e-12)


# ---------------------------------------------------------------------------
# Lens figures (focus, FWHM, focusing efficiency)
# ---------------------------------------------------------------------------
def test_fwhm_of_a_sampled_gaussian():
    """FWHM of exp(-x^2 / (2 s^2)) is 2 sqrt(2 ln 2) s; linear interpolation
    between samples at pitch s/5 is good to a few 1e-3."""
    from oracle import metrics as om
    s, d = 1.0, 0.2
    x = (np.arange(201) - 97.3) * d
    v = np.exp(-x * x / (2 * s * s))
    w = om.fwhm(v, int(np.argmax(v)), d)
    assert w == pytest.approx(2 * math.sqrt(2 * math.log(2)) * s, rel=3e-3)
    assert math.isnan(om.fwhm(np.ones(10), 5, d))


def test_plane_flux_of_plane_waves():
    """A plane wave of unit amplitude carries S_z = cos(theta) through a plane:
    normal incidence (x-polarised) and an oblique TM wave whose kx is a grid
    frequency, E = (cos t, 0, -sin t) exp(i k (x sin t + z cos t)) sampled in
    the plane z = 0 (only its transverse part enters)."""
    from oracle import metrics as om
    nx, ny, d = 64, 48, 0.1
    k = 2 * math.pi / 0.75
    x = np.arange(nx) * d
    Ex = np.ones((ny, nx), dtype=complex)
    Ey = np.zeros((ny, nx), dtype=complex)
    assert np.allclose(om.plane_flux(Ex, Ey, d, k), 1.0, atol=1e-12)
    m = 5
    kx = 2 * math.pi * m / (nx * d)
    t = math.asin(kx / k)
    Ex = np.broadcast_to(math.cos(t) * np.exp(1j * kx * x)[None, :], (ny, nx)).copy()
    assert np.allclose(om.plane_flux(Ex, Ey, d, k), math.cos(t), atol=1e-12)
    # an evanescent component carries nothing
    kx2 = 2 * math.pi * 20 / (nx * d)
    assert kx2 > k
    Ex2 = np.broadcast_to(np.exp(1j * kx2 * x)[None, :], (ny, nx)).copy()
    assert np.allclose(om.plane_flux(Ex2, Ey, d, k), 0.0, atol=1e-12)


def test_lens_figures_of_a_synthetic_focus():
    """Focus and FWHM of a Gaussian spot, and eta_f of a normally incident
    plane wave: the disc holds (voxel centres within the radius) x d^2 of
    flux, counted by brute force."""
    from oracle import metrics as om
    nx = ny = 81
    nz = 5
    d = 0.1
    s = 0.6
    y, x = np.meshgrid((np.arange(ny) - 40) * d, (np.arange(nx) - 40) * d, indexing="ij")
    plane = np.exp(-(x * x + y * y) / (2 * s * s))
    E = np.zeros((3, nz, ny, nx), dtype=np.complex128)
    E[0, 2] = np.sqrt(plane)
    E[0, 1] = 0.4 * np.sqrt(plane)
    E[0, 3] = 0.4 * np.sqrt(plane)
    k = 2 * math.pi / 0.75
    f = om.lens_figures(E, d, (0, 0, 0), (nx, ny, nz), aperture=1.0, k=k)
    assert f["focus"] == (40, 40, 2)
    fw = 2 * math.sqrt(2 * math.log(2)) * s
    assert f["fwhm"][0] == pytest.approx(fw, rel=5e-3) and f["fwhm"][1] == pytest.approx(fw, rel=5e-3)
    # a plane wave with a bump to fix the focus: eta_f from the disc count
    E2 = np.zeros((3, 3, 21, 21), dtype=np.complex128)
    E2[0] = 1.0
    f2 = om.lens_figures(E2 + 0.0, 0.1, (0, 0, 0), (21, 21, 3), aperture=1.0, k=k)
    assert math.isnan(f2["fwhm"][0])                  # a flat field has no width
    Sz = om.plane_flux(E2[0, 1], E2[1, 1], 0.1, k)
    assert np.allclose(Sz, 1.0)
    r = 4.3
    brute = sum(1 for j in range(21) for i in range(21) if (i - 10) ** 2 + (j - 10) ** 2 <= r * r)
    yy, xx = np.meshgrid(np.arange(21) - 10, np.arange(21) - 10, indexing="ij")
    assert float(np.sum(Sz[(xx * xx + yy * yy) <= r * r])) == pytest.approx(brute, rel=1e-12)
