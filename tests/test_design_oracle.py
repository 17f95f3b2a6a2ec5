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
