"""GPU tests of the autograd path (forward solve + adjoint gradient through the
C ABI) against the FP64 oracle's adjoint gradient and finite differences."""

import numpy as np
import pytest
import torch

from oracle import cbs as oc
from paper_2506_15411_amd import scenes
from paper_2506_15411_amd.autograd import cbs_solve, focal_intensity
from paper_2506_15411_amd.solver import Plan

pytestmark = pytest.mark.gpu
LAM = 1.064e-6
# the FP32 iteration's residual floor on these 16 x 14 x 18 grids is about
# 1.5e-7; solves to 5e-7 are converged and stop there
TOL = 5e-7


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def setup(device, shape=(16, 14, 18), pml=(2, 2, 3), seed=23):
    eps = scenes.random_passive_eps(shape, pml, seed)
    g = oc.Grid(*shape, LAM / 8, LAM, 1.0, pml)
    p = Plan(shape, LAM / 8, LAM, 1.0, pml, device=device)
    return g, p, eps


def test_focal_intensity_gradient_matches_oracle(device):
    g, p, eps = setup(device)
    r0 = (8, 7, 12)
    e = torch.from_numpy(eps).to(device).requires_grad_(True)
    L = focal_intensity(e, p, r0, tol=TOL, max_iter=5000)
    L.backward()
    Eo, _ = oc.solve_forward(g, eps, tol=1e-11, max_iter=40000)
    ga = oc.solve_adjoint(g, eps, oc.adjoint_point_source(g, Eo, r0), tol=1e-11, max_iter=40000)
    gref = oc.gradient(g, Eo, ga.E_s, scale=2.0)
    assert L.item() == pytest.approx(oc.focal_objective(Eo, r0), rel=1e-4)
    assert rel(e.grad.cpu().numpy(), gref) < 1e-3
    # the point-source adjoint path gives the same gradient
    E, _ = p.solve(tol=TOL, max_iter=5000)
    Ea, _ = p.adjoint(E_fwd=E, r0=r0, tol=TOL, max_iter=5000)
    gp = p.gradient(E, Ea, scale=2.0)
    assert rel(e.grad.cpu().numpy(), gp.cpu().numpy()) < 1e-4


def test_general_loss_gradient_matches_oracle(device):
    g, p, eps = setup(device, seed=29)
    e = torch.from_numpy(eps).to(device).requires_grad_(True)
    E = cbs_solve(e, p, tol=TOL, max_iter=5000)
    region = (slice(None), slice(9, 14), slice(5, 9), slice(6, 10))
    L = (E[region].abs() ** 2).sum() + E[0, 12, 7, 8].real - 0.5 * E[2, 11, 6, 9].imag
    L.backward()
    Eo, _ = oc.solve_forward(g, eps, tol=1e-11, max_iter=40000)
    gE = np.zeros_like(Eo)            # torch convention: gE = 2 dL/dE*
    gE[region] = 2 * Eo[region]
    gE[0, 12, 7, 8] += 1.0
    gE[2, 11, 6, 9] += -0.5 * 1j
    ga = oc.solve_adjoint(g, eps, np.conj(gE), tol=1e-11, max_iter=40000)
    gref = oc.gradient(g, Eo, ga.E_s, scale=1.0)
    assert rel(e.grad.cpu().numpy(), gref) < 1e-3


def test_directional_finite_difference(device):
    """GPU-only check: (L(eps + h v) - L(eps - h v)) / 2h against <grad, v> for
    the coherent direction v = sign(grad) over the interior, with h chosen so
    that L moves by about 1%.  The solves iterate to the FP32 floor of the
    residual (about 1.6e-7 on this grid: tol 1e-8 is not reached, so the
    20000-iteration cap ends them and strict is off)."""
    g, p, eps = setup(device, seed=31)
    r0 = (8, 7, 12)
    e = torch.from_numpy(eps).to(device).requires_grad_(True)
    L = focal_intensity(e, p, r0, tol=1e-8, max_iter=20000, strict=False)
    L.backward()
    mask = torch.zeros_like(e)
    mask[3:-3, 2:-2, 2:-2] = 1.0
    vt = torch.sign(e.grad) * mask
    dg = float((e.grad * vt).sum().item())
    h = 0.01 * L.item() / dg
    with torch.no_grad():
        Lp = focal_intensity(e + h * vt, p, r0, tol=1e-8, max_iter=20000, strict=False).item()
        Lm = focal_intensity(e - h * vt, p, r0, tol=1e-8, max_iter=20000, strict=False).item()
    fd = (Lp - Lm) / (2 * h)
    assert abs(fd - dg) <= 1e-3 * abs(dg)


def test_sphere64_design_slab_gradient_vs_oracle(device):
    """The gradient case on the 64^3 sphere grid: seeded design slab, objective
    |E(r0)|^2, GPU forward + adjoint + gradient against the FP64 oracle's
    adjoint gradient over the slab."""
    sc = scenes.sphere64()
    eps = sc.eps_r.copy()
    rng = np.random.default_rng(0)
    sl = (slice(18, 24), slice(8, 56), slice(8, 56))
    eps[sl] = np.clip(eps[sl] + rng.uniform(-0.25, 0.25, eps[sl].shape), 1.0, 2.1).astype(np.float32)
    r0, lo, hi = (32, 32, 44), (8, 8, 18), (56, 56, 24)
    g = oc.Grid(*sc.shape, sc.pitch, LAM, 1.0, sc.pml)
    p = Plan(sc.shape, sc.pitch, LAM, 1.0, sc.pml, device=device)
    p.set_permittivity(torch.from_numpy(eps).to(device))
    E, s1 = p.solve(tol=1e-6, max_iter=4000)
    Ea, s2 = p.adjoint(E_fwd=E, r0=r0, tol=1e-6, max_iter=4000)
    grad = p.gradient(E, Ea, lo, hi, scale=2.0)
    Eo, _ = oc.solve_forward(g, eps, tol=1e-9, max_iter=20000)
    ga = oc.solve_adjoint(g, eps, oc.adjoint_point_source(g, Eo, r0), tol=1e-9, max_iter=20000)
    gref = oc.gradient(g, Eo, ga.E_s, lo, hi, scale=2.0)
    assert rel(grad.cpu().numpy(), gref) < 1e-3
