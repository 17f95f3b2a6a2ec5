"""Converged GPU solves against FP64 fixtures written by tests/golden/make_converged.py
(oracle only; see that script for how each was computed).

* 275 x 275 x 315 zone plate (the Fig. 1 benchmark lens): the GPU's scattered
  field at tol 1e-6 against the FP64 CBS field the fixture stores (its own eta
  and estimated error are stored with it) on the focal plane, the xz plane
  through the axis, 4096 seeded voxels and the whole-volume norm.
* The same lens with its seeded design slab: forward and adjoint to tol 1e-6,
  the gradient of |E(r0)|^2 over the slab against the oracle's adjoint gradient
  (4096 slab voxels, the slab's middle plane, the norm).
* 64^3 sphere with a 6-voxel design slab: the GPU adjoint gradient against FP64
  central differences at 32 voxels (each within 1e-3 of the difference).
* The same slab gradient checked by a random +-1 directional difference on the
  GPU, reported with the FP32 noise floor of the objective.

Tolerance at convergence: 1e-3 relative (the FP32 iteration stops at eta 1e-6;
its distance to the exact solution is about eta / (1 - rho) plus FP32
round-off), or three times the fixture's own estimated error where that is
larger (the FP64 iteration of these lenses contracts by only about 0.999 per
step at the end, so its solution carries an error of about 1000 eta).
"""

import os

import numpy as np
import pytest
import torch

from paper_2506_15411_amd import libcbs as L
from paper_2506_15411_amd import scenes
from paper_2506_15411_amd.solver import Plan

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
LAM = scenes.LAMBDA0


def golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated (tests/golden/make_converged.py)")
    return np.load(path)


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel())
                 / np.linalg.norm(np.asarray(b).ravel()))


def fixture_tol(gd):
    """1e-3, or three times the fixture's estimated relative error if larger"""
    est = float(np.max(np.atleast_1d(gd["error_estimate"])))
    tol = max(1e-3, 3.0 * est)
    print(f"fixture eta {np.atleast_1d(gd['eta']).tolist()}, estimated error {est:.1e}: "
          f"tolerance {tol:.1e}")
    return tol


def check_samples(got, want, what, tol=1e-3, worst_tol=5e-2):
    """relative L2 over the samples within tol; the worst single sample, in units
    of the samples' rms magnitude, within worst_tol (the slow modes of these
    lenses live in the low-field region between the thin lateral layers, where
    a sample's error is a larger share of its own magnitude)"""
    got = np.asarray(got)
    want = np.asarray(want)
    r = rel(got, want)
    rms = np.sqrt(np.mean(np.abs(want) ** 2))
    worst = float(np.max(np.abs(got - want)) / rms)
    print(f"{what}: rel-L2 {r:.2e}, worst sample {worst:.2e} of rms")
    assert r < tol and worst < worst_tol, what


def test_lens16_converged_field_vs_fp64_fixture(device):
    gd = golden("lens16_converged.npz")
    sc = scenes.zoneplate16()
    assert tuple(gd["shape"]) == sc.shape and tuple(gd["r0"]) == sc.r0
    p = Plan(sc.shape, sc.pitch, LAM, 1.0, sc.pml, device=device)
    p.set_permittivity(torch.from_numpy(sc.eps_r).to(device))
    assert p.eps_shift == pytest.approx(float(gd["eps_shift"]), rel=1e-12)
    E, st = p.solve(tol=1e-6, max_iter=20000, scattered=True)
    assert st.status == L.CBS_OK
    print(f"GPU {st.iterations} iterations to {st.residual:.2e}; FP64 solution's own "
          f"eta {float(gd['eta']):.2e}")
    tol = fixture_tol(gd)
    x0, y0, z0 = sc.r0
    check_samples(E[:, z0].cpu().numpy(), gd["focal_plane"], "focal plane", tol)
    check_samples(E[:, :, y0, :].cpu().numpy(), gd["xz_plane"], "xz plane", tol)
    vx, vy, vz = (torch.from_numpy(v).to(device) for v in gd["vox"])
    check_samples(E[:, vz, vy, vx].cpu().numpy(), gd["vox_E"], "4096 voxels", tol)
    norm = float(torch.linalg.vector_norm(E.to(torch.complex128)).item())
    assert abs(norm - float(gd["norm"])) < tol * float(gd["norm"])
    # how far solves to the configs' tol 1e-4, and to 1e-5, are from the converged field
    for t in (1e-4, 1e-5):
        Et, s_t = p.solve(tol=t, max_iter=20000, scattered=True)
        d = rel(Et[:, vz, vy, vx].cpu().numpy(), gd["vox_E"])
        print(f"a solve to tol {t:.0e} ({s_t.iterations} iterations) is {d:.2e} from the "
              f"converged field at the 4096 voxels (the FP64 fixture's own estimated error "
              f"{float(gd['error_estimate']):.1e})")
    p.close()


def test_lens16_converged_gradient_vs_fp64_fixture(device):
    gd = golden("lens16_gradient_converged.npz")
    sc = scenes.zoneplate16_design(0)
    lo, hi = sc.design_box
    assert tuple(gd["box_lo"]) == tuple(lo) and tuple(gd["box_hi"]) == tuple(hi)
    p = Plan(sc.shape, sc.pitch, LAM, 1.0, sc.pml, device=device)
    p.set_permittivity(torch.from_numpy(sc.eps_r).to(device))
    E, s1 = p.solve(tol=1e-6, max_iter=20000)
    Ea, s2 = p.adjoint(E_fwd=E, r0=sc.r0, tol=1e-6, max_iter=20000)
    assert s1.status == L.CBS_OK and s2.status == L.CBS_OK
    print(f"GPU {s1.iterations} + {s2.iterations} iterations; FP64 solutions' own eta "
          f"{list(gd['eta'])}")
    tol = fixture_tol(gd)
    x0, y0, z0 = sc.r0
    fom = float((E[:, z0, y0, x0].abs() ** 2).sum().item())
    assert fom == pytest.approx(float(gd["objective"]), rel=tol)
    grad = p.gradient(E, Ea, lo, hi, scale=2.0)
    vx, vy, vz = (torch.from_numpy(v).to(device) for v in gd["vox"])
    check_samples(grad[vz, vy, vx].double().cpu().numpy(), gd["vox_grad"], "4096 slab voxels",
                  tol)
    bz = grad.shape[0]
    check_samples(grad[bz // 2].double().cpu().numpy(), gd["mid_plane"], "slab middle plane", tol)
    norm = float(torch.linalg.vector_norm(grad.double()).item())
    assert abs(norm - float(gd["norm"])) < tol * float(gd["norm"])
    p.close()


def sphere64_slab():
    """the 64^3 gradient case of make_converged.py (same seeds and geometry)"""
    sc = scenes.sphere64()
    eps = sc.eps_r.copy()
    rng = np.random.default_rng(0)
    sl = (slice(18, 24), slice(8, 56), slice(8, 56))
    eps[sl] = np.clip(eps[sl] + rng.uniform(-0.25, 0.25, eps[sl].shape), 1.0, 2.1).astype(np.float32)
    return sc, eps, (32, 32, 44), (8, 8, 18), (56, 56, 24)


def test_sphere64_gradient_vs_fp64_central_differences(device):
    gd = golden("sphere64_fd_gradient.npz")
    sc, eps, r0, lo, hi = sphere64_slab()
    assert tuple(gd["r0"]) == r0 and tuple(gd["box_lo"]) == lo and tuple(gd["box_hi"]) == hi
    p = Plan(sc.shape, sc.pitch, LAM, 1.0, sc.pml, device=device)
    p.set_permittivity(torch.from_numpy(eps).to(device))
    E, s1 = p.solve(tol=5e-7, max_iter=20000)
    Ea, s2 = p.adjoint(E_fwd=E, r0=r0, tol=5e-7, max_iter=20000)
    assert s1.status == L.CBS_OK and s2.status == L.CBS_OK
    grad = p.gradient(E, Ea, lo, hi, scale=2.0).double().cpu().numpy()
    worst = 0.0
    for (x, y, z), fd in zip(gd["vox"], gd["fd"]):
        gv = grad[z - lo[2], y - lo[1], x - lo[0]]
        worst = max(worst, abs(gv - fd) / abs(fd))
    print(f"64^3 slab: worst relative difference of 32 voxels to the FP64 central "
          f"difference {worst:.2e}")
    assert worst < 1e-3
    p.close()


def test_lens16_slab_random_direction_difference(device):
    """Directional difference of |E(r0)|^2 along a random +-1 direction over the
    whole 2 um slab of the 16 um lens (h = 1e-2), GPU solves to tol 1e-6 (the
    FP32 residual floor of this volume is about 5e-7), against <grad, v>.  The
    FP32 noise floor of the objective is measured as the spread of |E(r0)|^2
    over solves started from different fields; the difference must agree with
    <grad, v> within the floor's effect plus 2% (second-order terms of the
    central difference)."""
    sc = scenes.zoneplate16_design(0)
    lo, hi = sc.design_box
    x0, y0, z0 = sc.r0
    eps = torch.from_numpy(sc.eps_r).to(device)
    p = Plan(sc.shape, sc.pitch, LAM, 1.0, sc.pml, device=device)
    tol = 1e-6

    def fom(e, warm=None):
        p.set_permittivity(e)
        E = warm.clone() if warm is not None else p.new_field()
        E, st = p.solve(E, tol=tol, max_iter=20000, warm=warm is not None)
        assert st.status == L.CBS_OK
        return float((E[:, z0, y0, x0].to(torch.complex128).abs() ** 2).sum().item()), E

    L0, E = fom(eps)
    Ea, st = p.adjoint(E_fwd=E, r0=sc.r0, tol=tol, max_iter=20000)
    grad = p.gradient(E, Ea, lo, hi, scale=2.0).double()
    gen = torch.Generator(device="cpu").manual_seed(3)
    v = (torch.randint(0, 2, grad.shape, generator=gen) * 2 - 1).to(device, torch.float64)
    dg = float((grad * v).sum().item())
    h = 1e-2
    sl = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
    ep, em = eps.clone(), eps.clone()
    ep[sl] += (h * v).float()
    em[sl] -= (h * v).float()
    Lp, _ = fom(ep, E)
    Lm, _ = fom(em, E)
    fd = (Lp - Lm) / (2 * h)
    # noise floor: the same objective from a cold start and from a warm start
    L0w, _ = fom(eps, E * 0.5)
    floor = abs(L0w - L0) / (2 * h) * np.sqrt(2)
    print(f"random +-1 direction over {grad.numel()} slab voxels: <grad, v> {dg:.6e}, "
          f"central difference {fd:.6e} (relative {abs(fd - dg) / abs(dg):.2e}), "
          f"objective {L0:.6e}, FP32 noise floor of the difference {floor:.2e} "
          f"({floor / abs(dg):.2e} relative)")
    assert abs(fd - dg) <= 3 * floor + 2e-2 * abs(dg)
    p.close()
