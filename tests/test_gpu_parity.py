"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Tolerances (relative L2 over all voxels and components):
  * one Green's-operator application: 5e-6 (FP32 FFTs of these lengths carry
    ~1e-7 log2 N of round-off);
  * CBS at equal iteration count: 1e-4; at convergence: 1e-3.
"""

import math

import numpy as np
import pytest
import torch

from oracle import cbs as oc
from oracle import closed
from paper_2506_15411_amd import libcbs as L
from paper_2506_15411_amd import scenes
from paper_2506_15411_amd.solver import Plan

pytestmark = pytest.mark.gpu
LAM = 1.064e-6


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def to_dev(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def make(shape, pitch, pml, eps, dev, **kw):
    g = oc.Grid(*shape, pitch, LAM, 1.0, tuple(pml), **{k: v for k, v in kw.items()})
    p = Plan(shape, pitch, LAM, 1.0, pml, device=dev,
             pml_order=kw.get("pml_order", 2), sigma_max=kw.get("sigma_max", 1.0),
             shift_factor=kw.get("shift_factor", 1.1))
    p.set_permittivity(to_dev(eps, dev))
    return g, p


SHAPES = [(8, 8, 8), (5, 6, 7), (12, 10, 9), (16, 16, 16), (40, 36, 48), (27, 25, 29),
          (64, 64, 64), (100, 96, 36), (20, 18, 121)]


@pytest.mark.parametrize("shape", SHAPES)
def test_green_operator_matches_oracle(shape, device):
    pml = (1, 1, 1)
    eps = scenes.random_passive_eps(shape, pml, 3, loss=0.05)
    g, p = make(shape, LAM / 8, pml, eps, device)
    pot = oc.potentials(g, eps)
    assert p.eps_shift == pytest.approx(pot.eps, rel=1e-12)
    W = scenes.random_field(shape, 5)
    out = p.apply_green(to_dev(W, device))
    torch.cuda.synchronize()
    ref = oc.green_apply(g, W.astype(np.complex128), pot.kt2)
    assert rel(out.cpu().numpy(), ref) < 5e-6


@pytest.mark.parametrize("shape,pml,loss,k", [
    ((8, 8, 8), (2, 2, 2), 0.0, 30),
    ((12, 10, 9), (2, 2, 2), 0.1, 40),
    ((16, 16, 16), (3, 3, 4), 0.0, 25),
    ((40, 36, 48), (4, 4, 6), 0.02, 20),
])
def test_cbs_equal_iterations(shape, pml, loss, k, device):
    eps = scenes.random_passive_eps(shape, pml, 7, loss=loss)
    g, p = make(shape, LAM / 8, pml, eps, device)
    E, st = p.solve(tol=0.0, max_iter=k, check_every=7)
    assert st.iterations == k and st.status == L.CBS_NOT_CONVERGED
    Eo, res = oc.solve_forward(g, eps, tol=0.0, max_iter=k)
    assert res.iterations == k
    assert rel(E.cpu().numpy(), Eo) < 1e-4
    # scattered part alone
    Es, _ = p.solve(tol=0.0, max_iter=k, scattered=True)
    assert rel(Es.cpu().numpy(), res.E_s) < 1e-4
    assert abs(st.residual - res.history[-1]) < 1e-4 * res.history[-1] + 1e-6


def test_sphere64_equal_iterations_and_converged(device):
    sc = scenes.sphere64()
    g, p = make(sc.shape, sc.pitch, sc.pml, sc.eps_r, device)
    E, st = p.solve(tol=0.0, max_iter=20, check_every=10)
    Eo, res = oc.solve_forward(g, sc.eps_r, tol=0.0, max_iter=20)
    assert rel(E.cpu().numpy(), Eo) < 1e-4
    E, st = p.solve(tol=1e-6, max_iter=5000, check_every=10, history=True)
    assert st.status == L.CBS_OK and st.converged and st.residual <= 1e-6
    Eo, res = oc.solve_forward(g, sc.eps_r, tol=1e-9, max_iter=20000)
    print(f"sphere64: gpu {st.iterations} it (eta {st.residual:.2e}), oracle {res.iterations} it")
    assert rel(E.cpu().numpy(), Eo) < 1e-3
    h = p.history()
    assert len(h) == st.iterations and h[-1] == pytest.approx(st.residual)


def test_sphere64_scattered_field_against_mie(device):
    """The GPU's converged scattered field of the 64^3 sphere scene against the
    Mie series outside the sphere and the absorbing layer: the same
    discretisation-limited agreement the oracle reaches (0.111 at lambda/6)."""
    from oracle import mie
    sc = scenes.sphere64()
    g, p = make(sc.shape, sc.pitch, sc.pml, sc.eps_r, device)
    Es, st = p.solve(tol=1e-6, max_iter=5000, check_every=10, scattered=True)
    Es = Es.cpu().numpy().astype(np.complex128)
    nx, ny, nz = sc.shape
    d = sc.pitch
    c = ((nx - 1) / 2 * d, (ny - 1) / 2 * d, (nz - 1) / 2 * d)
    zz, yy, xx = np.meshgrid(np.arange(nz) * d, np.arange(ny) * d, np.arange(nx) * d, indexing="ij")
    r = np.sqrt((xx - c[0]) ** 2 + (yy - c[1]) ** 2 + (zz - c[2]) ** 2)
    px, py, pz = sc.pml
    inner = np.zeros(r.shape, bool)
    inner[pz + 2:nz - pz - 2, py + 2:ny - py - 2, px + 2:nx - px - 2] = True
    sel = inner & (r > sc.info["radius"] + d)
    k = 2 * np.pi / LAM
    Em = mie.scattered_field(k, sc.info["radius"], sc.info["n_sphere"],
                             np.stack([xx[sel], yy[sel], zz[sel]]), c) * np.exp(1j * k * c[2])
    Eg = np.stack([Es[i][sel] for i in range(3)])
    e = rel(Eg, Em)
    print(f"sphere64 vs Mie: rel-L2 {e:.4f} over {sel.sum()} voxels")
    assert e < 0.12


def test_homogeneous_medium_is_exact(device):
    shape, pml = (16, 12, 20), (2, 2, 4)
    eps = np.ones(shape[::-1], dtype=np.float32)
    g, p = make(shape, LAM / 8, pml, eps, device)
    Es, st = p.solve(tol=0.0, max_iter=12, scattered=True)
    assert torch.count_nonzero(Es).item() == 0
    E, _ = p.solve(tol=0.0, max_iter=12)
    Einc = oc.plane_wave(g)
    assert rel(E.cpu().numpy(), Einc) < 1e-6


def test_uniform_medium_closed_form(device):
    shape = (24, 20, 16)
    eps_c = complex(np.complex64(1.3 + 0.05j))
    eps = np.full(shape[::-1], eps_c, dtype=np.complex64)
    g, p = make(shape, LAM / 8, (0, 0, 0), eps, device)
    S = scenes.random_field(shape, 17, scale=1e13)      # units of k0^2
    for k in (1, 7, 30):
        Ek, _ = closed.uniform_medium(g, eps_c, S.astype(np.complex128), k)
        E, st = p.solve(tol=0.0, max_iter=k, field=to_dev(S, device))
        assert rel(E.cpu().numpy(), Ek) < 1e-4


def test_point_source_adjoint_and_gradient(device):
    shape, pml = (16, 14, 18), (2, 2, 3)
    eps = scenes.random_passive_eps(shape, pml, 23)
    g, p = make(shape, LAM / 8, pml, eps, device)
    r0 = (8, 7, 12)
    E, st = p.solve(tol=1e-7, max_iter=4000)
    Eo, res = oc.solve_forward(g, eps, tol=1e-11, max_iter=40000)
    assert rel(E.cpu().numpy(), Eo) < 1e-3
    Ea, sta = p.adjoint(E_fwd=E, r0=r0, tol=1e-7, max_iter=4000)
    ga = oc.solve_adjoint(g, eps, oc.adjoint_point_source(g, Eo, r0), tol=1e-11, max_iter=40000)
    assert rel(Ea.cpu().numpy(), ga.E_s) < 1e-3
    lo, hi = (2, 2, 3), (14, 12, 15)
    grad = p.gradient(E, Ea, lo, hi, scale=2.0)
    gref = oc.gradient(g, Eo, ga.E_s, lo, hi, scale=2.0)
    assert rel(grad.cpu().numpy(), gref) < 1e-3
    # explicit-amplitude point source equals the field-derived one
    amp = np.conj(Eo[:, r0[2], r0[1], r0[0]])
    Ea2, _ = p.adjoint(r0=r0, amp=amp, tol=1e-7, max_iter=4000)
    assert rel(Ea2.cpu().numpy(), ga.E_s) < 1e-3


def test_field_source_matches_oracle(device):
    shape, pml = (12, 12, 16), (2, 2, 3)
    eps = scenes.random_passive_eps(shape, pml, 31, loss=0.1)
    g, p = make(shape, LAM / 8, pml, eps, device)
    S = scenes.random_field(shape, 32, scale=1e13)
    E, st = p.solve(tol=0.0, max_iter=25, field=to_dev(S, device))
    ref = oc.cbs(g, eps, S.astype(np.complex128), tol=0.0, max_iter=25).E_s
    assert rel(E.cpu().numpy(), ref) < 1e-4


def test_warm_start_continues_the_iteration(device):
    shape, pml = (12, 10, 14), (2, 2, 3)
    eps = scenes.random_passive_eps(shape, pml, 41)
    g, p = make(shape, LAM / 8, pml, eps, device)
    E, _ = p.solve(tol=0.0, max_iter=15)
    E, _ = p.solve(E, tol=0.0, max_iter=10, warm=True)
    Eo, _ = oc.solve_forward(g, eps, tol=0.0, max_iter=25)
    assert rel(E.cpu().numpy(), Eo) < 1e-4


def test_non_finite_warm_start_reports_divergence(device):
    """A warm start from a field holding a NaN makes the residual non-finite:
    the solve stops at its first check with CBS_E_DIVERGED instead of running
    to max_iter, and the plan stays usable (a cold solve afterwards matches
    the oracle)."""
    shape, pml = (12, 10, 14), (2, 2, 3)
    eps = scenes.random_passive_eps(shape, pml, 41)
    g, p = make(shape, LAM / 8, pml, eps, device)
    E, _ = p.solve(tol=0.0, max_iter=15)
    E[1, 5, 4, 3] = complex(float("nan"), 0.0)
    with pytest.raises(L.CbsError) as ei:
        p.solve(E, tol=1e-6, max_iter=500, check_every=10, warm=True)
    assert ei.value.code == L.CBS_E_DIVERGED and "non-finite" in str(ei.value)
    E2, st = p.solve(tol=0.0, max_iter=15)
    Eo, _ = oc.solve_forward(g, eps, tol=0.0, max_iter=15)
    assert st.iterations == 15 and rel(E2.cpu().numpy(), Eo) < 1e-4


def test_repeat_is_bitwise_identical(device):
    sc = scenes.sphere_scene(32, LAM / 6, 0.8e-6, 1.45, 1.0, (4, 4, 6), supersample=4)
    _, p = make(sc.shape, sc.pitch, sc.pml, sc.eps_r, device)
    E1, s1 = p.solve(tol=0.0, max_iter=30)
    E2, s2 = p.solve(tol=0.0, max_iter=30)
    assert torch.equal(E1, E2) and s1.residual == s2.residual
    # a cold start ignores what the output buffer holds
    E3 = torch.full_like(E1, 3.0 - 1.0j)
    E3, s3 = p.solve(E3, tol=0.0, max_iter=30)
    assert torch.equal(E1, E3) and s3.residual == s1.residual
    Ea1, _ = p.adjoint(E_fwd=E1, r0=(16, 16, 20), tol=0.0, max_iter=10)
    Ea2, _ = p.adjoint(E_fwd=E1, r0=(16, 16, 20), E_adj=E3.clone(), tol=0.0, max_iter=10)
    assert torch.equal(Ea1, Ea2)


@pytest.mark.parametrize("bad,frag", [("gain", "gain"), ("layer", "absorbing layer"),
                                      ("nan", "non-finite"), ("huge", "FP32")])
def test_invalid_media_are_rejected(bad, frag, device):
    shape, pml = (8, 8, 8), (2, 2, 2)
    eps = scenes.random_passive_eps(shape, pml, 1, loss=0.1)
    if bad == "gain":
        eps[4, 4, 4] = 1.5 - 0.1j
    elif bad == "layer":
        eps[0, 4, 4] = 1.2
    elif bad == "huge":
        eps[3, 3, 3] = 1e35
    else:
        eps[3, 3, 3] = np.nan
    p = Plan(shape, LAM / 8, LAM, 1.0, pml, device=device)
    with pytest.raises(L.CbsError) as ei:
        p.set_permittivity(to_dev(eps, device))
    assert ei.value.code == L.CBS_E_INVALID and frag in str(ei.value)
    with pytest.raises(L.CbsError) as ei:
        p.solve(max_iter=3)
    assert ei.value.code == L.CBS_E_STATE
