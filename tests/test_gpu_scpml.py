"""The stretched-coordinate absorbing layer (reference [31] of the paper's
simulation-setup paragraph) on the GPU, against the FP64 oracle.

* The layer's operator (L_s - L) v: per-axis matrix products on the GPU, FFT
  derivatives in the oracle (oracle.scpml.delta_apply), on even and odd axes,
  through both forms of A and B: dense (y on 24 x 20 x 32, z on 25 x 27 x 15)
  and the two-launch form of a thin layer, 8p <= n (x and z on 24 x 20 x 32, x
  on 25 x 27 x 15; z in the reflection cases); and at the 275 x 275 x 315
  lens size on fields that vary along one axis only, against the oracle's
  operator on a grid of that axis alone.
* Equal GMRES steps: two restart cycles of GMRES(8) on the CBS-preconditioned
  system, GPU (FP32 fields, FP64 reductions) against scipy's GMRES on the
  oracle's operator (oracle.scpml.gmres_solve).
* Converged: against dense LU of the stretched operator on a tiny grid
  (oracle.scpml.solve_dense) and against the stored FP64 GMRES solution on
  24 x 20 x 32 (tests/golden/make_scpml.py).
* Reflection at normal incidence on the z layers of the 621 x 621 x 261 volume
  (18 voxels of 177 nm) and of the 64^3 sphere case (8 voxels at lambda/6, the
  thickness of its lateral layers), for alpha_max 1.5 (quadratic) and the
  default 0.75 (linear): below the graded potential's by orders of magnitude,
  near the oracle's exact 1D value.
"""

import os

import numpy as np
import pytest
import torch

from oracle import absorber as ab
from oracle import cbs as oc
from oracle import scpml
from paper_2506_15411_amd import libcbs as L
from paper_2506_15411_amd import scenes
from paper_2506_15411_amd.solver import Plan

pytestmark = pytest.mark.gpu
LAM = 1.064e-6
HERE = os.path.dirname(os.path.abspath(__file__))


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel())
                 / np.linalg.norm(np.asarray(b).ravel()))


def plan(shape, pml, device, pitch=LAM / 8, eps=None):
    p = Plan(shape, pitch, LAM, 1.0, pml, device=device, sigma_max=0.0)
    if eps is None:
        eps = np.ones(shape[::-1], dtype=np.float32)
    p.set_permittivity(torch.from_numpy(np.ascontiguousarray(eps)).to(device))
    return p


@pytest.mark.parametrize("shape,pml", [((24, 20, 32), (3, 3, 4)), ((25, 27, 15), (2, 0, 3))])
def test_layer_operator_matches_oracle(shape, pml, device):
    g = oc.Grid(*shape, LAM / 8, LAM, 1.0, pml, sigma_max=0.0)
    rng = np.random.default_rng(7)
    v = (rng.standard_normal((3,) + g.vshape) + 1j * rng.standard_normal((3,) + g.vshape))
    p = plan(shape, pml, device)
    vd = torch.from_numpy(v.astype(np.complex64)).to(device)
    for alpha, order in ((1.5, 2), (3.0, 3)):
        out = p.scpml_operator(vd, alpha, order).cpu().numpy()
        ref = scpml.delta_apply(g, v.astype(np.complex64).astype(np.complex128), alpha, order)
        err = rel(out, ref)
        print(f"{shape} alpha {alpha} order {order}: rel {err:.2e}")
        assert err < 2e-6
    # no stretch: the operator is exactly zero
    assert torch.count_nonzero(p.scpml_operator(vd, 0.0, 2)).item() == 0
    p.close()


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_layer_operator_at_the_lens_size_on_one_axis_fields(axis, device):
    """At the 275 x 275 x 315 size of the 16 um lens (lambda/16: thin 8-voxel x
    and y layers, a thick 48-voxel z layer, in the launch configuration of its
    solves): a field that varies along one axis only has no derivative along
    the other two, so (L_s - L) v is the one-axis operator applied along every
    line, whatever the other layers.  The oracle applies it on a grid of that
    axis alone (2 voxels and no layer on the others); every line of the GPU
    result must match it."""
    shape, pml, pitch = (275, 275, 315), (8, 8, 48), LAM / 16
    n = shape[axis]
    dims, lp = [2, 2, 2], [0, 0, 0]
    dims[axis], lp[axis] = n, pml[axis]
    g1 = oc.Grid(*dims, pitch, LAM, 1.0, tuple(lp), sigma_max=0.0)
    rng = np.random.default_rng(11 + axis)
    line = (rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))).astype(np.complex64)
    bshape = [3, 1, 1, 1]
    bshape[3 - axis] = n                      # field layout [c][z][y][x]
    v1 = np.broadcast_to(line.reshape(bshape), (3,) + g1.vshape).astype(np.complex128)
    p = plan(shape, pml, device, pitch=pitch)
    vd = torch.from_numpy(line).to(device).reshape(bshape).expand((3,) + p.vshape).contiguous()
    for alpha, order in ((0.75, 1), (1.5, 2)):
        ref1 = scpml.delta_apply(g1, v1, alpha, order)
        sel = [slice(None), 0, 0, 0]
        sel[3 - axis] = slice(None)
        ref_line = ref1[tuple(sel)]
        assert np.allclose(ref1, ref_line.reshape(bshape), rtol=0, atol=1e-9 * np.abs(ref1).max())
        out = p.scpml_operator(vd, alpha, order)
        exp = torch.from_numpy(ref_line.astype(np.complex64)).to(device).reshape(bshape)
        num = torch.linalg.vector_norm((out - exp).to(torch.complex128)).item()
        den = torch.linalg.vector_norm(exp.expand_as(out).to(torch.complex128)).item()
        print(f"axis {axis} (n {n}, layer {pml[axis]}), alpha {alpha} order {order}: "
              f"rel {num / den:.2e} over {out.numel() // 3} voxels")
        assert num / den < 5e-6
        del out, exp
    p.close()


def test_equal_gmres_steps_match_oracle(device):
    shape, pml = (24, 20, 32), (3, 3, 4)
    eps = scenes.random_passive_eps(shape, pml, 132, loss=0.02)
    g = oc.Grid(*shape, LAM / 8, LAM, 1.0, pml, sigma_max=0.0)
    p = plan(shape, pml, device, eps=eps)
    for steps in (8, 16):
        E, st = p.solve_scpml(alpha_max=1.5, order=2, restart=8, tol=0.0, max_iter=steps,
                              scattered=True)
        assert st.status == L.CBS_NOT_CONVERGED and st.iterations == steps
        Eo, res = scpml.gmres_solve(g, eps, oc.plane_wave_source(g, eps), 1.5, rtol=1e-30,
                                    restart=8, maxiter=steps // 8, require_convergence=False)
        err = rel(E.cpu().numpy(), Eo)
        print(f"{steps} GMRES steps: field rel {err:.2e}, residual gpu {st.residual:.4e} "
              f"oracle {res:.4e}")
        assert err < 1e-5
        assert abs(st.residual - res) < 1e-4 * res
    p.close()


@pytest.mark.parametrize("kind", ["oblique plane wave", "point source"])
def test_other_sources_at_equal_gmres_steps(kind, device):
    """The stretched-layer solve with an oblique p-polarised plane wave and with
    a point source (every source kind goes through the same first CBS step),
    12 GMRES(6) steps against the oracle's GMRES on the same source."""
    shape, pml = (24, 20, 32), (3, 3, 4)
    eps = scenes.random_passive_eps(shape, pml, 133, loss=0.02)
    g = oc.Grid(*shape, LAM / 8, LAM, 1.0, pml, sigma_max=0.0)
    p = plan(shape, pml, device, eps=eps)
    if kind == "point source":
        r0, amp = (11, 9, 17), (g.k0 ** 2, 0.5j * g.k0 ** 2, 0.0)
        S = oc.point_source(g, r0, amp)
        E, st = p.solve_scpml(alpha_max=0.75, order=1, restart=6, tol=0.0, max_iter=12,
                              point=(r0, amp))
    else:
        d = (0.3, 0.2)
        sx, sy = d
        cz, st_ = np.sqrt(1 - sx * sx - sy * sy), np.hypot(sx, sy)
        pol = (cz * sx / st_, cz * sy / st_, -st_)
        S = oc.plane_wave_source(g, eps, pol, d)
        E, st = p.solve_scpml(alpha_max=0.75, order=1, restart=6, tol=0.0, max_iter=12,
                              scattered=True, pol=pol, direction=d)
    assert st.status == L.CBS_NOT_CONVERGED and st.iterations == 12
    Eo, res = scpml.gmres_solve(g, eps, S, 0.75, 1, rtol=1e-30, restart=6, maxiter=2,
                                require_convergence=False)
    err = rel(E.cpu().numpy(), Eo)
    print(f"{kind}: 12 GMRES steps, field rel {err:.2e}, residual gpu {st.residual:.4e} "
          f"oracle {res:.4e}")
    assert err < 1e-5
    assert abs(st.residual - res) < 1e-4 * res
    p.close()


def test_converged_matches_dense_lu(device):
    shape, pml = (8, 8, 12), (2, 2, 3)
    eps = np.ones(shape[::-1], dtype=np.float32)
    eps[3:9, 2:6, 2:6] = 2.1
    g = oc.Grid(*shape, LAM / 6, LAM, 1.0, pml, sigma_max=0.0)
    Ed = scpml.solve_dense(g, eps, oc.plane_wave_source(g, eps), 2.0)
    p = plan(shape, pml, device, pitch=LAM / 6, eps=eps)
    E, st = p.solve_scpml(alpha_max=2.0, order=2, restart=30, tol=1e-6, max_iter=3000,
                          scattered=True, history=True)
    assert st.status == L.CBS_OK and st.converged and st.residual <= 1e-6
    h = p.history()
    assert len(h) == st.iterations and h[-1] <= 1.5e-6
    err = rel(E.cpu().numpy(), Ed)
    print(f"8x8x12: {st.iterations} steps, residual {st.residual:.2e}, field rel {err:.2e}")
    assert err < 1e-5
    # the total field adds the incident wave
    Et, _ = p.solve_scpml(alpha_max=2.0, order=2, restart=30, tol=1e-6, max_iter=3000)
    assert rel(Et.cpu().numpy(), Ed + oc.plane_wave(g)) < 1e-5
    p.close()


def test_converged_matches_fp64_fixture(device):
    gd = np.load(os.path.join(HERE, "golden", "scpml_24x20x32.npz"))
    shape, pml = tuple(int(v) for v in gd["shape"]), tuple(int(v) for v in gd["pml"])
    eps = scenes.random_passive_eps(shape, pml, int(gd["seed"]), loss=0.02)
    p = plan(shape, pml, device, eps=eps)
    E, st = p.solve_scpml(alpha_max=float(gd["alpha_max"]), order=int(gd["order"]), restart=40,
                          tol=1e-6, max_iter=4000, scattered=True)
    assert st.status == L.CBS_OK
    err = rel(E.cpu().numpy(), gd["E_s"])
    print(f"24x20x32: {st.iterations} GMRES steps, residual {st.residual:.2e}, "
          f"field rel to the FP64 fixture {err:.2e} (fixture residual {float(gd['residual']):.1e})")
    assert err < 5e-5
    p.close()


@pytest.mark.parametrize("alpha,order", [(1.5, 2), (0.75, 1)])
@pytest.mark.parametrize("case", ["621x621x261 z layer", "64^3 lateral thickness"])
def test_reflection_below_graded_potential(case, alpha, order, device):
    nz, pitch, pz = {"621x621x261 z layer": (261, 177e-9, 18),
                     "64^3 lateral thickness": (64, LAM / 6, 8)}[case]
    shape, pml = (4, 4, nz), (0, 0, pz)
    g = oc.Grid(*shape, pitch, LAM, 1.0, pml, sigma_max=0.0)
    z_src = pz + 6
    S = ab.oblique_source(g, 0, "s", z_src, amp=g.k0 ** 2)
    Sd = torch.from_numpy(S.astype(np.complex64)).to(device)
    p = plan(shape, pml, device, pitch=pitch)
    E, st = p.solve_scpml(alpha_max=alpha, order=order, restart=40, tol=2e-7, max_iter=4000,
                          field=Sd)
    assert st.status == L.CBS_OK
    R_s, _ = ab.reflection_from_field(g, E.cpu().numpy().astype(np.complex128), 0, "s", z_src)
    R_1d, _ = scpml.reflection_normal(nz, pitch, LAM, pz, alpha, order)
    R_graded, _ = ab.reflection_normal(nz, pitch, LAM, pz)
    print(f"{case}, alpha {alpha} order {order}: R stretched gpu {R_s:.2e} (oracle 1D "
          f"{R_1d:.2e}, {st.iterations} steps), graded potential {R_graded:.2e}")
    assert R_s < R_graded / 100
    # at R ~ 1e-11 the FP32 field resolves the returning wave to about 1e-1 of itself
    assert abs(R_s - R_1d) <= 0.3 * R_1d + 1e-12
    p.close()


def test_rejects_a_plan_with_a_graded_potential(device):
    p = Plan((8, 8, 12), LAM / 6, LAM, 1.0, (2, 2, 3), device=device)
    p.set_permittivity(torch.ones((12, 8, 8), dtype=torch.float32, device=device))
    with pytest.raises(L.CbsError) as e:
        p.solve_scpml(max_iter=5)
    assert e.value.code == L.CBS_E_STATE
    p.close()
    q = plan((8, 8, 12), (2, 2, 3), device)
    with pytest.raises(ValueError):
        q.solve_scpml(restart=65, max_iter=5)
    q.close()
