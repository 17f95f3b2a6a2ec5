"""The allocation-free entry point cbs_solve_static (scratch in a static device
array) against the plan-based cbs_solve on the same inputs: three calls in a
row on one device, each smaller than the one before, with plane-wave, point
and field sources.  The two entry points run the same kernels in the same
order, so the fields must be bit-identical and the iteration counts equal;
the first case is also checked against the FP64 oracle at equal iterations."""

import numpy as np
import pytest
import torch

from oracle import cbs as oc
from paper_2506_15411_amd import libcbs as L
from paper_2506_15411_amd import scenes
from paper_2506_15411_amd.solver import Plan

pytestmark = pytest.mark.gpu
LAM = 1.064e-6


def static_solve(shape, pitch, pml, eps, src, opts, device):
    E = torch.full((3,) + tuple(shape[::-1]), float("nan"), dtype=torch.complex64, device=device)
    stream = torch.cuda.current_stream(device).cuda_stream
    dtype = L.CBS_C64 if eps.dtype == torch.complex64 else L.CBS_F32
    rc, st = L.cbs_solve_static(*shape, pitch, LAM, 1.0, pml, eps.data_ptr(), dtype, src,
                                E.data_ptr(), opts, stream)
    return E, rc, st


def test_static_solve_matches_plan_solve(device):
    sc = scenes.sphere64()
    s2, p2 = (20, 18, 24), (3, 2, 3)
    s3, p3 = (16, 14, 18), (2, 2, 3)
    cases = [
        (sc.shape, sc.pitch, sc.pml, sc.eps_r, None, (1e-6, 5000, 10, 0)),
        (s2, LAM / 8, p2, scenes.random_passive_eps(s2, p2, 5, loss=0.02), None,
         (0.0, 37, 7, L.CBS_RETURN_SCATTERED)),
        (s3, LAM / 8, p3, scenes.random_passive_eps(s3, p3, 6), "point", (1e-6, 3000, 10, 0)),
    ]
    for n, (shape, pitch, pml, eps_np, kind, (tol, mx, every, flags)) in enumerate(cases):
        eps = torch.from_numpy(eps_np).to(device)
        opts = L.cbs_opts(tol, mx, every, flags)
        src = None
        if kind == "point":
            src = L.cbs_source()
            src.kind = L.CBS_SRC_POINT
            for c, v in enumerate((8, 7, 12)):
                src.r0[c] = v
            src.amp[0][0], src.amp[1][1], src.amp[2][0] = 1.0e12, -0.5e12, 0.25e12
        p = Plan(shape, pitch, LAM, 1.0, pml, device=device)
        p.set_permittivity(eps)
        Eref = p.new_field()
        rc_ref, st_ref = L.cbs_solve(p.handle, src, Eref.data_ptr(), opts)
        torch.cuda.synchronize()
        E, rc, st = static_solve(shape, pitch, pml, eps, src, opts, device)
        torch.cuda.synchronize()
        print(f"case {n} {shape}: static {st.iterations} it, plan {st_ref.iterations} it, "
              f"eta {st.residual:.3e}")
        assert rc == rc_ref and st.iterations == st_ref.iterations
        assert st.residual == st_ref.residual and st.eps_shift == st_ref.eps_shift
        assert torch.equal(E, Eref)
        if n == 1:
            g = oc.Grid(*shape, pitch, LAM, 1.0, pml)
            ref = oc.cbs(g, eps_np, oc.plane_wave_source(g, eps_np), tol=0.0, max_iter=mx)
            err = np.linalg.norm(E.cpu().numpy() - ref.E_s) / np.linalg.norm(ref.E_s)
            assert err < 1e-4
        p.close()


def test_static_solve_rejects_grids_beyond_its_scratch(device):
    shape = (275, 275, 315)
    assert L.cbs_plan_workspace_bytes(*shape) > L.CBS_STATIC_SCRATCH_BYTES
    eps = torch.ones(shape[::-1], dtype=torch.float32, device=device)
    E = torch.zeros((3,) + shape[::-1], dtype=torch.complex64, device=device)
    with pytest.raises(L.CbsError) as ei:
        L.cbs_solve_static(*shape, LAM / 16, LAM, 1.0, (8, 8, 48), eps.data_ptr(), L.CBS_F32,
                           None, E.data_ptr(), L.cbs_opts(1e-4, 10, 10, 0),
                           torch.cuda.current_stream(device).cuda_stream)
    assert ei.value.code == L.CBS_E_WORKSPACE and "static scratch" in str(ei.value)
