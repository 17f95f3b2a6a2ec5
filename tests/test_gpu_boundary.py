"""GPU tests of the C ABI's less-travelled entry points and options, against the
FP64 oracle or against the library's own blocking solves:

* the device-side stopping rule at y lengths whose y-pass work-groups are not a
  power of two wide (192 and 320 threads): stopping iteration and residual
  history against the oracle, and bit-identical histories whatever the host's
  polling interval (the lagged and the quantum-end reductions agree);
* cbs_batch_step over three plans of different grids against solo solves;
* a non-default absorbing profile (order 3, sigma_max 0.5) and shift factor 1.3;
* one Green's-operator application for every registered axis length on every
  axis it is registered for;
* the conjugated field source (FIELD_CONJ) of the adjoint of a general loss.
"""

import numpy as np
import pytest
import torch

from oracle import cbs as oc
from paper_2506_15411_amd import libcbs as L
from paper_2506_15411_amd import scenes
from paper_2506_15411_amd.autograd import NotConvergedError, cbs_solve
from paper_2506_15411_amd.solver import Plan

pytestmark = pytest.mark.gpu
LAM = 1.064e-6


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def to_dev(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def pick_stop(hist, first):
    """An iteration k >= first at which a tolerance between eta_{k-1} and eta_k
    stops the oracle, with a margin the FP32 residual cannot cross."""
    for k in range(first, len(hist) + 1):
        a, b = hist[k - 2], hist[k - 1]
        if a / b > 1.01 and b < min(hist[:k - 1]) / 1.01:
            return k, float(np.sqrt(a * b))
    raise AssertionError("no usable stopping point")


@pytest.mark.parametrize("shape", [(12, 18, 16), (10, 20, 9), (8, 315, 6)])
def test_stopping_rule_at_non_power_of_two_y_passes(shape, device):
    pml = (2, 2, 2)
    eps = scenes.random_passive_eps(shape, pml, 41, loss=0.02)
    g = oc.Grid(*shape, LAM / 8, LAM, 1.0, pml)
    ref = oc.cbs(g, eps, oc.plane_wave_source(g, eps), tol=0.0, max_iter=60)
    k, tol = pick_stop(ref.history, 12)
    p = Plan(shape, LAM / 8, LAM, 1.0, pml, device=device)
    p.set_permittivity(to_dev(eps, device))
    hists = []
    for every in (1, 7, 10, 64):
        E, st = p.solve(tol=tol, max_iter=200, check_every=every, history=True)
        assert st.status == L.CBS_OK and st.iterations == k, (every, st)
        hists.append(np.array(p.history()))
    for h in hists[1:]:
        assert np.array_equal(h, hists[0])
    h = hists[0]
    ho = np.array(ref.history[:k])
    assert np.all(np.abs(h - ho) <= 1e-4 * ho + 1e-7)
    Eo, _ = oc.solve_forward(g, eps, tol=0.0, max_iter=k)
    assert rel(E.cpu().numpy(), Eo) < 1e-4
    p.close()


def test_batch_step_matches_solo_solves(device):
    grids = [((16, 16, 16), (2, 2, 3)), ((20, 18, 24), (3, 2, 3)), ((12, 10, 9), (2, 2, 2))]
    eps = [to_dev(scenes.random_passive_eps(s, pm, 50 + i, loss=0.01), device)
           for i, (s, pm) in enumerate(grids)]
    torch.cuda.synchronize()
    plans = [Plan(s, LAM / 8, LAM, 1.0, pm, device=device, stream=torch.cuda.Stream(device))
             for s, pm in grids]
    for p, e in zip(plans, eps):
        p.set_permittivity(e)
    solo = []
    for p in plans:
        E, st = p.solve(tol=1e-6, max_iter=2000, check_every=10)
        p.stream.synchronize()
        solo.append((E.clone(), st.iterations))
        p.stream.synchronize()
    fields = [p.new_field() for p in plans]
    torch.cuda.synchronize()
    for p, E in zip(plans, fields):
        p.begin(E, tol=1e-6, max_iter=2000)
    done = [False] * 3
    steps = 0
    while not all(done):
        out = L.cbs_batch_step([p.handle for p in plans], 7)
        done = [d or o for d, o in zip(done, out)]
        steps += 1
        assert steps < 1000
    for p, E, (Es, its) in zip(plans, fields, solo):
        st = p.end()
        p.stream.synchronize()
        assert st.status == L.CBS_OK and st.iterations == its
        assert torch.equal(E, Es)
    for p in plans:
        p.close()


def test_non_default_absorber_and_shift(device):
    shape, pml = (20, 18, 24), (3, 3, 4)
    eps = scenes.random_passive_eps(shape, pml, 61, loss=0.03)
    kw = dict(pml_order=3, sigma_max=0.5, shift_factor=1.3)
    g = oc.Grid(*shape, LAM / 8, LAM, 1.0, pml, **kw)
    p = Plan(shape, LAM / 8, LAM, 1.0, pml, device=device, **kw)
    p.set_permittivity(to_dev(eps, device))
    assert p.eps_shift == pytest.approx(oc.potentials(g, eps).eps, rel=1e-12)
    E, st = p.solve(tol=0.0, max_iter=30, scattered=True)
    ref = oc.cbs(g, eps, oc.plane_wave_source(g, eps), tol=0.0, max_iter=30)
    assert rel(E.cpu().numpy(), ref.E_s) < 1e-4
    E, st = p.solve(tol=1e-6, max_iter=5000)
    assert st.status == L.CBS_OK
    Eo, _ = oc.solve_forward(g, eps, tol=1e-11, max_iter=40000)
    assert rel(E.cpu().numpy(), Eo) < 1e-3
    p.close()


def registered_lengths():
    return [n for n in range(2, 1024) if L.cbs_axis_supported(0, n)]


@pytest.mark.parametrize("n", registered_lengths())
def test_green_operator_every_axis_length(n, device):
    for axis in range(3):
        if not L.cbs_axis_supported(axis, n):
            assert axis == 2 and n == 621
            continue
        shape = [6, 5, 7]
        shape[axis] = n
        shape = tuple(shape)
        eps = scenes.random_passive_eps(shape, (0, 0, 0), 70 + axis, loss=0.05)
        g = oc.Grid(*shape, LAM / 8, LAM, 1.0, (0, 0, 0))
        p = Plan(shape, LAM / 8, LAM, 1.0, (0, 0, 0), device=device)
        p.set_permittivity(to_dev(eps, device))
        W = scenes.random_field(shape, 80 + axis)
        out = p.apply_green(to_dev(W, device))
        ref = oc.green_apply(g, W.astype(np.complex128), oc.potentials(g, eps).kt2)
        err = rel(out.cpu().numpy(), ref)
        p.close()
        assert err < 5e-6, (shape, err)


def test_conjugated_field_source(device):
    shape, pml = (16, 14, 18), (2, 2, 3)
    eps = scenes.random_passive_eps(shape, pml, 90)
    g = oc.Grid(*shape, LAM / 8, LAM, 1.0, pml)
    p = Plan(shape, LAM / 8, LAM, 1.0, pml, device=device)
    p.set_permittivity(to_dev(eps, device))
    F = scenes.random_field(shape, 91, scale=(2 * np.pi / LAM) ** 2)
    Fd = to_dev(F, device)
    Ea, st = p.adjoint(field=Fd, conj=True, tol=0.0, max_iter=25)
    Eb, _ = p.adjoint(field=torch.conj(Fd).resolve_conj(), tol=0.0, max_iter=25)
    assert torch.equal(Ea, Eb)
    ref = oc.solve_adjoint(g, eps, np.conj(F.astype(np.complex128)), tol=0.0, max_iter=25)
    assert rel(Ea.cpu().numpy(), ref.E_s) < 1e-4
    with pytest.raises(ValueError):
        p.adjoint(field=torch.conj(Fd), tol=0.0, max_iter=2)
    p.close()


def test_autograd_reports_unconverged_solves(device):
    shape, pml = (16, 14, 18), (2, 2, 3)
    eps = scenes.random_passive_eps(shape, pml, 92)
    p = Plan(shape, LAM / 8, LAM, 1.0, pml, device=device)
    e = to_dev(eps, device).requires_grad_(True)
    with pytest.raises(NotConvergedError):
        cbs_solve(e, p, tol=1e-9, max_iter=3)
    E = cbs_solve(e, p, tol=1e-9, max_iter=3, strict=False)
    assert p.last_forward_stats.status == L.CBS_NOT_CONVERGED
    (E.abs() ** 2).sum().backward()
    assert p.last_adjoint_stats.iterations == 3
    p.close()
