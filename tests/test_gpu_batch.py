"""Batched multi-illumination solves (cbs_solve_batch) and oblique plane waves.

* Three illuminations of one medium -- x- and y-polarised at normal incidence
  and a p-polarised wave at oblique incidence -- in one batch: at equal
  iteration counts each field equals the single solve of its source (bit for
  bit where both run the same x-pass instantiation), and each matches the
  FP64 oracle's plane wave of that polarisation and direction (equal
  iterations 1e-4, converged 1e-3).
* The batch stops when its largest residual reaches tol; every illumination's
  own residual is reported.
"""

import math

import numpy as np
import pytest
import torch

from oracle import cbs as oc
from paper_2506_15411_amd import libcbs as L
from paper_2506_15411_amd import scenes
from paper_2506_15411_amd.solver import Plan

pytestmark = pytest.mark.gpu
LAM = 1.064e-6


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel())
                 / np.linalg.norm(np.asarray(b).ravel()))


def p_polarised(direction):
    """a unit polarisation in the plane of incidence, transverse to k"""
    sx, sy = direction
    cz = math.sqrt(1 - sx * sx - sy * sy)
    st = math.hypot(sx, sy)
    ux, uy = sx / st, sy / st
    return (cz * ux, cz * uy, -st)


ILLUM = [((1, 0, 0), (0.0, 0.0)), ((0, 1, 0), (0.0, 0.0)),
         (p_polarised((0.3, 0.2)), (0.3, 0.2))]


def setup(device, shape=(24, 20, 32), pml=(3, 3, 4), seed=120):
    eps = scenes.random_passive_eps(shape, pml, seed, loss=0.02)
    g = oc.Grid(*shape, LAM / 8, LAM, 1.0, pml)
    p = Plan(shape, LAM / 8, LAM, 1.0, pml, device=device)
    p.set_permittivity(torch.from_numpy(eps).to(device))
    return g, p, eps


def test_batch_equals_single_solves_and_oracle(device):
    g, p, eps = setup(device)
    k = 25
    Eb, sts = p.solve_batch(ILLUM, tol=0.0, max_iter=k, check_every=7)
    assert all(s.iterations == k and s.status == L.CBS_NOT_CONVERGED for s in sts)
    for b, (pol, d) in enumerate(ILLUM):
        E1, s1 = p.solve(tol=0.0, max_iter=k, pol=pol, direction=d)
        if d == (0.0, 0.0):
            # a normal-incidence wave inside a batch that holds an oblique one runs
            # the x pass compiled with the per-element x phase (exactly 1 here):
            # the same arithmetic up to the compiler's FMA contraction
            assert rel(Eb[b].cpu().numpy(), E1.cpu().numpy()) < 1e-6, b
        else:
            assert torch.equal(Eb[b], E1), b
            assert s1.residual == sts[b].residual
        Eo, res = oc.solve_forward(g, eps, tol=0.0, max_iter=k, pol=pol, direction=d)
        assert rel(E1.cpu().numpy(), Eo) < 1e-4, b
        assert abs(sts[b].residual - res.eta) < 1e-4 * res.eta
    p.close()


def test_normal_incidence_batch_is_bit_identical_to_single_solves(device):
    g, p, eps = setup(device, seed=122)
    illum = ILLUM[:2]
    Eb, sts = p.solve_batch(illum, tol=0.0, max_iter=20, check_every=6)
    for b, (pol, d) in enumerate(illum):
        E1, s1 = p.solve(tol=0.0, max_iter=20, pol=pol, direction=d)
        assert torch.equal(Eb[b], E1), b
        assert s1.residual == sts[b].residual
    p.close()


def test_batch_converged_against_oracle(device):
    g, p, eps = setup(device, seed=121)
    Eb, sts = p.solve_batch(ILLUM, tol=1e-6, max_iter=5000)
    assert all(s.status == L.CBS_OK for s in sts)
    assert max(s.residual for s in sts) <= 1e-6
    assert all(s.converged for s in sts)
    for b, (pol, d) in enumerate(ILLUM):
        Eo, _ = oc.solve_forward(g, eps, tol=1e-11, max_iter=40000, pol=pol, direction=d)
        assert rel(Eb[b].cpu().numpy(), Eo) < 1e-3, b
    # the residual history is the largest of the illuminations' residuals
    Eb2, sts2 = p.solve_batch(ILLUM, tol=1e-6, max_iter=5000, history=True)
    h = p.history()
    assert len(h) == sts2[0].iterations and h[-1] == max(s.residual for s in sts2)
    assert torch.equal(Eb, Eb2)
    p.close()


def test_oblique_plane_wave_in_a_homogeneous_medium_is_exact(device):
    """With eps_r = n_bg^2 everywhere the scattered field of any plane wave is
    zero at every iteration, so the total field is the incident wave itself."""
    shape, pml = (24, 20, 32), (3, 3, 4)
    p = Plan(shape, LAM / 8, LAM, 1.0, pml, device=device)
    p.set_permittivity(torch.ones(shape[::-1], dtype=torch.float32, device=device))
    pol, d = ILLUM[2]
    Es, st = p.solve(tol=0.0, max_iter=5, pol=pol, direction=d, scattered=True)
    assert torch.count_nonzero(Es).item() == 0
    E, _ = p.solve(tol=0.0, max_iter=5, pol=pol, direction=d)
    g = oc.Grid(*shape, LAM / 8, LAM, 1.0, pml)
    assert rel(E.cpu().numpy(), oc.plane_wave(g, pol, d)) < 1e-6
    p.close()


def test_batch_rejects_bad_arguments(device):
    g, p, eps = setup(device)
    with pytest.raises(ValueError):
        p.solve_batch([(None, None)] * 9, tol=0.0, max_iter=2)
    with pytest.raises(L.CbsError):
        p.solve_batch([((1, 0, 0), (0.8, 0.7))], tol=0.0, max_iter=2)   # evanescent
    p.close()
