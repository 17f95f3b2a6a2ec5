"""Writes the converged-solution fixtures of the GPU parity tests.

Calls only the FP64 oracle (``oracle/``) and the seeded scene generator
(``paper_2506_15411_amd.scenes``, geometry and random numbers only).  Nothing
here reads anything the HIP library produced.

    python tests/golden/make_converged.py lens16          # 275 x 275 x 315 zone plate
    python tests/golden/make_converged.py lens16_grad     # the same with its design slab
    python tests/golden/make_converged.py sphere64_fd     # 64^3 finite-difference gradient

lens16       The 16 um zone plate of the Fig. 1 benchmark (275 x 275 x 315 at
             lambda/16): the FP64 CBS iteration run until eta <= 1e-6.  Past
             eta ~ 1e-4 the iteration of this lens contracts by only about 0.997
             per step (weakly damped modes between its thin lateral absorbing
             layers), so the field's distance to E_s* = A^-1 S is about
             eta rho / (1 - rho); the measured contraction rho over the last 100
             steps and that estimate are stored with the fields.  (GMRES on the
             CBS-preconditioned system, oracle.dense.cbs_gmres_solve, gains about
             3x per operator application on this tail: not enough to reach 1e-9
             either.)  Stored: the scattered field on the focal plane z = z0 and
             on the xz plane through the axis, at 4096 voxels drawn with
             default_rng(7), and the whole-volume norm.
lens16_grad  The same lens with its seed-0 design slab (the adjoint-gradient
             case, objective |E(r0)|^2; objective and optimisation paragraphs):
             forward and adjoint solves as above (the adjoint as the sum of the
             three unit-dipole solves at r0 weighted by conj(E(r0)), which
             lens16_dipole0..2 can compute beforehand), the gradient
             2 k0^2 Re(E_adj . E) over the slab at 4096 slab voxels
             (default_rng(8)), on the slab's middle plane, and its norm.
sphere64_fd  The 64^3 sphere at lambda/6 with a 6-voxel seeded design slab: the
             adjoint gradient and FP64 central differences (h = 1e-3, solves
             warm-started from the base field to eta <= 1e-12) at 32 slab voxels
             drawn without replacement with default_rng(1).

Long solves run in chunks of 50 iterations (each chunk continues exactly where
the previous stopped: the iteration depends only on the current field) and
write a checkpoint to the directory named by --ckpt, so an interrupted run
resumes.  --tol (default 1e-6) is the eta at which the lens solves stop; with
--gmres-restart R --gmres-cycles C the CBS iterate is then refined by C cycles
of GMRES(R) on the same preconditioned system (oracle.dense.cbs_gmres_solve),
which removes the slow tail faster than the iteration does.  A fixture stores
the eta it reached and the error estimate above, and the GPU tests compare
against it within the larger of 1e-3 and three times that estimate.
"""

from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import cbs as oc  # noqa: E402
from oracle import dense as _dense  # noqa: E402
from paper_2506_15411_amd import scenes  # noqa: E402

TOL = 1e-6
CHUNK = 50


def log(*a):
    print(time.strftime("%H:%M:%S"), *a, flush=True)


GMRES = {"restart": 0, "cycles": 0}   # set from --gmres-restart / --gmres-cycles


def converge(g, eps, S, tag, ckpt_dir, tol=TOL, max_iter=20000):
    """FP64 CBS from E_s = 0 until eta <= tol, in resumable chunks; then, if
    requested, oracle.dense.cbs_gmres_solve from that iterate (same
    preconditioned system, so its relative residual is eta's quantity)."""
    path = os.path.join(ckpt_dir, f"{tag}.npz") if ckpt_dir else None
    E, done, hist = None, 0, []
    if path and os.path.exists(path):
        z = np.load(path)
        E, done, hist = z["E"], int(z["iterations"]), list(z["history"])
        log(f"{tag}: resuming at iteration {done}, eta {hist[-1]:.3e}")
    eta = hist[-1] if hist else math.inf
    while eta > tol and done < max_iter:
        res = oc.cbs(g, eps, S, tol=tol, max_iter=min(CHUNK, max_iter - done), E0=E)
        E, done, eta = res.E_s, done + res.iterations, res.eta
        hist += res.history
        log(f"{tag}: iteration {done}, eta {eta:.3e}")
        if path:
            np.savez(path + ".tmp.npz", E=E, iterations=done, history=np.array(hist))
            os.replace(path + ".tmp.npz", path)
    if eta > tol:
        raise RuntimeError(f"{tag}: eta {eta:.3e} > {tol} after {done} iterations")
    h = np.array(hist)
    # contraction per iteration over the last 100 steps, and the distance to the
    # solution it implies (the slowest mode dominates the update)
    rho = float((h[-1] / h[-101]) ** (1.0 / 100)) if len(h) > 100 else float("nan")
    err = float(h[-1] * rho / (1.0 - rho)) if rho < 1 else float("inf")
    log(f"{tag}: {done} iterations, eta {h[-1]:.3e}, contraction {rho:.5f}, "
        f"estimated relative error {err:.1e}")
    if GMRES["restart"] > 0 and GMRES["cycles"] > 0:
        E, h, err = gmres_finish(g, eps, S, tag, E, h, rho)
    return E, done, h, rho, err


def gmres_finish(g, eps, S, tag, E, h, rho):
    """GMRES(restart) for a fixed number of cycles from the CBS iterate E.  The
    preconditioned residual r = gamma G S - gamma (I - G V) E is the CBS update,
    so |r| / |E| continues the eta history; the error estimate keeps the CBS
    tail's contraction rho: |r| / |E| * rho / (1 - rho)."""
    pot = oc.potentials(g, eps)
    b = pot.gamma[None] * oc.green_apply(g, np.asarray(S, dtype=np.complex128), pot.kt2)
    nb = float(np.linalg.norm(b))
    del b
    t0 = time.time()

    def cb(k, r):
        if k % 5 == 0:
            log(f"{tag}: GMRES step {k}, residual {r * nb / np.linalg.norm(E):.3e} of |E| "
                f"({time.time() - t0:.0f} s)")

    E = _dense.cbs_gmres_solve(g, eps, S, rtol=1e-14, restart=GMRES["restart"],
                               maxiter=GMRES["cycles"], x0=E, callback=cb,
                               require_convergence=False)
    E1 = oc.cbs(g, eps, S, tol=0.0, max_iter=1, E0=E)   # one CBS step: its eta is |r| / |E|
    eta = float(E1.eta)
    del E1
    err = float(eta * rho / (1.0 - rho)) if rho < 1 else float("inf")
    log(f"{tag}: after {GMRES['restart'] * GMRES['cycles']} GMRES steps eta {eta:.3e}, "
        f"estimated relative error {err:.1e}")
    return E, np.append(h, eta), err


def lens16(ckpt, tol=TOL):
    sc = scenes.zoneplate16()
    g = oc.Grid(*sc.shape, sc.pitch, sc.lambda0, sc.n_bg, sc.pml)
    oc.validate(g, sc.eps_r)
    E, its, hist, rho, err = converge(g, sc.eps_r, oc.plane_wave_source(g, sc.eps_r),
                                      "lens16_fwd", ckpt, tol)
    nx, ny, nz = sc.shape
    x0, y0, z0 = sc.r0
    rng = np.random.default_rng(7)
    vz, vy, vx = rng.integers(0, nz, 4096), rng.integers(0, ny, 4096), rng.integers(0, nx, 4096)
    out = os.path.join(HERE, "lens16_converged.npz")
    np.savez_compressed(
        out, shape=np.array(sc.shape), r0=np.array(sc.r0), tol=tol, iterations=its,
        eta=hist[-1], contraction=rho, error_estimate=err,
        eps_shift=oc.potentials(g, sc.eps_r).eps,
        focal_plane=E[:, z0].astype(np.complex64),          # [3, ny, nx] at z = z0
        xz_plane=E[:, :, y0, :].astype(np.complex64),       # [3, nz, nx] at y = y0
        vox=np.stack([vx, vy, vz]), vox_E=E[:, vz, vy, vx],  # complex128 [3, 4096]
        norm=float(np.sqrt(np.sum(np.abs(E) ** 2))))
    log(f"wrote {out}: {its} iterations, eta {hist[-1]:.3e}")


def lens16_grad(ckpt, tol=TOL):
    sc = scenes.zoneplate16_design(0)
    g = oc.Grid(*sc.shape, sc.pitch, sc.lambda0, sc.n_bg, sc.pml)
    oc.validate(g, sc.eps_r)
    Es, it1, h1, rho1, err1 = converge(g, sc.eps_r, oc.plane_wave_source(g, sc.eps_r),
                                       "lens16d_fwd", ckpt, tol)
    E = oc.plane_wave(g) + Es
    del Es
    # the adjoint source conj(E(r0)) delta_{r0} is a sum of three unit dipoles at
    # r0, so E_adj = sum_c conj(E_c(r0)) A^-1 (delta_{r0} e_c); the dipole solves
    # do not depend on the forward field and can run beforehand (lens16_dipole)
    ix, iy, iz = sc.r0
    w = np.conj(E[:, iz, iy, ix])
    Ea = np.zeros_like(E)
    it2, rho2, err2, eta2 = 0, 0.0, 0.0, 0.0
    for c in range(3):
        Gc, itc, hc, rhoc, errc = dipole(g, sc, c, ckpt, tol)
        Ea += w[c] * Gc
        del Gc
        it2, rho2, err2, eta2 = max(it2, itc), max(rho2, rhoc), max(err2, errc), max(eta2, hc[-1])
    h2 = [eta2]
    lo, hi = sc.design_box
    grad = oc.gradient(g, E, Ea, lo, hi, scale=2.0)          # [bz, by, bx]
    bz, by, bx = grad.shape
    rng = np.random.default_rng(8)
    vz, vy, vx = rng.integers(0, bz, 4096), rng.integers(0, by, 4096), rng.integers(0, bx, 4096)
    out = os.path.join(HERE, "lens16_gradient_converged.npz")
    np.savez_compressed(
        out, shape=np.array(sc.shape), r0=np.array(sc.r0), box_lo=np.array(lo),
        box_hi=np.array(hi), tol=tol, iterations=np.array([it1, it2]),
        eta=np.array([h1[-1], h2[-1]]), contraction=np.array([rho1, rho2]),
        error_estimate=np.array([err1, err2]), objective=oc.focal_objective(E, sc.r0),
        vox=np.stack([vx, vy, vz]), vox_grad=grad[vz, vy, vx],
        mid_plane=grad[bz // 2].astype(np.float32), norm=float(np.linalg.norm(grad)))
    log(f"wrote {out}")


def dipole(g, sc, c, ckpt, tol=TOL):
    """A^-1 (delta_{r0} e_c): the unit dipole at the focus, component c."""
    amp = [0.0, 0.0, 0.0]
    amp[c] = 1.0
    return converge(g, sc.eps_r, oc.point_source(g, sc.r0, amp), f"lens16d_dip{c}", ckpt, tol)


def lens16_dipole(ckpt, c, tol=TOL):
    sc = scenes.zoneplate16_design(0)
    g = oc.Grid(*sc.shape, sc.pitch, sc.lambda0, sc.n_bg, sc.pml)
    dipole(g, sc, c, ckpt, tol)


def sphere64_slab():
    """The 64^3 gradient case: the sphere scene with a 6-voxel slab of seeded
    random permittivity below it (z in [18, 24), x, y in [8, 56)), objective
    |E(r0)|^2 at r0 = (32, 32, 44)."""
    sc = scenes.sphere64()
    eps = sc.eps_r.copy()
    rng = np.random.default_rng(0)
    sl = (slice(18, 24), slice(8, 56), slice(8, 56))
    eps[sl] = np.clip(eps[sl] + rng.uniform(-0.25, 0.25, eps[sl].shape), 1.0, 2.1).astype(np.float32)
    return sc, eps, (32, 32, 44), (8, 8, 18), (56, 56, 24)


def sphere64_fd(ckpt):
    sc, eps32, r0, lo, hi = sphere64_slab()
    g = oc.Grid(*sc.shape, sc.pitch, sc.lambda0, sc.n_bg, sc.pml)
    eps = eps32.astype(np.float64)
    tol = 1e-12
    L0, res = oc.objective_of_eps(g, eps, r0, tol, 40000)
    E = oc.plane_wave(g) + res.E_s
    adj = oc.solve_adjoint(g, eps, oc.adjoint_point_source(g, E, r0), tol=tol, max_iter=40000)
    grad = oc.gradient(g, E, adj.E_s, lo, hi, scale=2.0)
    bz, by, bx = grad.shape
    pick = np.random.default_rng(1).choice(bz * by * bx, size=32, replace=False)
    h = 1e-3
    vox, fd, ga = [], [], []
    for n, v in enumerate(pick):
        zi, yi, xi = v // (by * bx), (v // bx) % by, v % bx
        x, y, z = lo[0] + xi, lo[1] + yi, lo[2] + zi
        ep, em = eps.copy(), eps.copy()
        ep[z, y, x] += h
        em[z, y, x] -= h
        Lp, rp = oc.objective_of_eps(g, ep, r0, tol, 40000, res.E_s)
        Lm, rm = oc.objective_of_eps(g, em, r0, tol, 40000, res.E_s)
        vox.append((x, y, z))
        fd.append((Lp - Lm) / (2 * h))
        ga.append(grad[zi, yi, xi])
        log(f"sphere64_fd {n + 1}/32: voxel {vox[-1]} fd {fd[-1]:.9e} adjoint {ga[-1]:.9e} "
            f"({rp.iterations} + {rm.iterations} iterations)")
    out = os.path.join(HERE, "sphere64_fd_gradient.npz")
    np.savez_compressed(out, r0=np.array(r0), box_lo=np.array(lo), box_hi=np.array(hi), h=h,
                        tol=tol, objective=L0, vox=np.array(vox), fd=np.array(fd),
                        adjoint=np.array(ga), grad_norm=float(np.linalg.norm(grad)),
                        grad_max=float(np.abs(grad).max()))
    log(f"wrote {out}")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="+",
                    choices=["lens16", "lens16_grad", "sphere64_fd", "lens16_dipole0",
                             "lens16_dipole1", "lens16_dipole2"])
    ap.add_argument("--ckpt", default=None, help="directory for resumable checkpoints")
    ap.add_argument("--tol", type=float, default=TOL, help="eta at which the lens solves stop")
    ap.add_argument("--gmres-restart", type=int, default=0,
                    help="after the CBS iteration, GMRES with this restart length ...")
    ap.add_argument("--gmres-cycles", type=int, default=0, help="... for this many cycles")
    a = ap.parse_args(argv)
    GMRES["restart"], GMRES["cycles"] = a.gmres_restart, a.gmres_cycles
    if a.ckpt:
        os.makedirs(a.ckpt, exist_ok=True)
    for w in a.which:
        if w.startswith("lens16_dipole"):
            lens16_dipole(a.ckpt, int(w[-1]), a.tol)
        elif w == "sphere64_fd":
            sphere64_fd(a.ckpt)
        else:
            {"lens16": lens16, "lens16_grad": lens16_grad}[w](a.ckpt, a.tol)


if __name__ == "__main__":
    main()
