"""Thickness-map inverse design of a diffractive lens on one GPU.

The loop of the optimisation paragraph (Fig. 2a) around the CBS solver:

    p (thickness map, voxel pitches)
      -> mirror symmetry (mean of the four mirror images about the centre)
      -> optional Gaussian smoothing (standard deviation 355 nm, zero outside)
      -> lens aperture (zero outside D and the absorbing layer)
      -> subpixel shape function: voxel z of column (x, y) is filled by
         clip(h - (z - z_b), 0, 1), eps_r = n_bg^2 + fill (n^2 - n_bg^2)
      -> forward CBS, L = |E(r0)|^2, adjoint CBS, dL/d eps_r over the lens slab
         (all in the HIP library, warm-started from the previous step's fields)
      -> dL/dp by torch autograd through the design map (linear and
         elementwise; the fill's derivative is taken one-sided from above so a
         zero thickness can grow)
      -> Adam ascent (step 0.3, decay rates 0.9 / 0.999, 1e-6; Adam
         paragraph), then p clipped to [0, h_max].

Thickness is measured in voxel pitches, and the Adam step is in the same unit
(the paper does not state it).  The design map is a few small torch tensor
operations on the lateral map and the lens slab; every solve and the gradient
product run in libcbs.
"""

from __future__ import annotations

import dataclasses
import math
import time

import numpy as np
import torch

from .scenes import LensDesign
from .solver import Plan


def _gauss1d(sigma: float) -> np.ndarray:
    r = int(math.ceil(4.0 * sigma))
    x = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-x * x / (2.0 * sigma * sigma))
    return g / g.sum()


class DesignMap:
    """p [ny, nx] -> eps_r of the lens slab [z1 - z0, ny, nx] (torch, differentiable)."""

    def __init__(self, d: LensDesign, device, smoothing: bool = True):
        self.d = d
        self.device = torch.device(device)
        self.smoothing = smoothing
        self.aperture = torch.from_numpy(np.asarray(d.aperture, np.float32)).to(self.device)
        g = torch.from_numpy(_gauss1d(d.sigma_vox).astype(np.float32)).to(self.device)
        self.r = (g.numel() - 1) // 2
        self.kx = g.view(1, 1, 1, -1)
        self.ky = g.view(1, 1, -1, 1)
        z0, z1 = d.slab
        self.dz = (torch.arange(z0, z1, device=self.device, dtype=torch.float32)
                   - float(d.z_base)).view(-1, 1, 1)
        self.contrast = float(d.n_lens ** 2 - d.n_bg ** 2)
        self.bg = float(d.n_bg ** 2)

    def thickness(self, p: torch.Tensor) -> torch.Tensor:
        h = 0.25 * (p + p.flip(1) + p.flip(0) + p.flip((0, 1)))
        if self.smoothing:
            x = h.view(1, 1, *h.shape)
            x = torch.nn.functional.conv2d(x, self.kx, padding=(0, self.r))
            x = torch.nn.functional.conv2d(x, self.ky, padding=(self.r, 0))
            h = x.view(h.shape)
        return h * self.aperture

    def slab_eps(self, h: torch.Tensor) -> torch.Tensor:
        u = h.unsqueeze(0) - self.dz
        fill = torch.where((u >= 0) & (u < 1), u, (u >= 1).to(u.dtype))
        return self.bg + fill * self.contrast

    def __call__(self, p: torch.Tensor) -> torch.Tensor:
        return self.slab_eps(self.thickness(p))


@dataclasses.dataclass
class DesignStep:
    step: int
    fom: float                    # |E(r0)|^2 before the update
    iterations: tuple             # (forward, adjoint)
    seconds: float


class LensOptimizer:
    """Adam ascent of |E(r0)|^2 over the thickness map of a LensDesign."""

    def __init__(self, d: LensDesign, device=None, smoothing: bool = True, tol: float = 1e-4,
                 max_iter: int = 20000, lr: float = 0.3, betas=(0.9, 0.999), adam_eps: float = 1e-6,
                 check_every: int = 20):
        nx, ny, nz = d.shape
        z0, z1 = d.slab
        if z0 < d.pml[2] or z1 > nz - d.pml[2]:
            raise ValueError(f"lens slab z [{z0}, {z1}) reaches into the absorbing layer")
        if not all(d.pml[a] <= d.r0[a] < d.shape[a] - d.pml[a] for a in range(3)):
            raise ValueError(f"focus {d.r0} lies in the absorbing layer")
        self.d = d
        self.device = torch.device(device) if device is not None else torch.device("cuda", 0)
        self.map = DesignMap(d, self.device, smoothing)
        self.plan = Plan(d.shape, d.pitch, d.lambda0, d.n_bg, d.pml, device=self.device)
        self.p = torch.tensor(d.h_init, dtype=torch.float32, device=self.device, requires_grad=True)
        self.opt = torch.optim.Adam([self.p], lr=lr, betas=betas, eps=adam_eps, maximize=True)
        self.eps = torch.full((nz, ny, nx), d.n_bg ** 2, dtype=torch.float32, device=self.device)
        self.E = self.plan.new_field()
        self.Ea = self.plan.new_field()
        self.warm = False
        self.tol, self.max_iter, self.check_every = tol, max_iter, check_every
        self.k = 0
        self.last_grad = None

    def gradient(self):
        """(L, dL/dp, (forward, adjoint) iterations) at the current p; no update."""
        d = self.d
        z0, z1 = d.slab
        nx, ny, nz = d.shape
        e_slab = self.map(self.p)
        with torch.no_grad():
            self.eps[z0:z1] = e_slab
        self.plan.set_permittivity(self.eps)
        E, s1 = self.plan.solve(self.E, tol=self.tol, max_iter=self.max_iter,
                                check_every=self.check_every, warm=self.warm)
        ix, iy, iz = d.r0
        L = float((E[:, iz, iy, ix].abs() ** 2).sum().item())
        Ea, s2 = self.plan.adjoint(E_fwd=E, r0=d.r0, E_adj=self.Ea, tol=self.tol,
                                   max_iter=self.max_iter, check_every=self.check_every,
                                   warm=self.warm)
        geps = self.plan.gradient(E, Ea, (0, 0, z0), (nx, ny, z1), scale=2.0)
        self.warm = True
        if self.p.grad is not None:
            self.p.grad = None
        e_slab.backward(geps)
        return L, self.p.grad.detach().clone(), (s1.iterations, s2.iterations)

    def step(self) -> DesignStep:
        t0 = time.perf_counter()
        L, g, its = self.gradient()
        self.last_grad = g
        self.opt.step()
        with torch.no_grad():
            self.p.clamp_(0.0, float(self.d.h_max))
        torch.cuda.synchronize(self.device)
        self.k += 1
        return DesignStep(self.k, L, its, time.perf_counter() - t0)

    def thickness(self) -> torch.Tensor:
        with torch.no_grad():
            return self.map.thickness(self.p)

    def close(self):
        self.plan.close()
