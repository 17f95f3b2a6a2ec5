"""Writes the converged stretched-layer fixture of the GPU parity tests.

Calls only the FP64 oracle (``oracle/``) and the seeded scene generator
(``paper_2506_15411_amd.scenes``, geometry and random numbers only).

    python tests/golden/make_scpml.py

scpml_24x20x32.npz  A random passive medium (scenes.random_passive_eps, seed
                    131, loss 0.02) on 24 x 20 x 32 voxels at lambda/8 with
                    stretched layers (3, 3, 4) per side (alpha_max 1.5, order 2)
                    and no graded potential, lit by the x-polarised plane wave
                    at normal incidence: the scattered field E_s = A_s^-1 S by
                    oracle.scpml.gmres_solve to a relative residual of 1e-10
                    (restart 40), stored in complex128 with the residual.
"""

from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import cbs as oc  # noqa: E402
from oracle import scpml  # noqa: E402
from paper_2506_15411_amd import scenes  # noqa: E402

LAM = 1.064e-6
SHAPE, PML, SEED, ALPHA, ORDER = (24, 20, 32), (3, 3, 4), 131, 1.5, 2


def main():
    eps = scenes.random_passive_eps(SHAPE, PML, SEED, loss=0.02)
    g = oc.Grid(*SHAPE, LAM / 8, LAM, 1.0, PML, sigma_max=0.0)
    S = oc.plane_wave_source(g, eps)
    E, res = scpml.gmres_solve(g, eps, S, ALPHA, ORDER, rtol=1e-10, restart=40, maxiter=100)
    out = os.path.join(HERE, "scpml_24x20x32.npz")
    np.savez_compressed(out, E_s=E, residual=res, shape=np.array(SHAPE), pml=np.array(PML),
                        seed=SEED, alpha_max=ALPHA, order=ORDER, pitch=LAM / 8, lambda0=LAM)
    print(out, "residual", res)


if __name__ == "__main__":
    main()
