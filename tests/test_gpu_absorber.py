"""Reflection of the absorbing z layer at the edge angle of an NA-0.84 lens
(asin 0.84 = 57 deg), measured on the GPU solution and in the FP64 oracle.

A current sheet J e^{i kx x} just inside the lower layer launches s- or
p-polarised plane waves at angle asin(kx / kb) towards the upper layer on a grid
periodic in x and y; the driven component's x-mode amplitude along z is split
into the outgoing and the returning wave (oracle.absorber).  The grids are the
z geometry of the two lens volumes: 261 planes of 177 nm with 18-voxel layers
(the 621 x 621 x 261 volume) and 315 planes at lambda/16 with 48-voxel layers
(the 275 x 275 x 315 volume), with the default profile (order 2, sigma_max 1).
"""

import numpy as np
import pytest
import torch

from oracle import absorber as ab
from oracle import cbs as oc
from paper_2506_15411_amd import libcbs as L
from paper_2506_15411_amd.solver import Plan

pytestmark = pytest.mark.gpu
LAM = 1.064e-6
CASES = {
    "621x621x261 z layer": ((36, 4, 261), 177e-9, (0, 0, 18), 5),     # 56.6 deg
    "275x275x315 z layer": ((96, 4, 315), LAM / 16, (0, 0, 48), 5),   # 56.4 deg
}


@pytest.mark.parametrize("pol", ["s", "p"])
@pytest.mark.parametrize("case", list(CASES))
def test_edge_angle_reflection_matches_oracle(case, pol, device):
    shape, pitch, pml, mx = CASES[case]
    g = oc.Grid(*shape, pitch, LAM, 1.0, pml)
    R_o, fit_o, ang = ab.reflection_oblique(g, mx, pol, tol=1e-10)
    z_src = pml[2] + 6
    S = ab.oblique_source(g, mx, pol, z_src, amp=g.k0 ** 2)
    p = Plan(shape, pitch, LAM, 1.0, pml, device=device)
    p.set_permittivity(torch.ones(shape[::-1], dtype=torch.float32, device=device))
    # the FP32 residual floor of these grids is about 1.7e-7
    E, st = p.solve(tol=5e-7, max_iter=100000,
                    field=torch.from_numpy(S.astype(np.complex64)).to(device))
    assert st.status == L.CBS_OK
    R_g, fit_g = ab.reflection_from_field(g, E.cpu().numpy().astype(np.complex128), mx, pol, z_src)
    print(f"{case}, {pol}-polarised at {ang:.1f} deg: R gpu {R_g:.3e} oracle {R_o:.3e} "
          f"({st.iterations} iterations)")
    assert R_o < 1e-5
    assert abs(R_g - R_o) <= 0.05 * R_o + 1e-9
    p.close()
