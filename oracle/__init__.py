"""FP64 CPU oracle for the vector convergent Born series (CBS) solver.

THIS PACKAGE IS TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import or call it. The product
path (the HIP library and its Python binding) never imports it and shares no
code with it; the only thing both sides consume is the seeded scene/input
generator module, which contains none of the solver's arithmetic.

Modules
-------
cbs       plain FP64 CBS iteration, sources, adjoint solve, gradient
dense     dense 3N x 3N operator from explicit DFT matrices, LU and GMRES solves
closed    closed forms: uniform-medium per-mode iteration, 1D slab reduction
mie       Mie series of a dielectric sphere in a plane wave (continuum closed form)
design    thickness-map lens design: eps_r(h), chain rule dL/dh, Adam step
metrics   lens figures: focus, FWHM, focusing efficiency (Poynting flux)

Every function cites the passage of the paper (arXiv 2506.15411) or of the CBS
literature the paper builds on (its references [25] and [26]) that it follows.
Where the paper is silent the reading taken is stated in the docstring.
"""

from . import cbs, dense, closed, mie, design, metrics  # noqa: F401
