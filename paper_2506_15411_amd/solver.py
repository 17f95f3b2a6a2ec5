"""Torch-facing wrapper of libcbs: device memory and streams come from torch,
every arithmetic step runs in the HIP library (include/cbs.h)."""

from __future__ import annotations

import dataclasses

import torch

from . import libcbs as L


@dataclasses.dataclass
class SolveStats:
    status: int
    iterations: int
    converged: bool
    residual: float
    eps_shift: float
    ms: float


def _stats(rc, st) -> SolveStats:
    return SolveStats(rc, st.iterations, bool(st.converged), st.residual, st.eps_shift, st.ms)


def _require_gpu(t: torch.Tensor, name: str, dtype, shape):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} shape {tuple(t.shape)} != {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Plan:
    """A CBS plan on one GPU: grid, optics, absorbing layer, workspace.

    shape = (nx, ny, nz); pml per side in voxels; lengths in metres.  The
    workspace is a torch uint8 tensor on ``device`` (exactly the bytes
    cbs_plan_workspace_bytes reports, 256-byte aligned)."""

    def __init__(self, shape, pitch, lambda0=1.064e-6, n_bg=1.0, pml=(0, 0, 0), device=None,
                 stream: torch.cuda.Stream | None = None, pml_order=2, sigma_max=1.0,
                 shift_factor=1.1):
        nx, ny, nz = (int(v) for v in shape)
        self.shape = (nx, ny, nz)
        self.pitch, self.lambda0, self.n_bg, self.pml = float(pitch), float(lambda0), float(n_bg), tuple(pml)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        nbytes = L.cbs_plan_workspace_bytes(nx, ny, nz)
        if nbytes == 0:
            raise ValueError(f"grid {shape} is not supported by libcbs")
        self.workspace_bytes = nbytes
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._raw = raw
        self.workspace = raw[off:off + nbytes]
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.handle = L.cbs_plan_create(nx, ny, nz, self.pitch, self.lambda0, self.n_bg, self.pml,
                                        self.workspace.data_ptr(), nbytes, self.stream.cuda_stream)
        if (pml_order, sigma_max) != (2, 1.0):
            L.cbs_plan_set_pml_profile(self.handle, int(pml_order), float(sigma_max))
        if shift_factor != 1.1:
            L.cbs_plan_set_shift_factor(self.handle, float(shift_factor))
        self._eps_ref = None

    # -- shapes ---------------------------------------------------------------
    @property
    def vshape(self):
        nx, ny, nz = self.shape
        return (nz, ny, nx)

    @property
    def fshape(self):
        return (3,) + self.vshape

    def new_field(self):
        """A zeroed complex64 [3, nz, ny, nx] field, allocated and cleared on the
        plan's stream so the plan's kernels are ordered after the clear."""
        with torch.cuda.stream(self.stream):
            return torch.zeros(self.fshape, dtype=torch.complex64, device=self.device)

    # -- entry points -----------------------------------------------------------
    def set_permittivity(self, eps_r: torch.Tensor):
        dtype = {torch.float32: L.CBS_F32, torch.complex64: L.CBS_C64}.get(eps_r.dtype)
        if dtype is None:
            raise ValueError("eps_r must be float32 or complex64")
        _require_gpu(eps_r, "eps_r", eps_r.dtype, self.vshape)
        L.cbs_set_permittivity(self.handle, eps_r.data_ptr(), dtype)
        self._eps_ref = eps_r
        return self.eps_shift

    @property
    def eps_shift(self) -> float:
        return L.cbs_eps_shift(self.handle)

    @staticmethod
    def _opts(tol, max_iter, check_every, warm=False, scattered=False, history=False):
        flags = (L.CBS_WARM_START if warm else 0) | (L.CBS_RETURN_SCATTERED if scattered else 0) \
            | (L.CBS_RECORD_HISTORY if history else 0)
        return L.cbs_opts(float(tol), int(max_iter), int(check_every), flags)

    def _forward_source(self, pol=None, field=None, point=None, kind=None, direction=None):
        src = L.cbs_source()
        if field is not None:
            _require_gpu(field, "field", torch.complex64, self.fshape)
            if field.is_conj():
                raise ValueError("field has torch's lazy conjugate bit; resolve it first")
            src.kind = L.CBS_SRC_FIELD
            src.field = field.data_ptr()
        elif point is not None:
            r0, amp = point
            src.kind = L.CBS_SRC_POINT
            for c in range(3):
                src.r0[c] = int(r0[c])
                a = complex(amp[c])
                src.amp[c][0], src.amp[c][1] = a.real, a.imag
        else:
            src.kind = L.CBS_SRC_PLANE_WAVE if kind is None else kind
            if pol is not None:
                for c in range(3):
                    a = complex(pol[c])
                    src.pol[c][0], src.pol[c][1] = a.real, a.imag
            if direction is not None:
                src.dir[0], src.dir[1] = float(direction[0]), float(direction[1])
        return src

    def _adjoint_source(self, E_fwd=None, r0=None, amp=None, field=None, conj=False):
        src = L.cbs_source()
        fptr = 0
        if field is not None:
            _require_gpu(field, "field", torch.complex64, self.fshape)
            if field.is_conj():
                raise ValueError("field has torch's lazy conjugate bit; pass conj=True "
                                 "with the unconjugated tensor instead")
            src.kind = L.CBS_SRC_FIELD_CONJ if conj else L.CBS_SRC_FIELD
            src.field = field.data_ptr()
        else:
            src.kind = L.CBS_SRC_POINT
            for c in range(3):
                src.r0[c] = int(r0[c])
            if amp is not None:
                for c in range(3):
                    a = complex(amp[c])
                    src.amp[c][0], src.amp[c][1] = a.real, a.imag
            else:
                _require_gpu(E_fwd, "E_fwd", torch.complex64, self.fshape)
                fptr = E_fwd.data_ptr()
        return src, fptr

    def solve(self, E: torch.Tensor | None = None, tol=1e-4, max_iter=20000, check_every=10,
              warm=False, scattered=False, history=False, pol=None, field=None, point=None,
              kind=None, direction=None):
        """Forward solve (plane wave by default: x-polarised, normal incidence;
        direction = (kx, ky) / kb tilts it).  Returns (E, SolveStats)."""
        if E is None:
            E = self.new_field()
        _require_gpu(E, "E", torch.complex64, self.fshape)
        src = self._forward_source(pol, field, point, kind, direction)
        self._src_keep = src
        rc, st = L.cbs_solve(self.handle, src, E.data_ptr(),
                             self._opts(tol, max_iter, check_every, warm, scattered, history))
        return E, _stats(rc, st)

    def adjoint(self, E_fwd: torch.Tensor | None = None, r0=None, amp=None, field=None,
                E_adj: torch.Tensor | None = None, tol=1e-4, max_iter=20000, check_every=10,
                warm=False, history=False, conj=False):
        """Adjoint solve.  With r0 and E_fwd: source conj(E_fwd(r0)) at r0
        (objective |E(r0)|^2).  With r0 and amp: that amplitude.  With field:
        a general source (conj=True: its complex conjugate, formed on the
        device).  Returns (E_adj, SolveStats)."""
        if E_adj is None:
            E_adj = self.new_field()
        _require_gpu(E_adj, "E_adj", torch.complex64, self.fshape)
        src, fptr = self._adjoint_source(E_fwd, r0, amp, field, conj)
        rc, st = L.cbs_adjoint_solve(self.handle, fptr, src, E_adj.data_ptr(),
                                     self._opts(tol, max_iter, check_every, warm, False, history))
        return E_adj, _stats(rc, st)

    def solve_batch(self, illuminations, E: torch.Tensor | None = None, tol=1e-4,
                    max_iter=20000, check_every=10, warm=False, scattered=False,
                    history=False):
        """Several plane-wave illuminations of the current medium in one batched
        solve (see cbs_solve_batch).  illuminations: list of (pol, direction)
        pairs (None for x-polarised / normal incidence).  Returns
        (E [count, 3, nz, ny, nx], [SolveStats per illumination])."""
        n = len(illuminations)
        shape = (n,) + self.fshape
        if E is None:
            with torch.cuda.stream(self.stream):
                E = torch.zeros(shape, dtype=torch.complex64, device=self.device)
        _require_gpu(E, "E", torch.complex64, shape)
        srcs = [self._forward_source(pol, None, None, None, d) for pol, d in illuminations]
        nbytes = L.cbs_batch_workspace_bytes(*self.shape, n)
        if nbytes == 0:
            raise ValueError(f"{n} illuminations: 1..{L.CBS_MAX_ILLUMINATIONS} supported")
        with torch.cuda.stream(self.stream):
            raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        rc, sts = L.cbs_solve_batch(self.handle, srcs, E.data_ptr(),
                                    self._opts(tol, max_iter, check_every, warm, scattered,
                                               history),
                                    raw.data_ptr() + off, nbytes)
        return E, [_stats(rc, st) for st in sts]

    def _scpml_work(self, restart):
        nbytes = L.cbs_scpml_workspace_bytes(*self.shape, int(restart))
        if nbytes == 0:
            raise ValueError(f"restart {restart}: 1..64 supported, every axis <= 1024")
        with torch.cuda.stream(self.stream):
            raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        return raw, raw.data_ptr() + (-raw.data_ptr()) % 256, nbytes

    def solve_scpml(self, E: torch.Tensor | None = None, alpha_max=0.75, order=1, restart=40,
                    tol=1e-5, max_iter=2000, scattered=False, history=False, pol=None,
                    field=None, point=None, kind=None, direction=None):
        """Forward solve with the stretched-coordinate layer instead of the graded
        potential (see cbs_solve_scpml; the plan must have sigma_max = 0).  tol is
        the relative residual of the preconditioned system, max_iter counts GMRES
        steps.  The default profile (alpha_max 0.75, linear) keeps GMRES
        converging on large grids: the stretched layer's high spatial
        frequencies act like s^-2, which winds further round the origin as
        alpha_max grows.  Returns (E, SolveStats)."""
        if E is None:
            E = self.new_field()
        _require_gpu(E, "E", torch.complex64, self.fshape)
        src = self._forward_source(pol, field, point, kind, direction)
        raw, ptr, nbytes = self._scpml_work(restart)
        layer = L.cbs_scpml(float(alpha_max), int(order), int(restart))
        rc, st = L.cbs_solve_scpml(self.handle, src, E.data_ptr(),
                                   self._opts(tol, max_iter, 1, False, scattered, history),
                                   layer, ptr, nbytes)
        del raw   # the call synchronised the plan's stream
        return E, _stats(rc, st)

    def scpml_operator(self, v: torch.Tensor, alpha_max=0.75, order=1,
                       out: torch.Tensor | None = None) -> torch.Tensor:
        """(L_s - L) v in 1/m^2 (see cbs_scpml_operator)."""
        _require_gpu(v, "v", torch.complex64, self.fshape)
        if out is None:
            out = self.new_field()
        _require_gpu(out, "out", torch.complex64, self.fshape)
        raw, ptr, nbytes = self._scpml_work(1)
        L.cbs_scpml_operator(self.handle, L.cbs_scpml(float(alpha_max), int(order), 1),
                             v.data_ptr(), out.data_ptr(), ptr, nbytes)
        self.stream.synchronize()   # the workspace is released on return
        return out

    # -- asynchronous solves (one at a time per plan; plans overlap) ---------
    def begin(self, E: torch.Tensor, adjoint=False, E_fwd=None, r0=None, amp=None, field=None,
              tol=1e-4, max_iter=20000, warm=False, scattered=False, history=False, pol=None):
        """Start a solve into E without waiting (see cbs_solve_begin)."""
        _require_gpu(E, "E", torch.complex64, self.fshape)
        if adjoint:
            src, fptr = self._adjoint_source(E_fwd, r0, amp, field)
        else:
            src, fptr = self._forward_source(pol, field, None, None), 0
        opts = self._opts(tol, max_iter, 1, warm, scattered, history)
        L.cbs_solve_begin(self.handle, 1 if adjoint else 0, fptr, src, E.data_ptr(), opts)
        self._async_keep = (E, E_fwd, field)
        return E

    def advance(self, iters: int):
        L.cbs_solve_advance(self.handle, iters)

    def poll(self):
        """(done, outstanding quanta) without waiting."""
        return L.cbs_solve_poll(self.handle)

    def end(self) -> SolveStats:
        rc, st = L.cbs_solve_end(self.handle)
        self._async_keep = None
        return _stats(rc, st)

    def lens_metrics(self, E: torch.Tensor, lo, hi, aperture_m: float, disc_factor: float = 3.0,
                     e0: float = 1.0) -> dict:
        """Focus (maximum of |E|^2 in [lo, hi)), FWHM along x, y, z (metres) and the
        focusing efficiency of the field E (see cbs_lens_metrics)."""
        _require_gpu(E, "E", torch.complex64, self.fshape)
        f = L.cbs_lens_metrics(self.handle, E.data_ptr(), lo, hi, disc_factor, aperture_m, e0)
        return {"focus": tuple(f.focus), "peak": f.peak, "fwhm": tuple(f.fwhm),
                "disc_flux": f.disc_flux, "eta_f": f.eta_f}

    def gradient(self, E: torch.Tensor, E_adj: torch.Tensor, box_lo=None, box_hi=None,
                 scale=2.0, out: torch.Tensor | None = None):
        """scale * k0^2 * Re(sum_c E_adj,c E_c) over [box_lo, box_hi) -> [z, y, x] float32."""
        nx, ny, nz = self.shape
        lo = tuple(box_lo) if box_lo is not None else (0, 0, 0)
        hi = tuple(box_hi) if box_hi is not None else (nx, ny, nz)
        bshape = (hi[2] - lo[2], hi[1] - lo[1], hi[0] - lo[0])
        _require_gpu(E, "E", torch.complex64, self.fshape)
        _require_gpu(E_adj, "E_adj", torch.complex64, self.fshape)
        if out is None:
            out = torch.empty(bshape, dtype=torch.float32, device=self.device)
        _require_gpu(out, "out", torch.float32, bshape)
        L.cbs_gradient(self.handle, E.data_ptr(), E_adj.data_ptr(), lo, hi, scale, out.data_ptr())
        return out

    def tfsf_source(self, lo, hi, pol=None, direction=None, out: torch.Tensor | None = None):
        """Total-field / scattered-field source of a plane wave for the box
        [lo, hi) (see cbs_tfsf_source); solve it with solve(field=...)."""
        if out is None:
            out = self.new_field()
        _require_gpu(out, "out", torch.complex64, self.fshape)
        src = self._forward_source(pol, None, None, None, direction)
        L.cbs_tfsf_source(self.handle, src, lo, hi, out.data_ptr())
        return out

    def apply_green(self, W: torch.Tensor, out: torch.Tensor | None = None):
        _require_gpu(W, "W", torch.complex64, self.fshape)
        if out is None:
            out = self.new_field()
        L.cbs_apply_green(self.handle, W.data_ptr(), out.data_ptr())
        return out

    PASSES = ("ky_forward", "kz_green", "ky_inverse", "kx_update", "residual")

    def time_passes(self, iters=10, E: torch.Tensor | None = None):
        """Mean device ms per launch of each pass over `iters` iterations."""
        if E is None:
            E = self.new_field()
        _require_gpu(E, "E", torch.complex64, self.fshape)
        return dict(zip(self.PASSES, L.cbs_time_passes(self.handle, E.data_ptr(), iters)))

    def history(self, n=1 << 16):
        return L.cbs_history(self.handle, n)

    def close(self):
        if getattr(self, "handle", None) is not None:
            L.cbs_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
