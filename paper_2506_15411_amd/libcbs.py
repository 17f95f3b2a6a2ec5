"""ctypes binding of libcbs (include/cbs.h): argument marshalling only.

Every function here has the name and argument order of the C entry point it
calls; device buffers are passed as raw pointers (``tensor.data_ptr()``).
The solver's arithmetic lives entirely in the HIP library: if the library is
missing this module raises instead of falling back to anything else.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libcbs.so")

# status codes (cbs_status)
CBS_OK = 0
CBS_NOT_CONVERGED = 1
CBS_E_INVALID = -1
CBS_E_WORKSPACE = -2
CBS_E_HIP = -3
CBS_E_DIVERGED = -4
CBS_E_STATE = -5

CBS_F32 = 0
CBS_C64 = 1

CBS_SRC_NONE = 0
CBS_SRC_PLANE_WAVE = 1
CBS_SRC_FIELD = 2
CBS_SRC_POINT = 3
CBS_SRC_FIELD_CONJ = 4

CBS_WARM_START = 1
CBS_RETURN_SCATTERED = 2
CBS_RECORD_HISTORY = 4


class cbs_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("check_every", ctypes.c_int), ("flags", ctypes.c_uint)]


class cbs_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int),
                ("residual", ctypes.c_double), ("eps_shift", ctypes.c_double),
                ("ms", ctypes.c_float)]


class cbs_lens_figures(ctypes.Structure):
    _fields_ = [("focus", ctypes.c_int * 3), ("peak", ctypes.c_double),
                ("fwhm", ctypes.c_double * 3), ("disc_flux", ctypes.c_double),
                ("eta_f", ctypes.c_double)]


class cbs_source(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("pol", (ctypes.c_double * 2) * 3),
                ("field", ctypes.c_void_p), ("r0", ctypes.c_int * 3),
                ("amp", (ctypes.c_double * 2) * 3), ("dir", ctypes.c_double * 2)]


class cbs_scpml(ctypes.Structure):
    _fields_ = [("alpha_max", ctypes.c_double), ("order", ctypes.c_int),
                ("restart", ctypes.c_int)]


class CbsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"cbs status {code}: {msg}")
        self.code = code


_lib = None

SYMBOLS = [
    "cbs_plan_workspace_bytes", "cbs_axis_supported", "cbs_plan_create",
    "cbs_plan_set_pml_profile", "cbs_plan_set_shift_factor", "cbs_set_permittivity", "cbs_solve", "cbs_adjoint_solve",
    "cbs_solve_begin", "cbs_solve_advance", "cbs_solve_poll", "cbs_solve_end", "cbs_batch_step",
    "cbs_gradient", "cbs_lens_metrics", "cbs_apply_green", "cbs_time_passes", "cbs_bandwidth_probe", "cbs_history", "cbs_eps_shift", "cbs_plan_destroy",
    "cbs_last_error", "cbs_solve_static", "cbs_batch_workspace_bytes", "cbs_solve_batch",
    "cbs_tfsf_source", "cbs_scpml_workspace_bytes", "cbs_solve_scpml", "cbs_scpml_operator",
]

CBS_MAX_ILLUMINATIONS = 8

CBS_STATIC_SCRATCH_BYTES = 96 << 20


def load(path: str | None = None):
    """Load libcbs.so (built by paper_2506_15411_amd.build); raises if absent."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"libcbs.so not found at {p}; run `python -m paper_2506_15411_amd.build`")
    lib = ctypes.CDLL(p)
    c_int, c_double, c_void_p, c_size_t = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
    P = ctypes.POINTER
    lib.cbs_plan_workspace_bytes.argtypes = [c_int, c_int, c_int]
    lib.cbs_plan_workspace_bytes.restype = c_size_t
    lib.cbs_axis_supported.argtypes = [c_int, c_int]
    lib.cbs_axis_supported.restype = c_int
    lib.cbs_plan_create.argtypes = [P(c_void_p), c_int, c_int, c_int, c_double, c_double, c_double,
                                    P(c_int), c_void_p, c_size_t, c_void_p]
    lib.cbs_plan_create.restype = c_int
    lib.cbs_plan_set_pml_profile.argtypes = [c_void_p, c_int, c_double]
    lib.cbs_plan_set_pml_profile.restype = c_int
    lib.cbs_plan_set_shift_factor.argtypes = [c_void_p, c_double]
    lib.cbs_plan_set_shift_factor.restype = c_int
    lib.cbs_set_permittivity.argtypes = [c_void_p, c_void_p, c_int]
    lib.cbs_set_permittivity.restype = c_int
    lib.cbs_solve.argtypes = [c_void_p, P(cbs_source), c_void_p, P(cbs_opts), P(cbs_stats)]
    lib.cbs_solve.restype = c_int
    lib.cbs_adjoint_solve.argtypes = [c_void_p, c_void_p, P(cbs_source), c_void_p, P(cbs_opts),
                                      P(cbs_stats)]
    lib.cbs_adjoint_solve.restype = c_int
    lib.cbs_solve_begin.argtypes = [c_void_p, c_int, c_void_p, P(cbs_source), c_void_p, P(cbs_opts)]
    lib.cbs_solve_begin.restype = c_int
    lib.cbs_solve_advance.argtypes = [c_void_p, c_int]
    lib.cbs_solve_advance.restype = c_int
    lib.cbs_solve_poll.argtypes = [c_void_p, P(c_int), P(c_int)]
    lib.cbs_solve_poll.restype = c_int
    lib.cbs_solve_end.argtypes = [c_void_p, P(cbs_stats)]
    lib.cbs_solve_end.restype = c_int
    lib.cbs_batch_step.argtypes = [P(c_void_p), c_int, c_int, P(c_int)]
    lib.cbs_batch_step.restype = c_int
    lib.cbs_gradient.argtypes = [c_void_p, c_void_p, c_void_p, P(c_int), P(c_int), c_double,
                                 c_void_p]
    lib.cbs_gradient.restype = c_int
    lib.cbs_lens_metrics.argtypes = [c_void_p, c_void_p, P(c_int), P(c_int), c_double, c_double,
                                     c_double, P(cbs_lens_figures)]
    lib.cbs_lens_metrics.restype = c_int
    lib.cbs_apply_green.argtypes = [c_void_p, c_void_p, c_void_p]
    lib.cbs_apply_green.restype = c_int
    lib.cbs_time_passes.argtypes = [c_void_p, c_void_p, c_int, P(ctypes.c_float)]
    lib.cbs_time_passes.restype = c_int
    lib.cbs_bandwidth_probe.argtypes = [c_void_p, c_void_p, c_size_t, c_int, c_void_p,
                                        P(ctypes.c_float)]
    lib.cbs_bandwidth_probe.restype = c_int
    lib.cbs_history.argtypes = [c_void_p, P(c_double), c_int]
    lib.cbs_history.restype = c_int
    lib.cbs_eps_shift.argtypes = [c_void_p]
    lib.cbs_eps_shift.restype = c_double
    lib.cbs_plan_destroy.argtypes = [c_void_p]
    lib.cbs_plan_destroy.restype = c_int
    lib.cbs_solve_static.argtypes = [c_int, c_int, c_int, c_double, c_double, c_double, P(c_int),
                                     c_void_p, c_int, P(cbs_source), c_void_p, P(cbs_opts),
                                     P(cbs_stats), c_void_p]
    lib.cbs_solve_static.restype = c_int
    lib.cbs_batch_workspace_bytes.argtypes = [c_int, c_int, c_int, c_int]
    lib.cbs_batch_workspace_bytes.restype = c_size_t
    lib.cbs_solve_batch.argtypes = [c_void_p, c_int, P(cbs_source), c_void_p, P(cbs_opts),
                                    P(cbs_stats), c_void_p, c_size_t]
    lib.cbs_solve_batch.restype = c_int
    lib.cbs_tfsf_source.argtypes = [c_void_p, P(cbs_source), P(c_int), P(c_int), c_void_p]
    lib.cbs_tfsf_source.restype = c_int
    lib.cbs_scpml_workspace_bytes.argtypes = [c_int, c_int, c_int, c_int]
    lib.cbs_scpml_workspace_bytes.restype = c_size_t
    lib.cbs_solve_scpml.argtypes = [c_void_p, P(cbs_source), c_void_p, P(cbs_opts), P(cbs_scpml),
                                    P(cbs_stats), c_void_p, c_size_t]
    lib.cbs_solve_scpml.restype = c_int
    lib.cbs_scpml_operator.argtypes = [c_void_p, P(cbs_scpml), c_void_p, c_void_p, c_void_p,
                                       c_size_t]
    lib.cbs_scpml_operator.restype = c_int
    lib.cbs_last_error.argtypes = []
    lib.cbs_last_error.restype = ctypes.c_char_p
    if path is None:
        _lib = lib
    return lib


def check(code: int, allow_not_converged: bool = False) -> int:
    """Raise CbsError for error statuses (and NOT_CONVERGED unless allowed)."""
    if code == CBS_OK or (allow_not_converged and code == CBS_NOT_CONVERGED):
        return code
    msg = load().cbs_last_error().decode(errors="replace")
    raise CbsError(code, msg)


def _ints3(v):
    return (ctypes.c_int * 3)(*[int(x) for x in v])


# --- one wrapper per entry point (same names) ------------------------------
def cbs_plan_workspace_bytes(nx, ny, nz) -> int:
    return int(load().cbs_plan_workspace_bytes(nx, ny, nz))


def cbs_axis_supported(axis, n) -> bool:
    return bool(load().cbs_axis_supported(axis, n))


def cbs_plan_create(nx, ny, nz, pitch, lambda0, n_bg, pml, workspace_ptr, workspace_bytes,
                    stream_ptr):
    h = ctypes.c_void_p()
    check(load().cbs_plan_create(ctypes.byref(h), nx, ny, nz, pitch, lambda0, n_bg, _ints3(pml),
                                 ctypes.c_void_p(workspace_ptr), workspace_bytes,
                                 ctypes.c_void_p(stream_ptr)))
    return h


def cbs_plan_set_pml_profile(plan, order, sigma_max):
    return check(load().cbs_plan_set_pml_profile(plan, order, sigma_max))


def cbs_plan_set_shift_factor(plan, kappa):
    return check(load().cbs_plan_set_shift_factor(plan, float(kappa)))


def cbs_set_permittivity(plan, eps_ptr, dtype):
    return check(load().cbs_set_permittivity(plan, ctypes.c_void_p(eps_ptr), dtype))


def cbs_solve(plan, src: cbs_source | None, E_ptr, opts: cbs_opts):
    st = cbs_stats()
    rc = load().cbs_solve(plan, ctypes.byref(src) if src is not None else None,
                          ctypes.c_void_p(E_ptr), ctypes.byref(opts), ctypes.byref(st))
    check(rc, allow_not_converged=True)
    return rc, st


def cbs_adjoint_solve(plan, E_fwd_ptr, src: cbs_source, E_adj_ptr, opts: cbs_opts):
    st = cbs_stats()
    rc = load().cbs_adjoint_solve(plan, ctypes.c_void_p(E_fwd_ptr), ctypes.byref(src),
                                  ctypes.c_void_p(E_adj_ptr), ctypes.byref(opts),
                                  ctypes.byref(st))
    check(rc, allow_not_converged=True)
    return rc, st


def cbs_solve_begin(plan, adjoint: int, E_fwd_ptr, src: cbs_source | None, E_ptr, opts: cbs_opts):
    return check(load().cbs_solve_begin(plan, int(adjoint), ctypes.c_void_p(E_fwd_ptr),
                                        ctypes.byref(src) if src is not None else None,
                                        ctypes.c_void_p(E_ptr), ctypes.byref(opts)))


def cbs_solve_advance(plan, iters):
    return check(load().cbs_solve_advance(plan, int(iters)))


def cbs_solve_poll(plan):
    """(done, outstanding quanta)"""
    done = ctypes.c_int(0)
    out = ctypes.c_int(0)
    check(load().cbs_solve_poll(plan, ctypes.byref(done), ctypes.byref(out)))
    return bool(done.value), int(out.value)


def cbs_solve_end(plan):
    st = cbs_stats()
    rc = load().cbs_solve_end(plan, ctypes.byref(st))
    check(rc, allow_not_converged=True)
    return rc, st


def cbs_batch_step(plans, iters):
    arr = (ctypes.c_void_p * len(plans))(*[p.value if isinstance(p, ctypes.c_void_p) else p for p in plans])
    done = (ctypes.c_int * max(1, len(plans)))()
    check(load().cbs_batch_step(arr, len(plans), int(iters), done))
    return [bool(done[i]) for i in range(len(plans))]


def cbs_gradient(plan, E_ptr, E_adj_ptr, box_lo, box_hi, scale, grad_ptr):
    return check(load().cbs_gradient(plan, ctypes.c_void_p(E_ptr), ctypes.c_void_p(E_adj_ptr),
                                     _ints3(box_lo), _ints3(box_hi), float(scale),
                                     ctypes.c_void_p(grad_ptr)))


def cbs_lens_metrics(plan, E_ptr, lo, hi, disc_factor, aperture_m, e0=1.0):
    out = cbs_lens_figures()
    check(load().cbs_lens_metrics(plan, ctypes.c_void_p(E_ptr), _ints3(lo), _ints3(hi),
                                  float(disc_factor), float(aperture_m), float(e0),
                                  ctypes.byref(out)))
    return out


def cbs_apply_green(plan, in_ptr, out_ptr):
    return check(load().cbs_apply_green(plan, ctypes.c_void_p(in_ptr), ctypes.c_void_p(out_ptr)))


def cbs_time_passes(plan, E_ptr, iters):
    ms = (ctypes.c_float * 5)()
    check(load().cbs_time_passes(plan, ctypes.c_void_p(E_ptr), int(iters), ms))
    return [float(v) for v in ms]


def cbs_bandwidth_probe(src_ptr, dst_ptr, nbytes, reps, stream_ptr) -> float:
    ms = ctypes.c_float()
    check(load().cbs_bandwidth_probe(ctypes.c_void_p(src_ptr), ctypes.c_void_p(dst_ptr), int(nbytes),
                                     int(reps), ctypes.c_void_p(stream_ptr), ctypes.byref(ms)))
    return float(ms.value)


def cbs_history(plan, max_n: int):
    buf = (ctypes.c_double * max(1, max_n))()
    n = load().cbs_history(plan, buf, max_n)
    if n < 0:
        check(n)
    return [buf[i] for i in range(min(n, max_n))]


def cbs_eps_shift(plan) -> float:
    return float(load().cbs_eps_shift(plan))


def cbs_plan_destroy(plan):
    return check(load().cbs_plan_destroy(plan))


def cbs_solve_static(nx, ny, nz, pitch, lambda0, n_bg, pml, eps_ptr, dtype,
                     src: cbs_source | None, E_ptr, opts: cbs_opts, stream_ptr):
    st = cbs_stats()
    rc = load().cbs_solve_static(nx, ny, nz, pitch, lambda0, n_bg, _ints3(pml),
                                 ctypes.c_void_p(eps_ptr), dtype,
                                 ctypes.byref(src) if src is not None else None,
                                 ctypes.c_void_p(E_ptr), ctypes.byref(opts), ctypes.byref(st),
                                 ctypes.c_void_p(stream_ptr))
    check(rc, allow_not_converged=True)
    return rc, st


def cbs_batch_workspace_bytes(nx, ny, nz, count) -> int:
    return int(load().cbs_batch_workspace_bytes(nx, ny, nz, count))


def cbs_solve_batch(plan, srcs, E_ptr, opts: cbs_opts, work_ptr, work_bytes):
    n = len(srcs)
    arr = (cbs_source * n)(*srcs)
    st = (cbs_stats * n)()
    rc = load().cbs_solve_batch(plan, n, arr, ctypes.c_void_p(E_ptr), ctypes.byref(opts), st,
                                ctypes.c_void_p(work_ptr), work_bytes)
    check(rc, allow_not_converged=True)
    return rc, [st[i] for i in range(n)]


def cbs_tfsf_source(plan, src: cbs_source | None, lo, hi, S_ptr):
    return check(load().cbs_tfsf_source(plan, ctypes.byref(src) if src is not None else None,
                                        _ints3(lo), _ints3(hi), ctypes.c_void_p(S_ptr)))


def cbs_scpml_workspace_bytes(nx, ny, nz, restart) -> int:
    return int(load().cbs_scpml_workspace_bytes(nx, ny, nz, restart))


def cbs_solve_scpml(plan, src: cbs_source | None, E_ptr, opts: cbs_opts, layer: cbs_scpml,
                    work_ptr, work_bytes):
    st = cbs_stats()
    code = load().cbs_solve_scpml(plan, ctypes.byref(src) if src is not None else None,
                                  ctypes.c_void_p(E_ptr), ctypes.byref(opts), ctypes.byref(layer),
                                  ctypes.byref(st), ctypes.c_void_p(work_ptr), work_bytes)
    check(code, allow_not_converged=True)
    return code, st


def cbs_scpml_operator(plan, layer: cbs_scpml, in_ptr, out_ptr, work_ptr, work_bytes):
    return check(load().cbs_scpml_operator(plan, ctypes.byref(layer), ctypes.c_void_p(in_ptr),
                                           ctypes.c_void_p(out_ptr), ctypes.c_void_p(work_ptr),
                                           work_bytes))


def cbs_last_error() -> str:
    return load().cbs_last_error().decode(errors="replace")
