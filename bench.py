"""Benchmark of the CBS hot path on one MI355X.

A step is one optimisation step of the 621 x 621 x 261 design volume (177 nm
pitch, zone-plate lens D = 100 um, NA 0.84, n = 1.45, lambda0 = 1064 nm):
set the permittivity, forward CBS solve of the x-polarised plane wave to
tol, adjoint CBS solve for the focal intensity |E(r0)|^2 to tol, and the
permittivity gradient over the 2 um design slab.  Inputs are resident in HBM
before the timed region.  value = voxels x CBS iterations / second.

Prints one JSON line (rank 0) with the per-kernel roofline of the dominant
pass (HIP events on the plan's stream) and the FP64 CPU oracle timed on a
bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import hashlib
import re
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CBS Gvoxel-iter/s (vector c64) + % HBM peak; p50/p99 served solve latency"
HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per voxel per launch of each pass (complex64, 3 comps):
#   y/z passes read and write the 24 B field; the x pass reads GW, E_s (24 B
#   each) and V0 (8 B) and writes E_s and the next W (24 B each).
PASS_BYTES = {"ky_forward": 48, "kz_green": 48, "ky_inverse": 48, "kx_update": 104}
ITER_BYTES = 248
PASS_SOURCES = ["paper_2506_15411_amd/csrc/kernels.hpp", "paper_2506_15411_amd/csrc/codelets.hpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    """Hash of the pass sources with comments and whitespace removed, so that
    counters stay attached to the code they were measured on."""
    h = hashlib.sha256()
    for p in PASS_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            src = f.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def workload(name: str):
    from paper_2506_15411_amd import scenes
    if name == "zoneplate100":
        return scenes.zoneplate100_design(0)
    if name == "zoneplate16":
        return scenes.zoneplate16_design(0)
    if name == "sphere64":
        sc = scenes.sphere64()
        import dataclasses
        return dataclasses.replace(sc, r0=(32, 32, 48), design_box=((8, 8, 16), (56, 56, 48)))
    raise SystemExit(f"unknown workload {name}")


def traffic_from_profile(name: str, kernel: str):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_hash") != kernel_hash():
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def copy_probe(dev, nbytes=1 << 30, reps=1):
    """Plain streaming copy of nbytes (read + write) in the library's probe kernel."""
    import torch
    from paper_2506_15411_amd import libcbs as L
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    ms = L.cbs_bandwidth_probe(src.data_ptr(), dst.data_ptr(), nbytes, reps,
                               torch.cuda.current_stream(dev).cuda_stream)
    del src, dst
    return ms


# iteration cap per served solve: high enough that every request of the served
# stream reaches tol (the slowest, large high-index spheres on the 128^3 grid,
# need about 5000-7000 iterations at tol 1e-4)
SERVE_MAX_ITER = 20000


SERVE_TRACE_LEN = 200   # the configured served stream; shorter runs take its prefix


def serving(dev, n_requests: int, loads, tol: float):
    """Served stream of mixed-grid forward/adjoint solves (Poisson arrivals,
    numpy default_rng(0)): every request is first served back to back, one at
    a time, which measures its service time; then, for each load, the stream
    arrives at load x the mean service rate and is served with continuous
    batching.  One-at-a-time latencies at that load follow from the measured
    service times by the FIFO recurrence (start = max(arrival, previous
    finish)): solves are deterministic, so a third pass would repeat them."""
    import dataclasses
    import numpy as np
    from paper_2506_15411_amd import scenes
    from paper_2506_15411_amd.serve import (Server, fifo_one_at_a_time, service_times,
                                            summarize)
    trace = scenes.served_trace(n_requests, 1.0, seed=0)
    unit_arrivals = [r.arrival for r in trace]
    srv = Server(dev, max_active=4, tol=tol, max_iter=SERVE_MAX_ITER)

    def prog(tag):
        def f(res, k):
            if k % 5 == 0 or k == len(trace):
                log(f"[bench] serving {tag}: {k}/{len(trace)} done (last: {res.shape} {res.kind} "
                    f"it {res.iterations} {res.latency * 1e3:.0f} ms)")
        return f

    back_to_back = [dataclasses.replace(r, arrival=0.0) for r in trace]
    b2b = srv.run_sequential(back_to_back, progress=prog("one-at-a-time service"))
    service = service_times(b2b)
    mean_service = float(np.mean([v.seconds for v in service.values()]))
    per = {}
    for r in b2b:
        per.setdefault(str(r.shape), []).append(sum(r.iterations))
    log(f"[bench] serving iterations per grid: " +
        ", ".join(f"{k}: median {int(np.median(v))} max {max(v)}" for k, v in per.items()))
    capped = [{"rid": r.rid, "grid": list(r.shape), "kind": r.kind, "iterations": list(r.iterations),
               "status": r.status} for r in b2b if r.status != 0]

    def rnd(d):
        return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}

    legs = []
    for load in loads:
        rate = load / mean_service
        timed = [dataclasses.replace(r, arrival=a / rate) for r, a in zip(trace, unit_arrivals)]
        log(f"[bench] serving at load {load}: mean service {mean_service * 1e3:.1f} ms, "
            f"rate {rate:.3f}/s")
        mixed = summarize(srv.run(timed, progress=prog(f"continuous batching, load {load}")))
        seq = summarize(fifo_one_at_a_time(timed, service))
        legs.append({"load": load, "arrival_rate_hz": round(rate, 4),
                     "continuous_batching": rnd(mixed), "one_at_a_time": rnd(seq)})
    srv.close()
    n_label = (f"{len(trace)}" if len(trace) >= SERVE_TRACE_LEN else
               f"{len(trace)} of {SERVE_TRACE_LEN} (prefix of the seeded stream)")
    return {
        "requests": n_label,
        "grids": ["64^3 lambda/6", "128^3 lambda/6", "192x192x256 lambda/12", "275x275x315 lambda/16"],
        "tol": tol, "max_iter_per_solve": SERVE_MAX_ITER,
        "scheduler": {"max_active": srv.max_active, "inflight_quanta": srv.inflight,
                      "quantum_target_ms": srv.target_ms,
                      "exclusive_after_s": srv.exclusive_after_s,
                      "exclusive_quantum_scale": srv.exclusive_scale},
        "mean_service_s": round(mean_service, 4),
        "one_at_a_time_method": "FIFO recurrence over the measured back-to-back service times",
        "iterations_per_grid": {k: {"median": int(np.median(v)), "max": int(max(v))}
                                for k, v in per.items()},
        "not_converged": capped,
        "loads": legs,
    }


def design_bench(args, dev):
    """One JSON line for the thickness-map optimisation (optimisation and
    benchmark paragraphs): W warm-up Adam steps, then K timed steps; value =
    voxel-iterations of all forward and adjoint solves per second of wall time."""
    import numpy as np
    import torch
    from paper_2506_15411_amd import scenes
    from paper_2506_15411_amd.design import LensOptimizer
    d = scenes.lens32_design()
    nvox = int(np.prod(d.shape))
    opt = LensOptimizer(d, dev, smoothing=not args.no_smoothing, tol=args.tol,
                        max_iter=args.max_iter, check_every=args.check_every)
    nx, ny, nz = d.shape
    z0, z1 = d.slab
    search = ((d.pml[0], d.pml[1], z1), (nx - d.pml[0], ny - d.pml[1], nz - d.pml[2]))

    def figures():
        # the field of the current design (the optimiser's last forward solve
        # is at the previous p, so solve once more at p)
        with torch.no_grad():
            opt.eps[z0:z1] = opt.map(opt.p)
        opt.plan.set_permittivity(opt.eps)
        E, _ = opt.plan.solve(tol=args.tol, max_iter=args.max_iter, check_every=args.check_every)
        f = opt.plan.lens_metrics(E, *search, aperture_m=d.D)

        def num(v, scale=1.0, nd=4):   # NaN (no half-maximum crossing) -> null
            return round(v * scale, nd) if math.isfinite(v) else None
        return {"eta_f": num(f["eta_f"]), "fwhm_um": [num(w, 1e6, 3) for w in f["fwhm"]],
                "focus": list(f["focus"]), "peak": num(f["peak"], 1.0, 3)}

    if args.profile_iters > 0:
        # the passes on the kinoform start, for rocprofv3 (no optimisation steps)
        with torch.no_grad():
            opt.eps[z0:z1] = opt.map(opt.p)
        opt.plan.set_permittivity(opt.eps)
        warm = max(1, int(1.0e3 / max(1e-3, sum(opt.plan.time_passes(iters=2, E=opt.E).values()))))
        opt.plan.time_passes(iters=warm, E=opt.E)
        passes = opt.plan.time_passes(iters=args.profile_iters, E=opt.E)
        ms = copy_probe(dev)
        log(f"[bench] profile mode: {args.profile_iters} iterations of lens32; passes (ms) {passes}; "
            f"copy probe 1 GiB: {ms:.4f} ms = {2 * 2**30 / ms / 1e6:.0f} GB/s")
        opt.close()
        return 0

    start = figures()
    log(f"[bench] design start: {start}")
    foms = []
    for i in range(args.warmup):
        st = opt.step()
        foms.append(st.fom)
        log(f"[bench] design warm-up {st.step}: |E(r0)|^2 {st.fom:.4e}, it {st.iterations}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = 0
    for i in range(args.steps):
        st = opt.step()
        foms.append(st.fom)
        iters += sum(st.iterations)
        if st.step % 10 == 0 or i == args.steps - 1:
            log(f"[bench] design step {st.step}: |E(r0)|^2 {st.fom:.4e} "
                f"({st.fom / foms[0]:.3f} x start), it {st.iterations}, {st.seconds:.3f} s")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    end = figures()
    log(f"[bench] design end: {end}")
    passes = opt.plan.time_passes(iters=10)
    it_ms = sum(passes.values())
    dom = max(PASS_BYTES, key=lambda k: passes[k])
    achieved = PASS_BYTES[dom] * nvox / (passes[dom] * 1e-3) / 1e9
    opt.close()
    k = max(1, args.steps)
    out = {
        "metric": METRIC, "value": round(nvox * iters / dt / 1e9, 3), "unit": "Gvoxel-iter/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3 / k, 2), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": f"lens32 {d.shape[0]}x{d.shape[1]}x{d.shape[2]} pitch 177 nm: "
                               f"thickness-map Adam step (forward + adjoint CBS to tol "
                               f"{args.tol:g}, gradient, design map), kinoform start D = 32 um "
                               f"NA 0.84 n = 1.54",
                   "voxels": nvox, "smoothing": not args.no_smoothing, "tol": args.tol,
                   "iterations_per_step": iters / k},
        "hbm_frac_iteration": round(ITER_BYTES * nvox / (it_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "iteration_ms": round(it_ms, 4),
        "passes_ms": {kk: round(v, 4) for kk, v in passes.items()},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_from_profile("lens32", dom),
                     "kernel": dom, "alg_bytes_per_launch": PASS_BYTES[dom] * nvox,
                     "avg_launch_ms": round(passes[dom], 4)},
        "design": {"fom_relative": [round(f / foms[0], 4) for f in foms],
                   "lens_start": start, "lens_end": end,
                   "paper_context_s_per_step": 3.7},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        import psutil
        phys = psutil.cpu_count(logical=False)
    except Exception:
        phys = None
    return model, phys, os.cpu_count()


def cpu_baseline(sc, samples: int = 5):
    """FP64 oracle on the host: one CBS iteration of the same workload, timed
    as one warm-up and then the median of `samples` timings.  Each timing is
    one oracle call with max_iter = 1 minus the oracle's own per-solve set-up
    (the potentials and the Green tensor's mode-wise scalars), timed just
    before it."""
    import statistics
    from oracle import cbs as oc
    g = oc.Grid(*sc.shape, sc.pitch, sc.lambda0, sc.n_bg, sc.pml)
    eps = sc.eps_r
    S = oc.plane_wave_source(g, eps)
    r = oc.cbs(g, eps, S, tol=0.0, max_iter=1)          # warm-up
    del r
    times = []
    for k in range(samples):
        t0 = time.perf_counter()
        pot = oc.potentials(g, eps)
        gf = oc.green_factors(g, pot.kt2)
        t1 = time.perf_counter()
        del pot, gf
        t2 = time.perf_counter()
        r = oc.cbs(g, eps, S, tol=0.0, max_iter=1)
        t3 = time.perf_counter()
        del r
        times.append((t3 - t2) - (t1 - t0))
        log(f"[bench] oracle iteration sample {k + 1}/{samples}: {times[-1]:.2f} s")
    med = statistics.median(times)
    model, phys, logical = cpu_info()
    return {
        "value": round(sc.n_vox / med / 1e9, 6),
        "unit": "Gvoxel-iter/s",
        "cores": oc._WORKERS,
        "kind": "oracle",
        "sample": (f"one FP64 oracle CBS iteration on the full {sc.shape[0]}x{sc.shape[1]}x"
                   f"{sc.shape[2]} volume: one warm-up, then the median of {samples} "
                   f"(the oracle's per-solve set-up, potentials and Green factors, timed separately and excluded)"),
        "samples": samples,
        "median_s": round(med, 3),
        "all_s": [round(t, 3) for t in times],
        "cpu_model": model,
        "physical_cores": phys,
        "logical_cpus": logical,
        "threads_note": (f"scipy.fft uses {oc._WORKERS} workers; numpy's elementwise "
                         f"operations run on one thread"),
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="zoneplate100",
                    choices=["zoneplate100", "zoneplate16", "sphere64", "lens32"],
                    help="lens32: the thickness-map optimisation of the 32 um kinoform "
                         "(189 x 189 x 121 at 177 nm); a step is one Adam step")
    ap.add_argument("--no-smoothing", action="store_true",
                    help="lens32: optimise without the Gaussian smoothing filter")
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--max-iter", type=int, default=20000)
    ap.add_argument("--check-every", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=40,
                    help="requests of the seeded 200-request served stream to replay (its "
                         "prefix; 0 = skip serving)")
    ap.add_argument("--serve-loads", default="0.7",
                    help="comma-separated arrival rates as fractions of the one-at-a-time "
                         "service rate")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving leg and print its JSON")
    ap.add_argument("--serve-out", default=None, help="also write the serving JSON here")
    ap.add_argument("--profile-iters", type=int, default=0,
                    help="profiling mode: about 1 s of warm-up iterations, then this many "
                         "CBS iterations of the workload (one launch of each pass per "
                         "iteration) and a 1 GiB device copy used to calibrate memory "
                         "counters; prints no JSON line")
    ap.add_argument("--scpml-steps", type=int, default=0,
                    help="measurement mode: this many GMRES steps of the stretched-layer "
                         "solve (alpha_max 0.75, order 1, restart 40, no graded potential) "
                         "on the workload's scene; logs ms per step, prints no JSON line")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the CBS solver of this package is a "
              "single-GPU path (no multi-GPU decomposition is built); use --gpus 1.",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_2506_15411_amd.solver import Plan

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    loads = [float(v) for v in args.serve_loads.split(",") if v]
    if args.serve_only:
        res = serving(dev, args.serve_requests, loads, args.tol)
        if args.serve_out:
            with open(args.serve_out, "w") as f:
                json.dump(res, f, indent=1)
        print(json.dumps({"serving": res}), flush=True)
        return 0
    if args.workload == "lens32":
        return design_bench(args, dev)
    log(f"[bench] building scene {args.workload}")
    sc = workload(args.workload)
    eps = torch.from_numpy(sc.eps_r).to(dev)
    if args.scpml_steps > 0:
        sp = Plan(sc.shape, sc.pitch, sc.lambda0, sc.n_bg, sc.pml, device=dev, sigma_max=0.0)
        sp.set_permittivity(eps)
        Es = sp.new_field()
        sp.solve_scpml(Es, restart=40, tol=0.0, max_iter=2)   # tables, first launches
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = sp.solve_scpml(Es, restart=40, tol=0.0, max_iter=args.scpml_steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        log(f"[bench] stretched layer on {sc.name}: {st.iterations} GMRES steps, "
            f"{1e3 * dt / st.iterations:.2f} ms per step, residual {st.residual:.3e}")
        return 0
    plan = Plan(sc.shape, sc.pitch, sc.lambda0, sc.n_bg, sc.pml, device=dev)
    plan_order, plan_sigma, plan_kappa = 2, 1.0, 1.1     # the Plan defaults
    E = plan.new_field()
    Ea = plan.new_field()
    lo, hi = sc.design_box
    grad = torch.empty((hi[2] - lo[2], hi[1] - lo[1], hi[0] - lo[0]), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()

    if args.profile_iters > 0:
        plan.set_permittivity(eps)
        # about a second of iterations first, so clocks are at their working level
        warm = max(1, int(1.0e3 / max(1e-3, sum(plan.time_passes(iters=2, E=E).values()))))
        plan.time_passes(iters=warm, E=E)
        passes = plan.time_passes(iters=args.profile_iters, E=E)
        ms = copy_probe(dev)
        log(f"[bench] profile mode: {args.profile_iters} iterations of {sc.name}; "
            f"passes (ms) {passes}; copy probe 1 GiB: {ms:.4f} ms = {2 * 2**30 / ms / 1e6:.0f} GB/s")
        return 0

    def step():
        plan.set_permittivity(eps)
        _, s1 = plan.solve(E, tol=args.tol, max_iter=args.max_iter, check_every=args.check_every)
        _, s2 = plan.adjoint(E_fwd=E, r0=sc.r0, E_adj=Ea, tol=args.tol, max_iter=args.max_iter,
                             check_every=args.check_every)
        plan.gradient(E, Ea, lo, hi, scale=2.0, out=grad)
        return s1, s2

    for i in range(args.warmup):
        s1, s2 = step()
        log(f"[bench] warmup {i}: fwd {s1.iterations} it ({s1.ms:.0f} ms, eta {s1.residual:.2e}), "
            f"adj {s2.iterations} it ({s2.ms:.0f} ms, eta {s2.residual:.2e})")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = 0
    solve_ms = 0.0
    for i in range(args.steps):
        s1, s2 = step()
        iters += s1.iterations + s2.iterations
        solve_ms += s1.ms + s2.ms
        log(f"[bench] step {i}: fwd {s1.iterations} it, adj {s2.iterations} it")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    nvox = sc.n_vox
    value = nvox * iters / dt / 1e9
    iter_rate = nvox * iters / (solve_ms / 1e3) / 1e9

    # per-pass device time (HIP events on the plan's stream)
    passes = plan.time_passes(iters=10)
    log(f"[bench] passes (ms): {passes}")
    dom = max(PASS_BYTES, key=lambda k: passes[k])
    achieved = PASS_BYTES[dom] * nvox / (passes[dom] * 1e-3) / 1e9
    traffic = traffic_from_profile(args.workload, dom)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "kernel": dom,
                "alg_bytes_per_launch": PASS_BYTES[dom] * nvox,
                "avg_launch_ms": round(passes[dom], 4)}
    it_ms = sum(passes.values())
    copy_ms = copy_probe(dev, reps=5)
    copy_gbs = 2 * (1 << 30) / (copy_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gvoxel-iter/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3 / args.steps, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": f"{sc.name} {sc.shape[0]}x{sc.shape[1]}x{sc.shape[2]} "
                               f"pitch {sc.pitch * 1e9:.1f} nm: forward + adjoint CBS (tol "
                               f"{args.tol:g}) + gradient over the design slab",
                   "voxels": nvox, "iterations_per_step": iters / args.steps,
                   "tol": args.tol, "shift_factor": plan_kappa, "pml_per_side": list(sc.pml),
                   "pml_order": plan_order, "sigma_max": plan_sigma},
        "hbm_frac_iteration": round(ITER_BYTES * nvox / (it_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "iteration_ms": round(it_ms, 3),
        "solve_only_gvoxel_iter_s": round(iter_rate, 3),
        "passes_ms": {k: round(v, 4) for k, v in passes.items()},
        "copy_probe_gbs": round(copy_gbs, 1),
        "roofline": roofline,
        "serving": None,
        "cpu_baseline": None,
    }
    if args.serve_requests > 0:
        del E, Ea, grad
        plan.close()
        del plan
        torch.cuda.empty_cache()
        out["serving"] = serving(dev, args.serve_requests, loads, args.tol)
        if args.serve_out:
            with open(args.serve_out, "w") as f:
                json.dump(out["serving"], f, indent=1)
        leg = out["serving"]["loads"][0]
        out["p50_served_latency_s"] = leg["continuous_batching"]["p50_latency_s"]
        out["p99_served_latency_s"] = leg["continuous_batching"]["p99_latency_s"]
    if not args.no_cpu_baseline:
        torch.cuda.empty_cache()
        log("[bench] timing the FP64 oracle on the host")
        out["cpu_baseline"] = cpu_baseline(sc)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
