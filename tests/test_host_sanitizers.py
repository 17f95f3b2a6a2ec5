"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only; no kernel is launched).

tests/host_sanitize/host_checks.cpp includes the C-ABI source and drives its
host paths: the size registry, the FP64 twiddle tables of every registered
split, the workspace carve-ups, the argument checks of every entry point, the
source set-up, the FWHM interpolation of the lens figures and, with no GPU,
plan creation up to its first HIP call and the clean-up after it fails.  It is
compiled with the sanitizers on its host code only and linked with the size
registries of the library build (paper_2506_15411_amd/_lib/obj).  Any report
of either sanitizer, a leak included, or a failed check fails the test.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OBJ = os.path.join(ROOT, "paper_2506_15411_amd", "_lib", "obj")
SIZES = [os.path.join(OBJ, f"sizes_{s}.o") for s in ("small", "mid", "large")]
SANITIZE = [
    "-Xarch_host", "-fsanitize=address",
    "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=undefined",
]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    return None


def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    cc = _hipcc()
    if cc is None:
        pytest.skip("hipcc not found")
    if not all(os.path.exists(o) for o in SIZES):
        pytest.skip("library objects not built (python -m paper_2506_15411_amd.build)")
    obj, exe = str(tmp_path / "host_checks.o"), str(tmp_path / "host_checks")
    common = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    r = subprocess.run(
        [cc, "-x", "hip", "-std=c++17", "-O1", "-g", *common, *SANITIZE,
         "-Xarch_host", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-c",
         os.path.join(ROOT, "tests", "host_sanitize", "host_checks.cpp"), "-o", obj],
        capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([cc, "--offload-arch=gfx950", *SANITIZE, obj, *SIZES, "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    out = r.stdout + r.stderr
    print(out[-2000:])
    assert "AddressSanitizer" not in out and "LeakSanitizer" not in out, out[-6000:]
    assert "runtime error" not in out, out[-6000:]
    assert r.returncode == 0, out[-6000:]
    assert "host checks passed" in out
