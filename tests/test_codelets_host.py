"""The register DFT codelets (csrc/codelets.hpp) compiled for the host and
checked against numpy's FFT in complex128, CPU only.

Every length the supported axis splits use, plus the primes that take the
Rader-ordered split form (17, 29, 37, 41, 53), forward and inverse: the FP32
result of dft<N, S> must match the DFT of the same FP32 inputs to a relative
L2 error of a few FP32 roundings times log N."""

import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2506_15411_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

LENGTHS = [2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 20, 21, 23, 24, 25,
           27, 29, 31, 32, 35, 36, 37, 41, 53]

HARNESS = r"""
#include "codelets.hpp"
#include <cstdio>
#include <vector>
template <int N, int S> void one(FILE* in, FILE* out) {
  float2 a[N];
  if (fread(a, sizeof(float2), N, in) != (size_t)N) return;
  cbs::dft<N, S>(a);
  fwrite(a, sizeof(float2), N, out);
}
template <int N> void both(FILE* in, FILE* out) { one<N, -1>(in, out); one<N, +1>(in, out); }
int main(int argc, char** argv) {
  FILE* in = fopen(argv[1], "rb");
  FILE* out = fopen(argv[2], "wb");
  if (!in || !out) return 1;
  %s
  fclose(in);
  fclose(out);
  return 0;
}
"""


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not found")
    d = tmp_path_factory.mktemp("codelets")
    src = d / "h.cpp"
    src.write_text(HARNESS % "\n  ".join(f"both<{n}>(in, out);" for n in LENGTHS))
    exe = d / "h"
    cmd = [HIPCC if os.path.exists(HIPCC) else "hipcc", "-std=c++17", "-O2", "-x", "hip",
           "--offload-host-only", "-I", CSRC, str(src), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return d, exe


def test_codelets_match_numpy_fft(harness):
    d, exe = harness
    rng = np.random.default_rng(11)
    cases = []
    for n in LENGTHS:
        for s in (-1, 1):
            x = (rng.normal(size=n) + 1j * rng.normal(size=n)).astype(np.complex64)
            cases.append((n, s, x))
    with open(d / "in.bin", "wb") as f:
        for _, _, x in cases:
            f.write(x.tobytes())
    subprocess.run([str(exe), str(d / "in.bin"), str(d / "out.bin")], check=True)
    out = np.fromfile(d / "out.bin", dtype=np.complex64)
    assert out.size == sum(n for n, _, _ in cases)
    o = 0
    for n, s, x in cases:
        got = out[o:o + n].astype(np.complex128)
        o += n
        xd = x.astype(np.complex128)
        ref = np.fft.fft(xd) if s < 0 else np.fft.ifft(xd) * n
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert err < 3e-7 * max(1.0, np.log2(n)), (n, s, err)
