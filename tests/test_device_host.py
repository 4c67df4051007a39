"""Host-side checks of the integer helpers in csrc/lfdpr_device.h (compiled for
the host with hipcc; no GPU needed): the double-based floor division that the
lattice rows use equals exact integer floor division over its whole range,
including quotients just below, at and above an integer."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

PROGRAM = r'''
#include "lfdpr_device.h"
#include <cstdio>
#include <random>
using namespace lfdpr;
static int check(int64_t a, int64_t b, long& bad) {
  if (floor_div_53(a, b) != floor_div(a, b)) {
    if (bad < 5) std::printf("mismatch a=%lld b=%lld got %lld want %lld\n", (long long)a, (long long)b,
                             (long long)floor_div_53(a, b), (long long)floor_div(a, b));
    ++bad;
  }
  return 1;
}
int main() {
  std::mt19937_64 rng(12345);
  long n = 0, bad = 0;
  for (int it = 0; it < 2000000; ++it) {
    const int eb = 1 + (int)(rng() % 31), ea = (int)(rng() % 51);
    const int64_t b = 1 + (int64_t)(rng() % (uint64_t)(1ll << eb));
    int64_t a = (int64_t)(rng() % (uint64_t)(1ll << ea));
    if (rng() & 1) a = -a;
    n += check(a, b, bad);
    // quotient boundaries: k*b - 1, k*b, k*b + 1
    const int64_t k = (int64_t)(rng() % (uint64_t)(1ll << 17)) * ((rng() & 1) ? 1 : -1);
    if (k * b < (1ll << 50) && -k * b < (1ll << 50))
      for (int d = -1; d <= 1; ++d) n += check(k * b + d, b, bad);
  }
  const int64_t edges[] = {(1ll << 48) - 1, -(1ll << 48), (1ll << 52) - 3, -(1ll << 52) + 5, 0, -1, 1};
  for (int64_t a : edges)
    for (int64_t b : {1ll, 2ll, 3ll, 255ll, 256ll, 1ll << 30, (1ll << 31) - 1}) n += check(a, b, bad);
  std::printf("checked %ld bad %ld\n", n, bad);
  return bad != 0;
}
'''


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_floor_div_53_equals_integer_floor_division():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "fd.hip")
        exe = os.path.join(d, "fd")
        open(src, "w").write(PROGRAM)
        cmd = [HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
               "-I", os.path.join(ROOT, "paper_2601_19901_amd", "csrc"), "-o", exe, src]
        subprocess.run(cmd, check=True, capture_output=True, timeout=600)
        out = subprocess.run([exe], capture_output=True, text=True, timeout=600)
        print(out.stdout)
        assert out.returncode == 0, out.stdout + out.stderr
        assert "bad 0" in out.stdout
