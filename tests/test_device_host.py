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


PRECHECK = r'''
#include "lfdpr_device.h"
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>
#include <algorithm>
using namespace lfdpr;
int main() {
  std::mt19937 rng(2024);
  std::uniform_real_distribution<float> U(0.0f, 1.0f);
  long culled = 0, seen_any = 0, wrong = 0, tris = 0;
  for (int rig = 0; rig < 400; ++rig) {
    Rig rg{};
    const int V = 2 + (int)(rng() % 63);
    rg.n_views = V;
    rg.W = 16 + (int)(rng() % 1024);
    rg.H = 16 + (int)(rng() % 1024);
    const float D = 0.5f + 4.0f * U(rng), cone = 0.05f + 1.2f * U(rng), fovy = 0.2f + 1.0f * U(rng);
    rg.fy = (float)((rg.H / 2.0) / std::tan(fovy / 2.0));
    rg.fx = rg.fy * (0.5f + U(rng));
    rg.cx = rg.W / 2.0f;
    rg.cy = rg.H / 2.0f;
    rg.rD = 1.0f / D;
    rg.znear = 0.05f * D;
    rg.fxfy = rg.fx * rg.fy;
    std::vector<float> eye(V);
    const bool jitter = rng() & 1;
    for (int r = 0; r < V; ++r) {
      const double q = jitter ? r + U(rng) : r + 0.5;
      eye[r] = (float)(D * std::tan(cone / 2.0) * (2.0 * q / V - 1.0));
    }
    rg.eye = eye.data();
    rg.eye_lo = *std::min_element(eye.begin(), eye.end());
    rg.eye_hi = *std::max_element(eye.begin(), eye.end());
    for (int t = 0; t < 2000; ++t) {
      // vertices around the frustum, some far outside it, all in front of z_near
      float P[3][3];
      const float spread = (rng() & 3) == 0 ? 20.0f : 1.5f;
      for (int k = 0; k < 3; ++k) {
        const float z = rg.znear + 3.0f * D * U(rng);
        P[k][0] = (2.0f * U(rng) - 1.0f) * spread * z;
        P[k][1] = (2.0f * U(rng) - 1.0f) * spread * z;
        P[k][2] = z;
      }
      const float e1[3] = {P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2]};
      const float e2[3] = {P[2][0] - P[0][0], P[2][1] - P[0][1], P[2][2] - P[0][2]};
      const float n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
      const float nl = sqrtf((n[0] * n[0] + n[1] * n[1]) + n[2] * n[2]);
      if (!(nl > 0.0f) || std::isinf(nl)) continue;
      TriRec R{};
      R.nx = n[0] / nl; R.ny = n[1] / nl; R.nz = n[2] / nl;
      R.p0x = P[0][0]; R.p0y = P[0][1]; R.p0z = P[0][2];
      R.h = (R.nx * P[0][0] + R.ny * P[0][1]) + R.nz * P[0][2];
      vertex_proj(rg, P[0][0], P[0][1], P[0][2], R.a0, R.c0, R.y0);
      vertex_proj(rg, P[1][0], P[1][1], P[1][2], R.a1, R.c1, R.y1);
      vertex_proj(rg, P[2][0], P[2][1], P[2][2], R.a2, R.c2, R.y2);
      ++tris;
      bool any = false;
      for (int r = 0; r < V && !any; ++r) {
        int32_t qx[3], qy[3];
        any = view_active(rg, R, eye[r], qx, qy);
      }
      const bool may = may_be_seen(rg, R);
      if (any) ++seen_any;
      if (!may) ++culled;
      if (any && !may) {
        if (wrong < 5) std::printf("wrongly culled: rig %d tri %d\n", rig, t);
        ++wrong;
      }
    }
  }
  std::printf("triangles %ld, seen by some view %ld, culled by the precheck %ld, wrongly culled %ld\n", tris, seen_any,
              culled, wrong);
  return wrong != 0 || culled == 0 || seen_any == 0;
}
'''


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_precheck_never_culls_a_visible_triangle():
    """The set-up's "no eye sees it" test (may_be_seen: behind the plane for
    both ends of the eye range, rows off the view, all vertices left or right
    of the view at both ends) is false only where view_active is false for
    every eye of the rig: random rigs (jittered eye tables included) and
    random triangles around and far outside the frustum."""
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "pc.hip")
        exe = os.path.join(d, "pc")
        open(src, "w").write(PRECHECK)
        cmd = [HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17", "-ffp-contract=off", "-I",
               os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2601_19901_amd", "csrc"), "-o", exe, src]
        subprocess.run(cmd, check=True, capture_output=True, timeout=600)
        out = subprocess.run([exe], capture_output=True, text=True, timeout=600)
        print(out.stdout)
        assert out.returncode == 0, out.stdout + out.stderr
        assert "wrongly culled 0" in out.stdout
