"""Tile order of the trailing update (host build of the device function ``update_tile``).

The update kernel maps a task-local tile number to a tile (i, j) of the lower-triangular tile set
{j < ct, j <= i < R}; the symbolic schedule sizes each launch as ct R - ct (ct - 1) / 2 tiles.  The
mapping must hit every tile of that set exactly once and report the numbers past it as empty,
or a tile would be updated twice or not at all.  Checked exhaustively for every shape up to 200
row tiles (fronts of up to 12,800 rows).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

CHECK = r"""
#include "kernels.h"
#include <cstdio>
#include <vector>
int main() {
  long bad = 0, cases = 0;
  for (int64_t R = 1; R <= 200; ++R)
    for (int64_t ct = 1; ct <= R; ++ct) {
      ++cases;
      const int64_t n = ct * R - ct * (ct - 1) / 2;
      std::vector<char> seen(R * ct, 0);
      for (int64_t lt = 0; lt < n; ++lt) {
        int64_t i = -1, j = -1;
        if (!sgn::update_tile(lt, R, ct, i, j) || j < 0 || j >= ct || i < j || i >= R || seen[i * ct + j]) {
          ++bad;
          break;
        }
        seen[i * ct + j] = 1;
      }
      int64_t i, j;
      if (sgn::update_tile(n, R, ct, i, j) || sgn::update_tile(n + 5, R, ct, i, j) ||
          sgn::update_tile(-1, R, ct, i, j))
        ++bad;
    }
  std::printf("%ld %ld\n", cases, bad);
  return 0;
}
"""


@pytest.mark.skipif(shutil.which(HIPCC) is None and not os.path.exists(HIPCC), reason="hipcc not available")
def test_update_tile_order_is_a_bijection_onto_the_lower_tiles(tmp_path):
    src = tmp_path / "check.cpp"
    src.write_text(CHECK)
    exe = tmp_path / "check"
    inc = os.path.join(ROOT, "paper_2107_03285_amd", "csrc")
    subprocess.run([HIPCC, "-O2", "-std=c++17", "-I", inc, str(src), "-o", str(exe)], check=True,
                   capture_output=True, timeout=300)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=300).stdout.split()
    assert out == ["20100", "0"]
