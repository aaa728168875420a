"""CPU check of the XCD-banded tile order of the tile kernels (kk_common.hpp):
for every tile count up to 6000, xcd_tile is a bijection on [0, n) (so every
tile is swept exactly once per launch, whatever the count), and the tiles of
each XCD (workgroups b with the same b mod 8) form one contiguous run.  The
header is compiled host-only with hipcc, without a GPU."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1309_4349_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

PROGRAM = r"""
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "kk_common.hpp"
int main(int argc, char** argv) {
  const int maxn = atoi(argv[1]);
  for (int n = 1; n <= maxn; ++n) {
    std::vector<int> seen(n, 0);
    std::vector<int> lo(8, n), hi(8, -1), cnt(8, 0);
    for (int b = 0; b < n; ++b) {
      const int t = kk::xcd_tile(b, n);
      if (t < 0 || t >= n || seen[t]) { printf("not a bijection: n=%d b=%d t=%d\n", n, b, t); return 1; }
      seen[t] = 1;
      const int x = b % 8;
      lo[x] = t < lo[x] ? t : lo[x];
      hi[x] = t > hi[x] ? t : hi[x];
      cnt[x] += 1;
    }
    for (int x = 0; x < 8; ++x)
      if (cnt[x] && hi[x] - lo[x] + 1 != cnt[x]) { printf("XCD %d not contiguous: n=%d\n", x, n); return 1; }
  }
  printf("ok %d\n", maxn);
  return 0;
}
"""


def test_xcd_tile_is_a_banded_bijection(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not installed")
    src = tmp_path / "xcd.cpp"
    exe = tmp_path / "xcd"
    src.write_text(PROGRAM)
    subprocess.run([HIPCC, "-x", "hip", "--cuda-host-only", "-O2", "-std=c++17", "-I", CSRC, "-o", str(exe),
                    str(src)], check=True, capture_output=True)
    r = subprocess.run([str(exe), "6000"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "ok 6000"
