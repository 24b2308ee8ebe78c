"""Unit test of the serving engine's first-fit range allocator (host C++),
built with the host compiler: random allocate/release sequences against a
brute-force occupancy model (first fit, no overlap, full coalescing)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2202_02264_amd", "csrc")

PROBE = r"""
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "dsmc_range_alloc.h"
int main() {
  const int cap = 200;
  dsmc::RangeAlloc ra;
  ra.reset(cap);
  std::vector<int> used(cap, 0);           // brute-force model
  std::vector<std::pair<int, int>> live;
  unsigned s = 12345u;
  auto rnd = [&]() { s = s * 1103515245u + 12345u; return (s >> 8) & 0xffff; };
  for (int it = 0; it < 20000; ++it) {
    if (live.empty() || rnd() % 3) {
      const int len = 1 + rnd() % 40;
      int want = -1;                        // first fit in the model
      for (int a = 0; a + len <= cap && want < 0; ++a) {
        bool ok = true;
        for (int i = a; i < a + len; ++i) ok = ok && !used[i];
        if (ok) want = a;
      }
      const int got = ra.alloc(len);
      if (got != want) { printf("alloc %d: got %d want %d\n", len, got, want); return 1; }
      if (got >= 0) {
        for (int i = got; i < got + len; ++i) used[i] = 1;
        live.push_back({got, len});
      }
    } else {
      const size_t k = rnd() % live.size();
      ra.release(live[k].first, live[k].second);
      for (int i = live[k].first; i < live[k].first + live[k].second; ++i) used[i] = 0;
      live.erase(live.begin() + k);
    }
    // free ranges are exactly the maximal runs of unused units
    int runs = 0;
    for (int i = 0; i < cap; ++i) runs += !used[i] && (i == 0 || used[i - 1]);
    if ((int)ra.free_ranges().size() != runs) { printf("not coalesced at %d\n", it); return 1; }
    for (auto& fr : ra.free_ranges())
      for (int i = fr.first; i < fr.first + fr.second; ++i)
        if (used[i]) { printf("free range overlaps a live one\n"); return 1; }
  }
  printf("ok\n");
  return 0;
}
"""


def test_range_alloc_against_model(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    src = tmp_path / "ra.cpp"
    src.write_text(PROBE)
    exe = tmp_path / "ra"
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout
