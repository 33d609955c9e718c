"""The sorting networks the builders sort their candidate lists with
(csrc/kfwave.h: 4, 6 and 8 inputs), checked on the CPU: by the 0-1 principle
a comparator network sorts every input iff it sorts every 0/1 input, so each
table is run over all 2^N 0/1 vectors (and, for N = 6, over all 720
permutations of distinct keys).  The program includes the header and applies
its comparator tables as they are; only the compare-exchange is written
here."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

PROGRAM = r"""
#include <algorithm>
#include <cstdio>
#include <vector>
#include "kfwave.h"
template <int N> static int check() {
  int bad = 0;
  for (int m = 0; m < (1 << N); ++m) {
    int v[N];
    for (int k = 0; k < N; ++k) v[k] = (m >> k) & 1;
    for (int t = 0; t < SortNet<N>::len; ++t) {
      const int a = SortNet<N>::c[t][0], b = SortNet<N>::c[t][1];
      if (!(a < b && b < N)) return -1;
      if (v[b] < v[a]) std::swap(v[a], v[b]);
    }
    if (!std::is_sorted(v, v + N)) ++bad;
  }
  return bad;
}
int main() {
  std::vector<int> p = {0, 1, 2, 3, 4, 5};
  int bad6 = 0;
  do {
    int v[6];
    for (int k = 0; k < 6; ++k) v[k] = p[k];
    for (int t = 0; t < SortNet<6>::len; ++t) {
      const int a = SortNet<6>::c[t][0], b = SortNet<6>::c[t][1];
      if (v[b] < v[a]) std::swap(v[a], v[b]);
    }
    if (!std::is_sorted(v, v + 6)) ++bad6;
  } while (std::next_permutation(p.begin(), p.end()));
  printf("%d %d %d %d\n", check<4>(), check<6>(), check<8>(), bad6);
  printf("%d %d %d\n", SortNet<4>::len, SortNet<6>::len, SortNet<8>::len);
  return 0;
}
"""


@pytest.fixture(scope="module")
def output(tmp_path_factory):
    if not os.path.exists(HIPCC) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("sortnet")
    src = d / "sortnet.hip"
    src.write_text(PROGRAM)
    exe = d / "sortnet"
    cmd = [HIPCC, "-O1", "-std=c++17", "--cuda-host-only", "-w", "-I", os.path.join(ROOT, "paper_1711_06571_amd", "csrc"),
           "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    return subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")


def test_every_network_sorts_all_zero_one_inputs(output):
    b4, b6, b8, bperm = (int(x) for x in output[0].split())
    assert (b4, b6, b8) == (0, 0, 0), output[0]
    assert bperm == 0


def test_network_sizes(output):
    # 5, 12 and 19 comparators: the known optimal sizes for 4 and 6 inputs
    # and Batcher's odd-even merge for 8
    assert output[1].split() == ["5", "12", "19"]
