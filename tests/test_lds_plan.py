"""The build kernel's LDS plan (csrc/kfplan.h), checked on the CPU: at the
benchmark's cap of 6 every variant (FP32 / FP64, plain / learned window,
Cartesian / hybrid state) fits two blocks of four waves in a CU's 160 KB,
so the launch keeps two waves per SIMD; the regions follow each other
without overlap, 16-byte aligned; an FP64 plan holds the state between
layers (6 + NPL doubles per lane) and a stash of only the 21 - NPL
covariance entries left in registers, an FP32 plan no state and the full
27-value stash.  The program includes the header and prints its plan."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CU_LDS = 160 * 1024

PROGRAM = r"""
#include <cstdio>
#include "kfplan.h"
int main() {
  for (int cap = 1; cap <= 8; ++cap)
    for (int t : {4, 8})
      for (int learned = 0; learned < 2; ++learned)
        for (int hyb = 0; hyb < 2; ++hyb) {
          const LdsPlan p = lds_plan(17, 4, cap, t, learned, hyb);
          printf("%d %d %d %d %d %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", cap, t, learned, hyb,
                 xs_npl(t, learned, hyb), p.stash, p.rec, p.recf, p.acc, p.pub, p.tl, p.mlp, p.xs, p.total);
        }
  return 0;
}
"""


@pytest.fixture(scope="module")
def plans(tmp_path_factory):
    if not os.path.exists(HIPCC) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("ldsplan")
    src = d / "ldsplan.hip"
    src.write_text(PROGRAM)
    exe = d / "ldsplan"
    cmd = [HIPCC, "-O1", "-std=c++17", "--cuda-host-only", "-w", "-I", os.path.join(ROOT, "paper_1711_06571_amd", "csrc"),
           "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    rows = []
    for line in out:
        if line.strip():
            v = [int(x) for x in line.split()]
            rows.append(dict(zip(["cap", "t", "learned", "hyb", "npl", "stash", "rec", "recf", "acc", "pub", "tl", "mlp",
                                  "xs", "total"], v)))
    return rows


def test_two_blocks_per_cu_at_cap_6(plans):
    for p in plans:
        if p["cap"] == 6:
            assert 2 * p["total"] <= CU_LDS, p


def test_regions_in_order_and_aligned(plans):
    for p in plans:
        offs = [p["stash"], p["rec"], p["recf"], p["acc"], p["pub"], p["tl"]]
        assert offs == sorted(offs) and all(o % 16 == 0 for o in offs), p
        assert p["xs"] % 16 == 0 and p["xs"] <= p["total"], p


def test_state_and_stash_sizes(plans):
    nw = 4
    for p in plans:
        if p["t"] == 8:
            assert p["npl"] == (2 if p["learned"] else 20 if p["hyb"] else 12), p
            assert p["rec"] - p["stash"] == nw * (21 - p["npl"]) * 64 * 4, p
            assert p["total"] - p["xs"] == nw * (6 + p["npl"]) * 64 * 8, p
        else:
            assert p["npl"] < 0, p
            assert p["rec"] - p["stash"] == nw * 27 * 64 * 4, p
            assert p["total"] == p["xs"], p
