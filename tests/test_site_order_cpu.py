"""Host-side check of the kernels' processing order (order_site in wd_device.h).

The operator and CG kernels map position L of their processing order to a
lattice site.  Every order must be a permutation of the sites (each site
computed exactly once, every index in bounds) and must keep each xy-plane
contiguous (coalesced wavefront accesses).  The function is compiled for the
host with hipcc and run on the CPU over ragged and regular lattices and every
strip width.
"""
import os
import shutil
import subprocess

import pytest

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_2111_14958_amd", "csrc")

PROGRAM = r"""
#include "wd_device.h"
#include <stdio.h>
#include <vector>
int main() {
    const int dims[][4] = {{4,4,4,4}, {14,14,14,14}, {16,16,16,32}, {3,5,7,2}, {8,8,13,5}, {2,2,2,2},
                           {6,4,9,3}};
    int bad = 0, checked = 0;
    for (auto &d : dims) {
        wd::Geom g;
        for (int k = 0; k < 4; ++k) g.L[k] = d[k];
        g.S[0] = 1; g.S[1] = d[0]; g.S[2] = d[0] * d[1]; g.S[3] = d[0] * d[1] * d[2];
        g.V = d[0] * d[1] * d[2] * d[3];
        const int P = g.S[2];
        for (int W = 0; W <= d[2] + 1; ++W) {
            std::vector<int> seen(g.V, 0);
            for (int L = 0; L < g.V; ++L) {
                const int s = wd::order_site(g, W, L);
                if (s < 0 || s >= g.V) { ++bad; continue; }
                ++seen[s];
                if (L % P && s != wd::order_site(g, W, L - 1) + 1) ++bad;   // plane contiguous
            }
            for (int s = 0; s < g.V; ++s) bad += seen[s] != 1;
            ++checked;
        }
    }
    printf("checked %d bad %d\n", checked, bad);
    return bad != 0;
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not found")
def test_processing_orders_are_permutations(tmp_path):
    src = tmp_path / "order.cpp"
    exe = tmp_path / "order"
    src.write_text(PROGRAM)
    subprocess.run(["hipcc", "-x", "hip", "--offload-arch=gfx950", "-std=c++17", "-O1", "-w",
                    "-I", CSRC, str(src), "-o", str(exe)], check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "bad 0" in r.stdout
