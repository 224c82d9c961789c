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
        const wd::Geom g = wd::geom_of(d, -1);
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


FASTDIV = r"""
#include "wd_device.h"
#include <stdio.h>
#include <stdint.h>
// every divisor up to 4200 against every dividend up to 70000, then a
// pseudo-random sample of large dividends and divisors, and the extremes
int main() {
    long bad = 0, checked = 0;
    auto check = [&](int n, int d, wd::FastDiv f) {
        ++checked;
        if (wd::fastdiv(n, f) != n / d) {
            if (bad < 5) printf("n %d d %d got %d\n", n, d, wd::fastdiv(n, f));
            ++bad;
        }
    };
    for (int d = 1; d <= 4200; ++d) {
        const wd::FastDiv f = wd::fastdiv_make(d);
        for (int n = 0; n < 70000; ++n) check(n, d, f);
        check(2147483647, d, f);
        check(2147483647 - d, d, f);
    }
    uint64_t x = 88172645463325252ull;
    for (int i = 0; i < 4000000; ++i) {
        x ^= x << 13; x ^= x >> 7; x ^= x << 17;
        const int d = 1 + (int)((x >> 33) % ((i & 1) ? 2147483646u : 100000u));
        const int n = (int)((x & 0x7fffffff) >> (i % 24));
        check(n, d, wd::fastdiv_make(d));
    }
    const int ds[] = {1, 2, 3, 1073741823, 1073741824, 1073741825, 2147483646, 2147483647};
    for (int d : ds)
        for (int n : {0, 1, d - 1, d, 2147483646, 2147483647})
            if (n >= 0) check(n, d, wd::fastdiv_make(d));
    printf("checked %ld bad %ld\n", checked, bad);
    return bad != 0;
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not found")
def test_fastdiv_matches_integer_division(tmp_path):
    """The kernels divide by lattice extents with a multiply-high, an add and
    a shift (division by invariant integers); the host build of the same
    functions against C's integer division."""
    src = tmp_path / "fastdiv.cpp"
    exe = tmp_path / "fastdiv"
    src.write_text(FASTDIV)
    subprocess.run(["hipcc", "-x", "hip", "--offload-arch=gfx950", "-std=c++17", "-O2", "-w",
                    "-I", CSRC, str(src), "-o", str(exe)], check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "bad 0" in r.stdout
