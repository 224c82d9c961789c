"""The autotuner's cache file format (csrc/tune_cache.h) round trip, without a
GPU: a small host program built with g++ writes entries for every kernel family
and shape field (hop order 5, z-marching, passes of rhs groups, planes per
block), parses them
back, and checks that lines of another arch or runtime version, of another
format version and malformed lines are skipped."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2111_14958_amd", "csrc")

PROG = r"""
#include "tune_cache.h"
#include <stdio.h>
#include <assert.h>
using namespace wd;
static bool same(const CacheKey &a, const CacheKey &b) {
    return a.fam == b.fam && a.L[0] == b.L[0] && a.L[1] == b.L[1] && a.L[2] == b.L[2] && a.L[3] == b.L[3] &&
           a.prec == b.prec && a.nrhs == b.nrhs && a.dag == b.dag;
}
static bool same(const CacheShape &a, const CacheShape &b) {
    return a.block == b.block && a.nr == b.nr && a.remap == b.remap && a.ordered == b.ordered &&
           a.rloop == b.rloop && a.strip == b.strip && a.gmajor == b.gmajor && a.xylds == b.xylds &&
           a.occ == b.occ && a.fpass == b.fpass && a.planes == b.planes;
}
int main() {
    const char *arch = "gfx950:sramecc+:xnack-";
    const int ver = 70226015;
    int n = 0;
    for (int fam = 0; fam < 4; ++fam)
        for (int ord : {1, 3, 5})
            for (int xy : {0, 1, 2}) {
                CacheKey k{fam, {14, 12, 16, 32}, fam % 3, 16 - fam, fam & 1};
                CacheShape s{xy ? 196 : 256, 1 + (ord == 3), 1, ord, 1, xy == 2 ? 2 : 4, xy == 2, xy, 3 * (xy == 1),
                             fam == 1 ? 7 : 0, xy == 1 && ord == 5 ? 2 : 1};
                std::string line = cache_line(arch, ver, k, s, 12.345);
                line.pop_back();   // the reader strips the newline
                CacheKey k2;
                CacheShape s2;
                double us = 0;
                if (!cache_parse(line.c_str(), arch, ver, &k2, &s2, &us) || !same(k, k2) || !same(s, s2) ||
                    us != 12.345) { printf("round trip failed: %s\n", line.c_str()); return 1; }
                // another GPU or another runtime: skipped
                if (cache_parse(line.c_str(), "gfx942:sramecc+:xnack-", ver, &k2, &s2, &us)) return 2;
                if (cache_parse(line.c_str(), arch, ver + 1, &k2, &s2, &us)) return 3;
                ++n;
            }
    CacheKey k; CacheShape s; double us;
    const char *bad[] = {
        "",
        "gfx950 14 14 14 14 1 16 0 256 1 1 3 1 4 0 1 0 45.000",   // the old format: no arch/runtime/family
        "wdtune 1 gfx950:sramecc+:xnack- 70226015 0 14 14 14 14 1 16 0 196 1 1 5 1 4 0 1 0 0 45.000",
        "wdtune 2 gfx950:sramecc+:xnack- 70226015 0 14 14 14 14 1 16 0 196 1 1 5 1 4 0 1 0 0 45.000",   // version 2
        "wdtune 3 gfx950:sramecc+:xnack- 70226015 0 14 14 14 14 1 16 0 196 1 1 5 1 4 0 1 0 0 45.000",   // a field short
        "wdtune 3 gfx950:sramecc+:xnack- 70226015 0 14 14 14 14 1 16 0 196 1 1 5 1 4 0 1 0 0 2 45.000 extra",
        "wdtune 3 gfx950:sramecc+:xnack- 70226015 0 14 14 14 14 1 16 0 196 1 1 5 1 4 0 1 0 0 2x 45.000",
    };
    for (const char *b : bad)
        if (cache_parse(b, "gfx950:sramecc+:xnack-", 70226015, &k, &s, &us)) { printf("accepted: %s\n", b); return 4; }
    printf("ok %d\n", n);
    return 0;
}
"""


def test_tune_cache_round_trip(tmp_path):
    src = tmp_path / "rt.cpp"
    src.write_text(PROG)
    exe = tmp_path / "rt"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-I", CSRC, str(src), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip() == "ok 36"
