// Text format of the autotuner's cache file (the file WD_TUNE_CACHE names):
// one line per tuned launch shape,
//
//   wdtune 3 <arch> <hip runtime> <family> <Lx> <Ly> <Lz> <Lt> <prec> <nrhs> <dagger>
//            <block> <nr> <remap> <hop order> <rhs loop> <strip> <group-major>
//            <xy_lds> <occ> <fpass> <planes> <us>
//
// arch is the device's gcnArchName (e.g. gfx950:sramecc+:xnack-), hip runtime
// the version hipRuntimeGetVersion reports, family the kernel family of the
// shape table (operator, CG phase A, CG phase B, reliable update), xy_lds 2 the
// z-marching variant, planes the xy-planes per plane-blocked block.  A line is
// used only when its format version is 3 and its arch and runtime version
// are the running process's: shapes tuned on another GPU or another ROCm are
// skipped, and so are malformed lines.  Later lines of a key replace earlier
// ones.  Plain host C++ (no HIP), so that the format can be tested without a GPU.
#pragma once

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>

namespace wd {

struct CacheKey {
    int fam, L[4], prec, nrhs, dag;
};
struct CacheShape {
    int block, nr, remap, ordered, rloop, strip, gmajor, xylds, occ, fpass, planes;
};

inline std::string cache_line(const char *arch, int hip_version, const CacheKey &k, const CacheShape &s, double us) {
    char buf[512];
    snprintf(buf, sizeof buf,
             "wdtune 3 %s %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %.3f\n", arch, hip_version,
             k.fam, k.L[0], k.L[1], k.L[2], k.L[3], k.prec, k.nrhs, k.dag, s.block, s.nr, s.remap, s.ordered, s.rloop,
             s.strip, s.gmajor, s.xylds, s.occ, s.fpass, s.planes, us);
    return buf;
}

// true when `line` is a well-formed entry for this arch and runtime version:
// exactly 24 space-separated tokens, every integer field a whole integer
inline bool cache_parse(const char *line, const char *arch, int hip_version, CacheKey *k, CacheShape *s,
                        double *us) {
    char buf[512];
    if (strlen(line) >= sizeof buf) return false;
    strcpy(buf, line);
    const char *tok[25];
    int n = 0;
    for (char *save = nullptr, *t = strtok_r(buf, " \t\r\n", &save); t; t = strtok_r(nullptr, " \t\r\n", &save)) {
        if (n == 25) return false;
        tok[n++] = t;
    }
    if (n != 24 || strcmp(tok[0], "wdtune") != 0 || strcmp(tok[1], "3") != 0 || strcmp(tok[2], arch) != 0)
        return false;
    int v[20];
    for (int i = 0; i < 20; ++i) {
        char *end = nullptr;
        const long x = strtol(tok[3 + i], &end, 10);
        if (end == tok[3 + i] || *end != '\0' || x < -2147483647L || x > 2147483647L) return false;
        v[i] = (int)x;
    }
    char *end = nullptr;
    const double t = strtod(tok[23], &end);
    if (end == tok[23] || *end != '\0') return false;
    if (v[0] != hip_version) return false;
    *k = CacheKey{v[1], {v[2], v[3], v[4], v[5]}, v[6], v[7], v[8]};
    *s = CacheShape{v[9], v[10], v[11], v[12], v[13], v[14], v[15], v[16], v[17], v[18], v[19]};
    *us = t;
    return true;
}

}  // namespace wd
