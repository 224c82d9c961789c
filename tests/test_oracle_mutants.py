"""Plant plausible mistakes in copies of the oracle source (on the CPU) and
check that the pins reject every one of them: a dropped term, a wrong sign,
a transposed operand, a wrong index, a wrong boundary, a wrong CG scalar."""
import os
import subprocess

import pytest

import oracle
import pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "wilson_oracle.c")

# (name, text to replace, replacement, which occurrence (0-based))
MUTANTS = [
    ("forward projector sign", "Pf[mu][a][b] = id - sgn", "Pf[mu][a][b] = id + sgn", 0),
    ("backward projector sign", "Pb[mu][a][b] = id + sgn", "Pb[mu][a][b] = id - sgn", 0),
    ("t direction dropped", "for (int mu = 0; mu < 4; ++mu) {\n            /* forward",
     "for (int mu = 0; mu < 3; ++mu) {\n            /* forward", 0),
    ("forward link transposed", "Uf[3 * a + b]", "Uf[3 * b + a]", 0),
    ("backward link not daggered", "conj(Ub[3 * b + a])", "Ub[3 * a + b]", 0),
    ("backward link taken at x", "(nb * 4 + mu) * 9", "(s * 4 + mu) * 9", 0),
    ("periodic time boundary forward", "(double)t_sign : 1.0;", "1.0 : 1.0;", 0),
    ("periodic time boundary backward", "(double)t_sign : 1.0;", "1.0 : 1.0;", 1),
    ("mass term", "(4.0 + m0) * ps", "(4.0 + 2.0 * m0) * ps", 0),
    ("hopping factor 1/2 dropped", "- 0.5 * acc[sp][a]", "- acc[sp][a]", 0),
    ("gamma_y entry sign", "G[1][0][3] = -1", "G[1][0][3] = 1", 0),
    ("gamma_z entry conjugated", "G[2][0][2] = I", "G[2][0][2] = -I", 0),
    ("dagger flag ignored", "const double sgn = dagger ? -1.0 : 1.0;",
     "const double sgn = 1.0;", 0),
    ("forward neighbour off by one", "cf[mu] = (c[mu] + 1) % L[mu];",
     "cf[mu] = (c[mu] + 2) % L[mu];", 0),
    ("colour index of spinor", "pf[3 * sp + b]", "pf[3 * b + sp % 3]", 0),
    ("CG alpha inverted", "double alpha = rho / sigma;", "double alpha = sigma / rho;", 0),
    ("CG beta inverted", "double beta = rho_new / rho;", "double beta = rho / rho_new;", 0),
    ("CG solution updated with p", "axpy(alpha, q, x, n);", "axpy(alpha, p, x, n);", 0),
    ("CG residual update sign", "axpy(-alpha, t, r, n);", "axpy(alpha, t, r, n);", 0),
    ("CG direction without beta", "p[i] = r[i] + beta * p[i];", "p[i] = r[i];", 0),
    ("BiCGSTAB residual update sign", "r[i] = sv[i] - omega * t[i];", "r[i] = sv[i] + omega * t[i];", 0),
    ("BiCGSTAB alpha inverted", "alpha = rho / rhv;", "alpha = rhv / rho;", 0),
    ("BiCGSTAB x update without omega s", "x[i] += alpha * p[i] + omega * sv[i];",
     "x[i] += alpha * p[i];", 0),
]


def _replace_nth(text, old, new, n):
    idx = -1
    for _ in range(n + 1):
        idx = text.find(old, idx + 1)
        assert idx >= 0, f"mutation anchor not found: {old!r}"
    return text[:idx] + new + text[idx + len(old):]


def _build(text, tmp_path, tag):
    c = tmp_path / f"m_{tag}.c"
    so = tmp_path / f"m_{tag}.so"
    c.write_text(text)
    subprocess.check_call(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                           "-o", str(so), str(c), "-lm"])
    return oracle.load_variant(str(so))


def _pins(lib):
    """Fast pins; returns the names of those that fail."""
    checks = {
        "gamma_algebra": lambda: pins.gamma_algebra(lib=lib),
        "plane_waves": lambda: pins.free_plane_waves((4, 4, 4, 6), 0.1, -1, lib=lib),
        "spectrum_2x4": lambda: pins.free_spectrum_2x4(0.1, lib=lib),
        "gamma5": lambda: pins.gamma5_hermiticity(dims=(4, 4, 4, 4), lib=lib),
        "covariance": lambda: pins.gauge_covariance(dims=(4, 4, 4, 6), lib=lib),
        "dense_solve": lambda: pins.dense_solve(dims=(2, 2, 4, 4), lib=lib, max_iter=1000),
        "pure_gauge": lambda: pins.pure_gauge_solve(dims=(4, 4, 4, 8), lib=lib, max_iter=1000),
        "bicgstab_dense": lambda: pins.bicgstab_dense_solve(dims=(2, 2, 4, 4), lib=lib, max_iter=1000),
    }
    failed = []
    for name, fn in checks.items():
        try:
            ok, _ = fn()
        except Exception:   # a broken build may also crash a pin's linear algebra
            ok = False
        if not bool(ok):
            failed.append(name)
    return failed


def test_unmutated_source_passes_fast_pins(tmp_path):
    lib = _build(open(SRC).read(), tmp_path, "clean")
    assert _pins(lib) == []


@pytest.mark.parametrize("name,old,new,nth", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new, nth):
    text = _replace_nth(open(SRC).read(), old, new, nth)
    lib = _build(text, tmp_path, str(abs(hash(name))))
    failed = _pins(lib)
    assert failed, f"mutation '{name}' passed every pin"


# Mistakes planted in the even-odd Schur complement (NumPy side of the oracle);
# the dense block-elimination pin must reject each one.
SCHUR_MUTANTS = [
    ("Schur sign", "return np.where(even, a * ve - z, 0)", "return np.where(even, a * ve + z, 0)"),
    ("A^-1 dropped", "dirac(U, ve, dims, m0, t_sign, dagger, lib=lib)) / a", "dirac(U, ve, dims, m0, t_sign, dagger, lib=lib))"),
    ("diagonal dropped", "return np.where(even, a * ve - z, 0)", "return np.where(even, -z, 0)"),
    ("parity of the intermediate", "w = np.where(even, 0, dirac(", "w = np.where(even, dirac("),
    ("dagger ignored in the second hop", "z = dirac(U, w, dims, m0, t_sign, dagger, lib=lib)",
     "z = dirac(U, w, dims, m0, t_sign, False, lib=lib)"),
]


@pytest.mark.parametrize("name,old,new", SCHUR_MUTANTS, ids=[m[0] for m in SCHUR_MUTANTS])
def test_schur_mutants_are_caught(name, old, new):
    import inspect

    import numpy as np
    import wdgen
    src = inspect.getsource(oracle.schur)
    assert old in src, name
    if name == "parity of the intermediate":
        new_src = src.replace("w = np.where(even, 0, dirac(U, ve, dims, m0, t_sign, dagger, lib=lib)) / a",
                              "w = np.where(even, dirac(U, ve, dims, m0, t_sign, dagger, lib=lib), 0) / a")
    else:
        new_src = src.replace(old, new)
    assert new_src != src
    ns = dict(vars(oracle))
    exec(new_src, ns)
    mutant = ns["schur"]
    dims, m0 = (2, 2, 4, 4), 0.13
    dagger = name.startswith("dagger")
    U = wdgen.gauge_field(dims, 0.6, 91)
    D = oracle.dense(U, dims, m0, dagger=dagger)
    par = oracle.parity(dims).ravel()
    rows = np.arange(par.size * 12)
    ie, io = rows[par[rows // 12] == 0], rows[par[rows // 12] == 1]
    S = D[np.ix_(ie, ie)] - D[np.ix_(ie, io)] @ np.linalg.solve(D[np.ix_(io, io)], D[np.ix_(io, ie)])
    v = wdgen.gaussian_source(dims, 1, 92)[0]
    got = mutant(U, v, dims, m0, dagger=dagger).ravel()
    want = S @ v.ravel()[ie]
    assert np.linalg.norm(got[ie] - want) > 1e-6 * np.linalg.norm(want), f"mutant {name} survived"
