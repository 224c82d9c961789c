"""TEST INFRASTRUCTURE ONLY -- the CPU oracle for the Wilson-Dirac solver.

Plain FP64 reference implementations (C for the operator and the Krylov
iteration, NumPy for the storage encodings and the coordinate-format matrix)
against which the GPU library is checked.  Only the tests, the smoke check and
the CPU-baseline leg of the benchmark may import this package; the GPU library
never does, and this package never imports the GPU library.

Functions and the passages they follow (arXiv 2111.14958):
  dirac, dirac_dag      -- Eq. (1) with the Wilson-Dirac operator; D^dagger from
                           gamma5-hermiticity (Sec. 2)
  cg                    -- CG on the normal equations (Sec. 2, CG algorithm)
  bicgstab              -- BiCGSTAB on D (one of the other Krylov methods, Sec. 1)
  coo                   -- the coordinate (Val, Row, Col) storage of D (Sec. 2)
  coo_matvec            -- the coordinate-format product out[Row] += Val*in[Col]
  dense                 -- D as a dense matrix, column by column from `dirac`
  fp16n_encode/decode   -- half-precision spinor storage with a per-site FP32
                           norm (storage format of the benchmark configurations;
                           the paper does not discuss precision)
  round_f32             -- FP32 rounding of inputs (RNE)
  parity, schur, cg_eo  -- even-odd preconditioning: the Schur complement of D
                           on the even sites and CG on its normal equations.
                           The paper asks for operator forms better suited to
                           the Dirac operator (Conclusions) but describes none;
                           this is the textbook block elimination of Eq. (1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wilson_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, no fast-math, no FMA contraction;
    OpenMP for the operator's independent site loop only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
            "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _bind(lib):
    P = ctypes.c_void_p
    lib.oracle_dirac.argtypes = [P, P, ctypes.c_int, ctypes.c_double, P, P, ctypes.c_int]
    lib.oracle_dirac.restype = None
    lib.oracle_cg.argtypes = [P, P, ctypes.c_int, ctypes.c_double, P, P, ctypes.c_int,
                              ctypes.c_double, ctypes.c_int, ctypes.c_int, P, P, P]
    lib.oracle_cg.restype = ctypes.c_int
    lib.oracle_gamma.argtypes = [ctypes.c_int, P]
    lib.oracle_gamma.restype = None
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = ctypes.c_int
    lib.oracle_bicgstab.argtypes = [P, P, ctypes.c_int, ctypes.c_double, P, P, ctypes.c_int,
                                    ctypes.c_double, ctypes.c_int, P, P]
    lib.oracle_bicgstab.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def load_variant(path: str):
    """Bind another build of the oracle source (used by the mutation tests, which
    compile deliberately broken copies and check that the pins reject them)."""
    return _bind(ctypes.CDLL(os.path.abspath(path)))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dims_arr(dims):
    return np.ascontiguousarray(np.array([int(d) for d in dims], dtype=np.int32))


def _check(U, psi, dims):
    lx, ly, lz, lt = (int(d) for d in dims)
    V = lx * ly * lz * lt
    U = np.ascontiguousarray(U, dtype=np.complex128)
    if U.size != V * 36:
        raise ValueError("gauge field does not match dims")
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    if psi.size % (V * 12):
        raise ValueError("spinor field does not match dims")
    return U, psi, V


def set_threads(n: int = 0) -> int:
    """Host threads for the operator's site loop (OpenMP); n <= 0 only reports
    the count in force.  Results do not depend on it: each site is computed by
    the same statements on whichever thread, and every sum stays sequential."""
    return int(_load().oracle_set_threads(int(n)))


def gamma(mu: int, lib=None) -> np.ndarray:
    """gamma_mu (DeGrand-Rossi basis) as used by the oracle's operator."""
    out = np.zeros(16, dtype=np.complex128)
    (lib or _load()).oracle_gamma(int(mu), _ptr(out))
    return out.reshape(4, 4)


def dirac(U, psi, dims, m0: float, t_sign: int = -1, dagger: bool = False,
          lib=None) -> np.ndarray:
    """D psi (or D^dagger psi) for one or more spinors in canonical layout."""
    U, psi, V = _check(U, psi, dims)
    shape = psi.shape
    flat = psi.reshape(-1, V * 12)
    out = np.empty_like(flat)
    d = _dims_arr(dims)
    lib = lib or _load()
    for i in range(flat.shape[0]):
        src = np.ascontiguousarray(flat[i])
        dst = np.empty_like(src)
        lib.oracle_dirac(_ptr(U), _ptr(d), int(t_sign), float(m0), _ptr(src), _ptr(dst),
                         1 if dagger else 0)
        out[i] = dst
    return out.reshape(shape)


def dirac_dag(U, psi, dims, m0: float, t_sign: int = -1, lib=None) -> np.ndarray:
    return dirac(U, psi, dims, m0, t_sign, dagger=True, lib=lib)


def true_residual(U, eta, x, dims, m0: float, t_sign: int = -1, lib=None) -> np.ndarray:
    """|eta - D x| / |eta| per right-hand side (FP64)."""
    U, eta, V = _check(U, eta, dims)
    x = np.ascontiguousarray(x, dtype=np.complex128).reshape(eta.shape)
    r = eta - dirac(U, x, dims, m0, t_sign, lib=lib)
    e = eta.reshape(-1, V * 12)
    r = r.reshape(-1, V * 12)
    en = np.linalg.norm(e, axis=1)
    rn = np.linalg.norm(r, axis=1)
    return np.where(en > 0, rn / np.where(en > 0, en, 1), rn)


def cg(U, eta, dims, m0: float, tol: float = 1e-10, max_iter: int = 20000,
       t_sign: int = -1, form: int = 0, x0=None, trace: bool = False, lib=None):
    """Solve D x = eta by CG on the normal equations, one spinor at a time.

    form 0: CG on D D^dagger (the paper's choice), form 1: CG on D^dagger D.
    Returns (x, iters[list], true_rel_res[list], status[list]) and, with
    trace=True, a list of per-iteration relative residual histories.
    """
    U, eta, V = _check(U, eta, dims)
    shape = eta.shape
    flat = eta.reshape(-1, V * 12)
    xs = np.zeros_like(flat)
    if x0 is not None:
        xs[:] = np.asarray(x0, dtype=np.complex128).reshape(flat.shape)
    d = _dims_arr(dims)
    lib = lib or _load()
    iters, res, st, traces = [], [], [], []
    for i in range(flat.shape[0]):
        e = np.ascontiguousarray(flat[i])
        x = np.ascontiguousarray(xs[i])
        it = ctypes.c_int(0)
        rr = ctypes.c_double(0.0)
        tr = np.zeros(max_iter, dtype=np.float64) if trace else None
        s = lib.oracle_cg(_ptr(U), _ptr(d), int(t_sign), float(m0), _ptr(e), _ptr(x),
                          1 if x0 is not None else 0, float(tol), int(max_iter), int(form),
                          ctypes.byref(it), ctypes.byref(rr),
                          _ptr(tr) if trace else None)
        xs[i] = x
        iters.append(it.value)
        res.append(rr.value)
        st.append(s)
        if trace:
            traces.append(tr[: it.value].copy())
    out = (xs.reshape(shape), iters, res, st)
    return out + (traces,) if trace else out


def bicgstab(U, eta, dims, m0: float, tol: float = 1e-10, max_iter: int = 20000,
             t_sign: int = -1, x0=None, lib=None):
    """Solve D x = eta by BiCGSTAB on D itself (Sec. 1 lists it), one field at a time.
    Returns (x, iters[list], true_rel_res[list], status[list])."""
    U, eta, V = _check(U, eta, dims)
    shape = eta.shape
    flat = eta.reshape(-1, V * 12)
    xs = np.zeros_like(flat)
    if x0 is not None:
        xs[:] = np.asarray(x0, dtype=np.complex128).reshape(flat.shape)
    d = _dims_arr(dims)
    lib = lib or _load()
    iters, res, st = [], [], []
    for i in range(flat.shape[0]):
        e = np.ascontiguousarray(flat[i])
        x = np.ascontiguousarray(xs[i])
        it = ctypes.c_int(0)
        rr = ctypes.c_double(0.0)
        s = lib.oracle_bicgstab(_ptr(U), _ptr(d), int(t_sign), float(m0), _ptr(e), _ptr(x),
                                1 if x0 is not None else 0, float(tol), int(max_iter),
                                ctypes.byref(it), ctypes.byref(rr))
        xs[i] = x
        iters.append(it.value)
        res.append(rr.value)
        st.append(s)
    return xs.reshape(shape), iters, res, st


def dense(U, dims, m0: float, t_sign: int = -1, dagger: bool = False, lib=None) -> np.ndarray:
    """D as a dense (12V x 12V) matrix, built column by column (small lattices only)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    V = lx * ly * lz * lt
    n = 12 * V
    if n > 12 * 4 ** 4:
        raise ValueError("dense matrix requested for a lattice larger than 4^4")
    eye = np.eye(n, dtype=np.complex128).reshape(n, V * 12)
    cols = dirac(U, eye, dims, m0, t_sign, dagger, lib=lib)
    return np.ascontiguousarray(cols.reshape(n, n).T)


# ---------------------------------------------------------------------------
# Coordinate (COO) storage of D, Sec. 2: three arrays Val, Row, Col holding each
# non-zero entry with its row and column index.  Row/column index of component
# (site n, spin alpha, colour A) is 12 n + 3 alpha + A.  Entries are generated
# term by term from the operator's definition (diagonal, then for each site and
# direction the forward and backward hops); duplicates are kept, and the product
# sums them exactly like the paper's loop out[Row[k]] += Val[k] * in[Col[k]].
# ---------------------------------------------------------------------------
def _gammas():
    return [gamma(mu) for mu in range(4)]


def coo(U, dims, m0: float, t_sign: int = -1, dagger: bool = False):
    """(Val, Row, Col) of D (or D^dagger) in the coordinate format of Sec. 2."""
    lx, ly, lz, lt = (int(d) for d in dims)
    L = (lx, ly, lz, lt)
    V = lx * ly * lz * lt
    U = np.ascontiguousarray(U, dtype=np.complex128).reshape(V, 4, 3, 3)
    G = _gammas()
    sgn = -1.0 if dagger else 1.0
    site = np.arange(V)
    coords = [site % lx, (site // lx) % ly, (site // (lx * ly)) % lz, site // (lx * ly * lz)]
    vals, rows, cols = [], [], []
    # diagonal (4 + m0)
    comp = np.arange(12)
    rows.append((12 * site[:, None] + comp[None, :]).ravel())
    cols.append((12 * site[:, None] + comp[None, :]).ravel())
    vals.append(np.full(12 * V, 4.0 + m0, dtype=np.complex128))
    for mu in range(4):
        Pf = np.eye(4) - sgn * G[mu]
        Pb = np.eye(4) + sgn * G[mu]
        strides = (1, lx, lx * ly, lx * ly * lz)
        c = coords[mu]
        fwd = site + np.where(c == L[mu] - 1, -(L[mu] - 1) * strides[mu], strides[mu])
        bwd = site + np.where(c == 0, (L[mu] - 1) * strides[mu], -strides[mu])
        sf = np.where((mu == 3) & (c == L[mu] - 1), float(t_sign), 1.0)
        sb = np.where((mu == 3) & (c == 0), float(t_sign), 1.0)
        Uf = U[:, mu]                       # U_mu(n)
        Ub = np.conj(np.swapaxes(U[bwd, mu], -1, -2))  # U_mu(n - mu)^dagger
        for al in range(4):
            for be in range(4):
                for A in range(3):
                    for B in range(3):
                        if Pf[al, be] != 0:
                            vals.append(-0.5 * Pf[al, be] * sf * Uf[:, A, B])
                            rows.append(12 * site + 3 * al + A)
                            cols.append(12 * fwd + 3 * be + B)
                        if Pb[al, be] != 0:
                            vals.append(-0.5 * Pb[al, be] * sb * Ub[:, A, B])
                            rows.append(12 * site + 3 * al + A)
                            cols.append(12 * bwd + 3 * be + B)
    return (np.concatenate(vals), np.concatenate(rows).astype(np.int64),
            np.concatenate(cols).astype(np.int64))


def coo_matvec(val, row, col, vec, n: int) -> np.ndarray:
    """out[Row[k]] += Val[k] * in[Col[k]] over all k (Sec. 2), duplicates summed."""
    out = np.zeros(n, dtype=np.complex128)
    np.add.at(out, row, val * vec[col])
    return out


# ---------------------------------------------------------------------------
# Storage encodings of the reduced-precision solver modes.
# ---------------------------------------------------------------------------
def round_f32(a: np.ndarray) -> np.ndarray:
    """Round complex128 data to complex64 (round to nearest even) and back."""
    return np.asarray(a, dtype=np.complex128).astype(np.complex64).astype(np.complex128)


def fp16n_encode(psi_f32: np.ndarray):
    """Half storage with a per-site FP32 norm for spinors [..., V, 4, 3].

    norm = max |component| over the 24 real numbers of the site (FP32);
    inv = 1 / norm rounded to FP32; code = half(v * inv) with the product
    rounded to FP32 first, then to half, all round-to-nearest-even (one
    division per site instead of one per component).  Where 1 / norm
    overflows FP32 (norm < 2^-128, a subnormal) the FP32 quotient v / norm
    takes the product's place.  A site that is all zero gets norm 0, codes 0.
    Input is complex64 (already rounded to FP32).
    Returns (codes float16 [..., V, 24] as (re, im) pairs, norms float32 [..., V]).
    """
    v = np.asarray(psi_f32, dtype=np.complex64)
    lead = v.shape[:-2]
    re = np.stack([v.real, v.imag], axis=-1).reshape(lead + (24,)).astype(np.float32)
    norm = np.max(np.abs(re), axis=-1).astype(np.float32)
    safe = np.where(norm > 0, norm, np.float32(1)).astype(np.float32)
    with np.errstate(over="ignore", invalid="ignore"):
        inv = (np.float32(1) / safe).astype(np.float32)
        q = np.where(np.isinf(inv)[..., None], re / safe[..., None], re * inv[..., None]).astype(np.float32)
    q = np.where(norm[..., None] > 0, q, np.float32(0))
    return q.astype(np.float16), norm


def fp16n_decode(codes: np.ndarray, norms: np.ndarray) -> np.ndarray:
    """Inverse of fp16n_encode: norm * float(code), returned as complex64 [..., V, 4, 3]."""
    f = codes.astype(np.float32) * norms.astype(np.float32)[..., None]
    f = f.reshape(f.shape[:-1] + (12, 2))
    c = (f[..., 0] + 1j * f[..., 1]).astype(np.complex64)
    return c.reshape(c.shape[:-1] + (4, 3))


# ------------------------------------------------------------ even-odd
def parity(dims) -> np.ndarray:
    """(x + y + z + t) mod 2 of every site, shape (Lt, Lz, Ly, Lx)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    return (x + y + z + t) % 2


def schur(U, v, dims, m0: float, t_sign: int = -1, dagger: bool = False, lib=None) -> np.ndarray:
    """Schur complement of D on the even sites, applied to v (canonical layout;
    only its even sites are read, the result is zero on odd sites):
        Dhat v = A v_e - D_eo A^-1 D_oe v_e,   A = 4 + m0 (the diagonal of Eq. (1)).
    D_oe v_e is the odd part of D applied to the even-supported v (D's diagonal
    keeps parity, its hopping flips it); likewise D_eo w for odd-supported w.
    dagger: the Schur complement of D^dagger, which is Dhat^dagger."""
    even = (parity(dims) == 0)[..., None, None]
    a = 4.0 + m0
    ve = np.where(even, v, 0)
    w = np.where(even, 0, dirac(U, ve, dims, m0, t_sign, dagger, lib=lib)) / a   # A^-1 D_oe v_e
    z = dirac(U, w, dims, m0, t_sign, dagger, lib=lib)                          # even part: D_eo w
    return np.where(even, a * ve - z, 0)


def cg_eo(U, eta, dims, m0: float, tol: float = 1e-10, max_iter: int = 20000, t_sign: int = -1,
          lib=None):
    """Solve D x = eta with even-odd preconditioning, one field at a time:
        b_e = eta_e - D_eo A^-1 eta_o
        CG on Dhat Dhat^dagger chi = b_e carried in x_e = Dhat^dagger chi (the
        CG algorithm of Sec. 2 on Dhat), until |b_e - Dhat x_e| <= tol |eta|
        x_o = A^-1 (eta_o - D_oe x_e)
    Then eta - D x vanishes on the odd sites and equals b_e - Dhat x_e on the even
    ones.  Returns (x, iters[list], true_rel_res[list] of the full system,
    status[list]: 0 converged, 1 not converged, 2 breakdown)."""
    U, eta, V = _check(U, eta, dims)
    lib = lib or _load()
    shape = eta.shape
    flat = eta.reshape((-1,) + shape[-6:]) if eta.ndim == 7 else eta.reshape((1,) + shape)
    even = (parity(dims) == 0)[..., None, None]
    a = 4.0 + m0
    xs, iters, res, st = [], [], [], []
    dot = lambda u, v: float(np.vdot(u, v).real)
    for e in flat:
        eta_norm = np.sqrt(dot(e, e))
        x = np.zeros_like(e)
        if eta_norm == 0.0:
            xs.append(x); iters.append(0); res.append(0.0); st.append(0)
            continue
        wo = np.where(even, 0, e) / a
        b = np.where(even, e - dirac(U, wo, dims, m0, t_sign, lib=lib), 0)
        stop = tol * eta_norm
        r = b.copy()
        p = r.copy()
        rho = dot(r, r)
        status, it = 1, 0
        while it < max_iter:
            q = schur(U, p, dims, m0, t_sign, dagger=True, lib=lib)
            sigma = dot(q, q)
            if not (sigma > 0.0 and np.isfinite(sigma)):
                status = 2
                break
            alpha = rho / sigma
            x = x + alpha * q
            r = r - alpha * schur(U, q, dims, m0, t_sign, lib=lib)
            rho_new = dot(r, r)
            it += 1
            if np.sqrt(rho_new) <= stop:
                rt = b - schur(U, x, dims, m0, t_sign, lib=lib)
                if np.sqrt(dot(rt, rt)) <= stop:
                    status = 0
                    break
                r = rt
                rho_new = dot(r, r)
            p = r + (rho_new / rho) * p
            rho = rho_new
        xo = np.where(even, 0, e - dirac(U, x, dims, m0, t_sign, lib=lib)) / a
        xf = np.where(even, x, xo)
        rf = e - dirac(U, xf, dims, m0, t_sign, lib=lib)
        xs.append(xf); iters.append(it); res.append(np.sqrt(dot(rf, rf)) / eta_norm); st.append(status)
    return np.stack(xs).reshape(shape), iters, res, st
