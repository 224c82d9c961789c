"""Seeded synthetic inputs for the Wilson-Dirac solver: gauge links, sources,
gauge transformations and request streams.

This module is shared by the CPU oracle, the tests, the smoke check and the
benchmark.  It holds none of the solver's arithmetic (no Dirac operator, no
Krylov iteration): only random fields and the canonical array layouts.

Canonical layouts (C order, complex128):
  gauge   U[t][z][y][x][mu][a][b]   -- link x -> x+mu, acting as (U psi)_a = sum_b U_ab psi_b
  spinor  psi[rhs][t][z][y][x][spin][colour]
Directions mu = 0,1,2,3 are x,y,z,t; dims are given as (Lx, Ly, Lz, Lt) and the
site index is x + Lx*(y + Ly*(z + Lz*t)).

The paper (Sec. 2) never says how its links are produced; the inputs follow the
generator of the benchmark configurations: U = exp(i eps H) with H a random
traceless Hermitian 3x3 matrix, H = sum_a h_a lambda_a / 2, h_a ~ N(0,1).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "lattice_shape", "volume", "gell_mann", "su3_from_generator", "gauge_field",
    "unit_gauge", "gaussian_source", "point_sources", "mixed_sources",
    "site_matrices", "transform_gauge", "pure_gauge", "apply_site_matrix",
    "shift_forward", "CONFIGS", "serving_requests",
]

# numpy axis of the (t, z, y, x) site block that direction mu runs along
_AXIS = {0: 3, 1: 2, 2: 1, 3: 0}


def lattice_shape(dims):
    """(Lx, Ly, Lz, Lt) -> numpy block shape (Lt, Lz, Ly, Lx)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    if min(lx, ly, lz, lt) < 1:
        raise ValueError(f"bad lattice dims {dims}")
    return (lt, lz, ly, lx)


def volume(dims) -> int:
    lx, ly, lz, lt = (int(d) for d in dims)
    return lx * ly * lz * lt


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3)."""
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1] = -1j
    l[1][1, 0] = 1j
    l[2][0, 0], l[2][1, 1] = 1, -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2] = -1j
    l[4][2, 0] = 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2] = -1j
    l[6][2, 1] = 1j
    l[7][0, 0] = l[7][1, 1] = 1 / np.sqrt(3)
    l[7][2, 2] = -2 / np.sqrt(3)
    return l


def su3_from_generator(h: np.ndarray, eps: float) -> np.ndarray:
    """exp(i eps H) for H = sum_a h[..., a] lambda_a / 2 (traceless Hermitian).

    Uses the spectral decomposition H = V diag(w) V^dagger, so the result is
    unitary to rounding and has det = exp(i eps tr H) = 1.
    """
    H = np.einsum("...a,aij->...ij", h, gell_mann()) / 2.0
    w, V = np.linalg.eigh(H)
    ph = np.exp(1j * eps * w)
    return np.einsum("...ik,...k,...jk->...ij", V, ph, V.conj())


def gauge_field(dims, eps: float, seed: int) -> np.ndarray:
    """Random SU(3) links U_mu(x) = exp(i eps H), draw order [t][z][y][x][mu][a]."""
    shp = lattice_shape(dims)
    rng = np.random.default_rng(seed)
    h = rng.standard_normal(shp + (4, 8))
    return np.ascontiguousarray(su3_from_generator(h, eps))


def unit_gauge(dims) -> np.ndarray:
    """Free field U = 1."""
    shp = lattice_shape(dims)
    U = np.zeros(shp + (4, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def gaussian_source(dims, nrhs: int, seed: int) -> np.ndarray:
    """Complex Gaussian spinors, Re and Im ~ N(0,1) i.i.d."""
    shp = lattice_shape(dims)
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((nrhs,) + shp + (4, 3, 2))
    return np.ascontiguousarray(a[..., 0] + 1j * a[..., 1])


def point_sources(dims, ks=range(12)) -> np.ndarray:
    """Unit point sources at the origin; source k has spin k // 3, colour k % 3."""
    ks = list(ks)
    shp = lattice_shape(dims)
    s = np.zeros((len(ks),) + shp + (4, 3), dtype=np.complex128)
    for i, k in enumerate(ks):
        s[(i, 0, 0, 0, 0, k // 3, k % 3)] = 1.0
    return s


def mixed_sources(dims, n_point: int, n_gauss: int, seed: int) -> np.ndarray:
    """n_point spin-colour point sources followed by n_gauss Gaussian sources."""
    parts = []
    if n_point:
        parts.append(point_sources(dims, range(n_point)))
    if n_gauss:
        parts.append(gaussian_source(dims, n_gauss, seed))
    return np.ascontiguousarray(np.concatenate(parts, axis=0))


def site_matrices(dims, eps: float, seed: int) -> np.ndarray:
    """One random SU(3) matrix per site (a gauge transformation Omega(x))."""
    shp = lattice_shape(dims)
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(su3_from_generator(rng.standard_normal(shp + (8,)), eps))


def shift_forward(field: np.ndarray, mu: int) -> np.ndarray:
    """f(x + mu_hat) for a field whose leading four axes are (t, z, y, x).

    A plain periodic relabelling; boundary phases are not part of the fields.
    """
    return np.roll(field, -1, axis=_AXIS[mu])


def transform_gauge(U: np.ndarray, Om: np.ndarray) -> np.ndarray:
    """U^Omega_mu(x) = Omega(x) U_mu(x) Omega(x + mu_hat)^dagger."""
    out = np.empty_like(U)
    for mu in range(4):
        Om_f = shift_forward(Om, mu)
        out[..., mu, :, :] = Om @ U[..., mu, :, :] @ np.conj(np.swapaxes(Om_f, -1, -2))
    return out


def pure_gauge(Om: np.ndarray) -> np.ndarray:
    """Links gauge-equivalent to U = 1: U_mu(x) = Omega(x) Omega(x + mu_hat)^dagger."""
    shp = Om.shape[:4]
    U = np.empty(shp + (4, 3, 3), dtype=np.complex128)
    for mu in range(4):
        U[..., mu, :, :] = Om @ np.conj(np.swapaxes(shift_forward(Om, mu), -1, -2))
    return U


def apply_site_matrix(Om: np.ndarray, psi: np.ndarray, dagger: bool = False) -> np.ndarray:
    """(Omega psi)(x) on the colour index of spinors psi[..., t, z, y, x, spin, colour]."""
    M = np.conj(np.swapaxes(Om, -1, -2)) if dagger else Om
    return np.einsum("tzyxab,...tzyxsb->...tzyxsa", M, psi)


# Benchmark / test workloads (lattice dims (Lx, Ly, Lz, Lt), bare mass m0, link
# disorder eps, seeds): gauge seeds 1001..1004 and source seeds 2001..2004 in the
# order of the workloads (the single-field lattices 8^4..14^4 share one pair).
CONFIGS = {
    "lat4x4_1rhs": dict(dims=(4, 4, 4, 4), m0=0.1, eps=0.3, gauge_seed=1001, src_seed=2001,
                   nrhs=1, tol=1e-10),
    "lat8x4_1rhs": dict(dims=(8, 8, 8, 8), m0=0.05, eps=0.5, gauge_seed=1002, src_seed=2002,
                   nrhs=1, tol=1e-10),
    "lat12x4_1rhs": dict(dims=(12, 12, 12, 12), m0=0.05, eps=0.5, gauge_seed=1002, src_seed=2002,
                    nrhs=1, tol=1e-10),
    "lat14x4_1rhs": dict(dims=(14, 14, 14, 14), m0=0.05, eps=0.5, gauge_seed=1002, src_seed=2002,
                    nrhs=1, tol=1e-10),
    # 12 spin-colour point sources at the origin, then 4 Gaussian sources
    "lat14x4_16rhs": dict(dims=(14, 14, 14, 14), m0=0.05, eps=0.5, gauge_seed=1003,
                          src_seed=2003, n_point=12, n_gauss=4, tol=1e-10),
    "lat16x3x32_12rhs": dict(dims=(16, 16, 16, 32), m0=0.02, eps=0.5, gauge_seed=1004,
                             src_seed=2004, n_point=12, n_gauss=0, tol=1e-10),
}

SERVING_VOLUMES = [(4, 4, 4, 4), (8, 8, 8, 8), (12, 12, 12, 12), (14, 14, 14, 14),
                   (16, 16, 16, 32)]


def serving_requests(n: int, rate: float, seed: int = 10_000, volumes=None,
                     max_rhs: int = 12, m0_range=(0.02, 0.2)):
    """Poisson arrival stream of solve requests.

    Each request draws a volume uniformly from `volumes`, 1..max_rhs right-hand
    sides and m0 uniform in m0_range; request i uses gauge seed seed + i.
    Returns a list of dicts with arrival time (s), dims, nrhs, m0, seeds.
    """
    vols = volumes or SERVING_VOLUMES
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n) if rate > 0 else np.zeros(n)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n):
        out.append(dict(
            arrival=float(t[i]),
            dims=tuple(vols[int(rng.integers(len(vols)))]),
            nrhs=int(rng.integers(1, max_rhs + 1)),
            m0=float(rng.uniform(*m0_range)),
            gauge_seed=seed + i,
            src_seed=seed + 50_000 + i,
        ))
    return out
