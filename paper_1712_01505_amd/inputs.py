"""Seeded synthetic lattice fields (inputs only; no operator arithmetic).

This module is shared by the tests, the benchmark and the CPU oracle checks as
the single source of *inputs*.  It contains no part of the Wilson operator, the
solvers or the force: only random gauge links, random spinors and point
sources, all numpy, all seeded.

Layouts (canonical, complex128):
  spinor  (Lt, Lz, Ly, Lx, 4, 3)          -- with nrhs: (nrhs, Lt, Lz, Ly, Lx, 4, 3)
  gauge   (4, Lt, Lz, Ly, Lx, 3, 3)
  dims    (Lx, Ly, Lz, Lt)

Generators:
  * ``haar_gauge``: Haar-random SU(3) links -- QR of a complex Gaussian 3x3
    matrix, phases of R's diagonal moved into Q, then det fixed to 1 by the
    principal cube root.
  * ``near_unity_gauge``: U = exp(i eps H), H = sum_a h_a lambda_a / 2 with
    h_a ~ N(0,1) i.i.d. over the 8 Gell-Mann matrices; built by eigen-
    decomposition so det U = 1 to rounding.
  * ``gaussian_spinor``: re and im each N(0,1).
  * ``point_source``: delta at one site, one spin, one colour.
Draw order for complex Gaussians: the real block, then the imaginary block,
each in canonical array order, from numpy's PCG64 ``default_rng(seed)``.
"""
from __future__ import annotations

import numpy as np

GAUGE_SEED = 1
SOURCE_SEED = 0


def volume(dims) -> int:
    Lx, Ly, Lz, Lt = dims
    return int(Lx) * int(Ly) * int(Lz) * int(Lt)


def spinor_shape(dims, nrhs: int | None = None):
    Lx, Ly, Lz, Lt = dims
    s = (Lt, Lz, Ly, Lx, 4, 3)
    return s if nrhs is None else (nrhs,) + s


def gauge_shape(dims):
    Lx, Ly, Lz, Lt = dims
    return (4, Lt, Lz, Ly, Lx, 3, 3)


def _complex_gaussian(rng, shape, scale=1.0):
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return scale * (re + 1j * im)


def gaussian_spinor(dims, seed: int = SOURCE_SEED, nrhs: int | None = None) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return _complex_gaussian(rng, spinor_shape(dims, nrhs))


def point_source(dims, site=(0, 0, 0, 0), spin: int = 0, colour: int = 0) -> np.ndarray:
    x, y, z, t = site
    out = np.zeros(spinor_shape(dims), dtype=np.complex128)
    out[t, z, y, x, spin, colour] = 1.0
    return out


def point_sources_all_spin_colour(dims, site=(0, 0, 0, 0)) -> np.ndarray:
    """The 12 point sources delta_{x,site} delta_{s,s0} delta_{c,c0}, k = 3 s0 + c0."""
    x, y, z, t = site
    out = np.zeros(spinor_shape(dims, 12), dtype=np.complex128)
    for k in range(12):
        out[k, t, z, y, x, k // 3, k % 3] = 1.0
    return out


def _fix_det(Q):
    det = np.linalg.det(Q)
    # principal cube root of det (det has modulus 1 for unitary Q)
    root = np.exp(1j * np.angle(det) / 3.0)
    return Q / root[..., None, None]


def haar_su3(n: int, rng) -> np.ndarray:
    Z = _complex_gaussian(rng, (n, 3, 3), scale=1.0 / np.sqrt(2.0))
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    ph = d / np.abs(d)
    Q = Q * ph[:, None, :]
    return _fix_det(Q)


def gell_mann() -> np.ndarray:
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


def exp_i_hermitian(H: np.ndarray, eps: float = 1.0) -> np.ndarray:
    """exp(i eps H) for a stack of Hermitian 3x3 matrices, by eigendecomposition."""
    w, V = np.linalg.eigh(H)
    return np.matmul(V * np.exp(1j * eps * w)[..., None, :], np.conj(np.swapaxes(V, -1, -2)))


def near_unity_su3(n: int, eps: float, rng, chunk: int = 1 << 20) -> np.ndarray:
    lam = gell_mann() / 2.0
    out = np.empty((n, 3, 3), dtype=np.complex128)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        h = rng.standard_normal((hi - lo, 8))
        H = np.einsum("na,aij->nij", h, lam)
        out[lo:hi] = exp_i_hermitian(H, eps)
    return out


def haar_gauge(dims, seed: int = GAUGE_SEED) -> np.ndarray:
    rng = np.random.default_rng(seed)
    n = 4 * volume(dims)
    return haar_su3(n, rng).reshape(gauge_shape(dims))


def near_unity_gauge(dims, eps: float = 0.3, seed: int = GAUGE_SEED) -> np.ndarray:
    rng = np.random.default_rng(seed)
    n = 4 * volume(dims)
    return near_unity_su3(n, eps, rng).reshape(gauge_shape(dims))


def unit_gauge(dims) -> np.ndarray:
    U = np.zeros(gauge_shape(dims), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def random_gauge_transform(dims, seed: int = 7) -> np.ndarray:
    """Omega(x) in SU(3) per site, shape (Lt, Lz, Ly, Lx, 3, 3)."""
    rng = np.random.default_rng(seed)
    Lx, Ly, Lz, Lt = dims
    return haar_su3(volume(dims), rng).reshape(Lt, Lz, Ly, Lx, 3, 3)
