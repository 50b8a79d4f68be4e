"""FP64 CPU oracle for the Wilson-Dirac operator (TEST INFRASTRUCTURE ONLY).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never imports, links or
calls it, and it shares no code with the GPU library: the arithmetic lives in
``wilson_oracle.c`` (plain C, FP64, dense gamma matrices, full 3x3 links) and
the few steps written here in numpy are the plain definitions.

Paper: Kanamori & Matsufuru, arXiv:1712.01505.
  Sec. II-A   field content (4 spin x 3 colour per site, SU(3) links)
  Sec. II-B   eq. (1), the Wilson fermion matrix
  Sec. II-B   eq. (2), the domain-wall fermion matrix (5-d fields, shape (Ns, Lt, Lz, Ly, Lx, 4, 3))
  Sec. II-C   BiCGStab for the Wilson matrix, CG on the normal equations
  Sec. II-C, Sec. VI-B   CG on D^dag D for the domain-wall matrix

Array conventions (numpy, complex128, canonical):
  spinor  shape (Lt, Lz, Ly, Lx, 4, 3)
  gauge   shape (4, Lt, Lz, Ly, Lx, 3, 3)
  dims    (Lx, Ly, Lz, Lt); bc (bx, by, bz, bt) with +1 periodic, -1 antiperiodic.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

DEFAULT_BC = (1, 1, 1, -1)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b  # noqa: WPS433
        _b.build()
    _lib = _configure(ctypes.CDLL(_LIB_PATH))
    return _lib


def _configure(lib):
    P = ctypes.c_void_p
    ip = ctypes.POINTER(ctypes.c_int)
    lib.oracle_gamma.argtypes = [ctypes.c_int, P]
    lib.oracle_hop.argtypes = [ip, ip, P, P, P, ctypes.c_int]
    lib.oracle_apply.argtypes = [ip, ip, ctypes.c_double, P, P, P, ctypes.c_int]
    lib.oracle_apply_sites.argtypes = [ip, ip, ctypes.c_double, P, P, ctypes.c_int, ctypes.c_long, P, P]
    lib.oracle_cgnr.argtypes = [ip, ip, ctypes.c_double, P, P, P, ctypes.c_double, ctypes.c_int,
                                ip, ctypes.POINTER(ctypes.c_double)]
    lib.oracle_cgnr.restype = ctypes.c_int
    lib.oracle_bicgstab.argtypes = [ip, ip, ctypes.c_double, P, P, P, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_int, ip, ctypes.POINTER(ctypes.c_double)]
    lib.oracle_bicgstab.restype = ctypes.c_int
    lib.oracle_force.argtypes = [ip, ip, ctypes.c_double, P, P, P]
    lib.oracle_dw_apply.argtypes = [ip, ip, ctypes.c_int, ctypes.c_double, ctypes.c_double, P, P, P, ctypes.c_int]
    lib.oracle_dw_cgnr.argtypes = [ip, ip, ctypes.c_int, ctypes.c_double, ctypes.c_double, P, P, P, ctypes.c_double,
                                   ctypes.c_int, ip, ctypes.POINTER(ctypes.c_double)]
    lib.oracle_dw_cgnr.restype = ctypes.c_int
    return lib


def _ivec(v):
    return (ctypes.c_int * 4)(*[int(a) for a in v])


def _c128(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a


def _dims_of_spinor(psi):
    Lt, Lz, Ly, Lx = psi.shape[:4]
    return (Lx, Ly, Lz, Lt)


def gamma(mu: int) -> np.ndarray:
    """The oracle's gamma_mu (mu = 0..3 for x, y, z, t) as a 4x4 complex matrix."""
    out = np.zeros(32, dtype=np.float64)
    _load().oracle_gamma(int(mu), out.ctypes.data)
    return (out[0::2] + 1j * out[1::2]).reshape(4, 4)


def hop(U, psi, bc=DEFAULT_BC, dagger=False):
    """H psi: the hopping term of eq. (1) (times -2 of its 1/2 prefactor),
    H psi(x) = sum_mu [s+ (1-g_mu) U_mu(x) psi(x+mu) + s- (1+g_mu) U_mu(x-mu)^dag psi(x-mu)].
    dagger=True gives the hopping term of D^dag (projector signs swapped)."""
    U = _c128(U)
    psi = _c128(psi)
    out = np.empty_like(psi)
    _load().oracle_hop(_ivec(_dims_of_spinor(psi)), _ivec(bc), U.ctypes.data, psi.ctypes.data,
                       out.ctypes.data, int(bool(dagger)))
    return out


def apply(U, psi, kappa, bc=DEFAULT_BC, dagger=False):
    """D psi = psi - kappa H psi (eq. (1) with D = 2 kappa D_W, kappa = 1/(2 m0 + 8));
    dagger=True gives D^dag psi."""
    U = _c128(U)
    psi = _c128(psi)
    out = np.empty_like(psi)
    _load().oracle_apply(_ivec(_dims_of_spinor(psi)), _ivec(bc), float(kappa), U.ctypes.data,
                         psi.ctypes.data, out.ctypes.data, int(bool(dagger)))
    return out


def apply_sites(U, psi, kappa, sites, bc=DEFAULT_BC, dagger=False):
    """(D psi) at the listed lexicographic site indices; returns shape (n, 4, 3)."""
    U = _c128(U)
    psi = _c128(psi)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    V = int(np.prod(psi.shape[:4]))
    if sites.size and (sites.min() < 0 or sites.max() >= V):
        raise IndexError("site index out of range")
    out = np.empty((len(sites), 4, 3), dtype=np.complex128)
    _load().oracle_apply_sites(_ivec(_dims_of_spinor(psi)), _ivec(bc), float(kappa), U.ctypes.data,
                               psi.ctypes.data, int(bool(dagger)), len(sites), sites.ctypes.data,
                               out.ctypes.data)
    return out


def cgnr(U, b, kappa, bc=DEFAULT_BC, tol=1e-12, maxiter=10000, x0=None):
    """CG on the normal equations (Saad Alg. 8.4); returns (x, status, iters, true_relres)."""
    U = _c128(U)
    b = _c128(b)
    x = np.zeros_like(b) if x0 is None else _c128(x0).copy()
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    st = _load().oracle_cgnr(_ivec(_dims_of_spinor(b)), _ivec(bc), float(kappa), U.ctypes.data,
                             b.ctypes.data, x.ctypes.data, float(tol), int(maxiter), ctypes.byref(it),
                             ctypes.byref(rel))
    return x, st, it.value, rel.value


def bicgstab(U, b, kappa, bc=DEFAULT_BC, tol=1e-12, maxiter=10000, dagger=False, x0=None):
    """BiCGStab (van der Vorst) for D x = b (or D^dag x = b); returns (x, status, iters, true_relres)."""
    U = _c128(U)
    b = _c128(b)
    x = np.zeros_like(b) if x0 is None else _c128(x0).copy()
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    st = _load().oracle_bicgstab(_ivec(_dims_of_spinor(b)), _ivec(bc), float(kappa), U.ctypes.data,
                                 b.ctypes.data, x.ctypes.data, int(bool(dagger)), float(tol), int(maxiter),
                                 ctypes.byref(it), ctypes.byref(rel))
    return x, st, it.value, rel.value


def force(U, x, mu_adj, kappa, bc=DEFAULT_BC):
    """G_mu(x) with dL = Re sum Tr[dU_mu(x) G_mu(x)] for x = D^{-1} b and adjoint
    mu = D^{-dag} dL/dx*; shape (4, Lt, Lz, Ly, Lx, 3, 3)."""
    x = _c128(x)
    mu_adj = _c128(mu_adj)
    dims = _dims_of_spinor(x)
    G = np.empty((4,) + x.shape[:4] + (3, 3), dtype=np.complex128)
    _load().oracle_force(_ivec(dims), _ivec(bc), float(kappa), x.ctypes.data, mu_adj.ctypes.data,
                         G.ctypes.data)
    return G


def su3_project(U, G):
    """P = traceless Hermitian part of A = i U G, per link.  Along U -> exp(i w T) U
    (T Hermitian traceless) the derivative of L is Tr[T P]; the tangent-space
    gradient is i P U."""
    A = 1j * np.matmul(U, G)
    H = 0.5 * (A + np.conj(np.swapaxes(A, -1, -2)))
    tr = np.trace(H, axis1=-2, axis2=-1)[..., None, None]
    return H - tr / 3.0 * np.eye(3)


def gradient(U, b, kappa, bc=DEFAULT_BC, tol=1e-13, maxiter=20000):
    """Gradients of L = ||D^{-1} b||^2.
    Returns dict(x, L, grad_b, G, P, grad_U_tangent):
      grad_b = mu = D^{-dag} (2 x)  (PyTorch convention dL/dRe b + i dL/dIm b),
      G      = link derivative (unconstrained autograd gradient is G^dag),
      P      = su(3) projection, grad_U_tangent = i P U."""
    x, st, _, rel = bicgstab(U, b, kappa, bc=bc, tol=tol, maxiter=maxiter)
    if st != 0:
        raise RuntimeError(f"oracle forward solve failed: status {st}, relres {rel}")
    g = 2.0 * x
    mu, st, _, rel = bicgstab(U, g, kappa, bc=bc, tol=tol, maxiter=maxiter, dagger=True)
    if st != 0:
        raise RuntimeError(f"oracle adjoint solve failed: status {st}, relres {rel}")
    G = force(U, x, mu, kappa, bc=bc)
    P = su3_project(U, G)
    return dict(x=x, L=float(np.vdot(x, x).real), grad_b=mu, G=G, P=P, grad_U_tangent=1j * np.matmul(P, U))


def dw_apply(U, psi, m0, m, bc=DEFAULT_BC, dagger=False):
    """D_DW psi (eq. (2)) for a 5-d field psi of shape (Ns, Lt, Lz, Ly, Lx, 4, 3):
    D_W + 1 on the diagonal in s (D_W = (m0 + 4) - H/2), -P_- above, -P_+ below,
    m P_+ / m P_- in the corners; P_pm = (1 pm gamma_5)/2.  dagger: D_DW^dag."""
    U = _c128(U)
    psi = _c128(psi)
    out = np.empty_like(psi)
    _load().oracle_dw_apply(_ivec(_dims_of_spinor(psi[0])), _ivec(bc), int(psi.shape[0]), float(m0), float(m),
                            U.ctypes.data, psi.ctypes.data, out.ctypes.data, int(bool(dagger)))
    return out


def dw_cgnr(U, b, m0, m, bc=DEFAULT_BC, tol=1e-12, maxiter=20000, x0=None):
    """CG on D_DW^dag D_DW x = D_DW^dag b; returns (x, status, iters, true_relres)."""
    U = _c128(U)
    b = _c128(b)
    x = np.zeros_like(b) if x0 is None else _c128(x0).copy()
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    st = _load().oracle_dw_cgnr(_ivec(_dims_of_spinor(b[0])), _ivec(bc), int(b.shape[0]), float(m0), float(m),
                                U.ctypes.data, b.ctypes.data, x.ctypes.data, float(tol), int(maxiter),
                                ctypes.byref(it), ctypes.byref(rel))
    return x, st, it.value, rel.value
