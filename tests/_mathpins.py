"""Independent mathematical pins for the Wilson-Dirac operator (test helpers).

Nothing here calls the oracle or the GPU library.  The constructions are
written from the mathematics, in a different form from the oracle's site loop:

* ``dense_wilson``: the operator as a sparse/dense matrix built from Kronecker
  products, D = 1 - kappa sum_mu [ (1-g_mu) (x) F_mu + (1+g_mu) (x) F_mu^dag ],
  where F_mu = blockdiag_x(U_mu(x)) . (S_mu (x) 1_3) and S_mu is the signed
  shift S_mu[x, x+mu] = boundary sign (paper Sec. II-B, eq. (1), in the
  hopping-parameter normalisation D = 2 kappa D_W).
* ``free_spectrum``: the closed-form eigenvalues of the free-field operator
  (U = 1): on a plane wave e^{ipx} u, D acts as
  D(p) = 1 - 2 kappa sum cos p_mu + 2 i kappa sum gamma_mu sin p_mu, whose
  eigenvalues are A(p) +/- 2 i kappa sqrt(sum sin^2 p_mu), each 6-fold.
* ``free_solve_fft``: x = D^{-1} b at U = 1 by FFT, using the inverse symbol
  D(p)^{-1} = [A(p) - 2 i kappa sum gamma_mu sin p_mu] / [A(p)^2 + 4 kappa^2 sum sin^2 p_mu].

The gamma matrices are the chiral (DeGrand-Rossi) basis, typed here a second
time on purpose (the oracle types its own copy); Clifford relations are
checked in the tests.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

I = 1j
GAMMAS = np.array([
    [[0, 0, 0, I], [0, 0, I, 0], [0, -I, 0, 0], [-I, 0, 0, 0]],
    [[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]],
    [[0, 0, I, 0], [0, 0, 0, -I], [-I, 0, 0, 0], [0, I, 0, 0]],
    [[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]],
], dtype=np.complex128)
GAMMA5 = GAMMAS[0] @ GAMMAS[1] @ GAMMAS[2] @ GAMMAS[3]


def _vol(dims):
    return int(np.prod(dims))


def shift(dims, mu, bc):
    """Signed forward shift S_mu (V x V): S[x, x+mu] = bc[mu] if the step wraps, else 1."""
    Lx, Ly, Lz, Lt = dims
    V = _vol(dims)
    idx = np.arange(V).reshape(Lt, Lz, Ly, Lx)
    axis = 3 - mu
    nb = np.roll(idx, -1, axis=axis)
    sign = np.ones_like(idx, dtype=np.float64)
    sl = [slice(None)] * 4
    sl[axis] = -1
    sign[tuple(sl)] = bc[mu]
    return sp.csr_matrix((sign.ravel(), (idx.ravel(), nb.ravel())), shape=(V, V))


def dense_wilson(U, kappa, dims, bc=(1, 1, 1, -1), dagger=False):
    """Dense D (or D^dag) as a (12V x 12V) matrix in the canonical index order
    site*12 + spin*3 + colour."""
    V = _vol(dims)
    Umu = np.asarray(U).reshape(4, V, 3, 3)
    H = None
    for mu in range(4):
        blk = sp.block_diag([sp.csr_matrix(Umu[mu, x]) for x in range(V)], format="csr")
        F = blk @ sp.kron(shift(dims, mu, bc), sp.identity(3), format="csr")
        one = np.eye(4)
        term = sp.kron(one - GAMMAS[mu], F) + sp.kron(one + GAMMAS[mu], F.conj().T)
        H = term if H is None else H + term
    # H is in (spin, site, colour) order; permute to (site, spin, colour)
    n = 12 * V
    spin = np.repeat(np.arange(4), 3 * V)
    site = np.tile(np.repeat(np.arange(V), 3), 4)
    col = np.tile(np.arange(3), 4 * V)
    canon = site * 12 + spin * 3 + col
    P = sp.csr_matrix((np.ones(n), (canon, np.arange(n))), shape=(n, n))
    Hc = (P @ H @ P.T).toarray()
    D = np.eye(n) - kappa * Hc
    return D.conj().T if dagger else D


def momenta(dims, bc=(1, 1, 1, -1)):
    """Allowed momenta per axis: 2 pi n / L (periodic) or (2 pi n + pi) / L (antiperiodic)."""
    out = []
    for mu, L in enumerate(dims):
        n = np.arange(L)
        out.append((2 * np.pi * n + (np.pi if bc[mu] < 0 else 0.0)) / L)
    return out


def free_spectrum(dims, kappa, bc=(1, 1, 1, -1)):
    """Closed-form eigenvalues of the free-field D, each repeated 6 times."""
    px, py, pz, pt = np.meshgrid(*momenta(dims, bc), indexing="ij")
    A = 1 - 2 * kappa * (np.cos(px) + np.cos(py) + np.cos(pz) + np.cos(pt))
    B = 2 * kappa * np.sqrt(np.sin(px) ** 2 + np.sin(py) ** 2 + np.sin(pz) ** 2 + np.sin(pt) ** 2)
    ev = np.concatenate([(A + 1j * B).ravel(), (A - 1j * B).ravel()])
    return np.repeat(ev, 6)


def free_solve_fft(b, kappa, bc=(1, 1, 1, -1)):
    """Exact x = D^{-1} b at U = 1 (canonical spinor layout, one right-hand side)."""
    Lt, Lz, Ly, Lx = b.shape[:4]
    dims = (Lx, Ly, Lz, Lt)
    # twist out the antiperiodic phases so a plain DFT applies
    coords = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    twist_angle = np.zeros((Lt, Lz, Ly, Lx))
    for mu, c in zip((3, 2, 1, 0), coords):
        if bc[mu] < 0:
            twist_angle = twist_angle + np.pi * c / dims[mu]
    phi = b * np.exp(-1j * twist_angle)[..., None, None]
    phit = np.fft.fftn(phi, axes=(0, 1, 2, 3))
    p = momenta(dims, bc)
    pt, pz, py, px = np.meshgrid(p[3], p[2], p[1], p[0], indexing="ij")
    s = [np.sin(px), np.sin(py), np.sin(pz), np.sin(pt)]
    A = 1 - 2 * kappa * (np.cos(px) + np.cos(py) + np.cos(pz) + np.cos(pt))
    den = A ** 2 + 4 * kappa ** 2 * (s[0] ** 2 + s[1] ** 2 + s[2] ** 2 + s[3] ** 2)
    num = A[..., None, None] * np.eye(4)
    for mu in range(4):
        num = num - 2j * kappa * s[mu][..., None, None] * GAMMAS[mu]
    Dinv = num / den[..., None, None]
    xt = np.einsum("tzyxab,tzyxbc->tzyxac", Dinv, phit)
    x = np.fft.ifftn(xt, axes=(0, 1, 2, 3))
    return x * np.exp(1j * twist_angle)[..., None, None]


def gamma5_spinor(psi):
    """gamma_5 acting on the spin index of a canonical spinor (..., 4, 3)."""
    return np.einsum("ab,...bc->...ac", GAMMA5, psi)


def gauge_transform_links(U, Om, dims):
    """U^Omega_mu(x) = Omega(x) U_mu(x) Omega(x+mu)^dag (gauge field (4,Lt,Lz,Ly,Lx,3,3))."""
    out = np.empty_like(U)
    for mu in range(4):
        axis = 3 - mu
        Om_fwd = np.roll(Om, -1, axis=axis)
        out[mu] = Om @ U[mu] @ np.conj(np.swapaxes(Om_fwd, -1, -2))
    return out


# ---------------------------------------------------------------- domain wall
# D_DW (paper Sec. II-B, eq. (2)) written as Kronecker products over the fifth
# index: I_s (x) (D_W + 1) - U_s (x) P_- - L_s (x) P_+ + m E_{0,Ns-1} (x) P_+
# + m E_{Ns-1,0} (x) P_-, with U_s / L_s the ones just above / below the
# diagonal, D_W = (m0 + 4) - H/2 and P_pm = (1 pm gamma_5)/2 acting on spin.

P_PLUS = 0.5 * (np.eye(4) + GAMMA5)
P_MINUS = 0.5 * (np.eye(4) - GAMMA5)


def dense_dw(U, m0, m, Ns, dims, bc=(1, 1, 1, -1), dagger=False):
    """Dense D_DW (or its conjugate transpose), index order s*12V + site*12 + spin*3 + colour."""
    V = _vol(dims)
    H = np.eye(12 * V) - dense_wilson(U, 1.0, dims, bc)  # D(kappa=1) = 1 - H
    DW = (m0 + 4.0) * np.eye(12 * V) - 0.5 * H
    site_p = lambda P: np.kron(np.eye(V), np.kron(P, np.eye(3)))
    Pp, Pm = site_p(P_PLUS), site_p(P_MINUS)
    up = np.eye(Ns, k=1)
    down = np.eye(Ns, k=-1)
    corner_top = np.zeros((Ns, Ns))
    corner_top[0, Ns - 1] = 1.0
    corner_bot = np.zeros((Ns, Ns))
    corner_bot[Ns - 1, 0] = 1.0
    D = (np.kron(np.eye(Ns), DW + np.eye(12 * V)) - np.kron(up, Pm) - np.kron(down, Pp)
         + m * np.kron(corner_top, Pp) + m * np.kron(corner_bot, Pm))
    return D.conj().T if dagger else D


def dw_symbol(p, m0, m, Ns):
    """Free-field D_DW on e^{ipx} v (v: Ns x 4 spin vectors), a (4 Ns x 4 Ns) matrix:
    D_W(p) = (m0 + 4) - sum cos p_mu + i sum gamma_mu sin p_mu in the diagonal blocks."""
    DWp = (m0 + 4.0 - np.sum(np.cos(p))) * np.eye(4, dtype=np.complex128)
    for mu in range(4):
        DWp = DWp + 1j * np.sin(p[mu]) * GAMMAS[mu]
    M = np.zeros((4 * Ns, 4 * Ns), dtype=np.complex128)
    for s in range(Ns):
        M[4 * s:4 * s + 4, 4 * s:4 * s + 4] = DWp + np.eye(4)
        if s + 1 < Ns:
            M[4 * s:4 * s + 4, 4 * (s + 1):4 * (s + 2)] = -P_MINUS
        if s > 0:
            M[4 * s:4 * s + 4, 4 * (s - 1):4 * s] = -P_PLUS
    M[0:4, 4 * (Ns - 1):4 * Ns] += m * P_PLUS
    M[4 * (Ns - 1):4 * Ns, 0:4] += m * P_MINUS
    return M
