"""The merged BiCGStab iteration the solver runs (rho' = <rh, s> - omega <rh, t>
formed before r' = s - omega t, x, r and the next p updated in one pass) is the
textbook recurrence of Sec. II-C regrouped: on a dense Wilson matrix both give
the same iterates to rounding, also across a residual replacement (reliable
update), and the GPU solver needs the oracle's iteration count."""
import numpy as np
import pytest

from paper_1712_01505_amd import inputs
from tests._mathpins import dense_wilson


def _dot(a, b):
    return np.vdot(a, b)  # sum conj(a) b


def textbook(A, b, iters, replace_at=None):
    x = np.zeros_like(b)
    r = b.copy()
    rh = r.copy()
    rho = _dot(rh, r)
    p = r.copy()
    out = []
    for k in range(iters):
        v = A @ p
        alpha = rho / _dot(rh, v)
        s = r - alpha * v
        t = A @ s
        omega = _dot(t, s) / _dot(t, t)
        x = x + alpha * p + omega * s
        r = s - omega * t
        if replace_at is not None and k == replace_at:
            r = b - A @ x  # reliable update: the true residual replaces r
        rho_new = _dot(rh, r)
        beta = (rho_new / rho) * (alpha / omega)
        rho = rho_new
        p = r + beta * (p - omega * v)
        out.append(x.copy())
    return out


def merged(A, b, iters, replace_at=None):
    x = np.zeros_like(b)
    r = b.copy()
    rh = r.copy()
    rho = _dot(rh, r)
    p = r.copy()
    v = np.zeros_like(b)
    out = []
    pending_p = False
    beta = 0.0
    for k in range(iters):
        if pending_p:
            p = r + beta * (p - omega * v)
            pending_p = False
        v = A @ p
        alpha = rho / _dot(rh, v)
        s = r - alpha * v
        t = A @ s
        # the second product's reduction: <s,t>, |t|^2, <rh,s>, <rh,t>
        st, tt, hs, ht = _dot(s, t), _dot(t, t).real, _dot(rh, s), _dot(rh, t)
        omega = np.conj(st) / tt
        rho_new = hs - omega * ht
        beta = (rho_new / rho) * (alpha / omega)
        rho_prev, rho = rho, rho_new
        x = x + alpha * p + omega * s
        r = s - omega * t
        if replace_at is not None and k == replace_at:
            r = b - A @ x
            rho = _dot(rh, r)  # recomputed from the replaced r
            beta = (rho / rho_prev) * (alpha / omega)
            pending_p = True
        else:
            p = r + beta * (p - omega * v)
        out.append(x.copy())
    return out


@pytest.mark.parametrize("replace_at", [None, 5])
def test_merged_iteration_equals_textbook(replace_at):
    dims = (2, 2, 2, 4)
    U = inputs.near_unity_gauge(dims, 0.5, seed=7)
    A = dense_wilson(U, 0.124, dims)
    b = inputs.gaussian_spinor(dims, seed=8).reshape(-1)
    xa = textbook(A, b, 14, replace_at)
    xb = merged(A, b, 14, replace_at)
    for k, (a, m) in enumerate(zip(xa, xb)):
        assert np.linalg.norm(a - m) <= 1e-11 * np.linalg.norm(a), k
    # and the iteration converges (the recurrence is the solver's, not a stand-in)
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(xb[-1] - xs) < 1e-3 * np.linalg.norm(xs)


def test_merged_rho_equals_explicit_dot():
    """rho' = <rh, s> - omega <rh, t> is <rh, s - omega t> (linearity in the
    second argument); a mutation that conjugates omega breaks it."""
    rng = np.random.default_rng(3)
    rh, s, t = (rng.standard_normal(96) + 1j * rng.standard_normal(96) for _ in range(3))
    omega = 0.3 - 0.7j
    explicit = _dot(rh, s - omega * t)
    assert abs((_dot(rh, s) - omega * _dot(rh, t)) - explicit) < 1e-12 * abs(explicit)
    assert abs((_dot(rh, s) - np.conj(omega) * _dot(rh, t)) - explicit) > 1e-3 * abs(explicit)


@pytest.fixture(scope="module")
def W():
    torch = pytest.importorskip("torch")
    from paper_1712_01505_amd import wilson
    assert torch.cuda.is_available()
    wilson.lib()
    return wilson


@pytest.mark.gpu
def test_gpu_bicgstab_iterations_match_oracle(W, oracle_mod):
    """FP64: the merged GPU iteration and the oracle's textbook BiCGStab stop
    within one iteration of each other at the same tolerance."""
    import torch
    dims = (8, 8, 8, 16)
    kappa = 0.124
    U = inputs.near_unity_gauge(dims, 0.3, seed=11)
    b = inputs.gaussian_spinor(dims, seed=12)
    x, st = W.solve(torch.from_numpy(U).cuda(), torch.from_numpy(b).cuda(), kappa, method="bicgstab", tol=1e-10,
                    return_stats=True)
    _, ost, oit, orel = oracle_mod.bicgstab(U, b, kappa, tol=1e-10)
    assert st["status"] == 0 and ost == 0
    assert abs(st["iters"] - oit) <= 1, (st["iters"], oit)
