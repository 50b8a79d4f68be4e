"""Multi-lattice solves (wilson_solve_multi): uneven lattices with several
right-hand sides each, every stencil application of the iteration one
multi-lattice launch, every column with its own scalars.  Each column's
solution is checked against the oracle's D (its true residual <= 1e-10) and
the iteration counts against the same systems solved one by one."""
import numpy as np
import pytest

from paper_1712_01505_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

C4 = [(8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 32), (20, 20, 20, 20)]


@pytest.fixture(scope="module")
def W():
    from paper_1712_01505_amd import wilson
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    wilson.lib()
    return wilson


def _systems(W, lattices, nrhs, hi_prec, lo_prec, seed, kappas=None):
    out, host = [], []
    for j, dims in enumerate(lattices):
        U = inputs.near_unity_gauge(dims, 0.3, seed=seed + j)
        b = inputs.gaussian_spinor(dims, seed=seed + 100 + j, nrhs=nrhs)
        kappa = kappas[j] if kappas else 0.12 + 0.001 * j
        Ud = torch.from_numpy(U).cuda()
        hi = W.Operator.create(Ud, kappa, W.PREC[hi_prec])
        lo = W.Operator.create(Ud, kappa, W.PREC[lo_prec]) if lo_prec else None
        out.append((hi, lo, hi.pack(torch.from_numpy(b).cuda())))
        host.append((U, b, kappa))
    return out, host


def _check_oracle(W, oracle_mod, systems, host, xs, nrhs, st):
    for j, ((hi, _, _), (U, b, kappa), x) in enumerate(zip(systems, host, xs)):
        xc = hi.unpack(x, nrhs).cpu().numpy()
        for r in range(nrhs):
            res = b[r] - oracle_mod.apply(U, xc[r], kappa)
            rel = np.linalg.norm(res) / np.linalg.norm(b[r])
            assert rel <= 1e-10, (j, r, rel, st[j * nrhs + r])


@pytest.mark.parametrize("method", ["bicgstab", "cgnr"])
def test_c4_mixed_f32_multi_solve_matches_oracle(W, oracle_mod, method):
    """The uneven set {8^4, 12^4, 16^3 x 32, 20^4} x 4 Gaussian sources, FP32
    inner solves in FP64 refinement, solved together."""
    nrhs = 4
    systems, host = _systems(W, C4, nrhs, "f64", "f32", seed=70)
    xs, st = W.solve_multi(systems, nrhs=nrhs, method=method, tol=1e-10, return_stats=True)
    assert all(s["status"] == 0 and s["converged"] for s in st), st
    _check_oracle(W, oracle_mod, systems, host, xs, nrhs, st)
    # each lattice solved on its own needs about as many inner iterations
    for j, (hi, lo, b) in enumerate(systems):
        _, sj = W.solve(None, hi.unpack(b, nrhs), hi.kappa, method=method, precision="mixed-f32", tol=1e-10,
                        ops=(hi, lo), return_stats=True)
        for r in range(nrhs):
            a, m = sj[r]["iters"], st[j * nrhs + r]["iters"]
            assert abs(a - m) <= max(4, 0.1 * a), (j, r, a, m)


def test_plain_fp64_multi_solve_ragged(W, oracle_mod):
    """Plain FP64 BiCGStab on lattices of very different size and
    conditioning (the easy one stops early and is frozen while the others
    go on); two right-hand sides each."""
    lattices = [(4, 4, 4, 4), (6, 4, 4, 8), (8, 8, 8, 16)]
    systems, host = _systems(W, lattices, 2, "f64", None, seed=80, kappas=[0.08, 0.12, 0.124])
    xs, st = W.solve_multi(systems, nrhs=2, method="bicgstab", tol=1e-10, return_stats=True)
    assert all(s["status"] == 0 for s in st), st
    _check_oracle(W, oracle_mod, systems, host, xs, 2, st)
    assert st[0]["iters"] < st[4]["iters"], st


@pytest.mark.parametrize("lo,method,kw", [("f16", "bicgstab", {"form": 1}), ("f32", "bicgstab", {"reliable": True}),
                                          ("f16", "cgnr", {})])
def test_multi_solve_variants(W, oracle_mod, lo, method, kw):
    """16-bit inner solves, the single-reduction form and reliable updates
    over several lattices."""
    lattices = [(8, 8, 8, 8), (8, 8, 8, 16), (12, 12, 12, 12)]
    systems, host = _systems(W, lattices, 2, "f64", lo, seed=90)
    xs, st = W.solve_multi(systems, nrhs=2, method=method, tol=1e-10, return_stats=True, **kw)
    assert all(s["status"] == 0 for s in st), st
    _check_oracle(W, oracle_mod, systems, host, xs, 2, st)
