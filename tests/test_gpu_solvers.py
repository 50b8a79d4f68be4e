"""GPU solvers against the oracle and the independent pins (dense LU, FFT
free-field solutions), plus failure handling.  The solution check is the
true relative residual ||b - D x|| / ||b|| recomputed by the FP64 oracle D,
and the forward error against an oracle or exact solution."""
import numpy as np
import pytest

from paper_1712_01505_amd import inputs
from tests import _mathpins as mp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def W():
    from paper_1712_01505_amd import wilson
    assert torch.cuda.is_available()
    wilson.lib()
    return wilson


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def true_res(oracle_mod, U, x, b, kappa):
    return rel(oracle_mod.apply(U, x, kappa), b)


@pytest.mark.parametrize("method", ["cgnr", "bicgstab"])
def test_plain_fp64_4x4_matches_dense_lu(W, oracle_mod, method):
    """4^4, kappa 0.12, Haar links, Gaussian source (seed 0), tolerance 1e-12."""
    dims = (4, 4, 4, 4)
    kappa = 0.12
    U = inputs.haar_gauge(dims, seed=inputs.GAUGE_SEED)
    b = inputs.gaussian_spinor(dims, seed=inputs.SOURCE_SEED)
    x, st = W.solve(dev(U), dev(b), kappa, method=method, precision="f64", tol=1e-12, return_stats=True)
    x = x.cpu().numpy()
    assert st["status"] == 0 and st["converged"] == 1
    assert true_res(oracle_mod, U, x, b, kappa) <= 1e-12
    D = mp.dense_wilson(U, kappa, dims)
    x_lu = np.linalg.solve(D, b.ravel()).reshape(b.shape)
    assert rel(x, x_lu) < 1e-10


@pytest.mark.parametrize("method", ["cgnr", "bicgstab"])
def test_free_field_matches_fft(W, method):
    dims = (8, 8, 8, 16)
    kappa = 0.124
    b = inputs.gaussian_spinor(dims, seed=3)
    x = W.solve(dev(inputs.unit_gauge(dims)), dev(b), kappa, method=method, tol=1e-11).cpu().numpy()
    assert rel(x, mp.free_solve_fft(b, kappa)) < 1e-9


@pytest.mark.parametrize("method", ["cgnr", "bicgstab"])
def test_fp64_16x32_true_residual(W, oracle_mod, method):
    """16^3 x 32, eps 0.3 links, kappa 0.125, Gaussian source, 1e-10."""
    dims = (16, 16, 16, 32)
    kappa = 0.125
    U = inputs.near_unity_gauge(dims, 0.3, seed=1)
    b = inputs.gaussian_spinor(dims, seed=0)
    x, st = W.solve(dev(U), dev(b), kappa, method=method, tol=1e-10, return_stats=True)
    assert st["status"] == 0
    r = true_res(oracle_mod, U, x.cpu().numpy(), b, kappa)
    assert r <= 1e-10
    assert abs(r - st["true_rel_res"]) < 1e-12


@pytest.mark.parametrize("method", ["cgnr", "bicgstab"])
@pytest.mark.parametrize("lo", ["f32", "bf16", "f16"])
def test_mixed_precision_reaches_fp64_accuracy(W, oracle_mod, method, lo):
    dims = (8, 8, 8, 16)
    kappa = 0.1255
    U = inputs.near_unity_gauge(dims, 0.3, seed=1)
    b = inputs.gaussian_spinor(dims, seed=0)
    x, st = W.solve(dev(U), dev(b), kappa, method=method, precision="mixed-" + lo, tol=1e-10, return_stats=True)
    x = x.cpu().numpy()
    assert st["status"] == 0, st
    assert true_res(oracle_mod, U, x, b, kappa) <= 1e-10
    x_ref, _, _, _ = oracle_mod.bicgstab(U, b, kappa, tol=1e-13)
    assert rel(x, x_ref) < 1e-8  # forward error <= cond(D) x residual


@pytest.mark.parametrize("method", ["cgnr", "bicgstab"])
def test_multi_rhs_solve_matches_single(W, oracle_mod, method):
    dims = (8, 8, 8, 8)
    kappa = 0.12
    U = inputs.near_unity_gauge(dims, 0.3, seed=4)
    srcs = inputs.point_sources_all_spin_colour(dims)
    xs, st = W.solve(dev(U), dev(srcs), kappa, method=method, tol=1e-10, return_stats=True)
    xs = xs.cpu().numpy()
    assert all(s["converged"] for s in st)
    for k in (0, 7, 11):
        assert true_res(oracle_mod, U, xs[k], srcs[k], kappa) <= 1e-10
        x1 = W.solve(dev(U), dev(srcs[k]), kappa, method=method, tol=1e-10).cpu().numpy()
        assert rel(xs[k], x1) < 1e-8


@pytest.mark.parametrize("method", ["cgnr", "bicgstab"])
def test_multi_rhs_solve_ragged_tiles(W, oracle_mod, method):
    """6 right-hand sides on 6x4x6x6 (tile counts not a multiple of 8, so the
    multi-RHS stencil pads its grid; 2 right-hand sides across the lanes by
    default, so the fused reductions are segmented) in FP64 and mixed FP32."""
    dims = (6, 4, 6, 6)
    kappa = 0.12
    U = inputs.near_unity_gauge(dims, 0.3, seed=6)
    bs = inputs.gaussian_spinor(dims, seed=8, nrhs=6)
    for prec in ("f64", "mixed-f32"):
        xs, st = W.solve(dev(U), dev(bs), kappa, method=method, precision=prec, tol=1e-10, return_stats=True)
        xs = xs.cpu().numpy()
        assert all(s["converged"] for s in st), (prec, st)
        for k in range(6):
            assert true_res(oracle_mod, U, xs[k], bs[k], kappa) <= 1e-10


def test_free_point_source_propagator_batched(W):
    dims = (8, 8, 8, 16)
    kappa = 0.12
    srcs = inputs.point_sources_all_spin_colour(dims)
    xs = W.solve(dev(inputs.unit_gauge(dims)), dev(srcs), kappa, method="bicgstab",
                 precision="mixed-f32", tol=1e-10).cpu().numpy()
    for k in (0, 4, 11):
        assert rel(xs[k], mp.free_solve_fft(srcs[k], kappa)) < 1e-8


# ---------------------------------------------------------------- failure handling
def test_zero_source_gives_zero_solution(W):
    dims = (4, 4, 4, 8)
    U = dev(inputs.haar_gauge(dims))
    b = torch.zeros(inputs.spinor_shape(dims), dtype=torch.complex128, device="cuda")
    for method in ("cgnr", "bicgstab"):
        x, st = W.solve(U, b, 0.12, method=method, return_stats=True)
        assert st["status"] == 0 and st["iters"] == 0 and not torch.any(x != 0)


def test_maxiter_one_is_not_converged(W):
    dims = (4, 4, 4, 8)
    U = dev(inputs.haar_gauge(dims))
    b = dev(inputs.gaussian_spinor(dims))
    for method in ("cgnr", "bicgstab"):
        x, st = W.solve(U, b, 0.12, method=method, maxiter=1, return_stats=True)
        assert st["status"] == W.WL_NOT_CONVERGED and st["converged"] == 0
        assert torch.isfinite(torch.view_as_real(x)).all()


def test_singular_operator_terminates(W):
    """Fully periodic free field at kappa = 1/8 has a zero mode."""
    dims = (4, 4, 4, 4)
    U = dev(inputs.unit_gauge(dims))
    b = torch.ones(inputs.spinor_shape(dims), dtype=torch.complex128, device="cuda")
    for method in ("cgnr", "bicgstab"):
        _, st = W.solve(U, b, 0.125, method=method, maxiter=300, bc=(1, 1, 1, 1), return_stats=True)
        assert st["status"] in (W.WL_NOT_CONVERGED, W.WL_BREAKDOWN) and not st["converged"]


def test_nan_source_reports_enan(W):
    dims = (4, 4, 4, 8)
    U = dev(inputs.haar_gauge(dims))
    b = inputs.gaussian_spinor(dims)
    b[0, 0, 0, 0, 0, 0] = np.nan
    with pytest.raises(W.WilsonError) as e:
        W.solve(U, dev(b), 0.12)
    assert e.value.code == W.WL_ENAN


def test_warm_restart_from_solution(W, oracle_mod):
    dims = (8, 8, 8, 8)
    U = inputs.near_unity_gauge(dims, 0.3, seed=2)
    b = inputs.gaussian_spinor(dims, seed=5)
    Ud, bd = dev(U), dev(b)
    x1 = W.solve(Ud, bd, 0.12, tol=1e-10)
    x2, st = W.solve(Ud, bd, 0.12, tol=1e-10, x0=x1, return_stats=True)
    assert st["iters"] <= 1
    assert rel(x2.cpu().numpy(), x1.cpu().numpy()) < 1e-9


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_solver_with_each_stencil_variant(W, oracle_mod, prec):
    """The fused-reduction stencils of every code variant drive a solve to the
    same answer (the variants differ in schedule, not in arithmetic)."""
    dims = (8, 8, 8, 16)
    kappa = 0.12
    U = inputs.near_unity_gauge(dims, 0.3, seed=2)
    b = inputs.gaussian_spinor(dims, seed=3)
    Ud = dev(U)
    hi = W.Operator.create(Ud, kappa, W.WL_F64)
    lo = None if prec == "f64" else W.Operator.create(Ud, kappa, W.PREC[prec])
    op = hi if lo is None else lo
    xs, vs = [], []
    for var in W.VARIANTS[op.prec]:
        if not W.try_set_launch(op.handle, 1, 128, 1, 1, var):
            continue
        x, st = W.solve(None, dev(b), kappa, method="bicgstab", precision="f64" if lo is None else "mixed-" + prec,
                        tol=1e-10, ops=(hi, lo), return_stats=True)
        assert st["converged"], (var, st)
        xs.append(x.cpu().numpy())
        vs.append(var)
    assert len(xs) >= 4
    for x in xs:
        assert rel(oracle_mod.apply(U, x, kappa), b) <= 1e-10
    if prec == "f64":
        # variants 0-3 share the per-workgroup partial layout, so even the
        # reductions round identically; t-walk sums its column first
        same = [x for x, v in zip(xs, vs) if v < 4]
        for x in same[1:]:
            assert np.array_equal(x, same[0])


@pytest.mark.parametrize("method", ["bicgstab", "cgnr"])
@pytest.mark.parametrize("lo", ["f32", "bf16", "f16"])
def test_reliable_updates_reach_fp64_accuracy(W, oracle_mod, lo, method):
    """Reliable updates (one inner run, FP64 solution and residual refreshed
    in place) meet the same bar as defect correction.  CG on the normal
    equations with 16-bit storage is offered with defect correction only:
    asking it for reliable updates is rejected (WL_EPREC), nothing runs."""
    dims = (8, 8, 8, 16)
    kappa = 0.1255
    U = inputs.near_unity_gauge(dims, 0.3, seed=1)
    b = inputs.gaussian_spinor(dims, seed=0)
    if method == "cgnr" and lo != "f32":
        with pytest.raises(W.WilsonError) as ei:
            W.solve(dev(U), dev(b), kappa, method=method, precision="mixed-" + lo, tol=1e-10, reliable=True)
        assert ei.value.code == W.WL_EPREC
        return
    x, st = W.solve(dev(U), dev(b), kappa, method=method, precision="mixed-" + lo, tol=1e-10,
                    reliable=True, return_stats=True)
    x = x.cpu().numpy()
    assert st["status"] == 0, st
    assert st["outer"] >= 2  # at least one in-run update besides the last check
    assert true_res(oracle_mod, U, x, b, kappa) <= 1e-10
    x_ref, _, _, _ = oracle_mod.bicgstab(U, b, kappa, tol=1e-13)
    assert rel(x, x_ref) < 1e-8


def test_reliable_updates_multi_rhs_and_adjoint(W, oracle_mod):
    """12 point sources together, and the adjoint system, with reliable updates."""
    dims = (8, 8, 8, 8)
    kappa = 0.12
    U = inputs.near_unity_gauge(dims, 0.3, seed=4)
    srcs = inputs.point_sources_all_spin_colour(dims)
    xs, st = W.solve(dev(U), dev(srcs), kappa, method="bicgstab", precision="mixed-f16", tol=1e-10,
                     reliable=True, return_stats=True)
    xs = xs.cpu().numpy()
    assert all(s["converged"] for s in st)
    for k in (0, 5, 11):
        assert true_res(oracle_mod, U, xs[k], srcs[k], kappa) <= 1e-10
    b = inputs.gaussian_spinor(dims, seed=9)
    y = W.solve(dev(U), dev(b), kappa, method="bicgstab", precision="mixed-bf16", tol=1e-10, reliable=True,
                dagger=True).cpu().numpy()
    g5 = mp.gamma5_spinor
    # D^dag = gamma5 D gamma5
    assert rel(g5(oracle_mod.apply(U, g5(y), kappa)), b) <= 1e-10
