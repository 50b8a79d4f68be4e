"""Domain-wall operator (paper Sec. II-B, eq. (2)) and CG on its normal
equations (Sec. II-C, Sec. VI-B) on the GPU, against the FP64 oracle."""
import numpy as np
import pytest

from paper_1712_01505_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

M0, MQ = -1.8, 0.05
TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2, "f16": 3e-3}


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def field5(dims, Ns, seed, nvec=None):
    f = np.stack([inputs.gaussian_spinor(dims, seed=seed + s) for s in range(Ns * (nvec or 1))])
    return f if nvec is None else f.reshape((nvec, Ns) + f.shape[1:])


@pytest.fixture(scope="module")
def W():
    from paper_1712_01505_amd import wilson
    assert torch.cuda.is_available()
    wilson.lib()
    return wilson


@pytest.mark.parametrize("dims,Ns", [((4, 4, 4, 8), 8), ((3, 5, 2, 7), 4), ((8, 8, 8, 8), 6)])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f16"])
def test_dw_apply_matches_oracle(W, oracle_mod, dims, Ns, prec):
    """Every launch shape the operator offers (variants, the t-walks, slices
    across lanes, tile orders), both D_DW and D_DW^dag."""
    U = inputs.near_unity_gauge(dims, 0.3, seed=1) if dims[0] == 8 else inputs.haar_gauge(dims, seed=1)
    psi = field5(dims, Ns, 10)
    p = W.PREC[prec]
    op = W.DWOperator.create(dev(U), M0, MQ, Ns, p)
    src = op.pack(dev(psi))
    for dagger in (False, True):
        ref = oracle_mod.dw_apply(U, psi, M0, MQ, dagger=dagger)
        n = 0
        for var in (0, 1, 2, 4, 5):
            for lanes in (1, 2, 4, 8):
                for block, xcd in ((64, 0), (256, 1), (512, 2), (128, 0)):
                    if not W.try_set_launch(op.handle, 1, block, 1, xcd, var, lanes):
                        continue
                    dst = op.new_field()
                    op.apply_packed(dst, src, 1, dagger)
                    out = op.unpack(dst).cpu().numpy()
                    assert rel(out, ref) < TOL[prec], (dagger, var, lanes, block, xcd)
                    n += 1
        assert n >= 4


def test_dw_launch_shapes_agree_bitwise(W):
    """The launch shape never changes an FP64/FP32 domain-wall result."""
    dims, Ns = (4, 4, 8, 8), 8
    U = inputs.near_unity_gauge(dims, 0.3, seed=2)
    psi = field5(dims, Ns, 30)
    for prec in ("f64", "f32"):
        op = W.DWOperator.create(dev(U), M0, MQ, Ns, W.PREC[prec])
        src = op.pack(dev(psi))
        outs = []
        for var in (0, 1, 2, 4, 5):
            for lanes in (1, 4, 8):
                for block, xcd in ((512, 0), (512, 2), (256, 5), (256, 0)):
                    if W.try_set_launch(op.handle, 1, block, 1, xcd, var, lanes):
                        dst = op.new_field()
                        op.apply_packed(dst, src)
                        outs.append(op.unpack(dst).cpu().numpy())
        assert len(outs) >= 6
        for o in outs[1:]:
            assert np.array_equal(o, outs[0])


def test_dw_several_vectors_equal_one_at_a_time(W, oracle_mod):
    dims, Ns = (4, 4, 4, 4), 4
    U = inputs.haar_gauge(dims, seed=3)
    psi = field5(dims, Ns, 50, nvec=3)
    op = W.DWOperator.create(dev(U), M0, MQ, Ns, W.WL_F64)
    both = W.dw_apply(None, dev(psi), M0, MQ, op=op).cpu().numpy()
    for k in range(3):
        one = W.dw_apply(None, dev(psi[k]), M0, MQ, op=op).cpu().numpy()
        assert np.array_equal(both[k], one)
        assert rel(one, oracle_mod.dw_apply(U, psi[k], M0, MQ)) < 1e-12


def test_dw_apply_16x32_full_compare(W, oracle_mod):
    """16^3 x 32 with Ns = 8 (the paper's per-node domain-wall lattice) in FP64 and FP32."""
    dims, Ns = (16, 16, 16, 32), 8
    U = inputs.near_unity_gauge(dims, 0.3, seed=1)
    psi = field5(dims, Ns, 0)
    ref = oracle_mod.dw_apply(U, psi, M0, MQ)
    Ud, pd = dev(U), dev(psi)
    for prec in ("f64", "f32"):
        out = W.dw_apply(Ud, pd, M0, MQ, prec=prec).cpu().numpy()
        assert rel(out, ref) < TOL[prec], prec
    del Ud, pd
    torch.cuda.empty_cache()


@pytest.mark.parametrize("precision,reliable", [("f64", 0), ("mixed-f32", 0), ("mixed-f16", 0),
                                                ("mixed-f32", 1), ("mixed-f16", 1)])
def test_dw_cgnr_reaches_tolerance(W, oracle_mod, precision, reliable):
    """CG on D_DW^dag D_DW to 1e-10 by the oracle's residual; 16-bit storage
    with reliable updates is not offered for CG (WL_EPREC, nothing runs)."""
    dims, Ns = (8, 8, 8, 8), 8
    U = inputs.near_unity_gauge(dims, 0.3, seed=1)
    b = field5(dims, Ns, 0)
    if precision == "mixed-f16" and reliable:
        with pytest.raises(W.WilsonError) as ei:
            W.dw_solve(dev(U), dev(b), M0, MQ, precision=precision, tol=1e-10, reliable=True)
        assert ei.value.code == W.WL_EPREC
        return
    x, st = W.dw_solve(dev(U), dev(b), M0, MQ, precision=precision, tol=1e-10, return_stats=True,
                       reliable=bool(reliable))
    assert st["status"] == 0 and st["converged"], st
    x = x.cpu().numpy()
    r = rel(oracle_mod.dw_apply(U, x, M0, MQ), b)
    assert r <= 1e-10
    assert abs(r - st["true_rel_res"]) < 1e-12
    x_ref, code, _, _ = oracle_mod.dw_cgnr(U, b, M0, MQ, tol=1e-13)
    assert code == 0 and rel(x, x_ref) < 1e-7


def test_dw_cgnr_several_vectors_and_dense_pin(W, oracle_mod):
    """Two 5-d right-hand sides at once on 2^3 x 4 (Ns = 4), each checked against a dense solve."""
    from tests import _mathpins as mp
    dims, Ns = (2, 2, 2, 4), 4
    U = inputs.haar_gauge(dims, seed=5)
    b = field5(dims, Ns, 70, nvec=2)
    xs, st = W.dw_solve(dev(U), dev(b), M0, MQ, precision="f64", tol=1e-12, return_stats=True)
    assert all(s["converged"] for s in st)
    D = mp.dense_dw(U, M0, MQ, Ns, dims)
    for k in range(2):
        x_lu = np.linalg.solve(D, b[k].ravel()).reshape(b[k].shape)
        assert rel(xs[k].cpu().numpy(), x_lu) < 1e-9
