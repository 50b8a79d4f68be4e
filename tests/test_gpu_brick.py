"""The LDS-staged brick walk (stencil code variant 7) against the FP64 CPU
oracle, element by element on the same seeded inputs, over brick shapes
that span a direction or not (halo faces or wrap inside the brick), walk
lengths, odd walks and every storage precision; FP64 and FP32 results must
equal the straight-line kernel's bit for bit (same order of additions).

Tolerances as in test_gpu_stencil: FP64 1e-12, FP32 1e-5, 16-bit storage
against its rounding bound."""
import numpy as np
import pytest

from paper_1712_01505_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2, "f16": 3e-3}


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def W():
    from paper_1712_01505_amd import wilson
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    wilson.lib()
    return wilson


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


# (dims, links, [(brick, t_steps), ...])
CASES = [
    ((4, 4, 4, 4), "haar", [((4, 4, 4), 4), ((4, 4, 4), 1)]),              # brick = whole slice: no halo
    ((8, 8, 8, 8), "near", [((8, 8, 1), 8), ((4, 4, 4), 2), ((8, 4, 4), 4), ((8, 8, 4), 8), ((8, 2, 8), 1)]),
    ((8, 4, 8, 6), "haar", [((8, 4, 2), 3), ((4, 4, 4), 6), ((8, 4, 8), 2)]),  # Lt = 6, odd walk of 3
    ((12, 12, 12, 12), "near", [((4, 4, 4), 4), ((4, 4, 12), 3)]),        # brick spans z only
    ((16, 16, 16, 32), "near", [((8, 8, 4), 16), ((16, 4, 4), 8), ((8, 4, 4), 4), ((16, 16, 1), 32)]),
]


def _gauge(dims, kind):
    return inputs.haar_gauge(dims, seed=1) if kind == "haar" else inputs.near_unity_gauge(dims, 0.3, seed=1)


@pytest.mark.parametrize("dims,kind,shapes", CASES)
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f16"])
def test_brick_apply_matches_oracle(W, oracle_mod, dims, kind, shapes, prec):
    kappa = 0.1255
    U = _gauge(dims, kind)
    psi = inputs.gaussian_spinor(dims, seed=0)
    p = W.PREC[prec]
    op = W.Operator.create(dev(U), kappa, p)
    src = op.pack(dev(psi))
    for dagger in (False, True):
        ref = oracle_mod.apply(U, psi, kappa, dagger=dagger)
        assert W.try_set_launch(op.handle, 1, 64, 1, 0, 0)
        base = op.new_field()
        op.apply_packed(base, src, 1, dagger)
        base = op.unpack(base).cpu().numpy()
        n = 0
        for brick, T in shapes:
            for xcd in (0, 1):
                block = brick[0] * brick[1] * brick[2]
                if not W.try_set_launch(op.handle, 1, block, 1, xcd, W.VAR_BRICK, brick=brick, t_steps=T):
                    continue
                dst = op.new_field()
                op.apply_packed(dst, src, 1, dagger)
                out = op.unpack(dst).cpu().numpy()
                assert rel(out, ref) < TOL[prec], (brick, T, xcd, dagger)
                if prec in ("f64", "f32"):
                    assert np.array_equal(out, base), (brick, T, xcd, dagger)
                n += 1
        assert n >= 2 * len(shapes) - 1


def test_brick_rejects_shapes_that_do_not_tile(W):
    dims = (8, 8, 8, 8)
    op = W.Operator.create(dev(inputs.near_unity_gauge(dims, 0.3, seed=1)), 0.12, W.WL_F32)
    bad = [((8, 8, 2), 8, 64),    # block != bx by bz
           ((6, 4, 4), 8, 96),    # 6 does not divide 8; 96 sites
           ((8, 8, 4), 3, 256),   # walk length does not divide Lt
           ((8, 8, 8), 8, 512),   # more than 256 sites
           ((4, 4, 2), 8, 32)]    # fewer than 64
    for brick, T, block in bad:
        assert not W.try_set_launch(op.handle, 1, block, 1, 0, W.VAR_BRICK, brick=brick, t_steps=T), brick
    assert not W.try_set_launch(op.handle, 2, 128, 1, 0, W.VAR_BRICK, lanes=2, brick=(8, 4, 4), t_steps=8)
    assert W.try_set_launch(op.handle, 1, 128, 1, 0, W.VAR_BRICK, brick=(8, 4, 4), t_steps=8)
    got = W.wl_get_launch(op.handle, 1)
    assert got[3] == W.VAR_BRICK and tuple(got[5:10]) == (8, 4, 4, 8, 0)
    # an occupancy cap: the staged slices must fit the LDS share
    assert W.try_set_launch(op.handle, 1, 128, 1, 0, W.VAR_BRICK, brick=(8, 4, 4), t_steps=8, wg_per_cu=4)
    assert W.wl_get_launch(op.handle, 1)[9] == 4
    assert not W.try_set_launch(op.handle, 1, 128, 1, 0, W.VAR_BRICK, brick=(8, 4, 4), t_steps=8, wg_per_cu=3)
    assert not W.try_set_launch(op.handle, 1, 128, 1, 0, 1, wg_per_cu=2)  # brick walk only


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_brick_multi_rhs_and_dslash(W, oracle_mod, prec):
    """Several right-hand sides (one workgroup set each) and the hopping term
    alone."""
    dims = (8, 8, 8, 16)
    U = inputs.near_unity_gauge(dims, 0.3, seed=3)
    psi = inputs.gaussian_spinor(dims, seed=7, nrhs=3)
    p = W.PREC[prec]
    op = W.Operator.create(dev(U), 0.125, p)
    assert W.try_set_launch(op.handle, 3, 128, 1, 1, W.VAR_BRICK, brick=(8, 4, 4), t_steps=8)
    out = W.apply(None, dev(psi), 0.125, prec=prec, op=op).cpu().numpy()
    for k in range(3):
        assert rel(out[k], oracle_mod.apply(U, psi[k], 0.125)) < TOL[prec], k
    assert W.try_set_launch(op.handle, 1, 256, 1, 0, W.VAR_BRICK, brick=(8, 8, 4), t_steps=4)
    h = op.new_field()
    src1 = op.pack(dev(psi[1]))
    op.dslash_packed(h, src1)
    assert rel(op.unpack(h).cpu().numpy(), oracle_mod.hop(U, psi[1])) < TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
@pytest.mark.parametrize("method", ["bicgstab", "cgnr"])
def test_brick_fused_reductions_drive_solves(W, oracle_mod, prec, method):
    """The brick walk's fused reductions (|out|^2 for CGNR; <rh, D p> and the
    merged <s, t>, |t|^2, <rh, s>, <rh, t> for BiCGStab) drive plain and
    mixed solves to the oracle's 1e-10."""
    dims = (8, 8, 8, 16)
    kappa = 0.12
    U = inputs.near_unity_gauge(dims, 0.3, seed=2)
    b = inputs.gaussian_spinor(dims, seed=3)
    Ud = dev(U)
    hi = W.Operator.create(Ud, kappa, W.WL_F64)
    lo = None if prec == "f64" else W.Operator.create(Ud, kappa, W.PREC[prec])
    for o in (hi, lo):
        if o is not None:
            assert W.try_set_launch(o.handle, 1, 128, 1, 1, W.VAR_BRICK, brick=(8, 4, 4), t_steps=4)
    x, st = W.solve(None, dev(b), kappa, method=method, precision="f64" if lo is None else "mixed-" + prec,
                    tol=1e-10, ops=(hi, lo), return_stats=True)
    assert st["converged"], st
    assert rel(oracle_mod.apply(U, x.cpu().numpy(), kappa), b) <= 1e-10


def test_autotune_writes_json_cache(W, tmp_path):
    """wl_autotune keeps its choices per (arch, extents, precision, nrhs,
    dagger, reduction) and writes them to the JSON file named by
    $WL_TUNE_CACHE; the entries name the shapes the op then launches with."""
    import json
    import os
    dims = (16, 16, 16, 32)
    op = W.Operator.create(dev(inputs.near_unity_gauge(dims, 0.3, seed=3)), 0.12, W.WL_F32)
    path = tmp_path / "tune.json"
    old = os.environ.get("WL_TUNE_CACHE")
    os.environ["WL_TUNE_CACHE"] = str(path)
    try:
        W.wl_autotune(op.handle, 1, 1, W._stream())
    finally:
        if old is None:
            del os.environ["WL_TUNE_CACHE"]
        else:
            os.environ["WL_TUNE_CACHE"] = old
    doc = json.loads(path.read_text())
    mine = [e for e in doc["entries"] if e.get("dims") == list(dims) and e.get("prec") == W.WL_F32
            and e.get("nrhs") == 1 and e.get("dagger") == 1]
    assert sorted(e["reduction"] for e in mine) == [0, 1, 2, 3, 4, 5], mine
    for e in mine:
        assert e["key"].endswith(f":16x16x16x32:p1:n1:d1:r{e['reduction']}") and e["us"] > 0
        assert e["arch"].startswith("gfx")
        if e["variant"] == W.VAR_BRICK:
            assert e["block"] == e["brick"][0] * e["brick"][1] * e["brick"][2] and e["t_steps"] > 0
