"""Launch shapes in which several columns share the gauge field (Sec. II-B:
it is common to every right-hand side): the t-walks (variants 4, 5) with
right-hand sides interleaved across the lanes of each wavefront, and the
brick walk (variant 7) with several right-hand sides per workgroup.
Outputs equal the one-column shapes bit for bit in FP64 and FP32, the fused
reductions of the solvers equal the inner products of the stored vectors
column by column, and the t-walk tile counts include grids with idle units
(nxyz not a multiple of the tile)."""
import numpy as np
import pytest

from paper_1712_01505_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KAPPA = 0.124


@pytest.fixture(scope="module")
def W():
    from paper_1712_01505_amd import wilson
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    wilson.lib()
    return wilson


def _cdot(a, b):
    return np.vdot(a.ravel(), b.ravel())


def _want(kind, W, inq, oq, vq):
    if kind == W.WL_DOT_BICG:
        return [_cdot(inq, oq), _cdot(oq, oq), _cdot(vq, inq), _cdot(vq, oq), _cdot(inq, inq)]
    if kind == W.WL_DOT_V:
        return [_cdot(vq, oq)]
    return [_cdot(oq, oq)]


def _got(kind, W, d):
    if kind == W.WL_DOT_BICG:
        return [d[0] + 1j * d[1], d[2], d[3] + 1j * d[4], d[5] + 1j * d[6], d[7]]
    if kind == W.WL_DOT_V:
        return [d[0] + 1j * d[1]]
    return [d[0]]


@pytest.mark.parametrize("dims", [(8, 4, 8, 8), (6, 6, 5, 8)])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_twalk_column_lanes_apply_and_reductions(W, oracle_mod, prec, dims):
    nrhs = 8
    U = inputs.near_unity_gauge(dims, 0.3, seed=12)
    psi = inputs.gaussian_spinor(dims, seed=13, nrhs=nrhs)
    vv = inputs.gaussian_spinor(dims, seed=14, nrhs=nrhs)
    p = W.PREC[prec]
    op = W.Operator.create(torch.from_numpy(U).cuda(), KAPPA, p)
    src = op.pack(torch.from_numpy(psi).cuda())
    vsrc = op.pack(torch.from_numpy(vv).cuda())
    inq = op.unpack(src, nrhs).cpu().numpy()
    vq = op.unpack(vsrc, nrhs).cpu().numpy()
    tol = {"f64": 1e-12, "f32": 1e-5, "f16": 3e-3}[prec]
    for dagger in (False, True):
        ref = np.stack([oracle_mod.apply(U, psi[r], KAPPA, dagger=dagger) for r in range(nrhs)])
        for var in (4, 5):
            assert W.try_set_launch(op.handle, nrhs, 128, 1, 1, var, 1)
            base = op.new_field(nrhs)
            op.apply_packed(base, src, nrhs, dagger)
            base = op.unpack(base, nrhs)
            n = 0
            for lanes, gm in ((2, 0), (4, 0), (8, 0), (2, 1), (4, 1)):
                for block, xcd in ((128, 0), (256, 1), (64, 1)):
                    if not W.try_set_launch(op.handle, nrhs, block, 1, xcd, var, lanes, rhs_major=gm):
                        continue
                    cfg = (dagger, var, lanes, block, xcd, gm)
                    dst = op.new_field(nrhs)
                    op.apply_packed(dst, src, nrhs, dagger)
                    out = op.unpack(dst, nrhs)
                    if prec == "f16":
                        assert np.linalg.norm((out - base).cpu().numpy()) <= 1e-6 * torch.linalg.norm(base).item(), cfg
                    else:
                        assert torch.equal(out, base), cfg
                    oc = out.cpu().numpy()
                    for r in range(nrhs):
                        assert np.linalg.norm(oc[r] - ref[r]) <= tol * np.linalg.norm(ref[r]), cfg + (r,)
                    for kind in (W.WL_DOT_BICG, W.WL_DOT_V, W.WL_DOT_NORM):
                        d2 = op.new_field(nrhs)
                        dots = W.apply_dot(op, d2, src, vsrc, dagger=dagger, nrhs=nrhs, kind=kind).cpu().numpy()
                        o2 = op.unpack(d2, nrhs)
                        if prec != "f16":
                            assert torch.equal(o2, out), cfg + (kind,)
                        oq = o2.cpu().numpy()
                        for r in range(nrhs):
                            for g_, w_ in zip(_got(kind, W, dots[:, r]), _want(kind, W, inq[r], oq[r], vq[r])):
                                assert abs(g_ - w_) <= 1e-12 * max(abs(w_), 1e-300) + 1e-9, cfg + (kind, r, g_, w_)
                    n += 1
            assert n >= 4, (var, n)


def test_twalk_column_lanes_rejected_shapes(W):
    """Fewer than 32 sites per workgroup, lanes not dividing the columns, the
    brick walk with lanes, a group order other than 0 or 1: rejected."""
    dims = (8, 8, 8, 8)
    U = inputs.near_unity_gauge(dims, 0.3, seed=1)
    op = W.Operator.create(torch.from_numpy(U).cuda(), KAPPA, W.WL_F32)
    assert not W.try_set_launch(op.handle, 8, 128, 1, 0, 4, 8)   # 16 sites per workgroup
    assert W.try_set_launch(op.handle, 8, 256, 1, 0, 4, 8)       # 32
    assert not W.try_set_launch(op.handle, 6, 256, 1, 0, 4, 4)   # 4 does not divide 6
    assert not W.try_set_launch(op.handle, 4, 512, 1, 0, 4, 4)   # t-walk: at most 256 threads
    assert not W.try_set_launch(op.handle, 4, 256, 1, 0, W.VAR_BRICK, 2, brick=(8, 8, 4), t_steps=4)
    assert not W.try_set_launch(op.handle, 8, 256, 1, 0, 4, 2, rhs_major=2)
    assert W.try_set_launch(op.handle, 8, 256, 1, 0, 4, 2, rhs_major=1)
    assert W.wl_get_launch(op.handle, 8)[10] == 1


def test_group_major_brick_and_solver_columns(W, oracle_mod):
    """Group-major order for the brick walk (12 right-hand sides, one per
    lane) equals the default order bit for bit; a 4-column CGNR solve whose
    stencils run group-major reaches the oracle's residual."""
    dims = (8, 8, 8, 8)
    U = inputs.near_unity_gauge(dims, 0.3, seed=21)
    psi = inputs.gaussian_spinor(dims, seed=22, nrhs=12)
    op = W.Operator.create(torch.from_numpy(U).cuda(), KAPPA, W.WL_F32)
    src = op.pack(torch.from_numpy(psi).cuda())
    outs = []
    for gm in (0, 1):
        assert W.try_set_launch(op.handle, 12, 128, 1, 1, W.VAR_BRICK, brick=(8, 4, 4), t_steps=4, rhs_major=gm)
        dst = op.new_field(12)
        op.apply_packed(dst, src, 12)
        outs.append(op.unpack(dst, 12))
    assert torch.equal(outs[0], outs[1])
    b = inputs.gaussian_spinor(dims, seed=23, nrhs=4)
    op64 = W.Operator.create(torch.from_numpy(U).cuda(), KAPPA, W.WL_F64)
    assert W.try_set_launch(op64.handle, 4, 128, 1, 1, 4, 2, rhs_major=1)
    x, st = W.solve(None, torch.from_numpy(b).cuda(), KAPPA, method="cgnr", tol=1e-10, return_stats=True,
                    ops=(op64, None))
    xs = x.cpu().numpy()
    for r in range(4):
        assert st[r]["status"] == 0, st[r]
        res = b[r] - oracle_mod.apply(U, xs[r], KAPPA)
        assert np.linalg.norm(res) <= 1e-10 * np.linalg.norm(b[r]), r


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f16"])
def test_brick_several_rhs_per_workgroup(W, oracle_mod, prec):
    """The brick walk holding 2 or 4 right-hand sides per workgroup (each
    with its own LDS stage, all behind the same barriers): every column equals
    the one-right-hand-side brick (bit for bit in FP64 / FP32), in both group
    orders, for the plain apply and every fused reduction of the solvers,
    whose inner products equal those of the stored vectors."""
    dims = (8, 8, 8, 8)
    nrhs = 8
    U = inputs.near_unity_gauge(dims, 0.3, seed=31)
    psi = inputs.gaussian_spinor(dims, seed=32, nrhs=nrhs)
    vv = inputs.gaussian_spinor(dims, seed=33, nrhs=nrhs)
    p = W.PREC[prec]
    op = W.Operator.create(torch.from_numpy(U).cuda(), KAPPA, p)
    src = op.pack(torch.from_numpy(psi).cuda())
    vsrc = op.pack(torch.from_numpy(vv).cuda())
    inq = op.unpack(src, nrhs).cpu().numpy()
    vq = op.unpack(vsrc, nrhs).cpu().numpy()
    tol = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2, "f16": 3e-3}[prec]
    for dagger in (False, True):
        ref = np.stack([oracle_mod.apply(U, psi[r], KAPPA, dagger=dagger) for r in range(nrhs)])
        assert W.try_set_launch(op.handle, nrhs, 128, 1, 1, W.VAR_BRICK, 1, brick=(8, 4, 4), t_steps=4)
        base = op.new_field(nrhs)
        op.apply_packed(base, src, nrhs, dagger)
        base = op.unpack(base, nrhs)
        n = 0
        for rw, brick, T, gm, xcd in ((2, (8, 4, 4), 4, 0, 1), (4, (4, 4, 4), 8, 0, 0), (4, (4, 4, 4), 4, 1, 1),
                                      (2, (4, 4, 4), 8, 1, 0)):
            block = brick[0] * brick[1] * brick[2] * rw
            assert W.try_set_launch(op.handle, nrhs, block, 1, xcd, W.VAR_BRICK, rw, brick=brick, t_steps=T,
                                    rhs_major=gm), (rw, brick, T)
            cfg = (dagger, rw, brick, T, gm, xcd)
            dst = op.new_field(nrhs)
            op.apply_packed(dst, src, nrhs, dagger)
            out = op.unpack(dst, nrhs)
            if prec in ("f64", "f32"):
                assert torch.equal(out, base), cfg
            else:
                assert np.linalg.norm((out - base).cpu().numpy()) <= 1e-6 * torch.linalg.norm(base).item(), cfg
            oc = out.cpu().numpy()
            for r in range(nrhs):
                assert np.linalg.norm(oc[r] - ref[r]) <= tol * np.linalg.norm(ref[r]), cfg + (r,)
            for kind in (W.WL_DOT_BICG, W.WL_DOT_V, W.WL_DOT_NORM):
                d2 = op.new_field(nrhs)
                dots = W.apply_dot(op, d2, src, vsrc, dagger=dagger, nrhs=nrhs, kind=kind).cpu().numpy()
                oq = op.unpack(d2, nrhs).cpu().numpy()
                for r in range(nrhs):
                    for g_, w_ in zip(_got(kind, W, dots[:, r]), _want(kind, W, inq[r], oq[r], vq[r])):
                        assert abs(g_ - w_) <= 1e-12 * max(abs(w_), 1e-300) + 1e-9, cfg + (kind, r, g_, w_)
            n += 1
        assert n == 4


def test_brick_several_rhs_rejected_shapes(W):
    """More than 256 threads, 8 right-hand sides per workgroup, a count not
    dividing the columns, stages beyond the LDS: rejected."""
    dims = (8, 8, 8, 8)
    U = inputs.near_unity_gauge(dims, 0.3, seed=1)
    op = W.Operator.create(torch.from_numpy(U).cuda(), KAPPA, W.WL_F64)
    B = W.VAR_BRICK
    assert W.try_set_launch(op.handle, 4, 256, 1, 0, B, 4, brick=(4, 4, 4), t_steps=4)
    assert not W.try_set_launch(op.handle, 4, 512, 1, 0, B, 4, brick=(8, 4, 4), t_steps=4)   # 512 threads
    assert not W.try_set_launch(op.handle, 8, 512, 1, 0, B, 8, brick=(4, 4, 4), t_steps=4)   # 8 per workgroup
    assert not W.try_set_launch(op.handle, 6, 256, 1, 0, B, 4, brick=(4, 4, 4), t_steps=4)   # 4 does not divide 6
    assert not W.try_set_launch(op.handle, 4, 256, 1, 0, B, 4, brick=(8, 4, 4), t_steps=4)   # block != sites x 4
    assert W.wl_get_launch(op.handle, 4)[4] == 4


def test_brick_several_rhs_in_a_solve(W, oracle_mod):
    """A 4-column mixed FP32 BiCGStab whose inner stencils run the brick with
    two right-hand sides per workgroup reaches the oracle's residual."""
    dims = (8, 8, 8, 8)
    U = inputs.near_unity_gauge(dims, 0.3, seed=41)
    b = inputs.gaussian_spinor(dims, seed=42, nrhs=4)
    Ud = torch.from_numpy(U).cuda()
    hi = W.Operator.create(Ud, KAPPA, W.WL_F64)
    lo = W.Operator.create(Ud, KAPPA, W.WL_F32)
    assert W.try_set_launch(lo.handle, 4, 256, 1, 1, W.VAR_BRICK, 2, brick=(8, 4, 4), t_steps=4)
    x, st = W.solve(None, torch.from_numpy(b).cuda(), KAPPA, method="bicgstab", tol=1e-10, return_stats=True,
                    ops=(hi, lo))
    xs = x.cpu().numpy()
    for r in range(4):
        assert st[r]["status"] == 0, st[r]
        res = b[r] - oracle_mod.apply(U, xs[r], KAPPA)
        assert np.linalg.norm(res) <= 1e-10 * np.linalg.norm(b[r]), r
