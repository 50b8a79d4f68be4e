"""GPU parity of the packed layouts and the Wilson stencil against the FP64
CPU oracle (element by element, same seeded inputs).

Tolerances (relative 2-norm over the whole field, inputs shared in FP64):
FP64 1e-12 and FP32 1e-5 (the stencil's accuracy target); the 16-bit storage
formats are checked against their own rounding bound: one rounding of each
input (u = 2^-8 BF16, 2^-11 FP16, relative to the site maximum) propagated
through 8 hops of unit-norm links, i.e. a few u.
"""
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


# ---------------------------------------------------------------- pack / unpack
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f16"])
def test_pack_unpack_roundtrip(W, prec):
    dims = (4, 6, 2, 10)
    psi = inputs.gaussian_spinor(dims, seed=3, nrhs=3)
    psi[1, 0, 0, 0, 0] = 0.0  # an all-zero site (scale 0)
    p = W.PREC[prec]
    back = W.unpack_spinor(W.pack_spinor(dev(psi), p), dims, p, nrhs=3).cpu().numpy()
    if prec == "f64":
        assert np.array_equal(back, psi)
    elif prec == "f32":
        assert np.array_equal(back, psi.astype(np.complex64).astype(np.complex128))
    else:
        u = 2.0 ** -8 if prec == "bf16" else 2.0 ** -11
        site_max = np.abs(np.stack([psi.real, psi.imag])).max(axis=(0, 5, 6), keepdims=False)
        err = np.maximum(np.abs(back.real - psi.real), np.abs(back.imag - psi.imag)).max(axis=(4, 5))
        assert np.all(err <= u * site_max * 1.0001)
        assert np.all(back[1, 0, 0, 0, 0] == 0)


# ---------------------------------------------------------------- stencil vs oracle
CASES = [
    ((2, 2, 2, 2), "haar"),          # every +mu and -mu neighbour coincide
    ((4, 4, 4, 4), "haar"),
    ((3, 5, 2, 7), "haar"),          # odd extents, V = 210 (ragged last tile)
    ((8, 8, 8, 8), "near"),
    ((12, 12, 12, 12), "near"),
    ((16, 16, 16, 32), "near"),
]


def _gauge(dims, kind):
    return inputs.haar_gauge(dims, seed=1) if kind == "haar" else inputs.near_unity_gauge(dims, 0.3, seed=1)


@pytest.mark.parametrize("dims,kind", CASES)
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f16"])
@pytest.mark.parametrize("dagger", [False, True])
def test_apply_matches_oracle(W, oracle_mod, dims, kind, prec, dagger):
    kappa = 0.1255
    U = _gauge(dims, kind)
    psi = inputs.gaussian_spinor(dims, seed=0)
    ref = oracle_mod.apply(U, psi, kappa, dagger=dagger)
    p = W.PREC[prec]
    op = W.Operator.create(dev(U), kappa, p)
    for var in W.VARIANTS[p]:
        for xcd in (0, 1, 2, 3, 4, 5):
            if not W.try_set_launch(op.handle, 1, 64, 1, xcd, var):
                continue  # e.g. a t-walk column length not dividing Lt, or no z-slabs
            out = W.apply(None, dev(psi), kappa, dagger=dagger, op=op).cpu().numpy()
            assert rel(out, ref) < TOL[prec], (var, xcd)


@pytest.mark.parametrize("dims,kind", CASES[:4])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_dslash_matches_oracle(W, oracle_mod, dims, kind, prec):
    U = _gauge(dims, kind)
    psi = inputs.gaussian_spinor(dims, seed=4)
    for dagger in (False, True):
        out = W.dslash(dev(U), dev(psi), dagger=dagger, prec=prec).cpu().numpy()
        ref = oracle_mod.hop(U, psi, dagger=dagger)
        assert rel(out, ref) < TOL[prec]


def test_bc_variants(W, oracle_mod):
    dims = (4, 2, 6, 4)
    U = inputs.haar_gauge(dims, seed=5)
    psi = inputs.gaussian_spinor(dims, seed=6)
    for bc in [(1, 1, 1, 1), (-1, -1, -1, -1), (1, -1, 1, -1), (-1, 1, 1, 1)]:
        out = W.apply(dev(U), dev(psi), 0.11, bc=bc).cpu().numpy()
        assert rel(out, oracle_mod.apply(U, psi, 0.11, bc=bc)) < 1e-12


def test_kappa_zero_identity_and_free_field(W):
    dims = (4, 4, 4, 8)
    psi = inputs.gaussian_spinor(dims, seed=2)
    U = inputs.haar_gauge(dims, seed=2)
    out = W.apply(dev(U), dev(psi), 0.0).cpu().numpy()
    assert np.array_equal(out, psi)


@pytest.mark.parametrize("dims", [(8, 4, 6, 8), (8, 4, 8, 8)])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_multi_rhs_columns_equal_single_rhs(W, prec, dims):
    """Every launch shape for 12 right-hand sides (tile counts that are and
    are not multiples of 8, slab order where Lz allows it) gives the
    single-RHS result bit for bit."""
    U = inputs.near_unity_gauge(dims, 0.3, seed=3)
    psi = inputs.gaussian_spinor(dims, seed=7, nrhs=12)
    p = W.PREC[prec]
    op = W.Operator.create(dev(U), 0.125, p)
    src = op.pack(dev(psi))
    outs, cfgs = [], []
    for rpt in (1, 2, 3, 4):
        if rpt > W.MAX_RPT[p]:
            continue
        for lanes in ((1, 2, 4) if rpt == 1 else (1,)):
            for block in (64, 256, 512):
                for xcd in (0, 1, 2, 4, 5):
                    for var in (W.VARIANTS[p] if rpt == 1 else (0,)):
                        for gm in ((0, 1) if block == 256 else (0,)):  # group-major order
                            if not W.try_set_launch(op.handle, 12, block, rpt, xcd, var, lanes, rhs_major=gm):
                                continue
                            dst = op.new_field(12)
                            op.apply_packed(dst, src, 12)
                            outs.append(op.unpack(dst, 12).cpu().numpy())
                            cfgs.append((block, rpt, xcd, var, lanes, gm))
    for o, cfg in zip(outs[1:], cfgs[1:]):
        if p in (W.WL_BF16S, W.WL_F16S) and cfg[3] >= 4:
            # t-walk applies a neighbour's 16-bit scale in a different place: equal to rounding
            assert rel(o, outs[0]) < 1e-6, cfg
        else:
            assert np.array_equal(o, outs[0]), cfg  # launch shape never changes a result
    for k in (0, 5, 11):
        single = W.apply(dev(U), dev(psi[k]), 0.125, prec=prec, op=op).cpu().numpy()
        assert np.array_equal(single, outs[0][k])


def test_full_size_sampled_parity_32x64(W, oracle_mod):
    """32^3 x 64 FP64 and FP32 apply (the benchmark size), checked on sampled sites."""
    dims = (32, 32, 32, 64)
    kappa = 0.1255
    U = inputs.near_unity_gauge(dims, 0.3, seed=1)
    psi = inputs.gaussian_spinor(dims, seed=0)
    rng = np.random.default_rng(11)
    V = inputs.volume(dims)
    sites = np.unique(np.concatenate([rng.integers(0, V, 3000), [0, 31, 32 * 31, V - 1, V - 32768, 32767]]))
    ref = oracle_mod.apply_sites(U, psi, kappa, sites)
    Ud, pd = dev(U), dev(psi)
    for prec, tol in (("f64", 1e-12), ("f32", 1e-5)):
        out = W.apply(Ud, pd, kappa, prec=prec).reshape(V, 4, 3)[torch.from_numpy(sites).cuda()].cpu().numpy()
        assert rel(out, ref) < tol, prec
    del Ud, pd
    torch.cuda.empty_cache()


def test_gamma5_hermiticity_on_gpu(W):
    dims = (8, 8, 8, 16)
    U = dev(inputs.haar_gauge(dims, seed=9))
    x = inputs.gaussian_spinor(dims, seed=1)
    y = inputs.gaussian_spinor(dims, seed=2)
    Dy = W.apply(U, dev(y), 0.125).cpu().numpy()
    Ddx = W.apply(U, dev(x), 0.125, dagger=True).cpu().numpy()
    lhs, rhs = np.vdot(x, Dy), np.vdot(Ddx, y)
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_multi_lattice_plan_every_shape(W):
    """A plan run in every launch shape (and again after each run: the
    queue counter resets itself) reproduces the separate launches."""
    lattices = [(4, 4, 4, 4), (6, 4, 6, 2), (8, 8, 8, 8)]
    for prec in ("f64", "f32", "bf16", "f16"):
        p = W.PREC[prec]
        ops, srcs, dsts, refs = [], [], [], []
        for j, dims in enumerate(lattices):
            op = W.Operator.create(dev(inputs.near_unity_gauge(dims, 0.3, seed=20 + j)), 0.12, p)
            src = op.pack(dev(inputs.gaussian_spinor(dims, seed=200 + j, nrhs=4)))
            ref = op.new_field(4)
            op.apply_packed(ref, src, 4)
            ops.append(op)
            srcs.append(src)
            dsts.append(op.new_field(4))
            refs.append(op.unpack(ref, 4))
        for dagger in (0, 1):
            if dagger:
                refs = []
                for o, s_ in zip(ops, srcs):
                    r = o.new_field(4)
                    o.apply_packed(r, s_, 4, dagger=True)
                    refs.append(o.unpack(r, 4))
            plan = W.MultiPlan([(o.handle, d.data_ptr(), s_.data_ptr()) for o, d, s_ in zip(ops, dsts, srcs)],
                               dagger, 4)
            n = 0
            for pers in (1, 0):
                for block in (64, 256):
                    for rpt in (1, 2, 4):
                        for var in (0, 1, 2, 3):
                            if not plan.set_launch(block, rpt, var, pers):
                                continue
                            for rep in range(2):
                                for d in dsts:
                                    d.zero_()
                                plan.run()
                                torch.cuda.synchronize()
                                for o, d, r in zip(ops, dsts, refs):
                                    assert torch.equal(o.unpack(d, 4), r), (prec, dagger, pers, block, rpt, var, rep)
                            n += 1
            assert n >= 12
            plan.tune()
            for d in dsts:
                d.zero_()
            plan.run()
            torch.cuda.synchronize()
            for o, d, r in zip(ops, dsts, refs):
                assert torch.equal(o.unpack(d, 4), r), (prec, dagger, "tuned", plan.launch())
            del plan


def test_multi_lattice_plan_many_small(W):
    """An ensemble of 40 small lattices of four shapes in one plan (tuned,
    then run twice) equals the separate launches bit for bit."""
    shapes = [(4, 4, 4, 4), (6, 6, 6, 6), (8, 8, 8, 8), (4, 4, 4, 8)]
    for prec in ("f32", "f16"):
        p = W.PREC[prec]
        ops, srcs, dsts, refs = [], [], [], []
        for j in range(40):
            dims = shapes[j % 4]
            op = W.Operator.create(dev(inputs.near_unity_gauge(dims, 0.3, seed=300 + j)), 0.12, p)
            src = op.pack(dev(inputs.gaussian_spinor(dims, seed=400 + j, nrhs=4)))
            ref = op.new_field(4)
            op.apply_packed(ref, src, 4)
            ops.append(op)
            srcs.append(src)
            dsts.append(op.new_field(4))
            refs.append(op.unpack(ref, 4))
        plan = W.MultiPlan([(o.handle, d.data_ptr(), s_.data_ptr()) for o, d, s_ in zip(ops, dsts, srcs)], 0, 4)
        plan.tune()
        for rep in range(2):
            for d in dsts:
                d.zero_()
            plan.run()
            torch.cuda.synchronize()
            for j, (o, d, r) in enumerate(zip(ops, dsts, refs)):
                assert torch.equal(o.unpack(d, 4), r), (prec, rep, j, plan.launch())


def test_multi_lattice_launch_matches_separate(W):
    lattices = [(8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 32), (20, 20, 20, 20)]
    for prec in ("f64", "f32"):
        p = W.PREC[prec]
        ops, srcs, dsts, refs = [], [], [], []
        for j, dims in enumerate(lattices):
            U = inputs.near_unity_gauge(dims, 0.3, seed=10 + j)
            psi = inputs.gaussian_spinor(dims, seed=100 * j, nrhs=4)
            op = W.Operator.create(dev(U), 0.12 + 0.001 * j, p)
            src = op.pack(dev(psi))
            ref = op.new_field(4)
            op.apply_packed(ref, src, 4)
            ops.append(op)
            srcs.append(src)
            dsts.append(op.new_field(4))
            refs.append(ref)
        W.wilson_multi_apply([(o.handle, d.data_ptr(), s.data_ptr()) for o, d, s in zip(ops, dsts, srcs)], 0, 4,
                             W._stream())
        torch.cuda.synchronize()
        for o, d, r in zip(ops, dsts, refs):
            assert torch.equal(o.unpack(d, 4), o.unpack(r, 4))
