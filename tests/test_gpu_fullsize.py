"""The benchmark-size lattice (32^3 x 64, eps = 0.3 links, kappa = 0.1255)
in the launch shapes the benchmark runs: every storage precision after the
autotuner has chosen its shapes, the plain apply and the three fused-reduction
launches the solvers use, checked against the FP64 oracle on sampled sites
(random sites plus both t faces, where the t walks start and end), and the
fused inner products against their definition.

Tolerances: FP64 1e-12, FP32 1e-5 (relative 2-norm over the sampled sites),
16-bit storage against its rounding bound; inner products of the kernel's own
stored output to 1e-12 relative (FP64 accumulation in another order)."""
import numpy as np
import pytest

from paper_1712_01505_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2, "f16": 3e-3}
DIMS = (32, 32, 32, 64)
KAPPA = 0.1255


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def W():
    from paper_1712_01505_amd import wilson
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    wilson.lib()
    return wilson


@pytest.fixture(scope="module")
def fields():
    U = inputs.near_unity_gauge(DIMS, 0.3, seed=inputs.GAUGE_SEED)
    psi = inputs.gaussian_spinor(DIMS, seed=inputs.SOURCE_SEED)
    v = inputs.gaussian_spinor(DIMS, seed=5)
    V = inputs.volume(DIMS)
    vs = DIMS[0] * DIMS[1] * DIMS[2]
    rng = np.random.default_rng(11)
    sites = np.unique(np.concatenate([rng.integers(0, V, 2000), rng.integers(0, vs, 300),
                                      V - vs + rng.integers(0, vs, 300), [0, vs - 1, V - vs, V - 1]]))
    return U, psi, v, sites


def _cdot(a, b):
    return np.vdot(a.ravel(), b.ravel())


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f16"])
def test_tuned_launches_match_oracle_32x64(W, oracle_mod, fields, prec):
    U, psi, v, sites = fields
    p = W.PREC[prec]
    Ud = torch.from_numpy(U).cuda()
    op = W.Operator.create(Ud, KAPPA, p)
    del Ud
    W.wl_autotune(op.handle, 1, 0, W._stream())
    src = op.pack(torch.from_numpy(psi).cuda())
    vsrc = op.pack(torch.from_numpy(v).cuda())
    idx = torch.from_numpy(sites).cuda()
    V = inputs.volume(DIMS)
    for dagger in (False, True):
        ref = oracle_mod.apply_sites(U, psi, KAPPA, sites, dagger=dagger)
        dst = op.new_field()
        op.apply_packed(dst, src, 1, dagger)
        out = op.unpack(dst)
        plain = out.reshape(V, 4, 3)[idx].cpu().numpy()
        assert rel(plain, ref) < TOL[prec], (prec, dagger, W.wl_get_launch(op.handle, 1))
        # the solvers' fused-reduction launches, each in its own tuned shape
        inq = op.unpack(src).cpu().numpy()
        vq = op.unpack(vsrc).cpu().numpy()
        for kind in (W.WL_DOT_BICG, W.WL_DOT_V, W.WL_DOT_NORM):
            d2 = op.new_field()
            dots = W.apply_dot(op, d2, src, vsrc, dagger=dagger, kind=kind).cpu().numpy()[:, 0]
            o2 = op.unpack(d2)
            got = o2.reshape(V, 4, 3)[idx].cpu().numpy()
            assert rel(got, ref) < TOL[prec], (prec, dagger, kind)
            if prec in ("f64", "f32"):
                assert torch.equal(o2, out), (prec, dagger, kind)  # every shape adds in the same order
            oq = o2.cpu().numpy()
            if kind == W.WL_DOT_BICG:
                want = [_cdot(inq, oq), _cdot(oq, oq), _cdot(vq, inq), _cdot(vq, oq), _cdot(inq, inq)]
                got_c = [dots[0] + 1j * dots[1], dots[2], dots[3] + 1j * dots[4], dots[5] + 1j * dots[6], dots[7]]
            elif kind == W.WL_DOT_V:
                want, got_c = [_cdot(vq, oq)], [dots[0] + 1j * dots[1]]
            else:
                want, got_c = [_cdot(oq, oq)], [dots[0]]
            for g_, w_ in zip(got_c, want):
                assert abs(g_ - w_) <= 1e-12 * max(abs(w_), 1e-300) + 1e-9, (prec, dagger, kind, g_, w_)
    if prec == "f64":
        # the inner products against the oracle's own D psi (FP64 inputs)
        Dpsi = oracle_mod.apply(U, psi, KAPPA)
        d2 = op.new_field()
        dots = W.apply_dot(op, d2, src, vsrc, kind=W.WL_DOT_BICG).cpu().numpy()[:, 0]
        for g_, w_ in zip([dots[0] + 1j * dots[1], dots[2], dots[5] + 1j * dots[6]],
                          [_cdot(psi, Dpsi), _cdot(Dpsi, Dpsi), _cdot(v, Dpsi)]):
            assert abs(g_ - w_) <= 1e-12 * abs(w_)
    del op, src, vsrc
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f16"])
def test_multi_lattice_plan_matches_oracle(W, oracle_mod, prec):
    """The uneven lattices {8^4, 12^4, 16^3 x 32, 20^4} x 4 Gaussian sources in
    one plan -- persistent queue, one workgroup per item, and the tuned shape --
    against the oracle column by column, for D and D^dag."""
    lattices = [(8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 32), (20, 20, 20, 20)]
    p = W.PREC[prec]
    Us, psis, kappas, ops, srcs, dsts = [], [], [], [], [], []
    for j, dims in enumerate(lattices):
        U = inputs.near_unity_gauge(dims, 0.3, seed=10 + j)
        psi = inputs.gaussian_spinor(dims, seed=100 * j, nrhs=4)
        kappa = 0.12 + 0.001 * j
        op = W.Operator.create(torch.from_numpy(U).cuda(), kappa, p)
        Us.append(U)
        psis.append(psi)
        kappas.append(kappa)
        ops.append(op)
        srcs.append(op.pack(torch.from_numpy(psi).cuda()))
        dsts.append(op.new_field(4))
    descs = [(o.handle, d.data_ptr(), s_.data_ptr()) for o, d, s_ in zip(ops, dsts, srcs)]
    for dagger in (0, 1):
        refs = [[oracle_mod.apply(U, psi[k], kappa, dagger=bool(dagger)) for k in range(4)]
                for U, psi, kappa in zip(Us, psis, kappas)]
        plan = W.MultiPlan(descs, dagger, 4)
        forms = [(256, 1, 1, 1), (128, 2, 0, 0), (64, 1, 0, 0), None]
        for form in forms:
            if form is None:
                plan.tune()
            else:
                block, rpt, var, pers = form
                assert plan.set_launch(block, rpt, var, pers), form
            for d in dsts:
                d.zero_()
            plan.run()
            torch.cuda.synchronize()
            for j, (o, d) in enumerate(zip(ops, dsts)):
                out = o.unpack(d, 4).cpu().numpy()
                for k in range(4):
                    assert rel(out[k], refs[j][k]) < TOL[prec], (prec, dagger, form, plan.launch(), j, k)
        del plan
