"""Enforced-halo apply (the paper's single-node runs with the boundary copy
enforced, Sec. IV): face pack, device copy, interior with the wrapping t hops
cut, boundary finish.  Its result must equal the plain apply (FP64/FP32: to
the order of additions) and the oracle."""
import numpy as np
import pytest

from paper_1712_01505_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2, "f16": 3e-3}
SAME = {"f64": 1e-14, "f32": 2e-6}


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.fixture(scope="module")
def W():
    from paper_1712_01505_amd import wilson
    assert torch.cuda.is_available()
    wilson.lib()
    return wilson


@pytest.mark.parametrize("dims,bc", [((4, 4, 4, 8), (1, 1, 1, -1)), ((3, 5, 2, 7), (1, 1, 1, -1)),
                                     ((8, 8, 8, 2), (1, 1, 1, 1)), ((4, 2, 6, 4), (-1, 1, -1, -1))])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f16"])
def test_halo_apply_matches_plain_and_oracle(W, oracle_mod, dims, bc, prec):
    kappa = 0.1255
    U = inputs.haar_gauge(dims, seed=2)
    psi = inputs.gaussian_spinor(dims, seed=3, nrhs=4)
    p = W.PREC[prec]
    op = W.Operator.create(dev(U), kappa, p, bc)
    src = op.pack(dev(psi))
    halo = op.halo_buffer(4)
    for dagger in (False, True):
        ref = np.stack([oracle_mod.apply(U, psi[k], kappa, bc=bc, dagger=dagger) for k in range(4)])
        plain = op.new_field(4)
        op.apply_packed(plain, src, 4, dagger)
        plain = op.unpack(plain, 4).cpu().numpy()
        n = 0
        for var, lanes, block, xcd in ((0, 1, 64, 0), (1, 1, 128, 1), (2, 2, 256, 1), (1, 4, 256, 0), (5, 1, 64, 1)):
            if not W.try_set_launch(op.handle, 4, block, 1, xcd, var, lanes):
                continue
            out = op.new_field(4)
            op.apply_halo_packed(out, src, halo, 4, dagger)
            got = op.unpack(out, 4).cpu().numpy()
            assert rel(got, ref) < TOL[prec], (dagger, var, lanes)
            if prec in SAME:
                assert rel(got, plain) < SAME[prec], (dagger, var, lanes)
            n += 1
        assert n >= 3


def test_halo_apply_32x64_sampled(W, oracle_mod):
    """32^3 x 64 FP32 through the halo path, checked on sampled sites of the t faces and the bulk."""
    dims = (32, 32, 32, 64)
    kappa = 0.1255
    U = inputs.near_unity_gauge(dims, 0.3, seed=1)
    psi = inputs.gaussian_spinor(dims, seed=0)
    V = inputs.volume(dims)
    vs = 32 ** 3
    rng = np.random.default_rng(5)
    sites = np.unique(np.concatenate([rng.integers(0, vs, 500), V - vs + rng.integers(0, vs, 500),
                                      rng.integers(0, V, 1000)]))
    ref = oracle_mod.apply_sites(U, psi, kappa, sites)
    op = W.Operator.create(dev(U), kappa, W.WL_F32)
    src = op.pack(dev(psi))
    out = op.new_field()
    op.apply_halo_packed(out, src, op.halo_buffer())
    got = op.unpack(out).reshape(V, 4, 3)[torch.from_numpy(sites).cuda()].cpu().numpy()
    assert rel(got, ref) < 1e-5
    del op, src, out
    torch.cuda.empty_cache()
