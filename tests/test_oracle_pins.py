"""Pins of the FP64 CPU oracle against mathematics (CPU only, no GPU).

Each test checks the oracle against something other than itself: the closed-
form free-field spectrum and plane waves, gamma_5-hermiticity, gauge
covariance, a dense matrix built independently by Kronecker products, dense LU,
the FFT-exact free-field solution, the kappa = 0 and D_W-normalisation special
cases, and finite differences of the solve.  A plausible slip in the oracle (a
wrong projector sign, a transposed link, a missed boundary sign, a swapped
dagger) fails at least one of them; the planted-mistake tests at the end prove
that for a few such slips.
"""
import numpy as np
import pytest

from paper_1712_01505_amd import inputs
from tests import _mathpins as mp

BC = (1, 1, 1, -1)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# ---------------------------------------------------------------- gamma basis
def test_oracle_gammas_are_chiral_basis(oracle_mod):
    g = [oracle_mod.gamma(mu) for mu in range(4)]
    for a in range(4):
        assert np.allclose(g[a], g[a].conj().T)
        for b in range(4):
            assert np.allclose(g[a] @ g[b] + g[b] @ g[a], 2 * np.eye(4) * (a == b))
        assert np.linalg.matrix_rank(np.eye(4) - g[a]) == 2
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    assert np.allclose(g5, np.diag([1, 1, -1, -1]))
    # the same basis as the independently typed copy in the test helpers
    assert np.allclose(np.array(g), mp.GAMMAS)


# ---------------------------------------------------------------- operator pins
@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 2, 2, 4), (4, 2, 2, 4)])
def test_free_field_spectrum_closed_form(oracle_mod, dims):
    kappa = 0.13
    U = inputs.unit_gauge(dims)
    V = inputs.volume(dims)
    n = 12 * V
    D = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[:] = 0
        e[j] = 1
        D[:, j] = oracle_mod.apply(U, e.reshape(inputs.spinor_shape(dims)), kappa, BC).ravel()
    ev = np.sort_complex(np.round(np.linalg.eigvals(D), 10))
    ref = np.sort_complex(np.round(mp.free_spectrum(dims, kappa, BC), 10))
    assert np.allclose(ev, ref, atol=1e-9)


def test_free_field_plane_wave_eigenvector(oracle_mod):
    dims = (4, 4, 4, 4)
    kappa = 0.12
    U = inputs.unit_gauge(dims)
    p = [2 * np.pi * 1 / 4, 2 * np.pi * 3 / 4, 0.0, (2 * np.pi * 2 + np.pi) / 4]
    Dp = (1 - 2 * kappa * sum(np.cos(q) for q in p)) * np.eye(4) + 2j * kappa * sum(
        mp.GAMMAS[mu] * np.sin(p[mu]) for mu in range(4))
    lam, vecs = np.linalg.eig(Dp)
    colour = np.array([0.3, -0.2j, 0.5])
    t, z, y, x = np.meshgrid(*[np.arange(4)] * 4, indexing="ij")
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    for k in range(4):
        psi = phase[..., None, None] * np.outer(vecs[:, k], colour)[None, None, None, None]
        out = oracle_mod.apply(U, psi, kappa, BC)
        assert rel(out, lam[k] * psi) < 1e-13


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 2, 2, 4), (3, 2, 2, 4), (4, 4, 4, 4)])
@pytest.mark.parametrize("dagger", [False, True])
def test_oracle_matches_independent_dense_builder(oracle_mod, dims, dagger):
    kappa = 0.12
    U = inputs.haar_gauge(dims, seed=3)
    D = mp.dense_wilson(U, kappa, dims, BC, dagger=dagger)
    psi = inputs.gaussian_spinor(dims, seed=5)
    ref = (D @ psi.ravel()).reshape(psi.shape)
    out = oracle_mod.apply(U, psi, kappa, BC, dagger=dagger)
    assert rel(out, ref) < 1e-14


def test_oracle_bc_all_periodic_and_all_antiperiodic(oracle_mod):
    dims = (2, 2, 2, 4)
    U = inputs.haar_gauge(dims, seed=11)
    psi = inputs.gaussian_spinor(dims, seed=12)
    for bc in [(1, 1, 1, 1), (-1, -1, -1, -1), (1, -1, 1, -1)]:
        D = mp.dense_wilson(U, 0.11, dims, bc)
        assert rel(oracle_mod.apply(U, psi, 0.11, bc), (D @ psi.ravel()).reshape(psi.shape)) < 1e-14


def test_gamma5_hermiticity(oracle_mod):
    dims = (4, 4, 4, 8)
    kappa = 0.125
    U = inputs.haar_gauge(dims, seed=2)
    x = inputs.gaussian_spinor(dims, seed=3)
    y = inputs.gaussian_spinor(dims, seed=4)
    lhs = np.vdot(x, oracle_mod.apply(U, y, kappa))
    g5Dg5x = mp.gamma5_spinor(oracle_mod.apply(U, mp.gamma5_spinor(x), kappa))
    rhs = np.vdot(g5Dg5x, y)
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)
    # the dagger apply is gamma5 D gamma5, site by site
    assert rel(oracle_mod.apply(U, x, kappa, dagger=True), g5Dg5x) < 1e-14
    # and it is the adjoint: <x, D y> = <D^dag x, y>
    assert abs(np.vdot(oracle_mod.apply(U, x, kappa, dagger=True), y) - lhs) < 1e-11 * abs(lhs)


def test_gauge_covariance(oracle_mod):
    dims = (4, 4, 2, 4)
    kappa = 0.13
    U = inputs.haar_gauge(dims, seed=8)
    Om = inputs.random_gauge_transform(dims, seed=9)
    psi = inputs.gaussian_spinor(dims, seed=10)
    UO = mp.gauge_transform_links(U, Om, dims)
    Om_psi = np.einsum("tzyxab,tzyxsb->tzyxsa", Om, psi)
    lhs = oracle_mod.apply(UO, Om_psi, kappa)
    rhs = np.einsum("tzyxab,tzyxsb->tzyxsa", Om, oracle_mod.apply(U, psi, kappa))
    assert rel(lhs, rhs) < 1e-14


def test_kappa_zero_is_identity(oracle_mod):
    dims = (2, 2, 2, 4)
    U = inputs.haar_gauge(dims)
    psi = inputs.gaussian_spinor(dims)
    assert np.array_equal(oracle_mod.apply(U, psi, 0.0), psi)


def test_paper_normalisation_DW(oracle_mod):
    """eq. (1): D_W = (m0+4) - 1/2 H equals D / (2 kappa) for m0 = 1/(2 kappa) - 4."""
    dims = (2, 2, 4, 4)
    U = inputs.haar_gauge(dims, seed=21)
    psi = inputs.gaussian_spinor(dims, seed=22)
    for kappa in (0.12, 0.125, 0.1255):
        m0 = 1 / (2 * kappa) - 4
        DW = (m0 + 4) * psi - 0.5 * oracle_mod.hop(U, psi)
        assert rel(DW, oracle_mod.apply(U, psi, kappa) / (2 * kappa)) < 1e-14


def test_nearest_neighbour_support(oracle_mod):
    """A point source couples only to itself and its 8 nearest neighbours."""
    dims = (6, 6, 6, 6)
    U = inputs.haar_gauge(dims, seed=4)
    src = inputs.point_source(dims, site=(2, 3, 4, 5), spin=1, colour=2)
    out = oracle_mod.apply(U, src, 0.12)
    nz = np.argwhere(np.abs(out).sum(axis=(4, 5)) > 0)
    got = {tuple(v) for v in nz}
    t, z, y, x = 5, 4, 3, 2
    want = {(t, z, y, x)}
    for d in (1, -1):
        want |= {((t + d) % 6, z, y, x), (t, (z + d) % 6, y, x), (t, z, (y + d) % 6, x), (t, z, y, (x + d) % 6)}
    assert got == want


def test_apply_sites_matches_full_apply(oracle_mod):
    dims = (4, 4, 4, 8)
    U = inputs.near_unity_gauge(dims)
    psi = inputs.gaussian_spinor(dims)
    full = oracle_mod.apply(U, psi, 0.125).reshape(-1, 4, 3)
    sites = np.array([0, 1, 63, 64, 500, 511])
    assert np.array_equal(oracle_mod.apply_sites(U, psi, 0.125, sites), full[sites])


# ---------------------------------------------------------------- solver pins
def test_cgnr_and_bicgstab_match_dense_lu_C1(oracle_mod):
    """Plain FP64 workload: 4^4, kappa = 0.12, Haar links, Gaussian source, tol 1e-12."""
    dims = (4, 4, 4, 4)
    kappa = 0.12
    U = inputs.haar_gauge(dims, seed=inputs.GAUGE_SEED)
    b = inputs.gaussian_spinor(dims, seed=inputs.SOURCE_SEED)
    D = mp.dense_wilson(U, kappa, dims, BC)
    x_lu = np.linalg.solve(D, b.ravel()).reshape(b.shape)
    x, st, it, rr = oracle_mod.cgnr(U, b, kappa, tol=1e-12)
    assert st == 0 and rr <= 1e-12 and it > 10
    assert rel(x, x_lu) < 1e-10
    x2, st2, it2, rr2 = oracle_mod.bicgstab(U, b, kappa, tol=1e-12)
    assert st2 == 0 and rr2 <= 1e-12
    assert rel(x2, x_lu) < 1e-10
    # D^dag solve
    x3, st3, _, _ = oracle_mod.bicgstab(U, b, kappa, tol=1e-12, dagger=True)
    assert st3 == 0
    assert rel(x3, np.linalg.solve(D.conj().T, b.ravel()).reshape(b.shape)) < 1e-10


@pytest.mark.parametrize("solver", ["cgnr", "bicgstab"])
def test_free_field_solve_matches_fft(oracle_mod, solver):
    dims = (8, 8, 8, 8)
    kappa = 0.124
    U = inputs.unit_gauge(dims)
    b = inputs.gaussian_spinor(dims, seed=3)
    x_fft = mp.free_solve_fft(b, kappa)
    x, st, it, rr = getattr(oracle_mod, solver)(U, b, kappa, tol=1e-12)
    assert st == 0
    assert rel(x, x_fft) < 1e-10


def test_fft_solver_pinned_by_dense_lu():
    dims = (2, 2, 2, 4)
    U = inputs.unit_gauge(dims)
    b = inputs.gaussian_spinor(dims, seed=1)
    D = mp.dense_wilson(U, 0.12, dims)
    assert rel(mp.free_solve_fft(b, 0.12), np.linalg.solve(D, b.ravel()).reshape(b.shape)) < 1e-12


def test_singular_free_field_is_not_solved(oracle_mod):
    """Fully periodic free field at kappa = 1/8 has an exact zero mode (p = 0)."""
    dims = (2, 2, 2, 2)
    U = inputs.unit_gauge(dims)
    ev = mp.free_spectrum(dims, 0.125, (1, 1, 1, 1))
    assert np.min(np.abs(ev)) < 1e-15
    b = np.ones(inputs.spinor_shape(dims), dtype=np.complex128)  # overlaps the zero mode
    _, st, it, rr = oracle_mod.cgnr(U, b, 0.125, bc=(1, 1, 1, 1), tol=1e-12, maxiter=200)
    assert st != 0 and rr > 1e-3


def test_zero_source_zero_solution(oracle_mod):
    dims = (2, 2, 2, 4)
    U = inputs.haar_gauge(dims)
    b = np.zeros(inputs.spinor_shape(dims), dtype=np.complex128)
    x, st, it, rr = oracle_mod.bicgstab(U, b, 0.12)
    assert st == 0 and it == 0 and not np.any(x)


# ---------------------------------------------------------------- gradient pins
def _loss_dense(U, b, kappa, dims):
    D = mp.dense_wilson(U, kappa, dims, BC)
    x = np.linalg.solve(D, b.ravel())
    return float(np.vdot(x, x).real)


def test_gradient_wrt_source_matches_central_fd(oracle_mod):
    dims = (2, 2, 2, 4)
    kappa = 0.12
    U = inputs.near_unity_gauge(dims, eps=0.3, seed=2)
    b = inputs.gaussian_spinor(dims, seed=3)
    g = oracle_mod.gradient(U, b, kappa)
    rng = np.random.default_rng(5)
    db = rng.standard_normal(b.shape) + 1j * rng.standard_normal(b.shape)
    h = 1e-5
    fd = (_loss_dense(U, b + h * db, kappa, dims) - _loss_dense(U, b - h * db, kappa, dims)) / (2 * h)
    an = float(np.real(np.vdot(g["grad_b"], db)))
    assert abs(fd - an) <= 1e-7 * abs(an) + 1e-9 * g["L"]


def test_gradient_wrt_links_matches_central_fd(oracle_mod):
    dims = (2, 2, 2, 4)
    kappa = 0.12
    U = inputs.near_unity_gauge(dims, eps=0.3, seed=2)
    b = inputs.gaussian_spinor(dims, seed=3)
    g = oracle_mod.gradient(U, b, kappa)
    lam = inputs.gell_mann() / 2
    rng = np.random.default_rng(9)
    h = 1e-5
    samples = [(3, (3, 1, 0, 1), a) for a in range(8)]  # t-boundary link (t = Lt-1)
    samples += [(int(rng.integers(4)), tuple(int(v) for v in rng.integers(0, [4, 2, 2, 2])), int(rng.integers(8)))
                for _ in range(16)]
    for mu, (t, z, y, x), a in samples:
        Up, Um = U.copy(), U.copy()
        E = inputs.exp_i_hermitian(lam[a], h)
        Up[mu, t, z, y, x] = E @ U[mu, t, z, y, x]
        Um[mu, t, z, y, x] = np.conj(E.T) @ U[mu, t, z, y, x]
        fd = (_loss_dense(Up, b, kappa, dims) - _loss_dense(Um, b, kappa, dims)) / (2 * h)
        an = float(np.real(np.trace(lam[a] @ g["P"][mu, t, z, y, x])))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)) + 1e-9 * g["L"], (mu, t, z, y, x, a, fd, an)


def test_force_matches_no_solve_fd_of_operator(oracle_mod):
    """d/dw Re<mu, D(e^{iwT}U) x> = -Tr[T P] with P from the oracle force (no solve)."""
    dims = (4, 2, 2, 4)
    kappa = 0.125
    U = inputs.haar_gauge(dims, seed=31)
    x = inputs.gaussian_spinor(dims, seed=32)
    muv = inputs.gaussian_spinor(dims, seed=33)
    P = oracle_mod.su3_project(U, oracle_mod.force(U, x, muv, kappa))
    lam = inputs.gell_mann() / 2
    h = 1e-4
    for mu, (t, z, y, xx), a in [(3, (3, 0, 1, 2), 2), (0, (0, 1, 1, 3), 7), (1, (2, 0, 0, 0), 4),
                                 (2, (1, 1, 1, 1), 0), (3, (0, 0, 0, 0), 5)]:
        E = inputs.exp_i_hermitian(lam[a], h)
        Up, Um = U.copy(), U.copy()
        Up[mu, t, z, y, xx] = E @ U[mu, t, z, y, xx]
        Um[mu, t, z, y, xx] = np.conj(E.T) @ U[mu, t, z, y, xx]
        fd = (np.vdot(muv, oracle_mod.apply(Up, x, kappa)).real - np.vdot(muv, oracle_mod.apply(Um, x, kappa)).real) / (2 * h)
        an = -np.real(np.trace(lam[a] @ P[mu, t, z, y, xx]))
        assert abs(fd - an) < 1e-7 * max(1.0, abs(an))


# ---------------------------------------------------------------- table I identities
def test_table1_cost_identities():
    """Sec. II-B, Table I: Wilson 1368 flop/site and 1536 B/site (float, no reuse)."""
    proj, su3_mv, accum, diag = 12, 132, 24, 48
    assert 8 * (proj + su3_mv) + 7 * accum + 48 == 1368
    assert 8 * (proj + su3_mv) + 7 * accum == 1320  # hopping term alone
    assert diag == 48
    spinor_f, link_f = 24 * 4, 18 * 4
    assert 8 * spinor_f + 8 * link_f + spinor_f + spinor_f == 1536
    assert round(1536 / 1368, 2) == 1.12
    # domain-wall row, N_s = 8
    assert 8 * (8 * spinor_f + spinor_f + spinor_f) + 8 * link_f == 8256
    assert round(8256 / 11520, 2) == 0.72


# ---------------------------------------------------------------- planted mistakes
# Each case compiles a copy of the oracle with one plausible slip and checks
# that the pins above catch it (the oracle source is mutated on the CPU only).
import ctypes  # noqa: E402
import os  # noqa: E402
import subprocess  # noqa: E402

_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "wilson_oracle.c")

_MUTATIONS = {
    "projector_sign": ("const double fwd_pm = dagger ? +1.0 : -1.0;", "const double fwd_pm = dagger ? -1.0 : +1.0;"),
    "boundary_sign_dropped": ("*sign = (double)bc[mu];\n    } else if", "*sign = 1.0;\n    } else if"),
    "link_not_conjugated": ("cplx m = adj ? conj(link[3 * b + a]) : link[3 * a + b];",
                            "cplx m = adj ? link[3 * b + a] : link[3 * a + b];"),
    "link_transposed": ("cplx m = adj ? conj(link[3 * b + a]) : link[3 * a + b];",
                        "cplx m = adj ? conj(link[3 * a + b]) : link[3 * b + a];"),
    "force_second_term_dropped": ("acc += mu_adj[12 * nf + 3 * sp + a] * conj(w[sp][b]);", ""),
    "dw_projectors_swapped": ("const double up = dagger ? +1.0 : -1.0, down = -up;",
                              "const double up = dagger ? -1.0 : +1.0, down = -up;"),
    "dw_diagonal_shift": ("(m0 + 5.0) * ps[12 * x + i]", "(m0 + 4.0) * ps[12 * x + i]"),
    "dw_corner_sign": ("add_chiral(os + 12 * x, psi + 12 * x, g5, up, m);",
                       "add_chiral(os + 12 * x, psi + 12 * x, g5, up, -m);"),
}


@pytest.fixture
def planted(tmp_path, oracle_mod, monkeypatch):
    def make(name):
        old, new = _MUTATIONS[name]
        src = open(_SRC).read()
        assert src.count(old) == 1, name
        path = tmp_path / f"{name}.c"
        path.write_text(src.replace(old, new))
        lib = tmp_path / f"{name}.so"
        subprocess.run(["gcc", "-std=c11", "-O1", "-fopenmp", "-fPIC", "-shared", "-o", str(lib), str(path), "-lm"],
                       check=True)
        monkeypatch.setattr(oracle_mod, "_lib", oracle_mod._configure(ctypes.CDLL(str(lib))))
        return oracle_mod
    return make


def _dense_pin_fails(o, dagger=False):
    dims = (2, 2, 2, 4)
    U = inputs.haar_gauge(dims, seed=3)
    psi = inputs.gaussian_spinor(dims, seed=5)
    ref = (mp.dense_wilson(U, 0.12, dims, BC, dagger=dagger) @ psi.ravel()).reshape(psi.shape)
    return rel(o.apply(U, psi, 0.12, BC, dagger=dagger), ref) > 1e-6


@pytest.mark.parametrize("name", ["projector_sign", "boundary_sign_dropped", "link_not_conjugated",
                                  "link_transposed"])
def test_planted_operator_mistakes_are_caught(planted, name):
    o = planted(name)
    assert _dense_pin_fails(o) or _dense_pin_fails(o, dagger=True)


def test_planted_boundary_mistake_caught_by_free_spectrum(planted):
    o = planted("boundary_sign_dropped")
    dims = (2, 2, 2, 4)
    b = inputs.gaussian_spinor(dims, seed=1)
    x, _, _, _ = o.bicgstab(inputs.unit_gauge(dims), b, 0.12, tol=1e-12)
    assert rel(x, mp.free_solve_fft(b, 0.12)) > 1e-3


def test_planted_force_mistake_caught_by_fd(planted):
    o = planted("force_second_term_dropped")
    dims = (4, 2, 2, 4)
    U = inputs.haar_gauge(dims, seed=31)
    x = inputs.gaussian_spinor(dims, seed=32)
    muv = inputs.gaussian_spinor(dims, seed=33)
    P = o.su3_project(U, o.force(U, x, muv, 0.125))
    lam = inputs.gell_mann() / 2
    h = 1e-4
    worst = 0.0
    for a in range(8):
        E = inputs.exp_i_hermitian(lam[a], h)
        Up, Um = U.copy(), U.copy()
        Up[1, 2, 0, 0, 0] = E @ U[1, 2, 0, 0, 0]
        Um[1, 2, 0, 0, 0] = np.conj(E.T) @ U[1, 2, 0, 0, 0]
        fd = (np.vdot(muv, o.apply(Up, x, 0.125)).real - np.vdot(muv, o.apply(Um, x, 0.125)).real) / (2 * h)
        worst = max(worst, abs(fd + np.real(np.trace(lam[a] @ P[1, 2, 0, 0, 0]))))
    assert worst > 1e-3


# ---------------------------------------------------------------- domain wall (eq. (2))
DW_M0, DW_M = -1.8, 0.05


def _dw_field(dims, Ns, seed):
    return np.stack([inputs.gaussian_spinor(dims, seed=seed + s) for s in range(Ns)])


@pytest.mark.parametrize("dims,Ns", [((2, 2, 2, 2), 4), ((2, 2, 2, 4), 3), ((3, 2, 2, 2), 2)])
@pytest.mark.parametrize("dagger", [False, True])
def test_dw_matches_kronecker_construction(oracle_mod, dims, Ns, dagger):
    U = inputs.haar_gauge(dims, seed=7)
    psi = _dw_field(dims, Ns, 40)
    ref = (mp.dense_dw(U, DW_M0, DW_M, Ns, dims, BC, dagger=dagger) @ psi.ravel()).reshape(psi.shape)
    assert rel(oracle_mod.dw_apply(U, psi, DW_M0, DW_M, BC, dagger=dagger), ref) < 1e-13


def test_dw_free_field_plane_waves(oracle_mod):
    """U = 1: a plane wave e^{ipx} times spin vectors v_s is mapped to e^{ipx} (M(p) v)_s."""
    dims, Ns = (4, 4, 4, 4), 5
    rng = np.random.default_rng(2)
    moms = mp.momenta(dims, BC)
    Lx, Ly, Lz, Lt = dims
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    for trial in range(3):
        p = np.array([moms[mu][rng.integers(0, dims[mu])] for mu in range(4)])
        wave = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
        v = rng.normal(size=(Ns, 4)) + 1j * rng.normal(size=(Ns, 4))
        col = rng.normal(size=3) + 1j * rng.normal(size=3)
        psi = wave[None, ..., None, None] * v[:, None, None, None, None, :, None] * col
        out = oracle_mod.dw_apply(inputs.unit_gauge(dims), psi, DW_M0, DW_M, BC)
        w = (mp.dw_symbol(p, DW_M0, DW_M, Ns) @ v.ravel()).reshape(Ns, 4)
        ref = wave[None, ..., None, None] * w[:, None, None, None, None, :, None] * col
        assert rel(out, ref) < 1e-12


def test_dw_gamma5_reflection_hermiticity(oracle_mod):
    """D_DW^dag = Gamma D_DW Gamma with Gamma = gamma_5 R_5 (R_5: s -> Ns-1-s), and <x, D y> = <D^dag x, y>."""
    dims, Ns = (4, 2, 2, 4), 6
    U = inputs.haar_gauge(dims, seed=11)
    x = _dw_field(dims, Ns, 60)
    y = _dw_field(dims, Ns, 70)
    gam = lambda f: mp.gamma5_spinor(f[::-1])
    lhs = oracle_mod.dw_apply(U, x, DW_M0, DW_M, BC, dagger=True)
    assert rel(lhs, gam(oracle_mod.dw_apply(U, gam(x), DW_M0, DW_M, BC))) < 1e-13
    a = np.vdot(x, oracle_mod.dw_apply(U, y, DW_M0, DW_M, BC))
    b = np.vdot(lhs, y)
    assert abs(a - b) < 1e-12 * abs(a)


def test_dw_cgnr_matches_dense_solve(oracle_mod):
    dims, Ns = (2, 2, 2, 4), 4
    U = inputs.haar_gauge(dims, seed=13)
    b = _dw_field(dims, Ns, 80)
    x, st, it, relres = oracle_mod.dw_cgnr(U, b, DW_M0, DW_M, BC, tol=1e-12)
    assert st == 0 and relres <= 1e-12 and it > 0
    D = mp.dense_dw(U, DW_M0, DW_M, Ns, dims, BC)
    x_lu = np.linalg.solve(D, b.ravel()).reshape(b.shape)
    assert rel(x, x_lu) < 1e-9


def test_dw_ns1_reduces_to_shifted_wilson(oracle_mod):
    """Ns = 1: both corners land on the diagonal, D_DW = D_W + 1 + m (P_+ + P_-) = D_W + 1 + m."""
    dims = (2, 2, 2, 4)
    U = inputs.haar_gauge(dims, seed=17)
    psi = _dw_field(dims, 1, 90)
    kappa = 1.0 / (2 * (DW_M0 + 1 + DW_M) + 8)  # D_W + 1 + m = (m0 + 1 + m + 4) - H/2 = D(kappa) / (2 kappa)
    ref = oracle_mod.apply(U, psi[0], kappa, BC) / (2 * kappa)
    assert rel(oracle_mod.dw_apply(U, psi, DW_M0, DW_M, BC)[0], ref) < 1e-13


@pytest.mark.parametrize("name", ["dw_projectors_swapped", "dw_diagonal_shift", "dw_corner_sign"])
def test_planted_dw_mistakes_are_caught(planted, name):
    o = planted(name)
    dims, Ns = (2, 2, 2, 2), 3
    U = inputs.haar_gauge(dims, seed=19)
    psi = _dw_field(dims, Ns, 95)
    bad = False
    for dagger in (False, True):
        ref = (mp.dense_dw(U, DW_M0, DW_M, Ns, dims, BC, dagger=dagger) @ psi.ravel()).reshape(psi.shape)
        bad = bad or rel(o.dw_apply(U, psi, DW_M0, DW_M, BC, dagger=dagger), ref) > 1e-6
    assert bad
