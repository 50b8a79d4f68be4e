"""ctypes binding of libwilson.so (the gfx950 Wilson-Dirac library).

Each ``wl_*`` / ``wilson_*`` / ``solve_*`` function here has the name and the
arguments of the C entry point in include/wilson.h and only marshals them:
every step of the computation runs in the HIP library.  On top of those,
``Operator``, ``apply``, ``dslash`` and ``solve`` take canonical complex128
torch tensors on the GPU (spinor ``(..., Lt, Lz, Ly, Lx, 4, 3)``, gauge
``(4, Lt, Lz, Ly, Lx, 3, 3)``) and use torch only for device memory and the
current stream.

The library must be built (``python -m paper_1712_01505_amd.build``); there is
no fallback: a missing library raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwilson.so")

WL_OK, WL_NOT_CONVERGED, WL_BREAKDOWN, WL_STAGNATED = 0, 1, 2, 3
WL_EINVAL, WL_EALIGN, WL_EPREC, WL_EHIP, WL_ENAN, WL_EWORKSPACE = -1, -2, -3, -4, -5, -6
WL_F64, WL_F32, WL_BF16S, WL_F16S = 0, 1, 2, 3
WL_SPINOR, WL_GAUGE = 0, 1
WL_SOLVER_CGNR, WL_SOLVER_BICGSTAB = 0, 1

PREC = {"f64": WL_F64, "f32": WL_F32, "bf16": WL_BF16S, "f16": WL_F16S}
SOLVER = {"cgnr": WL_SOLVER_CGNR, "bicgstab": WL_SOLVER_BICGSTAB}

# Symbols the header declares (checked by the CPU test suite).
EXPORTS = [
    "wl_field_bytes", "wl_pack_gauge", "wl_pack_spinor", "wl_unpack_spinor", "wl_convert_spinor",
    "wl_op_create", "wl_op_destroy", "wilson_dslash", "wilson_apply", "wl_solver_workspace_bytes",
    "solve_cgnr", "solve_bicgstab", "wilson_gauge_force", "wilson_multi_apply", "wl_autotune",
    "wl_get_launch", "wl_set_launch", "wl_prof_enable", "wl_prof_reset", "wl_prof_read", "wl_prof_read_aux",
    "wl_stream_copy", "wl_strerror", "wl_last_hip_error", "wl_multi_plan_create", "wl_multi_plan_run",
    "wl_multi_plan_tune", "wl_multi_plan_get_launch", "wl_multi_plan_set_launch", "wl_multi_plan_destroy",
    "wl_dw_op_create", "dwf_apply", "wl_halo_bytes", "wilson_apply_halo", "wl_eo_split", "wl_eo_merge",
    "wilson_schur_apply", "wl_apply_dot_workspace_bytes", "wilson_apply_dot", "wilson_apply_dot_noalloc",
    "wl_multi_solver_workspace_bytes", "wilson_solve_multi",
]


class wl_geom(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 4), ("bc", ctypes.c_int32 * 4)]


class wl_solve_params(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("max_outer", ctypes.c_int), ("reliable", ctypes.c_int), ("check_every", ctypes.c_int),
                ("use_x0", ctypes.c_int), ("dagger", ctypes.c_int), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t), ("eo", ctypes.c_int), ("form", ctypes.c_int)]


class wl_solve_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer", ctypes.c_int), ("stencil_calls", ctypes.c_int),
                ("converged", ctypes.c_int), ("iter_rel_res", ctypes.c_double), ("true_rel_res", ctypes.c_double),
                ("seconds", ctypes.c_double), ("kernels", ctypes.c_int), ("finalizes", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class wl_launch(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int), ("rhs_per_thread", ctypes.c_int), ("rhs_lanes", ctypes.c_int),
                ("xcd_remap", ctypes.c_int), ("variant", ctypes.c_int), ("brick", ctypes.c_int * 3),
                ("t_steps", ctypes.c_int), ("wg_per_cu", ctypes.c_int), ("rhs_major", ctypes.c_int)]


class wl_multi_desc(ctypes.Structure):
    _fields_ = [("op", ctypes.c_void_p), ("out", ctypes.c_void_p), ("in_", ctypes.c_void_p)]


class wl_multi_system(ctypes.Structure):
    _fields_ = [("hi", ctypes.c_void_p), ("lo", ctypes.c_void_p), ("x", ctypes.c_void_p), ("b", ctypes.c_void_p)]


class WilsonError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = lib().wl_strerror(code).decode()
        if code == WL_EHIP:
            msg += f" (hipError {lib().wl_last_hip_error()})"
        super().__init__(f"{where}: {msg} [{code}]")


_lib = None


def lib():
    """Load libwilson.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libwilson.so not found at {LIB_PATH}: build it with "
                           "`python -m paper_1712_01505_amd.build` (there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    P, I, D, SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    G = ctypes.POINTER(wl_geom)
    sig = {
        "wl_field_bytes": [G, I, I, I, ctypes.POINTER(SZ)],
        "wl_pack_gauge": [G, I, P, P, P],
        "wl_pack_spinor": [G, I, I, P, P, P],
        "wl_unpack_spinor": [G, I, I, P, P, P],
        "wl_convert_spinor": [G, I, I, I, P, P, P],
        "wl_op_create": [G, D, I, P, ctypes.POINTER(P)],
        "wl_op_destroy": [P],
        "wl_dw_op_create": [G, D, D, I, I, P, ctypes.POINTER(P)],
        "dwf_apply": [P, P, P, I, I, P],
        "wl_halo_bytes": [P, I, ctypes.POINTER(SZ)],
        "wl_eo_split": [G, I, I, P, P, P, P],
        "wl_eo_merge": [G, I, I, P, P, P, P],
        "wilson_schur_apply": [P, P, P, P, I, I, P],
        "wilson_apply_halo": [P, P, P, I, I, P, SZ, P],
        "wilson_dslash": [P, P, P, I, I, P],
        "wilson_apply": [P, P, P, I, I, P],
        "wl_solver_workspace_bytes": [P, P, I, I, ctypes.POINTER(SZ)],
        "solve_cgnr": [P, P, P, P, I, ctypes.POINTER(wl_solve_params), ctypes.POINTER(wl_solve_stats), P],
        "solve_bicgstab": [P, P, P, P, I, ctypes.POINTER(wl_solve_params), ctypes.POINTER(wl_solve_stats), P],
        "wilson_gauge_force": [P, P, P, P, I, P],
        "wilson_multi_apply": [ctypes.POINTER(wl_multi_desc), I, I, I, P],
        "wl_autotune": [P, I, I, P],
        "wl_get_launch": [P, I, ctypes.POINTER(wl_launch)],
        "wl_set_launch": [P, I, ctypes.POINTER(wl_launch)],
        "wl_prof_enable": [I],
        "wl_prof_reset": [],
        "wl_prof_read": [I, ctypes.POINTER(ctypes.c_long), ctypes.POINTER(D), ctypes.POINTER(D)],
        "wl_prof_read_aux": [I, ctypes.POINTER(D)],
        "wl_stream_copy": [P, P, SZ, P],
        "wl_strerror": [I],
        "wl_last_hip_error": [],
        "wl_multi_plan_create": [ctypes.POINTER(wl_multi_desc), I, I, I, ctypes.POINTER(P)],
        "wl_multi_plan_run": [P, P],
        "wl_multi_plan_tune": [P, P],
        "wl_multi_plan_get_launch": [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I),
                                     ctypes.POINTER(I)],
        "wl_multi_plan_set_launch": [P, I, I, I, I],
        "wl_multi_plan_destroy": [P],
        "wl_apply_dot_workspace_bytes": [P, I, ctypes.POINTER(SZ)],
        "wilson_apply_dot": [P, P, P, P, I, I, I, P, P, SZ, P],
        "wilson_apply_dot_noalloc": [P, P, P, P, I, I, I, P, P],
        "wl_multi_solver_workspace_bytes": [ctypes.POINTER(wl_multi_system), I, I, I, ctypes.POINTER(SZ)],
        "wilson_solve_multi": [ctypes.POINTER(wl_multi_system), I, I, I, ctypes.POINTER(wl_solve_params),
                               ctypes.POINTER(wl_solve_stats), P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_char_p if name == "wl_strerror" else I
    _lib = L
    return L


def _check(code, where, allow_positive=False):
    if code < 0 or (code > 0 and not allow_positive):
        raise WilsonError(code, where)
    return code


# ---------------------------------------------------------------- thin C-ABI mirrors
def make_geom(dims, bc=(1, 1, 1, -1)) -> wl_geom:
    g = wl_geom()
    for i in range(4):
        g.dims[i] = int(dims[i])
        g.bc[i] = int(bc[i])
    return g


def wl_field_bytes(geom, kind, prec, nrhs=1) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().wl_field_bytes(ctypes.byref(geom), kind, prec, nrhs, ctypes.byref(out)), "wl_field_bytes")
    return out.value


def wl_pack_gauge(geom, prec, U_canon, U_packed, stream):
    return _check(lib().wl_pack_gauge(ctypes.byref(geom), prec, U_canon, U_packed, stream), "wl_pack_gauge")


def wl_pack_spinor(geom, prec, nrhs, psi_canon, psi_packed, stream):
    return _check(lib().wl_pack_spinor(ctypes.byref(geom), prec, nrhs, psi_canon, psi_packed, stream),
                  "wl_pack_spinor")


def wl_unpack_spinor(geom, prec, nrhs, psi_packed, psi_canon, stream):
    return _check(lib().wl_unpack_spinor(ctypes.byref(geom), prec, nrhs, psi_packed, psi_canon, stream),
                  "wl_unpack_spinor")


def wl_convert_spinor(geom, prec_in, prec_out, nrhs, src, dst, stream):
    return _check(lib().wl_convert_spinor(ctypes.byref(geom), prec_in, prec_out, nrhs, src, dst, stream),
                  "wl_convert_spinor")


def wl_op_create(geom, kappa, prec, U_packed) -> int:
    h = ctypes.c_void_p(0)
    _check(lib().wl_op_create(ctypes.byref(geom), float(kappa), prec, U_packed, ctypes.byref(h)), "wl_op_create")
    return h.value


def wl_op_destroy(op):
    return _check(lib().wl_op_destroy(op), "wl_op_destroy")


def wilson_dslash(op, out, inp, dagger, nrhs, stream):
    return _check(lib().wilson_dslash(op, out, inp, int(dagger), nrhs, stream), "wilson_dslash")


def wilson_apply(op, out, inp, dagger, nrhs, stream):
    return _check(lib().wilson_apply(op, out, inp, int(dagger), nrhs, stream), "wilson_apply")


def wl_solver_workspace_bytes(hi, lo, solver, nrhs) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().wl_solver_workspace_bytes(hi, lo, solver, nrhs, ctypes.byref(out)), "wl_solver_workspace_bytes")
    return out.value


def solve_cgnr(hi, lo, x, b, nrhs, params, stats, stream):
    return _check(lib().solve_cgnr(hi, lo, x, b, nrhs, ctypes.byref(params), stats, stream), "solve_cgnr",
                  allow_positive=True)


def solve_bicgstab(hi, lo, x, b, nrhs, params, stats, stream):
    return _check(lib().solve_bicgstab(hi, lo, x, b, nrhs, ctypes.byref(params), stats, stream), "solve_bicgstab",
                  allow_positive=True)


def wilson_gauge_force(op, out_canon, x, mu, project, stream):
    return _check(lib().wilson_gauge_force(op, out_canon, x, mu, int(project), stream), "wilson_gauge_force")


def gauge_force(op, x_packed, mu_packed, project=2):
    """Link derivative from packed x and adjoint mu (op precision FP64/FP32):
    project 0 -> G^dag, 1 -> P (su(3) force), 2 -> i P U; canonical complex128 (4, Lt, Lz, Ly, Lx, 3, 3)."""
    torch = _torch()
    Lx, Ly, Lz, Lt = op.dims
    out = torch.empty((4, Lt, Lz, Ly, Lx, 3, 3), dtype=torch.complex128, device=op.U_packed.device)
    wilson_gauge_force(op.handle, _ptr(out), _ptr(x_packed), _ptr(mu_packed), project, _stream())
    return out


def wilson_multi_apply(descs, dagger, nrhs, stream):
    arr = (wl_multi_desc * len(descs))(*[wl_multi_desc(o, out, inp) for o, out, inp in descs])
    return _check(lib().wilson_multi_apply(arr, len(descs), int(dagger), nrhs, stream), "wilson_multi_apply")


class MultiPlan:
    """Several lattices in one persistent launch (wl_multi_plan_*): descs is
    a list of (op handle, out pointer, in pointer); the buffers must outlive
    the plan."""

    def __init__(self, descs, dagger, nrhs):
        arr = (wl_multi_desc * len(descs))(*[wl_multi_desc(o, out, inp) for o, out, inp in descs])
        h = ctypes.c_void_p()
        _check(lib().wl_multi_plan_create(arr, len(descs), int(dagger), int(nrhs), ctypes.byref(h)),
               "wl_multi_plan_create")
        self.handle = h.value

    def run(self, stream=None):
        _check(lib().wl_multi_plan_run(self.handle, _stream() if stream is None else stream), "wl_multi_plan_run")

    def tune(self, stream=None):
        _check(lib().wl_multi_plan_tune(self.handle, _stream() if stream is None else stream), "wl_multi_plan_tune")

    def launch(self):
        """(block, rhs_per_thread, variant, persistent, grid)."""
        v = [ctypes.c_int() for _ in range(5)]
        _check(lib().wl_multi_plan_get_launch(self.handle, *[ctypes.byref(x) for x in v]), "wl_multi_plan_get_launch")
        return tuple(x.value for x in v)

    def set_launch(self, block, rpt, variant, persistent=1):
        """Force a launch shape; returns False if the library rejects it."""
        return lib().wl_multi_plan_set_launch(self.handle, block, rpt, variant, int(persistent)) == WL_OK

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.wl_multi_plan_destroy(self.handle)
            self.handle = None


def wl_autotune(op, nrhs, dagger, stream):
    return _check(lib().wl_autotune(op, nrhs, int(dagger), stream), "wl_autotune")


def wl_get_launch(op, nrhs):
    """(block, rhs_per_thread, xcd_remap, variant, rhs_lanes, brick_x, brick_y, brick_z, t_steps,
    wg_per_cu, rhs_major) used for nrhs right-hand sides (the brick fields are 0 unless variant
    is 7)."""
    c = wl_launch()
    _check(lib().wl_get_launch(op, nrhs, ctypes.byref(c)), "wl_get_launch")
    return (c.block, c.rhs_per_thread, c.xcd_remap, c.variant, c.rhs_lanes, c.brick[0], c.brick[1], c.brick[2],
            c.t_steps, c.wg_per_cu, c.rhs_major)


def _launch(block, rpt, xcd, variant, lanes, brick, t_steps, wg_per_cu=0, rhs_major=0):
    c = wl_launch(block=block, rhs_per_thread=rpt, rhs_lanes=lanes, xcd_remap=xcd, variant=variant)
    if brick is not None:
        c.brick[0], c.brick[1], c.brick[2] = (int(b) for b in brick)
        c.t_steps = int(t_steps)
    c.wg_per_cu = int(wg_per_cu)
    c.rhs_major = int(rhs_major)
    return c


def wl_set_launch(op, nrhs, block, rpt, xcd, variant=0, lanes=1, brick=None, t_steps=0, wg_per_cu=0, rhs_major=0):
    c = _launch(block, rpt, xcd, variant, lanes, brick, t_steps, wg_per_cu, rhs_major)
    return _check(lib().wl_set_launch(op, nrhs, ctypes.byref(c)), "wl_set_launch")


# Stencil code variants per precision (see wl_set_launch in the header):
# 0 straight-line, 1-3 pipelined hops, 4-6 t-walk with columns of 4, 8, 16,
# 7 LDS-staged brick walk (needs a brick shape and a walk length).
VARIANTS = {WL_F64: (0, 1, 4, 5, 6), WL_F32: (0, 1, 2, 4, 5, 6), WL_BF16S: (0, 1, 2, 3, 4, 5, 6),
            WL_F16S: (0, 1, 2, 3, 4, 5, 6)}
VAR_BRICK = 7
MAX_VARIANT = {k: VAR_BRICK for k in VARIANTS}


def try_set_launch(op, nrhs, block, rpt, xcd, variant=0, lanes=1, brick=None, t_steps=0, wg_per_cu=0,
                   rhs_major=0):
    """wl_set_launch that returns False (instead of raising) for a configuration
    the library rejects."""
    c = _launch(block, rpt, xcd, variant, lanes, brick, t_steps, wg_per_cu, rhs_major)
    return lib().wl_set_launch(op, nrhs, ctypes.byref(c)) == WL_OK
MAX_RPT = {WL_F64: 2, WL_F32: 4, WL_BF16S: 4, WL_F16S: 4}


WL_DOT_BICG, WL_DOT_V, WL_DOT_NORM = 0, 1, 2
DOT_NVAL = {WL_DOT_BICG: 8, WL_DOT_V: 2, WL_DOT_NORM: 1}


def wl_apply_dot_workspace_bytes(op, nrhs) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().wl_apply_dot_workspace_bytes(op, nrhs, ctypes.byref(out)), "wl_apply_dot_workspace_bytes")
    return out.value


def wilson_apply_dot(op, out, inp, v, dagger, nrhs, kind, dots, workspace, workspace_bytes, stream):
    return _check(lib().wilson_apply_dot(op, out, inp, v, int(dagger), nrhs, kind, dots, workspace,
                                         workspace_bytes, stream), "wilson_apply_dot")


def apply_dot(op, out_packed, in_packed, v_packed=None, dagger=False, nrhs=1, kind=WL_DOT_BICG):
    """out = D in (packed, op precision) with the fused inner products of
    `kind`; returns a float64 CUDA tensor of shape (nval, nrhs)."""
    torch = _torch()
    dev = in_packed.device
    nb = wl_apply_dot_workspace_bytes(op.handle, nrhs)
    work = torch.empty(nb, dtype=torch.uint8, device=dev)
    dots = torch.empty((DOT_NVAL[kind], nrhs), dtype=torch.float64, device=dev)
    wilson_apply_dot(op.handle, _ptr(out_packed), _ptr(in_packed), _ptr(v_packed) if v_packed is not None else None,
                     dagger, nrhs, kind, _ptr(dots), _ptr(work), nb, _stream())
    return dots


def wl_stream_copy(dst, src, nbytes, stream):
    return _check(lib().wl_stream_copy(dst, src, nbytes, stream), "wl_stream_copy")


def wl_prof_enable(on):
    return _check(lib().wl_prof_enable(int(on)), "wl_prof_enable")


def wl_prof_reset():
    return _check(lib().wl_prof_reset(), "wl_prof_reset")


def wl_prof_read(prec):
    n, ms, sites = ctypes.c_long(), ctypes.c_double(), ctypes.c_double()
    _check(lib().wl_prof_read(prec, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(sites)), "wl_prof_read")
    return n.value, ms.value, sites.value


def wl_prof_read_aux(prec):
    aux = ctypes.c_double()
    _check(lib().wl_prof_read_aux(prec, ctypes.byref(aux)), "wl_prof_read_aux")
    return aux.value


# ---------------------------------------------------------------- torch conveniences
def _torch():
    import torch  # noqa: WPS433
    return torch


def _stream():
    return _torch().cuda.current_stream().cuda_stream


def _ptr(t) -> int:
    return t.data_ptr()


def dims_of_spinor(psi):
    Lt, Lz, Ly, Lx = psi.shape[-6:-2]
    return (Lx, Ly, Lz, Lt)


def _nrhs_of(psi):
    return 1 if psi.dim() == 6 else int(psi.shape[0])


def alloc_field(geom, kind, prec, nrhs=1, device="cuda"):
    torch = _torch()
    n = wl_field_bytes(geom, kind, prec, nrhs)
    return torch.empty(max(n, 16), dtype=torch.uint8, device=device)


def pack_spinor(psi, prec=WL_F64, bc=(1, 1, 1, -1)):
    """Canonical complex128 spinor(s) on the GPU -> packed uint8 tensor."""
    torch = _torch()
    if psi.dtype != torch.complex128 or not psi.is_cuda:
        raise TypeError("pack_spinor expects a complex128 CUDA tensor")
    psi = psi.contiguous()
    geom = make_geom(dims_of_spinor(psi), bc)
    nrhs = _nrhs_of(psi)
    out = alloc_field(geom, WL_SPINOR, prec, nrhs, psi.device)
    wl_pack_spinor(geom, prec, nrhs, _ptr(psi), _ptr(out), _stream())
    return out


def unpack_spinor(packed, dims, prec=WL_F64, nrhs=None, bc=(1, 1, 1, -1)):
    torch = _torch()
    geom = make_geom(dims, bc)
    Lx, Ly, Lz, Lt = dims
    shape = (Lt, Lz, Ly, Lx, 4, 3) if nrhs is None else (nrhs, Lt, Lz, Ly, Lx, 4, 3)
    out = torch.empty(shape, dtype=torch.complex128, device=packed.device)
    wl_unpack_spinor(geom, prec, 1 if nrhs is None else nrhs, _ptr(packed), _ptr(out), _stream())
    return out


@dataclass
class Operator:
    """D = 1 - kappa H on packed links of one precision (owns the packed links)."""

    dims: tuple
    kappa: float
    prec: int
    bc: tuple
    U_packed: object
    handle: int

    @classmethod
    def create(cls, U, kappa, prec=WL_F64, bc=(1, 1, 1, -1)):
        torch = _torch()
        if U.dtype != torch.complex128 or not U.is_cuda:
            raise TypeError("Operator.create expects a complex128 CUDA gauge tensor")
        U = U.contiguous()
        Lt, Lz, Ly, Lx = U.shape[1:5]
        dims = (Lx, Ly, Lz, Lt)
        geom = make_geom(dims, bc)
        Up = alloc_field(geom, WL_GAUGE, prec, 1, U.device)
        wl_pack_gauge(geom, prec, _ptr(U), _ptr(Up), _stream())
        h = wl_op_create(geom, kappa, prec, _ptr(Up))
        return cls(dims, float(kappa), prec, tuple(bc), Up, h)

    @property
    def geom(self):
        return make_geom(self.dims, self.bc)

    def close(self):
        if self.handle:
            wl_op_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 -- interpreter shutdown
            pass

    def pack(self, psi):
        return pack_spinor(psi, self.prec, self.bc)

    def unpack(self, packed, nrhs=None):
        return unpack_spinor(packed, self.dims, self.prec, nrhs, self.bc)

    def new_field(self, nrhs=1):
        return alloc_field(self.geom, WL_SPINOR, self.prec, nrhs, self.U_packed.device)

    def apply_packed(self, out, inp, nrhs=1, dagger=False):
        wilson_apply(self.handle, _ptr(out), _ptr(inp), dagger, nrhs, _stream())

    def dslash_packed(self, out, inp, nrhs=1, dagger=False):
        wilson_dslash(self.handle, _ptr(out), _ptr(inp), dagger, nrhs, _stream())

    def new_half(self, nrhs=1):
        """A packed half field (the V/2 sites of one parity)."""
        n = wl_field_bytes(self.geom, WL_SPINOR, self.prec, nrhs) // 2
        return _torch().empty(max(n, 16), dtype=_torch().uint8, device=self.U_packed.device)

    def eo_split(self, packed, nrhs=1):
        even, odd = self.new_half(nrhs), self.new_half(nrhs)
        g = self.geom
        _check(lib().wl_eo_split(ctypes.byref(g), self.prec, int(nrhs), _ptr(packed), _ptr(even), _ptr(odd),
                                 _stream()), "wl_eo_split")
        return even, odd

    def eo_merge(self, even, odd, nrhs=1):
        out = self.new_field(nrhs)
        g = self.geom
        _check(lib().wl_eo_merge(ctypes.byref(g), self.prec, int(nrhs), _ptr(even), _ptr(odd), _ptr(out),
                                 _stream()), "wl_eo_merge")
        return out

    def schur_packed(self, out_e, in_e, tmp_o, nrhs=1, dagger=False):
        """out_e = (1 - kappa^2 H_eo H_oe) in_e on packed even half fields."""
        _check(lib().wilson_schur_apply(self.handle, _ptr(out_e), _ptr(in_e), _ptr(tmp_o), int(bool(dagger)),
                                        int(nrhs), _stream()), "wilson_schur_apply")

    def halo_buffer(self, nrhs=1):
        n = ctypes.c_size_t(0)
        _check(lib().wl_halo_bytes(self.handle, int(nrhs), ctypes.byref(n)), "wl_halo_bytes")
        return _torch().empty(max(n.value, 16), dtype=_torch().uint8, device=self.U_packed.device)

    def apply_halo_packed(self, out, inp, halo, nrhs=1, dagger=False):
        """D in through the enforced-halo path (face pack, copy, interior, finish)."""
        _check(lib().wilson_apply_halo(self.handle, _ptr(out), _ptr(inp), int(bool(dagger)), int(nrhs), _ptr(halo),
                                       halo.numel(), _stream()), "wilson_apply_halo")


@dataclass
class DWOperator:
    """Domain-wall D_DW (eq. (2)) with Ns slices on packed links of one
    precision (owns the packed links).  5-d fields are canonical complex128
    tensors of shape (Ns, Lt, Lz, Ly, Lx, 4, 3), or (nvec, Ns, ...) for several."""

    dims: tuple
    m0: float
    m: float
    ns: int
    prec: int
    bc: tuple
    U_packed: object
    handle: int

    @classmethod
    def create(cls, U, m0, m, Ns, prec=WL_F64, bc=(1, 1, 1, -1)):
        torch = _torch()
        if U.dtype != torch.complex128 or not U.is_cuda:
            raise TypeError("DWOperator.create expects a complex128 CUDA gauge tensor")
        U = U.contiguous()
        Lt, Lz, Ly, Lx = U.shape[1:5]
        dims = (Lx, Ly, Lz, Lt)
        geom = make_geom(dims, bc)
        Up = alloc_field(geom, WL_GAUGE, prec, 1, U.device)
        wl_pack_gauge(geom, prec, _ptr(U), _ptr(Up), _stream())
        h = ctypes.c_void_p()
        _check(lib().wl_dw_op_create(ctypes.byref(geom), float(m0), float(m), int(Ns), prec, _ptr(Up),
                                     ctypes.byref(h)), "wl_dw_op_create")
        return cls(dims, float(m0), float(m), int(Ns), prec, tuple(bc), Up, h.value)

    @property
    def geom(self):
        return make_geom(self.dims, self.bc)

    def close(self):
        if self.handle:
            wl_op_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 -- interpreter shutdown
            pass

    def _nvec(self, psi):
        if psi.dim() == 7:
            return None
        if psi.dim() == 8:
            return int(psi.shape[0])
        raise ValueError("a 5-d field has shape (Ns, Lt, Lz, Ly, Lx, 4, 3) or (nvec, Ns, ...)")

    def pack(self, psi):
        if int(psi.shape[-7]) != self.ns:
            raise ValueError(f"expected Ns = {self.ns} slices")
        return pack_spinor(psi.reshape((-1,) + tuple(psi.shape[-6:])), self.prec, self.bc)

    def unpack(self, packed, nvec=None):
        x = unpack_spinor(packed, self.dims, self.prec, (nvec or 1) * self.ns, self.bc)
        lead = (nvec, self.ns) if nvec else (self.ns,)
        return x.reshape(lead + tuple(x.shape[1:]))

    def new_field(self, nvec=1):
        return alloc_field(self.geom, WL_SPINOR, self.prec, nvec * self.ns, self.U_packed.device)

    def apply_packed(self, out, inp, nvec=1, dagger=False):
        _check(lib().dwf_apply(self.handle, _ptr(out), _ptr(inp), int(bool(dagger)), int(nvec), _stream()),
               "dwf_apply")


def dw_apply(U, psi, m0, m, dagger=False, prec="f64", bc=(1, 1, 1, -1), op=None):
    """D_DW psi (or D_DW^dag psi) for a canonical 5-d complex128 CUDA tensor."""
    p = PREC[prec] if isinstance(prec, str) else prec
    ns = int(psi.shape[-7])
    op = op or DWOperator.create(U, m0, m, ns, p, bc)
    nvec = op._nvec(psi)
    src = op.pack(psi)
    dst = op.new_field(nvec or 1)
    op.apply_packed(dst, src, nvec or 1, dagger)
    return op.unpack(dst, nvec)


def dw_solve(U, b, m0, m, precision="f64", tol=1e-10, maxiter=20000, bc=(1, 1, 1, -1), inner_tol=0.0,
             check_every=0, x0=None, ops=None, return_stats=False, reliable=False, form=0):
    """x = D_DW^{-1} b by CG on D_DW^dag D_DW (Sec. II-C, Sec. VI-B) for a canonical 5-d
    complex128 CUDA tensor b (Ns, ...) or (nvec, Ns, ...).

    precision: "f64", "f32", or "mixed-f32" / "mixed-bf16" / "mixed-f16" (FP64
    refinement around an inner CG with that storage; reliable: reliable
    updates instead of restarts).  ops: optional (hi, lo) DWOperators to reuse."""
    torch = _torch()
    ns = int(b.shape[-7])
    if ops is not None:
        hi, lo = ops
    elif precision.startswith("mixed-"):
        hi = DWOperator.create(U, m0, m, ns, WL_F64, bc)
        lo = DWOperator.create(U, m0, m, ns, PREC[precision.split("-", 1)[1]], bc)
    else:
        hi = DWOperator.create(U, m0, m, ns, PREC[precision], bc)
        lo = None
    nvec = hi._nvec(b)
    n = nvec or 1
    bp = hi.pack(b)
    xp = hi.pack(x0) if x0 is not None else hi.new_field(n)
    prm = wl_solve_params(tol=tol, maxiter=maxiter, inner_tol=inner_tol, max_outer=0, reliable=int(reliable),
                          check_every=check_every, use_x0=1 if x0 is not None else 0, dagger=0,
                          workspace=None, workspace_bytes=0, form=int(form))
    ws = wl_solver_workspace_bytes(hi.handle, lo.handle if lo else None, WL_SOLVER_CGNR, n)
    work = torch.empty(ws, dtype=torch.uint8, device=b.device)
    prm.workspace = work.data_ptr()
    prm.workspace_bytes = ws
    stats = (wl_solve_stats * n)()
    code = solve_cgnr(hi.handle, lo.handle if lo else None, _ptr(xp), _ptr(bp), n, prm, stats, _stream())
    x = hi.unpack(xp, nvec)
    st = [s_.as_dict() for s_ in stats]
    for s_ in st:
        s_["status"] = code
    if return_stats:
        return x, (st[0] if nvec is None else st)
    return x


def apply(U, psi, kappa, dagger=False, prec="f64", bc=(1, 1, 1, -1), op=None):
    """D psi (or D^dag psi) for canonical complex128 CUDA tensors."""
    p = PREC[prec] if isinstance(prec, str) else prec
    op = op or Operator.create(U, kappa, p, bc)
    nrhs = None if psi.dim() == 6 else int(psi.shape[0])
    src = op.pack(psi)
    dst = op.new_field(nrhs or 1)
    op.apply_packed(dst, src, nrhs or 1, dagger)
    return op.unpack(dst, nrhs)


def dslash(U, psi, dagger=False, prec="f64", bc=(1, 1, 1, -1), op=None):
    """H psi (the hopping term) for canonical complex128 CUDA tensors."""
    p = PREC[prec] if isinstance(prec, str) else prec
    op = op or Operator.create(U, 0.0, p, bc)
    nrhs = None if psi.dim() == 6 else int(psi.shape[0])
    src = op.pack(psi)
    dst = op.new_field(nrhs or 1)
    op.dslash_packed(dst, src, nrhs or 1, dagger)
    return op.unpack(dst, nrhs)


def solve(U, b, kappa, method="bicgstab", precision="f64", tol=1e-10, maxiter=10000, bc=(1, 1, 1, -1),
          inner_tol=0.0, check_every=0, x0=None, ops=None, return_stats=False, dagger=False, reliable=False,
          eo=False, form=0):
    """x = D^{-1} b (dagger: x = D^{-dag} b) for canonical complex128 CUDA tensors.

    precision: "f64" (plain FP64), "f32" (plain FP32), or "mixed-f32", "mixed-bf16",
    "mixed-f16" (FP64 refinement around an inner solve with that storage).
    ops: optional (hi, lo) Operators to reuse (lo None for a plain solve).
    eo: even-odd preconditioning (Schur complement on the even sites).
    form: 0 merged two-phase iterations, 1 one reduction phase per iteration."""
    torch = _torch()
    nrhs = None if b.dim() == 6 else int(b.shape[0])
    n = nrhs or 1
    if ops is not None:
        hi, lo = ops
    elif precision.startswith("mixed-"):
        lo_prec = PREC[precision.split("-", 1)[1]]
        hi = Operator.create(U, kappa, WL_F64, bc)
        lo = Operator.create(U, kappa, lo_prec, bc)
    else:
        hi = Operator.create(U, kappa, PREC[precision], bc)
        lo = None
    bp = hi.pack(b)
    xp = hi.pack(x0) if x0 is not None else hi.new_field(n)
    prm = wl_solve_params(tol=tol, maxiter=maxiter, inner_tol=inner_tol, max_outer=0, reliable=int(reliable),
                          check_every=check_every, use_x0=1 if x0 is not None else 0, dagger=int(dagger),
                          workspace=None, workspace_bytes=0, eo=int(eo), form=int(form))
    ws = wl_solver_workspace_bytes(hi.handle, lo.handle if lo else None, SOLVER[method], n)
    work = torch.empty(ws, dtype=torch.uint8, device=b.device)
    prm.workspace = work.data_ptr()
    prm.workspace_bytes = ws
    stats = (wl_solve_stats * n)()
    fn = solve_cgnr if method == "cgnr" else solve_bicgstab
    code = fn(hi.handle, lo.handle if lo else None, _ptr(xp), _ptr(bp), n, prm, stats, _stream())
    x = hi.unpack(xp, nrhs)
    st = [s.as_dict() for s in stats]
    for s in st:
        s["status"] = code
    if return_stats:
        return x, (st[0] if nrhs is None else st)
    return x


def solve_multi(systems, nrhs=1, method="bicgstab", tol=1e-10, maxiter=10000, inner_tol=0.0, reliable=False,
                form=0, return_stats=False):
    """Several lattices solved together (wilson_solve_multi).  systems: list
    of (hi Operator, lo Operator or None, b packed in hi's precision with nrhs
    columns); returns the packed solutions (and the per-column stats, column
    i * nrhs + r)."""
    torch = _torch()
    n = len(systems)
    xs = [hi.new_field(nrhs) for hi, _, _ in systems]
    arr = (wl_multi_system * n)(*[wl_multi_system(hi.handle, lo.handle if lo is not None else None, _ptr(x), _ptr(b))
                                  for (hi, lo, b), x in zip(systems, xs)])
    ws = ctypes.c_size_t(0)
    _check(lib().wl_multi_solver_workspace_bytes(arr, n, SOLVER[method], nrhs, ctypes.byref(ws)),
           "wl_multi_solver_workspace_bytes")
    work = torch.empty(ws.value, dtype=torch.uint8, device=systems[0][2].device)
    prm = wl_solve_params(tol=tol, maxiter=maxiter, inner_tol=inner_tol, max_outer=0, reliable=int(reliable),
                          check_every=0, use_x0=0, dagger=0, workspace=work.data_ptr(), workspace_bytes=ws.value,
                          eo=0, form=int(form))
    stats = (wl_solve_stats * (n * nrhs))()
    code = lib().wilson_solve_multi(arr, n, SOLVER[method], nrhs, ctypes.byref(prm), stats, _stream())
    _check(code, "wilson_solve_multi", allow_positive=True)
    st = [s_.as_dict() for s_ in stats]
    for s_ in st:
        s_["status"] = code
    return (xs, st) if return_stats else xs
