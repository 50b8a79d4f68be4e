"""Short fixed sequences of launches for rocprofv3 runs (kernel statistics and
hardware counters), one case per invocation:

    python -m paper_1712_01505_amd.profile_cases apply <prec> [dims]
        the tuned apply of one precision (f64, f32, bf16, f16), 3 + reps launches
    python -m paper_1712_01505_amd.profile_cases multi_rhs
        24^3 x 48 FP32: the tuned 12-right-hand-side apply and the tuned
        single-right-hand-side apply, 3 + reps launches each
    python -m paper_1712_01505_amd.profile_cases dwf <prec>
        the domain-wall apply at 32^3 x 64, Ns = 8, tuned, 3 + reps launches
    python -m paper_1712_01505_amd.profile_cases halo <prec> [dims]
        the tuned apply, then the same apply with the boundary copy enforced
    python -m paper_1712_01505_amd.profile_cases shapes dwf|multi_rhs
        a fixed list of launch shapes (tile order, columns across lanes or
        right-hand sides per brick workgroup, group order, variant), 3
        launches each, in the order printed: the
        FP32 domain-wall apply at 32^3 x 64, Ns = 8, or the 12-RHS FP32 apply
        at 24^3 x 48 (after one single-RHS apply in the tuned default shape)

reps comes from $PROFILE_REPS (default 5).  Every case autotunes first
(keeping the choices in $WL_TUNE_CACHE when it is set) unless --no-tune is
given, as it is for the profiled runs, which then launch the cached shapes
only; it prints, per timed sequence, its launch shape and the time per launch
from HIP events, so a counter run's per-dispatch figures can be matched to
the shape.  Inputs are the benchmark's synthetic fields."""
import ctypes
import json
import os
import sys

import torch

from . import inputs
from . import wilson as W

PNAME = {"f64": W.WL_F64, "f32": W.WL_F32, "bf16": W.WL_BF16S, "f16": W.WL_F16S}
TUNE = True


def _tune(handle, nrhs):
    if TUNE:
        W.wl_autotune(handle, nrhs, 0, W._stream())


def _timed(fn, reps):
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps * 1e3


def _three(fn):
    """Three launches, timed together (ms per launch, in microseconds)."""
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(3):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / 3 * 1e3


def case_apply(prec, dims, reps):
    p = PNAME[prec]
    U = torch.from_numpy(inputs.near_unity_gauge(dims, 0.3, seed=inputs.GAUGE_SEED)).cuda()
    op = W.Operator.create(U, 0.1255, p)
    del U
    _tune(op.handle, 1)
    src = op.pack(torch.from_numpy(inputs.gaussian_spinor(dims, seed=inputs.SOURCE_SEED)).cuda())
    dst = op.new_field()
    us = _timed(lambda: op.apply_packed(dst, src), reps)
    return [{"case": f"apply {prec} {dims}", "launch": W.wl_get_launch(op.handle, 1), "launches": 3 + reps,
             "us": round(us, 2), "sites": inputs.volume(dims)}]


def case_multi_rhs(reps):
    dims, n = (24, 24, 24, 48), 12
    U = torch.from_numpy(inputs.near_unity_gauge(dims, 0.3, seed=inputs.GAUGE_SEED)).cuda()
    op = W.Operator.create(U, 0.12, W.WL_F32)
    del U
    _tune(op.handle, n)
    _tune(op.handle, 1)
    src = op.pack(torch.from_numpy(inputs.gaussian_spinor(dims, seed=inputs.SOURCE_SEED, nrhs=n)).cuda())
    dst = op.new_field(n)
    s1 = op.pack(torch.from_numpy(inputs.gaussian_spinor(dims, seed=inputs.SOURCE_SEED)).cuda())
    d1 = op.new_field()
    out = []
    us = _timed(lambda: op.apply_packed(dst, src, n), reps)
    out.append({"case": f"apply f32 {dims} nrhs {n}", "launch": W.wl_get_launch(op.handle, n), "launches": 3 + reps,
                "us": round(us, 2), "sites": inputs.volume(dims), "nrhs": n})
    us = _timed(lambda: op.apply_packed(d1, s1, 1), reps)
    out.append({"case": f"apply f32 {dims} nrhs 1", "launch": W.wl_get_launch(op.handle, 1), "launches": 3 + reps,
                "us": round(us, 2), "sites": inputs.volume(dims), "nrhs": 1})
    return out


def case_dwf(prec, reps):
    dims, ns = (32, 32, 32, 64), 8
    U = torch.from_numpy(inputs.near_unity_gauge(dims, 0.3, seed=inputs.GAUGE_SEED)).cuda()
    op = W.DWOperator.create(U, -1.8, 0.1, ns, PNAME[prec])
    del U
    _tune(op.handle, 1)
    dst = op.new_field()
    inp = op.pack(torch.from_numpy(inputs.gaussian_spinor(dims, seed=inputs.SOURCE_SEED, nrhs=ns)).cuda())
    us = _timed(lambda: op.apply_packed(dst, inp), reps)
    return [{"case": f"dwf {prec} {dims} Ns {ns}", "launch": W.wl_get_launch(op.handle, 1), "launches": 3 + reps,
             "us": round(us, 2), "sites": inputs.volume(dims), "ns": ns}]


def case_halo(prec, dims, reps):
    p = PNAME[prec]
    U = torch.from_numpy(inputs.near_unity_gauge(dims, 0.3, seed=inputs.GAUGE_SEED)).cuda()
    op = W.Operator.create(U, 0.1255, p)
    del U
    _tune(op.handle, 1)
    src = op.pack(torch.from_numpy(inputs.gaussian_spinor(dims, seed=inputs.SOURCE_SEED)).cuda())
    dst = op.new_field()
    nb = ctypes.c_size_t(0)
    W.lib().wl_halo_bytes(op.handle, 1, ctypes.byref(nb))
    halo = torch.empty(nb.value, dtype=torch.uint8, device=src.device)
    plain = _timed(lambda: op.apply_packed(dst, src), reps)
    fn = lambda: W.lib().wilson_apply_halo(op.handle, dst.data_ptr(), src.data_ptr(), 0, 1, halo.data_ptr(),
                                           nb.value, W._stream())
    enforced = _timed(fn, reps)
    return [{"case": f"halo {prec} {dims}", "launch": W.wl_get_launch(op.handle, 1), "plain_us": round(plain, 2),
             "halo_us": round(enforced, 2), "fixed_us": round(enforced - plain, 2),
             "overhead": round(enforced / plain - 1.0, 4)}]


# (block, xcd_remap, variant, rhs_lanes, rhs_major, brick or None, t_steps)
SHAPES = {
    "dwf": [(256, 1, 2, 1, 0, None, 0), (256, 3, 2, 1, 0, None, 0), (256, 5, 2, 1, 0, None, 0),
            (256, 3, 2, 4, 0, None, 0), (512, 3, 2, 8, 0, None, 0), (512, 5, 2, 8, 0, None, 0),
            (256, 1, 5, 1, 0, None, 0), (256, 1, 5, 8, 0, None, 0), (128, 0, 6, 1, 0, None, 0)],
    "multi_rhs": [(256, 0, 7, 1, 0, (8, 8, 4), 4), (256, 0, 7, 1, 1, (8, 8, 4), 4), (256, 1, 2, 4, 0, None, 0),
                  (256, 2, 2, 1, 1, None, 0), (256, 2, 2, 4, 1, None, 0), (128, 1, 5, 2, 0, None, 0),
                  (128, 1, 5, 2, 1, None, 0), (256, 1, 7, 2, 1, (8, 8, 2), 16), (256, 1, 7, 4, 1, (4, 4, 4), 8),
                  (256, 1, 7, 4, 0, (4, 4, 4), 8)],
}


def case_shapes(which):
    rows = []
    if which == "dwf":
        dims, ns = (32, 32, 32, 64), 8
        U = torch.from_numpy(inputs.near_unity_gauge(dims, 0.3, seed=inputs.GAUGE_SEED)).cuda()
        op = W.DWOperator.create(U, -1.8, 0.1, ns, W.WL_F32)
        del U
        nrhs, dst = 1, op.new_field()
        src = op.pack(torch.from_numpy(inputs.gaussian_spinor(dims, seed=inputs.SOURCE_SEED, nrhs=ns)).cuda())
        V = inputs.volume(dims)
        rd, wr = (96 * ns + 192) * V, 96 * ns * V  # FP32: spinors in (all slices) + links once; out
    else:
        dims = (24, 24, 24, 48)
        U = torch.from_numpy(inputs.near_unity_gauge(dims, 0.3, seed=inputs.GAUGE_SEED)).cuda()
        op = W.Operator.create(U, 0.12, W.WL_F32)
        del U
        s1 = op.pack(torch.from_numpy(inputs.gaussian_spinor(dims, seed=inputs.SOURCE_SEED)).cuda())
        d1 = op.new_field()
        V = inputs.volume(dims)
        us = _three(lambda: op.apply_packed(d1, s1, 1))
        rows.append({"case": f"shapes multi_rhs {dims} nrhs 1", "launch": W.wl_get_launch(op.handle, 1),
                     "launches": 3, "us_first3": round(us, 1), "compulsory_read": 288 * V, "compulsory_write": 96 * V})
        nrhs = 12
        src = op.pack(torch.from_numpy(inputs.gaussian_spinor(dims, seed=inputs.SOURCE_SEED, nrhs=nrhs)).cuda())
        dst = op.new_field(nrhs)
        rd, wr = (96 * nrhs + 192) * V, 96 * nrhs * V
    for block, xcd, var, lanes, gm, brick, T in SHAPES[which]:
        if not W.try_set_launch(op.handle, nrhs, block, 1, xcd, var, lanes, brick=brick, t_steps=T, rhs_major=gm):
            raise SystemExit(f"launch shape rejected: {(block, xcd, var, lanes, gm, brick, T)}")
        us = _three(lambda: op.apply_packed(dst, src, nrhs))
        rows.append({"case": f"shapes {which} {dims}", "launch": W.wl_get_launch(op.handle, nrhs), "launches": 3,
                     "us_first3": round(us, 1), "compulsory_read": rd, "compulsory_write": wr})
    return rows


def main(argv):
    global TUNE
    reps = int(os.environ.get("PROFILE_REPS", "5"))
    if "--no-tune" in argv:
        TUNE = False
        argv = [a for a in argv if a != "--no-tune"]
    if not argv:
        raise SystemExit(__doc__)
    if argv[0] == "apply":
        dims = tuple(int(v) for v in argv[2].split(",")) if len(argv) > 2 else (32, 32, 32, 64)
        rows = case_apply(argv[1], dims, reps)
    elif argv[0] == "multi_rhs":
        rows = case_multi_rhs(reps)
    elif argv[0] == "dwf":
        rows = case_dwf(argv[1], reps)
    elif argv[0] == "shapes" and len(argv) > 1 and argv[1] in SHAPES:
        rows = case_shapes(argv[1])
    elif argv[0] == "halo":
        dims = tuple(int(v) for v in argv[2].split(",")) if len(argv) > 2 else (32, 32, 32, 64)
        rows = case_halo(argv[1], dims, reps)
    else:
        raise SystemExit(__doc__)
    for r in rows:
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
