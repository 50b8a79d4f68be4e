#!/usr/bin/env python3
"""Benchmark: Wilson-Dirac stencil throughput and mixed vs FP64 solve time.

Workload (one GPU): 32^3 x 64 lattice, near-unity links U = exp(i 0.3 H)
(gauge seed 1), kappa = 0.1255, antiperiodic in t, complex Gaussian source
(seed 0); the paper's strong-scaling lattice.  All inputs are synthetic and
resident in HBM before the timed region starts.

One step = one mixed-precision solve of D x = b to a true relative residual
of 1e-10 (BiCGStab inner solve with FP16 storage + per-site scale and FP32
arithmetic, inside FP64 true-residual refinement).  `value` is the sustained
stencil rate over the step: stencil applications x 1368 flop/site (paper
Table I) x V / step time.  Outside the timed region the script also measures
each stencil precision on its own (GFLOP/s and GB/s on compulsory bytes), the
plain FP64 BiCGStab and CGNR solves, the other inner precisions, checks the
step's solution with the FP64 CPU oracle, and times the oracle on the host.

Every solve reports, beside the library's own FP64 residual, the true
residual recomputed by the FP64 CPU oracle and the forward error against the
oracle's solution x* (BiCGStab to 1e-12 from x = 0).  Further sections: the
paper's single-node lattice 16^3 x 32 (apply with one and with four rotated
buffer sets, FP64 BiCGStab and CGNR, the oracle's solvers timed on the host),
24^3 x 48 with 12 point sources (multi-RHS stencil, batched solve with every
column's oracle residual), multi-lattice plans, the differentiable solve, the
domain-wall operator and the enforced halo.  The CPU baseline is the oracle's
D on the benchmark lattice with all host threads and with one, with the CPU
model.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
Prints one JSON line on stdout (progress goes to stderr).
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FLOP_APPLY = 1368
# compulsory bytes per site per right-hand side (spinor in + 4 two-row links + spinor out)
BYTES = {0: 192 + 4 * 96 + 192, 1: 96 + 4 * 48 + 96, 2: 52 + 4 * 24 + 52, 3: 52 + 4 * 24 + 52}
# one spinor field per site (a fused reduction <rh, .> reads rh on top of BYTES)
SPINOR = {0: 192, 1: 96, 2: 52, 3: 52}
PNAME = {0: "f64", 1: "f32", 2: "bf16", 3: "f16"}
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(prec, dims):
    """HBM bytes per launch of the stencil of `prec`, from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary (scaled by the copy
    calibration), or None if there is none or the kernel sources changed."""
    from paper_1712_01505_amd import profiling
    path = os.path.join(ROOT, "profiles", "traffic_stencil_%dx%dx%dx%d.json" % tuple(dims))
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_hash") != profiling.source_hash():
        return None
    tot, n = 0.0, 0
    for k, v in d["kernels"].items():
        # the solver's stencils of this precision: stencil_kernel<prec, dagger,
        # rhs/thread, reduction, apply, variant>, twalk_kernel<prec, dagger,
        # reduction, apply> or brick_kernel<prec, dagger, reduction, apply>,
        # with a fused reduction (the profiled run does not autotune, so
        # these are the timed solve's launches)
        if k.startswith("wl::stencil_kernel<"):
            red_at = 3
        elif k.startswith("wl::twalk_kernel<") or k.startswith("wl::brick_kernel<"):
            red_at = 2
        else:
            continue
        targs = [int(a) if a.strip().lstrip("-").isdigit() else int(a.strip() == "true")
                 for a in k[k.index("<") + 1:k.index(">")].split(",")]
        if targs[0] == prec and targs[red_at] != 0:
            tot += v["hbm_bytes"] * v["dispatches"]
            n += v["dispatches"]
    return round(tot / n) if n else None


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo; lscpu reads the same)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    """Threads the oracle's OpenMP runtime uses: OMP_NUM_THREADS, else the
    cores this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def omp_set_threads(n):
    """Set the thread count of the OpenMP runtime the oracle is linked with."""
    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))


def oracle_errors(oracle, U, x, b, kappa, x_star=None, dagger=False):
    """The true relative residual ||b - D x|| / ||b|| with the FP64 oracle D
    and, given the oracle solution x*, the forward error ||x - x*|| / ||x*||."""
    import numpy as np
    r = oracle.apply(U, x, kappa, dagger=dagger) - b
    out = {"oracle_true_rel_res": float(np.linalg.norm(r) / np.linalg.norm(b))}
    if x_star is not None:
        out["forward_error_vs_oracle"] = float(np.linalg.norm(x - x_star) / np.linalg.norm(x_star))
    return out


def oracle_solve(oracle, U, b, kappa, tol=1e-12):
    """The oracle's BiCGStab from x = 0; on a breakdown (a point source as the
    shadow residual makes <rh, r> vanish exactly after one step for this
    operator) it restarts from its own current x, where rh = r is no longer a
    point.  Returns x and a summary."""
    x, code, it, rr = oracle.bicgstab(U, b, kappa, tol=tol)
    its, restarts = it, 0
    while code == 2 and restarts < 5:
        x, code, it, rr = oracle.bicgstab(U, b, kappa, tol=tol, x0=x)
        its += it
        restarts += 1
    return x, {"status": code, "iters": its, "restarts": restarts, "true_rel_res": rr}


def per_iteration(st, seconds):
    """Launch counts and time per Krylov iteration of a solve (whole call,
    set-up and final residual included, divided by the iterations)."""
    it = max(int(st["iters"]), 1)
    return {"kernels": st["kernels"], "finalizes": st["finalizes"],
            "kernels_per_iter": round(st["kernels"] / it, 2), "finalizes_per_iter": round(st["finalizes"] / it, 2),
            "ms_per_iter": round(1e3 * seconds / it, 4)}


def _time_ms(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_batching(W, inputs, torch, log, oracle=None):
    """24^3 x 48 with the 12 point sources (one per spin-colour at the origin):
    multi-RHS FP32 stencil vs one right-hand side at a time, and the batched
    mixed-precision solve vs 12 sequential solves; plus one persistent launch
    over the uneven lattices {8^4, 12^4, 16^3x32, 20^4} x 4 sources vs separate
    launches."""
    out = {}
    dims = (24, 24, 24, 48)
    V = inputs.volume(dims)
    kappa = 0.12
    log(f"[bench] batching: generating {dims}")
    U24 = inputs.near_unity_gauge(dims, 0.3, seed=inputs.GAUGE_SEED)
    src24 = inputs.point_sources_all_spin_colour(dims)
    Ud = torch.from_numpy(U24).cuda()
    src = torch.from_numpy(src24).cuda()
    hi = W.Operator.create(Ud, kappa, W.WL_F64)
    lo = W.Operator.create(Ud, kappa, W.WL_F32)
    del Ud
    st = W._stream()
    W.wl_autotune(lo.handle, 12, 0, st)
    W.wl_autotune(lo.handle, 1, 0, st)
    s12 = lo.pack(src)
    d12 = lo.new_field(12)
    ms12 = _time_ms(torch, lambda: lo.apply_packed(d12, s12, 12), 10)
    s1 = lo.pack(src[0])
    d1 = lo.new_field(1)
    ms1 = _time_ms(torch, lambda: lo.apply_packed(d1, s1, 1), 10)
    bytes12 = (2 * 96 + 4 * 48 / 12) * V * 12
    out["multi_rhs_stencil_f32"] = {
        "nrhs": 12, "launch": W.wl_get_launch(lo.handle, 12), "us": round(ms12 * 1e3, 1),
        "us_per_rhs": round(ms12 * 1e3 / 12, 1), "single_rhs_us": round(ms1 * 1e3, 1),
        "speedup_vs_12_single": round(12 * ms1 / ms12, 3),
        "GFLOP/s": round(1368 * V * 12 / (ms12 * 1e-3) / 1e9, 1),
        "GB/s": round(bytes12 / (ms12 * 1e-3) / 1e9, 1), "bytes_per_site_per_rhs": 208}
    log(f"[bench] multi-RHS stencil: {out['multi_rhs_stencil_f32']}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xb, sts = W.solve(None, src, kappa, method="bicgstab", precision="mixed-f32", tol=1e-10, ops=(hi, lo),
                      return_stats=True)
    t_batch = time.perf_counter() - t0
    xb = xb.cpu().numpy()
    t0 = time.perf_counter()
    iters = []
    for k in range(12):
        _, s_k = W.solve(None, src[k], kappa, method="bicgstab", precision="mixed-f32", tol=1e-10, ops=(hi, lo),
                         return_stats=True)
        iters.append(s_k["iters"])
    t_seq = time.perf_counter() - t0
    out["batched_solve"] = {"nrhs": 12, "precision": "mixed-f32", "seconds": round(t_batch, 4),
                            "sequential_seconds": round(t_seq, 4), "speedup": round(t_seq / t_batch, 3),
                            "max_true_rel_res": max(x["true_rel_res"] for x in sts),
                            "iters": [x["iters"] for x in sts], "sequential_iters": iters}
    if oracle is not None:
        # every column's true residual by the FP64 oracle; the forward error
        # against oracle solutions (BiCGStab to 1e-12) for two columns, a
        # bounded sample of the CPU work
        cols = {}
        for k in range(12):
            star = None
            info = None
            if k in (0, 11):
                t1 = time.perf_counter()
                star, info = oracle_solve(oracle, U24, src24[k], kappa)
                info["seconds"] = round(time.perf_counter() - t1, 2)
                log(f"[bench] oracle solution of column {k}: {info}")
            cols[k] = oracle_errors(oracle, U24, xb[k], src24[k], kappa, star)
            if info is not None:
                cols[k]["oracle_solution"] = info
        out["batched_solve"]["oracle_per_column"] = cols
        out["batched_solve"]["max_oracle_true_rel_res"] = max(c["oracle_true_rel_res"] for c in cols.values())
    del xb
    log(f"[bench] batched solve: {out['batched_solve']}")
    del hi, lo, src, s12, d12, s1, d1
    torch.cuda.empty_cache()
    # uneven lattices in one persistent launch
    lattices = [(8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 32), (20, 20, 20, 20)]
    ops, srcs, dsts = [], [], []
    for j, dj in enumerate(lattices):
        op = W.Operator.create(torch.from_numpy(inputs.near_unity_gauge(dj, 0.3, seed=10 + j)).cuda(), kappa, W.WL_F32)
        srcs.append(op.pack(torch.from_numpy(inputs.gaussian_spinor(dj, seed=100 * j, nrhs=4)).cuda()))
        dsts.append(op.new_field(4))
        ops.append(op)
    descs = [(o.handle, d.data_ptr(), s_.data_ptr()) for o, d, s_ in zip(ops, dsts, srcs)]
    plan = W.MultiPlan(descs, 0, 4)
    plan.tune(st)
    ms_multi = _time_ms(torch, lambda: plan.run(st), 20)
    for o in ops:
        W.wl_autotune(o.handle, 4, 0, st)

    def separate():
        for o, d, s_ in zip(ops, dsts, srcs):
            o.apply_packed(d, s_, 4)
    ms_sep = _time_ms(torch, separate, 20)
    Vt = sum(inputs.volume(d) for d in lattices)
    out["multi_lattice_f32"] = {"lattices": [list(d) for d in lattices], "nrhs": 4, "V_total": Vt,
                                "one_launch_us": round(ms_multi * 1e3, 1), "plan_launch": plan.launch(),
                                "separate_launches_us": round(ms_sep * 1e3, 1),
                                "speedup": round(ms_sep / ms_multi, 3),
                                "GFLOP/s": round(1368 * Vt * 4 / (ms_multi * 1e-3) / 1e9, 1)}
    log(f"[bench] multi-lattice: {out['multi_lattice_f32']}")
    del ops, srcs, dsts, plan
    torch.cuda.empty_cache()
    out["multi_lattice_solve"] = bench_multi_solve(W, inputs, torch, log, oracle, lattices, kappa)
    # an ensemble of small lattices (64 of 4^4 .. 8^4), where separate
    # launches are bound by their fixed cost
    shapes = [(4, 4, 4, 4), (6, 6, 6, 6), (8, 8, 8, 8), (4, 4, 4, 8)]
    ens = [shapes[j % 4] for j in range(64)]
    ops, srcs, dsts = [], [], []
    for j, dj in enumerate(ens):
        op = W.Operator.create(torch.from_numpy(inputs.near_unity_gauge(dj, 0.3, seed=300 + j)).cuda(), kappa,
                               W.WL_F32)
        srcs.append(op.pack(torch.from_numpy(inputs.gaussian_spinor(dj, seed=400 + j, nrhs=4)).cuda()))
        dsts.append(op.new_field(4))
        ops.append(op)
    plan = W.MultiPlan([(o.handle, d.data_ptr(), s_.data_ptr()) for o, d, s_ in zip(ops, dsts, srcs)], 0, 4)
    plan.tune(st)
    ms_multi = _time_ms(torch, lambda: plan.run(st), 50)
    for o in ops[:4]:
        W.wl_autotune(o.handle, 4, 0, st)
    ms_sep = _time_ms(torch, separate, 20)
    Vt = sum(inputs.volume(d) for d in ens)
    out["ensemble_64_small_f32"] = {"lattices": "16 each of 4^4, 6^4, 8^4, 4^3x8", "nrhs": 4, "V_total": Vt,
                                    "one_launch_us": round(ms_multi * 1e3, 1), "plan_launch": plan.launch(),
                                    "separate_launches_us": round(ms_sep * 1e3, 1),
                                    "speedup": round(ms_sep / ms_multi, 3),
                                    "GFLOP/s": round(1368 * Vt * 4 / (ms_multi * 1e-3) / 1e9, 1)}
    log(f"[bench] ensemble of small lattices: {out['ensemble_64_small_f32']}")
    return out


def _copy_launch(W, src_op, dst_op, nrhs=1):
    c = W.wl_get_launch(src_op.handle, nrhs)
    W.wl_set_launch(dst_op.handle, nrhs, c[0], c[1], c[2], c[3], c[4],
                    brick=c[5:8] if c[3] == W.VAR_BRICK else None, t_steps=c[8], wg_per_cu=c[9], rhs_major=c[10])


def bench_multi_solve(W, inputs, torch, log, oracle, lattices, kappa):
    """The uneven lattices x 4 Gaussian sources solved together (mixed FP32
    BiCGStab to 1e-10: every stencil one multi-lattice launch) against the
    same four systems solved one after the other, each column checked with
    the oracle's D."""
    import numpy as np
    st = W._stream()
    nrhs = 4
    systems, host = [], []
    for j, dj in enumerate(lattices):
        U = inputs.near_unity_gauge(dj, 0.3, seed=10 + j)
        b = inputs.gaussian_spinor(dj, seed=100 * j, nrhs=nrhs)
        Ud = torch.from_numpy(U).cuda()
        hi = W.Operator.create(Ud, kappa, W.WL_F64)
        lo = W.Operator.create(Ud, kappa, W.WL_F32)
        systems.append((hi, lo, hi.pack(torch.from_numpy(b).cuda())))
        host.append((U, b))
    # the multi-lattice stencil shape: the plan tuner's choice for these lattices
    plans = []
    for prec_op in (0, 1):
        fields = [(s_[prec_op], s_[prec_op].new_field(nrhs), s_[prec_op].new_field(nrhs)) for s_ in systems]
        plan = W.MultiPlan([(o.handle, d.data_ptr(), i.data_ptr()) for o, d, i in fields], 0, nrhs)
        plan.tune(st)
        plans.append(plan.launch())
        del plan, fields
    W.solve_multi(systems, nrhs=nrhs, method="bicgstab", tol=1e-10)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xs, stm = W.solve_multi(systems, nrhs=nrhs, method="bicgstab", tol=1e-10, return_stats=True)
    torch.cuda.synchronize()
    t_multi = time.perf_counter() - t0

    def separate():
        res = []
        for hi, lo, b in systems:
            res.append(W.solve(None, hi.unpack(b, nrhs), kappa, method="bicgstab", tol=1e-10, ops=(hi, lo),
                               return_stats=True)[1])
        return res
    separate()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sts = separate()
    torch.cuda.synchronize()
    t_sep = time.perf_counter() - t0
    r = {"lattices": [list(d) for d in lattices], "nrhs": nrhs, "precision": "mixed-f32", "method": "bicgstab",
         "tol": 1e-10, "seconds": round(t_multi, 4), "separate_seconds": round(t_sep, 4),
         "speedup": round(t_sep / t_multi, 3), "plan_launch_f64_f32": plans,
         "iters": [s_["iters"] for s_ in stm], "separate_iters": [s_["iters"] for sj in sts for s_ in sj],
         "kernels": stm[0]["kernels"], "separate_kernels": sum(sj[0]["kernels"] for sj in sts),
         "status": stm[0]["status"], "max_true_rel_res": max(s_["true_rel_res"] for s_ in stm)}
    if oracle is not None:
        worst = 0.0
        for (hi, _, _), (U, b), x in zip(systems, host, xs):
            xc = hi.unpack(x, nrhs).cpu().numpy()
            for k in range(nrhs):
                res = b[k] - oracle.apply(U, xc[k], kappa)
                worst = max(worst, float(np.linalg.norm(res) / np.linalg.norm(b[k])))
        r["max_oracle_true_rel_res"] = worst
    log(f"[bench] multi-lattice solve: {r}")
    del systems, xs
    torch.cuda.empty_cache()
    return r


def bench_c2(W, inputs, torch, log, oracle=None):
    """The paper's single-node lattice 16^3 x 32 (eps = 0.3, kappa = 0.125):
    FP64 and FP32 apply on one buffer set (it fits the 256 MB Infinity Cache)
    and rotated over four sets (links, source and output each; > 256 MB), the
    FP64 BiCGStab and CGNR solves to 1e-10 with their errors against the
    oracle, and the oracle's own BiCGStab and CGNR timed on the host."""
    import numpy as np
    dims = (16, 16, 16, 32)
    kappa = 0.125
    V = inputs.volume(dims)
    st = W._stream()
    log(f"[bench] single lattice {dims}: generating")
    U = inputs.near_unity_gauge(dims, 0.3, seed=inputs.GAUGE_SEED)
    b = inputs.gaussian_spinor(dims, seed=inputs.SOURCE_SEED)
    Ud = torch.from_numpy(U).cuda()
    bd = torch.from_numpy(b).cuda()
    out = {"dims": list(dims), "kappa": kappa, "eps": 0.3}
    app = {}
    nsets = 4
    for p in (0, 1):
        ops = [W.Operator.create(Ud, kappa, p) for _ in range(nsets)]  # four packed copies of the links
        W.wl_autotune(ops[0].handle, 1, 0, st)
        for o in ops[1:]:
            _copy_launch(W, ops[0], o)
        srcs = [o.pack(bd) for o in ops]
        dsts = [o.new_field() for o in ops]
        ms1 = _time_ms(torch, lambda: ops[0].apply_packed(dsts[0], srcs[0]), 200)

        def rotated():
            for k in range(nsets):
                ops[k].apply_packed(dsts[k], srcs[k])
        ms4 = _time_ms(torch, rotated, 50) / nsets
        gbs1 = BYTES[p] * V / (ms1 * 1e-3) / 1e9
        gbs4 = BYTES[p] * V / (ms4 * 1e-3) / 1e9
        app[PNAME[p]] = {"us": round(ms1 * 1e3, 2), "GFLOP/s": round(FLOP_APPLY * V / (ms1 * 1e-3) / 1e9, 1),
                         "GB/s": round(gbs1, 1), "hbm_frac": round(gbs1 / HBM_PEAK_GBS, 4),
                         "rotated_us": round(ms4 * 1e3, 2),
                         "rotated_GFLOP/s": round(FLOP_APPLY * V / (ms4 * 1e-3) / 1e9, 1),
                         "rotated_GB/s": round(gbs4, 1), "rotated_hbm_frac": round(gbs4 / HBM_PEAK_GBS, 4),
                         "rotated_sets": nsets, "set_MB": round(BYTES[p] * V / 1e6, 1),
                         "launch": W.wl_get_launch(ops[0].handle, 1)}
        log(f"[bench] {dims} apply {PNAME[p]}: {app[PNAME[p]]}")
        del ops, srcs, dsts
    out["apply"] = app
    hi = W.Operator.create(Ud, kappa, W.WL_F64)
    W.wl_autotune(hi.handle, 1, 0, st)
    x_star = None
    if oracle is not None:
        t1 = time.perf_counter()
        x_star, info = oracle_solve(oracle, U, b, kappa)
        info.update({"tol": 1e-12, "seconds": round(time.perf_counter() - t1, 2)})
        out["oracle_reference_solution"] = info
    solves = {}
    for method in ("bicgstab", "cgnr"):
        for form in (0, 1):
            W.solve(None, bd, kappa, method=method, precision="f64", tol=1e-10, ops=(hi, None), form=form)  # warm-up
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            x, sst = W.solve(None, bd, kappa, method=method, precision="f64", tol=1e-10, ops=(hi, None),
                             return_stats=True, form=form)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            r = {"seconds": round(dt, 4), "status": sst["status"], "iters": sst["iters"],
                 "stencil_calls": sst["stencil_calls"], "true_rel_res": sst["true_rel_res"]}
            r.update(per_iteration(sst, dt))
            if oracle is not None:
                r.update(oracle_errors(oracle, U, x.cpu().numpy(), b, kappa, x_star))
            key = method + "_f64" + ("_single_reduction" if form else "")
            solves[key] = r
            log(f"[bench] {dims} solve {key}: {r}")
    out["solves"] = solves
    if oracle is not None:
        # the oracle's solvers on the same system, timed on the host
        osol = {"threads": host_threads(), "cpu_model": cpu_model()}
        for method in ("bicgstab", "cgnr"):
            fn = oracle.bicgstab if method == "bicgstab" else oracle.cgnr
            t1 = time.perf_counter()
            _, code_o, it_o, rr_o = fn(U, b, kappa, tol=1e-10)
            dt = time.perf_counter() - t1
            osol[method] = {"seconds": round(dt, 2), "status": code_o, "iters": it_o, "true_rel_res": rr_o,
                            "gpu_speedup": round(dt / solves[method + "_f64"]["seconds"], 1)}
        out["oracle_solvers"] = osol
        log(f"[bench] {dims} oracle solvers: {osol}")
    del hi, Ud, bd
    torch.cuda.empty_cache()
    return out


def bench_halo(W, inputs, torch, log):
    """Enforced-halo apply (t faces through buffers on a side stream, interior
    meanwhile, boundary finish) against the plain apply, FP32 and FP64, at the
    paper's 16^3 x 32 and 32^3 x 64 Wilson lattices."""
    out = {}
    for dims in ((16, 16, 16, 32), (32, 32, 32, 64)):
        V = inputs.volume(dims)
        Ud = torch.from_numpy(inputs.near_unity_gauge(dims, 0.3, seed=inputs.GAUGE_SEED)).cuda()
        src = torch.from_numpy(inputs.gaussian_spinor(dims, seed=inputs.SOURCE_SEED)).cuda()
        res = {}
        for p in (0, 1):
            op = W.Operator.create(Ud, 0.1255, p)
            W.wl_autotune(op.handle, 1, 0, W._stream())
            a = op.pack(src)
            b = op.new_field()
            halo = op.halo_buffer()
            ms_plain = _time_ms(torch, lambda: op.apply_packed(b, a), 20)
            ms_halo = _time_ms(torch, lambda: op.apply_halo_packed(b, a, halo), 20)
            res[PNAME[p]] = {"plain_us": round(ms_plain * 1e3, 1), "halo_us": round(ms_halo * 1e3, 1),
                             "halo_GFLOP/s": round(FLOP_APPLY * V / (ms_halo * 1e-3) / 1e9, 1),
                             "overhead": round(ms_halo / ms_plain - 1.0, 3),
                             "face_bytes": int(halo.numel() // 2)}
            log(f"[bench] halo apply {dims} {PNAME[p]}: {res[PNAME[p]]}")
            del op, a, b, halo
        out["%dx%dx%dx%d" % dims] = res
        del Ud, src
        torch.cuda.empty_cache()
    out["paper_knl_context"] = {"wilson_copy_enforced_GFLOPs_16x16x16x32": 100.4,
                                "wilson_copy_enforced_GFLOPs_32x32x32x64": 176.0,
                                "note": "single KNL node, single precision, boundary copy enforced (context only)"}
    return out


DW_FLOP_PER_5D_SITE = 11520 // 8  # Table I: 11520 flop per 4-d site at Ns = 8


def bench_dwf(W, inputs, torch, log):
    """Domain-wall operator (eq. (2), Ns = 8, m0 = -1.8, m = 0.05): apply
    throughput per precision on the paper's per-node 16^3 x 32 lattice and on
    32^3 x 64, and CG on D^dag D (FP64, mixed FP32, mixed FP16) to 1e-10 at
    16^3 x 32.  Compulsory bytes per 5-d site: two spinors plus the links
    shared by the Ns slices (FP64 384 + 384/Ns, FP32 192 + 192/Ns, 16-bit
    104 + 96/Ns)."""
    out = {}
    Ns, m0, mq = 8, -1.8, 0.05
    spin = {0: 192, 1: 96, 2: 52, 3: 52}
    link4 = {0: 384, 1: 192, 2: 96, 3: 96}
    st = W._stream()
    for dims in ((16, 16, 16, 32), (32, 32, 32, 64)):
        V = inputs.volume(dims)
        log(f"[bench] domain wall: generating {dims} x Ns={Ns}")
        Ud = torch.from_numpy(inputs.near_unity_gauge(dims, 0.3, seed=inputs.GAUGE_SEED)).cuda()
        src = torch.stack([torch.from_numpy(inputs.gaussian_spinor(dims, seed=s)) for s in range(Ns)]).cuda()
        res = {}
        for p in (0, 1, 3):
            op = W.DWOperator.create(Ud, m0, mq, Ns, p)
            W.wl_autotune(op.handle, 1, 0, st)
            a = op.pack(src)
            b = op.new_field()
            ms = _time_ms(torch, lambda: op.apply_packed(b, a), 10)
            nbytes = (2 * spin[p] + link4[p] / Ns) * V * Ns
            res[PNAME[p]] = {"us": round(ms * 1e3, 1),
                             "GFLOP/s": round(DW_FLOP_PER_5D_SITE * V * Ns / (ms * 1e-3) / 1e9, 1),
                             "GB/s": round(nbytes / (ms * 1e-3) / 1e9, 1),
                             "hbm_frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                             "launch": W.wl_get_launch(op.handle, 1)}
            log(f"[bench] dw apply {dims} {PNAME[p]}: {res[PNAME[p]]}")
            del op, a, b
        out["apply_%dx%dx%dx%d" % dims] = res
        if dims == (16, 16, 16, 32):
            solves = {}
            hi = W.DWOperator.create(Ud, m0, mq, Ns, W.WL_F64)
            W.wl_autotune(hi.handle, 1, 0, st)
            los = {}
            for prec, rel in (("f64", 0), ("mixed-f32", 0), ("mixed-f16", 0), ("mixed-f32", 1)):
                lo = None
                if prec != "f64":
                    if prec not in los:
                        los[prec] = W.DWOperator.create(Ud, m0, mq, Ns, W.PREC[prec.split("-")[1]])
                        W.wl_autotune(los[prec].handle, 1, 0, st)
                    lo = los[prec]
                W.dw_solve(None, src, m0, mq, precision=prec, tol=1e-10, ops=(hi, lo), reliable=bool(rel))  # warm-up
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x, stt = W.dw_solve(None, src, m0, mq, precision=prec, tol=1e-10, ops=(hi, lo), return_stats=True,
                                    reliable=bool(rel))
                dt = time.perf_counter() - t0
                key = prec + ("_reliable" if rel else "")
                solves[key] = {"seconds": round(dt, 4), "status": stt["status"], "iters": stt["iters"],
                               "outer": stt["outer"], "true_rel_res": stt["true_rel_res"]}
                log(f"[bench] dw cgnr {key}: {solves[key]}")
            del los
            base = solves["f64"]["seconds"]
            for v in solves.values():
                v["speedup_vs_f64"] = round(base / v["seconds"], 3)
            out["cgnr_16x16x16x32"] = solves
            del hi
        del Ud, src
        torch.cuda.empty_cache()
    out["paper_knl_context"] = {"dw_mult_GFLOPs_16x16x16x32": 155.2, "dw_mult_GFLOPs_32x32x32x64": 211.8,
                                "note": "single KNL node, single precision, boundary copy enforced (context only)"}
    return out


def bench_autograd(W, inputs, torch, log):
    """Differentiable solve at 16^3 x 32, kappa 0.12: L = ||D^{-1} b||^2,
    forward (mixed FP32/FP64) + backward (adjoint solve + link force)."""
    from paper_1712_01505_amd.autograd import wilson_solve
    dims = (16, 16, 16, 32)
    U = torch.from_numpy(inputs.near_unity_gauge(dims, 0.3, seed=inputs.GAUGE_SEED)).cuda().requires_grad_(True)
    b = torch.from_numpy(inputs.gaussian_spinor(dims, seed=inputs.SOURCE_SEED)).cuda().requires_grad_(True)

    def step():
        U.grad = None
        b.grad = None
        x = wilson_solve(U, b, 0.12, precision="mixed-f32", tol=1e-10)
        (x.abs() ** 2).sum().backward()
    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    r = {"dims": list(dims), "kappa": 0.12, "forward_plus_backward_s": round(dt, 4),
         "grad_b_norm": float(b.grad.abs().pow(2).sum().sqrt()), "grad_U_norm": float(U.grad.abs().pow(2).sum().sqrt())}
    log(f"[bench] differentiable solve: {r}")
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dims", type=str, default="32,32,32,64")
    ap.add_argument("--inner", type=str, default="f16", choices=["f32", "bf16", "f16"])
    ap.add_argument("--reliable", type=int, default=0, choices=[0, 1],
                    help="timed solve: 1 = reliable updates, 0 = defect correction")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (launch shapes then come from $WL_TUNE_CACHE or the defaults)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline and check")
    ap.add_argument("--no-extra", action="store_true", help="skip the measurements outside the timed region")
    ap.add_argument("--no-batch", action="store_true", help="skip the multi-RHS / multi-lattice / autograd extras")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding is a design, not an implementation.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1712_01505_amd import inputs
    from paper_1712_01505_amd import wilson as W

    dims = tuple(int(v) for v in args.dims.split(","))
    V = inputs.volume(dims)
    kappa, eps, tol = 0.1255, 0.3, 1e-10
    log(f"[bench] generating inputs {dims} (V={V})")
    t0 = time.time()
    U = inputs.near_unity_gauge(dims, eps, seed=inputs.GAUGE_SEED)
    b = inputs.gaussian_spinor(dims, seed=inputs.SOURCE_SEED)
    log(f"[bench] inputs ready in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    Ud = torch.from_numpy(U).to(dev)
    bd = torch.from_numpy(b).to(dev)
    ops = {p: W.Operator.create(Ud, kappa, p) for p in (W.WL_F64, W.WL_F32, W.WL_BF16S, W.WL_F16S)}
    del Ud
    torch.cuda.synchronize()
    stream = W._stream()
    hi = ops[W.WL_F64]
    b64 = hi.pack(bd)
    x64 = hi.new_field()
    ws_bytes = max(W.wl_solver_workspace_bytes(hi.handle, lo, s, 1)
                   for lo in [None] + [ops[p].handle for p in (1, 2, 3)] for s in (0, 1))
    work = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)

    def run_solve(method, lo_prec, reliable=args.reliable, eo=0, form=0):
        prm = W.wl_solve_params(tol=tol, maxiter=20000, inner_tol=0.0, max_outer=0, reliable=int(reliable),
                                eo=int(eo), check_every=0, form=int(form),
                                use_x0=0, workspace=work.data_ptr(), workspace_bytes=ws_bytes)
        st = (W.wl_solve_stats * 1)()
        fn = W.solve_cgnr if method == "cgnr" else W.solve_bicgstab
        lo = ops[lo_prec].handle if lo_prec is not None else None
        code = fn(hi.handle, lo, x64.data_ptr(), b64.data_ptr(), 1, prm, st, stream)
        return code, st[0].as_dict()

    oracle = None
    if not args.no_cpu:
        import oracle  # the FP64 CPU checker (test infrastructure), never the product path
    inner = {"f32": W.WL_F32, "bf16": W.WL_BF16S, "f16": W.WL_F16S}[args.inner]
    tuned = {}
    for p, op in ops.items():
        if not args.no_tune:
            W.wl_autotune(op.handle, 1, 0, stream)
        tuned[PNAME[p]] = W.wl_get_launch(op.handle, 1)
    log(f"[bench] autotuned launch (block, rhs/thread, xcd, variant): {tuned}")

    # ---------------------------------------------------------------- timed region
    log(f"[bench] warmup {args.warmup} step(s)")
    for _ in range(args.warmup):
        code, st = run_solve("bicgstab", inner)
        if code != 0:
            raise SystemExit(f"warmup solve failed: status {code} {st}")
    W.wl_prof_reset()
    W.wl_prof_enable(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(args.steps):
        code, st = run_solve("bicgstab", inner)
        stats.append(st)
        if code != 0:
            raise SystemExit(f"timed solve failed: status {code} {st}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    W.wl_prof_enable(0)
    prof = {p: W.wl_prof_read(p) for p in range(4)}
    prof_aux = {p: W.wl_prof_read_aux(p) for p in range(4)}
    log(f"[bench] {args.steps} steps in {elapsed:.3f}s")
    ms_per_step = 1e3 * elapsed / args.steps
    calls = sum(s["stencil_calls"] for s in stats) / args.steps
    value = calls * FLOP_APPLY * V / (ms_per_step * 1e-3) / 1e9
    step_x = hi.unpack(x64).cpu().numpy()
    last = stats[-1]

    # dominant kernel: the stencil precision with the most time in the step
    dom = max(prof, key=lambda p: prof[p][1])
    n_l, ms_l, sites_l = prof[dom]
    avg_ms = ms_l / max(n_l, 1)
    # compulsory bytes of the launches: the stencil's own, plus the rh field
    # read by the launches whose fused reduction takes <rh, out>
    bytes_per_launch = (BYTES[dom] * sites_l + SPINOR[dom] * prof_aux[dom]) / max(n_l, 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm",
                "kernel": f"wilson stencil <{PNAME[dom]}> in the solve (stencil/t-walk/brick kernels, fused reductions)",
                "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(dom, dims),
                "bytes_per_site": round(bytes_per_launch / V, 1), "stencil_bytes_per_site": BYTES[dom],
                "fused_rh_read_fraction": round(prof_aux[dom] / max(sites_l, 1), 3),
                "sites_per_launch": V, "avg_launch_us": round(avg_ms * 1e3, 2),
                "launches": n_l}

    result = {
        "metric": "dslash GFLOP/s & HBM GB/s; mixed vs FP64 solve time at 1e-10 residual",
        "value": round(value, 1), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": f"fp32 arithmetic on {args.inner} storage inside fp64 refinement", "data": "synthetic",
        "config": {"workload": f"wilson-dirac mixed-precision BiCGStab solve, {dims[0]}^3x{dims[3]}"
                   if dims[0] == dims[1] == dims[2] else f"wilson-dirac solve {dims}",
                   "dims": list(dims), "kappa": kappa, "eps": eps, "bc": [1, 1, 1, -1], "tol": tol,
                   "inner": args.inner, "reliable_updates": bool(args.reliable), "value_counts": "1368 flop/site x stencil applications per step / step time"},
        "launch": tuned,
        "solve_step": {"iters": last["iters"], "outer": last["outer"], "stencil_calls": last["stencil_calls"],
                       "true_rel_res": last["true_rel_res"], "seconds": round(ms_per_step / 1e3, 4),
                       **per_iteration(last, ms_per_step / 1e3)},
        "roofline": roofline,
    }

    # ---------------------------------------------------------------- outside the timed region
    if not args.no_extra:
        dsl = {}
        for p in (0, 1, 2, 3):
            op = ops[p]
            src = op.pack(bd)
            dst = op.new_field()
            for _ in range(3):
                op.apply_packed(dst, src)
            reps = 20
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                op.apply_packed(dst, src)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            dsl[PNAME[p]] = {"us": round(ms * 1e3, 1), "GFLOP/s": round(FLOP_APPLY * V / (ms * 1e-3) / 1e9, 1),
                             "GB/s": round(BYTES[p] * V / (ms * 1e-3) / 1e9, 1),
                             "hbm_frac": round(BYTES[p] * V / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            del src, dst
            log(f"[bench] apply {PNAME[p]}: {dsl[PNAME[p]]}")
        result["dslash"] = dsl
        # the FP64 oracle's solution x* of the same system (BiCGStab to 1e-12,
        # zero start), against which every solve below states its error
        x_star, ref_info = None, None
        if oracle is not None:
            log("[bench] oracle reference solution x* (CPU, BiCGStab to 1e-12)")
            t1 = time.perf_counter()
            x_star, ref_info = oracle_solve(oracle, U, b, kappa)
            ref_info.update({"method": "oracle BiCGStab, FP64, zero start", "tol": 1e-12,
                             "seconds": round(time.perf_counter() - t1, 2), "threads": host_threads()})
            result["oracle_reference_solution"] = ref_info
            log(f"[bench] x*: {ref_info}")
            result["solve_step"].update(oracle_errors(oracle, U, step_x, b, kappa, x_star))
        solves = {}
        F16 = W.WL_F16S
        for method, lo, rel, eo, form in (
                ("bicgstab", None, 0, 0, 0), ("cgnr", None, 0, 0, 0), ("bicgstab", W.WL_F32, 0, 0, 0),
                ("bicgstab", W.WL_BF16S, 0, 0, 0), ("bicgstab", F16, 0, 0, 0), ("cgnr", F16, 0, 0, 0),
                ("bicgstab", W.WL_F32, 1, 0, 0), ("bicgstab", W.WL_BF16S, 1, 0, 0), ("bicgstab", F16, 1, 0, 0),
                ("cgnr", W.WL_F32, 0, 0, 0), ("cgnr", W.WL_F32, 1, 0, 0),
                ("bicgstab", None, 0, 1, 0), ("cgnr", None, 0, 1, 0), ("bicgstab", W.WL_F32, 1, 1, 0),
                ("bicgstab", F16, 0, 1, 0), ("bicgstab", F16, 1, 1, 0),
                # one reduction phase per iteration
                ("bicgstab", None, 0, 0, 1), ("cgnr", None, 0, 0, 1), ("bicgstab", F16, 0, 0, 1),
                ("cgnr", F16, 0, 0, 1)):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            code, st = run_solve(method, lo, rel, eo, form)
            dt = time.perf_counter() - t1
            key = (f"{method}_{'f64' if lo is None else 'mixed_' + PNAME[lo]}{'_reliable' if rel else ''}"
                   f"{'_evenodd' if eo else ''}{'_single_reduction' if form else ''}")
            solves[key] = {"seconds": round(dt, 4), "status": code, "iters": st["iters"], "outer": st["outer"],
                           "true_rel_res": st["true_rel_res"]}
            solves[key].update(per_iteration(st, dt))
            if oracle is not None:
                solves[key].update(oracle_errors(oracle, U, hi.unpack(x64).cpu().numpy(), b, kappa, x_star))
            log(f"[bench] solve {key}: {solves[key]}")
        base = solves["bicgstab_f64"]["seconds"]
        for k, v in solves.items():
            v["speedup_vs_bicgstab_f64"] = round(base / v["seconds"], 3)
        result["solves"] = solves

    c2 = None
    if not args.no_extra and not args.no_batch:
        del ops, hi, b64, x64, work
        torch.cuda.empty_cache()
        c2 = bench_c2(W, inputs, torch, log, oracle)
        result["single_lattice_16x16x16x32"] = c2
        result["batching"] = bench_batching(W, inputs, torch, log, oracle)
        result["differentiable"] = bench_autograd(W, inputs, torch, log)
        result["domain_wall"] = bench_dwf(W, inputs, torch, log)
        result["enforced_halo"] = bench_halo(W, inputs, torch, log)

    if oracle is not None:
        if "oracle_true_rel_res" not in result["solve_step"]:
            result["solve_step"].update(oracle_errors(oracle, U, step_x, b, kappa))
        # the oracle's D on the same lattice: all host threads, then one
        threads = host_threads()
        log(f"[bench] CPU baseline: oracle D on {dims}, {threads} threads then 1 ({cpu_model()})")
        t1 = time.perf_counter()
        oracle.apply(U, b, kappa)
        t_apply = time.perf_counter() - t1
        reps = max(1, min(10, int(12.0 / max(t_apply, 1e-3))))
        t1 = time.perf_counter()
        for _ in range(reps):
            oracle.apply(U, b, kappa)
        t_cpu = (time.perf_counter() - t1) / reps
        omp_set_threads(1)
        t1 = time.perf_counter()
        oracle.apply(U, b, kappa)
        t_one = time.perf_counter() - t1
        omp_set_threads(threads)
        result["cpu_baseline"] = {
            "value": round(FLOP_APPLY * V / t_cpu / 1e9, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{reps} FP64 oracle applications of D on the same {dims} lattice ({t_cpu:.3f} s each, "
                      f"OpenMP, {threads} threads); one more with 1 thread ({t_one:.2f} s)",
            "single_thread_value": round(FLOP_APPLY * V / t_one / 1e9, 3),
            "cpu_model": cpu_model(),
            "gpu_fp64_apply_vs_cpu": (round(result["dslash"]["f64"]["GFLOP/s"] / (FLOP_APPLY * V / t_cpu / 1e9), 1)
                                      if "dslash" in result else None)}
        if c2 is not None and "oracle_solvers" in c2:
            result["cpu_baseline"]["solvers_16x16x16x32"] = c2["oracle_solvers"]
        if "oracle_reference_solution" in result:
            result["cpu_baseline"]["reference_solve_32x32x32x64"] = result["oracle_reference_solution"]
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
