"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/wilson.h declares, and validates arguments before any
launch; the header compiles as C; the fast integer division used for site
coordinates is exact."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

from paper_1712_01505_amd import wilson

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wilson.h")


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|char\s*\*|const char\s*\*)\s*\*?\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_binding_exports():
    assert sorted(wilson.EXPORTS) == header_functions()


def test_library_exports_every_declared_symbol():
    L = wilson.lib()
    missing = [n for n in header_functions() if not hasattr(L, n)]
    assert not missing


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc missing")
def test_header_compiles_as_c(tmp_path):
    c = tmp_path / "t.c"
    c.write_text('#include "wilson.h"\nint main(void){ wl_geom g; (void)g; return WL_OK; }\n')
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), "-c", str(c),
                    "-o", str(tmp_path / "t.o")], check=True)


def test_field_bytes():
    g = wilson.make_geom((4, 4, 4, 8))
    V = 512
    assert wilson.wl_field_bytes(g, wilson.WL_SPINOR, wilson.WL_F64, 3) == 3 * V * 192
    assert wilson.wl_field_bytes(g, wilson.WL_SPINOR, wilson.WL_F32, 1) == V * 96
    assert wilson.wl_field_bytes(g, wilson.WL_SPINOR, wilson.WL_BF16S, 2) == 2 * V * 52
    assert wilson.wl_field_bytes(g, wilson.WL_GAUGE, wilson.WL_F64) == 4 * V * 96
    assert wilson.wl_field_bytes(g, wilson.WL_GAUGE, wilson.WL_F16S) == 4 * V * 24


@pytest.mark.parametrize("dims,bc", [((1, 4, 4, 4), (1, 1, 1, -1)), ((4, 4, 4, 0), (1, 1, 1, -1)),
                                     ((4, 4, 4, 4), (1, 1, 2, -1)), ((65536, 65536, 2, 2), (1, 1, 1, 1))])
def test_bad_geometry_rejected(dims, bc):
    L = wilson.lib()
    out = ctypes.c_size_t(0)
    assert L.wl_field_bytes(ctypes.byref(wilson.make_geom(dims, bc)), 0, 0, 1, ctypes.byref(out)) == wilson.WL_EINVAL
    h = ctypes.c_void_p()
    assert L.wl_op_create(ctypes.byref(wilson.make_geom(dims, bc)), 0.1, 0, 256, ctypes.byref(h)) == wilson.WL_EINVAL


def test_bad_arguments_rejected_before_launch():
    L = wilson.lib()
    g = wilson.make_geom((4, 4, 4, 4))
    out = ctypes.c_size_t(0)
    assert L.wl_field_bytes(ctypes.byref(g), 0, 7, 1, ctypes.byref(out)) == wilson.WL_EPREC
    assert L.wl_field_bytes(ctypes.byref(g), 0, 0, 0, ctypes.byref(out)) == wilson.WL_EINVAL
    assert L.wl_pack_spinor(ctypes.byref(g), 0, 1, 24, 256, None) == wilson.WL_EALIGN
    assert L.wl_pack_spinor(ctypes.byref(g), 0, 1, None, 256, None) == wilson.WL_EINVAL
    h = ctypes.c_void_p()
    assert L.wl_op_create(ctypes.byref(g), float("nan"), 0, 256, ctypes.byref(h)) == wilson.WL_EINVAL
    assert L.wl_op_create(ctypes.byref(g), 0.12, 0, 8, ctypes.byref(h)) == wilson.WL_EALIGN
    assert L.wl_op_create(ctypes.byref(g), 0.12, 0, 256, ctypes.byref(h)) == wilson.WL_OK
    op = h.value
    try:
        assert L.wilson_apply(op, 512, 512, 0, 1, None) == wilson.WL_EINVAL  # in == out
        assert L.wilson_apply(op, 512, 1024, 2, 1, None) == wilson.WL_EINVAL  # dagger flag
        assert L.wilson_apply(op, 512, 1024, 0, 0, None) == wilson.WL_EINVAL  # nrhs
        assert L.wilson_apply(op, 520, 1024, 0, 1, None) == wilson.WL_EALIGN
        def setl(nrhs, block, rpt, xcd, var, lanes=1):
            c = wilson.wl_launch(block=block, rhs_per_thread=rpt, rhs_lanes=lanes, xcd_remap=xcd, variant=var)
            return L.wl_set_launch(op, nrhs, ctypes.byref(c))
        assert setl(1, 96, 1, 1, 0) == wilson.WL_EINVAL
        assert setl(4, 256, 3, 1, 0) == wilson.WL_EINVAL  # 3 does not divide 4
        assert setl(4, 256, 4, 1, 0) == wilson.WL_EINVAL  # FP64 offers at most 2
        assert setl(4, 256, 2, 0, 1) == wilson.WL_EINVAL  # pipelined variants need 1 RHS/thread
        assert setl(1, 256, 1, 0, 2) == wilson.WL_EINVAL  # FP64 offers variants 0, 1
        assert setl(4, 256, 1, 0, 1, lanes=3) == wilson.WL_EINVAL  # lanes: 1, 2, 4, 8
        assert setl(2, 256, 1, 0, 1, lanes=4) == wilson.WL_EINVAL  # lanes must divide nrhs
        assert setl(4, 256, 2, 0, 0, lanes=2) == wilson.WL_EINVAL  # lanes need 1 RHS/thread
        assert setl(4, 128, 1, 0, 1, lanes=4) == wilson.WL_EINVAL  # at least 64 sites per workgroup
        assert setl(1, 256, 1, 6, 1) == wilson.WL_EINVAL  # tile orders 0..5
        assert setl(1, 256, 1, 2, 1) == wilson.WL_EINVAL  # no z-slabs for Lz = 4
        assert setl(1, 256, 1, 0, 1) == wilson.WL_OK
        assert setl(4, 256, 2, 0, 0) == wilson.WL_OK
        assert setl(4, 256, 1, 1, 1, lanes=4) == wilson.WL_OK
        got = wilson.wl_launch()
        assert L.wl_get_launch(op, 4, ctypes.byref(got)) == wilson.WL_OK
        assert (got.block, got.rhs_per_thread, got.rhs_lanes, got.xcd_remap, got.variant) == (256, 1, 4, 1, 1)
        # brick walk (variant 7): the brick tiles (x, y, z), has block sites and a walk dividing Lt
        def setb(block, brick, T, nrhs=1, lanes=1):
            c = wilson.wl_launch(block=block, rhs_per_thread=1, rhs_lanes=lanes, xcd_remap=1, variant=7)
            c.brick[0], c.brick[1], c.brick[2] = brick
            c.t_steps = T
            return L.wl_set_launch(op, nrhs, ctypes.byref(c))
        assert setb(64, (4, 4, 4), 4) == wilson.WL_OK
        assert setb(64, (4, 4, 4), 3) == wilson.WL_EINVAL  # 3 does not divide Lt = 4
        assert setb(128, (4, 4, 4), 4) == wilson.WL_EINVAL  # block != brick sites
        assert setb(64, (8, 4, 2), 4) == wilson.WL_EINVAL  # 8 does not divide Lx = 4
        # several right-hand sides per brick workgroup: block = brick sites x count, at most 256 threads
        assert setb(64, (4, 4, 4), 4, nrhs=2, lanes=2) == wilson.WL_EINVAL  # block != 64 sites x 2
        assert setb(512, (4, 4, 4), 4, nrhs=8, lanes=8) == wilson.WL_EINVAL  # at most 4 per workgroup
        assert setb(256, (4, 4, 4), 4, nrhs=6, lanes=4) == wilson.WL_EINVAL  # 4 does not divide 6
        assert setb(128, (4, 4, 4), 4, nrhs=2, lanes=2) == wilson.WL_OK
        assert L.wl_get_launch(op, 2, ctypes.byref(got)) == wilson.WL_OK
        assert (got.block, got.rhs_lanes, got.variant) == (128, 2, 7)
        assert L.wl_get_launch(op, 1, ctypes.byref(got)) == wilson.WL_OK
        assert (got.variant, tuple(got.brick), got.t_steps) == (7, (4, 4, 4), 4)
        # t-walks with right-hand sides across lanes (at least 32 sites per workgroup) and the group order
        assert setl(8, 256, 1, 0, 4, lanes=8) == wilson.WL_OK
        assert setl(8, 128, 1, 0, 4, lanes=8) == wilson.WL_EINVAL
        c = wilson.wl_launch(block=256, rhs_per_thread=1, rhs_lanes=2, xcd_remap=1, variant=4, rhs_major=2)
        assert L.wl_set_launch(op, 8, ctypes.byref(c)) == wilson.WL_EINVAL  # group order 0 or 1
        c.rhs_major = 1
        assert L.wl_set_launch(op, 8, ctypes.byref(c)) == wilson.WL_OK
        assert L.wl_get_launch(op, 8, ctypes.byref(got)) == wilson.WL_OK
        assert (got.rhs_lanes, got.variant, got.rhs_major) == (2, 4, 1)
        # fused apply + inner products: argument checks happen before any launch
        wb = ctypes.c_size_t(0)
        assert L.wl_apply_dot_workspace_bytes(op, 1, ctypes.byref(wb)) == wilson.WL_OK and wb.value % 256 == 0
        assert L.wl_apply_dot_workspace_bytes(op, 65, ctypes.byref(wb)) == wilson.WL_EINVAL
        assert L.wilson_apply_dot(op, 512, 1024, None, 0, 1, wilson.WL_DOT_BICG, 2048, 4096, wb.value,
                                  None) == wilson.WL_EINVAL  # BiCG kind needs v
        assert L.wilson_apply_dot(op, 512, 1024, 1536, 0, 1, 9, 2048, 4096, wb.value, None) == wilson.WL_EINVAL
        assert L.wilson_apply_dot(op, 512, 1024, 1536, 0, 1, wilson.WL_DOT_V, 2048, None, wb.value,
                                  None) == wilson.WL_EWORKSPACE
        assert L.wilson_apply_dot(op, 512, 1024, 1536, 0, 1, wilson.WL_DOT_V, 2048, 4096, wb.value - 8,
                                  None) == wilson.WL_EWORKSPACE
        assert L.wilson_apply_dot(op, 512, 1024, 1536, 0, 1, wilson.WL_DOT_V, 2052, 4096, wb.value,
                                  None) == wilson.WL_EALIGN  # dots not 8-byte aligned
        # the allocation-free variant rejects sizes beyond its scratch array before any launch
        big = ctypes.c_void_p()
        gb = wilson.make_geom((32, 32, 32, 64))
        assert L.wl_op_create(ctypes.byref(gb), 0.12, wilson.WL_F16S, 256, ctypes.byref(big)) == wilson.WL_OK
        try:
            assert L.wl_apply_dot_workspace_bytes(big, 16, ctypes.byref(wb)) == wilson.WL_OK
            assert wb.value > 16 << 20
            assert L.wilson_apply_dot_noalloc(big, 512, 1024, None, 0, 16, wilson.WL_DOT_NORM, 2048,
                                              None) == wilson.WL_EWORKSPACE
            assert L.wilson_apply_dot_noalloc(big, 512, 1024, None, 0, 1, 9, 2048, None) == wilson.WL_EINVAL
        finally:
            L.wl_op_destroy(big)
        # a solve allocates nothing: no workspace is an error
        prm = wilson.wl_solve_params(tol=1e-10, maxiter=10)
        assert L.solve_bicgstab(op, None, 512, 1024, 1, ctypes.byref(prm), None, None) == wilson.WL_EWORKSPACE
        prm = wilson.wl_solve_params(tol=0.0, maxiter=10)
        assert L.solve_cgnr(op, None, 512, 1024, 1, ctypes.byref(prm), None, None) == wilson.WL_EINVAL
        prm = wilson.wl_solve_params(tol=1e-10, maxiter=10)
        assert L.solve_cgnr(op, op, 512, 1024, 1, ctypes.byref(prm), None, None) == wilson.WL_EPREC
        assert L.solve_cgnr(op, None, 512, 1024, 65, ctypes.byref(prm), None, None) == wilson.WL_EINVAL
        prm = wilson.wl_solve_params(tol=1e-10, maxiter=10, form=2)  # no such iteration form
        assert L.solve_bicgstab(op, None, 512, 1024, 1, ctypes.byref(prm), None, None) == wilson.WL_EINVAL
        # the single-reduction forms take defect correction only
        prm = wilson.wl_solve_params(tol=1e-10, maxiter=10, form=1, reliable=1)
        assert L.solve_bicgstab(op, op, 512, 1024, 1, ctypes.byref(prm), None, None) == wilson.WL_EINVAL
        assert L.wilson_gauge_force(op, 512, 1024, 2048, 3, None) == wilson.WL_EINVAL
        hb = ctypes.c_size_t(0)
        assert L.wl_halo_bytes(op, 2, ctypes.byref(hb)) == wilson.WL_OK
        assert hb.value == 4 * 2 * 12 * 4 * 4 * 4 * 8  # send + receive, 2 faces, 2 RHS, 12 doubles per face site
        assert L.wilson_apply_halo(op, 512, 1024, 0, 2, None, hb.value, None) == wilson.WL_EINVAL
        assert L.wilson_apply_halo(op, 512, 1024, 0, 2, 4096, hb.value - 16, None) == wilson.WL_EWORKSPACE
        assert L.wilson_apply_halo(op, 512, 1024, 0, 2, 4104, hb.value, None) == wilson.WL_EALIGN
        plan = ctypes.c_void_p()
        d = (wilson.wl_multi_desc * 2)(wilson.wl_multi_desc(op, 512, 1024), wilson.wl_multi_desc(op, 2048, 2048))
        assert L.wl_multi_plan_create(d, 2, 0, 1, ctypes.byref(plan)) == wilson.WL_EINVAL  # out == in
        assert L.wl_multi_plan_create(d, 0, 0, 1, ctypes.byref(plan)) == wilson.WL_EINVAL
        assert L.wl_multi_plan_create(d, 1, 2, 1, ctypes.byref(plan)) == wilson.WL_EINVAL  # dagger flag
        assert L.wl_multi_plan_create(d, 1, 0, 0, ctypes.byref(plan)) == wilson.WL_EINVAL  # nrhs
        assert plan.value is None
        assert L.wl_multi_plan_run(None, None) == wilson.WL_EINVAL
        assert L.wl_multi_plan_destroy(None) == wilson.WL_EINVAL
    finally:
        L.wl_op_destroy(op)
    # domain-wall operators
    assert L.wl_dw_op_create(ctypes.byref(g), -1.8, 0.1, 0, 0, 256, ctypes.byref(h)) == wilson.WL_EINVAL  # Ns
    assert L.wl_dw_op_create(ctypes.byref(g), float("inf"), 0.1, 4, 0, 256, ctypes.byref(h)) == wilson.WL_EINVAL
    assert L.wl_dw_op_create(ctypes.byref(g), -1.8, 0.1, 4, 0, 8, ctypes.byref(h)) == wilson.WL_EALIGN
    assert L.wl_dw_op_create(ctypes.byref(g), -1.8, 0.1, 8, 0, 256, ctypes.byref(h)) == wilson.WL_OK
    dw = h.value
    try:
        assert L.wilson_apply(dw, 512, 1024, 0, 8, None) == wilson.WL_EINVAL  # not a Wilson op
        assert L.dwf_apply(dw, 512, 1024, 0, 0, None) == wilson.WL_EINVAL  # nvec
        assert L.dwf_apply(dw, 512, 512, 0, 1, None) == wilson.WL_EINVAL  # in == out
        prm = wilson.wl_solve_params(tol=1e-10, maxiter=10)
        assert L.solve_bicgstab(dw, None, 512, 1024, 1, ctypes.byref(prm), None, None) == wilson.WL_EINVAL
        assert L.solve_cgnr(dw, None, 512, 1024, 9, ctypes.byref(prm), None, None) == wilson.WL_EINVAL  # 72 columns
        c = wilson.wl_launch(block=256, rhs_per_thread=2, rhs_lanes=1, xcd_remap=0, variant=0)
        assert L.wl_set_launch(dw, 1, ctypes.byref(c)) == wilson.WL_EINVAL  # one slice per thread
        c = wilson.wl_launch(block=256, rhs_per_thread=1, rhs_lanes=4, xcd_remap=0, variant=2)
        assert L.wl_set_launch(dw, 1, ctypes.byref(c)) == wilson.WL_EINVAL  # FP64 offers variants 0, 1
        c = wilson.wl_launch(block=512, rhs_per_thread=1, rhs_lanes=8, xcd_remap=0, variant=1)
        assert L.wl_set_launch(dw, 1, ctypes.byref(c)) == wilson.WL_OK
        n = ctypes.c_size_t(0)
        assert L.wl_halo_bytes(dw, 1, ctypes.byref(n)) == wilson.WL_EINVAL  # Wilson ops only
    finally:
        L.wl_op_destroy(dw)
    godd = wilson.make_geom((4, 4, 3, 4))  # even-odd needs every extent even
    assert L.wl_eo_split(ctypes.byref(godd), 0, 1, 256, 512, 768, None) == wilson.WL_EINVAL
    assert L.wl_eo_split(ctypes.byref(g), 0, 1, 256, 512, 512, None) == wilson.WL_EINVAL  # even == odd
    assert L.wl_eo_merge(ctypes.byref(g), 0, 1, 256, 512, 8, None) == wilson.WL_EALIGN
    for c in (0, 1, 2, 3, -1, -2, -3, -4, -5, -6):
        assert L.wl_strerror(c).decode() != "unknown error"


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ missing")
def test_fastdiv_is_exact(tmp_path):
    """The magic-number division used to decode site coordinates (host copy of
    the same header routine, evaluated with 64-bit arithmetic) is exact."""
    src = tmp_path / "fd.cpp"
    src.write_text(r'''
#include <cstdint>
#include <cstdio>
#define __device__
#define __forceinline__ inline
static inline uint32_t __umulhi(uint32_t a, uint32_t b) { return (uint32_t)(((uint64_t)a * b) >> 32); }
''' + "".join(_fastdiv_source()) + r'''
int main() {
  const uint32_t ds[] = {1,2,3,4,5,6,7,8,12,16,20,24,32,48,64,96,100,1000,4096,13824,32768,65535,100000,1u<<20};
  for (uint32_t d : ds) {
    wl::FastDiv f = wl::make_fastdiv(d);
    for (uint64_t n = 0; n < 200000; ++n) if (wl::fdiv((uint32_t)n, f) != n / d) { printf("bad %u %llu\n", d, (unsigned long long)n); return 1; }
    for (uint64_t n = 0x7fffffffull - 200000; n <= 0x7fffffffull; ++n) if (wl::fdiv((uint32_t)n, f) != n / d) { printf("bad %u %llu\n", d, (unsigned long long)n); return 1; }
    for (uint64_t k = 1; k * d < 0x7fffffffull && k < 100000; k += 7) {
      uint64_t n = k * d; if (wl::fdiv((uint32_t)n, f) != k || wl::fdiv((uint32_t)(n - 1), f) != k - 1) { printf("bad %u\n", d); return 1; }
    }
  }
  puts("ok"); return 0;
}
''')
    exe = tmp_path / "fd"
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", str(exe), str(src)], check=True)
    assert subprocess.run([str(exe)], capture_output=True, text=True).stdout.strip() == "ok"


def _fastdiv_source():
    """Extract the FastDiv struct and its two functions from wl_common.h."""
    text = open(os.path.join(ROOT, "paper_1712_01505_amd", "csrc", "wl_common.h")).read()
    start = text.index("struct FastDiv {")
    end = text.index("// ---------------------------------------------------------------- tile order")
    return ["namespace wl {\n", text[start:end], "}\n"]


def test_tune_cache_json_is_read(tmp_path):
    """The launch-shape cache is JSON with one entry per line; a fresh process
    that finds an entry for its (arch, extents, precision, nrhs, dagger,
    reduction) key launches with it (no GPU: the architecture reads as
    "unknown")."""
    import json
    import subprocess
    import sys
    path = tmp_path / "tune.json"
    entry = {"key": "unknown:8x8x8x8:p1:n1:d0:r0", "arch": "unknown", "dims": [8, 8, 8, 8], "prec": 1, "nrhs": 1,
             "dagger": 0, "reduction": 0, "block": 128, "rhs_per_thread": 1, "rhs_lanes": 1, "xcd_remap": 0,
             "variant": 7, "brick": [8, 4, 4], "t_steps": 8, "wg_per_cu": 2, "us": 12.5}
    path.write_text(json.dumps({"format": "wilson launch shapes", "entries": [entry]}, indent=None)
                    .replace("[{", "[\n{").replace("}]", "}\n]") + "\n")
    code = (
        "import ctypes\n"
        "from paper_1712_01505_amd import wilson\n"
        "L = wilson.lib()\n"
        "g = wilson.make_geom((8, 8, 8, 8))\n"
        "op = ctypes.c_void_p()\n"
        "assert L.wl_op_create(ctypes.byref(g), 0.12, wilson.WL_F32, 256, ctypes.byref(op)) == 0\n"
        "c = wilson.wl_launch()\n"
        "assert L.wl_get_launch(op, 1, ctypes.byref(c)) == 0\n"
        "print(c.block, c.variant, tuple(c.brick), c.t_steps, c.wg_per_cu)\n")
    env = dict(os.environ, WL_TUNE_CACHE=str(path))
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120,
                         cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert out.returncode == 0, out.stderr
    assert out.stdout.split() == ["128", "7", "(8,", "4,", "4)", "8", "2"], out.stdout


def test_multi_solve_arguments_rejected():
    """wilson_solve_multi / wl_multi_solver_workspace_bytes reject bad system
    lists before touching the GPU."""
    L = wilson.lib()
    g1, g2 = wilson.make_geom((4, 4, 4, 4)), wilson.make_geom((6, 6, 6, 6))
    ops = []
    try:
        for g, p in ((g1, wilson.WL_F64), (g2, wilson.WL_F64), (g1, wilson.WL_F32), (g2, wilson.WL_F16S)):
            h = ctypes.c_void_p()
            assert L.wl_op_create(ctypes.byref(g), 0.12, p, 256, ctypes.byref(h)) == wilson.WL_OK
            ops.append(h.value)
        f64a, f64b, f32a, f16b = ops
        S = wilson.wl_multi_system
        n = ctypes.c_size_t()
        ok = (S * 2)(S(f64a, None, 512, 1024), S(f64b, None, 2048, 4096))
        assert L.wl_multi_solver_workspace_bytes(ok, 2, 1, 4, ctypes.byref(n)) == wilson.WL_OK and n.value > 0
        assert L.wl_multi_solver_workspace_bytes(ok, 0, 1, 4, ctypes.byref(n)) == wilson.WL_EINVAL
        assert L.wl_multi_solver_workspace_bytes(ok, 2, 1, 33, ctypes.byref(n)) == wilson.WL_EINVAL  # 66 columns
        assert L.wl_multi_solver_workspace_bytes(ok, 2, 2, 1, ctypes.byref(n)) == wilson.WL_EINVAL  # solver id
        mixed_plain = (S * 2)(S(f64a, f32a, 512, 1024), S(f64b, None, 2048, 4096))
        assert L.wl_multi_solver_workspace_bytes(mixed_plain, 2, 1, 1, ctypes.byref(n)) == wilson.WL_EINVAL
        lo_geom = (S * 1)(S(f64b, f32a, 512, 1024))  # lo on another lattice
        assert L.wl_multi_solver_workspace_bytes(lo_geom, 1, 1, 1, ctypes.byref(n)) == wilson.WL_EINVAL
        plain16 = (S * 1)(S(f16b, None, 512, 1024))
        assert L.wl_multi_solver_workspace_bytes(plain16, 1, 1, 1, ctypes.byref(n)) == wilson.WL_EPREC
        prm = wilson.wl_solve_params(tol=1e-10, maxiter=10, eo=1)
        assert L.wilson_solve_multi(ok, 2, 1, 1, ctypes.byref(prm), None, None) == wilson.WL_EINVAL  # no eo
        prm = wilson.wl_solve_params(tol=1e-10, maxiter=10)
        same = (S * 1)(S(f64a, None, 512, 512))
        assert L.wilson_solve_multi(same, 1, 1, 1, ctypes.byref(prm), None, None) == wilson.WL_EINVAL  # x == b
        odd = (S * 1)(S(f64a, None, 520, 1024))
        assert L.wilson_solve_multi(odd, 1, 1, 1, ctypes.byref(prm), None, None) == wilson.WL_EALIGN
        assert L.wilson_solve_multi(ok, 2, 1, 1, ctypes.byref(prm), None, None) == wilson.WL_EWORKSPACE
    finally:
        for h in ops:
            L.wl_op_destroy(h)


def test_profiling_shapes_summary(tmp_path):
    """The per-launch-shape summary pairs dispatches three by three with the
    printed shapes, sums counter rows per dispatch and scales them by the
    copy calibration; a count mismatch is refused."""
    import csv
    import json
    from paper_1712_01505_amd import profiling

    def write(path, rows, fields):
        path.parent.mkdir(parents=True, exist_ok=True)
        with open(path, "w", newline="") as f:
            w = csv.DictWriter(f, fieldnames=fields)
            w.writeheader()
            for r in rows:
                w.writerow(r)

    k = "void wl::stencil_kernel<1, 0, 1, 0, 2, 2>(wl::StencilParams)"
    write(tmp_path / "t" / "s_kernel_trace.csv",
          [{"Dispatch_Id": i, "Kernel_Name": k, "Start_Timestamp": 1000 * i, "End_Timestamp": 1000 * i + 2000}
           for i in range(1, 7)], ["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
    cf = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    for d, c, v in (("f", "FETCH_SIZE", 500.0), ("w", "WRITE_SIZE", 1000.0)):
        # two rows per dispatch (one per XCD, say): summed
        write(tmp_path / d / "s_counter_collection.csv",
              [{"Dispatch_Id": i, "Kernel_Name": k, "Counter_Name": c, "Counter_Value": v} for i in range(1, 7)
               for _ in range(2)], cf)
    for d, c, v in (("cf", "FETCH_SIZE", 512.0), ("cw", "WRITE_SIZE", 1024.0)):
        write(tmp_path / d / "s_counter_collection.csv",
              [{"Dispatch_Id": 1, "Kernel_Name": "void wl::stream_copy_kernel(x)", "Counter_Name": c,
                "Counter_Value": v}], cf)
    log = tmp_path / "case.log"
    log.write_text("".join(json.dumps({"case": f"c{j}", "launch": [256, 1, 1, 2, 1, 0, 0, 0, 0, 0, 0],
                                       "compulsory_read": 1024000, "compulsory_write": 2048000}) + "\n"
                           for j in range(2)))
    out = tmp_path / "out.md"
    profiling.shapes(str(tmp_path / "t"), str(tmp_path / "f"), str(tmp_path / "w"), str(log), str(tmp_path / "cf"),
                     str(tmp_path / "cw"), "1", str(out), "cmd")
    rows = [l for l in out.read_text().splitlines() if l.startswith("| c") and not l.startswith("| case")]
    assert len(rows) == 2
    cells = [x.strip() for x in rows[0].split("|")]
    # 2 us per dispatch; read = 2 x 500 KiB x (1024 / 512) = 2048000 B; write = 2 x 1000 KiB x 1 = 2048000 B
    assert cells[4] == "2.0" and cells[5] == "2" and cells[6] == "2.00" and cells[7] == "2" and cells[8] == "1.00"
    log.write_text(log.read_text().splitlines()[0] + "\n")
    with pytest.raises(SystemExit):
        profiling.shapes(str(tmp_path / "t"), str(tmp_path / "f"), str(tmp_path / "w"), str(log),
                         str(tmp_path / "cf"), str(tmp_path / "cw"), "1", str(out), "cmd")
