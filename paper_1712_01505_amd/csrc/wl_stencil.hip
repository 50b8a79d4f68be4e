// wl_stencil.hip -- the Wilson-Dirac hopping stencil on gfx950, its
// multi-lattice persistent variant and the link-force kernel.
//
// Operator (Kanamori & Matsufuru, Sec. II-B, eq. (1), kappa normalisation):
//   (H psi)(x) = sum_mu [ s+ (1 - g_mu) U_mu(x) psi(x+mu) + s- (1 + g_mu) U_mu(x-mu)^dag psi(x-mu) ]
//   D psi = psi - kappa H psi;   D^dag swaps the projector signs.
// Cost convention (Table I): 1368 flop/site for D, 1320 for H.
//
// Design (bandwidth-bound; no matrix cores: the 3x3 complex mat-vec has
// about 1.8 flop/byte in FP64, far below the machine balance):
//   * one thread per lattice site, R right-hand sides per thread so that a
//     link loaded once serves R spinors;
//   * site-contiguous packed fields: every component load of a wavefront is
//     a contiguous 1 KB (FP64) / 1 KB (FP32, 2 complex) / 1 KB (16-bit, 4 complex);
//   * spin projection: (1 -+ g_mu) has rank 2, so only a 2-spin half-spinor
//     is multiplied by the link and the other two spin rows are rebuilt
//     with 0, +-1, +-i coefficients (chiral basis);
//   * two-row links, row 2 = conj(row0 x row1) rebuilt in registers;
//   * the antiperiodic boundary sign multiplies the hop (never the link,
//     since -U has det -1 and would rebuild a wrong third row);
//   * XCD-aware tile order and fused reductions for the solvers.
#include <type_traits>

#include "wl_brick.h"

namespace wl {

// FP64 with G = 2 and FP32 with G = 4 exceed the register file and spill;
// variants 4-6 (t-walk) and 7 (LDS-staged brick walk) exist for every precision.
int max_var(int prec) { return VAR_BRICK; }
bool var_ok(int prec, int var) { return var <= 1 || var >= 4 || (var == 2 && prec != F64) || (var == 3 && prec >= BF16S); }

bool brick_ok(const int *L, int prec, int bx, int by, int bz, int T, int wpe, int rw)
{
    BrickGeom g{};
    if (!brick_setup(L, prec, bx, by, bz, T, g, rw))
        return false;
    return wpe == 0 ||
           ((wpe == 1 || wpe == 2 || wpe == 4 || wpe == 8) && (size_t)g.stage * rw <= brick_reserve(wpe));
}

bool slab_ok(const int *L, int block, int mode)
{
    if (mode < 2 || mode > 5)
        return false;
    const uint64_t slab = (uint64_t)L[0] * L[1] * (L[2] / 8) * L[3];
    return L[2] % 8 == 0 && L[1] % (1 << (mode - 2)) == 0 && slab % (uint64_t)block == 0;
}

int stencil_nval(int red) { return red_nval(red); }

static uint32_t pad8(uint32_t n) { return (n + 7u) & ~7u; }

// Number of per-workgroup partials (per right-hand side) a launch with this
// configuration writes.
int stencil_partials(const LaunchCfg &cfg, const int *L, uint32_t V, int nrhs)
{
    const uint32_t tile = (uint32_t)(cfg.block / cfg.lanes);
    uint32_t n = (V + tile - 1) / tile;
    if (cfg.rpt == 1 && cfg.var == VAR_BRICK && cfg.bx > 0 && cfg.by > 0 && cfg.bz > 0 && cfg.tsteps > 0) {
        n = (uint32_t)((L[0] / cfg.bx) * (L[1] / cfg.by) * (L[2] / cfg.bz)) * (uint32_t)(L[3] / cfg.tsteps);
    } else if (cfg.rpt == 1 && cfg.var >= 4) {
        const uint32_t nxyz = (uint32_t)L[0] * L[1] * L[2];
        n = ((nxyz + tile - 1) / tile) * (uint32_t)(L[3] / twalk_T(cfg.var));
    }
    return (int)(nrhs / (cfg.rpt * cfg.lanes) > 1 ? pad8(n) : n);
}

int max_rpt(int prec) { return prec == F64 ? 2 : 4; }

hipError_t launch_stencil(int prec, int dagger, const LaunchCfg &cfg, StencilParams p, hipStream_t st)
{
    const int lg = cfg.lanes == 1 ? 0 : cfg.lanes == 2 ? 1 : cfg.lanes == 4 ? 2 : cfg.lanes == 8 ? 3 : -1;
    if (cfg.rpt < 1 || cfg.rpt > 4 || p.nrhs % cfg.rpt != 0 || cfg.block < 64 || cfg.block > 512 ||
        cfg.block % 64 != 0 || lg < 0 ||
        (lg > 0 && (cfg.rpt != 1 || p.nrhs % cfg.lanes != 0 ||
                    (cfg.var != VAR_BRICK && (cfg.block >> lg) < (cfg.var >= 4 ? 32 : 64)))))
        return hipErrorInvalidValue;
    if (p.apply == 2 && (cfg.rpt != 1 || (cfg.var > 2 && cfg.var < 4) || cfg.var > 6 || p.ns < 1 || p.nrhs % p.ns != 0))
        return hipErrorInvalidValue;  // domain wall: one slice per thread, variants 0..2 and the t-walks
    if (p.apply == 3 && (!p.aux || (prec != F64 && prec != F32) || (p.red != RED_NONE && p.red != RED_NORM)))
        return hipErrorInvalidValue;  // residual: FP64 / FP32, with |r|^2 or without
    if (cfg.gmaj != 0 && cfg.gmaj != 1)
        return hipErrorInvalidValue;
    p.lanes_lg = lg;
    p.gmaj = cfg.gmaj;
    const int tile = cfg.block >> lg;
    p.nblk = (int)((p.V + tile - 1) / tile);
    p.xcd = cfg.xcd;
    p.one = 1.0f;
    if (p.xcd >= 2 && !(cfg.rpt == 1 && cfg.var >= 4)) {  // the t-walk kernels use modes 0 / 1 only
        if (!slab_ok(p.L, tile, p.xcd))
            return hipErrorInvalidValue;
        const uint32_t Lx = (uint32_t)p.L[0], Ly = (uint32_t)p.L[1], Lz = (uint32_t)p.L[2], Lt = (uint32_t)p.L[3];
        const uint32_t yc = Ly >> (p.xcd - 2);
        SlabOrder &o = p.slab;
        o.zs = Lz / 8;
        o.plane_n = Lx * yc;
        o.slice_n = o.plane_n * o.zs;
        o.chunk_n = o.slice_n * Lt;
        o.xy = Lx * Ly;
        o.vslice = o.xy * Lz;
        o.f_chunk = make_fastdiv(o.chunk_n);
        o.f_slice = make_fastdiv(o.slice_n);
        o.f_plane = make_fastdiv(o.plane_n);
    }
    switch (prec) {
    case F64: return launch_stencil_p<F64>(dagger, cfg, p, st);
    case F32: return launch_stencil_p<F32>(dagger, cfg, p, st);
    case BF16S: return launch_stencil_p<BF16S>(dagger, cfg, p, st);
    case F16S: return launch_stencil_p<F16S>(dagger, cfg, p, st);
    default: return hipErrorInvalidValue;
    }
}

// Multi-lattice launch shapes: R in {1, 2, 4} (FP64: 1, 2); R = 1 takes the
// pipelined code variants 1..3 where the precision offers them.
static bool multi_shape_ok(int prec, int rpt, int var)
{
    if (rpt != 1 && rpt != 2 && rpt != 4)
        return false;
    if (prec == F64 && rpt == 4)
        return false;
    if (rpt > 1)
        return var == 0;
    return var >= 0 && var <= 3 && var_ok(prec, var);
}

static const void *multi_kernel_ptr(int prec, int dagger, int rpt, int var, bool persistent)
{
    if (!multi_shape_ok(prec, rpt, var))
        return nullptr;
    switch (prec) {
    case F64: return multi_kernel_p<F64>(dagger, rpt, var, persistent);
    case F32: return multi_kernel_p<F32>(dagger, rpt, var, persistent);
    case BF16S: return multi_kernel_p<BF16S>(dagger, rpt, var, persistent);
    case F16S: return multi_kernel_p<F16S>(dagger, rpt, var, persistent);
    default: return nullptr;
    }
}

bool multi_launch_ok(int prec, int rpt, int block, int var)
{
    return block >= 64 && block <= 512 && block % 64 == 0 && multi_shape_ok(prec, rpt, var);
}

// Resident workgroups for a full machine: occupancy per CU x CUs.
int multi_grid_size(int prec, int dagger, int rpt, int block, int var)
{
    const void *fn = multi_kernel_ptr(prec, dagger, rpt, var, true);
    if (!fn)
        return 0;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, 0) != hipSuccess)
        per_cu = 1;
    int dev = 0, ncu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    return (per_cu < 1 ? 1 : per_cu) * (ncu < 1 ? 1 : ncu);
}

hipError_t launch_multi(int prec, int dagger, int rpt, int block, int var, const MultiEntry *E, int n,
                        uint32_t total, unsigned *counter, int grid, hipStream_t st)
{
    // grid > 0: persistent form with that many workgroups; grid == 0: one
    // workgroup per item
    const bool persistent = grid > 0;
    const void *fn = multi_kernel_ptr(prec, dagger, rpt, var, persistent);
    if (!fn || total == 0)
        return hipErrorInvalidValue;
    if (persistent) {
        void *args[] = {(void *)&E, (void *)&n, (void *)&total, (void *)&counter};
        return hipLaunchKernel(fn, dim3(grid), dim3(block), args, 0, st);
    }
    void *args[] = {(void *)&E, (void *)&n, (void *)&total};
    return hipLaunchKernel(fn, dim3(total), dim3(block), args, 0, st);
}

// ---------------------------------------------------------------- enforced halo
// The paper's single-node mode with the boundary copy enforced (Sec. IV): the
// lattice is treated as one rank of a t-decomposition whose neighbours are
// itself.  halo_pack writes, per face site j (Vs = Lx Ly Lz sites per slice),
//   face 0: the projected half-spinor of the t = 0 slice that the forward t
//           hop of t = Lt-1 needs (the receiver multiplies by its link), and
//   face 1: U_t^dag times the projected half-spinor of the t = Lt-1 slice, the
//           whole backward t hop of t = 0 (the sender owns that link);
// a device copy moves them to the receive buffer (on several GPUs: the
// exchange with the t neighbours), and halo_finish adds the received hops to
// the boundary slices of an output the stencil computed with those hops cut.
template <int P>
using HaloReal = typename std::conditional<P == F64, double, float>::type;

size_t halo_face_bytes(int prec, uint32_t vs, int nrhs)
{
    const size_t real = prec == F64 ? 8 : 4;
    return (size_t)nrhs * 12 * vs * real;
}

template <int P, int DAG>
__global__ __launch_bounds__(256) void halo_pack_kernel(StencilParams p)
{
    using T = typename Traits<P>::real;
    using H = HaloReal<P>;
    constexpr int SF = DAG ? 1 : -1;
    const uint32_t vs = (uint32_t)p.L[0] * p.L[1] * p.L[2];
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    const int face = blockIdx.y, rhs = blockIdx.z;
    if (j >= vs)
        return;
    const uint32_t s = face == 0 ? j : j + (uint32_t)(p.L[3] - 1) * vs;
    cx<T> ps[12], h[6], g[6];
    load_site<P>(p.in, p.V, p.nrhs, s, rhs, ps);
    if (face == 0) {
        project<3, SF>(ps, h, (T)1);  // the forward t hop's projection
#pragma unroll
        for (int k = 0; k < 6; ++k)
            g[k] = h[k];
    } else {
        project<3, -SF>(ps, h, (T)1);  // the backward t hop: U_t(s)^dag (projected)
        cx<T> u[9];
        load_link<P>(p.U, p.V, 3, s, u);
        su3_adj_mv(u, h, g);
    }
    H *b = reinterpret_cast<H *>(p.halo_send) + ((size_t)(face * p.nrhs + rhs) * 12) * vs;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        b[(size_t)(2 * k) * vs + j] = (H)g[k].re;
        b[(size_t)(2 * k + 1) * vs + j] = (H)g[k].im;
    }
}

template <int P, int DAG>
__global__ __launch_bounds__(256) void halo_finish_kernel(StencilParams p)
{
    using T = typename Traits<P>::real;
    using H = HaloReal<P>;
    constexpr int SF = DAG ? 1 : -1;
    const uint32_t vs = (uint32_t)p.L[0] * p.L[1] * p.L[2];
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    const int face = blockIdx.y, rhs = blockIdx.z;
    if (j >= vs)
        return;
    const H *b = reinterpret_cast<const H *>(p.halo_recv) + ((size_t)(face * p.nrhs + rhs) * 12) * vs;
    cx<T> h[6];
#pragma unroll
    for (int k = 0; k < 6; ++k)
        h[k] = cx<T>{(T)b[(size_t)(2 * k) * vs + j], (T)b[(size_t)(2 * k + 1) * vs + j]};
    const T sg = p.bc[3] < 0 ? T(-1) : T(1);  // both faces' hops wrap around the lattice
    cx<T> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k)
        acc[k] = cx<T>{T(0), T(0)};
    uint32_t s;
    if (face == 0) {  // received t = 0 half-spinors: the forward hop of t = Lt-1
        s = j + (uint32_t)(p.L[3] - 1) * vs;
        cx<T> u[9], g[6];
        load_link<P>(p.U, p.V, 3, s, u);
        su3_mv(u, h, g);
        accum<3, SF>(acc, g, sg);
    } else {  // received backward hops into t = 0
        s = j;
        accum<3, -SF>(acc, h, sg);
    }
    cx<T> o[12];
    load_site<P>(p.out, p.V, p.nrhs, s, rhs, o);
    const T c = p.apply ? -(T)p.kappa : T(1);  // D: out = in - kappa H in;  H alone: out = H in
#pragma unroll
    for (int k = 0; k < 12; ++k)
        o[k] = cx<T>{fma(c, acc[k].re, o[k].re), fma(c, acc[k].im, o[k].im)};
    store_site_q<P>(p.out, p.V, p.nrhs, s, rhs, o);
}

template <int DAG>
static hipError_t halo_launch(int prec, bool finish, const StencilParams &p, hipStream_t st)
{
    const uint32_t vs = (uint32_t)p.L[0] * p.L[1] * p.L[2];
    dim3 g((vs + 255) / 256, 2, p.nrhs), b(256);
    switch (prec) {
    case F64:
        if (finish) hipLaunchKernelGGL((halo_finish_kernel<F64, DAG>), g, b, 0, st, p);
        else hipLaunchKernelGGL((halo_pack_kernel<F64, DAG>), g, b, 0, st, p);
        break;
    case F32:
        if (finish) hipLaunchKernelGGL((halo_finish_kernel<F32, DAG>), g, b, 0, st, p);
        else hipLaunchKernelGGL((halo_pack_kernel<F32, DAG>), g, b, 0, st, p);
        break;
    case BF16S:
        if (finish) hipLaunchKernelGGL((halo_finish_kernel<BF16S, DAG>), g, b, 0, st, p);
        else hipLaunchKernelGGL((halo_pack_kernel<BF16S, DAG>), g, b, 0, st, p);
        break;
    case F16S:
        if (finish) hipLaunchKernelGGL((halo_finish_kernel<F16S, DAG>), g, b, 0, st, p);
        else hipLaunchKernelGGL((halo_pack_kernel<F16S, DAG>), g, b, 0, st, p);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_halo_pack(int prec, int dagger, const StencilParams &p, hipStream_t st)
{
    return dagger ? halo_launch<1>(prec, false, p, st) : halo_launch<0>(prec, false, p, st);
}

hipError_t launch_halo_finish(int prec, int dagger, const StencilParams &p, hipStream_t st)
{
    return dagger ? halo_launch<1>(prec, true, p, st) : halo_launch<0>(prec, true, p, st);
}

// ---------------------------------------------------------------- link force
// For each link (x, mu): G = kappa s_mu(x) [ sum_spin ((1-g_mu) x(x+mu)) mu(x)^dag
//                                           + sum_spin mu(x+mu) ((1+g_mu) x(x))^dag ],
// the derivative of Re<mu, D x> style terms with respect to U_mu(x)
// (dL = Re Tr[dU G]); written out as G^dag or as P = TH(i U G).
template <int P, int MU>
__device__ __forceinline__ void force_dir(const StencilParams &p, uint32_t s, int c, uint32_t stride,
                                          double2 *out, int want_p)
{
    using T = typename Traits<P>::real;
    const int L = p.L[MU];
    const bool wf = (c == L - 1);
    const uint32_t sf = wf ? s - (uint32_t)(L - 1) * stride : s + stride;
    const double sg = (wf && p.bc[MU] < 0) ? -1.0 : 1.0;
    cx<T> xf[12], xs[12], mf[12], ms[12];
    load_site<P>(p.in, p.V, 1, sf, 0, xf);
    load_site<P>(p.in, p.V, 1, s, 0, xs);
    load_site<P>(p.aux, p.V, 1, sf, 0, mf);
    load_site<P>(p.aux, p.V, 1, s, 0, ms);
    // v = (1 - g) x(x+mu), w = (1 + g) x(x): projected then expanded to 4 spins
    cx<T> h[6], v[12], w[12];
#pragma unroll
    for (int k = 0; k < 12; ++k)
        v[k] = w[k] = cx<T>{T(0), T(0)};
    project<MU, -1>(xf, h);
    accum<MU, -1>(v, h, T(1));
    project<MU, 1>(xs, h);
    accum<MU, 1>(w, h, T(1));
    cx<double> G[9];
    const double kf = p.kappa * sg;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            cx<double> acc{0.0, 0.0};
#pragma unroll
            for (int sp = 0; sp < 4; ++sp) {
                const cx<double> va{(double)v[3 * sp + a].re, (double)v[3 * sp + a].im};
                const cx<double> mb{(double)ms[3 * sp + b].re, (double)ms[3 * sp + b].im};
                const cx<double> fa{(double)mf[3 * sp + a].re, (double)mf[3 * sp + a].im};
                const cx<double> wb{(double)w[3 * sp + b].re, (double)w[3 * sp + b].im};
                acc = cfma(va, cconj(mb), acc);
                acc = cfma(fa, cconj(wb), acc);
            }
            G[3 * a + b] = cx<double>{kf * acc.re, kf * acc.im};
        }
    double2 *o = out + ((size_t)MU * p.V + s) * 9;
    if (!want_p) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
                o[3 * a + b] = make_double2(G[3 * b + a].re, -G[3 * b + a].im);
        return;
    }
    cx<T> ut[9];
    load_link<P>(p.U, p.V, MU, s, ut);
    cx<double> A[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            cx<double> acc{0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; ++k)
                acc = cfma(cx<double>{(double)ut[3 * a + k].re, (double)ut[3 * a + k].im}, G[3 * k + b], acc);
            A[3 * a + b] = cx<double>{-acc.im, acc.re};  // i U G
        }
    // P = (A + A^dag)/2 - Tr[(A + A^dag)/2]/3
    const double tr = (A[0].re + A[4].re + A[8].re) / 3.0;
    cx<double> Pm[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            double re = 0.5 * (A[3 * a + b].re + A[3 * b + a].re);
            double im = 0.5 * (A[3 * a + b].im - A[3 * b + a].im);
            if (a == b)
                re -= tr;
            Pm[3 * a + b] = cx<double>{re, im};
        }
    if (want_p == 1) {
#pragma unroll
        for (int k = 0; k < 9; ++k)
            o[k] = make_double2(Pm[k].re, Pm[k].im);
        return;
    }
    // tangent gradient i P U
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            cx<double> acc{0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; ++k)
                acc = cfma(Pm[3 * a + k], cx<double>{(double)ut[3 * k + b].re, (double)ut[3 * k + b].im}, acc);
            o[3 * a + b] = make_double2(-acc.im, acc.re);
        }
}

template <int P>
__global__ __launch_bounds__(256) void force_kernel(StencilParams p, double2 *out, int want_p)
{
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= p.V)
        return;
    const uint32_t q1 = fdiv(s, p.fx);
    const int x = (int)(s - q1 * (uint32_t)p.L[0]);
    const uint32_t q2 = fdiv(q1, p.fy);
    const int y = (int)(q1 - q2 * (uint32_t)p.L[1]);
    const uint32_t q3 = fdiv(q2, p.fz);
    const int z = (int)(q2 - q3 * (uint32_t)p.L[2]);
    const int t = (int)q3;
    const uint32_t sy = (uint32_t)p.L[0], sz = sy * (uint32_t)p.L[1], st = sz * (uint32_t)p.L[2];
    force_dir<P, 0>(p, s, x, 1u, out, want_p);
    force_dir<P, 1>(p, s, y, sy, out, want_p);
    force_dir<P, 2>(p, s, z, sz, out, want_p);
    force_dir<P, 3>(p, s, t, st, out, want_p);
}

hipError_t launch_force(int prec, const wl_op *op, void *out, const void *x, const void *mu, int project,
                        hipStream_t st)
{
    StencilParams p{};
    p.U = op->U;
    p.in = x;
    p.aux = mu;
    p.V = op->V;
    p.nrhs = 1;
    p.kappa = op->kappa;
    for (int i = 0; i < 4; ++i) {
        p.L[i] = op->g.dims[i];
        p.bc[i] = op->g.bc[i];
    }
    p.fx = make_fastdiv((uint32_t)p.L[0]);
    p.fy = make_fastdiv((uint32_t)p.L[1]);
    p.fz = make_fastdiv((uint32_t)p.L[2]);
    const int block = 256;
    dim3 grid((p.V + block - 1) / block);
    if (prec == F64)
        hipLaunchKernelGGL((force_kernel<F64>), grid, dim3(block), 0, st, p, (double2 *)out, project);
    else if (prec == F32)
        hipLaunchKernelGGL((force_kernel<F32>), grid, dim3(block), 0, st, p, (double2 *)out, project);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace wl
