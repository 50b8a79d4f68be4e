// wl_blas.hip -- fused BLAS-1 updates, deterministic reductions and the
// on-device scalar steps of CGNR and BiCGStab.
//
// The paper composes its solvers from a BLAS-like library (Sec. V-C) and
// finds that these streaming updates and their global reductions, not the
// stencil, limit the solver.  Here each solver step that touches vectors is
// one fused kernel (several axpy-type updates plus the norms/dots the next
// step needs), each reduction is a fixed-order two-stage sum (wavefront
// shuffles and LDS into per-workgroup partials, then one workgroup sums the
// partials in index order), and the scalar recurrences (alpha, beta, omega,
// rho, convergence) run on the device so the host only polls occasionally.
//
// Inner product <a, b> = sum conj(a_i) b_i; norms and dots accumulate in FP64.
#include "wl_internal.h"

namespace wl {

template <typename T>
__device__ __forceinline__ double n2(const cx<T> (&v)[12])
{
    double a = 0.0;
#pragma unroll
    for (int k = 0; k < 12; ++k)
        a = fma((double)v[k].re, (double)v[k].re, fma((double)v[k].im, (double)v[k].im, a));
    return a;
}
template <typename T>
__device__ __forceinline__ void dot(const cx<T> (&a)[12], const cx<T> (&b)[12], double &re, double &im)
{
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        re = fma((double)a[k].re, (double)b[k].re, fma((double)a[k].im, (double)b[k].im, re));
        im = fma((double)a[k].re, (double)b[k].im, fma(-(double)a[k].im, (double)b[k].re, im));
    }
}

template <int P>
__device__ __forceinline__ void round_if_scaled(cx<typename Traits<P>::real> (&v)[12])
{
    if constexpr (Traits<P>::SCALED) {
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < 12; ++k)
            m = fmaxf(m, fmaxf(fabsf(v[k].re), fabsf(v[k].im)));
        const float inv = m > 0.f ? 1.0f / m : 0.f;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            cx<float> q = unpack2<P>(pack2<P>(v[k].re * inv, v[k].im * inv));
            v[k] = cx<float>{q.re * m, q.im * m};
        }
    }
}

// values reduced by each op, and sites per thread (ops with many reduced
// values cover more sites per workgroup, so that the finalize reads fewer
// partial sums)
__host__ __device__ constexpr int blas_nv(int op)
{
    return (op == B_RES || op == B_CG_XR || op == B_NORM || op == B_BI_XRP || op == B_CG1 || op == B_SR_XR ||
            op == B_INIT)                                                                                   ? 1
           : (op == B_BI_XR || op == B_DOT_NORM)                                                           ? 3
           : op == B_SR_PV                                                                                 ? 9
                                                                                                           : 0;
}
__host__ __device__ constexpr int blas_spt(int op) { return op == B_SR_PV ? 4 : 1; }

template <int P, int OP>
__global__ __launch_bounds__(256) void blas_kernel(BlasParams p)
{
    using T = typename Traits<P>::real;
    constexpr int NV = blas_nv(OP);
    constexpr int NA = NV > 0 ? NV : 1;
    __shared__ double lds[NA * 4];
    // one column per blockIdx.y; segmented vectors: that column's lattice
    // segment (its sites, columns and offset into every buffer)
    const int col = blockIdx.y;
    uint32_t V = p.V;
    int nr = p.nrhs, r = col;
    size_t off = 0;
    if (p.seg) {
        const Seg g = p.seg[col];
        V = g.V;
        nr = g.nrhs;
        r = g.r;
        off = g.off;
    }
    void *const Y0 = p.y0 ? (char *)p.y0 + off : nullptr, *const Y1 = p.y1 ? (char *)p.y1 + off : nullptr;
    void *const Y2 = p.y2 ? (char *)p.y2 + off : nullptr, *const Y3 = p.y3 ? (char *)p.y3 + off : nullptr;
    const void *const A0 = p.a0 ? (const char *)p.a0 + off : nullptr;
    const void *const A1 = p.a1 ? (const char *)p.a1 + off : nullptr;
    const void *const A2 = p.a2 ? (const char *)p.a2 + off : nullptr;
    const void *const A3 = p.a3 ? (const char *)p.a3 + off : nullptr;
    if (p.skip_frozen && p.sc[col].frozen)  // whole workgroup
        return;
    if (OP == B_CG_RESTART && !p.sc[col].restart)
        return;
    double red[NA] = {};
    for (int j = 0; j < blas_spt(OP); ++j) {
    const uint32_t s = (blockIdx.x * blas_spt(OP) + j) * blockDim.x + threadIdx.x;
    if (s < V) {
        const Scalars &sc = p.sc[col];
        if constexpr (OP == B_RES) {  // r = b - w
            cx<T> b[12], w[12], o[12];
            load_site<P>(A0, V, nr, s, r, b);
            load_site<P>(A1, V, nr, s, r, w);
#pragma unroll
            for (int k = 0; k < 12; ++k)
                o[k] = cx<T>{b[k].re - w[k].re, b[k].im - w[k].im};
            round_if_scaled<P>(o);
            store_site<P>(Y0, V, nr, s, r, o);
            red[0] += n2(o);
        } else if constexpr (OP == B_CG_XR) {  // x += a p ; r -= a w
            const T a = (T)sc.alpha.x;
            cx<T> x[12], rr[12], pp[12], w[12];
            load_site<P>(Y0, V, nr, s, r, x);
            load_site<P>(Y1, V, nr, s, r, rr);
            load_site<P>(A0, V, nr, s, r, pp);
            load_site<P>(A1, V, nr, s, r, w);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                x[k] = rfma(a, pp[k], x[k]);
                rr[k] = rfma(-a, w[k], rr[k]);
            }
            round_if_scaled<P>(rr);
            store_site<P>(Y0, V, nr, s, r, x);
            store_site<P>(Y1, V, nr, s, r, rr);
            red[0] += n2(rr);
        } else if constexpr (OP == B_CG_P) {  // p = z + beta p
            const T b = (T)sc.beta.x;
            cx<T> pp[12], z[12];
            load_site<P>(Y0, V, nr, s, r, pp);
            load_site<P>(A0, V, nr, s, r, z);
#pragma unroll
            for (int k = 0; k < 12; ++k)
                pp[k] = rfma(b, pp[k], z[k]);
            store_site<P>(Y0, V, nr, s, r, pp);
        } else if constexpr (OP == B_BI_P) {  // p = r + beta (p - omega v)
            const cx<T> b{(T)sc.beta.x, (T)sc.beta.y}, om{(T)sc.omega.x, (T)sc.omega.y};
            cx<T> pp[12], rr[12], v[12];
            load_site<P>(Y0, V, nr, s, r, pp);
            load_site<P>(A0, V, nr, s, r, rr);
            load_site<P>(A1, V, nr, s, r, v);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                cx<T> d = cfma(cx<T>{-om.re, -om.im}, v[k], pp[k]);
                pp[k] = cfma(b, d, rr[k]);
            }
            store_site<P>(Y0, V, nr, s, r, pp);
        } else if constexpr (OP == B_BI_S) {  // s = r - alpha v (|s|^2 comes with t = D s)
            const cx<T> a{(T)sc.alpha.x, (T)sc.alpha.y};
            cx<T> rr[12], v[12];
            load_site<P>(A0, V, nr, s, r, rr);
            load_site<P>(A1, V, nr, s, r, v);
#pragma unroll
            for (int k = 0; k < 12; ++k)
                rr[k] = cfma(cx<T>{-a.re, -a.im}, v[k], rr[k]);
            store_site<P>(Y0, V, nr, s, r, rr);
        } else if constexpr (OP == B_CG1) {
            // p = z + beta p ; w = q + beta w ; x += alpha p ; r -= alpha w
            const T a = (T)sc.alpha.x, b = (T)sc.beta.x;
            cx<T> x[12], rr[12], pp[12], w[12], z[12], q[12];
            load_site<P>(Y2, V, nr, s, r, pp);
            load_site<P>(Y3, V, nr, s, r, w);
            load_site<P>(A0, V, nr, s, r, z);
            load_site<P>(A1, V, nr, s, r, q);
            load_site<P>(Y0, V, nr, s, r, x);
            load_site<P>(Y1, V, nr, s, r, rr);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                pp[k] = rfma(b, pp[k], z[k]);
                w[k] = rfma(b, w[k], q[k]);
            }
            // the stored p and w are what the next iteration reads
            round_if_scaled<P>(pp);
            round_if_scaled<P>(w);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                x[k] = rfma(a, pp[k], x[k]);
                rr[k] = rfma(-a, w[k], rr[k]);
            }
            round_if_scaled<P>(rr);
            store_site<P>(Y2, V, nr, s, r, pp);
            store_site<P>(Y3, V, nr, s, r, w);
            store_site<P>(Y0, V, nr, s, r, x);
            store_site<P>(Y1, V, nr, s, r, rr);
            red[0] += n2(rr);
        } else if constexpr (OP == B_SR_PV) {
            // p = r + beta (p - omega v) ; v = u + beta (v - omega q) ; then
            // <rh, v>, <rh, u>, <u, r>, <u, v>, |u|^2 of the stored values
            const cx<T> b{(T)sc.beta.x, (T)sc.beta.y}, om{(T)sc.omega.x, (T)sc.omega.y};
            const cx<T> mom{-om.re, -om.im};
            cx<T> pp[12], v[12], rr[12], u[12], q[12];
            load_site<P>(Y0, V, nr, s, r, pp);
            load_site<P>(Y1, V, nr, s, r, v);
            load_site<P>(A0, V, nr, s, r, rr);
            load_site<P>(A1, V, nr, s, r, u);
            load_site<P>(A2, V, nr, s, r, q);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                pp[k] = cfma(b, cfma(mom, v[k], pp[k]), rr[k]);
                v[k] = cfma(b, cfma(mom, q[k], v[k]), u[k]);
            }
            round_if_scaled<P>(v);
            store_site<P>(Y0, V, nr, s, r, pp);
            store_site<P>(Y1, V, nr, s, r, v);
            cx<T> rh[12];
            load_site<P>(A3, V, nr, s, r, rh);
            dot(rh, v, red[0], red[1]);
            dot(rh, u, red[2], red[3]);
            dot(u, rr, red[4], red[5]);
            dot(u, v, red[6], red[7]);
            red[8] += n2(u);
        } else if constexpr (OP == B_SR_XR) {
            // s = r - alpha v ; x += alpha p + omega s ; r = s - omega (u - alpha q)
            const cx<T> a{(T)sc.alpha.x, (T)sc.alpha.y}, om{(T)sc.omega.x, (T)sc.omega.y};
            const cx<T> ma{-a.re, -a.im}, mom{-om.re, -om.im};
            cx<T> x[12], rr[12], pp[12], v[12];
            load_site<P>(Y0, V, nr, s, r, x);
            load_site<P>(Y1, V, nr, s, r, rr);
            load_site<P>(A0, V, nr, s, r, pp);
            load_site<P>(A1, V, nr, s, r, v);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                rr[k] = cfma(ma, v[k], rr[k]);  // s
                x[k] = cfma(a, pp[k], x[k]);
                x[k] = cfma(om, rr[k], x[k]);
            }
            cx<T> u[12], q[12];
            load_site<P>(A2, V, nr, s, r, u);
            load_site<P>(A3, V, nr, s, r, q);
#pragma unroll
            for (int k = 0; k < 12; ++k)
                rr[k] = cfma(mom, cfma(ma, q[k], u[k]), rr[k]);
            round_if_scaled<P>(rr);
            store_site<P>(Y0, V, nr, s, r, x);
            store_site<P>(Y1, V, nr, s, r, rr);
            red[0] += n2(rr);
        } else if constexpr (OP == B_BI_XR) {  // x += alpha p + omega s ; r = s - omega t
            const cx<T> a{(T)sc.alpha.x, (T)sc.alpha.y}, om{(T)sc.omega.x, (T)sc.omega.y};
            cx<T> x[12], pp[12], ss[12], t[12];
            load_site<P>(Y0, V, nr, s, r, x);
            load_site<P>(A0, V, nr, s, r, pp);
            load_site<P>(A1, V, nr, s, r, ss);
            load_site<P>(A2, V, nr, s, r, t);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                x[k] = cfma(a, pp[k], x[k]);
                x[k] = cfma(om, ss[k], x[k]);
                ss[k] = cfma(cx<T>{-om.re, -om.im}, t[k], ss[k]);
            }
            round_if_scaled<P>(ss);
            store_site<P>(Y0, V, nr, s, r, x);
            store_site<P>(Y1, V, nr, s, r, ss);
            red[0] += n2(ss);
            cx<T> rh[12];
            load_site<P>(A3, V, nr, s, r, rh);
            dot(rh, ss, red[1], red[2]);
        } else if constexpr (OP == B_BI_XRP) {
            // B_BI_XR and the next B_BI_P in one pass (beta is known before r
            // is formed, see F_BI_OMEGA_RHO); p' is formed from the r that is
            // stored, as a separate B_BI_P would load it
            const cx<T> a{(T)sc.alpha.x, (T)sc.alpha.y}, om{(T)sc.omega.x, (T)sc.omega.y};
            const cx<T> b{(T)sc.beta.x, (T)sc.beta.y};
            cx<T> x[12], pp[12], ss[12], t[12];
            load_site<P>(Y0, V, nr, s, r, x);
            load_site<P>(Y2, V, nr, s, r, pp);
            load_site<P>(A1, V, nr, s, r, ss);
            load_site<P>(A2, V, nr, s, r, t);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                x[k] = cfma(a, pp[k], x[k]);
                x[k] = cfma(om, ss[k], x[k]);
                ss[k] = cfma(cx<T>{-om.re, -om.im}, t[k], ss[k]);
            }
            round_if_scaled<P>(ss);
            store_site<P>(Y0, V, nr, s, r, x);
            store_site<P>(Y1, V, nr, s, r, ss);
            red[0] += n2(ss);
            cx<T> v[12];
            load_site<P>(A3, V, nr, s, r, v);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                const cx<T> d = cfma(cx<T>{-om.re, -om.im}, v[k], pp[k]);
                pp[k] = cfma(b, d, ss[k]);
            }
            store_site<P>(Y2, V, nr, s, r, pp);
        } else if constexpr (OP == B_COPY) {
            cx<T> v[12];
            load_site<P>(A0, V, nr, s, r, v);
            store_site<P>(Y0, V, nr, s, r, v);
        } else if constexpr (OP == B_ZERO) {
            cx<T> v[12];
#pragma unroll
            for (int k = 0; k < 12; ++k)
                v[k] = cx<T>{T(0), T(0)};
            store_site<P>(Y0, V, nr, s, r, v);
        } else if constexpr (OP == B_INIT) {  // x = 0 ; r (and y2, y3) = b ; |b|^2
            cx<T> v[12], z[12];
            load_site<P>(A0, V, nr, s, r, v);
#pragma unroll
            for (int k = 0; k < 12; ++k)
                z[k] = cx<T>{T(0), T(0)};
            store_site<P>(Y0, V, nr, s, r, z);
            store_site<P>(Y1, V, nr, s, r, v);
            if (Y2)
                store_site<P>(Y2, V, nr, s, r, v);
            if (Y3)
                store_site<P>(Y3, V, nr, s, r, v);
            red[0] += n2(v);
        } else if constexpr (OP == B_NORM) {
            cx<T> v[12];
            load_site<P>(A0, V, nr, s, r, v);
            red[0] += n2(v);
        } else if constexpr (OP == B_CG_RESTART) {  // p = z
            cx<T> v[12];
            load_site<P>(A0, V, nr, s, r, v);
            store_site<P>(Y0, V, nr, s, r, v);
        } else if constexpr (OP == B_DOT_NORM) {
            cx<T> a[12], b[12];
            load_site<P>(A0, V, nr, s, r, a);
            load_site<P>(A1, V, nr, s, r, b);
            dot(a, b, red[0], red[1]);
            red[2] += n2(b);
        }
    }
    }
    if constexpr (NV > 0) {
        block_sum<NV>(red, lds);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < NV; ++k)
                p.partials[((size_t)k * gridDim.y + col) * p.nblk + blockIdx.x] = red[k];
        }
    }
}

int blas_nval(int op) { return blas_nv(op); }
int blas_sites_per_thread(int op) { return blas_spt(op); }

template <int P>
static hipError_t launch_blas_p(int op, const BlasParams &p, dim3 g, dim3 b, hipStream_t st)
{
    switch (op) {
    case B_RES: hipLaunchKernelGGL((blas_kernel<P, B_RES>), g, b, 0, st, p); break;
    case B_CG_XR: hipLaunchKernelGGL((blas_kernel<P, B_CG_XR>), g, b, 0, st, p); break;
    case B_CG_P: hipLaunchKernelGGL((blas_kernel<P, B_CG_P>), g, b, 0, st, p); break;
    case B_BI_P: hipLaunchKernelGGL((blas_kernel<P, B_BI_P>), g, b, 0, st, p); break;
    case B_BI_S: hipLaunchKernelGGL((blas_kernel<P, B_BI_S>), g, b, 0, st, p); break;
    case B_BI_XR: hipLaunchKernelGGL((blas_kernel<P, B_BI_XR>), g, b, 0, st, p); break;
    case B_COPY: hipLaunchKernelGGL((blas_kernel<P, B_COPY>), g, b, 0, st, p); break;
    case B_ZERO: hipLaunchKernelGGL((blas_kernel<P, B_ZERO>), g, b, 0, st, p); break;
    case B_NORM: hipLaunchKernelGGL((blas_kernel<P, B_NORM>), g, b, 0, st, p); break;
    case B_DOT_NORM: hipLaunchKernelGGL((blas_kernel<P, B_DOT_NORM>), g, b, 0, st, p); break;
    case B_CG_RESTART: hipLaunchKernelGGL((blas_kernel<P, B_CG_RESTART>), g, b, 0, st, p); break;
    case B_BI_XRP: hipLaunchKernelGGL((blas_kernel<P, B_BI_XRP>), g, b, 0, st, p); break;
    case B_CG1: hipLaunchKernelGGL((blas_kernel<P, B_CG1>), g, b, 0, st, p); break;
    case B_SR_PV: hipLaunchKernelGGL((blas_kernel<P, B_SR_PV>), g, b, 0, st, p); break;
    case B_SR_XR: hipLaunchKernelGGL((blas_kernel<P, B_SR_XR>), g, b, 0, st, p); break;
    case B_INIT: hipLaunchKernelGGL((blas_kernel<P, B_INIT>), g, b, 0, st, p); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// One workgroup per `block` sites and column.  (A grid-stride variant capped
// at 2048 workgroups, which shrinks the finalize's input, measured slower
// overall: the streaming kernels lost more than the finalize gained.)
int blas_partials(uint32_t V, int op, int block)
{
    const uint32_t per = (uint32_t)block * (uint32_t)blas_spt(op);
    return (int)((V + per - 1) / per);
}

hipError_t launch_blas(int prec, int op, const BlasParams &p0, int block, hipStream_t st)
{
    BlasParams p = p0;
    p.nblk = blas_partials(p.V, op, block);
    dim3 g(p.nblk, p.nrhs), b(block);
    switch (prec) {
    case F64: return launch_blas_p<F64>(op, p, g, b, st);
    case F32: return launch_blas_p<F32>(op, p, g, b, st);
    case BF16S: return launch_blas_p<BF16S>(op, p, g, b, st);
    case F16S: return launch_blas_p<F16S>(op, p, g, b, st);
    default: return hipErrorInvalidValue;
    }
}

// x64 += f[rhs] * e
template <int PI>
__global__ __launch_bounds__(256) void accum_kernel(uint32_t V, int nrhs, void *x64, const void *e, const double *f,
                                                    int fstride)
{
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= V)
        return;
    const double a = f[(size_t)r * fstride];
    cx<typename Traits<PI>::real> ev[12];
    cx<double> x[12];
    load_site<PI>(e, V, nrhs, s, r, ev);
    load_site<F64>(x64, V, nrhs, s, r, x);
#pragma unroll
    for (int k = 0; k < 12; ++k)
        x[k] = cx<double>{fma(a, (double)ev[k].re, x[k].re), fma(a, (double)ev[k].im, x[k].im)};
    store_site<F64>(x64, V, nrhs, s, r, x);
}

hipError_t launch_accum(int pin, uint32_t V, int nrhs, void *x64, const void *e, const double *s, int sstride,
                        hipStream_t st)
{
    const int B = 256;
    dim3 g((V + B - 1) / B, nrhs);
    switch (pin) {
    case F64: hipLaunchKernelGGL(accum_kernel<F64>, g, dim3(B), 0, st, V, nrhs, x64, e, s, sstride); break;
    case F32: hipLaunchKernelGGL(accum_kernel<F32>, g, dim3(B), 0, st, V, nrhs, x64, e, s, sstride); break;
    case BF16S: hipLaunchKernelGGL(accum_kernel<BF16S>, g, dim3(B), 0, st, V, nrhs, x64, e, s, sstride); break;
    case F16S: hipLaunchKernelGGL(accum_kernel<F16S>, g, dim3(B), 0, st, V, nrhs, x64, e, s, sstride); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- finalize
// One workgroup sums every (value, right-hand side) row of the partial
// arrays in a fixed order and then runs the scalar recurrence per column.
// Rows are summed G at a time; a pass loads U values of each of the G rows
// per thread before it adds any of them.
constexpr int FIN_THREADS = 1024;
constexpr int FIN_MAX = RED_NVAL_MAX * 64;  // values x right-hand sides per partial set
// rows summed per pass: a template parameter G, 1 or 2 when the call has
// that few rows, else 4 (measured: one pass of 8 rows took 13.8 us where
// two passes of 4 took 12.1 us; a 1-row call with G = 1 5.8 us, with G = 4
// 7.5 us)
constexpr int FIN_U = 4;         // loads per thread per row and pass

__device__ __forceinline__ bool finite2(double a) { return isfinite(a); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b)  // b != 0
{
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

struct RowRef {
    const double *p;
    int n;
};

__device__ __forceinline__ RowRef fin_row(const FinParams &p, int c)
{
    const int na = p.nvalA * p.nrhs, nb = p.nvalB * p.nrhs;
    if (c < na)
        return RowRef{p.A + (size_t)c * p.nblkA, p.lenA ? p.lenA[c % p.nrhs] : p.nblkA};
    c -= na;
    if (c < nb)
        return RowRef{p.B + (size_t)c * p.nblkB, p.lenB ? p.lenB[c % p.nrhs] : p.nblkB};
    c -= nb;
    return RowRef{p.C + (size_t)c * p.nblkC, p.lenC ? p.lenC[c % p.nrhs] : p.nblkC};
}

template <int FIN_G>
__global__ __launch_bounds__(FIN_THREADS) void finalize_kernel(FinParams p, int op)
{
    __shared__ double lds[FIN_G * FIN_THREADS / 64];
    __shared__ double sums[3 * FIN_MAX];
    __shared__ double gsums[3 * FIN_MAX];
    const int nr = p.nrhs;
    const int na = p.nvalA * nr, nb = p.nvalB * nr, ncomb = na + nb + p.nvalC * nr;
    for (int c0 = 0; c0 < ncomb; c0 += FIN_G) {
        // one pass issues the loads of all G rows before any add: a single
        // workgroup is bound by its load issue rate, not by latency
        RowRef row[FIN_G];
        int nmax = 0;
#pragma unroll
        for (int g = 0; g < FIN_G; ++g) {
            row[g] = c0 + g < ncomb ? fin_row(p, c0 + g) : RowRef{nullptr, 0};
            nmax = max(nmax, row[g].n);
        }
        double v[FIN_G];
#pragma unroll
        for (int g = 0; g < FIN_G; ++g)
            v[g] = 0.0;
        for (int base = 0; base < nmax; base += FIN_U * FIN_THREADS) {
            double x[FIN_G][FIN_U];
#pragma unroll
            for (int g = 0; g < FIN_G; ++g) {
                if (base < row[g].n) {  // uniform: rows shorter than nmax stop early
#pragma unroll
                    for (int j = 0; j < FIN_U; ++j) {
                        const int i = base + j * FIN_THREADS + (int)threadIdx.x;
                        x[g][j] = row[g].p[i < row[g].n ? i : 0];
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < FIN_U; ++j)
                        x[g][j] = 0.0;
                }
            }
#pragma unroll
            for (int g = 0; g < FIN_G; ++g) {
#pragma unroll
                for (int j = 0; j < FIN_U; ++j)
                    if (base + j * FIN_THREADS + (int)threadIdx.x >= row[g].n)
                        x[g][j] = 0.0;
                // fixed pairwise order within a pass
#pragma unroll
                for (int w = FIN_U / 2; w > 0; w >>= 1)
#pragma unroll
                    for (int j = 0; j < w; ++j)
                        x[g][j] += x[g][j + w];
                v[g] += x[g][0];
            }
        }
        block_sum<FIN_G>(v, lds);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int g = 0; g < FIN_G; ++g)
                if (c0 + g < ncomb)
                    sums[c0 + g] = v[g];
        }
        __syncthreads();
    }
    const double *S = sums;
    if (p.group > 1) {
        // several columns form one linear system (a 5-d domain-wall vector):
        // every column of a group gets the group's total, in a fixed order
        __syncthreads();
        for (int c = threadIdx.x; c < ncomb; c += blockDim.x) {
            const int first = c - (c % nr) % p.group;  // sets start at multiples of nr
            double a = 0.0;
            for (int j = 0; j < p.group; ++j)
                a += sums[first + j];
            gsums[c] = a;
        }
        S = gsums;
    }
    const double *sA = S, *sB = S + na, *sC = S + na + nb;
    __syncthreads();
    const int r = threadIdx.x;
    if (r >= nr)
        return;
    if (op == F_SUM) {
        for (int v = 0; v < p.nvalA; ++v)
            p.out[v * nr + r] = sA[v * nr + r];
        return;
    }
    Scalars sc = p.sc[r];
    const double2 zero = make_double2(0.0, 0.0), one = make_double2(1.0, 0.0);
    switch (op) {
    case F_INIT_CG: {
        sc.rr = sA[r];
        sc.zz = p.nvalB > 0 ? sB[r] : 0.0;  // the single-reduction form computes z in its loop
        sc.bb = sC[r];
        sc.rr_upd = sc.rr;
        sc.restart = 0;
        sc.tol2 = p.tol2v ? p.tol2v[r] : p.tol2;
        sc.alpha = sc.beta = zero;
        sc.flag = 0;
        sc.conv_iter = 0;
        if (!finite2(sc.rr) || !finite2(sc.zz) || !finite2(sc.bb))
            sc.flag = 3;
        else if (sc.rr <= sc.tol2 * sc.bb)
            sc.flag = 1;
        sc.frozen = sc.flag != 0;
        break;
    }
    case F_CG_ALPHA: {
        const double ww = sA[r];
        if (sc.flag == 0) {
            if (!finite2(ww))
                sc.flag = 3;
            else if (ww > 0.0) {
                sc.alpha = make_double2(sc.zz / ww, 0.0);
                break;
            } else
                sc.flag = 2;
        }
        sc.alpha = zero;
        break;
    }
    case F_CG_BETA: {
        const double rr = sA[r], zz = sB[r];
        if (sc.flag == 0) {
            sc.rr = rr;
            if (!finite2(rr) || !finite2(zz))
                sc.flag = 3;
            else if (rr <= sc.tol2 * sc.bb) {
                sc.flag = 1;
                sc.conv_iter = p.iter + 1;
            } else if (sc.zz > 0.0) {
                sc.beta = make_double2(zz / sc.zz, 0.0);
                sc.zz = zz;
                break;
            } else
                sc.flag = 2;
        }
        sc.beta = zero;
        sc.frozen = 1;  // end of the iteration with flag != 0
        break;
    }
    case F_CG_RELIABLE: {
        // r was replaced by the (converted) true residual and z = D^dag r
        // recomputed; the search direction is kept
        if (sc.flag == 0) {
            const double rr = sA[r], zz = sB[r];
            sc.rr = rr;
            if (!finite2(rr) || !finite2(zz))
                sc.flag = 3;
            else if (rr <= sc.tol2 * sc.bb) {
                sc.flag = 1;
                sc.conv_iter = p.iter + 1;
            } else if (zz > 0.0) {
                sc.zz = zz;
                // |r| has grown since the previous update: the low-precision
                // recurrence has lost its search space; start it again from z
                sc.restart = rr > sc.rr_upd;
                sc.rr_upd = rr;
            } else
                sc.flag = 2;
            if (sc.flag != 0) {
                sc.alpha = sc.beta = zero;
                sc.frozen = 1;
            }
        }
        break;
    }
    case F_INIT_BI: {
        sc.rr = sA[r];
        sc.bb = sC[r];
        sc.tol2 = p.tol2v ? p.tol2v[r] : p.tol2;
        sc.rho = make_double2(sc.rr, 0.0);
        sc.rho_prev = sc.rho;  // <rh, r0> with rh = r0
        sc.alpha = sc.omega = one;
        sc.beta = zero;  // p = v = 0 -> first p = r
        sc.brk = 0;
        sc.flag = 0;
        sc.conv_iter = 0;
        if (!finite2(sc.rr) || !finite2(sc.bb))
            sc.flag = 3;
        else if (sc.rr <= sc.tol2 * sc.bb)
            sc.flag = 1;
        sc.frozen = sc.flag != 0;
        break;
    }
    case F_BI_ALPHA: {
        const double2 rv = make_double2(sA[r], sA[nr + r]);
        if (sc.flag == 0) {
            const double d = rv.x * rv.x + rv.y * rv.y;
            if (!finite2(d))
                sc.flag = 3;
            else if (d > 0.0) {  // alpha = rho / <rh, v>
                sc.alpha = make_double2((sc.rho.x * rv.x + sc.rho.y * rv.y) / d, (sc.rho.y * rv.x - sc.rho.x * rv.y) / d);
                break;
            } else
                sc.flag = 2;
        }
        sc.alpha = zero;
        break;
    }
    case F_BI_OMEGA_RHO: {
        // omega = <t, s> / <t, t> (or stop: converged on |s|, t = 0, NaN);
        // then, with r' = s - omega t still to be formed,
        // rho' = <rh, r'> = <rh, s> - omega <rh, t> and beta = (rho'/rho)(alpha/omega)
        const double ss = sA[7 * nr + r];
        const double st_re = sA[r], st_im = sA[nr + r], tt = sA[2 * nr + r];
        const double2 hs = make_double2(sA[3 * nr + r], sA[4 * nr + r]);
        const double2 ht = make_double2(sA[5 * nr + r], sA[6 * nr + r]);
        sc.ss = ss;
        sc.brk = 0;
        sc.beta = zero;
        if (sc.flag == 0) {
            if (!finite2(ss) || !finite2(tt) || !finite2(st_re) || !finite2(st_im))
                sc.flag = 3;
            else if (ss <= sc.tol2 * sc.bb) {  // x += alpha p ; r = s  (omega = 0)
                sc.flag = 1;
                sc.conv_iter = p.iter + 1;
            } else if (tt > 0.0) {
                const double2 om = make_double2(st_re / tt, -st_im / tt);
                sc.omega = om;
                const double2 rho_new = make_double2(hs.x - (om.x * ht.x - om.y * ht.y), hs.y - (om.x * ht.y + om.y * ht.x));
                const double om2 = om.x * om.x + om.y * om.y;
                const double rho2 = sc.rho.x * sc.rho.x + sc.rho.y * sc.rho.y;
                if (!finite2(rho_new.x) || !finite2(rho_new.y))
                    sc.brk = 2;
                else if (om2 > 0.0 && rho2 > 0.0 && (rho_new.x != 0.0 || rho_new.y != 0.0)) {
                    const double2 q1 = make_double2((rho_new.x * sc.rho.x + rho_new.y * sc.rho.y) / rho2,
                                                    (rho_new.y * sc.rho.x - rho_new.x * sc.rho.y) / rho2);
                    const double2 q2 = make_double2((sc.alpha.x * om.x + sc.alpha.y * om.y) / om2,
                                                    (sc.alpha.y * om.x - sc.alpha.x * om.y) / om2);
                    sc.beta = make_double2(q1.x * q2.x - q1.y * q2.y, q1.x * q2.y + q1.y * q2.x);
                    sc.rho_prev = sc.rho;
                    sc.rho = rho_new;
                } else
                    sc.brk = 1;
                break;
            } else
                sc.flag = 2;
        } else
            sc.alpha = zero;
        sc.omega = zero;
        break;
    }
    case F_BI_CONV: {
        const double rr = sA[r];
        if (sc.flag == 0) {
            sc.rr = rr;
            if (!finite2(rr) || sc.brk == 2)
                sc.flag = 3;
            else if (rr <= sc.tol2 * sc.bb) {
                sc.flag = 1;
                sc.conv_iter = p.iter + 1;
            } else if (sc.brk == 1)
                sc.flag = 2;
            else
                break;
        } else if (sc.flag == 1 && sc.conv_iter == p.iter + 1) {
            sc.rr = rr;  // converged on |s| this iteration: r = s
        }
        sc.beta = zero;
        sc.alpha = zero;
        sc.omega = zero;
        sc.frozen = 1;  // end of the iteration with flag != 0
        break;
    }
    case F_CG1: {
        // CG on the normal equations with one reduction phase per iteration
        // (Chronopoulos and Gear's form): gamma = |z|^2 with z = D^dag r,
        // delta = |D z|^2; beta = gamma / gamma_prev and
        // alpha = gamma / (delta - beta gamma / alpha_prev), where the
        // denominator equals |D p|^2 for p = z + beta p_prev
        const double rr = p.nvalC > 0 ? sC[r] : sc.rr, gam = sA[r], del = sB[r];
        if (sc.flag == 0) {
            sc.rr = rr;
            if (!finite2(rr) || !finite2(gam) || !finite2(del))
                sc.flag = 3;
            else if (rr <= sc.tol2 * sc.bb) {
                sc.flag = 1;
                sc.conv_iter = p.iter;
            } else {
                const double beta = p.iter > 0 && sc.zz > 0.0 ? gam / sc.zz : 0.0;
                const double den = beta != 0.0 ? del - beta * gam / sc.alpha.x : del;
                if (gam > 0.0 && den > 0.0 && finite2(den)) {
                    sc.alpha = make_double2(gam / den, 0.0);
                    sc.beta = make_double2(beta, 0.0);
                    sc.zz = gam;
                    break;
                }
                sc.flag = 2;
            }
        }
        sc.alpha = sc.beta = zero;
        sc.frozen = 1;  // the update pass of this iteration is skipped
        break;
    }
    case F_SR: {
        // BiCGStab with one reduction phase per iteration.  With u = D r,
        // v = D p and q = D v known, s = r - alpha v and t = D s = u - alpha q
        // never need to be formed before the scalars:
        //   <t, s> = <u, r> - alpha <u, v> - conj(alpha) <q, r> + |alpha|^2 <q, v>
        //   <t, t> = |u|^2 - 2 Re(alpha <u, q>) + |alpha|^2 |q|^2
        //   rho'   = <rh, s> - omega <rh, t>
        //          = rho - alpha <rh, v> - omega (<rh, u> - alpha <rh, q>)
        const double rr = p.nvalC > 0 ? sC[r] : sc.rr;
        const double2 hv = make_double2(sA[r], sA[nr + r]), hu = make_double2(sA[2 * nr + r], sA[3 * nr + r]);
        const double2 ur = make_double2(sA[4 * nr + r], sA[5 * nr + r]), uv = make_double2(sA[6 * nr + r], sA[7 * nr + r]);
        const double uu = sA[8 * nr + r];
        const double2 vq = make_double2(sB[r], sB[nr + r]);
        const double qq = sB[2 * nr + r];
        const double2 hq = make_double2(sB[3 * nr + r], sB[4 * nr + r]), rq = make_double2(sB[5 * nr + r], sB[6 * nr + r]);
        const double2 uq = make_double2(sB[7 * nr + r], sB[8 * nr + r]);
        if (sc.flag == 0) {
            sc.rr = rr;
            const double d = hv.x * hv.x + hv.y * hv.y;
            if (!finite2(rr) || !finite2(d) || !finite2(uu) || !finite2(qq) || sc.brk == 2)
                sc.flag = 3;
            else if (rr <= sc.tol2 * sc.bb) {
                sc.flag = 1;
                sc.conv_iter = p.iter;
            } else if (sc.brk == 1 || !(d > 0.0))
                sc.flag = 2;
            if (sc.flag == 0) {
                const double2 a = cdiv(sc.rho, hv);
                const double a2 = a.x * a.x + a.y * a.y;
                // <t, s>
                const double2 auv = cmul(a, uv);
                const double2 aqr = cmul(make_double2(a.x, -a.y), make_double2(rq.x, -rq.y));
                const double2 ts = make_double2(ur.x - auv.x - aqr.x + a2 * vq.x, ur.y - auv.y - aqr.y - a2 * vq.y);
                const double tt = uu - 2.0 * cmul(a, uq).x + a2 * qq;
                sc.brk = 0;
                if (!finite2(ts.x) || !finite2(ts.y) || !finite2(tt)) {
                    sc.flag = 3;
                } else if (!(tt > 0.0)) {
                    sc.flag = 2;
                } else {
                    const double2 om = make_double2(ts.x / tt, ts.y / tt);
                    const double2 ahq = cmul(a, hq);
                    const double2 w1 = cmul(om, make_double2(hu.x - ahq.x, hu.y - ahq.y));
                    const double2 ahv = cmul(a, hv);
                    const double2 rho_new = make_double2(sc.rho.x - ahv.x - w1.x, sc.rho.y - ahv.y - w1.y);
                    sc.alpha = a;
                    sc.omega = om;
                    sc.beta = zero;
                    if (!finite2(rho_new.x) || !finite2(rho_new.y))
                        sc.brk = 2;
                    else if ((om.x != 0.0 || om.y != 0.0) && (rho_new.x != 0.0 || rho_new.y != 0.0))
                        sc.beta = cmul(cdiv(rho_new, sc.rho), cdiv(a, om));
                    else
                        sc.brk = 1;  // this step is taken; the next check reports the breakdown
                    sc.rho_prev = sc.rho;
                    sc.rho = rho_new;
                    break;
                }
            }
        }
        sc.alpha = sc.beta = sc.omega = zero;
        sc.frozen = 1;
        break;
    }
    case F_BI_RELIABLE: {
        // r was just replaced by the (converted) true residual; recompute
        // rho = <rh, r> and beta = (rho / rho_prev)(alpha / omega) from it
        if (sc.flag == 0) {
            const double rr = sA[2 * nr + r];
            const double2 rho_new = make_double2(sA[r], sA[nr + r]);
            const double om2 = sc.omega.x * sc.omega.x + sc.omega.y * sc.omega.y;
            const double rp2 = sc.rho_prev.x * sc.rho_prev.x + sc.rho_prev.y * sc.rho_prev.y;
            sc.rr = rr;
            if (!finite2(rr) || !finite2(rho_new.x) || !finite2(rho_new.y)) {
                sc.flag = 3;
            } else if (rr <= sc.tol2 * sc.bb) {
                sc.flag = 1;
                sc.conv_iter = p.iter + 1;
            } else if (om2 > 0.0 && rp2 > 0.0 && (rho_new.x != 0.0 || rho_new.y != 0.0)) {
                const double2 q1 = make_double2((rho_new.x * sc.rho_prev.x + rho_new.y * sc.rho_prev.y) / rp2,
                                                (rho_new.y * sc.rho_prev.x - rho_new.x * sc.rho_prev.y) / rp2);
                const double2 q2 = make_double2((sc.alpha.x * sc.omega.x + sc.alpha.y * sc.omega.y) / om2,
                                                (sc.alpha.y * sc.omega.x - sc.alpha.x * sc.omega.y) / om2);
                sc.beta = make_double2(q1.x * q2.x - q1.y * q2.y, q1.x * q2.y + q1.y * q2.x);
                sc.rho = rho_new;
            } else {
                sc.flag = 2;
            }
            if (sc.flag != 0) {
                sc.alpha = sc.beta = sc.omega = zero;
                sc.frozen = 1;
            }
        }
        break;
    }
    default: break;
    }
    p.sc[r] = sc;
    if (p.hflag) {  // mirror the status into host-visible memory for polling
        p.hrr[r] = sc.rr;
        p.hflag[r] = sc.flag;
        if (p.hsc)
            p.hsc[r] = sc;
    }
}

hipError_t launch_finalize(int op, const FinParams &p, hipStream_t st)
{
    if (p.nrhs > 64 || p.nvalA * p.nrhs > FIN_MAX || p.nvalB * p.nrhs > FIN_MAX || p.nvalC * p.nrhs > FIN_MAX)
        return hipErrorInvalidValue;
    const int rows = (p.nvalA + p.nvalB + p.nvalC) * p.nrhs;
    if (rows <= 1)
        hipLaunchKernelGGL(finalize_kernel<1>, dim3(1), dim3(FIN_THREADS), 0, st, p, op);
    else if (rows <= 2)
        hipLaunchKernelGGL(finalize_kernel<2>, dim3(1), dim3(FIN_THREADS), 0, st, p, op);
    else
        hipLaunchKernelGGL(finalize_kernel<4>, dim3(1), dim3(FIN_THREADS), 0, st, p, op);
    return hipGetLastError();
}

}  // namespace wl
