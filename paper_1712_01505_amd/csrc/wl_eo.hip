// wl_eo.hip -- even-odd (red-black) decomposition of the Wilson operator.
//
// With sites coloured by the parity of x + y + z + t, the hopping term only
// couples opposite parities, so D = 1 - kappa H reads, in (even, odd) blocks,
//   D = [[1, -kappa H_eo], [-kappa H_oe, 1]],
// and D x = b is equivalent to the Schur system on the even sites
//   M x_e = b_e + kappa H_eo b_o,   M = 1 - kappa^2 H_eo H_oe,
// followed by x_o = b_o + kappa H_oe x_e.  (The paper leaves
// preconditioning out, Sec. II-C; this is the standard first step, with the
// same solution.)
//
// Half fields hold the sites of one parity in the packed spinor format with
// V/2 sites: the site x + Lx (y + Ly (z + Lz t)) of parity p sits at half
// index (x + Lx (y + ...)) / 2.  Every extent must be even (a hop that wraps
// around an odd extent would keep the parity).  Links stay in the full
// packed layout.
#include "wl_hop.h"
#include "wl_internal.h"

namespace wl {

// Copy whole packed sites between the full layout and the two half layouts
// (raw 16-byte chunks and, for 16-bit formats, the scale: bit-exact).
template <int P, bool SPLIT>
__global__ void eo_copy_kernel(uint32_t V, int nrhs, const void *__restrict__ full_in, void *__restrict__ full_out,
                               void *__restrict__ even, void *__restrict__ odd, FastDiv fx, FastDiv fy, FastDiv fz,
                               int Lx, int Ly, int Lz)
{
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= V)
        return;
    const uint32_t q1 = fdiv(s, fx);
    const int x = (int)(s - q1 * (uint32_t)Lx);
    const uint32_t q2 = fdiv(q1, fy);
    const int y = (int)(q1 - q2 * (uint32_t)Ly);
    const uint32_t q3 = fdiv(q2, fz);
    const int z = (int)(q2 - q3 * (uint32_t)Lz);
    const int t = (int)q3;
    const int par = (x + y + z + t) & 1;
    const uint32_t Vh = V / 2, i = s >> 1;
    constexpr int NCH = Traits<P>::NCH;
    const uint4 *src;
    uint4 *dst;
    uint32_t sv, dv, si, di;
    char *half = reinterpret_cast<char *>(par ? odd : even);
    if constexpr (SPLIT) {
        src = reinterpret_cast<const uint4 *>(full_in);
        dst = reinterpret_cast<uint4 *>(half);
        sv = V;
        dv = Vh;
        si = s;
        di = i;
    } else {
        src = reinterpret_cast<const uint4 *>(half);
        dst = reinterpret_cast<uint4 *>(full_out);
        sv = Vh;
        dv = V;
        si = i;
        di = s;
    }
#pragma unroll
    for (int k = 0; k < NCH; ++k)
        dst[((size_t)r * NCH + k) * dv + di] = src[((size_t)r * NCH + k) * sv + si];
    if constexpr (Traits<P>::SCALED) {
        const float *ss = reinterpret_cast<const float *>(reinterpret_cast<const char *>(src) + (size_t)nrhs * NCH * sv * 16);
        float *ds = reinterpret_cast<float *>(reinterpret_cast<char *>(dst) + (size_t)nrhs * NCH * dv * 16);
        ds[(size_t)r * dv + di] = ss[(size_t)r * sv + si];
    }
}

hipError_t launch_eo_copy(int prec, bool split, const int *L, int nrhs, const void *full_in, void *full_out,
                          void *even, void *odd, hipStream_t st)
{
    const uint32_t V = (uint32_t)L[0] * L[1] * L[2] * L[3];
    const FastDiv fx = make_fastdiv((uint32_t)L[0]), fy = make_fastdiv((uint32_t)L[1]),
                  fz = make_fastdiv((uint32_t)L[2]);
    dim3 g((V + 255) / 256, nrhs), b(256);
#define WL_EO_COPY(PP)                                                                                         \
    if (split)                                                                                                 \
        hipLaunchKernelGGL((eo_copy_kernel<PP, true>), g, b, 0, st, V, nrhs, full_in, full_out, even, odd, fx, \
                           fy, fz, L[0], L[1], L[2]);                                                          \
    else                                                                                                       \
        hipLaunchKernelGGL((eo_copy_kernel<PP, false>), g, b, 0, st, V, nrhs, full_in, full_out, even, odd,    \
                           fx, fy, fz, L[0], L[1], L[2]);
    switch (prec) {
    case F64: WL_EO_COPY(F64) break;
    case F32: WL_EO_COPY(F32) break;
    case BF16S: WL_EO_COPY(BF16S) break;
    case F16S: WL_EO_COPY(F16S) break;
    default: return hipErrorInvalidValue;
    }
#undef WL_EO_COPY
    return hipGetLastError();
}

// One hop direction MU (both signs) into acc for the half-lattice site with
// full coordinates c and full index s; neighbours are read from the half
// field `in` (the other parity), links from the full layout.
template <int P, int DAG, int MU>
__device__ __forceinline__ void eo_hop_dir(const EoParams &p, const int (&c)[4], uint32_t s, int rhs,
                                           cx<typename Traits<P>::real> (&acc)[12])
{
    using T = typename Traits<P>::real;
    constexpr int SF = DAG ? 1 : -1;
    uint32_t stride = 1;
#pragma unroll
    for (int m = 0; m < MU; ++m)
        stride *= (uint32_t)p.L[m];
    const int L = p.L[MU];
    const bool wf = c[MU] == L - 1, wb = c[MU] == 0;
    const uint32_t span = (uint32_t)(L - 1) * stride;
    const uint32_t sf = wf ? s - span : s + stride;
    const uint32_t sb = wb ? s + span : s - stride;
    const bool anti = p.bc[MU] < 0;
    const T gf = (wf && anti) ? T(-1) : T(1);
    const T gb = (wb && anti) ? T(-1) : T(1);
    cx<T> u[9], ps[12], h[6], g[6];
    load_link<P>(p.U, p.V, MU, s, u);
    load_site<P>(p.in, p.Vh, p.nrhs, sf >> 1, rhs, ps);
    project<MU, SF>(ps, h);
    su3_mv(u, h, g);
    accum<MU, SF>(acc, g, gf);
    load_link<P>(p.U, p.V, MU, sb, u);
    load_site<P>(p.in, p.Vh, p.nrhs, sb >> 1, rhs, ps);
    project<MU, -SF>(ps, h);
    su3_adj_mv(u, h, g);
    accum<MU, -SF>(acc, g, gb);
}

// out(parity) = c_self * self + c_hop * H_{parity, other} in, with optional
// fused reductions over out: |out|^2 (RED_NORM), <v, out> (RED_DOTV, v =
// dotv) or <self, out> and |out|^2 (RED_DOTIN_NORM); with self the Schur
// input, the BiCGStab sets RED_BICG and RED_SR.
template <int P, int DAG, int RED>
__global__ __launch_bounds__(256) void eo_hop_kernel(EoParams p)
{
    using T = typename Traits<P>::real;
    constexpr int NV = red_nval(RED);
    __shared__ double lds[(NV > 0 ? NV : 1) * 4];
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const int rhs = blockIdx.y;
    if (p.skip && p.skip[rhs].frozen)
        return;
    double red[NV > 0 ? NV : 1] = {};
    if (i < p.Vh) {
        // half index -> coordinates: x = 2 (i mod Lx/2) + parity bit
        const uint32_t q1 = fdiv(i, p.fxh);
        const uint32_t k = i - q1 * (uint32_t)(p.L[0] / 2);
        const uint32_t q2 = fdiv(q1, p.fy);
        const int y = (int)(q1 - q2 * (uint32_t)p.L[1]);
        const uint32_t q3 = fdiv(q2, p.fz);
        const int z = (int)(q2 - q3 * (uint32_t)p.L[2]);
        const int t = (int)q3;
        const int x = 2 * (int)k + ((y + z + t + p.parity) & 1);
        const int c[4] = {x, y, z, t};
        const uint32_t s = (uint32_t)x + (uint32_t)p.L[0] * q1;
        cx<T> acc[12];
#pragma unroll
        for (int n = 0; n < 12; ++n)
            acc[n] = cx<T>{T(0), T(0)};
        eo_hop_dir<P, DAG, 0>(p, c, s, rhs, acc);
        eo_hop_dir<P, DAG, 1>(p, c, s, rhs, acc);
        eo_hop_dir<P, DAG, 2>(p, c, s, rhs, acc);
        eo_hop_dir<P, DAG, 3>(p, c, s, rhs, acc);
        const T ch = (T)p.c_hop, cs = (T)p.c_self;
        cx<T> o[12], sf[12];
        if (p.self) {
            load_site<P>(p.self, p.Vh, p.nrhs, i, rhs, sf);
#pragma unroll
            for (int n = 0; n < 12; ++n)
                o[n] = cx<T>{fma(ch, acc[n].re, cs * sf[n].re), fma(ch, acc[n].im, cs * sf[n].im)};
        } else {
#pragma unroll
            for (int n = 0; n < 12; ++n) {
                sf[n] = cx<T>{T(0), T(0)};
                o[n] = cx<T>{ch * acc[n].re, ch * acc[n].im};
            }
        }
        store_site_q<P, true>(p.out, p.Vh, p.nrhs, i, rhs, o);
        if constexpr (RED == RED_NORM || RED == RED_DOTIN_NORM) {
            double n2 = 0.0;
#pragma unroll
            for (int n = 0; n < 12; ++n)
                n2 = fma((double)o[n].re, (double)o[n].re, fma((double)o[n].im, (double)o[n].im, n2));
            red[NV - 1] = n2;
        }
        if constexpr (RED == RED_DOTV || RED == RED_DOTIN_NORM) {
            cx<T> v[12];
            if constexpr (RED == RED_DOTV)
                load_site<P>(p.dotv, p.Vh, p.nrhs, i, rhs, v);
            else
#pragma unroll
                for (int n = 0; n < 12; ++n)
                    v[n] = sf[n];
            double re = 0.0, im = 0.0;
#pragma unroll
            for (int n = 0; n < 12; ++n) {
                re = fma((double)v[n].re, (double)o[n].re, fma((double)v[n].im, (double)o[n].im, re));
                im = fma((double)v[n].re, (double)o[n].im, fma(-(double)v[n].im, (double)o[n].re, im));
            }
            red[0] = re;
            red[1] = im;
        }
        if constexpr (RED == RED_BICG) {  // self = the Schur input s, dotv = rh
            cx<T> v[12];
            load_site<P>(p.dotv, p.Vh, p.nrhs, i, rhs, v);
            bicg_values(sf, o, v, red);
        }
        if constexpr (RED == RED_SR) {  // self = the Schur input v; dotv, dotv2, dotv3 = rh, r, u
            cx<T> a[12], b[12], c[12];
            load_site<P>(p.dotv, p.Vh, p.nrhs, i, rhs, a);
            load_site<P>(p.dotv2, p.Vh, p.nrhs, i, rhs, b);
            load_site<P>(p.dotv3, p.Vh, p.nrhs, i, rhs, c);
            sr_values(sf, o, a, b, c, red);
        }
    }
    if constexpr (NV > 0) {
        block_sum<NV>(red, lds);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < NV; ++k)
                p.partials[((size_t)k * p.nrhs + rhs) * p.nblk + blockIdx.x] = red[k];
        }
    }
}

int eo_partials(uint32_t Vh) { return (int)((Vh + 255) / 256); }

EoParams eo_params(const wl_op *op, int parity, int nrhs)
{
    EoParams p{};
    p.U = op->U;
    for (int i = 0; i < 4; ++i) {
        p.L[i] = op->g.dims[i];
        p.bc[i] = op->g.bc[i];
    }
    p.parity = parity;
    p.nrhs = nrhs;
    return p;
}

hipError_t launch_eo_hop(int prec, int dagger, int red, EoParams p, hipStream_t st)
{
    if (p.L[0] % 2 != 0 || p.L[1] % 2 != 0 || p.L[2] % 2 != 0 || p.L[3] % 2 != 0)
        return hipErrorInvalidValue;
    p.V = (uint32_t)p.L[0] * p.L[1] * p.L[2] * p.L[3];
    p.Vh = p.V / 2;
    p.fxh = make_fastdiv((uint32_t)(p.L[0] / 2));
    p.fy = make_fastdiv((uint32_t)p.L[1]);
    p.fz = make_fastdiv((uint32_t)p.L[2]);
    p.nblk = eo_partials(p.Vh);
    dim3 g(p.nblk, p.nrhs), b(256);
#define WL_EO_RED(PP, DD)                                                                                      \
    switch (red) {                                                                                             \
    case RED_NONE: hipLaunchKernelGGL((eo_hop_kernel<PP, DD, RED_NONE>), g, b, 0, st, p); break;              \
    case RED_NORM: hipLaunchKernelGGL((eo_hop_kernel<PP, DD, RED_NORM>), g, b, 0, st, p); break;              \
    case RED_DOTV: hipLaunchKernelGGL((eo_hop_kernel<PP, DD, RED_DOTV>), g, b, 0, st, p); break;              \
    case RED_DOTIN_NORM: hipLaunchKernelGGL((eo_hop_kernel<PP, DD, RED_DOTIN_NORM>), g, b, 0, st, p); break;  \
    case RED_BICG: hipLaunchKernelGGL((eo_hop_kernel<PP, DD, RED_BICG>), g, b, 0, st, p); break;              \
    case RED_SR: hipLaunchKernelGGL((eo_hop_kernel<PP, DD, RED_SR>), g, b, 0, st, p); break;                  \
    default: return hipErrorInvalidValue;                                                                      \
    }
    switch (prec * 2 + (dagger ? 1 : 0)) {
    case 0: WL_EO_RED(F64, 0) break;
    case 1: WL_EO_RED(F64, 1) break;
    case 2: WL_EO_RED(F32, 0) break;
    case 3: WL_EO_RED(F32, 1) break;
    case 4: WL_EO_RED(BF16S, 0) break;
    case 5: WL_EO_RED(BF16S, 1) break;
    case 6: WL_EO_RED(F16S, 0) break;
    case 7: WL_EO_RED(F16S, 1) break;
    default: return hipErrorInvalidValue;
    }
#undef WL_EO_RED
    return hipGetLastError();
}

}  // namespace wl
