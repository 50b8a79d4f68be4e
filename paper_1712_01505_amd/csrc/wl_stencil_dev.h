// wl_stencil_dev.h -- device building blocks of the Wilson-Dirac stencil
// kernels (paper Sec. II-B, eq. (1)): the hops of one site, straight-line
// or software-pipelined over raw (still packed) loads, the t-walk helpers,
// the domain-wall epilogue and the workgroup -> (tile, right-hand side)
// map.  Included by the per-precision kernel files.
#pragma once

#include "wl_hop.h"
#include "wl_hop16.h"
#include "wl_internal.h"

namespace wl {

// FP16 storage: a link's two stored rows as packed f16 complex with the
// third row rebuilt, and a site's stored spinor (unscaled) with its scale.
__device__ __forceinline__ void raw_link16(const StencilParams &p, int mu, uint32_t s, hf2 (&u)[9])
{
    const uint2 *b = reinterpret_cast<const uint2 *>(p.U) + (size_t)mu * 3 * p.V + s;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const uint2 d = b[(size_t)k * p.V];
        u[2 * k] = as_hf2(d.x);
        u[2 * k + 1] = as_hf2(d.y);
    }
    rebuild_row16(u);
}
__device__ __forceinline__ void raw_spinor16(const StencilParams &p, uint32_t s, int rhs, hf2 (&ps)[12], float &sc)
{
    const uint4 *b = reinterpret_cast<const uint4 *>(p.in) + (size_t)rhs * 3 * p.V + s;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const uint4 d = b[(size_t)k * p.V];
        ps[4 * k] = as_hf2(d.x);
        ps[4 * k + 1] = as_hf2(d.y);
        ps[4 * k + 2] = as_hf2(d.z);
        ps[4 * k + 3] = as_hf2(d.w);
    }
    sc = scale_ptr<F16S>(p.in, p.V, p.nrhs)[(size_t)rhs * p.V + s];
}

// Both hops in direction MU for R right-hand sides.
template <int P, int DAG, int R, int MU>
__device__ __forceinline__ void hop_dir(const StencilParams &p, uint32_t s, int c, uint32_t stride, int r0,
                                        cx<typename Traits<P>::real> (&acc)[R][12])
{
    using T = typename Traits<P>::real;
    constexpr int SF = DAG ? 1 : -1;  // forward hop uses (1 + SF g), backward (1 - SF g)
    const int L = p.L[MU];
    const bool wf = (c == L - 1), wb = (c == 0);
    const uint32_t span = (uint32_t)(L - 1) * stride;
    const uint32_t sf = wf ? s - span : s + stride;
    const uint32_t sb = wb ? s + span : s - stride;
    const bool anti = p.bc[MU] < 0;
    // an enforced halo takes the t hops that wrap out of the face buffers
    const bool cut = MU == 3 && p.halo_t;
    const T gf = (wf && cut) ? T(0) : (wf && anti) ? T(-1) : T(1);
    const T gb = (wb && cut) ? T(0) : (wb && anti) ? T(-1) : T(1);
    if constexpr (P == F16S) {  // packed f16 projection, dot2 products (wl_hop16.h)
        hf2 u[9];
        raw_link16(p, MU, s, u);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            hf2 ps[12], h[6];
            float sc;
            raw_spinor16(p, sf, r0 + r, ps, sc);
            project16<MU, SF>(ps, h);
            cx<float> g[6];
            su3_mv16<0>(u, h, g);
            accum<MU, SF>(acc[r], g, gf * sc);
        }
        if constexpr (R > 1)
            __builtin_amdgcn_sched_barrier(0);
        raw_link16(p, MU, sb, u);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            hf2 ps[12], h[6];
            float sc;
            raw_spinor16(p, sb, r0 + r, ps, sc);
            project16<MU, -SF>(ps, h);
            cx<float> g[6];
            su3_mv16<1>(u, h, g);
            accum<MU, -SF>(acc[r], g, gb * sc);
        }
        if constexpr (R > 1)
            __builtin_amdgcn_sched_barrier(0);
        return;
    }
    cx<T> u[9];
    load_link<P>(p.U, p.V, MU, s, u);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        cx<T> ps[12], h[6], g[6];
        T sc;
        load_site_unscaled<P>(p.in, p.V, p.nrhs, sf, r0 + r, ps, sc);
        project<MU, SF>(ps, h, (T)p.one);
        su3_mv(u, h, g);
        accum<MU, SF>(acc[r], g, gf * sc);
    }
    // with several right-hand sides per thread, keep the scheduler from
    // hoisting every neighbour load of the site (it would spill)
    if constexpr (R > 1)
        __builtin_amdgcn_sched_barrier(0);
    load_link<P>(p.U, p.V, MU, sb, u);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        cx<T> ps[12], h[6], g[6];
        T sc;
        load_site_unscaled<P>(p.in, p.V, p.nrhs, sb, r0 + r, ps, sc);
        project<MU, -SF>(ps, h, (T)p.one);
        su3_adj_mv(u, h, g);
        accum<MU, -SF>(acc[r], g, gb * sc);
    }
    if constexpr (R > 1)
        __builtin_amdgcn_sched_barrier(0);
}

template <int P, int DAG, int R>
__device__ __forceinline__ void hop_site(const StencilParams &p, uint32_t s, int r0,
                                         cx<typename Traits<P>::real> (&acc)[R][12])
{
    const uint32_t q1 = fdiv(s, p.fx);
    const int x = (int)(s - q1 * (uint32_t)p.L[0]);
    const uint32_t q2 = fdiv(q1, p.fy);
    const int y = (int)(q1 - q2 * (uint32_t)p.L[1]);
    const uint32_t q3 = fdiv(q2, p.fz);
    const int z = (int)(q2 - q3 * (uint32_t)p.L[2]);
    const int t = (int)q3;
    const uint32_t sy = (uint32_t)p.L[0], sz = sy * (uint32_t)p.L[1], st = sz * (uint32_t)p.L[2];
    hop_dir<P, DAG, R, 0>(p, s, x, 1u, r0, acc);
    hop_dir<P, DAG, R, 1>(p, s, y, sy, r0, acc);
    hop_dir<P, DAG, R, 2>(p, s, z, sz, r0, acc);
    hop_dir<P, DAG, R, 3>(p, s, t, st, r0, acc);
}

// ---------------------------------------------------------------- pipelined hops
// The eight hops of a site as a software pipeline: the raw (still packed)
// spinor and link data of the next G hops are loaded while the current G
// hops are decoded and computed, so each wavefront keeps up to 2G hops of
// loads in flight instead of draining after every hop.
template <int P>
struct RawHop;
template <>
struct RawHop<F64> {
    double2 sp[12];
    double2 lk[6];
};
template <>
struct RawHop<F32> {
    float4 sp[6];
    float4 lk[3];
};
template <>
struct RawHop<BF16S> {
    uint4 sp[3];
    uint2 lk[3];
    float sc;
};
template <>
struct RawHop<F16S> {
    uint4 sp[3];
    uint2 lk[3];
    float sc;
};

struct Hops {
    uint32_t nb[8];  // neighbour site of hop h = 2 mu + (0 forward, 1 backward)
    float sg[8];     // boundary sign of the hop
};

__device__ __forceinline__ void make_hops(const StencilParams &p, uint32_t s, Hops &h)
{
    const uint32_t q1 = fdiv(s, p.fx);
    const int x = (int)(s - q1 * (uint32_t)p.L[0]);
    const uint32_t q2 = fdiv(q1, p.fy);
    const int y = (int)(q1 - q2 * (uint32_t)p.L[1]);
    const uint32_t q3 = fdiv(q2, p.fz);
    const int z = (int)(q2 - q3 * (uint32_t)p.L[2]);
    const int t = (int)q3;
    const int c[4] = {x, y, z, t};
    uint32_t stride = 1u;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const int L = p.L[mu];
        const bool wf = (c[mu] == L - 1), wb = (c[mu] == 0);
        const uint32_t span = (uint32_t)(L - 1) * stride;
        h.nb[2 * mu] = wf ? s - span : s + stride;
        h.nb[2 * mu + 1] = wb ? s + span : s - stride;
        const bool anti = p.bc[mu] < 0;
        const bool cut = mu == 3 && p.halo_t;  // enforced halo: face buffers carry these hops
        h.sg[2 * mu] = (wf && cut) ? 0.f : (wf && anti) ? -1.f : 1.f;
        h.sg[2 * mu + 1] = (wb && cut) ? 0.f : (wb && anti) ? -1.f : 1.f;
        stride *= (uint32_t)L;
    }
}

template <int P>
__device__ __forceinline__ void raw_load(const StencilParams &p, uint32_t nb, uint32_t ls, int mu, int rhs,
                                         RawHop<P> &r)
{
    const uint32_t V = p.V;
    const size_t so = (size_t)rhs * Traits<P>::NCH * V + nb;  // chunk 0 of the neighbour, this right-hand side
    if constexpr (P == F64) {
        const double2 *b = reinterpret_cast<const double2 *>(p.in) + so;
#pragma unroll
        for (int k = 0; k < 12; ++k)
            r.sp[k] = b[(size_t)k * V];
        const double2 *u = reinterpret_cast<const double2 *>(p.U) + (size_t)mu * 6 * V + ls;
#pragma unroll
        for (int k = 0; k < 6; ++k)
            r.lk[k] = u[(size_t)k * V];
    } else if constexpr (P == F32) {
        const float4 *b = reinterpret_cast<const float4 *>(p.in) + so;
#pragma unroll
        for (int k = 0; k < 6; ++k)
            r.sp[k] = b[(size_t)k * V];
        const float4 *u = reinterpret_cast<const float4 *>(p.U) + (size_t)mu * 3 * V + ls;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            r.lk[k] = u[(size_t)k * V];
    } else {
        const uint4 *b = reinterpret_cast<const uint4 *>(p.in) + so;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            r.sp[k] = b[(size_t)k * V];
        r.sc = scale_ptr<P>(p.in, V, p.nrhs)[(size_t)rhs * V + nb];
        const uint2 *u = reinterpret_cast<const uint2 *>(p.U) + (size_t)mu * 3 * V + ls;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            r.lk[k] = u[(size_t)k * V];
    }
}

template <int P>
__device__ __forceinline__ void decode(const RawHop<P> &r, cx<typename Traits<P>::real> (&ps)[12],
                                       cx<typename Traits<P>::real> (&u)[9])
{
    using T = typename Traits<P>::real;
    if constexpr (P == F64) {
#pragma unroll
        for (int k = 0; k < 12; ++k)
            ps[k] = cx<double>{r.sp[k].x, r.sp[k].y};
#pragma unroll
        for (int k = 0; k < 6; ++k)
            u[k] = cx<double>{r.lk[k].x, r.lk[k].y};
    } else if constexpr (P == F32) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            ps[2 * k] = cx<float>{r.sp[k].x, r.sp[k].y};
            ps[2 * k + 1] = cx<float>{r.sp[k].z, r.sp[k].w};
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            u[2 * k] = cx<float>{r.lk[k].x, r.lk[k].y};
            u[2 * k + 1] = cx<float>{r.lk[k].z, r.lk[k].w};
        }
    } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const uint32_t w[4] = {r.sp[k].x, r.sp[k].y, r.sp[k].z, r.sp[k].w};
#pragma unroll
            for (int j = 0; j < 4; ++j)
                ps[4 * k + j] = unpack2<P>(w[j]);  // site scale applied in the accumulate
            u[2 * k] = unpack2<P>(r.lk[k].x);
            u[2 * k + 1] = unpack2<P>(r.lk[k].y);
        }
    }
    // row 2 = conj(row0 x row1)
    const cx<T> a0 = u[0], a1 = u[1], a2 = u[2], b0 = u[3], b1 = u[4], b2 = u[5];
    cx<T> c0 = cmul(a1, b2), c1 = cmul(a2, b0), c2 = cmul(a0, b1);
    c0 = cfma(cx<T>{-a2.re, -a2.im}, b1, c0);
    c1 = cfma(cx<T>{-a0.re, -a0.im}, b2, c1);
    c2 = cfma(cx<T>{-a1.re, -a1.im}, b0, c2);
    u[6] = cconj(c0);
    u[7] = cconj(c1);
    u[8] = cconj(c2);
}

// The projected hop of raw (still packed) data: g = U (1 + SIG g_MU) psi
// (ADJ = 0) or U^dag (1 + SIG g_MU) psi (ADJ = 1), the 16-bit site scale not
// applied.  FP16 storage takes the packed f16 / dot2 path of wl_hop16.h.
template <int P, int MU, int SIG, int ADJ>
__device__ __forceinline__ void hop_g(const RawHop<P> &r, cx<typename Traits<P>::real> (&g)[6],
                                      typename Traits<P>::real one)
{
    using T = typename Traits<P>::real;
    if constexpr (P == F16S) {
        hf2 ps[12], u[9], h[6];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            ps[4 * k] = as_hf2(r.sp[k].x);
            ps[4 * k + 1] = as_hf2(r.sp[k].y);
            ps[4 * k + 2] = as_hf2(r.sp[k].z);
            ps[4 * k + 3] = as_hf2(r.sp[k].w);
            u[2 * k] = as_hf2(r.lk[k].x);
            u[2 * k + 1] = as_hf2(r.lk[k].y);
        }
        rebuild_row16(u);
        project16<MU, SIG>(ps, h);
        su3_mv16<ADJ>(u, h, g);
    } else {
        cx<T> ps[12], u[9], h[6];
        decode<P>(r, ps, u);
        project<MU, SIG>(ps, h, one);
        if constexpr (ADJ)
            su3_adj_mv(u, h, g);
        else
            su3_mv(u, h, g);
    }
}

template <int P, int DAG, int H>
__device__ __forceinline__ void compute_hop(const RawHop<P> &r, float sg, cx<typename Traits<P>::real> (&acc)[12],
                                            typename Traits<P>::real one)
{
    using T = typename Traits<P>::real;
    constexpr int MU = H / 2;
    constexpr int SF = DAG ? 1 : -1;
    constexpr int SIG = (H % 2 == 0) ? SF : -SF;
    cx<T> g[6];
    hop_g<P, MU, SIG, H % 2>(r, g, one);
    // the hop is linear in the neighbour spinor, so a 16-bit site's scale
    // multiplies the accumulate coefficient instead of its 24 components
    if constexpr (Traits<P>::SCALED)
        accum<MU, SIG>(acc, g, (T)sg * r.sc);
    else
        accum<MU, SIG>(acc, g, (T)sg);
}

template <int P, int G, int H>
__device__ __forceinline__ void load_group(const StencilParams &p, uint32_t s, int rhs, const Hops &hp,
                                           RawHop<P> (&buf)[2 * G])
{
    constexpr int slot = ((H / G) % 2) * G;
#pragma unroll
    for (int j = 0; j < G; ++j) {
        const int h = H + j;
        raw_load<P>(p, hp.nb[h], (h % 2 == 0) ? s : hp.nb[h], h / 2, rhs, buf[slot + j]);
    }
    // keep the group's loads here: the scheduler would otherwise sink them
    // next to their first use and serialise the pipeline
    __builtin_amdgcn_sched_barrier(0);
}

template <int P, int DAG, int G, int H, int NH = 8>
__device__ __forceinline__ void pipe(const StencilParams &p, uint32_t s, int rhs, const Hops &hp,
                                     RawHop<P> (&buf)[2 * G], cx<typename Traits<P>::real> (&acc)[12])
{
    if constexpr (H < NH) {
        if constexpr (H % G == 0 && H + G < NH)
            load_group<P, G, H + G>(p, s, rhs, hp, buf);
        compute_hop<P, DAG, H>(buf[((H / G) % 2) * G + H % G], hp.sg[H], acc, (typename Traits<P>::real)p.one);
        pipe<P, DAG, G, H + 1, NH>(p, s, rhs, hp, buf, acc);
    }
}

template <int P, int DAG, int G>
__device__ __forceinline__ void hop_site_pipe(const StencilParams &p, uint32_t s, int rhs,
                                              cx<typename Traits<P>::real> (&acc)[12])
{
    Hops hp;
    make_hops(p, s, hp);
    RawHop<P> buf[2 * G];
    load_group<P, G, 0>(p, s, rhs, hp, buf);
    pipe<P, DAG, G, 0>(p, s, rhs, hp, buf, acc);
}

// Stencil code variants (chosen per launch by the autotuner):
//   0: straight-line hops, compiler-scheduled loads (any R)
//   1, 2, 3: pipelined hops with G = 1, 2, 4 hops per stage (R = 1)
template <int P, int VAR>
struct VarG {
    static constexpr int G = VAR == 1 ? 1 : VAR == 2 ? 2 : 4;
};

template <int P>
__device__ __forceinline__ void scale_site(cx<typename Traits<P>::real> (&v)[12], typename Traits<P>::real sc)
{
#pragma unroll
    for (int k = 0; k < 12; ++k)
        v[k] = cx<typename Traits<P>::real>{v[k].re * sc, v[k].im * sc};
}

// Spatial hops of the t-walk are pipelined G at a time; FP64 does not carry
// the site's own spinor (register budget) and reloads it, a near reuse.
// Workgroup -> (tile, right-hand-side group).  Single-group launches use
// blockIdx.x as the tile.  With ng > 1 groups the grid is one-dimensional
// and, among the workgroups that land on one XCD (b = 8 k + xcd under the
// round-robin dispatch), the group index runs fastest: the ng groups of a
// tile execute back to back on the same XCD, so the links and neighbour
// spinors they share are re-read from that XCD's L2 instead of HBM.  The
// tile keeps b's XCD (bt = b mod 8), so the per-XCD tile orders below still
// apply; ntile is a multiple of 8 there, which makes the map a bijection.
// Group-major order (gmaj = 1) runs one group after the other over all
// tiles instead: each group then streams the lattice as a one-group launch
// does (its neighbour spinors stay in L2 as there), at the price of fetching
// the links once per group; b mod 8 = bt mod 8 again keeps the tile orders.
__device__ __forceinline__ uint32_t tile_group(const StencilParams &p, int &g)
{
    const uint32_t b = blockIdx.x;
    if (p.ng == 1) {
        g = 0;
        return b;
    }
    if (p.gmaj) {
        const uint32_t q = fdiv(b, p.f_ntile);
        g = (int)q;
        return b - q * p.ntile;
    }
    const uint32_t k = b >> 3;
    const uint32_t q = fdiv(k, p.f_ng);
    g = (int)(k - q * p.ng);
    return (q << 3) | (b & 7u);
}

template <int P>
struct TwalkG {
    static constexpr int G = P == F64 ? 1 : P == F32 ? 2 : 3;
    static constexpr bool CARRY_SELF = P != F64;
    static constexpr bool EARLY_T = P != F64;  // issue the forward-t loads before the spatial hops
};

// t-walk column length of code variants 4, 5, 6
__host__ __device__ constexpr int twalk_T(int var) { return var == 4 ? 4 : var == 5 ? 8 : 16; }

// Round a site to what the 16-bit format will store (so that fused
// reductions see exactly the stored values).
template <int P>
__device__ __forceinline__ void round_site(cx<float> (&v)[12])
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

// Domain-wall epilogue (Sec. II-B, eq. (2)) for slice s5 = col mod ns of a
// 5-d vector: out = (m0 + 5) in - H in / 2 - P_up in(s5 + 1) - P_dn in(s5 - 1),
// where the neighbour past either end of the fifth dimension is replaced by
// -m times the slice at the other end.  P_up = P_- and P_dn = P_+ for D_DW;
// the adjoint swaps them (the hop then already uses the adjoint projectors).
// With gamma_5 = diag(1, 1, -1, -1), P_+ keeps spins 0, 1 (components 0..5)
// and P_- spins 2, 3 (components 6..11).
template <int P, int DAG>
__device__ __forceinline__ void dw_epilogue(const StencilParams &p, uint32_t s, int col,
                                            const cx<typename Traits<P>::real> (&in)[12],
                                            const cx<typename Traits<P>::real> (&acc)[12],
                                            cx<typename Traits<P>::real> (&o)[12])
{
    using T = typename Traits<P>::real;
    const int ns = p.ns;
    const int s5 = col % ns, base = col - s5;
    const bool top = s5 + 1 == ns, bot = s5 == 0;
    const T cu = top ? (T)p.dw_m : T(-1), cd = bot ? (T)p.dw_m : T(-1);
    cx<T> up[12], dn[12];
    load_site<P>(p.in, p.V, p.nrhs, s, top ? base : col + 1, up);
    load_site<P>(p.in, p.V, p.nrhs, s, bot ? base + ns - 1 : col - 1, dn);
    const T diag = (T)p.dw_diag, half = T(0.5);
    // P_up selects components [ub, ub + 6), P_dn the other six
    constexpr int ub = DAG ? 0 : 6, db = DAG ? 6 : 0;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        cx<T> v{fma(-half, acc[k].re, diag * in[k].re), fma(-half, acc[k].im, diag * in[k].im)};
        if (k >= ub && k < ub + 6)
            v = rfma(cu, up[k], v);
        if (k >= db && k < db + 6)
            v = rfma(cd, dn[k], v);
        o[k] = v;
    }
}

// Residual epilogue (apply 3): o = aux - o, o holding D in at this site,
// exactly as a separate pass r = b - w over the stored w would form it.
template <int P>
__device__ __forceinline__ void residual_epilogue(const StencilParams &p, uint32_t s, int col,
                                                  cx<typename Traits<P>::real> (&o)[12])
{
    cx<typename Traits<P>::real> b[12];
    load_site<P>(p.aux, p.V, p.nrhs, s, col, b);
#pragma unroll
    for (int k = 0; k < 12; ++k)
        o[k] = cx<typename Traits<P>::real>{b[k].re - o[k].re, b[k].im - o[k].im};
}

// Tile count and right-hand-side groups of a launch (see tile_group).
inline void set_groups(StencilParams &p, uint32_t tiles, uint32_t ng)
{
    p.ng = ng;
    p.f_ng = make_fastdiv(ng);
    p.ntile = ng > 1 ? (tiles + 7u) & ~7u : tiles;
    p.f_ntile = make_fastdiv(p.ntile);
    p.nblk = (int)p.ntile;
}

}  // namespace wl
