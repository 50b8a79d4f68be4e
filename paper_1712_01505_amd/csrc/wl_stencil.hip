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

#include "wl_hop.h"
#include "wl_internal.h"

namespace wl {

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

template <int P, int DAG, int H>
__device__ __forceinline__ void compute_hop(const RawHop<P> &r, float sg, cx<typename Traits<P>::real> (&acc)[12],
                                            typename Traits<P>::real one)
{
    using T = typename Traits<P>::real;
    constexpr int MU = H / 2;
    constexpr int SF = DAG ? 1 : -1;
    constexpr int SIG = (H % 2 == 0) ? SF : -SF;
    cx<T> ps[12], u[9], h[6], g[6];
    decode<P>(r, ps, u);
    project<MU, SIG>(ps, h, one);
    if constexpr (H % 2 == 0)
        su3_mv(u, h, g);
    else
        su3_adj_mv(u, h, g);
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
// FP64 with G = 2 and FP32 with G = 4 exceed the register file and spill;
// variants 4-6 (t-walk) exist for every precision.
int max_var(int prec) { return 6; }
bool var_ok(int prec, int var) { return var <= 1 || var >= 4 || (var == 2 && prec != F64) || (var == 3 && prec >= BF16S); }

// ---------------------------------------------------------------- t-walk
// Each thread walks a column of T sites along t.  The decoded spinor of the
// current site and the backward-t contribution of the next site,
// U_t(x)^dag (1 -+ g_t) psi(x), computed while U_t(x) and psi(x) are in
// registers, are carried to the next step; every t-direction spinor and
// link is therefore read from memory once per column instead of three and
// two times, and the accesses of the co-resident workgroups (the same t
// steps of neighbouring (x, y, z) blocks) stay close in time.
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
__device__ __forceinline__ uint32_t tile_group(const StencilParams &p, int &g)
{
    const uint32_t b = blockIdx.x;
    if (p.ng == 1) {
        g = 0;
        return b;
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

template <int P, int DAG, int RED, int APPLY>
// At most 256 threads per workgroup: the walk's live state (carried spinor,
// t-term, pipelined hops) needs more than the 256 registers a 512-thread
// bound leaves (FP64 and FP32 spilled to scratch there); with this bound the
// compiler can spill into accumulation registers instead.
__global__ __launch_bounds__(256) void twalk_kernel(StencilParams p, int T, uint32_t nxyz, uint32_t nbxyz)
{
    using R_ = typename Traits<P>::real;
    constexpr int NV = red_nval(RED);
    constexpr int SF = DAG ? 1 : -1;  // forward hops use (1 + SF g), backward (1 - SF g)
    constexpr int G = TwalkG<P>::G;
    constexpr bool CARRY = TwalkG<P>::CARRY_SELF;
    __shared__ double lds[(NV > 0 ? NV : 1) * 8];
    int rhs;
    const uint32_t bt = tile_group(p, rhs);
    if (p.skip && p.skip[rhs].frozen)
        return;
    const uint32_t unit = tile_of(bt, p.ntile, p.xcd ? 1 : 0);
    const uint32_t chunk = unit / nbxyz;
    const uint32_t sx = (unit - chunk * nbxyz) * blockDim.x + threadIdx.x;
    double red[NV > 0 ? NV : 1];
#pragma unroll
    for (int i = 0; i < (NV > 0 ? NV : 1); ++i)
        red[i] = 0.0;
    if (sx < nxyz && (int)chunk * T < p.L[3]) {  // padded multi-RHS grids have idle units
        // spatial coordinates and neighbours (in the xyz index), fixed along the walk
        const uint32_t q1 = fdiv(sx, p.fx);
        const int x = (int)(sx - q1 * (uint32_t)p.L[0]);
        const uint32_t q2 = fdiv(q1, p.fy);
        const int y = (int)(q1 - q2 * (uint32_t)p.L[1]);
        const int z = (int)q2;
        const int c[3] = {x, y, z};
        Hops sp;  // spatial hops 0..5 (h = 2 mu + dir), sites relative to t = 0
        uint32_t stride = 1u;
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
            const int L = p.L[mu];
            const bool wf = c[mu] == L - 1, wb = c[mu] == 0;
            const uint32_t span = (uint32_t)(L - 1) * stride;
            sp.nb[2 * mu] = wf ? sx - span : sx + stride;
            sp.nb[2 * mu + 1] = wb ? sx + span : sx - stride;
            sp.sg[2 * mu] = (wf && p.bc[mu] < 0) ? -1.f : 1.f;
            sp.sg[2 * mu + 1] = (wb && p.bc[mu] < 0) ? -1.f : 1.f;
            stride *= (uint32_t)L;
        }
        const int Lt = p.L[3];
        const bool anti_t = p.bc[3] < 0;
        const int t0 = (int)chunk * T;
        cx<R_> self[12], C[12];
        // prologue: the backward-t hop into the site at t0
        {
            if constexpr (CARRY)
                load_site<P>(p.in, p.V, p.nrhs, sx + nxyz * (uint32_t)t0, rhs, self);
            const int tb = t0 == 0 ? Lt - 1 : t0 - 1;
            const uint32_t sb = sx + nxyz * (uint32_t)tb;
            RawHop<P> rb;
            raw_load<P>(p, sb, sb, 3, rhs, rb);
            cx<R_> ps[12], u[9], h[6], g[6];
            decode<P>(rb, ps, u);
            project<3, -SF>(ps, h, (R_)p.one);
            su3_adj_mv(u, h, g);
            R_ gb = (t0 == 0 && anti_t) ? R_(-1) : R_(1);
            if constexpr (Traits<P>::SCALED)
                gb *= rb.sc;
#pragma unroll
            for (int k = 0; k < 12; ++k)
                C[k] = cx<R_>{R_(0), R_(0)};
            accum<3, -SF>(C, g, gb);
        }
        const R_ kap = (R_)p.kappa;
        for (int k = 0; k < T; ++k) {
            const int t = t0 + k;
            const uint32_t toff = nxyz * (uint32_t)t;
            const uint32_t s = sx + toff;
            // forward t neighbour and link U_t(x): the far loads, issued first
            const bool wf = t == Lt - 1;
            const uint32_t sn = sx + nxyz * (uint32_t)(wf ? 0 : t + 1);
            RawHop<P> rf;
            if constexpr (TwalkG<P>::EARLY_T)
                raw_load<P>(p, sn, s, 3, rhs, rf);
            Hops hp;
#pragma unroll
            for (int h = 0; h < 6; ++h) {
                hp.nb[h] = sp.nb[h] + toff;
                hp.sg[h] = sp.sg[h];
            }
            // hop order +x, -x, +y, -y, +z, -z, +t, -t as in the other variants; with
            // FP64/FP32 storage the carried -t term is exact (its coefficients are
            // +-1), so the site result rounds exactly as there
            cx<R_> acc[12];
#pragma unroll
            for (int i = 0; i < 12; ++i)
                acc[i] = cx<R_>{R_(0), R_(0)};
            {
                RawHop<P> buf[2 * G];
                load_group<P, G, 0>(p, s, rhs, hp, buf);
                pipe<P, DAG, G, 0, 6>(p, s, rhs, hp, buf, acc);
            }
            if constexpr (!TwalkG<P>::EARLY_T)
                raw_load<P>(p, sn, s, 3, rhs, rf);
            if constexpr (!CARRY)
                load_site<P>(p.in, p.V, p.nrhs, s, rhs, self);
            cx<R_> nxt[12], u[9];
            decode<P>(rf, nxt, u);
            {
                cx<R_> h[6], g[6];
                project<3, SF>(nxt, h, (R_)p.one);
                su3_mv(u, h, g);
                R_ gf = (wf && anti_t) ? R_(-1) : R_(1);
                if constexpr (Traits<P>::SCALED)
                    gf *= rf.sc;
                accum<3, SF>(acc, g, gf);
            }
#pragma unroll
            for (int i = 0; i < 12; ++i)
                acc[i] = cx<R_>{acc[i].re + C[i].re, acc[i].im + C[i].im};
            // backward-t contribution of the next site: U_t(x)^dag (1 - SF g_t) psi(x)
            {
                cx<R_> h[6], g[6];
                project<3, -SF>(self, h, (R_)p.one);
                su3_adj_mv(u, h, g);
#pragma unroll
                for (int i = 0; i < 12; ++i)
                    C[i] = cx<R_>{R_(0), R_(0)};
                accum<3, -SF>(C, g, R_(1));
            }
            // epilogue for site s
            cx<R_> o[12];
            if constexpr (APPLY) {
#pragma unroll
                for (int i = 0; i < 12; ++i)
                    o[i] = cx<R_>{fma(-kap, acc[i].re, self[i].re), fma(-kap, acc[i].im, self[i].im)};
            } else {
#pragma unroll
                for (int i = 0; i < 12; ++i)
                    o[i] = acc[i];
            }
            store_site_q<P, true>(p.out, p.V, p.nrhs, s, rhs, o);
            if constexpr (RED == RED_NORM || RED == RED_DOTIN_NORM) {
#pragma unroll
                for (int i = 0; i < 12; ++i)
                    red[NV - 1] = fma((double)o[i].re, (double)o[i].re, fma((double)o[i].im, (double)o[i].im, red[NV - 1]));
            }
            if constexpr (RED == RED_DOTIN_NORM) {
#pragma unroll
                for (int i = 0; i < 12; ++i) {
                    red[0] = fma((double)self[i].re, (double)o[i].re, fma((double)self[i].im, (double)o[i].im, red[0]));
                    red[1] = fma((double)self[i].re, (double)o[i].im, fma(-(double)self[i].im, (double)o[i].re, red[1]));
                }
            }
            if constexpr (RED == RED_DOTV) {
                cx<R_> v[12];
                load_site<P>(p.aux, p.V, p.nrhs, s, rhs, v);
#pragma unroll
                for (int i = 0; i < 12; ++i) {
                    red[0] = fma((double)v[i].re, (double)o[i].re, fma((double)v[i].im, (double)o[i].im, red[0]));
                    red[1] = fma((double)v[i].re, (double)o[i].im, fma(-(double)v[i].im, (double)o[i].re, red[1]));
                }
            }
            if constexpr (RED == RED_BICG) {
                cx<R_> v[12];
                load_site<P>(p.aux, p.V, p.nrhs, s, rhs, v);
                bicg_values(self, o, v, red);  // accumulates over the t-walk
            }
            if constexpr (CARRY) {  // the forward neighbour becomes the next site
                if constexpr (Traits<P>::SCALED)
                    scale_site<P>(nxt, rf.sc);
#pragma unroll
                for (int i = 0; i < 12; ++i)
                    self[i] = nxt[i];
            }
        }
    }
    if constexpr (NV > 0) {
        block_sum<NV>(red, lds);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < NV; ++k)
                p.partials[((size_t)k * p.nrhs + rhs) * p.nblk + bt] = red[k];
        }
    }
}

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

template <int P, int DAG, int R, int RED, int APPLY, int VAR>
__global__ __launch_bounds__(512) void stencil_kernel(StencilParams p)
{
    using T = typename Traits<P>::real;
    constexpr int NV = red_nval(RED);
    __shared__ double lds[(NV > 0 ? NV : 1) * (R > 1 ? R : 8) * 8];
    int grp;
    const uint32_t bt = tile_group(p, grp);
    // right-hand sides across lanes (R = 1 only): segment j of 64 >> lg lanes
    // of every wavefront serves right-hand side grp 2^lg + j, so the links of
    // a site are fetched once per instruction for all 2^lg of them
    const int lg = p.lanes_lg;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t seg = 64u >> lg;
    const uint32_t tsite = ((threadIdx.x >> 6) << (6 - lg)) + (lane & (seg - 1u));
    const uint32_t tile = blockDim.x >> lg;
    const uint32_t s = p.xcd >= 2 ? slab_site(bt, tsite, tile, p.slab) : tile_of(bt, p.ntile, p.xcd) * tile + tsite;
    const int r0 = (grp << lg) * R + (int)(lane >> (6 - lg));
    if (p.skip) {  // solver loop: every column of this workgroup has stopped
        bool all = true;
        const int rb = (grp << lg) * R;
        for (int r = 0; r < (R << lg); ++r)
            all = all && p.skip[rb + r].frozen;
        if (all)
            return;
    }
    const bool active = s < p.V;
    double red[(NV > 0 ? NV : 1) * R];
#pragma unroll
    for (int i = 0; i < (NV > 0 ? NV : 1) * R; ++i)
        red[i] = 0.0;
    if (active) {
        cx<T> acc[R][12];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < 12; ++k)
                acc[r][k] = cx<T>{T(0), T(0)};
        if constexpr (VAR == 0 || R > 1)
            hop_site<P, DAG, R>(p, s, r0, acc);
        else
            hop_site_pipe<P, DAG, VarG<P, VAR>::G>(p, s, r0, acc[0]);
        const T kap = (T)p.kappa;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            cx<T> o[12];
            if constexpr (APPLY || RED == RED_DOTIN_NORM) {
                cx<T> in[12];
                load_site<P>(p.in, p.V, p.nrhs, s, r0 + r, in);
                if constexpr (APPLY == 2) {
                    dw_epilogue<P, DAG>(p, s, r0 + r, in, acc[r], o);
                } else if constexpr (APPLY) {
#pragma unroll
                    for (int k = 0; k < 12; ++k)
                        o[k] = cx<T>{fma(-kap, acc[r][k].re, in[k].re), fma(-kap, acc[r][k].im, in[k].im)};
                } else {
#pragma unroll
                    for (int k = 0; k < 12; ++k)
                        o[k] = acc[r][k];
                }

                if constexpr (RED == RED_DOTIN_NORM) {
                    double re = 0.0, im = 0.0;
#pragma unroll
                    for (int k = 0; k < 12; ++k) {
                        re = fma((double)in[k].re, (double)o[k].re, fma((double)in[k].im, (double)o[k].im, re));
                        im = fma((double)in[k].re, (double)o[k].im, fma(-(double)in[k].im, (double)o[k].re, im));
                    }
                    red[NV * r + 0] = re;
                    red[NV * r + 1] = im;
                }
            } else {
#pragma unroll
                for (int k = 0; k < 12; ++k)
                    o[k] = acc[r][k];

            }
            store_site_q<P, true>(p.out, p.V, p.nrhs, s, r0 + r, o);
            if constexpr (RED == RED_NORM || RED == RED_DOTIN_NORM) {
                double n2 = 0.0;
#pragma unroll
                for (int k = 0; k < 12; ++k)
                    n2 = fma((double)o[k].re, (double)o[k].re, fma((double)o[k].im, (double)o[k].im, n2));
                red[NV * r + NV - 1] = n2;
            }
            if constexpr (RED == RED_BICG) {
                cx<T> in[12], v[12];
                load_site<P>(p.in, p.V, p.nrhs, s, r0 + r, in);
                load_site<P>(p.aux, p.V, p.nrhs, s, r0 + r, v);
                bicg_values(in, o, v, &red[NV * r]);
            }
            if constexpr (RED == RED_DOTV) {
                cx<T> v[12];
                load_site<P>(p.aux, p.V, p.nrhs, s, r0 + r, v);
                double re = 0.0, im = 0.0;
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    re = fma((double)v[k].re, (double)o[k].re, fma((double)v[k].im, (double)o[k].im, re));
                    im = fma((double)v[k].re, (double)o[k].im, fma(-(double)v[k].im, (double)o[k].re, im));
                }
                red[NV * r + 0] = re;
                red[NV * r + 1] = im;
            }
        }
    }
    if constexpr (NV > 0) {
        if constexpr (R == 1) {
            block_sum_lanes<NV>(red, lds, lg);
            if ((int)threadIdx.x < (1 << lg)) {
#pragma unroll
                for (int k = 0; k < NV; ++k)
                    p.partials[((size_t)k * p.nrhs + (grp << lg) + threadIdx.x) * p.nblk + bt] = red[k];
            }
        } else {
            block_sum<NV * R>(red, lds);
            if (threadIdx.x == 0) {
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int k = 0; k < NV; ++k)
                        p.partials[((size_t)k * p.nrhs + r0 + r) * p.nblk + bt] = red[NV * r + k];
            }
        }
    }
}

bool slab_ok(const int *L, int block, int mode)
{
    if (mode < 2 || mode > 5)
        return false;
    const uint64_t slab = (uint64_t)L[0] * L[1] * (L[2] / 8) * L[3];
    return L[2] % 8 == 0 && L[1] % (1 << (mode - 2)) == 0 && slab % (uint64_t)block == 0;
}

int stencil_nval(int red) { return red_nval(red); }

// Tile count and right-hand-side groups of a launch (see tile_group).
static void set_groups(StencilParams &p, uint32_t tiles, uint32_t ng)
{
    p.ng = ng;
    p.f_ng = make_fastdiv(ng);
    p.ntile = ng > 1 ? (tiles + 7u) & ~7u : tiles;
    p.nblk = (int)p.ntile;
}

template <int P, int DAG, int R, int VAR>
static hipError_t launch_v(dim3 grid, dim3 block, const StencilParams &p, hipStream_t st)
{
    if (p.apply == 2) {  // domain wall: R = 1, variants 0..2, the reductions CG needs
        if constexpr (R == 1 && VAR <= 2) {
            switch (p.red) {
            case RED_NONE: hipLaunchKernelGGL((stencil_kernel<P, DAG, 1, RED_NONE, 2, VAR>), grid, block, 0, st, p); break;
            case RED_NORM: hipLaunchKernelGGL((stencil_kernel<P, DAG, 1, RED_NORM, 2, VAR>), grid, block, 0, st, p); break;
            default: return hipErrorInvalidValue;
            }
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    if (!p.apply) {  // the hopping term alone is only offered without fused reductions
        if (p.red != RED_NONE)
            return hipErrorInvalidValue;
        hipLaunchKernelGGL((stencil_kernel<P, DAG, R, RED_NONE, 0, VAR>), grid, block, 0, st, p);
        return hipGetLastError();
    }
    switch (p.red) {
    case RED_NONE: hipLaunchKernelGGL((stencil_kernel<P, DAG, R, RED_NONE, 1, VAR>), grid, block, 0, st, p); break;
    case RED_NORM: hipLaunchKernelGGL((stencil_kernel<P, DAG, R, RED_NORM, 1, VAR>), grid, block, 0, st, p); break;
    case RED_DOTV: hipLaunchKernelGGL((stencil_kernel<P, DAG, R, RED_DOTV, 1, VAR>), grid, block, 0, st, p); break;
    case RED_DOTIN_NORM:
        hipLaunchKernelGGL((stencil_kernel<P, DAG, R, RED_DOTIN_NORM, 1, VAR>), grid, block, 0, st, p);
        break;
    case RED_BICG: hipLaunchKernelGGL((stencil_kernel<P, DAG, R, RED_BICG, 1, VAR>), grid, block, 0, st, p); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int P, int DAG>
static hipError_t launch_twalk(const LaunchCfg &cfg, StencilParams p, hipStream_t st)
{
    const int T = twalk_T(cfg.var);
    if (p.L[3] % T != 0 || cfg.block > 256)
        return hipErrorInvalidValue;
    const uint32_t nxyz = (uint32_t)p.L[0] * p.L[1] * p.L[2];
    const uint32_t nbxyz = (nxyz + cfg.block - 1) / cfg.block;
    const uint32_t units = nbxyz * (uint32_t)(p.L[3] / T);
    set_groups(p, units, (uint32_t)p.nrhs);
    if ((uint64_t)p.ntile * p.ng > 0x7fffffffull)
        return hipErrorInvalidValue;
    dim3 grid(p.ntile * p.ng), block(cfg.block);
    if (!p.apply) {
        if (p.red != RED_NONE)
            return hipErrorInvalidValue;
        hipLaunchKernelGGL((twalk_kernel<P, DAG, RED_NONE, 0>), grid, block, 0, st, p, T, nxyz, nbxyz);
        return hipGetLastError();
    }
    switch (p.red) {
    case RED_NONE: hipLaunchKernelGGL((twalk_kernel<P, DAG, RED_NONE, 1>), grid, block, 0, st, p, T, nxyz, nbxyz); break;
    case RED_NORM: hipLaunchKernelGGL((twalk_kernel<P, DAG, RED_NORM, 1>), grid, block, 0, st, p, T, nxyz, nbxyz); break;
    case RED_DOTV: hipLaunchKernelGGL((twalk_kernel<P, DAG, RED_DOTV, 1>), grid, block, 0, st, p, T, nxyz, nbxyz); break;
    case RED_DOTIN_NORM:
        hipLaunchKernelGGL((twalk_kernel<P, DAG, RED_DOTIN_NORM, 1>), grid, block, 0, st, p, T, nxyz, nbxyz);
        break;
    case RED_BICG: hipLaunchKernelGGL((twalk_kernel<P, DAG, RED_BICG, 1>), grid, block, 0, st, p, T, nxyz, nbxyz); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static uint32_t pad8(uint32_t n) { return (n + 7u) & ~7u; }

// Number of per-workgroup partials (per right-hand side) a launch with this
// configuration writes.
int stencil_partials(const LaunchCfg &cfg, const int *L, uint32_t V, int nrhs)
{
    const uint32_t tile = (uint32_t)(cfg.block / cfg.lanes);
    uint32_t n = (V + tile - 1) / tile;
    if (cfg.rpt == 1 && cfg.var >= 4) {
        const uint32_t nxyz = (uint32_t)L[0] * L[1] * L[2];
        n = ((nxyz + cfg.block - 1) / cfg.block) * (uint32_t)(L[3] / twalk_T(cfg.var));
    }
    return (int)(nrhs / (cfg.rpt * cfg.lanes) > 1 ? pad8(n) : n);
}

template <int P, int DAG, int R>
static hipError_t launch_t(const LaunchCfg &cfg, StencilParams p, hipStream_t st)
{
    set_groups(p, (uint32_t)p.nblk, (uint32_t)(p.nrhs / (R << p.lanes_lg)));
    if ((uint64_t)p.ntile * p.ng > 0x7fffffffull)
        return hipErrorInvalidValue;
    dim3 grid(p.ntile * p.ng), block(cfg.block);
    if constexpr (R == 1) {
        switch (cfg.var) {
        case 0: return launch_v<P, DAG, 1, 0>(grid, block, p, st);
        case 1: return launch_v<P, DAG, 1, 1>(grid, block, p, st);
        case 2:
            if constexpr (P != F64)
                return launch_v<P, DAG, 1, 2>(grid, block, p, st);
            return hipErrorInvalidValue;
        case 3:
            if constexpr (P == BF16S || P == F16S)
                return launch_v<P, DAG, 1, 3>(grid, block, p, st);
            return hipErrorInvalidValue;
        case 4:
        case 5:
        case 6: return launch_twalk<P, DAG>(cfg, p, st);
        default: return hipErrorInvalidValue;
        }
    } else {
        if (cfg.var != 0)
            return hipErrorInvalidValue;
        return launch_v<P, DAG, R, 0>(grid, block, p, st);
    }
}

// Right-hand sides per thread: FP64 keeps at most 2 (24 FP64 accumulators
// per right-hand side; 3 or more spill at the 256-VGPR budget of a
// 512-thread workgroup), the FP32-arithmetic formats up to 4.
template <int P, int DAG>
static hipError_t launch_r(const LaunchCfg &cfg, StencilParams p, hipStream_t st)
{
    switch (cfg.rpt) {
    case 1: return launch_t<P, DAG, 1>(cfg, p, st);
    case 2: return launch_t<P, DAG, 2>(cfg, p, st);
    case 3:
        if constexpr (P != F64)
            return launch_t<P, DAG, 3>(cfg, p, st);
        return hipErrorInvalidValue;
    case 4:
        if constexpr (P != F64)
            return launch_t<P, DAG, 4>(cfg, p, st);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

int max_rpt(int prec) { return prec == F64 ? 2 : 4; }

hipError_t launch_stencil(int prec, int dagger, const LaunchCfg &cfg, StencilParams p, hipStream_t st)
{
    const int lg = cfg.lanes == 1 ? 0 : cfg.lanes == 2 ? 1 : cfg.lanes == 4 ? 2 : cfg.lanes == 8 ? 3 : -1;
    if (cfg.rpt < 1 || cfg.rpt > 4 || p.nrhs % cfg.rpt != 0 || cfg.block < 64 || cfg.block > 512 ||
        cfg.block % 64 != 0 || lg < 0 ||
        (lg > 0 && (cfg.rpt != 1 || cfg.var >= 4 || p.nrhs % cfg.lanes != 0 || (cfg.block >> lg) < 64)))
        return hipErrorInvalidValue;
    if (p.apply == 2 && (cfg.rpt != 1 || cfg.var > 2 || p.ns < 1 || p.nrhs % p.ns != 0))
        return hipErrorInvalidValue;  // domain wall: one slice per thread, variants 0..2
    if (p.halo_t && cfg.rpt == 1 && cfg.var >= 4)
        return hipErrorInvalidValue;  // the t-walk carries its t hops in registers
    p.lanes_lg = lg;
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
    switch (prec * 2 + (dagger ? 1 : 0)) {
    case 0: return launch_r<F64, 0>(cfg, p, st);
    case 1: return launch_r<F64, 1>(cfg, p, st);
    case 2: return launch_r<F32, 0>(cfg, p, st);
    case 3: return launch_r<F32, 1>(cfg, p, st);
    case 4: return launch_r<BF16S, 0>(cfg, p, st);
    case 5: return launch_r<BF16S, 1>(cfg, p, st);
    case 6: return launch_r<F16S, 0>(cfg, p, st);
    case 7: return launch_r<F16S, 1>(cfg, p, st);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------- multi-lattice
// One persistent grid; each workgroup pops work items (lattice, site tile,
// RHS group; the group index fastest within a lattice) from a device-wide
// counter until the queue is empty, so uneven lattices share one launch.
// counter[0] is the queue head, counter[1] counts workgroups that have left
// the loop: the last one to leave resets both to zero, so the queue is ready
// for the next launch without a host-side reset.  Every workgroup leaves the
// loop once the head passes the total, so the grid always drains.
// One work item: entry (lattice) found by binary search over tile_begin,
// then site tile and RHS group (the group fastest) within it.
template <int P, int DAG, int R, int VAR>
__device__ __forceinline__ void multi_item(const MultiEntry *E, int n, uint32_t t)
{
    using T = typename Traits<P>::real;
    int lo = 0, hi = n - 1;  // last entry with tile_begin <= t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (E[mid].tile_begin <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    const StencilParams &p = E[lo].p;  // fields are read (scalar loads) where used
    const uint32_t local = t - E[lo].tile_begin;
    const uint32_t lt = fdiv(local, p.f_ng);
    const int r0 = (int)(local - lt * p.ng) * R;
    const uint32_t s = lt * blockDim.x + threadIdx.x;
    if (s < p.V) {
        cx<T> acc[R][12];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < 12; ++k)
                acc[r][k] = cx<T>{T(0), T(0)};
        if constexpr (VAR == 0 || R > 1)
            hop_site<P, DAG, R>(p, s, r0, acc);
        else
            hop_site_pipe<P, DAG, VarG<P, VAR>::G>(p, s, r0, acc[0]);
        const T kap = (T)p.kappa;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            cx<T> in[12], o[12];
            load_site<P>(p.in, p.V, p.nrhs, s, r0 + r, in);
#pragma unroll
            for (int k = 0; k < 12; ++k)
                o[k] = cx<T>{fma(-kap, acc[r][k].re, in[k].re), fma(-kap, acc[r][k].im, in[k].im)};
            store_site_q<P, true>(p.out, p.V, p.nrhs, s, r0 + r, o);
        }
    }
}

// Persistent form: a resident grid whose workgroups pop work items from a
// device-wide counter until the queue is empty, so uneven lattices share one
// launch.  counter[0] is the queue head, counter[1] counts workgroups that
// have left the loop: the last one to leave resets both to zero, so the
// queue is ready for the next launch without a host-side reset.  Every
// workgroup leaves the loop once the head passes the total, so the grid
// always drains.
template <int P, int DAG, int R, int VAR>
__global__ __launch_bounds__(512) void multi_kernel(const MultiEntry *E, int n, uint32_t total, unsigned *counter)
{
    __shared__ unsigned item_s;
    if (threadIdx.x == 0)
        item_s = atomicAdd(&counter[0], 1u);
    __syncthreads();
    // the item is uniform across the workgroup: keep it (and the entry
    // lookup that follows from it) in scalar registers
    unsigned t = __builtin_amdgcn_readfirstlane(item_s);
    for (;;) {
        __syncthreads();  // everyone has read item_s
        if (t >= total)
            break;
        // pop the next item now, so the atomic's latency overlaps this one
        if (threadIdx.x == 0)
            item_s = atomicAdd(&counter[0], 1u);
        multi_item<P, DAG, R, VAR>(E, n, t);
        __syncthreads();  // item_s written
        t = __builtin_amdgcn_readfirstlane(item_s);
    }
    if (threadIdx.x == 0) {
        __threadfence();  // this workgroup's last pop precedes its exit count
        if (atomicAdd(&counter[1], 1u) == gridDim.x - 1) {
            atomicExch(&counter[0], 0u);
            atomicExch(&counter[1], 0u);
        }
    }
}

// Direct form: one workgroup per work item (the hardware dispatcher is the
// queue); same items, same results.
template <int P, int DAG, int R, int VAR>
__global__ __launch_bounds__(512) void multi_direct_kernel(const MultiEntry *E, int n, uint32_t total)
{
    const uint32_t t = blockIdx.x;
    if (t < total)
        multi_item<P, DAG, R, VAR>(E, n, t);
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

template <int P, int DAG, int R, int VAR>
static const void *multi_fn(bool persistent)
{
    return persistent ? reinterpret_cast<const void *>(&multi_kernel<P, DAG, R, VAR>)
                      : reinterpret_cast<const void *>(&multi_direct_kernel<P, DAG, R, VAR>);
}

template <int P, int DAG>
static const void *multi_pick(int rpt, int var, bool persistent)
{
    if (rpt == 2)
        return multi_fn<P, DAG, 2, 0>(persistent);
    if constexpr (P != F64)
        if (rpt == 4)
            return multi_fn<P, DAG, 4, 0>(persistent);
    switch (var) {
    case 0: return multi_fn<P, DAG, 1, 0>(persistent);
    case 1: return multi_fn<P, DAG, 1, 1>(persistent);
    case 2:
        if constexpr (P != F64)
            return multi_fn<P, DAG, 1, 2>(persistent);
        return nullptr;
    case 3:
        if constexpr (P == BF16S || P == F16S)
            return multi_fn<P, DAG, 1, 3>(persistent);
        return nullptr;
    default: return nullptr;
    }
}

static const void *multi_kernel_ptr(int prec, int dagger, int rpt, int var, bool persistent)
{
    if (!multi_shape_ok(prec, rpt, var))
        return nullptr;
    switch (prec * 2 + (dagger ? 1 : 0)) {
    case 0: return multi_pick<F64, 0>(rpt, var, persistent);
    case 1: return multi_pick<F64, 1>(rpt, var, persistent);
    case 2: return multi_pick<F32, 0>(rpt, var, persistent);
    case 3: return multi_pick<F32, 1>(rpt, var, persistent);
    case 4: return multi_pick<BF16S, 0>(rpt, var, persistent);
    case 5: return multi_pick<BF16S, 1>(rpt, var, persistent);
    case 6: return multi_pick<F16S, 0>(rpt, var, persistent);
    case 7: return multi_pick<F16S, 1>(rpt, var, persistent);
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
