// wl_stencil_kern.h -- the stencil kernels as templates over the storage
// precision and their launchers; each wl_stencil_<prec>.hip instantiates
// them for one precision (paper Sec. II-B, eq. (1); Table I cost).
#pragma once

#include "wl_brick.h"
#include "wl_stencil_dev.h"

namespace wl {

// ---------------------------------------------------------------- t-walk
// Each thread walks a column of T sites along t.  The decoded spinor of the
// current site and the backward-t contribution of the next site,
// U_t(x)^dag (1 -+ g_t) psi(x), computed while U_t(x) and psi(x) are in
// registers, are carried to the next step; every t-direction spinor and
// link is therefore read from memory once per column instead of three and
// two times, and the accesses of the co-resident workgroups (the same t
// steps of neighbouring (x, y, z) blocks) stay close in time.
// Columns across lanes (lanes_lg = lg > 0): segment j of the 64 >> lg lanes
// of every wavefront walks column grp 2^lg + j of the same sites, so one
// link fetch per instruction serves 2^lg right-hand sides or domain-wall
// slices (whose s +- 1 neighbours the slice's own wavefront loaded).
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
    __shared__ double lds[(NV > 0 ? NV : 1) * 8 * 4];
    int grp;
    const uint32_t bt = tile_group(p, grp);
    const int lg = p.lanes_lg;
    const uint32_t lane = threadIdx.x & 63u, seg = 64u >> lg;
    const uint32_t tsite = ((threadIdx.x >> 6) << (6 - lg)) + (lane & (seg - 1u));
    const int rhs = (grp << lg) + (int)(lane >> (6 - lg));
    if (p.skip) {  // solver loop: every column of this workgroup has stopped
        bool all = true;
        for (int r = 0; r < (1 << lg); ++r)
            all = all && p.skip[(grp << lg) + r].frozen;
        if (all)
            return;
    }
    const uint32_t unit = tile_of(bt, p.ntile, p.xcd ? 1 : 0);
    const uint32_t chunk = unit / nbxyz;
    const uint32_t sx = (unit - chunk * nbxyz) * (blockDim.x >> lg) + tsite;
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
            // (enforced halo: the wrapping hop into t = 0 comes from the face buffer)
            R_ gb = (t0 == 0 && p.halo_t) ? R_(0) : (t0 == 0 && anti_t) ? R_(-1) : R_(1);
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
                R_ gf = (wf && p.halo_t) ? R_(0) : (wf && anti_t) ? R_(-1) : R_(1);
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
            if constexpr (APPLY == 2) {
                dw_epilogue<P, DAG>(p, s, rhs, self, acc, o);
            } else if constexpr (APPLY) {
#pragma unroll
                for (int i = 0; i < 12; ++i)
                    o[i] = cx<R_>{fma(-kap, acc[i].re, self[i].re), fma(-kap, acc[i].im, self[i].im)};
            } else {
#pragma unroll
                for (int i = 0; i < 12; ++i)
                    o[i] = acc[i];
            }
            if constexpr (APPLY == 3)
                residual_epilogue<P>(p, s, rhs, o);
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
            if constexpr (RED == RED_SR) {
                cx<R_> a[12], b[12], c[12];
                load_site<P>(p.aux, p.V, p.nrhs, s, rhs, a);
                load_site<P>(p.aux2, p.V, p.nrhs, s, rhs, b);
                load_site<P>(p.aux3, p.V, p.nrhs, s, rhs, c);
                sr_values(self, o, a, b, c, red);
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
        if (lg == 0) {
            block_sum<NV>(red, lds);
            if (threadIdx.x == 0) {
#pragma unroll
                for (int k = 0; k < NV; ++k)
                    p.partials[((size_t)k * p.nrhs + rhs) * p.nblk + bt] = red[k];
            }
        } else {
            block_sum_lanes<NV>(red, lds, lg);
            if ((int)threadIdx.x < (1 << lg)) {
#pragma unroll
                for (int k = 0; k < NV; ++k)
                    p.partials[((size_t)k * p.nrhs + (grp << lg) + threadIdx.x) * p.nblk + bt] = red[k];
            }
        }
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
                    if constexpr (APPLY == 3)
                        residual_epilogue<P>(p, s, r0 + r, o);
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
            if constexpr (RED == RED_SR) {
                cx<T> in[12], a[12], b[12], c[12];
                load_site<P>(p.in, p.V, p.nrhs, s, r0 + r, in);
                load_site<P>(p.aux, p.V, p.nrhs, s, r0 + r, a);
                load_site<P>(p.aux2, p.V, p.nrhs, s, r0 + r, b);
                load_site<P>(p.aux3, p.V, p.nrhs, s, r0 + r, c);
                sr_values(in, o, a, b, c, &red[NV * r]);
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

template <int P, int DAG, int R, int VAR>
inline hipError_t launch_v(dim3 grid, dim3 block, const StencilParams &p, hipStream_t st)
{
    if (p.apply == 3) {  // the residual aux - D in (FP64 / FP32)
        if constexpr (P == F64 || P == F32) {
            if (p.red == RED_NONE)
                hipLaunchKernelGGL((stencil_kernel<P, DAG, R, RED_NONE, 3, VAR>), grid, block, 0, st, p);
            else if (p.red == RED_NORM)
                hipLaunchKernelGGL((stencil_kernel<P, DAG, R, RED_NORM, 3, VAR>), grid, block, 0, st, p);
            else
                return hipErrorInvalidValue;
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
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
    case RED_SR: hipLaunchKernelGGL((stencil_kernel<P, DAG, R, RED_SR, 1, VAR>), grid, block, 0, st, p); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int P, int DAG>
inline hipError_t launch_twalk(const LaunchCfg &cfg, StencilParams p, hipStream_t st)
{
    const int T = twalk_T(cfg.var);
    if (p.L[3] % T != 0 || cfg.block > 256)
        return hipErrorInvalidValue;
    const uint32_t nxyz = (uint32_t)p.L[0] * p.L[1] * p.L[2];
    const uint32_t tile = (uint32_t)cfg.block >> p.lanes_lg;
    const uint32_t nbxyz = (nxyz + tile - 1) / tile;
    const uint32_t units = nbxyz * (uint32_t)(p.L[3] / T);
    set_groups(p, units, (uint32_t)p.nrhs >> p.lanes_lg);
    if ((uint64_t)p.ntile * p.ng > 0x7fffffffull)
        return hipErrorInvalidValue;
    dim3 grid(p.ntile * p.ng), block(cfg.block);
    if (p.apply == 3) {  // the residual aux - D in (FP64 / FP32)
        if constexpr (P == F64 || P == F32) {
            if (p.red == RED_NONE)
                hipLaunchKernelGGL((twalk_kernel<P, DAG, RED_NONE, 3>), grid, block, 0, st, p, T, nxyz, nbxyz);
            else if (p.red == RED_NORM)
                hipLaunchKernelGGL((twalk_kernel<P, DAG, RED_NORM, 3>), grid, block, 0, st, p, T, nxyz, nbxyz);
            else
                return hipErrorInvalidValue;
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    if (p.apply == 2) {  // domain wall: the reductions CG on the normal equations needs
        switch (p.red) {
        case RED_NONE: hipLaunchKernelGGL((twalk_kernel<P, DAG, RED_NONE, 2>), grid, block, 0, st, p, T, nxyz, nbxyz); break;
        case RED_NORM: hipLaunchKernelGGL((twalk_kernel<P, DAG, RED_NORM, 2>), grid, block, 0, st, p, T, nxyz, nbxyz); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
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
    case RED_SR: hipLaunchKernelGGL((twalk_kernel<P, DAG, RED_SR, 1>), grid, block, 0, st, p, T, nxyz, nbxyz); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int P, int DAG, int R>
inline hipError_t launch_t(const LaunchCfg &cfg, StencilParams p, hipStream_t st)
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
        case VAR_BRICK: return launch_brick<P, DAG>(cfg, p, st);
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
inline hipError_t launch_r(const LaunchCfg &cfg, StencilParams p, hipStream_t st)
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
    // a multi-lattice solve (one column per thread): frozen columns are
    // skipped, and the fused reduction (chosen at run time, uniform over the
    // item) goes to partial [value][pcol0 + column][site tile]
    const int red = R == 1 ? p.red : RED_NONE;
    if (R == 1 && p.skip && p.skip[p.pcol0 + r0].frozen)
        return;
    double rv[RED_NVAL_MAX] = {};
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
            if constexpr (R == 1) {
                if (red == RED_NORM) {
#pragma unroll
                    for (int k = 0; k < 12; ++k)
                        rv[0] = fma((double)o[k].re, (double)o[k].re, fma((double)o[k].im, (double)o[k].im, rv[0]));
                } else if (red == RED_DOTV) {
                    cx<T> v[12];
                    load_site<P>(p.aux, p.V, p.nrhs, s, r0, v);
#pragma unroll
                    for (int k = 0; k < 12; ++k) {
                        rv[0] = fma((double)v[k].re, (double)o[k].re, fma((double)v[k].im, (double)o[k].im, rv[0]));
                        rv[1] = fma((double)v[k].re, (double)o[k].im, fma(-(double)v[k].im, (double)o[k].re, rv[1]));
                    }
                } else if (red == RED_BICG) {
                    cx<T> v[12];
                    load_site<P>(p.aux, p.V, p.nrhs, s, r0, v);
                    bicg_values(in, o, v, rv);
                } else if (red == RED_SR) {
                    cx<T> a[12], b[12], c[12];
                    load_site<P>(p.aux, p.V, p.nrhs, s, r0, a);
                    load_site<P>(p.aux2, p.V, p.nrhs, s, r0, b);
                    load_site<P>(p.aux3, p.V, p.nrhs, s, r0, c);
                    sr_values(in, o, a, b, c, rv);
                }
            }
        }
    }
    if (red != RED_NONE) {  // uniform: every thread of the workgroup takes part
        __shared__ double lds_mr[RED_NVAL_MAX * 8];
        block_sum<RED_NVAL_MAX>(rv, lds_mr);
        if (threadIdx.x == 0) {
            const int nv = red_nval(red);
            for (int k = 0; k < nv; ++k)
                p.partials[((size_t)k * p.pncol + p.pcol0 + r0) * p.pstride + lt] = rv[k];
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

template <int P, int DAG, int R, int VAR>
inline const void *multi_fn(bool persistent)
{
    return persistent ? reinterpret_cast<const void *>(&multi_kernel<P, DAG, R, VAR>)
                      : reinterpret_cast<const void *>(&multi_direct_kernel<P, DAG, R, VAR>);
}

template <int P, int DAG>
inline const void *multi_pick(int rpt, int var, bool persistent)
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

// Stencil launch of one storage precision (instantiated per precision).
template <int P>
hipError_t launch_stencil_p(int dagger, const LaunchCfg &cfg, const StencilParams &p, hipStream_t st)
{
    return dagger ? launch_r<P, 1>(cfg, p, st) : launch_r<P, 0>(cfg, p, st);
}

// Multi-lattice kernel of one storage precision (instantiated per precision).
template <int P>
const void *multi_kernel_p(int dagger, int rpt, int var, bool persistent)
{
    return dagger ? multi_pick<P, 1>(rpt, var, persistent) : multi_pick<P, 0>(rpt, var, persistent);
}

}  // namespace wl
