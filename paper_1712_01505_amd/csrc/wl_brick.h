// wl_brick.h -- the LDS-staged brick walk (stencil code variant 7) of the
// Wilson-Dirac hopping term (paper Sec. II-B, eq. (1)).
//
// A workgroup owns a brick of B0 x B1 x B2 sites in (x, y, z), one site per
// thread, and walks T consecutive t-slices.  For every slice the packed
// spinors of the brick and of its six face halos (the sites one step outside
// the brick in x, y or z) are staged in LDS:
//   * the brick's own spinors come from registers: each thread loaded its
//     site's spinor at t one step earlier, as the forward-t neighbour of
//     t - 1, and writes it into its LDS slot;
//   * the halo spinors are copied HBM -> LDS by the gfx950 direct-to-LDS
//     loads (global_load_lds_dwordx4 / _dword), which occupy no registers
//     while in flight.
// The six spatial neighbours of a site are then read from LDS (a halo slot
// for the sites on the brick's faces), so every spinor of the slice is read
// from memory once by its owner plus once per face halo it belongs to,
// instead of once per neighbour.  The t direction is carried through the
// walk as in the register t-walk: the forward-t neighbour's raw spinor is
// loaded into registers (it becomes the next slice's own spinor) and the
// backward-t term U_t(x, t-1)^dag (1 -+ g_t) psi(x, t-1) is computed one step
// early and carried.  Links are read by the threads that use them, straight
// into registers.
//
// Several right-hand sides per workgroup (RW > 1): the workgroup is RW
// copies of the brick's threads, copy r serving right-hand side
// group x RW + r with its own LDS stage; all copies pass the same barriers,
// so they load the links of a slice within one step of each other (served
// once from HBM, the rest from L1 / L2) -- the gauge field is common to every
// right-hand side (Sec. II-B).
//
// The hops are accumulated in the order +x, -x, +y, -y, +z, -z, +t, -t as in
// every other variant, so FP64 and FP32 results are bit-identical to them
// (16-bit storage: equal to rounding, as for the t-walk).
#pragma once

#include "wl_stencil_dev.h"

namespace wl {

typedef __attribute__((address_space(3))) void lds_void_t;

// Brick walk geometry (host-computed; see brick_setup).
struct BrickGeom {
    int B[3];         // brick extents in x, y, z; B0 B1 B2 = workgroup size
    int nb[3];        // bricks per direction
    int T;            // t-slices per work unit
    int NB;           // sites per brick
    int NH;           // halo slots in use
    int NHG;          // halo slot groups of 64 (one direct-to-LDS load per group and chunk)
    int NSP;          // slots per chunk in LDS: NB + 64 NHG
    int RW;           // right-hand sides per workgroup (workgroup = RW NB threads)
    uint32_t stage;   // LDS bytes of one right-hand side's stage
    int hoff[7];      // first halo slot of face -x, +x, -y, +y, -z, +z (hoff[6] = NH)
    uint32_t nxyz;    // Lx Ly Lz
    uint32_t nbrick;  // bricks per t-slice
    FastDiv f_b0, f_b01, f_nb0, f_nb01, f_nbrick;
};

// Packed spinor of one site as stored (raw chunks, plus the 16-bit scale).
template <int P>
struct RawSp {
    using C = typename std::conditional<P == F64, double2, typename std::conditional<P == F32, float4, uint4>::type>::type;
    C sp[Traits<P>::NCH];
    float sc;
};

template <int P>
__device__ __forceinline__ void raw_spinor(const StencilParams &p, uint32_t s, int rhs, RawSp<P> &r)
{
    using C = typename RawSp<P>::C;
    const C *b = reinterpret_cast<const C *>(p.in) + (size_t)rhs * Traits<P>::NCH * p.V + s;
#pragma unroll
    for (int k = 0; k < Traits<P>::NCH; ++k)
        r.sp[k] = b[(size_t)k * p.V];
    if constexpr (Traits<P>::SCALED)
        r.sc = scale_ptr<P>(p.in, p.V, p.nrhs)[(size_t)rhs * p.V + s];
    else
        r.sc = 1.f;
}

template <int P>
__device__ __forceinline__ void raw_link(const StencilParams &p, uint32_t s, int mu, RawHop<P> &r)
{
    if constexpr (P == F64) {
        const double2 *u = reinterpret_cast<const double2 *>(p.U) + (size_t)mu * 6 * p.V + s;
#pragma unroll
        for (int k = 0; k < 6; ++k)
            r.lk[k] = u[(size_t)k * p.V];
    } else if constexpr (P == F32) {
        const float4 *u = reinterpret_cast<const float4 *>(p.U) + (size_t)mu * 3 * p.V + s;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            r.lk[k] = u[(size_t)k * p.V];
    } else {
        const uint2 *u = reinterpret_cast<const uint2 *>(p.U) + (size_t)mu * 3 * p.V + s;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            r.lk[k] = u[(size_t)k * p.V];
    }
}

// Copy a stored spinor slot (LDS) into the spinor part of a raw hop.
template <int P>
__device__ __forceinline__ void lds_spinor(const char *smem, int NSP, int slot, RawHop<P> &r)
{
    using C = typename RawSp<P>::C;
    const C *b = reinterpret_cast<const C *>(smem);
#pragma unroll
    for (int k = 0; k < Traits<P>::NCH; ++k)
        r.sp[k] = b[k * NSP + slot];
    if constexpr (Traits<P>::SCALED)
        r.sc = reinterpret_cast<const float *>(smem + (size_t)NSP * Traits<P>::NCH * 16)[slot];
}

// Global (x, y, z) index of halo slot h of the brick with origin o.
__device__ __forceinline__ uint32_t halo_site(const StencilParams &p, const BrickGeom &g, const int (&o)[3], int h)
{
    int f = 0;
#pragma unroll
    for (int i = 1; i < 6; ++i)
        f += h >= g.hoff[i] ? 1 : 0;
    const int mu = f >> 1, pos = h - g.hoff[f];
    // the two brick coordinates across the face, in index order
    const int a = mu == 0 ? 1 : 0, b = mu == 2 ? 1 : 2;
    const int ia = pos % g.B[a], ib = pos / g.B[a];
    int c[3];
    c[a] = o[a] + ia;
    c[b] = o[b] + ib;
    const int L = p.L[mu];
    c[mu] = (f & 1) ? (o[mu] + g.B[mu] == L ? 0 : o[mu] + g.B[mu]) : (o[mu] == 0 ? L - 1 : o[mu] - 1);
    return (uint32_t)c[0] + (uint32_t)p.L[0] * ((uint32_t)c[1] + (uint32_t)p.L[1] * (uint32_t)c[2]);
}

template <int P, int DAG, int RED, int APPLY, int MULTI>
__global__ __launch_bounds__(256) void brick_kernel(StencilParams p, BrickGeom g)
{
    using R_ = typename Traits<P>::real;
    using Ch = typename RawSp<P>::C;
    constexpr int NCH = Traits<P>::NCH;
    constexpr int NV = red_nval(RED);
    constexpr int SF = DAG ? 1 : -1;  // forward hops use (1 + SF g), backward (1 - SF g)
    constexpr bool LINKS_EARLY = Traits<P>::SCALED;  // FP32 and FP64 load each hop's link where it is used (registers)
    extern __shared__ __align__(16) char smem_all[];
    __shared__ double lds_red[(NV > 0 ? NV : 1) * 4];
    int grp;
    const uint32_t bt = tile_group(p, grp);
    // this thread's right-hand side within the workgroup: uniform per
    // wavefront (NB is a multiple of 64), kept in a scalar register so that
    // the address arithmetic that depends on it stays scalar
    const int rl = MULTI ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6) / (g.NB >> 6)) : 0;
    const int rhs = MULTI ? grp * g.RW + rl : grp;
    if (p.skip) {
        bool all = true;
        for (int r = 0; r < (MULTI ? g.RW : 1); ++r)
            all = all && p.skip[(MULTI ? grp * g.RW : grp) + r].frozen;
        if (all)
            return;
    }
    char *smem = smem_all + (size_t)rl * g.stage;
    const uint32_t unit = tile_of(bt, p.ntile, p.xcd ? 1 : 0);
    const uint32_t chunk = fdiv(unit, g.f_nbrick);
    const uint32_t brick = unit - chunk * g.nbrick;
    const int tid = (int)threadIdx.x - rl * g.NB;
    double red[NV > 0 ? NV : 1];
#pragma unroll
    for (int i = 0; i < (NV > 0 ? NV : 1); ++i)
        red[i] = 0.0;
    const int Lt = p.L[3];
    if ((int)chunk * g.T < Lt) {  // padded multi-RHS grids have idle units (uniform per workgroup)
        // brick origin and this thread's site
        const uint32_t q0 = fdiv(brick, g.f_nb0), q1 = fdiv(brick, g.f_nb01);
        const int o[3] = {(int)(brick - q0 * (uint32_t)g.nb[0]) * g.B[0],
                          (int)(q0 - q1 * (uint32_t)g.nb[1]) * g.B[1], (int)q1 * g.B[2]};
        const uint32_t r0 = fdiv((uint32_t)tid, g.f_b0), r1 = fdiv((uint32_t)tid, g.f_b01);
        const int bc_[3] = {tid - (int)r0 * g.B[0], (int)(r0 - r1 * (uint32_t)g.B[1]), (int)r1};
        const int c[3] = {o[0] + bc_[0], o[1] + bc_[1], o[2] + bc_[2]};
        const uint32_t sx = (uint32_t)c[0] + (uint32_t)p.L[0] * ((uint32_t)c[1] + (uint32_t)p.L[1] * (uint32_t)c[2]);
        // spatial neighbours: LDS slot, (x, y, z) index (for the backward links) and boundary sign
        int slot[6];
        uint32_t nbx[6];
        float sg[6];
        {
            const int bstride[3] = {1, g.B[0], g.B[0] * g.B[1]};
            const int pos[3] = {bc_[1] + g.B[1] * bc_[2], bc_[0] + g.B[0] * bc_[2], bc_[0] + g.B[0] * bc_[1]};
            uint32_t stride = 1u;
#pragma unroll
            for (int mu = 0; mu < 3; ++mu) {
                const int L = p.L[mu], B = g.B[mu];
                const bool full = B == L;  // the brick spans the direction: neighbours wrap inside it
                const bool wf = c[mu] == L - 1, wb = c[mu] == 0;
                slot[2 * mu] = bc_[mu] + 1 < B ? tid + bstride[mu]
                               : full        ? tid - (B - 1) * bstride[mu]
                                             : g.NB + g.hoff[2 * mu + 1] + pos[mu];
                slot[2 * mu + 1] = bc_[mu] > 0 ? tid - bstride[mu]
                                   : full      ? tid + (B - 1) * bstride[mu]
                                               : g.NB + g.hoff[2 * mu] + pos[mu];
                const uint32_t span = (uint32_t)(L - 1) * stride;
                nbx[2 * mu] = wf ? sx - span : sx + stride;
                nbx[2 * mu + 1] = wb ? sx + span : sx - stride;
                sg[2 * mu] = (wf && p.bc[mu] < 0) ? -1.f : 1.f;
                sg[2 * mu + 1] = (wb && p.bc[mu] < 0) ? -1.f : 1.f;
                stride *= (uint32_t)L;
            }
        }
        // halo slots this wavefront copies: groups w, w + nw, ... (at most 4)
        const int lane = tid & 63, w = tid >> 6, nw = g.NB >> 6;
        uint32_t hsite[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int h = (w + j * nw) * 64 + lane;
            hsite[j] = h < g.NH ? halo_site(p, g, o, h) : sx;  // padding lanes copy a valid site
        }
        const bool anti_t = p.bc[3] < 0;
        const int t0 = (int)chunk * g.T;
        const R_ one = (R_)p.one;
        RawSp<P> cur;
        raw_spinor<P>(p, sx + g.nxyz * (uint32_t)t0, rhs, cur);
        // prologue: the backward-t hop into the site at t0, carried as the
        // projected half-spinor Cg and its coefficient Cs (sign and 16-bit scale)
        cx<R_> Cg[6];
        R_ Cs;
        {
            const int tb = t0 == 0 ? Lt - 1 : t0 - 1;
            const uint32_t sb = sx + g.nxyz * (uint32_t)tb;
            RawHop<P> rb;
            raw_load<P>(p, sb, sb, 3, rhs, rb);
            hop_g<P, 3, -SF, 1>(rb, Cg, one);
            // (enforced halo: the wrapping hop into t = 0 comes from the face buffer)
            Cs = (t0 == 0 && p.halo_t) ? R_(0) : (t0 == 0 && anti_t) ? R_(-1) : R_(1);
            if constexpr (Traits<P>::SCALED)
                Cs *= rb.sc;
        }
        Ch *lsp = reinterpret_cast<Ch *>(smem);
        float *lsc = reinterpret_cast<float *>(smem + (size_t)g.NSP * NCH * 16);
        const R_ kap = (R_)p.kappa;
        for (int k = 0; k < g.T; ++k) {
            const int t = t0 + k;
            const uint32_t toff = g.nxyz * (uint32_t)t;
            const uint32_t s = sx + toff;
            __syncthreads();  // every read of the previous slice's LDS stage is done
            // stage the slice: own spinor from registers, halo by direct-to-LDS copies
#pragma unroll
            for (int q = 0; q < NCH; ++q)
                lsp[q * g.NSP + tid] = cur.sp[q];
            if constexpr (Traits<P>::SCALED)
                lsc[tid] = cur.sc;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int grp = w + j * nw;
                if (grp < g.NHG) {  // uniform per wavefront
                    const uint32_t hs = hsite[j] + toff;
#pragma unroll
                    for (int q = 0; q < NCH; ++q) {
                        const Ch *src = reinterpret_cast<const Ch *>(p.in) + ((size_t)rhs * NCH + q) * p.V + hs;
                        __builtin_amdgcn_global_load_lds((const void *)src, (lds_void_t *)(lsp + q * g.NSP + g.NB + grp * 64), 16, 0, 0);
                    }
                    if constexpr (Traits<P>::SCALED) {
                        const float *src = scale_ptr<P>(p.in, p.V, p.nrhs) + (size_t)rhs * p.V + hs;
                        __builtin_amdgcn_global_load_lds((const void *)src, (lds_void_t *)(lsc + g.NB + grp * 64), 4, 0, 0);
                    }
                }
            }
            // forward t neighbour (the next slice's own spinor) and U_t(x, t)
            const bool wf = t == Lt - 1;
            const uint32_t sn = sx + g.nxyz * (uint32_t)(wf ? 0 : t + 1);
            RawSp<P> nxt;
            raw_spinor<P>(p, sn, rhs, nxt);
            RawHop<P> rf;
            raw_link<P>(p, s, 3, rf);
            RawHop<P> lnk[6];
            if constexpr (LINKS_EARLY) {
#pragma unroll
                for (int h = 0; h < 6; ++h)
                    raw_link<P>(p, (h & 1) ? nbx[h] + toff : s, h >> 1, lnk[h]);
            }
            __syncthreads();  // the slice is in LDS (waits for the direct-to-LDS copies)
            cx<R_> acc[12];
#pragma unroll
            for (int i = 0; i < 12; ++i)
                acc[i] = cx<R_>{R_(0), R_(0)};
#pragma unroll
            for (int h = 0; h < 6; ++h) {
                RawHop<P> r;
                if constexpr (LINKS_EARLY) {
#pragma unroll
                    for (int q = 0; q < (P == F64 ? 6 : 3); ++q)
                        r.lk[q] = lnk[h].lk[q];
                } else {
                    raw_link<P>(p, (h & 1) ? nbx[h] + toff : s, h >> 1, r);
                }
                lds_spinor<P>(smem, g.NSP, slot[h], r);
                switch (h) {
                case 0: compute_hop<P, DAG, 0>(r, sg[0], acc, one); break;
                case 1: compute_hop<P, DAG, 1>(r, sg[1], acc, one); break;
                case 2: compute_hop<P, DAG, 2>(r, sg[2], acc, one); break;
                case 3: compute_hop<P, DAG, 3>(r, sg[3], acc, one); break;
                case 4: compute_hop<P, DAG, 4>(r, sg[4], acc, one); break;
                default: compute_hop<P, DAG, 5>(r, sg[5], acc, one); break;
                }
            }
            // the site's own spinor (the stored values, scaled), with U_t(x)
            RawHop<P> rs;
            lds_spinor<P>(smem, g.NSP, tid, rs);
            for (int q = 0; q < (P == F64 ? 6 : 3); ++q)
                rs.lk[q] = rf.lk[q];
            cx<R_> self[12];
            {
                cx<R_> u_unused[9];
                decode<P>(rs, self, u_unused);
                if constexpr (Traits<P>::SCALED)
                    scale_site<P>(self, rs.sc);
            }
            // forward t hop: U_t(x) (1 + SF g_t) psi(x + t)
            {
                RawHop<P> r;
                for (int q = 0; q < NCH; ++q)
                    r.sp[q] = nxt.sp[q];
                for (int q = 0; q < (P == F64 ? 6 : 3); ++q)
                    r.lk[q] = rf.lk[q];
                cx<R_> gg[6];
                hop_g<P, 3, SF, 0>(r, gg, one);
                R_ gf = (wf && p.halo_t) ? R_(0) : (wf && anti_t) ? R_(-1) : R_(1);
                if constexpr (Traits<P>::SCALED)
                    gf *= nxt.sc;
                accum<3, SF>(acc, gg, gf);
            }
            // the -t hop last, as in every variant
            accum<3, -SF>(acc, Cg, Cs);
            // backward-t contribution of the next site: U_t(x)^dag (1 - SF g_t) psi(x)
            hop_g<P, 3, -SF, 1>(rs, Cg, one);
            if constexpr (Traits<P>::SCALED)
                Cs = rs.sc;
            else
                Cs = R_(1);
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
                bicg_values(self, o, v, red);
            }
            if constexpr (RED == RED_SR) {
                cx<R_> a[12], b[12], c[12];
                load_site<P>(p.aux, p.V, p.nrhs, s, rhs, a);
                load_site<P>(p.aux2, p.V, p.nrhs, s, rhs, b);
                load_site<P>(p.aux3, p.V, p.nrhs, s, rhs, c);
                sr_values(self, o, a, b, c, red);
            }
            cur = nxt;
        }
    }
    if constexpr (NV > 0) {
        if constexpr (!MULTI) {
            block_sum<NV>(red, lds_red);
            if (threadIdx.x == 0) {
#pragma unroll
                for (int k = 0; k < NV; ++k)
                    p.partials[((size_t)k * p.nrhs + rhs) * p.nblk + bt] = red[k];
            }
        } else {
            // per right-hand side: wavefront sums, then thread r adds the
            // wavefronts of copy r in order
            const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6, nwv = (int)blockDim.x >> 6;
#pragma unroll
            for (int i = 0; i < NV; ++i)
                red[i] = wave_sum(red[i]);
            if (lane == 0) {
#pragma unroll
                for (int i = 0; i < NV; ++i)
                    lds_red[i * nwv + wv] = red[i];
            }
            __syncthreads();
            if ((int)threadIdx.x < g.RW) {
                const int per = g.NB >> 6, r = (int)threadIdx.x;
#pragma unroll
                for (int k = 0; k < NV; ++k) {
                    double a = 0.0;
                    for (int j = 0; j < per; ++j)
                        a += lds_red[k * nwv + r * per + j];
                    p.partials[((size_t)k * p.nrhs + grp * g.RW + r) * p.nblk + bt] = a;
                }
            }
        }
    }
}

// LDS bytes of one staged slice.
inline size_t brick_lds_bytes(int prec, int nsp)
{
    return (size_t)nsp * (prec == F64 ? 192 : prec == F32 ? 96 : 52);
}

// Brick geometry for launch shape (bx, by, bz, T) with rw right-hand sides
// per workgroup on extents L; false if the shape does not tile the lattice
// or exceeds the kernel's limits.
inline bool brick_setup(const int *L, int prec, int bx, int by, int bz, int T, BrickGeom &g, int rw = 1)
{
    const int B[3] = {bx, by, bz};
    const int nbk = bx * by * bz;
    if (nbk < 64 || nbk > 256 || nbk % 64 != 0 || T < 1 || L[3] % T != 0)
        return false;
    int NH = 0;
    for (int mu = 0; mu < 3; ++mu) {
        if (B[mu] < 1 || L[mu] % B[mu] != 0)
            return false;
        g.B[mu] = B[mu];
        g.nb[mu] = L[mu] / B[mu];
    }
    for (int mu = 0; mu < 3; ++mu) {
        const int face = B[mu] == L[mu] ? 0 : nbk / B[mu];
        g.hoff[2 * mu] = NH;
        g.hoff[2 * mu + 1] = NH + face;
        NH += 2 * face;
    }
    g.hoff[6] = NH;
    g.T = T;
    g.NB = nbk;
    g.NH = NH;
    g.NHG = (NH + 63) / 64;
    if (g.NHG > 4 * (nbk / 64))
        return false;  // at most four halo groups per wavefront
    g.NSP = nbk + 64 * g.NHG;
    if ((rw != 1 && rw != 2 && rw != 4) || nbk * rw > 256)
        return false;  // at most 256 threads: the walk's registers need the 256-thread budget
    g.RW = rw;
    g.stage = (uint32_t)brick_lds_bytes(prec, g.NSP);
    if ((size_t)g.stage * rw > 160 * 1024 - 1024)
        return false;
    g.nxyz = (uint32_t)L[0] * L[1] * L[2];
    g.nbrick = (uint32_t)(g.nb[0] * g.nb[1] * g.nb[2]);
    g.f_b0 = make_fastdiv((uint32_t)bx);
    g.f_b01 = make_fastdiv((uint32_t)(bx * by));
    g.f_nb0 = make_fastdiv((uint32_t)g.nb[0]);
    g.f_nb01 = make_fastdiv((uint32_t)(g.nb[0] * g.nb[1]));
    g.f_nbrick = make_fastdiv(g.nbrick);
    return true;
}

template <int P, int DAG, int RED, int APPLY, int MULTI>
inline hipError_t brick_go1(dim3 grid, dim3 block, size_t smem, const StencilParams &p, const BrickGeom &g,
                            hipStream_t st)
{
    // dynamic LDS beyond the default 64 KB: raise this kernel's limit to what
    // the launch needs (the kernel's static LDS counts against the same
    // 160 KB, so the limit is set to the size asked for, not to the maximum)
    static size_t granted = 65536;
    if (smem > granted) {
        const hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void *>(&brick_kernel<P, DAG, RED, APPLY, MULTI>),
            hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess)
            return e;
        granted = smem;
    }
    hipLaunchKernelGGL((brick_kernel<P, DAG, RED, APPLY, MULTI>), grid, block, smem, st, p, g);
    return hipGetLastError();
}

template <int P, int DAG, int RED, int APPLY>
inline hipError_t brick_go(dim3 grid, dim3 block, size_t smem, const StencilParams &p, const BrickGeom &g,
                           hipStream_t st)
{
    return brick_go1<P, DAG, RED, APPLY, 0>(grid, block, smem, p, g, st);
}

// The form with several right-hand sides per workgroup, launched from its
// own translation unit (wl_brick_multi.hip): compiled next to it, the
// one-right-hand-side kernels came out with more registers (FP16 with the
// <r, D p> reduction: 188 instead of 167, one wave per SIMD fewer).
template <int P>
hipError_t brick_multi_dispatch(int dagger, const StencilParams &p, const BrickGeom &g, dim3 grid, dim3 block,
                                size_t smem, hipStream_t st);

template <int P, int DAG>
inline hipError_t launch_brick(const LaunchCfg &cfg, StencilParams p, hipStream_t st)
{
    BrickGeom g{};
    if (!brick_setup(p.L, P, cfg.bx, cfg.by, cfg.bz, cfg.tsteps, g, cfg.lanes) || cfg.block != g.NB * g.RW ||
        p.nrhs % g.RW != 0)
        return hipErrorInvalidValue;
    const uint32_t units = g.nbrick * (uint32_t)(p.L[3] / g.T);
    set_groups(p, units, (uint32_t)(p.nrhs / g.RW));
    if ((uint64_t)p.ntile * p.ng > 0x7fffffffull)
        return hipErrorInvalidValue;
    const dim3 grid(p.ntile * p.ng), block(cfg.block);
    const size_t need = (size_t)g.stage * g.RW, cap = brick_reserve(cfg.wpe);
    if (cap && need > cap)
        return hipErrorInvalidValue;
    const size_t smem = cap ? cap : need;  // a cap reserves more LDS than the slices need
    if (g.RW > 1)
        return brick_multi_dispatch<P>(DAG, p, g, grid, block, smem, st);
    if (p.apply == 3) {  // the residual aux - D in (FP64 / FP32)
        if constexpr (P == F64 || P == F32) {
            if (p.red == RED_NONE)
                return brick_go<P, DAG, RED_NONE, 3>(grid, block, smem, p, g, st);
            if (p.red == RED_NORM)
                return brick_go<P, DAG, RED_NORM, 3>(grid, block, smem, p, g, st);
        }
        return hipErrorInvalidValue;
    }
    if (!p.apply) {
        if (p.red != RED_NONE)
            return hipErrorInvalidValue;
        return brick_go<P, DAG, RED_NONE, 0>(grid, block, smem, p, g, st);
    }
    if (p.apply != 1)
        return hipErrorInvalidValue;
    switch (p.red) {
    case RED_NONE: return brick_go<P, DAG, RED_NONE, 1>(grid, block, smem, p, g, st);
    case RED_NORM: return brick_go<P, DAG, RED_NORM, 1>(grid, block, smem, p, g, st);
    case RED_DOTV: return brick_go<P, DAG, RED_DOTV, 1>(grid, block, smem, p, g, st);
    case RED_DOTIN_NORM: return brick_go<P, DAG, RED_DOTIN_NORM, 1>(grid, block, smem, p, g, st);
    case RED_BICG: return brick_go<P, DAG, RED_BICG, 1>(grid, block, smem, p, g, st);
    case RED_SR: return brick_go<P, DAG, RED_SR, 1>(grid, block, smem, p, g, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace wl
