// wl_hop.h -- device building blocks of one hop of the Wilson stencil, shared
// by the stencil kernels and the even-odd kernels: the rank-2 spin projection
// (1 +- gamma_mu) in the chiral basis, the SU(3) mat-vec with a link or its
// adjoint, and the reconstruction of the four spin rows from the projected
// result (paper Sec. II-B, eq. (1)).
#pragma once

#include "wl_common.h"

namespace wl {

// Upper two spin rows of (1 + SIG g_MU) psi, per colour: h[3*spin + colour].
// Chiral basis: g_MU = [[0, A],[A^dag, 0]], so h = psi_up + SIG A psi_dn.
// `one` is 1 at run time; multiplying the +-1 coefficients by it keeps
// the compiler from turning the fused form into an add, so a 16-bit input
// feeds a mixed-precision FMA directly (no separate conversion).
template <int MU, int SIG, typename T>
__device__ __forceinline__ void project(const cx<T> (&ps)[12], cx<T> (&h)[6], T one = T(1))
{
    const T s = (T)SIG * one;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cx<T> p0 = ps[a], p1 = ps[3 + a], p2 = ps[6 + a], p3 = ps[9 + a];
        if constexpr (MU == 0) {  // A = [[0, i], [i, 0]]
            h[a] = ifma(s, p3, p0);
            h[3 + a] = ifma(s, p2, p1);
        } else if constexpr (MU == 1) {  // A = [[0, -1], [1, 0]]
            h[a] = rfma(-s, p3, p0);
            h[3 + a] = rfma(s, p2, p1);
        } else if constexpr (MU == 2) {  // A = [[i, 0], [0, -i]]
            h[a] = ifma(s, p2, p0);
            h[3 + a] = ifma(-s, p3, p1);
        } else {  // A = 1
            h[a] = rfma(s, p2, p0);
            h[3 + a] = rfma(s, p3, p1);
        }
    }
}

// acc += sg * [g ; SIG A^dag g]  (the full 4-spinor of a projected hop).
template <int MU, int SIG, typename T>
__device__ __forceinline__ void accum(cx<T> (&acc)[12], const cx<T> (&g)[6], T sg)
{
    const T s = sg * (T)SIG;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cx<T> g0 = g[a], g1 = g[3 + a];
        acc[a] = rfma(sg, g0, acc[a]);
        acc[3 + a] = rfma(sg, g1, acc[3 + a]);
        if constexpr (MU == 0) {  // A^dag g = (-i g1, -i g0)
            acc[6 + a] = ifma(-s, g1, acc[6 + a]);
            acc[9 + a] = ifma(-s, g0, acc[9 + a]);
        } else if constexpr (MU == 1) {  // A^dag g = (g1, -g0)
            acc[6 + a] = rfma(s, g1, acc[6 + a]);
            acc[9 + a] = rfma(-s, g0, acc[9 + a]);
        } else if constexpr (MU == 2) {  // A^dag g = (-i g0, i g1)
            acc[6 + a] = ifma(-s, g0, acc[6 + a]);
            acc[9 + a] = ifma(s, g1, acc[9 + a]);
        } else {  // A^dag g = g
            acc[6 + a] = rfma(s, g0, acc[6 + a]);
            acc[9 + a] = rfma(s, g1, acc[9 + a]);
        }
    }
}

// g = U h for both spin rows.
template <typename T>
__device__ __forceinline__ void su3_mv(const cx<T> (&u)[9], const cx<T> (&h)[6], cx<T> (&g)[6])
{
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cx<T> v = cmul(u[3 * a], h[3 * sp]);
            v = cfma(u[3 * a + 1], h[3 * sp + 1], v);
            v = cfma(u[3 * a + 2], h[3 * sp + 2], v);
            g[3 * sp + a] = v;
        }
}
// g = U^dag h for both spin rows.
template <typename T>
__device__ __forceinline__ void su3_adj_mv(const cx<T> (&u)[9], const cx<T> (&h)[6], cx<T> (&g)[6])
{
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cx<T> v = cmul(cconj(u[a]), h[3 * sp]);
            v = cjfma(u[3 + a], h[3 * sp + 1], v);
            v = cjfma(u[6 + a], h[3 * sp + 2], v);
            g[3 * sp + a] = v;
        }
}

}  // namespace wl
