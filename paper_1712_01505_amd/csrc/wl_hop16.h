// wl_hop16.h -- one hop of the Wilson stencil (paper Sec. II-B, eq. (1)) for
// FP16 storage with the gfx950 packed half-precision units: the rank-2 spin
// projection in packed f16 adds, and the SU(3) x half-spinor product and the
// rebuilt third link row with v_dot2 (two f16 x f16 products, exact in FP32,
// added to an FP32 accumulator).  Compared with converting every stored value
// to FP32 first, a complex multiply-add takes two instructions instead of
// four; the products are exact and every sum is FP32, and the only further
// roundings are the projected half-spinor and the rebuilt third row, each
// held in f16 like the stored operands they come from.
#pragma once

#include "wl_common.h"

namespace wl {

typedef _Float16 hf2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ hf2 as_hf2(uint32_t w) { return __builtin_bit_cast(hf2, w); }
__device__ __forceinline__ hf2 h_i(hf2 z) { return hf2{-z.y, z.x}; }  // i z

// Upper two spin rows of (1 + SIG g_MU) psi in packed f16 (chiral basis, as
// project() in wl_hop.h): p[3 spin + colour], h[3 spin + colour].
template <int MU, int SIG>
__device__ __forceinline__ void project16(const hf2 (&p)[12], hf2 (&h)[6])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const hf2 p0 = p[a], p1 = p[3 + a], p2 = p[6 + a], p3 = p[9 + a];
        if constexpr (MU == 0) {  // A = [[0, i], [i, 0]]
            h[a] = SIG > 0 ? p0 + h_i(p3) : p0 - h_i(p3);
            h[3 + a] = SIG > 0 ? p1 + h_i(p2) : p1 - h_i(p2);
        } else if constexpr (MU == 1) {  // A = [[0, -1], [1, 0]]
            h[a] = SIG > 0 ? p0 - p3 : p0 + p3;
            h[3 + a] = SIG > 0 ? p1 + p2 : p1 - p2;
        } else if constexpr (MU == 2) {  // A = [[i, 0], [0, -i]]
            h[a] = SIG > 0 ? p0 + h_i(p2) : p0 - h_i(p2);
            h[3 + a] = SIG > 0 ? p1 - h_i(p3) : p1 + h_i(p3);
        } else {  // A = 1
            h[a] = SIG > 0 ? p0 + p2 : p0 - p2;
            h[3 + a] = SIG > 0 ? p1 + p3 : p1 - p3;
        }
    }
}

// v_dot2_f32_f16 computes a.x b.x + a.y b.y + c with exact f16 products and
// an FP32 sum; neg_hi / neg_lo negate the high / low half of b.  The compiler
// emits only the accumulate-in-place form without source modifiers (each
// negation or zero start would cost another instruction), so the products are
// written as whole blocks of these instructions.  A DOT result must not be
// read by another kind of instruction for three wait states (the compiler
// pads its own DOTs; it cannot see into an asm block), so every block ends
// with s_nop 2; inside a block results are only read back as the
// accumulator of the same instruction, which needs no wait.  Outputs are
// early-clobber: the block writes them while it still reads its inputs.

#define CHAIN0 \
        "v_dot2_f32_f16 %0, %6, %15, 0 neg_hi:[0,1,0]\n" \
        "v_dot2_f32_f16 %3, %6, %18, 0\n" \
        "v_dot2_f32_f16 %1, %9, %15, 0 neg_hi:[0,1,0]\n" \
        "v_dot2_f32_f16 %4, %9, %18, 0\n" \
        "v_dot2_f32_f16 %2, %12, %15, 0 neg_hi:[0,1,0]\n" \
        "v_dot2_f32_f16 %5, %12, %18, 0\n" \
        "v_dot2_f32_f16 %0, %7, %16, %0 neg_hi:[0,1,0]\n" \
        "v_dot2_f32_f16 %3, %7, %19, %3\n" \
        "v_dot2_f32_f16 %1, %10, %16, %1 neg_hi:[0,1,0]\n" \
        "v_dot2_f32_f16 %4, %10, %19, %4\n" \
        "v_dot2_f32_f16 %2, %13, %16, %2 neg_hi:[0,1,0]\n" \
        "v_dot2_f32_f16 %5, %13, %19, %5\n" \
        "v_dot2_f32_f16 %0, %8, %17, %0 neg_hi:[0,1,0]\n" \
        "v_dot2_f32_f16 %3, %8, %20, %3\n" \
        "v_dot2_f32_f16 %1, %11, %17, %1 neg_hi:[0,1,0]\n" \
        "v_dot2_f32_f16 %4, %11, %20, %4\n" \
        "v_dot2_f32_f16 %2, %14, %17, %2 neg_hi:[0,1,0]\n" \
        "v_dot2_f32_f16 %5, %14, %20, %5\n" \
        "s_nop 2"
#define CHAIN1 \
        "v_dot2_f32_f16 %0, %6, %15, 0\n" \
        "v_dot2_f32_f16 %3, %6, %18, 0 neg_hi:[0,1,0]\n" \
        "v_dot2_f32_f16 %1, %9, %15, 0\n" \
        "v_dot2_f32_f16 %4, %9, %18, 0 neg_hi:[0,1,0]\n" \
        "v_dot2_f32_f16 %2, %12, %15, 0\n" \
        "v_dot2_f32_f16 %5, %12, %18, 0 neg_hi:[0,1,0]\n" \
        "v_dot2_f32_f16 %0, %7, %16, %0\n" \
        "v_dot2_f32_f16 %3, %7, %19, %3 neg_hi:[0,1,0]\n" \
        "v_dot2_f32_f16 %1, %10, %16, %1\n" \
        "v_dot2_f32_f16 %4, %10, %19, %4 neg_hi:[0,1,0]\n" \
        "v_dot2_f32_f16 %2, %13, %16, %2\n" \
        "v_dot2_f32_f16 %5, %13, %19, %5 neg_hi:[0,1,0]\n" \
        "v_dot2_f32_f16 %0, %8, %17, %0\n" \
        "v_dot2_f32_f16 %3, %8, %20, %3 neg_hi:[0,1,0]\n" \
        "v_dot2_f32_f16 %1, %11, %17, %1\n" \
        "v_dot2_f32_f16 %4, %11, %20, %4 neg_hi:[0,1,0]\n" \
        "v_dot2_f32_f16 %2, %14, %17, %2\n" \
        "v_dot2_f32_f16 %5, %14, %20, %5 neg_hi:[0,1,0]\n" \
        "s_nop 2"
#define ROWBLOCK \
        "v_dot2_f32_f16 %0, %8, %10, 0 neg_lo:[0,1,0]\n" \
        "v_dot2_f32_f16 %3, %8, %13, 0 neg_lo:[0,1,0] neg_hi:[0,1,0]\n" \
        "v_dot2_f32_f16 %1, %6, %11, 0 neg_lo:[0,1,0]\n" \
        "v_dot2_f32_f16 %4, %6, %14, 0 neg_lo:[0,1,0] neg_hi:[0,1,0]\n" \
        "v_dot2_f32_f16 %2, %7, %9, 0 neg_lo:[0,1,0]\n" \
        "v_dot2_f32_f16 %5, %7, %12, 0 neg_lo:[0,1,0] neg_hi:[0,1,0]\n" \
        "v_dot2_f32_f16 %0, %7, %11, %0 neg_hi:[0,1,0]\n" \
        "v_dot2_f32_f16 %3, %7, %14, %3\n" \
        "v_dot2_f32_f16 %1, %8, %9, %1 neg_hi:[0,1,0]\n" \
        "v_dot2_f32_f16 %4, %8, %12, %4\n" \
        "v_dot2_f32_f16 %2, %6, %10, %2 neg_hi:[0,1,0]\n" \
        "v_dot2_f32_f16 %5, %6, %13, %5\n" \
        "s_nop 2"

// g = M h for one spin row, M(a, b) = U(a, b) (ADJ = 0) or conj(U(b, a))
// (ADJ = 1); m in a-major order, hs = h with halves swapped:
//   U h:      re = U.re h.re - U.im h.im,   im = U.re h.im + U.im h.re
//   U^dag h:  re = U.re h.re + U.im h.im,   im = U.re h.im - U.im h.re
template <int ADJ>
__device__ __forceinline__ void mv3_16(const hf2 (&m)[9], const hf2 *h, const hf2 *hs, float (&re)[3], float (&im)[3])
{
    if constexpr (ADJ == 0) {
        asm(CHAIN0
            : "=&v"(re[0]), "=&v"(re[1]), "=&v"(re[2]), "=&v"(im[0]), "=&v"(im[1]), "=&v"(im[2])
            : "v"(m[0]), "v"(m[1]), "v"(m[2]), "v"(m[3]), "v"(m[4]), "v"(m[5]), "v"(m[6]), "v"(m[7]), "v"(m[8]),
              "v"(h[0]), "v"(h[1]), "v"(h[2]), "v"(hs[0]), "v"(hs[1]), "v"(hs[2]));
    } else {
        asm(CHAIN1
            : "=&v"(re[0]), "=&v"(re[1]), "=&v"(re[2]), "=&v"(im[0]), "=&v"(im[1]), "=&v"(im[2])
            : "v"(m[0]), "v"(m[1]), "v"(m[2]), "v"(m[3]), "v"(m[4]), "v"(m[5]), "v"(m[6]), "v"(m[7]), "v"(m[8]),
              "v"(h[0]), "v"(h[1]), "v"(h[2]), "v"(hs[0]), "v"(hs[1]), "v"(hs[2]));
    }
}

__device__ __forceinline__ hf2 h_swap(hf2 z) { return hf2{z.y, z.x}; }

// Third row of a two-row SU(3) link, u[6..8] = conj(row0 x row1): with
// x = row 0, y = row 1 and (b, c, d) cyclic,
//   x_c y_d - x_d y_c:  re = [x_c.re y_d.re - x_c.im y_d.im] + [-x_d.re y_c.re + x_d.im y_c.im]
//                       im = [x_c.re y_d.im + x_c.im y_d.re] + [-x_d.re y_c.im - x_d.im y_c.re]
// (each bracket one v_dot2); the row is rounded to f16 like the stored rows.
__device__ __forceinline__ void rebuild_row16(hf2 (&u)[9])
{
    const hf2 ys0 = h_swap(u[3]), ys1 = h_swap(u[4]), ys2 = h_swap(u[5]);
    float re[3], im[3];
    // operands: %0..%2 re, %3..%5 im, %6..%8 x, %9..%11 y, %12..%14 swapped y
    asm(ROWBLOCK
        : "=&v"(re[0]), "=&v"(re[1]), "=&v"(re[2]), "=&v"(im[0]), "=&v"(im[1]), "=&v"(im[2])
        : "v"(u[0]), "v"(u[1]), "v"(u[2]), "v"(u[3]), "v"(u[4]), "v"(u[5]), "v"(ys0), "v"(ys1), "v"(ys2));
#pragma unroll
    for (int b = 0; b < 3; ++b)
        u[6 + b] = hf2{(_Float16)re[b], (_Float16)(-im[b])};
}

// g = U h (ADJ = 0) or U^dag h (ADJ = 1) for both spin rows, in FP32.
template <int ADJ>
__device__ __forceinline__ void su3_mv16(const hf2 (&u)[9], const hf2 (&h)[6], cx<float> (&g)[6])
{
    hf2 m[9], hs[6];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            m[3 * a + b] = ADJ ? u[3 * b + a] : u[3 * a + b];
#pragma unroll
    for (int k = 0; k < 6; ++k)
        hs[k] = h_swap(h[k]);
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) {
        float re[3], im[3];
        mv3_16<ADJ>(m, &h[3 * sp], &hs[3 * sp], re, im);
#pragma unroll
        for (int a = 0; a < 3; ++a)
            g[3 * sp + a] = cx<float>{re[a], im[a]};
    }
}

#undef CHAIN0
#undef CHAIN1
#undef ROWBLOCK

}  // namespace wl
