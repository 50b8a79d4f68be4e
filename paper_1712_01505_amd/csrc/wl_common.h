// wl_common.h -- device-side building blocks shared by the gfx950 kernels:
// storage traits of the packed layouts, site/link loads and stores with
// precision conversion, complex arithmetic, fast integer division, the
// XCD-aware tile order and deterministic wavefront/block reductions.
//
// Packed layouts (see include/wilson.h):
//   spinor  [nrhs][chunk][V] of 16-byte chunks; component k = 3*spin + colour
//           lives in chunk k / CPC at slot k % CPC (CPC = complex per chunk).
//           16-bit formats append [nrhs][V] FP32 per-site scales.
//   gauge   [mu][unit][V]; the two stored rows (6 complex) are split into
//           LINK_UNITS units of LINK_CPU complex each.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wl {

enum Prec { F64 = 0, F32 = 1, BF16S = 2, F16S = 3 };

template <typename T>
struct cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }

// a*b + c
template <typename T>
__device__ __forceinline__ cx<T> cfma(cx<T> a, cx<T> b, cx<T> c)
{
    c.re = fma(a.re, b.re, c.re);
    c.re = fma(-a.im, b.im, c.re);
    c.im = fma(a.re, b.im, c.im);
    c.im = fma(a.im, b.re, c.im);
    return c;
}
// conj(a)*b + c
template <typename T>
__device__ __forceinline__ cx<T> cjfma(cx<T> a, cx<T> b, cx<T> c)
{
    c.re = fma(a.re, b.re, c.re);
    c.re = fma(a.im, b.im, c.re);
    c.im = fma(a.re, b.im, c.im);
    c.im = fma(-a.im, b.re, c.im);
    return c;
}
// a*b with explicit fused operations (the library is built with
// -ffp-contract=off so that every kernel variant rounds identically)
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b)
{
    return cx<T>{fma(a.re, b.re, -(a.im * b.im)), fma(a.re, b.im, a.im * b.re)};
}
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) { return cx<T>{a.re, -a.im}; }
// s*a + c (real s)
template <typename T>
__device__ __forceinline__ cx<T> rfma(T s, cx<T> a, cx<T> c) { return cx<T>{fma(s, a.re, c.re), fma(s, a.im, c.im)}; }
// s*(i a) + c (real s)
template <typename T>
__device__ __forceinline__ cx<T> ifma(T s, cx<T> a, cx<T> c) { return cx<T>{fma(-s, a.im, c.re), fma(s, a.re, c.im)}; }

// ---------------------------------------------------------------- 16-bit reals
__device__ __forceinline__ uint32_t f32_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u)
        return 0x7fc0u;  // NaN stays NaN
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return u >> 16;
}
__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ uint32_t f32_to_f16(float f)
{
    _Float16 h = (_Float16)f;  // round to nearest even
    return (uint32_t)__builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float f16_to_f32(uint32_t h) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(h & 0xffffu)); }

template <int P>
__device__ __forceinline__ uint32_t pack2(float re, float im)
{
    if constexpr (P == BF16S)
        return f32_to_bf16(re) | (f32_to_bf16(im) << 16);
    else
        return f32_to_f16(re) | (f32_to_f16(im) << 16);
}
template <int P>
__device__ __forceinline__ cx<float> unpack2(uint32_t w)
{
    if constexpr (P == BF16S)
        return cx<float>{bf16_to_f32(w & 0xffffu), bf16_to_f32(w >> 16)};
    else
        return cx<float>{f16_to_f32(w & 0xffffu), f16_to_f32(w >> 16)};
}

// ---------------------------------------------------------------- traits
template <int P>
struct Traits;
template <>
struct Traits<F64> {
    using real = double;
    static constexpr int CPC = 1, NCH = 12, SCALED = 0;
    static constexpr int LINK_UNITS = 6, LINK_CPU = 1, LINK_UNIT_BYTES = 16;
};
template <>
struct Traits<F32> {
    using real = float;
    static constexpr int CPC = 2, NCH = 6, SCALED = 0;
    static constexpr int LINK_UNITS = 3, LINK_CPU = 2, LINK_UNIT_BYTES = 16;
};
template <>
struct Traits<BF16S> {
    using real = float;
    static constexpr int CPC = 4, NCH = 3, SCALED = 1;
    static constexpr int LINK_UNITS = 3, LINK_CPU = 2, LINK_UNIT_BYTES = 8;
};
template <>
struct Traits<F16S> {
    using real = float;
    static constexpr int CPC = 4, NCH = 3, SCALED = 1;
    static constexpr int LINK_UNITS = 3, LINK_CPU = 2, LINK_UNIT_BYTES = 8;
};

// Bytes per site per right-hand side of a packed spinor / per direction of a link.
__host__ __device__ constexpr int spinor_site_bytes(int p) { return p == F64 ? 192 : p == F32 ? 96 : 52; }
__host__ __device__ constexpr int link_site_bytes(int p) { return p == F64 ? 96 : p == F32 ? 48 : 24; }

// ---------------------------------------------------------------- spinor access
// A packed spinor field: base pointer, volume, number of right-hand sides.
struct Field {
    void *p;
    uint32_t V;
    int nrhs;
};
struct CField {
    const void *p;
    uint32_t V;
    int nrhs;
};

// Stores of a kernel's final output that nothing in the same kernel reads
// again can bypass the caches' allocation (non-temporal), leaving L2 to the
// neighbour data the stencil re-reads.
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef unsigned nt_u4 __attribute__((ext_vector_type(4)));
template <bool NT>
__device__ __forceinline__ void st16(double2 *p, double2 v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(nt_d2{v.x, v.y}, reinterpret_cast<nt_d2 *>(p));
    else
        *p = v;
}
template <bool NT>
__device__ __forceinline__ void st16(float4 *p, float4 v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(nt_f4{v.x, v.y, v.z, v.w}, reinterpret_cast<nt_f4 *>(p));
    else
        *p = v;
}
template <bool NT>
__device__ __forceinline__ void st16(uint4 *p, uint4 v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(nt_u4{v.x, v.y, v.z, v.w}, reinterpret_cast<nt_u4 *>(p));
    else
        *p = v;
}
template <bool NT>
__device__ __forceinline__ void st4(float *p, float v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <int P>
__device__ __forceinline__ const float *scale_ptr(const void *base, uint32_t V, int nrhs)
{
    return reinterpret_cast<const float *>(reinterpret_cast<const char *>(base) + (size_t)nrhs * V * 48);
}

template <int P>
__device__ __forceinline__ void load_site(const void *base, uint32_t V, int nrhs, uint32_t s, int rhs,
                                          cx<typename Traits<P>::real> (&v)[12])
{
    const size_t off = (size_t)rhs * Traits<P>::NCH * V + s;
    if constexpr (P == F64) {
        const double2 *b = reinterpret_cast<const double2 *>(base) + off;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            double2 d = b[(size_t)k * V];
            v[k] = cx<double>{d.x, d.y};
        }
    } else if constexpr (P == F32) {
        const float4 *b = reinterpret_cast<const float4 *>(base) + off;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            float4 d = b[(size_t)k * V];
            v[2 * k] = cx<float>{d.x, d.y};
            v[2 * k + 1] = cx<float>{d.z, d.w};
        }
    } else {
        const uint4 *b = reinterpret_cast<const uint4 *>(base) + off;
        const float sc = scale_ptr<P>(base, V, nrhs)[(size_t)rhs * V + s];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uint4 d = b[(size_t)k * V];
            cx<float> a0 = unpack2<P>(d.x), a1 = unpack2<P>(d.y), a2 = unpack2<P>(d.z), a3 = unpack2<P>(d.w);
            v[4 * k + 0] = cx<float>{a0.re * sc, a0.im * sc};
            v[4 * k + 1] = cx<float>{a1.re * sc, a1.im * sc};
            v[4 * k + 2] = cx<float>{a2.re * sc, a2.im * sc};
            v[4 * k + 3] = cx<float>{a3.re * sc, a3.im * sc};
        }
    }
}

// As load_site, but 16-bit formats return the stored (unit-range) values and
// the site scale separately (sc = 1 for FP64/FP32).
template <int P>
__device__ __forceinline__ void load_site_unscaled(const void *base, uint32_t V, int nrhs, uint32_t s, int rhs,
                                                   cx<typename Traits<P>::real> (&v)[12],
                                                   typename Traits<P>::real &sc)
{
    if constexpr (Traits<P>::SCALED) {
        const size_t off = (size_t)rhs * Traits<P>::NCH * V + s;
        const uint4 *b = reinterpret_cast<const uint4 *>(base) + off;
        sc = scale_ptr<P>(base, V, nrhs)[(size_t)rhs * V + s];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uint4 d = b[(size_t)k * V];
            v[4 * k + 0] = unpack2<P>(d.x);
            v[4 * k + 1] = unpack2<P>(d.y);
            v[4 * k + 2] = unpack2<P>(d.z);
            v[4 * k + 3] = unpack2<P>(d.w);
        }
    } else {
        load_site<P>(base, V, nrhs, s, rhs, v);
        sc = typename Traits<P>::real(1);
    }
}

template <int P, bool NT = false>
__device__ __forceinline__ void store_site(void *base, uint32_t V, int nrhs, uint32_t s, int rhs,
                                           const cx<typename Traits<P>::real> (&v)[12])
{
    const size_t off = (size_t)rhs * Traits<P>::NCH * V + s;
    if constexpr (P == F64) {
        double2 *b = reinterpret_cast<double2 *>(base) + off;
#pragma unroll
        for (int k = 0; k < 12; ++k)
            st16<NT>(&b[(size_t)k * V], make_double2(v[k].re, v[k].im));
    } else if constexpr (P == F32) {
        float4 *b = reinterpret_cast<float4 *>(base) + off;
#pragma unroll
        for (int k = 0; k < 6; ++k)
            st16<NT>(&b[(size_t)k * V], make_float4(v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im));
    } else {
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < 12; ++k)
            m = fmaxf(m, fmaxf(fabsf(v[k].re), fabsf(v[k].im)));
        const float inv = m > 0.f ? 1.0f / m : 0.f;
        uint4 *b = reinterpret_cast<uint4 *>(base) + off;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uint4 d;
            d.x = pack2<P>(v[4 * k + 0].re * inv, v[4 * k + 0].im * inv);
            d.y = pack2<P>(v[4 * k + 1].re * inv, v[4 * k + 1].im * inv);
            d.z = pack2<P>(v[4 * k + 2].re * inv, v[4 * k + 2].im * inv);
            d.w = pack2<P>(v[4 * k + 3].re * inv, v[4 * k + 3].im * inv);
            st16<NT>(&b[(size_t)k * V], d);
        }
        float *scp = const_cast<float *>(scale_ptr<P>(base, V, nrhs));
        st4<NT>(&scp[(size_t)rhs * V + s], m);
    }
}

// Store a site and replace v by exactly what was stored (16-bit formats
// quantise once: site maximum, scale, round to nearest even).
template <int P, bool NT = false>
__device__ __forceinline__ void store_site_q(void *base, uint32_t V, int nrhs, uint32_t s, int rhs,
                                             cx<typename Traits<P>::real> (&v)[12])
{
    if constexpr (Traits<P>::SCALED) {
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < 12; ++k)
            m = fmaxf(m, fmaxf(fabsf(v[k].re), fabsf(v[k].im)));
        const float inv = m > 0.f ? 1.0f / m : 0.f;
        const size_t off = (size_t)rhs * 3 * V + s;
        uint4 *b = reinterpret_cast<uint4 *>(base) + off;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uint32_t w[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                w[j] = pack2<P>(v[4 * k + j].re * inv, v[4 * k + j].im * inv);
                const cx<float> q = unpack2<P>(w[j]);
                v[4 * k + j] = cx<float>{q.re * m, q.im * m};
            }
            st16<NT>(&b[(size_t)k * V], make_uint4(w[0], w[1], w[2], w[3]));
        }
        float *scp = const_cast<float *>(scale_ptr<P>(base, V, nrhs));
        st4<NT>(&scp[(size_t)rhs * V + s], m);
    } else {
        store_site<P, NT>(base, V, nrhs, s, rhs, v);
    }
}

// Load the two stored rows of U_mu(s) and rebuild row 2 = conj(row0 x row1)
// (valid for SU(3): unitary with det 1).  u[3*row + col].
template <int P>
__device__ __forceinline__ void load_link(const void *U, uint32_t V, int mu, uint32_t s,
                                          cx<typename Traits<P>::real> (&u)[9])
{
    using T = typename Traits<P>::real;
    if constexpr (P == F64) {
        const double2 *b = reinterpret_cast<const double2 *>(U) + (size_t)mu * 6 * V + s;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            double2 d = b[(size_t)k * V];
            u[k] = cx<double>{d.x, d.y};
        }
    } else if constexpr (P == F32) {
        const float4 *b = reinterpret_cast<const float4 *>(U) + (size_t)mu * 3 * V + s;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float4 d = b[(size_t)k * V];
            u[2 * k] = cx<float>{d.x, d.y};
            u[2 * k + 1] = cx<float>{d.z, d.w};
        }
    } else {
        const uint2 *b = reinterpret_cast<const uint2 *>(U) + (size_t)mu * 3 * V + s;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uint2 d = b[(size_t)k * V];
            u[2 * k] = unpack2<P>(d.x);
            u[2 * k + 1] = unpack2<P>(d.y);
        }
    }
    // row 2 = conj(row0 x row1)
    cx<T> a0 = u[0], a1 = u[1], a2 = u[2], b0 = u[3], b1 = u[4], b2 = u[5];
    cx<T> c0 = cmul(a1, b2), c1 = cmul(a2, b0), c2 = cmul(a0, b1);
    c0 = cfma(cx<T>{-a2.re, -a2.im}, b1, c0);
    c1 = cfma(cx<T>{-a0.re, -a0.im}, b2, c1);
    c2 = cfma(cx<T>{-a1.re, -a1.im}, b0, c2);
    u[6] = cconj(c0);
    u[7] = cconj(c1);
    u[8] = cconj(c2);
}

// ---------------------------------------------------------------- fast division
// q = floor(n / d) for n < 2^31 via a 32-bit multiply-high (round-up magic
// number, Granlund & Montgomery 1994).
struct FastDiv {
    uint32_t d, m, l;
};
static inline FastDiv make_fastdiv(uint32_t d)
{
    uint32_t l = 0;
    while ((1ull << l) < d)
        ++l;
    uint64_t m = ((1ull << 32) * ((1ull << l) - d)) / d + 1;
    return FastDiv{d, (uint32_t)m, l};
}
__device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv f) { return (__umulhi(n, f.m) + n) >> f.l; }

// ---------------------------------------------------------------- tile order
// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  With remapping, XCD k processes one contiguous range of tiles, so the
// +-x, +-y, +-z neighbours of a tile are mostly in the same L2.
__device__ __forceinline__ uint32_t tile_of(uint32_t b, uint32_t nb, int xcd)
{
    if (!xcd)
        return b;
    const uint32_t q = nb >> 3, r = nb & 7u, k = b & 7u, j = b >> 3;
    return k * q + (k < r ? k : r) + j;
}

// Slab orders (xcd modes 2..5): XCD k owns the z-slab [k Zs, (k+1) Zs),
// Zs = Lz / 8, cut into y-chunks of Yc = Ly >> (mode - 2) rows; it walks the
// chunks one after the other, each t-major (t, z, y, x).  The +-t (and +-z)
// neighbours of the sites in flight were then fetched at most two chunk
// t-slices (Lx Yc Zs sites) earlier by the same XCD, i.e. are in its L2;
// smaller chunks shorten that distance at the price of misses on the chunk
// faces in y.  Needs Lz % 8 == 0, Ly % 2^(mode - 2) == 0 and a block size
// dividing V / 8 (the host checks).
struct SlabOrder {
    FastDiv f_chunk, f_slice, f_plane;  // divisions by chunk_n, slice_n, plane_n
    uint32_t chunk_n;                   // Lx Yc Zs Lt: sites of one chunk
    uint32_t slice_n;                   // Lx Yc Zs: one t-slice of a chunk
    uint32_t plane_n;                   // Lx Yc: one z-plane of a chunk slice
    uint32_t xy;                        // Lx Ly
    uint32_t zs;                        // Lz / 8
    uint32_t vslice;                    // Lx Ly Lz
};

__device__ __forceinline__ uint32_t slab_site(uint32_t b, uint32_t tid, uint32_t block, const SlabOrder &o)
{
    const uint32_t k = b & 7u, j = b >> 3;
    uint32_t r = j * block + tid;  // position in XCD k's walk
    const uint32_t c = fdiv(r, o.f_chunk);
    r -= c * o.chunk_n;
    const uint32_t t = fdiv(r, o.f_slice);
    r -= t * o.slice_n;
    const uint32_t z = fdiv(r, o.f_plane);
    r -= z * o.plane_n;  // r = x + Lx (y - c Yc)
    return r + o.plane_n * c + o.xy * (k * o.zs + z) + o.vslice * t;
}

// ---------------------------------------------------------------- reductions
// RED_BICG values of one site, added to r[0..7]: <in, out> (re, im), |out|^2,
// <v, in> (re, im), <v, out> (re, im), |in|^2; <a, b> = sum conj(a) b, in FP64.
template <typename T>
__device__ __forceinline__ void bicg_values(const cx<T> (&in)[12], const cx<T> (&out)[12], const cx<T> (&v)[12],
                                            double *r)
{
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const double ir = in[k].re, ii = in[k].im, orr = out[k].re, oi = out[k].im, vr = v[k].re, vi = v[k].im;
        r[0] = fma(ir, orr, fma(ii, oi, r[0]));
        r[1] = fma(ir, oi, fma(-ii, orr, r[1]));
        r[2] = fma(orr, orr, fma(oi, oi, r[2]));
        r[3] = fma(vr, ir, fma(vi, ii, r[3]));
        r[4] = fma(vr, ii, fma(-vi, ir, r[4]));
        r[5] = fma(vr, orr, fma(vi, oi, r[5]));
        r[6] = fma(vr, oi, fma(-vi, orr, r[6]));
        r[7] = fma(ir, ir, fma(ii, ii, r[7]));
    }
}
// RED_SR: <in, out>, |out|^2, <a, out>, <b, out>, <c, out> (9 values, accumulated)
template <typename T>
__device__ __forceinline__ void sr_values(const cx<T> (&in)[12], const cx<T> (&out)[12], const cx<T> (&a)[12],
                                          const cx<T> (&b)[12], const cx<T> (&c)[12], double *r)
{
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const double orr = out[k].re, oi = out[k].im;
        r[0] = fma((double)in[k].re, orr, fma((double)in[k].im, oi, r[0]));
        r[1] = fma((double)in[k].re, oi, fma(-(double)in[k].im, orr, r[1]));
        r[2] = fma(orr, orr, fma(oi, oi, r[2]));
        r[3] = fma((double)a[k].re, orr, fma((double)a[k].im, oi, r[3]));
        r[4] = fma((double)a[k].re, oi, fma(-(double)a[k].im, orr, r[4]));
        r[5] = fma((double)b[k].re, orr, fma((double)b[k].im, oi, r[5]));
        r[6] = fma((double)b[k].re, oi, fma(-(double)b[k].im, orr, r[6]));
        r[7] = fma((double)c[k].re, orr, fma((double)c[k].im, oi, r[7]));
        r[8] = fma((double)c[k].re, oi, fma(-(double)c[k].im, orr, r[8]));
    }
}
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

// Deterministic block sum of N values per thread; thread 0 returns the sums.
// `lds` must hold N * (blockDim.x / 64) doubles.
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double *lds)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int i = 0; i < N; ++i)
        v[i] = wave_sum(v[i]);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i)
            lds[i * nw + w] = v[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            double a = 0.0;
            for (int k = 0; k < nw; ++k)
                a += lds[i * nw + k];
            v[i] = a;
        }
    }
}

// Block sums of N values per thread for lane-interleaved right-hand sides:
// a wavefront holds 2^lg segments of 64 >> lg lanes, segment j serving
// right-hand side j.  Thread j < 2^lg returns the sums of segment j over the
// block (lg = 0 is block_sum).  Fixed order, so deterministic.  `lds` must
// hold N * 2^lg * (blockDim.x / 64) doubles.
template <int N>
__device__ __forceinline__ void block_sum_lanes(double (&v)[N], double *lds, int lg)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int seg = 64 >> lg, nl = 1 << lg;
#pragma unroll
    for (int i = 0; i < N; ++i)
        for (int o = seg >> 1; o > 0; o >>= 1)
            v[i] += __shfl_xor(v[i], o, 64);
    if ((lane & (seg - 1)) == 0) {
        const int j = lane / seg;
#pragma unroll
        for (int i = 0; i < N; ++i)
            lds[(i * nl + j) * nw + w] = v[i];
    }
    __syncthreads();
    if ((int)threadIdx.x < nl) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            double a = 0.0;
            for (int k = 0; k < nw; ++k)
                a += lds[(i * nl + threadIdx.x) * nw + k];
            v[i] = a;
        }
    }
}

}  // namespace wl
