// wl_internal.h -- host-side internals shared by the library's translation
// units: the operator object, kernel parameter blocks and the launch entry
// points each .hip file exports to the host code.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "../../include/wilson.h"
#include "wl_common.h"

namespace wl {

// Launch configuration of the stencil.
struct LaunchCfg {
    int block = 256;  // threads per workgroup (= sites per tile x lanes)
    int rpt = 1;      // right-hand sides per thread
    int xcd = 1;      // tile order: 0 natural, 1 contiguous range per XCD, 2..5 z-slab per XCD walked
                      // t-major in y-chunks of Ly >> (xcd - 2) rows
    int var = 0;      // stencil code variant (0 = straight-line hops; 1..3 = pipelined, R = 1 only)
    int lanes = 1;    // right-hand sides interleaved across the lanes of a wavefront (1, 2, 4, 8; rpt = 1)
    // variant 7 (LDS-staged brick walk): brick extents in x, y, z (bx by bz = block) and t-slices per unit
    int bx = 0, by = 0, bz = 0, tsteps = 0;
    // variant 7: cap of workgroups per CU (0 = none): each workgroup reserves
    // 1/wpe of the CU's LDS, which bounds the waves per SIMD
    int wpe = 0;
    // several right-hand-side groups: 0 = the groups of a tile back to back
    // on one XCD, 1 = one group after the other over the whole lattice
    int gmaj = 0;
};

}  // namespace wl

struct wl_op {
    wl_geom g;
    double kappa;     // Wilson: hopping parameter
    int prec;
    int ns = 0;       // domain wall: fifth-dimension extent (0 = Wilson operator)
    double m0 = 0.0;  // domain wall: Wilson mass of D_W and quark mass m
    double mq = 0.0;
    const void *U;
    uint32_t V;
    std::mutex mu;
    std::map<int, wl::LaunchCfg> launch;  // keyed by nrhs
};

namespace wl {

struct Scalars;

// Reduction requested from a kernel epilogue (partials [nval][nrhs][nblk]).
enum Red {
    RED_NONE = 0,
    RED_NORM = 1,      // |out|^2                           (1 value)
    RED_DOTV = 2,      // <v, out> with v = aux              (2 values: re, im)
    RED_DOTIN_NORM = 3,// <in, out> and |out|^2              (3 values)
    RED_BICG = 4,      // <in, out>, |out|^2, <v, in>, <v, out>, |in|^2 with v = aux (8 values;
                       // BiCGStab's second product: omega, the next rho and |s|^2 together)
    RED_SR = 5         // <in, out>, |out|^2, <aux, out>, <aux2, out>, <aux3, out> (9 values;
                       // the single-reduction BiCGStab's q = D v with aux = rh, aux2 = r, aux3 = u)
};
constexpr int RED_NVAL_MAX = 9;  // values per right-hand side of the largest reduction
constexpr int RED_LAST = RED_SR;
__host__ __device__ constexpr int red_nval(int red)
{
    return red == RED_NORM ? 1 : red == RED_DOTV ? 2 : red == RED_DOTIN_NORM ? 3 : red == RED_BICG ? 8
           : red == RED_SR ? 9 : 0;
}

struct StencilParams {
    const void *U;
    const void *in;
    void *out;
    const void *aux;   // RED_DOTV: the v of <v, out>
    const void *aux2, *aux3;  // RED_SR: the second and third vectors dotted with out
    double *partials;  // per-block partial sums
    FastDiv fx, fy, fz;
    int L[4];
    int bc[4];
    uint32_t V;
    int nrhs;
    double kappa;
    int apply;  // 1: out = in - kappa H in; 0: out = H in; 2: domain wall (ns, dw_diag, dw_m);
                // 3: out = aux - (in - kappa H in), the residual of D in = aux (FP64 / FP32)
    int ns;          // apply 2: columns r form 5-d vectors of ns slices (s = r mod ns)
    double dw_diag;  // apply 2: m0 + 5 (the diagonal of D_W + 1); the hop enters with -1/2
    double dw_m;     // apply 2: quark mass m of the corner blocks
    int red;
    int xcd;
    int nblk;   // number of site tiles (partials per right-hand side)
    // multi-RHS launches: ng right-hand-side groups per tile, interleaved
    // with the tiles (see tile_group); ntile = tiles in the launch, padded
    // to a multiple of 8 when ng > 1
    uint32_t ng, ntile;
    FastDiv f_ng;
    int gmaj;      // 1: group-major block order (see tile_group)
    FastDiv f_ntile;
    int lanes_lg;  // log2 of the right-hand sides interleaved across lanes
    SlabOrder slab;  // xcd >= 2
    const struct Scalars *skip;  // in a solver loop: skip a workgroup whose columns are all frozen
    float one;                   // 1.0 (see project())
    // enforced halo: the t hops that wrap around the lattice are left out
    // here (halo_t = 1) and come from face buffers (halo_pack / halo_finish)
    int halo_t;
    void *halo_send;             // [face 2][rhs][6 complex][Vs], real = double (FP64) or float
    const void *halo_recv;       // same layout, filled by the face copy
    // multi-lattice solves (multi_item): this lattice's columns start at
    // pcol0 of pncol; partials [nval][pncol][pstride] indexed by site tile,
    // and skip[] is indexed by the same global column
    int pcol0, pncol, pstride;
};

// ---- even-odd (wl_eo.hip)
struct EoParams {
    const void *U;
    const void *in;      // half field of the other parity
    const void *self;    // half field of the output parity (c_self term, <self, out>), or null
    const void *dotv;    // RED_DOTV: the v of <v, out>
    const void *dotv2, *dotv3;  // RED_SR: the second and third vectors dotted with out
    void *out;           // half field of the output parity
    double *partials;
    const struct Scalars *skip;
    int L[4], bc[4];
    int parity;          // of the output sites
    int nrhs;
    double c_self, c_hop;  // out = c_self self + c_hop H in
    uint32_t V, Vh;      // set by the launcher
    FastDiv fxh, fy, fz;
    int nblk;
};
hipError_t launch_eo_hop(int prec, int dagger, int red, EoParams p, hipStream_t st);
hipError_t launch_eo_copy(int prec, bool split, const int *L, int nrhs, const void *full_in, void *full_out,
                          void *even, void *odd, hipStream_t st);
int eo_partials(uint32_t Vh);  // per-right-hand-side partials of one eo_hop launch
EoParams eo_params(const wl_op *op, int parity, int nrhs);  // links, extents, parity

// ---- stencil (wl_stencil.hip)
hipError_t launch_stencil(int prec, int dagger, const LaunchCfg &cfg, StencilParams p, hipStream_t st);
// the stencil and multi-lattice kernels of one storage precision P, each
// instantiated in its own translation unit (wl_stencil_<prec>.hip)
template <int P>
hipError_t launch_stencil_p(int dagger, const LaunchCfg &cfg, const StencilParams &p, hipStream_t st);
template <int P>
const void *multi_kernel_p(int dagger, int rpt, int var, bool persistent);
// enforced halo: pack the two t faces' projected half-spinors, and add the
// received faces' hops to the boundary slices
hipError_t launch_halo_pack(int prec, int dagger, const StencilParams &p, hipStream_t st);
hipError_t launch_halo_finish(int prec, int dagger, const StencilParams &p, hipStream_t st);
size_t halo_face_bytes(int prec, uint32_t vs, int nrhs);  // one face, all right-hand sides
int stencil_nval(int red);
int max_rpt(int prec);  // largest right-hand sides per thread the stencil offers
int max_var(int prec);  // largest stencil code variant for R = 1
bool var_ok(int prec, int var);  // variant exists for this precision
int stencil_partials(const LaunchCfg &cfg, const int *L, uint32_t V, int nrhs);  // partials per RHS of one launch
bool slab_ok(const int *L, int block, int mode);  // slab order `mode` usable for these extents and block size
// variant 7: the brick (bx, by, bz) and walk length T tile extents L and fit the kernel's LDS and halo limits
bool brick_ok(const int *L, int prec, int bx, int by, int bz, int T, int wpe = 0, int rw = 1);
constexpr size_t LDS_PER_CU = 160 * 1024;
// dynamic LDS a brick launch reserves for its occupancy cap (0: none)
inline size_t brick_reserve(int wpe) { return wpe > 0 ? (LDS_PER_CU / (size_t)wpe - 512) / 256 * 256 : 0; }
constexpr int VAR_BRICK = 7;

struct MultiEntry {
    StencilParams p;      // per lattice; ng / f_ng = RHS groups per tile
    uint32_t tile_begin;  // first work item of this lattice
};
bool multi_launch_ok(int prec, int rpt, int block, int var);
hipError_t launch_multi(int prec, int dagger, int rpt, int block, int var, const MultiEntry *dev_entries, int n,
                        uint32_t total_items, unsigned *counter, int grid, hipStream_t st);
int multi_grid_size(int prec, int dagger, int rpt, int block, int var);

// Kind-specific stencil parameters of an operator (domain wall: apply 2).
void op_apply_params(const wl_op *op, StencilParams &p);
// Stencil columns of nrhs vectors: nrhs for Wilson, nrhs x ns for domain wall.
inline int op_cols(const wl_op *op, int nrhs) { return op->ns > 0 ? nrhs * op->ns : nrhs; }

hipError_t launch_force(int prec, const wl_op *op, void *out, const void *x, const void *mu, int project,
                        hipStream_t st);

// ---- pack (wl_pack.hip)
hipError_t launch_pack_gauge(int prec, uint32_t V, const void *canon, void *packed, hipStream_t st);
hipError_t launch_pack_spinor(int prec, uint32_t V, int nrhs, const void *canon, void *packed, hipStream_t st);
hipError_t launch_unpack_spinor(int prec, uint32_t V, int nrhs, const void *packed, void *canon, hipStream_t st);
// out = in * f(rhs) where f = 1 (mode 0), s[rhs] (mode 1) or 1/s[rhs] (mode 2, 0 if s == 0);
// s[] is read from device memory with stride `sstride` doubles.
hipError_t launch_convert(int pin, int pout, uint32_t V, int nrhs, const void *in, void *out, const double *s,
                          int sstride, int mode, hipStream_t st);
hipError_t launch_fill_u32(unsigned *p, unsigned v, int n, hipStream_t st);
hipError_t launch_stream_copy(void *dst, const void *src, size_t bytes, hipStream_t st);

// ---- BLAS-1 and solver scalars (wl_blas.hip)
// Per-right-hand-side solver scalars, kept on the device.
struct Scalars {
    double bb;            // |b|^2 of the system being solved
    double rr;            // |r|^2 (iterated)
    double zz;            // CGNR |z|^2
    double ss;            // BiCGStab |s|^2
    double2 alpha, beta, omega, rho;
    double2 rho_prev;     // BiCGStab: rho before the last F_BI_OMEGA_RHO (for reliable updates)
    double tol2;          // converge when rr <= tol2 * bb
    double rr_upd;        // reliable updates: |r|^2 after the previous update (or at the start)
    int flag;             // 0 running, 1 converged, 2 breakdown, 3 NaN/Inf
    int conv_iter;
    int frozen;           // set at the end of an iteration once flag != 0: loop kernels skip the column
    int restart;          // CGNR reliable update without progress: restart the search direction
    int brk;              // merged BiCGStab: 1 rho or omega degenerate, 2 non-finite (acted on at F_BI_CONV)
};

enum BlasOp {
    B_RES = 0,        // r = b - w                      ; |r|^2
    B_CG_XR = 1,      // x += a p ; r -= a w            ; |r|^2
    B_CG_P = 2,       // p = z + beta p
    B_BI_P = 3,       // p = r + beta (p - omega v)
    B_BI_S = 4,       // s = r - alpha v                ; |s|^2
    B_BI_XR = 5,      // x += alpha p + omega s ; r = s - omega t ; |r|^2, <rh, r>  (a3 = rh)
    B_COPY = 6,       // y = x
    B_ZERO = 7,       // y = 0
    B_NORM = 8,       // |x|^2
    B_DOT_NORM = 9,   // <a0, a1> and |a1|^2  (3 values)
    B_CG_RESTART = 10,// p = z for columns whose restart flag is set
    B_BI_XRP = 11,    // x += alpha p + omega s ; r = s - omega t ; p = r + beta (p - omega v) ; |r|^2
                      // (y0 = x, y1 = r, y2 = p, a1 = s, a2 = t, a3 = v)
    // single-reduction forms (one finalize per iteration)
    B_CG1 = 12,       // CGNR: p = z + beta p ; w = q + beta w ; x += alpha p ; r -= alpha w ; |r|^2
                      // (y0 = x, y1 = r, y2 = p, y3 = w, a0 = z, a1 = q)
    B_SR_PV = 13,     // BiCGStab: p = r + beta (p - omega v) ; v = u + beta (v - omega q) ;
                      // <rh, v>, <rh, u>, <u, r>, <u, v>, |u|^2  (9 values;
                      // y0 = p, y1 = v, a0 = r, a1 = u, a2 = q, a3 = rh)
    B_SR_XR = 14,     // BiCGStab: s = r - alpha v ; x += alpha p + omega s ; r = s - omega (u - alpha q) ;
                      // |r|^2  (y0 = x, y1 = r, a0 = p, a1 = v, a2 = u, a3 = q)
    B_INIT = 15       // start of a run from x = 0: x = 0 ; r = b, and y2, y3 = b where given ; |b|^2
                      // (y0 = x, y1 = r, a0 = b)
};
// One column of a segmented (multi-lattice) vector: its lattice's fields
// start `off` bytes into every vector buffer, with V sites and nrhs columns,
// of which this is column r.
struct Seg {
    uint64_t off;
    uint32_t V;
    int nrhs;
    int r;
    int pad;
};
struct BlasParams {
    const Seg *seg;    // segmented vectors: per-column table (blockIdx.y = global column), or null
    void *y0;          // first output / in-out vector
    void *y1;          // second output / in-out vector
    void *y2;          // third in-out vector (B_BI_XRP, B_CG1: p)
    void *y3;          // fourth in-out vector (B_CG1: w)
    const void *a0, *a1, *a2, *a3;  // inputs
    const Scalars *sc;
    double *partials;
    uint32_t V;
    int nrhs;
    int nblk;
    int skip_frozen;   // in a solver loop: skip frozen columns
};
hipError_t launch_blas(int prec, int op, const BlasParams &p, int block, hipStream_t st);
int blas_partials(uint32_t V, int op, int block);  // workgroups (= partial sums per RHS) of one launch
int blas_nval(int op);
int blas_sites_per_thread(int op);

// x64 += s[rhs] * e (e in precision pin); s read from device with stride.
hipError_t launch_accum(int pin, uint32_t V, int nrhs, void *x64, const void *e, const double *s, int sstride,
                        hipStream_t st);

enum FinOp {
    F_INIT_CG = 0,    // vals: |r|^2 (set A), |z|^2 (set B); bb from |b|^2 set C
    F_CG_ALPHA = 1,   // vals: |w|^2
    F_CG_BETA = 2,    // vals: |r|^2 (A), |z|^2 (B)
    F_INIT_BI = 3,    // vals: |r|^2 (A), bb (C)
    F_BI_ALPHA = 4,   // vals: <rh, v>
    F_SUM = 7,        // just reduce set A into out[] (nval x nrhs)
    F_BI_RELIABLE = 8, // after a reliable update replaced r: A = (<rh, r>, |r|^2) -> rr,
                       // convergence, rho and beta = (rho'/rho_prev)(alpha/omega)
    F_CG_RELIABLE = 9, // CGNR after a reliable update replaced r and z = D^dag r: A = |r|^2, B = |z|^2
    F_BI_OMEGA_RHO = 10, // merged BiCGStab: A = RED_BICG of t = D s with v = rh (|s|^2 its last value):
                         // omega, then rho' = <rh, s> - omega <rh, t> and beta before r is formed
    F_BI_CONV = 11,      // merged BiCGStab, end of an iteration: A = |r|^2 -> convergence / stop
    // single-reduction forms: the iteration's only finalize.  C = |r|^2 of
    // the previous update (absent in the first iteration: the value from the init)
    F_CG1 = 12,          // CGNR: A = |z|^2 (z = D^dag r), B = |q|^2 (q = D z)
    F_SR = 13            // BiCGStab: A = B_SR_PV's 9 values, B = RED_SR's 9 values
};
struct FinParams {
    const double *A;
    const double *B;
    const double *C;
    int nblkA, nblkB, nblkC;
    int nvalA, nvalB, nvalC;
    Scalars *sc;
    double *out;      // F_SUM destination [nval][nrhs]
    int *hflag;       // optional host-visible copy of flag[nrhs] ...
    double *hrr;      // ... and rr[nrhs] (device pointers to mapped host memory)
    Scalars *hsc;     // optional host-visible copy of every column's scalars (mapped host memory)
    int nrhs;
    int iter;
    double tol2;
    const double *tol2v;  // optional per-column tol2 for the F_INIT_* ops (overrides tol2)
    int group;            // columns per linear system (domain wall: ns); sums are taken per group
    // segmented vectors: rows of column c hold lenX[c] partials (stride nblkX)
    const int *lenA, *lenB, *lenC;
};
hipError_t launch_finalize(int op, const FinParams &p, hipStream_t st);
hipError_t launch_scalars_init(Scalars *sc, int nrhs, double tol2, hipStream_t st);

}  // namespace wl
