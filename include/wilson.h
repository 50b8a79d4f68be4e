/*
 * wilson.h -- C ABI of the MI355X (gfx950) Wilson-Dirac stencil and Krylov
 * solver library (libwilson.so).
 *
 * What it computes (Kanamori & Matsufuru, arXiv:1712.01505):
 *   Sec. II-B, eq. (1): the Wilson fermion matrix on a 4-D lattice with SU(3)
 *   links U_mu(x) and 4-spin x 3-colour fields, periodic or antiperiodic
 *   boundaries.  The library uses the hopping-parameter normalisation
 *       D = 1 - kappa H = 2 kappa D_W,   kappa = 1 / (2 m0 + 8),
 *       (H psi)(x) = sum_mu [ s+ (1 - g_mu) U_mu(x) psi(x+mu)
 *                           + s- (1 + g_mu) U_mu(x-mu)^dag psi(x-mu) ],
 *   where s+/s- are the boundary signs of hops that wrap around the lattice.
 *   Sec. II-C: linear solves D x = b by BiCGStab (the paper's solver for the
 *   Wilson matrix) and a mixed-precision solve whose inner solver runs in a
 *   lower precision.  The paper applies CG to the normal equations D^dag D
 *   of the domain-wall matrix (Sec. II-C, Sec. VI-B); the library offers the
 *   same CG on the normal equations (CGNR) for the Wilson matrix as well.
 *   Sec. IV-A: the solver is offloaded from the host code to a separately
 *   tuned library whose fields may take any data layout and type; here that
 *   library is this C ABI, with caller-owned device buffers.
 *
 * Gamma matrices: chiral (DeGrand-Rossi) basis, Hermitian,
 *   gamma_5 = gamma_x gamma_y gamma_z gamma_t = diag(1, 1, -1, -1).
 *
 * CONVENTIONS
 *   dims = {Lx, Ly, Lz, Lt}, each >= 2; site index s = x + Lx*(y + Ly*(z + Lz*t));
 *   V = Lx*Ly*Lz*Lt <= 2^31 - 1.  bc[mu] = +1 periodic, -1 antiperiodic
 *   (default {1, 1, 1, -1}).
 *   Canonical (caller) layouts, complex128 (re, im interleaved):
 *     spinor  [nrhs][Lt][Lz][Ly][Lx][spin 4][colour 3]
 *     gauge   [mu 4][Lt][Lz][Ly][Lx][row 3][col 3]   (links must be SU(3):
 *             the library stores two rows and rebuilds the third as
 *             conj(row0 x row1), which holds only for unitary det-1 links)
 *   Packed (library) layouts, produced by wl_pack_* and sized by
 *   wl_field_bytes; opaque to callers except for their size:
 *     spinor  [nrhs][chunk][V] 16-byte chunks, site-contiguous per component
 *             (WL_F64: 12 chunks of 1 complex; WL_F32: 6 chunks of 2 complex;
 *              WL_BF16S / WL_F16S: 3 chunks of 4 complex of 16-bit reals, then
 *              [nrhs][V] FP32 per-site scales = max |real| of the site).
 *     gauge   [mu 4][V][2 rows x 3 cols] in the same site-contiguous form.
 *
 * MEMORY AND STREAMS
 *   Every field pointer is a device pointer to a caller-owned allocation
 *   (typically a torch tensor's data_ptr), 16-byte aligned.  `stream` is a
 *   hipStream_t (NULL = the default stream).  wl_op borrows the packed-link
 *   pointer: keep it alive and unchanged while the op exists.
 *   Stencil, pack and force calls are asynchronous on `stream`.  Solvers
 *   synchronise `stream` (they read convergence scalars) and return after
 *   completion.
 *
 * ERRORS
 *   0 = WL_OK.  Positive = completed, result usable, see stats.  Negative =
 *   nothing was launched (argument error) or the HIP runtime reported an
 *   error (WL_EHIP; wl_last_hip_error() returns the hipError_t).
 */
#ifndef WILSON_H
#define WILSON_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    WL_OK = 0,
    WL_NOT_CONVERGED = 1, /* maxiter reached; x is the last iterate */
    WL_BREAKDOWN = 2,     /* BiCGStab rho, <r^,v> or omega vanished */
    WL_STAGNATED = 3,     /* mixed solve stopped reducing the true residual */
    WL_EINVAL = -1,       /* bad dims/bc/nrhs/NULL/flag */
    WL_EALIGN = -2,       /* a pointer is not 16-byte aligned */
    WL_EPREC = -3,        /* unsupported precision or precision pairing */
    WL_EHIP = -4,         /* HIP runtime error */
    WL_ENAN = -5,         /* NaN/Inf in a residual */
    WL_EWORKSPACE = -6    /* workspace too small */
};

/* Storage precision of packed fields.  *S = 16-bit storage with an FP32
 * per-site scale for spinors; arithmetic is FP64 for WL_F64, FP32 otherwise. */
typedef enum { WL_F64 = 0, WL_F32 = 1, WL_BF16S = 2, WL_F16S = 3 } wl_prec;

enum { WL_SPINOR = 0, WL_GAUGE = 1 };
enum { WL_SOLVER_CGNR = 0, WL_SOLVER_BICGSTAB = 1 };

typedef struct {
    int32_t dims[4]; /* Lx, Ly, Lz, Lt */
    int32_t bc[4];   /* +1 periodic, -1 antiperiodic */
} wl_geom;

typedef struct wl_op wl_op; /* geometry + kappa + precision + borrowed links */

/* Bytes of a packed field of `kind` (WL_SPINOR with nrhs right-hand sides,
 * or WL_GAUGE with nrhs ignored) in precision `prec`. */
int wl_field_bytes(const wl_geom *g, int kind, int prec, int nrhs, size_t *out_bytes);

/* Canonical complex128 gauge field -> packed links (two rows) in `prec`.
 * Paper Sec. IV-A (data layout flexible per architecture). Async. */
int wl_pack_gauge(const wl_geom *g, int prec, const void *U_canon, void *U_packed, void *stream);

/* Canonical complex128 spinors -> packed spinors (round to nearest even).  Async. */
int wl_pack_spinor(const wl_geom *g, int prec, int nrhs, const void *psi_canon, void *psi_packed, void *stream);

/* Packed spinors -> canonical complex128.  Async. */
int wl_unpack_spinor(const wl_geom *g, int prec, int nrhs, const void *psi_packed, void *psi_canon, void *stream);

/* Packed -> packed precision conversion, out = in (both packed).  Async. */
int wl_convert_spinor(const wl_geom *g, int prec_in, int prec_out, int nrhs, const void *in, void *out,
                      void *stream);

/* Create/destroy an operator.  `U_packed` must have been packed in `prec`. */
int wl_op_create(const wl_geom *g, double kappa, int prec, const void *U_packed, wl_op **out);
int wl_op_destroy(wl_op *op);

/* out = H in (dagger = 0), or the hopping term of D^dag (dagger = 1); eq. (1)
 * without the diagonal; 1320 flop/site per right-hand side.  `in` and `out`
 * are packed spinors of the op's precision with nrhs right-hand sides and
 * must not overlap.  Async. */
int wilson_dslash(const wl_op *op, void *out, const void *in, int dagger, int nrhs, void *stream);

/* out = D in = in - kappa H in (dagger = 1: D^dag in = gamma5 D gamma5 in);
 * eq. (1) in the kappa normalisation; 1368 flop/site per right-hand side
 * (paper Table I).  Same buffer rules as wilson_dslash.  Async. */
int wilson_apply(const wl_op *op, void *out, const void *in, int dagger, int nrhs, void *stream);

/* ---- Enforced halo (Sec. IV: single-node runs with the boundary copy
 * enforced) ----
 * out = D in (dagger: D^dag in) computed as one rank of a lattice decomposed
 * in t whose neighbours are itself: the projected half-spinors of the two t
 * faces are packed into buffers (12 reals per face site; the t = Lt-1 face
 * already multiplied by its link) and copied device to device (the
 * exchange), the interior stencil runs in the tuned launch shape with the
 * wrapping t hops left out, and a last kernel adds the received faces to
 * the t = 0 and t = Lt-1 slices; all four in that order on `stream` (on one
 * GPU the copy costs less than a synchronisation with a second stream).
 * The result equals wilson_apply's up to the order of the additions.  halo: device buffer of
 * wl_halo_bytes (send and receive regions; FP64 ops use double, the others
 * float), owned by the caller and not used concurrently by two calls.
 * Wilson ops only.  Async with respect to the host. */
int wl_halo_bytes(const wl_op *op, int nrhs, size_t *out_bytes);
int wilson_apply_halo(const wl_op *op, void *out, const void *in, int dagger, int nrhs, void *halo,
                      size_t halo_bytes, void *stream);

/* ---- Even-odd (red-black) decomposition ----
 * Sites of even and odd parity of x + y + z + t; the hopping term couples
 * only opposite parities, D = [[1, -kappa H_eo], [-kappa H_oe, 1]].  A half
 * field holds the V/2 sites of one parity in the packed spinor format with
 * V/2 in place of V (wl_field_bytes / 2 bytes); site s of parity p sits at
 * half index s / 2.  Needs every extent even (a hop wrapping around an odd
 * extent keeps the parity); WL_EINVAL otherwise.
 * wl_eo_split / wl_eo_merge: full packed field <-> its two halves (bit-exact
 * copies).  wilson_schur_apply: out_e = M in_e with the Schur complement
 * M = 1 - kappa^2 H_eo H_oe (dagger: M^dag = 1 - kappa^2 H'_eo H'_oe with
 * the adjoint hops); tmp_o is a caller half field receiving H_oe in_e.
 * Wilson ops only; async. */
int wl_eo_split(const wl_geom *g, int prec, int nrhs, const void *full, void *even, void *odd, void *stream);
int wl_eo_merge(const wl_geom *g, int prec, int nrhs, const void *even, const void *odd, void *full, void *stream);
int wilson_schur_apply(const wl_op *op, void *out_e, const void *in_e, void *tmp_o, int dagger, int nrhs,
                       void *stream);

/* ---- Domain-wall operator (Sec. II-B, eq. (2)) ----
 * D_DW acts on 5-d fields: Ns four-dimensional spinors psi_0 .. psi_{Ns-1}
 * sharing the links.  In packed form a 5-d field is Ns consecutive
 * right-hand-side columns ([vec][s][chunk][V]; pack it with
 * wl_pack_spinor and nrhs = nvec * Ns from a canonical (nvec, Ns, Lt, Lz,
 * Ly, Lx, 4, 3) array).  Block-tridiagonal in s:
 *   (D_DW psi)_s = (D_W + 1) psi_s - P_- psi_{s+1} - P_+ psi_{s-1},
 *   D_W = (m0 + 4) - H/2 (eq. (1)), P_pm = (1 pm gamma_5)/2,
 * where psi_{Ns} stands for -m psi_0 and psi_{-1} for -m psi_{Ns-1}
 * (the corner blocks m P_+ and m P_-).  m0 is the Wilson mass of D_W (the
 * domain-wall height is -m0), m the quark mass.  dagger = 1 applies
 * D_DW^dag (adjoint hop, P_+ and P_- exchanged).  11520 flop per 4-d site
 * at Ns = 8, i.e. 1440 per 5-d site (Table I).
 * The op borrows U_packed like wl_op_create; Ns in [1, 64].  Such an op
 * takes dwf_apply, solve_cgnr (CG on D_DW^dag D_DW, Sec. II-C and VI-B; nrhs there
 * counts 5-d vectors, nrhs * Ns <= 64), wl_autotune / wl_get_launch /
 * wl_set_launch (nrhs = 5-d vectors; one slice per thread, variants 0..2
 * and the t-walks 4..6, slices across lanes allowed)
 * and wl_op_destroy; the Wilson entry points, solve_bicgstab (its spectrum
 * reaches Re < 0), the force and multi-lattice plans reject it with
 * WL_EINVAL. */
int wl_dw_op_create(const wl_geom *g, double m0, double m, int Ns, int prec, const void *U_packed, wl_op **out);
/* out = D_DW in (dagger: D_DW^dag in) for nvec 5-d vectors (nvec * Ns <= 65535);
 * buffer rules as wilson_apply.  Async. */
int dwf_apply(const wl_op *op, void *out, const void *in, int dagger, int nvec, void *stream);

typedef struct {
    double tol;           /* stop when ||b - D x|| <= tol ||b|| (true residual, FP64; the
                             library accepts at tol (1 - 1e-4), so that an independent FP64
                             evaluation of the residual, rounded in another order, also
                             finds <= tol) */
    int maxiter;          /* Krylov iterations (summed over inner solves when mixed) */
    double inner_tol;     /* mixed: defect correction: relative tolerance of each inner solve;
                             reliable updates: residual drop that triggers an FP64 update
                             (0 = default: 1e-5 FP32, 3e-2 16-bit, FP16 BiCGStab 0.1;
                             reliable updates 0.1, FP16 BiCGStab 0.01) */
    int max_outer;        /* mixed: maximum outer (refinement) cycles (0 = default 50) */
    int reliable;         /* mixed: 0 = defect correction (restart the inner solve per cycle),
                             1 = reliable updates (one inner run, FP64 solution and residual
                             refreshed in place; BiCGStab re-derives rho and beta, CGNR
                             recomputes z = D^dag r and keeps its search direction unless
                             |r| has grown since the previous update).  CGNR with a
                             16-bit inner op takes defect correction only: reliable = 1
                             returns WL_EPREC for that pairing. */
    int check_every;      /* host convergence check period in iterations (0 = default) */
    int use_x0;           /* 1 = x holds the initial guess on entry, 0 = start from x = 0 */
    int dagger;           /* 1 = solve D^dag x = b (the adjoint system; D^dag = gamma5 D gamma5) */
    void *workspace;      /* device scratch of at least wl_solver_workspace_bytes, owned by
                             the caller and not used by two concurrent solves; a solve
                             allocates no device memory itself (NULL or too small:
                             WL_EWORKSPACE) */
    size_t workspace_bytes;
    int eo;               /* 1 = even-odd preconditioned: solve the Schur system
                             (1 - kappa^2 H_eo H_oe) x_e = b_e + kappa H_eo b_o on the even
                             sites, then x_o = b_o + kappa H_oe x_e; Wilson ops with every
                             extent even.  x, b stay full packed fields; tol applies to
                             the full system, whose residual is recomputed at the end. */
    int form;             /* iteration form (Sec. V-C: the vector updates and global
                             reductions, not the stencil, bound the solver):
                             0 = merged two-phase iterations (CGNR: 4 kernels and 2
                             finalizes per iteration; BiCGStab: 4 kernels and 3
                             finalizes, see below);
                             1 = one reduction phase per iteration.  CGNR in
                             Chronopoulos and Gear's form: z = D^dag r and q = D z
                             with their norms, one finalize (alpha from
                             |z|^2 / (|q|^2 - beta |z|^2 / alpha_prev)), one pass
                             updating p, w = D p, x and r: 3 kernels + 1 finalize.
                             BiCGStab rearranged around u = D r, v = D p and q = D v
                             (s and t = D s are never formed before the scalars):
                             4 kernels + 1 finalize, with more vector traffic.
                             Both check |r| one iteration later (two extra stencils
                             at the end); the same recurrences in exact
                             arithmetic.  Form 1 with a mixed solve needs
                             reliable = 0 (WL_EINVAL otherwise). */
} wl_solve_params;

typedef struct {
    int iters;            /* Krylov iterations performed for this right-hand side */
    int outer;            /* mixed: FP64 residual refreshes (refinement cycles + reliable updates) */
    int stencil_calls;    /* stencil applications (all precisions) */
    int converged;        /* 1 if the final true relative residual <= tol */
    double iter_rel_res;  /* final iterated (recursive) relative residual */
    double true_rel_res;  /* final true relative residual ||b - D x|| / ||b|| (FP64) */
    double seconds;       /* wall time of the whole call */
    int kernels;          /* kernel launches of the call (finalizes included) */
    int finalizes;        /* single-workgroup finalize launches (the reduction phases) */
} wl_solve_stats;

/* Device workspace needed by a solve (hi op; lo op or NULL; solver id). */
int wl_solver_workspace_bytes(const wl_op *hi, const wl_op *lo, int solver, int nrhs, size_t *out_bytes);

/* Solve D x = b for nrhs right-hand sides at once (per-right-hand-side
 * scalars; converged columns are frozen).  x, b: packed spinors of hi's
 * precision.  lo == NULL: plain solve in hi's precision (BiCGStab: Sec. II-C,
 * Sec. V-C; CGNR: the CG on the normal equations that Sec. II-C and VI-B apply
 * to the domain-wall matrix, offered for the Wilson matrix too).  lo != NULL: mixed precision --
 * FP64 outer true-residual refinement around an inner solve in lo's
 * precision (Sec. II-C: the inner low-precision solver sets the speed).
 * With domain-wall ops (wl_dw_op_create; hi and lo with equal Ns, m0, m)
 * only solve_cgnr is offered and nrhs counts 5-d vectors.
 * BiCGStab (form 0) runs a merged iteration: the second product t = D s
 * also returns <rh, s>, <rh, t> and |s|^2, so rho' = <rh, s> - omega <rh, t>
 * and beta are known before r' = s - omega t is formed, and one pass updates
 * x, r and the next p (the same recurrences; two vector passes and one
 * kernel fewer per iteration; an iteration followed by a reliable update
 * updates x and r only, and the next forms p from the replaced r).
 * stats: array of nrhs entries (may be NULL).  Synchronises `stream`.
 * Returns the worst status over right-hand sides. */
int solve_cgnr(const wl_op *hi, const wl_op *lo, void *x, const void *b, int nrhs, const wl_solve_params *p,
               wl_solve_stats *stats, void *stream);
int solve_bicgstab(const wl_op *hi, const wl_op *lo, void *x, const void *b, int nrhs, const wl_solve_params *p,
                   wl_solve_stats *stats, void *stream);

/* Derivative of a solve with respect to the links, for x = D^{-1} b and the
 * adjoint mu = D^{-dag} g (g = dL/dRe x + i dL/dIm x):
 *   dL = Re sum_{x,mu} Tr[dU_mu(x) G_mu(x)],
 *   G_mu(x) = kappa s_mu(x) [ sum_spin ((1 - g_mu) x(x+mu)) mu(x)^dag
 *                           + sum_spin mu(x+mu) ((1 + g_mu) x(x))^dag ].
 * project = 0: out = G^dag (the unconstrained complex gradient dL/dRe U + i dL/dIm U);
 * project = 1: out = P = traceless Hermitian part of i U G (the su(3) force:
 *              along U -> exp(i w T) U, dL/dw = Tr[T P]);
 * project = 2: out = i P U (the gradient in the tangent space of SU(3)).
 * x, mu: packed spinors of the op's precision (WL_F64 or WL_F32), nrhs = 1.
 * out: canonical complex128 gauge layout.  Async. */
int wilson_gauge_force(const wl_op *op, void *out_canon, const void *x, const void *mu, int project,
                       void *stream);

/* Several lattices of different sizes in one persistent launch: entry i
 * computes out_i = D_i in_i (or D_i^dag in_i) with nrhs right-hand sides.
 * All ops must share one precision; out_i and in_i are packed spinors of
 * it, distinct, 16-byte aligned.  The work is cut into fixed-size site
 * tiles x right-hand-side groups, drawn by resident workgroups from one
 * device-wide queue, so small lattices fill the gaps of large ones. */
typedef struct {
    const wl_op *op;
    void *out;
    const void *in;
} wl_multi_desc;

/* A plan uploads the descriptor table once (and owns the queue counter);
 * each run is then one kernel launch.  The ops and buffers named in the
 * descriptors must outlive the plan.  Runs of one plan must not overlap
 * in time (they share the counter): issue them on one stream.
 * create: n in [1, 1024], nrhs in [1, 65535]; synchronous.
 * run: async on `stream`.
 * tune: times the launch shapes (sites per workgroup, RHS per thread, code
 *   variant, persistent or direct form) with HIP events, keeps the fastest
 *   (also in $WL_TUNE_CACHE); synchronous; leaves out_i = D_i in_i.
 * get_launch: current block size, RHS per thread, variant, form and grid.
 * set_launch: force a shape: block in {64,...,512} (multiple of 64); RHS per
 *   thread 1, 2 or 4 (WL_F64: 1, 2) dividing nrhs; variant 0 (any RHS per
 *   thread) or a pipelined variant 1..3 the precision offers (1 RHS per
 *   thread); persistent = 1: resident workgroups pop work items from the
 *   queue, 0: one workgroup per work item (the same items and results);
 *   synchronous, the plan must be idle. */
typedef struct wl_multi_plan wl_multi_plan;
int wl_multi_plan_create(const wl_multi_desc *d, int n, int dagger, int nrhs, wl_multi_plan **plan);
int wl_multi_plan_run(wl_multi_plan *plan, void *stream);
int wl_multi_plan_tune(wl_multi_plan *plan, void *stream);
int wl_multi_plan_get_launch(const wl_multi_plan *plan, int *block, int *rhs_per_thread, int *variant,
                             int *persistent, int *grid);
int wl_multi_plan_set_launch(wl_multi_plan *plan, int block, int rhs_per_thread, int variant, int persistent);
int wl_multi_plan_destroy(wl_multi_plan *plan);

/* One-shot form: create a plan, run it, wait for `stream`, destroy it. */
int wilson_multi_apply(const wl_multi_desc *d, int n, int dagger, int nrhs, void *stream);

/* ---- Multi-lattice solve (Sec. II-C solvers over several lattices at once)
 * n linear systems D_i x_i = b_i on lattices of any extents (each with its
 * own links, kappa and boundary signs), nrhs right-hand sides each, solved
 * together: every stencil application of the Krylov iteration is ONE
 * multi-lattice launch over all lattices (the plan kernel with the solver's
 * fused reduction, one descriptor table per call site, uploaded once per
 * solve), every vector update one launch over all columns and every
 * reduction one finalize; each (lattice, right-hand side) column keeps its
 * own scalars and stops on its own tolerance.  Solver, params, precision
 * pairing and stats as solve_cgnr / solve_bicgstab: hi ops all of one
 * precision (plain: WL_F64 or WL_F32; mixed: WL_F64 with lo ops all of one
 * lower precision, lo_i on the geometry and kappa of hi_i), Wilson ops only,
 * n * nrhs <= 64, eo = 0.  x_i, b_i: packed fields of hi_i's precision with
 * nrhs columns (x_i holds the start if use_x0).  The workspace
 * (wl_multi_solver_workspace_bytes) holds the segmented vectors; the right-
 * hand sides are gathered into it and the solutions scattered back (device
 * copies).  The stencil shape is the multi-lattice plan tuner's choice for
 * these lattices (one right-hand side per thread) if one is cached, else the
 * default.  stats: n * nrhs entries, column i * nrhs + r.  Synchronises
 * `stream`; returns the worst status. */
typedef struct {
    const wl_op *hi;
    const wl_op *lo;  /* NULL for a plain solve (then NULL for every system) */
    void *x;
    const void *b;
} wl_multi_system;
int wl_multi_solver_workspace_bytes(const wl_multi_system *s, int n, int solver, int nrhs, size_t *out_bytes);
int wilson_solve_multi(const wl_multi_system *s, int n, int solver, int nrhs, const wl_solve_params *p,
                       wl_solve_stats *stats, void *stream);

/* Time the stencil launch candidates for (op geometry, precision, nrhs,
 * dagger), for the plain apply and for each fused reduction the solvers use,
 * with HIP events (a reduction with its finalize), and keep the fastest; the
 * best brick walk is timed again with each occupancy cap (wg_per_cu).  The
 * choices are kept in memory and, if $WL_TUNE_CACHE names a file, in that
 * JSON file: {"entries": [...]}, one object per line with "key", the key's
 * fields ("arch", "dims", "prec", "nrhs", "dagger", "reduction"), the launch
 * shape (the wl_launch fields) and "us", the measured time per launch.  A
 * later process reads the file on its first launch.  Synchronous. */
int wl_autotune(const wl_op *op, int nrhs, int dagger, void *stream);

/* Stencil launch configuration for (op, nrhs):
 * block           threads per workgroup, 64..512, a multiple of 64;
 * rhs_per_thread  right-hand sides per thread sharing its link registers:
 *                 dividing nrhs, at most 2 for WL_F64 and 4 otherwise;
 * rhs_lanes       right-hand sides interleaved across the lanes of every
 *                 wavefront (1, 2, 4 or 8, dividing nrhs; > 1 needs
 *                 rhs_per_thread = 1 and block / rhs_lanes >= 64, or >= 32
 *                 for the t-walks): the links of a site are fetched once
 *                 per load instruction for all of them, and a workgroup
 *                 covers block / rhs_lanes sites (t-walk: columns of
 *                 sites).  Variant 7: right-hand sides per workgroup, each
 *                 in wavefronts of its own with its own LDS stage, passing
 *                 the same barriers (so their link loads of a slice hit
 *                 the caches after the first);
 * xcd_remap       0 natural tile order, 1 one contiguous site range per XCD,
 *                 2..5 one z-slab per XCD, walked in y-chunks of
 *                 Ly >> (xcd_remap - 2) rows, each chunk t-major (needs
 *                 Lz % 8 == 0, Ly divisible by the chunk count and
 *                 block / rhs_lanes dividing V/8; the t-walk variants treat
 *                 2..5 as 1);
 * variant         0 straight-line hops; with rhs_per_thread = 1 a
 *                 software-pipelined hop loop 1 (all precisions), 2 (not
 *                 WL_F64), 3 (16-bit formats only), or a t-walk 4, 5, 6
 *                 (columns of 4, 8, 16 sites along t; Lt divisible by that;
 *                 block <= 256), or 7, the LDS-staged brick walk: a
 *                 workgroup of brick[0] x brick[1] x brick[2] (64..256,
 *                 a multiple of 64) threads per right-hand side owns that
 *                 brick of (x, y, z) sites and
 *                 walks t_steps t-slices; each slice's spinors of the brick
 *                 and of its face halos are staged in LDS (the halo by
 *                 direct-to-LDS copies) and the spatial neighbours are read
 *                 from there (brick extents dividing Lx, Ly, Lz; t_steps
 *                 dividing Lt; block = brick sites x rhs_lanes <= 256,
 *                 rhs_lanes 1, 2 or 4, the stages of all of them within
 *                 the LDS; rhs_per_thread = 1; Wilson ops).
 * brick, t_steps  variant 7 only (ignored otherwise).
 * wg_per_cu       variant 7 only (else 0): 0 no cap, or 1, 2, 4, 8 -- each
 *                 workgroup reserves 1/wg_per_cu of the CU's 160 KB of LDS,
 *                 so at most that many workgroups (wg_per_cu x block / 256
 *                 waves per SIMD) share a CU; the slices must fit the share.
 * rhs_major       with several groups of right-hand sides (nrhs larger than
 *                 rhs_per_thread x rhs_lanes): 0 runs the groups of a site
 *                 tile back to back on one XCD (they share its links and
 *                 neighbours in L2 while they are resident), 1 runs one
 *                 group after the other over the whole lattice (each group
 *                 streams like a one-group launch and fetches the links
 *                 again); 0 or 1.
 * Results do not depend on the configuration (16-bit t-walk and brick walk:
 * to rounding). */
typedef struct {
    int block;
    int rhs_per_thread;
    int rhs_lanes;
    int xcd_remap;
    int variant;
    int brick[3];
    int t_steps;
    int wg_per_cu;
    int rhs_major;
} wl_launch;
int wl_get_launch(const wl_op *op, int nrhs, wl_launch *cfg);
/* Force a configuration (WL_EINVAL if it breaks a rule above).  Used by
 * tests and the autotuner. */
int wl_set_launch(wl_op *op, int nrhs, const wl_launch *cfg);

/* Stencil timing: when enabled, every stencil launch is bracketed by HIP
 * events on its stream; wl_prof_read synchronises and returns, for stencil
 * launches of storage precision `prec`, the number of launches, their summed
 * duration in ms and the summed sites x right-hand sides processed. */
int wl_prof_enable(int on);
int wl_prof_reset(void);
int wl_prof_read(int prec, long *launches, double *total_ms, double *site_rhs);
/* Of those sites x right-hand sides, the ones whose launch also read a
 * further spinor field for its fused reduction (the solvers' <rh, D p> and
 * <rh, D s>, with rh the BiCGStab shadow residual): one more field of
 * compulsory traffic per site.  WL_EINVAL for a bad precision or null. */
int wl_prof_read_aux(int prec, double *aux_site_rhs);

/* ---- Fused apply with the solvers' inner products ----
 * out = D in (dagger: D^dag in) and, from the same pass over the sites, the
 * inner products the Krylov solvers fuse into their operator products
 * (paper Sec. V-C: the solver's linear algebra and reductions, not the
 * stencil, dominate its time):
 *   kind WL_DOT_BICG: 8 values per right-hand side r, <in, out>, |out|^2,
 *        <v, in>, <v, out>, |in|^2 (BiCGStab's second product: omega, the
 *        next rho and |s|^2);
 *   kind WL_DOT_V:    2 values, <v, out> (BiCGStab's <rh, D p>);
 *   kind WL_DOT_NORM: 1 value, |out|^2 (CG on the normal equations).
 * Complex values take two entries (re, im); <a, b> = sum conj(a_i) b_i,
 * accumulated in FP64 in a fixed order.  dots: DEVICE array of nval x nrhs
 * doubles, value-major (entry k of column r at dots[k nrhs + r]), 8-byte
 * aligned; for WL_DOT_BICG the order is Re<in,out>, Im<in,out>, |out|^2,
 * Re<v,in>, Im<v,in>, Re<v,out>, Im<v,out>, |in|^2.  v: packed spinor of the op's
 * precision (nrhs columns; may equal in; NULL only for WL_DOT_NORM).  The
 * stencil runs in the launch shape tuned for that reduction.  workspace:
 * caller-owned device scratch of wl_apply_dot_workspace_bytes (256-byte
 * aligned), not shared by concurrent calls.  Wilson ops, nrhs <= 64.  Async
 * (nothing is copied to the host). */
enum { WL_DOT_BICG = 0, WL_DOT_V = 1, WL_DOT_NORM = 2 };
int wl_apply_dot_workspace_bytes(const wl_op *op, int nrhs, size_t *out_bytes);
int wilson_apply_dot(const wl_op *op, void *out, const void *in, const void *v, int dagger, int nrhs, int kind,
                     double *dots, void *workspace, size_t workspace_bytes, void *stream);

/* ---- The same fused apply for callers that cannot allocate ----
 * For code under HIP graph capture, tight serving loops and harnesses that
 * forbid device allocation: wilson_apply_dot without a workspace argument.
 * Its partial sums live in a library-owned device array of
 * WL_NOALLOC_SCRATCH_BYTES (one per GPU the library runs on, held until the
 * process ends); the call itself allocates nothing.  A size needing more
 * than that (wl_apply_dot_workspace_bytes > WL_NOALLOC_SCRATCH_BYTES, e.g.
 * more than 7 right-hand sides at 32^3 x 64) returns WL_EWORKSPACE before
 * any launch.  Every call on one GPU shares that GPU's array: calls that
 * overlap in time on one GPU (two streams, two threads) race and must not
 * be issued; calls in one stream are ordered and safe.  The array keeps the
 * last call's partials; nothing in it needs to start at zero.  Arguments,
 * results and errors as wilson_apply_dot.  Async. */
#define WL_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
int wilson_apply_dot_noalloc(const wl_op *op, void *out, const void *in, const void *v, int dagger, int nrhs,
                             int kind, double *dots, void *stream);

/* Plain device-to-device streaming copy of `bytes` (a multiple of 16, no
 * overlap): the reference point for achievable HBM bandwidth and for
 * calibrating hardware byte counters against a kernel of known traffic.
 * Async. */
int wl_stream_copy(void *dst, const void *src, size_t bytes, void *stream);

const char *wl_strerror(int code);
int wl_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* WILSON_H */
