/*
 * wilson_oracle.c -- plain FP64 CPU oracle for the Wilson-Dirac operator,
 * its Krylov solvers and the gauge-link derivative of a solve.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no source, header, table or helper with the GPU library: the gamma
 * matrices below are typed here from the chiral basis definition, the links
 * are full 3x3 matrices, the spin structure is a dense 4x4 multiply and there
 * is no spin projection, no link compression and no blocking.
 *
 * Paper: I. Kanamori, H. Matsufuru, "Practical Implementation of Lattice QCD
 * Simulation on Intel Xeon Phi Knights Landing" (arXiv:1712.01505).
 *   - Sec. II-A: fields; a site x = (x1..x4), links U_mu(x) in SU(3), the
 *     fermion field carries 4 spin x 3 colour complex values per site.
 *   - Sec. II-B, eq. (1): the Wilson fermion matrix
 *       D_W = (m0+4) delta_{x,y} - 1/2 sum_mu [ (1-gamma_mu) U_mu(x) delta_{x+mu,y}
 *                                              + (1+gamma_mu) U_mu^dag(x-mu) delta_{x-mu,y} ],
 *     with periodic or antiperiodic boundary conditions.
 *   - Sec. II-C: BiCGStab for the Wilson matrix; CG on the normal equations.
 *
 * Normalisation: this oracle works with the hopping-parameter form
 *   D = 1 - kappa * H,   H psi(x) = sum_mu [ s+ (1-g_mu) U_mu(x) psi(x+mu)
 *                                            + s- (1+g_mu) U_mu(x-mu)^dag psi(x-mu) ]
 * which equals 2*kappa*D_W with kappa = 1/(2 m0 + 8).  s+ / s- are the
 * boundary signs of a hop that wraps around the lattice in direction mu
 * (bc[mu] = +1 periodic, -1 antiperiodic), applied to the hop and never
 * folded into a link.
 *
 * Layout (canonical, the same one callers of the library use):
 *   spinor  psi[t][z][y][x][spin 4][colour 3]          complex double
 *   gauge   U[mu][t][z][y][x][row 3][col 3]            complex double
 *   site index s = x + Lx*(y + Ly*(z + Lz*t)),  dims = {Lx, Ly, Lz, Lt}.
 *
 * Inner product <a,b> = sum conj(a_i) b_i; norms are FP64.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* Euclidean gamma matrices in the chiral (DeGrand-Rossi) basis, mu = x,y,z,t.
 * Hermitian, gamma_mu^2 = 1, {gamma_mu, gamma_nu} = 2 delta;
 * gamma_5 = gamma_x gamma_y gamma_z gamma_t = diag(1,1,-1,-1). */
static const cplx GAMMA[4][4][4] = {
    {{0, 0, 0, I}, {0, 0, I, 0}, {0, -I, 0, 0}, {-I, 0, 0, 0}},
    {{0, 0, 0, -1}, {0, 0, 1, 0}, {0, 1, 0, 0}, {-1, 0, 0, 0}},
    {{0, 0, I, 0}, {0, 0, 0, -I}, {-I, 0, 0, 0}, {0, I, 0, 0}},
    {{0, 0, 1, 0}, {0, 0, 0, 1}, {1, 0, 0, 0}, {0, 1, 0, 0}},
};

void oracle_gamma(int mu, double *out_re_im /* 16 complex, row-major */)
{
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            out_re_im[2 * (4 * a + b)] = creal(GAMMA[mu][a][b]);
            out_re_im[2 * (4 * a + b) + 1] = cimag(GAMMA[mu][a][b]);
        }
}

static long volume(const int *L) { return (long)L[0] * L[1] * L[2] * L[3]; }

static void coords_of(const int *L, long s, int *c)
{
    c[0] = (int)(s % L[0]);
    s /= L[0];
    c[1] = (int)(s % L[1]);
    s /= L[1];
    c[2] = (int)(s % L[2]);
    c[3] = (int)(s / L[2]);
}

static long index_of(const int *L, const int *c)
{
    return c[0] + (long)L[0] * (c[1] + (long)L[1] * (c[2] + (long)L[2] * c[3]));
}

/* Site reached from coordinates c by one step (+1 or -1) in direction mu.
 * *sign is bc[mu] when the step wraps around the lattice, else +1. */
static long step_site(const int *L, const int *bc, const int *c, int mu, int dir, double *sign)
{
    int n[4] = {c[0], c[1], c[2], c[3]};
    n[mu] += dir;
    *sign = 1.0;
    if (n[mu] == L[mu]) {
        n[mu] = 0;
        *sign = (double)bc[mu];
    } else if (n[mu] < 0) {
        n[mu] = L[mu] - 1;
        *sign = (double)bc[mu];
    }
    return index_of(L, n);
}

/* out[spin][colour] += coef * (1 + pm*gamma_mu) * M * in, where M is the
 * colour matrix `link` (or its Hermitian conjugate if `adj`). */
static void add_hop(cplx out[4][3], const cplx *link, int adj, const cplx *in, int mu, double pm, double coef)
{
    cplx Min[4][3];
    for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) {
            cplx acc = 0;
            for (int b = 0; b < 3; ++b) {
                cplx m = adj ? conj(link[3 * b + a]) : link[3 * a + b];
                acc += m * in[3 * s + b];
            }
            Min[s][a] = acc;
        }
    for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) {
            cplx acc = Min[s][a];
            for (int r = 0; r < 4; ++r)
                acc += pm * GAMMA[mu][s][r] * Min[r][a];
            out[s][a] += coef * acc;
        }
}

/* Hopping term at one site: out12 = (H psi)(s) (dagger = 0) or the hopping
 * term of D^dag (dagger = 1), which swaps the projector signs. */
static void hop_site(const int *L, const int *bc, const cplx *U, const cplx *psi, long s, int dagger, cplx *out12)
{
    const long V = volume(L);
    int c[4];
    coords_of(L, s, c);
    cplx acc[4][3];
    memset(acc, 0, sizeof acc);
    const double fwd_pm = dagger ? +1.0 : -1.0; /* (1 - gamma) forward for D */
    for (int mu = 0; mu < 4; ++mu) {
        double sg;
        long nf = step_site(L, bc, c, mu, +1, &sg);
        add_hop(acc, U + 9 * (mu * V + s), 0, psi + 12 * nf, mu, fwd_pm, sg);
        long nb = step_site(L, bc, c, mu, -1, &sg);
        add_hop(acc, U + 9 * (mu * V + nb), 1, psi + 12 * nb, mu, -fwd_pm, sg);
    }
    for (int sp = 0; sp < 4; ++sp)
        for (int a = 0; a < 3; ++a)
            out12[3 * sp + a] = acc[sp][a];
}

/* out = H psi (dagger = 0) or out = H' psi with H' the hopping term of D^dag. */
void oracle_hop(const int *L, const int *bc, const cplx *U, const cplx *psi, cplx *out, int dagger)
{
    const long V = volume(L);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s)
        hop_site(L, bc, U, psi, s, dagger, out + 12 * s);
}

/* out = D psi = psi - kappa H psi  (dagger = 1: D^dag psi). */
void oracle_apply(const int *L, const int *bc, double kappa, const cplx *U, const cplx *psi, cplx *out, int dagger)
{
    const long V = volume(L);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s) {
        cplx h[12];
        hop_site(L, bc, U, psi, s, dagger, h);
        for (int i = 0; i < 12; ++i)
            out[12 * s + i] = psi[12 * s + i] - kappa * h[i];
    }
}

/* D psi evaluated only at the listed sites: out[k*12 + i] = (D psi)(sites[k])_i.
 * Used to check a large GPU result on sampled sites. */
void oracle_apply_sites(const int *L, const int *bc, double kappa, const cplx *U, const cplx *psi, int dagger,
                        long nsites, const long *sites, cplx *out)
{
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nsites; ++k) {
        cplx h[12];
        long s = sites[k];
        hop_site(L, bc, U, psi, s, dagger, h);
        for (int i = 0; i < 12; ++i)
            out[12 * k + i] = psi[12 * s + i] - kappa * h[i];
    }
}

/* ---- vector helpers (plain loops) ---- */
static cplx vdot(long n, const cplx *a, const cplx *b)
{
    double re = 0, im = 0;
#pragma omp parallel for reduction(+ : re, im) schedule(static)
    for (long i = 0; i < n; ++i) {
        cplx p = conj(a[i]) * b[i];
        re += creal(p);
        im += cimag(p);
    }
    return re + I * im;
}
static double vnorm2(long n, const cplx *a) { return creal(vdot(n, a, a)); }

/* CG on the normal equations D^dag D x = D^dag b (CGNR), following the
 * standard algorithm (Saad, Iterative Methods for Sparse Linear Systems,
 * Alg. 8.4); the paper uses CG on the normal equations in Sec. II-C.
 * x holds the initial guess on entry.  Stops when ||b - D x|| <= tol ||b||
 * by the recursively updated residual, then recomputes the true residual.
 * Returns 0 if the true relative residual is <= tol, 1 otherwise. */
int oracle_cgnr(const int *L, const int *bc, double kappa, const cplx *U, const cplx *b, cplx *x, double tol,
                int maxiter, int *iters, double *true_relres)
{
    const long n = 12 * volume(L);
    cplx *r = malloc(n * sizeof(cplx)), *z = malloc(n * sizeof(cplx));
    cplx *p = malloc(n * sizeof(cplx)), *w = malloc(n * sizeof(cplx));
    const double bnorm = sqrt(vnorm2(n, b));
    int k = 0;
    oracle_apply(L, bc, kappa, U, x, w, 0);
    for (long i = 0; i < n; ++i)
        r[i] = b[i] - w[i];
    oracle_apply(L, bc, kappa, U, r, z, 1);
    memcpy(p, z, n * sizeof(cplx));
    double zz = vnorm2(n, z);
    double rr = vnorm2(n, r);
    while (k < maxiter && sqrt(rr) > tol * bnorm) {
        oracle_apply(L, bc, kappa, U, p, w, 0);
        double ww = vnorm2(n, w);
        if (ww == 0.0)
            break;
        double alpha = zz / ww;
        for (long i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * w[i];
        }
        rr = vnorm2(n, r);
        oracle_apply(L, bc, kappa, U, r, z, 1);
        double zz_new = vnorm2(n, z);
        double beta = zz_new / zz;
        zz = zz_new;
        for (long i = 0; i < n; ++i)
            p[i] = z[i] + beta * p[i];
        ++k;
    }
    oracle_apply(L, bc, kappa, U, x, w, 0);
    for (long i = 0; i < n; ++i)
        r[i] = b[i] - w[i];
    double rel = bnorm > 0 ? sqrt(vnorm2(n, r)) / bnorm : 0.0;
    *iters = k;
    *true_relres = rel;
    free(r);
    free(z);
    free(p);
    free(w);
    return rel <= tol ? 0 : 1;
}

/* BiCGStab (van der Vorst 1992) for M x = b with M = D (dagger = 0) or
 * M = D^dag (dagger = 1); the paper's solver for the Wilson matrix
 * (Sec. II-C, Sec. V-C).  Shadow residual r^ = r0.  x holds the initial
 * guess on entry.  Returns 0 when the true relative residual is <= tol,
 * 1 when not converged, 2 on breakdown (rho or <r^,v> or omega zero). */
int oracle_bicgstab(const int *L, const int *bc, double kappa, const cplx *U, const cplx *b, cplx *x, int dagger,
                    double tol, int maxiter, int *iters, double *true_relres)
{
    const long n = 12 * volume(L);
    cplx *r = malloc(n * sizeof(cplx)), *rh = malloc(n * sizeof(cplx));
    cplx *p = calloc(n, sizeof(cplx)), *v = calloc(n, sizeof(cplx));
    cplx *s = malloc(n * sizeof(cplx)), *t = malloc(n * sizeof(cplx));
    const double bnorm = sqrt(vnorm2(n, b));
    int status = 1, k = 0;
    oracle_apply(L, bc, kappa, U, x, t, dagger);
    for (long i = 0; i < n; ++i)
        r[i] = b[i] - t[i];
    memcpy(rh, r, n * sizeof(cplx));
    cplx rho = 1, alpha = 1, omega = 1;
    double rr = vnorm2(n, r);
    while (k < maxiter && sqrt(rr) > tol * bnorm) {
        cplx rho_new = vdot(n, rh, r);
        if (cabs(rho_new) == 0.0) {
            status = 2;
            break;
        }
        cplx beta = (rho_new / rho) * (alpha / omega);
        rho = rho_new;
        for (long i = 0; i < n; ++i)
            p[i] = r[i] + beta * (p[i] - omega * v[i]);
        oracle_apply(L, bc, kappa, U, p, v, dagger);
        cplx rv = vdot(n, rh, v);
        if (cabs(rv) == 0.0) {
            status = 2;
            break;
        }
        alpha = rho / rv;
        for (long i = 0; i < n; ++i)
            s[i] = r[i] - alpha * v[i];
        ++k;
        if (sqrt(vnorm2(n, s)) <= tol * bnorm) {
            for (long i = 0; i < n; ++i)
                x[i] += alpha * p[i];
            rr = vnorm2(n, s);
            break;
        }
        oracle_apply(L, bc, kappa, U, s, t, dagger);
        double tt = vnorm2(n, t);
        omega = tt > 0 ? vdot(n, t, s) / tt : 0;
        if (cabs(omega) == 0.0) {
            status = 2;
            break;
        }
        for (long i = 0; i < n; ++i) {
            x[i] += alpha * p[i] + omega * s[i];
            r[i] = s[i] - omega * t[i];
        }
        rr = vnorm2(n, r);
    }
    oracle_apply(L, bc, kappa, U, x, t, dagger);
    for (long i = 0; i < n; ++i)
        r[i] = b[i] - t[i];
    double rel = bnorm > 0 ? sqrt(vnorm2(n, r)) / bnorm : 0.0;
    *iters = k;
    *true_relres = rel;
    if (status != 2)
        status = rel <= tol ? 0 : 1;
    free(r);
    free(rh);
    free(p);
    free(v);
    free(s);
    free(t);
    return status;
}

/* Derivative of a solve with respect to the links.
 * For L(x) with x = D^{-1} b, upstream g = dL/dRe x + i dL/dIm x and
 * adjoint mu = D^{-dag} g, the variation is
 *   dL = Re sum_{x,mu} Tr[ dU_mu(x) G_mu(x) ],
 *   G_mu(x) = kappa s_mu(x) [ sum_spin ((1-g_mu) x(x+mu))_spin mu(x)_spin^dag
 *                           + sum_spin mu(x+mu)_spin ((1+g_mu) x(x))_spin^dag ],
 * obtained by differentiating D = 1 - kappa H term by term (each link enters
 * the forward hop at x and the backward hop at x+mu).  s_mu(x) is the
 * boundary sign of the hop x -> x+mu.  Output G in the gauge layout. */
void oracle_force(const int *L, const int *bc, double kappa, const cplx *x, const cplx *mu_adj, cplx *G)
{
    const long V = volume(L);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s) {
        int c[4];
        coords_of(L, s, c);
        for (int mu = 0; mu < 4; ++mu) {
            double sg;
            long nf = step_site(L, bc, c, mu, +1, &sg);
            cplx v[4][3], w[4][3];
            for (int sp = 0; sp < 4; ++sp)
                for (int a = 0; a < 3; ++a) {
                    cplx gv = 0, gw = 0;
                    for (int r = 0; r < 4; ++r) {
                        gv += GAMMA[mu][sp][r] * x[12 * nf + 3 * r + a];
                        gw += GAMMA[mu][sp][r] * x[12 * s + 3 * r + a];
                    }
                    v[sp][a] = x[12 * nf + 3 * sp + a] - gv; /* (1 - g) x(x+mu) */
                    w[sp][a] = x[12 * s + 3 * sp + a] + gw;  /* (1 + g) x(x)    */
                }
            cplx *g = G + 9 * (mu * V + s);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    cplx acc = 0;
                    for (int sp = 0; sp < 4; ++sp) {
                        acc += v[sp][a] * conj(mu_adj[12 * s + 3 * sp + b]);
                        acc += mu_adj[12 * nf + 3 * sp + a] * conj(w[sp][b]);
                    }
                    g[3 * a + b] = kappa * sg * acc;
                }
        }
    }
}

/* ---- Domain-wall operator (Sec. II-B, eq. (2)) ------------------------------
 * A 5-d field is Ns four-dimensional spinor fields one after the other,
 * psi[s][t][z][y][x][spin][colour], s = 0..Ns-1.  The matrix is block
 * tridiagonal in s:
 *   block (s, s)       D_W + 1,  with D_W = (m0 + 4) - 1/2 H   (eq. (1))
 *   block (s, s+1)     -P_-          block (s, s-1)     -P_+
 *   block (0, Ns-1)    m P_+         block (Ns-1, 0)    m P_-
 * with the chiral projectors P_pm = (1 pm gamma_5)/2 (the paper does not spell
 * them out; this is their standard meaning).  The links are the same for every
 * s.  The conjugate transpose has D_W^dag + 1 on the diagonal, -P_+ in block
 * (s, s+1), -P_- in block (s, s-1), m P_- in block (0, Ns-1) and m P_+ in
 * block (Ns-1, 0). */

/* gamma_5 as the product gamma_x gamma_y gamma_z gamma_t, by plain 4x4 products. */
static void gamma5_matrix(cplx g5[4][4])
{
    cplx a[4][4], b[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
            a[i][j] = GAMMA[0][i][j];
    for (int mu = 1; mu < 4; ++mu) {
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                cplx acc = 0;
                for (int k = 0; k < 4; ++k)
                    acc += a[i][k] * GAMMA[mu][k][j];
                b[i][j] = acc;
            }
        memcpy(a, b, sizeof a);
    }
    memcpy(g5, a, sizeof a);
}

/* out12 += coef * P_pm in12, P_pm = (1 pm gamma_5) / 2 (pm = +1 or -1). */
static void add_chiral(cplx *out12, const cplx *in12, const cplx g5[4][4], double pm, cplx coef)
{
    for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) {
            cplx acc = 0.5 * in12[3 * s + a];
            for (int r = 0; r < 4; ++r)
                acc += 0.5 * pm * g5[s][r] * in12[3 * r + a];
            out12[3 * s + a] += coef * acc;
        }
}

/* out = D_DW psi (dagger = 0) or D_DW^dag psi (dagger = 1). */
void oracle_dw_apply(const int *L, const int *bc, int Ns, double m0, double m, const cplx *U, const cplx *psi,
                     cplx *out, int dagger)
{
    const long V = volume(L), n4 = 12 * V;
    cplx g5[4][4];
    gamma5_matrix(g5);
    /* the projector in block (s, s+1) and in block (s, s-1) */
    const double up = dagger ? +1.0 : -1.0, down = -up;
    for (int s = 0; s < Ns; ++s) {
        const cplx *ps = psi + s * n4;
        cplx *os = out + s * n4;
#pragma omp parallel for schedule(static)
        for (long x = 0; x < V; ++x) {
            cplx h[12];
            hop_site(L, bc, U, ps, x, dagger, h);
            for (int i = 0; i < 12; ++i)
                os[12 * x + i] = (m0 + 5.0) * ps[12 * x + i] - 0.5 * h[i];
            /* block (s, s+1): -P_up psi_{s+1}; for s = Ns-1 the corner m P_up psi_0 */
            if (s + 1 < Ns)
                add_chiral(os + 12 * x, psi + (s + 1) * n4 + 12 * x, g5, up, -1.0);
            else
                add_chiral(os + 12 * x, psi + 12 * x, g5, up, m);
            /* block (s, s-1): -P_down psi_{s-1}; for s = 0 the corner m P_down psi_{Ns-1} */
            if (s > 0)
                add_chiral(os + 12 * x, psi + (s - 1) * n4 + 12 * x, g5, down, -1.0);
            else
                add_chiral(os + 12 * x, psi + (Ns - 1) * n4 + 12 * x, g5, down, m);
        }
    }
}

/* CG on the normal equations of the domain-wall matrix, D^dag D x = D^dag b
 * (Sec. II-C and Sec. VI-B: the paper applies CG to D^dag D for this operator), following
 * the same textbook steps as oracle_cgnr (Saad, Alg. 8.4).  x holds the
 * initial guess.  Returns 0 if the true relative residual ||b - D x|| / ||b||
 * is <= tol, 1 otherwise. */
int oracle_dw_cgnr(const int *L, const int *bc, int Ns, double m0, double m, const cplx *U, const cplx *b, cplx *x,
                   double tol, int maxiter, int *iters, double *true_relres)
{
    const long n = 12 * volume(L) * Ns;
    cplx *r = malloc(n * sizeof(cplx)), *z = malloc(n * sizeof(cplx));
    cplx *p = malloc(n * sizeof(cplx)), *w = malloc(n * sizeof(cplx));
    const double bnorm = sqrt(vnorm2(n, b));
    int k = 0;
    oracle_dw_apply(L, bc, Ns, m0, m, U, x, w, 0);
    for (long i = 0; i < n; ++i)
        r[i] = b[i] - w[i];
    oracle_dw_apply(L, bc, Ns, m0, m, U, r, z, 1);
    memcpy(p, z, n * sizeof(cplx));
    double zz = vnorm2(n, z);
    double rr = vnorm2(n, r);
    while (k < maxiter && sqrt(rr) > tol * bnorm) {
        oracle_dw_apply(L, bc, Ns, m0, m, U, p, w, 0);
        double ww = vnorm2(n, w);
        if (ww == 0.0)
            break;
        double alpha = zz / ww;
        for (long i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * w[i];
        }
        rr = vnorm2(n, r);
        oracle_dw_apply(L, bc, Ns, m0, m, U, r, z, 1);
        double zz_new = vnorm2(n, z);
        double beta = zz_new / zz;
        zz = zz_new;
        for (long i = 0; i < n; ++i)
            p[i] = z[i] + beta * p[i];
        ++k;
    }
    oracle_dw_apply(L, bc, Ns, m0, m, U, x, w, 0);
    for (long i = 0; i < n; ++i)
        r[i] = b[i] - w[i];
    double rel = bnorm > 0 ? sqrt(vnorm2(n, r)) / bnorm : 0.0;
    *iters = k;
    *true_relres = rel;
    free(r);
    free(z);
    free(p);
    free(w);
    return rel <= tol ? 0 : 1;
}
