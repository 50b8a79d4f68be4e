// wl_solver.cpp -- host drivers of the Krylov solvers: CGNR and BiCGStab
// (paper Sec. II-C; BiCGStab for the Wilson matrix, CG on the normal
// equations) and the mixed-precision refinement around a low-precision
// inner solve (Sec. II-C: the inner solver sets the performance).
//
// Every vector operation is a kernel on the caller's stream; the scalar
// recurrences live on the device (wl_blas.hip), so an iteration issues only
// kernel launches; the finalize kernels mirror each column's status into
// host-visible memory, and the host checks it behind a lookahead of
// `check_every` queued iterations (HIP events, no copies, no stream drain
// while iterating).  All right-hand sides run together; a converged
// or broken-down column is frozen by zeroing its coefficients on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <mutex>
#include <vector>

#include "wl_internal.h"

namespace wl {

hipError_t prof_stencil(int prec, const wl_op *op, int dagger, const LaunchCfg &cfg, StencilParams p,
                        hipStream_t st);  // wl_api.cpp
LaunchCfg launch_for(const wl_op *op, int nrhs, int red, int dagger);  // wl_api.cpp
void set_last_hip_error(hipError_t e);           // wl_api.cpp

namespace {

constexpr int BLAS_BLOCK = 256;
constexpr size_t ALIGN = 256;

size_t align_up(size_t n) { return (n + ALIGN - 1) / ALIGN * ALIGN; }

size_t vec_bytes(int prec, uint32_t V, int nrhs) { return (size_t)nrhs * V * spinor_site_bytes(prec); }

// Largest number of per-workgroup partials any kernel here produces (the
// t-walk stencil writes at most one per 64 (x,y,z) sites per t-column step,
// i.e. at most V/64 + Lt; multi-RHS launches pad the tile count to a
// multiple of 8).
size_t max_nblk(uint32_t V, int Lt) { return (V + 63) / 64 + (size_t)Lt + 8; }
size_t partial_bytes(uint32_t V, int Lt, int nrhs)
{
    return align_up(RED_NVAL_MAX * (size_t)nrhs * max_nblk(V, Lt) * sizeof(double));
}

struct Arena {
    char *base;
    size_t cap, off = 0;
    void *take(size_t n)
    {
        n = align_up(n);
        if (off + n > cap)
            return nullptr;
        void *p = base + off;
        off += n;
        return p;
    }
};

// Bytes of one Krylov engine for op precision `prec`.
size_t engine_bytes(int solver, int prec, uint32_t V, int Lt, int nrhs)
{
    const int nvec = solver == WL_SOLVER_CGNR ? 5 : 6;
    return nvec * align_up(vec_bytes(prec, V, nrhs)) + 3 * partial_bytes(V, Lt, nrhs) +
           align_up(sizeof(Scalars) * nrhs) + align_up(sizeof(double) * 3 * nrhs);
}

#define WL_TRY(expr)                                                                                           \
    do {                                                                                                       \
        hipError_t e_ = (expr);                                                                                \
        if (e_ != hipSuccess) {                                                                                \
            set_last_hip_error(e_);                                                                            \
            return WL_EHIP;                                                                                    \
        }                                                                                                      \
    } while (0)

// Host-side buffers of one solve, kept in a pool and allocated once: coherent
// mapped host memory that the kernels read and write directly (no copy
// kernels): the per-RHS scalars mirrored by the finalize kernels, the status
// they mirror every iteration, scalar inputs and sums (d), and lookahead
// events.
constexpr int MAX_RHS = 64;
constexpr int MAX_LOOK = 8;
struct HostBufs {
    Scalars *sc = nullptr;   // mirror of the device scalars (written by the finalize kernels)
    double *d = nullptr;     // scratch [4 * MAX_RHS]: sums written by kernels, scalars read by kernels
    int *hflag = nullptr;    // status mirror
    double *hrr = nullptr;
    Scalars *dsc = nullptr;  // device views of sc, d, hflag, hrr
    double *dd = nullptr;
    int *dflag = nullptr;
    double *drr = nullptr;
    hipEvent_t ev[MAX_LOOK + 1] = {};
    bool ok = false;
    void create()
    {
        const unsigned f = hipHostMallocMapped | hipHostMallocCoherent;
        ok = hipHostMalloc((void **)&sc, sizeof(Scalars) * MAX_RHS, f) == hipSuccess &&
             hipHostMalloc((void **)&d, sizeof(double) * 4 * MAX_RHS, f) == hipSuccess &&
             hipHostMalloc((void **)&hflag, sizeof(int) * MAX_RHS, f) == hipSuccess &&
             hipHostMalloc((void **)&hrr, sizeof(double) * MAX_RHS, f) == hipSuccess &&
             hipHostGetDevicePointer((void **)&dsc, sc, 0) == hipSuccess &&
             hipHostGetDevicePointer((void **)&dd, d, 0) == hipSuccess &&
             hipHostGetDevicePointer((void **)&dflag, hflag, 0) == hipSuccess &&
             hipHostGetDevicePointer((void **)&drr, hrr, 0) == hipSuccess;
        for (int i = 0; ok && i <= MAX_LOOK; ++i)
            ok = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) == hipSuccess;
    }
    // device view of a location in d (the host writes it only while the
    // stream is idle; kernels read or write it in stream order)
    double *dev(double *h) const { return dd + (h - d); }
};
std::mutex g_pool_mu;
std::vector<HostBufs *> g_pool;

struct HostLease {
    HostBufs *b = nullptr;
    HostLease()
    {
        {
            std::lock_guard<std::mutex> lk(g_pool_mu);
            if (!g_pool.empty()) {
                b = g_pool.back();
                g_pool.pop_back();
            }
        }
        if (!b) {
            b = new HostBufs();
            b->create();
        }
    }
    ~HostLease()
    {
        if (b && b->ok) {
            std::lock_guard<std::mutex> lk(g_pool_mu);
            g_pool.push_back(b);
        }
        // a lease whose creation failed is leaked on purpose: its partially
        // created resources are not reused
    }
};

// Several lattices solved together (one column per (lattice, right-hand
// side)): the operators, the columns per lattice and the shape of the
// multi-lattice stencil launch (one site per thread).
struct MultiSpec {
    std::vector<const wl_op *> hi, lo;
    int nrhs = 1;
    LaunchCfg cfg, cfg_lo;  // the hi and lo operators' stencil shapes
};
constexpr int MAX_TABLES = 10;  // multi-lattice stencil call sites of one engine

// Stencil parameters of one operator (as the single-operator launch sets
// them up), for the multi-lattice descriptor tables.
StencilParams op_params(const wl_op *op, void *out, const void *in, int nrhs)
{
    StencilParams p{};
    p.U = op->U;
    p.in = in;
    p.out = out;
    for (int i = 0; i < 4; ++i) {
        p.L[i] = op->g.dims[i];
        p.bc[i] = op->g.bc[i];
    }
    p.fx = make_fastdiv((uint32_t)p.L[0]);
    p.fy = make_fastdiv((uint32_t)p.L[1]);
    p.fz = make_fastdiv((uint32_t)p.L[2]);
    p.V = op->V;
    p.nrhs = nrhs;
    p.kappa = op->kappa;
    p.apply = 1;
    p.one = 1.0f;
    return p;
}

// Bytes of one segmented vector (every lattice's field, 256-byte aligned).
size_t seg_vec_bytes(const std::vector<const wl_op *> &ops, int prec, int nrhs)
{
    size_t n = 0;
    for (const wl_op *o : ops)
        n += align_up(vec_bytes(prec, o->V, nrhs));
    return n;
}
// Partials per column of a multi-lattice engine: the BLAS kernels' (256
// sites per workgroup) or the stencil's site tiles (at least 64 sites).
int seg_stride(const std::vector<const wl_op *> &ops, int block)
{
    uint32_t vmax = 0;
    for (const wl_op *o : ops)
        vmax = std::max(vmax, o->V);
    return std::max(blas_partials(vmax, B_NORM, BLAS_BLOCK), (int)((vmax + block - 1) / block));
}
size_t multi_engine_bytes(int solver, int prec, const std::vector<const wl_op *> &ops, int nrhs)
{
    const int nvec = solver == WL_SOLVER_CGNR ? 5 : 6;
    const int ncol = (int)ops.size() * nrhs;
    return nvec * seg_vec_bytes(ops, prec, nrhs) +
           3 * align_up((size_t)RED_NVAL_MAX * ncol * seg_stride(ops, 64) * sizeof(double)) +
           align_up(sizeof(Scalars) * ncol) + align_up(sizeof(double) * 3 * ncol) + align_up(sizeof(Seg) * ncol) +
           align_up(sizeof(int) * 3 * ncol) + align_up(sizeof(MultiEntry) * MAX_TABLES * ops.size()) + 8 * ALIGN;
}

// A Krylov solver instance on one operator (one precision), nrhs columns.
struct Engine {
    const wl_op *op;
    int solver, nrhs, prec;
    uint32_t V;
    hipStream_t st;
    void *v[6];
    double *part[3];
    int nblk[3] = {0, 0, 0}, nval[3] = {0, 0, 0};
    Scalars *sc;
    double *sums;
    Scalars *sc_host;  // pinned
    HostBufs *hb;
    int lookahead = 2;
    int adj = 0;  // solving with D^dag: every stencil's dagger flag is flipped
    int stencil_calls = 0;
    int kernels = 0, finalizes = 0;  // launches issued (kernels includes the finalizes)
    int form = 0;   // 1: one reduction phase per iteration (single-reduction CGNR / BiCGStab)
    int group = 1;  // columns per linear system (domain wall: the fifth-dimension extent)
    bool eo = false;       // even-odd: vectors are even half fields, the operator is the Schur complement
    void *eo_tmp = nullptr;  // odd half field for H_oe in
    const double *tol2v = nullptr;  // optional per-column tolerance^2 (device)
    // Called after each queued CGNR iteration that did not stop the run
    // (the reliable-update check of the mixed solver).
    std::function<int(int)> on_iter;
    // The same check for BiCGStab, split in two: whether iteration it ends
    // with a reliable update (asked before its last BLAS pass, which then
    // leaves p alone), and the update itself.
    std::function<bool(int)> rel_decide;
    std::function<int(int)> rel_act;

    // ---- multi-lattice mode (init_multi): vectors are segmented, one
    // segment per lattice; nrhs counts all columns, lat_nrhs those of a lattice
    struct Lat {
        const wl_op *op;
        uint32_t V;
        size_t off;
        int tiles;  // stencil site tiles
    };
    std::vector<Lat> lats;
    int lat_nrhs = 0;
    size_t seg_bytes = 0;
    LaunchCfg mcfg;
    int mstride = 0;             // partials per column
    Seg *dseg = nullptr;         // device [nrhs]
    int *dlen = nullptr;         // device [3][nrhs]: partial rows of BLAS, BLAS with 4 sites/thread, stencil
    MultiEntry *dtab = nullptr;  // device [MAX_TABLES][lattices]
    std::vector<Seg> hseg;
    std::vector<int> hlen;
    struct Table {
        const void *out, *in, *aux, *aux2, *aux3;
        int dagger, red, slot;
        bool loop;
        uint32_t total;
        std::vector<MultiEntry> host;
    };
    std::vector<Table> tables;
    const int *lenp[3] = {nullptr, nullptr, nullptr};  // row lengths of each partial set's producer

    int init_multi(Arena &a, const std::vector<const wl_op *> &ops, int solv, int nl, hipStream_t s, HostBufs *h,
                   const LaunchCfg &mc)
    {
        op = ops[0];
        solver = solv;
        lat_nrhs = nl;
        nrhs = (int)ops.size() * nl;
        prec = op->prec;
        group = 1;
        eo = false;
        st = s;
        hb = h;
        sc_host = h->sc;
        mcfg = mc;
        size_t off = 0;
        uint32_t vmax = 0;
        for (const wl_op *o : ops) {
            lats.push_back(Lat{o, o->V, off, (int)((o->V + mc.block - 1) / mc.block)});
            off += align_up(vec_bytes(prec, o->V, nl));
            vmax = std::max(vmax, o->V);
        }
        seg_bytes = off;
        V = vmax;
        mstride = seg_stride(ops, mc.block);
        const int nvec = solver == WL_SOLVER_CGNR ? 5 : 6;
        for (int i = 0; i < nvec; ++i)
            if (!(v[i] = a.take(seg_bytes)))
                return WL_EWORKSPACE;
        for (int i = 0; i < 3; ++i)
            if (!(part[i] = (double *)a.take((size_t)RED_NVAL_MAX * nrhs * mstride * sizeof(double))))
                return WL_EWORKSPACE;
        if (!(sc = (Scalars *)a.take(sizeof(Scalars) * nrhs)) || !(sums = (double *)a.take(sizeof(double) * 3 * nrhs)))
            return WL_EWORKSPACE;
        if (!(dseg = (Seg *)a.take(sizeof(Seg) * nrhs)) || !(dlen = (int *)a.take(sizeof(int) * 3 * nrhs)) ||
            !(dtab = (MultiEntry *)a.take(sizeof(MultiEntry) * MAX_TABLES * lats.size())))
            return WL_EWORKSPACE;
        hseg.resize(nrhs);
        hlen.resize(3 * nrhs);
        for (size_t i = 0; i < lats.size(); ++i)
            for (int r = 0; r < nl; ++r) {
                const int c = (int)i * nl + r;
                hseg[c] = Seg{lats[i].off, lats[i].V, nl, r, 0};
                hlen[c] = blas_partials(lats[i].V, B_NORM, BLAS_BLOCK);
                hlen[nrhs + c] = blas_partials(lats[i].V, B_SR_PV, BLAS_BLOCK);
                hlen[2 * nrhs + c] = lats[i].tiles;
            }
        WL_TRY(hipMemcpyAsync(dseg, hseg.data(), sizeof(Seg) * nrhs, hipMemcpyHostToDevice, st));
        WL_TRY(hipMemcpyAsync(dlen, hlen.data(), sizeof(int) * 3 * nrhs, hipMemcpyHostToDevice, st));
        kernels += 2;
        return WL_OK;
    }

    // One multi-lattice launch: every lattice's segment of out = D in (with
    // the fused reduction into the segmented partials); the descriptor table
    // of each call site is built and uploaded once.
    int stencil_multi(void *out, const void *in, int dagger, int red, const void *aux, int slot, bool loop,
                      const void *aux2, const void *aux3)
    {
        const int n = (int)lats.size();
        int idx = -1;
        for (size_t i = 0; i < tables.size() && idx < 0; ++i) {
            const Table &t = tables[i];
            if (t.out == out && t.in == in && t.aux == aux && t.aux2 == aux2 && t.aux3 == aux3 && t.dagger == dagger &&
                t.red == red && t.slot == slot && t.loop == loop)
                idx = (int)i;
        }
        if (idx < 0) {
            if ((int)tables.size() >= MAX_TABLES)
                return WL_EWORKSPACE;
            Table t{out, in, aux, aux2, aux3, dagger, red, slot, loop, 0, std::vector<MultiEntry>(n)};
            uint64_t total = 0;
            auto at = [](const void *q, size_t off) { return q ? (const char *)q + off : nullptr; };
            for (int i = 0; i < n; ++i) {
                const Lat &L = lats[i];
                StencilParams p = op_params(L.op, (char *)out + L.off, at(in, L.off), lat_nrhs);
                p.red = red;
                p.aux = at(aux, L.off);
                p.aux2 = at(aux2, L.off);
                p.aux3 = at(aux3, L.off);
                p.partials = slot >= 0 ? part[slot] : nullptr;
                p.skip = loop ? sc : nullptr;
                p.pcol0 = i * lat_nrhs;
                p.pncol = nrhs;
                p.pstride = mstride;
                p.nblk = L.tiles;
                p.ng = (uint32_t)lat_nrhs;
                p.f_ng = make_fastdiv((uint32_t)lat_nrhs);
                t.host[i].p = p;
                t.host[i].tile_begin = (uint32_t)total;
                total += (uint64_t)L.tiles * lat_nrhs;
            }
            if (total > 0x7fffffffull)
                return WL_EINVAL;
            t.total = (uint32_t)total;
            idx = (int)tables.size();
            WL_TRY(hipMemcpyAsync(dtab + (size_t)idx * n, t.host.data(), sizeof(MultiEntry) * n, hipMemcpyHostToDevice,
                                  st));
            ++kernels;
            tables.push_back(std::move(t));
        }
        if (slot >= 0) {
            nblk[slot] = mstride;
            nval[slot] = red_nval(red);
            lenp[slot] = dlen + 2 * nrhs;
        }
        ++stencil_calls;
        ++kernels;
        WL_TRY(launch_multi(prec, dagger, 1, mcfg.block, mcfg.var, dtab + (size_t)idx * n, n, tables[idx].total,
                            nullptr, 0, st));
        return WL_OK;
    }

    int init(Arena &a, const wl_op *o, int solv, int n, hipStream_t s, HostBufs *h, bool even_odd = false)
    {
        op = o;
        solver = solv;
        nrhs = n;
        prec = o->prec;
        group = o->ns > 0 ? o->ns : 1;
        eo = even_odd;
        V = eo ? o->V / 2 : o->V;
        if (eo && !(eo_tmp = a.take(vec_bytes(prec, V, nrhs))))
            return WL_EWORKSPACE;
        st = s;
        hb = h;
        sc_host = h->sc;
        const int nvec = solver == WL_SOLVER_CGNR ? 5 : 6;
        for (int i = 0; i < nvec; ++i)
            if (!(v[i] = a.take(vec_bytes(prec, V, nrhs))))
                return WL_EWORKSPACE;
        for (int i = 0; i < 3; ++i)
            if (!(part[i] = (double *)a.take(partial_bytes(V, o->g.dims[3], nrhs))))
                return WL_EWORKSPACE;
        if (!(sc = (Scalars *)a.take(sizeof(Scalars) * nrhs)))
            return WL_EWORKSPACE;
        if (!(sums = (double *)a.take(sizeof(double) * 3 * nrhs)))
            return WL_EWORKSPACE;
        return WL_OK;
    }

    int stencil(void *out, const void *in, int dagger, int red, const void *aux, int slot, bool loop = false,
                const void *aux2 = nullptr, const void *aux3 = nullptr, int apply = 1)
    {
        if (!lats.empty())
            return stencil_multi(out, in, dagger ^ adj, red, aux, slot, loop, aux2, aux3);
        if (eo) {  // out = (1 - kappa^2 H_eo H_oe) in on even half fields
            EoParams a = eo_params(op, 1, nrhs);
            a.in = in;
            a.out = eo_tmp;
            a.c_hop = 1.0;
            a.skip = loop ? sc : nullptr;
            WL_TRY(launch_eo_hop(prec, dagger ^ adj, RED_NONE, a, st));
            EoParams b = eo_params(op, 0, nrhs);
            b.in = eo_tmp;
            b.self = in;
            b.dotv = aux;
            b.dotv2 = aux2;
            b.dotv3 = aux3;
            b.out = out;
            b.c_self = 1.0;
            b.c_hop = -op->kappa * op->kappa;
            b.skip = loop ? sc : nullptr;
            b.partials = slot >= 0 ? part[slot] : nullptr;
            if (slot >= 0) {
                nblk[slot] = eo_partials(V);
                nval[slot] = stencil_nval(red);
            }
            ++stencil_calls;
            kernels += 2;
            WL_TRY(launch_eo_hop(prec, dagger ^ adj, red, b, st));
            return WL_OK;
        }
        StencilParams p{};
        p.skip = loop ? sc : nullptr;
        p.U = op->U;
        p.in = in;
        p.out = out;
        p.aux = aux;
        p.aux2 = aux2;
        p.aux3 = aux3;
        p.partials = slot >= 0 ? part[slot] : nullptr;
        for (int i = 0; i < 4; ++i) {
            p.L[i] = op->g.dims[i];
            p.bc[i] = op->g.bc[i];
        }
        p.fx = make_fastdiv((uint32_t)p.L[0]);
        p.fy = make_fastdiv((uint32_t)p.L[1]);
        p.fz = make_fastdiv((uint32_t)p.L[2]);
        p.V = V;
        p.nrhs = nrhs;
        p.kappa = op->kappa;
        p.apply = apply;
        p.red = red;
        op_apply_params(op, p);
        LaunchCfg cfg = launch_for(op, nrhs, red, dagger ^ adj);
        if (slot >= 0) {
            nblk[slot] = stencil_partials(cfg, p.L, V, nrhs);
            nval[slot] = stencil_nval(red);
        }
        ++stencil_calls;
        ++kernels;
        WL_TRY(prof_stencil(prec, op, dagger ^ adj, cfg, p, st));
        return WL_OK;
    }

    int blas(int bop, void *y0, void *y1, const void *a0, const void *a1, const void *a2, const void *a3, int slot,
             bool loop = false, void *y2 = nullptr, void *y3 = nullptr)
    {
        BlasParams p{};
        p.skip_frozen = loop ? 1 : 0;
        p.y0 = y0;
        p.y1 = y1;
        p.y2 = y2;
        p.y3 = y3;
        p.a0 = a0;
        p.a1 = a1;
        p.a2 = a2;
        p.a3 = a3;
        p.sc = sc;
        p.partials = slot >= 0 ? part[slot] : nullptr;
        p.V = V;
        p.nrhs = nrhs;
        p.seg = lats.empty() ? nullptr : dseg;
        if (slot >= 0) {
            nblk[slot] = blas_partials(V, bop, BLAS_BLOCK);
            nval[slot] = blas_nval(bop);
            lenp[slot] = lats.empty() ? nullptr : dlen + (blas_sites_per_thread(bop) > 1 ? nrhs : 0);
        }
        ++kernels;
        WL_TRY(launch_blas(prec, bop, p, BLAS_BLOCK, st));
        return WL_OK;
    }

    // out: F_SUM destination (default: the engine's device sums)
    int fin(int fop, int a, int b, int c, int iter, double tol2, double *out = nullptr)
    {
        FinParams p{};
        if (a >= 0) {
            p.A = part[a];
            p.nblkA = nblk[a];
            p.nvalA = nval[a];
            p.lenA = lenp[a];
        }
        if (b >= 0) {
            p.B = part[b];
            p.nblkB = nblk[b];
            p.nvalB = nval[b];
            p.lenB = lenp[b];
        }
        if (c >= 0) {
            p.C = part[c];
            p.nblkC = nblk[c];
            p.nvalC = nval[c];
            p.lenC = lenp[c];
        }
        p.sc = sc;
        p.out = out ? out : sums;
        // the host reads the status at iteration ends only: the mid-iteration
        // steps skip the (PCIe) mirror writes
        const bool mid = fop == F_CG_ALPHA || fop == F_BI_ALPHA || fop == F_BI_OMEGA_RHO;
        p.hflag = mid ? nullptr : hb->dflag;
        p.hrr = mid ? nullptr : hb->drr;
        p.hsc = mid ? nullptr : hb->dsc;
        p.nrhs = nrhs;
        p.iter = iter;
        p.tol2 = tol2;
        p.tol2v = tol2v;
        p.group = group;
        ++kernels;
        ++finalizes;
        WL_TRY(launch_finalize(fop, p, st));
        return WL_OK;
    }

    // Status as last mirrored by a finalize kernel (valid once an event
    // recorded after that kernel has completed).
    bool host_all_done() const
    {
        for (int r = 0; r < nrhs; ++r)
            if (((volatile int *)hb->hflag)[r] == 0)
                return false;
        return true;
    }

    // Record the end of iteration `it` (0-based) and, once `lookahead`
    // iterations are queued behind it, wait for an older one and check the
    // mirrored status.  Returns true when every column has stopped.
    int mark(int it, bool *stop)
    {
        const int L = lookahead, n = L + 1;
        WL_TRY(hipEventRecord(hb->ev[it % n], st));
        *stop = false;
        if (it >= L) {
            WL_TRY(hipEventSynchronize(hb->ev[(it - L) % n]));
            *stop = host_all_done();
        }
        return WL_OK;
    }

    // The per-RHS scalars as the last end-of-iteration finalize mirrored them
    // into host memory (synchronises the stream).
    int poll()
    {
        WL_TRY(hipStreamSynchronize(st));
        return WL_OK;
    }

    bool all_done() const
    {
        for (int r = 0; r < nrhs; ++r)
            if (sc_host[r].flag == 0)
                return false;
        return true;
    }

    // Run the Krylov iteration for D x = b from x (zero_x: x := 0 first).
    // Afterwards sc_host holds the final per-RHS scalars.  *iters_done is
    // the number of iterations executed.
    int run(void *x, const void *b, bool zero_x, double tol, int maxiter, int *iters_done)
    {
        const double tol2 = tol * tol;
        int rc;
        void *r = v[0];
        // the merged BiCGStab from x = 0: one pass sets x, r, rh and p and
        // sums |b|^2 (= |r|^2), which the start finalize then reads twice
        const bool one_pass = zero_x && solver == WL_SOLVER_BICGSTAB && form == 0;
        if (one_pass) {
            if ((rc = blas(B_INIT, x, r, b, nullptr, nullptr, nullptr, 0, false, v[1], v[2])))
                return rc;
        } else if (zero_x) {
            if ((rc = blas(B_ZERO, x, nullptr, nullptr, nullptr, nullptr, nullptr, -1)))
                return rc;
            if ((rc = blas(B_COPY, r, nullptr, b, nullptr, nullptr, nullptr, -1)))
                return rc;
            if ((rc = blas(B_NORM, nullptr, nullptr, r, nullptr, nullptr, nullptr, 0)))
                return rc;
        } else {
            void *w = v[1];
            if ((rc = stencil(w, x, 0, RED_NONE, nullptr, -1)))
                return rc;
            if ((rc = blas(B_RES, r, nullptr, b, w, nullptr, nullptr, 0)))
                return rc;
        }
        if (!one_pass)
            if ((rc = blas(B_NORM, nullptr, nullptr, b, nullptr, nullptr, nullptr, 2)))
                return rc;
        int it = 0;
        if (solver == WL_SOLVER_CGNR && form == 1) {
            // one reduction phase per iteration: z = D^dag r (|z|^2), q = D z
            // (|q|^2), one finalize, then one pass updates p, w = D p, x and r
            // (|r|^2, checked by the next iteration's finalize)
            void *z = v[1], *p = v[2], *w = v[3], *q = v[4];
            if ((rc = blas(B_ZERO, p, nullptr, nullptr, nullptr, nullptr, nullptr, -1)))
                return rc;
            if ((rc = blas(B_ZERO, w, nullptr, nullptr, nullptr, nullptr, nullptr, -1)))
                return rc;
            if ((rc = fin(F_INIT_CG, 0, -1, 2, 0, tol2)))
                return rc;
            WL_TRY(hipStreamSynchronize(st));
            bool stop = host_all_done();
            while (!stop && it < maxiter) {
                if ((rc = stencil(z, r, 1, RED_NORM, nullptr, 0, true)))
                    return rc;
                if ((rc = stencil(q, z, 0, RED_NORM, nullptr, 1, true)))
                    return rc;
                if ((rc = fin(F_CG1, 0, 1, it > 0 ? 2 : -1, it, tol2)))
                    return rc;
                if ((rc = blas(B_CG1, x, r, z, q, nullptr, nullptr, 2, true, p, w)))
                    return rc;
                if ((rc = mark(it, &stop)))
                    return rc;
                ++it;
            }
        } else if (solver == WL_SOLVER_BICGSTAB && form == 1) {
            // one reduction phase per iteration: u = D r; p and v = D p from
            // their recurrences (with <rh, v>, <rh, u>, <u, r>, <u, v>, |u|^2);
            // q = D v (with <v, q>, |q|^2, <rh, q>, <r, q>, <u, q>); one
            // finalize forms alpha, omega, rho' and beta; one pass updates x
            // and r (|r|^2, checked by the next iteration's finalize)
            if (op->ns > 0)
                return WL_EINVAL;
            void *rh = v[1], *p = v[2], *vv = v[3], *u = v[4], *q = v[5];
            if ((rc = blas(B_COPY, rh, nullptr, r, nullptr, nullptr, nullptr, -1)))
                return rc;
            for (void *z0 : {p, vv, q})
                if ((rc = blas(B_ZERO, z0, nullptr, nullptr, nullptr, nullptr, nullptr, -1)))
                    return rc;
            if ((rc = fin(F_INIT_BI, 0, -1, 2, 0, tol2)))
                return rc;
            WL_TRY(hipStreamSynchronize(st));
            bool stop = host_all_done();
            while (!stop && it < maxiter) {
                if ((rc = stencil(u, r, 0, RED_NONE, nullptr, -1, true)))
                    return rc;
                if ((rc = blas(B_SR_PV, p, vv, r, u, q, rh, 0, true)))
                    return rc;
                if ((rc = stencil(q, vv, 0, RED_SR, rh, 1, true, r, u)))
                    return rc;
                if ((rc = fin(F_SR, 0, 1, it > 0 ? 2 : -1, it, tol2)))
                    return rc;
                if ((rc = blas(B_SR_XR, x, r, p, vv, u, q, 2, true)))
                    return rc;
                if ((rc = mark(it, &stop)))
                    return rc;
                ++it;
            }
        } else if (solver == WL_SOLVER_CGNR) {
            void *z = v[1], *p = v[2], *w = v[3];
            if ((rc = stencil(z, r, 1, RED_NORM, nullptr, 1)))
                return rc;
            if ((rc = fin(F_INIT_CG, 0, 1, 2, 0, tol2)))
                return rc;
            if ((rc = blas(B_COPY, p, nullptr, z, nullptr, nullptr, nullptr, -1)))
                return rc;
            WL_TRY(hipStreamSynchronize(st));
            bool stop = host_all_done();
            while (!stop && it < maxiter) {
                if ((rc = stencil(w, p, 0, RED_NORM, nullptr, 0, true)))
                    return rc;
                if ((rc = fin(F_CG_ALPHA, 0, -1, -1, it, tol2)))
                    return rc;
                if ((rc = blas(B_CG_XR, x, r, p, w, nullptr, nullptr, 0, true)))
                    return rc;
                if ((rc = stencil(z, r, 1, RED_NORM, nullptr, 1, true)))
                    return rc;
                if ((rc = fin(F_CG_BETA, 0, 1, -1, it, tol2)))
                    return rc;
                if ((rc = blas(B_CG_P, p, nullptr, z, nullptr, nullptr, nullptr, -1, true)))
                    return rc;
                if ((rc = mark(it, &stop)))
                    return rc;
                if (!stop && on_iter && (rc = on_iter(it)))
                    return rc;
                ++it;
            }
        } else {
            void *rh = v[1], *p = v[2], *vv = v[3], *s = v[4], *t = v[5];
            // Merged iteration: the second product also yields <rh, s> and
            // <rh, t>, so rho' and beta are known before r' = s - omega t is
            // formed and one pass updates x, r and the next p.  An iteration
            // followed by a reliable update updates x and r only; the next
            // one forms p from the replaced r.
            if (op->ns > 0)
                return WL_EINVAL;  // BiCGStab is offered for the Wilson operator only
            bool pending_p = false;  // a reliable update replaced r: p is formed from it next
            if (!one_pass) {
                if ((rc = blas(B_COPY, rh, nullptr, r, nullptr, nullptr, nullptr, -1)))
                    return rc;
                if ((rc = blas(B_COPY, p, nullptr, r, nullptr, nullptr, nullptr, -1)))
                    return rc;
            }
            if ((rc = blas(B_ZERO, vv, nullptr, nullptr, nullptr, nullptr, nullptr, -1)))
                return rc;
            if ((rc = fin(F_INIT_BI, 0, -1, one_pass ? 0 : 2, 0, tol2)))
                return rc;
            WL_TRY(hipStreamSynchronize(st));
            bool stop = host_all_done();
            while (!stop && it < maxiter) {
                if (pending_p) {  // p = r + beta (p - omega v) with the replaced r and its beta
                    if ((rc = blas(B_BI_P, p, nullptr, r, vv, nullptr, nullptr, -1, true)))
                        return rc;
                    pending_p = false;
                }
                if ((rc = stencil(vv, p, 0, RED_DOTV, rh, 0, true)))
                    return rc;
                if ((rc = fin(F_BI_ALPHA, 0, -1, -1, it, tol2)))
                    return rc;
                if ((rc = blas(B_BI_S, s, nullptr, r, vv, nullptr, nullptr, -1, true)))
                    return rc;
                if ((rc = stencil(t, s, 0, RED_BICG, rh, 1, true)))  // with |s|^2
                    return rc;
                if ((rc = fin(F_BI_OMEGA_RHO, 1, -1, -1, it, tol2)))
                    return rc;
                // the host has the status through iteration it - 1 at most, so
                // the check runs as it would have after that iteration
                const bool upd = rel_decide && rel_decide(it - 1);
                if (upd) {  // x and r only: p follows the replaced r
                    if ((rc = blas(B_BI_XR, x, r, p, s, t, rh, 0, true)))
                        return rc;
                } else if ((rc = blas(B_BI_XRP, x, r, nullptr, s, t, vv, 0, true, p))) {
                    return rc;
                }
                if ((rc = fin(F_BI_CONV, 0, -1, -1, it, tol2)))  // |r|^2 is the first value of either
                    return rc;
                if ((rc = mark(it, &stop)))
                    return rc;
                if (upd && !stop) {
                    if ((rc = rel_act(it)))
                        return rc;
                    pending_p = true;
                }
                ++it;
            }
        }
        if ((rc = poll()))
            return rc;
        *iters_done = it;
        return WL_OK;
    }

    // out[r] = |b - D x|^2 per right-hand side, into host array (synchronous).
    int true_res2(void *x, const void *b, double *out_host)
    {
        int rc;
        void *w = v[1], *r = v[0];
        if (lats.empty() && !eo && op->ns == 0 && (prec == WL_F64 || prec == WL_F32)) {
            // one pass: r = b - D x with |r|^2 in the stencil's epilogue
            if ((rc = stencil(r, x, 0, RED_NORM, b, 0, false, nullptr, nullptr, 3)))
                return rc;
        } else {
            if ((rc = stencil(w, x, 0, RED_NONE, nullptr, -1)))
                return rc;
            if ((rc = blas(B_RES, r, nullptr, b, w, nullptr, nullptr, 0)))
                return rc;
        }
        if ((rc = fin(F_SUM, 0, -1, -1, 0, 0.0, hb->dev(out_host))))
            return rc;
        WL_TRY(hipStreamSynchronize(st));
        return WL_OK;
    }

    int norm2(const void *b, double *out_host)
    {
        int rc;
        if ((rc = blas(B_NORM, nullptr, nullptr, b, nullptr, nullptr, nullptr, 2)))
            return rc;
        if ((rc = fin(F_SUM, 2, -1, -1, 0, 0.0, hb->dev(out_host))))
            return rc;
        WL_TRY(hipStreamSynchronize(st));
        return WL_OK;
    }
};

// Iterations the host lets the GPU run ahead of its convergence check
// (check_every); the status is read from host-visible memory without a copy.
int lookahead_of(const wl_solve_params *prm)
{
    const int c = prm->check_every > 0 ? prm->check_every : 2;
    return c > MAX_LOOK ? MAX_LOOK : c;
}

int status_of(const wl_solve_stats &s, int flag)
{
    if (s.converged)
        return WL_OK;
    if (flag == 2)
        return WL_BREAKDOWN;
    return WL_NOT_CONVERGED;
}

// Plain solve in the op's own precision.
int solve_plain(int solver, const wl_op *op, void *x, const void *b, int nrhs, const wl_solve_params *prm,
                wl_solve_stats *stats, hipStream_t st, Arena &arena, bool eo = false, const double *tolc = nullptr,
                const MultiSpec *ms = nullptr)
{
    HostLease lease;
    if (!lease.b->ok)
        return WL_EHIP;
    Engine E{};
    int rc = ms ? E.init_multi(arena, ms->hi, solver, ms->nrhs, st, lease.b, ms->cfg)
                : E.init(arena, op, solver, nrhs, st, lease.b, eo);
    if (rc)
        return rc;
    // per-column tolerance (even-odd: scaled to the Schur right-hand side)
    std::vector<double> tol(nrhs, prm->tol);
    if (tolc) {
        double *t2h = lease.b->d + 3 * nrhs;  // read by the kernels through its device view
        WL_TRY(hipStreamSynchronize(st));     // no earlier kernel still reads this location
        for (int r = 0; r < nrhs; ++r) {
            tol[r] = tolc[r];
            t2h[r] = tolc[r] * tolc[r];
        }
        E.tol2v = lease.b->dev(t2h);
    }
    E.adj = prm->dagger;
    E.form = prm->form;
    E.lookahead = lookahead_of(prm);
    double *bb = lease.b->d, *rr = lease.b->d + nrhs;
    if ((rc = E.norm2(b, bb)))
        return rc;
    std::vector<int> iters(nrhs, 0), flags(nrhs, 0);
    std::vector<double> itres(nrhs, 0.0);
    int total = 0;
    bool zero_x = !prm->use_x0;
    for (int attempt = 0; attempt < 4 && total < prm->maxiter; ++attempt) {
        int done = 0;
        if ((rc = E.run(x, b, zero_x, prm->tol, prm->maxiter - total, &done)))
            return rc;
        zero_x = false;
        for (int r = 0; r < nrhs; ++r) {
            const Scalars &s = E.sc_host[r];
            iters[r] += s.flag == 1 ? s.conv_iter : done;
            flags[r] = s.flag;
            itres[r] = bb[r] > 0 ? std::sqrt(s.rr / bb[r]) : 0.0;
            if (s.flag == 3)
                return WL_ENAN;
        }
        total += done;
        if ((rc = E.true_res2(x, b, rr)))
            return rc;
        bool all_ok = true;
        for (int r = 0; r < nrhs; ++r) {
            if (!std::isfinite(rr[r]))
                return WL_ENAN;
            if (!(rr[r] <= tol[r] * tol[r] * bb[r]))
                all_ok = false;
        }
        if (all_ok)
            break;
        // recursive and true residual disagree, or breakdown: restart from x
    }
    int worst = WL_OK;
    for (int r = 0; r < nrhs; ++r) {
        wl_solve_stats s{};
        s.iters = iters[r];
        s.outer = 0;
        s.stencil_calls = E.stencil_calls;
        s.kernels = E.kernels;
        s.finalizes = E.finalizes;
        s.true_rel_res = bb[r] > 0 ? std::sqrt(rr[r] / bb[r]) : 0.0;
        s.iter_rel_res = itres[r];
        s.converged = s.true_rel_res <= tol[r];
        const int code = status_of(s, flags[r]);
        if (code > worst)
            worst = code;
        if (stats)
            stats[r] = s;
    }
    return worst;
}

// Mixed precision: FP64 outer true-residual refinement around an inner solve
// in lo's precision.  Two forms (Sec. II-C names mixed precision without
// fixing one):
//  * defect correction (reliable = 0): each cycle solves D e = r/|r| to the
//    relative tolerance delta from e = 0, then x += |r| e;
//  * reliable updates (reliable = 1): one inner Krylov run is continued
//    across cycles.  Whenever the iterated low-precision residual has fallen
//    by delta below its largest value since the last update, the partial
//    solution is folded into x (FP64), the residual is recomputed as b - D x
//    in FP64 and replaces the iterated one (Sleijpen & van der Vorst's
//    reliable updates); BiCGStab re-derives rho and beta from it, CGNR
//    recomputes z = D^dag r and its norm and keeps the search direction.
//    The inner run then stops on the global tolerance; the outer loop
//    confirms it with a last FP64 residual.
int solve_mixed(int solver, const wl_op *hi, const wl_op *lo, void *x, const void *b, int nrhs,
                const wl_solve_params *prm, wl_solve_stats *stats, hipStream_t st, Arena &arena, bool eo = false,
                const double *tolc = nullptr, const MultiSpec *ms = nullptr)
{
    HostLease lease;
    if (!lease.b->ok)
        return WL_EHIP;
    Engine H{}, L{};
    int rc;
    // the outer engine only needs r, w and the partial/scalar buffers; it is
    // initialised as a CGNR engine for simplicity of layout
    if ((rc = ms ? H.init_multi(arena, ms->hi, WL_SOLVER_CGNR, ms->nrhs, st, lease.b, ms->cfg)
                 : H.init(arena, hi, WL_SOLVER_CGNR, nrhs, st, lease.b, eo)))
        return rc;
    if ((rc = ms ? L.init_multi(arena, ms->lo, solver, ms->nrhs, st, lease.b, ms->cfg_lo)
                 : L.init(arena, lo, solver, nrhs, st, lease.b, eo)))
        return rc;
    H.adj = L.adj = prm->dagger;
    L.form = prm->form;
    int direct = 0;  // accumulate / convert launches issued here
    const size_t lo_bytes = ms ? L.seg_bytes : vec_bytes(lo->prec, L.V, nrhs);
    void *r_lo = arena.take(lo_bytes);
    void *e_lo = arena.take(lo_bytes);
    if (!r_lo || !e_lo)
        return WL_EWORKSPACE;
    H.lookahead = L.lookahead = lookahead_of(prm);
    double *bb = lease.b->d, *rr = lease.b->d + nrhs, *sig = lease.b->d + 2 * nrhs, *t2 = lease.b->d + 3 * nrhs;
    // sigma and the inner tolerances are written by the host between cycles
    // (the stream idle after each true-residual check) and read by the kernels
    // through the device view of that host memory
    double *sig_dev = lease.b->dev(sig), *tol2_dev = lease.b->dev(t2);
    // x64 += sigma e  and  r_lo = r64 / sigma, one launch per lattice segment
    // in a multi-lattice solve
    auto accum = [&]() -> hipError_t {
        if (!ms) {
            ++direct;
            return launch_accum(lo->prec, H.V, nrhs, x, e_lo, sig_dev, 1, st);
        }
        for (size_t i = 0; i < H.lats.size(); ++i) {
            ++direct;
            const hipError_t e = launch_accum(lo->prec, H.lats[i].V, ms->nrhs, (char *)x + H.lats[i].off,
                                              (char *)e_lo + L.lats[i].off, sig_dev + i * ms->nrhs, 1, st);
            if (e != hipSuccess)
                return e;
        }
        return hipSuccess;
    };
    auto convert = [&](const void *r64, void *rlo) -> hipError_t {
        if (!ms) {
            ++direct;
            return launch_convert(WL_F64, lo->prec, H.V, nrhs, r64, rlo, sig_dev, 1, 2, st);
        }
        for (size_t i = 0; i < H.lats.size(); ++i) {
            ++direct;
            const hipError_t e = launch_convert(WL_F64, lo->prec, H.lats[i].V, ms->nrhs, (const char *)r64 + H.lats[i].off,
                                                (char *)rlo + L.lats[i].off, sig_dev + i * ms->nrhs, 1, 2, st);
            if (e != hipSuccess)
                return e;
        }
        return hipSuccess;
    };
    if ((rc = H.norm2(b, bb)))
        return rc;
    if (!prm->use_x0)
        if ((rc = H.blas(B_ZERO, x, nullptr, nullptr, nullptr, nullptr, nullptr, -1)))
            return rc;
    std::vector<double> tolv(nrhs, prm->tol);  // per column (even-odd: scaled to the Schur system)
    if (tolc)
        for (int r = 0; r < nrhs; ++r)
            tolv[r] = tolc[r];
    // (CG on the normal equations with 16-bit storage and reliable updates is
    // rejected with WL_EPREC before this point)
    const bool reliable = prm->reliable != 0;
    // defaults measured on 32^3 x 64 (six sources, BiCGStab to 1e-10): an
    // FP16 BiCGStab is fastest restarted from the FP64 residual every 0.1
    // (defect correction) or updated every 0.01 (reliable updates); CG on
    // the normal equations keeps 3e-2 (0.1 cost the domain-wall system 17 %)
    const bool f16_bicg = lo->prec == WL_F16S && solver == WL_SOLVER_BICGSTAB;
    const double delta = prm->inner_tol > 0  ? prm->inner_tol
                         : reliable          ? (f16_bicg ? 1e-2 : 0.1)
                         : lo->prec == WL_F32 ? 1e-5
                         : f16_bicg           ? 0.1
                                              : 3e-2;
    const int max_outer = prm->max_outer > 0 ? prm->max_outer : 50;
    std::vector<int> iters(nrhs, 0);
    std::vector<double> best(nrhs, INFINITY), rmax(nrhs, 0.0);
    std::vector<int> stall(nrhs, 0);
    int total = 0, outer = 0, updates = 0, worst_flag = 0, next_read = 0, last_update = 0, last_gap = 0;
    bool stagnated = false;
    if (reliable) {
        // the inner run's stopping rule is the global one, in units of the
        // scaled system (|r_lo|^2 ~ 1 at the start of a cycle); 0.8 leaves
        // room for the rounding of the iterated residual
        L.tol2v = tol2_dev;
        const double d2 = delta * delta;
        auto decide = [&](int it) -> bool {
            if (it < next_read)
                return false;
            const volatile int *hf = lease.b->hflag;
            const volatile double *hr = lease.b->hrr;
            // update when the iterated residual has dropped by delta, and also
            // when that has taken three times longer than the previous drop
            // (at least 64 iterations): a low-precision recurrence can stall
            // while the true residual drifts away
            const int gap = std::max(64, 3 * last_gap);
            bool need = it - last_update >= gap;
            for (int r = 0; r < nrhs; ++r) {
                if (hf[r] != 0)
                    continue;
                const double v = hr[r];
                if (v > rmax[r])
                    rmax[r] = v;
                else if (v < d2 * rmax[r])
                    need = true;
            }
            return need;
        };
        auto act = [&](int it) -> int {
            last_gap = it - last_update;
            last_update = it;
            int e;
            // x64 += sigma e ; e = 0 ; r64 = b - D64 x ; r_lo = r64 / sigma
            WL_TRY(accum());
            if ((e = L.blas(B_ZERO, e_lo, nullptr, nullptr, nullptr, nullptr, nullptr, -1)))
                return e;
            if ((e = H.stencil(H.v[1], x, 0, RED_NONE, nullptr, -1)))
                return e;
            if ((e = H.blas(B_RES, H.v[0], nullptr, b, H.v[1], nullptr, nullptr, 0)))
                return e;
            WL_TRY(convert(H.v[0], L.v[0]));
            if (solver == WL_SOLVER_BICGSTAB) {
                // rho = <rh, r>, |r|^2 of the replaced residual, then beta
                if ((e = L.blas(B_DOT_NORM, nullptr, nullptr, L.v[1], L.v[0], nullptr, nullptr, 0)))
                    return e;
                if ((e = L.fin(F_BI_RELIABLE, 0, -1, -1, it, 0.0)))
                    return e;
            } else {
                // |r|^2, then z = D^dag r with |z|^2; the search direction stays
                if ((e = L.blas(B_NORM, nullptr, nullptr, L.v[0], nullptr, nullptr, nullptr, 0)))
                    return e;
                if ((e = L.stencil(L.v[1], L.v[0], 1, RED_NORM, nullptr, 1)))
                    return e;
                if ((e = L.fin(F_CG_RELIABLE, 0, 1, -1, it, 0.0)))
                    return e;
                if ((e = L.blas(B_CG_RESTART, L.v[2], nullptr, L.v[1], nullptr, nullptr, nullptr, -1)))
                    return e;
            }
            ++updates;
            // the status mirrored by iteration it + 1 onwards includes this
            // update; observations before that are skipped
            next_read = it + L.lookahead + 1;
            for (int r = 0; r < nrhs; ++r)
                rmax[r] = 0.0;
            return WL_OK;
        };
        if (solver == WL_SOLVER_BICGSTAB) {
            L.rel_decide = decide;
            L.rel_act = act;
        } else {
            L.on_iter = [decide, act](int it) -> int { return decide(it) ? act(it) : WL_OK; };
        }
    }
    for (;;) {
        if ((rc = H.true_res2(x, b, rr)))
            return rc;
        bool all_ok = true;
        for (int r = 0; r < nrhs; ++r) {
            if (!std::isfinite(rr[r]))
                return WL_ENAN;
            const double tol = tolv[r];
            const bool ok = rr[r] <= tol * tol * bb[r];
            sig[r] = ok ? 0.0 : std::sqrt(rr[r]);
            t2[r] = ok ? 0.0 : 0.64 * tol * tol * bb[r] / rr[r];
            if (!ok) {
                all_ok = false;
                const double rel = std::sqrt(rr[r] / bb[r]);
                if (rel > 0.9 * best[r])
                    ++stall[r];
                else
                    stall[r] = 0;
                if (rel < best[r])
                    best[r] = rel;
                if (stall[r] >= 2)
                    stagnated = true;
            }
        }
        if (all_ok || stagnated || outer >= max_outer || total >= prm->maxiter)
            break;
        // r_lo = r64 / sigma (0 for converged columns)
        WL_TRY(convert(H.v[0], r_lo));
        int done = 0;
        next_read = 0;
        last_update = 0;
        last_gap = 0;
        for (int r = 0; r < nrhs; ++r)
            rmax[r] = 0.0;
        if ((rc = L.run(e_lo, r_lo, true, delta, prm->maxiter - total, &done)))
            return rc;
        for (int r = 0; r < nrhs; ++r) {
            const Scalars &s = L.sc_host[r];
            if (sig[r] != 0.0)
                iters[r] += s.flag == 1 ? s.conv_iter : done;
            if (s.flag == 3)
                return WL_ENAN;
            if (s.flag == 2 && worst_flag < 2)
                worst_flag = 2;
        }
        total += done;
        // x64 += sigma e
        WL_TRY(accum());
        ++outer;
    }
    int worst = WL_OK;
    for (int r = 0; r < nrhs; ++r) {
        wl_solve_stats s{};
        s.iters = iters[r];
        s.outer = outer + updates;
        s.stencil_calls = H.stencil_calls + L.stencil_calls;
        s.kernels = H.kernels + L.kernels + direct;
        s.finalizes = H.finalizes + L.finalizes;
        s.true_rel_res = bb[r] > 0 ? std::sqrt(rr[r] / bb[r]) : 0.0;
        s.iter_rel_res = s.true_rel_res;
        s.converged = s.true_rel_res <= tolv[r];
        int code = s.converged ? WL_OK : (stagnated ? WL_STAGNATED : worst_flag == 2 ? WL_BREAKDOWN : WL_NOT_CONVERGED);
        if (code > worst)
            worst = code;
        if (stats)
            stats[r] = s;
    }
    return worst;
}

size_t plain_or_mixed_bytes(const wl_op *hi, const wl_op *lo, int solver, int nrhs, uint32_t V)
{
    const int Lt = hi->g.dims[3];
    if (!lo)
        return engine_bytes(solver, hi->prec, V, Lt, nrhs) + 4 * ALIGN;
    return engine_bytes(WL_SOLVER_CGNR, hi->prec, V, Lt, nrhs) + engine_bytes(solver, lo->prec, V, Lt, nrhs) +
           2 * align_up(vec_bytes(lo->prec, V, nrhs)) + 2 * align_up(sizeof(double) * nrhs) + 8 * ALIGN;
}

// Even-odd solves: engines on half fields (plus each engine's odd scratch),
// five half fields in hi's precision for the split, the Schur right-hand side
// and the reconstruction, a half engine for |bh|, a full engine for the final
// residual of D x = b, and the per-column tolerances.
size_t eo_bytes(const wl_op *hi, const wl_op *lo, int solver, int nrhs)
{
    const uint32_t Vh = hi->V / 2;
    const int Lt = hi->g.dims[3];
    size_t n = plain_or_mixed_bytes(hi, lo, solver, nrhs, Vh) + align_up(vec_bytes(hi->prec, Vh, nrhs)) +
               (lo ? align_up(vec_bytes(lo->prec, Vh, nrhs)) : 0);
    n += 5 * align_up(vec_bytes(hi->prec, Vh, nrhs));
    n += engine_bytes(WL_SOLVER_CGNR, hi->prec, Vh, Lt, nrhs) + align_up(vec_bytes(hi->prec, Vh, nrhs));
    n += engine_bytes(WL_SOLVER_CGNR, hi->prec, hi->V, Lt, nrhs);
    n += 2 * align_up(sizeof(double) * nrhs) + 16 * ALIGN;
    return n;
}

// Even-odd preconditioned solve (Schur complement on the even sites):
//   b_e, b_o = split(b);  bh = b_e + kappa H_eo b_o;  M x_e = bh;
//   x_o = b_o + kappa H_oe x_e;  x = merge(x_e, x_o)
// (with the adjoint hops for D^dag).  The Schur system is solved to
// |bh - M x_e| <= 0.9 tol |b| per column, which is the residual of D x = b
// on the even sites (the odd ones vanish by construction); the reported
// residual is recomputed on the full system.
int solve_eo(int solver, const wl_op *hi, const wl_op *lo, void *x, const void *b, int nrhs,
             const wl_solve_params *prm, wl_solve_stats *stats, hipStream_t st, Arena &arena)
{
    for (int i = 0; i < 4; ++i)
        if (hi->g.dims[i] % 2 != 0)
            return WL_EINVAL;
    if (hi->ns > 0)
        return WL_EINVAL;
    const uint32_t Vh = hi->V / 2;
    const size_t hb = vec_bytes(hi->prec, Vh, nrhs);
    void *b_e = arena.take(hb), *b_o = arena.take(hb), *bh = arena.take(hb), *x_e = arena.take(hb),
         *x_o = arena.take(hb);
    if (!b_e || !b_o || !bh || !x_e || !x_o)
        return WL_EWORKSPACE;
    HostLease lease;
    if (!lease.b->ok)
        return WL_EHIP;
    Engine F{};  // full lattice: |b| and the final true residual
    int rc = F.init(arena, hi, WL_SOLVER_CGNR, nrhs, st, lease.b, false);
    if (rc)
        return rc;
    F.adj = prm->dagger;
    Engine Hh{};  // half lattice: |bh|
    if ((rc = Hh.init(arena, hi, WL_SOLVER_CGNR, nrhs, st, lease.b, true)))
        return rc;
    WL_TRY(launch_eo_copy(hi->prec, true, hi->g.dims, nrhs, b, nullptr, b_e, b_o, st));
    EoParams pp = eo_params(hi, 0, nrhs);  // bh = b_e + kappa H_eo b_o
    pp.in = b_o;
    pp.self = b_e;
    pp.out = bh;
    pp.c_self = 1.0;
    pp.c_hop = hi->kappa;
    WL_TRY(launch_eo_hop(hi->prec, prm->dagger, RED_NONE, pp, st));
    if (prm->use_x0)
        WL_TRY(launch_eo_copy(hi->prec, true, hi->g.dims, nrhs, x, nullptr, x_e, x_o, st));
    // per-column tolerance of the Schur system: 0.9 tol |b| / |bh|
    std::vector<double> nb(nrhs), nh(nrhs), tolc(nrhs);
    double *tmp = lease.b->d;
    if ((rc = F.norm2(b, tmp)))
        return rc;
    for (int r = 0; r < nrhs; ++r)
        nb[r] = tmp[r];
    if ((rc = Hh.norm2(bh, tmp)))
        return rc;
    for (int r = 0; r < nrhs; ++r) {
        nh[r] = tmp[r];
        tolc[r] = nh[r] > 0 ? 0.9 * prm->tol * std::sqrt(nb[r] / nh[r]) : prm->tol;
    }
    std::vector<wl_solve_stats> es(nrhs);
    const int src = lo ? solve_mixed(solver, hi, lo, x_e, bh, nrhs, prm, es.data(), st, arena, true, tolc.data())
                       : solve_plain(solver, hi, x_e, bh, nrhs, prm, es.data(), st, arena, true, tolc.data());
    if (src < 0)
        return src;
    EoParams pr = eo_params(hi, 1, nrhs);  // x_o = b_o + kappa H_oe x_e
    pr.in = x_e;
    pr.self = b_o;
    pr.out = x_o;
    pr.c_self = 1.0;
    pr.c_hop = hi->kappa;
    WL_TRY(launch_eo_hop(hi->prec, prm->dagger, RED_NONE, pr, st));
    WL_TRY(launch_eo_copy(hi->prec, false, hi->g.dims, nrhs, nullptr, x, x_e, x_o, st));
    double *rr = lease.b->d + nrhs;
    if ((rc = F.true_res2(x, b, rr)))
        return rc;
    int worst = WL_OK;
    for (int r = 0; r < nrhs; ++r) {
        if (!std::isfinite(rr[r]))
            return WL_ENAN;
        wl_solve_stats s = es[r];
        s.kernels += F.kernels + Hh.kernels + 4 + (prm->use_x0 ? 1 : 0);  // the splits, two hops, the merge
        s.finalizes += F.finalizes + Hh.finalizes;
        s.true_rel_res = nb[r] > 0 ? std::sqrt(rr[r] / nb[r]) : 0.0;
        s.iter_rel_res = nb[r] > 0 ? es[r].iter_rel_res * std::sqrt(nh[r] / nb[r]) : 0.0;
        s.converged = s.true_rel_res <= prm->tol;
        const int code = s.converged ? WL_OK : (src > 0 ? src : WL_NOT_CONVERGED);
        if (code > worst)
            worst = code;
        stats[r] = s;
    }
    return worst;
}

size_t multi_bytes(const MultiSpec &ms, int solver)
{
    const int ph = ms.hi[0]->prec;
    size_t n = 2 * seg_vec_bytes(ms.hi, ph, ms.nrhs) + 16 * ALIGN;  // the segmented x and b
    if (ms.lo.empty())
        return n + multi_engine_bytes(solver, ph, ms.hi, ms.nrhs);
    const int pl = ms.lo[0]->prec;
    return n + multi_engine_bytes(WL_SOLVER_CGNR, ph, ms.hi, ms.nrhs) + multi_engine_bytes(solver, pl, ms.lo, ms.nrhs) +
           2 * seg_vec_bytes(ms.lo, pl, ms.nrhs);
}

}  // namespace

size_t multi_solver_workspace_bytes(const std::vector<const wl_op *> &hi, const std::vector<const wl_op *> &lo,
                                    int solver, int nrhs)
{
    MultiSpec ms;
    ms.hi = hi;
    ms.lo = lo;
    ms.nrhs = nrhs;
    return multi_bytes(ms, solver);
}

// Several lattices, nrhs right-hand sides each, solved together: every
// stencil application of the iteration is one multi-lattice launch (one
// descriptor table per call site), every vector update one segmented BLAS
// launch and every reduction one finalize over all columns; each column keeps
// its own scalars and stops on its own.  The right-hand sides are gathered
// into segmented buffers in the workspace and the solutions scattered back.
int solve_multi(int solver, const std::vector<const wl_op *> &hi, const std::vector<const wl_op *> &lo,
                void *const *x, const void *const *b, int nrhs, const LaunchCfg &cfg, const LaunchCfg &cfg_lo,
                const wl_solve_params *prm, wl_solve_stats *stats, hipStream_t st)
{
    const auto t0 = std::chrono::steady_clock::now();
    MultiSpec ms;
    ms.hi = hi;
    ms.lo = lo;
    ms.nrhs = nrhs;
    ms.cfg = cfg;
    ms.cfg_lo = cfg_lo;
    const size_t need = multi_bytes(ms, solver);
    if (!prm->workspace || prm->workspace_bytes < need)
        return WL_EWORKSPACE;
    Arena arena{(char *)prm->workspace, prm->workspace_bytes};
    const size_t mis = (uintptr_t)arena.base % ALIGN;
    if (mis)
        arena.off = ALIGN - mis;
    wl_solve_params q = *prm;
    q.tol = prm->tol * (1.0 - 1e-4);  // as for a single lattice
    const int ph = hi[0]->prec;
    const size_t sb = seg_vec_bytes(hi, ph, nrhs);
    char *xs = (char *)arena.take(sb), *bs = (char *)arena.take(sb);
    if (!xs || !bs)
        return WL_EWORKSPACE;
    const int n = (int)hi.size(), ncols = n * nrhs;
    std::vector<size_t> off(n);
    size_t o = 0;
    for (int i = 0; i < n; ++i) {
        off[i] = o;
        const size_t bytes = vec_bytes(ph, hi[i]->V, nrhs);
        WL_TRY(hipMemcpyAsync(bs + o, b[i], bytes, hipMemcpyDeviceToDevice, st));
        if (prm->use_x0)
            WL_TRY(hipMemcpyAsync(xs + o, x[i], bytes, hipMemcpyDeviceToDevice, st));
        o += align_up(bytes);
    }
    std::vector<wl_solve_stats> cst(ncols);
    int rc = lo.empty() ? solve_plain(solver, hi[0], xs, bs, ncols, &q, cst.data(), st, arena, false, nullptr, &ms)
                        : solve_mixed(solver, hi[0], lo[0], xs, bs, ncols, &q, cst.data(), st, arena, false, nullptr, &ms);
    if (rc >= 0)
        for (int i = 0; i < n; ++i)
            WL_TRY(hipMemcpyAsync(x[i], xs + off[i], vec_bytes(ph, hi[i]->V, nrhs), hipMemcpyDeviceToDevice, st));
    (void)hipStreamSynchronize(st);
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats && rc >= 0)
        for (int c = 0; c < ncols; ++c) {
            stats[c] = cst[c];
            stats[c].kernels += (prm->use_x0 ? 3 : 2) * n;  // gathers and scatters
            stats[c].seconds = secs;
        }
    return rc;
}

size_t solver_workspace_bytes(const wl_op *hi, const wl_op *lo, int solver, int nrhs)
{
    const size_t plain = plain_or_mixed_bytes(hi, lo, solver, nrhs, hi->V);
    bool even = hi->ns == 0;
    for (int i = 0; i < 4; ++i)
        even = even && hi->g.dims[i] % 2 == 0;
    if (!even)
        return plain;
    const size_t e = eo_bytes(hi, lo, solver, nrhs);
    return plain > e ? plain : e;
}

int solve(int solver, const wl_op *hi, const wl_op *lo, void *x, const void *b, int nrhs, const wl_solve_params *prm,
          wl_solve_stats *stats, hipStream_t st)
{
    const auto t0 = std::chrono::steady_clock::now();
    // a domain-wall system spans ns columns; the engines work on columns and
    // every reduction is taken over a system's columns, so the per-column
    // results of one system agree and its first column reports them
    const int G = hi->ns > 0 ? hi->ns : 1;
    const int ncols = nrhs * G;
    const size_t need = solver_workspace_bytes(hi, lo, solver, ncols);
    // the caller provides every device buffer: no allocation in a solve
    if (!prm->workspace || prm->workspace_bytes < need)
        return WL_EWORKSPACE;
    Arena arena{(char *)prm->workspace, prm->workspace_bytes};
    // The solve is accepted once the FP64 true residual is <= tol (1 - 1e-4):
    // an independent FP64 evaluation of b - D x (another summation order)
    // differs from the library's by a relative few 1e-6 at these residuals,
    // so it also finds <= tol.
    wl_solve_params q = *prm;
    q.tol = prm->tol * (1.0 - 1e-4);
    prm = &q;
    // align the arena start
    const size_t mis = (uintptr_t)arena.base % ALIGN;
    if (mis) {
        arena.off = ALIGN - mis;
    }
    std::vector<wl_solve_stats> cst(ncols);
    int rc = prm->eo ? solve_eo(solver, hi, lo, x, b, ncols, prm, cst.data(), st, arena)
             : lo    ? solve_mixed(solver, hi, lo, x, b, ncols, prm, cst.data(), st, arena)
                     : solve_plain(solver, hi, x, b, ncols, prm, cst.data(), st, arena);
    (void)hipStreamSynchronize(st);
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats && rc >= 0)
        for (int r = 0; r < nrhs; ++r) {
            stats[r] = cst[(size_t)r * G];
            stats[r].seconds = secs;
        }
    return rc;
}

}  // namespace wl
