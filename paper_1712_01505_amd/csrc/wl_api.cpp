// wl_api.cpp -- the C ABI (include/wilson.h): argument checking, operator
// objects, launch-configuration choice and autotuning, stencil timing, and
// the dispatch into the kernels and solver drivers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "wl_internal.h"

// A multi-lattice plan: the descriptors, the device table built from them
// for the current launch shape, and the work-queue counter.
struct wl_multi_plan {
    int n = 0, nrhs = 0, dagger = 0, prec = 0;
    std::vector<wl_multi_desc> desc;
    wl::LaunchCfg cfg{};
    int grid = 0;
    uint32_t total = 0;
    void *buf = nullptr;             // device: table, then the counter
    wl::MultiEntry *dE = nullptr;
    unsigned *counter = nullptr;     // [0] queue head, [1] exit count; zero between launches
};

namespace wl {
size_t solver_workspace_bytes(const wl_op *hi, const wl_op *lo, int solver, int nrhs);
size_t multi_solver_workspace_bytes(const std::vector<const wl_op *> &hi, const std::vector<const wl_op *> &lo,
                                    int solver, int nrhs);
int solve_multi(int solver, const std::vector<const wl_op *> &hi, const std::vector<const wl_op *> &lo,
                void *const *x, const void *const *b, int nrhs, const LaunchCfg &cfg, const LaunchCfg &cfg_lo,
                const wl_solve_params *prm, wl_solve_stats *stats, hipStream_t st);
int solve(int solver, const wl_op *hi, const wl_op *lo, void *x, const void *b, int nrhs, const wl_solve_params *prm,
          wl_solve_stats *stats, hipStream_t st);

static thread_local int g_last_hip = 0;
void set_last_hip_error(hipError_t e) { g_last_hip = (int)e; }

// ---------------------------------------------------------------- argument checks
static bool geom_ok(const wl_geom *g)
{
    if (!g)
        return false;
    uint64_t V = 1;
    for (int i = 0; i < 4; ++i) {
        if (g->dims[i] < 2)
            return false;
        if (g->bc[i] != 1 && g->bc[i] != -1)
            return false;
        V *= (uint64_t)g->dims[i];
    }
    return V <= 0x7fffffffull;
}
static uint32_t vol(const wl_geom *g) { return (uint32_t)g->dims[0] * g->dims[1] * g->dims[2] * g->dims[3]; }
static bool prec_ok(int p) { return p >= WL_F64 && p <= WL_F16S; }
static bool al16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

#define CHECK_HIP(expr)                                                                                        \
    do {                                                                                                       \
        hipError_t e_ = (expr);                                                                                \
        if (e_ != hipSuccess) {                                                                                \
            set_last_hip_error(e_);                                                                            \
            return WL_EHIP;                                                                                    \
        }                                                                                                      \
    } while (0)

// ---------------------------------------------------------------- stencil timing
struct ProfRec {
    int prec;
    hipEvent_t a, b;
    double sites;
    double aux_sites;  // sites x RHS of launches whose reduction reads a further field (aux)
};
static std::atomic<int> g_prof_on{0};
static std::mutex g_prof_mu;
static std::vector<ProfRec> g_prof_pending;
static double g_prof_ms[4] = {0, 0, 0, 0}, g_prof_sites[4] = {0, 0, 0, 0}, g_prof_aux[4] = {0, 0, 0, 0};
static long g_prof_n[4] = {0, 0, 0, 0};
static std::vector<hipEvent_t> g_event_pool;

static hipEvent_t take_event()
{
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

static void drain_prof_locked()
{
    for (auto &r : g_prof_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            g_prof_ms[r.prec] += ms;
            g_prof_sites[r.prec] += r.sites;
            g_prof_aux[r.prec] += r.aux_sites;
            g_prof_n[r.prec] += 1;
        }
        g_event_pool.push_back(r.a);
        g_event_pool.push_back(r.b);
    }
    g_prof_pending.clear();
}

hipError_t prof_stencil(int prec, const wl_op *op, int dagger, const LaunchCfg &cfg, StencilParams p, hipStream_t st)
{
    if (!g_prof_on.load(std::memory_order_relaxed))
        return launch_stencil(prec, dagger, cfg, p, st);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (g_prof_pending.size() > 4096)
        drain_prof_locked();
    hipEvent_t a = take_event(), b = take_event();
    if (!a || !b)
        return launch_stencil(prec, dagger, cfg, p, st);
    hipError_t e = hipEventRecord(a, st);
    if (e == hipSuccess)
        e = launch_stencil(prec, dagger, cfg, p, st);
    if (e == hipSuccess)
        e = hipEventRecord(b, st);
    // sites of extra vectors the fused reduction reads (RED_SR: three)
    const int naux = p.red == RED_SR ? 3 : (p.aux && (p.red == RED_DOTV || p.red == RED_BICG)) ? 1 : 0;
    if (e == hipSuccess)
        g_prof_pending.push_back(ProfRec{prec, a, b, (double)p.V * p.nrhs, (double)naux * p.V * p.nrhs});
    (void)op;
    return e;
}

// ---------------------------------------------------------------- launch choice and autotune cache
// Tuned launch shapes, keyed by (architecture, extents, precision, columns,
// dagger, fused reduction) for single operators and by (architecture,
// precision, columns, dagger, lattice list) for multi-lattice plans; kept in
// memory and, if $WL_TUNE_CACHE names a file, in that JSON file (one entry
// per line, each with its key, the key's fields and the launch shape).
struct TuneEntry {
    LaunchCfg c;
    double us = 0.0;       // measured time of the choice (per launch; reductions with their finalize)
    std::string fields;    // the key's fields as JSON members (written out as they came)
};
static std::mutex g_tune_mu;
static std::map<std::string, TuneEntry> g_tune;
static bool g_tune_loaded = false;

static std::string arch_name()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    std::string n = prop.gcnArchName;
    const size_t c = n.find(':');
    return c == std::string::npos ? n : n.substr(0, c);
}

static std::string tune_key(const wl_op *op, int nrhs, int dagger, int red)
{
    char buf[160];
    snprintf(buf, sizeof buf, "%s:%dx%dx%dx%d:p%d:n%d:d%d:r%d", arch_name().c_str(), op->g.dims[0], op->g.dims[1],
             op->g.dims[2], op->g.dims[3], op->prec, nrhs, dagger, red);
    return buf;
}

static std::string tune_fields(const wl_op *op, int nrhs, int dagger, int red)
{
    char buf[200];
    snprintf(buf, sizeof buf,
             "\"arch\": \"%s\", \"dims\": [%d, %d, %d, %d], \"prec\": %d, \"nrhs\": %d, \"dagger\": %d, "
             "\"reduction\": %d",
             arch_name().c_str(), op->g.dims[0], op->g.dims[1], op->g.dims[2], op->g.dims[3], op->prec, nrhs, dagger,
             red);
    return buf;
}

// the number after "name": in a line of the cache file
static bool json_num(const std::string &line, const char *name, double *v)
{
    const std::string pat = std::string("\"") + name + "\":";
    const size_t at = line.find(pat);
    return at != std::string::npos && sscanf(line.c_str() + at + pat.size(), " %lf", v) == 1;
}
static bool json_int(const std::string &line, const char *name, int *v)
{
    double d = 0.0;
    if (!json_num(line, name, &d))
        return false;
    *v = (int)d;
    return true;
}

static void load_tune_cache_locked()
{
    if (g_tune_loaded)
        return;
    g_tune_loaded = true;
    const char *path = getenv("WL_TUNE_CACHE");
    if (!path)
        return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t k0 = line.find("\"key\": \"");
        if (k0 == std::string::npos)
            continue;
        const size_t ks = k0 + 8, ke = line.find('"', ks);
        if (ke == std::string::npos)
            continue;
        TuneEntry t;
        LaunchCfg &c = t.c;
        bool ok = json_int(line, "block", &c.block) && json_int(line, "rhs_per_thread", &c.rpt) &&
                  json_int(line, "rhs_lanes", &c.lanes) && json_int(line, "xcd_remap", &c.xcd) &&
                  json_int(line, "variant", &c.var);
        if (!ok)
            continue;
        const size_t br = line.find("\"brick\":");
        if (br == std::string::npos || sscanf(line.c_str() + br + 8, " [%d , %d , %d ]", &c.bx, &c.by, &c.bz) != 3)
            c.bx = c.by = c.bz = 0;
        if (!json_int(line, "t_steps", &c.tsteps))
            c.tsteps = 0;
        if (!json_int(line, "wg_per_cu", &c.wpe))
            c.wpe = 0;
        if (!json_int(line, "rhs_major", &c.gmaj))
            c.gmaj = 0;
        (void)json_num(line, "us", &t.us);
        // the key's fields: everything between the key and the launch shape
        const size_t fs = line.find(',', ke), fe = line.find(", \"block\":");
        if (fs != std::string::npos && fe != std::string::npos && fe > fs + 2)
            t.fields = line.substr(fs + 2, fe - fs - 2);
        g_tune[line.substr(ks, ke - ks)] = t;
    }
}

static void save_tune_cache_locked()
{
    const char *path = getenv("WL_TUNE_CACHE");
    if (!path)
        return;
    std::ofstream f(path, std::ios::trunc);
    f << "{\"format\": \"wilson launch shapes\", \"entries\": [\n";
    size_t i = 0;
    for (auto &kv : g_tune) {
        const LaunchCfg &c = kv.second.c;
        char buf[512];
        snprintf(buf, sizeof buf,
                 "\"block\": %d, \"rhs_per_thread\": %d, \"rhs_lanes\": %d, \"xcd_remap\": %d, \"variant\": %d, "
                 "\"brick\": [%d, %d, %d], \"t_steps\": %d, \"wg_per_cu\": %d, \"rhs_major\": %d, \"us\": %.3f",
                 c.block, c.rpt, c.lanes, c.xcd, c.var, c.bx, c.by, c.bz, c.tsteps, c.wpe, c.gmaj, kv.second.us);
        f << "{\"key\": \"" << kv.first << "\", ";
        if (!kv.second.fields.empty())
            f << kv.second.fields << ", ";
        f << buf << "}" << (++i < g_tune.size() ? "," : "") << "\n";
    }
    f << "]}\n";
}

// Untuned defaults (measured on MI355X at 32^3 x 64): one right-hand side
// runs the pipelined hop loop with small workgroups; several right-hand
// sides share each link load across RHS_per_thread spinors.
static LaunchCfg default_launch(const wl_op *op, int nrhs)
{
    const int prec = op->prec;
    LaunchCfg c;
    if (nrhs == 1) {
        c.rpt = 1;
        if (prec == WL_F64 || prec == WL_F32) {
            c.block = 256;
            c.xcd = slab_ok(op->g.dims, 256, 2) ? 2 : 0;
            c.var = prec == WL_F64 ? 1 : 2;
        } else {
            c.block = 128;
            c.xcd = 1;
            c.var = 2;
        }
        return c;
    }
    // several right-hand sides: interleave them across the lanes of each
    // wavefront (one link fetch per instruction serves all of them)
    c.block = 256;
    c.xcd = 1;
    c.rpt = 1;
    c.var = prec == WL_F64 ? 1 : 2;
    c.lanes = nrhs % 4 == 0 ? 4 : nrhs % 2 == 0 ? 2 : 1;
    return c;
}

static bool launch_ok(const wl_op *op, int nrhs, const LaunchCfg &c)
{
    const int prec = op->prec;
    if (op->ns > 0 && (c.rpt != 1 || c.var == 3 || c.var > 6 || nrhs % op->ns != 0))
        return false;  // domain wall: one slice per thread, variants 0..2 and the t-walks
    // columns across lanes: at least 64 sites per workgroup, 32 for the
    // t-walks; the brick walk takes rhs_lanes right-hand sides per workgroup
    const bool lanes_ok = c.lanes == 1 || ((c.lanes == 2 || c.lanes == 4 || c.lanes == 8) && c.rpt == 1 &&
                                           nrhs % c.lanes == 0 &&
                                           (c.var == VAR_BRICK || c.block / c.lanes >= (c.var >= 4 ? 32 : 64)));
    return c.block >= 64 && c.block <= 512 && c.block % 64 == 0 && c.rpt >= 1 && c.rpt <= max_rpt(prec) &&
           nrhs % c.rpt == 0 && lanes_ok && c.xcd >= 0 && c.xcd <= 5 &&
           (c.xcd < 2 || slab_ok(op->g.dims, c.block / c.lanes, c.xcd)) && c.var >= 0 && c.var <= max_var(prec) &&
           var_ok(prec, c.var) && (c.var == 0 || c.rpt == 1) &&
           (c.var < 4 || c.var == VAR_BRICK ||
            (c.block <= 256 && op->g.dims[3] % (c.var == 4 ? 4 : c.var == 5 ? 8 : 16) == 0)) &&
           (c.var != VAR_BRICK || (op->ns == 0 && c.bx * c.by * c.bz * c.lanes == c.block &&
                                   brick_ok(op->g.dims, prec, c.bx, c.by, c.bz, c.tsteps, c.wpe, c.lanes))) &&
           (c.wpe == 0 || c.var == VAR_BRICK) && (c.gmaj == 0 || c.gmaj == 1);
}

// Brick shapes (variant 7) for extents L: x extent 8, 16 or 32, the rest
// as close to cubic as the divisors allow, 128 or 256 sites; walks of 4, 8
// or 16 t-slices.  With several right-hand sides also 64- and 128-site
// bricks (x extent 4 too) holding 2 or 4 of them per workgroup.
static void brick_candidates(const wl_op *op, int nrhs, std::vector<LaunchCfg> &out)
{
    const int *L = op->g.dims;
    if (op->ns > 0)
        return;
    const int sites[] = {64, 128, 256};
    const int bxs[] = {4, 8, 16, 32};
    const int ts[] = {4, 8, 16};
    for (int rw = 1; rw <= 4; rw *= 2) {
        if (nrhs % rw != 0)
            continue;
        for (int nb : sites) {
            if ((rw == 1 && nb == 64) || nb * rw > 256)
                continue;
            for (int bx : bxs) {
                if (nb % bx != 0 || (bx == 4 && rw == 1))
                    continue;
                const int rest = nb / bx;
                for (int by = 1; by <= rest; by *= 2) {
                    const int bz = rest / by;
                    if (by * bz != rest || by > 4 * bz || bz > 4 * by)
                        continue;
                    for (int T : ts)
                        for (int xcd = 0; xcd <= 1; ++xcd) {
                            LaunchCfg c{nb * rw, 1, xcd, VAR_BRICK, rw};
                            c.bx = bx;
                            c.by = by;
                            c.bz = bz;
                            c.tsteps = T;
                            if (brick_ok(L, op->prec, bx, by, bz, T, 0, rw))
                                out.push_back(c);
                        }
                }
            }
        }
    }
}

// Launch configurations are kept per (nrhs, fused reduction, dagger): the
// solver's stencils with a reduction epilogue are tuned separately from the
// plain apply.  A combination without its own entry takes the other dagger's,
// then the plain apply's, then the default.
static int launch_key(int nrhs, int red, int dagger) { return (nrhs * 8 + red) * 2 + dagger; }

LaunchCfg launch_for(const wl_op *op, int nrhs, int red, int dagger)
{
    wl_op *o = const_cast<wl_op *>(op);
    {
        std::lock_guard<std::mutex> lk(o->mu);
        auto it = o->launch.find(launch_key(nrhs, red, dagger));
        if (it != o->launch.end())
            return it->second;
    }
    // first use of this (nrhs, reduction, dagger): search the op's choices
    // and the tune cache in the order above
    LaunchCfg c = default_launch(op, nrhs);
    const int order[4][2] = {{red, dagger}, {red, 1 - dagger}, {RED_NONE, dagger}, {RED_NONE, 1 - dagger}};
    bool have = false;
    for (int k = 0; k < 4 && !have; ++k) {
        {
            std::lock_guard<std::mutex> lk(o->mu);
            auto it = o->launch.find(launch_key(nrhs, order[k][0], order[k][1]));
            if (it != o->launch.end()) {
                c = it->second;
                have = true;
                break;
            }
        }
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_tune_cache_locked();
        auto it = g_tune.find(tune_key(op, nrhs, order[k][1], order[k][0]));
        if (it != g_tune.end() && launch_ok(op, nrhs, it->second.c)) {
            c = it->second.c;
            have = true;
        }
    }
    std::lock_guard<std::mutex> lk(o->mu);
    o->launch[launch_key(nrhs, red, dagger)] = c;
    return c;
}

static StencilParams base_params(const wl_op *op, void *out, const void *in, int nrhs, int apply)
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
    p.apply = apply;
    p.red = RED_NONE;
    p.one = 1.0f;
    if (apply)
        op_apply_params(op, p);
    return p;
}

void op_apply_params(const wl_op *op, StencilParams &p)
{
    if (op->ns > 0) {
        p.apply = 2;
        p.ns = op->ns;
        p.dw_diag = op->m0 + 5.0;
        p.dw_m = op->mq;
        p.kappa = 0.5;
    }
}

// ---------------------------------------------------------------- multi-lattice plans
// Plan shapes reuse LaunchCfg: block, rpt, var, and xcd = 1 for the
// persistent work-queue form, 0 for one workgroup per work item.
static LaunchCfg multi_default(int prec, int nrhs)
{
    (void)nrhs;
    return LaunchCfg{256, 1, 1, prec == WL_F64 ? 1 : 2, 1};
}

static std::string multi_key_of(int prec, int nrhs, int dagger, const std::vector<const wl_op *> &ops)
{
    std::string k = arch_name() + ":multi:p" + std::to_string(prec) + ":n" + std::to_string(nrhs) + ":d" +
                    std::to_string(dagger);
    for (const wl_op *op : ops) {
        char buf[64];
        snprintf(buf, sizeof buf, ":%dx%dx%dx%d", op->g.dims[0], op->g.dims[1], op->g.dims[2], op->g.dims[3]);
        k += buf;
    }
    return k;
}

static std::string multi_key(const wl_multi_plan *pl)
{
    std::vector<const wl_op *> ops;
    for (const auto &d : pl->desc)
        ops.push_back(d.op);
    return multi_key_of(pl->prec, pl->nrhs, pl->dagger, ops);
}

// Launch shape of a multi-lattice solve's stencils (one site per thread, the
// direct form): the plan tuner's choice for these lattices if it has one
// with one right-hand side per thread, else the default.
static LaunchCfg multi_solve_shape(int prec, int nrhs, const std::vector<const wl_op *> &ops)
{
    LaunchCfg c = multi_default(prec, nrhs);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_cache_locked();
    auto it = g_tune.find(multi_key_of(prec, nrhs, 0, ops));
    if (it != g_tune.end() && it->second.c.rpt == 1 && multi_launch_ok(prec, 1, it->second.c.block, it->second.c.var))
        c = it->second.c;
    c.rpt = 1;
    c.xcd = 0;
    return c;
}

static std::string multi_fields(const wl_multi_plan *pl)
{
    std::string f = "\"arch\": \"" + arch_name() + "\", \"multi_lattice\": [";
    for (size_t i = 0; i < pl->desc.size(); ++i) {
        const int *L = pl->desc[i].op->g.dims;
        char buf[64];
        snprintf(buf, sizeof buf, "%s[%d, %d, %d, %d]", i ? ", " : "", L[0], L[1], L[2], L[3]);
        f += buf;
    }
    return f + "], \"prec\": " + std::to_string(pl->prec) + ", \"nrhs\": " + std::to_string(pl->nrhs) +
           ", \"dagger\": " + std::to_string(pl->dagger);
}

// (Re)build the descriptor table for launch shape c and upload it
// (synchronous; the plan must be idle).
static int plan_build(wl_multi_plan *pl, const LaunchCfg &c)
{
    if (pl->nrhs % c.rpt != 0 || !multi_launch_ok(pl->prec, c.rpt, c.block, c.var))
        return WL_EINVAL;
    std::vector<MultiEntry> E(pl->n);
    const uint32_t ng = (uint32_t)(pl->nrhs / c.rpt);
    uint64_t total = 0;
    for (int i = 0; i < pl->n; ++i) {
        const wl_multi_desc &d = pl->desc[i];
        E[i].p = base_params(d.op, d.out, d.in, pl->nrhs, 1);
        E[i].p.nblk = (int)((d.op->V + c.block - 1) / c.block);
        E[i].p.ng = ng;
        E[i].p.f_ng = make_fastdiv(ng);
        E[i].tile_begin = (uint32_t)total;
        total += (uint64_t)E[i].p.nblk * ng;
        if (total > 0x7fffffffull)
            return WL_EINVAL;
    }
    CHECK_HIP(hipMemcpy(pl->dE, E.data(), sizeof(MultiEntry) * pl->n, hipMemcpyHostToDevice));
    int grid = 0;  // direct form: one workgroup per item
    if (c.xcd == 1) {  // persistent form: resident workgroups only
        grid = multi_grid_size(pl->prec, pl->dagger, c.rpt, c.block, c.var);
        if (grid < 1)
            return WL_EINVAL;
        if ((uint64_t)grid > total)
            grid = (int)total;
    }
    pl->cfg = c;
    pl->total = (uint32_t)total;
    pl->grid = grid;
    return WL_OK;
}

static void plan_free(wl_multi_plan *pl)
{
    if (pl->buf)
        (void)hipFree(pl->buf);
    delete pl;
}

}  // namespace wl

using namespace wl;

extern "C" {

const char *wl_strerror(int code)
{
    switch (code) {
    case WL_OK: return "ok";
    case WL_NOT_CONVERGED: return "not converged (maxiter reached)";
    case WL_BREAKDOWN: return "Krylov breakdown";
    case WL_STAGNATED: return "mixed-precision refinement stagnated";
    case WL_EINVAL: return "invalid argument";
    case WL_EALIGN: return "pointer not 16-byte aligned";
    case WL_EPREC: return "unsupported precision";
    case WL_EHIP: return "HIP runtime error";
    case WL_ENAN: return "NaN/Inf in residual";
    case WL_EWORKSPACE: return "workspace too small";
    default: return "unknown error";
    }
}

int wl_last_hip_error(void) { return g_last_hip; }

int wl_field_bytes(const wl_geom *g, int kind, int prec, int nrhs, size_t *out_bytes)
{
    if (!geom_ok(g) || !out_bytes || (kind != WL_SPINOR && kind != WL_GAUGE))
        return WL_EINVAL;
    if (!prec_ok(prec))
        return WL_EPREC;
    const uint32_t V = vol(g);
    if (kind == WL_SPINOR) {
        if (nrhs < 1)
            return WL_EINVAL;
        *out_bytes = (size_t)nrhs * V * spinor_site_bytes(prec);
    } else {
        *out_bytes = (size_t)4 * V * link_site_bytes(prec);
    }
    return WL_OK;
}

int wl_pack_gauge(const wl_geom *g, int prec, const void *U_canon, void *U_packed, void *stream)
{
    if (!geom_ok(g) || !U_canon || !U_packed)
        return WL_EINVAL;
    if (!prec_ok(prec))
        return WL_EPREC;
    if (!al16(U_canon) || !al16(U_packed))
        return WL_EALIGN;
    CHECK_HIP(launch_pack_gauge(prec, vol(g), U_canon, U_packed, (hipStream_t)stream));
    return WL_OK;
}

int wl_pack_spinor(const wl_geom *g, int prec, int nrhs, const void *psi_canon, void *psi_packed, void *stream)
{
    if (!geom_ok(g) || !psi_canon || !psi_packed || nrhs < 1 || nrhs > 65535)
        return WL_EINVAL;
    if (!prec_ok(prec))
        return WL_EPREC;
    if (!al16(psi_canon) || !al16(psi_packed))
        return WL_EALIGN;
    CHECK_HIP(launch_pack_spinor(prec, vol(g), nrhs, psi_canon, psi_packed, (hipStream_t)stream));
    return WL_OK;
}

int wl_unpack_spinor(const wl_geom *g, int prec, int nrhs, const void *psi_packed, void *psi_canon, void *stream)
{
    if (!geom_ok(g) || !psi_canon || !psi_packed || nrhs < 1 || nrhs > 65535)
        return WL_EINVAL;
    if (!prec_ok(prec))
        return WL_EPREC;
    if (!al16(psi_canon) || !al16(psi_packed))
        return WL_EALIGN;
    CHECK_HIP(launch_unpack_spinor(prec, vol(g), nrhs, psi_packed, psi_canon, (hipStream_t)stream));
    return WL_OK;
}

int wl_convert_spinor(const wl_geom *g, int prec_in, int prec_out, int nrhs, const void *in, void *out, void *stream)
{
    if (!geom_ok(g) || !in || !out || nrhs < 1 || nrhs > 65535)
        return WL_EINVAL;
    if (!prec_ok(prec_in) || !prec_ok(prec_out))
        return WL_EPREC;
    if (!al16(in) || !al16(out))
        return WL_EALIGN;
    CHECK_HIP(launch_convert(prec_in, prec_out, vol(g), nrhs, in, out, nullptr, 0, 0, (hipStream_t)stream));
    return WL_OK;
}

int wl_op_create(const wl_geom *g, double kappa, int prec, const void *U_packed, wl_op **out)
{
    if (!geom_ok(g) || !U_packed || !out || !std::isfinite(kappa))
        return WL_EINVAL;
    if (!prec_ok(prec))
        return WL_EPREC;
    if (!al16(U_packed))
        return WL_EALIGN;
    wl_op *op = new wl_op();
    op->g = *g;
    op->kappa = kappa;
    op->prec = prec;
    op->U = U_packed;
    op->V = vol(g);
    *out = op;
    return WL_OK;
}

int wl_dw_op_create(const wl_geom *g, double m0, double m, int Ns, int prec, const void *U_packed, wl_op **out)
{
    if (!geom_ok(g) || !U_packed || !out || !std::isfinite(m0) || !std::isfinite(m) || Ns < 1 || Ns > 64)
        return WL_EINVAL;
    if (!prec_ok(prec))
        return WL_EPREC;
    if (!al16(U_packed))
        return WL_EALIGN;
    wl_op *op = new wl_op();
    op->g = *g;
    op->kappa = 0.0;
    op->prec = prec;
    op->U = U_packed;
    op->V = vol(g);
    op->ns = Ns;
    op->m0 = m0;
    op->mq = m;
    *out = op;
    return WL_OK;
}

int wl_op_destroy(wl_op *op)
{
    delete op;
    return WL_OK;
}

static int stencil_call(const wl_op *op, void *out, const void *in, int dagger, int nrhs, void *stream, int apply)
{
    if (!op || !out || !in || nrhs < 1 || nrhs > 65535 || (dagger != 0 && dagger != 1) || out == in)
        return WL_EINVAL;
    if (!al16(out) || !al16(in))
        return WL_EALIGN;
    LaunchCfg cfg = launch_for(op, nrhs, RED_NONE, dagger);
    if (nrhs % cfg.rpt != 0) {
        cfg.rpt = 1;
        cfg.var = 0;
    }
    StencilParams p = base_params(op, out, in, nrhs, apply);
    CHECK_HIP(prof_stencil(op->prec, op, dagger, cfg, p, (hipStream_t)stream));
    return WL_OK;
}

// Enforced halo: face pack, the face copy, the interior and the finish, in
// that order on the caller's stream.  On one GPU the copy takes a few
// microseconds, less than a synchronisation between two streams would; with
// several GPUs the exchange goes to a communication stream and overlaps the
// interior.

int wl_halo_bytes(const wl_op *op, int nrhs, size_t *out_bytes)
{
    if (!op || op->ns > 0 || nrhs < 1 || nrhs > 65535 || !out_bytes)
        return WL_EINVAL;
    const uint32_t vs = (uint32_t)op->g.dims[0] * op->g.dims[1] * op->g.dims[2];
    *out_bytes = 4 * halo_face_bytes(op->prec, vs, nrhs);  // send and receive, two faces each
    return WL_OK;
}

int wilson_apply_halo(const wl_op *op, void *out, const void *in, int dagger, int nrhs, void *halo,
                      size_t halo_bytes, void *stream)
{
    size_t need = 0;
    if (!op || !out || !in || !halo || out == in || (dagger != 0 && dagger != 1) ||
        wl_halo_bytes(op, nrhs, &need) != WL_OK)
        return WL_EINVAL;
    if (halo_bytes < need)
        return WL_EWORKSPACE;
    if (!al16(out) || !al16(in) || !al16(halo))
        return WL_EALIGN;
    // the interior runs in the tuned shape (every variant leaves out the
    // wrapping t hops when halo_t is set)
    const LaunchCfg cfg = launch_for(op, nrhs, RED_NONE, dagger);
    StencilParams p = base_params(op, out, in, nrhs, 1);
    p.halo_t = 1;
    p.halo_send = halo;
    p.halo_recv = (char *)halo + need / 2;
    hipStream_t st = (hipStream_t)stream;
    CHECK_HIP(launch_halo_pack(op->prec, dagger, p, st));
    // the exchange (here with itself): a streaming copy kernel
    CHECK_HIP(launch_stream_copy(const_cast<void *>(p.halo_recv), p.halo_send, need / 2, st));
    // interior: every site, the wrapping t hops left out
    CHECK_HIP(prof_stencil(op->prec, op, dagger, cfg, p, st));
    // then the received faces into the boundary slices
    CHECK_HIP(launch_halo_finish(op->prec, dagger, p, st));
    return WL_OK;
}

// ---------------------------------------------------------------- even-odd
// the hopping term couples only opposite parities when every extent is even
static bool eo_geom_ok(const wl_geom *g)
{
    return geom_ok(g) && g->dims[0] % 2 == 0 && g->dims[1] % 2 == 0 && g->dims[2] % 2 == 0 && g->dims[3] % 2 == 0;
}

int wl_eo_split(const wl_geom *g, int prec, int nrhs, const void *full, void *even, void *odd, void *stream)
{
    if (!eo_geom_ok(g) || !full || !even || !odd || nrhs < 1 || nrhs > 65535 || even == odd)
        return WL_EINVAL;
    if (!prec_ok(prec))
        return WL_EPREC;
    if (!al16(full) || !al16(even) || !al16(odd))
        return WL_EALIGN;
    CHECK_HIP(launch_eo_copy(prec, true, g->dims, nrhs, full, nullptr, even, odd, (hipStream_t)stream));
    return WL_OK;
}

int wl_eo_merge(const wl_geom *g, int prec, int nrhs, const void *even, const void *odd, void *full, void *stream)
{
    if (!eo_geom_ok(g) || !full || !even || !odd || nrhs < 1 || nrhs > 65535 || even == odd)
        return WL_EINVAL;
    if (!prec_ok(prec))
        return WL_EPREC;
    if (!al16(full) || !al16(even) || !al16(odd))
        return WL_EALIGN;
    CHECK_HIP(launch_eo_copy(prec, false, g->dims, nrhs, nullptr, full, const_cast<void *>(even),
                             const_cast<void *>(odd), (hipStream_t)stream));
    return WL_OK;
}

int wilson_schur_apply(const wl_op *op, void *out_e, const void *in_e, void *tmp_o, int dagger, int nrhs,
                       void *stream)
{
    if (!op || op->ns > 0 || !eo_geom_ok(&op->g) || !out_e || !in_e || !tmp_o || out_e == in_e ||
        tmp_o == in_e || tmp_o == out_e || nrhs < 1 || nrhs > 65535 || (dagger != 0 && dagger != 1))
        return WL_EINVAL;
    if (!al16(out_e) || !al16(in_e) || !al16(tmp_o))
        return WL_EALIGN;
    hipStream_t st = (hipStream_t)stream;
    EoParams a = eo_params(op, 1, nrhs);  // tmp_o = H_oe in_e
    a.in = in_e;
    a.out = tmp_o;
    a.c_hop = 1.0;
    CHECK_HIP(launch_eo_hop(op->prec, dagger, RED_NONE, a, st));
    EoParams b = eo_params(op, 0, nrhs);  // out_e = in_e - kappa^2 H_eo tmp_o
    b.in = tmp_o;
    b.self = in_e;
    b.out = out_e;
    b.c_self = 1.0;
    b.c_hop = -op->kappa * op->kappa;
    CHECK_HIP(launch_eo_hop(op->prec, dagger, RED_NONE, b, st));
    return WL_OK;
}

int dwf_apply(const wl_op *op, void *out, const void *in, int dagger, int nvec, void *stream)
{
    if (!op || op->ns < 1 || nvec < 1 || (long)nvec * op->ns > 65535)
        return WL_EINVAL;
    return stencil_call(op, out, in, dagger, nvec * op->ns, stream, 1);
}

int wilson_dslash(const wl_op *op, void *out, const void *in, int dagger, int nrhs, void *stream)
{
    if (op && op->ns > 0)
        return WL_EINVAL;  // a domain-wall operator: dwf_apply
    return stencil_call(op, out, in, dagger, nrhs, stream, 0);
}

int wilson_apply(const wl_op *op, void *out, const void *in, int dagger, int nrhs, void *stream)
{
    if (op && op->ns > 0)
        return WL_EINVAL;
    return stencil_call(op, out, in, dagger, nrhs, stream, 1);
}

int wl_solver_workspace_bytes(const wl_op *hi, const wl_op *lo, int solver, int nrhs, size_t *out_bytes)
{
    if (!hi || !out_bytes || nrhs < 1 || op_cols(hi, nrhs) > 64 ||
        (solver != WL_SOLVER_CGNR && solver != WL_SOLVER_BICGSTAB))
        return WL_EINVAL;
    *out_bytes = solver_workspace_bytes(hi, lo, solver, op_cols(hi, nrhs));
    return WL_OK;
}

static int solve_entry(int solver, const wl_op *hi, const wl_op *lo, void *x, const void *b, int nrhs,
                       const wl_solve_params *p, wl_solve_stats *stats, void *stream)
{
    if (!hi || !x || !b || !p || nrhs < 1 || op_cols(hi, nrhs) > 64 || x == b || !(p->tol > 0) ||
        p->maxiter < 1 || (p->dagger != 0 && p->dagger != 1) || (p->form != 0 && p->form != 1))
        return WL_EINVAL;
    // the single-reduction forms keep recurrences (w = D p; v = D p and
    // q = D v) that a residual replacement would break: defect correction only
    if (p->form == 1 && lo && p->reliable)
        return WL_EINVAL;
    if (hi->ns > 0 && solver != WL_SOLVER_CGNR)
        return WL_EINVAL;  // domain wall: CG on the normal equations only (Sec. II-C, Sec. VI-B)
    if (!al16(x) || !al16(b))
        return WL_EALIGN;
    if (lo) {
        if (hi->prec != WL_F64 || lo->prec == WL_F64)
            return WL_EPREC;
        // CG on the normal equations cannot carry its recurrence between
        // reliable updates with 16-bit storage (measured: BF16 stalls, FP16
        // drifts into thousands of iterations or overflows); those pairs take
        // defect correction (reliable = 0) only
        if (p->reliable && solver == WL_SOLVER_CGNR && lo->prec != WL_F32)
            return WL_EPREC;
        for (int i = 0; i < 4; ++i)
            if (lo->g.dims[i] != hi->g.dims[i] || lo->g.bc[i] != hi->g.bc[i])
                return WL_EINVAL;
        if (lo->kappa != hi->kappa || lo->ns != hi->ns || lo->m0 != hi->m0 || lo->mq != hi->mq)
            return WL_EINVAL;
    } else if (hi->prec != WL_F64 && hi->prec != WL_F32) {
        return WL_EPREC;  // plain solves run in FP64 or FP32 storage
    }
    return solve(solver, hi, lo, x, b, nrhs, p, stats, (hipStream_t)stream);
}

int solve_cgnr(const wl_op *hi, const wl_op *lo, void *x, const void *b, int nrhs, const wl_solve_params *p,
               wl_solve_stats *stats, void *stream)
{
    return solve_entry(WL_SOLVER_CGNR, hi, lo, x, b, nrhs, p, stats, stream);
}

int solve_bicgstab(const wl_op *hi, const wl_op *lo, void *x, const void *b, int nrhs, const wl_solve_params *p,
                   wl_solve_stats *stats, void *stream)
{
    return solve_entry(WL_SOLVER_BICGSTAB, hi, lo, x, b, nrhs, p, stats, stream);
}

// Multi-lattice solves: validation shared by the workspace query and the solve.
static int multi_systems(const wl_multi_system *s, int n, int solver, int nrhs, std::vector<const wl_op *> &hi,
                         std::vector<const wl_op *> &lo)
{
    if (!s || n < 1 || nrhs < 1 || (long)n * nrhs > 64 || (solver != WL_SOLVER_CGNR && solver != WL_SOLVER_BICGSTAB))
        return WL_EINVAL;
    const bool mixed = s[0].lo != nullptr;
    for (int i = 0; i < n; ++i) {
        const wl_multi_system &q = s[i];
        if (!q.hi || q.hi->ns > 0 || (q.lo != nullptr) != mixed || q.hi->prec != s[0].hi->prec)
            return WL_EINVAL;
        if (mixed) {
            if (q.lo->ns > 0 || q.lo->prec != s[0].lo->prec)
                return WL_EINVAL;
            for (int k = 0; k < 4; ++k)
                if (q.lo->g.dims[k] != q.hi->g.dims[k] || q.lo->g.bc[k] != q.hi->g.bc[k])
                    return WL_EINVAL;
            if (q.lo->kappa != q.hi->kappa)
                return WL_EINVAL;
        }
        hi.push_back(q.hi);
        if (mixed)
            lo.push_back(q.lo);
    }
    if (mixed ? (s[0].hi->prec != WL_F64 || s[0].lo->prec == WL_F64)
              : (s[0].hi->prec != WL_F64 && s[0].hi->prec != WL_F32))
        return WL_EPREC;
    return WL_OK;
}

int wl_multi_solver_workspace_bytes(const wl_multi_system *s, int n, int solver, int nrhs, size_t *out_bytes)
{
    std::vector<const wl_op *> hi, lo;
    if (!out_bytes)
        return WL_EINVAL;
    const int rc = multi_systems(s, n, solver, nrhs, hi, lo);
    if (rc != WL_OK)
        return rc;
    *out_bytes = multi_solver_workspace_bytes(hi, lo, solver, nrhs);
    return WL_OK;
}

int wilson_solve_multi(const wl_multi_system *s, int n, int solver, int nrhs, const wl_solve_params *p,
                       wl_solve_stats *stats, void *stream)
{
    std::vector<const wl_op *> hi, lo;
    int rc = multi_systems(s, n, solver, nrhs, hi, lo);
    if (rc != WL_OK)
        return rc;
    if (!p || !(p->tol > 0) || p->maxiter < 1 || (p->dagger != 0 && p->dagger != 1) || (p->form != 0 && p->form != 1) ||
        p->eo != 0 || (p->form == 1 && !lo.empty() && p->reliable))
        return WL_EINVAL;
    if (p->reliable && solver == WL_SOLVER_CGNR && !lo.empty() && lo[0]->prec != WL_F32)
        return WL_EPREC;
    std::vector<void *> x(n);
    std::vector<const void *> b(n);
    for (int i = 0; i < n; ++i) {
        if (!s[i].x || !s[i].b || s[i].x == s[i].b)
            return WL_EINVAL;
        if (!al16(s[i].x) || !al16(s[i].b))
            return WL_EALIGN;
        x[i] = s[i].x;
        b[i] = s[i].b;
    }
    const LaunchCfg cfg = multi_solve_shape(hi[0]->prec, nrhs, hi);
    const LaunchCfg cfg_lo = lo.empty() ? cfg : multi_solve_shape(lo[0]->prec, nrhs, lo);
    return solve_multi(solver, hi, lo, x.data(), b.data(), nrhs, cfg, cfg_lo, p, stats, (hipStream_t)stream);
}

int wilson_gauge_force(const wl_op *op, void *out_canon, const void *x, const void *mu, int project, void *stream)
{
    if (!op || !out_canon || !x || !mu || project < 0 || project > 2 || op->ns > 0)
        return WL_EINVAL;
    if (op->prec != WL_F64 && op->prec != WL_F32)
        return WL_EPREC;
    if (!al16(out_canon) || !al16(x) || !al16(mu))
        return WL_EALIGN;
    CHECK_HIP(launch_force(op->prec, op, out_canon, x, mu, project, (hipStream_t)stream));
    return WL_OK;
}

int wl_multi_plan_create(const wl_multi_desc *d, int n, int dagger, int nrhs, wl_multi_plan **out)
{
    if (!out)
        return WL_EINVAL;
    *out = nullptr;
    if (!d || n < 1 || n > 1024 || (dagger != 0 && dagger != 1) || nrhs < 1 || nrhs > 65535)
        return WL_EINVAL;
    const int prec = d[0].op ? d[0].op->prec : -1;
    for (int i = 0; i < n; ++i) {
        if (!d[i].op || !d[i].out || !d[i].in || d[i].out == d[i].in || d[i].op->ns > 0)
            return WL_EINVAL;
        if (d[i].op->prec != prec)
            return WL_EPREC;
        if (!al16(d[i].out) || !al16(d[i].in))
            return WL_EALIGN;
    }
    wl_multi_plan *pl = new wl_multi_plan();
    pl->n = n;
    pl->nrhs = nrhs;
    pl->dagger = dagger;
    pl->prec = prec;
    pl->desc.assign(d, d + n);
    const size_t bytes = sizeof(MultiEntry) * n + 256;
    hipError_t e = hipMalloc(&pl->buf, bytes);
    pl->dE = (MultiEntry *)pl->buf;
    if (e == hipSuccess)
        pl->counter = (unsigned *)((char *)pl->buf + (sizeof(MultiEntry) * n + 127) / 128 * 128);
    if (e == hipSuccess)
        e = hipMemset(pl->counter, 0, 2 * sizeof(unsigned));
    if (e != hipSuccess) {
        set_last_hip_error(e);
        plan_free(pl);
        return WL_EHIP;
    }
    LaunchCfg c = multi_default(prec, nrhs);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_tune_cache_locked();
        auto it = g_tune.find(multi_key(pl));
        if (it != g_tune.end() && nrhs % it->second.c.rpt == 0 &&
            multi_launch_ok(prec, it->second.c.rpt, it->second.c.block, it->second.c.var))
            c = it->second.c;
    }
    const int rc = plan_build(pl, c);
    if (rc != WL_OK) {
        plan_free(pl);
        return rc;
    }
    *out = pl;
    return WL_OK;
}

int wl_multi_plan_run(wl_multi_plan *pl, void *stream)
{
    if (!pl)
        return WL_EINVAL;
    CHECK_HIP(launch_multi(pl->prec, pl->dagger, pl->cfg.rpt, pl->cfg.block, pl->cfg.var, pl->dE, pl->n, pl->total,
                           pl->counter, pl->grid, (hipStream_t)stream));
    return WL_OK;
}

int wl_multi_plan_tune(wl_multi_plan *pl, void *stream)
{
    if (!pl)
        return WL_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    CHECK_HIP(hipStreamSynchronize(st));
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess)
        e = hipEventCreate(&b);
    LaunchCfg best = pl->cfg;
    float best_ms = INFINITY;
    const int blocks[] = {64, 128, 256, 512};
    int rc = WL_OK;
    for (int pers = 0; pers <= 1 && e == hipSuccess && rc == WL_OK; ++pers)
        for (int bi = 0; bi < 4 && e == hipSuccess && rc == WL_OK; ++bi)
            for (int rpt = 1; rpt <= 4 && e == hipSuccess && rc == WL_OK; ++rpt)
                for (int var = 0; var <= 3 && e == hipSuccess && rc == WL_OK; ++var) {
                    if (pl->nrhs % rpt != 0 || !multi_launch_ok(pl->prec, rpt, blocks[bi], var))
                        continue;
                    if ((rc = plan_build(pl, LaunchCfg{blocks[bi], rpt, pers, var, 1})) != WL_OK)
                        break;
                    for (int w = 0; w < 2 && e == hipSuccess; ++w)
                        e = launch_multi(pl->prec, pl->dagger, rpt, blocks[bi], var, pl->dE, pl->n, pl->total,
                                         pl->counter, pl->grid, st);
                    const int reps = 10;
                    if (e == hipSuccess)
                        e = hipEventRecord(a, st);
                    for (int k = 0; k < reps && e == hipSuccess; ++k)
                        e = launch_multi(pl->prec, pl->dagger, rpt, blocks[bi], var, pl->dE, pl->n, pl->total,
                                         pl->counter, pl->grid, st);
                    if (e == hipSuccess)
                        e = hipEventRecord(b, st);
                    if (e == hipSuccess)
                        e = hipEventSynchronize(b);
                    float ms = 0.f;
                    if (e == hipSuccess)
                        e = hipEventElapsedTime(&ms, a, b);
                    if (e == hipSuccess && ms < best_ms) {
                        best_ms = ms;
                        best = pl->cfg;
                    }
                }
    if (a)
        (void)hipEventDestroy(a);
    if (b)
        (void)hipEventDestroy(b);
    CHECK_HIP(e);
    if (rc != WL_OK)
        return rc;
    if ((rc = plan_build(pl, best)) != WL_OK)
        return rc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_cache_locked();
    TuneEntry te;
    te.c = best;
    te.us = best_ms * 1e3 / 10;
    te.fields = multi_fields(pl);
    g_tune[multi_key(pl)] = te;
    save_tune_cache_locked();
    return WL_OK;
}

int wl_multi_plan_get_launch(const wl_multi_plan *pl, int *block, int *rpt, int *variant, int *persistent,
                             int *grid)
{
    if (!pl || !block || !rpt || !variant || !persistent || !grid)
        return WL_EINVAL;
    *block = pl->cfg.block;
    *rpt = pl->cfg.rpt;
    *variant = pl->cfg.var;
    *persistent = pl->cfg.xcd;
    *grid = pl->grid > 0 ? pl->grid : (int)pl->total;
    return WL_OK;
}

int wl_multi_plan_set_launch(wl_multi_plan *pl, int block, int rpt, int variant, int persistent)
{
    if (!pl || (persistent != 0 && persistent != 1))
        return WL_EINVAL;
    return plan_build(pl, LaunchCfg{block, rpt, persistent, variant, 1});
}

int wl_multi_plan_destroy(wl_multi_plan *pl)
{
    if (!pl)
        return WL_EINVAL;
    plan_free(pl);
    return WL_OK;
}

int wilson_multi_apply(const wl_multi_desc *d, int n, int dagger, int nrhs, void *stream)
{
    wl_multi_plan *pl = nullptr;
    int rc = wl_multi_plan_create(d, n, dagger, nrhs, &pl);
    if (rc != WL_OK)
        return rc;
    rc = wl_multi_plan_run(pl, stream);
    // the plan's table must outlive the launch
    const hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    plan_free(pl);
    if (rc != WL_OK)
        return rc;
    CHECK_HIP(e);
    return WL_OK;
}

int wl_get_launch(const wl_op *op, int nrhs, wl_launch *cfg)
{
    if (!op || nrhs < 1 || !cfg)
        return WL_EINVAL;
    const LaunchCfg c = launch_for(op, op_cols(op, nrhs), RED_NONE, 0);
    cfg->block = c.block;
    cfg->rhs_per_thread = c.rpt;
    cfg->rhs_lanes = c.lanes;
    cfg->xcd_remap = c.xcd;
    cfg->variant = c.var;
    cfg->brick[0] = c.bx;
    cfg->brick[1] = c.by;
    cfg->brick[2] = c.bz;
    cfg->t_steps = c.tsteps;
    cfg->wg_per_cu = c.wpe;
    cfg->rhs_major = c.gmaj;
    return WL_OK;
}

int wl_set_launch(wl_op *op, int nrhs, const wl_launch *cfg)
{
    if (!op || nrhs < 1 || !cfg)
        return WL_EINVAL;
    nrhs = op_cols(op, nrhs);
    LaunchCfg c;
    c.block = cfg->block;
    c.rpt = cfg->rhs_per_thread;
    c.lanes = cfg->rhs_lanes;
    c.xcd = cfg->xcd_remap;
    c.var = cfg->variant;
    if (c.var == VAR_BRICK) {
        c.bx = cfg->brick[0];
        c.by = cfg->brick[1];
        c.bz = cfg->brick[2];
        c.tsteps = cfg->t_steps;
        c.wpe = cfg->wg_per_cu;
    } else if (cfg->wg_per_cu != 0) {
        return WL_EINVAL;
    }
    c.gmaj = cfg->rhs_major;
    if (!launch_ok(op, nrhs, c))
        return WL_EINVAL;
    std::lock_guard<std::mutex> lk(op->mu);
    for (int red = RED_NONE; red <= RED_LAST; ++red)  // every stencil of this nrhs
        for (int d = 0; d <= 1; ++d)
            op->launch[launch_key(nrhs, red, d)] = c;
    return WL_OK;
}

int wl_autotune(const wl_op *op, int nrhs, int dagger, void *stream)
{
    if (!op || nrhs < 1 || op_cols(op, nrhs) > 64 || (dagger != 0 && dagger != 1))
        return WL_EINVAL;
    nrhs = op_cols(op, nrhs);
    hipStream_t st = (hipStream_t)stream;
    const size_t vb = (size_t)nrhs * op->V * spinor_site_bytes(op->prec);
    void *in = nullptr, *out = nullptr;
    CHECK_HIP(hipMalloc(&in, vb));
    if (hipMalloc(&out, vb) != hipSuccess) {
        (void)hipFree(in);
        return WL_EHIP;
    }
    hipError_t e = hipMemsetAsync(in, 0, vb, st);
    hipEvent_t a = nullptr, b = nullptr;
    if (e == hipSuccess)
        e = hipEventCreate(&a);
    if (e == hipSuccess)
        e = hipEventCreate(&b);
    const int blocks[] = {64, 128, 256, 512};
    std::vector<LaunchCfg> cands;
    for (int bi = 0; bi < 4; ++bi)
        for (int rpt = 1; rpt <= max_rpt(op->prec); ++rpt)
            for (int lanes = 1; lanes <= 8; lanes *= 2)
                for (int xcd = 0; xcd <= 5; ++xcd)
                    for (int var = 0; var <= max_var(op->prec); ++var) {
                        const LaunchCfg c{blocks[bi], rpt, xcd, var, lanes};
                        if (var >= 4 && xcd >= 2)
                            continue;  // the t-walk orders only distinguish 0 and 1
                        if (var == VAR_BRICK)
                            continue;  // brick shapes below
                        if (launch_ok(op, nrhs, c))
                            cands.push_back(c);
                    }
    {
        std::vector<LaunchCfg> bc;
        brick_candidates(op, nrhs, bc);
        for (const LaunchCfg &c : bc)
            if (launch_ok(op, nrhs, c))
                cands.push_back(c);
    }
    // several right-hand-side groups: each shape also in group-major order
    for (size_t i = 0, n0 = cands.size(); i < n0; ++i)
        if (nrhs / (cands[i].rpt * cands[i].lanes) > 1) {
            LaunchCfg c = cands[i];
            c.gmaj = 1;
            cands.push_back(c);
        }
    // the plain apply, then each fused reduction of the solvers (partials
    // and the <v, out> operands in scratch)
    LaunchCfg bests[RED_LAST + 1];
    double best_us[RED_LAST + 1] = {};
    double *parts = nullptr, *sums = nullptr;
    if (e == hipSuccess)
        e = hipMalloc(&parts, RED_NVAL_MAX * sizeof(double) * (size_t)nrhs * ((op->V + 63) / 64 + op->g.dims[3] + 8));
    if (e == hipSuccess)
        e = hipMalloc(&sums, RED_NVAL_MAX * sizeof(double) * (size_t)nrhs);
    // time one shape for one reduction kind (ms per launch, or < 0 when the
    // shape cannot be launched for lack of resources)
    auto time_shape = [&](const LaunchCfg &c, int red, int reps) -> float {
        StencilParams p = base_params(op, out, in, nrhs, 1);
        p.red = red;
        p.partials = parts;
        p.aux = p.aux2 = p.aux3 = in;
        // a fused reduction is timed with the finalize that sums its
        // partials: fewer, larger workgroups leave it less to read
        FinParams fp{};
        fp.A = parts;
        fp.nblkA = stencil_partials(c, p.L, op->V, nrhs);
        fp.nvalA = stencil_nval(red);
        fp.out = sums;
        fp.nrhs = nrhs;
        fp.group = 1;
        auto step = [&]() {
            hipError_t r = launch_stencil(op->prec, dagger, c, p, st);
            if (r == hipSuccess && red != RED_NONE)
                r = launch_finalize(F_SUM, fp, st);
            return r;
        };
        for (int w = 0; w < 2 && e == hipSuccess; ++w)
            e = step();
        if (e == hipErrorInvalidValue || e == hipErrorInvalidConfiguration || e == hipErrorLaunchOutOfResources) {
            (void)hipGetLastError();  // a shape this kernel cannot be launched with: skip it
            e = hipSuccess;
            return -1.f;
        }
        if (e == hipSuccess)
            e = hipEventRecord(a, st);
        for (int k = 0; k < reps && e == hipSuccess; ++k)
            e = step();
        if (e == hipSuccess)
            e = hipEventRecord(b, st);
        if (e == hipSuccess)
            e = hipEventSynchronize(b);
        float ms = 0.f;
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms, a, b);
        return e == hipSuccess ? ms / reps : -1.f;
    };
    // a domain-wall operator has only the reductions of CG on the normal equations
    const int last_red = op->ns > 0 ? (int)RED_NORM : (int)RED_LAST;
    for (int red = RED_NONE; red <= RED_LAST && e == hipSuccess; ++red) {
        if (red > last_red) {
            bests[red] = bests[last_red];
            best_us[red] = best_us[last_red];
            continue;
        }
        // a short timing of every candidate, then the fastest few again with
        // four times the repetitions (the first pass's order is noisy where
        // shapes lie within a few per cent)
        std::vector<std::pair<float, size_t>> timed;
        for (size_t ci = 0; ci < cands.size() && e == hipSuccess; ++ci) {
            const float ms = time_shape(cands[ci], red, 10);
            if (ms >= 0.f)
                timed.emplace_back(ms, ci);
        }
        std::sort(timed.begin(), timed.end());
        float best_ms = INFINITY;
        LaunchCfg best = default_launch(op, nrhs);
        for (size_t j = 0; j < timed.size() && j < 6 && e == hipSuccess; ++j) {
            const float ms = time_shape(cands[timed[j].second], red, 40);
            if (ms >= 0.f && ms < best_ms) {
                best_ms = ms;
                best = cands[timed[j].second];
            }
        }
        // the fastest brick walk of the first pass again with its occupancy
        // capped (workgroups per CU, i.e. waves per SIMD), which trades latency
        // hiding for L2 reuse -- also when another variant won uncapped
        const LaunchCfg *brick0 = nullptr;
        for (size_t j = 0; j < timed.size() && !brick0; ++j)
            if (cands[timed[j].second].var == VAR_BRICK)
                brick0 = &cands[timed[j].second];
        if (brick0)
            for (int wpe = 1; wpe <= 8 && e == hipSuccess; wpe *= 2) {
                LaunchCfg c = *brick0;
                c.wpe = wpe;
                if (!launch_ok(op, nrhs, c))
                    continue;
                const float ms = time_shape(c, red, 40);
                if (ms >= 0.f && ms < best_ms) {
                    best_ms = ms;
                    best = c;
                }
            }
        bests[red] = best;
        best_us[red] = std::isfinite(best_ms) ? 1e3 * best_ms : 0.0;
    }
    if (a)
        (void)hipEventDestroy(a);
    if (b)
        (void)hipEventDestroy(b);
    if (parts)
        (void)hipFree(parts);
    if (sums)
        (void)hipFree(sums);
    (void)hipFree(in);
    (void)hipFree(out);
    CHECK_HIP(e);
    {
        wl_op *o = const_cast<wl_op *>(op);
        std::lock_guard<std::mutex> lk(o->mu);
        for (int red = RED_NONE; red <= RED_LAST; ++red)
            o->launch[launch_key(nrhs, red, dagger)] = bests[red];
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_cache_locked();
    for (int red = RED_NONE; red <= RED_LAST; ++red) {
        TuneEntry t;
        t.c = bests[red];
        t.us = best_us[red];
        t.fields = tune_fields(op, nrhs, dagger, red);
        g_tune[tune_key(op, nrhs, dagger, red)] = t;
    }
    save_tune_cache_locked();
    return WL_OK;
}

// ---------------------------------------------------------------- fused apply + inner products
static int dot_red(int kind)
{
    return kind == WL_DOT_BICG ? RED_BICG : kind == WL_DOT_V ? RED_DOTV : kind == WL_DOT_NORM ? RED_NORM : -1;
}

// Per-workgroup partials of any launch shape (the smallest tile has 64
// sites; t-walk and brick units are no more numerous) plus the sums.
static size_t apply_dot_bytes(const wl_op *op, int nrhs)
{
    const size_t nblk = (size_t)(op->V + 63) / 64 + (size_t)op->g.dims[3] + 8;
    return ((size_t)red_nval(RED_BICG) * nrhs * nblk * sizeof(double) + 255) / 256 * 256;  // the largest kind
}

int wl_apply_dot_workspace_bytes(const wl_op *op, int nrhs, size_t *out_bytes)
{
    if (!op || op->ns > 0 || nrhs < 1 || nrhs > 64 || !out_bytes)
        return WL_EINVAL;
    *out_bytes = apply_dot_bytes(op, nrhs);
    return WL_OK;
}

// The fused apply on `work` (partials, apply_dot_bytes of them); shared by
// wilson_apply_dot and its allocation-free variant.
int apply_dot_run(const wl_op *op, void *out, const void *in, const void *v, int dagger, int nrhs, int kind,
                  double *dots, double *work, hipStream_t st)
{
    const int red = dot_red(kind);
    StencilParams p = base_params(op, out, in, nrhs, 1);
    p.red = red;
    p.aux = v;
    p.partials = work;
    LaunchCfg cfg = launch_for(op, nrhs, red, dagger);
    FinParams fp{};
    fp.A = work;
    fp.nblkA = stencil_partials(cfg, p.L, op->V, nrhs);
    fp.nvalA = stencil_nval(red);
    fp.out = dots;
    fp.nrhs = nrhs;
    fp.group = 1;
    CHECK_HIP(prof_stencil(op->prec, op, dagger, cfg, p, st));
    CHECK_HIP(launch_finalize(F_SUM, fp, st));
    return WL_OK;
}

static int apply_dot_args(const wl_op *op, void *out, const void *in, const void *v, int dagger, int nrhs, int kind,
                          double *dots)
{
    if (!op || op->ns > 0 || !out || !in || !dots || out == in || nrhs < 1 || nrhs > 64 ||
        (dagger != 0 && dagger != 1) || dot_red(kind) < 0 || ((kind == WL_DOT_BICG || kind == WL_DOT_V) && !v) ||
        v == out)
        return WL_EINVAL;
    if (!al16(out) || !al16(in) || (v && !al16(v)) || ((uintptr_t)dots & 7u) != 0)
        return WL_EALIGN;
    return WL_OK;
}

int wilson_apply_dot(const wl_op *op, void *out, const void *in, const void *v, int dagger, int nrhs, int kind,
                     double *dots, void *workspace, size_t workspace_bytes, void *stream)
{
    int rc = apply_dot_args(op, out, in, v, dagger, nrhs, kind, dots);
    if (rc != WL_OK)
        return rc;
    if (!workspace || workspace_bytes < apply_dot_bytes(op, nrhs))
        return WL_EWORKSPACE;
    if (((uintptr_t)workspace & 255u) != 0)
        return WL_EALIGN;
    return apply_dot_run(op, out, in, v, dagger, nrhs, kind, dots, (double *)workspace, (hipStream_t)stream);
}

// ---------------------------------------------------------------- allocation-free fused apply
// The partial sums of wilson_apply_dot_noalloc live in this file-scope array
// (one copy per GPU, held until the process ends).  Host code never uses
// its name as an address: the device address comes from hipGetSymbolAddress,
// taken once per device with that device current.
static __device__ __align__(256) char scratch[WL_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
constexpr int SCRATCH_MAX_DEV = 64;
static void *g_scratch_ptr[SCRATCH_MAX_DEV] = {};

static int scratch_on_current_device(void **out)
{
    int dev = 0;
    CHECK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= SCRATCH_MAX_DEV)
        return WL_EINVAL;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        CHECK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return WL_OK;
}

int wilson_apply_dot_noalloc(const wl_op *op, void *out, const void *in, const void *v, int dagger, int nrhs,
                             int kind, double *dots, void *stream)
{
    int rc = apply_dot_args(op, out, in, v, dagger, nrhs, kind, dots);
    if (rc != WL_OK)
        return rc;
    if (apply_dot_bytes(op, nrhs) > WL_NOALLOC_SCRATCH_BYTES)
        return WL_EWORKSPACE;
    void *work = nullptr;
    if ((rc = scratch_on_current_device(&work)) != WL_OK)
        return rc;
    // every partial the finalize reads is written by the stencil first, so
    // the array needs no clearing between calls
    return apply_dot_run(op, out, in, v, dagger, nrhs, kind, dots, (double *)work, (hipStream_t)stream);
}

int wl_stream_copy(void *dst, const void *src, size_t bytes, void *stream)
{
    if (!dst || !src || bytes % 16 != 0)
        return WL_EINVAL;
    if (!al16(dst) || !al16(src))
        return WL_EALIGN;
    const char *d = (const char *)dst, *s = (const char *)src;
    if (d < s + bytes && s < d + bytes)
        return WL_EINVAL;  // overlapping ranges
    if (bytes == 0)
        return WL_OK;
    CHECK_HIP(launch_stream_copy(dst, src, bytes, (hipStream_t)stream));
    return WL_OK;
}

int wl_prof_enable(int on)
{
    g_prof_on.store(on ? 1 : 0);
    return WL_OK;
}

int wl_prof_reset(void)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    drain_prof_locked();
    for (int i = 0; i < 4; ++i) {
        g_prof_ms[i] = 0;
        g_prof_sites[i] = 0;
        g_prof_aux[i] = 0;
        g_prof_n[i] = 0;
    }
    return WL_OK;
}

int wl_prof_read(int prec, long *launches, double *total_ms, double *site_rhs)
{
    if (!prec_ok(prec) || !launches || !total_ms || !site_rhs)
        return WL_EINVAL;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    drain_prof_locked();
    *launches = g_prof_n[prec];
    *total_ms = g_prof_ms[prec];
    *site_rhs = g_prof_sites[prec];
    return WL_OK;
}

int wl_prof_read_aux(int prec, double *aux_site_rhs)
{
    if (!prec_ok(prec) || !aux_site_rhs)
        return WL_EINVAL;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    drain_prof_locked();
    *aux_site_rhs = g_prof_aux[prec];
    return WL_OK;
}

}  // extern "C"
