// Host runtime and C ABI of the restarted-PDHG optimal-transport library (include/pdot.h).
//
// A solve is a batch of one or more instances sharing one workspace.  The runtime lays out
// every instance's buffers, materialises stored costs, writes the device-resident control
// blocks, captures a HIP graph of `slots` iteration slots (each: one streaming-pass launch
// per kernel variant present in the batch, then one combine launch), and relaunches that
// graph until every instance reports idle.  All decisions of the method (Section 5 of
// the paper: restart candidate, restart conditions, step-size check, primal weight,
// termination) are taken on the device; the host only reads the mode words between
// graph launches and enforces the wall-clock limit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pdot.h"
#include "pdot_internal.h"

namespace pdot {
hipError_t launch_pass(int fp32, int vec, int cost, const Inst *insts, const Tile *tiles,
                       int ntiles, int grid, hipStream_t s);
hipError_t launch_combine(const Inst *insts, const CombEntry *ents, int nents, int grid,
                          hipStream_t s);
hipError_t launch_materialize(int fp32, void *dst, int64_t m, int64_t n, int64_t ld, int kind,
                              const double *src, int64_t ldc, const double *xs, const double *ys,
                              int dim, int side, double scale, hipStream_t s);
}  // namespace pdot

using namespace pdot;

namespace {

thread_local std::string g_err;

ot_status fail(ot_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(OT_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
constexpr int kMaxGrid = 4096;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Per-instance layout inside the workspace.
struct Layout {
    int64_t m = 0, n = 0, ld = 0, m_alloc = 0;
    int fp32 = 1, vec = 4, rows = 64, ncb = 0, nrb = 0, ntiles = 0, ncomb = 0;
    int cost = C_STORED, dim = 0, side = 0;
    bool stored = true;
    size_t es = 4;
    size_t off_X[4] = {0, 0, 0, 0}, off_C = 0, off_xs = 0, off_ys = 0, off_f = 0, off_g = 0;
    size_t off_rowv = 0, off_colv = 0, off_rowpart = 0, off_colpart = 0;
    size_t off_tiles = 0, off_comb = 0, off_counter = 0, off_ctl = 0;
    size_t bytes = 0;
};

bool finite_nonneg(const std::vector<double> &v)
{
    for (double x : v)
        if (!std::isfinite(x) || x < 0.0) return false;
    return true;
}

int default_vec(int64_t n)
{
    if (n >= 256) return 4;
    if (n >= 128) return 2;
    return 1;
}

int default_rows(int64_t m, int ncb)
{
    // aim for about four tiles per compute unit on large instances while keeping the column
    // partials (one row of n values per row block) small against the plan
    int64_t r = (m * ncb + 1023) / 1024;
    r = std::max<int64_t>(16, std::min<int64_t>(256, r));
    r = (r + 15) / 16 * 16;
    return (int)r;
}

ot_status plan_instance(const ot_problem &pb, const ot_params &prm, Layout &L)
{
    if (pb.m < 1 || pb.n < 1) return fail(OT_ERR_INVALID, "m and n must be >= 1");
    if (pb.m > (int64_t)1 << 31 || pb.n > (int64_t)1 << 31)
        return fail(OT_ERR_INVALID, "m or n too large");
    if (!pb.f || !pb.g) return fail(OT_ERR_INVALID, "f and g are required");
    L.m = pb.m;
    L.n = pb.n;
    L.fp32 = prm.precision == OT_PREC_FP32 ? 1 : 0;
    if (prm.precision != OT_PREC_FP32 && prm.precision != OT_PREC_FP64)
        return fail(OT_ERR_INVALID, "unknown precision");
    L.es = L.fp32 ? 4 : 8;
    L.ld = (pb.n + 63) / 64 * 64;
    L.m_alloc = (pb.m + 15) / 16 * 16;
    const ot_cost &c = pb.cost;
    switch (c.kind) {
    case OT_COST_DENSE:
        if (!c.C) return fail(OT_ERR_INVALID, "dense cost needs C");
        if (c.ldc < pb.n) return fail(OT_ERR_INVALID, "ldc < n");
        L.cost = C_STORED;
        L.stored = true;
        break;
    case OT_COST_POINTS_SQEUCLID:
    case OT_COST_POINTS_EUCLID:
        if (!c.x || !c.y) return fail(OT_ERR_INVALID, "points cost needs x and y");
        if (c.dim < 1 || c.dim > 3) return fail(OT_ERR_INVALID, "dim must be 1..3");
        L.dim = c.dim;
        L.stored = c.store != 0;
        L.cost = L.stored ? C_STORED : (c.kind == OT_COST_POINTS_SQEUCLID ? C_PTS_SQ : C_PTS_EU);
        break;
    case OT_COST_GRID_SQEUCLID:
        if (c.side < 1 || (int64_t)c.side * c.side != pb.m || pb.m != pb.n)
            return fail(OT_ERR_INVALID, "grid cost needs m = n = side^2");
        if (!std::isfinite(c.scale)) return fail(OT_ERR_INVALID, "grid scale not finite");
        L.side = c.side;
        L.stored = c.store != 0;
        L.cost = L.stored ? C_STORED : C_GRID_SQ;
        break;
    default:
        return fail(OT_ERR_INVALID, "unknown cost kind");
    }
    L.vec = prm.tile_vec ? prm.tile_vec : default_vec(pb.n);
    if (L.vec != 1 && L.vec != 2 && L.vec != 4) return fail(OT_ERR_INVALID, "tile_vec must be 1, 2 or 4");
    L.ncb = (int)((pb.n + 64 * L.vec - 1) / (64 * L.vec));
    L.rows = prm.tile_rows ? prm.tile_rows : default_rows(pb.m, L.ncb);
    if (L.rows < 16 || L.rows % 16) return fail(OT_ERR_INVALID, "tile_rows must be a positive multiple of 16");
    L.nrb = (int)((pb.m + L.rows - 1) / L.rows);
    const int64_t nt = (int64_t)L.ncb * L.nrb;
    if (nt > (1 << 30)) return fail(OT_ERR_INVALID, "too many tiles");
    L.ntiles = (int)nt;
    L.ncomb = (int)((pb.m + kCombEntries - 1) / kCombEntries + (pb.n + kCombEntries - 1) / kCombEntries);

    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    const size_t mat = (size_t)L.m_alloc * (size_t)L.ld * L.es;
    for (int b = 0; b < 4; ++b) L.off_X[b] = take(mat);
    L.off_C = L.stored ? take(mat) : 0;
    L.off_xs = L.dim ? take(sizeof(double) * (size_t)L.m * L.dim) : 0;
    L.off_ys = L.dim ? take(sizeof(double) * (size_t)L.n * L.dim) : 0;
    L.off_f = take(sizeof(double) * (size_t)L.m);
    L.off_g = take(sizeof(double) * (size_t)L.n);
    L.off_rowv = take(sizeof(double) * (size_t)L.m * 10);   // p[2] pb[2] pa rs[2] rsb (+2 spare)
    L.off_colv = take(sizeof(double) * (size_t)L.n * 10);
    L.off_rowpart = take(sizeof(double) * (size_t)L.ncb * (size_t)L.m);
    L.off_colpart = take(sizeof(double) * (size_t)L.nrb * (size_t)L.n);
    L.off_tiles = take(sizeof(double) * (size_t)L.ntiles * kNS);
    L.off_comb = take(sizeof(double) * (size_t)L.ncomb * kNC);
    L.off_counter = take(sizeof(uint32_t) * 4);
    L.off_ctl = take(sizeof(Ctl));
    L.bytes = off;
    return OT_OK;
}

Prm device_params(const ot_params &p, double tol)
{
    Prm d;
    memset(&d, 0, sizeof(d));
    d.tol = tol;
    d.max_iters = p.max_iters;
    d.max_passes = p.max_passes;
    d.kkt_mode = p.kkt_mode;
    d.step_rule = p.step_rule;
    d.restart_rule = p.restart_rule;
    d.avg_weighting = p.avg_weighting;
    d.pwu = p.primal_weight_update;
    d.output = p.output;
    d.beta_suff = p.beta_sufficient;
    d.beta_nec = p.beta_necessary;
    d.beta_art = p.beta_artificial;
    d.beta_basic = p.beta_basic;
    d.theta = p.theta;
    d.eps_zero = p.eps_zero;
    d.red_exp = p.step_reduction_exp;
    d.grow_exp = p.step_growth_exp;
    return d;
}

bool is_device_ptr(const void *p)
{
    if (!p) return false;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

// Copy n doubles from a host or device pointer to host memory.
ot_status fetch_host(const double *src, size_t count, std::vector<double> &out, hipStream_t s)
{
    out.resize(count);
    if (count == 0) return OT_OK;
    if (is_device_ptr(src)) {
        HIP_TRY(hipMemcpyAsync(out.data(), src, count * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    } else {
        memcpy(out.data(), src, count * sizeof(double));
    }
    return OT_OK;
}

struct Batch {
    std::vector<Layout> L;
    std::vector<size_t> base;   // workspace offset of every instance
    size_t inst_tab = 0, tile_tab = 0, comb_tab = 0, total = 0;
    int ntiles_total = 0, ncomb_total = 0;
    struct Group { int fp32, vec, cost, first, count; };
    std::vector<Group> groups;
    std::vector<Tile> tiles;
    std::vector<CombEntry> combs;
};

ot_status plan_batch(const ot_problem *probs, int count, const ot_params &prm, Batch &B)
{
    B.L.resize(count);
    B.base.resize(count);
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
        ot_status st = plan_instance(probs[i], prm, B.L[i]);
        if (st != OT_OK) return fail(st, "instance " + std::to_string(i) + ": " + g_err);
        B.base[i] = off;
        off = align_up(off + B.L[i].bytes);
    }
    // tiles grouped by kernel variant; every tile knows its instance and local index
    struct Key { int fp32, vec, cost; };
    std::vector<Key> keys;
    for (int i = 0; i < count; ++i) {
        Key k{B.L[i].fp32, B.L[i].vec, B.L[i].cost};
        bool seen = false;
        for (auto &q : keys) seen |= (q.fp32 == k.fp32 && q.vec == k.vec && q.cost == k.cost);
        if (!seen) keys.push_back(k);
    }
    for (auto &k : keys) {
        Batch::Group g{k.fp32, k.vec, k.cost, (int)B.tiles.size(), 0};
        for (int i = 0; i < count; ++i) {
            const Layout &l = B.L[i];
            if (l.fp32 != k.fp32 || l.vec != k.vec || l.cost != k.cost) continue;
            for (int rb = 0; rb < l.nrb; ++rb)
                for (int cb = 0; cb < l.ncb; ++cb)
                    B.tiles.push_back(Tile{i, rb, cb, rb * l.ncb + cb});
        }
        g.count = (int)B.tiles.size() - g.first;
        B.groups.push_back(g);
    }
    for (int i = 0; i < count; ++i) {
        const Layout &l = B.L[i];
        int local = 0;
        for (int64_t r = 0; r < l.m; r += kCombEntries) B.combs.push_back(CombEntry{i, 0, (int)r, local++});
        for (int64_t c = 0; c < l.n; c += kCombEntries) B.combs.push_back(CombEntry{i, 1, (int)c, local++});
    }
    B.ntiles_total = (int)B.tiles.size();
    B.ncomb_total = (int)B.combs.size();
    B.inst_tab = off;
    off = align_up(off + sizeof(Inst) * (size_t)count);
    B.tile_tab = off;
    off = align_up(off + sizeof(Tile) * B.tiles.size());
    B.comb_tab = off;
    off = align_up(off + sizeof(CombEntry) * B.combs.size());
    B.total = off;
    return OT_OK;
}

int auto_slots(const Batch &B)
{
    // about 2 ms of streaming per graph launch at roughly 5 TB/s, 16..512 slots
    double bytes = 0.0;
    for (auto &l : B.L) bytes += (double)l.m * (double)l.ld * (double)l.es * 5.0;
    const double t_pass = bytes / 5e12 + 6e-6;
    int s = (int)(2e-3 / t_pass);
    return std::max(16, std::min(512, s));
}

ot_status run_batch(const ot_problem *probs, int count, const ot_params &prm, ot_result *res,
                    void *workspace, size_t ws_bytes, hipStream_t user_stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (count < 1 || !probs) return fail(OT_ERR_INVALID, "no problems");
    if (!(prm.tol > 0.0)) return fail(OT_ERR_INVALID, "tol must be > 0");
    if (prm.max_iters < 0 || prm.max_passes < 0) return fail(OT_ERR_INVALID, "negative limits");
    Batch B;
    ot_status st = plan_batch(probs, count, prm, B);
    if (st != OT_OK) return st;

    hipStream_t s = user_stream;
    bool own_stream = false;
    if (!s) {
        HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        own_stream = true;
    }
    struct Cleanup {
        hipStream_t s = nullptr;
        bool own = false;
        void *ws = nullptr;
        std::vector<void *> tmp;
        void *pinned = nullptr;
        std::vector<hipEvent_t> events;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        ~Cleanup()
        {
            if (s) (void)hipStreamSynchronize(s);
            if (exec) (void)hipGraphExecDestroy(exec);
            if (graph) (void)hipGraphDestroy(graph);
            for (void *p : tmp) (void)hipFree(p);
            if (ws) (void)hipFree(ws);
            if (pinned) (void)hipHostFree(pinned);
            for (auto e : events) (void)hipEventDestroy(e);
            if (own && s) (void)hipStreamDestroy(s);
        }
    } cl;
    cl.s = s;
    cl.own = own_stream;

    // host-side validation of the marginals (paper: f, g probability vectors, eq. ot)
    std::vector<std::vector<double>> fh(count), gh(count);
    std::vector<double> tols(count);
    for (int i = 0; i < count; ++i) {
        st = fetch_host(probs[i].f, (size_t)probs[i].m, fh[i], s);
        if (st != OT_OK) return st;
        st = fetch_host(probs[i].g, (size_t)probs[i].n, gh[i], s);
        if (st != OT_OK) return st;
        if (!finite_nonneg(fh[i]) || !finite_nonneg(gh[i]))
            return fail(OT_ERR_INVALID, "instance " + std::to_string(i) + ": f and g must be finite and >= 0");
        double sf = 0.0, sg = 0.0;
        for (double v : fh[i]) sf += v;
        for (double v : gh[i]) sg += v;
        if (!(std::fabs(sf - sg) <= 1e-12 * std::max(sf, sg)))
            return fail(OT_ERR_INVALID, "instance " + std::to_string(i) + ": sum f != sum g");
        tols[i] = probs[i].tol > 0.0 ? probs[i].tol : prm.tol;
    }

    char *ws = (char *)workspace;
    if (ws) {
        if (ws_bytes < B.total) return fail(OT_ERR_OOM, "workspace too small");
        if ((uintptr_t)ws % kAlign) return fail(OT_ERR_INVALID, "workspace must be 256-byte aligned");
    } else {
        void *p = nullptr;
        if (hipMalloc(&p, B.total) != hipSuccess) {
            (void)hipGetLastError();
            return fail(OT_ERR_OOM, "hipMalloc of " + std::to_string(B.total) + " bytes failed");
        }
        cl.ws = p;
        ws = (char *)p;
    }
    HIP_TRY(hipMemsetAsync(ws, 0, B.total, s));

    std::vector<Inst> insts(count);
    for (int i = 0; i < count; ++i) {
        const Layout &l = B.L[i];
        const ot_problem &pb = probs[i];
        char *b = ws + B.base[i];
        Inst &I = insts[i];
        memset(&I, 0, sizeof(I));
        I.m = l.m;
        I.n = l.n;
        I.ld = l.ld;
        I.m_alloc = l.m_alloc;
        I.cost = l.cost;
        I.dim = l.dim;
        I.side = l.side;
        I.vec = l.vec;
        I.rows = l.rows;
        I.ncb = l.ncb;
        I.nrb = l.nrb;
        I.ntiles = l.ntiles;
        I.ncomb = l.ncomb;
        I.scale = pb.cost.scale;
        for (int k = 0; k < 4; ++k) I.X[k] = b + l.off_X[k];
        I.C = l.stored ? (const void *)(b + l.off_C) : nullptr;
        I.xs = l.dim ? (const double *)(b + l.off_xs) : nullptr;
        I.ys = l.dim ? (const double *)(b + l.off_ys) : nullptr;
        I.f = (const double *)(b + l.off_f);
        I.g = (const double *)(b + l.off_g);
        double *rv = (double *)(b + l.off_rowv);
        double *cv = (double *)(b + l.off_colv);
        const int64_t m = l.m, n = l.n;
        I.p[0] = rv + 0 * m; I.p[1] = rv + 1 * m; I.pb[0] = rv + 2 * m; I.pb[1] = rv + 3 * m;
        I.pa = rv + 4 * m; I.rs[0] = rv + 5 * m; I.rs[1] = rv + 6 * m; I.rsb = rv + 7 * m;
        I.q[0] = cv + 0 * n; I.q[1] = cv + 1 * n; I.qb[0] = cv + 2 * n; I.qb[1] = cv + 3 * n;
        I.qa = cv + 4 * n; I.cs[0] = cv + 5 * n; I.cs[1] = cv + 6 * n; I.csb = cv + 7 * n;
        I.rowpart = (double *)(b + l.off_rowpart);
        I.colpart = (double *)(b + l.off_colpart);
        I.tilescal = (double *)(b + l.off_tiles);
        I.combscal = (double *)(b + l.off_comb);
        I.counter = (uint32_t *)(b + l.off_counter);
        I.ctl = (Ctl *)(b + l.off_ctl);
        I.prm = device_params(prm, tols[i]);

        HIP_TRY(hipMemcpyAsync((void *)I.f, fh[i].data(), sizeof(double) * m, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync((void *)I.g, gh[i].data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
        if (l.dim) {
            HIP_TRY(hipMemcpyAsync((void *)I.xs, pb.cost.x, sizeof(double) * m * l.dim, hipMemcpyDefault, s));
            HIP_TRY(hipMemcpyAsync((void *)I.ys, pb.cost.y, sizeof(double) * n * l.dim, hipMemcpyDefault, s));
        }
        if (l.stored) {
            int kind = C_STORED;
            const double *src = nullptr;
            int64_t ldc = 0;
            if (pb.cost.kind == OT_COST_DENSE) {
                ldc = pb.cost.ldc;
                if (is_device_ptr(pb.cost.C)) {
                    src = pb.cost.C;
                } else {
                    void *tmp = nullptr;
                    const size_t bytes = sizeof(double) * (size_t)((m - 1) * ldc + n);
                    if (hipMalloc(&tmp, bytes) != hipSuccess) {
                        (void)hipGetLastError();
                        return fail(OT_ERR_OOM, "staging allocation for C failed");
                    }
                    cl.tmp.push_back(tmp);
                    HIP_TRY(hipMemcpyAsync(tmp, pb.cost.C, bytes, hipMemcpyHostToDevice, s));
                    src = (const double *)tmp;
                }
            } else if (pb.cost.kind == OT_COST_GRID_SQEUCLID) {
                kind = C_GRID_SQ;
            } else {
                kind = pb.cost.kind == OT_COST_POINTS_SQEUCLID ? C_PTS_SQ : C_PTS_EU;
            }
            HIP_TRY(launch_materialize(l.fp32, (void *)I.C, m, n, l.ld, kind, src, ldc, I.xs, I.ys,
                                       l.dim, l.side, pb.cost.scale, s));
        }
        Ctl c;
        memset(&c, 0, sizeof(c));
        c.mode = M_INIT;
        c.status = -1;
        for (int k = 0; k < 4; ++k) c.xr[k] = k;
        c.eta = prm.eta0 > 0.0 ? prm.eta0 : 1.0 / std::sqrt((double)(m + n));
        c.omega = prm.omega0 > 0.0 ? prm.omega0 : 1.0;
        c.tol_eff = tols[i];
        HIP_TRY(hipMemcpyAsync(I.ctl, &c, sizeof(Ctl), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));   // host staging buffers above are on the stack
    }
    const Inst *d_insts = (const Inst *)(ws + B.inst_tab);
    const Tile *d_tiles = (const Tile *)(ws + B.tile_tab);
    const CombEntry *d_combs = (const CombEntry *)(ws + B.comb_tab);
    HIP_TRY(hipMemcpyAsync((void *)d_insts, insts.data(), sizeof(Inst) * count, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync((void *)d_tiles, B.tiles.data(), sizeof(Tile) * B.tiles.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync((void *)d_combs, B.combs.data(), sizeof(CombEntry) * B.combs.size(), hipMemcpyHostToDevice, s));

    // one graph of `slots` iteration slots
    const int slots = prm.graph_slots > 0 ? prm.graph_slots : auto_slots(B);
    const int comb_grid = std::min(B.ncomb_total, kMaxGrid);
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (int sl = 0; sl < slots; ++sl) {
        for (auto &g : B.groups) {
            const int grid = std::min(g.count, kMaxGrid);
            hipError_t e = launch_pass(g.fp32, g.vec, g.cost, d_insts, d_tiles + g.first, g.count, grid, s);
            if (e != hipSuccess) {
                hipGraph_t junk = nullptr;
                (void)hipStreamEndCapture(s, &junk);
                if (junk) (void)hipGraphDestroy(junk);
                return fail(OT_ERR_DEVICE, std::string("pass launch: ") + hipGetErrorString(e));
            }
        }
        hipError_t e = launch_combine(d_insts, d_combs, B.ncomb_total, comb_grid, s);
        if (e != hipSuccess) {
            hipGraph_t junk = nullptr;
            (void)hipStreamEndCapture(s, &junk);
            if (junk) (void)hipGraphDestroy(junk);
            return fail(OT_ERR_DEVICE, std::string("combine launch: ") + hipGetErrorString(e));
        }
    }
    HIP_TRY(hipStreamEndCapture(s, &cl.graph));
    HIP_TRY(hipGraphInstantiate(&cl.exec, cl.graph, nullptr, nullptr, 0));

    HIP_TRY(hipHostMalloc(&cl.pinned, sizeof(Ctl) * count, hipHostMallocDefault));
    Ctl *hc = (Ctl *)cl.pinned;
    for (int i = 0; i < count; ++i) hc[i].mode = M_INIT;
    // every slot either evaluates a step trial, restarts, or finishes; bound the launches
    const int64_t max_slots = 3 * std::max<int64_t>(prm.max_passes, 1) + 16;
    int64_t launched = 0;
    bool stop_sent = false;
    std::vector<double> pass_ms(count, 0.0), comb_ms(count, 0.0);
    std::vector<hipEvent_t> ev;
    if (prm.profile) {
        ev.resize(3);
        for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
        cl.events = ev;
    }
    while (true) {
        if (prm.profile) {
            // one slot at a time, pass and combine launches bracketed by events
            HIP_TRY(hipEventRecord(ev[0], s));
            for (auto &g : B.groups)
                HIP_TRY(launch_pass(g.fp32, g.vec, g.cost, d_insts, d_tiles + g.first, g.count,
                                    std::min(g.count, kMaxGrid), s));
            HIP_TRY(hipEventRecord(ev[1], s));
            HIP_TRY(launch_combine(d_insts, d_combs, B.ncomb_total, comb_grid, s));
            HIP_TRY(hipEventRecord(ev[2], s));
            launched += 1;
            HIP_TRY(hipEventSynchronize(ev[2]));
            float a = 0.f, b = 0.f;
            HIP_TRY(hipEventElapsedTime(&a, ev[0], ev[1]));
            HIP_TRY(hipEventElapsedTime(&b, ev[1], ev[2]));
            // attribute to every instance still running (single instance in practice)
            for (int i = 0; i < count; ++i)
                if (hc[i].mode != M_IDLE) {
                    pass_ms[i] += a;
                    comb_ms[i] += b;
                }
        } else {
            HIP_TRY(hipGraphLaunch(cl.exec, s));
            launched += slots;
        }
        for (int i = 0; i < count; ++i)
            HIP_TRY(hipMemcpyAsync(hc + i, insts[i].ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        bool running = false;
        for (int i = 0; i < count; ++i) running |= hc[i].mode != M_IDLE;
        if (!running) break;
        if (launched > max_slots) return fail(OT_ERR_DEVICE, "solver did not reach a final state");
        if (!stop_sent && prm.time_limit_s > 0.0) {
            const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (el >= prm.time_limit_s) {
                const int32_t one = 1;
                for (int i = 0; i < count; ++i)
                    HIP_TRY(hipMemcpyAsync((char *)insts[i].ctl + offsetof(Ctl, stop), &one, sizeof(one),
                                           hipMemcpyHostToDevice, s));
                HIP_TRY(hipStreamSynchronize(s));
                stop_sent = true;
            }
        }
    }

    // outputs
    ot_status first_bad = OT_OK;
    for (int i = 0; i < count; ++i) {
        const Layout &l = B.L[i];
        const ot_problem &pb = probs[i];
        const Ctl &c = hc[i];
        const Inst &I = insts[i];
        const ot_status ist = c.status < 0 ? OT_ERR_DEVICE : (ot_status)c.status;
        if (ist != OT_OK && first_bad == OT_OK) first_bad = ist;
        if (ist == OT_OK || ist == OT_NOT_CONVERGED) {
            if (pb.X_out)
                HIP_TRY(hipMemcpy2DAsync(pb.X_out, l.n * l.es, I.X[c.ret_x], l.ld * l.es, l.n * l.es,
                                         l.m, hipMemcpyDefault, s));
            const double *pr = c.ret_avg ? I.pb[c.pbv] : I.p[c.pv];
            const double *qr = c.ret_avg ? I.qb[c.pbv] : I.q[c.pv];
            if (pb.u_out) HIP_TRY(hipMemcpyAsync(pb.u_out, pr, sizeof(double) * l.m, hipMemcpyDefault, s));
            if (pb.v_out) HIP_TRY(hipMemcpyAsync(pb.v_out, qr, sizeof(double) * l.n, hipMemcpyDefault, s));
        }
        if (res) {
            ot_result &r = res[i];
            memset(&r, 0, sizeof(r));
            r.status = ist;
            r.returned_average = c.ret_avg;
            r.iterations = c.T;
            r.passes = c.passes;
            r.restarts = c.restarts;
            r.kernel_passes = c.kpasses;
            r.objective = c.r_obj;
            r.dual_objective = c.r_dobj;
            r.rel_primal = c.r_relP;
            r.rel_dual = c.r_relD;
            r.rel_gap = c.r_relG;
            r.rel_kkt = c.r_kkt;
            r.eta = c.eta;
            r.omega = c.omega;
            // algorithmic bytes per element of each pass kind (plan element size b, cost
            // element size bc, 0 when regenerated): start-point KKT reads C; a trial reads
            // X and C and writes X+; the full pass also reads and writes the average; the
            // restart pass reads two plans; verification reads X and C
            const double b = (double)l.es, bc = l.stored ? (double)l.es : 0.0;
            const double per[6] = {0.0, bc, 2 * b + bc, 4 * b + bc, 2 * b, b + bc};
            const double elems = (double)l.m * (double)l.n;
            double bytes = 0.0;
            for (int k = 0; k < 6; ++k) {
                r.mode_passes[k] = c.mcount[k];
                bytes += per[k] * elems * (double)c.mcount[k];
            }
            r.pass_bytes = bytes;
            r.pass_ms = pass_ms[i];
            r.combine_ms = comb_ms[i];
        }
    }
    HIP_TRY(hipStreamSynchronize(s));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (res)
        for (int i = 0; i < count; ++i) res[i].seconds = secs;
    if (first_bad != OT_OK) {
        g_err = first_bad == OT_NOT_CONVERGED ? "iteration, pass or time limit reached"
                                               : "numerical failure (NaN/Inf in KKT or step scalars)";
    } else {
        g_err.clear();
    }
    return first_bad;
}

}  // namespace

extern "C" {

void ot_params_default(ot_params *p)
{
    if (!p) return;
    memset(p, 0, sizeof(*p));
    p->tol = 1e-4;
    p->max_iters = 1000000;
    p->max_passes = 4000000;
    p->time_limit_s = 3600.0;
    p->precision = OT_PREC_FP32;
    p->kkt_mode = 0;
    p->step_rule = 0;
    p->restart_rule = 0;
    p->avg_weighting = 0;
    p->primal_weight_update = 1;
    p->output = 0;
    p->graph_slots = 0;
    p->beta_sufficient = 0.1;
    p->beta_necessary = 0.9;
    p->beta_artificial = 0.36;
    p->beta_basic = 0.2;
    p->theta = 0.5;
    p->omega0 = 1.0;
    p->eta0 = 0.0;
    p->eps_zero = 1e-10;
    p->step_reduction_exp = 0.3;
    p->step_growth_exp = 0.6;
    p->tile_vec = 0;
    p->tile_rows = 0;
}

size_t ot_workspace_size(const ot_problem *prob, const ot_params *prm)
{
    if (!prob || !prm) {
        fail(OT_ERR_INVALID, "null argument");
        return 0;
    }
    Batch B;
    if (plan_batch(prob, 1, *prm, B) != OT_OK) return 0;
    return B.total;
}

ot_status ot_solve(const ot_problem *prob, const ot_params *prm, ot_result *res, void *workspace,
                   size_t workspace_bytes, void *stream)
{
    if (!prob || !prm) return fail(OT_ERR_INVALID, "null argument");
    return run_batch(prob, 1, *prm, res, workspace, workspace_bytes, (hipStream_t)stream);
}

ot_status ot_solve_batch(const ot_problem *probs, int32_t count, const ot_params *prm,
                         ot_result *res, void *stream)
{
    if (!probs || !prm || count < 1) return fail(OT_ERR_INVALID, "null argument or empty batch");
    return run_batch(probs, count, *prm, res, nullptr, 0, (hipStream_t)stream);
}

const char *ot_last_error(void) { return g_err.c_str(); }

const char *ot_version(void) { return "pdot-mi355x 0.1"; }

}  // extern "C"
