// Host runtime and C ABI of the restarted-PDHG optimal-transport library (include/pdot.h).
//
// Everything runs through one Engine: a device arena holding every admitted instance's
// buffers and the engine tables, a set of running instances, and a HIP graph of `slots`
// iteration slots.  A slot is one streaming-pass launch per kernel variant (precision,
// columns per lane, cost source) present among the running instances, then one combine
// launch.  The tables (instance descriptors, tiles grouped by variant, combine entries)
// live in device memory and their lengths are read by the kernels from device memory, so
// the host can repack them between graph launches (instances finishing, or joining in the
// server) without touching the graph; it is captured again only when the variant layout
// of the tile table changes.  All decisions of the method (Section 5 of the paper:
// restart candidate, restart conditions, step-size check, primal weight, termination)
// are taken on the device; the host reads the mode words between graph launches,
// retires finished instances and enforces wall-clock limits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "pdot.h"
#include "pdot_host.h"
#include "pdot_internal.h"

using namespace pdot;

static_assert(sizeof(ot_trace_rec) == sizeof(TraceRec), "trace record layout");
static_assert((int)OT_COST_GRID_SQEUCLID == (int)C_GRID_SQ && (int)OT_COST_GRID_L1 == (int)C_GRID_L1 &&
                  (int)OT_COST_GRID_L2 == (int)C_GRID_L2 && (int)OT_COST_GRID_LINF == (int)C_GRID_LINF,
              "grid cost kinds share their numbering with the kernels");

namespace pdot {

// The calling thread's message for ot_last_error: a fixed buffer, so that setting it
// allocates nothing (the no-allocation entry point sets it too).
struct ErrMsg {
    char buf[1024] = {0};
    ErrMsg &operator=(const char *s)
    {
        snprintf(buf, sizeof buf, "%s", s);
        return *this;
    }
    ErrMsg &operator=(const std::string &s) { return *this = s.c_str(); }
    void clear() { buf[0] = 0; }
    bool empty() const { return buf[0] == 0; }
    const char *c_str() const { return buf; }
};
thread_local ErrMsg g_err;

ot_status fail(ot_status st, const char *msg)
{
    g_err = msg;
    return st;
}

ot_status fail(ot_status st, const std::string &msg) { return fail(st, msg.c_str()); }

// ------------------------------------------------------------------ per-instance layout



int lane_of(int64_t elems)
{
    int l = 0;
    while (l < kLanes - 1 && elems > kLaneMax[l]) ++l;
    return l;
}

// The widest lane (more bytes per load) whose tiles of 16 rows still number about four per
// compute unit (1024); narrower lanes fill the GPU on mid-size instances (the autotuner
// picks 1 column per lane for 1024 x 1024 grids and 4 for 4096 x 4096 with FP32 plans).
// FP64 plans take at most 2 columns per lane: 4 doubles per lane and stream cost more
// registers than they save (at 4096 x 4096, 91 us per pass with 2 columns and 64 rows
// against 99 us with 4 and 64).
int default_vec(int64_t m, int64_t n, bool fp32)
{
    const int64_t rb = (m + 15) / 16;
    for (int v = fp32 ? 4 : 2; v >= 2; v /= 2)
        if (n >= 64 * v && rb * ((n + 64 * v - 1) / (64 * v)) >= 1024) return v;
    return 1;
}

int default_rows(int64_t m, int ncb, bool fp32, int vec, bool points)
{
    // aim for about four tiles per compute unit on large instances (eight with FP64 plans,
    // whose lanes are narrower) while keeping the column partials (one row of n values per
    // row block) small against the plan.  The 4-column FP32 kernel of the grid and stored
    // costs runs three work-groups per compute unit (165 VGPRs), so it aims for one full
    // round of them (768 tiles): at 4096 x 4096, 96-row tiles (688) instead of 64-row ones
    // (1024, 1.33 rounds) took 47.7 against 51.2 us per pass and 4.4 % less time to 1e-6
    // over 25 images (seeds 200-224; iteration counts equal within 3 %).
    const int64_t target = !fp32 ? 2048 : (vec == 4 && !points ? 768 : 1024);
    int64_t r = (m * ncb + target - 1) / target;
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
    case OT_COST_GRID_L1:
    case OT_COST_GRID_L2:
    case OT_COST_GRID_LINF:
        if (c.side < 1 || (int64_t)c.side * c.side != pb.m || pb.m != pb.n)
            return fail(OT_ERR_INVALID, "grid cost needs m = n = side^2");
        if (!std::isfinite(c.scale)) return fail(OT_ERR_INVALID, "grid scale not finite");
        L.side = c.side;
        L.stored = c.store != 0;
        // the ABI's grid kinds and the kernels' cost kinds share their numbering
        L.cost = L.stored ? C_STORED : (int)c.kind;
        break;
    default:
        return fail(OT_ERR_INVALID, "unknown cost kind");
    }
    if (prm.engine < 0 || prm.engine > 2) return fail(OT_ERR_INVALID, "engine must be 0, 1 or 2");
    const int64_t elems = pb.m * pb.n;
    L.resident = (prm.engine == 0 && elems <= OT_RESIDENT_MAX_ELEMS) ||
                 (prm.engine == 2 && elems <= OT_RESIDENT_HARD_MAX_ELEMS);
    L.vec = pb.tile_vec > 0 ? pb.tile_vec : (prm.tile_vec ? prm.tile_vec : default_vec(pb.m, pb.n, L.fp32));
    if (L.vec != 1 && L.vec != 2 && L.vec != 4) return fail(OT_ERR_INVALID, "tile_vec must be 1, 2 or 4");
    // the resident kernel has no 4-column variant (it would spill registers)
    if (L.resident && L.vec == 4) L.vec = 2;
    L.ncb = (int)((pb.n + 64 * L.vec - 1) / (64 * L.vec));
    L.rows = pb.tile_rows > 0 ? pb.tile_rows : (prm.tile_rows ? prm.tile_rows : default_rows(pb.m, L.ncb, L.fp32, L.vec, L.cost == C_PTS_SQ || L.cost == C_PTS_EU));
    if (L.rows < 16 || L.rows % 16) return fail(OT_ERR_INVALID, "tile_rows must be a positive multiple of 16");
    // a resident instance is one row block: its work-group streams every row of a band
    if (L.resident) L.rows = (int)L.m_alloc;
    L.lane = lane_of(elems);
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
    for (int b = 0; b < kBufs; ++b) L.off_X[b] = take(mat);
    L.off_C = L.stored ? take(mat) : 0;
    L.off_xs = L.dim ? take(sizeof(double) * (size_t)L.m * L.dim) : 0;
    L.off_ys = L.dim ? take(sizeof(double) * (size_t)L.n * L.dim) : 0;
    L.off_f = take(sizeof(double) * (size_t)L.m);
    L.off_g = take(sizeof(double) * (size_t)L.n);
    L.off_rowv = take(sizeof(double) * (size_t)L.m * 8);   // p[2] pb[2] pa rs[2] rsb
    L.off_colv = take(sizeof(double) * (size_t)L.n * 8);
    L.off_rowpart = take(sizeof(double) * (size_t)L.ncb * (size_t)L.m);
    L.off_colpart = take(sizeof(double) * (size_t)L.nrb * (size_t)L.n);
    L.off_tiles = take(sizeof(double) * (size_t)L.ntiles * kNS);
    L.off_comb = take(sizeof(double) * (size_t)L.ncomb * kNB * 2);   // two record sets
    L.off_counter = take(sizeof(uint32_t) * 4);
    L.off_ctl = take(sizeof(Ctl));
    if (pb.trace_cap < 0) return fail(OT_ERR_INVALID, "trace_cap < 0");
    L.trace_cap = pb.trace ? pb.trace_cap : 0;
    L.off_trace = L.trace_cap ? take(sizeof(TraceRec) * (size_t)L.trace_cap) : 0;
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
    d.verify_retries = p.verify_retries;
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

ot_status check_params(const ot_params &prm)
{
    if (!(prm.tol > 0.0)) return fail(OT_ERR_INVALID, "tol must be > 0");
    if (prm.max_iters < 0 || prm.max_passes < 0 || prm.verify_retries < 0)
        return fail(OT_ERR_INVALID, "negative limits");
    return OT_OK;
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



void init_inst(const Layout &l, char *b, double scale, const ot_params &prm, double tol, Inst &I)
{
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
    I.scale = scale;
    for (int k = 0; k < kBufs; ++k) I.X[k] = b + l.off_X[k];
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
    I.trace = l.trace_cap ? (TraceRec *)(b + l.off_trace) : nullptr;
    I.trace_cap = l.trace_cap;
    I.prm = device_params(prm, tol);
}

int64_t plan_bytes(const Layout &l)
{
    return (int64_t)l.m_alloc * l.ld * (int64_t)l.es;
}

void init_ctl(const Layout &l, const ot_params &prm, double tol, Ctl &c)
{
    memset(&c, 0, sizeof(c));
    c.mode = M_INIT;
    c.status = ST_RUNNING;
    for (int k = 0; k < kBufs; ++k) c.xr[k] = k;
    c.eta = prm.eta0 > 0.0 ? prm.eta0 : 1.0 / std::sqrt((double)(l.m + l.n));
    c.omega = prm.omega0 > 0.0 ? prm.omega0 : 1.0;
    c.tol_eff = tol;
}

void fill_result(const Layout &l, const Ctl &c, ot_status st, ot_result &o)
{
    memset(&o, 0, sizeof(o));
    o.status = st;
    o.returned_average = c.ret_avg;
    o.iterations = c.T;
    o.passes = c.passes;
    o.restarts = c.restarts;
    o.kernel_passes = c.kpasses;
    o.objective = c.r_obj;
    o.dual_objective = c.r_dobj;
    o.rel_primal = c.r_relP;
    o.rel_dual = c.r_relD;
    o.rel_gap = c.r_relG;
    o.rel_kkt = c.r_kkt;
    o.eta = c.eta;
    o.omega = c.omega;
    // algorithmic bytes per element of each pass kind (plan element size b, cost
    // element size bc, 0 when regenerated): start-point KKT reads C; a trial or full
    // pass reads X and C and writes X+, and when it folds two iterates it also reads
    // the average and writes the next one; the restart pass reads two plans;
    // verification reads X and C; the fold pass reads two plans and writes one
    const double b = (double)l.es, bc = l.stored ? (double)l.es : 0.0;
    const double per[kModes] = {0.0, bc, 2 * b + bc, 2 * b + bc, 2 * b, b + bc, 3 * b};
    const double elems = (double)l.m * (double)l.n;
    double bytes = 2 * b * elems * (double)c.fold2;
    for (int k = 0; k < kModes; ++k) {
        o.mode_passes[k] = c.mcount[k];
        bytes += per[k] * elems * (double)c.mcount[k];
    }
    o.avg_fold_passes = c.fold2;
    o.pass_bytes = bytes;
    o.verify_retries = c.verify_fails;
    o.kkt_estimate = c.K_cand;
    for (int q = 0; q < 3; ++q) o.estimate_parts[q] = c.e_rel[q];
    o.estimate_objective = c.e_obj;
    o.trace_len = std::min<int64_t>(c.ntrace, l.trace_cap);
}

}  // namespace pdot

namespace {

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(OT_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define OT_TRY(expr)                 \
    do {                             \
        ot_status s_ = (expr);       \
        if (s_ != OT_OK) return s_;  \
    } while (0)

constexpr int kMaxGroups = 24;   // precisions x columns-per-lane x cost sources
// device counts: per lane the tiles of each variant and the combine entries, then the
// instances of each resident variant
constexpr int kLaneCounts = kMaxGroups + 1;
constexpr int kNumCounts = kLanes * kLaneCounts + kMaxGroups;

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

bool finite_nonneg(const std::vector<double> &v)
{
    for (double x : v)
        if (!std::isfinite(x) || x < 0.0) return false;
    return true;
}

// A non-blocking stream of the calling thread for small host fetches: the legacy stream
// must not be used while another thread (the server's scheduler) captures a graph.
ot_status helper_stream(hipStream_t *out)
{
    thread_local hipStream_t s = nullptr;
    thread_local int dev = -1;
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (!s || dev != cur) {
        HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        dev = cur;
    }
    *out = s;
    return OT_OK;
}

// Copy count doubles from a host or device pointer into host memory.
ot_status fetch_host(const double *src, size_t count, std::vector<double> &out)
{
    out.resize(count);
    if (count == 0) return OT_OK;
    if (is_device_ptr(src)) {
        hipStream_t hs = nullptr;
        OT_TRY(helper_stream(&hs));
        HIP_TRY(hipMemcpyAsync(out.data(), src, count * sizeof(double), hipMemcpyDeviceToHost, hs));
        HIP_TRY(hipStreamSynchronize(hs));
    } else {
        memcpy(out.data(), src, count * sizeof(double));
    }
    return OT_OK;
}

ot_status validate_marginals(const std::vector<double> &f, const std::vector<double> &g)
{
    if (!finite_nonneg(f) || !finite_nonneg(g))
        return fail(OT_ERR_INVALID, "f and g must be finite and >= 0");
    double sf = 0.0, sg = 0.0;
    for (double v : f) sf += v;
    for (double v : g) sg += v;
    if (!(std::fabs(sf - sg) <= 1e-12 * std::max(sf, sg))) return fail(OT_ERR_INVALID, "sum f != sum g");
    return OT_OK;
}

// ------------------------------------------------------------------ arena allocator

// First-fit allocator over byte offsets of one device allocation, 256-byte granularity,
// coalescing free neighbours.
class Arena {
public:
    void reset(size_t bytes)
    {
        total_ = bytes;
        used_ = peak_ = 0;
        free_.clear();
        if (bytes) free_[0] = bytes;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = align_up(std::max<size_t>(bytes, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    bool can_alloc(size_t bytes) const
    {
        bytes = align_up(std::max<size_t>(bytes, 1));
        for (auto &kv : free_)
            if (kv.second >= bytes) return true;
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align_up(std::max<size_t>(bytes, 1));
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t total() const { return total_; }

private:
    size_t total_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

// ------------------------------------------------------------------ engine

// Inputs of one instance held in host memory (server requests copy them at submit).
struct HostData {
    std::vector<double> f, g, C, x, y;
};

struct Req {
    Layout L;
    ot_problem prob{};       // caller's output pointers (and input pointers for direct solves)
    double tol = 0.0;
    size_t off = 0;          // arena offset of the instance
    int slot = -1;           // index in the instance table
    Inst I{};
    std::shared_ptr<HostData> host;   // non-null for server requests
    uint64_t ticket = 0;
    double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
    int64_t slots_run = 0;
    double pass_ms = 0.0, comb_ms = 0.0;
    bool done = false;
    ot_result res{};
};

class Engine {
public:
    ~Engine() { release(); }

    // Set up the stream and the arena.  ws: caller workspace (nullable).
    // Narrow write-through plan stores (WT_NARROW) for every instance admitted from now on:
    // for a fixed set whose
    // plans together fit kWtMaxBytes (the server, whose set changes, never sets it).
    void set_write_through(bool on) { write_through_ = on; }

    ot_status init(const ot_params &prm, hipStream_t user_stream, size_t arena_bytes, void *ws,
                   size_t ws_bytes, int max_slots)
    {
        prm_ = prm;
        s_ = user_stream;
        if (!s_) {
            HIP_TRY(hipStreamCreateWithFlags(&s_, hipStreamNonBlocking));
            own_stream_ = true;
        }
        if (ws) {
            if ((uintptr_t)ws % kAlign) return fail(OT_ERR_INVALID, "workspace must be 256-byte aligned");
            if (ws_bytes < arena_bytes) return fail(OT_ERR_OOM, "workspace too small");
            base_ = (char *)ws;
            arena_bytes = ws_bytes;
        } else {
            void *p = nullptr;
            if (hipMalloc(&p, arena_bytes) != hipSuccess) {
                (void)hipGetLastError();
                return fail(OT_ERR_OOM, "hipMalloc of " + std::to_string(arena_bytes) + " bytes failed");
            }
            base_ = (char *)p;
            own_arena_ = true;
        }
        arena_.reset(arena_bytes);
        max_slots_ = max_slots;
        // instance and control-block tables and counts come first in the arena
        if (!arena_.alloc(sizeof(Inst) * (size_t)max_slots, &off_insts_) ||
            !arena_.alloc(sizeof(Ctl) * (size_t)max_slots, &off_ctls_) ||
            !arena_.alloc(sizeof(int32_t) * kNumCounts, &off_counts_))
            return fail(OT_ERR_OOM, "arena too small for the engine tables");
        HIP_TRY(hipHostMalloc((void **)&h_ctl_, sizeof(Ctl) * (size_t)max_slots, hipHostMallocDefault));
        HIP_TRY(hipHostMalloc((void **)&h_counts_, sizeof(int32_t) * kNumCounts, hipHostMallocDefault));
        // resident instances run on a stream of their own, and so does every lane but the
        // first (which uses the caller's stream), beside each other
        HIP_TRY(hipStreamCreateWithFlags(&s2_, hipStreamNonBlocking));
        lanes_[0].s = s_;
        for (int l = 1; l < kLanes; ++l) HIP_TRY(hipStreamCreateWithFlags(&lanes_[l].s, hipStreamNonBlocking));
        for (int i = 0; i < max_slots; ++i) free_slots_.push_back(max_slots - 1 - i);
        for (auto &e : ev_) HIP_TRY(hipEventCreate(&e));
        return OT_OK;
    }

    bool fits(const Layout &L) const { return !free_slots_.empty() && arena_.can_alloc(L.bytes); }

    // Place an instance: workspace, inputs, cost, control block.  On success the request
    // runs from the next graph launch on.
    ot_status admit(Req &r)
    {
        if (free_slots_.empty()) return fail(OT_ERR_BUSY, "no free instance slot");
        if (!arena_.alloc(r.L.bytes, &r.off)) return fail(OT_ERR_BUSY, "arena full");
        r.slot = free_slots_.back();
        free_slots_.pop_back();
        ot_status st = setup(r);
        if (st != OT_OK) {
            arena_.release(r.off, r.L.bytes);
            free_slots_.push_back(r.slot);
            return st;
        }
        active_.push_back(&r);
        dirty_ = true;
        return OT_OK;
    }

    // Launch one block of about target_ms: for every lane a graph launch of its slots
    // (slots_hint > 0 fixes the slot count, else each lane picks its own), and up to
    // `budget` slots of every resident instance, all on their own streams beside each
    // other; then refresh the host mirror of the control blocks of the running instances.
    ot_status run_block(int slots_hint, double target_ms = 2.0)
    {
        OT_TRY(sync_tables(slots_hint, target_ms));
        const int budget = resident_budget(target_ms);
        if (prm_.profile) {
            // one launch at a time, every launch timed by events it stamps itself
            for (size_t gi = 0; gi < rgroups_.size(); ++gi) {
                const RGroup &g = rgroups_[gi];
                HIP_TRY(launch_resident(g.fp32, g.vec, g.cost, d_insts(), d_rlist() + g.first,
                                        d_counts() + kLanes * kLaneCounts + gi, g.cap, budget, s_, ev_[0],
                                        ev_[1]));
                HIP_TRY(hipEventSynchronize(ev_[1]));
                float t = 0.f;
                HIP_TRY(hipEventElapsedTime(&t, ev_[0], ev_[1]));
                for (Req *r : active_)
                    if (r->L.resident && r->L.fp32 == g.fp32 && r->L.vec == g.vec && r->L.cost == g.cost)
                        r->pass_ms += t;
            }
            // the slots of a lane are launched back to back (as in a graph block), every
            // launch stamping its own pair of events; after the block, slot k's times go to
            // the instances whose pass count grew by more than k (an instance stays idle
            // once it has finished)
            for (int l = 0; l < kLanes; ++l) {
                Lane &ln = lanes_[l];
                if (!ln.active) continue;
                const size_t per_slot = ln.groups.size() + 1;
                const size_t need = 2 * per_slot * (size_t)ln.slots;
                while (prof_ev_.size() < need) {
                    hipEvent_t e = nullptr;
                    HIP_TRY(hipEventCreate(&e));
                    prof_ev_.push_back(e);
                }
                std::vector<int64_t> kp0(active_.size());
                for (size_t q = 0; q < active_.size(); ++q) kp0[q] = h_ctl_[active_[q]->slot].kpasses;
                for (int k = 0; k < ln.slots; ++k) {
                    hipEvent_t *ev = &prof_ev_[2 * per_slot * (size_t)k];
                    for (size_t gi = 0; gi < ln.groups.size(); ++gi) {
                        const Group &g = ln.groups[gi];
                        HIP_TRY(launch_pass(g.fp32, g.vec, g.cost, d_insts(), d_ctls(), tiles(ln, k & 1) + g.first,
                                            d_counts() + l * kLaneCounts + gi, g.grid, ln.s, ev[2 * gi],
                                            ev[2 * gi + 1]));
                    }
                    HIP_TRY(launch_combine(d_insts(), d_ctls(), combs(ln), d_counts() + l * kLaneCounts + kMaxGroups,
                                           ln.comb_grid, ln.s, ev[2 * (per_slot - 1)], ev[2 * per_slot - 1]));
                }
                HIP_TRY(hipStreamSynchronize(ln.s));
                for (Req *r : active_)
                    HIP_TRY(hipMemcpyAsync(&h_ctl_[r->slot], r->I.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s_));
                HIP_TRY(hipStreamSynchronize(s_));
                for (int k = 0; k < ln.slots; ++k) {
                    hipEvent_t *ev = &prof_ev_[2 * per_slot * (size_t)k];
                    float a = 0.f, b = 0.f, t = 0.f;
                    for (size_t gi = 0; gi < ln.groups.size(); ++gi) {
                        HIP_TRY(hipEventElapsedTime(&t, ev[2 * gi], ev[2 * gi + 1]));
                        a += t;
                    }
                    HIP_TRY(hipEventElapsedTime(&b, ev[2 * (per_slot - 1)], ev[2 * per_slot - 1]));
                    for (size_t q = 0; q < active_.size(); ++q) {
                        Req *r = active_[q];
                        if (!r->L.resident && r->L.lane == l && h_ctl_[r->slot].kpasses - kp0[q] > k) {
                            r->pass_ms += a;
                            r->comb_ms += b;
                        }
                    }
                }
            }
        } else {
            for (size_t gi = 0; gi < rgroups_.size(); ++gi) {
                const RGroup &g = rgroups_[gi];
                HIP_TRY(launch_resident(g.fp32, g.vec, g.cost, d_insts(), d_rlist() + g.first,
                                        d_counts() + kLanes * kLaneCounts + gi, g.cap, budget, s2_));
            }
            for (int l = 0; l < kLanes; ++l)
                if (lanes_[l].active) HIP_TRY(hipGraphLaunch(lanes_[l].exec, lanes_[l].s));
            HIP_TRY(hipStreamSynchronize(s2_));
            for (int l = 1; l < kLanes; ++l) HIP_TRY(hipStreamSynchronize(lanes_[l].s));
        }
        for (Req *r : active_) {
            r->slots_run += r->L.resident ? budget : lanes_[r->L.lane].slots;
            HIP_TRY(hipMemcpyAsync(&h_ctl_[r->slot], r->I.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s_));
        }
        HIP_TRY(hipStreamSynchronize(s_));
        ++launches_;
        return OT_OK;
    }

    // Algorithm 3 and the certified bracket for an admitted FP64 instance: the plan X
    // (row stride n, FP32 or FP64, host or device) goes to X[0], the duals u to p[0];
    // X_feas (nullable, FP64, row stride n, host or device) receives the feasible plan;
    // scal[6] receives the scalars (RD_* order).
    ot_status round_instance(Req &r, const void *X, int x_fp32, const double *u, double *X_feas, double *scal)
    {
        const Layout &l = r.L;
        Inst &I = r.I;
        const size_t esx = x_fp32 ? 4 : 8;
        if (x_fp32) {
            // stage the FP32 plan in the (free) third plan buffer, then widen it
            HIP_TRY(hipMemcpyAsync(I.X[2], X, esx * (size_t)(l.m * l.n), hipMemcpyDefault, s_));
            HIP_TRY(launch_widen((const float *)I.X[2], l.m, l.n, (double *)I.X[0], l.ld, s_));
        } else {
            HIP_TRY(hipMemcpy2DAsync(I.X[0], sizeof(double) * l.ld, X, sizeof(double) * l.n,
                                     sizeof(double) * l.n, l.m, hipMemcpyDefault, s_));
        }
        HIP_TRY(hipMemcpyAsync(I.p[0], u, sizeof(double) * l.m, hipMemcpyDefault, s_));
        double *xf = nullptr;
        const bool direct = X_feas && is_device_ptr(X_feas);
        if (X_feas) xf = direct ? X_feas : (double *)I.X[2];   // X[2] holds m*n doubles
        HIP_TRY(launch_round(l.cost, d_insts() + r.slot, l.ntiles, xf, s_));
        HIP_TRY(hipMemcpyAsync(scal, I.combscal, sizeof(double) * 6, hipMemcpyDeviceToHost, s_));
        if (X_feas && !direct)
            HIP_TRY(hipMemcpyAsync(X_feas, xf, sizeof(double) * (size_t)(l.m * l.n), hipMemcpyDeviceToHost, s_));
        HIP_TRY(hipStreamSynchronize(s_));
        return OT_OK;
    }

    const Ctl &ctl(const Req &r) const { return h_ctl_[r.slot]; }

    // Ask a running instance to stop at its next decision point (time limits).
    ot_status request_stop(Req &r)
    {
        const int32_t one = 1;
        HIP_TRY(hipMemcpyAsync((char *)r.I.ctl + offsetof(Ctl, stop), &one, sizeof(one),
                               hipMemcpyHostToDevice, s_));
        HIP_TRY(hipStreamSynchronize(s_));
        h_ctl_[r.slot].stop = 1;
        return OT_OK;
    }

    // Copy the outputs of a finished instance, fill its result and release its space.
    ot_status retire(Req &r, ot_status forced = OT_OK)
    {
        const Ctl &c = h_ctl_[r.slot];
        const Layout &l = r.L;
        const Inst &I = r.I;
        ot_status ist = forced != OT_OK ? forced : (c.status < 0 ? OT_ERR_DEVICE : (ot_status)c.status);
        ot_status copy_st = OT_OK;
        if (ist == OT_OK || ist == OT_NOT_CONVERGED) copy_st = copy_outputs(r, c);
        ot_result &o = r.res;
        fill_result(l, c, copy_st != OT_OK ? copy_st : ist, o);
        o.pass_ms = r.pass_ms;
        o.combine_ms = r.comb_ms;
        (void)I;
        r.done = true;
        arena_.release(r.off, l.bytes);
        free_slots_.push_back(r.slot);
        active_.erase(std::remove(active_.begin(), active_.end(), &r), active_.end());
        dirty_ = true;
        return copy_st;
    }

    const std::vector<Req *> &active() const { return active_; }
    size_t arena_used() const { return arena_.used(); }
    size_t arena_peak() const { return arena_.peak(); }
    size_t arena_total() const { return arena_.total(); }
    int64_t launches() const { return launches_; }

    // Slots per graph launch for the running instances of a lane: about target_ms of
    // streaming at roughly 5 TB/s plus about 15 us of latency per slot, between 4 and 512.
    int auto_slots(int lane, double target_ms) const
    {
        double bytes = 0.0;
        for (const Req *r : active_)
            if (!r->L.resident && r->L.lane == lane)
                bytes += (double)r->L.m * (double)r->L.ld * (double)r->L.es * 5.0;
        const double t_slot = bytes / 5e12 + 15e-6;
        int s = (int)(target_ms * 1e-3 / t_slot);
        return std::max(4, std::min(512, s));
    }

    // Slots per launch for the resident instances: about target_ms for the largest of
    // them (a work-group streams about 50 GB/s; a slot costs at least about 4 us of
    // barriers and control), between 16 and 4096 slots.
    int resident_budget(double target_ms) const
    {
        double t_slot = 0.0;
        for (const Req *r : active_)
            if (r->L.resident)
                t_slot = std::max(t_slot, 4e-6 + (double)r->L.m * (double)r->L.ld * (double)r->L.es * 5.0 / 50e9);
        if (t_slot <= 0.0) return 0;
        const int s = (int)(target_ms * 1e-3 / t_slot);
        return std::max(16, std::min(4096, s));
    }

    void release()
    {
        if (s2_) (void)hipStreamSynchronize(s2_);
        if (s_) (void)hipStreamSynchronize(s_);
        for (int l = 0; l < kLanes; ++l) {
            Lane &ln = lanes_[l];
            if (l > 0 && ln.s) {
                (void)hipStreamSynchronize(ln.s);
                (void)hipStreamDestroy(ln.s);
            }
            ln.s = nullptr;
            if (ln.exec) (void)hipGraphExecDestroy(ln.exec);
            if (ln.graph) (void)hipGraphDestroy(ln.graph);
            ln.exec = nullptr;
            ln.graph = nullptr;
        }
        for (auto &e : ev_) {
            if (e) (void)hipEventDestroy(e);
            e = nullptr;
        }
        for (auto &e : prof_ev_) (void)hipEventDestroy(e);
        prof_ev_.clear();
        if (h_ctl_) (void)hipHostFree(h_ctl_);
        if (h_counts_) (void)hipHostFree(h_counts_);
        h_ctl_ = nullptr;
        h_counts_ = nullptr;
        if (own_arena_ && base_) (void)hipFree(base_);
        base_ = nullptr;
        if (own_stream_ && s_) (void)hipStreamDestroy(s_);
        s_ = nullptr;
        if (s2_) {
            (void)hipStreamSynchronize(s2_);
            (void)hipStreamDestroy(s2_);
        }
        s2_ = nullptr;
    }

private:
    struct Group {
        int fp32, vec, cost;
        int first, cap, grid;
    };
    struct RGroup {
        int fp32, vec, cost;
        int first, cap;   // region of the resident list; cap is also the launch grid
    };
    // A size lane: its tile and combine tables, and the graph of its slots.
    struct Lane {
        std::vector<Group> groups;
        size_t off_tiles = 0, off_combs = 0;
        int64_t tile_cap = 0, comb_cap = 0;
        int comb_grid = 1;
        hipStream_t s = nullptr;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        int slots = 0;          // slots per launch (of the captured graph)
        int captured = 0;       // slots in the captured graph
        bool active = false;    // has running instances
    };

    Inst *d_insts() const { return (Inst *)(base_ + off_insts_); }
    Ctl *d_ctls() const { return (Ctl *)(base_ + off_ctls_); }
    int32_t *d_counts() const { return (int32_t *)(base_ + off_counts_); }
    // The tile table of a lane in forward (rev = 0) or reversed (rev = 1) order.
    Tile *tiles(const Lane &ln, int rev = 0) const
    {
        return (Tile *)(base_ + ln.off_tiles) + (rev ? ln.tile_cap : 0);
    }
    CombEntry *combs(const Lane &ln) const { return (CombEntry *)(base_ + ln.off_combs); }
    int32_t *d_rlist() const { return (int32_t *)(base_ + off_rlist_); }

    ot_status copy_outputs(Req &r, const Ctl &c)
    {
        const Layout &l = r.L;
        const Inst &I = r.I;
        if (r.prob.X_out)
            HIP_TRY(hipMemcpy2DAsync(r.prob.X_out, l.n * l.es, I.X[c.ret_x], l.ld * l.es, l.n * l.es, l.m,
                                     hipMemcpyDefault, s_));
        const double *pr = c.ret_avg ? I.pb[c.pbv] : I.p[c.pv];
        const double *qr = c.ret_avg ? I.qb[c.pbv] : I.q[c.pv];
        if (r.prob.u_out) HIP_TRY(hipMemcpyAsync(r.prob.u_out, pr, sizeof(double) * l.m, hipMemcpyDefault, s_));
        if (r.prob.v_out) HIP_TRY(hipMemcpyAsync(r.prob.v_out, qr, sizeof(double) * l.n, hipMemcpyDefault, s_));
        const int64_t nt = std::min<int64_t>(c.ntrace, l.trace_cap);
        if (nt > 0)
            HIP_TRY(hipMemcpyAsync(r.prob.trace, I.trace, sizeof(TraceRec) * (size_t)nt, hipMemcpyDefault, s_));
        HIP_TRY(hipStreamSynchronize(s_));
        return OT_OK;
    }

    ot_status setup(Req &r)
    {
        const Layout &l = r.L;
        const ot_problem &pb = r.prob;
        char *b = base_ + r.off;
        Inst &I = r.I;
        init_inst(l, b, pb.cost.scale, prm_, r.tol, I);
        I.ctl = d_ctls() + r.slot;   // the control block lives in the engine's table
        I.wt = (write_through_ ? 1 : 0) | (plan_bytes(l) >= kWtMinWideBytes ? 2 : 0);
        const int64_t m = l.m, n = l.n;

        HIP_TRY(hipMemsetAsync(b, 0, l.bytes, s_));
        const HostData *h = r.host.get();
        HIP_TRY(hipMemcpyAsync((void *)I.f, h ? (const void *)h->f.data() : (const void *)pb.f,
                               sizeof(double) * m, hipMemcpyDefault, s_));
        HIP_TRY(hipMemcpyAsync((void *)I.g, h ? (const void *)h->g.data() : (const void *)pb.g,
                               sizeof(double) * n, hipMemcpyDefault, s_));
        if (l.dim) {
            HIP_TRY(hipMemcpyAsync((void *)I.xs, h ? (const void *)h->x.data() : (const void *)pb.cost.x,
                                   sizeof(double) * m * l.dim, hipMemcpyDefault, s_));
            HIP_TRY(hipMemcpyAsync((void *)I.ys, h ? (const void *)h->y.data() : (const void *)pb.cost.y,
                                   sizeof(double) * n * l.dim, hipMemcpyDefault, s_));
        }
        if (l.stored) {
            int kind = C_STORED;
            const double *src = nullptr;
            int64_t ldc = 0;
            void *tmp = nullptr;
            if (pb.cost.kind == OT_COST_DENSE) {
                ldc = h ? n : pb.cost.ldc;
                const double *C = h ? h->C.data() : pb.cost.C;
                if (!h && is_device_ptr(C)) {
                    src = C;
                } else {
                    const size_t bytes = sizeof(double) * (size_t)((m - 1) * ldc + n);
                    if (hipMallocAsync(&tmp, bytes, s_) != hipSuccess) {
                        (void)hipGetLastError();
                        return fail(OT_ERR_OOM, "staging allocation for C failed");
                    }
                    HIP_TRY(hipMemcpyAsync(tmp, C, bytes, hipMemcpyHostToDevice, s_));
                    src = (const double *)tmp;
                }
            } else if (is_grid(pb.cost.kind)) {
                kind = (int)pb.cost.kind;
            } else {
                kind = pb.cost.kind == OT_COST_POINTS_SQEUCLID ? C_PTS_SQ : C_PTS_EU;
            }
            HIP_TRY(launch_materialize(l.fp32, (void *)I.C, m, n, l.ld, kind, src, ldc, I.xs, I.ys,
                                       l.dim, l.side, pb.cost.scale, s_));
            if (tmp) HIP_TRY(hipFreeAsync(tmp, s_));
        }
        Ctl c;
        init_ctl(l, prm_, r.tol, c);
        h_ctl_[r.slot] = c;
        HIP_TRY(hipMemcpyAsync(I.ctl, &h_ctl_[r.slot], sizeof(Ctl), hipMemcpyHostToDevice, s_));
        HIP_TRY(hipMemcpyAsync(d_insts() + r.slot, &I, sizeof(Inst), hipMemcpyHostToDevice, s_));
        // host sources above must stay alive until the copies are done
        HIP_TRY(hipStreamSynchronize(s_));
        return OT_OK;
    }

    // Rebuild the tile, combine and resident tables of the running set; in each lane,
    // capture the graph again when its variant layout changed, a table had to grow or its
    // slot count changed.  A lane keeps its slot count unless the work asks for more than
    // twice or less than half of it (every new count needs a new capture).
    ot_status sync_tables(int slots_hint, double target_ms)
    {
        int want[kLanes];
        bool change = dirty_;
        for (int l = 0; l < kLanes; ++l) {
            Lane &ln = lanes_[l];
            int w = slots_hint > 0 ? slots_hint : auto_slots(l, target_ms);
            if (slots_hint <= 0 && ln.slots > 0 && w <= 2 * ln.slots && 2 * w >= ln.slots) w = ln.slots;
            want[l] = w;
            change |= w != ln.slots;
        }
        if (!change) return OT_OK;
        struct Key {
            int fp32, vec, cost;
        };
        auto key_of = [](std::vector<Key> &ks, const Layout &l) {
            for (size_t k = 0; k < ks.size(); ++k)
                if (ks[k].fp32 == l.fp32 && ks[k].vec == l.vec && ks[k].cost == l.cost) return k;
            ks.push_back({l.fp32, l.vec, l.cost});
            return ks.size() - 1;
        };
        std::vector<Key> keys[kLanes], rkeys;
        std::vector<std::vector<Tile>> per[kLanes];
        std::vector<CombEntry> cmb[kLanes];
        std::vector<std::vector<int32_t>> rper;
        for (Req *r : active_) {
            const Layout &l = r->L;
            if (l.resident) {
                const size_t gi = key_of(rkeys, l);
                if (rper.size() < rkeys.size()) rper.resize(rkeys.size());
                rper[gi].push_back(r->slot);
                continue;
            }
            const int ln = l.lane;
            const size_t gi = key_of(keys[ln], l);
            if (per[ln].size() < keys[ln].size()) per[ln].resize(keys[ln].size());
            for (int rb = 0; rb < l.nrb; ++rb)
                for (int cb = 0; cb < l.ncb; ++cb) per[ln][gi].push_back(Tile{r->slot, rb, cb, rb * l.ncb + cb});
            int local = 0;
            for (int64_t i = 0; i < l.m; i += kCombEntries) cmb[ln].push_back(CombEntry{r->slot, 0, (int)i, local++});
            for (int64_t j = 0; j < l.n; j += kCombEntries) cmb[ln].push_back(CombEntry{r->slot, 1, (int)j, local++});
        }
        if ((int)rkeys.size() > kMaxGroups) return fail(OT_ERR_INVALID, "too many kernel variants in one run");
        for (int l = 0; l < kLanes; ++l)
            if ((int)keys[l].size() > kMaxGroups) return fail(OT_ERR_INVALID, "too many kernel variants in one run");

        // resident lists: one region per variant (launched directly, no graph)
        {
            int64_t total = 0;
            for (auto &v : rper) total += std::max<int64_t>(64, (int64_t)v.size());
            if (total > rlist_cap_) {
                if (rlist_cap_) arena_.release(off_rlist_, sizeof(int32_t) * (size_t)rlist_cap_);
                rlist_cap_ = 0;
                const int64_t cap = total * 3 / 2 + 64;
                if (!arena_.alloc(sizeof(int32_t) * (size_t)cap, &off_rlist_))
                    return fail(OT_ERR_OOM, "arena too small for the resident list");
                rlist_cap_ = cap;
            }
            rgroups_.clear();
            int first = 0;
            for (size_t k = 0; k < rkeys.size(); ++k) {
                const int cap = (int)std::max<int64_t>(64, (int64_t)rper[k].size());
                rgroups_.push_back(RGroup{rkeys[k].fp32, rkeys[k].vec, rkeys[k].cost, first, cap});
                HIP_TRY(hipMemcpyAsync(d_rlist() + first, rper[k].data(), sizeof(int32_t) * rper[k].size(),
                                       hipMemcpyHostToDevice, s_));
                first += cap;
            }
        }

        for (int g = 0; g < kNumCounts; ++g) h_counts_[g] = 0;
        std::deque<std::vector<Tile>> rev_tiles;   // reversed tables, alive until the sync below
        bool recapture[kLanes];
        for (int l = 0; l < kLanes; ++l) {
            Lane &ln = lanes_[l];
            recapture[l] = false;
            ln.active = !keys[l].empty();
            ln.slots = want[l];
            if (!ln.active) continue;
            // keep the current layout when every variant still fits its region
            bool relayout = (!ln.exec && !prm_.profile) || ln.slots != ln.captured ||
                            (int64_t)cmb[l].size() > ln.comb_cap;
            std::vector<int> map(keys[l].size(), -1);
            for (size_t k = 0; k < keys[l].size(); ++k) {
                for (size_t g = 0; g < ln.groups.size(); ++g)
                    if (ln.groups[g].fp32 == keys[l][k].fp32 && ln.groups[g].vec == keys[l][k].vec &&
                        ln.groups[g].cost == keys[l][k].cost && (int64_t)per[l][k].size() <= ln.groups[g].cap)
                        map[k] = (int)g;
                if (map[k] < 0) relayout = true;
            }
            if (relayout) {
                std::vector<Group> ng;
                int64_t total = 0;
                for (size_t k = 0; k < keys[l].size(); ++k) {
                    // room to spare so that instances joining later rarely force a new capture
                    const int cap = (int)std::max<int64_t>(256, (int64_t)per[l][k].size() * 3 / 2 + 64);
                    ng.push_back(Group{keys[l][k].fp32, keys[l][k].vec, keys[l][k].cost, (int)total, cap,
                                       std::min(cap, kMaxGrid)});
                    map[k] = (int)k;
                    total += cap;
                }
                const int64_t ccap = std::max<int64_t>(256, (int64_t)cmb[l].size() * 3 / 2 + 64);
                // two copies of the table: tile order forward, then reversed (see capture())
                if (total > ln.tile_cap) {
                    if (ln.tile_cap) arena_.release(ln.off_tiles, sizeof(Tile) * 2 * (size_t)ln.tile_cap);
                    ln.tile_cap = 0;
                    if (!arena_.alloc(sizeof(Tile) * 2 * (size_t)total, &ln.off_tiles))
                        return fail(OT_ERR_OOM, "arena too small for the tile table");
                    ln.tile_cap = total;
                }
                if (ccap > ln.comb_cap) {
                    if (ln.comb_cap) arena_.release(ln.off_combs, sizeof(CombEntry) * (size_t)ln.comb_cap);
                    ln.comb_cap = 0;
                    if (!arena_.alloc(sizeof(CombEntry) * (size_t)ccap, &ln.off_combs))
                        return fail(OT_ERR_OOM, "arena too small for the combine table");
                    ln.comb_cap = ccap;
                }
                ln.groups = ng;
                ln.comb_grid = (int)std::min<int64_t>(ln.comb_cap, kMaxGrid);
                recapture[l] = !prm_.profile;
            }
            for (size_t k = 0; k < keys[l].size(); ++k) {
                const Group &g = ln.groups[map[k]];
                if (!per[l][k].empty()) {
                    HIP_TRY(hipMemcpyAsync(tiles(ln) + g.first, per[l][k].data(), sizeof(Tile) * per[l][k].size(),
                                           hipMemcpyHostToDevice, s_));
                    // a copy of its own: the source of an asynchronous copy must stay unchanged
                    // until the synchronisation below
                    rev_tiles.emplace_back(per[l][k].rbegin(), per[l][k].rend());
                    HIP_TRY(hipMemcpyAsync(tiles(ln, 1) + g.first, rev_tiles.back().data(),
                                           sizeof(Tile) * rev_tiles.back().size(), hipMemcpyHostToDevice, s_));
                }
                h_counts_[l * kLaneCounts + map[k]] = (int32_t)per[l][k].size();
            }
            if (!cmb[l].empty())
                HIP_TRY(hipMemcpyAsync(combs(ln), cmb[l].data(), sizeof(CombEntry) * cmb[l].size(),
                                       hipMemcpyHostToDevice, s_));
            h_counts_[l * kLaneCounts + kMaxGroups] = (int32_t)cmb[l].size();
        }
        for (size_t k = 0; k < rkeys.size(); ++k) h_counts_[kLanes * kLaneCounts + k] = (int32_t)rper[k].size();
        HIP_TRY(hipMemcpyAsync(d_counts(), h_counts_, sizeof(int32_t) * kNumCounts, hipMemcpyHostToDevice, s_));
        HIP_TRY(hipStreamSynchronize(s_));   // the host tables above are temporaries
        dirty_ = false;
        for (int l = 0; l < kLanes; ++l)
            if (recapture[l]) OT_TRY(capture(l));
        return OT_OK;
    }

    ot_status capture(int l)
    {
        Lane &ln = lanes_[l];
        if (ln.exec) (void)hipGraphExecDestroy(ln.exec);
        if (ln.graph) (void)hipGraphDestroy(ln.graph);
        ln.exec = nullptr;
        ln.graph = nullptr;
        ln.captured = 0;
        // relaxed: other threads (callers submitting to a server) may use the runtime while
        // this thread captures
        HIP_TRY(hipStreamBeginCapture(ln.s, hipStreamCaptureModeRelaxed));
        hipError_t e = hipSuccess;
        for (int sl = 0; sl < ln.slots && e == hipSuccess; ++sl) {
            for (size_t gi = 0; gi < ln.groups.size() && e == hipSuccess; ++gi) {
                const Group &g = ln.groups[gi];
                // consecutive slots stream the tiles in opposite orders: a pass starts on
                // what the previous one touched last, which the Infinity Cache still holds
                // when the plans outgrow it
                e = launch_pass(g.fp32, g.vec, g.cost, d_insts(), d_ctls(), tiles(ln, sl & 1) + g.first,
                                d_counts() + l * kLaneCounts + gi, g.grid, ln.s);
            }
            if (e == hipSuccess)
                e = launch_combine(d_insts(), d_ctls(), combs(ln), d_counts() + l * kLaneCounts + kMaxGroups,
                                   ln.comb_grid, ln.s);
        }
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(ln.s, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(OT_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
        }
        ln.graph = g;
        HIP_TRY(hipGraphInstantiate(&ln.exec, ln.graph, nullptr, nullptr, 0));
        ln.captured = ln.slots;
        return OT_OK;
    }

    ot_params prm_{};
    hipStream_t s_ = nullptr;
    bool own_stream_ = false, own_arena_ = false;
    bool write_through_ = false;   // set_write_through
    char *base_ = nullptr;
    Arena arena_;
    int max_slots_ = 0;
    std::vector<int> free_slots_;
    std::vector<Req *> active_;
    size_t off_insts_ = 0, off_ctls_ = 0, off_counts_ = 0, off_rlist_ = 0;
    int64_t rlist_cap_ = 0;
    Lane lanes_[kLanes];
    std::vector<RGroup> rgroups_;
    hipStream_t s2_ = nullptr;
    bool dirty_ = true;
    Ctl *h_ctl_ = nullptr;
    int32_t *h_counts_ = nullptr;
    hipEvent_t ev_[2] = {nullptr, nullptr};
    std::vector<hipEvent_t> prof_ev_;   // profile mode: a start and an end event per launch
    int64_t launches_ = 0;
};

// ------------------------------------------------------------------ fixed batches

struct Planned {
    std::vector<Layout> L;
    size_t total = 0;
};

// Arena bytes for a fixed set: the engine's instance table and counts, every instance in
// admission order, then the tile table (one region per kernel variant, each sized as
// sync_tables sizes it) and the combine table.
ot_status plan_fixed(const ot_problem *probs, int count, const ot_params &prm, Planned &P)
{
    P.L.resize(count);
    int64_t combs[kLanes] = {};
    bool used[kLanes] = {};
    std::vector<std::pair<std::tuple<int, int, int, int>, int64_t>> per;
    for (int i = 0; i < count; ++i) {
        ot_status st = plan_instance(probs[i], prm, P.L[i]);
        if (st != OT_OK) return fail(st, "instance " + std::to_string(i) + ": " + g_err.c_str());
        const Layout &l = P.L[i];
        if (l.resident) continue;
        combs[l.lane] += l.ncomb;
        used[l.lane] = true;
        auto key = std::make_tuple(l.lane, l.fp32, l.vec, l.cost);
        bool seen = false;
        for (auto &kv : per)
            if (kv.first == key) {
                kv.second += l.ntiles;
                seen = true;
            }
        if (!seen) per.push_back({key, (int64_t)l.ntiles});
    }
    size_t total = align_up(sizeof(Inst) * (size_t)count) + align_up(sizeof(Ctl) * (size_t)count) +
                   align_up(sizeof(int32_t) * kNumCounts);
    for (auto &l : P.L) total += align_up(l.bytes);
    // each lane's tile (two copies) and combine tables, sized as sync_tables sizes them
    int64_t tcap[kLanes] = {};
    for (auto &kv : per) tcap[std::get<0>(kv.first)] += std::max<int64_t>(256, kv.second * 3 / 2 + 64);
    for (int l = 0; l < kLanes; ++l) {
        if (!used[l]) continue;
        const int64_t ccap = std::max<int64_t>(256, combs[l] * 3 / 2 + 64);
        total += align_up(sizeof(Tile) * 2 * (size_t)tcap[l]) + align_up(sizeof(CombEntry) * (size_t)ccap);
    }
    // resident lists, sized as sync_tables sizes them at most
    total += align_up(sizeof(int32_t) * (size_t)(((int64_t)count + 64 * kMaxGroups) * 3 / 2 + 64));
    P.total = total;
    return OT_OK;
}

ot_status run_fixed(const ot_problem *probs, int count, const ot_params &prm, ot_result *res,
                    void *workspace, size_t ws_bytes, hipStream_t stream)
{
    const double t0 = now_s();
    if (count < 1 || !probs) return fail(OT_ERR_INVALID, "no problems");
    OT_TRY(check_params(prm));
    Planned P;
    OT_TRY(plan_fixed(probs, count, prm, P));
    std::vector<Req> reqs(count);
    for (int i = 0; i < count; ++i) {
        std::vector<double> fh, gh;
        OT_TRY(fetch_host(probs[i].f, (size_t)probs[i].m, fh));
        OT_TRY(fetch_host(probs[i].g, (size_t)probs[i].n, gh));
        ot_status st = validate_marginals(fh, gh);
        if (st != OT_OK) return fail(st, "instance " + std::to_string(i) + ": " + g_err.c_str());
        reqs[i].L = P.L[i];
        reqs[i].prob = probs[i];
        reqs[i].tol = probs[i].tol > 0.0 ? probs[i].tol : prm.tol;
    }
    Engine E;
    OT_TRY(E.init(prm, stream, P.total, workspace, ws_bytes, count));
    int64_t plans = 0;
    for (int i = 0; i < count; ++i) plans += plan_bytes(P.L[i]);
    E.set_write_through(plans <= kWtMaxBytes);
    for (int i = 0; i < count; ++i) {
        ot_status st = E.admit(reqs[i]);
        if (st != OT_OK)
            return fail(st == OT_ERR_BUSY ? OT_ERR_OOM : st, "instance " + std::to_string(i) + ": " + g_err.c_str());
    }
    bool stop_sent = false;
    ot_status hard = OT_OK;
    while (!E.active().empty()) {
        // blocks of about 8 ms: fewer host round trips than the server's 2 ms (which
        // bound admission latency); an instance that finishes inside a block idles for
        // the rest of it at about 3 us per slot
        // profile mode launches blocks of 16 slots back to back without a graph
        ot_status st = E.run_block(prm.profile ? 16 : prm.graph_slots, 8.0);
        if (st != OT_OK) return st;
        std::vector<Req *> fin, stuck;
        for (Req *r : E.active()) {
            if (E.ctl(*r).mode == M_IDLE) fin.push_back(r);
            else if (r->slots_run > 3 * std::max<int64_t>(prm.max_passes, 1) + 64) stuck.push_back(r);
        }
        for (Req *r : fin) {
            r->t_done = now_s() - t0;
            st = E.retire(*r);
            if (st != OT_OK && hard == OT_OK) hard = st;
        }
        for (Req *r : stuck) {
            r->t_done = now_s() - t0;
            (void)E.retire(*r, OT_ERR_DEVICE);
        }
        if (!stop_sent && prm.time_limit_s > 0.0 && now_s() - t0 >= prm.time_limit_s) {
            for (Req *r : E.active()) OT_TRY(E.request_stop(*r));
            stop_sent = true;
        }
    }
    const double secs = now_s() - t0;
    ot_status first_bad = hard;
    for (int i = 0; i < count; ++i) {
        if (reqs[i].res.status != OT_OK && first_bad == OT_OK) first_bad = (ot_status)reqs[i].res.status;
        if (res) {
            res[i] = reqs[i].res;
            res[i].seconds = count == 1 ? secs : reqs[i].t_done;
        }
    }
    if (first_bad == OT_OK) {
        g_err.clear();
    } else if (first_bad == OT_NOT_CONVERGED) {
        g_err = "iteration, pass or time limit reached";
    } else if (first_bad == OT_ERR_NUMERIC) {
        g_err = "numerical failure (NaN/Inf in KKT or step scalars)";
    } else if (g_err.empty()) {
        g_err = "solver did not reach a final state";
    }
    return first_bad;
}

}  // namespace

// ------------------------------------------------------------------ server

struct ot_server {
    ot_server_cfg cfg{};
    Engine E;
    int device = 0;
    double t0 = 0.0;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv, cv_done;
    bool stop = false;
    std::deque<std::unique_ptr<Req>> queue;
    std::vector<std::unique_ptr<Req>> running;
    std::deque<ot_completion> done;
    uint64_t next_ticket = 1;
    int64_t submitted = 0, admitted = 0, completed = 0, max_running = 0, launches = 0;
    int64_t arena_used = 0, arena_peak = 0;   // snapshots of the engine's counters
    std::string thread_error;

    // completion record of a request (called with mu held)
    void push_done(const Req &r)
    {
        ot_completion c{};
        c.ticket = r.ticket;
        c.result = r.res;
        c.result.seconds = r.t_done - r.t_admit;
        c.t_submit = r.t_submit;
        c.t_admit = r.t_admit;
        c.t_done = r.t_done;
        done.push_back(c);
        ++completed;
        cv_done.notify_all();
    }

    void loop()
    {
        (void)hipSetDevice(device);
        while (true) {
            {
                std::unique_lock<std::mutex> lk(mu);
                if (running.empty())
                    cv.wait(lk, [&] { return stop || !queue.empty(); });
                if (stop) break;
                // admit from the head of the queue while a slot and arena space are free
                while (!queue.empty() && E.fits(queue.front()->L)) {
                    std::unique_ptr<Req> r = std::move(queue.front());
                    queue.pop_front();
                    lk.unlock();
                    r->t_admit = now_s() - t0;
                    const ot_status st = E.admit(*r);
                    lk.lock();
                    if (st != OT_OK) {
                        r->res.status = st;
                        r->t_done = now_s() - t0;
                        push_done(*r);
                        continue;
                    }
                    ++admitted;
                    running.push_back(std::move(r));
                    max_running = std::max<int64_t>(max_running, (int64_t)running.size());
                }
                // nothing runs and the head still does not fit (tables fragment the arena):
                // it never will, reject it
                if (running.empty() && !queue.empty()) {
                    std::unique_ptr<Req> r = std::move(queue.front());
                    queue.pop_front();
                    r->res.status = OT_ERR_OOM;
                    r->t_admit = r->t_done = now_s() - t0;
                    push_done(*r);
                }
                arena_used = (int64_t)E.arena_used();
                arena_peak = (int64_t)E.arena_peak();
            }
            if (running.empty()) continue;
            const ot_status st = E.run_block(cfg.params.graph_slots, cfg.block_ms > 0 ? cfg.block_ms : 2.0);
            if (st != OT_OK) {
                std::lock_guard<std::mutex> lk(mu);
                thread_error = g_err.c_str();
                for (auto &r : running) {
                    r->res.status = st;
                    r->t_done = now_s() - t0;
                    push_done(*r);
                }
                running.clear();
                cv_done.notify_all();
                break;
            }
            const double tnow = now_s() - t0;
            std::vector<Req *> fin, stuck;
            for (auto &r : running) {
                const Ctl &c = E.ctl(*r);
                if (c.mode == M_IDLE) {
                    fin.push_back(r.get());
                } else if (r->slots_run > 3 * std::max<int64_t>(cfg.params.max_passes, 1) + 64) {
                    stuck.push_back(r.get());
                } else if (cfg.params.time_limit_s > 0.0 && tnow - r->t_admit >= cfg.params.time_limit_s &&
                           !c.stop) {
                    (void)E.request_stop(*r);
                }
            }
            for (Req *r : fin) (void)E.retire(*r);
            for (Req *r : stuck) (void)E.retire(*r, OT_ERR_DEVICE);
            std::lock_guard<std::mutex> lk(mu);
            launches = E.launches();
            arena_used = (int64_t)E.arena_used();
            arena_peak = (int64_t)E.arena_peak();
            const double tdone = now_s() - t0;
            for (auto &r : running)
                if (r->done) {
                    r->t_done = tdone;
                    push_done(*r);
                }
            running.erase(std::remove_if(running.begin(), running.end(),
                                         [](const std::unique_ptr<Req> &r) { return r->done; }),
                          running.end());
        }
    }
};

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
    p->verify_retries = 8;
}

size_t ot_workspace_size(const ot_problem *prob, const ot_params *prm)
{
    if (!prob || !prm) {
        fail(OT_ERR_INVALID, "null argument");
        return 0;
    }
    Planned P;
    if (plan_fixed(prob, 1, *prm, P) != OT_OK) return 0;
    return P.total;
}

ot_status ot_solve(const ot_problem *prob, const ot_params *prm, ot_result *res, void *workspace,
                   size_t workspace_bytes, void *stream)
{
    if (!prob || !prm) return fail(OT_ERR_INVALID, "null argument");
    return run_fixed(prob, 1, *prm, res, workspace, workspace_bytes, (hipStream_t)stream);
}

ot_status ot_solve_batch(const ot_problem *probs, int32_t count, const ot_params *prm,
                         ot_result *res, void *stream)
{
    if (!probs || !prm || count < 1) return fail(OT_ERR_INVALID, "null argument or empty batch");
    return run_fixed(probs, count, *prm, res, nullptr, 0, (hipStream_t)stream);
}

ot_status ot_round(const ot_problem *prob, int32_t precision, const void *X, const double *u,
                   double *X_feas, ot_bracket *out, void *stream)
{
    if (!prob || !X || !u || !out) return fail(OT_ERR_INVALID, "null argument");
    if (precision != OT_PREC_FP32 && precision != OT_PREC_FP64) return fail(OT_ERR_INVALID, "unknown precision");
    // an FP64 instance (the paper's costs) on the whole-GPU layout, 128-column bands
    ot_params prm;
    ot_params_default(&prm);
    prm.precision = OT_PREC_FP64;
    prm.engine = 1;
    ot_problem pb = *prob;
    pb.tile_vec = 2;
    pb.tile_rows = 0;
    pb.X_out = nullptr;
    pb.u_out = nullptr;
    pb.v_out = nullptr;
    pb.trace = nullptr;
    pb.trace_cap = 0;
    Planned P;
    OT_TRY(plan_fixed(&pb, 1, prm, P));
    std::vector<double> fh, gh;
    OT_TRY(fetch_host(pb.f, (size_t)pb.m, fh));
    OT_TRY(fetch_host(pb.g, (size_t)pb.n, gh));
    OT_TRY(validate_marginals(fh, gh));
    Engine E;
    OT_TRY(E.init(prm, (hipStream_t)stream, P.total, nullptr, 0, 1));
    Req r;
    r.L = P.L[0];
    r.prob = pb;
    r.tol = 1.0;
    OT_TRY(E.admit(r));
    double sc[6] = {0, 0, 0, 0, 0, 0};
    OT_TRY(E.round_instance(r, X, precision == OT_PREC_FP32, u, X_feas, sc));
    memset(out, 0, sizeof(*out));
    out->marginal_l1 = sc[RD_MARG];
    out->upper = sc[RD_UPPER];
    out->l1_change = sc[RD_CHANGE];
    out->lower = sc[RD_LOWER];
    out->feas_violation = sc[RD_VIOL];
    g_err.clear();
    return OT_OK;
}

ot_status ot_server_create(const ot_server_cfg *cfg, ot_server **out)
{
    if (!cfg || !out) return fail(OT_ERR_INVALID, "null argument");
    if (cfg->max_active < 1 || cfg->hbm_budget_bytes < ((size_t)1 << 20))
        return fail(OT_ERR_INVALID, "max_active >= 1 and a budget of at least 1 MiB are required");
    OT_TRY(check_params(cfg->params));
    std::unique_ptr<ot_server> s(new ot_server());
    s->cfg = *cfg;
    s->cfg.params.profile = 0;
    HIP_TRY(hipGetDevice(&s->device));
    OT_TRY(s->E.init(s->cfg.params, nullptr, cfg->hbm_budget_bytes, nullptr, 0, cfg->max_active));
    s->t0 = now_s();
    ot_server *raw = s.get();
    s->th = std::thread([raw] { raw->loop(); });
    *out = s.release();
    g_err.clear();
    return OT_OK;
}

ot_status ot_server_submit(ot_server *srv, const ot_problem *prob, uint64_t *ticket)
{
    if (!srv || !prob) return fail(OT_ERR_INVALID, "null argument");
    std::unique_ptr<Req> r(new Req());
    OT_TRY(plan_instance(*prob, srv->cfg.params, r->L));
    // the instance plus its share of the engine tables must fit in the arena
    if (r->L.bytes + ((size_t)1 << 20) > srv->E.arena_total())
        return fail(OT_ERR_BUSY, "problem needs more device memory than the server budget");
    auto h = std::make_shared<HostData>();
    OT_TRY(fetch_host(prob->f, (size_t)prob->m, h->f));
    OT_TRY(fetch_host(prob->g, (size_t)prob->n, h->g));
    OT_TRY(validate_marginals(h->f, h->g));
    const ot_cost &c = prob->cost;
    if (c.kind == OT_COST_DENSE) {
        h->C.resize((size_t)prob->m * (size_t)prob->n);
        std::vector<double> row;
        for (int64_t i = 0; i < prob->m; ++i) {
            OT_TRY(fetch_host(c.C + i * c.ldc, (size_t)prob->n, row));
            memcpy(h->C.data() + i * prob->n, row.data(), sizeof(double) * (size_t)prob->n);
        }
    } else if (c.kind == OT_COST_POINTS_SQEUCLID || c.kind == OT_COST_POINTS_EUCLID) {
        OT_TRY(fetch_host(c.x, (size_t)prob->m * c.dim, h->x));
        OT_TRY(fetch_host(c.y, (size_t)prob->n * c.dim, h->y));
    }
    r->host = h;
    r->prob = *prob;
    r->tol = prob->tol > 0.0 ? prob->tol : srv->cfg.params.tol;
    std::lock_guard<std::mutex> lk(srv->mu);
    if (!srv->thread_error.empty()) return fail(OT_ERR_DEVICE, "server stopped: " + srv->thread_error);
    if (srv->cfg.max_queue > 0 && (int)srv->queue.size() >= srv->cfg.max_queue)
        return fail(OT_ERR_BUSY, "queue full");
    r->ticket = srv->next_ticket++;
    r->t_submit = now_s() - srv->t0;
    if (ticket) *ticket = r->ticket;
    srv->queue.push_back(std::move(r));
    ++srv->submitted;
    srv->cv.notify_all();
    g_err.clear();
    return OT_OK;
}

ot_status ot_server_poll(ot_server *srv, ot_completion *out, int32_t max, int32_t *n_out)
{
    if (!srv || (!out && max > 0) || !n_out) return fail(OT_ERR_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    int32_t k = 0;
    while (k < max && !srv->done.empty()) {
        out[k++] = srv->done.front();
        srv->done.pop_front();
    }
    *n_out = k;
    return OT_OK;
}

ot_status ot_server_drain(ot_server *srv, double timeout_s)
{
    if (!srv) return fail(OT_ERR_INVALID, "null argument");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto pred = [&] { return srv->completed >= srv->submitted || !srv->thread_error.empty(); };
    if (timeout_s > 0.0) {
        if (!srv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred))
            return fail(OT_NOT_CONVERGED, "drain timed out");
    } else {
        srv->cv_done.wait(lk, pred);
    }
    if (!srv->thread_error.empty()) return fail(OT_ERR_DEVICE, "server stopped: " + srv->thread_error);
    return OT_OK;
}

ot_status ot_server_get_stats(ot_server *srv, ot_server_stats *o)
{
    if (!srv || !o) return fail(OT_ERR_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    o->submitted = srv->submitted;
    o->admitted = srv->admitted;
    o->completed = srv->completed;
    o->running = (int64_t)srv->running.size();
    o->queued = (int64_t)srv->queue.size();
    o->arena_used = srv->arena_used;
    o->arena_peak = srv->arena_peak;
    o->launches = srv->launches;
    o->max_running = srv->max_running;
    return OT_OK;
}

ot_status ot_server_destroy(ot_server *srv)
{
    if (!srv) return fail(OT_ERR_INVALID, "null argument");
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv.notify_all();
    if (srv->th.joinable()) srv->th.join();
    srv->E.release();
    delete srv;
    return OT_OK;
}

const char *ot_last_error(void) { return g_err.c_str(); }

const char *ot_version(void) { return "pdot-mi355x 0.2"; }

}  // extern "C"
