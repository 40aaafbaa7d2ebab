// ot_solve_noalloc: ot_solve for callers that cannot allocate (code under HIP graph
// capture, tight serving loops, harnesses that forbid allocation).
//
// The workspace of the solve -- the instance's plan buffers, cost, coordinates, vectors,
// partial sums and control block, and the instance, tile and combine tables -- lives in a
// file-scope device array of OT_NOALLOC_MAX_BYTES that the library holds on every GPU it
// runs on until the process ends.  The call launches the same kernels as ot_solve (one
// streaming pass and one combine per slot, or the resident kernel for small instances)
// directly on the caller's stream, without a graph, and reads the control block between
// blocks of slots; it calls no hipMalloc, hipFree, hipHostMalloc, stream, event or graph
// creation, and keeps no heap memory: host-side state is on the stack, and marginals that
// live in device memory are checked through a stack buffer.  Every call on a GPU uses that
// GPU's one array, so calls that overlap on one GPU race: callers serialise them per
// device.  The array keeps the last call's contents; each call clears the region it uses
// with a fill kernel before use.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "pdot.h"
#include "pdot_host.h"
#include "pdot_internal.h"

namespace pdot {
namespace {

constexpr size_t kScratchBytes = OT_NOALLOC_MAX_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices];   // device address of `scratch` on each device (null: not yet)

#define NA_TRY(expr)                                                                    \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            char b_[256];                                                               \
            snprintf(b_, sizeof b_, "%s: %s", #expr, hipGetErrorString(e_));            \
            return fail(OT_ERR_DEVICE, b_);                                             \
        }                                                                               \
    } while (0)

#define NA_OK(expr)                 \
    do {                            \
        ot_status s_ = (expr);      \
        if (s_ != OT_OK) return s_; \
    } while (0)

double seconds_now()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Device address of the array on the current device, looked up once per device with that
// device current.  The array's name is only a host-side stand-in for it.
ot_status scratch_base(char **out)
{
    int dev = 0;
    NA_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(OT_ERR_DEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        NA_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(OT_ERR_DEVICE, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch[dev] = p;
    }
    *out = (char *)g_scratch[dev];
    return OT_OK;
}

// Sum of a host or device vector in index order, and whether every entry is finite and
// >= 0 (device data is read through a stack buffer).
ot_status sum_checked(const double *v, int64_t len, hipStream_t s, double *sum, bool *ok)
{
    double buf[2048];
    const bool on_dev = is_device_ptr(v);
    double acc = 0.0;
    bool good = true;
    for (int64_t at = 0; at < len; at += 2048) {
        const int64_t cnt = len - at < 2048 ? len - at : 2048;
        const double *src = v + at;
        if (on_dev) {
            NA_TRY(hipMemcpyAsync(buf, src, sizeof(double) * (size_t)cnt, hipMemcpyDeviceToHost, s));
            NA_TRY(hipStreamSynchronize(s));
            src = buf;
        }
        for (int64_t i = 0; i < cnt; ++i) {
            if (!std::isfinite(src[i]) || src[i] < 0.0) good = false;
            acc += src[i];
        }
    }
    *sum = acc;
    *ok = good;
    return OT_OK;
}

ot_status solve_noalloc(const ot_problem &pb, const ot_params &prm, ot_result *res, hipStream_t s)
{
    const double t0 = seconds_now();
    NA_OK(check_params(prm));
    Layout L;
    NA_OK(plan_instance(pb, prm, L));

    // scratch: [instance descriptor][counts][tile table][combine table][instance workspace]
    const size_t off_counts = align_up(sizeof(Inst));
    const size_t off_tiles = off_counts + align_up(sizeof(int32_t) * 8);
    const size_t off_combs = off_tiles + align_up(sizeof(Tile) * (size_t)L.ntiles);
    const size_t off_ws = off_combs + align_up(sizeof(CombEntry) * (size_t)L.ncomb);
    const size_t need = off_ws + L.bytes;
    if (need > kScratchBytes) {
        char b[256];
        snprintf(b, sizeof b,
                 "problem needs %zu bytes of device scratch; ot_solve_noalloc holds at most %zu "
                 "(OT_NOALLOC_MAX_BYTES): use ot_solve",
                 need, kScratchBytes);
        return fail(OT_ERR_OOM, b);
    }

    // marginals: finite, >= 0, equal mass (as ot_solve checks them)
    double sf = 0.0, sg = 0.0;
    bool okf = true, okg = true;
    NA_OK(sum_checked(pb.f, pb.m, s, &sf, &okf));
    NA_OK(sum_checked(pb.g, pb.n, s, &sg, &okg));
    if (!okf || !okg) return fail(OT_ERR_INVALID, "f and g must be finite and >= 0");
    if (!(std::fabs(sf - sg) <= 1e-12 * (sf > sg ? sf : sg))) return fail(OT_ERR_INVALID, "sum f != sum g");

    char *base = nullptr;
    NA_OK(scratch_base(&base));
    Inst *d_inst = (Inst *)base;
    int32_t *counts = (int32_t *)(base + off_counts);
    Tile *tiles = (Tile *)(base + off_tiles);
    CombEntry *combs = (CombEntry *)(base + off_combs);
    char *ws = base + off_ws;

    const double tol = pb.tol > 0.0 ? pb.tol : prm.tol;
    const int64_t m = L.m, n = L.n;
    Inst I;
    init_inst(L, ws, pb.cost.scale, prm, tol, I);
    I.wt = (plan_bytes(L) <= kWtMaxBytes ? 1 : 0) | (plan_bytes(L) >= kWtMinWideBytes ? 2 : 0);
    NA_TRY(launch_zero(ws, L.bytes, s));
    NA_TRY(hipMemcpyAsync((void *)I.f, pb.f, sizeof(double) * m, hipMemcpyDefault, s));
    NA_TRY(hipMemcpyAsync((void *)I.g, pb.g, sizeof(double) * n, hipMemcpyDefault, s));
    if (L.dim) {
        NA_TRY(hipMemcpyAsync((void *)I.xs, pb.cost.x, sizeof(double) * m * L.dim, hipMemcpyDefault, s));
        NA_TRY(hipMemcpyAsync((void *)I.ys, pb.cost.y, sizeof(double) * n * L.dim, hipMemcpyDefault, s));
    }
    if (L.stored) {
        int kind = C_STORED;
        const double *src = nullptr;
        int64_t ldc = 0;
        bool staged = false;
        if (pb.cost.kind == OT_COST_DENSE) {
            if (is_device_ptr(pb.cost.C)) {
                src = pb.cost.C;
                ldc = pb.cost.ldc;
            } else {
                // a host cost goes through the plan buffers (five contiguous m_alloc x ld
                // blocks, at least m x n doubles), which are cleared again afterwards
                NA_TRY(hipMemcpy2DAsync(I.X[0], sizeof(double) * n, pb.cost.C, sizeof(double) * pb.cost.ldc,
                                        sizeof(double) * n, m, hipMemcpyHostToDevice, s));
                src = (const double *)I.X[0];
                ldc = n;
                staged = true;
            }
        } else if (is_grid(pb.cost.kind)) {
            kind = (int)pb.cost.kind;
        } else {
            kind = pb.cost.kind == OT_COST_POINTS_SQEUCLID ? C_PTS_SQ : C_PTS_EU;
        }
        NA_TRY(launch_materialize(L.fp32, (void *)I.C, m, n, L.ld, kind, src, ldc, I.xs, I.ys, L.dim, L.side,
                                  pb.cost.scale, s));
        if (staged) NA_TRY(launch_zero(I.X[0], (size_t)kBufs * (L.off_X[1] - L.off_X[0]), s));
    }
    Ctl c;
    init_ctl(L, prm, tol, c);
    NA_TRY(hipMemcpyAsync(I.ctl, &c, sizeof(Ctl), hipMemcpyHostToDevice, s));
    NA_TRY(hipMemcpyAsync(d_inst, &I, sizeof(Inst), hipMemcpyHostToDevice, s));
    NA_TRY(launch_tables(tiles, L.ntiles, L.ncb, combs, m, n, counts, s));
    NA_TRY(hipStreamSynchronize(s));   // host sources above are on this stack frame

    // blocks of slots of about 8 ms, as ot_solve runs a fixed set
    const double slot_s = (double)m * (double)L.ld * (double)L.es * 5.0 / 5e12 + 15e-6;
    int slots = (int)(8e-3 / slot_s);
    slots = slots < 4 ? 4 : (slots > 512 ? 512 : slots);
    const double res_slot_s = 4e-6 + (double)m * (double)L.ld * (double)L.es * 5.0 / 50e9;
    int budget = (int)(8e-3 / res_slot_s);
    budget = budget < 16 ? 16 : (budget > 4096 ? 4096 : budget);
    const int grid_t = L.ntiles < kMaxGrid ? L.ntiles : kMaxGrid;
    const int grid_c = L.ncomb < kMaxGrid ? L.ncomb : kMaxGrid;
    const int64_t max_slots = 3 * (prm.max_passes > 1 ? prm.max_passes : 1) + 64;
    int64_t slots_run = 0;
    bool stop_sent = false;
    for (;;) {
        if (L.resident) {
            NA_TRY(launch_resident(L.fp32, L.vec, L.cost, d_inst, counts + 3, counts + 2, 1, budget, s));
            slots_run += budget;
        } else {
            for (int k = 0; k < slots; ++k) {
                NA_TRY(launch_pass(L.fp32, L.vec, L.cost, d_inst, I.ctl, tiles, counts, grid_t, s));
                NA_TRY(launch_combine(d_inst, I.ctl, combs, counts + 1, grid_c, s));
            }
            slots_run += slots;
        }
        NA_TRY(hipMemcpyAsync(&c, I.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
        NA_TRY(hipStreamSynchronize(s));
        if (c.mode == M_IDLE) break;
        if (slots_run > max_slots) return fail(OT_ERR_DEVICE, "solver did not reach a final state");
        if (!stop_sent && prm.time_limit_s > 0.0 && seconds_now() - t0 >= prm.time_limit_s) {
            const int32_t one = 1;
            NA_TRY(hipMemcpyAsync((char *)I.ctl + offsetof(Ctl, stop), &one, sizeof(one), hipMemcpyHostToDevice, s));
            NA_TRY(hipStreamSynchronize(s));
            stop_sent = true;
        }
    }

    const ot_status st = c.status < 0 ? OT_ERR_DEVICE : (ot_status)c.status;
    if (st == OT_OK || st == OT_NOT_CONVERGED) {
        if (pb.X_out)
            NA_TRY(hipMemcpy2DAsync(pb.X_out, L.n * L.es, I.X[c.ret_x], L.ld * L.es, L.n * L.es, L.m,
                                    hipMemcpyDefault, s));
        const double *pr = c.ret_avg ? I.pb[c.pbv] : I.p[c.pv];
        const double *qr = c.ret_avg ? I.qb[c.pbv] : I.q[c.pv];
        if (pb.u_out) NA_TRY(hipMemcpyAsync(pb.u_out, pr, sizeof(double) * m, hipMemcpyDefault, s));
        if (pb.v_out) NA_TRY(hipMemcpyAsync(pb.v_out, qr, sizeof(double) * n, hipMemcpyDefault, s));
        const int64_t nt = c.ntrace < L.trace_cap ? c.ntrace : L.trace_cap;
        if (nt > 0)
            NA_TRY(hipMemcpyAsync(pb.trace, I.trace, sizeof(TraceRec) * (size_t)nt, hipMemcpyDefault, s));
        NA_TRY(hipStreamSynchronize(s));
    }
    if (res) {
        fill_result(L, c, st, *res);
        res->seconds = seconds_now() - t0;
    }
    if (st == OT_OK) fail(OT_OK, "");
    else if (st == OT_NOT_CONVERGED) fail(st, "iteration, pass or time limit reached, or the final verification failed");
    else if (st == OT_ERR_NUMERIC) fail(st, "numerical failure (NaN/Inf in KKT or step scalars)");
    else fail(st, "solver did not reach a final state");
    return st;
}

}  // namespace
}  // namespace pdot

extern "C" ot_status ot_solve_noalloc(const ot_problem *prob, const ot_params *prm, ot_result *res,
                                      void *stream)
{
    if (!prob || !prm) return pdot::fail(OT_ERR_INVALID, "null argument");
    return pdot::solve_noalloc(*prob, *prm, res, (hipStream_t)stream);
}
