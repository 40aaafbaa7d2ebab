// Internal layout shared by the HIP kernels and the host runtime of the PDHG optimal
// transport library.  Not part of the public ABI (include/pdot.h is).
//
// One iteration "slot" is two launches: the streaming pass kernel over the m x n tiles of
// every running instance, then the combine kernel over row and column slices, whose last
// work-group per instance runs the scalar control of Section 5 (restart candidate,
// restart conditions, step-size check, primal weight, termination) and writes the mode of
// the next slot into the instance's device-resident control block.  Kernels of a slot
// whose instance is idle return at once, so a graph of many slots needs no host sync.
#pragma once
#include <stdint.h>

namespace pdot {

// What the next pass/combine pair does for an instance.
enum Mode : int32_t {
    M_IDLE = 0,     // finished (or never started): both kernels return immediately
    M_INIT = 1,     // KKT of the start point: ||C||_F and ||[-C]^+||_F, ||[f;g]||
    M_TRIAL = 2,    // step trial from the current point (first step of an epoch or retry)
    M_FULL = 3,     // fold the newly accepted iterate into the average, KKT of current and
                    // average, restart/termination checks, and a speculative trial step
    M_RESTART = 4,  // distance of the restart point to the previous one (primal weight)
    M_VERIFY = 5,   // exact KKT and objective of the returned triple
    M_FOLD = 6      // fold the current iterate into the stored average (before a restart
                    // to the average, or before returning it, when the fold is pending)
};
constexpr int kModes = 7;

enum CostKind : int32_t {
    C_STORED = 0, C_PTS_SQ = 1, C_PTS_EU = 2, C_GRID_SQ = 3, C_GRID_L1 = 4, C_GRID_L2 = 5, C_GRID_LINF = 6
};
constexpr bool is_grid(int c) { return c >= C_GRID_SQ && c <= C_GRID_LINF; }

// Roles of the five m x ld plan buffers.  The trial buffer is never the current, the
// average, the next average or the restart anchor, so a role swap replaces every copy.
// The stored average lags: a pass that starts from an iterate not yet in the average
// folds it and the trial it produces (both are in registers) into the next-average
// buffer, and the pass after an accepted trial leaves the average alone, so the average
// is read and written every other pass.
enum Role : int32_t { R_CUR = 0, R_TRIAL = 1, R_AVG = 2, R_ANCHOR = 3, R_AVGN = 4 };
constexpr int kBufs = 5;

constexpr int kWG = 256;          // threads per work-group (4 wave64)
constexpr int kCombEntries = 64;  // rows or columns handled by one combine work-group
constexpr int kNS = 6;            // per-tile scalars
constexpr int kNC = 8;            // per-combine-entry scalars
constexpr int kNB = kNC + kNS;
constexpr int64_t kWtMaxBytes = (int64_t)8 << 20;         // narrow write-through: plans together
constexpr int64_t kWtMinWideBytes = (int64_t)128 << 20;   // wide write-through: one plan    // combine record: entry scalars, then its share of tile scalars

// scalars of the rounding passes (in combscal of the rounding instance)
enum { RD_MARG = 0, RD_L1 = 1, RD_UPPER = 2, RD_CHANGE = 3, RD_LOWER = 4, RD_VIOL = 5 };

// tile scalar slots (TS_AUX: ||C||_F^2 at the start point, the squared distance of the restart
// pass, and <C, next average> in a pass that folds two iterates)
enum { TS_DX2 = 0, TS_DRES = 1, TS_DRESB = 2, TS_POBJ = 3, TS_POBJB = 4, TS_AUX = 5 };
// combine scalar slots
enum { CS_PRES = 0, CS_DOBJ = 1, CS_PRESB = 2, CS_DOBJB = 3, CS_DY2 = 4, CS_INTER = 5,
       CS_AUX = 6, CS_SPARE = 7 };

struct Prm {
    double tol;
    int64_t max_iters, max_passes;
    int32_t kkt_mode, step_rule, restart_rule, avg_weighting;
    int32_t pwu, output, verify_retries, pad1;
    double beta_suff, beta_nec, beta_art, beta_basic;
    double theta, eps_zero, red_exp, grow_exp;
};

// Device-resident control block of one instance (written only by the combine kernel's
// last work-group, or by the host between graph launches).
struct Ctl {
    int32_t mode, status;
    int32_t xr[kBufs];      // role -> physical plan buffer
    int32_t pv, pbv, rsv;   // current version of p/q, of the averaged p/q, of the sums
    int32_t lag;            // the current iterate is not yet folded into the stored average
    int32_t pending;        // after an M_FOLD pass: M_RESTART or M_VERIFY
    int32_t cand_avg;       // last restart candidate is the average
    int32_t ret_x, ret_avg; // returned plan buffer / returned duals are the averages
    int32_t stop;           // host request: stop at the next decision point
    int32_t verify_fails;   // final verifications that did not confirm the tolerance
    int64_t T, k, passes, restarts, kpasses;
    int64_t mcount[kModes]; // slots executed per mode (index: Mode)
    int64_t fold2;          // trial passes that also folded two iterates into the average
    double eta, omega, wsum, a_fold;
    double tol_eff;         // internal termination threshold (tightened on a failed verify)
    double K_start, K_prev, K_cand;
    double norm_b, norm_c;
    double r_obj, r_dobj, r_relP, r_relD, r_relG, r_kkt;
    double e_rel[3], e_obj;  // running estimate of the candidate (rel_P, rel_D, rel_G, <C,X>)
    double pobjb;           // <C, Xbar> of the stored average when it holds the current
                            // iterate (computed by the pass that wrote it, before rounding)
    int64_t ntrace;         // control records written to the instance's trace buffer
    int64_t tr_pass;        // accepted trial awaiting its record: its pass number, the
    double tr_eta, tr_eta_bar;   // step it used and the step bound it met
};

// One control record (the layout of ot_trace_rec in the public header): a rejected trial,
// or an accepted iteration with its KKT values, candidate and restart decision.
struct TraceRec {
    int64_t pass, iter;
    int32_t accepted, restart, cand_avg, pad;
    double eta_used, eta_bar, k_cur, k_avg, omega;
};

struct Inst {
    int64_t m, n, ld;       // ld: row stride (elements) of every m x n buffer
    int64_t m_alloc;        // rows allocated for plan/cost buffers: m rounded up to 16
    int32_t cost, dim, side, vec;
    int32_t rows, ncb, nrb, ntiles;
    int32_t ncomb;
    int32_t wt;             // write-through plan stores: 1 narrow lanes of a solve whose plans
                            // fit kWtMaxBytes, 2 wide lanes of a plan of kWtMinWideBytes or more
    double scale;
    void *X[kBufs];
    const void *C;          // stored cost in the working precision (C_STORED)
    const double *xs, *ys;  // coordinates (points kinds)
    const double *f, *g;
    double *p[2], *q[2], *pb[2], *qb[2];
    double *pa, *qa;
    double *rs[2], *cs[2];
    double *rsb, *csb;
    double *rowpart;        // [ncb][m]  row sums of each column band
    double *colpart;        // [nrb][n]  column sums of each row block
    double *tilescal;       // [ntiles][kNS]
    double *combscal;       // [2][ncomb][kNB]: combine records of even and odd slots
    uint32_t *counter;
    Ctl *ctl;
    TraceRec *trace;        // nullable: control records of the solve
    int64_t trace_cap;
    Prm prm;
};

struct Tile {
    int32_t inst, rb, cb, local;
};

struct CombEntry {
    int32_t inst, kind, start, local;  // kind 0: rows [start, start+64), 1: columns
};

}  // namespace pdot
