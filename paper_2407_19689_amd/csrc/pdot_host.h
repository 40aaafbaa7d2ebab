// Host-side pieces shared by the runtime (pdot_runtime.cpp) and the no-allocation entry
// point (pdot_noalloc.hip): kernel launchers, the per-instance workspace layout, parameter
// checks and the filling of results.  Not part of the public ABI (include/pdot.h is).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "pdot.h"
#include "pdot_internal.h"

namespace pdot {

// ---- kernel launchers (pdot_kernels.hip)
// ctls: the control blocks, indexed like the instance table (the control block of the
// instance in slot k is ctls[k]; Inst::ctl points to it)
hipError_t launch_pass(int fp32, int vec, int cost, const Inst *insts, const Ctl *ctls, const Tile *tiles,
                       const int32_t *ntiles, int grid, hipStream_t s, hipEvent_t ev0 = nullptr,
                       hipEvent_t ev1 = nullptr);
hipError_t launch_combine(const Inst *insts, Ctl *ctls, const CombEntry *ents, const int32_t *nents, int grid,
                          hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_resident(int fp32, int vec, int cost, const Inst *insts, const int32_t *list,
                           const int32_t *count, int grid, int32_t budget, hipStream_t s,
                           hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_materialize(int fp32, void *dst, int64_t m, int64_t n, int64_t ld, int kind,
                              const double *src, int64_t ldc, const double *xs, const double *ys,
                              int dim, int side, double scale, hipStream_t s);
hipError_t launch_round(int cost, const Inst *inst, int ntiles, double *xfeas, hipStream_t s);
hipError_t launch_widen(const float *src, int64_t m, int64_t n, double *dst, int64_t ld, hipStream_t s);
// Zero `bytes` (a multiple of 8) at a 256-byte aligned device address (a kernel, not a
// memset node, so that it behaves alike inside and outside graph capture).
hipError_t launch_zero(void *dst, size_t bytes, hipStream_t s);
// Tile table (row block, column band of every tile, in row-major order), combine table
// (row slices, then column slices) and the two counts of one instance in slot 0.
hipError_t launch_tables(Tile *tiles, int ntiles, int ncb, CombEntry *combs, int64_t m, int64_t n,
                         int32_t *counts, hipStream_t s);

// ---- sizes and limits
constexpr size_t kAlign = 256;
constexpr int kMaxGrid = 4096;   // work-groups of a streaming or combine launch at most
// Instances that run on the whole GPU are split by size into lanes; each lane has its own
// graph and stream, so small instances keep their short slots while large ones run.
constexpr int kLanes = 3;
constexpr int64_t kLaneMax[kLanes - 1] = {(int64_t)1 << 18, (int64_t)1 << 24};   // plan entries
enum { ST_RUNNING = -1 };

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// ---- per-instance layout of one workspace
struct Layout {
    int64_t m = 0, n = 0, ld = 0, m_alloc = 0;
    int fp32 = 1, vec = 4, rows = 64, ncb = 0, nrb = 0, ntiles = 0, ncomb = 0;
    int cost = C_STORED, dim = 0, side = 0;
    bool stored = true;
    bool resident = false;    // one work-group runs the whole instance
    int lane = 0;             // size lane (instances on the whole GPU)
    size_t es = 4;
    size_t off_X[kBufs] = {}, off_C = 0, off_xs = 0, off_ys = 0, off_f = 0, off_g = 0;
    size_t off_rowv = 0, off_colv = 0, off_rowpart = 0, off_colpart = 0;
    size_t off_tiles = 0, off_comb = 0, off_counter = 0, off_ctl = 0, off_trace = 0;
    int64_t trace_cap = 0;
    size_t bytes = 0;
};

// Set the calling thread's ot_last_error message and return st (no allocation).
ot_status fail(ot_status st, const char *msg);
ot_status fail(ot_status st, const std::string &msg);

ot_status plan_instance(const ot_problem &pb, const ot_params &prm, Layout &L);
Prm device_params(const ot_params &p, double tol);
ot_status check_params(const ot_params &prm);
bool is_device_ptr(const void *p);
// Descriptor of an instance whose workspace starts at `base` (device address).
void init_inst(const Layout &l, char *base, double scale, const ot_params &prm, double tol, Inst &I);
// Bytes of one m x n plan buffer of the instance.
int64_t plan_bytes(const Layout &l);
// Control block of an instance before its first slot.
void init_ctl(const Layout &l, const ot_params &prm, double tol, Ctl &c);
// Result of a finished instance from its final control block (st: its status).
void fill_result(const Layout &l, const Ctl &c, ot_status st, ot_result &o);

}  // namespace pdot
