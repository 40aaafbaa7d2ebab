// HIP kernels (gfx950) of restarted PDHG for discrete optimal transport.
//
// Paper: Lu & Yang, "PDOT" (arXiv 2407.19689).  Algorithm 2 (alg:rpd) gives the
// iteration in matrix form; Section 3.1 the matrix-free products A vec(X) = [X1; X^T 1]
// and A^T [p;q] = p1^T + 1q^T and the KKT error; Section 5 the restart candidate, the
// three restart conditions, the step-size rule with tau = eta/omega, sigma = eta*omega and
// the primal-weight update; Section 5.1 the relative-KKT termination.
//
// k_pass streams the plan once per slot.  A tile is `rows` rows by 64*VEC columns; each
// lane owns VEC adjacent columns for the whole tile and the four waves of the work-group
// take interleaved rows.  Per element the kernel evaluates (FP64 arithmetic, FP32 or FP64
// storage):
//   gradient   G_ij = C_ij - p_i - q_j
//   trial      X+_ij = max(0, X_ij - tau G_ij)                    (primal step, Algorithm 2)
//   sums       X+ 1, (X+ - X) 1, X+^T 1, (X+ - X)^T 1            (matrix-free A, Section 3.1)
//   step norm  ||X+ - X||_F^2                                     (step-size rule, Section 5)
//   average    Xbar <- (1-a) Xbar + a X                           (Algorithm 2, last update)
//              every other pass, for the start iterate and then for the trial (two folds
//              in registers, one store)
//   KKT parts  ||[p_i+q_j-C_ij]^+||^2 for (p,q) and (pbar,qbar), <C,X>, <C,Xbar>
// Row sums are wave reductions; column sums stay in registers over the tile's rows, are
// combined across the four waves in LDS and written as one partial row per tile; k_combine
// adds the partials in a fixed order (deterministic, no floating-point atomics).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "pdot_internal.h"

// Rows each wave keeps in flight per loop step, for FP32 and FP64 plans: passes that
// stream one plan (and the cost), and passes that stream two plans (a fold into the
// average, the restart distance).
#ifndef PDOT_RU_F32
#define PDOT_RU_F32 2
#endif
#ifndef PDOT_RU_F64
#define PDOT_RU_F64 2
#endif
#ifndef PDOT_RU_F32_AVG
#define PDOT_RU_F32_AVG 1
#endif
#ifndef PDOT_RU_F64_AVG
#define PDOT_RU_F64_AVG 1
#endif
// Rows each wave keeps in flight in the resident kernel (one work-group per instance has
// few waves, so each needs more rows in flight).
#ifndef PDOT_RU_RES
#define PDOT_RU_RES 2
#endif
// Row ranges of tiles are multiples of 16 rows and the four waves step through them 4*RU
// rows at a time, so RU must divide 4.
#define PDOT_RU_OK(r) ((r) == 1 || (r) == 2 || (r) == 4)
static_assert(PDOT_RU_OK(PDOT_RU_F32) && PDOT_RU_OK(PDOT_RU_F64) && PDOT_RU_OK(PDOT_RU_F32_AVG) &&
                  PDOT_RU_OK(PDOT_RU_F64_AVG) && PDOT_RU_OK(PDOT_RU_RES),
              "rows in flight must divide 4");
// Loop steps of rows whose loads are in flight while a step is computed (register sets
// in the ring: this plus one).
#ifndef PDOT_PF
#define PDOT_PF 1
#endif
#ifndef PDOT_PF_AVG
#define PDOT_PF_AVG 1
#endif
static_assert(PDOT_PF >= 1 && PDOT_PF <= 3 && PDOT_PF_AVG >= 1 && PDOT_PF_AVG <= 3, "prefetch depth 1..3");
// Waves per SIMD the streaming kernel is compiled for (bounds its registers).
#ifndef PDOT_PASS_WAVES
#define PDOT_PASS_WAVES 2
#endif
#ifndef PDOT_NT_STORES
#define PDOT_NT_STORES 1
#endif
#ifndef PDOT_NT_LOADS
#define PDOT_NT_LOADS 1
#endif
#ifndef PDOT_NT_LOADS_F64
#define PDOT_NT_LOADS_F64 0
#endif

namespace pdot {

// ------------------------------------------------------------------ small helpers

// Every buffer lives in device global memory.  Pointers read out of the instance table
// are generic pointers; qualifying them as global lets the compiler use global (not flat)
// memory instructions, whose completion counters do not serialise against scalar loads.
// The instance and tile tables (and, inside the streaming kernel, the control blocks) do
// not change while a kernel runs; reading them through the constant address space lets
// the compiler use scalar loads into SGPRs instead of vector loads into VGPRs.
// (The host compilation pass of this file only type-checks kernels; it gets no qualifier.)
#if defined(__HIP_DEVICE_COMPILE__)
#define PDOT_GLOBAL __attribute__((address_space(1)))
#define PDOT_CONST __attribute__((address_space(4)))
#else
#define PDOT_GLOBAL
#define PDOT_CONST
#endif

template <typename T>
__device__ __forceinline__ PDOT_GLOBAL T *gp(T *p)
{
    return (PDOT_GLOBAL T *)p;
}

template <typename T>
__device__ __forceinline__ const PDOT_CONST T *cp(const T *p)
{
    return (const PDOT_CONST T *)p;
}

template <typename T, int N>
struct alignas(sizeof(T) * N) Pack {
    T v[N];
};

template <typename T, int N>
__device__ __forceinline__ void load_pack(const PDOT_GLOBAL T *__restrict__ p, T (&o)[N])
{
    const Pack<T, N> t = *reinterpret_cast<const PDOT_GLOBAL Pack<T, N> *>(p);
#pragma unroll
    for (int i = 0; i < N; ++i) o[i] = t.v[i];
}

template <typename T, int N>
__device__ __forceinline__ void store_pack(PDOT_GLOBAL T *__restrict__ p, const T (&o)[N])
{
    Pack<T, N> t;
#pragma unroll
    for (int i = 0; i < N; ++i) t.v[i] = o[i];
    *reinterpret_cast<PDOT_GLOBAL Pack<T, N> *>(p) = t;
}

// Squared distance of two points (dim <= 3), summed over coordinates in index order with
// every product and sum rounded separately (the same value wherever it is evaluated).
// The coordinate loop is unrolled with a predicate, so register arrays are indexed by
// constants only and stay in registers.
template <typename P1, typename P2>
__device__ __forceinline__ double sqdist(P1 xi, P2 yj, int dim)
{
#pragma clang fp contract(off)
    double t = xi[0] - yj[0];
    double s = t * t;
#pragma unroll
    for (int k = 1; k < 3; ++k) {
        if (k < dim) {
            t = xi[k] - yj[k];
            s = s + t * t;
        }
    }
    return s;
}

// Costs are evaluated in the working precision TX and widened to FP64; the materialising
// kernel calls the same functions, so stored and regenerated costs are bit-identical.
// Points kinds: the squared distance of the FP64 coordinates in FP64 (exact differences,
// each product and sum rounded once); an FP32 plan then rounds it to FP32 once, and the
// Euclidean kind takes the square root of that FP32 value in FP32, so the FP32 form pays
// no FP64 square root per entry (the cost stays within an FP32 ulp or two of the FP64
// distance, the rounding the FP32 cost stream has anyway).
template <typename TX, int COST, typename P1, typename P2>
__device__ __forceinline__ double point_cost(P1 xi, P2 yj, int dim)
{
    const double s2 = sqdist(xi, yj, dim);
    if constexpr (sizeof(TX) == 8) {
        return COST == C_PTS_EU ? sqrt(s2) : s2;
    } else {
        const float s = (float)s2;
        return (double)(COST == C_PTS_EU ? sqrtf(s) : s);
    }
}

// Grid kinds, C_ij = scale * d(pixel_i, pixel_j) for pixels (a, b), with d the squared
// Euclidean, l1, l2 or l-infinity distance.  The coordinates are small integers held
// exactly in floats.  FP64: the integer distance exact, then the square root (l2) and the
// product by scale each rounded once, in numpy's order (the oracle's value).  FP32: the
// same steps in FP32 with scale rounded to FP32.
template <typename TX, int COST>
__device__ __forceinline__ double grid_cost(float ia, float ib, float ja, float jb, double scale,
                                            float scale32)
{
#pragma clang fp contract(off)
    if constexpr (sizeof(TX) == 8) {
        const double da = (double)ia - (double)ja, db = (double)ib - (double)jb;
        if constexpr (COST == C_GRID_SQ) return (da * da + db * db) * scale;
        else if constexpr (COST == C_GRID_L1) return (fabs(da) + fabs(db)) * scale;
        else if constexpr (COST == C_GRID_L2) return sqrt(da * da + db * db) * scale;
        else return fmax(fabs(da), fabs(db)) * scale;
    } else {
        const float da = ia - ja, db = ib - jb;
        float d;
        if constexpr (COST == C_GRID_SQ) d = da * da + db * db;   // exact: an integer below 2^24
        else if constexpr (COST == C_GRID_L1) d = fabsf(da) + fabsf(db);
        else if constexpr (COST == C_GRID_L2) d = sqrtf(da * da + db * db);
        else d = fmaxf(fabsf(da), fabsf(db));
        return (double)(d * scale32);
    }
}

// 32-bit integer mixer "lowbias32" (C. Wellons, hash-prospector): a bijection on 32-bit
// words with low avalanche bias.  Used as a counter-based generator for the rounding below.
__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

// Store of the running average.  FP64 storage keeps the value.  FP32 storage rounds
// stochastically: for v >= 0 the 29 FP64 mantissa bits that FP32 drops are incremented by
// 29 random bits and then cleared, so v is stored as its upper FP32 neighbour with
// probability (v - lo)/(hi - lo) and as the lower one otherwise (exact in the FP32 normal
// range).  Round-to-nearest would drop every fold increment below half an ulp, a bias that
// grows linearly with the epoch length; the stochastic store is unbiased.
template <typename TX>
__device__ __forceinline__ TX store_avg(double v, uint32_t h);

template <>
__device__ __forceinline__ double store_avg<double>(double v, uint32_t)
{
    return v;
}

template <>
__device__ __forceinline__ float store_avg<float>(double v, uint32_t h)
{
    uint64_t b = (uint64_t)__double_as_longlong(v);
    b += (uint64_t)(h >> 3);
    b &= ~(uint64_t)0x1FFFFFFFu;
    return (float)__longlong_as_double((long long)b);
}

// Move of a 64-bit value between lanes with a DPP pattern (two 32-bit moves); lanes whose
// source is outside the pattern, or whose row is masked off, read 0.
template <int CTRL, int ROW_MASK, bool BOUND_ZERO>
__device__ __forceinline__ double dpp64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xF, BOUND_ZERO);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xF, BOUND_ZERO);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes with DPP moves: a scan inside each row of 16 lanes (shifts 1, 2,
// 4, 8), then the row totals are carried across rows with the row broadcasts of lanes 15
// and 31.  The total is in lane 63; the combination order is fixed.
__device__ __forceinline__ double wave_sum_to63(double v)
{
    v += dpp64<0x111, 0xF, true>(v);   // row_shr:1
    v += dpp64<0x112, 0xF, true>(v);   // row_shr:2
    v += dpp64<0x114, 0xF, true>(v);   // row_shr:4
    v += dpp64<0x118, 0xF, true>(v);   // row_shr:8
    v += dpp64<0x142, 0xA, false>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp64<0x143, 0xC, false>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// ------------------------------------------------------------------ streaming pass

// Store of VEC plan entries: non-temporal vector stores (16-byte pieces) by default; the
// plan and the average are written once per pass and read back only by the next pass.
// Two write-through forms (Inst::wt), which leave no dirty plan lines in the chiplet's L2:
//  * WT_NARROW, solves whose plans together fit kWtMaxBytes, on lanes of under 16 bytes:
//    agent-scope word stores, so the release at the end of the pass has nothing to write
//    back (at 1024 x 1024 an FP32 pass went from 7.8 to 6.9 us, FP64 from 8.9 to 7.7 us).
//    On plans beyond the caches word stores halve the stream rate (at 8100 x 8100, 4.6
//    against 2.3 TB/s), hence the limit.
//  * WT_WIDE, plans of at least kWtMinWideBytes (beyond the Infinity Cache), on 16-byte
//    lanes: buffer stores with the device-scope and non-temporal bits (the buffer
//    descriptor's base is the row's first entry, uniform across the wave), 4.75 against
//    4.48 TB/s at 8100 x 8100.  On plans the Infinity Cache still holds they cost a third
//    of the rate (at 4096 x 4096, 46 against 34 us per pass), hence the floor.
enum { WT_NARROW = 1, WT_WIDE = 2 };
template <typename T, int N>
__device__ __forceinline__ void store_pack_nt(PDOT_GLOBAL T *__restrict__ p, const T (&o)[N], int wt)
{
    if constexpr (sizeof(T) * N < 16) {
        if (wt & WT_NARROW) {
            if constexpr (sizeof(T) * N == 8) {
                uint64_t w;
                __builtin_memcpy(&w, o, 8);
                __hip_atomic_store(reinterpret_cast<PDOT_GLOBAL uint64_t *>(p), w, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            } else {
#pragma unroll
                for (int e = 0; e < N; ++e)
                    __hip_atomic_store(p + e, o[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            return;
        }
    }
    if constexpr (!PDOT_NT_STORES) {
        store_pack<T, N>(p, o);
    } else if constexpr (sizeof(T) * N >= 16) {
        constexpr int E = 16 / sizeof(T);   // entries per 16-byte piece
        typedef T V __attribute__((ext_vector_type(E)));
        if (wt & WT_WIDE) {
            typedef unsigned int U4 __attribute__((ext_vector_type(4)));
            // the lanes of a wave store one row of the tile: descriptor base = its first
            // entry (the same for every lane), bounds = the row's 64 * N entries
            const int ln = threadIdx.x & 63;
            const uint64_t a = (uint64_t)(uintptr_t)(p - ln * N);
            const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
            const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(uintptr_t)(((uint64_t)hi << 32) | lo), (short)0, 64 * N * (int)sizeof(T), 0x00020000);
#pragma unroll
            for (int c = 0; c < N / E; ++c) {
                V v;
#pragma unroll
                for (int e = 0; e < E; ++e) v[e] = o[c * E + e];
                U4 u;
                __builtin_memcpy(&u, &v, 16);
                __builtin_amdgcn_raw_buffer_store_b128(u, rs, (ln * N + c * E) * (int)sizeof(T), 0,
                                                       16 /* device scope */ | 2 /* non-temporal */);
            }
            return;
        }
#pragma unroll
        for (int c = 0; c < N / E; ++c) {
            V v;
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = o[c * E + e];
            __builtin_nontemporal_store(v, reinterpret_cast<PDOT_GLOBAL V *>(p) + c);
        }
    } else {
#pragma unroll
        for (int e = 0; e < N; ++e) __builtin_nontemporal_store(o[e], p + e);
    }
}

// Non-temporal vector load of VEC plan entries: in the trial and fold passes the plan and
// the average are read for the last time (the next pass reads what this one writes).
// Measured on FP32 plans 4.6 % faster at 4096 x 4096; on FP64 plans, whose passes do not
// fit the Infinity Cache, ordinary loads were 2-7 % faster, so those keep them.
template <typename T, int N>
__device__ __forceinline__ void load_pack_nt(const PDOT_GLOBAL T *__restrict__ p, T (&o)[N])
{
    if constexpr (!PDOT_NT_LOADS || (sizeof(T) == 8 && !PDOT_NT_LOADS_F64)) {
        load_pack<T, N>(p, o);
    } else {
        constexpr int B = sizeof(T) * N < 16 ? (int)sizeof(T) * N : 16;   // bytes per piece
        constexpr int E = B / (int)sizeof(T);                            // entries per piece
        if constexpr (E == 1) {
#pragma unroll
            for (int e = 0; e < N; ++e) o[e] = __builtin_nontemporal_load(p + e);
        } else {
            typedef T V __attribute__((ext_vector_type(E)));
#pragma unroll
            for (int c = 0; c < N / E; ++c) {
                const V v = __builtin_nontemporal_load(reinterpret_cast<const PDOT_GLOBAL V *>(p) + c);
#pragma unroll
                for (int e = 0; e < E; ++e) o[c * E + e] = v[e];
            }
        }
    }
}

// Per-row dual of the streaming pass.  In the resident kernel the duals are rewritten by
// other threads of the same work-group between passes, so they are read with vector
// loads (a workgroup-scope atomic load is never turned into a scalar-cache load); in the
// grid kernel they do not change during the launch and may come through the scalar cache.
template <bool RES>
__device__ __forceinline__ double row_dual(const PDOT_GLOBAL double *p, int64_t i)
{
    if constexpr (RES)
        return __hip_atomic_load(p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    else
        return p[i];
}

// One tile of the streaming pass.  Rows are processed RU at a time per wave (wave w takes
// rows i0+w, i0+w+4, ...); the tile's row range is a multiple of 4*RU inside the padded
// allocation, so every row touched exists in memory.  Padding rows (i >= m) use p_i = -inf
// and padding columns (j >= n) q_j = -inf: the gradient is then +inf, the projected step
// is 0 and no residual term is positive, so padding contributes exactly zero without a
// masked code path.  Plan padding is zero and stays zero.  Per-row quantities (row base,
// duals, pixel coordinates, hash) are wave-uniform and live in scalar registers.
// F2 (trial and full passes whose start iterate is not yet in the stored average): fold
// the start iterate and then the trial into the average, in FP64 registers, and store the
// result (the average after the trial, should it be accepted) in the next-average buffer;
// the two folds are the sequential ones, so an FP64 plan gets exactly the running average.
template <typename TX, int VEC, int COST, int MODE, bool RES = false, bool F2 = false>
__device__ void tile_body(const PDOT_CONST Inst &I, const Ctl &st, const Tile &tl, double *lds)
{
    // Every product and sum below is rounded as written (fused multiply-adds only where
    // fma() is spelled out), so all kernel variants (cost source, tile shape) round alike.
#pragma clang fp contract(off)
    constexpr bool kX = MODE != M_INIT;         // reads the plan
    constexpr bool kCost = MODE != M_RESTART && MODE != M_FOLD;   // needs C
    constexpr bool kTrial = MODE == M_TRIAL || MODE == M_FULL;
    constexpr bool kFold2 = kTrial && F2;                  // folds two iterates
    constexpr bool kAvgIn = kFold2 || MODE == M_FOLD;      // reads the stored average
    constexpr bool kTwo = kAvgIn || MODE == M_RESTART;    // streams two plans
    constexpr int RU = RES ? PDOT_RU_RES
                           : (sizeof(TX) == 4 ? (kTwo ? PDOT_RU_F32_AVG : PDOT_RU_F32)
                                              : (kTwo ? PDOT_RU_F64_AVG : PDOT_RU_F64));   // rows in flight per wave
    constexpr bool kAvgOut = kAvgIn;                       // writes the next average
    constexpr bool kAvgKKT = MODE == M_FULL;               // KKT pieces of the average
    constexpr bool kRowCol = kTrial || MODE == M_VERIFY;
    constexpr bool kGrid = is_grid(COST);
    constexpr bool kPts = COST == C_PTS_SQ || COST == C_PTS_EU;
    constexpr double kNegInf = -__builtin_huge_val();

    const int lane = threadIdx.x & 63;
    // wave index as a wave-uniform value, so row indices and per-row data stay scalar
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t m = I.m, n = I.n, ld = I.ld;
    const int wthru = I.wt;   // write-through plan stores (WT_NARROW, WT_WIDE)
    const int64_t i0 = (int64_t)tl.rb * I.rows;
    const int64_t ie = min(I.m_alloc, i0 + (int64_t)I.rows);
    const int64_t jband = (int64_t)tl.cb * (64 * VEC);   // first column of the tile (uniform)
    const uint32_t jl = (uint32_t)lane * VEC;            // lane's first column in the tile
    const int64_t j0 = jband + jl;
    const bool active = j0 < n;   // lanes wholly beyond n touch no memory

    const int xc = (MODE == M_VERIFY) ? st.ret_x : st.xr[R_CUR];
    const PDOT_GLOBAL TX *__restrict__ Xc = gp((const TX *)I.X[xc]);
    PDOT_GLOBAL TX *__restrict__ Xt = gp((TX *)I.X[st.xr[R_TRIAL]]);
    const PDOT_GLOBAL TX *__restrict__ Xb = gp((const TX *)I.X[st.xr[R_AVG]]);
    PDOT_GLOBAL TX *__restrict__ Xn = gp((TX *)I.X[st.xr[R_AVGN]]);
    const PDOT_GLOBAL TX *__restrict__ Xa = gp((const TX *)I.X[st.xr[R_ANCHOR]]);
    const PDOT_GLOBAL TX *__restrict__ Cs = gp((const TX *)I.C);
    const bool use_avg_duals = (MODE == M_VERIFY) && st.ret_avg;
    const PDOT_GLOBAL double *__restrict__ pc = gp(use_avg_duals ? I.pb[st.pbv] : I.p[st.pv]);
    const PDOT_GLOBAL double *__restrict__ qc = gp(use_avg_duals ? I.qb[st.pbv] : I.q[st.pv]);
    const PDOT_GLOBAL double *__restrict__ pbc = gp(I.pb[st.pbv]);
    const PDOT_GLOBAL double *__restrict__ qbc = gp(I.qb[st.pbv]);
    const PDOT_GLOBAL double *__restrict__ xs = gp(I.xs);
    const PDOT_GLOBAL double *__restrict__ ys = gp(I.ys);
    PDOT_GLOBAL double *__restrict__ rowpart = gp(I.rowpart);
    PDOT_GLOBAL double *__restrict__ colpart = gp(I.colpart);
    const double tau = st.eta / st.omega;
    const double a = st.a_fold;   // weight of the start iterate in the average
    const bool first_fold = st.k == 1;
    // weight of the trial in the average, as the control computes it on acceptance
    const double wt = I.prm.avg_weighting == 1 ? 1.0 : st.eta;
    const double a2 = wt / (st.wsum + wt);
    const uint32_t hiter = mix32((uint32_t)st.T * 0x85EBCA77U + 0x27D4EB2FU);
    const double scale = I.scale;
    const float scale32 = (float)I.scale;
    const int dim = I.dim, side = I.side;

    // per-lane column context
    uint32_t hcol[VEC];
    double qv[VEC], qbv[VEC];
    bool colok[VEC];
    float gja[VEC], gjb[VEC];
    double yc[VEC][3];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        const int64_t j = j0 + v;
        const bool ok = j < n;
        const int64_t jc = ok ? j : n - 1;
        colok[v] = ok;
        hcol[v] = mix32((uint32_t)j * 0x9E3779B9U + 0x632BE5ABU);
        qv[v] = ok ? qc[jc] : kNegInf;
        qbv[v] = (ok && kAvgKKT) ? qbc[jc] : kNegInf;
        gja[v] = gjb[v] = 0.0f;
        yc[v][0] = yc[v][1] = yc[v][2] = 0.0;
        if constexpr (kGrid) {
            gja[v] = (float)(int)((uint32_t)jc / (uint32_t)side);
            gjb[v] = (float)(int)((uint32_t)jc % (uint32_t)side);
        }
        if constexpr (kPts) {
#pragma unroll
            for (int k = 0; k < 3; ++k)
                if (k < dim) yc[v][k] = ys[jc * dim + k];
        }
    }

    double csv[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) csv[v] = 0.0;
    double s_dx2 = 0.0, s_dres = 0.0, s_dresb = 0.0, s_pobj = 0.0, s_pobjb = 0.0, s_aux = 0.0;

    // pixel coordinates of this wave's next row to load, advanced by 4 rows at a time
    int ga = 0, gb = 0;
    if constexpr (kGrid) {
        const uint32_t r0 = (uint32_t)(i0 + wave);
        ga = (int)(r0 / (uint32_t)side);
        gb = (int)(r0 % (uint32_t)side);
    }

    // Registers of RU rows: the plan entries and the wave-uniform row data.
    struct Rows {
        TX x[RU][VEC], c[RU][VEC], b[RU][VEC], an[RU][VEC];
        double pi[RU], pbi[RU];
        double xi[RU][3];
        float gia[RU], gib[RU];
    };

    auto load_rows = [&](int64_t ib, Rows &R) {
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int64_t i = ib + 4 * u;
            const bool rok = i < m;
            const int64_t ic = rok ? i : m - 1;
            const int64_t rowoff = i * ld + jband;   // uniform row base; lanes add jl
            R.pi[u] = rok ? row_dual<RES>(pc, i) : kNegInf;
            R.pbi[u] = (rok && kAvgKKT) ? row_dual<RES>(pbc, i) : kNegInf;
            R.gia[u] = (float)ga;
            R.gib[u] = (float)gb;
            if constexpr (kGrid) {
                gb += 4;
                while (gb >= side) {
                    gb -= side;
                    ga += 1;
                }
            }
            R.xi[u][0] = R.xi[u][1] = R.xi[u][2] = 0.0;
            if constexpr (kPts) {
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    if (k < dim) R.xi[u][k] = xs[ic * dim + k];
            }
#pragma unroll
            for (int v = 0; v < VEC; ++v) R.x[u][v] = R.c[u][v] = R.b[u][v] = R.an[u][v] = (TX)0;
            if (active) {
                if constexpr (kX) {
                    if constexpr (kTrial || MODE == M_FOLD) load_pack_nt<TX, VEC>(Xc + rowoff + jl, R.x[u]);
                    else load_pack<TX, VEC>(Xc + rowoff + jl, R.x[u]);
                }
                if constexpr (kCost && COST == C_STORED) load_pack<TX, VEC>(Cs + rowoff + jl, R.c[u]);
                if constexpr (kAvgIn) load_pack_nt<TX, VEC>(Xb + rowoff + jl, R.b[u]);
                if constexpr (MODE == M_RESTART) load_pack<TX, VEC>(Xa + rowoff + jl, R.an[u]);
            }
        }
    };

    auto compute_rows = [&](int64_t ib, const Rows &R) {
        double rsum[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            rsum[u] = 0.0;
            const int64_t i = ib + 4 * u;
            const uint32_t hrow = mix32((uint32_t)i ^ hiter);
            TX xn_out[VEC], xb_out[VEC];
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                const double xd = (double)R.x[u][v];
                double cd = 0.0;
                if constexpr (kCost) {
                    if constexpr (COST == C_STORED) {
                        cd = (double)R.c[u][v];
                    } else if constexpr (kGrid) {
                        cd = grid_cost<TX, COST>(R.gia[u], R.gib[u], gja[v], gjb[v], scale, scale32);
                    } else {
                        cd = point_cost<TX, COST>(R.xi[u], yc[v], dim);
                    }
                }
                xn_out[v] = (TX)0;
                xb_out[v] = (TX)0;
                if constexpr (MODE == M_INIT) {
                    const double cm = (colok[v] && i < m) ? cd : 0.0;
                    s_aux = fma(cm, cm, s_aux);
                    const double nd = fmax((R.pi[u] + qv[v]) - cd, 0.0);
                    s_dres = fma(nd, nd, s_dres);
                }
                if constexpr (MODE == M_RESTART) {
                    const double d = xd - (double)R.an[u][v];
                    s_aux = fma(d, d, s_aux);
                }
                if constexpr (MODE == M_VERIFY) {
                    const double nd = fmax((R.pi[u] + qv[v]) - cd, 0.0);
                    s_dres = fma(nd, nd, s_dres);
                    s_pobj = fma(cd, xd, s_pobj);
                    rsum[u] += xd;
                    csv[v] += xd;
                }
                // fold of the start iterate into the running average
                double xbn = 0.0;
                if constexpr (kAvgIn) {
                    const double xbd = (double)R.b[u][v];
                    xbn = first_fold ? xd : fma(a, xd, (1.0 - a) * xbd);
                }
                if constexpr (MODE == M_FOLD) xb_out[v] = store_avg<TX>(xbn, hrow ^ hcol[v]);
                if constexpr (kTrial) {
                    const double sg = R.pi[u] + qv[v];
                    const double gr = cd - sg;                // G_ij = C_ij - p_i - q_j
                    if constexpr (kAvgKKT) {
                        // KKT pieces of the current iterate (its duals are p, q) and of the
                        // average (averaged duals); the averaged objective uses the value
                        // before storage rounding, like the averaged row and column sums
                        // (the final verification measures the stored arrays).  Without F2
                        // the average already holds the current iterate and its objective
                        // came from the pass that wrote it.
                        const double ng = fmin(gr, 0.0);
                        s_dres = fma(ng, ng, s_dres);
                        s_pobj = fma(cd, xd, s_pobj);
                        const double nb = fmax((R.pbi[u] + qbv[v]) - cd, 0.0);
                        s_dresb = fma(nb, nb, s_dresb);
                        if constexpr (kFold2) s_pobjb = fma(cd, xbn, s_pobjb);
                    }
                    const double y = fma(-tau, gr, xd);
                    const TX xn = (TX)fmax(y, 0.0);
                    xn_out[v] = xn;
                    const double xnd = (double)xn;
                    const double d = xnd - xd;
                    rsum[u] += xnd;
                    csv[v] += xnd;
                    s_dx2 = fma(d, d, s_dx2);
                    if constexpr (kFold2) {
                        // second fold: the trial as stored, with its own weight
                        const double xbt = fma(a2, xnd, (1.0 - a2) * xbn);
                        xb_out[v] = store_avg<TX>(xbt, hrow ^ hcol[v]);
                        s_aux = fma(cd, xbt, s_aux);
                    }
                }
            }
            if (active) {
                const int64_t rowoff = i * ld + jband;
                if constexpr (kTrial) store_pack_nt<TX, VEC>(Xt + rowoff + jl, xn_out, wthru);
                if constexpr (kAvgOut) store_pack_nt<TX, VEC>(Xn + rowoff + jl, xb_out, wthru);
            }
            // keep one row's arithmetic together: bounds the live temporaries
            __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (kRowCol) {
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const double sr = wave_sum_to63(rsum[u]);
                const int64_t i = ib + 4 * u;
                if (lane == 63 && i < m) rowpart[(int64_t)tl.cb * m + i] = sr;
            }
        }
    };

    // Software pipeline: the loads of the next PF steps of RU rows are in flight while a
    // step is computed, in a ring of PF + 1 register sets (the ring loop is unrolled, so
    // every set index is a constant).
    constexpr int PF = RES ? 1 : (kTwo ? PDOT_PF_AVG : PDOT_PF);
    constexpr int NS = PF + 1;
    const int64_t step = 4 * RU;
    Rows S[NS];
    int64_t ib = i0 + wave;
#pragma unroll
    for (int s = 0; s < PF; ++s)
        if (ib + s * step < ie) load_rows(ib + s * step, S[s]);
    while (ib < ie) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (ib + PF * step < ie) load_rows(ib + PF * step, S[(s + PF) % NS]);
            __builtin_amdgcn_sched_barrier(0);
            compute_rows(ib, S[s]);
            ib += step;
            if (ib >= ie) break;
        }
    }

    // column partials: combine the four waves in a fixed order
    if constexpr (kRowCol) {
        double *cl = lds;   // [3][VEC][64]
        if (wave > 0) {
#pragma unroll
            for (int v = 0; v < VEC; ++v) cl[((wave - 1) * VEC + v) * 64 + lane] = csv[v];
        }
        __syncthreads();
        if (wave == 0 && active) {
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                double sv = csv[v];
                for (int w = 0; w < 3; ++w) sv += cl[(w * VEC + v) * 64 + lane];
                const int64_t j = j0 + v;
                if (j < n) colpart[(int64_t)tl.rb * n + j] = sv;
            }
        }
        __syncthreads();
    }

    // tile scalars
    {
        double *sl = lds + 3 * 2 * 4 * 64;   // after the largest column area
        double vals[kNS] = {s_dx2, s_dres, s_dresb, s_pobj, s_pobjb, s_aux};
#pragma unroll
        for (int s = 0; s < kNS; ++s) {
            const double r = wave_sum_to63(vals[s]);
            if (lane == 63) sl[wave * kNS + s] = r;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            PDOT_GLOBAL double *dst = gp(I.tilescal) + (int64_t)tl.local * kNS;
            for (int s = 0; s < kNS; ++s)
                dst[s] = ((sl[s] + sl[kNS + s]) + sl[2 * kNS + s]) + sl[3 * kNS + s];
        }
        __syncthreads();
    }
}

// The tile count is read from device memory, so a captured graph stays valid when the
// host repacks the tile table between launches (instances joining or finishing).
template <typename TX, int VEC, int COST>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(PDOT_PASS_WAVES)))
void k_pass(const Inst *__restrict__ insts, const Ctl *__restrict__ ctls, const Tile *__restrict__ tiles,
            const int32_t *__restrict__ count)
{
    __shared__ double lds[3 * 2 * 4 * 64 + 4 * kNS];
    // The launch grid never exceeds the tile table's capacity, so the first tile entry is
    // read before the count (both loads in flight); it is used only if it is in the count.
    Tile next = cp(tiles)[blockIdx.x];
    const int ntiles = *cp(count);
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const Tile tl = next;
        if (t + (int)gridDim.x < ntiles) next = cp(tiles)[t + gridDim.x];
        // the descriptor and the control block come from tables indexed by the instance,
        // so both loads are in flight together
        const PDOT_CONST Inst &I = cp(insts)[tl.inst];
        const Ctl st = cp(ctls)[tl.inst];
        switch (st.mode) {
        case M_INIT: tile_body<TX, VEC, COST, M_INIT>(I, st, tl, lds); break;
        case M_TRIAL:
            if (st.lag) tile_body<TX, VEC, COST, M_TRIAL, false, true>(I, st, tl, lds);
            else tile_body<TX, VEC, COST, M_TRIAL>(I, st, tl, lds);
            break;
        case M_FULL:
            if (st.lag) tile_body<TX, VEC, COST, M_FULL, false, true>(I, st, tl, lds);
            else tile_body<TX, VEC, COST, M_FULL>(I, st, tl, lds);
            break;
        case M_RESTART: tile_body<TX, VEC, COST, M_RESTART>(I, st, tl, lds); break;
        case M_VERIFY: tile_body<TX, VEC, COST, M_VERIFY>(I, st, tl, lds); break;
        case M_FOLD: tile_body<TX, VEC, COST, M_FOLD>(I, st, tl, lds); break;
        default: break;
        }
    }
}

// ------------------------------------------------------------------ control (one thread)

// Relative KKT error (Section 3.1 stacked norm, each block over its own scale; kkt_mode 1
// uses 1 + scale denominators).  out = {rel_P, rel_D, rel_G}.
__device__ __forceinline__ double rel_kkt(const Prm &P, double nb, double nc, double pres2, double dres2,
                          double pobj, double dobj, double *out)
{
    const double ap = sqrt(pres2), ad = sqrt(dres2), gap = fabs(pobj - dobj);
    double rp, rd, rg;
    if (P.kkt_mode == 1) {
        rp = ap / (1.0 + nb);
        rd = ad / (1.0 + nc);
        rg = gap / (1.0 + fabs(pobj) + fabs(dobj));
    } else {
        rp = nb > 0.0 ? ap / nb : ap;
        rd = nc > 0.0 ? ad / nc : ad;
        const double den = fabs(pobj) + fabs(dobj);
        rg = den > 0.0 ? gap / den : 0.0;
    }
    if (out) {
        out[0] = rp;
        out[1] = rd;
        out[2] = rg;
    }
    return sqrt(rp * rp + rd * rd + rg * rg);
}

enum { ST_RUNNING = -1, ST_OK = 0, ST_DEVICE = 3, ST_NOT_CONVERGED = 4, ST_NUMERIC = 5 };

__device__ __forceinline__ void finish(Ctl &c, const Prm &P, int status)
{
    c.status = status;
    c.ret_avg = (P.output == 0 && c.cand_avg && c.T > 0 && c.k > 0) ? 1 : 0;
    if (c.ret_avg && c.lag) {   // the average does not hold the current iterate yet
        c.pending = M_VERIFY;
        c.mode = M_FOLD;
        return;
    }
    c.ret_x = c.ret_avg ? c.xr[R_AVG] : c.xr[R_CUR];
    c.mode = M_VERIFY;
}

__device__ __forceinline__ void swap_avg(Ctl &c)
{
    const int t = c.xr[R_AVG];
    c.xr[R_AVG] = c.xr[R_AVGN];
    c.xr[R_AVGN] = t;
}

__device__ __forceinline__ bool limits_hit(const Ctl &c, const Prm &P)
{
    return c.T >= P.max_iters || c.passes >= P.max_passes || c.stop;
}

// Where the control appends its records (null: no trace), and how many fit.
struct TraceOut {
    TraceRec *buf;
    int64_t cap;
};

__device__ __forceinline__ void trace_put(Ctl &c, const TraceOut &to, int64_t pass, int32_t accepted,
                                          int32_t restart, double eta_used, double eta_bar, double kc,
                                          double ka)
{
    if (!to.buf || c.ntrace >= to.cap) return;
    TraceRec r;
    r.pass = pass;
    r.iter = c.T;
    r.accepted = accepted;
    r.restart = restart;
    r.cand_avg = accepted ? c.cand_avg : 0;
    r.pad = 0;
    r.eta_used = eta_used;
    r.eta_bar = eta_bar;
    r.k_cur = kc;
    r.k_avg = ka;
    r.omega = c.omega;
    gp(to.buf)[c.ntrace] = r;
    c.ntrace += 1;
}

// Step-size check of the trial (Section 5, adaptive step size).
// g_red = (T+1)^-a and g_grow = (T+1)^-b are evaluated by the caller (step_factors, on
// other lanes) for the current T.
// aux: <C, next average> of a pass that folded two iterates.
// A rejected trial is traced at once; an accepted one when its KKT values and restart
// decision are known (the next M_FULL control), from the fields kept in tr_*.
__device__ __forceinline__ void step_decide(Ctl &c, const Prm &P, double dx2, double dy2, double inter,
                            double aux, double g_red, double g_grow, const TraceOut &to)
{
    c.passes += 1;
    const double eta_used = c.eta;
    bool accept = true;
    double eta_bar = INFINITY;
    if (P.step_rule == 0) {
        const double num = c.omega * dx2 + dy2 / c.omega;
        const double den = 2.0 * fabs(inter);
        eta_bar = den > 0.0 ? num / den : INFINITY;
        accept = c.eta <= eta_bar;
        const double shrink = (1.0 - g_red) * eta_bar;
        const double grow = (1.0 + g_grow) * c.eta;
        c.eta = shrink < grow ? shrink : grow;
        if (!(num == num) || !(c.eta == c.eta)) {   // NaN guard
            c.status = ST_NUMERIC;
            c.mode = M_IDLE;
            return;
        }
    }
    if (accept) {
        if (c.lag) {
            // the pass folded the current iterate and the trial: the next average is the
            // average of the new current iterate
            swap_avg(c);
            c.pobjb = aux;
            c.lag = 0;
        } else {
            c.lag = 1;
        }
        const int old_cur = c.xr[R_CUR];
        const int new_cur = c.xr[R_TRIAL];
        int nt = old_cur;
        if (old_cur == c.xr[R_ANCHOR]) {
            for (int b = 0; b < kBufs; ++b)
                if (b != new_cur && b != c.xr[R_AVG] && b != c.xr[R_AVGN] && b != c.xr[R_ANCHOR]) nt = b;
        }
        c.xr[R_CUR] = new_cur;
        c.xr[R_TRIAL] = nt;
        c.pv ^= 1;
        c.pbv ^= 1;
        c.rsv ^= 1;
        c.T += 1;
        c.k += 1;
        const double w = P.avg_weighting == 1 ? 1.0 : eta_used;
        c.wsum += w;
        c.a_fold = w / c.wsum;
        c.tr_pass = c.passes;
        c.tr_eta = eta_used;
        c.tr_eta_bar = eta_bar;
        c.mode = M_FULL;
    } else {
        trace_put(c, to, c.passes, 0, 0, eta_used, eta_bar, 0.0, 0.0);
        c.mode = M_TRIAL;
        if (c.passes >= P.max_passes || c.stop) finish(c, P, ST_NOT_CONVERGED);
    }
}

__device__ __forceinline__ void control(Ctl &c, const Prm &P, int mode, const double *cs, const double *ts,
                        double g_red, double g_grow, const TraceOut &to)
{
    // Constant indices only: an array of the control block indexed at run time goes to
    // scratch memory, and its load-add-store would put a memory round trip on the slot's
    // critical path (a switch over the modes is folded back into such an index).
    c.kpasses += 1;
#pragma unroll
    for (int k = M_INIT; k < kModes; ++k) c.mcount[k] += mode == k ? 1 : 0;
    if ((mode == M_TRIAL || mode == M_FULL) && c.lag) c.fold2 += 1;
    if (mode == M_INIT) {
        c.norm_b = sqrt(cs[CS_AUX]);
        c.norm_c = sqrt(ts[TS_AUX]);
        const double K = rel_kkt(P, c.norm_b, c.norm_c, cs[CS_AUX], ts[TS_DRES], 0.0, 0.0, nullptr);
        c.K_start = c.K_prev = c.K_cand = K;
        c.cand_avg = 0;
        if (!(K == K) || !(c.norm_c < INFINITY)) {
            c.status = ST_NUMERIC;
            c.mode = M_IDLE;
        } else if (K <= c.tol_eff) {
            finish(c, P, ST_OK);
        } else if (limits_hit(c, P)) {
            finish(c, P, ST_NOT_CONVERGED);
        } else {
            c.mode = M_TRIAL;
        }
        return;
    }
    if (mode == M_TRIAL) {
        step_decide(c, P, ts[TS_DX2], cs[CS_DY2], cs[CS_INTER], ts[TS_AUX], g_red, g_grow, to);
        return;
    }
    if (mode == M_FULL) {
        double ec[3], ea[3];
        const double kc = rel_kkt(P, c.norm_b, c.norm_c, cs[CS_PRES], ts[TS_DRES], ts[TS_POBJ],
                                  cs[CS_DOBJ], ec);
        // <C, average>: from this pass when it folded the current iterate, else from the
        // pass that wrote the stored average
        const double pobjb = c.lag ? ts[TS_POBJB] : c.pobjb;
        const double ka = rel_kkt(P, c.norm_b, c.norm_c, cs[CS_PRESB], ts[TS_DRESB],
                                  pobjb, cs[CS_DOBJB], ea);
        // restart candidate (Section 5): the current iterate only if strictly better
        c.cand_avg = !(kc < ka);
        for (int q = 0; q < 3; ++q) c.e_rel[q] = c.cand_avg ? ea[q] : ec[q];
        c.e_obj = c.cand_avg ? pobjb : ts[TS_POBJ];
        double K = c.cand_avg ? ka : kc;
        if (!(K == K)) {
            c.status = ST_NUMERIC;
            c.mode = M_IDLE;
            return;
        }
        c.K_cand = K;
        if (K <= c.tol_eff) {
            trace_put(c, to, c.tr_pass, 1, 0, c.tr_eta, c.tr_eta_bar, kc, ka);
            finish(c, P, ST_OK);
            return;
        }
        int restart = 0;
        if (P.restart_rule == 0) {
            if (K <= P.beta_suff * c.K_start) restart = 1;                          // (i)
            else if (K <= P.beta_nec * c.K_start && K > c.K_prev) restart = 2;      // (ii)
            else if ((double)c.k >= P.beta_art * (double)c.T) restart = 3;          // (iii)
        } else if (P.restart_rule == 1) {
            if (ka <= P.beta_basic * c.K_start) {
                restart = 1;
                c.cand_avg = 1;
                K = ka;
                c.K_cand = K;
            }
        }
        trace_put(c, to, c.tr_pass, 1, restart, c.tr_eta, c.tr_eta_bar, kc, ka);
        if (restart) {
            c.K_start = K;
            c.K_prev = K;
            if (c.cand_avg && c.lag) {   // materialise the average first
                c.pending = M_RESTART;
                c.mode = M_FOLD;
                return;
            }
            if (c.cand_avg) c.xr[R_CUR] = c.xr[R_AVG];
            c.mode = M_RESTART;
            return;
        }
        c.K_prev = K;
        if (limits_hit(c, P)) {
            finish(c, P, ST_NOT_CONVERGED);
            return;
        }
        step_decide(c, P, ts[TS_DX2], cs[CS_DY2], cs[CS_INTER], ts[TS_AUX], g_red, g_grow, to);
        return;
    }
    if (mode == M_FOLD) {
        swap_avg(c);
        c.lag = 0;
        if (c.pending == M_RESTART) {
            c.xr[R_CUR] = c.xr[R_AVG];
            c.mode = M_RESTART;
        } else {
            c.ret_x = c.xr[R_AVG];
            c.mode = M_VERIFY;
        }
        return;
    }
    if (mode == M_RESTART) {
        // primal weight (Section 5): distances between consecutive restart points
        const double dX = sqrt(ts[TS_AUX]);
        const double dY = sqrt(cs[CS_AUX]);
        if (P.pwu && dX > P.eps_zero && dY > P.eps_zero)
            c.omega = exp(P.theta * log(dY / dX) + (1.0 - P.theta) * log(c.omega));
        const int cur = c.xr[R_CUR];
        c.xr[R_ANCHOR] = cur;
        // the three lowest buffer indices other than the restart point, in role order
        int o0 = -1, o1 = -1, o2 = -1;
#pragma unroll
        for (int b = kBufs - 1; b >= 0; --b)
            if (b != cur) {
                o2 = o1;
                o1 = o0;
                o0 = b;
            }
        c.xr[R_TRIAL] = o0;
        c.xr[R_AVG] = o1;
        c.xr[R_AVGN] = o2;
        c.lag = 0;
        c.wsum = 0.0;
        c.k = 0;
        c.restarts += 1;
        c.cand_avg = 0;
        if (limits_hit(c, P)) finish(c, P, ST_NOT_CONVERGED);
        else c.mode = M_TRIAL;
        return;
    }
    if (mode == M_VERIFY) {
        double rel[3];
        const double K = rel_kkt(P, c.norm_b, c.norm_c, cs[CS_PRES], ts[TS_DRES], ts[TS_POBJ],
                                 cs[CS_DOBJ], rel);
        c.r_obj = ts[TS_POBJ];
        c.r_dobj = cs[CS_DOBJ];
        c.r_relP = rel[0];
        c.r_relD = rel[1];
        c.r_relG = rel[2];
        c.r_kkt = K;
        if (c.status == ST_OK && !(K == K)) {
            c.status = ST_NUMERIC;
        } else if (c.status == ST_OK && K > P.tol) {
            if (c.verify_fails < P.verify_retries && !limits_hit(c, P)) {
                // The running estimate met the tolerance but the returned arrays do not
                // (FP32 storage of the average); tighten the internal threshold and keep
                // iterating from the unchanged state.
                c.verify_fails += 1;
                const double ratio = P.tol / K;
                c.tol_eff = c.tol_eff * (ratio < 0.9 ? ratio : 0.9);
                c.status = ST_RUNNING;
                c.mode = M_TRIAL;
                return;
            }
            // the returned arrays (filled) fail the termination test: not converged
            c.status = ST_NOT_CONVERGED;
        }
        c.mode = M_IDLE;
        return;
    }
}

// ------------------------------------------------------------------ combine + control

// Inputs of the work on one row (rows) or one column, loaded before its partial sums so
// that both sets of loads are in flight together.
struct IndexIn {
    double fi, pc0, pb0, rc0, sb0, an0;
};

__device__ __forceinline__ IndexIn index_load(const PDOT_CONST Inst &I, const Ctl &st, int mode, bool rows,
                                              int64_t idx)
{
    IndexIn in{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    in.fi = rows ? gp(I.f)[idx] : gp(I.g)[idx];
    if (mode == M_INIT || mode == M_FOLD) return in;
    in.pc0 = gp(rows ? I.p[st.pv] : I.q[st.pv])[idx];
    in.pb0 = gp(rows ? I.pb[st.pbv] : I.qb[st.pbv])[idx];
    in.rc0 = gp(rows ? I.rs[st.rsv] : I.cs[st.rsv])[idx];
    if (mode == M_FULL || mode == M_RESTART) in.sb0 = gp(rows ? I.rsb : I.csb)[idx];
    if (mode == M_RESTART) in.an0 = gp(rows ? I.pa : I.qa)[idx];
    return in;
}

// The same inputs for every mode and both versions of the double-buffered vectors, loaded
// before the control block has arrived (which version is current is known only then).
struct IndexPre {
    double fi, pc[2], pb[2], rc[2], sb0, an0;
};

__device__ __forceinline__ IndexPre index_prefetch(const PDOT_CONST Inst &I, bool rows, int64_t idx)
{
    IndexPre x;
    x.fi = rows ? gp(I.f)[idx] : gp(I.g)[idx];
#pragma unroll
    for (int v = 0; v < 2; ++v) {
        x.pc[v] = gp(rows ? I.p[v] : I.q[v])[idx];
        x.pb[v] = gp(rows ? I.pb[v] : I.qb[v])[idx];
        x.rc[v] = gp(rows ? I.rs[v] : I.cs[v])[idx];
    }
    x.sb0 = gp(rows ? I.rsb : I.csb)[idx];
    x.an0 = gp(rows ? I.pa : I.qa)[idx];
    return x;
}

// The inputs index_load would have loaded for this mode and these versions.
__device__ __forceinline__ IndexIn index_select(const IndexPre &x, const Ctl &st, int mode)
{
    IndexIn in{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    in.fi = x.fi;
    if (mode == M_INIT || mode == M_FOLD) return in;
    // selects, not a run-time index (which could put the arrays in scratch memory)
    in.pc0 = st.pv ? x.pc[1] : x.pc[0];
    in.pb0 = st.pbv ? x.pb[1] : x.pb[0];
    in.rc0 = st.rsv ? x.rc[1] : x.rc[0];
    if (mode == M_FULL || mode == M_RESTART) in.sb0 = x.sb0;
    if (mode == M_RESTART) in.an0 = x.an0;
    return in;
}

// Work on one row (rows) or one column once its sums of the pass are complete (sv; 0 for
// modes that need none): KKT pieces of the current iterate and of the average, the dual
// step of the trial (Algorithm 2, with the extrapolated sums) and its running average,
// the step-size terms (Section 5), the move of the duals to the restart candidate, or the
// verified KKT pieces.  Adds the index's scalar pieces to acc.
__device__ __forceinline__ void index_work(const PDOT_CONST Inst &I, const Ctl &st, int mode, bool rows,
                                           int64_t idx, const IndexIn &in, double sv, double (&acc)[kNC])
{
    const double fi = in.fi, pc0 = in.pc0, pb0 = in.pb0, rc0 = in.rc0;
    if (mode == M_INIT) {
        acc[CS_AUX] += fi * fi;
        return;
    }
    if (mode == M_TRIAL || mode == M_FULL) {
        if (mode == M_FULL) {
            // KKT of the current iterate: its sums were kept when it was accepted
            double dl = rc0 - fi;
            acc[CS_PRES] += dl * dl;
            acc[CS_DOBJ] += fi * pc0;
            // averaged sums (linear in the plan), same weights as the plan average
            const double nb = (st.k == 1) ? rc0 : (1.0 - st.a_fold) * in.sb0 + st.a_fold * rc0;
            gp(rows ? I.rsb : I.csb)[idx] = nb;
            dl = nb - fi;
            acc[CS_PRESB] += dl * dl;
            acc[CS_DOBJB] += fi * pb0;
        }
        // dual step with the extrapolated sums: (2X+ - X) 1 = 2 X+ 1 - X 1, where X 1 (the
        // current iterate's sums) was kept when X was accepted; the trial's change of the
        // sums is X+ 1 - X 1
        const double sigma = st.eta * st.omega;
        const double sd = sv - rc0;
        const double er = sv + sd;
        const double pn = pc0 + sigma * (fi - er);
        const double d = pn - pc0;
        gp(rows ? I.p[st.pv ^ 1] : I.q[st.pv ^ 1])[idx] = pn;
        gp(rows ? I.rs[st.rsv ^ 1] : I.cs[st.rsv ^ 1])[idx] = sv;
        acc[CS_DY2] += d * d;
        acc[CS_INTER] += d * sd;
        // tentative running average of the duals for the trial
        const double w = I.prm.avg_weighting == 1 ? 1.0 : st.eta;
        const double a2 = w / (st.wsum + w);
        gp(rows ? I.pb[st.pbv ^ 1] : I.qb[st.pbv ^ 1])[idx] = (st.k == 0) ? pn : (1.0 - a2) * pb0 + a2 * pn;
    } else if (mode == M_RESTART) {
        const double pnew = st.cand_avg ? pb0 : pc0;
        const double dd = pnew - in.an0;
        acc[CS_AUX] += dd * dd;
        gp(rows ? I.p[st.pv] : I.q[st.pv])[idx] = pnew;
        gp(rows ? I.pa : I.qa)[idx] = pnew;
        if (st.cand_avg) gp(rows ? I.rs[st.rsv] : I.cs[st.rsv])[idx] = in.sb0;
    } else if (mode == M_VERIFY) {
        const double dl = sv - fi;
        acc[CS_PRES] += dl * dl;
        acc[CS_DOBJ] += fi * (st.ret_avg ? pb0 : pc0);
    }
}

// Record words of the combine hand-off.  A word holds the bits of its value plus one, so
// zero (its state before the value is written) is never a value: a computed double never
// has the all-ones bit pattern (a NaN payload the arithmetic does not produce).  Records
// alternate between two sets by slot parity: in a slot, each work-group writes its record
// in the set of the slot and clears its record in the other set, which the previous slot
// used and the next will write; kernel boundaries order the clear after the previous
// slot's reads and before the next slot's values.  So every word a slot reads is either
// its value of this slot or zero.
__device__ __forceinline__ void rec_put(PDOT_GLOBAL uint64_t *w, double v)
{
    __hip_atomic_store(w, (uint64_t)__double_as_longlong(v) + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The other set is read by no work-group during this slot (the previous slot's last
// work-group has read it, the next slot's will), so its words are cleared with plain
// stores, after the counter has moved; the kernel boundary makes them visible.
__device__ __forceinline__ void rec_clear(PDOT_GLOBAL uint64_t *w)
{
    *w = 0;
}

// Take the kNB words of one record: all loads in flight together, then, while any word is
// still zero, a short sleep and the zero words loaded again, all together (bounded: after
// kRecSpin rounds `lost` is set and the caller stops the instance with a device error
// instead of waiting on).
constexpr int kRecSpin = 1 << 20;
__device__ __forceinline__ void rec_take(PDOT_GLOBAL uint64_t *w, double (&v)[kNB], bool &lost)
{
    uint64_t b[kNB];
#pragma unroll
    for (int q = 0; q < kNB; ++q) b[q] = __hip_atomic_load(w + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int k = 0; k < kRecSpin; ++k) {
        bool all = true;
#pragma unroll
        for (int q = 0; q < kNB; ++q) all = all && b[q] != 0;
        if (all) break;
        __builtin_amdgcn_s_sleep(1);
#pragma unroll
        for (int q = 0; q < kNB; ++q)
            if (b[q] == 0) b[q] = __hip_atomic_load(w + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
#pragma unroll
    for (int q = 0; q < kNB; ++q) {
        if (b[q] == 0) lost = true;
        v[q] = b[q] ? __longlong_as_double((long long)(b[q] - 1u)) : 0.0;
    }
}

// The step rule's factors (T+1)^-a and (T+1)^-b (Section 5), a pow each (about a hundred
// FP64 instructions): evaluated by one lane of waves 1 and 2 and handed to the control
// thread through LDS at the barrier that precedes it, so they run beside the other waves'
// work instead of on the control thread's chain (the compiler would otherwise sink them
// into the single thread that uses them).
__device__ __forceinline__ void step_factors(double red_exp, double grow_exp, int64_t T, double *dst)
{
    if (threadIdx.x == 64 || threadIdx.x == 128) {
        const double tt = (double)(T + 1);
        dst[threadIdx.x == 128 ? 1 : 0] = pow(tt, -(threadIdx.x == 64 ? red_exp : grow_exp));
    }
}

// The run parameters of an instance, with vector loads all in flight together.  Through
// the scalar cache the control would fetch each field where it first uses it, one
// dependent miss after another on the slot's critical path.
static_assert(sizeof(Prm) % 8 == 0, "Prm is loaded in 8-byte words");
__device__ __forceinline__ Prm prm_load(const Prm *p)
{
    const PDOT_GLOBAL uint64_t *src = gp((const uint64_t *)p);
    uint64_t w[sizeof(Prm) / 8];
#pragma unroll
    for (int q = 0; q < (int)(sizeof(Prm) / 8); ++q)
        w[q] = __hip_atomic_load(src + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    Prm P;
    __builtin_memcpy(&P, w, sizeof(Prm));
    return P;
}

// The combine kernel: one work-group per slice of 64 rows or 64 columns of an instance.
//  1. adds the per-tile partial sums of the slice (the four waves split the partials; all
//     loads of a wave are in flight together; fixed order);
//  2. per row/column (wave 0): the index work above; meanwhile wave 1 adds the scalars of
//     the slice's share of the pass's tiles;
//  3. hands its record (eight slice scalars, six tile scalars) to the last work-group of
//     the instance (agent-scope atomic stores and a counter), which reduces the records in
//     a fixed order and runs the control of Section 5 for the next slot.
__global__ __launch_bounds__(kWG) void k_combine(const Inst *__restrict__ insts, Ctl *__restrict__ ctls,
                                                 const CombEntry *__restrict__ ents,
                                                 const int32_t *__restrict__ count)
{
    __shared__ double part[4][64];
    __shared__ double tsum[kNS];
    __shared__ double fin[4][kNB];
    __shared__ int is_last, lost_any;
    __shared__ double gfac[2];   // step factors for the control thread
    if (threadIdx.x == 0) lost_any = 0;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // The launch grid never exceeds the entry table's capacity: the first entry is read
    // before the count (both loads in flight) and used only if it is in the count.
    CombEntry next = cp(ents)[blockIdx.x];
    const int nents = *cp(count);

    for (int e = blockIdx.x; e < nents; e += gridDim.x) {
        const CombEntry E = next;
        if (e + (int)gridDim.x < nents) next = cp(ents)[e + gridDim.x];
        const PDOT_CONST Inst &I = cp(insts)[E.inst];
        const Ctl st = gp(ctls)[E.inst];

        const bool rows = E.kind == 0;
        const int64_t len = rows ? I.m : I.n;
        const int64_t idx = (int64_t)E.start + lane;
        const bool valid = idx < len;

        // The per-entry vectors (wave 0) and the per-tile partial sums of this slice are
        // loaded before the control block has arrived, so that the three sets of loads are
        // in flight together; modes that use no sums (and idle instances) discard them.
        IndexPre pre{};
        if (wave == 0 && valid) pre = index_prefetch(I, rows, idx);

        // phase 1: the per-tile partial sums of this slice, in a fixed order (wave w adds
        // partials w, w+4, w+8, ... with up to 16 loads in flight)
        double sv = 0.0;
        {
            const int np = rows ? I.ncb : I.nrb;
            const PDOT_GLOBAL double *src = gp(rows ? (const double *)I.rowpart : (const double *)I.colpart);
            if (valid) {
                for (int base = wave; base < np; base += 64) {
                    double v[16];
#pragma unroll
                    for (int k = 0; k < 16; ++k) {
                        const int pp = base + 4 * k;
                        v[k] = pp < np ? src[(int64_t)pp * len + idx] : 0.0;
                    }
#pragma unroll
                    for (int k = 0; k < 16; ++k)
                        if (base + 4 * k < np) sv += v[k];
                }
            }
        }
        const int mode = st.mode;
        if (mode == M_IDLE) continue;
        const bool sums = mode == M_TRIAL || mode == M_FULL || mode == M_VERIFY;
        if (sums) part[wave][lane] = sv;
        IndexIn in{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (wave == 0 && valid) in = index_select(pre, st, mode);

        // the tile scalars of this entry's share of the pass's tiles (wave 1)
        if (wave == 1) {
            const int t0 = (int)((int64_t)E.local * I.ntiles / I.ncomb);
            const int t1 = (int)((int64_t)(E.local + 1) * I.ntiles / I.ncomb);
            double ts[kNS];
#pragma unroll
            for (int q = 0; q < kNS; ++q) ts[q] = 0.0;
            for (int t = t0 + lane; t < t1; t += 64) {
                const PDOT_GLOBAL double *src = gp((const double *)I.tilescal) + (int64_t)t * kNS;
#pragma unroll
                for (int q = 0; q < kNS; ++q) ts[q] += src[q];
            }
#pragma unroll
            for (int q = 0; q < kNS; ++q) ts[q] = wave_sum_to63(ts[q]);
            if (lane == 63) {
#pragma unroll
                for (int q = 0; q < kNS; ++q) tsum[q] = ts[q];
            }
        }
        __syncthreads();
        if (sums && wave == 0) sv = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];

        // phase 2: per-entry vector work (wave 0, one row or column per lane)
        if (wave == 0) {
            double acc[kNC];
#pragma unroll
            for (int q = 0; q < kNC; ++q) acc[q] = 0.0;
            if (valid) index_work(I, st, mode, rows, idx, in, sv, acc);
            // The record goes to the last work-group (elected by a counter) through record
            // words that carry their own state: agent-scope atomic stores and loads of each
            // 64-bit word (coherent across the chiplets' L2 caches), a word holding zero until
            // its value has been written (see rec_put).  So the last work-group needs no
            // ordering between the records and the counter, and no cache write-back or
            // invalidation: it waits for each word itself (rec_take).
            double r[kNC];
#pragma unroll
            for (int q = 0; q < kNC; ++q) r[q] = wave_sum_to63(acc[q]);
            if (lane == 63) {
                const int64_t set = (int64_t)(st.kpasses & 1) * I.ncomb * kNB;
                const int64_t other = (int64_t)((st.kpasses & 1) ^ 1) * I.ncomb * kNB;
                PDOT_GLOBAL uint64_t *dst = gp((uint64_t *)I.combscal) + set + (int64_t)E.local * kNB;
                PDOT_GLOBAL uint64_t *old = gp((uint64_t *)I.combscal) + other + (int64_t)E.local * kNB;
#pragma unroll
                for (int q = 0; q < kNC; ++q) rec_put(dst + q, r[q]);
#pragma unroll
                for (int q = 0; q < kNS; ++q) rec_put(dst + kNC + q, tsum[q]);
                // not needed for correctness: the record stores complete before the counter
                // moves, so the last work-group normally finds every word on its first load
                __builtin_amdgcn_s_waitcnt(0);
                const unsigned prev = __hip_atomic_fetch_add(gp(I.counter), 1u, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT);
                is_last = (prev == (unsigned)(I.ncomb - 1)) ? 1 : 0;
#pragma unroll
                for (int q = 0; q < kNB; ++q) rec_clear(old + q);
            }
        }
        __syncthreads();
        if (!is_last) continue;

        // phase 3 (last work-group of the instance): reduce every record in a fixed order
        // and run the control
        const Prm P = prm_load(&insts[E.inst].prm);
        step_factors(P.red_exp, P.grow_exp, st.T, gfac);
        double loc[kNB];
#pragma unroll
        for (int q = 0; q < kNB; ++q) loc[q] = 0.0;
        bool lost = false;
        const int64_t set = (int64_t)(st.kpasses & 1) * I.ncomb * kNB;
        for (int c = threadIdx.x; c < I.ncomb; c += kWG) {
            double v[kNB];
            rec_take(gp((uint64_t *)I.combscal) + set + (int64_t)c * kNB, v, lost);
#pragma unroll
            for (int q = 0; q < kNB; ++q) loc[q] += v[q];
        }
        if (lost) lost_any = 1;
#pragma unroll
        for (int q = 0; q < kNB; ++q) loc[q] = wave_sum_to63(loc[q]);
        if (lane == 63) {
#pragma unroll
            for (int q = 0; q < kNB; ++q) fin[wave][q] = loc[q];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double tot[kNB];
            for (int q = 0; q < kNB; ++q)
                tot[q] = ((fin[0][q] + fin[1][q]) + fin[2][q]) + fin[3][q];
            // the control block is unchanged since this work-group read it (only the last
            // work-group of the instance writes it, below)
            Ctl c = st;
            if (lost_any) {   // a record word never arrived: stop the instance, report it
                c.status = ST_DEVICE;
                c.mode = M_IDLE;
            } else {
                control(c, P, mode, tot, tot + kNC, gfac[0], gfac[1], TraceOut{I.trace, I.trace_cap});
            }
            gp(ctls)[E.inst] = c;
            __hip_atomic_store(gp(I.counter), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            lost_any = 0;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ resident instances

// One work-group runs a whole instance for up to `budget` slots per launch: it streams
// every column band of the plan itself (the tile body with all rows in one row block),
// so the row and column sums of a pass are complete inside the work-group, then does the
// index work of every row and column, reduces the scalars in a fixed order and runs the
// control, with work-group barriers in place of the grid-wide kernel boundaries.  Meant
// for small instances, whose passes are too short to fill the GPU: many of them run side
// by side, one per work-group, without a launch per iteration.  The control block lives
// in LDS during the launch.  Every value exchanged between threads goes through vector
// memory operations and the barriers' workgroup-scope fences.
template <typename TX, int VEC, int COST>
__device__ void resident_pass(const PDOT_CONST Inst &I, const Ctl &st, int slot, double *lds)
{
    for (int cb = 0; cb < I.ncb; ++cb) {
        const Tile tl{slot, 0, cb, cb};
        switch (st.mode) {
        case M_INIT: tile_body<TX, VEC, COST, M_INIT, true>(I, st, tl, lds); break;
        case M_TRIAL:
            if (st.lag) tile_body<TX, VEC, COST, M_TRIAL, true, true>(I, st, tl, lds);
            else tile_body<TX, VEC, COST, M_TRIAL, true>(I, st, tl, lds);
            break;
        case M_FULL:
            if (st.lag) tile_body<TX, VEC, COST, M_FULL, true, true>(I, st, tl, lds);
            else tile_body<TX, VEC, COST, M_FULL, true>(I, st, tl, lds);
            break;
        case M_RESTART: tile_body<TX, VEC, COST, M_RESTART, true>(I, st, tl, lds); break;
        case M_VERIFY: tile_body<TX, VEC, COST, M_VERIFY, true>(I, st, tl, lds); break;
        case M_FOLD: tile_body<TX, VEC, COST, M_FOLD, true>(I, st, tl, lds); break;
        default: break;
        }
    }
}

template <typename TX, int VEC, int COST>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(PDOT_PASS_WAVES)))
void k_resident(const Inst *__restrict__ insts, const int32_t *__restrict__ list,
                const int32_t *__restrict__ count, int32_t budget)
{
    const int nres = *cp(count);
    __shared__ double lds[3 * 2 * 4 * 64 + 4 * kNS];
    __shared__ double red[4][kNB];
    __shared__ double gfac[2];   // step factors for the control thread
    __shared__ Ctl sctl;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    for (int w = blockIdx.x; w < nres; w += gridDim.x) {
        const int slot = cp(list)[w];
        const PDOT_CONST Inst &I = cp(insts)[slot];
        if (threadIdx.x == 0) sctl = *gp(I.ctl);
        __syncthreads();
        for (int it = 0; it < budget; ++it) {
            const Ctl st = sctl;
            const int mode = st.mode;
            if (mode == M_IDLE) break;
            resident_pass<TX, VEC, COST>(I, st, slot, lds);
            __syncthreads();

            // index work over all rows, then all columns; the tile scalars of the pass
            const bool sums = mode == M_TRIAL || mode == M_FULL || mode == M_VERIFY;
            double acc[kNC], ts[kNS];
#pragma unroll
            for (int q = 0; q < kNC; ++q) acc[q] = 0.0;
#pragma unroll
            for (int q = 0; q < kNS; ++q) ts[q] = 0.0;
            for (int t = threadIdx.x; t < I.ncb; t += kWG) {
                const PDOT_GLOBAL double *src = gp((const double *)I.tilescal) + (int64_t)t * kNS;
#pragma unroll
                for (int q = 0; q < kNS; ++q) ts[q] += src[q];
            }
            for (int64_t i = threadIdx.x; i < I.m; i += kWG) {
                const IndexIn in = index_load(I, st, mode, true, i);
                double sv = 0.0;
                if (sums) {
                    const PDOT_GLOBAL double *src = gp((const double *)I.rowpart) + i;
                    for (int c = 0; c < I.ncb; ++c) sv += src[(int64_t)c * I.m];
                }
                index_work(I, st, mode, true, i, in, sv, acc);
            }
            for (int64_t j = threadIdx.x; j < I.n; j += kWG) {
                const IndexIn in = index_load(I, st, mode, false, j);
                const double sv = sums ? gp((const double *)I.colpart)[j] : 0.0;
                index_work(I, st, mode, false, j, in, sv, acc);
            }
            double r[kNB];
#pragma unroll
            for (int q = 0; q < kNC; ++q) r[q] = wave_sum_to63(acc[q]);
#pragma unroll
            for (int q = 0; q < kNS; ++q) r[kNC + q] = wave_sum_to63(ts[q]);
            if (lane == 63) {
#pragma unroll
                for (int q = 0; q < kNB; ++q) red[wave][q] = r[q];
            }
            step_factors(I.prm.red_exp, I.prm.grow_exp, st.T, gfac);
            __syncthreads();
            if (threadIdx.x == 0) {
                const Prm P = I.prm;
                double tot[kNB];
                for (int q = 0; q < kNB; ++q)
                    tot[q] = ((red[0][q] + red[1][q]) + red[2][q]) + red[3][q];
                Ctl c = sctl;
                control(c, P, mode, tot, tot + kNC, gfac[0], gfac[1], TraceOut{I.trace, I.trace_cap});
                sctl = c;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) *gp(I.ctl) = sctl;
        __syncthreads();
    }
}

// ------------------------------------------------------------------ rounding and bracket

// Rounding of an approximately feasible plan to an exactly feasible one (Algorithm 3,
// Section 3.2) and the certified bracket of the optimal value, on an FP64 copy of the plan
// in an instance workspace (plan in X[0], duals u in p[0], the FP64 cost stored or
// regenerated).  Four tiled passes, each followed by a one-work-group vector step:
//   1. X 1 and X^T 1                    -> x_i = min(f_i / (X 1)_i, 1)
//   2. column sums of D_x X             -> y_j = min(g_j / (D_x X)^T 1)_j, 1)
//   3. row and column sums of D_x X D_y -> err_r = f - ..., err_c = g - ..., ||err_r||_1
//   4. X_feas = D_x X D_y + err_r err_c^T / ||err_r||_1 (written when asked), <C, X_feas>,
//      ||X_feas - X||_1, the sums of X_feas, and min_i (C_ij - u_i) per column
// Vectors: x in rs[0], y in cs[0], err_r in rs[1], err_c in cs[1], the c-transform in csb;
// the column minima of pass 4 use the free plan buffer X[1]; scalars in combscal[0..15].
// Every sum runs in a fixed order.
template <int COST>
__device__ __forceinline__ double cost64(const PDOT_CONST Inst &I, int64_t i, int64_t j)
{
    if constexpr (COST == C_STORED) {
        return gp((const double *)I.C)[i * I.ld + j];
    } else if constexpr (is_grid(COST)) {
        const uint32_t s = (uint32_t)I.side;
        return grid_cost<double, COST>((float)(int)((uint32_t)i / s), (float)(int)((uint32_t)i % s),
                                       (float)(int)((uint32_t)j / s), (float)(int)((uint32_t)j % s),
                                       I.scale, (float)I.scale);
    } else {
        double xi[3] = {0.0, 0.0, 0.0}, yj[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (k < I.dim) {
                xi[k] = gp(I.xs)[i * I.dim + k];
                yj[k] = gp(I.ys)[j * I.dim + k];
            }
        double d = sqdist(xi, yj, I.dim);
        if constexpr (COST == C_PTS_EU) d = sqrt(d);
        return d;
    }
}

template <int COST, int PHASE>
__global__ __launch_bounds__(kWG) void k_round_tiles(const Inst *__restrict__ inst, double *__restrict__ xfeas)
{
#pragma clang fp contract(off)
    const PDOT_CONST Inst &I = *cp(inst);
    __shared__ double cl[3][2][64];
    __shared__ double sl[4][2];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t m = I.m, n = I.n, ld = I.ld;
    const PDOT_GLOBAL double *X = gp((const double *)I.X[0]);
    const PDOT_GLOBAL double *xr = gp((const double *)I.rs[0]);
    const PDOT_GLOBAL double *yc = gp((const double *)I.cs[0]);
    const PDOT_GLOBAL double *er = gp((const double *)I.rs[1]);
    const PDOT_GLOBAL double *ec = gp((const double *)I.cs[1]);
    const PDOT_GLOBAL double *u = gp((const double *)I.p[0]);
    PDOT_GLOBAL double *rowpart = gp(I.rowpart);
    PDOT_GLOBAL double *colpart = gp(I.colpart);
    PDOT_GLOBAL double *colmin = gp((double *)I.X[1]);
    const double l1 = PHASE == 4 ? gp((const double *)I.combscal)[RD_L1] : 0.0;
    constexpr double kInf = __builtin_huge_val();
    for (int t = blockIdx.x; t < I.ntiles; t += gridDim.x) {
        const int rb = t / I.ncb, cb = t % I.ncb;
        const int64_t i0 = (int64_t)rb * I.rows, ie = min(m, i0 + (int64_t)I.rows);
        double csum[2] = {0.0, 0.0}, cmin[2] = {kInf, kInf};
        double s_up = 0.0, s_ch = 0.0;
        int64_t jj[2];
        bool ok[2];
        double ycol[2] = {1.0, 1.0}, ecol[2] = {0.0, 0.0};
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            jj[v] = (int64_t)cb * 128 + lane * 2 + v;
            ok[v] = jj[v] < n;
            if (ok[v] && PHASE >= 3) ycol[v] = yc[jj[v]];
            if (ok[v] && PHASE == 4) ecol[v] = ec[jj[v]];
        }
        for (int64_t i = i0 + wave; i < ie; i += 4) {
            const double xi = PHASE >= 2 ? xr[i] : 1.0;
            const double eri = PHASE == 4 ? er[i] : 0.0;
            const double ui = PHASE == 4 ? u[i] : 0.0;
            double rsum = 0.0;
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                if (!ok[v]) continue;
                const int64_t j = jj[v];
                const double x = X[i * ld + j];
                double val = x;
                if (PHASE >= 2) val = xi * x;
                if (PHASE >= 3) val = val * ycol[v];
                if (PHASE == 4) {
                    if (l1 > 0.0) val = val + eri * ecol[v] / l1;
                    const double c = cost64<COST>(I, i, j);
                    s_up = fma(c, val, s_up);
                    s_ch += fabs(val - x);
                    const double d = c - ui;
                    cmin[v] = d < cmin[v] ? d : cmin[v];
                    if (xfeas) xfeas[i * n + j] = val;
                }
                rsum += val;
                csum[v] += val;
            }
            if (PHASE != 2) {
                const double r = wave_sum_to63(rsum);
                if (lane == 63) rowpart[(int64_t)cb * m + i] = r;
            }
        }
        // column partials (sums; minima in pass 4): the four waves in a fixed order
        if (wave > 0) {
            cl[wave - 1][0][lane] = csum[0];
            cl[wave - 1][1][lane] = csum[1];
        }
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                const double sv = ((csum[v] + cl[0][v][lane]) + cl[1][v][lane]) + cl[2][v][lane];
                if (ok[v]) colpart[(int64_t)rb * n + jj[v]] = sv;
            }
        }
        __syncthreads();
        if (PHASE == 4) {
            if (wave > 0) {
                cl[wave - 1][0][lane] = cmin[0];
                cl[wave - 1][1][lane] = cmin[1];
            }
            __syncthreads();
            if (wave == 0) {
#pragma unroll
                for (int v = 0; v < 2; ++v) {
                    double mv = cmin[v];
                    for (int w = 0; w < 3; ++w) mv = cl[w][v][lane] < mv ? cl[w][v][lane] : mv;
                    if (ok[v]) colmin[(int64_t)rb * n + jj[v]] = mv;
                }
            }
            const double a = wave_sum_to63(s_up), b = wave_sum_to63(s_ch);
            if (lane == 63) {
                sl[wave][0] = a;
                sl[wave][1] = b;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                PDOT_GLOBAL double *ts = gp(I.tilescal) + (int64_t)t * kNS;
                ts[0] = ((sl[0][0] + sl[1][0]) + sl[2][0]) + sl[3][0];
                ts[1] = ((sl[0][1] + sl[1][1]) + sl[2][1]) + sl[3][1];
            }
            __syncthreads();
        }
    }
}

// The vector step after each pass (one work-group; thread t takes indices t, t+256, ...;
// per-thread terms are combined by DPP and LDS in a fixed order).
template <int PHASE>
__global__ __launch_bounds__(kWG) void k_round_vec(const Inst *__restrict__ inst)
{
#pragma clang fp contract(off)
    const PDOT_CONST Inst &I = *cp(inst);
    __shared__ double red[4][4];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t m = I.m, n = I.n;
    const PDOT_GLOBAL double *rowpart = gp((const double *)I.rowpart);
    const PDOT_GLOBAL double *colpart = gp((const double *)I.colpart);
    const PDOT_GLOBAL double *f = gp(I.f);
    const PDOT_GLOBAL double *g = gp(I.g);
    PDOT_GLOBAL double *sc = gp(I.combscal);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};   // sums, or a maximum in acc[3]
    for (int64_t i = threadIdx.x; i < m && PHASE != 2; i += kWG) {
        double r = 0.0;
        for (int c = 0; c < I.ncb; ++c) r += rowpart[(int64_t)c * m + i];
        const double fi = f[i];
        if (PHASE == 1) {
            gp((double *)I.rs[0])[i] = r > 0.0 ? fmin(fi / r, 1.0) : 1.0;
            acc[0] += fabs(fi - r);
        } else if (PHASE == 3) {
            const double e = fi - r;
            gp((double *)I.rs[1])[i] = e;
            acc[1] += fabs(e);
        } else {
            acc[3] = fmax(acc[3], fabs(r - fi));
            acc[2] = fma(fi, gp((const double *)I.p[0])[i], acc[2]);
        }
    }
    for (int64_t j = threadIdx.x; j < n; j += kWG) {
        double c = 0.0;
        for (int r = 0; r < I.nrb; ++r) c += colpart[(int64_t)r * n + j];
        const double gj = g[j];
        if (PHASE == 1) {
            acc[0] += fabs(gj - c);
        } else if (PHASE == 2) {
            gp((double *)I.cs[0])[j] = c > 0.0 ? fmin(gj / c, 1.0) : 1.0;
        } else if (PHASE == 3) {
            gp((double *)I.cs[1])[j] = gj - c;
        } else {
            acc[3] = fmax(acc[3], fabs(c - gj));
            const PDOT_GLOBAL double *cm = gp((const double *)I.X[1]);
            double v = cm[j];
            for (int r = 1; r < I.nrb; ++r) v = cm[(int64_t)r * n + j] < v ? cm[(int64_t)r * n + j] : v;
            gp((double *)I.csb)[j] = v;
            acc[2] = fma(gj, v, acc[2]);
        }
    }
    double r[4];
#pragma unroll
    for (int q = 0; q < 3; ++q) r[q] = wave_sum_to63(acc[q]);
    // maximum over the wave: every lane's value, read by lane 63 through LDS
    __shared__ double mx[kWG];
    mx[threadIdx.x] = acc[3];
    __syncthreads();
    if (lane == 63) {
        double v = 0.0;
        for (int k = 0; k < 64; ++k) v = fmax(v, mx[wave * 64 + k]);
        r[3] = v;
#pragma unroll
        for (int q = 0; q < 4; ++q) red[wave][q] = r[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[4];
        for (int q = 0; q < 3; ++q) t[q] = ((red[0][q] + red[1][q]) + red[2][q]) + red[3][q];
        t[3] = fmax(fmax(red[0][3], red[1][3]), fmax(red[2][3], red[3][3]));
        if (PHASE == 1) sc[RD_MARG] = t[0];
        if (PHASE == 3) sc[RD_L1] = t[1];
        if (PHASE == 4) {
            double up = 0.0, ch = 0.0;
            const PDOT_GLOBAL double *ts = gp((const double *)I.tilescal);
            for (int k = 0; k < I.ntiles; ++k) {
                up += ts[(int64_t)k * kNS];
                ch += ts[(int64_t)k * kNS + 1];
            }
            sc[RD_UPPER] = up;
            sc[RD_CHANGE] = ch;
            sc[RD_LOWER] = t[2];
            sc[RD_VIOL] = t[3];
        }
    }
}

// ------------------------------------------------------------------ setup kernels

// Materialise the cost in the working precision with padding columns set to zero.
// kind: C_STORED reads a dense FP64 source with row stride ldc.
template <typename TX>
__global__ __launch_bounds__(kWG) void k_materialize(TX *__restrict__ dst, int64_t m, int64_t n,
                                                     int64_t ld, int kind, const double *__restrict__ src,
                                                     int64_t ldc, const double *__restrict__ xs,
                                                     const double *__restrict__ ys, int dim,
                                                     int side, double scale)
{
    const int64_t total = m * ld;
    for (int64_t e = (int64_t)blockIdx.x * kWG + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kWG) {
        const int64_t i = e / ld, j = e % ld;
        double v = 0.0;
        if (j < n) {
            if (kind == C_STORED) {
                v = src[i * ldc + j];
            } else if (is_grid(kind)) {
                const float ia = (float)(int)(i / side), ib = (float)(int)(i % side);
                const float ja = (float)(int)(j / side), jb = (float)(int)(j % side);
                const float s32 = (float)scale;
                if (kind == C_GRID_SQ) v = grid_cost<TX, C_GRID_SQ>(ia, ib, ja, jb, scale, s32);
                else if (kind == C_GRID_L1) v = grid_cost<TX, C_GRID_L1>(ia, ib, ja, jb, scale, s32);
                else if (kind == C_GRID_L2) v = grid_cost<TX, C_GRID_L2>(ia, ib, ja, jb, scale, s32);
                else v = grid_cost<TX, C_GRID_LINF>(ia, ib, ja, jb, scale, s32);
            } else if (kind == C_PTS_EU) {
                v = point_cost<TX, C_PTS_EU>(xs + i * dim, ys + j * dim, dim);
            } else {
                v = point_cost<TX, C_PTS_SQ>(xs + i * dim, ys + j * dim, dim);
            }
        }
        dst[e] = (TX)v;
    }
}

// Zero fill (8-byte words) of a workspace region.
__global__ __launch_bounds__(kWG) void k_zero(uint64_t *__restrict__ dst, int64_t words)
{
    for (int64_t e = (int64_t)blockIdx.x * kWG + threadIdx.x; e < words; e += (int64_t)gridDim.x * kWG)
        dst[e] = 0;
}

// The tile and combine tables of one instance in slot 0 (the order the runtime uses: tiles
// by row block then column band, combine entries for the row slices then the column
// slices), the two counts, and a one-entry resident list {0} with its count.
__global__ __launch_bounds__(kWG) void k_tables(Tile *__restrict__ tiles, int ntiles, int ncb,
                                                CombEntry *__restrict__ combs, int nrows, int ncomb,
                                                int32_t *__restrict__ counts)
{
    const int stride = gridDim.x * kWG;
    for (int t = blockIdx.x * kWG + threadIdx.x; t < ntiles; t += stride)
        tiles[t] = Tile{0, t / ncb, t % ncb, t};
    for (int e = blockIdx.x * kWG + threadIdx.x; e < ncomb; e += stride)
        combs[e] = e < nrows ? CombEntry{0, 0, e * kCombEntries, e}
                             : CombEntry{0, 1, (e - nrows) * kCombEntries, e};
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        counts[0] = ntiles;
        counts[1] = ncomb;
        counts[2] = 1;
        counts[3] = 0;
    }
}

}  // namespace pdot

// ------------------------------------------------------------------ launchers (host)

namespace pdot {

// Launch of the streaming pass.  With events (profiling), the events are stamped with the
// kernel's own start and end (hipExtLaunchKernel), not with the enqueue times.
template <typename K>
static hipError_t launch_k(K kernel, int grid, const Inst *insts, const Ctl *ctls, const Tile *tiles,
                           const int32_t *count, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    if (ev0 && ev1)
        hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(kWG), 0, s, ev0, ev1, 0, insts, ctls, tiles, count);
    else
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(kWG), 0, s, insts, ctls, tiles, count);
    return hipGetLastError();
}

template <typename TX, int VEC>
static hipError_t launch_pass_vec(int cost, const Inst *insts, const Ctl *ctls, const Tile *tiles,
                                  const int32_t *ntiles, int grid, hipStream_t s, hipEvent_t ev0,
                                  hipEvent_t ev1)
{
    switch (cost) {
    case C_STORED: return launch_k(k_pass<TX, VEC, C_STORED>, grid, insts, ctls, tiles, ntiles, s, ev0, ev1);
    case C_PTS_SQ: return launch_k(k_pass<TX, VEC, C_PTS_SQ>, grid, insts, ctls, tiles, ntiles, s, ev0, ev1);
    case C_PTS_EU: return launch_k(k_pass<TX, VEC, C_PTS_EU>, grid, insts, ctls, tiles, ntiles, s, ev0, ev1);
    case C_GRID_SQ: return launch_k(k_pass<TX, VEC, C_GRID_SQ>, grid, insts, ctls, tiles, ntiles, s, ev0, ev1);
    case C_GRID_L1: return launch_k(k_pass<TX, VEC, C_GRID_L1>, grid, insts, ctls, tiles, ntiles, s, ev0, ev1);
    case C_GRID_L2: return launch_k(k_pass<TX, VEC, C_GRID_L2>, grid, insts, ctls, tiles, ntiles, s, ev0, ev1);
    case C_GRID_LINF: return launch_k(k_pass<TX, VEC, C_GRID_LINF>, grid, insts, ctls, tiles, ntiles, s, ev0, ev1);
    default: return hipErrorInvalidValue;
    }
}

template <typename TX>
static hipError_t launch_pass_t(int vec, int cost, const Inst *insts, const Ctl *ctls, const Tile *tiles,
                                const int32_t *ntiles, int grid, hipStream_t s, hipEvent_t ev0,
                                hipEvent_t ev1)
{
    switch (vec) {
    case 1: return launch_pass_vec<TX, 1>(cost, insts, ctls, tiles, ntiles, grid, s, ev0, ev1);
    case 2: return launch_pass_vec<TX, 2>(cost, insts, ctls, tiles, ntiles, grid, s, ev0, ev1);
    case 4: return launch_pass_vec<TX, 4>(cost, insts, ctls, tiles, ntiles, grid, s, ev0, ev1);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pass(int fp32, int vec, int cost, const Inst *insts, const Ctl *ctls, const Tile *tiles,
                       const int32_t *ntiles, int grid, hipStream_t s, hipEvent_t ev0,
                       hipEvent_t ev1)
{
    return fp32 ? launch_pass_t<float>(vec, cost, insts, ctls, tiles, ntiles, grid, s, ev0, ev1)
                : launch_pass_t<double>(vec, cost, insts, ctls, tiles, ntiles, grid, s, ev0, ev1);
}

hipError_t launch_combine(const Inst *insts, Ctl *ctls, const CombEntry *ents, const int32_t *nents, int grid,
                          hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    if (ev0 && ev1)
        hipExtLaunchKernelGGL(k_combine, dim3(grid), dim3(kWG), 0, s, ev0, ev1, 0, insts, ctls, ents, nents);
    else
        hipLaunchKernelGGL(k_combine, dim3(grid), dim3(kWG), 0, s, insts, ctls, ents, nents);
    return hipGetLastError();
}

template <typename K>
static hipError_t launch_r(K kernel, int grid, const Inst *insts, const int32_t *list,
                           const int32_t *count, int32_t budget, hipStream_t s, hipEvent_t ev0,
                           hipEvent_t ev1)
{
    if (ev0 && ev1)
        hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(kWG), 0, s, ev0, ev1, 0, insts, list, count, budget);
    else
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(kWG), 0, s, insts, list, count, budget);
    return hipGetLastError();
}

template <typename TX, int VEC>
static hipError_t launch_resident_vec(int cost, const Inst *insts, const int32_t *list,
                                      const int32_t *count, int grid, int32_t budget, hipStream_t s,
                                      hipEvent_t ev0, hipEvent_t ev1)
{
    switch (cost) {
    case C_STORED: return launch_r(k_resident<TX, VEC, C_STORED>, grid, insts, list, count, budget, s, ev0, ev1);
    case C_PTS_SQ: return launch_r(k_resident<TX, VEC, C_PTS_SQ>, grid, insts, list, count, budget, s, ev0, ev1);
    case C_PTS_EU: return launch_r(k_resident<TX, VEC, C_PTS_EU>, grid, insts, list, count, budget, s, ev0, ev1);
    case C_GRID_SQ: return launch_r(k_resident<TX, VEC, C_GRID_SQ>, grid, insts, list, count, budget, s, ev0, ev1);
    case C_GRID_L1: return launch_r(k_resident<TX, VEC, C_GRID_L1>, grid, insts, list, count, budget, s, ev0, ev1);
    case C_GRID_L2: return launch_r(k_resident<TX, VEC, C_GRID_L2>, grid, insts, list, count, budget, s, ev0, ev1);
    case C_GRID_LINF: return launch_r(k_resident<TX, VEC, C_GRID_LINF>, grid, insts, list, count, budget, s, ev0, ev1);
    default: return hipErrorInvalidValue;
    }
}

template <typename TX>
static hipError_t launch_resident_t(int vec, int cost, const Inst *insts, const int32_t *list,
                                    const int32_t *count, int grid, int32_t budget, hipStream_t s,
                                    hipEvent_t ev0, hipEvent_t ev1)
{
    switch (vec) {
    case 1: return launch_resident_vec<TX, 1>(cost, insts, list, count, grid, budget, s, ev0, ev1);
    case 2: return launch_resident_vec<TX, 2>(cost, insts, list, count, grid, budget, s, ev0, ev1);
    default: return hipErrorInvalidValue;   // resident instances use 1 or 2 columns per lane
    }
}

hipError_t launch_resident(int fp32, int vec, int cost, const Inst *insts, const int32_t *list,
                           const int32_t *count, int grid, int32_t budget, hipStream_t s,
                           hipEvent_t ev0, hipEvent_t ev1)
{
    return fp32 ? launch_resident_t<float>(vec, cost, insts, list, count, grid, budget, s, ev0, ev1)
                : launch_resident_t<double>(vec, cost, insts, list, count, grid, budget, s, ev0, ev1);
}

template <int COST>
static hipError_t launch_round_cost(const Inst *inst, double *xfeas, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((k_round_tiles<COST, 1>), dim3(grid), dim3(kWG), 0, s, inst, (double *)nullptr);
    hipLaunchKernelGGL(k_round_vec<1>, dim3(1), dim3(kWG), 0, s, inst);
    hipLaunchKernelGGL((k_round_tiles<COST, 2>), dim3(grid), dim3(kWG), 0, s, inst, (double *)nullptr);
    hipLaunchKernelGGL(k_round_vec<2>, dim3(1), dim3(kWG), 0, s, inst);
    hipLaunchKernelGGL((k_round_tiles<COST, 3>), dim3(grid), dim3(kWG), 0, s, inst, (double *)nullptr);
    hipLaunchKernelGGL(k_round_vec<3>, dim3(1), dim3(kWG), 0, s, inst);
    hipLaunchKernelGGL((k_round_tiles<COST, 4>), dim3(grid), dim3(kWG), 0, s, inst, xfeas);
    hipLaunchKernelGGL(k_round_vec<4>, dim3(1), dim3(kWG), 0, s, inst);
    return hipGetLastError();
}

// FP32 plan (row stride n) widened into an FP64 buffer of row stride ld.
__global__ __launch_bounds__(kWG) void k_widen(const float *__restrict__ src, int64_t m, int64_t n,
                                               double *__restrict__ dst, int64_t ld)
{
    const int64_t total = m * n;
    for (int64_t e = (int64_t)blockIdx.x * kWG + threadIdx.x; e < total; e += (int64_t)gridDim.x * kWG) {
        const int64_t i = e / n, j = e % n;
        dst[i * ld + j] = (double)src[e];
    }
}

hipError_t launch_widen(const float *src, int64_t m, int64_t n, double *dst, int64_t ld, hipStream_t s)
{
    int64_t blocks = (m * n + kWG - 1) / kWG;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_widen, dim3((unsigned)blocks), dim3(kWG), 0, s, src, m, n, dst, ld);
    return hipGetLastError();
}

// Rounding passes of one FP64 instance (inst: device pointer to its descriptor).
hipError_t launch_round(int cost, const Inst *inst, int ntiles, double *xfeas, hipStream_t s)
{
    const int grid = ntiles < 65536 ? ntiles : 65536;
    switch (cost) {
    case C_STORED: return launch_round_cost<C_STORED>(inst, xfeas, grid, s);
    case C_PTS_SQ: return launch_round_cost<C_PTS_SQ>(inst, xfeas, grid, s);
    case C_PTS_EU: return launch_round_cost<C_PTS_EU>(inst, xfeas, grid, s);
    case C_GRID_SQ: return launch_round_cost<C_GRID_SQ>(inst, xfeas, grid, s);
    case C_GRID_L1: return launch_round_cost<C_GRID_L1>(inst, xfeas, grid, s);
    case C_GRID_L2: return launch_round_cost<C_GRID_L2>(inst, xfeas, grid, s);
    case C_GRID_LINF: return launch_round_cost<C_GRID_LINF>(inst, xfeas, grid, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_zero(void *dst, size_t bytes, hipStream_t s)
{
    const int64_t words = (int64_t)(bytes / 8);
    if (words <= 0) return hipSuccess;
    int64_t blocks = (words + kWG - 1) / kWG;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(kWG), 0, s, (uint64_t *)dst, words);
    return hipGetLastError();
}

hipError_t launch_tables(Tile *tiles, int ntiles, int ncb, CombEntry *combs, int64_t m, int64_t n,
                         int32_t *counts, hipStream_t s)
{
    const int nrows = (int)((m + kCombEntries - 1) / kCombEntries);
    const int ncomb = nrows + (int)((n + kCombEntries - 1) / kCombEntries);
    const int most = ntiles > ncomb ? ntiles : ncomb;
    int blocks = (most + kWG - 1) / kWG;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_tables, dim3(blocks), dim3(kWG), 0, s, tiles, ntiles, ncb, combs, nrows, ncomb,
                       counts);
    return hipGetLastError();
}

hipError_t launch_materialize(int fp32, void *dst, int64_t m, int64_t n, int64_t ld, int kind,
                              const double *src, int64_t ldc, const double *xs, const double *ys,
                              int dim, int side, double scale, hipStream_t s)
{
    const int64_t total = m * ld;
    int64_t blocks = (total + kWG - 1) / kWG;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    if (fp32)
        hipLaunchKernelGGL(k_materialize<float>, dim3((unsigned)blocks), dim3(kWG), 0, s,
                           (float *)dst, m, n, ld, kind, src, ldc, xs, ys, dim, side, scale);
    else
        hipLaunchKernelGGL(k_materialize<double>, dim3((unsigned)blocks), dim3(kWG), 0, s,
                           (double *)dst, m, n, ld, kind, src, ldc, xs, ys, dim, side, scale);
    return hipGetLastError();
}

}  // namespace pdot
