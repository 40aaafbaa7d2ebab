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
//   KKT parts  ||[p_i+q_j-C_ij]^+||^2 for (p,q) and (pbar,qbar), <C,X>, <C,Xbar>
// Row sums are wave reductions; column sums stay in registers over the tile's rows, are
// combined across the four waves in LDS and written as one partial row per tile; k_combine
// adds the partials in a fixed order (deterministic, no floating-point atomics).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "pdot_internal.h"

namespace pdot {

// ------------------------------------------------------------------ small helpers

// Butterfly sum over the 64 lanes of a wave.  Every lane ends with the same value and the
// pairing is fixed, so the result does not depend on timing.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename T, int N>
struct alignas(sizeof(T) * N) Pack {
    T v[N];
};

template <typename T, int N>
__device__ __forceinline__ void load_pack(const T *__restrict__ p, T (&o)[N])
{
    const Pack<T, N> t = *reinterpret_cast<const Pack<T, N> *>(p);
#pragma unroll
    for (int i = 0; i < N; ++i) o[i] = t.v[i];
}

template <typename T, int N>
__device__ __forceinline__ void store_pack(T *__restrict__ p, const T (&o)[N])
{
    Pack<T, N> t;
#pragma unroll
    for (int i = 0; i < N; ++i) t.v[i] = o[i];
    *reinterpret_cast<Pack<T, N> *>(p) = t;
}

// Squared distance of two points, summed over coordinates in index order with every
// product and sum rounded separately (the same value wherever it is evaluated).
__device__ __forceinline__ double sqdist(const double *xi, const double *yj, int dim)
{
    double t = xi[0] - yj[0];
    double s = __dmul_rn(t, t);
    for (int k = 1; k < dim; ++k) {
        t = xi[k] - yj[k];
        s = __dadd_rn(s, __dmul_rn(t, t));
    }
    return s;
}

// Cost entry in the working precision TX, returned widened to FP64.  Used both by the
// materialising kernel and inside the pass, so stored and regenerated costs are equal.
template <typename TX>
__device__ __forceinline__ double round_to(double v)
{
    return (double)(TX)v;
}

__device__ __forceinline__ double grid_cost(int ia, int ib, int ja, int jb, double scale)
{
    const int da = ia - ja, db = ib - jb;
    return (double)(da * da + db * db) * scale;
}

// ------------------------------------------------------------------ streaming pass

template <typename TX, int VEC, int COST, int MODE>
__device__ void tile_body(const Inst &I, const Ctl &st, const Tile &tl, double *lds)
{
    constexpr int RU = 2;                       // rows in flight per wave
    constexpr bool kX = MODE != M_INIT;         // reads the plan
    constexpr bool kCost = MODE != M_RESTART;   // needs C
    constexpr bool kTrial = MODE == M_TRIAL || MODE == M_FULL;
    constexpr bool kFold = MODE == M_FULL;
    constexpr bool kRowCol = kTrial || MODE == M_VERIFY;
    constexpr bool kDres = MODE == M_FULL || MODE == M_VERIFY || MODE == M_INIT;

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t m = I.m, n = I.n, ld = I.ld;
    const int64_t i0 = (int64_t)tl.rb * I.rows;
    const int64_t i1 = min(m, i0 + (int64_t)I.rows);
    const int64_t j0 = (int64_t)tl.cb * (64 * VEC) + (int64_t)lane * VEC;
    const bool active = j0 < n;
    const bool full = j0 + VEC <= n;

    const int xc = (MODE == M_VERIFY) ? st.ret_x : st.xr[R_CUR];
    const TX *__restrict__ Xc = (const TX *)I.X[xc];
    TX *__restrict__ Xt = (TX *)I.X[st.xr[R_TRIAL]];
    TX *__restrict__ Xb = (TX *)I.X[st.xr[R_AVG]];
    const TX *__restrict__ Xa = (const TX *)I.X[st.xr[R_ANCHOR]];
    const TX *__restrict__ Cs = (const TX *)I.C;
    const bool use_avg_duals = (MODE == M_VERIFY) && st.ret_avg;
    const double *__restrict__ pc = use_avg_duals ? I.pb[st.pbv] : I.p[st.pv];
    const double *__restrict__ qc = use_avg_duals ? I.qb[st.pbv] : I.q[st.pv];
    const double *__restrict__ pbc = I.pb[st.pbv];
    const double *__restrict__ qbc = I.qb[st.pbv];
    const double tau = st.eta / st.omega;
    const double a = st.a_fold;
    const bool first_fold = st.k == 1;
    const double scale = I.scale;
    const int dim = I.dim, side = I.side;

    // per-lane column context
    double qv[VEC], qbv[VEC];
    int gja[VEC], gjb[VEC];
    double yc[VEC][3];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        const int64_t j = j0 + v;
        const bool ok = j < n;
        qv[v] = (ok && kDres) || (ok && kTrial) ? qc[j] : 0.0;
        qbv[v] = (ok && kFold) ? qbc[j] : 0.0;
        gja[v] = 0;
        gjb[v] = 0;
        yc[v][0] = yc[v][1] = yc[v][2] = 0.0;
        if constexpr (COST == C_GRID_SQ) {
            if (ok) {
                gja[v] = (int)(j / side);
                gjb[v] = (int)(j % side);
            }
        }
        if constexpr (COST == C_PTS_SQ || COST == C_PTS_EU) {
            if (ok)
                for (int k = 0; k < dim; ++k) yc[v][k] = I.ys[j * dim + k];
        }
    }

    double csv[VEC], csd[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) csv[v] = csd[v] = 0.0;
    double s_dx2 = 0.0, s_dres = 0.0, s_dresb = 0.0, s_pobj = 0.0, s_pobjb = 0.0, s_aux = 0.0;

    for (int64_t ib = i0 + wave; ib < i1; ib += 4 * RU) {
        TX xr[RU][VEC], cr[RU][VEC], br[RU][VEC], ar[RU][VEC];
        double pi[RU], pbi[RU];
        double xi[RU][3];
        int gia[RU], gib[RU];
        bool rv_ok[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int64_t i = ib + 4 * u;
            rv_ok[u] = i < i1;
            const int64_t ii = rv_ok[u] ? i : ib;      // clamp: loads stay in bounds
            const int64_t off = ii * ld + j0;
            pi[u] = (kTrial || kDres) ? pc[ii] : 0.0;
            pbi[u] = kFold ? pbc[ii] : 0.0;
            gia[u] = gib[u] = 0;
            xi[u][0] = xi[u][1] = xi[u][2] = 0.0;
            if constexpr (COST == C_GRID_SQ) {
                gia[u] = (int)(ii / side);
                gib[u] = (int)(ii % side);
            }
            if constexpr (COST == C_PTS_SQ || COST == C_PTS_EU) {
                for (int k = 0; k < dim; ++k) xi[u][k] = I.xs[ii * dim + k];
            }
#pragma unroll
            for (int v = 0; v < VEC; ++v) xr[u][v] = cr[u][v] = br[u][v] = ar[u][v] = (TX)0;
            if (active) {
                if constexpr (kX) load_pack<TX, VEC>(Xc + off, xr[u]);
                if constexpr (kCost && COST == C_STORED) load_pack<TX, VEC>(Cs + off, cr[u]);
                if constexpr (kFold) load_pack<TX, VEC>(Xb + off, br[u]);
                if constexpr (MODE == M_RESTART) load_pack<TX, VEC>(Xa + off, ar[u]);
            }
        }

        double rsum[RU], rdel[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            rsum[u] = rdel[u] = 0.0;
            if (!active || !rv_ok[u]) continue;
            const int64_t off = (ib + 4 * u) * ld + j0;
            TX xn_out[VEC], xb_out[VEC];
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                const bool ok = full || (j0 + v < n);
                const double xd = (double)xr[u][v];
                double cd = 0.0;
                if constexpr (kCost) {
                    if constexpr (COST == C_STORED) {
                        cd = (double)cr[u][v];
                    } else if constexpr (COST == C_GRID_SQ) {
                        cd = round_to<TX>(grid_cost(gia[u], gib[u], gja[v], gjb[v], scale));
                    } else {
                        double s2 = sqdist(xi[u], yc[v], dim);
                        if constexpr (COST == C_PTS_EU) s2 = sqrt(s2);
                        cd = round_to<TX>(s2);
                    }
                }
                xn_out[v] = (TX)0;
                xb_out[v] = (TX)0;
                if (!ok) continue;
                if constexpr (MODE == M_INIT) {
                    s_aux += cd * cd;
                    const double nd = (pi[u] + qv[v]) - cd;
                    s_dres += nd > 0.0 ? nd * nd : 0.0;
                }
                if constexpr (MODE == M_RESTART) {
                    const double d = xd - (double)ar[u][v];
                    s_aux += d * d;
                }
                if constexpr (MODE == M_VERIFY) {
                    const double nd = (pi[u] + qv[v]) - cd;
                    s_dres += nd > 0.0 ? nd * nd : 0.0;
                    s_pobj += cd * xd;
                    rsum[u] += xd;
                    csv[v] += xd;
                }
                if constexpr (kTrial) {
                    const double s = pi[u] + qv[v];
                    const double gr = cd - s;                 // G_ij = C_ij - p_i - q_j
                    if constexpr (kFold) {
                        // KKT pieces of the current iterate (its duals are p, q)
                        s_dres += gr < 0.0 ? gr * gr : 0.0;
                        s_pobj += cd * xd;
                        // fold the current iterate into the running average
                        const double xbn = first_fold ? xd : (1.0 - a) * (double)br[u][v] + a * xd;
                        const TX xbt = (TX)xbn;
                        xb_out[v] = xbt;
                        const double nb = (pbi[u] + qbv[v]) - cd;
                        s_dresb += nb > 0.0 ? nb * nb : 0.0;
                        s_pobjb += cd * (double)xbt;
                    }
                    const double y = xd - tau * gr;
                    const TX xn = (TX)(y > 0.0 ? y : 0.0);
                    xn_out[v] = xn;
                    const double xnd = (double)xn;
                    const double d = xnd - xd;
                    rsum[u] += xnd;
                    rdel[u] += d;
                    csv[v] += xnd;
                    csd[v] += d;
                    s_dx2 += d * d;
                }
            }
            if constexpr (kTrial) store_pack<TX, VEC>(Xt + off, xn_out);
            if constexpr (kFold) store_pack<TX, VEC>(Xb + off, xb_out);
        }
        if constexpr (kRowCol) {
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const double s = wave_sum(rsum[u]);
                double d = 0.0;
                if constexpr (kTrial) d = wave_sum(rdel[u]);
                if (lane == 0 && rv_ok[u]) {
                    const int64_t i = ib + 4 * u;
                    I.rowpart[(int64_t)(2 * tl.cb) * m + i] = s;
                    if constexpr (kTrial) I.rowpart[(int64_t)(2 * tl.cb + 1) * m + i] = d;
                }
            }
        }
    }

    // column partials: combine the four waves in a fixed order
    if constexpr (kRowCol) {
        double *cl = lds;   // [3][2*VEC][64]
        if (wave > 0) {
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                cl[((wave - 1) * 2 * VEC + 2 * v) * 64 + lane] = csv[v];
                cl[((wave - 1) * 2 * VEC + 2 * v + 1) * 64 + lane] = csd[v];
            }
        }
        __syncthreads();
        if (wave == 0 && active) {
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                double sv = csv[v], sd = csd[v];
                for (int w = 0; w < 3; ++w) {
                    sv += cl[(w * 2 * VEC + 2 * v) * 64 + lane];
                    sd += cl[(w * 2 * VEC + 2 * v + 1) * 64 + lane];
                }
                const int64_t j = j0 + v;
                if (j < n) {
                    I.colpart[(int64_t)(2 * tl.rb) * n + j] = sv;
                    if constexpr (kTrial) I.colpart[(int64_t)(2 * tl.rb + 1) * n + j] = sd;
                }
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
            const double r = wave_sum(vals[s]);
            if (lane == 0) sl[wave * kNS + s] = r;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double *dst = I.tilescal + (int64_t)tl.local * kNS;
            for (int s = 0; s < kNS; ++s)
                dst[s] = ((sl[s] + sl[kNS + s]) + sl[2 * kNS + s]) + sl[3 * kNS + s];
        }
        __syncthreads();
    }
}

template <typename TX, int VEC, int COST>
__global__ __launch_bounds__(kWG) void k_pass(const Inst *__restrict__ insts,
                                              const Tile *__restrict__ tiles, int ntiles)
{
    __shared__ double lds[3 * 2 * 4 * 64 + 4 * kNS];
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const Tile tl = tiles[t];
        const Inst &I = insts[tl.inst];
        const Ctl st = *I.ctl;
        switch (st.mode) {
        case M_INIT: tile_body<TX, VEC, COST, M_INIT>(I, st, tl, lds); break;
        case M_TRIAL: tile_body<TX, VEC, COST, M_TRIAL>(I, st, tl, lds); break;
        case M_FULL: tile_body<TX, VEC, COST, M_FULL>(I, st, tl, lds); break;
        case M_RESTART: tile_body<TX, VEC, COST, M_RESTART>(I, st, tl, lds); break;
        case M_VERIFY: tile_body<TX, VEC, COST, M_VERIFY>(I, st, tl, lds); break;
        default: break;
        }
    }
}

// ------------------------------------------------------------------ control (one thread)

// Relative KKT error (Section 3.1 stacked norm, each block over its own scale; kkt_mode 1
// uses 1 + scale denominators).  out = {rel_P, rel_D, rel_G}.
__device__ double rel_kkt(const Prm &P, double nb, double nc, double pres2, double dres2,
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

enum { ST_RUNNING = -1, ST_OK = 0, ST_NOT_CONVERGED = 4, ST_NUMERIC = 5 };

__device__ void finish(Ctl &c, const Prm &P, int status)
{
    c.status = status;
    c.ret_avg = (P.output == 0 && c.cand_avg && c.T > 0 && c.k > 0) ? 1 : 0;
    c.ret_x = c.ret_avg ? c.xr[R_AVG] : c.xr[R_CUR];
    c.mode = M_VERIFY;
}

__device__ bool limits_hit(const Ctl &c, const Prm &P)
{
    return c.T >= P.max_iters || c.passes >= P.max_passes || c.stop;
}

// Step-size check of the trial (Section 5, adaptive step size).
__device__ void step_decide(Ctl &c, const Prm &P, double dx2, double dy2, double inter)
{
    c.passes += 1;
    const double eta_used = c.eta;
    bool accept = true;
    if (P.step_rule == 0) {
        const double num = c.omega * dx2 + dy2 / c.omega;
        const double den = 2.0 * fabs(inter);
        const double eta_bar = den > 0.0 ? num / den : INFINITY;
        accept = c.eta <= eta_bar;
        const double tt = (double)(c.T + 1);
        const double shrink = (1.0 - pow(tt, -P.red_exp)) * eta_bar;
        const double grow = (1.0 + pow(tt, -P.grow_exp)) * c.eta;
        c.eta = shrink < grow ? shrink : grow;
        if (!(num == num) || !(c.eta == c.eta)) {   // NaN guard
            c.status = ST_NUMERIC;
            c.mode = M_IDLE;
            return;
        }
    }
    if (accept) {
        const int old_cur = c.xr[R_CUR];
        const int new_cur = c.xr[R_TRIAL];
        int nt = old_cur;
        if (old_cur == c.xr[R_ANCHOR]) {
            for (int b = 0; b < 4; ++b)
                if (b != new_cur && b != c.xr[R_AVG] && b != c.xr[R_ANCHOR]) nt = b;
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
        c.mode = M_FULL;
    } else {
        c.mode = M_TRIAL;
        if (c.passes >= P.max_passes || c.stop) finish(c, P, ST_NOT_CONVERGED);
    }
}

__device__ void control(Ctl &c, const Prm &P, int mode, const double *cs, const double *ts)
{
    c.kpasses += 1;
    if (mode == M_INIT) {
        c.norm_b = sqrt(cs[CS_AUX]);
        c.norm_c = sqrt(ts[TS_AUX]);
        const double K = rel_kkt(P, c.norm_b, c.norm_c, cs[CS_AUX], ts[TS_DRES], 0.0, 0.0, nullptr);
        c.K_start = c.K_prev = c.K_cand = K;
        c.cand_avg = 0;
        if (!(K == K) || !(c.norm_c < INFINITY)) {
            c.status = ST_NUMERIC;
            c.mode = M_IDLE;
        } else if (K <= P.tol) {
            finish(c, P, ST_OK);
        } else if (limits_hit(c, P)) {
            finish(c, P, ST_NOT_CONVERGED);
        } else {
            c.mode = M_TRIAL;
        }
        return;
    }
    if (mode == M_TRIAL) {
        step_decide(c, P, ts[TS_DX2], cs[CS_DY2], cs[CS_INTER]);
        return;
    }
    if (mode == M_FULL) {
        const double kc = rel_kkt(P, c.norm_b, c.norm_c, cs[CS_PRES], ts[TS_DRES], ts[TS_POBJ],
                                  cs[CS_DOBJ], nullptr);
        const double ka = rel_kkt(P, c.norm_b, c.norm_c, cs[CS_PRESB], ts[TS_DRESB],
                                  ts[TS_POBJB], cs[CS_DOBJB], nullptr);
        // restart candidate (Section 5): the current iterate only if strictly better
        c.cand_avg = !(kc < ka);
        double K = c.cand_avg ? ka : kc;
        if (!(K == K)) {
            c.status = ST_NUMERIC;
            c.mode = M_IDLE;
            return;
        }
        c.K_cand = K;
        if (K <= P.tol) {
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
        if (restart) {
            if (c.cand_avg) c.xr[R_CUR] = c.xr[R_AVG];
            c.K_start = K;
            c.K_prev = K;
            c.mode = M_RESTART;
            return;
        }
        c.K_prev = K;
        if (limits_hit(c, P)) {
            finish(c, P, ST_NOT_CONVERGED);
            return;
        }
        step_decide(c, P, ts[TS_DX2], cs[CS_DY2], cs[CS_INTER]);
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
        int others[3], no = 0;
        for (int b = 0; b < 4; ++b)
            if (b != cur) others[no++] = b;
        c.xr[R_TRIAL] = others[0];
        c.xr[R_AVG] = others[1];
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
        if (c.status == ST_OK && !(K == K)) c.status = ST_NUMERIC;
        c.mode = M_IDLE;
        return;
    }
}

// ------------------------------------------------------------------ combine + control

__device__ __forceinline__ double block_sum(double v, double *sl)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) sl[wave] = v;
    __syncthreads();
    const double r = ((sl[0] + sl[1]) + sl[2]) + sl[3];
    return r;
}

__global__ __launch_bounds__(kWG) void k_combine(const Inst *__restrict__ insts,
                                                 const CombEntry *__restrict__ ents, int nents)
{
    __shared__ double part[4][2][64];
    __shared__ double sl[8];
    __shared__ double fin[kNC + kNS];
    __shared__ int is_last;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

    for (int e = blockIdx.x; e < nents; e += gridDim.x) {
        const CombEntry E = ents[e];
        const Inst &I = insts[E.inst];
        const Ctl st = *I.ctl;
        const int mode = st.mode;
        if (mode == M_IDLE) continue;
        const Prm &P = I.prm;

        const bool rows = E.kind == 0;
        const int64_t len = rows ? I.m : I.n;
        const int64_t idx = (int64_t)E.start + lane;
        const bool valid = idx < len;

        // phase 1: add the per-tile partial sums of this slice in a fixed order
        double sv = 0.0, sd = 0.0;
        if (mode == M_TRIAL || mode == M_FULL || mode == M_VERIFY) {
            const int P4 = rows ? I.ncb : I.nrb;
            const double *src = rows ? I.rowpart : I.colpart;
            const int pb = (wave * P4) / 4, pe = ((wave + 1) * P4) / 4;
            if (valid) {
                for (int pp = pb; pp < pe; ++pp) {
                    sv += src[(int64_t)(2 * pp) * len + idx];
                    if (mode != M_VERIFY) sd += src[(int64_t)(2 * pp + 1) * len + idx];
                }
            }
            part[wave][0][lane] = sv;
            part[wave][1][lane] = sd;
            __syncthreads();
            if (wave == 0) {
                sv = ((part[0][0][lane] + part[1][0][lane]) + part[2][0][lane]) + part[3][0][lane];
                sd = ((part[0][1][lane] + part[1][1][lane]) + part[2][1][lane]) + part[3][1][lane];
            }
            __syncthreads();
        }

        // phase 2: per-entry vector work (wave 0, one row or column per lane)
        if (wave == 0) {
            double acc[kNC];
#pragma unroll
            for (int s = 0; s < kNC; ++s) acc[s] = 0.0;
            if (valid) {
                const double fi = rows ? I.f[idx] : I.g[idx];
                double *const *pv2 = rows ? I.p : I.q;
                double *const *pb2 = rows ? I.pb : I.qb;
                double *const *rs2 = rows ? I.rs : I.cs;
                double *sbar = rows ? I.rsb : I.csb;
                double *anc = rows ? I.pa : I.qa;
                double *pcur = pv2[st.pv];
                double *pbcur = pb2[st.pbv];
                if (mode == M_INIT) {
                    acc[CS_AUX] = fi * fi;
                } else if (mode == M_TRIAL || mode == M_FULL) {
                    if (mode == M_FULL) {
                        // KKT of the current iterate: its sums were kept when it was accepted
                        const double rc = rs2[st.rsv][idx];
                        double dl = rc - fi;
                        acc[CS_PRES] = dl * dl;
                        acc[CS_DOBJ] = fi * pcur[idx];
                        // averaged sums (linear in the plan), same weights as the plan average
                        const double nb = (st.k == 1) ? rc : (1.0 - st.a_fold) * sbar[idx] + st.a_fold * rc;
                        sbar[idx] = nb;
                        dl = nb - fi;
                        acc[CS_PRESB] = dl * dl;
                        acc[CS_DOBJB] = fi * pbcur[idx];
                    }
                    // dual step with the extrapolated sums (2X+ - X) = X+ + (X+ - X)
                    const double sigma = st.eta * st.omega;
                    const double er = sv + sd;
                    const double pold = pcur[idx];
                    const double pn = pold + sigma * (fi - er);
                    const double d = pn - pold;
                    pv2[st.pv ^ 1][idx] = pn;
                    rs2[st.rsv ^ 1][idx] = sv;
                    acc[CS_DY2] = d * d;
                    acc[CS_INTER] = d * sd;
                    // tentative running average of the duals for the trial
                    const double w = P.avg_weighting == 1 ? 1.0 : st.eta;
                    const double a2 = w / (st.wsum + w);
                    pb2[st.pbv ^ 1][idx] = (st.k == 0) ? pn : (1.0 - a2) * pbcur[idx] + a2 * pn;
                } else if (mode == M_RESTART) {
                    const double pnew = st.cand_avg ? pbcur[idx] : pcur[idx];
                    const double dd = pnew - anc[idx];
                    acc[CS_AUX] = dd * dd;
                    pcur[idx] = pnew;
                    anc[idx] = pnew;
                    if (st.cand_avg) rs2[st.rsv][idx] = sbar[idx];
                } else if (mode == M_VERIFY) {
                    const double *pret = st.ret_avg ? pbcur : pcur;
                    const double dl = sv - fi;
                    acc[CS_PRES] = dl * dl;
                    acc[CS_DOBJ] = fi * pret[idx];
                }
            }
#pragma unroll
            for (int s = 0; s < kNC; ++s) {
                const double r = wave_sum(acc[s]);
                if (lane == 0) I.combscal[(int64_t)E.local * kNC + s] = r;
            }
        }

        // phase 3: the last work-group of this instance runs the control
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned prev = atomicAdd(I.counter, 1u);
            is_last = (prev == (unsigned)(I.ncomb - 1)) ? 1 : 0;
        }
        __syncthreads();
        if (!is_last) continue;
        __threadfence();

        double loc[kNC + kNS];
#pragma unroll
        for (int s = 0; s < kNC + kNS; ++s) loc[s] = 0.0;
        for (int c = threadIdx.x; c < I.ncomb; c += kWG) {
            const double *src = I.combscal + (int64_t)c * kNC;
#pragma unroll
            for (int s = 0; s < kNC; ++s) loc[s] += __hip_atomic_load(src + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        for (int t = threadIdx.x; t < I.ntiles; t += kWG) {
            const double *src = I.tilescal + (int64_t)t * kNS;
#pragma unroll
            for (int s = 0; s < kNS; ++s) loc[kNC + s] += src[s];
        }
        for (int s = 0; s < kNC + kNS; ++s) {
            const double r = block_sum(loc[s], sl);
            if (threadIdx.x == 0) fin[s] = r;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            Ctl c = *I.ctl;
            control(c, P, mode, fin, fin + kNC);
            *I.ctl = c;
            __hip_atomic_store(I.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
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
            } else if (kind == C_GRID_SQ) {
                v = grid_cost((int)(i / side), (int)(i % side), (int)(j / side), (int)(j % side), scale);
            } else {
                v = sqdist(xs + i * dim, ys + j * dim, dim);
                if (kind == C_PTS_EU) v = sqrt(v);
            }
        }
        dst[e] = (TX)v;
    }
}

}  // namespace pdot

// ------------------------------------------------------------------ launchers (host)

namespace pdot {

template <typename TX, int VEC>
static hipError_t launch_pass_vec(int cost, const Inst *insts, const Tile *tiles, int ntiles,
                                  int grid, hipStream_t s)
{
    switch (cost) {
    case C_STORED: hipLaunchKernelGGL((k_pass<TX, VEC, C_STORED>), dim3(grid), dim3(kWG), 0, s, insts, tiles, ntiles); break;
    case C_PTS_SQ: hipLaunchKernelGGL((k_pass<TX, VEC, C_PTS_SQ>), dim3(grid), dim3(kWG), 0, s, insts, tiles, ntiles); break;
    case C_PTS_EU: hipLaunchKernelGGL((k_pass<TX, VEC, C_PTS_EU>), dim3(grid), dim3(kWG), 0, s, insts, tiles, ntiles); break;
    case C_GRID_SQ: hipLaunchKernelGGL((k_pass<TX, VEC, C_GRID_SQ>), dim3(grid), dim3(kWG), 0, s, insts, tiles, ntiles); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename TX>
static hipError_t launch_pass_t(int vec, int cost, const Inst *insts, const Tile *tiles,
                                int ntiles, int grid, hipStream_t s)
{
    switch (vec) {
    case 1: return launch_pass_vec<TX, 1>(cost, insts, tiles, ntiles, grid, s);
    case 2: return launch_pass_vec<TX, 2>(cost, insts, tiles, ntiles, grid, s);
    case 4: return launch_pass_vec<TX, 4>(cost, insts, tiles, ntiles, grid, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pass(int fp32, int vec, int cost, const Inst *insts, const Tile *tiles,
                       int ntiles, int grid, hipStream_t s)
{
    return fp32 ? launch_pass_t<float>(vec, cost, insts, tiles, ntiles, grid, s)
                : launch_pass_t<double>(vec, cost, insts, tiles, ntiles, grid, s);
}

hipError_t launch_combine(const Inst *insts, const CombEntry *ents, int nents, int grid,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_combine, dim3(grid), dim3(kWG), 0, s, insts, ents, nents);
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
