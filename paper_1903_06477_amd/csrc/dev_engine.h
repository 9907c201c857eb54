// SuperSCS engine on the device, written once for any team (dev_common.h).
//
//   linear_step   u~ = (I + Q)^{-1} r, equation (drs) first line, by block
//                 elimination to (I + A^T A) px = rx - A^T ry, Jacobi-
//                 preconditioned CG, py = ry + A px, then the rank-one tau
//                 correction with g = M^{-1} (c, b) and delta = 1 + (c, b)^T g.
//   residual      u-bar = Pi_C(2 u~ - u), R u = u~ - u-bar  (equation (drs), R = I - T)
//   termination   pr, dr, gap, ic, uc of Sec. IV-C from (u, u~, u-bar)
//   directions    Anderson (Sec. IV-D-2) and restarted Broyden (Algorithm 2)
//   line search   w = u + a d, w~ = u~ + a d~ (linearity of (I+Q)^{-1}, Sec. IV-B),
//                 Rw = w~ - Pi_C(2 w~ - w), K1 / K2 tests of Algorithm 1
//   solve         Algorithm 1
//
// All scalar control (CG recurrences, step decisions, Gram solves) is FP64 and
// is computed identically by every thread from deterministic team reductions,
// so no decision ever diverges across the team and no host round trip sits
// inside an iteration.
#pragma once
#include "dev_common.h"
#include "dev_cones.h"

namespace sscs {

enum { ST_SOLVED = 1, ST_INFEASIBLE = 2, ST_UNBOUNDED = 3, ST_MAX_ITERS = 4, ST_TIME_LIMIT = 5,
       ST_NUMERICAL = 6 };
enum { DIR_RB = 0, DIR_AA = 1, DIR_RES = 2, DIR_ZERO = 3, DIR_SCS = 4, DIR_AA_QR = 5 };

struct Prob {
    int n, m, N;
    Csr<double> A, At;
    Csr<float> Af, Atf;     // FP32 copies of the values (mixed precision; same rp, ci)
    const double* b;
    const double* c;
    const double* dinv;     // 1 / (1 + ||A e_j||^2), Jacobi preconditioner of I + A^T A
    const double* g;        // M^{-1} (c, b), length n + m
    const int* partA;       // row partition of A over the workgroups of a grid (G + 1)
    const int* partAt;      // row partition of A^T
    int lds_cache;          // grid kernels keep their rows of A and A^T in LDS
    // direct linear step: (I + A^T A)^{-1}, n x n and symmetric (row j is
    // contiguous); null for the CG
    const double* Minv;
    double delta;           // 1 + (c, b)^T g
    double nb, nc;          // ||b||, ||c||
    ConeDev K;
};

struct Vecs {
    double *u, *ut, *ub, *Ru, *d, *dt, *Rw, *pz, *pxi;   // length N
    double *xw_u, *xw_d;                                 // CG warm starts, length n
    double *q_u, *q_d;                                   // K xw_u, K xw_d as the CG left them, length n
    double *cg_b, *cg_u, *cg_w, *cg_p, *cg_r, *cg_s;     // length n
    double* rhs_u;                                       // the u~ solve's right-hand side (grid teams), length n
    double *cg_g[2];                                     // 4 n each: gathered (D r, D s, D w, -) per column
    double *cg_t;                                        // length m
    double *Zb, *Yb;                                     // mem x N memory buffers
    double* Qb;                                          // mem x N: Q of Xi = Q R (Anderson by QR)
    const double* u0;                                    // warm start or null
    double *out_x, *out_y, *out_s;                       // results
    double* tr_res;                                      // trace (may be null)
    int *tr_kind, *tr_ls;
    double *tr_eta, *tr_rsafe;                           // eta and r_safe after each step
    long long tr_cap;
};

struct Params {
    double eps, c0, c1, q, sigma, lam, thetabar, aa_reg;
    double cg_tol;
    double cg_adapt;        // > 0: CG tolerance cg_adapt ||R u|| / ||u||, within [cg_tol, 1e-3]
    int cg_d_match;         // with cg_adapt > 0: d~'s CG stops at the absolute threshold of u~'s
    int direction, mem, ls_max, cg_max;
    int check_every;        // termination test every check_every-th iteration
    long long max_iters;
    long long max_ticks;    // time limit in wall-clock ticks, <= 0: none
    double setup_tol;       // CG tolerance of the one-off solve for g
    int setup_max;
};

struct Result {
    int status, err;
    long long iters, k0, k1, k2, km, bt, cg;
    double pr, dr, gap, ic, uc, pobj, dobj, res;
};

// ------------------------------------------------------------------ linear step

// out[0 .. n+m) = M^{-1} r[0 .. n+m), warm-starting CG from xw (updated in place).
// Leaves h^T M^{-1} r in sh.out[0]; returns the CG iteration count.  CG stops
// once ||K x - rhs||^2 <= thr, where thr = thr_abs if thr_abs > 0, else
// tol^2 ||rhs||^2 (rhs = r_x - A^T r_y); the threshold used is stored to
// *thr_used when given.
//
// The CG on K = I + A^T A (Jacobi preconditioner D) is the single-reduction
// (Chronopoulos-Gear) recurrence: with u = D r and w = K u,
//   gamma = <r, u>, delta = <w, u>,  beta = gamma / gamma_old,
//   alpha = gamma / (delta - beta gamma / alpha_old),
//   p = u + beta p,  s = w + beta s,  x += alpha p,  r -= alpha s.
// One iteration is two team-wide phases:
//   X: element owners update p, s, x, r, u; the owners of the rows of A form
//      t = A u_new, gathering u_new,k = D_k r_k - alpha (D_k w_k + beta D_k s_k)
//      from one 32-byte record (D r, D s, D w) per column of the previous
//      step -- no barrier is needed between the update and the product, and
//      each gathered column costs one cache line;
//   Y: the owners of the rows of A^T form w = u + A^T t, the record's D w and
//      the partial sums of gamma, delta and ||r||^2; one reduction.
// The records are double-buffered: X reads buffer cur and fills (D r, D s)
// of buffer cur^1, Y fills its D w.  The first pass runs with alpha = 0 and
// p = s = w = 0, which turns phase X into u = D r0, t = A u.
// The CG operator I + A^T A in value type T: FP64 (the parity path) or the
// FP32 copies of A and A^T (mixed precision).  Every other product uses FP64.
template <typename T>
__device__ __forceinline__ const Csr<T>& op_mat(const Prob& P, int which) {
    if constexpr (std::is_same<T, float>::value) return which ? P.Atf : P.Af;
    else return which ? P.At : P.A;
}

// Refinement rounds of a mixed-precision solve: each round recomputes the
// residual r0 = rhs - K xw with the FP64 operator and runs CG with the FP32
// one from there; a round whose FP64 residual already meets the tolerance
// ends the solve.  FP64 solves take a single round.
template <typename T>
__device__ __forceinline__ int cg_rounds() {
    return std::is_same<T, float>::value ? 4 : 1;
}

// One-workgroup form of solve_M: the workgroup owns every row, so the vectors
// the two products gather from (u for A, t for A^T) live in LDS and the
// column records are not needed; each iteration is: update and store u in
// LDS, reduce ||r||^2 | t = A u into LDS | w = u + A^T t and the dots.  Same
// recurrence as solve_M; since a workgroup barrier is cheap, the stopping
// test runs right after the update, before the product the next step would
// need (solve_M folds it into the dots' reduction to save a grid barrier, at
// the price of one product more per solve).  q and refresh as in solve_M.
template <typename TV, typename Team>
__device__ int solve_M_staged(Team& tm, Shared& sh, const Prob& P, const Vecs& V, const double* r, double* out,
                              double* xw, double tol, int maxit, double thr_abs, double* thr_used, double* q,
                              bool refresh) {
    const int n = P.n, m = P.m;
    // the small-instance kernel holds the staging, the CG's vectors, the warm
    // start and K xw, and D, b, c in LDS (Team::kLds)
    constexpr bool L = Team::kLds;
    const auto ul = vec_at<L>(tm.lu);
    const auto tl = vec_at<L>(tm.lt);
    const auto cr = vec_at<L>(V.cg_r);
    const auto cs = vec_at<L>(V.cg_s);
    const auto cu = vec_at<L>(V.cg_u);
    const auto cw = vec_at<L>(V.cg_w);
    const auto cp = vec_at<L>(V.cg_p);
    const auto cb = vec_at<L>(V.cg_b);
    const auto xl = vec_at<L>(xw);
    const auto dv = vec_at<L>(P.dinv);
    const auto bv = vec_at<L>(P.b);
    const auto cv = vec_at<L>(P.c);
    const Csr<TV>& KA = op_mat<TV>(P, 0);
    const Csr<TV>& KAt = op_mat<TV>(P, 1);
    constexpr bool kQ = std::is_same<TV, double>::value;
    if constexpr (!kQ) q = nullptr;
    const bool use_q = q != nullptr && !refresh;
    auto start = [&](int j, double rj) {          // r0 = rj; p = s = w = 0
        cr[j] = rj;
        cs[j] = 0.0;
        cu[j] = 0.0;
        cw[j] = 0.0;
        cp[j] = 0.0;
    };
    for (int i = tm.rank(); i < m; i += tm.size()) tl[i] = r[n + i];
    tm.sync();
    // rhs = rx - A^T ry
    double a_bb = 0.0;
    spmv_part<1>(tm, P.At, 1, [&](int c_) { return tl[c_]; }, [&](int j, double s) {
        const double bj = r[j] - s;
        cb[j] = bj;
        a_bb += bj * bj;
        if (use_q) start(j, bj - vec_at<L>(q)[j]);
    });
    double thr = 0.0;
    int it = 0;
    const int rounds = cg_rounds<TV>();
    for (int round = 0; round < rounds; ++round) {
        if (!(use_q && round == 0)) {
            // r0 = rhs - (xw + A^T A xw) in FP64
            for (int j = tm.rank(); j < n; j += tm.size()) ul[j] = xl[j];
            tm.sync();
            spmv_part<1>(tm, P.A, 0, [&](int c_) { return ul[c_]; }, [&](int i, double s) { tl[i] = s; });
            tm.sync();
            spmv_part<1>(tm, P.At, 1, [&](int c_) { return tl[c_]; },
                         [&](int j, double s) { start(j, cb[j] - (xl[j] + s)); });
        }
        tm.sync();
        double alpha = 0.0, beta = 0.0, gamma_old = 1.0, alpha_old = 1.0;
        bool done = false;
        for (int pass = 0;; ++pass) {
            double a_rr = 0.0;
            for (int j = tm.rank(); j < n; j += tm.size()) {
                const double pj = cu[j] + beta * cp[j];
                const double sj = cw[j] + beta * cs[j];
                const double rj = cr[j] - alpha * sj;
                const double uj = dv[j] * rj;
                xl[j] += alpha * pj;
                cp[j] = pj;
                cs[j] = sj;
                cr[j] = rj;
                cu[j] = uj;
                ul[j] = uj;
                a_rr += rj * rj;
            }
            put(sh, 0, a_rr);
            if (round == 0 && pass == 0) put(sh, 1, a_bb);
            tm.reduce(sh, (round == 0 && pass == 0) ? 2 : 1);
            const double rr = sh.out[0];
            if (round == 0 && pass == 0) {
                thr = thr_abs > 0.0 ? thr_abs : tol * tol * sh.out[1];
                if (thr_used) *thr_used = thr;
            }
            // at least one step per solve: a warm start that already meets the
            // tolerance would otherwise be returned as is, and its error would
            // stay at the tolerance from one outer iteration to the next
            if (!(rr > thr) && (it > 0 || round > 0)) {
                done = pass == 0;            // the FP64 residual itself meets the tolerance
                break;
            }
            if (it >= maxit) {
                done = true;
                break;
            }
            spmv_part<4>(tm, KA, 0, [&](int c) { return ul[c]; }, [&](int i, double acc) { tl[i] = acc; });
            tm.sync();
            double a_g = 0.0, a_d = 0.0;
            spmv_part<4>(tm, KAt, 1, [&](int c) { return tl[c]; }, [&](int j, double s) {
                const double uj = cu[j];
                const double rj = cr[j];
                const double wj = uj + s;
                cw[j] = wj;
                a_g += rj * uj;
                a_d += wj * uj;
            });
            put(sh, 0, a_g);
            put(sh, 1, a_d);
            tm.reduce(sh, 2);
            const double gamma = sh.out[0], delta = sh.out[1];
            double den = delta;
            if (pass == 0) {
                beta = 0.0;
            } else {
                beta = gamma / gamma_old;
                den = delta - beta * gamma / alpha_old;
            }
            if (!(gamma > 0.0) || !(den > 0.0)) break;
            alpha = gamma / den;
            gamma_old = gamma;
            alpha_old = alpha;
            ++it;
        }
        if (done) break;
    }
    // py = ry + A px ; h^T p
    for (int j = tm.rank(); j < n; j += tm.size()) ul[j] = xl[j];
    tm.sync();
    double a_hp = 0.0;
    spmv_part<1>(tm, P.A, 0, [&](int c_) { return ul[c_]; }, [&](int i, double s) {
        const double py = r[n + i] + s;
        out[n + i] = py;
        a_hp += bv[i] * py;
    });
    for (int j = tm.rank(); j < n; j += tm.size()) {
        out[j] = xl[j];
        a_hp += cv[j] * xl[j];
        if (q) vec_at<L>(q)[j] = cb[j] - cr[j];
    }
    put(sh, 0, a_hp);
    tm.reduce(sh, 1);
    return it;
}

// Out of line: the CG loop then gets a register allocation of its own,
// independent of the rest of the solve kernel it is called from.
// Direct form of solve_M (Sec. IV-A, the reduced system solved directly):
// rhs = r_x - A^T r_y, then x = M^{-1} rhs with the inverse formed once from
// the Cholesky factor (a dense symmetric product: one wavefront per row,
// coalesced, over the whole team, so the step is bound by reading M^{-1}
// rather than by the substitutions' chain of dependent blocks), then
// (x, r_y + A x) and h^T p.  xw and q are set to x and K x = rhs, so the
// CG's bookkeeping stays consistent.  Returns 0 (no CG iterations).
template <typename Team>
__device__ __noinline__ int solve_direct(Team& tm, Shared& sh, const Prob& P, const Vecs& V, const double* r,
                                         double* out, double* xw, double* q) {
    const int n = P.n;
    double* rh = V.cg_b;
    double* xs = V.cg_r;
    spmv_part<1>(tm, P.At, 1, [&](int c_) { return r[n + c_]; }, [&](int j, double s) { rh[j] = r[j] - s; });
    tm.sync();
    const int lane = threadIdx.x & (WAVE - 1);
    for (int j = tm.wave(); j < n; j += tm.nwaves()) {
        const double* row = P.Minv + (size_t)j * n;
        double a0 = 0.0, a1 = 0.0;
        int k = lane;
        for (; k + WAVE < n; k += 2 * WAVE) {
            a0 += row[k] * rh[k];
            a1 += row[k + WAVE] * rh[k + WAVE];
        }
        if (k < n) a0 += row[k] * rh[k];
        const double x = group_sum(a0 + a1, WAVE);
        if (lane == WAVE - 1) xs[j] = x;
    }
    tm.sync();
    // py = ry + A x ; h^T p
    double a_hp = 0.0;
    spmv_part<1>(tm, P.A, 0, [&](int c_) { return xs[c_]; }, [&](int i, double s) {
        const double py = r[n + i] + s;
        out[n + i] = py;
        a_hp += P.b[i] * py;
    });
    for (int j = tm.rank(); j < n; j += tm.size()) {
        const double xj = xs[j];
        out[j] = xj;
        a_hp += P.c[j] * xj;
        xw[j] = xj;
        if (q) q[j] = rh[j];
    }
    put(sh, 0, a_hp);
    tm.reduce(sh, 1);
    return 0;
}

// Per-row operands a pass prefetches ahead of the row's gathers (spmv_part_pre).
struct Row3 {
    double a, b, c;
};
struct Row4 {
    double a, b, c, d;
};

template <typename TV, typename Team>
__device__ __noinline__ int solve_M(Team& tm, Shared& sh, const Prob& P, const Vecs& V, const double* r, double* out,
                       double* xw, double tol, int maxit, double thr_abs = 0.0, double* thr_used = nullptr,
                       double* q = nullptr, bool refresh = true, double* rb = nullptr, bool prestarted = false,
                       double bb_part = 0.0) {
    if (P.Minv) return solve_direct(tm, sh, P, V, r, out, xw, q);
    if constexpr (Team::kBlock) {
        if (tm.lu) return solve_M_staged<TV>(tm, sh, P, V, r, out, xw, tol, maxit, thr_abs, thr_used, q, refresh);
    }
    const int n = P.n;
    const Csr<TV>& KA = op_mat<TV>(P, 0);
    const Csr<TV>& KAt = op_mat<TV>(P, 1);
    // q (optional, FP64 operator only) holds K xw as the previous solve's
    // recurrence left it (K x = rhs - r): then r0 = rhs - q needs no product,
    // which saves two products and a barrier per solve.  The recurrence
    // residual drifts from the true one by rounding only; refresh recomputes
    // r0 from scratch.
    constexpr bool kQ = std::is_same<TV, double>::value;
    if constexpr (!kQ) q = nullptr;
    const bool use_q = q != nullptr && !refresh;
    // FP64 solves end one pass early: the reduction that gives alpha and beta
    // also gives <r,w>, <r,s>, <w,w>, <w,s> and <s,s>, from which the
    // recurrence residual after the step, ||r - alpha (w + beta s)||^2,
    // follows without the step's products.  When it meets the threshold the
    // step is left pending and the closing pass applies it (x + alpha (u +
    // beta p), formed where it is gathered): the last pass's two products and
    // two barriers are saved.  The iterates are the same as without it.
    constexpr bool kPred = kQ && !Team::kBlock;   // grid teams (the one-workgroup kernel has no registers to spare)
    constexpr int KD = kPred ? 8 : 3;             // dot products per CG reduction
    bool pend = false;
    double fa = 0.0, fb = 0.0;
    int cur = 0;
    auto start = [&](int j, double rj) {          // r0 = rj; u = w = p = s = 0; record (D r0, 0, 0)
        V.cg_r[j] = rj;
        V.cg_s[j] = 0.0;
        V.cg_u[j] = 0.0;
        V.cg_w[j] = 0.0;
        V.cg_p[j] = 0.0;
        double* g = V.cg_g[cur] + 4 * (size_t)j;
        g[0] = P.dinv[j] * rj;
        g[1] = 0.0;
        g[2] = 0.0;
    };
    // rhs = rx - A^T ry, into rb (default the CG's own buffer).  prestarted:
    // the caller has already formed the rhs in rb and, with use_q, started
    // the CG from it (r0 = rhs - q, as start() below) in a pass that ended
    // with a team barrier; bb_part is this thread's part of ||rhs||^2.
    double* const B = rb ? rb : V.cg_b;
    double a_bb = bb_part;
    if (!prestarted)
        spmv_part_pre<4>(tm, P.At, 1, [&](int c_) { return (r + n)[c_]; },
                         [&](int j) { return Row3{r[j], use_q ? q[j] : 0.0, use_q ? P.dinv[j] : 0.0}; },
                         [&](int j, double s, const Row3& o) {     // o = (r_j, q_j, D_j)
                             const double bj = o.a - s;
                             B[j] = bj;
                             a_bb += bj * bj;
                             if (use_q) {                  // start(j, bj - q_j) with D_j prefetched
                                 const double rj = bj - o.b;
                                 V.cg_r[j] = rj;
                                 V.cg_s[j] = 0.0;
                                 V.cg_u[j] = 0.0;
                                 V.cg_w[j] = 0.0;
                                 V.cg_p[j] = 0.0;
                                 double* g = V.cg_g[cur] + 4 * (size_t)j;
                                 g[0] = o.c * rj;
                                 g[1] = 0.0;
                                 g[2] = 0.0;
                             }
                         });
    double thr = 0.0;
    int it = 0;
    const int rounds = cg_rounds<TV>();
    for (int round = 0; round < rounds; ++round) {
        if (!(use_q && round == 0)) {
            // t = A xw ; r0 = rhs - (xw + A^T t) in FP64
            spmv_part<1>(tm, P.A, 0, [&](int c_) { return (xw)[c_]; }, [&](int i, double s) { V.cg_t[i] = s; });
            tm.sync();
            spmv_part<1>(tm, P.At, 1, [&](int c_) { return (V.cg_t)[c_]; },
                         [&](int j, double s) { start(j, B[j] - (xw[j] + s)); });
        }
        if (!(prestarted && use_q && round == 0)) tm.sync();
        double alpha = 0.0, beta = 0.0, gamma_old = 1.0, alpha_old = 1.0;
        bool done = false;
        for (int pass = 0;; ++pass) {
            // ---- phase X
            const double* go = V.cg_g[cur];
            double* gn = V.cg_g[cur ^ 1];
            for (int j = tm.rank(); j < n; j += tm.size()) {
                const double pj = V.cg_u[j] + beta * V.cg_p[j];
                const double sj = V.cg_w[j] + beta * V.cg_s[j];
                const double rj = V.cg_r[j] - alpha * sj;
                const double dj = P.dinv[j];
                const double xj = xw[j] + alpha * pj;
                xw[j] = xj;
                V.cg_p[j] = pj;
                V.cg_s[j] = sj;
                V.cg_r[j] = rj;
                V.cg_u[j] = dj * rj;
                gn[4 * (size_t)j] = dj * rj;
                gn[4 * (size_t)j + 1] = dj * sj;
                if constexpr (kPred) gn[4 * (size_t)j + 3] = xj;   // read by a closing pass with a pending step
            }
            spmv_part<4>(tm, KA, 0,
                         [&](int c) {
                             const double2 ab = *reinterpret_cast<const double2*>(go + 4 * (size_t)c);
                             const double dw = go[4 * (size_t)c + 2];
                             return ab.x - alpha * (dw + beta * ab.y);
                         },
                         [&](int i, double acc) { V.cg_t[i] = acc; });
            tm.sync();
            cur ^= 1;
            // ---- phase Y
            double a_g = 0.0, a_d = 0.0, a_rr = 0.0;
            double a_rw = 0.0, a_rs = 0.0, a_ww = 0.0, a_ws = 0.0, a_ss = 0.0;
            spmv_part_pre<4>(tm, KAt, 1, [&](int c) { return V.cg_t[c]; },
                             [&](int j) { return Row4{V.cg_u[j], V.cg_r[j], P.dinv[j], kPred ? V.cg_s[j] : 0.0}; },
                             [&](int j, double s, const Row4& o) {     // o = (u_j, r_j, D_j, s_j)
                const double uj = o.a;
                const double rj = o.b;
                const double wj = uj + s;
                V.cg_w[j] = wj;
                V.cg_g[cur][4 * (size_t)j + 2] = o.c * wj;
                a_g += rj * uj;
                a_d += wj * uj;
                a_rr += rj * rj;
                if constexpr (kPred) {
                    const double sj = o.d;
                    a_rw += rj * wj;
                    a_rs += rj * sj;
                    a_ww += wj * wj;
                    a_ws += wj * sj;
                    a_ss += sj * sj;
                }
            });
            put(sh, 0, a_g);
            put(sh, 1, a_d);
            put(sh, 2, a_rr);
            if constexpr (kPred) {
                put(sh, 3, a_rw);
                put(sh, 4, a_rs);
                put(sh, 5, a_ww);
                put(sh, 6, a_ws);
                put(sh, 7, a_ss);
            }
            if (round == 0 && pass == 0) put(sh, KD, a_bb);
            tm.reduce(sh, (round == 0 && pass == 0) ? KD + 1 : KD);
            const double gamma = sh.out[0], delta = sh.out[1], rr = sh.out[2];
            if (round == 0 && pass == 0) {
                thr = thr_abs > 0.0 ? thr_abs : tol * tol * sh.out[KD];
                if (thr_used) *thr_used = thr;
            }
            if (!(rr > thr) && (it > 0 || round > 0)) {   // at least one step, as in solve_M_staged
                done = pass == 0;            // the FP64 residual itself meets the tolerance
                break;
            }
            if (it >= maxit || tm.aborted()) {
                done = true;
                break;
            }
            double den = delta;
            if (pass == 0) {
                beta = 0.0;
            } else {
                beta = gamma / gamma_old;
                den = delta - beta * gamma / alpha_old;
            }
            if (!(gamma > 0.0) || !(den > 0.0)) break;      // breakdown: residual at rounding level
            alpha = gamma / den;
            gamma_old = gamma;
            alpha_old = alpha;
            ++it;
            if constexpr (kPred) {
                // ||r - alpha s'||^2 with s' = w + beta s
                const double rs1 = sh.out[3] + beta * sh.out[4];
                const double ss1 = sh.out[5] + beta * (2.0 * sh.out[6] + beta * sh.out[7]);
                const double rr1 = rr - 2.0 * alpha * rs1 + alpha * alpha * ss1;
                if (!(rr1 > thr)) {
                    pend = true;
                    fa = alpha;
                    fb = beta;
                    done = true;
                    break;
                }
            }
        }
        if (done) break;
    }
    // py = ry + A px ; h^T p.  With a pending step, x + alpha p' (p' = u +
    // beta p) is formed where it is read: gathers take x and u from the
    // column records (the owners overwrite x in this pass), p from its vector.
    double a_hp = 0.0;
    const double* gf = V.cg_g[cur];
    spmv_part_pre<4>(tm, P.A, 0, [&](int c_) {
        if (pend) {
            const double* g = gf + 4 * (size_t)c_;
            return g[3] + fa * (g[0] + fb * V.cg_p[c_]);
        }
        return xw[c_];
    }, [&](int i) { return double2{r[n + i], P.b[i]}; }, [&](int i, double s, const double2& rb) {
        const double py = rb.x + s;
        out[n + i] = py;
        a_hp += rb.y * py;
    });
    for (int j = tm.rank(); j < n; j += tm.size()) {
        double xj = xw[j], rj = V.cg_r[j];
        if (pend) {
            const double pj = V.cg_u[j] + fb * V.cg_p[j];
            const double sj = V.cg_w[j] + fb * V.cg_s[j];
            rj = rj - fa * sj;
            xj = xj + fa * pj;
            xw[j] = xj;
        }
        out[j] = xj;
        a_hp += P.c[j] * xj;
        if (q) q[j] = B[j] - rj;
    }
    put(sh, 0, a_hp);
    tm.reduce(sh, 1);
    return it;
}

// (I + Q)^{-1} r = (p - tau g, tau) with p = M^{-1} r[0 .. n+m) written to
// out[0 .. n+m) and tau = (r_tau + h^T p) / delta returned.  The rank-one
// correction is left to the consumer (corrected(), below), which applies it
// on the fly in its own pass, saving a barrier.  r and out must not alias.
template <typename TV, typename Team>
__device__ double linear_step(Team& tm, Shared& sh, const Prob& P, const Vecs& V, const double* r, double* out,
                              double* xw, double tol, int maxit, long long* cg_iters, double thr_abs = 0.0,
                              double* thr_used = nullptr, double* q = nullptr, bool refresh = true,
                              double* rb = nullptr, bool prestarted = false, double bb_part = 0.0) {
    *cg_iters += solve_M<TV>(tm, sh, P, V, r, out, xw, tol, maxit, thr_abs, thr_used, q, refresh, rb, prestarted,
                             bb_part);
    return (r[P.N - 1] + sh.out[0]) / P.delta;
}

// Entry i of (I + Q)^{-1} r from the uncorrected output p of linear_step.
__device__ __forceinline__ double corrected(const Prob& P, const double* p, double tau, int i) {
    return (i < P.N - 1) ? p[i] - tau * P.g[i] : tau;
}

// Per-instance constants of the linear step: ||b||, ||c||, g = M^{-1} (c, b)
// (written to g) and delta = 1 + (c, b)^T g, stored into P.  V.d is scratch.
template <typename Team>
__device__ int setup_gdelta(Team& tm, Shared& sh, Prob& P, const Vecs& V, double* g, double tol, int maxit) {
    const int n = P.n, m = P.m;
    double nb2 = 0.0, nc2 = 0.0;
    for (int i = tm.rank(); i < m; i += tm.size()) { nb2 += P.b[i] * P.b[i]; V.d[n + i] = P.b[i]; }
    for (int j = tm.rank(); j < n; j += tm.size()) {
        nc2 += P.c[j] * P.c[j];
        V.d[j] = P.c[j];
        V.xw_d[j] = 0.0;
    }
    if (tm.rank() == 0) V.d[P.N - 1] = 0.0;
    put(sh, 0, nb2);
    put(sh, 1, nc2);
    tm.reduce(sh, 2);
    P.nb = sqrt(sh.out[0]);
    P.nc = sqrt(sh.out[1]);
    const int it = solve_M<double>(tm, sh, P, V, V.d, g, V.xw_d, tol, maxit);
    P.delta = 1.0 + sh.out[0];
    P.g = g;
    return it;
}

// ------------------------------------------------------------------ passes
//
// The passes of an outer iteration are out-of-line functions: the solve loop
// that calls them then holds only its own few values across the calls, and
// each pass gets a register allocation of its own (inlined, they made the
// solve kernel spill heavily).

// u-bar = Pi_C(2 u~ - u), R u = u~ - u-bar, where u~ is formed from the
// uncorrected linear-step output in V.ut and tau (and stored back corrected);
// returns ||R u||^2 and leaves ||u||^2 in sh.out[1].
template <typename Team>
__device__ __noinline__ double residual_pass(Team& tm, Shared& sh, const Prob& P, const Vecs& V, double tau) {
    double acc = 0.0, au = 0.0;
    project_C(tm, sh, P.n, P.N, P.K,
              [&](int i) { return 2.0 * corrected(P, V.ut, tau, i) - V.u[i]; },
              [&](int i, double v) {
                  const double ut = corrected(P, V.ut, tau, i);
                  V.ut[i] = ut;
                  V.ub[i] = v;
                  const double r = ut - v;
                  V.Ru[i] = r;
                  acc += r * r;
                  au += V.u[i] * V.u[i];
              });
    put(sh, 0, acc);
    put(sh, 1, au);
    tm.reduce(sh, 2);
    return sh.out[0];
}

struct Term {
    double pr, dr, gap, ic, uc, pobj, dobj, tau, cx, by;
    int status;
    int timeout;
};

// Sec. IV-C.  sig-bar = psi-bar - 2 psi~ + psi; candidate (chi, psi, sig)-bar / tau-bar.
// The measures land in sh.term (LDS), read by every thread after the call,
// which keeps them out of the registers of the long-lived solve loop.
// Partial sums of the termination measures (Sec. IV-C) into slots 0..6; the
// candidate is the barred iterate.  Returns its tau.
// scs: the candidate's sigma is psi-bar - z_psi (SCS's splitting, z in V.u)
// instead of psi-bar - 2 psi~ + psi.
template <typename Team>
__device__ __forceinline__ double term_partials(Team& tm, Shared& sh, const Prob& P, const Vecs& V, bool timed_out,
                                                bool scs = false) {
    const int n = P.n;
    const double tau = V.ub[P.N - 1];
    double a_p = 0.0, a_u = 0.0, a_d = 0.0, a_i = 0.0, a_cx = 0.0, a_by = 0.0;
    // <b, y> and <c, x> ride along with the products: every row of A and of
    // A^T is reported exactly once; each row's operands are prefetched
    spmv_part_pre<4>(tm, P.A, 0, [&](int c_) { return V.ub[c_]; },
                     [&](int i) { return Row4{V.ub[n + i], scs ? 0.0 : V.ut[n + i], V.u[n + i], P.b[i]}; },
                     [&](int i, double s, const Row4& o) {     // o = (ybar_i, ytilde_i, y_i, b_i)
        const double yb = o.a;
        const double sig = scs ? yb - o.c : yb - 2.0 * o.b + o.c;
        const double v = s + sig;
        a_u += v * v;
        const double bi = o.d;
        const double w = v - bi * tau;
        a_p += w * w;
        a_by += bi * yb;
    });
    spmv_part_pre<4>(tm, P.At, 1, [&](int c_) { return V.ub[n + c_]; },
                     [&](int j) { return double2{P.c[j], V.ub[j]}; }, [&](int j, double s, const double2& o) {   // (c_j, xbar_j)
        a_i += s * s;
        const double cj = o.x;
        const double w = s + cj * tau;
        a_d += w * w;
        a_cx += cj * o.y;
    });
    put(sh, 0, a_p);
    put(sh, 1, a_u);
    put(sh, 2, a_d);
    put(sh, 3, a_i);
    put(sh, 4, a_cx);
    put(sh, 5, a_by);
    put(sh, 6, (tm.rank() == 0 && timed_out) ? 1.0 : 0.0);
    return tau;
}

// The measures and status from the reduced slots 0..6 into sh.term (thread 0).
__device__ __forceinline__ void term_finish(Shared& sh, const Prob& P, const Params& S, double tau) {
    Term T;
    const auto out = vec_at<true>(sh.out);     // LDS-typed (see small_chol_solve)
    const double cx = out[4], by = out[5];
    T.tau = tau;
    T.cx = cx;
    T.by = by;
    T.timeout = out[6] > 0.0;
    T.pr = T.dr = T.gap = T.ic = T.uc = INFINITY;
    T.pobj = T.dobj = NAN;
    if (tau > 0.0) {
        T.pr = sqrt(out[0]) / tau / (1.0 + P.nb);
        T.dr = sqrt(out[2]) / tau / (1.0 + P.nc);
        T.gap = fabs(cx + by) / tau / (1.0 + fabs(cx) / tau + fabs(by) / tau);
        T.pobj = cx / tau;
        T.dobj = -by / tau;
    }
    if (by < 0.0) T.ic = P.nb * sqrt(out[3]) / (-by);
    if (cx < 0.0) T.uc = P.nc * sqrt(out[1]) / (-cx);
    T.status = 0;
    if (tau > 0.0 && T.pr <= S.eps && T.dr <= S.eps && T.gap <= S.eps) T.status = ST_SOLVED;
    else if (T.ic < S.eps) T.status = ST_INFEASIBLE;
    else if (T.uc < S.eps) T.status = ST_UNBOUNDED;
    *reinterpret_cast<Term*>(sh.term) = T;
}

template <typename Team>
__device__ __noinline__ void termination_pass(Team& tm, Shared& sh, const Prob& P, const Vecs& V, const Params& S,
                                              bool timed_out) {
    const double tau = term_partials(tm, sh, P, V, timed_out);
    tm.reduce(sh, 7);
    if (threadIdx.x == 0) term_finish(sh, P, S, tau);
    __syncthreads();
}

// ------------------------------------------------------------------ directions

// Solves (G + mu I) t = rhs (k x k, SPD) by Cholesky into t; false if not
// finite.  Every array is in LDS (the workgroup's Shared); they are reached
// through LDS-typed pointers, since a generic pointer would send each of the
// routine's dependent accesses down the vector-memory path.  The forward
// substitution's result is kept in t and overwritten in place by the
// backward one.
__device__ inline bool small_chol_solve(const double* G_, int ld, int k, double mu, const double* rhs_, double* t_,
                                        double* L_) {
    const auto G = vec_at<true>(G_);
    const auto rhs = vec_at<true>(rhs_);
    const auto t = vec_at<true>(t_);
    const auto L = vec_at<true>(L_);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = G[i * ld + j] + (i == j ? mu : 0.0);
            for (int e = 0; e < j; ++e) s -= L[i * MEMMAX + e] * L[j * MEMMAX + e];
            if (i == j) {
                if (!(s > 0.0)) return false;
                L[i * MEMMAX + i] = sqrt(s);
            } else {
                L[i * MEMMAX + j] = s / L[j * MEMMAX + j];
            }
        }
    for (int i = 0; i < k; ++i) {
        double s = rhs[i];
        for (int e = 0; e < i; ++e) s -= L[i * MEMMAX + e] * t[e];
        t[i] = s / L[i * MEMMAX + i];
    }
    for (int i = k - 1; i >= 0; --i) {
        double s = t[i];
        for (int e = i + 1; e < k; ++e) s -= L[e * MEMMAX + i] * t[e];
        t[i] = s / L[i * MEMMAX + i];
        if (!isfinite(t[i])) return false;
    }
    return true;
}

struct DirState {
    int pend;       // 0: no pending pair; 1: (pz, pxi) complete; 2: pxi still needs + R u
    int aa_k, aa_head;
    int rb_m;
    int aa_old;     // Anderson by QR: ring slot of the oldest pair (logical column 0)
};

// Memory columns whose loads one pass keeps in flight together (fewer in the
// one-workgroup engine, whose register budget is smaller).
template <typename Team>
constexpr int aa_chunk() { return Team::kBlock ? 2 : 8; }

// Anderson: push the pending pair into the ring, update the Gram matrix and
// solve for t; then d = -Ru - (Z - Xi) t, fused with the K0 update of u.
// Anderson (Sec. IV-D-2), in three parts so that the dot products can share
// a reduction with the termination check.  (1) Push the pending (z, xi) pair
// into the FIFO memory and put <Xi_i, Ru> (and <Xi_i, Xi_new> for a new
// column) into slots base.. (same element-to-thread map as the copy: no
// barrier needed); returns the new column's slot or -1.
template <typename Team>
__device__ __forceinline__ int aa_push_dots(Team& tm, Shared& sh, const Vecs& V, const Params& S, DirState& ds, int N,
                                            int base) {
    const int mem = S.mem;
    int slot = -1;
    if (ds.pend) {
        slot = ds.aa_head;
        const bool fix = ds.pend == 2;   // a K0 pair: xi from the next R u
        double* Zs = V.Zb + (size_t)slot * N;
        double* Ys = V.Yb + (size_t)slot * N;
        for (int e = tm.rank(); e < N; e += tm.size()) {
            Zs[e] = V.pz[e];
            Ys[e] = V.pxi[e] + (fix ? V.Ru[e] : 0.0);
        }
        ds.aa_head = (ds.aa_head + 1) % mem;
        if (ds.aa_k < mem) ds.aa_k++;
    }
    const int k = ds.aa_k;
    if (k == 0) return slot;
    // memory columns in chunks of AA_CHUNK, each chunk one pass whose loads
    // are all in flight together (a loop over the columns with a run-time
    // bound would wait for each column's loads in turn)
    const bool nc = slot >= 0;
    const bool fix = ds.pend == 2;
    constexpr int AA_CHUNK = aa_chunk<Team>();
    for (int i0 = 0; i0 < k; i0 += AA_CHUNK) {
        double a_r[AA_CHUNK], a_n[AA_CHUNK];
#pragma unroll
        for (int q = 0; q < AA_CHUNK; ++q) { a_r[q] = 0.0; a_n[q] = 0.0; }
        for (int e = tm.rank(); e < N; e += tm.size()) {
            const double ru = V.Ru[e];
            const double ys = nc ? V.pxi[e] + (fix ? ru : 0.0) : 0.0;   // the new column, as stored above
#pragma unroll
            for (int q = 0; q < AA_CHUNK; ++q) {
                if (i0 + q < k) {
                    const double yi = V.Yb[(size_t)(i0 + q) * N + e];
                    a_r[q] += yi * ru;
                    if (nc) a_n[q] += yi * ys;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < AA_CHUNK; ++q) {
            if (i0 + q < k) {
                put(sh, base + i0 + q, a_r[q]);
                if (nc) put(sh, base + k + i0 + q, a_n[q]);
            }
        }
    }
    return slot;
}

// Slots the dot products of aa_push_dots take.
__device__ __forceinline__ int aa_slots(int k, int slot) { return k == 0 ? 0 : (slot >= 0 ? 2 * k : k); }

// (2) Thread 0: the Gram matrix's new column and t from the reduced slots
// base.. ((Xi^T Xi + mu I) t = Xi^T Ru, by Cholesky) into sh.coef.
__device__ __forceinline__ void aa_gram(Shared& sh, const Params& S, int k, int slot, int base) {
    const auto G = vec_at<true>(sh.G);          // LDS-typed (see small_chol_solve)
    const auto out = vec_at<true>(sh.out);
    if (slot >= 0)
        for (int i = 0; i < k; ++i) {
            G[slot * MEMMAX + i] = out[base + k + i];
            G[i * MEMMAX + slot] = out[base + k + i];
        }
    double tr = 0.0;
    for (int i = 0; i < k; ++i) tr += G[i * MEMMAX + i];
    const bool ok = small_chol_solve(sh.G, MEMMAX, k, S.aa_reg * tr / k, sh.out + base, sh.coef, sh.L);
    if (!ok)
        for (int i = 0; i < k; ++i) vec_at<true>(sh.coef)[i] = 0.0;
}

// (3) d = -Ru - sum_i (Z_i - Y_i) t_i (d = -Ru with an empty memory); a K0
// step applies it at once.
template <typename Team>
__device__ __noinline__ void aa_apply(Team& tm, Shared& sh, const Prob& P, const Vecs& V, int k, bool k0) {
    const int N = P.N;
    constexpr int AA_CHUNK = aa_chunk<Team>();
    for (int e = tm.rank(); e < N; e += tm.size()) {
        double d = -V.Ru[e];
        for (int i0 = 0; i0 < k; i0 += AA_CHUNK) {      // loads of a chunk in flight together
#pragma unroll
            for (int q = 0; q < AA_CHUNK; ++q)
                if (i0 + q < k)
                    d -= (V.Zb[(size_t)(i0 + q) * N + e] - V.Yb[(size_t)(i0 + q) * N + e]) * sh.coef[i0 + q];
        }
        V.d[e] = d;
        if (k0) { V.u[e] += d; V.pz[e] = d; V.pxi[e] = -V.Ru[e]; }
    }
    tm.sync();
}

// The termination check and Anderson's dot products in one pass and one
// reduction (they depend only on the residual pass's output, not on each
// other): one barrier fewer per iteration.  aa_apply follows once the
// status is known.
// On iterations without a termination test (check false) only the dot
// products are reduced.
template <typename Team>
__device__ __noinline__ void termination_aa_pass(Team& tm, Shared& sh, const Prob& P, const Vecs& V, const Params& S,
                                                 DirState& ds, bool timed_out, bool check) {
    const int base = check ? 7 : 0;
    const double tau = check ? term_partials(tm, sh, P, V, timed_out) : 0.0;
    const int slot = aa_push_dots(tm, sh, V, S, ds, P.N, base);
    const int k = ds.aa_k;
    tm.reduce(sh, base + aa_slots(k, slot));
    // the two serial parts (disjoint LDS fields) on different wavefronts, at
    // the same time
    if (threadIdx.x == 0 && check) term_finish(sh, P, S, tau);
    if (threadIdx.x == (blockDim.x > WAVE ? WAVE : 0) && k > 0) aa_gram(sh, S, k, slot, base);
    __syncthreads();
}

// Anderson by an updated QR factorisation of Xi (Sec. IV-D-2): Xi = Q R with
// Q (N x k, columns in logical order oldest first, in V.Qb) and R upper
// triangular (k x k, in sh.G, replicated in every workgroup); Z and Xi stay in
// the ring of V.Zb / V.Yb, logical column j in slot (aa_old + j) % mem.  Per
// iteration: (1) with a full memory the oldest column is dropped: Givens
// rotations restore R[:, 1:] to triangular form and are applied to Q's columns
// element by element in the pass that also stores the new pair and forms
// Q^T xi, Q^T R u, <xi, R u>, ||xi||^2 (one reduction, shared with the
// termination check); (2) q1 = xi - Q c1 and its re-orthogonalisation
// coefficients c2 = Q^T q1 and ||q1||^2 (one reduction); (3) R gains the column
// (c1 + c2, r) with r^2 = ||q1||^2 - ||c2||^2 (q1 - Q c2 is orthogonal to Q),
// unless r <= 1e-14 ||xi|| (xi in the span: the pair is not stored), and
// t = R^{-1} Q^T R u, where the new column's entry of Q^T R u is
// (<xi, R u> - (c1 + c2)^T Q^T R u) / r; (4) the new Q column
// (q1 - Q c2) / r is written in the pass that forms d = -R u - (Z - Xi) t.

// Thread 0: Givens rotations dropping logical column 0 from R (k x k) into
// sh.L (c_i, s_i pairs), R replaced by the k-1 x k-1 triangular result.
__device__ inline void aaqr_drop_rotations(Shared& sh, int k) {
    double* R = sh.G;
    for (int i = 0; i < k; ++i)                 // H = R[:, 1:] (k x k-1), in place
        for (int j = 0; j < k - 1; ++j) R[i * MEMMAX + j] = R[i * MEMMAX + j + 1];
    for (int i = 0; i < k - 1; ++i) {
        const double a = R[i * MEMMAX + i], b = R[(i + 1) * MEMMAX + i];
        const double r = hypot(a, b);
        const double c = r == 0.0 ? 1.0 : a / r, s = r == 0.0 ? 0.0 : b / r;
        sh.L[2 * i] = c;
        sh.L[2 * i + 1] = s;
        for (int j = i; j < k - 1; ++j) {
            const double hi = R[i * MEMMAX + j], hj = R[(i + 1) * MEMMAX + j];
            R[i * MEMMAX + j] = c * hi + s * hj;
            R[(i + 1) * MEMMAX + j] = -s * hi + c * hj;
        }
        R[(i + 1) * MEMMAX + i] = 0.0;
    }
}

// (1): the termination partials (when check) and the Anderson-QR dot
// products in one reduction; slots base.. : c1 (k), Q^T R u (k), <xi, R u>,
// ||xi||^2.  Returns the number of kept columns k.
template <typename Team>
__device__ __noinline__ int termination_aaqr_pass(Team& tm, Shared& sh, const Prob& P, const Vecs& V, const Params& S,
                                                  DirState& ds, bool timed_out, bool check) {
    const int N = P.N, mem = S.mem;
    const int base = check ? 7 : 0;
    const double tau = check ? term_partials(tm, sh, P, V, timed_out) : 0.0;
    const bool push = ds.pend != 0;
    const bool drop = push && ds.aa_k == mem;
    if (drop) {
        if (threadIdx.x == 0) aaqr_drop_rotations(sh, mem);
        __syncthreads();
        ds.aa_old = (ds.aa_old + 1) % mem;
        ds.aa_k -= 1;
    }
    const int k = ds.aa_k;
    const int slot = (ds.aa_old + k) % mem;
    const bool fix = ds.pend == 2;
    double a1[MEMMAX], aR[MEMMAX];
    for (int j = 0; j < k; ++j) { a1[j] = 0.0; aR[j] = 0.0; }
    double axr = 0.0, axx = 0.0;
    for (int e = tm.rank(); e < N; e += tm.size()) {
        double q[MEMMAX];
        const int kq = drop ? k + 1 : k;
        for (int j = 0; j < kq; ++j) q[j] = V.Qb[(size_t)j * N + e];
        if (drop) {
            for (int i = 0; i < k; ++i) {
                const double c = sh.L[2 * i], s = sh.L[2 * i + 1];
                const double qi = q[i], qj = q[i + 1];
                q[i] = c * qi + s * qj;
                q[i + 1] = -s * qi + c * qj;
            }
            for (int j = 0; j < k; ++j) V.Qb[(size_t)j * N + e] = q[j];
        }
        const double ru = V.Ru[e];
        double xi = 0.0;
        if (push) {
            xi = V.pxi[e] + (fix ? ru : 0.0);
            V.Zb[(size_t)slot * N + e] = V.pz[e];
            V.Yb[(size_t)slot * N + e] = xi;
            axr += xi * ru;
            axx += xi * xi;
        }
        for (int j = 0; j < k; ++j) {
            a1[j] += q[j] * xi;
            aR[j] += q[j] * ru;
        }
    }
    for (int j = 0; j < k; ++j) {
        put(sh, base + j, a1[j]);
        put(sh, base + k + j, aR[j]);
    }
    put(sh, base + 2 * k, axr);
    put(sh, base + 2 * k + 1, axx);
    tm.reduce(sh, base + 2 * k + 2);
    if (threadIdx.x == 0 && check) term_finish(sh, P, S, tau);
    __syncthreads();
    // keep the reduced values the next steps need (sh.out is reused)
    if (threadIdx.x == 0)
        for (int j = 0; j < 2 * k + 2; ++j) sh.coef[2 * MEMMAX + j] = sh.out[base + j];
    __syncthreads();
    return k;
}

// (2) and (3): re-orthogonalisation sums, then (thread 0) R's new column and t
// into sh.coef[slot]; returns the number of stored columns after the step.
// sh.coef layout: [0, mem) t by ring slot; [2 MEMMAX, ..) c1, Q^T R u, <xi, R u>,
// ||xi||^2 from (1); sh.L[0, MEMMAX) c2, sh.L[MEMMAX] r, sh.L[MEMMAX + 1] 1 if
// the column was stored.
template <typename Team>
__device__ __noinline__ int aaqr_solve(Team& tm, Shared& sh, const Prob& P, const Vecs& V, const Params& S,
                                       DirState& ds, int k) {
    const int N = P.N, mem = S.mem;
    const bool push = ds.pend != 0;
    const double* c1 = sh.coef + 2 * MEMMAX;
    if (push) {
        const int slot = (ds.aa_old + k) % mem;
        double a2[MEMMAX];
        for (int j = 0; j < k; ++j) a2[j] = 0.0;
        double an = 0.0;
        for (int e = tm.rank(); e < N; e += tm.size()) {
            double q1 = V.Yb[(size_t)slot * N + e];
            double qv[MEMMAX];
            for (int j = 0; j < k; ++j) {
                qv[j] = V.Qb[(size_t)j * N + e];
                q1 -= qv[j] * c1[j];
            }
            V.Qb[(size_t)k * N + e] = q1;
            for (int j = 0; j < k; ++j) a2[j] += qv[j] * q1;
            an += q1 * q1;
        }
        for (int j = 0; j < k; ++j) put(sh, j, a2[j]);
        put(sh, k, an);
        tm.reduce(sh, k + 1);
    }
    if (threadIdx.x == 0) {
        double* R = sh.G;
        const double* qru = c1 + k;
        double rhs[MEMMAX];
        for (int j = 0; j < k; ++j) rhs[j] = qru[j];
        int kn = k;
        sh.L[MEMMAX + 1] = 0.0;
        if (push) {
            double c2n = 0.0;
            for (int j = 0; j < k; ++j) {
                sh.L[j] = sh.out[j];
                c2n += sh.out[j] * sh.out[j];
            }
            const double r2 = sh.out[k] - c2n;
            const double xr = c1[2 * k], xx = c1[2 * k + 1];
            if (r2 > 1e-28 * xx && isfinite(r2)) {
                const double r = sqrt(r2);
                double proj = 0.0;
                for (int j = 0; j < k; ++j) {
                    const double col = c1[j] + sh.L[j];
                    R[j * MEMMAX + k] = col;
                    proj += col * qru[j];
                }
                for (int j = 0; j < k; ++j) R[k * MEMMAX + j] = 0.0;
                R[k * MEMMAX + k] = r;
                rhs[k] = (xr - proj) / r;
                sh.L[MEMMAX] = r;
                sh.L[MEMMAX + 1] = 1.0;
                kn = k + 1;
            }
        }
        double t[MEMMAX];
        bool ok = true;
        for (int i = kn - 1; i >= 0; --i) {
            double v = rhs[i];
            for (int j = i + 1; j < kn; ++j) v -= R[i * MEMMAX + j] * t[j];
            t[i] = v / R[i * MEMMAX + i];
            ok = ok && isfinite(t[i]);
        }
        for (int j = 0; j < MEMMAX; ++j) sh.coef[j] = 0.0;
        if (ok)
            for (int j = 0; j < kn; ++j) sh.coef[(ds.aa_old + j) % mem] = t[j];
    }
    __syncthreads();
    return sh.L[MEMMAX + 1] > 0.0 ? k + 1 : k;
}

// (4) d = -Ru - (Z - Xi) t over the stored slots, the new Q column finished
// in the same pass; a K0 step applies d at once.
template <typename Team>
__device__ __noinline__ void aaqr_apply(Team& tm, Shared& sh, const Prob& P, const Vecs& V, const Params& S, int k,
                                        bool stored, bool k0) {
    const int N = P.N, mem = S.mem;
    const double r = sh.L[MEMMAX];
    const int kq = stored ? k - 1 : k;      // columns of Q before the new one
    for (int e = tm.rank(); e < N; e += tm.size()) {
        if (stored) {
            double q = V.Qb[(size_t)kq * N + e];
            for (int j = 0; j < kq; ++j) q -= V.Qb[(size_t)j * N + e] * sh.L[j];
            V.Qb[(size_t)kq * N + e] = q / r;
        }
        double d = -V.Ru[e];
        for (int i = 0; i < mem; ++i) {
            const double t = sh.coef[i];
            if (t != 0.0) d -= (V.Zb[(size_t)i * N + e] - V.Yb[(size_t)i * N + e]) * t;
        }
        V.d[e] = d;
        if (k0) { V.u[e] += d; V.pz[e] = d; V.pxi[e] = -V.Ru[e]; }
    }
    tm.sync();
}

// Restarted Broyden (Algorithm 2).  H = (I + zt_m z_m^T) ... (I + zt_1 z_1^T);
// applying H to a vector v0 gives v0 + sum_j c_j zt_j with the scalar
// recurrence c_i = <z_i, v0> + sum_{j<i} c_j <z_i, zt_j>, so one reduction of
// all inner products replaces the m' sequential dot/axpy steps.  W holds
// <z_i, zt_j> and is updated with every new pair.
template <typename Team>
__device__ __noinline__ void direction_rb(Team& tm, Shared& sh, const Prob& P, const Vecs& V, const Params& S,
                             DirState& ds, bool k0) {
    const int N = P.N, mem = S.mem;
    const int mp = ds.rb_m;
    const bool pair = ds.pend != 0;
    const bool fix = ds.pend == 2;
    // pxi gets its + R u completion in place (same element map everywhere below)
    if (fix)
        for (int e = tm.rank(); e < N; e += tm.size()) V.pxi[e] += V.Ru[e];
    // inner products: a_i = <z_i, xi>, b_i = <z_i, Ru>, c_i = <z_i, z>, e_j = <z, zt_j>,
    // f1 = <z, xi>, f2 = <z, Ru>, f3 = <z, z>
    for (int i = 0; i < mp; ++i) {
        const double* Zi = V.Zb + (size_t)i * N;
        double ab = 0.0;
        for (int e = tm.rank(); e < N; e += tm.size()) ab += Zi[e] * V.Ru[e];
        put(sh, mp + i, ab);
        if (pair) {
            const double* Zti = V.Yb + (size_t)i * N;
            double aa = 0.0, ac = 0.0, ae = 0.0;
            for (int e = tm.rank(); e < N; e += tm.size()) {
                aa += Zi[e] * V.pxi[e];
                ac += Zi[e] * V.pz[e];
                ae += V.pz[e] * Zti[e];
            }
            put(sh, i, aa);
            put(sh, 2 * mp + i, ac);
            put(sh, 3 * mp + i, ae);
        }
    }
    if (pair) {
        double f1 = 0.0, f2 = 0.0, f3 = 0.0;
        for (int e = tm.rank(); e < N; e += tm.size()) {
            const double z = V.pz[e];
            f1 += z * V.pxi[e];
            f2 += z * V.Ru[e];
            f3 += z * z;
        }
        put(sh, 4 * mp, f1);
        put(sh, 4 * mp + 1, f2);
        put(sh, 4 * mp + 2, f3);
    }
    tm.reduce(sh, pair ? 4 * mp + 3 : 2 * mp);
    // scalar phase (one thread per workgroup), coefficients broadcast in sh.coef:
    //   coef[0 .. mp)      multipliers of zt_j in d
    //   coef[mp]           multiplier of (z - xi) in d
    //   coef[mp+1 .. 2mp+1) multipliers of zt_j in the new zt (times -1 scale below)
    //   coef[2mp+1]        scale of the new zt: zt_new = s (z - xi - sum cx_j zt_j)
    //   coef[2mp+2]        slot that receives the new pair
    if (threadIdx.x == 0) {
        const double* o = sh.out;
        double* cr = sh.L;                 // LDS scratch of the scalar phase
        double* cx = sh.L + MEMMAX;
        for (int i = 0; i < mp; ++i) {
            double s = -o[mp + i];                 // <z_i, -Ru>
            for (int j = 0; j < i; ++j) s += cr[j] * sh.W[i * MEMMAX + j];
            cr[i] = s;
        }
        if (!pair) {
            for (int i = 0; i < mp; ++i) sh.coef[i] = cr[i];
            sh.coef[mp] = 0.0;
        } else {
            for (int i = 0; i < mp; ++i) {
                double s = o[i];                   // <z_i, xi>
                for (int j = 0; j < i; ++j) s += cx[j] * sh.W[i * MEMMAX + j];
                cx[i] = s;
            }
            const double f1 = o[4 * mp], f2 = o[4 * mp + 1], f3 = o[4 * mp + 2];
            double zHxi = f1, zv = -f2;
            for (int j = 0; j < mp; ++j) {
                zHxi += cx[j] * o[3 * mp + j];
                zv += cr[j] * o[3 * mp + j];
            }
            const double gamma = zHxi / f3;
            double theta = 1.0;
            if (fabs(gamma) < S.thetabar) {
                const double sg = (gamma >= 0.0) ? 1.0 : -1.0;
                theta = (1.0 - sg * S.thetabar) / (1.0 - gamma);
            }
            const double den = (1.0 - theta) * f3 + theta * zHxi;   // <z, H xi~>
            const double sc = theta / den;                            // zt_new = sc (z - H xi)
            // d = -Ru + sum cr_j zt_j + zv * zt_new
            for (int j = 0; j < mp; ++j) sh.coef[j] = cr[j] - zv * sc * cx[j];
            sh.coef[mp] = zv * sc;
            for (int j = 0; j < mp; ++j) sh.coef[mp + 1 + j] = cx[j];
            sh.coef[2 * mp + 1] = sc;
            // new inner products
            double* wcol = sh.L + 2 * MEMMAX;
            for (int i = 0; i < mp; ++i) {
                double zH = o[i];                  // <z_i, H xi> = a_i + sum cx_j W_ij
                for (int j = 0; j < mp; ++j) zH += cx[j] * sh.W[i * MEMMAX + j];
                wcol[i] = sc * (o[2 * mp + i] - zH);
            }
            const double wnn = sc * (f3 - zHxi);
            const bool restart = (mp == mem);
            const int slot = restart ? 0 : mp;
            sh.coef[2 * mp + 2] = (double)slot;
            if (restart) {
                sh.W[0] = wnn;
            } else {
                for (int j = 0; j < mp; ++j) sh.W[slot * MEMMAX + j] = o[3 * mp + j];
                for (int i = 0; i < mp; ++i) sh.W[i * MEMMAX + slot] = wcol[i];
                sh.W[slot * MEMMAX + slot] = wnn;
            }
        }
    }
    __syncthreads();
    const double cdz = sh.coef[mp];
    double sc = 0.0;
    int slot = -1;
    if (pair) {
        sc = sh.coef[2 * mp + 1];
        slot = (int)sh.coef[2 * mp + 2];
    }
    for (int e = tm.rank(); e < N; e += tm.size()) {
        const double ru = V.Ru[e];
        double d = -ru;
        double hx = 0.0;
        for (int j = 0; j < mp; ++j) {
            const double ztj = V.Yb[(size_t)j * N + e];
            d += sh.coef[j] * ztj;
            if (pair) hx += sh.coef[mp + 1 + j] * ztj;
        }
        if (pair) {
            const double z = V.pz[e], xi = V.pxi[e];
            d += cdz * (z - xi);
            const double ztn = sc * (z - xi - hx);
            V.Zb[(size_t)slot * N + e] = z;
            V.Yb[(size_t)slot * N + e] = ztn;
        }
        V.d[e] = d;
        if (k0) { V.u[e] += d; V.pz[e] = d; V.pxi[e] = -ru; }
    }
    if (pair) ds.rb_m = (mp == mem) ? 1 : mp + 1;
    tm.sync();
}

// ------------------------------------------------------------------ Algorithm 1

template <typename Team>
__device__ void write_trace(Team& tm, const Vecs& V, long long nu, double res, int kind, int ls, double eta,
                            double r_safe) {
    if (V.tr_res != nullptr && tm.rank() == 0 && nu < V.tr_cap) {
        V.tr_res[nu] = res;
        V.tr_kind[nu] = kind;
        V.tr_ls[nu] = ls;
        V.tr_eta[nu] = eta;
        V.tr_rsafe[nu] = r_safe;
    }
}

// Trial point w = u + a d of the line search (Algorithm 1): w~ = u~ + a d~ by
// linearity (Sec. IV-B), R w = w~ - Pi_C(2 w~ - w) into V.Rw; leaves ||R w||^2
// in sh.out[0] and <R w, d> in sh.out[1].  Out of line, like the other
// passes, so the solve loop's registers stay its own.
template <typename Team>
__device__ __noinline__ void trial_pass(Team& tm, Shared& sh, const Prob& P, const Vecs& V, double a, double tau_d) {
    double acc_w = 0.0, acc_d = 0.0;
    project_C(tm, sh, P.n, P.N, P.K,
              [&](int i) { return 2.0 * (V.ut[i] + a * corrected(P, V.dt, tau_d, i)) - (V.u[i] + a * V.d[i]); },
              [&](int i, double v) {
                  const double rw = (V.ut[i] + a * corrected(P, V.dt, tau_d, i)) - v;
                  V.Rw[i] = rw;
                  acc_w += rw * rw;
                  acc_d += rw * V.d[i];
              });
    put(sh, 0, acc_w);
    put(sh, 1, acc_d);
    tm.reduce(sh, 2);
}

template <typename TV, typename Team>
__device__ void solve(Team& tm, Shared& sh, const Prob& P, const Vecs& V, const Params& S, Result* res) {
    const int n = P.n, m = P.m, N = P.N;
    const long long t_start = wall_clock64();
    for (int i = tm.rank(); i < N; i += tm.size())
        V.u[i] = V.u0 ? V.u0[i] : (i == N - 1 ? 1.0 : 0.0);
    for (int j = tm.rank(); j < n; j += tm.size()) {
        V.xw_u[j] = 0.0;
        V.xw_d[j] = 0.0;
        V.q_u[j] = 0.0;
        V.q_d[j] = 0.0;
    }
    // CG starts from the stored K xw (saving two products per linear step),
    // recomputing the true residual every 64th iteration and always when the
    // solves are exact
    double* const qu = V.q_u;
    double* const qd = V.q_d;
    tm.sync();
    DirState ds = {0, 0, 0, 0, 0};
    double eta0 = 0.0, eta = 0.0, r_safe = 0.0;
    long long k0c = 0, k1c = 0, k2c = 0, kmc = 0, btc = 0, cgc = 0;
    const Term& T = *reinterpret_cast<const Term*>(sh.term);
    double nRu = 0.0;
    int status = 0;
    long long nu = 0;
    double tol = S.cg_adapt > 0.0 ? 1e-6 : S.cg_tol;
    double thr_u = 0.0;                                // the u step's CG threshold (absolute)
    // After a K1 step u+ = u + a d, the next u~ solve's right-hand side is
    // rhs_u + a rhs_d by linearity (the one of Sec. IV-B), and its CG starts
    // from x_u + a x_d with r0 = rhs - q: both are formed in the step's own
    // pass, so that solve needs neither the product with A^T nor its barrier
    // (grid teams, FP64 operator, iterative linear step).
    constexpr bool kPre = !Team::kBlock && std::is_same<TV, double>::value;
    const bool pre_ok = kPre && P.Minv == nullptr;
    bool pre = false;            // the next u~ solve is prestarted
    double bb_part = 0.0;        // this thread's part of that solve's ||rhs||^2
    for (nu = 0;; ++nu) {
        const bool refresh = !(S.cg_adapt > 0.0) || nu % 64 == 0;
        const double tau_u = linear_step<TV>(tm, sh, P, V, V.u, V.ut, V.xw_u, tol, S.cg_max, &cgc, 0.0, &thr_u, qu,
                                             refresh, pre_ok ? V.rhs_u : nullptr, pre, bb_part);
        pre = false;
        bb_part = 0.0;
        nRu = sqrt(residual_pass(tm, sh, P, V, tau_u));
        if (S.cg_adapt > 0.0) {
            // inexact linear steps: accuracy relative to the current fixed-point residual
            const double nu_ = sqrt(sh.out[1]);
            tol = fmin(1e-3, fmax(S.cg_tol, S.cg_adapt * nRu / fmax(nu_, 1e-300)));
        }
        const bool late = S.max_ticks > 0 && (wall_clock64() - t_start) > S.max_ticks;
        // termination test (Sec. IV-C) every check_every-th iteration and at the
        // iteration cap; the candidate returned is always that of a tested iteration
        const bool check = S.check_every <= 1 || nu % S.check_every == 0 || nu >= S.max_iters;
        int qr_k = 0;
        if (S.direction == DIR_AA) termination_aa_pass(tm, sh, P, V, S, ds, late, check);
        else if (S.direction == DIR_AA_QR) qr_k = termination_aaqr_pass(tm, sh, P, V, S, ds, late, check);
        else if (check) termination_pass(tm, sh, P, V, S, late);
        if (nu == 0) eta0 = eta = r_safe = nRu;
        status = check ? T.status : 0;
        if (!isfinite(nRu)) status = ST_NUMERICAL;
        if (tm.aborted()) status = ST_NUMERICAL;
        if (!status && nu >= S.max_iters) status = ST_MAX_ITERS;
        if (!status && check && T.timeout) status = ST_TIME_LIMIT;
        if (status) { write_trace(tm, V, nu, nRu, -1, 0, eta, r_safe); break; }
        const bool k0 = nRu <= S.c0 * eta;
        if (S.direction == DIR_AA) {
            aa_apply(tm, sh, P, V, ds.aa_k, k0);            // its dot products went with the termination check
        } else if (S.direction == DIR_AA_QR) {
            const int kn = aaqr_solve(tm, sh, P, V, S, ds, qr_k);
            ds.aa_k = kn;
            aaqr_apply(tm, sh, P, V, S, kn, kn > qr_k, k0);
        } else if (S.direction == DIR_RB) {
            direction_rb(tm, sh, P, V, S, ds, k0);
        } else {
            const bool zero = S.direction == DIR_ZERO;
            for (int e = tm.rank(); e < N; e += tm.size()) {
                const double d = zero ? 0.0 : -V.Ru[e];
                V.d[e] = d;
                if (k0) { V.u[e] += d; V.pz[e] = d; V.pxi[e] = -V.Ru[e]; }
            }
            tm.sync();
        }
        if (k0) {                                          // K0: u+ = u + d (w = u + d)
            eta = nRu;
            ds.pend = 2;
            ++k0c;
            write_trace(tm, V, nu, nRu, 0, 0, eta, r_safe);
            continue;
        }
        if (S.direction == DIR_ZERO) {
            // d = 0: the linear step of d is 0, every trial point is w = u with
            // Rw = Ru and rho = ||Ru||^2, so the first trial is the K2 step
            // u - lambda R u (the relaxed DRS / KM iteration of Sec. IV-A);
            // taken directly, without the redundant linear step and projection
            for (int e = tm.rank(); e < N; e += tm.size()) {
                V.pz[e] = 0.0;
                V.pxi[e] = 0.0;
                V.u[e] -= S.lam * V.Ru[e];
            }
            ds.pend = 1;
            ++k2c;
            tm.sync();
            write_trace(tm, V, nu, nRu, 2, 0, eta, r_safe);
            continue;
        }
        // inexact steps (cg_d_match): d~ to the same absolute accuracy as u~,
        // since trial points combine them as u~ + alpha d~ (Sec. IV-B); a
        // tolerance relative to d's own, much smaller, right-hand side solves
        // d~ far more accurately than u~ is known
        const double tau_d = linear_step<TV>(tm, sh, P, V, V.d, V.dt, V.xw_d, tol, S.cg_max, &cgc,
                                             S.cg_adapt > 0.0 && S.cg_d_match ? thr_u : 0.0, nullptr, qd, refresh);
        double alpha = 1.0;
        int kind = 3, ls = 0;
        double coef = 0.0;
        for (ls = 0; ls < S.ls_max; ++ls) {
            const double a = alpha;
            trial_pass(tm, sh, P, V, a, tau_d);
            const double nRw2 = sh.out[0];
            const double nRw = sqrt(nRw2);
            const double rho = nRw2 - a * sh.out[1];        // <Rw, u - T w>, T w = w - Rw
            if (nRu <= r_safe && nRw <= S.c1 * nRu) {        // K1
                kind = 1;
                r_safe = nRw + pow(S.q, (double)nu) * eta0;
                break;
            }
            if (rho >= S.sigma * nRu * nRw) {                // K2
                kind = 2;
                coef = S.lam * rho / nRw2;
                break;
            }
            alpha *= 0.5;
            ++btc;
        }
        const double a = alpha;
        if (kind == 1) {
            for (int e = tm.rank(); e < N; e += tm.size()) {
                const double z = a * V.d[e];
                V.u[e] += z;
                V.pz[e] = z;
                V.pxi[e] = V.Rw[e] - V.Ru[e];
            }
            // the next linear step solves for u + a d: by linearity (the same
            // property the line search uses, Sec. IV-B) its CG starts from the
            // sum of the two solutions already at hand
            const bool use_q = S.cg_adapt > 0.0 && (nu + 1) % 64 != 0;   // the next solve's refresh rule
            for (int j = tm.rank(); j < n; j += tm.size()) {
                V.xw_u[j] += a * V.xw_d[j];
                const double qj = qu[j] + a * qd[j];
                qu[j] = qj;
                if (pre_ok) {
                    // rhs_d is in the CG's buffer (d~ was the last solve)
                    const double bj = V.rhs_u[j] + a * V.cg_b[j];
                    V.rhs_u[j] = bj;
                    bb_part += bj * bj;
                    if (use_q) {                       // start(j, bj - q_j) of solve_M
                        const double rj = bj - qj;
                        V.cg_r[j] = rj;
                        V.cg_s[j] = 0.0;
                        V.cg_u[j] = 0.0;
                        V.cg_w[j] = 0.0;
                        V.cg_p[j] = 0.0;
                        double* g = V.cg_g[0] + 4 * (size_t)j;
                        g[0] = P.dinv[j] * rj;
                        g[1] = 0.0;
                        g[2] = 0.0;
                    }
                }
            }
            pre = pre_ok;
            ds.pend = 1;
            ++k1c;
        } else if (kind == 2) {
            for (int e = tm.rank(); e < N; e += tm.size()) {
                V.pz[e] = a * V.d[e];
                V.pxi[e] = V.Rw[e] - V.Ru[e];
                V.u[e] -= coef * V.Rw[e];
            }
            ds.pend = 1;
            ++k2c;
        } else {                                           // backtracking cap: u - lambda R u
            for (int e = tm.rank(); e < N; e += tm.size()) V.u[e] -= S.lam * V.Ru[e];
            ds.pend = 0;
            ++kmc;
        }
        tm.sync();
        write_trace(tm, V, nu, nRu, kind == 3 ? 3 : kind, ls, eta, r_safe);
    }
    // outputs: the candidate or the normalised certificate
    const double tau = T.tau;
    const double nan = NAN;
    for (int j = tm.rank(); j < n; j += tm.size()) {
        double x = nan;
        if (status == ST_UNBOUNDED) x = V.ub[j] / (-T.cx);
        else if (status != ST_INFEASIBLE && tau > 0.0) x = V.ub[j] / tau;
        V.out_x[j] = x;
    }
    for (int i = tm.rank(); i < m; i += tm.size()) {
        const double psi = V.ub[n + i];
        const double sig = psi - 2.0 * V.ut[n + i] + V.u[n + i];
        double y = nan, s = nan;
        if (status == ST_INFEASIBLE) y = psi / (-T.by);
        else if (status == ST_UNBOUNDED) s = sig / (-T.cx);
        else if (tau > 0.0) { y = psi / tau; s = sig / tau; }
        V.out_y[i] = y;
        V.out_s[i] = s;
    }
    if (tm.rank() == 0) {
        res->status = status;
        res->err = tm.aborted() ? 1 : 0;
        res->iters = nu;
        res->k0 = k0c; res->k1 = k1c; res->k2 = k2c; res->km = kmc; res->bt = btc; res->cg = cgc;
        res->pr = T.pr; res->dr = T.dr; res->gap = T.gap; res->ic = T.ic; res->uc = T.uc;
        res->pobj = T.pobj; res->dobj = T.dobj; res->res = nRu;
    }
    tm.sync();
}

// SCS's splitting (Sec. IV-A, "SCS and DRS"): Douglas-Rachford splitting on
// N_C + Q, the reverse order of equation (drs), relaxed by lambda, without
// SuperMann steps:
//   u-bar = Pi_C(z),  u~ = (I + Q)^{-1}(2 u-bar - z),  R z = u-bar - u~,
//   z+ = z - lambda R z.
// z lives in V.u, u-bar in V.ub, 2 u-bar - z in V.d, u~ in V.ut, R z in V.Ru.
// Termination (Sec. IV-C) on the candidate u-bar with sigma = psi-bar - z_psi
// (at a fixed point u-bar - z = Q u-bar).  The same linear step, projections,
// termination read-out and inexact-CG rule as Algorithm 1; out of line, so
// Algorithm 1's loop keeps its register allocation.
template <typename TV, typename Team>
__device__ __noinline__ void solve_scs(Team& tm, Shared& sh, const Prob& P, const Vecs& V, const Params& S,
                                       Result* res) {
    const int n = P.n, m = P.m, N = P.N;
    const long long t_start = wall_clock64();
    for (int i = tm.rank(); i < N; i += tm.size())
        V.u[i] = V.u0 ? V.u0[i] : (i == N - 1 ? 1.0 : 0.0);
    for (int j = tm.rank(); j < n; j += tm.size()) {
        V.xw_u[j] = 0.0;
        V.q_u[j] = 0.0;
    }
    tm.sync();
    const Term& T = *reinterpret_cast<const Term*>(sh.term);
    long long cgc = 0, nu = 0;
    int status = 0;
    double nRz = 0.0, tol = S.cg_adapt > 0.0 ? 1e-6 : S.cg_tol, thr = 0.0;
    for (nu = 0;; ++nu) {
        // u-bar = Pi_C(z), the linear step's input 2 u-bar - z
        project_C(tm, sh, n, N, P.K, [&](int i) { return V.u[i]; }, [&](int i, double v) {
            V.ub[i] = v;
            V.d[i] = 2.0 * v - V.u[i];
        });
        tm.sync();
        const bool refresh = !(S.cg_adapt > 0.0) || nu % 64 == 0;
        const double tau = linear_step<TV>(tm, sh, P, V, V.d, V.ut, V.xw_u, tol, S.cg_max, &cgc, 0.0, &thr, V.q_u,
                                           refresh);
        // R z = u-bar - u~ and the termination sums in one reduction
        double a_r = 0.0, a_z = 0.0;
        for (int i = tm.rank(); i < N; i += tm.size()) {
            const double ut = corrected(P, V.ut, tau, i);
            V.ut[i] = ut;
            const double r = V.ub[i] - ut;
            V.Ru[i] = r;
            a_r += r * r;
            a_z += V.u[i] * V.u[i];
        }
        const bool late = S.max_ticks > 0 && (wall_clock64() - t_start) > S.max_ticks;
        const bool check = S.check_every <= 1 || nu % S.check_every == 0 || nu >= S.max_iters;
        double ttau = 0.0;
        if (check) ttau = term_partials(tm, sh, P, V, late, true);
        put(sh, 7, a_r);
        put(sh, 8, a_z);
        if (check) {
            tm.reduce(sh, 9);
            if (threadIdx.x == 0) term_finish(sh, P, S, ttau);
        } else {
            for (int k = 0; k < 7; ++k) put(sh, k, 0.0);
            tm.reduce(sh, 9);
        }
        __syncthreads();
        nRz = sqrt(sh.out[7]);
        if (S.cg_adapt > 0.0) tol = fmin(1e-3, fmax(S.cg_tol, S.cg_adapt * nRz / fmax(sqrt(sh.out[8]), 1e-300)));
        status = check ? T.status : 0;
        if (!isfinite(nRz)) status = ST_NUMERICAL;
        if (tm.aborted()) status = ST_NUMERICAL;
        if (!status && nu >= S.max_iters) status = ST_MAX_ITERS;
        if (!status && check && T.timeout) status = ST_TIME_LIMIT;
        if (status) {
            write_trace(tm, V, nu, nRz, -1, 0, 0.0, 0.0);
            break;
        }
        for (int i = tm.rank(); i < N; i += tm.size()) V.u[i] -= S.lam * V.Ru[i];
        tm.sync();
        write_trace(tm, V, nu, nRz, 2, 0, 0.0, 0.0);
    }
    // outputs: the candidate (u-bar with sigma = psi-bar - z_psi) or the certificate
    const double tau = T.tau;
    const double nan = NAN;
    for (int j = tm.rank(); j < n; j += tm.size()) {
        double x = nan;
        if (status == ST_UNBOUNDED) x = V.ub[j] / (-T.cx);
        else if (status != ST_INFEASIBLE && tau > 0.0) x = V.ub[j] / tau;
        V.out_x[j] = x;
    }
    for (int i = tm.rank(); i < m; i += tm.size()) {
        const double psi = V.ub[n + i];
        const double sig = psi - V.u[n + i];
        double y = nan, s = nan;
        if (status == ST_INFEASIBLE) y = psi / (-T.by);
        else if (status == ST_UNBOUNDED) s = sig / (-T.cx);
        else if (tau > 0.0) { y = psi / tau; s = sig / tau; }
        V.out_y[i] = y;
        V.out_s[i] = s;
    }
    if (tm.rank() == 0) {
        res->status = status;
        res->err = tm.aborted() ? 1 : 0;
        res->iters = nu;
        res->k0 = 0; res->k1 = 0; res->k2 = nu; res->km = 0; res->bt = 0; res->cg = cgc;
        res->pr = T.pr; res->dr = T.dr; res->gap = T.gap; res->ic = T.ic; res->uc = T.uc;
        res->pobj = T.pobj; res->dobj = T.dobj; res->res = nRz;
    }
    tm.sync();
}

// Algorithm 1 or SCS's splitting, as the settings ask.
template <typename TV, typename Team>
__device__ void run_solve(Team& tm, Shared& sh, const Prob& P, const Vecs& V, const Params& S, Result* res) {
    if (S.direction == DIR_SCS) solve_scs<TV>(tm, sh, P, V, S, res);
    else solve<TV>(tm, sh, P, V, S, res);
}

}  // namespace sscs
