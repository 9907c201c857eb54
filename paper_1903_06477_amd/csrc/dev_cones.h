// Projections onto the dual cone K* (Sec. II cones; projection step of
// equation (drs), Sec. IV-A) as one team-wide streaming pass.
//
// project_C(tm, P, in, emit) evaluates u-bar = Pi_C(p) for C = R^n x K* x R+
// where in(i) returns p_i for the state index i in [0, N) and emit(i, v)
// receives u-bar_i.  Every index is emitted exactly once, by the thread that
// owns its block:
//   x part, zero rows (dual = free), R+ rows, tau     one thread per entry
//   second-order cones (t last)                       one wavefront per cone
//   exponential cones                                  one thread per cone
//   PSD blocks                                         one workgroup per block
#pragma once
#include <float.h>

#include "dev_common.h"

namespace sscs {

struct ConeDev {
    int z, l;                 // zero and R+ row counts
    int nq;                   // SOC count; qoff[nq + 1] row offsets inside the SOC region
    const int* qoff;
    int ns;                   // PSD count; sord[ns] orders, soff[ns + 1] offsets in the PSD region
    const int* sord;
    const int* soff;
    int ep;                   // exponential cones
    int soc0, psd0, exp0;     // first row of each region (relative to the start of y)
    double* psd_scratch;      // per-workgroup scratch for PSD blocks (psd_scratch_doubles(kmax) each)
    double* psd_team;         // grid-team scratch for blocks above kPsdTeamOrder (psd_team_doubles(kmax))
    int psd_kmax;
    double* psd_vecs;         // per block: the eigenvectors of its last projection (kmax^2
                              // doubles each), or null: every projection starts cold
    int* psd_warm;            // per block: 1 once psd_vecs holds an orthogonal basis
    int psd_lds;              // grid teams: bytes of dynamic LDS (at its start) holding the matrix
                              // and eigenvectors of the blocks projected one per workgroup, 0: none
    int psd_small;            // the largest order of those blocks (the LDS area holds 2 of its squares)
};

// ---------------------------------------------------------------- exponential cone
//
// K_e = cl{(x1, x2, x3): x1 >= x2 exp(x3 / x2), x2 > 0}.  For v0 outside K_e
// and outside its polar, the projection is p = s (e^rho, 1, rho) with s > 0 and
// v0 - p = beta (-1, e^rho (1 - rho), e^rho), beta > 0 (the outward normal at p).
// Eliminating s and beta leaves a scalar equation in rho (the formulation of
// Friberg, "Projection onto the exponential cone: a univariate root-finding
// problem"); it is solved here by a bracketed Illinois iteration.

__device__ __forceinline__ double exp_h_scaled(double rho, double t0, double s0, double r0) {
    // h(rho) = ((rho-1) r0 + s0) e^rho - (r0 - rho s0) e^-rho - (rho^2 - rho + 1) t0,
    // multiplied by e^-|rho| (same sign, no overflow).
    const double q = rho * (rho - 1.0) + 1.0;
    if (rho >= 0.0)
        return ((rho - 1.0) * r0 + s0) - (r0 - rho * s0) * exp(-2.0 * rho) - q * t0 * exp(-rho);
    return ((rho - 1.0) * r0 + s0) * exp(2.0 * rho) - (r0 - rho * s0) - q * t0 * exp(rho);
}

__device__ __noinline__ void proj_exp_primal(double t0, double s0, double r0, double* p) {
    const double eps = DBL_EPSILON;
    // inside K_e (points within rounding of the boundary count as inside)
    if (s0 > 0.0) {
        const double e = r0 / s0;
        const double g = (e < 700.0) ? s0 * exp(e) : INFINITY;
        if (t0 - g >= -4.0 * eps * fmax(fabs(t0), g)) { p[0] = t0; p[1] = s0; p[2] = r0; return; }
    } else if (s0 == 0.0 && t0 >= 0.0 && r0 <= 0.0) {
        p[0] = t0; p[1] = s0; p[2] = r0; return;
    }
    // inside the polar cone -K_e*: projection is the apex
    if (r0 > 0.0) {
        const double e = s0 / r0;
        if (e < 700.0 && r0 * exp(e) <= -M_E * t0) { p[0] = p[1] = p[2] = 0.0; return; }
    } else if (r0 == 0.0 && t0 <= 0.0 && s0 <= 0.0) {
        p[0] = p[1] = p[2] = 0.0; return;
    }
    // x2 <= 0 and x3 <= 0: nearest point of the face {x2 = 0, x1 >= 0, x3 <= 0}
    if (r0 <= 0.0 && s0 <= 0.0) { p[0] = fmax(t0, 0.0); p[1] = 0.0; p[2] = r0; return; }
    // boundary case: both multipliers positive confine rho to an interval on
    // which h goes from negative to positive
    double lo, hi;
    if (s0 > 0.0 && r0 > 0.0) { lo = 1.0 - s0 / r0; hi = r0 / s0; }
    else if (s0 > 0.0) {
        hi = r0 / s0;
        double step = 1.0;
        lo = hi - step;
        for (int k = 0; k < 80 && exp_h_scaled(lo, t0, s0, r0) > 0.0; ++k) { step *= 2.0; lo = hi - step; }
    } else {
        lo = 1.0 - s0 / r0;
        double step = 1.0;
        hi = lo + step;
        for (int k = 0; k < 80 && exp_h_scaled(hi, t0, s0, r0) < 0.0; ++k) { step *= 2.0; hi = lo + step; }
    }
    double fa = exp_h_scaled(lo, t0, s0, r0), fb = exp_h_scaled(hi, t0, s0, r0);
    double rho;
    if (fa >= 0.0) rho = lo;
    else if (fb <= 0.0) rho = hi;
    else {
        double a = lo, b = hi;
        int side = 0;
        rho = 0.5 * (a + b);
        for (int it = 0; it < 200; ++it) {
            double c = (a * fb - b * fa) / (fb - fa);
            if (!(c > a && c < b)) c = 0.5 * (a + b);
            const double fc = exp_h_scaled(c, t0, s0, r0);
            rho = c;
            if (fc == 0.0) break;
            if ((fc < 0.0) == (fa < 0.0)) {
                a = c; fa = fc;
                if (side == -1) fb *= 0.5;
                side = -1;
            } else {
                b = c; fb = fc;
                if (side == 1) fa *= 0.5;
                side = 1;
            }
            if (b - a <= 4.0 * eps * fmax(1.0, fabs(c))) { rho = 0.5 * (a + b); break; }
        }
    }
    // recover the point by the better conditioned of the two equivalent formulas
    const double qq = rho * rho - rho + 1.0;
    const double num_p = s0 + (rho - 1.0) * r0;     // s * qq
    const double num_d = r0 - rho * s0;             // beta e^rho * qq
    const double vmax = fmax(fabs(t0), fmax(fabs(s0), fabs(r0)));
    const double na = sqrt(1.0 + rho * rho + (rho < 350.0 ? exp(2.0 * rho) : INFINITY));
    const double err_p = eps * (fabs(s0) + fabs((rho - 1.0) * r0)) / qq * na;
    const double nns = sqrt((rho > -350.0 ? exp(-2.0 * rho) : INFINITY) + 1.0 + (1.0 - rho) * (1.0 - rho));
    const double err_d = eps * (fabs(r0) + fabs(rho * s0)) / qq * nns + eps * vmax;
    double c0, c1, c2;
    if (err_p <= err_d) {
        const double s = num_p / qq;
        c0 = (s > 0.0) ? exp(log(s) + rho) : 0.0;
        c1 = s;
        c2 = s * rho;
    } else {
        const double bexp = num_d / qq;
        const double beta = bexp * exp(-rho);
        c0 = t0 + beta;
        c1 = s0 - bexp * (1.0 - rho);
        c2 = r0 - bexp;
    }
    // keep the nearest of the boundary point, the face point and the apex
    const double f0 = fmax(t0, 0.0), f2 = fmin(r0, 0.0);
    const double d_c = (c0 - t0) * (c0 - t0) + (c1 - s0) * (c1 - s0) + (c2 - r0) * (c2 - r0);
    const double d_f = (f0 - t0) * (f0 - t0) + s0 * s0 + (f2 - r0) * (f2 - r0);
    const double d_0 = t0 * t0 + s0 * s0 + r0 * r0;
    if (d_c <= d_f && d_c <= d_0) { p[0] = c0; p[1] = c1; p[2] = c2; }
    else if (d_f <= d_0) { p[0] = f0; p[1] = 0.0; p[2] = f2; }
    else { p[0] = p[1] = p[2] = 0.0; }
}

// Pi_{K_e*}(v) = v + Pi_{K_e}(-v) (Moreau decomposition with the polar cone -K_e*).
__device__ inline void proj_exp_dual(const double* v, double* out) {
    double p[3];
    proj_exp_primal(-v[0], -v[1], -v[2], p);
    out[0] = v[0] + p[0];
    out[1] = v[1] + p[1];
    out[2] = v[2] + p[2];
}

// ---------------------------------------------------------------- PSD blocks
//
// Pi of a PSD block: mat(x) = V diag(lam) V^T, keep max(lam, 0), back to the
// packed layout (Sec. II).  The eigendecomposition is a cyclic two-sided
// Jacobi method run by one workgroup on the k x k matrix (global scratch
// private to the workgroup): each sweep visits every pair (p, q) once in
// round-robin order, k/2 disjoint rotations J per round in parallel.
//
// A round writes C = J^T A J to a second buffer in one pass over the 2 x 2
// blocks the disjoint rotations cut A into, so a round costs one barrier; the
// eigenvectors are kept as the rows of Vt = V^T (Vt <- J^T Vt), which makes
// their updates and the reconstruction walk rows.
//
// Warm start: the iterates the method projects change little from one call to
// the next, so a block keeps the eigenvectors of its previous projection
// (Vt0).  Jacobi then starts from B = Vt0 mat(x) Vt0^T (similar to mat(x),
// nearly diagonal) with Vt = Vt0, which leaves one to three sweeps instead
// of eight to ten.

// Scratch of one workgroup for blocks of order <= kmax: a, vm, tmp (k x k
// each), the packed input and output.
__host__ __device__ inline size_t psd_scratch_doubles(int kmax) {
    return 3 * (size_t)kmax * kmax + (size_t)kmax * (kmax + 1);
}

// Scratch of the grid-team projection: four k x k matrices, the packed input
// and output.
__host__ __device__ inline size_t psd_team_doubles(int kmax) {
    return 4 * (size_t)kmax * kmax + (size_t)kmax * (kmax + 1);
}

// Column j and row i of packed index idx (column-major lower triangle).
__device__ __forceinline__ void psd_unpack_index(int k, int idx, int& i, int& j) {
    const double b = 2.0 * k + 1.0;
    j = (int)((b - sqrt(b * b - 8.0 * idx)) * 0.5);
    if (j < 0) j = 0;
    if (j > k - 1) j = k - 1;
    while (j > 0 && j * k - j * (j - 1) / 2 > idx) --j;               // off(j) = j k - j (j - 1) / 2
    while (j + 1 < k && (j + 1) * k - (j + 1) * j / 2 <= idx) ++j;
    i = j + (idx - (j * k - j * (j - 1) / 2));
}

// Dense products of the PSD projection (the warm start Vt0 X Vt0^T and the
// reconstruction V max(lam, 0) V^T) on the FP64 matrix cores.
typedef double psd_d4 __attribute__((ext_vector_type(4)));

// One 16 x 16 tile (rows i0.., columns j0..) of op(A) op(B) for k x k
// row-major matrices, op(X) = X or X^T (TA, TB), by one wavefront with
// v_mfma_f64_16x16x4 steps: for step s, lane l supplies A's entry (i0 + l % 16,
// 4 s + l / 16) and B's entry (4 s + l / 16, j0 + l % 16), and the lane's
// result r (r < 4) is row i0 + 4 r + l / 16 of column j0 + l % 16.  Entries
// past k read as zero.  Eight steps' loads are issued before their products.
// The whole wavefront must take part.  Out of line: its registers stay out of
// the allocation of the projection routines that call it.
template <bool TA, bool TB>
__device__ __noinline__ psd_d4 psd_mfma_tile(int k, const double* A, const double* B, int i0, int j0) {
    const int l = threadIdx.x & (WAVE - 1);
    const int ia = i0 + (l & 15), jb = j0 + (l & 15), lk = l >> 4;
    psd_d4 acc = {0.0, 0.0, 0.0, 0.0};
    constexpr int kBatch = 8;
#pragma unroll 1
    for (int k0 = 0; k0 < k; k0 += 4 * kBatch) {
        double av[kBatch], bv[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int kk = k0 + 4 * u + lk;
            av[u] = (kk < k && ia < k) ? (TA ? A[(size_t)kk * k + ia] : A[(size_t)ia * k + kk]) : 0.0;
            bv[u] = (kk < k && jb < k) ? (TB ? B[(size_t)jb * k + kk] : B[(size_t)kk * k + jb]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
    }
    return acc;
}

// Stores a tile from psd_mfma_tile into C (k x k, row-major).
__device__ __forceinline__ void psd_tile_store(int k, const psd_d4& acc, int i0, int j0, double* C) {
    const int l = threadIdx.x & (WAVE - 1);
    const int col = j0 + (l & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = i0 + 4 * r + (l >> 4);
        if (row < k && col < k) C[(size_t)row * k + col] = acc[r];
    }
}

// Stores the entries on and below the diagonal of a tile of V max(lam, 0) V^T
// into the packed output (column-major lower triangle, off-diagonals times
// sqrt(2)).
__device__ __forceinline__ void psd_tile_store_packed(int k, const psd_d4& acc, int i0, int j0, double* outv) {
    const int l = threadIdx.x & (WAVE - 1);
    const int j = j0 + (l & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = i0 + 4 * r + (l >> 4);
        if (i < k && j <= i) {
            const size_t idx = (size_t)j * k - (size_t)j * (j - 1) / 2 + (i - j);
            outv[idx] = (i == j) ? acc[r] : acc[r] * 1.41421356237309504880;
        }
    }
}

// C = op(A) op(B) (k x k) by the wavefronts of one workgroup, a tile each in turn.
template <bool TA, bool TB>
__device__ __forceinline__ void psd_block_mma(int k, const double* A, const double* B, double* C) {
    const int nt = (k + 15) / 16, w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
#pragma unroll 1
    for (int t = w; t < nt * nt; t += nw) {
        const int i0 = (t / nt) * 16, j0 = (t % nt) * 16;
        psd_tile_store(k, psd_mfma_tile<TA, TB>(k, A, B, i0, j0), i0, j0, C);
    }
}

// outv = svec(Wt^T Vt) by the wavefronts of one workgroup (tiles on and below
// the diagonal).
__device__ __forceinline__ void psd_block_recon(int k, const double* wt, const double* vt, double* outv) {
    const int nt = (k + 15) / 16, w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
#pragma unroll 1
    for (int t = w; t < nt * nt; t += nw) {
        const int ti = t / nt, tj = t % nt;
        if (tj > ti) continue;
        psd_tile_store_packed(k, psd_mfma_tile<true, false>(k, wt, vt, ti * 16, tj * 16), ti * 16, tj * 16, outv);
    }
}

// Rotation (c, s) of a Jacobi step that zeroes apq in the symmetric 2 x 2
// block [app apq; apq aqq]: the smaller of the two angles, t = tan = sign(d)
// e / (|d| + sqrt(d^2 + e^2)) with d = aqq - app, e = 2 apq (the textbook
// t = sign(tau) / (|tau| + sqrt(1 + tau^2)), tau = d / e, multiplied through
// by |e|), so that with w = |d| + sqrt(d^2 + e^2): c = w / sqrt(w^2 + e^2),
// s = sign(d) e / sqrt(w^2 + e^2); one division.  Returns false (c = 1, s = 0)
// when apq is below the rounding of the diagonal, where a rotation changes
// nothing.  Branch-free (the identity is selected afterwards), so that a lane's
// rotations overlap.
__device__ __forceinline__ bool jacobi_rotation(double app, double aqq, double apq, double& c, double& s) {
    const double d = aqq - app, e = 2.0 * apq;
    const double w = fabs(d) + sqrt(d * d + e * e);
    const double g = 1.0 / sqrt(w * w + e * e);
    const bool act = apq != 0.0 && apq * apq > (2.2e-16 * 2.2e-16) * fabs(app * aqq);
    c = act ? w * g : 1.0;
    s = act ? (d >= 0.0 ? e : -e) * g : 0.0;
    return act;
}

// Tile width of the grid-team block Jacobi (psd_project_team) and the order
// of its subproblems (two tiles).
constexpr int kPsdTile = 8;
constexpr int kPsdSub = 2 * kPsdTile;

// Rotation tables of one Jacobi round (LDS, shared by both PSD routines).
struct PsdRound {
    double cs[512], sn[512];
    int pp[512], qq[512];
    double offn;
    int nact;
};

// Inputs of one piece of a team block Jacobi round, gathered from global
// memory in one burst (every load in flight together) and then read from
// LDS: a submatrix of the matrix being turned (up to two pairs' slots by two
// pairs' slots) and the two pairs' Q.  The team path runs after a workgroup's
// one-workgroup blocks, so it shares the rotation tables' LDS.
struct PsdStage {
    double M[2 * kPsdSub][2 * kPsdSub + 1];
    double Qa[kPsdSub][kPsdSub + 1];
    double Qb[kPsdSub][kPsdSub + 1];
};

union PsdLds {
    PsdRound round;
    PsdStage stage;
};

__device__ __forceinline__ PsdLds& psd_lds() {
    __shared__ PsdLds r;
    return r;
}

__device__ __forceinline__ PsdRound& psd_round_lds() { return psd_lds().round; }

// Pairs of round `round` of the round-robin ordering over kk (even) indices:
// position 0 stays, the others rotate; pair h is (pp[h], qq[h]) with p < q.
// Fills rotation (cs, sn) from `mat` for pairs with q < k; counts active ones.
// Called by the threads of one workgroup; ends with a workgroup barrier.
template <bool L = false>
__device__ __forceinline__ void psd_round_params(int k, int kk, int round, const double* mat_, PsdRound& R) {
    const auto mat = vec_at<L>(mat_);
    if (threadIdx.x == 0) R.nact = 0;
    __syncthreads();
    int act = 0;
    for (int h = threadIdx.x; h < kk / 2; h += blockDim.x) {
        const int x = (h == 0) ? 0 : 1 + ((h - 1 + round) % (kk - 1));
        const int y = 1 + ((kk - 2 - h + round) % (kk - 1));
        const int p = x < y ? x : y, q = x < y ? y : x;
        double c = 1.0, s = 0.0;
        if (q < k && jacobi_rotation(mat[p * k + p], mat[q * k + q], mat[p * k + q], c, s)) act = 1;
        R.pp[h] = p; R.qq[h] = q; R.cs[h] = c; R.sn[h] = s;
    }
    if (act) atomicAdd(&R.nact, 1);
    __syncthreads();
}

// One Jacobi round as A <- J^T A J, in place: the rotations are disjoint
// 2 x 2 blocks, so entry block (p1, q1) x (p2, q2) of the result depends only
// on the same block of A and on the two rotations, and each thread reads and
// then overwrites only its own blocks; thread `r` of `nr` takes blocks r,
// r + nr, ...  Rows p, q of Vt turn with J^T in place.  L: A and Vt in LDS.
template <bool L = false>
__device__ __forceinline__ void psd_round_apply(int k, int np, const PsdRound& R, double* mat_, double* vt_, int r,
                                                int nr) {
    const auto mat = vec_at<L>(mat_);
    const auto vt = vec_at<L>(vt_);
    // a thread's items are taken kCh at a time, all loads before any store
    // (the items' entries are distinct), so their loads are in flight together
    constexpr int kCh = 2;
    for (int i0 = r; i0 < np * np; i0 += kCh * nr) {
        int p1[kCh], q1[kCh], p2[kCh], q2[kCh];
        double c1[kCh], s1[kCh], c2[kCh], s2[kCh], app[kCh], apq[kCh], aqp[kCh], aqq[kCh];
#pragma unroll
        for (int u = 0; u < kCh; ++u) {
            const int idx = min(i0 + u * nr, np * np - 1);   // a repeated last item is not stored
            const int h1 = idx / np, h2 = idx - (idx / np) * np;
            p1[u] = R.pp[h1]; q1[u] = R.qq[h1]; p2[u] = R.pp[h2]; q2[u] = R.qq[h2];
            c1[u] = R.cs[h1]; s1[u] = R.sn[h1]; c2[u] = R.cs[h2]; s2[u] = R.sn[h2];
        }
#pragma unroll
        for (int u = 0; u < kCh; ++u) {
            const bool e1 = q1[u] < k, e2 = q2[u] < k;   // the dummy index has no row / column
            app[u] = mat[p1[u] * k + p2[u]];
            apq[u] = e2 ? mat[p1[u] * k + q2[u]] : 0.0;
            aqp[u] = e1 ? mat[q1[u] * k + p2[u]] : 0.0;
            aqq[u] = (e1 && e2) ? mat[q1[u] * k + q2[u]] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kCh; ++u) {
            if (i0 + u * nr >= np * np) continue;
            const bool e1 = q1[u] < k, e2 = q2[u] < k;
            // B = J^T A (rows), then C = B J (columns)
            const double bpp = c1[u] * app[u] - s1[u] * aqp[u], bpq = c1[u] * apq[u] - s1[u] * aqq[u];
            const double bqp = s1[u] * app[u] + c1[u] * aqp[u], bqq = s1[u] * apq[u] + c1[u] * aqq[u];
            mat[p1[u] * k + p2[u]] = c2[u] * bpp - s2[u] * bpq;
            if (e2) mat[p1[u] * k + q2[u]] = s2[u] * bpp + c2[u] * bpq;
            if (e1) mat[q1[u] * k + p2[u]] = c2[u] * bqp - s2[u] * bqq;
            if (e1 && e2) mat[q1[u] * k + q2[u]] = s2[u] * bqp + c2[u] * bqq;
        }
    }
    constexpr int kChV = 4;
    for (int i0 = r; i0 < np * k; i0 += kChV * nr) {
        int pv[kChV], qv[kChV], jv[kChV];
        double cv[kChV], sv[kChV], vp[kChV], vq[kChV];
#pragma unroll
        for (int u = 0; u < kChV; ++u) {
            const int idx = min(i0 + u * nr, np * k - 1);
            const int h = idx / k;
            jv[u] = idx - h * k;
            pv[u] = R.pp[h];
            qv[u] = min(R.qq[h], k - 1);               // dummy partner: read in range, not stored
            cv[u] = R.cs[h];
            sv[u] = R.sn[h];
        }
#pragma unroll
        for (int u = 0; u < kChV; ++u) {
            vp[u] = vt[pv[u] * k + jv[u]];
            vq[u] = vt[qv[u] * k + jv[u]];
        }
#pragma unroll
        for (int u = 0; u < kChV; ++u) {
            const int idx = i0 + u * nr;
            if (idx >= np * k) continue;
            const int h = idx / k;
            if (R.qq[h] >= k || sv[u] == 0.0) continue;
            vt[pv[u] * k + jv[u]] = cv[u] * vp[u] - sv[u] * vq[u];
            vt[qv[u] * k + jv[u]] = sv[u] * vp[u] + cv[u] * vq[u];
        }
    }
}

// `a`, `vm` and `tmp` hold k*k doubles each, `in` and `outv` the packed
// block (in is consumed); V0 (k*k, rows are eigenvectors) and *warm persist
// between calls, or V0 is null.
// L: a and vm are in LDS (tmp, the packed vectors and V0 are not).
template <typename Team, bool L = false>
__device__ __noinline__ void psd_project_block(Team& tm, int k, double* a, double* vm, double* tmp, double* in,
                                               double* outv, double* V0, int* warm) {
    const int t = threadIdx.x, nt = blockDim.x;
    const double rs2 = 0.70710678118654752440;
    // unpack into a: column-major lower triangle, off-diagonals scaled by sqrt(2)
    for (int idx = t; idx < k * (k + 1) / 2; idx += nt) {
        int i, j;
        psd_unpack_index(k, idx, i, j);
        const double v = in[idx];
        if (i == j) a[i * k + i] = v;
        else { a[i * k + j] = v * rs2; a[j * k + i] = v * rs2; }
    }
    __syncthreads();
    double* mat = a;        // the matrix being diagonalised; tmp is the transpose buffer
    const bool use_warm = V0 != nullptr && *warm != 0;
    if (use_warm) {
        psd_block_mma<false, false>(k, V0, a, tmp);    // tmp = Vt0 A
        __syncthreads();
        psd_block_mma<false, true>(k, tmp, V0, a);     // a = (Vt0 A) Vt0^T
        __syncthreads();
        for (int idx = t; idx < k * k; idx += nt) {     // symmetrise (rounding) and start from Vt0
            const int i = idx / k, j = idx - (idx / k) * k;
            if (i < j) {
                const double v = 0.5 * (mat[i * k + j] + mat[j * k + i]);
                mat[i * k + j] = v;
                mat[j * k + i] = v;
            }
            vm[idx] = V0[idx];
        }
    } else {
        for (int idx = t; idx < k * k; idx += nt) vm[idx] = ((idx / k) == (idx % k)) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (k > 1) {
        const int kk = (k & 1) ? k + 1 : k;   // pad to even with a dummy index
        PsdRound& R = psd_round_lds();
        // stop once the off-diagonal part is at the rounding level of a k x k
        // matrix, or when a sweep near that level no longer gains the quadratic factor
        const double tol2 = fmax(1e-30, (1e-16 * k) * (1e-16 * k));
        double prev = 1.0;
        for (int sweep = 0; sweep < 30; ++sweep) {
            // squared off-diagonal Frobenius norm relative to the whole matrix
            {
                __shared__ double red2[2 * NWMAX];
                double off = 0.0, tot = 0.0;
                const auto ml = vec_at<L>(mat);
                for (int idx = t; idx < k * k; idx += nt) {
                    const double v = ml[idx] * ml[idx];
                    tot += v;
                    if ((idx / k) != (idx % k)) off += v;
                }
                off = wave_sum(off);
                tot = wave_sum(tot);
                if ((t & (WAVE - 1)) == 0) { red2[t / WAVE] = off; red2[NWMAX + t / WAVE] = tot; }
                __syncthreads();
                if (t == 0) {
                    double so = 0.0, st = 0.0;
                    for (int w = 0; w < nt / WAVE; ++w) { so += red2[w]; st += red2[NWMAX + w]; }
                    R.offn = (st > 0.0) ? so / st : 0.0;
                }
                __syncthreads();
            }
            const double cur = R.offn;
            if (cur <= tol2 || (cur <= 1e-24 && cur > 0.25 * prev)) break;
            prev = cur;
            for (int round = 0; round < kk - 1; ++round) {
                psd_round_params<L>(k, kk, round, mat, R);
                if (R.nact == 0) continue;                  // uniform: nothing to rotate this round
                psd_round_apply<L>(k, kk / 2, R, mat, vm, t, nt);
                __syncthreads();
            }
        }
    }
    // reconstruct V max(lam, 0) V^T in packed form with Vt = V^T: lam into
    // `in` (consumed), Wt = diag(lam+) Vt into tmp, then Wt^T Vt
    for (int e = t; e < k; e += nt) in[e] = fmax(mat[e * k + e], 0.0);
    __syncthreads();
    for (int idx = t; idx < k * k; idx += nt) tmp[idx] = vm[idx] * in[idx / k];
    __syncthreads();
    psd_block_recon(k, tmp, vm, outv);
    if (V0 != nullptr) {
        for (int idx = t; idx < k * k; idx += nt) V0[idx] = vm[idx];
        if (t == 0) *warm = 1;
    }
    __syncthreads();
}

// The same projection computed by a team of workgroups (the grid, or its PSD
// sub-team), for blocks too large for one workgroup to turn over quickly (the
// order-256 block of the sparse-PCA instance): a two-sided *block* Jacobi
// method.  The indices are cut into tiles of kPsdTile; each round pairs the
// tiles round-robin, one workgroup per pair diagonalises (approximately: one
// inner sweep) the pair's 2-tile principal submatrix in LDS, producing an
// orthogonal Q_w, and the team turns A into
// Q^T A Q and Vt into Q^T Vt, block by block.  One team barrier per round and
// k/kPsdTile - 1 rounds per sweep, instead of one barrier per round over
// k - 1 rounds (the round structure is described at psd_project_team).  Warm
// start and stopping rule as in psd_project_block.

struct PsdSub {
    double S[kPsdSub][kPsdSub + 1];
    double Q[kPsdSub][kPsdSub + 1];
};

__device__ __forceinline__ PsdSub& psd_sub_lds() {
    __shared__ PsdSub r;
    return r;
}

// Global index of slot `a` (0 .. kPsdSub-1) of tile pair (t1, t2), or -1 when
// the slot lies past k or in the dummy tile.
__device__ __forceinline__ int psd_slot_index(int k, int nt, int t1, int t2, int a) {
    const int t = a < kPsdTile ? t1 : t2;
    if (t >= nt) return -1;
    const int g = t * kPsdTile + (a % kPsdTile);
    return g < k ? g : -1;
}

// Tile pair h of round `round` over ntt (even) tile positions.
__device__ __forceinline__ void psd_tile_pair(int ntt, int round, int h, int& t1, int& t2) {
    const int x = (h == 0) ? 0 : 1 + ((h - 1 + round) % (ntt - 1));
    const int y = 1 + ((ntt - 2 - h + round) % (ntt - 1));
    t1 = x < y ? x : y;
    t2 = x < y ? y : x;
}

// Tile pair containing tile t in round `round`, and t's side (0: first tile):
// psd_tile_pair inverted.  Tile 0 is in pair 0; a tile t > 0 is the moving
// entry x of pair h = ((t - 1 - round) mod (ntt - 1)) + 1 when that h is a
// pair, else the entry y of pair (ntt - 2 + round - (t - 1)) mod (ntt - 1).
__device__ __forceinline__ int psd_tile_owner(int ntt, int round, int t, int& side) {
    int h = 0;
    if (t > 0) {
        const int m = ntt - 1, a = t - 1;
        const int hx = ((a - round) % m + m) % m + 1;
        h = hx <= ntt / 2 - 1 ? hx : (ntt - 2 + round - a) % m;
    }
    int t1, t2;
    psd_tile_pair(ntt, round, h, t1, t2);
    side = t == t1 ? 0 : 1;
    return h;
}

// Orders LDS accesses between the lanes of one wavefront (a wavefront runs in
// lockstep and its LDS operations complete in issue order; the fences keep
// the compiler from moving accesses across this point).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inner sweeps per tile subproblem of the team block Jacobi.  The outer
// method converges with approximate subproblem solutions (each inner sweep
// is a block of the scalar method's rotations); the outer stopping test
// alone decides the accuracy.
constexpr int kPsdInnerSweeps = 1;

// Cyclic Jacobi on the symmetric kPsdSub x kPsdSub matrix in L.S (filled and
// visible to the workgroup); writes its eigenvectors Q (slot x slot,
// row-major, new column b = sum_a Q[a][b] old column a) to q.  Called by a
// whole workgroup: the sweeps run on the first wavefront alone (the eight
// rotations of a round, eight lanes per rotation, each lane computing its
// rotation itself; wavefront ordering instead of workgroup barriers).
__device__ __noinline__ void psd_sub_jacobi(double* q) {
    PsdSub& L = psd_sub_lds();
    const int t = threadIdx.x, n = blockDim.x;
    for (int e = t; e < kPsdSub * kPsdSub; e += n) L.Q[e / kPsdSub][e % kPsdSub] = (e / kPsdSub == e % kPsdSub) ? 1.0 : 0.0;
    __syncthreads();
    if (t < WAVE) {
        constexpr int kHalf = kPsdSub / 2;                      // rotations per round
        constexpr int kLanes = WAVE / kHalf;                    // lanes per rotation
        constexpr int kPer = kPsdSub / kLanes;                  // indices per lane
        static_assert(kLanes * kHalf == WAVE && kPer * kLanes == kPsdSub, "one wavefront per subproblem");
        const double tol2 = (1e-16 * kPsdSub) * (1e-16 * kPsdSub);
        double prev = 1.0;
        for (int sweep = 0; sweep < kPsdInnerSweeps; ++sweep) {
            double off = 0.0, tot = 0.0;
            for (int e = t; e < kPsdSub * kPsdSub; e += WAVE) {
                const double v = L.S[e / kPsdSub][e % kPsdSub] * L.S[e / kPsdSub][e % kPsdSub];
                tot += v;
                if (e / kPsdSub != e % kPsdSub) off += v;
            }
            off = wave_sum(off);
            tot = wave_sum(tot);
            const double cur = tot > 0.0 ? off / tot : 0.0;
            if (cur <= tol2 || (cur <= 1e-24 && cur > 0.25 * prev)) break;
            prev = cur;
            for (int round = 0; round < kPsdSub - 1; ++round) {
                // lane t serves pair h = t / kLanes (kLanes lanes per pair) at
                // indices (t % kLanes) + r kLanes, r < kPer, and computes that
                // pair's rotation itself (the lanes of a pair agree: same
                // inputs).  Each step issues all its LDS loads before its
                // stores (the items touch distinct entries), so they are in
                // flight together.
                int p, qq;
                psd_tile_pair(kPsdSub, round, t / kLanes, p, qq);
                double c, sn;
                jacobi_rotation(L.S[p][p], L.S[qq][qq], L.S[p][qq], c, sn);
                double x0[kPer], x1[kPer], x2[kPer], x3[kPer];
                wave_lds_sync();
                // rows p, q of S <- J^T S (an identity rotation rewrites its
                // entries unchanged: c x - 0 y = x)
#pragma unroll
                for (int r = 0; r < kPer; ++r) {
                    const int j = t % kLanes + r * kLanes;
                    x0[r] = L.S[p][j];
                    x1[r] = L.S[qq][j];
                }
#pragma unroll
                for (int r = 0; r < kPer; ++r) {
                    const int j = t % kLanes + r * kLanes;
                    L.S[p][j] = c * x0[r] - sn * x1[r];
                    L.S[qq][j] = sn * x0[r] + c * x1[r];
                }
                wave_lds_sync();
                // columns p, q of S and of Q <- (.) J
#pragma unroll
                for (int r = 0; r < kPer; ++r) {
                    const int i = t % kLanes + r * kLanes;
                    x0[r] = L.S[i][p];
                    x1[r] = L.S[i][qq];
                    x2[r] = L.Q[i][p];
                    x3[r] = L.Q[i][qq];
                }
#pragma unroll
                for (int r = 0; r < kPer; ++r) {
                    const int i = t % kLanes + r * kLanes;
                    L.S[i][p] = c * x0[r] - sn * x1[r];
                    L.S[i][qq] = sn * x0[r] + c * x1[r];
                    L.Q[i][p] = c * x2[r] - sn * x3[r];
                    L.Q[i][qq] = sn * x2[r] + c * x3[r];
                }
                wave_lds_sync();
            }
        }
    }
    __syncthreads();
    for (int e = t; e < kPsdSub * kPsdSub; e += n) q[e] = L.Q[e / kPsdSub][e % kPsdSub];
    __syncthreads();
}

template <typename At>
__device__ void psd_sub_diag(int k, int nt, int t1, int t2, At at, double* q) {
    PsdSub& L = psd_sub_lds();
    for (int e = threadIdx.x; e < kPsdSub * kPsdSub; e += blockDim.x) {
        const int a = e / kPsdSub, b = e % kPsdSub;
        const int ga = psd_slot_index(k, nt, t1, t2, a), gb = psd_slot_index(k, nt, t1, t2, b);
        L.S[a][b] = (ga >= 0 && gb >= 0) ? at(ga, gb) : 0.0;
    }
    __syncthreads();
    psd_sub_jacobi(q);
}

// Subproblem of tile pair h of round `nr`, taken from the matrix after round
// r (B = Q_r^T A Q_r, A = mat, Q_r of every round-r pair at qr), computed from
// A and Q_r directly.  The two new tiles u1, u2 sit in two different round-r
// pairs o1, o2 (a pair meets once per sweep), so B restricted to them needs
// only A on the slots of o1 and o2 (32 x 32) and Q_o1, Q_o2: these are staged
// in LDS first.  Then T = A[slots of o(u), slots of o(b)] Q_o(b)[:, b]
// (2 x 16 x 16, in the LDS of L) and S[a][b] = sum_x Q_o(a)[x][a'] T[x][b],
// with a', b the new slots' places in their round-r pairs.  Then diagonalised;
// Q to q.  Whole workgroup.
__device__ __noinline__ void psd_next_sub(int k, int nt, int ntt, int r, int nr, int h, const double* mat,
                                          const double* qr, double* q) {
    PsdSub& L = psd_sub_lds();
    PsdStage& G = psd_lds().stage;
    double* T = &L.S[0][0];                        // 2 * kPsdSub * kPsdSub doubles over S and Q
    const int t = threadIdx.x, n = blockDim.x;
    int u1, u2;
    psd_tile_pair(ntt, nr, h, u1, u2);
    int s1, s2;                                    // sides of u1, u2 in their round-r pairs
    const int o1 = psd_tile_owner(ntt, r, u1, s1), o2 = psd_tile_owner(ntt, r, u2, s2);
    int a1, a2, b1, b2;
    psd_tile_pair(ntt, r, o1, a1, a2);
    psd_tile_pair(ntt, r, o2, b1, b2);
    for (int e = t; e < 4 * kPsdSub * kPsdSub; e += n) {
        const int x = e / (2 * kPsdSub), y = e - (e / (2 * kPsdSub)) * (2 * kPsdSub);
        const int gx = x < kPsdSub ? psd_slot_index(k, nt, a1, a2, x) : psd_slot_index(k, nt, b1, b2, x - kPsdSub);
        const int gy = y < kPsdSub ? psd_slot_index(k, nt, a1, a2, y) : psd_slot_index(k, nt, b1, b2, y - kPsdSub);
        G.M[x][y] = (gx >= 0 && gy >= 0) ? mat[(size_t)gx * k + gy] : 0.0;
    }
    for (int e = t; e < 2 * kPsdSub * kPsdSub; e += n) {
        const int w = e / (kPsdSub * kPsdSub), f = e - w * (kPsdSub * kPsdSub);
        const double v = qr[(size_t)(w ? o2 : o1) * kPsdSub * kPsdSub + f];
        if (w) G.Qb[f / kPsdSub][f % kPsdSub] = v;
        else G.Qa[f / kPsdSub][f % kPsdSub] = v;
    }
    __syncthreads();
    for (int e = t; e < 2 * kPsdSub * kPsdSub; e += n) {
        const int sr = e / (kPsdSub * kPsdSub), x = (e / kPsdSub) % kPsdSub, b = e % kPsdSub;
        const int cb = (b < kPsdTile ? s1 : s2) * kPsdTile + b % kPsdTile;
        const int yo = b < kPsdTile ? 0 : kPsdSub;
        double v = 0.0;
#pragma unroll
        for (int y = 0; y < kPsdSub; ++y)
            v += G.M[sr * kPsdSub + x][yo + y] * (b < kPsdTile ? G.Qa[y][cb] : G.Qb[y][cb]);
        T[e] = v;
    }
    __syncthreads();
    double s_ = 0.0;
    if (t < kPsdSub * kPsdSub) {
        const int a = t / kPsdSub, b = t % kPsdSub;
        const int ga = psd_slot_index(k, nt, u1, u2, a), gb = psd_slot_index(k, nt, u1, u2, b);
        if (ga >= 0 && gb >= 0) {
            const int ca = (a < kPsdTile ? s1 : s2) * kPsdTile + a % kPsdTile;
            const double* tr = T + (size_t)(a / kPsdTile) * kPsdSub * kPsdSub;
#pragma unroll
            for (int x = 0; x < kPsdSub; ++x) s_ += (a < kPsdTile ? G.Qa[x][ca] : G.Qb[x][ca]) * tr[x * kPsdSub + b];
        }
    }
    __syncthreads();
    if (t < kPsdSub * kPsdSub) L.S[t / kPsdSub][t % kPsdSub] = s_;
    __syncthreads();
    psd_sub_jacobi(q);
}

// Pieces of the team block Jacobi, out of line and with bounded unrolling:
// the solve kernel calls the PSD team path from inside its projection passes,
// and every register this call tree touches is one the kernel cannot keep a
// value in across the call, so the tree is kept small.  Each piece is run by
// every thread of the team over the index range r0, r0 + R, ...

// C = op(A) op(B) (k x k, row-major) by the team's wavefronts, a 16 x 16
// tile each: tile t goes to workgroup t % nblk, so a small product spreads
// over the whole grid.
template <bool TA, bool TB>
__device__ __noinline__ void psd_team_mma(int blk, int nblk, int k, const double* A, const double* B, double* C) {
    const int nt = (k + 15) / 16, w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
#pragma unroll 1
    for (int t = blk + nblk * w; t < nt * nt; t += nblk * nw) {
        const int i0 = (t / nt) * 16, j0 = (t % nt) * 16;
        psd_tile_store(k, psd_mfma_tile<TA, TB>(k, A, B, i0, j0), i0, j0, C);
    }
}

// Step (a) of a team block Jacobi round: output blocks (pair hi, pair hc) of
// Q^T mat Q into out, one workgroup per block (workgroups blk, blk + nblk,
// ... of the ones taking part); the input block and the two Q are staged in
// LDS first.  On the sweep's last round also the squared off-diagonal and
// total mass of the output (added to off, tot).
__device__ __noinline__ void psd_team_blocks(int blk, int nblk, int k, int nt, int ntt, int np, int round, bool last,
                                             const double* mat, double* out, const double* qr, double* acc) {
    PsdSub& L = psd_sub_lds();
    PsdStage& G = psd_lds().stage;
    double off = 0.0, tot = 0.0;
    const int e = threadIdx.x;
    for (int bid = blk; bid < np * np; bid += nblk) {
        const int hi = bid / np, hc = bid - (bid / np) * np;
        int i1, i2, c1, c2;
        psd_tile_pair(ntt, round, hi, i1, i2);
        psd_tile_pair(ntt, round, hc, c1, c2);
        const double* qi = qr + (size_t)hi * kPsdSub * kPsdSub;
        const double* qc = qr + (size_t)hc * kPsdSub * kPsdSub;
        for (int f = e; f < 3 * kPsdSub * kPsdSub; f += blockDim.x) {
            const int w = f / (kPsdSub * kPsdSub), g = f - w * (kPsdSub * kPsdSub);
            const int x = g / kPsdSub, y = g % kPsdSub;
            if (w == 0) {
                const int gx = psd_slot_index(k, nt, i1, i2, x), gy = psd_slot_index(k, nt, c1, c2, y);
                G.M[x][y] = (gx >= 0 && gy >= 0) ? mat[(size_t)gx * k + gy] : 0.0;
            } else if (w == 1) {
                G.Qa[x][y] = qi[g];
            } else {
                G.Qb[x][y] = qc[g];
            }
        }
        __syncthreads();
        if (e < kPsdSub * kPsdSub) {               // L.S = mat[block] Q_c
            const int x = e / kPsdSub, cb = e % kPsdSub;
            double v = 0.0;
#pragma unroll
            for (int y = 0; y < kPsdSub; ++y) v += G.M[x][y] * G.Qb[y][cb];
            L.S[x][cb] = v;
        }
        __syncthreads();
        if (e < kPsdSub * kPsdSub) {               // block of the output = Q_i^T L.S
            const int ia = e / kPsdSub, cb = e % kPsdSub;
            const int gi = psd_slot_index(k, nt, i1, i2, ia), gc = psd_slot_index(k, nt, c1, c2, cb);
            if (gi >= 0 && gc >= 0) {
                double v = 0.0;
#pragma unroll
                for (int x = 0; x < kPsdSub; ++x) v += G.Qa[x][ia] * L.S[x][cb];
                out[(size_t)gi * k + gc] = v;
                if (last) {
                    tot += v * v;
                    if (gi != gc) off += v * v;
                }
            }
        }
        __syncthreads();
    }
    acc[0] = off;
    acc[1] = tot;
}

// Step (b): vout = Q^T vin on the rows of each pair of the round, one row per
// workgroup (rows w, w + nw, ... of the workgroups taking part), a thread per
// column; the row's sixteen source rows are read in one burst.
__device__ __noinline__ void psd_team_rows(int w, int nw, int k, int nt, int ntt, int round, const double* qr,
                                           const double* vin, double* vout) {
    for (int rw = w; rw < k; rw += nw) {
        int side;
        const int h = psd_tile_owner(ntt, round, rw / kPsdTile, side);
        int t1, t2;
        psd_tile_pair(ntt, round, h, t1, t2);
        const double* q = qr + (size_t)h * kPsdSub * kPsdSub;
        const int ip = side * kPsdTile + rw % kPsdTile;
        for (int j = threadIdx.x; j < k; j += blockDim.x) {
            double src[kPsdSub];
#pragma unroll
            for (int x = 0; x < kPsdSub; ++x) {
                const int gx = psd_slot_index(k, nt, t1, t2, x);
                src[x] = gx >= 0 ? vin[(size_t)gx * k + j] : 0.0;
            }
            double sv = 0.0;
#pragma unroll
            for (int x = 0; x < kPsdSub; ++x) sv += q[x * kPsdSub + ip] * src[x];
            vout[(size_t)rw * k + j] = sv;
        }
    }
}

// Packed output: outv = svec(Wt^T Vt), Wt = diag(lam+) Vt, by the team's
// wavefronts (tiles on and below the diagonal).
__device__ __noinline__ void psd_team_recon(int blk, int nblk, int k, const double* wt, const double* vt, double* outv) {
    const int nt = (k + 15) / 16, w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
#pragma unroll 1
    for (int t = blk + nblk * w; t < nt * nt; t += nblk * nw) {
        const int ti = t / nt, tj = t % nt;
        if (tj > ti) continue;
        psd_tile_store_packed(k, psd_mfma_tile<true, false>(k, wt, vt, ti * 16, tj * 16), ti * 16, tj * 16, outv);
    }
}

// `buf` holds 4 k*k doubles (matrix, its turned copy, Vt and its turned copy);
// `in` (packed input, filled by the caller) and `outv` are contiguous, with
// room for two rounds' Q matrices (k (k + 1) doubles in all, k > 2 kPsdTile).
// A round is one phase and one team barrier: (a) every 16 x 16 output block
// of Q^T A Q turned from its input block and the two pairs' Q, (b) the pairs'
// rows of Vt turned, and, at the same time on np workgroups of their own,
// (c) the next round's subproblems built from A and this round's Q directly
// and diagonalised (psd_next_sub).  `Team` is the grid team or its PSD
// sub-team.
template <typename Team>
__device__ __noinline__ void psd_project_team(Team& tm, Shared& sh, int k, double* buf, double* in, double* outv, double* V0,
                                 int* warm) {
    const int r0 = tm.rank(), R_ = tm.size();
    const double rs2 = 0.70710678118654752440;
    double* mat = buf;
    double* tmp = buf + (size_t)k * k;
    double* vm = tmp + (size_t)k * k;
    double* vm2 = vm + (size_t)k * k;
    double* qbuf[2] = {in, in + (size_t)((k / kPsdTile + 2) / 2) * kPsdSub * kPsdSub};   // Q of two rounds
    for (int idx = r0; idx < k * (k + 1) / 2; idx += R_) {
        int i, j;
        psd_unpack_index(k, idx, i, j);
        const double v = in[idx];
        if (i == j) mat[i * k + i] = v;
        else { mat[i * k + j] = v * rs2; mat[j * k + i] = v * rs2; }
    }
    tm.sync();
    const bool use_warm = V0 != nullptr && *warm != 0;
    if (use_warm) {
        psd_team_mma<false, false>(tm.blk(), tm.nblk(), k, V0, mat, tmp);    // tmp = Vt0 A
        tm.sync();
        psd_team_mma<false, true>(tm.blk(), tm.nblk(), k, tmp, V0, vm2);     // vm2 = (Vt0 A) Vt0^T
        tm.sync();
        for (int idx = r0; idx < k * k; idx += R_) {
            const int i = idx / k, j = idx - (idx / k) * k;
            mat[idx] = 0.5 * (vm2[i * k + j] + vm2[j * k + i]);   // symmetrise (rounding)
            vm[idx] = V0[idx];
        }
    } else {
        for (int idx = r0; idx < k * k; idx += R_) vm[idx] = ((idx / k) == (idx % k)) ? 1.0 : 0.0;
    }
    tm.sync();
    const int nt = (k + kPsdTile - 1) / kPsdTile;        // tiles
    const int ntt = nt + (nt & 1);                        // even, with a dummy tile
    const int np = ntt / 2;
    const double tol2 = fmax(1e-30, (1e-16 * k) * (1e-16 * k));
    PsdSub& L = psd_sub_lds();
    // off-diagonal mass of the starting matrix
    {
        double off = 0.0, tot = 0.0;
        for (int idx = r0; idx < k * k; idx += R_) {
            const double v = mat[idx] * mat[idx];
            tot += v;
            if ((idx / k) != (idx % k)) off += v;
        }
        put(sh, 0, off);
        put(sh, 1, tot);
        tm.reduce(sh, 2);
    }
    double cur = sh.out[1] > 0.0 ? sh.out[0] / sh.out[1] : 0.0;
    if (cur > tol2) {
        // Q of round 0 from the matrix itself
        for (int h = tm.blk(); h < np; h += tm.nblk()) {
            int t1, t2;
            psd_tile_pair(ntt, 0, h, t1, t2);
            psd_sub_diag(k, nt, t1, t2, [&](int i, int j) { return mat[(size_t)i * k + j]; },
                         qbuf[0] + (size_t)h * kPsdSub * kPsdSub);
        }
        tm.sync();
        double prev = 1.0;
        long long g = 0;                                  // rounds done; Q of round g is in qbuf[g & 1]
        // (a) and (b) below run on the workgroups under `split`, (c) on the
        // np from it: (c) is the longest piece, so its workgroups take no other
        // work (with few workgroups, every one takes all three)
        const int nb = tm.nblk(), wb = tm.blk();
        const int split = nb > 2 * np ? nb - np : nb;
        const int h0 = split < nb ? wb - split : wb, hs = split < nb ? np : nb;
        for (int sweep = 0; sweep < 30; ++sweep) {
            double acc[2] = {0.0, 0.0};
            for (int round = 0; round < ntt - 1; ++round, ++g) {
                const double* qr = qbuf[g & 1];
                const bool last = round == ntt - 2;
                if (wb < split) {
                    // (a) mat2 = Q^T mat Q, block by block: output block (pair hi,
                    // pair hc) needs input block (hi, hc) and the two pairs' Q
                    // only; (b) the pairs' rows of Vt
                    psd_team_blocks(wb, split, k, nt, ntt, np, round, last, mat, tmp, qr, acc);
                    psd_team_rows(wb, split, k, nt, ntt, round, qr, vm, vm2);
                }
                // (c) Q of the next round (the next sweep's first after the last)
                // from mat and this round's Q; unused if the sweeps stop here
                for (int h = h0; h >= 0 && h < np; h += hs)
                    psd_next_sub(k, nt, ntt, round, last ? 0 : round + 1, h, mat, qr,
                                 qbuf[(g + 1) & 1] + (size_t)h * kPsdSub * kPsdSub);
                double* sw = mat;
                mat = tmp;
                tmp = sw;
                sw = vm;
                vm = vm2;
                vm2 = sw;
                if (last) {
                    put(sh, 0, acc[0]);
                    put(sh, 1, acc[1]);
                    tm.reduce(sh, 2);
                } else {
                    tm.sync();
                }
            }
            cur = sh.out[1] > 0.0 ? sh.out[0] / sh.out[1] : 0.0;
            if (cur <= tol2 || (cur <= 1e-24 && cur > 0.25 * prev)) break;
            prev = cur;
        }
    }
    // reconstruct from Vt: lam into `in`, Wt = diag(lam+) Vt into tmp
    for (int e = r0; e < k; e += R_) in[e] = fmax(mat[e * k + e], 0.0);
    tm.sync();
    for (int idx = r0; idx < k * k; idx += R_) tmp[idx] = vm[idx] * in[idx / k];
    tm.sync();
    psd_team_recon(tm.blk(), tm.nblk(), k, tmp, vm, outv);
    if (V0 != nullptr) {
        for (int idx = r0; idx < k * k; idx += R_) V0[idx] = vm[idx];
        if (r0 == 0) *warm = 1;
    }
    tm.sync();
}

// Blocks of order above this go to the whole grid team.
constexpr int kPsdTeamOrder = 64;

// First workgroup of the PSD sub-team (PsdSubTeam) for a grid of G
// workgroups: when an instance has both blocks up to kPsdTeamOrder and larger
// ones, workgroups 0 .. s - 1 project the s small blocks, one each, while the
// others project the large blocks together, at the same time.  0 (the small
// blocks first, then the large ones by the whole grid) when there are no
// small blocks, or when they would leave the large blocks fewer than half the
// grid or too few workgroups for a round's subproblems and turns.
__device__ inline int psd_sub_start(const ConeDev& K, int G) {
    if (K.ns == 0 || K.psd_kmax <= kPsdTeamOrder) return 0;
    int small = 0;
    for (int c = 0; c < K.ns; ++c) small += K.sord[c] <= kPsdTeamOrder ? 1 : 0;
    const int nt = (K.psd_kmax + kPsdTile - 1) / kPsdTile, np = (nt + (nt & 1)) / 2;
    if (small == 0 || G - small < max(2 * np + 1, G / 2)) return 0;
    return small;
}

// The blocks above kPsdTeamOrder, projected by team t (the grid team, or its
// PSD sub-team).
template <typename T2, typename In, typename Emit>
__device__ __forceinline__ void psd_project_large(T2& t, Shared& sh, int n, const ConeDev& K, In& in, Emit& emit) {
    double* tb = K.psd_team;                     // 4 kmax^2 matrices, then input / output
    double* tin = tb + 4 * (size_t)K.psd_kmax * K.psd_kmax;
    double* tout = tin + (size_t)K.psd_kmax * (K.psd_kmax + 1) / 2;
    for (int c = 0; c < K.ns; ++c) {
        const int k = K.sord[c];
        if (k <= kPsdTeamOrder) continue;
        const int o = n + K.psd0 + K.soff[c];
        const int len = k * (k + 1) / 2;
        t.sync();
        for (int e = t.rank(); e < len; e += t.size()) tin[e] = in(o + e);
        t.sync();
        psd_project_team(t, sh, k, tb, tin, tout, K.psd_vecs ? K.psd_vecs + (size_t)c * K.psd_kmax * K.psd_kmax : nullptr,
                         K.psd_warm ? K.psd_warm + c : nullptr);
        for (int e = t.rank(); e < len; e += t.size()) emit(o + e, tout[e]);
    }
}

// ---------------------------------------------------------------- Pi_C pass

template <typename Team, typename In, typename Emit>
__device__ __forceinline__ void project_C(Team& tm, Shared& sh, int n, int N, const ConeDev& K, In&& in,
                                          Emit&& emit) {
    // elementwise part: x, zero rows, R+ rows, tau
    const int nel = n + K.z + K.l;
    for (int i = tm.rank(); i <= nel; i += tm.size()) {
        const int gi = (i < nel) ? i : N - 1;
        double v = in(gi);
        if (gi >= n + K.z) v = fmax(v, 0.0);
        emit(gi, v);
    }
    // second-order cones, t last: one wavefront per cone
    const int lane = threadIdx.x & (WAVE - 1);
    for (int c = tm.wave(); c < K.nq; c += tm.nwaves()) {
        const int o = n + K.soc0 + K.qoff[c];
        const int k = K.qoff[c + 1] - K.qoff[c];
        double ss = 0.0;
        for (int e = lane; e < k - 1; e += WAVE) { const double v = in(o + e); ss += v * v; }
        ss = wave_sum(ss);
        const double nx = sqrt(ss);
        const double t = in(o + k - 1);
        if (nx <= t) {
            for (int e = lane; e < k; e += WAVE) emit(o + e, in(o + e));
        } else if (nx <= -t) {
            for (int e = lane; e < k; e += WAVE) emit(o + e, 0.0);
        } else {
            const double a = 0.5 * (nx + t), sc = a / nx;
            for (int e = lane; e < k - 1; e += WAVE) emit(o + e, sc * in(o + e));
            if (lane == 0) emit(o + k - 1, a);
        }
    }
    // exponential cones: one thread per cone
    for (int c = tm.rank(); c < K.ep; c += tm.size()) {
        const int o = n + K.exp0 + 3 * c;
        double v[3] = {in(o), in(o + 1), in(o + 2)}, p[3];
        proj_exp_dual(v, p);
        emit(o, p[0]);
        emit(o + 1, p[1]);
        emit(o + 2, p[2]);
    }
    // PSD blocks: one workgroup per block (the whole workgroup takes the loop
    // together, so the barriers inside are uniform); in a grid team, blocks of
    // order above kPsdTeamOrder are then projected by the whole team
    if (K.ns > 0) {
        constexpr bool kGrid = !Team::kBlock;
        double* a = K.psd_scratch + (size_t)tm.blk() * psd_scratch_doubles(K.psd_kmax);
        double* vm = a + (size_t)K.psd_kmax * K.psd_kmax;
        double* tmpm = vm + (size_t)K.psd_kmax * K.psd_kmax;
        double* pin = tmpm + (size_t)K.psd_kmax * K.psd_kmax;
        double* pout = pin + (size_t)K.psd_kmax * (K.psd_kmax + 1) / 2;
        // grid teams: the blocks projected one per workgroup keep their matrix
        // and eigenvectors in LDS when the launch reserved the area
        bool lds = false;
        if constexpr (kGrid) {
            if (K.psd_lds > 0) {
                lds = true;
                a = sscs_dyn_lds;
                vm = a + (size_t)K.psd_small * K.psd_small;
            }
        }
        // with a PSD sub-team, the small blocks go to the workgroups before it
        int cstride = tm.nblk();
        bool small_here = true;
        if constexpr (kGrid && Team::kPsdTeam) {
            if (tm.sub0 > 0) {
                cstride = tm.sub0;
                small_here = tm.blk() < tm.sub0;
            }
        }
        for (int c = small_here ? tm.blk() : K.ns; c < K.ns; c += cstride) {
            const int k = K.sord[c];
            if (kGrid && k > kPsdTeamOrder) continue;
            const int o = n + K.psd0 + K.soff[c];
            const int len = k * (k + 1) / 2;
            for (int e = threadIdx.x; e < len; e += blockDim.x) pin[e] = in(o + e);
            __syncthreads();
            double* V0 = K.psd_vecs ? K.psd_vecs + (size_t)c * K.psd_kmax * K.psd_kmax : nullptr;
            int* wf = K.psd_warm ? K.psd_warm + c : nullptr;
            if (lds) psd_project_block<Team, true>(tm, k, a, vm, tmpm, pin, pout, V0, wf);
            else psd_project_block<Team, false>(tm, k, a, vm, tmpm, pin, pout, V0, wf);
            for (int e = threadIdx.x; e < len; e += blockDim.x) emit(o + e, pout[e]);
            __syncthreads();
        }
        if constexpr (kGrid && Team::kPsdTeam) {
            if (K.psd_kmax > kPsdTeamOrder) {
                if (tm.sub0 > 0) {
                    if (tm.blk() >= tm.sub0) {
                        PsdSubTeam<Team> st{tm};
                        psd_project_large(st, sh, n, K, in, emit);
                    }
                } else {
                    psd_project_large(tm, sh, n, K, in, emit);
                }
            }
        }
    }
}

}  // namespace sscs
