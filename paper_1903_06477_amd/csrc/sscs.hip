// libsscs: kernels and the C ABI declared in include/sscs.h.
//
// Kernels
//   k_solve_grid   whole Algorithm 1 for one large instance; cooperative
//                  launch, the grid is one GridTeam (grid barriers).
//   k_op_grid      one component call (linear step, residual, projection,
//                  setup of g and delta) on the same device code.
//   k_solve_batch  persistent batched solve: each workgroup pops instances from
//                  a device queue and runs Algorithm 1 as a BlockTeam.
//   k_spmv         stand-alone row-segmented SpMV (the CG's SpMV, timed alone).
//   setup kernels  CSR transpose (count, scan, scatter, per-row sort), Jacobi
//                  diagonal.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <map>
#include <vector>

#include "../../include/sscs.h"
#include "dev_engine.h"

using namespace sscs;

namespace {

constexpr int kBlock = 512;            // threads per workgroup of the grid-team kernels
constexpr int kBatchBlock = 256;
constexpr int kStageMax = 12288;       // doubles of LDS for the one-workgroup CG's gathered vectors (96 KB)

enum { OP_LINEAR = 0, OP_RESIDUAL = 1, OP_PROJECT = 2, OP_SETUP = 3 };

struct OpArgs {
    int op;
    const double* in;
    double* out1;
    double* out2;
    double* scal;     // OP_SETUP: [delta, ||b||, ||c||]
    double tol;
    int maxit;
};

}  // namespace

// ------------------------------------------------------------------ kernels

// Workgroup b of a grid kernel owns rows [part[b], part[b+1]) of A and of A^T
// and, when the operator fits, keeps them in LDS for the whole launch.
template <bool LDS, typename TL, bool PT>
__device__ inline void grid_team_init(GridTeam<LDS, TL, PT>& tm, const Prob& P) {
    int off = P.K.psd_lds;                   // the PSD blocks' area comes first
    load_part(tm.mp[0], op_mat<TL>(P, 0), P.partA, blockIdx.x, LDS, &off);
    load_part(tm.mp[1], op_mat<TL>(P, 1), P.partAt, blockIdx.x, LDS, &off);
    __syncthreads();
    tm.set_up(PT ? psd_sub_start(P.K, gridDim.x) : 0);
}

// stage_doubles: dynamic LDS of the launch (in doubles) for the CG's gathered
// vectors; an instance uses it when its n + m entries fit.
template <bool LDS>
__device__ inline void block_team_init(BlockTeamT<LDS>& tm, const Prob& P, int stage_doubles) {
    tm.mp[0] = MatPart{0, P.A.rows, 0, 0, 0, 0};
    tm.mp[1] = MatPart{0, P.At.rows, 0, 0, 0, 0};
    const bool fit = P.n + P.m <= stage_doubles;
    tm.lu = fit ? sscs_dyn_lds : nullptr;
    tm.lt = fit ? sscs_dyn_lds + P.n : nullptr;
}

// The solve kernels keep the instance descriptors (Prob, Vecs, Params) in
// LDS: every field read is then a broadcast LDS load instead of a load from a
// per-lane private copy.
struct Desc {
    Prob P;
    Vecs V;
    Params S;
};

// TV: value type of the CG operator (double, or float for mixed precision).
template <bool LDS, typename TV, bool PT>
__global__ void __launch_bounds__(kBlock) k_solve_grid(Prob P, Vecs V, Params S, Result* res,
                                                       unsigned long long* bar, int* abort_flag,
                                                       double* part, long long timeout_ticks) {
    __shared__ Shared sh;
    __shared__ Desc d;
    if (threadIdx.x == 0) {
        d.P = P;
        d.V = V;
        d.S = S;
    }
    __syncthreads();
    GridTeam<LDS, TV, PT> tm{{}, bar, abort_flag, part, 0ull, timeout_ticks, 0, 0u, 1u, 1ull};
    grid_team_init(tm, d.P);
    sscs::run_solve<TV>(tm, sh, d.P, d.V, d.S, res);
}

template <bool LDS, typename TV, bool PT>
__global__ void __launch_bounds__(kBlock) k_op_grid(Prob P, Vecs V, OpArgs a, unsigned long long* bar,
                                                    int* abort_flag, double* part, long long timeout_ticks) {
    __shared__ Shared sh;
    GridTeam<LDS, TV, PT> tm{{}, bar, abort_flag, part, 0ull, timeout_ticks, 0, 0u, 1u, 1ull};
    grid_team_init(tm, P);
    const int n = P.n, m = P.m, N = P.N;
    if (a.op == OP_LINEAR) {
        for (int j = tm.rank(); j < n; j += tm.size()) V.xw_d[j] = 0.0;
        tm.sync();
        long long it = 0;
        const double tau = linear_step<TV>(tm, sh, P, V, a.in, a.out1, V.xw_d, a.tol, a.maxit, &it);
        for (int i = tm.rank(); i < N; i += tm.size()) a.out1[i] = corrected(P, a.out1, tau, i);
        if (tm.rank() == 0 && a.scal) a.scal[0] = (double)it;
    } else if (a.op == OP_RESIDUAL) {
        for (int i = tm.rank(); i < N; i += tm.size()) V.u[i] = a.in[i];
        for (int j = tm.rank(); j < n; j += tm.size()) V.xw_u[j] = 0.0;
        tm.sync();
        long long it = 0;
        const double tau = linear_step<TV>(tm, sh, P, V, V.u, V.ut, V.xw_u, a.tol, a.maxit, &it);
        const double r2 = residual_pass(tm, sh, P, V, tau);
        for (int i = tm.rank(); i < N; i += tm.size()) {
            if (a.out1) a.out1[i] = V.ut[i];
            a.out2[i] = V.Ru[i];
        }
        if (tm.rank() == 0 && a.scal) a.scal[0] = r2;
    } else if (a.op == OP_PROJECT) {
        project_C(tm, sh, n, N, P.K,
                  [&](int i) { return (i >= n && i < n + m) ? a.in[i - n] : 0.0; },
                  [&](int i, double v) { if (i >= n && i < n + m) a.out1[i - n] = v; });
    } else if (a.op == OP_SETUP) {
        Prob Q = P;
        const int it = setup_gdelta(tm, sh, Q, V, a.out1, a.tol, a.maxit);
        if (tm.rank() == 0) {
            a.scal[0] = Q.delta;
            a.scal[1] = Q.nb;
            a.scal[2] = Q.nc;
            a.scal[3] = (double)it;
        }
    }
    tm.sync();
}

struct BatchInst {
    Prob P;
    Vecs V;
};

// Three workgroups per CU (waves_per_eu 3, up to 168 registers per lane):
// the one-workgroup engine is bound by memory latency, so resident instances
// hide latency, but at four per CU the 128-register budget made the rest of
// the solve (projections, directions, termination) spill heavily; three was
// measured fastest (two and four slower).
template <typename TV>
__global__ void __launch_bounds__(kBatchBlock) __attribute__((amdgpu_waves_per_eu(3, 3))) k_solve_batch(
    const BatchInst* __restrict__ insts, const int* __restrict__ order, int count, int nq, Params S, Result* res,
    int* queue, int stage_doubles) {
    __shared__ Shared sh;
    __shared__ Desc d;
    BlockTeam tm;
    if (threadIdx.x == 0) d.S = S;
    for (;;) {
        if (threadIdx.x == 0) {
            const int q = atomicAdd(queue, 1);
            sh.qhead = q < nq ? order[q] : count;
        }
        __syncthreads();
        const int idx = __builtin_amdgcn_readfirstlane(sh.qhead);
        __syncthreads();
        if (idx >= count) break;
        if (threadIdx.x == 0) {
            d.P = insts[idx].P;
            d.V = insts[idx].V;
        }
        __syncthreads();
        block_team_init(tm, d.P, stage_doubles);
        setup_gdelta(tm, sh, d.P, d.V, const_cast<double*>(d.P.g), d.S.setup_tol, d.S.setup_max);
        sscs::run_solve<TV>(tm, sh, d.P, d.V, d.S, res + idx);
    }
}

// Algorithm 1 for one instance small enough for a single workgroup.
template <typename TV>
__global__ void __launch_bounds__(kBatchBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) k_solve_block(Prob P, Vecs V, Params S, Result* res,
                                                             int stage_doubles) {
    __shared__ Shared sh;
    __shared__ Desc d;
    if (threadIdx.x == 0) {
        d.P = P;
        d.V = V;
        d.S = S;
    }
    __syncthreads();
    BlockTeam tm;
    block_team_init(tm, d.P, stage_doubles);
    sscs::run_solve<TV>(tm, sh, d.P, d.V, d.S, res);
}

// LDS plan of the small-instance kernel: after the CG's staging region, the
// operator (A, then A^T: values, column indices, row pointers), then groups
// of vectors, each group placed only when it fits, in this order: the
// problem's vectors (D, b, c, g), the CG's n- and m-vectors, the N-vectors of
// Algorithm 1, the quasi-Newton memory.  The host computes the plan with the
// same function, so the kernel's carving and the launch's size agree.
enum : int { SP_OP = 1, SP_PROB = 2, SP_CG = 4, SP_ITER = 8, SP_MEM = 16 };
__host__ __device__ inline int sp_align(long long b) { return (int)((b + 15) & ~15ll); }
__host__ __device__ inline long long sp_op_bytes(int rows, long long nnz) {
    return sp_align(8 * nnz + 4 * nnz + 4 * (long long)(rows + 1));
}
__host__ __device__ inline long long sp_group_bytes(int g, int n, int m, int N, int mem, bool qr) {
    switch (g) {
        case SP_PROB: return sp_align(8ll * n) * 2 + sp_align(8ll * m) + sp_align(8ll * (n + m));
        case SP_CG: return sp_align(8ll * n) * 10 + sp_align(8ll * m);
        case SP_ITER: return sp_align(8ll * N) * 9;
        case SP_MEM: return sp_align(8ll * N) * (long long)mem * (qr ? 3 : 2);
        default: return 0;
    }
}

// Algorithm 1 for one small instance in a single workgroup with its working
// set in LDS (plan `mask`, above): every pass then reads and writes LDS
// instead of waiting on the memory hierarchy.  Vectors are reached through
// the same descriptors as in global memory (generic addresses), so the engine
// code is shared; the outputs, the trace and the PSD buffers stay global.
// OPL (launched only when the plan holds the operator, the problem's vectors
// and the CG's vectors): the CG addresses those through LDS pointers.
template <bool OPL>
__global__ void __launch_bounds__(kBatchBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) k_solve_small(
    Prob P, Vecs V, Params S, Result* res, int stage_doubles, int mask) {
    __shared__ Shared sh;
    __shared__ Desc d;
    if (threadIdx.x == 0) {
        d.P = P;
        d.V = V;
        d.S = S;
    }
    __syncthreads();
    BlockTeamT<OPL> tm;
    block_team_init(tm, d.P, stage_doubles);
    const int n = P.n, m = P.m, N = P.N, mem = S.mem;
    int off = sp_align(8ll * stage_doubles);
    if constexpr (OPL) {
        const int pa[2] = {0, m}, pt[2] = {0, n};
        load_part(tm.mp[0], P.A, pa, 0, true, &off);
        load_part(tm.mp[1], P.At, pt, 0, true, &off);
    }
    char* lds = reinterpret_cast<char*>(sscs_dyn_lds);
    auto take = [&](long long cnt) {
        double* q = reinterpret_cast<double*>(lds + off);
        off += sp_align(8 * cnt);
        return q;
    };
    auto copy_in = [&](double* dst, const double* src, long long cnt) {
        for (long long i = threadIdx.x; i < cnt; i += blockDim.x) dst[i] = src[i];
    };
    Prob& Q = d.P;
    Vecs& W = d.V;
    __syncthreads();                  // every thread has read d.P / d.V before thread 0 rewires them
    if (mask & SP_PROB) {
        double* dinv = take(n); double* c = take(n); double* b = take(m); double* g = take(n + m);
        copy_in(dinv, P.dinv, n); copy_in(c, P.c, n); copy_in(b, P.b, m); copy_in(g, P.g, n + m);
        if (threadIdx.x == 0) { Q.dinv = dinv; Q.c = c; Q.b = b; Q.g = g; }
    }
    if (mask & SP_CG) {
        double* v[10];
        for (int i = 0; i < 10; ++i) v[i] = take(n);
        double* t = take(m);
        if (threadIdx.x == 0) {
            W.xw_u = v[0]; W.xw_d = v[1]; W.q_u = v[2]; W.q_d = v[3]; W.cg_b = v[4];
            W.cg_u = v[5]; W.cg_w = v[6]; W.cg_p = v[7]; W.cg_r = v[8]; W.cg_s = v[9]; W.cg_t = t;
        }
    }
    if (mask & SP_ITER) {
        double* v[9];
        for (int i = 0; i < 9; ++i) v[i] = take(N);
        if (threadIdx.x == 0) {
            W.u = v[0]; W.ut = v[1]; W.ub = v[2]; W.Ru = v[3]; W.d = v[4]; W.dt = v[5]; W.Rw = v[6];
            W.pz = v[7]; W.pxi = v[8];
        }
    }
    if (mask & SP_MEM) {
        double* z = take((long long)mem * N);
        double* y = take((long long)mem * N);
        double* qb = S.direction == DIR_AA_QR ? take((long long)mem * N) : nullptr;
        if (threadIdx.x == 0) { W.Zb = z; W.Yb = y; if (qb) W.Qb = qb; }
    }
    __syncthreads();
    sscs::run_solve<double>(tm, sh, d.P, d.V, d.S, res);
}

// ------------------------------------------------------------ direct linear step
// Dense Cholesky of the reduced system M = I + A^T A (Sec. IV-A), column-major
// and in place, by blocks of DIRECT_B: the diagonal block factored (and
// inverted) by one workgroup in LDS, the panel below it by triangular solves
// against that inverse, the trailing lower triangle updated tile by tile.

constexpr int DIRECT_B = 64;    // block order of the factorisation

// M = I + A^T A: entry (i, j) is 1[i = j] + <A e_i, A e_j>, the sorted rows i and
// j of A^T merged; one thread per entry of the lower triangle, both halves written.
__global__ void k_form_normal(const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ v,
                              int n, double* __restrict__ M) {
    const int i = blockIdx.y * blockDim.y + threadIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || j > i) return;
    int a = rp[i], ae = rp[i + 1], b = rp[j], be = rp[j + 1];
    double s = (i == j) ? 1.0 : 0.0;
    while (a < ae && b < be) {
        const int ca = ci[a], cb = ci[b];
        if (ca == cb) { s += v[a] * v[b]; ++a; ++b; }
        else if (ca < cb) ++a;
        else ++b;
    }
    M[(size_t)j * n + i] = s;
    M[(size_t)i * n + j] = s;
}

// Factors the diagonal block at k0 (order kn) in LDS, writes L_bb into M and
// L_bb^{-1} (row-major, zero-padded to DIRECT_B) into Li.  *err = 1 on a
// non-positive pivot.
__global__ void __launch_bounds__(256) k_chol_diag(double* __restrict__ M, int n, int k0, int kn,
                                                   double* __restrict__ Li, int* err) {
    __shared__ double A[DIRECT_B][DIRECT_B + 1];
    __shared__ double X[DIRECT_B][DIRECT_B + 1];
    const int t = threadIdx.x, nt = blockDim.x;
    for (int e = t; e < DIRECT_B * DIRECT_B; e += nt) {
        const int i = e / DIRECT_B, j = e % DIRECT_B;
        A[i][j] = (i < kn && j < kn) ? M[(size_t)(k0 + j) * n + (k0 + i)] : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < kn; ++k) {
        if (t == 0) {
            const double d = A[k][k];
            if (!(d > 0.0)) *err = 1;
            A[k][k] = sqrt(fmax(d, 1e-300));
        }
        __syncthreads();
        const double d = A[k][k];
        for (int i = k + 1 + t; i < kn; i += nt) A[i][k] /= d;
        __syncthreads();
        const int w = kn - k - 1;
        for (int e = t; e < w * w; e += nt) {
            const int i = k + 1 + e / w, j = k + 1 + e % w;
            if (j <= i) A[i][j] -= A[i][k] * A[j][k];
        }
        __syncthreads();
    }
    // X = L^{-1}, column c by thread c: forward substitution of L X e_c = e_c
    for (int c = t; c < DIRECT_B; c += nt) {
        for (int i = 0; i < DIRECT_B; ++i) X[i][c] = 0.0;
        if (c < kn) {
            for (int i = c; i < kn; ++i) {
                double s = (i == c) ? 1.0 : 0.0;
                for (int k = c; k < i; ++k) s -= A[i][k] * X[k][c];
                X[i][c] = s / A[i][i];
            }
        }
    }
    __syncthreads();
    for (int e = t; e < DIRECT_B * DIRECT_B; e += nt) {
        const int i = e / DIRECT_B, j = e % DIRECT_B;
        Li[e] = X[i][j];
        if (i < kn && j < kn && j <= i) M[(size_t)(k0 + j) * n + (k0 + i)] = A[i][j];
    }
}

// The panel below the diagonal block: L[i, k0 + c] = sum_k M[i, k0 + k] Li[c][k]
// for the DIRECT_B rows of this workgroup (i >= k0 + kn).
__global__ void __launch_bounds__(256) k_chol_panel(double* __restrict__ M, int n, int k0, int kn,
                                                    const double* __restrict__ Li) {
    __shared__ double R[DIRECT_B][DIRECT_B + 1];   // rows of this workgroup, panel columns
    __shared__ double I_[DIRECT_B][DIRECT_B + 1];
    const int t = threadIdx.x, nt = blockDim.x;
    const int r0 = k0 + kn + blockIdx.x * DIRECT_B;
    const int rn = min(DIRECT_B, n - r0);
    if (rn <= 0) return;
    for (int e = t; e < DIRECT_B * DIRECT_B; e += nt) {
        const int a = e % DIRECT_B, k = e / DIRECT_B;   // consecutive threads: consecutive rows
        R[a][k] = (a < rn && k < kn) ? M[(size_t)(k0 + k) * n + (r0 + a)] : 0.0;
        I_[k][a] = Li[(size_t)k * DIRECT_B + a];
    }
    __syncthreads();
    for (int e = t; e < DIRECT_B * DIRECT_B; e += nt) {
        const int a = e % DIRECT_B, c = e / DIRECT_B;
        if (a >= rn || c >= kn) continue;
        double s = 0.0;
        for (int k = 0; k <= c; ++k) s += R[a][k] * I_[c][k];
        M[(size_t)(k0 + c) * n + (r0 + a)] = s;
    }
}

// Trailing update of the lower triangle below and right of the panel:
// M[i, j] -= sum_k L[i, k0 + k] L[j, k0 + k], one DIRECT_B x DIRECT_B tile per
// workgroup (tiles above the diagonal return at once).
__global__ void __launch_bounds__(256) k_chol_update(double* __restrict__ M, int n, int k0, int kn) {
    const int ti = blockIdx.y, tj = blockIdx.x;
    if (tj > ti) return;
    __shared__ double Pi[DIRECT_B][DIRECT_B + 1];
    __shared__ double Pj[DIRECT_B][DIRECT_B + 1];
    const int base = k0 + kn;
    const int i0 = base + ti * DIRECT_B, j0 = base + tj * DIRECT_B;
    const int in_ = min(DIRECT_B, n - i0), jn = min(DIRECT_B, n - j0);
    if (in_ <= 0 || jn <= 0) return;
    const int t = threadIdx.x, nt = blockDim.x;
    for (int e = t; e < DIRECT_B * DIRECT_B; e += nt) {
        const int a = e % DIRECT_B, k = e / DIRECT_B;
        Pi[a][k] = (a < in_ && k < kn) ? M[(size_t)(k0 + k) * n + (i0 + a)] : 0.0;
        Pj[a][k] = (a < jn && k < kn) ? M[(size_t)(k0 + k) * n + (j0 + a)] : 0.0;
    }
    __syncthreads();
    for (int e = t; e < DIRECT_B * DIRECT_B; e += nt) {
        const int a = e % DIRECT_B, b = e / DIRECT_B;      // row i0 + a, column j0 + b
        if (a >= in_ || b >= jn) continue;
        if (ti == tj && b > a) continue;
        double s = 0.0;
        for (int k = 0; k < kn; ++k) s += Pi[a][k] * Pj[b][k];
        M[(size_t)(j0 + b) * n + (i0 + a)] -= s;
    }
}

// M^{-1} = L^{-T} L^{-1} from the factor, by substitution with the n columns of
// the identity as right-hand sides (W, column-major, starts as I): forward,
// for each block b, the rows of b are multiplied by L_bb^{-1} and the rows
// below lose L[rows, b] times them; backward the same with L^T from the last
// block up.  Each step is one launch over 64 x 64 tiles of W.

// W[k0 .. k0+kn, c0 .. c0+64] = Li (or Li^T) times itself, one column tile per workgroup.
__global__ void __launch_bounds__(256) k_inv_apply(double* __restrict__ W, int n, int k0, int kn,
                                                   const double* __restrict__ Li, int transpose) {
    __shared__ double B[DIRECT_B][DIRECT_B + 1];
    __shared__ double I_[DIRECT_B][DIRECT_B + 1];
    const int c0 = blockIdx.x * DIRECT_B;
    const int cn = min(DIRECT_B, n - c0);
    const int t = threadIdx.x, nt = blockDim.x;
    for (int e = t; e < DIRECT_B * DIRECT_B; e += nt) {
        const int a = e % DIRECT_B, c = e / DIRECT_B;          // row k0 + a, column c0 + c
        B[a][c] = (a < kn && c < cn) ? W[(size_t)(c0 + c) * n + (k0 + a)] : 0.0;
        const int r = e / DIRECT_B, q = e % DIRECT_B;
        I_[r][q] = transpose ? Li[(size_t)q * DIRECT_B + r] : Li[(size_t)r * DIRECT_B + q];
    }
    __syncthreads();
    for (int e = t; e < DIRECT_B * DIRECT_B; e += nt) {
        const int a = e % DIRECT_B, c = e / DIRECT_B;
        if (a >= kn || c >= cn) continue;
        double s = 0.0;
        for (int k = 0; k < kn; ++k) s += I_[a][k] * B[k][c];
        W[(size_t)(c0 + c) * n + (k0 + a)] = s;
    }
}

// W[i, c] -= sum_k F[i, k0 + k] W[k0 + k, c] for the row tile of this
// workgroup (blockIdx.y) and column tile (blockIdx.x); F = L (forward, rows
// below the block) or L^T (backward, rows above it), L column-major in Lc.
__global__ void __launch_bounds__(256) k_inv_update(double* __restrict__ W, const double* __restrict__ Lc, int n,
                                                    int k0, int kn, int forward) {
    __shared__ double F[DIRECT_B][DIRECT_B + 1];
    __shared__ double B[DIRECT_B][DIRECT_B + 1];
    const int base = forward ? k0 + kn : 0;
    const int lim = forward ? n : k0;
    const int i0 = base + blockIdx.y * DIRECT_B, c0 = blockIdx.x * DIRECT_B;
    const int in_ = min(DIRECT_B, lim - i0), cn = min(DIRECT_B, n - c0);
    if (in_ <= 0 || cn <= 0) return;
    const int t = threadIdx.x, nt = blockDim.x;
    for (int e = t; e < DIRECT_B * DIRECT_B; e += nt) {
        const int a = e % DIRECT_B, k = e / DIRECT_B;
        double f = 0.0;
        if (a < in_ && k < kn)
            f = forward ? Lc[(size_t)(k0 + k) * n + (i0 + a)]      // L[i, k0 + k]
                        : Lc[(size_t)(i0 + a) * n + (k0 + k)];     // L^T[i, k0 + k] = L[k0 + k, i]
        F[a][k] = f;
        B[a][k] = (a < kn && k < cn) ? W[(size_t)(c0 + k) * n + (k0 + a)] : 0.0;   // B[row k0 + a][col c0 + k]
    }
    __syncthreads();
    for (int e = t; e < DIRECT_B * DIRECT_B; e += nt) {
        const int a = e % DIRECT_B, c = e / DIRECT_B;
        if (a >= in_ || c >= cn) continue;
        double s = 0.0;
        for (int k = 0; k < kn; ++k) s += F[a][k] * B[k][c];
        W[(size_t)(c0 + c) * n + (i0 + a)] -= s;
    }
}

__global__ void k_identity(double* __restrict__ W, int n) {
    const long long nn = (long long)n * n;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn; e += (long long)gridDim.x * blockDim.x)
        W[e] = (e / n == e % n) ? 1.0 : 0.0;
}

__global__ void k_to_f32(const double* __restrict__ a, long long n, float* __restrict__ b) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

// Stand-alone SpMV for operators that stay in the caches: the CG's
// row-segmented scheme over a flat grid (seg lanes per row, chosen from the
// mean row length).
struct FlatTeam {
    __device__ int rank() const { return blockIdx.x * blockDim.x + threadIdx.x; }
    __device__ int size() const { return gridDim.x * blockDim.x; }
};

__global__ void k_spmv(Csr<double> M, const double* __restrict__ x, double* __restrict__ y) {
    FlatTeam tm;
    spmv_gather<1>(tm, M, [&](int c) { return x[c]; }, [&](int r, double s) { y[r] = s; });
}

// Stand-alone SpMV, column-panel form, for operators that stream from HBM:
// the input vector is cut into panels of at most kPanelCols entries, and a
// workgroup of 1024 threads (one per CU: the panel fills the LDS) stages its
// panel of x in LDS once and then runs the row-segmented product over its
// share of the rows, gathering from LDS instead of the cache hierarchy
// (measured: with x in L2 each 8-byte gather costs a cache-line transfer and
// caps the product far below the streaming rate of the operator).  Work item
// i is (panel p, share c, shares C) in items[3 i .. 3 i + 2]: the C workgroups
// of panel p interleave its rows segment by segment (at any moment the grid
// streams through one region of the operator).  The operator is given panel
// by panel: rows r of panel p are [rp[p rows + r], rp[p rows + r + 1]) of
// (ci, v), column indices relative to the panel (one panel: the CSR itself).
// With one panel the sums go to y; with several, row r's partial sum of panel
// p goes to part[p rows + r], summed over the panels in order by k_panel_sum.
// With R = 1 a segment walks its rows one at a time, the next row's pointers
// loaded before the current row's entries, and takes a row's entries U steps
// at a time (each lane's U loads in flight together, at constant offsets from
// one address), then the at most U - 1 steps left over as one more batch
// whose loads past the row's end read its last entry (and are not added);
// the additions are in the same order as one step at a time.  Measured on
// 5e6 x 2e4 operators: 20 entries per row, S = 4, U = 5 (a row in one batch)
// 249 us against 306-321 us for S = 8 one step at a time (clamping every
// batch's loads instead, 302 us); rows of 20.4 entries on average
// (binomial), the left-over steps as a batch 316 us, one by one 346 us.
// With R > 1 a segment takes R of its rows at a time: each step loads the
// next entry of all of them (at index min(k, nnz - 1) for a row already done),
// then adds those of the rows still going (the same additions in the same
// order as one row at a time).
constexpr int kPanelCols = 20480;      // 160 KB of FP64 entries per panel
constexpr int kPanelThreads = 1024;
template <int S, int U, int R>
__global__ void __launch_bounds__(kPanelThreads) k_spmv_panel(const int* __restrict__ rp, const int* __restrict__ ci,
                                                              const double* __restrict__ v, int rows, int cols,
                                                              const int* __restrict__ items, int nitems, int P, int pc,
                                                              const double* __restrict__ x, double* __restrict__ y,
                                                              double* __restrict__ part, long long nnz) {
    double* xs = sscs_dyn_lds;
    int cur = -1;
    const int seg = threadIdx.x / S, nseg = blockDim.x / S, ls = threadIdx.x & (S - 1);
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int p = items[3 * it], c = items[3 * it + 1], C = items[3 * it + 2];
        if (p != cur) {
            // stage panel p of x: kStage loads per thread in flight before
            // their stores (loads past the panel's end read its last entry)
            constexpr int kStage = 8;
            __syncthreads();
            const int c0 = p * pc, len = min(pc, cols - c0);
            for (int i0 = threadIdx.x; i0 < len; i0 += kStage * blockDim.x) {
                double t[kStage];
#pragma unroll
                for (int u = 0; u < kStage; ++u) t[u] = x[c0 + min(i0 + u * (int)blockDim.x, len - 1)];
#pragma unroll
                for (int u = 0; u < kStage; ++u)
                    if (i0 + u * (int)blockDim.x < len) xs[i0 + u * blockDim.x] = t[u];
            }
            __syncthreads();
            cur = p;
        }
        const int* prp = rp + (size_t)p * rows;
        if constexpr (R == 1) {
            const int step = C * nseg;
            int r = c * nseg + seg, kb = 0, ke = 0;
            if (r < rows) {
                kb = prp[r];
                ke = prp[r + 1];
            }
            for (; r < rows; r += step) {
                int kbn = 0, ken = 0;                // the next row's pointers, loaded ahead
                if (r + step < rows) {
                    kbn = prp[r + step];
                    ken = prp[r + step + 1];
                }
                double acc = 0.0;
                int k = kb + ls;
                for (; k < ke - (U - 1) * S; k += U * S) {   // U steps whose loads are in flight together
                    double vu[U];
                    int cu[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        vu[u] = v[k + u * S];
                        cu[u] = ci[k + u * S];
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) acc += vu[u] * xs[cu[u]];
                }
                if constexpr (U > 1) {
                    if (k < ke) {                    // at most U - 1 steps left: one batch as well
                        const int kl = ke - 1;       // loads past the end read the row's last entry
                        double vu[U - 1];
                        int cu[U - 1];
#pragma unroll
                        for (int u = 0; u < U - 1; ++u) {
                            const int kk = min(k + u * S, kl);
                            vu[u] = v[kk];
                            cu[u] = ci[kk];
                        }
#pragma unroll
                        for (int u = 0; u < U - 1; ++u) {
                            const double t = vu[u] * xs[cu[u]];
                            if (k + u * S < ke) acc += t;
                        }
                    }
                }
#pragma unroll
                for (int o = S >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, WAVE);
                if (ls == 0) {
                    if (P == 1) y[r] = acc;
                    else part[(size_t)p * rows + r] = acc;
                }
                kb = kbn;
                ke = ken;
            }
            continue;
        }
        const long long last = nnz - 1;
        for (int r0 = c * nseg + seg; r0 < rows; r0 += R * C * nseg) {
            long long kb[R], ke[R];
            double acc[R];
            bool more = false;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int r = r0 + q * C * nseg;
                kb[q] = r < rows ? (long long)prp[r] + ls : 0;
                ke[q] = r < rows ? prp[r + 1] : 0;
                acc[q] = 0.0;
                more = more || kb[q] < ke[q];
            }
            while (more) {                         // some row still going, so nnz > 0
                double vq[R];
                int cq[R];
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const long long k = kb[q] < last ? kb[q] : last;
                    vq[q] = v[k];
                    cq[q] = ci[k];
                }
                more = false;
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const double xv = xs[cq[q]];
                    if (kb[q] < ke[q]) {
                        acc[q] += vq[q] * xv;
                        kb[q] += S;
                        more = more || kb[q] < ke[q];
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < R; ++q) {
                double a = acc[q];
#pragma unroll
                for (int o = S >> 1; o > 0; o >>= 1) a += __shfl_xor(a, o, WAVE);
                const int r = r0 + q * C * nseg;
                if (ls == 0 && r < rows) {
                    if (P == 1) y[r] = a;
                    else part[(size_t)p * rows + r] = a;
                }
            }
        }
    }
}

// y[r] = sum over panels p in order of part[p rows + r].  A thread loads kB
// panels' partials before adding them (the same additions in the same order),
// so its loads are in flight together instead of one round trip per panel;
// the last, partial batch loads the row's last partial in place of those past
// the end (not added).  Launched with small workgroups, so that a few
// thousand rows still spread over every CU.  Measured on A^T of the 1e8-
// nonzero operator (245 panels, 20 000 rows): 26.7 us with batches of eight,
// branch-guarded, in 79 workgroups of 256.
constexpr int kPanelSumThreads = 64;
__global__ void __launch_bounds__(kPanelSumThreads) k_panel_sum(const double* __restrict__ part, int P, int rows,
                                                                 double* __restrict__ y) {
    constexpr int kB = 32;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x) {
        double a = 0.0;
        int p0 = 0;
        for (; p0 + kB <= P; p0 += kB) {
            double v[kB];
#pragma unroll
            for (int q = 0; q < kB; ++q) v[q] = part[(size_t)(p0 + q) * rows + r];
#pragma unroll
            for (int q = 0; q < kB; ++q) a += v[q];
        }
        if (p0 < P) {
            double v[kB];
#pragma unroll
            for (int q = 0; q < kB; ++q) v[q] = part[(size_t)min(p0 + q, P - 1) * rows + r];
#pragma unroll
            for (int q = 0; q < kB; ++q)
                if (p0 + q < P) a += v[q];
        }
        y[r] = a;
    }
}

// First entry of row r with column >= key (columns sorted).
__device__ inline int row_lower(const int* __restrict__ rp, const int* __restrict__ ci, int r, int key) {
    int lo = rp[r], hi = rp[r + 1];
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ci[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Panel-major copy of a CSR matrix with sorted columns: (1) the entry count of
// every (panel p, row r) into len[p rows + r]; (2) an exclusive scan of len
// (k_scan) gives the panel-major row pointers; (3) every (p, r) segment is
// copied with panel-relative columns.
__global__ void k_panel_lens(const int* __restrict__ rp, const int* __restrict__ ci, int rows, int P, int pc,
                             int* __restrict__ len) {
    const long long total = (long long)rows * P;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
         t += (long long)gridDim.x * blockDim.x) {
        const int p = (int)(t / rows), r = (int)(t % rows);
        len[t] = row_lower(rp, ci, r, (p + 1) * pc) - row_lower(rp, ci, r, p * pc);
    }
}

__global__ void k_panel_scatter(const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ v,
                                int rows, int P, int pc, const int* __restrict__ off, int* __restrict__ pci,
                                double* __restrict__ pv) {
    const long long total = (long long)rows * P;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
         t += (long long)gridDim.x * blockDim.x) {
        const int p = (int)(t / rows), r = (int)(t % rows);
        const int key = p * pc;
        const int lo = row_lower(rp, ci, r, key);
        const int o = off[t], cnt = off[t + 1] - o;
        for (int e = 0; e < cnt; ++e) {
            pci[o + e] = ci[lo + e] - key;
            pv[o + e] = v[lo + e];
        }
    }
}

// --- setup: CSR transpose ------------------------------------------------------

__global__ void k_count_cols(const int* __restrict__ ci, long long nnz, int* __restrict__ cnt) {
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nnz; k += (long long)gridDim.x * blockDim.x)
        atomicAdd(cnt + ci[k], 1);
}

// Exclusive scan of cnt[0..len) into out[0..len]; one workgroup, each thread a
// contiguous chunk, then a scan of the chunk totals.
__global__ void __launch_bounds__(1024) k_scan(const int* __restrict__ cnt, int len, int* __restrict__ out) {
    __shared__ int tot[1024];
    const int t = threadIdx.x, nt = blockDim.x;
    const int chunk = (len + nt - 1) / nt;
    const int b0 = min(len, t * chunk), b1 = min(len, b0 + chunk);
    int s = 0;
    for (int i = b0; i < b1; ++i) s += cnt[i];
    tot[t] = s;
    __syncthreads();
    if (t == 0) {
        int run = 0;
        for (int i = 0; i < nt; ++i) { const int v = tot[i]; tot[i] = run; run += v; }
        out[len] = run;
    }
    __syncthreads();
    int run = tot[t];
    for (int i = b0; i < b1; ++i) { out[i] = run; run += cnt[i]; }
}

__global__ void k_scatter_t(const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ v,
                            int rows, const int* __restrict__ trp, int* __restrict__ fill,
                            int* __restrict__ tci, double* __restrict__ tv) {
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x)
        for (int k = rp[r]; k < rp[r + 1]; ++k) {
            const int j = ci[k];
            const int pos = trp[j] + atomicAdd(fill + j, 1);
            tci[pos] = r;
            tv[pos] = v[k];
        }
}

// Shellsort gaps of Ciura (2001, "Best increments for the average case of
// Shellsort"), extended by the factor 2.25, up to the int range.
__constant__ int kShellGaps[26] = {1,       4,        10,       23,        57,        132,       301,
                                   701,     1750,     3937,     8858,      19930,     44842,     100894,
                                   227011,  510774,   1149241,  2585792,   5818032,   13090572,  29453787,
                                   66271020, 149109795, 335497038, 754868335, 1698453753};

// Sorts each row of the transpose by column (Shellsort, one thread per row:
// the scatter leaves a long column of A, thousands of entries, in arbitrary
// order, where insertion sort's quadratic count of dependent moves took over a
// second), so that its order, and every sum over it, is
// deterministic: the keys of a row are distinct, so the sorted order is
// unique.  Then the Jacobi diagonal 1 / (1 + ||row||^2).
__global__ void k_sort_rows(const int* __restrict__ trp, int rows, int* __restrict__ tci, double* __restrict__ tv,
                            double* __restrict__ dinv) {
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x) {
        const int k0 = trp[r], k1 = trp[r + 1];
        const int len = k1 - k0;
        int gi = 0;
        while (gi < 25 && kShellGaps[gi + 1] < len) ++gi;
        for (; gi >= 0; --gi) {
            const int g = kShellGaps[gi];
            for (int k = k0 + g; k < k1; ++k) {
                const int key = tci[k];
                const double val = tv[k];
                int j = k - g;
                while (j >= k0 && tci[j] > key) {
                    tci[j + g] = tci[j];
                    tv[j + g] = tv[j];
                    j -= g;
                }
                tci[j + g] = key;
                tv[j + g] = val;
            }
        }
        double s = 0.0;
        for (int k = k0; k < k1; ++k) s += tv[k] * tv[k];
        dinv[r] = 1.0 / (1.0 + s);
    }
}

// ------------------------------------------------------------------ host side

namespace {

thread_local std::string g_last_hip;
thread_local const char* g_unsupported = nullptr;   // reason of the last SSCS_E_UNSUPPORTED, if given

#define HIP_TRY(expr)                                                      \
    do {                                                                   \
        hipError_t _e = (expr);                                            \
        if (_e != hipSuccess) {                                            \
            g_last_hip = std::string(#expr) + ": " + hipGetErrorString(_e); \
            return SSCS_E_HIP;                                             \
        }                                                                  \
    } while (0)

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// LDS (in doubles) the one-workgroup kernels stage the CG's gathered
// vectors in, for an instance with `entries` = n + m; 0 when they do not fit
// (the CG then gathers from global memory).  The dynamic-LDS limit is raised
// on every instantiation that takes the staging buffer.
int stage_doubles(long long entries) {
    if (entries <= 0 || entries > kStageMax) return 0;
    static const bool attr = [] {
        const int bytes = kStageMax * (int)sizeof(double);
        const void* fns[] = {(const void*)k_solve_batch<double>, (const void*)k_solve_block<double>,
                             (const void*)k_solve_block<float>};
        bool ok = true;
        for (const void* f : fns)
            ok = ok && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
        return ok;
    }();
    return attr ? (int)entries : 0;
}

// Dynamic LDS the small-instance kernel may take (its static LDS and a margin
// subtracted from the device's per-workgroup limit); the limit is raised on
// both instantiations once.
int small_lds_budget() {
    static const int budget = [] {
        int dev = 0, lds_max = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 0;
        if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
        long long stat = 0;
        for (const void* f : {(const void*)k_solve_small<true>, (const void*)k_solve_small<false>}) {
            hipFuncAttributes fa{};
            if (hipFuncGetAttributes(&fa, f) != hipSuccess) return 0;
            stat = std::max<long long>(stat, (long long)fa.sharedSizeBytes);
        }
        const int b = (int)std::max<long long>(0, (long long)lds_max - stat - 256);
        for (const void* f : {(const void*)k_solve_small<true>, (const void*)k_solve_small<false>})
            if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, b) != hipSuccess) return 0;
        return b;
    }();
    return budget;
}

// Lanes per row of the row-segmented SpMV (the mean-row-length rule): the
// smallest power of two that gives each lane about `div` nonzeros of a
// mean-length row (more rows in flight per wavefront, several independent
// loads per lane); sscs_batch_autotune can replace it per size class.
int pow2_seg(double avg) {
    const double div = 4.0;
    int s = 1;
    while (s < 64 && s < avg / div) s <<= 1;
    return s;
}

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

// Everything one instance needs on the device.
struct Inst {
    int n = 0, m = 0, N = 0;
    long long nnz = 0;
    int *A_rp = nullptr, *A_ci = nullptr, *At_rp = nullptr, *At_ci = nullptr;
    double *A_v = nullptr, *At_v = nullptr;
    float *A_vf = nullptr, *At_vf = nullptr;   // FP32 copies (mixed precision)
    int *A_long = nullptr, *At_long = nullptr;   // rows summed by a whole workgroup
    int nlongA = 0, nlongAt = 0, lthrA = 1 << 30, lthrAt = 1 << 30;
    bool mixed = false;
    double *b = nullptr, *c = nullptr, *dinv = nullptr, *g = nullptr;
    double delta = 1.0, nb = 0.0, nc = 0.0;
    int *qoff = nullptr, *sord = nullptr, *soff = nullptr;
    int segA = 1, segAt = 1;
    ConeDev K{};
    bool owns_A = true;
    std::vector<int> h_rpA, h_rpAt;        // host row pointers (partitioning)
    int *partA = nullptr, *partAt = nullptr;
    int lds_bytes = 0;                     // dynamic LDS of the grid kernels
    bool op_lds = false;                   // the grid kernels hold their operator rows in LDS
    int psd_small = 0;                     // largest PSD order projected one block per workgroup
    double *Minv = nullptr;                // direct linear step: (I + A^T A)^{-1}, n x n
};

// The small kernel's plan for an FP64 instance: mask of what goes to LDS (see
// k_solve_small) and the dynamic LDS bytes; mask 0 when the CG's staging
// region itself does not fit.
int small_plan(const Inst& I, const sscs_settings& st, int* bytes) {
    *bytes = 0;
    const long long stage = I.n + (long long)I.m;
    const int budget = small_lds_budget();
    if (I.mixed || stage > kStageMax || budget <= 0) return 0;
    long long off = sp_align(8 * stage);
    if (off > budget) return 0;
    int mask = 0;
    const long long op = sp_op_bytes(I.m, I.nnz) + sp_op_bytes(I.n, I.nnz);
    if (off + op <= budget) { off += op; mask |= SP_OP; }
    for (int g : {(int)SP_PROB, (int)SP_CG, (int)SP_ITER, (int)SP_MEM}) {
        const long long gb = sp_group_bytes(g, I.n, I.m, I.N, st.mem, st.direction == SSCS_DIR_AA_QR);
        if (off + gb <= budget) { off += gb; mask |= g; }
    }
    *bytes = (int)off;
    return mask;
}

// A single instance runs on the small kernel (one workgroup, working set in
// LDS) when its operator, problem vectors, CG vectors and iterates all fit.
bool small_fits(const Inst& I, const sscs_settings& st) {
    int bytes = 0;
    const int need = SP_OP | SP_PROB | SP_CG | SP_ITER;
    return (small_plan(I, st, &bytes) & need) == need;
}

// check_csr = false skips the walk over A (an instance that shares instance
// 0's arrays, already checked).
int validate(const sscs_data* d, const sscs_cone* k, bool check_csr = true) {
    if (!d || !k) return SSCS_E_INVALID;
    if (d->m < 1 || d->n < 1 || d->nnz < 0) return SSCS_E_INVALID;
    if (!d->rowptr || (d->nnz > 0 && (!d->colind || !d->val)) || !d->b || !d->c) return SSCS_E_INVALID;
    if (d->nnz >= (1ll << 31)) return SSCS_E_UNSUPPORTED;
    if (d->rowptr[0] != 0 || d->rowptr[d->m] != d->nnz) return SSCS_E_INVALID;
    for (int i = 0; check_csr && i < d->m; ++i) {
        if (d->rowptr[i + 1] < d->rowptr[i]) return SSCS_E_INVALID;
        for (int kk = d->rowptr[i]; kk < d->rowptr[i + 1]; ++kk) {
            const int j = d->colind[kk];
            if (j < 0 || j >= d->n) return SSCS_E_INVALID;
            if (kk > d->rowptr[i] && j <= d->colind[kk - 1]) return SSCS_E_INVALID;
        }
    }
    if (k->z < 0 || k->l < 0 || k->nq < 0 || k->ns < 0 || k->ep < 0) return SSCS_E_INVALID;
    if ((k->nq > 0 && !k->q) || (k->ns > 0 && !k->s)) return SSCS_E_INVALID;
    long long rows = (long long)k->z + k->l + 3ll * k->ep;
    for (int i = 0; i < k->nq; ++i) {
        if (k->q[i] < 1) return SSCS_E_INVALID;
        rows += k->q[i];
    }
    for (int i = 0; i < k->ns; ++i) {
        if (k->s[i] < 1) return SSCS_E_INVALID;
        if (k->s[i] > 1023) return SSCS_E_UNSUPPORTED;
        rows += (long long)k->s[i] * (k->s[i] + 1) / 2;
    }
    if (rows != d->m) return SSCS_E_INVALID;
    return SSCS_OK;
}

int validate_settings(const sscs_settings* st) {
    if (!st) return SSCS_E_INVALID;
    if (!(st->eps > 0)) return SSCS_E_INVALID;
    if (st->direction < 0 || st->direction > 5) return SSCS_E_INVALID;
    if (st->mem < 1 || st->mem > MEMMAX) return SSCS_E_INVALID;
    if (st->ls_max < 0 || st->max_iters < 0 || st->cg_max < 0) return SSCS_E_INVALID;
    if (!(st->lambda > 0 && st->lambda < 2)) return SSCS_E_INVALID;
    if (!(st->sigma > 0 && st->sigma < 1)) return SSCS_E_INVALID;
    if (st->c0 < 0 || st->c1 < 0 || st->q < 0 || st->q >= 1) return SSCS_E_INVALID;
    if (!(st->thetabar > 0 && st->thetabar < 1)) return SSCS_E_INVALID;
    if (!(st->cg_tol > 0) || !(st->cg_adapt >= 0)) return SSCS_E_INVALID;
    if (st->cg_d_match != 0 && st->cg_d_match != 1) return SSCS_E_INVALID;
    if (st->precision != SSCS_PREC_FP64 && st->precision != SSCS_PREC_MIXED) return SSCS_E_INVALID;
    if (st->check_every < 0 || st->workgroups < 0) return SSCS_E_INVALID;
    if (st->linsys != SSCS_LINSYS_CG && st->linsys != SSCS_LINSYS_DIRECT) return SSCS_E_INVALID;
    return SSCS_OK;
}

Params make_params(const sscs_settings& st, double ticks_per_s) {
    Params p{};
    p.eps = st.eps;
    p.c0 = st.c0;
    p.c1 = st.c1;
    p.q = st.q;
    p.sigma = st.sigma;
    p.lam = st.lambda;
    p.thetabar = st.thetabar;
    p.aa_reg = st.aa_reg;
    p.cg_tol = st.cg_tol;
    p.cg_adapt = st.cg_adapt;
    p.cg_d_match = st.cg_d_match;
    p.direction = st.direction;
    p.mem = st.mem;
    p.ls_max = st.ls_max;
    p.cg_max = st.cg_max;
    p.check_every = std::max(1, st.check_every);
    p.max_iters = st.max_iters;
    p.max_ticks = st.max_time_s > 0 ? (long long)(st.max_time_s * ticks_per_s) : 0;
    p.setup_tol = std::min(1e-14, st.cg_tol);
    p.setup_max = std::max(st.cg_max, 1000);
    return p;
}

// Cone layout tables (host) -> device, offsets relative to the start of y.
struct ConeHost {
    std::vector<int> qoff, sord, soff;
    int z = 0, l = 0, ep = 0, soc0 = 0, psd0 = 0, exp0 = 0, kmax = 0;
};

ConeHost cone_host(const sscs_cone* k) {
    ConeHost h;
    h.z = k->z;
    h.l = k->l;
    h.ep = k->ep;
    h.soc0 = k->z + k->l;
    h.qoff.push_back(0);
    for (int i = 0; i < k->nq; ++i) h.qoff.push_back(h.qoff.back() + k->q[i]);
    h.psd0 = h.soc0 + h.qoff.back();
    h.soff.push_back(0);
    for (int i = 0; i < k->ns; ++i) {
        h.sord.push_back(k->s[i]);
        h.soff.push_back(h.soff.back() + k->s[i] * (k->s[i] + 1) / 2);
        h.kmax = std::max(h.kmax, k->s[i]);
    }
    h.exp0 = h.psd0 + h.soff.back();
    return h;
}

template <typename T>
int dmalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) {
        g_last_hip = std::string("hipMalloc: ") + hipGetErrorString(e);
        return SSCS_E_NOMEM;
    }
    return SSCS_OK;
}

#define TRY(expr)                    \
    do {                             \
        int _r = (expr);             \
        if (_r != SSCS_OK) return _r; \
    } while (0)

// Uploads A (unless shared), b, c and the cone tables; builds A^T and dinv.
int upload_instance(Inst& I, const sscs_data* d, const sscs_cone* k, hipStream_t s, const Inst* share,
                    bool mixed) {
    I.mixed = mixed;
    I.m = d->m;
    I.n = d->n;
    I.N = d->n + d->m + 1;
    I.nnz = d->nnz;
    const size_t nnz = (size_t)d->nnz;
    if (share) {
        I.A_rp = share->A_rp; I.A_ci = share->A_ci; I.A_v = share->A_v;
        I.At_rp = share->At_rp; I.At_ci = share->At_ci; I.At_v = share->At_v;
        I.A_vf = share->A_vf; I.At_vf = share->At_vf;
        I.A_long = share->A_long; I.At_long = share->At_long;
        I.nlongA = share->nlongA; I.nlongAt = share->nlongAt;
        I.lthrA = share->lthrA; I.lthrAt = share->lthrAt;
        I.h_rpA = share->h_rpA; I.h_rpAt = share->h_rpAt;
        I.dinv = share->dinv;
        I.owns_A = false;
    } else {
        TRY(dmalloc(&I.A_rp, I.m + 1));
        TRY(dmalloc(&I.A_ci, nnz));
        TRY(dmalloc(&I.A_v, nnz));
        TRY(dmalloc(&I.At_rp, I.n + 1));
        TRY(dmalloc(&I.At_ci, nnz));
        TRY(dmalloc(&I.At_v, nnz));
        TRY(dmalloc(&I.dinv, I.n));
        HIP_TRY(hipMemcpyAsync(I.A_rp, d->rowptr, (I.m + 1) * sizeof(int), hipMemcpyHostToDevice, s));
        if (nnz) {
            HIP_TRY(hipMemcpyAsync(I.A_ci, d->colind, nnz * sizeof(int), hipMemcpyHostToDevice, s));
            HIP_TRY(hipMemcpyAsync(I.A_v, d->val, nnz * sizeof(double), hipMemcpyHostToDevice, s));
        }
        int* cnt = nullptr;
        TRY(dmalloc(&cnt, I.n));
        HIP_TRY(hipMemsetAsync(cnt, 0, I.n * sizeof(int), s));
        if (nnz) k_count_cols<<<std::min<long long>(4096, (nnz + 255) / 256), 256, 0, s>>>(I.A_ci, (long long)nnz, cnt);
        k_scan<<<1, 1024, 0, s>>>(cnt, I.n, I.At_rp);
        HIP_TRY(hipMemsetAsync(cnt, 0, I.n * sizeof(int), s));
        k_scatter_t<<<std::min(4096, (I.m + 255) / 256), 256, 0, s>>>(I.A_rp, I.A_ci, I.A_v, I.m, I.At_rp, cnt,
                                                                     I.At_ci, I.At_v);
        k_sort_rows<<<std::min(4096, (I.n + 255) / 256), 256, 0, s>>>(I.At_rp, I.n, I.At_ci, I.At_v, I.dinv);
        if (mixed) {
            TRY(dmalloc(&I.A_vf, nnz));
            TRY(dmalloc(&I.At_vf, nnz));
            const int gb = (int)std::min<long long>(4096, ((long long)nnz + 255) / 256 + 1);
            k_to_f32<<<gb, 256, 0, s>>>(I.A_v, (long long)nnz, I.A_vf);
            k_to_f32<<<gb, 256, 0, s>>>(I.At_v, (long long)nnz, I.At_vf);
        }
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(s));
        hipFree(cnt);
        I.h_rpA.assign(d->rowptr, d->rowptr + I.m + 1);
        I.h_rpAt.resize(I.n + 1);
        HIP_TRY(hipMemcpy(I.h_rpAt.data(), I.At_rp, (I.n + 1) * sizeof(int), hipMemcpyDeviceToHost));
    }
    I.segA = pow2_seg((double)d->nnz / std::max(1, I.m));
    I.segAt = pow2_seg((double)d->nnz / std::max(1, I.n));
    if (!share) {
        // rows longer than 64 strides of their segment go to a whole workgroup
        auto longs = [&](const std::vector<int>& rp, int rows, int seg, int** dst, int* cnt, int* thr) -> int {
            *thr = 64 * seg;
            std::vector<int> lr;
            for (int r = 0; r < rows; ++r)
                if (rp[r + 1] - rp[r] > *thr) lr.push_back(r);
            *cnt = (int)lr.size();
            if (lr.empty()) return SSCS_OK;
            TRY(dmalloc(dst, lr.size()));
            HIP_TRY(hipMemcpy(*dst, lr.data(), lr.size() * sizeof(int), hipMemcpyHostToDevice));
            return SSCS_OK;
        };
        TRY(longs(I.h_rpA, I.m, I.segA, &I.A_long, &I.nlongA, &I.lthrA));
        TRY(longs(I.h_rpAt, I.n, I.segAt, &I.At_long, &I.nlongAt, &I.lthrAt));
    }
    TRY(dmalloc(&I.b, I.m));
    TRY(dmalloc(&I.c, I.n));
    TRY(dmalloc(&I.g, I.n + I.m));
    HIP_TRY(hipMemcpyAsync(I.b, d->b, I.m * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(I.c, d->c, I.n * sizeof(double), hipMemcpyHostToDevice, s));
    ConeHost h = cone_host(k);
    TRY(dmalloc(&I.qoff, h.qoff.size()));
    TRY(dmalloc(&I.sord, std::max<size_t>(1, h.sord.size())));
    TRY(dmalloc(&I.soff, h.soff.size()));
    HIP_TRY(hipMemcpyAsync(I.qoff, h.qoff.data(), h.qoff.size() * sizeof(int), hipMemcpyHostToDevice, s));
    if (!h.sord.empty())
        HIP_TRY(hipMemcpyAsync(I.sord, h.sord.data(), h.sord.size() * sizeof(int), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(I.soff, h.soff.data(), h.soff.size() * sizeof(int), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    I.K.z = h.z; I.K.l = h.l; I.K.nq = (int)h.qoff.size() - 1; I.K.qoff = I.qoff;
    I.K.ns = (int)h.sord.size(); I.K.sord = I.sord; I.K.soff = I.soff; I.K.ep = h.ep;
    I.K.soc0 = h.soc0; I.K.psd0 = h.psd0; I.K.exp0 = h.exp0;
    I.K.psd_scratch = nullptr;
    I.K.psd_kmax = h.kmax;
    I.psd_small = 0;
    for (int o : h.sord) if (o <= kPsdTeamOrder) I.psd_small = std::max(I.psd_small, o);
    I.K.psd_vecs = nullptr;
    I.K.psd_warm = nullptr;
    I.K.psd_team = nullptr;
    return SSCS_OK;
}

void free_instance(Inst& I) {
    if (I.owns_A) {
        hipFree(I.A_rp); hipFree(I.A_ci); hipFree(I.A_v);
        hipFree(I.At_rp); hipFree(I.At_ci); hipFree(I.At_v); hipFree(I.dinv);
        hipFree(I.A_vf); hipFree(I.At_vf);
        hipFree(I.A_long); hipFree(I.At_long);
    }
    hipFree(I.b); hipFree(I.c); hipFree(I.g);
    hipFree(I.qoff); hipFree(I.sord); hipFree(I.soff);
    hipFree(I.K.psd_scratch);
    hipFree(I.K.psd_vecs);
    hipFree(I.K.psd_team);
    hipFree(I.K.psd_warm);
    hipFree(I.partA); hipFree(I.partAt);
    hipFree(I.Minv);
    I = Inst{};
}

Prob make_prob(const Inst& I) {
    Prob P{};
    P.n = I.n; P.m = I.m; P.N = I.N;
    P.A = Csr<double>{I.A_rp, I.A_ci, I.A_v, I.m, I.n, I.segA, I.A_long, I.nlongA, I.lthrA};
    P.At = Csr<double>{I.At_rp, I.At_ci, I.At_v, I.n, I.m, I.segAt, I.At_long, I.nlongAt, I.lthrAt};
    P.Af = Csr<float>{I.A_rp, I.A_ci, I.A_vf, I.m, I.n, I.segA, I.A_long, I.nlongA, I.lthrA};
    P.Atf = Csr<float>{I.At_rp, I.At_ci, I.At_vf, I.n, I.m, I.segAt, I.At_long, I.nlongAt, I.lthrAt};
    P.b = I.b; P.c = I.c; P.dinv = I.dinv; P.g = I.g;
    P.partA = I.partA; P.partAt = I.partAt; P.lds_cache = I.op_lds ? 1 : 0;
    P.delta = I.delta; P.nb = I.nb; P.nc = I.nc;
    P.K = I.K;
    P.Minv = I.Minv;
    return P;
}

size_t vec_doubles(int n, int m, int mem) {
    const size_t N = (size_t)n + m + 1;
    return 9 * N + 19 * (size_t)n + (size_t)m + 3 * (size_t)mem * N + 8;
}

// Carves the Vecs of one instance from a contiguous device buffer.
Vecs carve(double* base, int n, int m, int mem) {
    const size_t N = (size_t)n + m + 1;
    Vecs V{};
    double* p = base;
    auto take = [&](size_t len) { double* q = p; p += len; return q; };
    V.u = take(N); V.ut = take(N); V.ub = take(N); V.Ru = take(N); V.d = take(N);
    V.dt = take(N); V.Rw = take(N); V.pz = take(N); V.pxi = take(N);
    V.xw_u = take(n); V.xw_d = take(n);
    V.q_u = take(n); V.q_d = take(n);
    V.cg_b = take(n); V.cg_u = take(n); V.cg_w = take(n); V.cg_p = take(n);
    V.cg_r = take(n); V.cg_s = take(n); V.rhs_u = take(n);
    p = reinterpret_cast<double*>((reinterpret_cast<uintptr_t>(p) + 31) & ~uintptr_t(31));   // 32-byte records
    V.cg_g[0] = take(4 * (size_t)n); V.cg_g[1] = take(4 * (size_t)n);
    V.cg_t = take(m);
    V.Zb = take((size_t)mem * N); V.Yb = take((size_t)mem * N); V.Qb = take((size_t)mem * N);
    return V;
}

}  // namespace

// ------------------------------------------------------------------ single instance

// Plan of the column-panel SpMV for one matrix (built at its first
// stand-alone product).
struct PanelPlan {
    bool built = false, use = false;
    int P = 1, pc = 0, S = 8, U = 1, R = 1, nitems = 0;
    int* items = nullptr;
    int* prp = nullptr;          // panel-major row pointers (P rows + 1), several panels
    int* pci = nullptr;          // panel-major column indices (panel-relative)
    double* pv = nullptr;        // panel-major values
    double* part = nullptr;      // P x rows partial sums
};

struct sscs_work {
    hipStream_t stream = nullptr;
    PanelPlan panel[2];          // A, A^T
    sscs_settings st{};
    Inst I;
    double* vecbuf = nullptr;
    Vecs V{};
    double* io = nullptr;        // staging for host vectors: 4 N
    double* scal = nullptr;      // device scalars
    Result* res = nullptr;
    unsigned long long* bar = nullptr;
    int* abort_flag = nullptr;
    double* part = nullptr;
    double* tr_res = nullptr;
    int* tr_kind = nullptr;
    int* tr_ls = nullptr;
    double* tr_eta = nullptr;
    double* tr_rsafe = nullptr;
    long long tr_cap = 0;
    long long last_iters = -1;
    int grid = 1, max_grid = 1, ncu = 1;
    double ticks_per_s = 1e8;
    long long timeout_ticks = 0;
    double setup_s = 0;
};

namespace {

int launch_grid_kernel(sscs_work* w, void* fn, void** args) {
    HIP_TRY(hipMemsetAsync(w->bar, 0, BAR_WORDS * sizeof(unsigned long long), w->stream));
    HIP_TRY(hipMemsetAsync(w->abort_flag, 0, sizeof(int), w->stream));
    HIP_TRY(hipLaunchCooperativeKernel(fn, dim3(w->grid), dim3(kBlock), args, (size_t)w->I.lds_bytes, w->stream));
    return SSCS_OK;
}

int check_abort(sscs_work* w) {
    int flag = 0;
    HIP_TRY(hipMemcpyAsync(&flag, w->abort_flag, sizeof(int), hipMemcpyDeviceToHost, w->stream));
    HIP_TRY(hipStreamSynchronize(w->stream));
    if (flag) {
        g_last_hip = "grid barrier timed out";
        return SSCS_E_DEVICE;
    }
    return SSCS_OK;
}

// Kernel instantiation for the operator placement (LDS or global) and the
// precision of the CG operator.
// The grid kernels for an instance: operator in LDS or not, FP32 or FP64 CG
// operator, with or without the team path for PSD blocks above order 64.
template <template <bool, typename, bool> class K_>
const void* pick_grid(bool lds, bool mixed, bool pt) {
    if (pt) {
        if (mixed) return lds ? (const void*)K_<true, float, true>::fn : (const void*)K_<false, float, true>::fn;
        return lds ? (const void*)K_<true, double, true>::fn : (const void*)K_<false, double, true>::fn;
    }
    if (mixed) return lds ? (const void*)K_<true, float, false>::fn : (const void*)K_<false, float, false>::fn;
    return lds ? (const void*)K_<true, double, false>::fn : (const void*)K_<false, double, false>::fn;
}
template <bool L, typename T, bool P> struct SolveGridK { static constexpr auto fn = k_solve_grid<L, T, P>; };
template <bool L, typename T, bool P> struct OpGridK { static constexpr auto fn = k_op_grid<L, T, P>; };

bool team_psd(const Inst& I) { return I.K.psd_kmax > kPsdTeamOrder; }
const void* solve_grid_fn(bool lds, const Inst& I) { return pick_grid<SolveGridK>(lds, I.mixed, team_psd(I)); }
const void* op_grid_fn(bool lds, const Inst& I) { return pick_grid<OpGridK>(lds, I.mixed, team_psd(I)); }

// The column-panel kernel for S lanes per row, U steps per batch (U > 1
// only with S = 4) and R rows per segment step (1 or 4).
template <int S>
const void* panel_kernel_s(int R) {
    return R > 1 ? (const void*)k_spmv_panel<S, 1, 4> : (const void*)k_spmv_panel<S, 1, 1>;
}
const void* panel_kernel(int S, int U, int R) {
    if (S == 4 && U > 1 && R == 1) {
        switch (U) {
            case 2: return (const void*)k_spmv_panel<4, 2, 1>;
            case 3: return (const void*)k_spmv_panel<4, 3, 1>;
            case 4: return (const void*)k_spmv_panel<4, 4, 1>;
            case 5: return (const void*)k_spmv_panel<4, 5, 1>;
            case 6: return (const void*)k_spmv_panel<4, 6, 1>;
            case 7: return (const void*)k_spmv_panel<4, 7, 1>;
            default: return (const void*)k_spmv_panel<4, 8, 1>;
        }
    }
    switch (S) {
        case 1: return panel_kernel_s<1>(R);
        case 2: return panel_kernel_s<2>(R);
        case 4: return panel_kernel_s<4>(R);
        case 8: return panel_kernel_s<8>(R);
        case 16: return panel_kernel_s<16>(R);
        case 32: return panel_kernel_s<32>(R);
        default: return panel_kernel_s<64>(R);
    }
}

// The column-panel plan of A (which = 0) or A^T (1).  It is used when staging
// the panels costs at most a quarter of the operator's bytes (so large
// operators take it, small cache-resident ones keep the stream form).
int panel_plan(sscs_work* w, int which) {
    PanelPlan& pl = w->panel[which];
    if (pl.built) return SSCS_OK;
    pl.built = true;
    const Inst& I = w->I;
    const int rows = which ? I.n : I.m, cols = which ? I.m : I.n;
    const long long nnz = I.nnz;
    pl.P = (cols + kPanelCols - 1) / kPanelCols;
    pl.pc = (cols + pl.P - 1) / pl.P;
    const int G = std::max(1, w->ncu);
    const int chunks = pl.P >= G ? 1 : (G + pl.P - 1) / pl.P;
    const double staging = (double)pl.P * chunks * pl.pc * 8.0;
    // (and when a lane's entry index plus a batch, k + U S, stays within int32)
    pl.use = staging * 4.0 <= (double)nnz * 12.0 && nnz <= (long long)INT_MAX - 1024;
    if (!pl.use) return SSCS_OK;
    const double mean = (double)nnz / std::max(1.0, (double)rows * pl.P);
    if (mean >= 6.0 && mean <= 40.0) {           // four lanes per row, about a row per batch
        pl.S = 4;
        pl.U = std::min(8, std::max(2, (int)std::lround(mean / 4.0)));
        pl.R = 1;
    } else {                                      // S a power of two near a third of the row length
        pl.S = 1;
        while (pl.S < 64 && pl.S < mean / 3.0) pl.S <<= 1;
        pl.U = 1;
        pl.R = pl.P > 1 ? 4 : 1;
    }
    std::vector<int> items;
    for (int p = 0; p < pl.P; ++p)
        for (int c = 0; c < chunks; ++c) items.insert(items.end(), {p, c, chunks});
    pl.nitems = (int)items.size() / 3;
    TRY(dmalloc(&pl.items, items.size()));
    HIP_TRY(hipMemcpy(pl.items, items.data(), items.size() * sizeof(int), hipMemcpyHostToDevice));
    if (pl.P > 1) {
        const int* drp = which ? I.At_rp : I.A_rp;
        const int* dci = which ? I.At_ci : I.A_ci;
        const double* dv = which ? I.At_v : I.A_v;
        const long long total = (long long)rows * pl.P;
        if (total >= (1ll << 31) - 1) { pl.use = false; return SSCS_OK; }
        int* len = nullptr;
        TRY(dmalloc(&len, total));
        TRY(dmalloc(&pl.prp, total + 1));
        TRY(dmalloc(&pl.pci, (size_t)nnz));
        TRY(dmalloc(&pl.pv, (size_t)nnz));
        TRY(dmalloc(&pl.part, (size_t)rows * pl.P));
        const int g = (int)std::min<long long>(65535, (total + 255) / 256);
        k_panel_lens<<<g, 256, 0, w->stream>>>(drp, dci, rows, pl.P, pl.pc, len);
        k_scan<<<1, 1024, 0, w->stream>>>(len, (int)total, pl.prp);
        k_panel_scatter<<<g, 256, 0, w->stream>>>(drp, dci, dv, rows, pl.P, pl.pc, pl.prp, pl.pci, pl.pv);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(w->stream));
        hipFree(len);
    }
    static const bool attr = [] {
        bool ok = true;
        std::vector<const void*> fns;
        for (int S = 1; S <= 64; S <<= 1)
            for (int R : {1, 4}) fns.push_back(panel_kernel(S, 1, R));
        for (int U = 2; U <= 8; ++U) fns.push_back(panel_kernel(4, U, 1));
        for (const void* f : fns)
            ok = ok && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           kPanelCols * (int)sizeof(double)) == hipSuccess;
        return ok;
    }();
    if (!attr) pl.use = false;
    return SSCS_OK;
}

// y = M x for M = A (transpose 0) or A^T (1), device vectors, on the
// workspace stream: the column-panel form when the plan takes it, the stream
// form otherwise.
int launch_spmv(sscs_work* w, int transpose, const double* dx, double* dy) {
    TRY(panel_plan(w, transpose ? 1 : 0));
    const PanelPlan& pl = w->panel[transpose ? 1 : 0];
    Prob P = make_prob(w->I);
    const Csr<double>& M = transpose ? P.At : P.A;
    if (pl.use) {
        const int grid = std::max(1, std::min(pl.nitems, w->ncu));
        const int* rp = pl.P > 1 ? pl.prp : M.rp;
        const int* ci = pl.P > 1 ? pl.pci : M.ci;
        const double* v = pl.P > 1 ? pl.pv : M.v;
        int rows = M.rows, cols = M.cols;
        const int* items = pl.items;
        int nitems = pl.nitems, np = pl.P, pc = pl.pc;
        double* part = pl.part;
        long long nnz = w->I.nnz;                // the panel-major copy holds the same entries
        void* args[] = {&rp, &ci, &v, &rows, &cols, &items, &nitems, &np, &pc, &dx, &dy, &part, &nnz};
        HIP_TRY(hipLaunchKernel(panel_kernel(pl.S, pl.U, pl.R), dim3(grid), dim3(kPanelThreads), args,
                                (size_t)pl.pc * sizeof(double), w->stream));
        if (pl.P > 1)
            k_panel_sum<<<std::max(1, std::min(65535, (M.rows + kPanelSumThreads - 1) / kPanelSumThreads)),
                          kPanelSumThreads, 0, w->stream>>>(pl.part, pl.P, M.rows, dy);
    } else {
        const long long threads = (long long)M.rows * M.seg;
        const int grid = (int)std::max<long long>(1, std::min<long long>(65535, (threads + 255) / 256));
        k_spmv<<<grid, 256, 0, w->stream>>>(M, dx, dy);
    }
    HIP_TRY(hipGetLastError());
    return SSCS_OK;
}

int run_op(sscs_work* w, int op, const double* in, double* out1, double* out2, double tol, int maxit) {
    Prob P = make_prob(w->I);
    OpArgs a{op, in, out1, out2, w->scal, tol, maxit};
    void* args[] = {&P, &w->V, &a, &w->bar, &w->abort_flag, &w->part, &w->timeout_ticks};
    TRY(launch_grid_kernel(w, const_cast<void*>(op_grid_fn(w->I.op_lds, w->I)), args));
    HIP_TRY(hipGetLastError());
    return check_abort(w);
}

// Host or device vector in, device pointer out (staged through w->io).
int stage_in(sscs_work* w, const double* src, size_t len, int slot, const double** dev) {
    if (w->st.data_on_device) { *dev = src; return SSCS_OK; }
    double* dst = w->io + (size_t)slot * w->I.N;
    HIP_TRY(hipMemcpyAsync(dst, src, len * sizeof(double), hipMemcpyHostToDevice, w->stream));
    *dev = dst;
    return SSCS_OK;
}

double* out_ptr(sscs_work* w, double* user, int slot) {
    return w->st.data_on_device ? user : w->io + (size_t)slot * w->I.N;
}

int stage_out(sscs_work* w, double* user, const double* dev, size_t len) {
    if (w->st.data_on_device || user == nullptr) return SSCS_OK;
    HIP_TRY(hipMemcpyAsync(user, dev, len * sizeof(double), hipMemcpyDeviceToHost, w->stream));
    return SSCS_OK;
}

// Row partition of a CSR matrix over G workgroups, balanced by nonzeros.
std::vector<int> partition_rows(const std::vector<int>& rp, int rows, int G) {
    std::vector<int> part(G + 1, 0);
    const long long nnz = rp[rows];
    for (int b = 1; b < G; ++b) {
        const long long target = nnz * b / G;
        int r = (int)(std::lower_bound(rp.begin(), rp.begin() + rows + 1, (int)target) - rp.begin());
        part[b] = std::max(part[b - 1], std::min(r, rows));
    }
    part[G] = rows;
    return part;
}

// LDS bytes workgroup b needs to hold its rows (values, column indices, local
// row pointers), with the layout load_part() uses.
long long part_lds_bytes(const std::vector<int>& rp, const std::vector<int>& part, int b, int vbytes) {
    const long long rows = part[b + 1] - part[b];
    const long long nnz = rp[part[b + 1]] - rp[part[b]];
    return ((vbytes + 4) * nnz + 4 * (rows + 1) + 15) & ~15ll;
}

int set_partitions(sscs_work* w, bool try_lds);

int choose_grid(sscs_work* w) {
    int dev = 0, ncu = 0, occ = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, solve_grid_fn(false, w->I), kBlock, 0));
    int occ2 = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ2, op_grid_fn(false, w->I), kBlock, 0));
    occ = std::max(1, std::min(occ, occ2));
    w->ncu = ncu;
    w->max_grid = std::max(1, ncu * occ);
    // one workgroup per CU once there are about two nonzeros of A per thread
    const long long want = std::max<long long>((w->I.nnz + 2ll * kBlock - 1) / (2ll * kBlock),
                                               ((long long)w->I.N + kBlock - 1) / kBlock);
    w->grid = (int)std::max<long long>(1, std::min<long long>(want, w->max_grid));
    if (small_fits(w->I, w->st)) w->grid = 1;     // one workgroup with its working set in LDS
    if (w->st.workgroups >= 1) w->grid = std::min(w->st.workgroups, w->max_grid);
    int rate_khz = 0;
    HIP_TRY(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev));
    w->ticks_per_s = rate_khz > 0 ? rate_khz * 1000.0 : 1e8;
    w->timeout_ticks = (long long)(60.0 * w->ticks_per_s);
    return set_partitions(w, true);
}

// Row partitions for the grid size; caches the operator in LDS when every
// workgroup's share fits next to the static LDS and the grid stays co-resident.
int set_partitions(sscs_work* w, bool try_lds) {
    Inst& I = w->I;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    int lds_max = 0;
    HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    // dynamic LDS left next to the kernels' static LDS (Shared, descriptors,
    // the PSD rotation tables)
    long long stat = 0;
    for (const void* f : {solve_grid_fn(true, I), op_grid_fn(true, I)}) {
        hipFuncAttributes fa{};
        HIP_TRY(hipFuncGetAttributes(&fa, f));
        stat = std::max<long long>(stat, (long long)fa.sharedSizeBytes);
    }
    const long long limit = (long long)lds_max - stat - 256;
    // the PSD blocks projected one per workgroup get their matrix and
    // eigenvectors in LDS first (their Jacobi rounds are the projection's
    // critical path); the operator rows are cached after them if they fit
    long long psd = ((2ll * I.psd_small * I.psd_small * 8) + 15) & ~15ll;
    if (psd > limit) psd = 0;
    std::vector<int> pA, pAt;
    long long need = 0;
    const int vb = I.mixed ? 4 : 8;       // bytes per cached value
    for (int attempt = 0; attempt < 2; ++attempt) {
        pA = partition_rows(I.h_rpA, I.m, w->grid);
        pAt = partition_rows(I.h_rpAt, I.n, w->grid);
        need = psd;
        for (int b = 0; b < w->grid; ++b)
            need = std::max(need, psd + part_lds_bytes(I.h_rpA, pA, b, vb) + part_lds_bytes(I.h_rpAt, pAt, b, vb));
        I.lds_bytes = (int)psd;
        I.op_lds = false;
        if (!try_lds || w->grid < 2 || need > limit) break;
        int o1 = 0, o2 = 0;
        HIP_TRY(hipFuncSetAttribute(solve_grid_fn(true, I), hipFuncAttributeMaxDynamicSharedMemorySize, (int)need));
        HIP_TRY(hipFuncSetAttribute(op_grid_fn(true, I), hipFuncAttributeMaxDynamicSharedMemorySize, (int)need));
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&o1, solve_grid_fn(true, I), kBlock, (size_t)need));
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&o2, op_grid_fn(true, I), kBlock, (size_t)need));
        const int cap = w->ncu * std::min(o1, o2);
        if (cap >= w->grid) { I.lds_bytes = (int)need; I.op_lds = true; break; }
        if (cap < 2) break;
        w->grid = cap;                        // shrink to a co-resident grid and re-partition
    }
    if (!I.op_lds && psd > 0) {
        // the PSD area alone, on the kernels without the operator cache
        int o1 = 0, o2 = 0;
        HIP_TRY(hipFuncSetAttribute(solve_grid_fn(false, I), hipFuncAttributeMaxDynamicSharedMemorySize, (int)psd));
        HIP_TRY(hipFuncSetAttribute(op_grid_fn(false, I), hipFuncAttributeMaxDynamicSharedMemorySize, (int)psd));
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&o1, solve_grid_fn(false, I), kBlock, (size_t)psd));
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&o2, op_grid_fn(false, I), kBlock, (size_t)psd));
        if (w->ncu * std::min(o1, o2) < w->grid) psd = 0;     // not co-resident with it: keep the area global
        I.lds_bytes = (int)psd;
    }
    I.K.psd_lds = (int)psd;
    I.K.psd_small = I.psd_small;
    hipFree(I.partA);
    hipFree(I.partAt);
    TRY(dmalloc(&I.partA, pA.size()));
    TRY(dmalloc(&I.partAt, pAt.size()));
    HIP_TRY(hipMemcpy(I.partA, pA.data(), pA.size() * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(I.partAt, pAt.data(), pAt.size() * sizeof(int), hipMemcpyHostToDevice));
    return SSCS_OK;
}

int alloc_work_vectors(sscs_work* w) {
    const int mem = MEMMAX;     // memory buffers sized for the largest mem so settings may change
    TRY(dmalloc(&w->vecbuf, vec_doubles(w->I.n, w->I.m, mem)));
    w->V = carve(w->vecbuf, w->I.n, w->I.m, mem);
    TRY(dmalloc(&w->io, 4 * (size_t)w->I.N));
    TRY(dmalloc(&w->scal, 16));
    TRY(dmalloc(&w->res, 1));
    TRY(dmalloc(&w->bar, BAR_WORDS));
    TRY(dmalloc(&w->abort_flag, 1));
    TRY(dmalloc(&w->part, 4 * (size_t)KMAX * w->max_grid));   // two buffers for the grid, two for its PSD sub-team
    if (w->I.K.ns > 0) {
        const size_t k = w->I.K.psd_kmax;
        const size_t per = psd_scratch_doubles((int)k);
        const size_t nblk = std::min<size_t>(w->grid, w->I.K.ns);
        TRY(dmalloc(&w->I.K.psd_scratch, per * nblk));
        TRY(dmalloc(&w->I.K.psd_vecs, k * k * (size_t)w->I.K.ns));
        if ((int)k > kPsdTeamOrder) TRY(dmalloc(&w->I.K.psd_team, psd_team_doubles((int)k)));
        TRY(dmalloc(&w->I.K.psd_warm, (size_t)w->I.K.ns));
        HIP_TRY(hipMemsetAsync(w->I.K.psd_warm, 0, w->I.K.ns * sizeof(int), w->stream));
    }
    return SSCS_OK;
}

// The direct linear step's operator, on the device: M = I + A^T A formed
// from the rows of A^T, its blocked Cholesky factor in place, then
// M^{-1} = L^{-T} L^{-1} by substitution with the identity; the factor is
// freed once the inverse is formed.
int build_direct(sscs_work* w) {
    Inst& I = w->I;
    const int n = I.n;
    if (n > SSCS_DIRECT_NMAX || I.mixed) {
        g_unsupported = n > SSCS_DIRECT_NMAX ? "the direct linear step takes n <= SSCS_DIRECT_NMAX"
                                             : "the direct linear step is FP64 only";
        return SSCS_E_UNSUPPORTED;
    }
    const int nb = (n + DIRECT_B - 1) / DIRECT_B;
    double *Lc = nullptr, *Li = nullptr;
    int* err = nullptr;
    int r = dmalloc(&Lc, (size_t)n * n);
    if (r == SSCS_OK) r = dmalloc(&Li, (size_t)nb * DIRECT_B * DIRECT_B);
    if (r == SSCS_OK) r = dmalloc(&I.Minv, (size_t)n * n);
    if (r == SSCS_OK) r = dmalloc(&err, 1);
    auto release = [&] { hipFree(Lc); hipFree(Li); hipFree(err); };
    if (r != SSCS_OK) { release(); return r; }
    const hipStream_t st = w->stream;
    hipError_t e = hipMemsetAsync(err, 0, sizeof(int), st);
    k_form_normal<<<dim3((n + 15) / 16, (n + 15) / 16), dim3(16, 16), 0, st>>>(I.At_rp, I.At_ci, I.At_v, n, Lc);
    for (int b = 0; b < nb; ++b) {
        const int k0 = b * DIRECT_B, kn = std::min(DIRECT_B, n - k0);
        double* Lib = Li + (size_t)b * DIRECT_B * DIRECT_B;
        k_chol_diag<<<1, 256, 0, st>>>(Lc, n, k0, kn, Lib, err);
        const int rest = n - k0 - kn;
        if (rest > 0) {
            const int nt = (rest + DIRECT_B - 1) / DIRECT_B;
            k_chol_panel<<<nt, 256, 0, st>>>(Lc, n, k0, kn, Lib);
            k_chol_update<<<dim3(nt, nt), 256, 0, st>>>(Lc, n, k0, kn);
        }
    }
    double* W = I.Minv;
    k_identity<<<1024, 256, 0, st>>>(W, n);
    for (int b = 0; b < nb; ++b) {                                   // L Y = I
        const int k0 = b * DIRECT_B, kn = std::min(DIRECT_B, n - k0);
        k_inv_apply<<<nb, 256, 0, st>>>(W, n, k0, kn, Li + (size_t)b * DIRECT_B * DIRECT_B, 0);
        const int rest = n - k0 - kn;
        if (rest > 0) k_inv_update<<<dim3(nb, (rest + DIRECT_B - 1) / DIRECT_B), 256, 0, st>>>(W, Lc, n, k0, kn, 1);
    }
    for (int b = nb - 1; b >= 0; --b) {                              // L^T X = Y
        const int k0 = b * DIRECT_B, kn = std::min(DIRECT_B, n - k0);
        k_inv_apply<<<nb, 256, 0, st>>>(W, n, k0, kn, Li + (size_t)b * DIRECT_B * DIRECT_B, 1);
        if (k0 > 0) k_inv_update<<<dim3(nb, (k0 + DIRECT_B - 1) / DIRECT_B), 256, 0, st>>>(W, Lc, n, k0, kn, 0);
    }
    int h = 0;
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&h, err, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    release();
    if (e != hipSuccess) {
        g_last_hip = hipGetErrorString(e);
        return SSCS_E_HIP;
    }
    if (h) {
        g_last_hip = "the Cholesky factor of I + A^T A met a non-positive pivot";
        return SSCS_E_DEVICE;
    }
    return SSCS_OK;
}

int setup_linear(sscs_work* w) {
    // g = M^{-1} (c, b) and delta = 1 + (c, b)^T g, solved tightly once
    double* h = w->io;
    HIP_TRY(hipMemcpyAsync(h, w->I.c, w->I.n * sizeof(double), hipMemcpyDeviceToDevice, w->stream));
    HIP_TRY(hipMemcpyAsync(h + w->I.n, w->I.b, w->I.m * sizeof(double), hipMemcpyDeviceToDevice, w->stream));
    HIP_TRY(hipMemsetAsync(h + w->I.n + w->I.m, 0, sizeof(double), w->stream));
    TRY(run_op(w, OP_SETUP, h, w->I.g, nullptr, std::min(1e-14, w->st.cg_tol), std::max(w->st.cg_max, 1000)));
    double sc[4];
    HIP_TRY(hipMemcpyAsync(sc, w->scal, sizeof(sc), hipMemcpyDeviceToHost, w->stream));
    HIP_TRY(hipStreamSynchronize(w->stream));
    w->I.delta = sc[0];
    w->I.nb = sc[1];
    w->I.nc = sc[2];
    if (!std::isfinite(sc[0])) return SSCS_E_INVALID;
    return SSCS_OK;
}

int alloc_trace(sscs_work* w) {
    hipFree(w->tr_res); hipFree(w->tr_kind); hipFree(w->tr_ls); hipFree(w->tr_eta); hipFree(w->tr_rsafe);
    w->tr_res = nullptr; w->tr_kind = nullptr; w->tr_ls = nullptr; w->tr_eta = nullptr; w->tr_rsafe = nullptr;
    w->tr_cap = 0;
    if (!w->st.record_trace) return SSCS_OK;
    w->tr_cap = std::min<long long>(w->st.max_iters + 1, 4 << 20);
    TRY(dmalloc(&w->tr_res, w->tr_cap));
    TRY(dmalloc(&w->tr_kind, w->tr_cap));
    TRY(dmalloc(&w->tr_ls, w->tr_cap));
    TRY(dmalloc(&w->tr_eta, w->tr_cap));
    TRY(dmalloc(&w->tr_rsafe, w->tr_cap));
    return SSCS_OK;
}

void fill_info(sscs_info* info, const Result& r, double setup_s, double solve_s) {
    if (!info) return;
    info->status = r.status;
    info->iters = r.iters;
    info->k0 = r.k0; info->k1 = r.k1; info->k2 = r.k2; info->km = r.km;
    info->backtracks = r.bt;
    info->cg_iters = r.cg;
    info->pr = r.pr; info->dr = r.dr; info->gap = r.gap; info->ic = r.ic; info->uc = r.uc;
    info->pobj = r.pobj; info->dobj = r.dobj; info->res_fp = r.res;
    info->setup_s = setup_s;
    info->solve_s = solve_s;
}

}  // namespace

extern "C" {

int sscs_default_settings(sscs_settings* st) {
    if (!st) return SSCS_E_INVALID;
    std::memset(st, 0, sizeof(*st));
    st->eps = 1e-6;
    st->direction = SSCS_DIR_AA;
    st->mem = 5;
    st->c0 = 0.99;
    st->c1 = 0.9999;
    st->q = 0.999;
    st->sigma = 0.01;
    st->lambda = 1.5;
    st->thetabar = 0.1;
    st->ls_max = 10;
    st->max_iters = 10000;
    st->max_time_s = 0.0;
    st->precision = SSCS_PREC_FP64;
    st->cg_tol = 1e-10;
    st->cg_max = 500;
    st->data_on_device = 0;
    st->record_trace = 0;
    st->aa_reg = 1e-12;
    st->cg_adapt = 0.0;
    st->cg_d_match = 1;
    st->check_every = 1;
    st->workgroups = 0;
    st->linsys = SSCS_LINSYS_CG;
    return SSCS_OK;
}

int sscs_create(const sscs_data* data, const sscs_cone* cone, const sscs_settings* st, void* hip_stream,
                sscs_work** out) {
    try {
        g_unsupported = nullptr;
        if (!out) return SSCS_E_INVALID;
        *out = nullptr;
        TRY(validate(data, cone));
        TRY(validate_settings(st));
        const double t0 = now_s();
        sscs_work* w = new (std::nothrow) sscs_work();
        if (!w) return SSCS_E_NOMEM;
        w->stream = (hipStream_t)hip_stream;
        w->st = *st;
        int r = upload_instance(w->I, data, cone, w->stream, nullptr, st->precision == SSCS_PREC_MIXED);
        if (r == SSCS_OK) r = choose_grid(w);
        if (r == SSCS_OK) r = alloc_work_vectors(w);
        if (r == SSCS_OK) r = alloc_trace(w);
        if (r == SSCS_OK && st->linsys == SSCS_LINSYS_DIRECT) r = build_direct(w);
        if (r == SSCS_OK) r = setup_linear(w);
        if (r != SSCS_OK) { sscs_destroy(w); return r; }
        w->setup_s = now_s() - t0;
        *out = w;
        return SSCS_OK;
    } catch (...) {
        return SSCS_E_NOMEM;
    }
}

int sscs_update_settings(sscs_work* w, const sscs_settings* st) {
    if (!w) return SSCS_E_INVALID;
    TRY(validate_settings(st));
    if (st->precision != w->st.precision || st->workgroups != w->st.workgroups || st->linsys != w->st.linsys)
        return SSCS_E_INVALID;
    const bool retrace = st->record_trace != w->st.record_trace || st->max_iters != w->st.max_iters;
    w->st = *st;
    if (retrace) TRY(alloc_trace(w));
    return SSCS_OK;
}

int sscs_update_bc(sscs_work* w, const double* b, const double* c) {
    if (!w || !b || !c) return SSCS_E_INVALID;
    const hipMemcpyKind kind = w->st.data_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIP_TRY(hipMemcpyAsync(w->I.b, b, w->I.m * sizeof(double), kind, w->stream));
    HIP_TRY(hipMemcpyAsync(w->I.c, c, w->I.n * sizeof(double), kind, w->stream));
    return setup_linear(w);
}

int sscs_destroy(sscs_work* w) {
    if (!w) return SSCS_OK;
    if (w->stream) hipStreamSynchronize(w->stream);
    else hipDeviceSynchronize();
    free_instance(w->I);
    hipFree(w->vecbuf); hipFree(w->io); hipFree(w->scal); hipFree(w->res);
    hipFree(w->bar); hipFree(w->abort_flag); hipFree(w->part);
    hipFree(w->tr_res); hipFree(w->tr_kind); hipFree(w->tr_ls); hipFree(w->tr_eta); hipFree(w->tr_rsafe);
    for (auto& pl : w->panel) {
        hipFree(pl.items); hipFree(pl.prp); hipFree(pl.pci); hipFree(pl.pv); hipFree(pl.part);
    }
    delete w;
    return SSCS_OK;
}

int sscs_solve(sscs_work* w, const double* u0, double* x, double* y, double* s, sscs_info* info) {
    if (!w || !x || !y || !s) return SSCS_E_INVALID;
    const double t0 = now_s();
    const int n = w->I.n, m = w->I.m, N = w->I.N;
    const double* du0 = nullptr;
    if (u0) TRY(stage_in(w, u0, N, 0, &du0));
    Vecs V = w->V;
    V.u0 = du0;
    V.out_x = out_ptr(w, x, 1);
    V.out_y = out_ptr(w, y, 2);
    V.out_s = out_ptr(w, s, 3);
    V.tr_res = w->tr_res; V.tr_kind = w->tr_kind; V.tr_ls = w->tr_ls; V.tr_cap = w->tr_cap;
    V.tr_eta = w->tr_eta; V.tr_rsafe = w->tr_rsafe;
    Prob P = make_prob(w->I);
    Params S = make_params(w->st, w->ticks_per_s);
    // every solve starts its PSD projections cold (same input, same bits)
    if (w->I.K.psd_warm) HIP_TRY(hipMemsetAsync(w->I.K.psd_warm, 0, w->I.K.ns * sizeof(int), w->stream));
    if (w->grid == 1) {
        HIP_TRY(hipMemsetAsync(w->abort_flag, 0, sizeof(int), w->stream));
        const int sd = stage_doubles(w->I.n + w->I.m);
        int bytes = 0;
        const int mask = small_plan(w->I, w->st, &bytes);
        if (w->I.mixed)
            k_solve_block<float><<<1, kBatchBlock, sd * sizeof(double), w->stream>>>(P, V, S, w->res, sd);
        else if ((mask & (SP_OP | SP_PROB | SP_CG)) == (SP_OP | SP_PROB | SP_CG))
            k_solve_small<true><<<1, kBatchBlock, bytes, w->stream>>>(P, V, S, w->res, (int)(w->I.n + w->I.m), mask);
        else if (mask)
            k_solve_small<false><<<1, kBatchBlock, bytes, w->stream>>>(P, V, S, w->res, (int)(w->I.n + w->I.m), mask);
        else
            k_solve_block<double><<<1, kBatchBlock, sd * sizeof(double), w->stream>>>(P, V, S, w->res, sd);
    } else {
        void* args[] = {&P, &V, &S, &w->res, &w->bar, &w->abort_flag, &w->part, &w->timeout_ticks};
        TRY(launch_grid_kernel(w, const_cast<void*>(solve_grid_fn(w->I.op_lds, w->I)), args));
    }
    HIP_TRY(hipGetLastError());
    TRY(stage_out(w, x, V.out_x, n));
    TRY(stage_out(w, y, V.out_y, m));
    TRY(stage_out(w, s, V.out_s, m));
    Result r{};
    HIP_TRY(hipMemcpyAsync(&r, w->res, sizeof(Result), hipMemcpyDeviceToHost, w->stream));
    TRY(check_abort(w));
    w->last_iters = r.iters;
    fill_info(info, r, w->setup_s, now_s() - t0);
    return SSCS_OK;
}

int sscs_linear_step(sscs_work* w, const double* r, double* out) {
    if (!w || !r || !out) return SSCS_E_INVALID;
    const double* dr = nullptr;
    TRY(stage_in(w, r, w->I.N, 0, &dr));
    double* dout = out_ptr(w, out, 1);
    TRY(run_op(w, OP_LINEAR, dr, dout, nullptr, w->st.cg_tol, w->st.cg_max));
    TRY(stage_out(w, out, dout, w->I.N));
    HIP_TRY(hipStreamSynchronize(w->stream));
    return SSCS_OK;
}

int sscs_residual(sscs_work* w, const double* u, double* ut, double* Ru) {
    if (!w || !u || !Ru) return SSCS_E_INVALID;
    const double* du = nullptr;
    TRY(stage_in(w, u, w->I.N, 0, &du));
    double* dut = ut ? out_ptr(w, ut, 1) : nullptr;
    double* dRu = out_ptr(w, Ru, 2);
    TRY(run_op(w, OP_RESIDUAL, du, dut, dRu, w->st.cg_tol, w->st.cg_max));
    if (ut) TRY(stage_out(w, ut, dut, w->I.N));
    TRY(stage_out(w, Ru, dRu, w->I.N));
    HIP_TRY(hipStreamSynchronize(w->stream));
    return SSCS_OK;
}

int sscs_project_dual_cone(sscs_work* w, const double* in, double* out) {
    if (!w || !in || !out) return SSCS_E_INVALID;
    const double* din = nullptr;
    TRY(stage_in(w, in, w->I.m, 0, &din));
    double* dout = out_ptr(w, out, 1);
    TRY(run_op(w, OP_PROJECT, din, dout, nullptr, 0.0, 0));
    TRY(stage_out(w, out, dout, w->I.m));
    HIP_TRY(hipStreamSynchronize(w->stream));
    return SSCS_OK;
}

int sscs_spmv(sscs_work* w, int32_t transpose, const double* x, double* y) {
    if (!w || !x || !y) return SSCS_E_INVALID;
    const int lin = transpose ? w->I.m : w->I.n, lout = transpose ? w->I.n : w->I.m;
    const double* dx = nullptr;
    TRY(stage_in(w, x, lin, 0, &dx));
    double* dy = out_ptr(w, y, 1);
    TRY(launch_spmv(w, transpose, dx, dy));
    TRY(stage_out(w, y, dy, lout));
    HIP_TRY(hipStreamSynchronize(w->stream));
    return SSCS_OK;
}

int sscs_spmv_bench(sscs_work* w, int32_t transpose, int32_t reps, double* ms) {
    if (!w || !ms || reps < 1) return SSCS_E_INVALID;
    const double* dx = transpose ? w->V.Ru + w->I.n : w->V.Ru;   // any resident vector of the right length
    double* dy = w->V.Rw;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    TRY(launch_spmv(w, transpose, dx, dy));     // warm-up (and the plan)
    HIP_TRY(hipEventRecord(e0, w->stream));
    for (int r = 0; r < reps; ++r) TRY(launch_spmv(w, transpose, dx, dy));
    HIP_TRY(hipEventRecord(e1, w->stream));
    HIP_TRY(hipEventSynchronize(e1));
    float f = 0.f;
    HIP_TRY(hipEventElapsedTime(&f, e0, e1));
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    *ms = f;
    return SSCS_OK;
}

int sscs_get_trace(sscs_work* w, int64_t cap, double* res, int32_t* kind, int32_t* ls, double* eta, double* r_safe,
                   int64_t* count) {
    if (!w || !count) return SSCS_E_INVALID;
    if (!w->tr_res || w->last_iters < 0) { *count = 0; return SSCS_OK; }
    const long long avail = std::min<long long>(w->last_iters + 1, w->tr_cap);
    *count = avail;
    const long long c = std::min<long long>(cap, avail);
    if (c > 0) {
        if (res) HIP_TRY(hipMemcpy(res, w->tr_res, c * sizeof(double), hipMemcpyDeviceToHost));
        if (kind) HIP_TRY(hipMemcpy(kind, w->tr_kind, c * sizeof(int), hipMemcpyDeviceToHost));
        if (ls) HIP_TRY(hipMemcpy(ls, w->tr_ls, c * sizeof(int), hipMemcpyDeviceToHost));
        if (eta) HIP_TRY(hipMemcpy(eta, w->tr_eta, c * sizeof(double), hipMemcpyDeviceToHost));
        if (r_safe) HIP_TRY(hipMemcpy(r_safe, w->tr_rsafe, c * sizeof(double), hipMemcpyDeviceToHost));
    }
    return SSCS_OK;
}

const char* sscs_error_string(int code) {
    static thread_local std::string msg;
    switch (code) {
        case SSCS_OK: return "ok";
        case SSCS_E_INVALID: return "invalid argument";
        case SSCS_E_NOMEM: msg = "out of memory"; break;
        case SSCS_E_HIP: msg = "HIP error"; break;
        case SSCS_E_UNSUPPORTED:
            if (!g_unsupported) return "unsupported";
            msg = std::string("unsupported: ") + g_unsupported;
            return msg.c_str();
        case SSCS_E_DEVICE: msg = "device engine failure"; break;
        default: return "unknown error";
    }
    if (!g_last_hip.empty()) msg += ": " + g_last_hip;
    return msg.c_str();
}

}  // extern "C"

// ------------------------------------------------------------------ batched

struct sscs_batch {
    hipStream_t stream = nullptr;
    sscs_settings st{};
    int count = 0;
    std::vector<Inst> inst;
    std::vector<size_t> off_x, off_y, off_u;     // packed offsets
    size_t tot_x = 0, tot_y = 0, tot_u = 0;
    double* vecbuf = nullptr;
    BatchInst* d_insts = nullptr;
    std::vector<BatchInst> h_insts;
    double* io = nullptr;        // staging: u0 (tot_u), x, y, s
    Result* res = nullptr;
    int* queue = nullptr;
    int* order = nullptr;        // queue position -> instance, most work per iteration first
    int grid = 1;
    int stage = 0;               // dynamic LDS of k_solve_batch, in doubles
    double ticks_per_s = 1e8;
    double setup_s = 0;
};


extern "C" {

int sscs_batch_destroy(sscs_batch* bt) {
    if (!bt) return SSCS_OK;
    if (bt->stream) hipStreamSynchronize(bt->stream);
    else hipDeviceSynchronize();
    for (auto& I : bt->inst) free_instance(I);
    hipFree(bt->vecbuf); hipFree(bt->d_insts); hipFree(bt->io); hipFree(bt->res); hipFree(bt->queue); hipFree(bt->order);
    delete bt;
    return SSCS_OK;
}

int sscs_batch_create(int32_t count, const sscs_data* data, const sscs_cone* cones, const sscs_settings* st,
                      void* hip_stream, sscs_batch** out) {
    try {
        g_unsupported = nullptr;
        if (!out || count < 1 || !data || !cones) return SSCS_E_INVALID;
        *out = nullptr;
        TRY(validate_settings(st));
        // the batched engine runs the FP64 operator only: its mixed-precision
        // form ran without finishing in a test whose cause has not been shown
        if (st->precision != SSCS_PREC_FP64) return SSCS_E_UNSUPPORTED;
        if (st->linsys != SSCS_LINSYS_CG) {
            g_unsupported = "batches run the CG linear step only";
            return SSCS_E_UNSUPPORTED;
        }
        for (int i = 0; i < count; ++i) {
            const bool shared = i > 0 && data[i].rowptr == data[0].rowptr && data[i].colind == data[0].colind &&
                                data[i].val == data[0].val && data[i].m == data[0].m && data[i].n == data[0].n &&
                                data[i].nnz == data[0].nnz;
            TRY(validate(&data[i], &cones[i], !shared));
            for (int j = 0; j < cones[i].ns; ++j)
                if (cones[i].s[j] > 64) return SSCS_E_UNSUPPORTED;
        }
        const double t0 = now_s();
        sscs_batch* bt = new (std::nothrow) sscs_batch();
        if (!bt) return SSCS_E_NOMEM;
        bt->stream = (hipStream_t)hip_stream;
        bt->st = *st;
        bt->count = count;
        bt->inst.resize(count);
        int r = SSCS_OK;
        for (int i = 0; i < count && r == SSCS_OK; ++i) {
            const bool share = i > 0 && data[i].rowptr == data[0].rowptr && data[i].colind == data[0].colind &&
                               data[i].val == data[0].val && data[i].m == data[0].m && data[i].n == data[0].n;
            r = upload_instance(bt->inst[i], &data[i], &cones[i], bt->stream, share ? &bt->inst[0] : nullptr,
                                st->precision == SSCS_PREC_MIXED);
        }
        size_t tot = 0;
        for (int i = 0; i < count && r == SSCS_OK; ++i) {
            const Inst& I = bt->inst[i];
            bt->off_x.push_back(bt->tot_x); bt->tot_x += I.n;
            bt->off_y.push_back(bt->tot_y); bt->tot_y += I.m;
            bt->off_u.push_back(bt->tot_u); bt->tot_u += I.N;
            tot += vec_doubles(I.n, I.m, st->mem);
        }
        if (r == SSCS_OK) r = dmalloc(&bt->vecbuf, tot);
        if (r == SSCS_OK) r = dmalloc(&bt->io, bt->tot_u + bt->tot_x + 2 * bt->tot_y);
        if (r == SSCS_OK) r = dmalloc(&bt->res, count);
        if (r == SSCS_OK) r = dmalloc(&bt->queue, 1);
        if (r == SSCS_OK) r = dmalloc(&bt->order, count);
        if (r == SSCS_OK) r = dmalloc(&bt->d_insts, count);
        // PSD scratch: one workgroup owns an instance at a time, so each instance
        // with PSD blocks gets its own (the batched engine allows orders <= 64)
        for (int i = 0; i < count && r == SSCS_OK; ++i) {
            Inst& I = bt->inst[i];
            if (I.K.ns > 0) {
                const size_t k = I.K.psd_kmax;
                r = dmalloc(&I.K.psd_scratch, psd_scratch_doubles((int)k));
            }
        }
        if (r == SSCS_OK) {
            bt->h_insts.resize(count);
            double* p = bt->vecbuf;
            for (int i = 0; i < count; ++i) {
                const Inst& I = bt->inst[i];
                bt->h_insts[i].P = make_prob(I);
                bt->h_insts[i].V = carve(p, I.n, I.m, st->mem);
                p += vec_doubles(I.n, I.m, st->mem);
            }
            hipError_t e = hipMemcpyAsync(bt->d_insts, bt->h_insts.data(), count * sizeof(BatchInst),
                                          hipMemcpyHostToDevice, bt->stream);
            if (e != hipSuccess) { g_last_hip = hipGetErrorString(e); r = SSCS_E_HIP; }
        }
        if (r == SSCS_OK) {
            // workgroups take instances in decreasing work per iteration (nonzeros
            // of A plus n + m; ties in index order), so the large instances start
            // first and the end of the launch is not held up by one of them
            std::vector<int> ord(count);
            for (int i = 0; i < count; ++i) ord[i] = i;
            auto cost = [&](int i) { return (long long)bt->inst[i].nnz + bt->inst[i].n + bt->inst[i].m; };
            std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return cost(a) > cost(b); });
            hipError_t e = hipMemcpy(bt->order, ord.data(), count * sizeof(int), hipMemcpyHostToDevice);
            if (e != hipSuccess) { g_last_hip = hipGetErrorString(e); r = SSCS_E_HIP; }
        }
        if (r == SSCS_OK) {
            int dev = 0, ncu = 0, occ = 0, rate = 0;
            hipGetDevice(&dev);
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
            long long big = 0;
            for (int i = 0; i < count; ++i) {
                const long long e = (long long)bt->inst[i].n + bt->inst[i].m;
                if (e <= kStageMax) big = std::max(big, e);
            }
            bt->stage = stage_doubles(big);
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k_solve_batch<double>, kBatchBlock,
                                                         bt->stage * sizeof(double));
            hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, dev);
            bt->ticks_per_s = rate > 0 ? rate * 1000.0 : 1e8;
            bt->grid = std::max(1, std::min(count, ncu * std::max(1, occ)));
            hipError_t e = hipStreamSynchronize(bt->stream);
            if (e != hipSuccess) { g_last_hip = hipGetErrorString(e); r = SSCS_E_HIP; }
        }
        if (r != SSCS_OK) { sscs_batch_destroy(bt); return r; }
        bt->setup_s = now_s() - t0;
        *out = bt;
        return SSCS_OK;
    } catch (...) {
        return SSCS_E_NOMEM;
    }
}

int sscs_batch_update_bc(sscs_batch* bt, const double* b_packed, const double* c_packed) {
    if (!bt || !b_packed || !c_packed) return SSCS_E_INVALID;
    const hipMemcpyKind kind = bt->st.data_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    for (int i = 0; i < bt->count; ++i) {
        Inst& I = bt->inst[i];
        HIP_TRY(hipMemcpyAsync(I.b, b_packed + bt->off_y[i], I.m * sizeof(double), kind, bt->stream));
        HIP_TRY(hipMemcpyAsync(I.c, c_packed + bt->off_x[i], I.n * sizeof(double), kind, bt->stream));
    }
    HIP_TRY(hipStreamSynchronize(bt->stream));
    return SSCS_OK;
}

int sscs_batch_solve(sscs_batch* bt, const double* u0_packed, double* x_packed, double* y_packed,
                     double* s_packed, sscs_info* infos) {
    if (!bt || !x_packed || !y_packed || !s_packed) return SSCS_E_INVALID;
    const double t0 = now_s();
    const bool dev = bt->st.data_on_device != 0;
    double* dio_u = bt->io;
    double* dio_x = dio_u + bt->tot_u;
    double* dio_y = dio_x + bt->tot_x;
    double* dio_s = dio_y + bt->tot_y;
    const double* du0 = nullptr;
    if (u0_packed) {
        if (dev) du0 = u0_packed;
        else {
            HIP_TRY(hipMemcpyAsync(dio_u, u0_packed, bt->tot_u * sizeof(double), hipMemcpyHostToDevice, bt->stream));
            du0 = dio_u;
        }
    }
    double* ox = dev ? x_packed : dio_x;
    double* oy = dev ? y_packed : dio_y;
    double* os = dev ? s_packed : dio_s;
    for (int i = 0; i < bt->count; ++i) {
        Vecs& V = bt->h_insts[i].V;
        V.u0 = du0 ? du0 + bt->off_u[i] : nullptr;
        V.out_x = ox + bt->off_x[i];
        V.out_y = oy + bt->off_y[i];
        V.out_s = os + bt->off_y[i];
        V.tr_res = nullptr; V.tr_kind = nullptr; V.tr_ls = nullptr; V.tr_cap = 0;
        V.tr_eta = nullptr; V.tr_rsafe = nullptr;
    }
    HIP_TRY(hipMemcpyAsync(bt->d_insts, bt->h_insts.data(), bt->count * sizeof(BatchInst), hipMemcpyHostToDevice,
                           bt->stream));
    HIP_TRY(hipMemsetAsync(bt->queue, 0, sizeof(int), bt->stream));
    Params S = make_params(bt->st, bt->ticks_per_s);
    const size_t lds = bt->stage * sizeof(double);
    k_solve_batch<double><<<bt->grid, kBatchBlock, lds, bt->stream>>>(bt->d_insts, bt->order, bt->count, bt->count,
                                                                      S, bt->res, bt->queue, bt->stage);
    HIP_TRY(hipGetLastError());
    if (!dev) {
        HIP_TRY(hipMemcpyAsync(x_packed, dio_x, bt->tot_x * sizeof(double), hipMemcpyDeviceToHost, bt->stream));
        HIP_TRY(hipMemcpyAsync(y_packed, dio_y, bt->tot_y * sizeof(double), hipMemcpyDeviceToHost, bt->stream));
        HIP_TRY(hipMemcpyAsync(s_packed, dio_s, bt->tot_y * sizeof(double), hipMemcpyDeviceToHost, bt->stream));
    }
    std::vector<Result> r(bt->count);
    HIP_TRY(hipMemcpyAsync(r.data(), bt->res, bt->count * sizeof(Result), hipMemcpyDeviceToHost, bt->stream));
    HIP_TRY(hipStreamSynchronize(bt->stream));
    const double el = now_s() - t0;
    if (infos)
        for (int i = 0; i < bt->count; ++i) fill_info(&infos[i], r[i], bt->setup_s, el);
    return SSCS_OK;
}

int sscs_batch_autotune(sscs_batch* bt, int32_t iters, int32_t cap, int32_t* n_classes, int32_t* class_seg,
                        int32_t* chosen_seg, double* ms) {
    if (!bt || iters < 1 || cap < 0 || !n_classes) return SSCS_E_INVALID;
    // classes: the width the mean-row-length rule gives each instance's A
    std::map<int, std::vector<int>> cls;
    for (int i = 0; i < bt->count; ++i) cls[bt->inst[i].segA].push_back(i);
    *n_classes = (int32_t)cls.size();
    int* d_ord = nullptr;
    TRY(dmalloc(&d_ord, bt->count));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int r = SSCS_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) r = SSCS_E_HIP;
    // timing runs: cold starts, outputs to the staging buffers, a fixed
    // iteration count (eps 0: no instance stops early)
    sscs_settings st = bt->st;
    st.max_iters = iters;
    st.eps = 0.0;
    st.max_time_s = 0.0;
    const Params S = make_params(st, bt->ticks_per_s);
    for (int i = 0; i < bt->count; ++i) {
        Vecs& V = bt->h_insts[i].V;
        V.u0 = nullptr;
        V.out_x = bt->io + bt->tot_u + bt->off_x[i];
        V.out_y = bt->io + bt->tot_u + bt->tot_x + bt->off_y[i];
        V.out_s = bt->io + bt->tot_u + bt->tot_x + bt->tot_y + bt->off_y[i];
        V.tr_res = nullptr; V.tr_kind = nullptr; V.tr_ls = nullptr; V.tr_cap = 0;
        V.tr_eta = nullptr; V.tr_rsafe = nullptr;
    }
    auto set_width = [&](const std::vector<int>& ids, int f2) {   // width x 2^f2, within 1..64
        for (int i : ids) {
            const Inst& I = bt->inst[i];
            auto scale = [&](int w) { return f2 >= 0 ? std::min(64, w << f2) : std::max(1, w >> -f2); };
            bt->h_insts[i].P.A.seg = scale(I.segA);
            bt->h_insts[i].P.At.seg = scale(I.segAt);
        }
    };
    auto run = [&](const std::vector<int>& ids, float* out_ms) -> int {
        HIP_TRY(hipMemcpyAsync(bt->d_insts, bt->h_insts.data(), bt->count * sizeof(BatchInst),
                               hipMemcpyHostToDevice, bt->stream));
        HIP_TRY(hipMemcpyAsync(d_ord, ids.data(), ids.size() * sizeof(int), hipMemcpyHostToDevice, bt->stream));
        HIP_TRY(hipMemsetAsync(bt->queue, 0, sizeof(int), bt->stream));
        HIP_TRY(hipEventRecord(e0, bt->stream));
        k_solve_batch<double><<<bt->grid, kBatchBlock, bt->stage * sizeof(double), bt->stream>>>(
            bt->d_insts, d_ord, bt->count, (int)ids.size(), S, bt->res, bt->queue, bt->stage);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipEventRecord(e1, bt->stream));
        HIP_TRY(hipEventSynchronize(e1));
        HIP_TRY(hipEventElapsedTime(out_ms, e0, e1));
        return SSCS_OK;
    };
    int c = 0;
    for (auto it = cls.begin(); it != cls.end() && r == SSCS_OK; ++it, ++c) {
        const int w0 = it->first;
        const std::vector<int>& ids = it->second;
        float t = 0.0f;
        double best = 1e300;
        int best_f = 0;
        set_width(ids, 0);
        r = run(ids, &t);                       // warm-up at the rule's width
        for (int f2 = -2; f2 <= 2 && r == SSCS_OK; ++f2) {
            const int w = f2 >= 0 ? (w0 << f2) : (w0 >> -f2);
            const bool in = w >= 1 && w <= 64 && (f2 >= 0 || (w << -f2) == w0);
            double tm = -1.0;
            if (in) {                           // the better of two timed runs
                set_width(ids, f2);
                float t1 = 0.0f, t2 = 0.0f;
                r = run(ids, &t1);
                if (r == SSCS_OK) r = run(ids, &t2);
                tm = std::min(t1, t2);
                if (r == SSCS_OK && tm < best) { best = tm; best_f = f2; }
            }
            if (ms && c < cap) ms[c * 5 + (f2 + 2)] = tm;
        }
        set_width(ids, best_f);
        if (c < cap) {
            if (class_seg) class_seg[c] = w0;
            if (chosen_seg) chosen_seg[c] = best_f >= 0 ? std::min(64, w0 << best_f) : std::max(1, w0 >> -best_f);
        }
    }
    if (r == SSCS_OK) {
        hipError_t e = hipMemcpyAsync(bt->d_insts, bt->h_insts.data(), bt->count * sizeof(BatchInst),
                                      hipMemcpyHostToDevice, bt->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(bt->stream);
        if (e != hipSuccess) { g_last_hip = hipGetErrorString(e); r = SSCS_E_HIP; }
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipFree(d_ord);
    return r;
}

}  // extern "C"

// ------------------------------------------------------------------ allocation-free one-shot solve
//
// sscs_solve_noalloc: the one-instance batched solve (sscs_batch_create +
// sscs_batch_solve + sscs_batch_destroy for count = 1, the same kernels) with
// every device buffer carved from one file-scope device array instead of
// hipMalloc'd memory.  Each GPU holds its own copy of the array until the
// process ends; calls on one GPU share it, so calls that overlap on one GPU
// race (one call at a time per GPU).

namespace {
constexpr size_t kScratchBytes = size_t(32) << 20;      // 32 MiB per GPU
}  // namespace

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, looked up once per
// device with that device current.  In host code the array's name is only a
// host-side handle, never a device address.
int scratch_base(double** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        g_unsupported = "device index beyond the scratch table";
        return SSCS_E_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            g_last_hip = "hipGetSymbolAddress returned no address for the scratch array";
            return SSCS_E_HIP;
        }
        g_scratch_dev[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_dev[dev];
    return SSCS_OK;
}

// Bump allocator over the scratch array (256-byte aligned pieces); only
// computes offsets, so running it with base = nullptr gives the footprint.
struct Carver {
    char* base;
    size_t off = 0;
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += std::max<size_t>(count, 1) * sizeof(T);
        return p;
    }
};

__global__ void k_fill_int(int* __restrict__ a, long long n, int v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        a[i] = v;
}

// Cone offset tables from the block sizes (one thread: the tables of one
// instance are short).
__global__ void k_cone_tables(const int* __restrict__ q, int nq, const int* __restrict__ s, int ns,
                              int* __restrict__ qoff, int* __restrict__ soff) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int run = 0;
    qoff[0] = 0;
    for (int i = 0; i < nq; ++i) { run += q[i]; qoff[i + 1] = run; }
    run = 0;
    soff[0] = 0;
    for (int i = 0; i < ns; ++i) { run += s[i] * (s[i] + 1) / 2; soff[i + 1] = run; }
}

// Ascending list of the rows longer than thr nonzeros (one workgroup; each
// chunk of rows is compacted with a prefix sum of its flags); *count gets the
// list length.
__global__ void __launch_bounds__(256) k_long_rows(const int* __restrict__ rp, int rows, int thr,
                                                   int* __restrict__ out, int* __restrict__ count) {
    __shared__ int flag[256];
    int base = 0;
    for (int r0 = 0; r0 < rows; r0 += blockDim.x) {
        const int r = r0 + threadIdx.x;
        const int f = (r < rows && rp[r + 1] - rp[r] > thr) ? 1 : 0;
        flag[threadIdx.x] = f;
        __syncthreads();
        for (int o = 1; o < (int)blockDim.x; o <<= 1) {
            const int v = threadIdx.x >= (unsigned)o ? flag[threadIdx.x - o] : 0;
            __syncthreads();
            flag[threadIdx.x] += v;
            __syncthreads();
        }
        if (f) out[base + flag[threadIdx.x] - 1] = r;
        const int tot = flag[blockDim.x - 1];
        __syncthreads();
        base += tot;
    }
    if (threadIdx.x == 0) *count = base;
}

}  // namespace

extern "C" {

int sscs_solve_noalloc(const sscs_data* data, const sscs_cone* cone, const sscs_settings* st, void* hip_stream,
                       const double* u0, double* x, double* y, double* s, sscs_info* info) {
    try {
        g_unsupported = nullptr;
        if (!x || !y || !s) return SSCS_E_INVALID;
        TRY(validate(data, cone));
        TRY(validate_settings(st));
        if (st->precision != SSCS_PREC_FP64) {                      // as the batched engine
            g_unsupported = "sscs_solve_noalloc runs the FP64 operator only";
            return SSCS_E_UNSUPPORTED;
        }
        if (st->linsys != SSCS_LINSYS_CG) {
            g_unsupported = "sscs_solve_noalloc runs the CG linear step only";
            return SSCS_E_UNSUPPORTED;
        }
        int kmax = 0;
        long long qsum = 0;
        for (int i = 0; i < cone->ns; ++i) kmax = std::max(kmax, cone->s[i]);
        for (int i = 0; i < cone->nq; ++i) qsum += cone->q[i];
        if (kmax > 64) {
            g_unsupported = "sscs_solve_noalloc takes PSD blocks up to order 64";
            return SSCS_E_UNSUPPORTED;
        }
        const double t0 = now_s();
        const hipStream_t strm = (hipStream_t)hip_stream;
        const int n = data->n, m = data->m, N = n + m + 1, mem = st->mem;
        const long long nnz = data->nnz;
        const bool dev = st->data_on_device != 0;
        // layout of the scratch array for this instance (footprint first)
        auto carve_all = [&](Carver& c, Inst& I, BatchInst** bi, int** order, int** queue, Result** res,
                             int** qsz, int** ssz, int** cnt, int** nlong, double** vec, double** io) {
            *res = c.take<Result>(1);
            *bi = c.take<BatchInst>(1);
            *order = c.take<int>(1);
            *queue = c.take<int>(1);
            *nlong = c.take<int>(2);
            I.A_rp = c.take<int>(m + 1);
            I.A_ci = c.take<int>(nnz);
            I.A_v = c.take<double>(nnz);
            I.At_rp = c.take<int>(n + 1);
            I.At_ci = c.take<int>(nnz);
            I.At_v = c.take<double>(nnz);
            I.A_long = c.take<int>(m);
            I.At_long = c.take<int>(n);
            *cnt = c.take<int>(n);
            I.dinv = c.take<double>(n);
            I.b = c.take<double>(m);
            I.c = c.take<double>(n);
            I.g = c.take<double>(n + m);
            *qsz = c.take<int>(cone->nq);
            *ssz = c.take<int>(cone->ns);
            I.qoff = c.take<int>(cone->nq + 1);
            I.sord = *ssz;
            I.soff = c.take<int>(cone->ns + 1);
            I.K.psd_scratch = cone->ns > 0 ? c.take<double>(psd_scratch_doubles(kmax)) : nullptr;
            *vec = c.take<double>(vec_doubles(n, m, mem));
            *io = dev ? nullptr : c.take<double>((size_t)N + n + 2 * (size_t)m);
        };
        {
            Carver probe{nullptr};
            Inst I;
            BatchInst* bi; int *order, *queue, *qsz, *ssz, *cnt, *nlong; Result* res; double *vec, *io;
            carve_all(probe, I, &bi, &order, &queue, &res, &qsz, &ssz, &cnt, &nlong, &vec, &io);
            if (probe.off > kScratchBytes) {
                g_unsupported = "the instance does not fit the 32 MiB device scratch of sscs_solve_noalloc";
                return SSCS_E_UNSUPPORTED;
            }
        }
        double* base = nullptr;
        TRY(scratch_base(&base));
        Carver cv{reinterpret_cast<char*>(base)};
        Inst I;
        BatchInst* d_bi; int *d_order, *d_queue, *d_qsz, *d_ssz, *d_cnt, *d_nlong; Result* d_res; double *d_vec, *d_io;
        carve_all(cv, I, &d_bi, &d_order, &d_queue, &d_res, &d_qsz, &d_ssz, &d_cnt, &d_nlong, &d_vec, &d_io);
        I.m = m; I.n = n; I.N = N; I.nnz = nnz; I.owns_A = false;
        // problem data in (the caller's host arrays, as sscs_create takes them)
        HIP_TRY(hipMemcpyAsync(I.A_rp, data->rowptr, (m + 1) * sizeof(int), hipMemcpyHostToDevice, strm));
        if (nnz) {
            HIP_TRY(hipMemcpyAsync(I.A_ci, data->colind, nnz * sizeof(int), hipMemcpyHostToDevice, strm));
            HIP_TRY(hipMemcpyAsync(I.A_v, data->val, nnz * sizeof(double), hipMemcpyHostToDevice, strm));
        }
        HIP_TRY(hipMemcpyAsync(I.b, data->b, m * sizeof(double), hipMemcpyHostToDevice, strm));
        HIP_TRY(hipMemcpyAsync(I.c, data->c, n * sizeof(double), hipMemcpyHostToDevice, strm));
        if (cone->nq) HIP_TRY(hipMemcpyAsync(d_qsz, cone->q, cone->nq * sizeof(int), hipMemcpyHostToDevice, strm));
        if (cone->ns) HIP_TRY(hipMemcpyAsync(d_ssz, cone->s, cone->ns * sizeof(int), hipMemcpyHostToDevice, strm));
        // A^T and the Jacobi diagonal: the kernels and launch shapes of upload_instance;
        // counters cleared by a fill kernel (the array keeps the previous call's contents)
        const int fb = (int)std::min<long long>(4096, (n + 255) / 256 + 1);
        k_fill_int<<<fb, 256, 0, strm>>>(d_cnt, n, 0);
        if (nnz) k_count_cols<<<std::min<long long>(4096, (nnz + 255) / 256), 256, 0, strm>>>(I.A_ci, nnz, d_cnt);
        k_scan<<<1, 1024, 0, strm>>>(d_cnt, n, I.At_rp);
        k_fill_int<<<fb, 256, 0, strm>>>(d_cnt, n, 0);
        k_scatter_t<<<std::min(4096, (m + 255) / 256), 256, 0, strm>>>(I.A_rp, I.A_ci, I.A_v, m, I.At_rp, d_cnt,
                                                                       I.At_ci, I.At_v);
        k_sort_rows<<<std::min(4096, (n + 255) / 256), 256, 0, strm>>>(I.At_rp, n, I.At_ci, I.At_v, I.dinv);
        I.segA = pow2_seg((double)nnz / std::max(1, m));
        I.segAt = pow2_seg((double)nnz / std::max(1, n));
        I.lthrA = 64 * I.segA;
        I.lthrAt = 64 * I.segAt;
        k_long_rows<<<1, 256, 0, strm>>>(I.A_rp, m, I.lthrA, I.A_long, d_nlong);
        k_long_rows<<<1, 256, 0, strm>>>(I.At_rp, n, I.lthrAt, I.At_long, d_nlong + 1);
        k_cone_tables<<<1, 1, 0, strm>>>(d_qsz, cone->nq, d_ssz, cone->ns, I.qoff, I.soff);
        HIP_TRY(hipGetLastError());
        int nl[2] = {0, 0};
        HIP_TRY(hipMemcpyAsync(nl, d_nlong, sizeof(nl), hipMemcpyDeviceToHost, strm));
        HIP_TRY(hipStreamSynchronize(strm));
        I.nlongA = nl[0];
        I.nlongAt = nl[1];
        I.K.z = cone->z; I.K.l = cone->l; I.K.nq = cone->nq; I.K.qoff = I.qoff;
        I.K.ns = cone->ns; I.K.sord = I.sord; I.K.soff = I.soff; I.K.ep = cone->ep;
        I.K.soc0 = cone->z + cone->l;
        I.K.psd0 = I.K.soc0 + (int)qsum;
        long long psum = 0;
        for (int i = 0; i < cone->ns; ++i) psum += (long long)cone->s[i] * (cone->s[i] + 1) / 2;
        I.K.exp0 = I.K.psd0 + (int)psum;
        I.K.psd_kmax = kmax;
        I.K.psd_team = nullptr; I.K.psd_vecs = nullptr; I.K.psd_warm = nullptr;
        // the instance record of the batched kernel
        BatchInst h{};
        h.P = make_prob(I);
        h.V = carve(d_vec, n, m, mem);
        const double* du0 = nullptr;
        if (u0) {
            if (dev) du0 = u0;
            else {
                HIP_TRY(hipMemcpyAsync(d_io, u0, N * sizeof(double), hipMemcpyHostToDevice, strm));
                du0 = d_io;
            }
        }
        h.V.u0 = du0;
        h.V.out_x = dev ? x : d_io + N;
        h.V.out_y = dev ? y : d_io + N + n;
        h.V.out_s = dev ? s : d_io + N + n + m;
        h.V.tr_res = nullptr; h.V.tr_kind = nullptr; h.V.tr_ls = nullptr; h.V.tr_cap = 0;
        h.V.tr_eta = nullptr; h.V.tr_rsafe = nullptr;
        HIP_TRY(hipMemcpyAsync(d_bi, &h, sizeof(h), hipMemcpyHostToDevice, strm));
        k_fill_int<<<1, 64, 0, strm>>>(d_order, 1, 0);
        k_fill_int<<<1, 64, 0, strm>>>(d_queue, 1, 0);
        int dv = 0, rate = 0;
        HIP_TRY(hipGetDevice(&dv));
        HIP_TRY(hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, dv));
        Params P = make_params(*st, rate > 0 ? rate * 1000.0 : 1e8);
        const int stage = stage_doubles((long long)n + m);
        k_solve_batch<double><<<1, kBatchBlock, stage * sizeof(double), strm>>>(d_bi, d_order, 1, 1, P, d_res,
                                                                                d_queue, stage);
        HIP_TRY(hipGetLastError());
        if (!dev) {
            HIP_TRY(hipMemcpyAsync(x, d_io + N, n * sizeof(double), hipMemcpyDeviceToHost, strm));
            HIP_TRY(hipMemcpyAsync(y, d_io + N + n, m * sizeof(double), hipMemcpyDeviceToHost, strm));
            HIP_TRY(hipMemcpyAsync(s, d_io + N + n + m, m * sizeof(double), hipMemcpyDeviceToHost, strm));
        }
        Result r{};
        HIP_TRY(hipMemcpyAsync(&r, d_res, sizeof(Result), hipMemcpyDeviceToHost, strm));
        HIP_TRY(hipStreamSynchronize(strm));
        const double el = now_s() - t0;
        fill_info(info, r, 0.0, el);
        return SSCS_OK;
    } catch (...) {
        return SSCS_E_NOMEM;
    }
}

}  // extern "C"
