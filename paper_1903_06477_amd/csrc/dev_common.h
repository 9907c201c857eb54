// Device building blocks shared by every kernel of libsscs (gfx950, wave64).
//
// A "team" is the set of threads that cooperates on one problem instance:
//   GridTeam  -- every thread of a cooperatively launched grid (one large instance);
//   BlockTeam -- the threads of one workgroup (one instance of a batch).
// Both expose the same interface, so the solver code in dev_engine.h is
// written once:
//   rank()/size()         thread index within the team and team size
//   wave()/nwaves()       wavefront index within the team and their number
//   blk()/nblk()          workgroup index within the team and their number
//   sync()                barrier over the team (grid barrier or __syncthreads)
//   reduce(sh, K)         sums K per-wave partials (written with put()) over the
//                         team; every thread then reads the totals in sh.out[0..K)
// Reductions are deterministic: partial sums are always combined in the same
// order, so every workgroup of a grid computes bit-identical totals and all
// control decisions derived from them agree across the grid.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <stdint.h>

namespace sscs {

constexpr int WAVE = 64;
constexpr int NWMAX = 16;      // waves per workgroup (<= 1024 threads)
constexpr int KMAX = 72;       // values per reduction
constexpr int MEMMAX = 16;     // quasi-Newton memory

// Per-workgroup LDS state.
struct Shared {
    double red[KMAX * NWMAX];   // per-wave partials
    double out[KMAX];           // reduction totals (broadcast)
    double G[MEMMAX * MEMMAX];  // Anderson Gram matrix Xi^T Xi (slot-indexed)
    double W[MEMMAX * MEMMAX];  // restarted Broyden inner products <z_i, zt_j>
    double coef[4 * MEMMAX + 8];
    double L[MEMMAX * MEMMAX];  // small factorisations (one thread)
    double term[12];            // termination measures of the current iteration
    int    qhead;               // batched engine: instance popped from the queue
};

// v of another lane by a data-parallel-primitive move (both halves with the
// same control); lanes of rows outside ROWM receive 0.
template <int CTRL, int ROWM>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWM, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWM, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Sum over aligned groups of S lanes (S a power of two, uniform over the
// wave), by moves within quads, half-rows and rows, then the broadcasts of a
// row's last lane into the next row: the group's total is in its last lane
// (S - 1), and in all of its lanes for S <= 16.  Moves that stay inside the
// group keep groups independent, so a group whose lanes are all active may sum
// while others of the wave are not.
__device__ __forceinline__ double group_sum(double v, int S) {
    if (S >= 2) v += dpp_f64<0xB1, 0xf>(v);      // quad_perm [1,0,3,2]
    if (S >= 4) v += dpp_f64<0x4E, 0xf>(v);      // quad_perm [2,3,0,1]
    if (S >= 8) v += dpp_f64<0x141, 0xf>(v);     // row_half_mirror
    if (S >= 16) v += dpp_f64<0x140, 0xf>(v);    // row_mirror
    if (S >= 32) v += dpp_f64<0x142, 0xa>(v);    // row_bcast:15 into rows 1 and 3
    if (S >= 64) v += dpp_f64<0x143, 0xc>(v);    // row_bcast:31 into rows 2 and 3
    return v;
}

// Sum over the wave, returned to every lane (all lanes must be active).
__device__ __forceinline__ double wave_sum(double v) {
    v = group_sum(v, WAVE);
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), WAVE - 1);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), WAVE - 1);
    return __hiloint2double(hi, lo);
}

// A double in LDS (address space 3).
typedef __attribute__((address_space(3))) double lds_f64;

// Writes the wave-sum of v into slot k of the per-wave partials.  (Shared
// always lives in LDS: the kernels declare it __shared__.  Its fields are
// reached through LDS-typed pointers where the callers hold a plain
// reference, which would otherwise compile to generic accesses.)
__device__ __forceinline__ void put(Shared& sh, int k, double v) {
    v = group_sum(v, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == WAVE - 1) ((lds_f64*)sh.red)[k * NWMAX + (threadIdx.x / WAVE)] = v;
}

// Sums the per-wave partials of slot k in wave order.
__device__ __forceinline__ double block_total(const Shared& sh, int k) {
    const int nw = blockDim.x / WAVE;
    const lds_f64* red = (const lds_f64*)sh.red;
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[k * NWMAX + w];
    return s;
}

// The rows of one matrix (A or A^T) that a workgroup owns, and where they
// live: in global memory, or copied into the workgroup's LDS (offsets in bytes
// into the dynamic LDS segment) for the lifetime of a persistent kernel.
struct MatPart {
    int r0, rows;     // first global row, row count
    int lds;          // 1: values, column indices and row pointers are in LDS
    int off_v, off_ci, off_rp;
};

extern __shared__ __attribute__((aligned(16))) double sscs_dyn_lds[];

// Vectors a kernel holds in LDS but reaches through generic pointers (shared
// descriptors) are cast back to LDS pointers where the code knows they live
// there: LDS instructions then replace flat ones, which take the longer
// vector-memory path even for LDS addresses.
template <bool L> struct VecPtr { using type = double*; };
template <> struct VecPtr<true> { using type = lds_f64*; };
template <bool L>
__device__ __forceinline__ typename VecPtr<L>::type vec_at(const double* p) {
    if constexpr (L) return (lds_f64*)const_cast<double*>(p);
    else return const_cast<double*>(p);
}

// One workgroup; LDS: the operator (A and A^T, FP64) is held in LDS.
template <bool LDS>
struct BlockTeamT {
    static constexpr bool kLds = LDS;
    static constexpr bool kBlock = true;
    static constexpr bool kPsdTeam = false;
    using lds_t = double;
    MatPart mp[2];    // A, A^T: all rows (global memory, or LDS)
    double* lu = nullptr;   // LDS copies of the CG's gathered vectors (n and m
    double* lt = nullptr;   // entries), or null when they do not fit
    __device__ int rank() const { return threadIdx.x; }
    __device__ int size() const { return blockDim.x; }
    __device__ int wave() const { return threadIdx.x / WAVE; }
    __device__ int nwaves() const { return blockDim.x / WAVE; }
    __device__ int blk() const { return 0; }
    __device__ int nblk() const { return 1; }
    __device__ bool aborted() const { return false; }
    __device__ void sync() { __syncthreads(); }
    __device__ void reduce(Shared& sh, int K) {
        __syncthreads();
        for (int k = threadIdx.x; k < K; k += blockDim.x) sh.out[k] = block_total(sh, k);
        __syncthreads();
    }
};
using BlockTeam = BlockTeamT<false>;

// Words of the grid barrier, each on its own 128-byte line: the global
// arrival counter, one arrival counter and one release word per group, one
// workgroup count per group and the set-up counter.  Groups are the XCDs
// (the hardware XCC_ID, four bits).  From BAR_SUB, the same words (less the
// set-up counter) of a second barrier among a subset of the workgroups (the
// PSD sub-team, PsdSubTeam).
constexpr int BAR_STRIDE = 16;
constexpr int BAR_GROUPS = 16;
constexpr int BAR_SUB = BAR_STRIDE * (2 + 3 * BAR_GROUPS);
constexpr int BAR_WORDS = BAR_SUB + BAR_STRIDE * (1 + 3 * BAR_GROUPS);

// The XCD (accelerator complex die) the calling wave runs on.
__device__ __forceinline__ unsigned xcc_id() {
    return __builtin_amdgcn_s_getreg(20 | (0 << 6) | ((16 - 1) << 11)) & 0xF;   // HW_REG_XCC_ID, bits 0..15
}

// Waits with relaxed loads (an acquiring load per poll would invalidate the
// caches the rest of the grid is working from); the caller orders what
// follows.  False when the wait timed out or the grid aborted.
__device__ __forceinline__ bool spin_until(unsigned long long* addr, unsigned long long target, int* abort_flag,
                                           long long timeout_ticks) {
    const long long t0 = wall_clock64();
    while (__hip_atomic_load(addr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
        __builtin_amdgcn_s_sleep(1);
        if (wall_clock64() - t0 > timeout_ticks) {
            __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
    return true;
}

// After a team reduction's barrier: sh.out[k] = sum over j in [j0, G) of
// p[k * G + j], k < K, summed by every workgroup in the same fixed order (lane
// l adds entries l, l + 64, ... in turn, then the wavefront sum).  A
// wavefront issues the loads of kR sums by kJ entries per lane before adding
// any, so they are in flight together: after the barrier the partials come
// from the memory-side cache, and one round trip per sum in turn cost
// microseconds.  Out of line, so its registers stay out of the callers'.
__device__ __noinline__ void sum_partials(Shared& sh, const double* p, int K, int G, int j0) {
    constexpr int kR = 3, kJ = 4;
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    for (int k0 = w; k0 < K; k0 += kR * nw) {
        double acc[kR];
#pragma unroll
        for (int r = 0; r < kR; ++r) acc[r] = 0.0;
        for (int jb = j0 + lane; jb < G; jb += kJ * WAVE) {
            double v[kR][kJ];
#pragma unroll
            for (int r = 0; r < kR; ++r)
#pragma unroll
                for (int q = 0; q < kJ; ++q) {
                    const int k = k0 + r * nw, j = jb + q * WAVE;
                    v[r][q] = (k < K && j < G) ? p[(size_t)k * G + j] : 0.0;
                }
#pragma unroll
            for (int r = 0; r < kR; ++r)
#pragma unroll
                for (int q = 0; q < kJ; ++q)
                    if (jb + q * WAVE < G) acc[r] += v[r][q];
        }
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const int k = k0 + r * nw;
            const double t = wave_sum(acc[r]);
            if (k < K && lane == 0) sh.out[k] = t;
        }
    }
}

// Thread 0's part of the k-th barrier among a team with `members` workgroups
// on this workgroup's XCD `grp` and `ngrp` XCDs in all, on the words from
// `base` (laid out as at BAR_WORDS); see GridTeam::sync.
__device__ __forceinline__ void xcd_barrier(unsigned long long* base, unsigned grp, unsigned long long members,
                                            unsigned ngrp, unsigned long long k, int* abort_flag,
                                            long long timeout_ticks) {
    unsigned long long* cnt = base + BAR_STRIDE * (1 + grp);
    unsigned long long* rel = base + BAR_STRIDE * (1 + BAR_GROUPS + grp);
    const unsigned long long old = __hip_atomic_fetch_add(cnt, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old + 1 == k * members) {
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");     // the XCD's L2 written back
        __hip_atomic_fetch_add(base, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        spin_until(base, k * ngrp, abort_flag, timeout_ticks);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");     // and the other XCDs' data acquired
        __hip_atomic_store(rel, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        spin_until(rel, k, abort_flag, timeout_ticks);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
}

// Two-level grid barrier over the XCDs.  Each XCD has its own L2, which is
// not coherent with the others'.  An agent-scope release writes the L2's
// dirty lines back, which costs about the same whichever workgroup of the XCD
// issues it, so only one workgroup per XCD does:
//   * every wave waits until its own stores are acknowledged (they are then in
//     the XCD's L2), the workgroup joins, and its first thread counts itself
//     in at its XCD's arrival counter (relaxed atomic);
//   * the last arrival of an XCD writes the L2 back (agent release), bumps the
//     global counter, waits for every XCD, acquires (L1 and L2 invalidated)
//     and stores the barrier's number into its XCD's release word;
//   * the other workgroups of the XCD wait for that word, then acquire at
//     agent scope themselves: their CU's L1 may hold stale lines, and the
//     only invalidation that reaches the L1 outside thread-group-split mode
//     is the agent-scope one (a workgroup-scope invalidate leaves it as is).
// Measured on 256 workgroups with 1 MiB written per phase: 4.8 us per
// barrier, against 8.6 us when every workgroup also writes the L2 back.
// Groups come from the hardware XCC_ID, counted once at kernel start (set_up),
// not from an assumed placement of workgroups.  All counters grow
// monotonically (the k-th barrier completes at k * members), so nothing is
// reset inside the kernel.  A wait that exceeds `timeout_ticks` of the wall
// clock raises the abort flag; later barriers then return at once, so every
// wave of the grid still reaches the kernel's end.
// PT: the form that projects PSD blocks above order 64 with the whole team;
// instances without such blocks run the form without that code, so the
// registers its call tree takes do not cost the solve kernel spills.
template <bool LDS, typename TL = double, bool PT = true>
struct GridTeam {
    static constexpr bool kLds = LDS;   // operator rows held in LDS ...
    using lds_t = TL;                   // ... with values of this type
    static constexpr bool kBlock = false;
    static constexpr bool kPsdTeam = PT;
    MatPart mp[2];              // this workgroup's rows of A and A^T
    unsigned long long* bar;    // BAR_WORDS words, zero at launch
    int* abort_flag;
    double* part;               // [4][KMAX][gridDim.x] partials (2 and 3: the PSD sub-team's)
    unsigned long long k;       // barriers passed so far
    long long timeout_ticks;
    int flip;
    unsigned grp, ngrp;         // this workgroup's XCD; XCDs the grid occupies
    unsigned long long members; // workgroups on this XCD
    // the PSD sub-team (workgroups sub0 .. gridDim.x - 1; none when sub0 is 0):
    // its workgroups on this XCD, its XCDs, its barriers passed, its partials' buffer
    int sub0 = 0;
    unsigned long long sub_members = 0;
    unsigned sub_ngrp = 0;
    unsigned long long sub_k = 0;
    int sub_flip = 0;

    __device__ int rank() const { return blockIdx.x * blockDim.x + threadIdx.x; }
    __device__ int size() const { return gridDim.x * blockDim.x; }
    __device__ int wave() const { return rank() / WAVE; }
    __device__ int nwaves() const { return size() / WAVE; }
    __device__ int blk() const { return blockIdx.x; }
    __device__ int nblk() const { return gridDim.x; }

    __device__ bool aborted() const {
        return __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    }

    // Counts the workgroups per XCD, of the grid and of the PSD sub-team
    // (workgroups from `sub_start`, none when 0), in one fully fenced
    // rendezvous of the grid.
    __device__ void set_up(int sub_start = 0) {
        __shared__ unsigned s_grp, s_ngrp, s_sub_ngrp;
        __shared__ unsigned long long s_members, s_sub_members;
        unsigned long long* cnt = bar + BAR_STRIDE * (1 + 2 * BAR_GROUPS);
        unsigned long long* scnt = bar + BAR_SUB + BAR_STRIDE * (1 + 2 * BAR_GROUPS);
        unsigned long long* arrived = bar + BAR_STRIDE * (1 + 3 * BAR_GROUPS);
        if (threadIdx.x == 0) {
            const unsigned x = xcc_id();
            __hip_atomic_fetch_add(cnt + BAR_STRIDE * x, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (sub_start > 0 && (int)blockIdx.x >= sub_start)
                __hip_atomic_fetch_add(scnt + BAR_STRIDE * x, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_fetch_add(arrived, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            spin_until(arrived, gridDim.x, abort_flag, timeout_ticks);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            unsigned ng = 0, sng = 0;
            for (int i = 0; i < BAR_GROUPS; ++i) {
                ng += __hip_atomic_load(cnt + BAR_STRIDE * i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? 1u : 0u;
                sng += __hip_atomic_load(scnt + BAR_STRIDE * i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? 1u : 0u;
            }
            s_grp = x;
            s_ngrp = ng;
            s_sub_ngrp = sng;
            s_members = __hip_atomic_load(cnt + BAR_STRIDE * x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_sub_members = __hip_atomic_load(scnt + BAR_STRIDE * x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        grp = s_grp;
        ngrp = s_ngrp;
        members = s_members;
        sub0 = sub_start;
        sub_ngrp = s_sub_ngrp;
        sub_members = s_sub_members;
        __syncthreads();
    }

    __device__ void sync() {
        __builtin_amdgcn_s_waitcnt(0);          // this wave's stores acknowledged (in the XCD's L2)
        __syncthreads();
        ++k;
        if (threadIdx.x == 0) xcd_barrier(bar, grp, members, ngrp, k, abort_flag, timeout_ticks);
        __syncthreads();
    }

    __device__ void reduce(Shared& sh, int K) {
        __syncthreads();
        const int G = gridDim.x;
        double* p = part + (size_t)flip * KMAX * G;
        for (int k = threadIdx.x; k < K; k += blockDim.x) p[(size_t)k * G + blockIdx.x] = block_total(sh, k);
        sync();
        sum_partials(sh, p, K, G, 0);          // every workgroup, the same fixed order
        __syncthreads();
        flip ^= 1;
    }
};

// The workgroups sub0 .. gridDim.x - 1 of a grid team as a team of their own
// (same interface), with their own barrier (the words from BAR_SUB, the same
// protocol as GridTeam::sync) and partial buffers: the order-256 PSD block is
// projected by them while workgroups 0 .. sub0 - 1 project the small blocks,
// one each.  Only members call its sync and reduce.
template <typename GT>
struct PsdSubTeam {
    static constexpr bool kBlock = false;
    static constexpr bool kPsdTeam = true;
    GT& g;
    __device__ int blk() const { return (int)blockIdx.x - g.sub0; }
    __device__ int nblk() const { return (int)gridDim.x - g.sub0; }
    __device__ int rank() const { return blk() * blockDim.x + threadIdx.x; }
    __device__ int size() const { return nblk() * blockDim.x; }
    __device__ bool aborted() const { return g.aborted(); }
    __device__ void sync() {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        ++g.sub_k;
        if (threadIdx.x == 0)
            xcd_barrier(g.bar + BAR_SUB, g.grp, g.sub_members, g.sub_ngrp, g.sub_k, g.abort_flag, g.timeout_ticks);
        __syncthreads();
    }
    __device__ void reduce(Shared& sh, int K) {
        __syncthreads();
        const int G = gridDim.x;
        double* p = g.part + (size_t)(2 + g.sub_flip) * KMAX * G;
        for (int k = threadIdx.x; k < K; k += blockDim.x) p[(size_t)k * G + blockIdx.x] = block_total(sh, k);
        sync();
        sum_partials(sh, p, K, G, g.sub0);     // every member, the same fixed order
        __syncthreads();
        g.sub_flip ^= 1;
    }
};

// CSR matrix on the device.  `seg` is the number of lanes that cooperate on one
// row (a power of two <= 64), chosen on the host from the mean row length.
// Rows longer than `lthr` nonzeros (ascending list `lrows`, `nlong` of them)
// are summed by a whole workgroup in the team products instead, so one long
// row (a variable shared by every cone, say) does not serialise a segment.
template <typename T>
struct Csr {
    const int* rp;
    const int* ci;
    const T* v;
    int rows, cols, seg;
    const int* lrows;
    int nlong, lthr;
};

// Row-segmented SpMV over the team: for every row r, f(r, sum_k v[k] gx(ci[k]))
// is called by the last lane of the segment that owns r.  Segments of `seg`
// consecutive lanes stride a row's nonzeros, so loads of ci and v coalesce;
// each segment keeps ROWS rows in flight at once (independent load chains,
// which is what hides the memory latency of a persistent kernel; the CG's
// products use four, the other passes one), and each
// row's sum is a group sum over the segment's lanes (reported by its last lane).  gx(c) returns the
// input vector's entry c, so callers can gather values formed on the fly.
template <int ROWS, typename Team, typename T, typename Gx, typename F>
__device__ __forceinline__ void spmv_gather(Team& tm, const Csr<T>& M, Gx&& gx, F&& f) {
    const int S = M.seg;
    const int seg = tm.rank() / S;
    const int nseg = tm.size() / S;
    const int ls = tm.rank() & (S - 1);
    for (int r0 = seg; r0 < M.rows; r0 += ROWS * nseg) {
        int kb[ROWS], ke[ROWS];
        double acc[ROWS];
#pragma unroll
        for (int q = 0; q < ROWS; ++q) {
            const int r = r0 + q * nseg;
            const bool in = r < M.rows;
            kb[q] = in ? M.rp[r] + ls : 0;
            ke[q] = in ? M.rp[r + 1] : 0;
            acc[q] = 0.0;
        }
        bool more = true;
        while (more) {
            more = false;
#pragma unroll
            for (int q = 0; q < ROWS; ++q) {
                if (kb[q] < ke[q]) {
                    acc[q] += (double)M.v[kb[q]] * (double)gx(M.ci[kb[q]]);
                    kb[q] += S;
                    more = true;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < ROWS; ++q) {
            double a = acc[q];
            a = group_sum(a, S);
            const int r = r0 + q * nseg;
            if (ls == S - 1 && r < M.rows) f(r, a);
        }
    }
}

// Team SpMV over the rows a workgroup owns (MatPart): for every owned row r,
// f(r, sum_k v[k] gx(ci[k])) is called by the last lane of the segment that
// owns r.  Same segment scheme and ROWS-way batching as spmv_gather, with the
// row range local to the workgroup and the operator read from LDS when cached.
// pre(r), when given, is called by the reporting lane when row r is set up,
// before its gathers, and its value is passed on as f(r, sum, pre(r)): the
// per-row operands of f (the vectors it combines with the row's sum) are then
// loaded while the gathers are in flight, not in a second round trip after
// them (f's stores keep the compiler from moving later rows' loads above
// earlier rows' f).
struct NoPre {
    __device__ int operator()(int) const { return 0; }
};

template <int ROWS, bool LDS, typename T, typename Gx, typename Pre, typename F>
__device__ __forceinline__ void spmv_part_impl(const Csr<T>& M, const MatPart& mp, Gx&& gx, Pre&& pre, F&& f) {
    using PV = decltype(pre(0));
    const int S = M.seg;
    const int seg = threadIdx.x / S;
    const int nseg = blockDim.x / S;
    const int ls = threadIdx.x & (S - 1);
    const char* lds = reinterpret_cast<const char*>(sscs_dyn_lds);
    const T* lv = reinterpret_cast<const T*>(lds + mp.off_v);
    const int* lci = reinterpret_cast<const int*>(lds + mp.off_ci);
    const int* lrp = reinterpret_cast<const int*>(lds + mp.off_rp);
    for (int l0 = seg; l0 < mp.rows; l0 += ROWS * nseg) {
        int kb[ROWS], ke[ROWS];
        double acc[ROWS];
        bool own[ROWS];
        PV pv[ROWS];
#pragma unroll
        for (int q = 0; q < ROWS; ++q) {
            const int l = l0 + q * nseg;
            const bool in = l < mp.rows;
            int b = 0, e = 0;
            if (LDS) {
                b = in ? lrp[l] : 0;
                e = in ? lrp[l + 1] : 0;
            } else {
                b = in ? M.rp[mp.r0 + l] : 0;
                e = in ? M.rp[mp.r0 + l + 1] : 0;
            }
            own[q] = in && (e - b) <= M.lthr;          // long rows are summed below
            kb[q] = own[q] ? b + ls : 0;
            ke[q] = own[q] ? e : 0;
            acc[q] = 0.0;
            pv[q] = (own[q] && ls == S - 1) ? pre(mp.r0 + l) : PV{};
        }
        bool more = true;
        while (more) {
            more = false;
#pragma unroll
            for (int q = 0; q < ROWS; ++q) {
                if (kb[q] < ke[q]) {
                    const double v = LDS ? (double)lv[kb[q]] : (double)M.v[kb[q]];
                    const int c = LDS ? lci[kb[q]] : M.ci[kb[q]];
                    acc[q] += v * (double)gx(c);
                    kb[q] += S;
                    more = true;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < ROWS; ++q) {
            double a = acc[q];
            a = group_sum(a, S);
            const int l = l0 + q * nseg;
            if (ls == S - 1 && own[q]) f(mp.r0 + l, a, pv[q]);
        }
    }
    if (M.nlong > 0) {
        // long rows of this part: the whole workgroup per row, summed in a
        // fixed order (lanes, then waves); the first thread reports the row
        __shared__ double lred[NWMAX];
        int lo = 0, hi = M.nlong;
        while (lo < hi) {                              // first long row >= mp.r0
            const int mid = (lo + hi) >> 1;
            if (M.lrows[mid] < mp.r0) lo = mid + 1; else hi = mid;
        }
        for (int li = lo; li < M.nlong && M.lrows[li] < mp.r0 + mp.rows; ++li) {
            const int r = M.lrows[li], l = r - mp.r0;
            const int b = LDS ? lrp[l] : M.rp[r], e = LDS ? lrp[l + 1] : M.rp[r + 1];
            double a = 0.0;
            for (int kk = b + (int)threadIdx.x; kk < e; kk += blockDim.x) {
                const double v = LDS ? (double)lv[kk] : (double)M.v[kk];
                const int c = LDS ? lci[kk] : M.ci[kk];
                a += v * (double)gx(c);
            }
            a = wave_sum(a);
            if ((threadIdx.x & (WAVE - 1)) == 0) lred[threadIdx.x / WAVE] = a;
            __syncthreads();
            if (threadIdx.x == 0) {
                double t = 0.0;
                for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) t += lred[w];
                f(r, t, pre(r));
            }
            __syncthreads();
        }
    }
}

// The LDS copy is used when the team holds one and its value type is T.
template <int ROWS, typename Team, typename T, typename Gx, typename F>
__device__ __forceinline__ void spmv_part(Team& tm, const Csr<T>& M, int which, Gx&& gx, F&& f) {
    constexpr bool kUse = Team::kLds && std::is_same<T, typename Team::lds_t>::value;
    spmv_part_impl<ROWS, kUse>(M, tm.mp[which], gx, NoPre{}, [&](int r, double s, int) { f(r, s); });
}

// The same with per-row operands prefetched: f(r, sum, pre(r)).
template <int ROWS, typename Team, typename T, typename Gx, typename Pre, typename F>
__device__ __forceinline__ void spmv_part_pre(Team& tm, const Csr<T>& M, int which, Gx&& gx, Pre&& pre, F&& f) {
    constexpr bool kUse = Team::kLds && std::is_same<T, typename Team::lds_t>::value;
    spmv_part_impl<ROWS, kUse>(M, tm.mp[which], gx, pre, f);
}

// Fills a workgroup's MatPart for rows [part[b], part[b+1]) and, when `cache`
// is set, copies those rows into LDS starting at byte offset `*lds_off`.
template <typename T>
__device__ inline void load_part(MatPart& mp, const Csr<T>& M, const int* part, int b, bool cache, int* lds_off) {
    const int r0 = part[b], r1 = part[b + 1];
    mp.r0 = r0;
    mp.rows = r1 - r0;
    mp.lds = cache ? 1 : 0;
    if (!cache) { mp.off_v = mp.off_ci = mp.off_rp = 0; return; }
    const int k0 = M.rp[r0], k1 = M.rp[r1];
    const int nnz = k1 - k0;
    mp.off_v = *lds_off;
    mp.off_ci = mp.off_v + (int)sizeof(T) * nnz;
    mp.off_rp = mp.off_ci + 4 * nnz;
    *lds_off = (mp.off_rp + 4 * (mp.rows + 1) + 15) & ~15;
    char* lds = reinterpret_cast<char*>(sscs_dyn_lds);
    T* lv = reinterpret_cast<T*>(lds + mp.off_v);
    int* lci = reinterpret_cast<int*>(lds + mp.off_ci);
    int* lrp = reinterpret_cast<int*>(lds + mp.off_rp);
    for (int k = threadIdx.x; k < nnz; k += blockDim.x) {
        lv[k] = M.v[k0 + k];
        lci[k] = M.ci[k0 + k];
    }
    for (int l = threadIdx.x; l <= mp.rows; l += blockDim.x) lrp[l] = M.rp[r0 + l] - k0;
}

}  // namespace sscs
