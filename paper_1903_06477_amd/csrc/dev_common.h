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
    int    qhead;               // batched engine: instance popped from the queue
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

// Writes the wave-sum of v into slot k of the per-wave partials.
__device__ __forceinline__ void put(Shared& sh, int k, double v) {
    v = wave_sum(v);
    if ((threadIdx.x & (WAVE - 1)) == 0) sh.red[k * NWMAX + (threadIdx.x / WAVE)] = v;
}

// Sums the per-wave partials of slot k in wave order.
__device__ __forceinline__ double block_total(const Shared& sh, int k) {
    const int nw = blockDim.x / WAVE;
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += sh.red[k * NWMAX + w];
    return s;
}

struct BlockTeam {
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

// Grid barrier on a monotonically increasing 64-bit arrival counter.  Every
// workgroup of the cooperative grid passes the same number of barriers, so the
// k-th barrier completes when the counter reaches k * gridDim.x.  A wait that
// exceeds `timeout_ticks` of the 100 MHz wall clock raises the abort flag; all
// later barriers then return at once, so every wave of the grid still reaches
// the kernel's end.
struct GridTeam {
    unsigned long long* bar;
    int* abort_flag;
    double* part;               // [2][KMAX][gridDim.x] partials
    unsigned long long epoch;   // barriers passed so far, times gridDim.x
    long long timeout_ticks;
    int flip;

    __device__ int rank() const { return blockIdx.x * blockDim.x + threadIdx.x; }
    __device__ int size() const { return gridDim.x * blockDim.x; }
    __device__ int wave() const { return rank() / WAVE; }
    __device__ int nwaves() const { return size() / WAVE; }
    __device__ int blk() const { return blockIdx.x; }
    __device__ int nblk() const { return gridDim.x; }

    __device__ bool aborted() const {
        return __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    }

    __device__ void sync() {
        __syncthreads();
        epoch += gridDim.x;
        if (threadIdx.x == 0) {
            __threadfence();
            __hip_atomic_fetch_add(bar, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const long long t0 = wall_clock64();
            while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
                if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                __builtin_amdgcn_s_sleep(1);
                if (wall_clock64() - t0 > timeout_ticks) {
                    __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
            __threadfence();
        }
        __syncthreads();
    }

    __device__ void reduce(Shared& sh, int K) {
        __syncthreads();
        const int G = gridDim.x;
        double* p = part + (size_t)flip * KMAX * G;
        for (int k = threadIdx.x; k < K; k += blockDim.x) p[(size_t)k * G + blockIdx.x] = block_total(sh, k);
        sync();
        // every workgroup sums all partials in the same fixed order
        const int lane = threadIdx.x & (WAVE - 1);
        const int nw = blockDim.x / WAVE;
        for (int k = threadIdx.x / WAVE; k < K; k += nw) {
            double s = 0.0;
            for (int j = lane; j < G; j += WAVE) s += p[(size_t)k * G + j];
            s = wave_sum(s);
            if (lane == 0) sh.out[k] = s;
        }
        __syncthreads();
        flip ^= 1;
    }
};

// CSR matrix on the device.  `seg` is the number of lanes that cooperate on one
// row (a power of two <= 64), chosen on the host from the mean row length.
template <typename T>
struct Csr {
    const int* rp;
    const int* ci;
    const T* v;
    int rows, cols, seg;
};

// Row-segmented SpMV over the team: for every row r, f(r, sum_k v[k] x[ci[k]])
// is called by the first lane of the segment that owns r.  Segments of `seg`
// consecutive lanes stride the row's nonzeros, so loads of ci and v coalesce;
// the segment sum is a butterfly over the segment's lanes.
template <typename Team, typename T, typename TX, typename F>
__device__ __forceinline__ void spmv_rows(Team& tm, const Csr<T>& M, const TX* __restrict__ x, F&& f) {
    const int S = M.seg;
    const int seg = tm.rank() / S;
    const int nseg = tm.size() / S;
    const int ls = tm.rank() & (S - 1);
    for (int r = seg; r < M.rows; r += nseg) {
        const int k1 = M.rp[r + 1];
        double acc = 0.0;
        for (int k = M.rp[r] + ls; k < k1; k += S) acc += (double)M.v[k] * (double)x[M.ci[k]];
        for (int off = S >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off, WAVE);
        if (ls == 0) f(r, acc);
    }
}

}  // namespace sscs
