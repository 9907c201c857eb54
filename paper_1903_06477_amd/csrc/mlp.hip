// The warm-start network of libsscs: a ReLU multilayer perceptron trained
// and evaluated by the kernels below (C ABI in include/sscs_mlp.h).
//
// Matrix products run on the CDNA4 matrix cores: v_mfma_f32_16x16x32_bf16,
// BF16 operands, FP32 accumulation.  Every product is written as
// C = A B^T with both operands K-contiguous ("NT"); the backward pass gets
// that form from transposed BF16 copies.  Operand buffers keep their leading
// dimension a multiple of 32 and their padding zero, so the K loop needs no
// bounds checks.  Master weights, biases, Adam moments and all reductions are
// FP32 (losses and column sums accumulate in FP64), in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/sscs.h"
#include "../../include/sscs_mlp.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float x) {
    // round to nearest, ties to even; NaN stays NaN
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return 0x7fc0;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

int pad32(int k) { return (k + 31) & ~31; }

// C (M x N) = A (M x Kp) * B (N x Kp)^T.  256 threads, 64 x 64 tile; wave w
// computes rows 32 (w / 2) .. +32 and columns 32 (w % 2) .. +32 as 2 x 2
// matrix-core tiles of 16 x 16.  Operand layout of the 16x16x32 instruction:
// lane l holds A[row l % 16][k (l / 16) * 8 .. +8] and B[col l % 16][same k];
// the result lane l holds rows (l / 16) * 4 .. +4 of column l % 16.
// Epilogue: + bias[col], optional ReLU, FP32 and/or BF16 output.
__global__ void __launch_bounds__(256) k_gemm_nt(const uint16_t* __restrict__ A, int lda,
                                                 const uint16_t* __restrict__ B, int ldb, int M, int N, int Kp,
                                                 const float* __restrict__ bias, int relu, float* __restrict__ C,
                                                 int ldc, uint16_t* __restrict__ Cb, int ldcb) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int row0 = blockIdx.y * 64 + (w >> 1) * 32;
    const int col0 = blockIdx.x * 64 + (w & 1) * 32;
    const int lr = lane & 15, lk = (lane >> 4) * 8;
    const int ra0 = row0 + lr, ra1 = row0 + 16 + lr;
    const int cb0 = col0 + lr, cb1 = col0 + 16 + lr;
    const bool va0 = ra0 < M, va1 = ra1 < M, vb0 = cb0 < N, vb1 = cb1 < N;
    const uint16_t* pa0 = A + (size_t)(va0 ? ra0 : 0) * lda + lk;
    const uint16_t* pa1 = A + (size_t)(va1 ? ra1 : 0) * lda + lk;
    const uint16_t* pb0 = B + (size_t)(vb0 ? cb0 : 0) * ldb + lk;
    const uint16_t* pb1 = B + (size_t)(vb1 ? cb1 : 0) * ldb + lk;
    f32x4 acc00 = {0.f, 0.f, 0.f, 0.f}, acc01 = acc00, acc10 = acc00, acc11 = acc00;
    const uint4 z = {0u, 0u, 0u, 0u};
    for (int k0 = 0; k0 < Kp; k0 += 32) {
        const uint4 a0 = va0 ? *reinterpret_cast<const uint4*>(pa0 + k0) : z;
        const uint4 a1 = va1 ? *reinterpret_cast<const uint4*>(pa1 + k0) : z;
        const uint4 b0 = vb0 ? *reinterpret_cast<const uint4*>(pb0 + k0) : z;
        const uint4 b1 = vb1 ? *reinterpret_cast<const uint4*>(pb1 + k0) : z;
        const bf16x8 fa0 = __builtin_bit_cast(bf16x8, a0), fa1 = __builtin_bit_cast(bf16x8, a1);
        const bf16x8 fb0 = __builtin_bit_cast(bf16x8, b0), fb1 = __builtin_bit_cast(bf16x8, b1);
        acc00 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa0, fb0, acc00, 0, 0, 0);
        acc01 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa0, fb1, acc01, 0, 0, 0);
        acc10 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa1, fb0, acc10, 0, 0, 0);
        acc11 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa1, fb1, acc11, 0, 0, 0);
    }
    const f32x4* accs[4] = {&acc00, &acc01, &acc10, &acc11};
    for (int t = 0; t < 4; ++t) {
        const int ti = t >> 1, tj = t & 1;
        const int col = col0 + 16 * tj + (lane & 15);
        if (col >= N) continue;
        const float bv = bias ? bias[col] : 0.f;
        for (int r = 0; r < 4; ++r) {
            const int row = row0 + 16 * ti + (lane >> 4) * 4 + r;
            if (row >= M) continue;
            float v = (*accs[t])[r] + bv;
            if (relu) v = fmaxf(v, 0.f);
            if (C) C[(size_t)row * ldc + col] = v;
            if (Cb) Cb[(size_t)row * ldcb + col] = f2bf(v);
        }
    }
}

// dst (rows x ldd, BF16) = src (rows x cols, FP32, leading dim lds); columns cols..ldd-1 zero.
__global__ void k_to_bf16(const float* __restrict__ src, int lds, int rows, int cols, uint16_t* __restrict__ dst,
                          int ldd) {
    const size_t total = (size_t)rows * ldd;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(i / ldd), c = (int)(i % ldd);
        dst[i] = c < cols ? f2bf(src[(size_t)r * lds + c]) : (uint16_t)0;
    }
}

// dst (cols x ldd, BF16) = transpose of src (rows x cols); dst columns rows..ldd-1 zero.
// 32 x 32 tiles through LDS so both sides coalesce.  SRC is float or uint16_t (BF16).
template <typename SRC>
__global__ void k_transpose_bf16(const SRC* __restrict__ src, int lds, int rows, int cols, uint16_t* __restrict__ dst,
                                 int ldd) {
    __shared__ uint16_t tile[32][33];
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 256 threads: 32 x 8
    for (int yy = ty; yy < 32; yy += 8) {
        const int r = r0 + yy, c = c0 + tx;
        uint16_t v = 0;
        if (r < rows && c < cols) {
            if constexpr (sizeof(SRC) == 4) v = f2bf(src[(size_t)r * lds + c]);
            else v = src[(size_t)r * lds + c];
        }
        tile[yy][tx] = v;
    }
    __syncthreads();
    for (int yy = ty; yy < 32; yy += 8) {
        const int c = c0 + yy, r = r0 + tx;           // dst row c, dst column r
        if (c < cols && r < ldd) dst[(size_t)c * ldd + r] = tile[tx][yy];
    }
}

// G = scale (Y - T); per-block partial sums of (Y - T)^2 (FP64).
__global__ void k_mse(const float* __restrict__ Y, const float* __restrict__ T, size_t n, float scale,
                      float* __restrict__ G, double* __restrict__ part) {
    __shared__ double red[256];
    double acc = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float d = Y[i] - T[i];
        if (G) G[i] = scale * d;
        acc += (double)d * d;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_sum(const double* __restrict__ part, int n, double scale, double* __restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += part[i];
        out[0] = s * scale;
    }
}

// G = dH where the (BF16) activation H is positive, else 0 (ReLU backward).
__global__ void k_relu_back(const float* __restrict__ dH, int rows, int cols, const uint16_t* __restrict__ H,
                            int ldh, float* __restrict__ G) {
    const size_t total = (size_t)rows * cols;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(i / cols), c = (int)(i % cols);
        G[i] = bf2f(H[(size_t)r * ldh + c]) > 0.f ? dH[i] : 0.f;
    }
}

// out[j] = sum_r G[r][j] (bias gradients), rows summed in order.
// 256 threads = 16 columns x 16 row groups; row group g sums rows g, g + 16, ...
// of its column, then the 16 partial sums are added in group order.
__global__ void __launch_bounds__(256) k_colsum(const float* __restrict__ G, int rows, int cols,
                                                float* __restrict__ out) {
    __shared__ double part[16][17];
    const int c = threadIdx.x & 15, g = threadIdx.x >> 4;
    const int j = blockIdx.x * 16 + c;
    double s = 0.0;
    if (j < cols)
        for (int r = g; r < rows; r += 16) s += G[(size_t)r * cols + j];
    part[g][c] = s;
    __syncthreads();
    if (g == 0 && j < cols) {
        double t = 0.0;
        for (int q = 0; q < 16; ++q) t += part[q][c];
        out[j] = (float)t;
    }
}

__global__ void k_adam(float* __restrict__ W, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, size_t n, float lr, float b1, float b2, float eps, float bc1,
                       float bc2) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        W[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    }
}

// Counter-based initialisation: splitmix64 of (seed, stream, index) ->
// uniform in [-a, a) with a = 1 / sqrt(fan_in), for weights (stream 2 l) and
// biases (stream 2 l + 1) of layer l.  (A wider range with zero biases leaves
// most ReLU units of this network dead after a few Adam steps.)
__global__ void k_init(float* __restrict__ W, size_t n, int fan_in, unsigned long long seed, int stream) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        unsigned long long z = seed + 0x9e3779b97f4a7c15ull * ((unsigned long long)stream * 0x100000000ull + i + 1);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        z = z ^ (z >> 31);
        const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);   // [0, 1)
        W[i] = (float)((2.0 * u - 1.0) / sqrt((double)fan_in));
    }
}

__global__ void k_assemble_u0(int count, int n, int m, const float* __restrict__ pred, double* __restrict__ u0) {
    const size_t N = (size_t)n + m + 1, P = (size_t)n + 2 * (size_t)m;
    const size_t total = (size_t)count * N;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const size_t r = i / N, c = i % N;
        const float* p = pred + r * P;
        double v;
        if (c < (size_t)n) v = p[c];
        else if (c < (size_t)n + m) v = (double)p[c] + (double)p[c + m];
        else v = 1.0;
        u0[i] = v;
    }
}

int grid_for(size_t n) { return (int)std::min<size_t>(65535, std::max<size_t>(1, (n + 255) / 256)); }

thread_local std::string g_err;

#define HTRY(expr)                                                          \
    do {                                                                    \
        hipError_t _e = (expr);                                             \
        if (_e != hipSuccess) { g_err = hipGetErrorString(_e); return SSCS_E_HIP; } \
    } while (0)

template <typename T>
int dalloc(T** p, size_t n) {
    *p = nullptr;
    if (hipMalloc((void**)p, std::max<size_t>(1, n) * sizeof(T)) != hipSuccess) return SSCS_E_NOMEM;
    if (hipMemset(*p, 0, std::max<size_t>(1, n) * sizeof(T)) != hipSuccess) return SSCS_E_HIP;
    return SSCS_OK;
}

int launch_gemm(hipStream_t s, const uint16_t* A, int lda, const uint16_t* B, int ldb, int M, int N, int Kp,
                const float* bias, int relu, float* C, int ldc, uint16_t* Cb, int ldcb) {
    dim3 grid((N + 63) / 64, (M + 63) / 64);
    k_gemm_nt<<<grid, 256, 0, s>>>(A, lda, B, ldb, M, N, Kp, bias, relu, C, ldc, Cb, ldcb);
    HTRY(hipGetLastError());
    return SSCS_OK;
}

}  // namespace

struct sscs_mlp {
    hipStream_t stream = nullptr;
    int L = 0, max_batch = 0, ldb = 0;
    std::vector<int> w, ld;                 // widths, padded widths
    std::vector<float*> W, b, gW, gb, mW, vW, mb, vb;
    std::vector<uint16_t*> Wb, WTb;         // BF16 W (out x ld_in) and W^T (in x ld_out)
    std::vector<uint16_t*> H;               // BF16 activations, layer inputs (batch x ld_l)
    float *G = nullptr, *G2 = nullptr, *dH = nullptr, *Y = nullptr;
    uint16_t *GT = nullptr, *HT = nullptr, *Gb = nullptr;
    double *part = nullptr, *lossd = nullptr;
    long long step = 0;
    int maxw = 0, maxld = 0;
};

namespace {

int refresh_bf16(sscs_mlp* n, int l) {
    const int out = n->w[l + 1], in = n->w[l];
    k_to_bf16<<<grid_for((size_t)out * n->ld[l]), 256, 0, n->stream>>>(n->W[l], in, out, in, n->Wb[l], n->ld[l]);
    dim3 g((in + 31) / 32, (out + 31) / 32);
    k_transpose_bf16<float><<<g, 256, 0, n->stream>>>(n->W[l], in, out, in, n->WTb[l], n->ld[l + 1]);
    HTRY(hipGetLastError());
    return SSCS_OK;
}

int forward(sscs_mlp* n, int batch, const float* X, float* Y) {
    k_to_bf16<<<grid_for((size_t)batch * n->ld[0]), 256, 0, n->stream>>>(X, n->w[0], batch, n->w[0], n->H[0], n->ld[0]);
    HTRY(hipGetLastError());
    for (int l = 0; l < n->L; ++l) {
        const bool last = l == n->L - 1;
        int r = launch_gemm(n->stream, n->H[l], n->ld[l], n->Wb[l], n->ld[l], batch, n->w[l + 1], n->ld[l],
                            n->b[l], last ? 0 : 1, last ? Y : nullptr, n->w[l + 1],
                            last ? nullptr : n->H[l + 1], last ? 0 : n->ld[l + 1]);
        if (r != SSCS_OK) return r;
    }
    return SSCS_OK;
}

// Loss and gradients for the batch (fills n->gW, n->gb); loss into n->lossd.
int backward(sscs_mlp* n, int batch, const float* X, const float* T, float* Y) {
    int r = forward(n, batch, X, Y);
    if (r != SSCS_OK) return r;
    const int wl = n->w[n->L];
    const size_t ny = (size_t)batch * wl;
    const int nblk = 512;
    k_mse<<<nblk, 256, 0, n->stream>>>(Y, T, ny, (float)(2.0 / (double)ny), n->G, n->part);
    k_sum<<<1, 1, 0, n->stream>>>(n->part, nblk, 1.0 / (double)ny, n->lossd);
    HTRY(hipGetLastError());
    const int ldB = pad32(batch);
    float* G = n->G;
    float* Gn = n->G2;
    for (int l = n->L - 1; l >= 0; --l) {
        const int out = n->w[l + 1], in = n->w[l];
        // dW_l = G^T H_l : operands G^T (out x batch) and H_l^T (in x batch), K = batch
        dim3 g1((out + 31) / 32, (batch + 31) / 32);
        k_transpose_bf16<float><<<g1, 256, 0, n->stream>>>(G, out, batch, out, n->GT, ldB);
        dim3 g2((in + 31) / 32, (batch + 31) / 32);
        k_transpose_bf16<uint16_t><<<g2, 256, 0, n->stream>>>(n->H[l], n->ld[l], batch, in, n->HT, ldB);
        HTRY(hipGetLastError());
        r = launch_gemm(n->stream, n->GT, ldB, n->HT, ldB, out, in, ldB, nullptr, 0, n->gW[l], in, nullptr, 0);
        if (r != SSCS_OK) return r;
        k_colsum<<<(out + 15) / 16, 256, 0, n->stream>>>(G, batch, out, n->gb[l]);
        HTRY(hipGetLastError());
        if (l == 0) break;
        // dH = G W_l : operands G (batch x out) and W_l^T (in x out), K = out; then ReLU mask of H_l
        k_to_bf16<<<grid_for((size_t)batch * n->ld[l + 1]), 256, 0, n->stream>>>(G, out, batch, out, n->Gb,
                                                                                  n->ld[l + 1]);
        HTRY(hipGetLastError());
        r = launch_gemm(n->stream, n->Gb, n->ld[l + 1], n->WTb[l], n->ld[l + 1], batch, in, n->ld[l + 1], nullptr,
                        0, n->dH, in, nullptr, 0);
        if (r != SSCS_OK) return r;
        k_relu_back<<<grid_for((size_t)batch * in), 256, 0, n->stream>>>(n->dH, batch, in, n->H[l], n->ld[l], Gn);
        HTRY(hipGetLastError());
        std::swap(G, Gn);
    }
    return SSCS_OK;
}

int check(sscs_mlp* n, int batch) {
    if (!n || batch < 1 || batch > n->max_batch) return SSCS_E_INVALID;
    return SSCS_OK;
}

}  // namespace

extern "C" {

int sscs_mlp_destroy(sscs_mlp* n) {
    if (!n) return SSCS_OK;
    if (n->stream) hipStreamSynchronize(n->stream);
    else hipDeviceSynchronize();
    for (auto* v : {&n->W, &n->b, &n->gW, &n->gb, &n->mW, &n->vW, &n->mb, &n->vb})
        for (float* p : *v) hipFree(p);
    for (uint16_t* p : n->Wb) hipFree(p);
    for (uint16_t* p : n->WTb) hipFree(p);
    for (uint16_t* p : n->H) hipFree(p);
    hipFree(n->G); hipFree(n->G2); hipFree(n->dH); hipFree(n->Y); hipFree(n->GT); hipFree(n->HT); hipFree(n->Gb);
    hipFree(n->part); hipFree(n->lossd);
    delete n;
    return SSCS_OK;
}

int sscs_mlp_create(int32_t nlayers, const int32_t* widths, int32_t max_batch, uint64_t seed, void* hip_stream,
                    sscs_mlp** out) {
    if (!out || nlayers < 1 || !widths || max_batch < 1) return SSCS_E_INVALID;
    *out = nullptr;
    for (int i = 0; i <= nlayers; ++i)
        if (widths[i] < 1) return SSCS_E_INVALID;
    sscs_mlp* n = new (std::nothrow) sscs_mlp();
    if (!n) return SSCS_E_NOMEM;
    n->stream = (hipStream_t)hip_stream;
    n->L = nlayers;
    n->max_batch = max_batch;
    for (int i = 0; i <= nlayers; ++i) {
        n->w.push_back(widths[i]);
        n->ld.push_back(pad32(widths[i]));
        n->maxw = std::max(n->maxw, widths[i]);
        n->maxld = std::max(n->maxld, pad32(widths[i]));
    }
    const int ldB = pad32(max_batch);
    int r = SSCS_OK;
    auto fal = [&](float** p, size_t k) { if (r == SSCS_OK) r = dalloc(p, k); };
    auto bal = [&](uint16_t** p, size_t k) { if (r == SSCS_OK) r = dalloc(p, k); };
    n->W.resize(nlayers); n->b.resize(nlayers); n->gW.resize(nlayers); n->gb.resize(nlayers);
    n->mW.resize(nlayers); n->vW.resize(nlayers); n->mb.resize(nlayers); n->vb.resize(nlayers);
    n->Wb.resize(nlayers); n->WTb.resize(nlayers); n->H.resize(nlayers);
    for (int l = 0; l < nlayers; ++l) {
        const size_t nw = (size_t)widths[l + 1] * widths[l];
        fal(&n->W[l], nw); fal(&n->gW[l], nw); fal(&n->mW[l], nw); fal(&n->vW[l], nw);
        fal(&n->b[l], widths[l + 1]); fal(&n->gb[l], widths[l + 1]);
        fal(&n->mb[l], widths[l + 1]); fal(&n->vb[l], widths[l + 1]);
        bal(&n->Wb[l], (size_t)widths[l + 1] * n->ld[l]);
        bal(&n->WTb[l], (size_t)widths[l] * n->ld[l + 1]);
        bal(&n->H[l], (size_t)max_batch * n->ld[l]);
    }
    fal(&n->G, (size_t)max_batch * n->maxw);
    fal(&n->G2, (size_t)max_batch * n->maxw);
    fal(&n->dH, (size_t)max_batch * n->maxw);
    fal(&n->Y, (size_t)max_batch * widths[nlayers]);
    bal(&n->GT, (size_t)n->maxw * ldB);
    bal(&n->HT, (size_t)n->maxw * ldB);
    bal(&n->Gb, (size_t)max_batch * n->maxld);
    if (r == SSCS_OK) r = dalloc(&n->part, 512);
    if (r == SSCS_OK) r = dalloc(&n->lossd, 1);
    for (int l = 0; l < nlayers && r == SSCS_OK; ++l) {
        const size_t nw = (size_t)widths[l + 1] * widths[l];
        k_init<<<grid_for(nw), 256, 0, n->stream>>>(n->W[l], nw, widths[l], (unsigned long long)seed, 2 * l);
        k_init<<<grid_for(widths[l + 1]), 256, 0, n->stream>>>(n->b[l], widths[l + 1], widths[l],
                                                              (unsigned long long)seed, 2 * l + 1);
        if (hipGetLastError() != hipSuccess) r = SSCS_E_HIP;
        if (r == SSCS_OK) r = refresh_bf16(n, l);
    }
    if (r == SSCS_OK && hipStreamSynchronize(n->stream) != hipSuccess) r = SSCS_E_HIP;
    if (r != SSCS_OK) { sscs_mlp_destroy(n); return r; }
    *out = n;
    return SSCS_OK;
}

int sscs_mlp_set_params(sscs_mlp* n, const float* const* W, const float* const* b) {
    if (!n || !W || !b) return SSCS_E_INVALID;
    for (int l = 0; l < n->L; ++l) {
        HTRY(hipMemcpyAsync(n->W[l], W[l], (size_t)n->w[l + 1] * n->w[l] * sizeof(float), hipMemcpyHostToDevice,
                            n->stream));
        HTRY(hipMemcpyAsync(n->b[l], b[l], (size_t)n->w[l + 1] * sizeof(float), hipMemcpyHostToDevice, n->stream));
        int r = refresh_bf16(n, l);
        if (r != SSCS_OK) return r;
    }
    HTRY(hipStreamSynchronize(n->stream));
    return SSCS_OK;
}

int sscs_mlp_get_params(sscs_mlp* n, float* const* W, float* const* b) {
    if (!n || !W || !b) return SSCS_E_INVALID;
    for (int l = 0; l < n->L; ++l) {
        HTRY(hipMemcpyAsync(W[l], n->W[l], (size_t)n->w[l + 1] * n->w[l] * sizeof(float), hipMemcpyDeviceToHost,
                            n->stream));
        HTRY(hipMemcpyAsync(b[l], n->b[l], (size_t)n->w[l + 1] * sizeof(float), hipMemcpyDeviceToHost, n->stream));
    }
    HTRY(hipStreamSynchronize(n->stream));
    return SSCS_OK;
}

int sscs_mlp_forward(sscs_mlp* n, int32_t batch, const float* X, float* Y) {
    int r = check(n, batch);
    if (r != SSCS_OK) return r;
    if (!X || !Y) return SSCS_E_INVALID;
    r = forward(n, batch, X, Y);
    if (r != SSCS_OK) return r;
    HTRY(hipStreamSynchronize(n->stream));
    return SSCS_OK;
}

int sscs_mlp_gradients(sscs_mlp* n, int32_t batch, const float* X, const float* T, float* const* dW,
                       float* const* db, float* loss) {
    int r = check(n, batch);
    if (r != SSCS_OK) return r;
    if (!X || !T || !dW || !db) return SSCS_E_INVALID;
    r = backward(n, batch, X, T, n->Y);
    if (r != SSCS_OK) return r;
    for (int l = 0; l < n->L; ++l) {
        HTRY(hipMemcpyAsync(dW[l], n->gW[l], (size_t)n->w[l + 1] * n->w[l] * sizeof(float), hipMemcpyDeviceToHost,
                            n->stream));
        HTRY(hipMemcpyAsync(db[l], n->gb[l], (size_t)n->w[l + 1] * sizeof(float), hipMemcpyDeviceToHost, n->stream));
    }
    double L = 0.0;
    HTRY(hipMemcpyAsync(&L, n->lossd, sizeof(double), hipMemcpyDeviceToHost, n->stream));
    HTRY(hipStreamSynchronize(n->stream));
    if (loss) *loss = (float)L;
    return SSCS_OK;
}

int sscs_mlp_train_step(sscs_mlp* n, int32_t batch, const float* X, const float* T, float lr, float* loss) {
    int r = check(n, batch);
    if (r != SSCS_OK) return r;
    if (!X || !T || !(lr > 0)) return SSCS_E_INVALID;
    r = backward(n, batch, X, T, n->Y);
    if (r != SSCS_OK) return r;
    n->step += 1;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float bc1 = (float)(1.0 - std::pow(0.9, (double)n->step));
    const float bc2 = (float)(1.0 - std::pow(0.999, (double)n->step));
    for (int l = 0; l < n->L; ++l) {
        const size_t nw = (size_t)n->w[l + 1] * n->w[l];
        k_adam<<<grid_for(nw), 256, 0, n->stream>>>(n->W[l], n->gW[l], n->mW[l], n->vW[l], nw, lr, b1, b2, eps, bc1,
                                                    bc2);
        k_adam<<<grid_for(n->w[l + 1]), 256, 0, n->stream>>>(n->b[l], n->gb[l], n->mb[l], n->vb[l], n->w[l + 1], lr,
                                                            b1, b2, eps, bc1, bc2);
        HTRY(hipGetLastError());
        r = refresh_bf16(n, l);
        if (r != SSCS_OK) return r;
    }
    double L = 0.0;
    HTRY(hipMemcpyAsync(&L, n->lossd, sizeof(double), hipMemcpyDeviceToHost, n->stream));
    HTRY(hipStreamSynchronize(n->stream));
    if (loss) *loss = (float)L;
    return SSCS_OK;
}

int sscs_assemble_u0(int32_t count, int32_t n, int32_t m, const float* pred, double* u0, void* hip_stream) {
    if (count < 1 || n < 1 || m < 1 || !pred || !u0) return SSCS_E_INVALID;
    hipStream_t s = (hipStream_t)hip_stream;
    k_assemble_u0<<<grid_for((size_t)count * (n + m + 1)), 256, 0, s>>>(count, n, m, pred, u0);
    HTRY(hipGetLastError());
    HTRY(hipStreamSynchronize(s));
    return SSCS_OK;
}

int sscs_mlp_gemm_nt(int32_t M, int32_t N, int32_t K, const float* A, const float* B, float* C, void* hip_stream) {
    if (M < 1 || N < 1 || K < 1 || !A || !B || !C) return SSCS_E_INVALID;
    hipStream_t s = (hipStream_t)hip_stream;
    const int Kp = pad32(K);
    uint16_t *Ab = nullptr, *Bb = nullptr;
    int r = dalloc(&Ab, (size_t)M * Kp);
    if (r == SSCS_OK) r = dalloc(&Bb, (size_t)N * Kp);
    if (r == SSCS_OK) {
        k_to_bf16<<<grid_for((size_t)M * Kp), 256, 0, s>>>(A, K, M, K, Ab, Kp);
        k_to_bf16<<<grid_for((size_t)N * Kp), 256, 0, s>>>(B, K, N, K, Bb, Kp);
        r = launch_gemm(s, Ab, Kp, Bb, Kp, M, N, Kp, nullptr, 0, C, N, nullptr, 0);
    }
    if (hipStreamSynchronize(s) != hipSuccess && r == SSCS_OK) r = SSCS_E_HIP;
    hipFree(Ab);
    hipFree(Bb);
    return r;
}

}  // extern "C"
