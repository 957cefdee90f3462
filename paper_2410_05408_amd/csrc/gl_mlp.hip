// gl_mlp.hip -- the residual surrogate network on the GPU: BF16 matrix-core
// (MFMA) GEMMs with FP32 accumulation, fused bias/GELU epilogues, backward
// pass, MSE loss and Adam on FP32 master weights.
//
// Network: x[n][16] -> [Linear -> GELU] x 4 (width 256) -> Linear -> y[n]
// (input width 16: the encoded features, zero-padded).  Activations and the
// weights fed to the matrix cores are BF16; accumulation, biases, the output
// layer, the loss, gradients of the output layer and the optimizer are FP32.
// All reductions run in a fixed order (no floating-point atomics).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "gl.h"
#include "gl_internal.h"

namespace {

constexpr int D_IN = GL_MLP_DIN;   // 16
constexpr int W = GL_MLP_WIDTH;    // 256
constexpr int DEPTH = 4;           // hidden layers

using bf16 = unsigned short;

__device__ __forceinline__ bf16 f2bf(float f)
{
    unsigned int u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    return (bf16)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16 h) { return __uint_as_float(((unsigned int)h) << 16); }

constexpr float kGeluC = 0.7978845608028654f;  // sqrt(2/pi)

// tanh(u) = 1 - 2 / (exp(2u) + 1) from the hardware exponential and
// reciprocal (relative error ~1e-6, far below the BF16 rounding of the
// activations; exp overflow gives exactly 1, underflow exactly -1)
__device__ __forceinline__ float tanh_fast(float u)
{
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(__expf(2.0f * u) + 1.0f);
}

__device__ __forceinline__ float gelu(float z)
{
    return 0.5f * z * (1.0f + tanh_fast(kGeluC * (z + 0.044715f * z * z * z)));
}
__device__ __forceinline__ float gelu_grad(float z)
{
    const float th = tanh_fast(kGeluC * (z + 0.044715f * z * z * z));
    const float du = kGeluC * (1.0f + 3.0f * 0.044715f * z * z);
    return 0.5f * (1.0f + th) + 0.5f * z * (1.0f - th * th) * du;
}

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16x8_t as_bf8(u32x4_t v) { return __builtin_bit_cast(bf16x8_t, v); }
// BF16 values are handled as 16-bit halves of 32-bit words (element j in
// word j/2, low half first); single elements are never read out of a bf16x8_t
__device__ __forceinline__ bf16 half_of(u32x4_t v, int j) { return (bf16)(v[j >> 1] >> (16 * (j & 1))); }
__device__ __forceinline__ unsigned pack2(bf16 lo, bf16 hi) { return (unsigned)lo | ((unsigned)hi << 16); }

// MFMA 16x16x32 BF16 (gfx950), FP32 accumulate.  Lane l holds row l%16 of A
// and column l%16 of B, each with 8 values of the K dimension (lane group
// l/16 picks which 8: the same choice for both operands, so the K order in
// which values are laid out only has to agree between A and B); the result
// D[4(l/16)+i][l%16], i < 4, lands in lane l.
__device__ __forceinline__ float4_t mfma32(bf16x8_t a, bf16x8_t b, float4_t c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

enum Epi { EPI_FWD = 0, EPI_DX = 1, EPI_DW = 2 };

constexpr int kGT = 64;       // block tile (M and N)
constexpr int kGK = 32;       // K per LDS stage (one MFMA deep)
constexpr int kGP = kGK + 8;  // LDS row pitch in bf16 (80 B: rows land on different banks)

// C[M][N] = op(A)[M][K] op(B)[K][N] over the K range of split blockIdx.z
// ([z kchunk, min(K, (z + 1) kchunk))): 64x64 block tile, 4 wavefronts each
// owning a 32x32 quadrant of 2x2 MFMA 16x16x32 tiles; K staged 32 at a time
// through two LDS buffers (the next stage's global loads are in flight while
// the current one runs), one 16-byte global load per thread and operand.
// TA: A is stored [K][M] (read transposed).  TB: B is stored [N][K].  In LDS
// both operands are kept K-contiguous (As[m][k], Bs[n][k]) so that an MFMA
// operand is one 16-byte read.  Out-of-range elements load as zero and are
// not stored.
//  EPI_FWD: z = acc + bias[n]; Z = bf16(z), H = bf16(gelu(z))
//  EPI_DX : out_bf = bf16(acc * gelu'(Zp[m][n]))
//  EPI_DW : Fout[z][m][n] = acc (one slice per split, summed in order later)
template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(256)
k_gemm(int M, int N, int K, int kchunk, const bf16* __restrict__ A, int lda, const bf16* __restrict__ B,
       int ldb, const float* __restrict__ bias, const bf16* __restrict__ Zp, bf16* __restrict__ Zout,
       bf16* __restrict__ Hout, float* __restrict__ Fout, int ldc)
{
    __shared__ __align__(16) bf16 As[2][kGT][kGP];
    __shared__ __align__(16) bf16 Bs[2][kGT][kGP];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int m0 = blockIdx.y * kGT, n0 = blockIdx.x * kGT;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int kb0 = blockIdx.z * kchunk;
    const int kb1 = min(K, kb0 + kchunk);
    // this thread's piece of each tile: a row and 8 consecutive K (K-contiguous
    // source) or a K row and 8 consecutive M / N (transposed source)
    const int rq = tid >> 2, cq = (tid & 3) * 8;  // row 0..63, K offset 0..24
    const int kr = tid >> 3, xq = (tid & 7) * 8;  // K row 0..31, M/N offset 0..56
    u32x4_t ra = {0u, 0u, 0u, 0u}, rb = {0u, 0u, 0u, 0u};
    auto load8 = [](const bf16* src, bool full, int avail) {
        u32x4_t v = {0u, 0u, 0u, 0u};
        if (full) {
            v = *reinterpret_cast<const u32x4_t*>(src);
        } else if (avail > 0) {
            for (int j = 0; j < 8 && j < avail; ++j) v[j >> 1] |= (unsigned)src[j] << (16 * (j & 1));
        }
        return v;
    };
    auto load = [&](int k0) {
        if (!TA) {  // A[m][k]
            const int m = m0 + rq, k = k0 + cq;
            ra = m < M ? load8(A + (size_t)m * lda + k, k + 8 <= kb1, kb1 - k) : u32x4_t{0u, 0u, 0u, 0u};
        } else {    // A[k][m]
            const int k = k0 + kr, m = m0 + xq;
            ra = k < kb1 ? load8(A + (size_t)k * lda + m, m + 8 <= M, M - m) : u32x4_t{0u, 0u, 0u, 0u};
        }
        if (!TB) {  // B[k][n]
            const int k = k0 + kr, n = n0 + xq;
            rb = k < kb1 ? load8(B + (size_t)k * ldb + n, n + 8 <= N, N - n) : u32x4_t{0u, 0u, 0u, 0u};
        } else {    // B[n][k]
            const int n = n0 + rq, k = k0 + cq;
            rb = n < N ? load8(B + (size_t)n * ldb + k, k + 8 <= kb1, kb1 - k) : u32x4_t{0u, 0u, 0u, 0u};
        }
    };
    auto store = [&](int st) {
        if (!TA) {
            *reinterpret_cast<u32x4_t*>(&As[st][rq][cq]) = ra;
        } else {
            for (int j = 0; j < 8; ++j) As[st][xq + j][kr] = half_of(ra, j);
        }
        if (TB) {
            *reinterpret_cast<u32x4_t*>(&Bs[st][rq][cq]) = rb;
        } else {
            for (int j = 0; j < 8; ++j) Bs[st][xq + j][kr] = half_of(rb, j);
        }
    };
    float4_t acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
    const int nk = kb1 > kb0 ? (kb1 - kb0 + kGK - 1) / kGK : 0;
    if (nk > 0) {
        load(kb0);
        store(0);
    }
    __syncthreads();
    const int lr = lane & 15, lg = (lane >> 4) * 8;
    for (int it = 0; it < nk; ++it) {
        const int st = it & 1;
        if (it + 1 < nk) load(kb0 + (it + 1) * kGK);
        bf16x8_t a[2], b[2];
        for (int t = 0; t < 2; ++t) {
            a[t] = *reinterpret_cast<const bf16x8_t*>(&As[st][wm + t * 16 + lr][lg]);
            b[t] = *reinterpret_cast<const bf16x8_t*>(&Bs[st][wn + t * 16 + lr][lg]);
        }
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) acc[i][j] = mfma32(a[i], b[j], acc[i][j]);
        if (it + 1 < nk) store(st ^ 1);
        __syncthreads();
    }
    float* Fz = EPI == EPI_DW ? Fout + (size_t)blockIdx.z * (size_t)M * ldc : nullptr;
    for (int ti = 0; ti < 2; ++ti)
        for (int tj = 0; tj < 2; ++tj)
            for (int i = 0; i < 4; ++i) {
                const int m = m0 + wm + ti * 16 + (lane >> 4) * 4 + i;
                const int n = n0 + wn + tj * 16 + (lane & 15);
                if (m >= M || n >= N) continue;
                const float v = acc[ti][tj][i];
                const size_t o = (size_t)m * ldc + n;
                if (EPI == EPI_FWD) {
                    const float z = v + bias[n];
                    Zout[o] = f2bf(z);
                    Hout[o] = f2bf(gelu(z));
                } else if (EPI == EPI_DX) {
                    Hout[o] = f2bf(v * gelu_grad(bf2f(Zp[o])));
                } else {
                    Fz[o] = v;
                }
            }
}

// out[e] = sum over s < S of part[s][e], in order of s (deterministic)
__global__ void k_reduce_parts(const float* __restrict__ part, int S, int64_t count, float* __restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    float a = 0.f;
    for (int s = 0; s < S; ++s) a += part[(size_t)s * count + e];
    out[e] = a;
}

// Column sums over rows [r z rows_per, ...) of a [n][ld] matrix, 64 columns per
// block (one per lane, rows in four phases), partial sums part[z][c] for
// k_reduce_parts; BF: BF16 input; SCALE: each row weighted by s[m].
template <bool BF, bool SCALE>
__global__ void __launch_bounds__(256)
k_colsum(const void* __restrict__ Xv, int ld, int n, int rows_per, const float* __restrict__ s,
         float* __restrict__ part)
{
    __shared__ float red[4][64];
    const int c = blockIdx.x * 64 + (threadIdx.x & 63), ph = threadIdx.x >> 6;
    const int r0 = blockIdx.y * rows_per, r1 = min(n, r0 + rows_per);
    float acc = 0.f;
    if (c < ld)
        for (int m = r0 + ph; m < r1; m += 4) {
            float v = BF ? bf2f(((const bf16*)Xv)[(size_t)m * ld + c]) : ((const float*)Xv)[(size_t)m * ld + c];
            if (SCALE) v *= s[m];
            acc += v;
        }
    red[ph][threadIdx.x & 63] = acc;
    __syncthreads();
    if (ph == 0 && c < ld)
        part[(size_t)blockIdx.y * ld + c] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) +
                                            red[3][threadIdx.x];
}

// sum of a vector in a fixed order (one block): rows in 256 phases, then a tree
__global__ void __launch_bounds__(256) k_vecsum(const float* __restrict__ x, int n, float* __restrict__ out)
{
    __shared__ float red[256];
    const int tid = threadIdx.x;
    float acc = 0.f;
    for (int m = tid; m < n; m += 256) acc += x[m];
    red[tid] = acc;
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if (tid < d) red[tid] += red[tid + d];
        __syncthreads();
    }
    if (tid == 0) out[0] = red[0];
}

// x (fp32 [n][16]) -> bf16
__global__ void k_to_bf16(const float* __restrict__ x, bf16* __restrict__ y, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

// y[m] = sum_k H[m][k] w[k] + b (FP32, k in order)
__global__ void k_out_fwd(const bf16* __restrict__ H, const float* __restrict__ w, const float* __restrict__ b,
                          float* __restrict__ y, int n)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    float s = 0.f;
    for (int k = 0; k < W; ++k) s = fmaf(bf2f(H[(size_t)m * W + k]), w[k], s);
    y[m] = s + b[0];
}

// dy[m] = 2 (y - t)/n ; dZ4[m][k] = bf16(dy w[k] gelu'(Z4[m][k])); also (y - t)^2 per row
__global__ void k_out_bwd(const float* __restrict__ y, const float* __restrict__ t, const float* __restrict__ w,
                          const bf16* __restrict__ Z4, float* __restrict__ dy, float* __restrict__ sq,
                          bf16* __restrict__ dZ4, int n)
{
    const int m = blockIdx.x;
    const int k = threadIdx.x;  // 256 threads
    if (m >= n) return;
    const float r = y[m] - t[m];
    const float d = 2.0f * r / (float)n;
    if (k == 0) {
        dy[m] = d;
        sq[m] = r * r;
    }
    const size_t o = (size_t)m * W + k;
    dZ4[o] = f2bf(d * w[k] * gelu_grad(bf2f(Z4[o])));
}

// Adam on FP32 master weights; refreshes the BF16 copy when bf is given.
// c1 = 1 - b1^step and c2 = 1 - b2^step come from the host in FP64 (in FP32,
// 1 - 0.999^step loses ~1e-5 to cancellation), and 1 - b1, 1 - b2 are the
// FP32 roundings of 0.1 and 0.001 rather than differences of rounded betas.
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, bf16* __restrict__ bf, int64_t n, float lr, float c1,
                       float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float b1 = 0.9f, b2 = 0.999f, omb1 = 0.1f, omb2 = 0.001f, eps = 1e-8f;
    const float gi = g[i];
    const float mi = b1 * m[i] + omb1 * gi;
    const float vi = b2 * v[i] + omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (bf) bf[i] = f2bf(wi);
}

// Training batch: rows perm(step * batch + i) of X / T, where perm(j) =
// (a j + c) mod n for a coprime to n (a fresh permutation every epoch).
__global__ void k_gather_rows(const bf16* __restrict__ Xall, const float* __restrict__ Tall, int64_t n,
                              uint64_t a, uint64_t c, int64_t j0, int batch, bf16* __restrict__ X,
                              float* __restrict__ T)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)batch * D_IN) return;
    const int64_t i = e / D_IN, f = e % D_IN;
    const uint64_t r = ((unsigned __int128)a * (uint64_t)(j0 + i) + c) % (uint64_t)n;
    X[e] = Xall[r * D_IN + f];
    if (f == 0) T[i] = Tall[r];
}

// hist[0] += loss[0] / n (one thread: the epoch's mean squared error)
__global__ void k_add_loss(const float* __restrict__ loss, float inv_n, float* __restrict__ hist)
{
    hist[0] += loss[0] * inv_n;
}

__global__ void k_refresh_bf16(const float* __restrict__ w, bf16* __restrict__ bf, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) bf[i] = f2bf(w[i]);
}

// packed parameter layout (FP32): W0[16][256] b0[256] W1[256][256] b1 W2 b2 W3 b3 w4[256] b4[1]
constexpr int64_t kSizeW0 = (int64_t)D_IN * W;
constexpr int64_t kSizeWh = (int64_t)W * W;
constexpr int64_t kOffW4 = kSizeW0 + W + 3 * (kSizeWh + W);
constexpr int64_t kOffB4 = kOffW4 + W;
constexpr int64_t kNParam = kOffB4 + 1;

__host__ __device__ constexpr int64_t off_w(int l) { return l == 0 ? 0 : kSizeW0 + W + (int64_t)(l - 1) * (kSizeWh + W); }
__host__ __device__ constexpr int64_t off_b(int l) { return off_w(l) + (l == 0 ? kSizeW0 : kSizeWh); }
constexpr int64_t in_dim(int l) { return l == 0 ? D_IN : W; }

// ---------------------------------------------------------------- fused inference
// The whole network for a block of rows in one kernel, activations kept in
// registers from layer to layer.  Each layer is computed transposed,
// H^T[out][row] = W^T[out][in] X^T[in][row], with the weights as the MFMA A
// operand (from LDS, one layer at a time) and the activations as the B
// operand: lane l holds sample l%16.  The accumulator tiles of one layer are
// then the B operands of the next with no data movement: the two 16-feature
// tiles 2kb and 2kb+1 give lane group g the features
// {32kb + 4g + i} and {32kb + 16 + 4g + i} (i < 4), which become the 8 K values
// of K block kb when the next layer's weights are stored with their input
// features in that order (kInK below).
constexpr int kInferWaves = 4;                              // one wavefront per SIMD (512 registers)
constexpr int kInferTiles = 2;                              // 16-sample tiles per wavefront
constexpr int kInferRows = kInferWaves * kInferTiles * 16;  // rows per block and round
constexpr int kW0K = 32;                                    // layer-0 K (16 features, zero-padded)
constexpr int kWP = W + 8;                                  // LDS pitch of a prepared weight row
// weight loads in flight per thread: 8 measured 3.5 % faster per gated step
// than 16 (whose 32 more registers per lane keep the hard chain's larger
// kernels off the SIMDs the inference holds) and 0.5 % faster than 4
constexpr int kInferStage = 8;
static_assert(W == kInferWaves * 64, "one bias per thread of the inference block");
constexpr int64_t kInferW = (int64_t)W * kW0K + 3 * (int64_t)W * W;  // prepared weights (bf16)

// input feature at position kp of the permuted K order of a hidden layer
__host__ __device__ constexpr int kInK(int kp)
{
    return 32 * (kp / 32) + 4 * ((kp % 32) / 8) + ((kp % 8) < 4 ? (kp % 8) : 12 + (kp % 8));
}

// prepared weights: layer 0 as [256 out][32 k] (k >= 16 zero), layers 1..3 as
// [256 out][256 k'] with input feature kInK(k') at position k'
__global__ void k_prep_infer(const float* __restrict__ p, bf16* __restrict__ wt)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kInferW) return;
    if (i < (int64_t)W * kW0K) {
        const int out = (int)(i / kW0K), k = (int)(i % kW0K);
        wt[i] = k < D_IN ? f2bf(p[(int64_t)k * W + out]) : (bf16)0;
        return;
    }
    const int64_t e = i - (int64_t)W * kW0K;
    const int l = 1 + (int)(e / ((int64_t)W * W));
    const int r = (int)(e % ((int64_t)W * W));
    const int out = r / W, kp = r % W;
    wt[i] = f2bf(p[off_w(l) + (int64_t)kInK(kp) * W + out]);
}

// y[r] = network(X[r]) for r < n, n = min(n_cap, *n_dev) (or n_cap); X BF16
// [rows][16]; persistent over blocks of kInferRows rows
__global__ void __launch_bounds__(kInferWaves * 64)
k_mlp_infer(const bf16* __restrict__ X, int64_t n_cap, const unsigned long long* __restrict__ n_dev,
            const bf16* __restrict__ wt, const float* __restrict__ p, float* __restrict__ y)
{
    __shared__ __align__(16) bf16 Wl[W][kWP];
    __shared__ float bl[W];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, lg = lane >> 4;
    int64_t n = n_cap;
    if (n_dev) n = min(n, (int64_t)*n_dev);
    const float b4 = p[kOffB4];
    for (int64_t r0 = (int64_t)blockIdx.x * kInferRows; r0 < n; r0 += (int64_t)gridDim.x * kInferRows) {
        u32x4_t hb[kInferTiles][W / 32];   // B operands of the next layer (BF16 pairs)
        float4_t acc[kInferTiles][W / 16];
        // layer 0 input: K values 8 lg .. 8 lg + 7 of sample lr (features >= 16 are zero)
        bf16x8_t xb[kInferTiles];
        for (int s = 0; s < kInferTiles; ++s) {
            const int64_t row = r0 + (int64_t)(wave * kInferTiles + s) * 16 + lr;
            u32x4_t v = {0u, 0u, 0u, 0u};
            if (lg < 2 && row < n) v = *reinterpret_cast<const u32x4_t*>(X + row * D_IN + 8 * lg);
            xb[s] = as_bf8(v);
        }
        for (int l = 0; l < DEPTH; ++l) {
            const int kw = l == 0 ? kW0K : W;
            const bf16* src = l == 0 ? wt : wt + (int64_t)W * kW0K + (int64_t)(l - 1) * W * W;
            __syncthreads();  // the previous layer is done with Wl
            {
                // the layer's weights (16-byte pieces) and biases into LDS,
                // kInferStage loads in flight per thread before the first
                // store (a load-wait-store loop waits once per piece)
                constexpr int kT = kInferWaves * 64;
                const int n16 = W * kw / 8;
                const float bv = p[off_b(l) + tid];  // W == kT: one bias per thread
                for (int e0 = tid; e0 < n16; e0 += kT * kInferStage) {
                    u32x4_t v[kInferStage];
#pragma unroll
                    for (int j = 0; j < kInferStage; ++j)
                        if (e0 + j * kT < n16) v[j] = *reinterpret_cast<const u32x4_t*>(src + 8 * (e0 + j * kT));
#pragma unroll
                    for (int j = 0; j < kInferStage; ++j) {
                        const int e = 8 * (e0 + j * kT);
                        if (e0 + j * kT < n16) *reinterpret_cast<u32x4_t*>(&Wl[e / kw][e % kw]) = v[j];
                    }
                }
                bl[tid] = bv;
            }
            __syncthreads();
            for (int t = 0; t < W / 16; ++t) {
                for (int s = 0; s < kInferTiles; ++s) acc[s][t] = float4_t{0.f, 0.f, 0.f, 0.f};
                if (l == 0) {
                    const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(&Wl[t * 16 + lr][8 * lg]);
                    for (int s = 0; s < kInferTiles; ++s) acc[s][t] = mfma32(a, xb[s], acc[s][t]);
                } else {
                    for (int kb = 0; kb < W / 32; ++kb) {
                        const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(&Wl[t * 16 + lr][32 * kb + 8 * lg]);
                        for (int s = 0; s < kInferTiles; ++s) acc[s][t] = mfma32(a, as_bf8(hb[s][kb]), acc[s][t]);
                    }
                }
            }
            // bias + GELU, rounded to BF16: tiles 2kb, 2kb+1 -> K block kb
            for (int s = 0; s < kInferTiles; ++s)
                for (int kb = 0; kb < W / 32; ++kb) {
                    bf16 h[8];
                    for (int u = 0; u < 2; ++u)
                        for (int i = 0; i < 4; ++i) {
                            const int f = (2 * kb + u) * 16 + 4 * lg + i;
                            h[4 * u + i] = f2bf(gelu(acc[s][2 * kb + u][i] + bl[f]));
                        }
                    hb[s][kb] = u32x4_t{pack2(h[0], h[1]), pack2(h[2], h[3]), pack2(h[4], h[5]), pack2(h[6], h[7])};
                }
        }
        // output layer in FP32 on the BF16 activations, features summed over
        // the four lane groups
        for (int s = 0; s < kInferTiles; ++s) {
            float a = 0.f;
            for (int kb = 0; kb < W / 32; ++kb)
                for (int j = 0; j < 8; ++j) {
                    const int f = 32 * kb + 4 * lg + (j < 4 ? j : 12 + j);
                    a = fmaf(bf2f(half_of(hb[s][kb], j)), p[kOffW4 + f], a);
                }
            a += __shfl_xor(a, 16);
            a += __shfl_xor(a, 32);
            const int64_t row = r0 + (int64_t)(wave * kInferTiles + s) * 16 + lr;
            if (lg == 0 && row < n) y[row] = a + b4;
        }
    }
}

}  // namespace

struct gl_mlp {
    int device = 0;
    int max_batch = 0;
    int64_t step = 0;
    std::string err;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;  // master, grad, Adam
    bf16* pb = nullptr;                                             // BF16 copy of all params
    bf16 *X = nullptr, *Z[DEPTH] = {}, *H[DEPTH] = {}, *dA = nullptr, *dB = nullptr;
    float *y = nullptr, *dy = nullptr, *sq = nullptr, *lossbuf = nullptr;
    float* part = nullptr;      // split-K and column-sum partials
    bf16* wt = nullptr;         // weights prepared for the fused inference kernel
    bool wt_stale = true;       // master weights changed since wt was prepared
    int n_cu = 256;
};

namespace {

gl_status mfail(gl_mlp* m, gl_status st, const char* what, hipError_t e = hipSuccess)
{
    if (m) {
        m->err = what;
        if (e != hipSuccess) {
            m->err += ": ";
            m->err += hipGetErrorString(e);
        }
    }
    return st;
}

#define GM_HIP(call, what)                                                 \
    do {                                                                   \
        hipError_t e_ = (call);                                            \
        if (e_ != hipSuccess) return mfail(mm, GL_ERR_DEVICE, what, e_);   \
    } while (0)

constexpr int64_t kPartFloats = (int64_t)1 << 22;  // partial sums buffer (16 MB)
constexpr int kColRows = 256;                          // rows per column-sum partial

unsigned blocks(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

template <bool TA, bool TB, int EPI>
void gemm(hipStream_t s, int M, int N, int K, const bf16* A, int lda, const bf16* B, int ldb,
          const float* bias, const bf16* Zp, bf16* Zout, bf16* Hout, float* Fout, int ldc)
{
    dim3 grid((N + kGT - 1) / kGT, (M + kGT - 1) / kGT, 1);
    hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), grid, dim3(256), 0, s, M, N, K, K, A, lda, B, ldb, bias,
                       Zp, Zout, Hout, Fout, ldc);
}

// out[M][N] = A^T B with A stored [K][M], B [K][N] and K long (a weight
// gradient over the batch): K split over enough blocks to fill the GPU, the
// splits summed in order
void gemm_dw(gl_mlp* mm, hipStream_t s, int M, int N, int K, const bf16* A, const bf16* B, float* out)
{
    const int tiles = ((M + kGT - 1) / kGT) * ((N + kGT - 1) / kGT);
    int S = std::max(1, std::min(64, (2 * mm->n_cu + tiles - 1) / tiles));
    int kchunk = ((K + S - 1) / S + kGK - 1) / kGK * kGK;
    S = (K + kchunk - 1) / kchunk;
    while ((int64_t)S * M * N > kPartFloats) {
        kchunk *= 2;
        S = (K + kchunk - 1) / kchunk;
    }
    dim3 grid((N + kGT - 1) / kGT, (M + kGT - 1) / kGT, S);
    hipLaunchKernelGGL((k_gemm<true, false, EPI_DW>), grid, dim3(256), 0, s, M, N, K, kchunk, A, M, B, N,
                       nullptr, nullptr, nullptr, nullptr, mm->part, N);
    hipLaunchKernelGGL(k_reduce_parts, dim3(blocks((int64_t)M * N)), dim3(256), 0, s, mm->part, S,
                       (int64_t)M * N, out);
}

// out[c] = sum_m X[m][c] (* w[m]) over n rows of a [n][ld] BF16 matrix, in a fixed order
template <bool SCALE>
void colsum(gl_mlp* mm, hipStream_t s, const bf16* X, int ld, int n, const float* w, float* out)
{
    const int R = (n + kColRows - 1) / kColRows;
    hipLaunchKernelGGL((k_colsum<true, SCALE>), dim3((ld + 63) / 64, R), dim3(256), 0, s, X, ld, n, kColRows, w,
                       mm->part);
    hipLaunchKernelGGL(k_reduce_parts, dim3(blocks(ld)), dim3(256), 0, s, mm->part, R, (int64_t)ld, out);
}

// forward of n <= max_batch rows already converted to BF16 in mm->X
void forward_bf(gl_mlp* mm, int n, hipStream_t s)
{
    const bf16* in = mm->X;
    for (int l = 0; l < DEPTH; ++l) {
        gemm<false, false, EPI_FWD>(s, n, W, (int)in_dim(l), in, (int)in_dim(l), mm->pb + off_w(l), W,
                                    mm->p + off_b(l), nullptr, mm->Z[l], mm->H[l], nullptr, W);
        in = mm->H[l];
    }
    hipLaunchKernelGGL(k_out_fwd, dim3(blocks(n)), dim3(256), 0, s, mm->H[DEPTH - 1], mm->p + kOffW4,
                       mm->p + kOffB4, mm->y, n);
}

// gradients of the mean squared error into mm->g (after forward_bf)
void backward(gl_mlp* mm, const float* t, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_out_bwd, dim3(n), dim3(256), 0, s, mm->y, t, mm->p + kOffW4, mm->Z[DEPTH - 1],
                       mm->dy, mm->sq, mm->dA, n);
    // output layer: g_w4[k] = sum_m dy[m] H4[m][k], g_b4 = sum_m dy[m], loss = sum sq
    colsum<true>(mm, s, mm->H[DEPTH - 1], W, n, mm->dy, mm->g + kOffW4);
    hipLaunchKernelGGL(k_vecsum, dim3(1), dim3(256), 0, s, mm->dy, n, mm->g + kOffB4);
    hipLaunchKernelGGL(k_vecsum, dim3(1), dim3(256), 0, s, mm->sq, n, mm->lossbuf);
    bf16* dZ = mm->dA;   // dL/dZ of the current layer
    bf16* spare = mm->dB;
    for (int l = DEPTH - 1; l >= 0; --l) {
        const bf16* in = (l == 0) ? mm->X : mm->H[l - 1];
        const int K_l = (int)in_dim(l);
        // dW_l[K_l][W] = in^T dZ  (A = in stored [n][K_l], read transposed)
        gemm_dw(mm, s, K_l, W, n, in, dZ, mm->g + off_w(l));
        colsum<false>(mm, s, dZ, W, n, nullptr, mm->g + off_b(l));
        if (l > 0) {
            // dZ_{l-1} = (dZ W_l^T) * gelu'(Z_{l-1}); W_l stored [K_l][W] = B^T layout
            gemm<false, true, EPI_DX>(s, n, K_l, W, dZ, W, mm->pb + off_w(l), W, nullptr, mm->Z[l - 1],
                                      nullptr, spare, nullptr, W);
            bf16* tmp = dZ;
            dZ = spare;
            spare = tmp;
        }
    }
}

// refreshes the fused kernel's prepared weights if the masters changed
void prepare_infer(gl_mlp* mm, hipStream_t s)
{
    if (!mm->wt_stale) return;
    hipLaunchKernelGGL(k_prep_infer, dim3(blocks(kInferW)), dim3(256), 0, s, mm->p, mm->wt);
    mm->wt_stale = false;
}

void launch_infer(gl_mlp* mm, const bf16* X, int64_t n_cap, const unsigned long long* n_dev, float* y,
                  hipStream_t s)
{
    prepare_infer(mm, s);
    const int64_t rounds = (n_cap + kInferRows - 1) / kInferRows;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(rounds, mm->n_cu));
    hipLaunchKernelGGL(k_mlp_infer, dim3(grid), dim3(kInferWaves * 64), 0, s, X, n_cap, n_dev, mm->wt, mm->p, y);
}

}  // namespace

extern "C" {

int gl_mlp_num_params(void) { return (int)kNParam; }

gl_status gl_mlp_create(gl_mlp** out, int device, int max_batch)
{
    if (!out) return GL_ERR_NULL;
    *out = nullptr;
    if (max_batch < 64 || max_batch > (1 << 22) || max_batch % 64) return GL_ERR_SIZE;
    if (hipSetDevice(device) != hipSuccess) return GL_ERR_DEVICE;
    gl_mlp* mm = new (std::nothrow) gl_mlp();
    if (!mm) return GL_ERR_NOMEM;
    mm->device = device;
    mm->max_batch = max_batch;
    bool ok = true;
    auto al = [&](void** pp, size_t bytes) {
        if (hipMalloc(pp, bytes) != hipSuccess) ok = false;
    };
    al((void**)&mm->p, sizeof(float) * kNParam);
    al((void**)&mm->g, sizeof(float) * kNParam);
    al((void**)&mm->m, sizeof(float) * kNParam);
    al((void**)&mm->v, sizeof(float) * kNParam);
    al((void**)&mm->pb, sizeof(bf16) * kNParam);
    al((void**)&mm->X, sizeof(bf16) * (size_t)max_batch * D_IN);
    for (int l = 0; l < DEPTH; ++l) {
        al((void**)&mm->Z[l], sizeof(bf16) * (size_t)max_batch * W);
        al((void**)&mm->H[l], sizeof(bf16) * (size_t)max_batch * W);
    }
    al((void**)&mm->dA, sizeof(bf16) * (size_t)max_batch * W);
    al((void**)&mm->dB, sizeof(bf16) * (size_t)max_batch * W);
    al((void**)&mm->y, sizeof(float) * 2 * (size_t)max_batch);  // outputs, then a batch's targets
    al((void**)&mm->dy, sizeof(float) * max_batch);
    al((void**)&mm->sq, sizeof(float) * max_batch);
    al((void**)&mm->lossbuf, sizeof(float) * 4);
    al((void**)&mm->part, sizeof(float) * kPartFloats);
    al((void**)&mm->wt, sizeof(bf16) * kInferW);
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
        mm->n_cu = ncu;
    if (ok) {
        ok = hipMemset(mm->p, 0, sizeof(float) * kNParam) == hipSuccess &&
             hipMemset(mm->g, 0, sizeof(float) * kNParam) == hipSuccess &&
             hipMemset(mm->m, 0, sizeof(float) * kNParam) == hipSuccess &&
             hipMemset(mm->v, 0, sizeof(float) * kNParam) == hipSuccess &&
             hipMemset(mm->pb, 0, sizeof(bf16) * kNParam) == hipSuccess &&
             hipDeviceSynchronize() == hipSuccess;
    }
    if (!ok) {
        gl_mlp_destroy(mm);
        return GL_ERR_NOMEM;
    }
    *out = mm;
    return GL_OK;
}

void gl_mlp_destroy(gl_mlp* mm)
{
    if (!mm) return;
    (void)hipSetDevice(mm->device);
    (void)hipDeviceSynchronize();
    void* bufs[] = {mm->p, mm->g, mm->m, mm->v, mm->pb, mm->X, mm->dA, mm->dB, mm->y, mm->dy, mm->sq,
                    mm->lossbuf, mm->part, mm->wt};
    for (void* b : bufs) (void)hipFree(b);
    for (int l = 0; l < DEPTH; ++l) {
        (void)hipFree(mm->Z[l]);
        (void)hipFree(mm->H[l]);
    }
    delete mm;
}

const char* gl_mlp_last_error(const gl_mlp* mm) { return mm ? mm->err.c_str() : "null network"; }

gl_status gl_mlp_set_weights(gl_mlp* mm, const float* host, int64_t n)
{
    if (!mm || !host) return GL_ERR_NULL;
    if (n != kNParam) return mfail(mm, GL_ERR_SIZE, "parameter count");
    GM_HIP(hipSetDevice(mm->device), "hipSetDevice");
    GM_HIP(hipMemcpy(mm->p, host, sizeof(float) * kNParam, hipMemcpyHostToDevice), "hipMemcpy");
    GM_HIP(hipMemset(mm->m, 0, sizeof(float) * kNParam), "hipMemset");
    GM_HIP(hipMemset(mm->v, 0, sizeof(float) * kNParam), "hipMemset");
    hipLaunchKernelGGL(k_refresh_bf16, dim3(blocks(kNParam)), dim3(256), 0, 0, mm->p, mm->pb, kNParam);
    mm->wt_stale = true;
    prepare_infer(mm, 0);
    GM_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    mm->step = 0;
    return GL_OK;
}

gl_status gl_mlp_get_weights(const gl_mlp* mmc, float* host, int64_t n)
{
    gl_mlp* mm = const_cast<gl_mlp*>(mmc);
    if (!mm || !host) return GL_ERR_NULL;
    if (n != kNParam) return mfail(mm, GL_ERR_SIZE, "parameter count");
    GM_HIP(hipSetDevice(mm->device), "hipSetDevice");
    GM_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    GM_HIP(hipMemcpy(host, mm->p, sizeof(float) * kNParam, hipMemcpyDeviceToHost), "hipMemcpy");
    return GL_OK;
}

gl_status gl_mlp_forward(gl_mlp* mm, const float* x, int64_t n, float* y, void* stream)
{
    if (!mm || !x || !y) return GL_ERR_NULL;
    if (n < 0) return mfail(mm, GL_ERR_SIZE, "n < 0");
    GM_HIP(hipSetDevice(mm->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    // fused kernel over chunks of max_batch rows converted to BF16
    for (int64_t r0 = 0; r0 < n; r0 += mm->max_batch) {
        const int nb = (int)std::min<int64_t>(mm->max_batch, n - r0);
        hipLaunchKernelGGL(k_to_bf16, dim3(blocks((int64_t)nb * D_IN)), dim3(256), 0, s,
                           x + r0 * D_IN, mm->X, (int64_t)nb * D_IN);
        launch_infer(mm, mm->X, nb, nullptr, y + r0, s);
    }
    GM_HIP(hipGetLastError(), "kernel launch");
    return GL_OK;
}

gl_status gl_mlp_grads(gl_mlp* mm, const float* x, const float* t, int64_t n, float* host_grads,
                       float* host_loss, void* stream)
{
    if (!mm || !x || !t || !host_grads) return GL_ERR_NULL;
    if (n < 1 || n > mm->max_batch) return mfail(mm, GL_ERR_SIZE, "1 <= n <= max_batch");
    GM_HIP(hipSetDevice(mm->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks(n * D_IN)), dim3(256), 0, s, x, mm->X, n * D_IN);
    forward_bf(mm, (int)n, s);
    backward(mm, t, (int)n, s);
    GM_HIP(hipGetLastError(), "kernel launch");
    GM_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    GM_HIP(hipMemcpy(host_grads, mm->g, sizeof(float) * kNParam, hipMemcpyDeviceToHost), "hipMemcpy");
    if (host_loss) {
        float l = 0.f;
        GM_HIP(hipMemcpy(&l, mm->lossbuf, sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy");
        *host_loss = l / (float)n;
    }
    return GL_OK;
}

// loss_dev (device, optional) receives the batch's sum of squared residuals
gl_status gl_mlp_train_step(gl_mlp* mm, const float* x, const float* t, int64_t n, float lr,
                            float* loss_dev, void* stream)
{
    if (!mm || !x || !t) return GL_ERR_NULL;
    if (n < 1 || n > mm->max_batch) return mfail(mm, GL_ERR_SIZE, "1 <= n <= max_batch");
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks(n * D_IN)), dim3(256), 0, s, x, mm->X, n * D_IN);
    forward_bf(mm, (int)n, s);
    backward(mm, t, (int)n, s);
    mm->step += 1;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)mm->step));
    const float c2 = (float)(1.0 - std::pow(0.999, (double)mm->step));
    hipLaunchKernelGGL(k_adam, dim3(blocks(kNParam)), dim3(256), 0, s, mm->p, mm->g, mm->m, mm->v,
                       mm->pb, kNParam, lr, c1, c2);
    mm->wt_stale = true;
    if (loss_dev)
        GM_HIP(hipMemcpyAsync(loss_dev, mm->lossbuf, sizeof(float), hipMemcpyDeviceToDevice, s),
               "hipMemcpyAsync");
    GM_HIP(hipGetLastError(), "kernel launch");
    return GL_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- internal calls
namespace gl_net {

namespace {
uint64_t mix64(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
uint64_t gcd64(uint64_t a, uint64_t b)
{
    while (b) {
        const uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}
}  // namespace

int max_batch(const gl_mlp* mm) { return mm->max_batch; }

gl_status train_rows(gl_mlp* mm, const uint16_t* X, const float* T, int64_t n, int epochs, int batch,
                     float lr, float lr_final, uint64_t seed, float* hist_dev, hipStream_t s)
{
    if (!mm || !X || !T) return GL_ERR_NULL;
    if (batch < 64 || batch > mm->max_batch || n < batch || epochs < 1) return mfail(mm, GL_ERR_SIZE, "training sizes");
    GM_HIP(hipSetDevice(mm->device), "hipSetDevice");
    const int64_t per_epoch = n / batch;
    const int64_t steps = per_epoch * epochs;
    int64_t step = 0;
    for (int ep = 0; ep < epochs; ++ep) {
        // a fresh permutation j -> (a j + c) mod n
        uint64_t a = (mix64(seed * 1315423911ull + (uint64_t)ep) % (uint64_t)n) | 1ull;
        while (gcd64(a, (uint64_t)n) != 1ull) a += 2;
        const uint64_t c = mix64(seed + 7919ull * (uint64_t)(ep + 1)) % (uint64_t)n;
        for (int64_t b = 0; b < per_epoch; ++b, ++step) {
            hipLaunchKernelGGL(k_gather_rows, dim3(blocks((int64_t)batch * D_IN)), dim3(256), 0, s, (const bf16*)X, T, n,
                               a % (uint64_t)n, c, b * batch, batch, mm->X, mm->y + mm->max_batch);
            const float lr_s = (float)((double)lr * std::pow((double)lr_final / (double)lr,
                                                             (double)step / (double)std::max<int64_t>(1, steps - 1)));
            forward_bf(mm, batch, s);
            backward(mm, mm->y + mm->max_batch, batch, s);
            mm->step += 1;
            const float c1 = (float)(1.0 - std::pow(0.9, (double)mm->step));
            const float c2 = (float)(1.0 - std::pow(0.999, (double)mm->step));
            hipLaunchKernelGGL(k_adam, dim3(blocks(kNParam)), dim3(256), 0, s, mm->p, mm->g, mm->m, mm->v, mm->pb,
                               kNParam, lr_s, c1, c2);
            if (hist_dev)
                hipLaunchKernelGGL(k_add_loss, dim3(1), dim3(1), 0, s, mm->lossbuf, 1.0f / (float)(per_epoch * batch),
                                   hist_dev + ep);
        }
    }
    mm->wt_stale = true;
    GM_HIP(hipGetLastError(), "kernel launch");
    return GL_OK;
}

void infer(gl_mlp* mm, const uint16_t* X, int64_t n_cap, const unsigned long long* n_dev, float* y, hipStream_t s)
{
    launch_infer(mm, (const bf16*)X, n_cap, n_dev, y, s);
}

gl_status get_state(const gl_mlp* mmc, float* m, float* v, int64_t* step)
{
    gl_mlp* mm = const_cast<gl_mlp*>(mmc);
    if (!mm || !m || !v || !step) return GL_ERR_NULL;
    GM_HIP(hipSetDevice(mm->device), "hipSetDevice");
    GM_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    GM_HIP(hipMemcpy(m, mm->m, sizeof(float) * kNParam, hipMemcpyDeviceToHost), "hipMemcpy");
    GM_HIP(hipMemcpy(v, mm->v, sizeof(float) * kNParam, hipMemcpyDeviceToHost), "hipMemcpy");
    *step = mm->step;
    return GL_OK;
}

gl_status set_state(gl_mlp* mm, const float* m, const float* v, int64_t step)
{
    if (!mm || !m || !v) return GL_ERR_NULL;
    GM_HIP(hipSetDevice(mm->device), "hipSetDevice");
    GM_HIP(hipMemcpy(mm->m, m, sizeof(float) * kNParam, hipMemcpyHostToDevice), "hipMemcpy");
    GM_HIP(hipMemcpy(mm->v, v, sizeof(float) * kNParam, hipMemcpyHostToDevice), "hipMemcpy");
    mm->step = step;
    return GL_OK;
}

}  // namespace gl_net
