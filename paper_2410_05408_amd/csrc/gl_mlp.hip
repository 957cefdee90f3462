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

__device__ __forceinline__ float gelu(float z)
{
    return 0.5f * z * (1.0f + tanhf(kGeluC * (z + 0.044715f * z * z * z)));
}
__device__ __forceinline__ float gelu_grad(float z)
{
    const float th = tanhf(kGeluC * (z + 0.044715f * z * z * z));
    const float du = kGeluC * (1.0f + 3.0f * 0.044715f * z * z);
    return 0.5f * (1.0f + th) + 0.5f * z * (1.0f - th * th) * du;
}

typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

enum Epi { EPI_FWD = 0, EPI_DX = 1, EPI_DW = 2 };

// C[M][N] = op(A)[M][K] * op(B)[K][N], 64x64 block tile, 4 wavefronts each
// owning a 32x32 quadrant made of 2x2 MFMA 16x16x16 tiles, K staged through
// LDS 16 at a time.  TA: A is stored [K][M] (read transposed).  TB: B is
// stored [N][K].  Out-of-range elements load as zero and are not stored.
//  EPI_FWD: z = acc + bias[n]; Z = bf16(z), H = bf16(gelu(z))
//  EPI_DX : out_bf = bf16(acc * gelu'(Zp[m][n]))
//  EPI_DW : out_f = acc
template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(256)
k_gemm(int M, int N, int K, const bf16* __restrict__ A, int lda, const bf16* __restrict__ B,
       int ldb, const float* __restrict__ bias, const bf16* __restrict__ Zp, bf16* __restrict__ Zout,
       bf16* __restrict__ Hout, float* __restrict__ Fout, int ldc)
{
    __shared__ bf16 As[64][16 + 2];
    __shared__ bf16 Bs[16][64 + 2];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    float4_t acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
        // stage A (64 x 16) and B (16 x 64): 1024 elements each, 4 per thread
        for (int e = tid; e < 64 * 16; e += 256) {
            const int r = e / 16, c = e % 16;  // A tile row r (m), col c (k)
            const int m = m0 + r, k = k0 + c;
            bf16 v = 0;
            if (m < M && k < K) v = TA ? A[(size_t)k * lda + m] : A[(size_t)m * lda + k];
            As[r][c] = v;
            const int kr = e / 64, nc = e % 64;  // B tile row kr (k), col nc (n)
            const int kk = k0 + kr, n = n0 + nc;
            bf16 w = 0;
            if (kk < K && n < N) w = TB ? B[(size_t)n * ldb + kk] : B[(size_t)kk * ldb + n];
            Bs[kr][nc] = w;
        }
        __syncthreads();
        // MFMA 16x16x16: a[i] = A[lane%16][4(lane/16)+i], b[i] = B[4(lane/16)+i][lane%16]
        const int lr = lane & 15, lk = (lane >> 4) * 4;
        short4_t a[2], b[2];
        for (int t = 0; t < 2; ++t) {
            for (int i = 0; i < 4; ++i) {
                a[t][i] = (short)As[wm + t * 16 + lr][lk + i];
                b[t][i] = (short)Bs[lk + i][wn + t * 16 + lr];
            }
        }
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // D[4(lane/16)+i][lane%16] of each 16x16 tile
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
                    Fout[o] = v;
                }
            }
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

// out[c] = sum_m X[m][c] (* s[m] if s), fixed-order tree over 256 threads; one block per column
template <bool BF, bool SCALE>
__global__ void __launch_bounds__(256)
k_colsum(const void* __restrict__ Xv, int ld, int n, const float* __restrict__ s, float* __restrict__ out)
{
    __shared__ float red[256];
    const int c = blockIdx.x, tid = threadIdx.x;
    float acc = 0.f;
    for (int m = tid; m < n; m += 256) {
        float v = BF ? bf2f(((const bf16*)Xv)[(size_t)m * ld + c]) : ((const float*)Xv)[(size_t)m * ld + c];
        if (SCALE) v *= s[m];
        acc += v;
    }
    red[tid] = acc;
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if (tid < d) red[tid] += red[tid + d];
        __syncthreads();
    }
    if (tid == 0) out[c] = red[0];
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

int64_t off_w(int l) { return l == 0 ? 0 : kSizeW0 + W + (int64_t)(l - 1) * (kSizeWh + W); }
int64_t off_b(int l) { return off_w(l) + (l == 0 ? kSizeW0 : kSizeWh); }
int64_t size_w(int l) { return l == 0 ? kSizeW0 : kSizeWh; }
int64_t in_dim(int l) { return l == 0 ? D_IN : W; }

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

template <bool TA, bool TB, int EPI>
void gemm(hipStream_t s, int M, int N, int K, const bf16* A, int lda, const bf16* B, int ldb,
          const float* bias, const bf16* Zp, bf16* Zout, bf16* Hout, float* Fout, int ldc)
{
    dim3 grid((N + 63) / 64, (M + 63) / 64);
    hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, bias,
                       Zp, Zout, Hout, Fout, ldc);
}

unsigned blocks(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

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
    // output layer: g_w4[k] = sum_m dy[m] H4[m][k], g_b4 = sum_m dy[m], loss = mean sq
    hipLaunchKernelGGL((k_colsum<true, true>), dim3(W), dim3(256), 0, s, mm->H[DEPTH - 1], W, n, mm->dy,
                       mm->g + kOffW4);
    hipLaunchKernelGGL((k_colsum<false, false>), dim3(1), dim3(256), 0, s, mm->dy, 1, n, nullptr,
                       mm->g + kOffB4);
    hipLaunchKernelGGL((k_colsum<false, false>), dim3(1), dim3(256), 0, s, mm->sq, 1, n, nullptr,
                       mm->lossbuf);
    bf16* dZ = mm->dA;   // dL/dZ of the current layer
    bf16* spare = mm->dB;
    for (int l = DEPTH - 1; l >= 0; --l) {
        const bf16* in = (l == 0) ? mm->X : mm->H[l - 1];
        const int K_l = (int)in_dim(l);
        // dW_l[K_l][W] = in^T dZ  (A = in stored [n][K_l], read transposed)
        gemm<true, false, EPI_DW>(s, K_l, W, n, in, K_l, dZ, W, nullptr, nullptr, nullptr, nullptr,
                                  mm->g + off_w(l), W);
        hipLaunchKernelGGL((k_colsum<true, false>), dim3(W), dim3(256), 0, s, dZ, W, n, nullptr,
                           mm->g + off_b(l));
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
    al((void**)&mm->y, sizeof(float) * max_batch);
    al((void**)&mm->dy, sizeof(float) * max_batch);
    al((void**)&mm->sq, sizeof(float) * max_batch);
    al((void**)&mm->lossbuf, sizeof(float) * 4);
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
                    mm->lossbuf};
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
    for (int64_t r0 = 0; r0 < n; r0 += mm->max_batch) {
        const int nb = (int)std::min<int64_t>(mm->max_batch, n - r0);
        hipLaunchKernelGGL(k_to_bf16, dim3(blocks((int64_t)nb * D_IN)), dim3(256), 0, s,
                           x + r0 * D_IN, mm->X, (int64_t)nb * D_IN);
        forward_bf(mm, nb, s);
        GM_HIP(hipMemcpyAsync(y + r0, mm->y, sizeof(float) * nb, hipMemcpyDeviceToDevice, s),
               "hipMemcpyAsync");
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
    if (loss_dev)
        GM_HIP(hipMemcpyAsync(loss_dev, mm->lossbuf, sizeof(float), hipMemcpyDeviceToDevice, s),
               "hipMemcpyAsync");
    GM_HIP(hipGetLastError(), "kernel launch");
    return GL_OK;
}

}  // extern "C"
