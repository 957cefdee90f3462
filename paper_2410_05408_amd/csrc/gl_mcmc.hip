// gl_mcmc.hip -- the glue an MCMC fit puts around the light curves (Section 3
// and Appendix A of arXiv:2410.05408):
//
//   k_prior_mu_nu   the inverse-transform sampler of the (mu, nu) prior: two
//                   uniforms per draw, supplied by the caller, give
//                   nu = u^2 / (u^2 - 2u + 2) (inverse of the marginal CDF of
//                   nu) and mu (inverse of the conditional CDF F(mu | nu))
//   k_walk_params   walker block (the fitting parameters r, mu, nu, xi, b,
//                   d/R*, P, t0, q1, q2) to the oblate parameter block:
//                   f = f_min + (1 - f_min) nu with f_min = 1 - sqrt((mu+1)/2),
//                   cos(2 eta) from eq. mu (eta in [0, pi/2]), theta = pi/2 - eta,
//                   equatorial radius k = r / cbrt(1 - f) (r: geometric mean
//                   of the three semi-axes, r^3 = k^3 (1 - f))
//   k_loglike       per-walker white-noise chi^2 and log-likelihood of a
//                   model light curve against data: one wavefront per walker,
//                   a fixed-order reduction (bitwise reproducible)
// (the light-curve batch of gl_loglike_batch converts its walkers inside its
// own set-up kernel, with the same walker_to_params)
//
// All three are bandwidth-light elementwise or streaming kernels; the
// light-curve batch between the first two and the last is the work.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "gl.h"
#include "gl_device.h"
#include "gl_internal.h"

namespace {

constexpr int kLLThreads = 256;
constexpr double kLog2Pi = 1.8378770664093454836;  // log(2 pi)

__device__ __forceinline__ bool finite(double x) { return fabs(x) <= 1.7976931348623157e308; }

__global__ void __launch_bounds__(256)
k_prior_mu_nu(const double* __restrict__ uw, int64_t n, double* __restrict__ mu_nu)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double u = uw[i], w = uw[n + i];
    double mu = __builtin_nan(""), nu = __builtin_nan("");
    // u = 1 is nu = 1, where the conditional CDF degenerates (f = 1)
    if (finite(u) && finite(w) && u >= 0.0 && u < 1.0 && w >= 0.0 && w <= 1.0) {
        nu = u * u / (u * u - 2.0 * u + 2.0);
        const double s = sqrt(nu * (2.0 - nu));
        const double g = (nu - 1.0) * (nu - 1.0);
        mu = (4.0 * w + 4.0 * (w * w - w) * s + 2.0 * (nu * (nu - 2.0) - 1.0) * w * w - g) / g;
    }
    mu_nu[i] = mu;
    mu_nu[n + i] = nu;
}

__global__ void __launch_bounds__(256)
k_walk_params(const double* __restrict__ walk, int64_t n, double* __restrict__ params)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double w[gl::kWalkParams], p[GL_NPARAM];
    for (int row = 0; row < gl::kWalkParams; ++row) w[row] = walk[row * n + i];
    gl::walker_to_params(w, p);
    for (int row = 0; row < GL_NPARAM; ++row) params[row * n + i] = p[row];
}

// Sum of a value per thread over the workgroup in a fixed order: butterfly
// within each wavefront, then the wavefronts' sums in index order.
__device__ double block_sum(double v, double* lds)
{
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) lds[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < kLLThreads / 64; ++k) s += lds[k];
    __syncthreads();
    return s;  // valid in thread 0
}

// Shared grid: the normalisation sum log(sigma) + (N/2) log(2 pi) is the same
// for every walker, so one workgroup forms it once and finishes every
// walker's log-likelihood from the chi^2 that k_loglike left in ll.
__global__ void __launch_bounds__(kLLThreads) k_loglike_finish(const double* __restrict__ sigma, int64_t n_times,
                                                              int64_t n_sets, double* __restrict__ ll)
{
    __shared__ double lds[kLLThreads / 64];
    __shared__ double norm;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n_times; i += kLLThreads) acc += log(sigma[i]);
    const double s = block_sum(acc, lds);
    if (threadIdx.x == 0) norm = s + 0.5 * (double)n_times * kLog2Pi;
    __syncthreads();
    for (int64_t w = threadIdx.x; w < n_sets; w += kLLThreads) ll[w] = -0.5 * ll[w] - norm;
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

// One wavefront per walker (four per workgroup: a shared grid's data and
// sigma are read once per workgroup from the caches).  The data set of a
// likelihood batch is about one latency-bandwidth product of HBM, so each
// lane issues all kLLUnroll loads of a 64 x kLLUnroll slice before it does any
// arithmetic; per-lane sums run in a fixed order, then a fixed butterfly.
// With `norm` (a shared grid's sum log(sigma) + (N/2) log(2 pi), computed
// before) the log-likelihood is finished here; without it, a shared grid
// leaves chi^2 in ll for k_loglike_finish.
constexpr int kLLUnroll = 16;

template <bool CSR>
__global__ void __launch_bounds__(kLLThreads)
k_loglike(const double* __restrict__ model, int64_t n_sets, const int64_t* __restrict__ offsets, int64_t n_times,
          const double* __restrict__ data, const double* __restrict__ sigma, const double* __restrict__ norm,
          double* __restrict__ chi2, double* __restrict__ ll)
{
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (kLLThreads / 64);
    for (int64_t s = (int64_t)blockIdx.x * (kLLThreads / 64) + (threadIdx.x >> 6); s < n_sets; s += waves) {
        int64_t a = 0, len = n_times;
        bool ok = true;
        if (CSR) {
            a = offsets[s];
            const int64_t b = offsets[s + 1];
            ok = a >= 0 && b >= a && b <= n_times;
            len = ok ? b - a : 0;
        }
        const double* m = model + (CSR ? a : s * n_times);
        const double* d = data + a;
        const double* sg = sigma + a;
        double acc = 0.0, accl = 0.0;
        for (int64_t i0 = 0; i0 < len; i0 += 64 * kLLUnroll) {
            double mv[kLLUnroll], dv[kLLUnroll], sv[kLLUnroll];
#pragma unroll
            for (int k = 0; k < kLLUnroll; ++k) {
                const int64_t j = i0 + lane + 64 * k;
                const bool in = j < len;
                mv[k] = in ? m[j] : 0.0;
                dv[k] = in ? d[j] : 0.0;
                sv[k] = in ? sg[j] : 1.0;
            }
#pragma unroll
            for (int k = 0; k < kLLUnroll; ++k) {
                const double r = (dv[k] - mv[k]) / sv[k];
                acc += r * r;
                if (CSR && i0 + lane + 64 * k < len) accl += log(sv[k]);
            }
        }
        const double c = wave_sum(acc);
        const double l = CSR ? wave_sum(accl) : 0.0;
        if (lane == 0) {
            const double cc = ok ? c : __builtin_nan("");
            if (chi2) chi2[s] = cc;
            if (ll) {
                if (CSR) ll[s] = -0.5 * cc - (l + 0.5 * (double)len * kLog2Pi);
                else ll[s] = norm ? -0.5 * cc - norm[0] : cc;  // finished later without norm
            }
        }
    }
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

namespace gl_mcmc {

void launch_walk_params(const double* walk, int64_t n, double* params, hipStream_t st)
{
    hipLaunchKernelGGL(k_walk_params, dim3(blocks_for(n)), dim3(256), 0, st, walk, n, params);
}

void launch_loglike(const double* model, int64_t n_sets, const int64_t* offsets, int64_t n_times,
                    const double* data, const double* sigma, const double* norm, double* chi2, double* ll,
                    hipStream_t st)
{
    const int64_t blocks = (n_sets + kLLThreads / 64 - 1) / (kLLThreads / 64);
    const unsigned grid = (unsigned)(blocks < (int64_t)1 << 20 ? blocks : (int64_t)1 << 20);
    if (offsets)
        hipLaunchKernelGGL(k_loglike<true>, dim3(grid), dim3(kLLThreads), 0, st, model, n_sets, offsets, n_times, data,
                           sigma, norm, chi2, ll);
    else
        hipLaunchKernelGGL(k_loglike<false>, dim3(grid), dim3(kLLThreads), 0, st, model, n_sets, offsets, n_times,
                           data, sigma, norm, chi2, ll);
    if (!offsets && ll && !norm)
        hipLaunchKernelGGL(k_loglike_finish, dim3(1), dim3(kLLThreads), 0, st, sigma, n_times, n_sets, ll);
}

}  // namespace gl_mcmc

extern "C" {

gl_status gl_prior_mu_nu(const double* uw, int64_t n, double* mu_nu, void* stream)
{
    if (!uw || !mu_nu) return GL_ERR_NULL;
    if (n < 1) return GL_ERR_SIZE;
    hipLaunchKernelGGL(k_prior_mu_nu, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, uw, n, mu_nu);
    return hipGetLastError() == hipSuccess ? GL_OK : GL_ERR_DEVICE;
}

gl_status gl_walkers_to_params(const double* walkers, int64_t n, double* params, void* stream)
{
    if (!walkers || !params) return GL_ERR_NULL;
    if (n < 1) return GL_ERR_SIZE;
    gl_mcmc::launch_walk_params(walkers, n, params, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? GL_OK : GL_ERR_DEVICE;
}

gl_status gl_loglike_of_model(const double* model, int64_t n_sets, const int64_t* offsets, int64_t n_times,
                              const double* data, const double* sigma, double* chi2, double* loglike, void* stream)
{
    if (!model || !data || !sigma || (!chi2 && !loglike)) return GL_ERR_NULL;
    if (n_sets < 1 || n_times < (offsets ? 0 : 1)) return GL_ERR_SIZE;
    gl_mcmc::launch_loglike(model, n_sets, offsets, n_times, data, sigma, nullptr, chi2, loglike,
                            (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? GL_OK : GL_ERR_DEVICE;
}

}  // extern "C"
