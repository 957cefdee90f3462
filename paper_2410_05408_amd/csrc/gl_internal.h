// gl_internal.h -- calls between the library's translation units (not part
// of the C ABI): the surrogate network's training loop, fused inference and
// optimizer state, used by the surrogate path of the light-curve library; the
// MCMC glue's launches, captured with a light-curve batch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gl.h"

namespace gl_net {

// Trains on n rows (X: BF16 [n][GL_MLP_DIN], T: FP32 targets), all device
// memory: `epochs` passes in a permuted order drawn from `seed`, `batch` rows
// per Adam step, learning rate log-linear from lr to lr_final.  hist_dev
// (device float[epochs], may be NULL) receives each epoch's mean squared
// error.  Enqueued on stream.
gl_status train_rows(gl_mlp* mm, const uint16_t* X, const float* T, int64_t n, int epochs, int batch,
                     float lr, float lr_final, uint64_t seed, float* hist_dev, hipStream_t stream);

// y[r] = network(X[r]) for r < min(n_cap, *n_dev) (n_dev may be NULL);
// X BF16 [n_cap][GL_MLP_DIN], device memory; enqueued on stream.
void infer(gl_mlp* mm, const uint16_t* X, int64_t n_cap, const unsigned long long* n_dev, float* y,
           hipStream_t stream);

// Adam state (host copies, gl_mlp_num_params() floats each) and step count.
gl_status get_state(const gl_mlp* mm, float* m, float* v, int64_t* step);
gl_status set_state(gl_mlp* mm, const float* m, const float* v, int64_t step);

int max_batch(const gl_mlp* mm);

}  // namespace gl_net

namespace gl_mcmc {

// Walker block [GL_W_NPARAM][n] -> oblate parameter block [GL_NPARAM][n].
void launch_walk_params(const double* walk, int64_t n, double* params, hipStream_t st);

// Per-walker chi^2 and log-likelihood of model against data / sigma (shared
// grid: model [n_sets][n_times], data and sigma [n_times]; CSR: all indexed
// alike by offsets).  chi2 or ll may be NULL.  norm (device, may be NULL):
// a shared grid's sum log(sigma) + (N/2) log(2 pi), already computed.
void launch_loglike(const double* model, int64_t n_sets, const int64_t* offsets, int64_t n_times,
                    const double* data, const double* sigma, const double* norm, double* chi2, double* ll,
                    hipStream_t st);

}  // namespace gl_mcmc
