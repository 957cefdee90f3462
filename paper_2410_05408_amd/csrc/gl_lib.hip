// gl_lib.hip -- kernels and C ABI of the oblate transit light-curve library.
//
// Pipeline of one gl_lightcurve_batch call (all on the caller's stream):
//   k_prep     one thread per parameter set: domain checks, derived constants
//              (projected ellipse from eqs. dx, dy1, dy2, orbit, limb darkening),
//              CSR segment checks, number of 64-output chunks per set.
//   k_scan     one workgroup: exclusive scan of the chunk counts.
//   k_fill     one wavefront per chunk of 64 consecutive outputs of one set:
//              outputs whose exposure cannot overlap the star are written as
//              1 (NaN for an invalid set); a 64-bit mask of the others is kept.
//   k_compute  persistent wavefronts pull chunks from an atomic head; for each
//              chunk with work, lanes take (output, sub-sample) pairs, evaluate
//              the instantaneous flux in FP64 and the sub-samples of an output
//              are averaged in a fixed order through LDS (deterministic).
// The four launches are captured once into a HIP graph and replayed while the
// arguments stay the same.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>

#include "gl.h"
#include "gl_device.h"

namespace {

constexpr int kChunk = 64;
constexpr int kScanThreads = 1024;

constexpr int kCensus = 8;

struct Counters {
    unsigned long long total_chunks;  // written by k_scan
    unsigned long long head;          // work head of k_compute (reset by k_prep)
    unsigned int status;              // bit 0: invalid set, bit 1: bad CSR segment, bit 2: non-finite time
    unsigned int pad;
    // work census (census launches only): in-window sub-samples, whole-on-star,
    // intersecting, in-window but off the star, full-turn rules, arc rules,
    // Newton steps, limb arcs
    unsigned long long census[kCensus];
};

// ---------------------------------------------------------------- kernels
__global__ void k_prep(const double* __restrict__ params, int64_t n_sets,
                       const int64_t* __restrict__ offsets, int64_t n_times,
                       const int32_t* __restrict__ n_ss, const double* __restrict__ t_exp,
                       gl::SetConst* __restrict__ sc, int64_t* __restrict__ seg_begin,
                       int64_t* __restrict__ seg_len, int64_t* __restrict__ chunk_off,
                       Counters* __restrict__ ctr)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s == 0) {
        ctr->head = 0ull;
        for (int i = 0; i < kCensus; ++i) ctr->census[i] = 0ull;
    }
    if (s >= n_sets) return;
    double p[GL_NPARAM];
#pragma unroll
    for (int i = 0; i < GL_NPARAM; ++i) p[i] = params[(int64_t)i * n_sets + s];
    const int nss = n_ss ? n_ss[s] : 1;
    const double te = t_exp ? t_exp[s] : 0.0;
    gl::SetConst c;
    const bool ok = gl::make_set_const(p, te, nss, c);
    int64_t b, e;
    unsigned int flag = ok ? 0u : 1u;
    if (offsets) {
        b = offsets[s];
        e = offsets[s + 1];
        bool seg_ok = (b >= 0) && (e >= b) && (e <= n_times);
        if (s == 0) seg_ok = seg_ok && (b == 0);
        if (s == n_sets - 1) seg_ok = seg_ok && (e == n_times);
        if (!seg_ok) {
            b = 0;
            e = 0;
            flag |= 2u;
        }
    } else {
        b = s * n_times;
        e = b + n_times;
    }
    if (flag) atomicOr(&ctr->status, flag);
    sc[s] = c;
    seg_begin[s] = b;
    seg_len[s] = e - b;
    chunk_off[s] = (e - b + kChunk - 1) / kChunk;
}

// exclusive scan of chunk_off[0..n) in place; chunk_off[n] = total.  A total
// above the workspace capacity (only possible when CSR offsets decrease and
// later segments overlap earlier ones) schedules no work and is reported.
__global__ void __launch_bounds__(kScanThreads)
k_scan(int64_t* __restrict__ chunk_off, int64_t n, int64_t max_chunks, Counters* __restrict__ ctr)
{
    __shared__ int64_t part[kScanThreads];
    const int tid = threadIdx.x;
    const int64_t per = (n + kScanThreads - 1) / kScanThreads;
    const int64_t lo = std::min<int64_t>(n, per * tid), hi = std::min<int64_t>(n, lo + per);
    int64_t sum = 0;
    for (int64_t i = lo; i < hi; ++i) sum += chunk_off[i];
    part[tid] = sum;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {
        const int64_t v = (tid >= d) ? part[tid - d] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int64_t run = part[tid] - sum;  // exclusive prefix of this thread's range
    for (int64_t i = lo; i < hi; ++i) {
        const int64_t v = chunk_off[i];
        chunk_off[i] = run;
        run += v;
    }
    if (tid == kScanThreads - 1) {
        int64_t total = part[tid];
        if (total > max_chunks) {
            atomicOr(&ctr->status, 2u);
            total = 0;
        }
        chunk_off[n] = total;
        ctr->total_chunks = (unsigned long long)total;
    }
}

__global__ void k_reset_head(Counters* __restrict__ ctr) { ctr->head = 0ull; }

__device__ __forceinline__ int64_t set_of_chunk(const int64_t* __restrict__ chunk_off,
                                                int64_t n_sets, int64_t c)
{
    int64_t lo = 0, hi = n_sets;  // chunk_off[lo] <= c < chunk_off[hi]
    while (hi - lo > 1) {
        const int64_t m = (lo + hi) >> 1;
        if (chunk_off[m] <= c) lo = m;
        else hi = m;
    }
    return lo;
}

__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const unsigned int lo = __builtin_amdgcn_readfirstlane((unsigned int)(v & 0xffffffffll));
    const unsigned int hi = __builtin_amdgcn_readfirstlane((unsigned int)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__global__ void __launch_bounds__(256)
k_fill(const double* __restrict__ times, int64_t n_sets, int shared_grid, int64_t cps,
       const gl::SetConst* __restrict__ sc, const int64_t* __restrict__ seg_begin,
       const int64_t* __restrict__ seg_len, const int64_t* __restrict__ chunk_off,
       Counters* __restrict__ ctr, unsigned long long* __restrict__ masks,
       int* __restrict__ chunk_set, double* __restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int64_t c = uniform64((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    const int64_t total = (int64_t)ctr->total_chunks;
    if (c >= total) return;
    const int64_t s = uniform64(shared_grid ? c / cps : set_of_chunk(chunk_off, n_sets, c));
    const int64_t lc = c - chunk_off[s];
    const int64_t pos = lc * kChunk + lane;  // position inside the set's segment
    const bool in_seg = pos < seg_len[s];
    const int64_t i = seg_begin[s] + pos;
    const gl::SetConst& S = sc[s];
    bool work = false;
    if (in_seg) {
        const double t = shared_grid ? times[pos] : times[i];
        if (!S.valid || !gl::finite_d(t)) {
            out[i] = __builtin_nan("");
            if (S.valid) atomicOr(&ctr->status, 4u);
        } else {
            const double tau = gl::phase_time(S, t);
            work = fabs(tau) < S.half_win + 0.5 * S.t_exp;
            if (!work) out[i] = 1.0;
        }
    }
    const unsigned long long m = __ballot(work);
    if (lane == 0) {
        masks[c] = m;
        chunk_set[c] = (int)s;
    }
}

// Sub-samples of one chunk kept in LDS by the three-phase path (n_ss <= 16).
constexpr int kMaxSubLds = kChunk * 16;

template <bool CENSUS>
struct Counter {
    unsigned long long v[kCensus];
    __device__ void add_sample(int cls, const gl::Census& ct)
    {
        if (!CENSUS) return;
        v[0] += 1;
        v[cls == gl::CLS_FULL ? 1 : (cls == gl::CLS_PARTIAL ? 2 : 3)] += 1;
        v[4] += ct.trap_nodes;
        v[5] += ct.arcs;
        v[6] += ct.iters;
        v[7] += ct.limbs;
    }
};

// Instantaneous flux, easy part only: returns false (and leaves F) when the
// sample needs the intersection machinery.
template <bool CENSUS>
__device__ __attribute__((noinline)) bool flux_easy(const gl::SetConst& S, double t, double& F,
                                          Counter<CENSUS>& cnt)
{
    double x0, y0;
    gl::Census ct;
    int cls = gl::CLS_OUT;
    if (!gl::centre_at(S, t, x0, y0)) {
        F = 1.0;
        cnt.add_sample(gl::CLS_OUT, ct);
        return true;
    }
    double d;
    bool easy;
    if (CENSUS) easy = gl::occulted_easy<gl::Census>(S, x0, y0, d, &cls, ct);
    else {
        gl::NoCensus nc;
        easy = gl::occulted_easy<gl::NoCensus>(S, x0, y0, d, nullptr, nc);
    }
    if (easy) {
        F = 1.0 - d;
        cnt.add_sample(cls, ct);
    }
    return easy;
}

template <bool CENSUS>
__device__ __attribute__((noinline)) double flux_hard(const gl::SetConst& S, double t, Counter<CENSUS>& cnt)
{
    double x0, y0;
    (void)gl::centre_at(S, t, x0, y0);
    if (CENSUS) {
        gl::Census ct;
        int cls = gl::CLS_OUT;
        const double d = gl::occulted_hard<gl::Census>(S, x0, y0, &cls, ct);
        cnt.add_sample(cls, ct);
        return 1.0 - d;
    }
    gl::NoCensus nc;
    return 1.0 - gl::occulted_hard<gl::NoCensus>(S, x0, y0, nullptr, nc);
}

// Occupancy target of the compute kernel (waves per SIMD; 0 = compiler's choice).
#ifndef GL_COMPUTE_WAVES_PER_EU
#define GL_COMPUTE_WAVES_PER_EU 0
#endif
#if GL_COMPUTE_WAVES_PER_EU > 0
#define GL_COMPUTE_ATTR __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(GL_COMPUTE_WAVES_PER_EU)))
#else
#define GL_COMPUTE_ATTR __launch_bounds__(64)
#endif

template <bool CENSUS>
__global__ void GL_COMPUTE_ATTR
k_compute(const double* __restrict__ times, int shared_grid, const gl::SetConst* __restrict__ sc,
          const int64_t* __restrict__ seg_begin, const int64_t* __restrict__ chunk_off,
          Counters* __restrict__ ctr, const unsigned long long* __restrict__ masks,
          const int* __restrict__ chunk_set, double* __restrict__ out)
{
    __shared__ double lds_f[kMaxSubLds];   // sub-sample fluxes of the chunk
    __shared__ short lds_def[kMaxSubLds];  // deferred (hard) sub-samples
    __shared__ int lds_idx[kChunk];        // chunk lanes with work, compacted
    const int lane = threadIdx.x;
    const int64_t total = (int64_t)ctr->total_chunks;
    Counter<CENSUS> cnt;
    for (int i = 0; i < kCensus; ++i) cnt.v[i] = 0ull;
    for (;;) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(&ctr->head, (unsigned long long)kChunk);
        base = (unsigned long long)uniform64((int64_t)base);  // lane 0's value
        if ((int64_t)base >= total) break;
        const int64_t my = (int64_t)base + lane;
        const unsigned long long mym = (my < total) ? masks[my] : 0ull;
        unsigned long long todo = __ballot(mym != 0ull);
        while (todo) {
            const int b = __builtin_ctzll(todo);
            todo &= todo - 1ull;
            const int64_t c = (int64_t)base + b;
            const unsigned long long M = (unsigned long long)uniform64((int64_t)masks[c]);
            const int64_t s = uniform64(chunk_set[c]);
            const gl::SetConst S = sc[s];
            const int64_t lc = c - chunk_off[s];
            const int64_t i0 = seg_begin[s] + lc * kChunk;
            const int64_t tb = shared_grid ? lc * kChunk : i0;
            // compact the chunk's working lanes
            if ((M >> lane) & 1ull) lds_idx[__popcll(M & ((1ull << lane) - 1ull))] = lane;
            __syncthreads();
            const int n_in = __popcll(M);
            const int nss = S.n_ss;
            const double inv_nss = 1.0 / (double)nss;
            // f / nss for f < 1024, nss <= 16 from an exact float product
            const float inv_nss_f = 1.0f / (float)nss;
            if (nss <= 16) {
                // phase 1: easy sub-samples now, hard ones into the deferred list
                const int N = n_in * nss;
                int ndef = 0;
                for (int f0 = 0; f0 < N; f0 += kChunk) {
                    const int f = f0 + lane;
                    bool hard = false;
                    if (f < N) {
                        const int o = (int)(((float)f + 0.5f) * inv_nss_f), j = f - o * nss;
                        const double t = times[tb + lds_idx[o]] + (((double)j + 0.5) * inv_nss - 0.5) * S.t_exp;
                        double F = 1.0;
                        hard = !flux_easy<CENSUS>(S, t, F, cnt);
                        if (!hard) lds_f[f] = F;
                    }
                    const unsigned long long hm = __ballot(hard);
                    if (hard) lds_def[ndef + __popcll(hm & ((1ull << lane) - 1ull))] = (short)f;
                    ndef += __popcll(hm);
                }
                __syncthreads();
                // phase 2: hard sub-samples, 64 at a time
                for (int k0 = 0; k0 < ndef; k0 += kChunk) {
                    const int k = k0 + lane;
                    if (k < ndef) {
                        const int f = lds_def[k];
                        const int o = (int)(((float)f + 0.5f) * inv_nss_f), j = f - o * nss;
                        const double t = times[tb + lds_idx[o]] + (((double)j + 0.5) * inv_nss - 0.5) * S.t_exp;
                        lds_f[f] = flux_hard<CENSUS>(S, t, cnt);
                    }
                }
                __syncthreads();
                // phase 3: box average per output, sub-samples in order
                for (int o = lane; o < n_in; o += kChunk) {
                    double sum = 0.0;
                    for (int jj = 0; jj < nss; ++jj) sum += lds_f[o * nss + jj];
                    out[i0 + lds_idx[o]] = sum / (double)nss;
                }
                __syncthreads();
            } else {
                // long exposures (n_ss > 16): lanes take (output, sub-sample)
                // pairs, averaged through LDS
                const int opw = kChunk / nss;
                const int lo = lane / nss, j = lane - lo * nss;
                const double frac = ((double)j + 0.5) * inv_nss - 0.5;
                for (int g = 0; g < n_in; g += opw) {
                    const int o = g + lo;
                    const bool act = (lo < opw) && (o < n_in);
                    double F = 1.0;
                    int off = 0;
                    if (act) {
                        off = lds_idx[o];
                        const double t = times[tb + off] + frac * S.t_exp;
                        if (!flux_easy<CENSUS>(S, t, F, cnt)) F = flux_hard<CENSUS>(S, t, cnt);
                    }
                    lds_f[lane] = F;
                    __syncthreads();
                    if (act && j == 0) {
                        double sum = 0.0;
                        for (int jj = 0; jj < nss; ++jj) sum += lds_f[lane + jj];
                        out[i0 + off] = sum / (double)nss;
                    }
                    __syncthreads();
                }
            }
        }
    }
    if (CENSUS) {
        for (int i = 0; i < kCensus; ++i) {
            unsigned long long v = cnt.v[i];
            for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
            if (lane == 0) atomicAdd(&ctr->census[i], v);
        }
    }
}

using ComputeFn = void (*)(const double*, int, const gl::SetConst*, const int64_t*,
                           const int64_t*, Counters*, const unsigned long long*, const int*,
                           double*);

}  // namespace

// ---------------------------------------------------------------- context
struct gl_ctx {
    int device = 0;
    int n_cu = 256;
    int waves_per_cu = 8;
    bool use_graph = true;
    std::string err;
    // workspace
    gl::SetConst* sc = nullptr;
    int64_t* seg_begin = nullptr;
    int64_t* seg_len = nullptr;
    int64_t* chunk_off = nullptr;
    int64_t cap_sets = 0;
    unsigned long long* masks = nullptr;
    int* chunk_set = nullptr;
    int64_t cap_chunks = 0;
    Counters* ctr = nullptr;
    // graph cache
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    struct Key {
        const double* params;
        int64_t n_sets;
        const double* times;
        const int64_t* offsets;
        int64_t n_times;
        const int32_t* n_ss;
        const double* t_exp;
        double* out;
        void* stream;
        int waves;
        void* ws;
    } key{};
    bool have_graph = false;
    // surrogate path buffers (grown on demand)
    int64_t* chunk_sub = nullptr;  // sub-sample offset per chunk (+1 total)
    int64_t cap_sub_chunks = 0;
    float* s_feat = nullptr;
    float* s_pred = nullptr;
    double* s_fsph = nullptr;
    double* s_scale = nullptr;
    double* s_t = nullptr;
    double* s_F = nullptr;
    int* s_bin = nullptr;
    int* s_set = nullptr;
    int64_t* s_fb = nullptr;
    int64_t cap_sub = 0;
    // per-launch timing (events around the compute kernel and the pipeline)
    int t_slots = 0, t_used = 0;
    hipEvent_t* ev = nullptr;  // 3 events per slot: pipeline start, compute start, end
};

namespace {

gl_status fail(gl_ctx* ctx, gl_status st, const char* what, hipError_t e = hipSuccess)
{
    if (ctx) {
        ctx->err = what;
        if (e != hipSuccess) {
            ctx->err += ": ";
            ctx->err += hipGetErrorString(e);
        }
    }
    return st;
}

#define GL_HIP(call, what)                                                   \
    do {                                                                     \
        hipError_t e_ = (call);                                              \
        if (e_ != hipSuccess) return fail(ctx, GL_ERR_DEVICE, what, e_);     \
    } while (0)

void drop_graph(gl_ctx* ctx)
{
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->gexec = nullptr;
    ctx->graph = nullptr;
    ctx->have_graph = false;
}

void free_sur(gl_ctx* ctx)
{
    void* b[] = {ctx->chunk_sub, ctx->s_feat, ctx->s_pred, ctx->s_fsph, ctx->s_scale, ctx->s_t,
                 ctx->s_F,       ctx->s_bin,  ctx->s_set,  ctx->s_fb};
    for (void* p : b) (void)hipFree(p);
    ctx->chunk_sub = nullptr;
    ctx->s_feat = ctx->s_pred = nullptr;
    ctx->s_fsph = ctx->s_scale = ctx->s_t = ctx->s_F = nullptr;
    ctx->s_bin = ctx->s_set = nullptr;
    ctx->s_fb = nullptr;
    ctx->cap_sub_chunks = ctx->cap_sub = 0;
}

void free_ws(gl_ctx* ctx)
{
    free_sur(ctx);
    (void)hipFree(ctx->sc);
    (void)hipFree(ctx->seg_begin);
    (void)hipFree(ctx->seg_len);
    (void)hipFree(ctx->chunk_off);
    (void)hipFree(ctx->masks);
    (void)hipFree(ctx->chunk_set);
    ctx->sc = nullptr;
    ctx->seg_begin = ctx->seg_len = ctx->chunk_off = nullptr;
    ctx->masks = nullptr;
    ctx->chunk_set = nullptr;
    ctx->cap_sets = ctx->cap_chunks = 0;
}

gl_status ensure_ws(gl_ctx* ctx, int64_t n_sets, int64_t n_chunks)
{
    if (n_sets > ctx->cap_sets) {
        drop_graph(ctx);
        GL_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
        (void)hipFree(ctx->sc);
        (void)hipFree(ctx->seg_begin);
        (void)hipFree(ctx->seg_len);
        (void)hipFree(ctx->chunk_off);
        ctx->sc = nullptr;
        ctx->seg_begin = ctx->seg_len = ctx->chunk_off = nullptr;
        ctx->cap_sets = 0;
        const int64_t cap = std::max<int64_t>(n_sets, 1024);
        if (hipMalloc(&ctx->sc, sizeof(gl::SetConst) * cap) != hipSuccess ||
            hipMalloc(&ctx->seg_begin, sizeof(int64_t) * cap) != hipSuccess ||
            hipMalloc(&ctx->seg_len, sizeof(int64_t) * cap) != hipSuccess ||
            hipMalloc(&ctx->chunk_off, sizeof(int64_t) * (cap + 1)) != hipSuccess) {
            free_ws(ctx);
            return fail(ctx, GL_ERR_NOMEM, "workspace allocation (sets)");
        }
        ctx->cap_sets = cap;
    }
    if (n_chunks > ctx->cap_chunks) {
        drop_graph(ctx);
        GL_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
        (void)hipFree(ctx->masks);
        (void)hipFree(ctx->chunk_set);
        ctx->masks = nullptr;
        ctx->chunk_set = nullptr;
        ctx->cap_chunks = 0;
        const int64_t cap = std::max<int64_t>(n_chunks, 4096);
        if (hipMalloc(&ctx->masks, sizeof(unsigned long long) * cap) != hipSuccess ||
            hipMalloc(&ctx->chunk_set, sizeof(int) * cap) != hipSuccess) {
            free_ws(ctx);
            return fail(ctx, GL_ERR_NOMEM, "workspace allocation (chunks)");
        }
        ctx->cap_chunks = cap;
    }
    return GL_OK;
}

struct Batch {
    const double* params;
    int64_t n_sets;
    const double* times;
    const int64_t* offsets;
    int64_t n_times;
    const int32_t* n_ss;
    const double* t_exp;
    double* out;
    hipStream_t stream;
    int64_t max_chunks;
};

gl_status check_args(gl_ctx* ctx, Batch& b)
{
    if (!ctx) return GL_ERR_NULL;
    ctx->err.clear();
    if (!b.params || !b.times || !b.out) return fail(ctx, GL_ERR_NULL, "params, times and out are required");
    if (b.n_sets < 1) return fail(ctx, GL_ERR_SIZE, "n_sets must be >= 1");
    if (b.n_sets > (int64_t)INT32_MAX) return fail(ctx, GL_ERR_SIZE, "n_sets too large");
    if (b.offsets) {
        if (b.n_times < 0) return fail(ctx, GL_ERR_SIZE, "CSR n_times must be >= 0");
        b.max_chunks = b.n_times / kChunk + b.n_sets;
    } else {
        if (b.n_times < 1) return fail(ctx, GL_ERR_SIZE, "n_times must be >= 1");
        const int64_t cps = (b.n_times + kChunk - 1) / kChunk;
        if (b.n_sets > ((int64_t)1 << 62) / std::max<int64_t>(b.n_times, 1))
            return fail(ctx, GL_ERR_SIZE, "n_sets * n_times overflows");
        b.max_chunks = cps * b.n_sets;
    }
    if (b.max_chunks > ((int64_t)1 << 40)) return fail(ctx, GL_ERR_SIZE, "batch too large");
    return GL_OK;
}

gl_status enqueue(gl_ctx* ctx, const Batch& b, bool census = false)
{
    const int shared = b.offsets ? 0 : 1;
    hipEvent_t* ev = nullptr;
    if (ctx->t_slots > 0 && ctx->t_used < ctx->t_slots && !census) {
        ev = ctx->ev + 3 * ctx->t_used;
        ctx->t_used++;
        GL_HIP(hipEventRecord(ev[0], b.stream), "hipEventRecord");
    }
    const unsigned prep_blocks = (unsigned)((b.n_sets + 255) / 256);
    hipLaunchKernelGGL(k_prep, dim3(prep_blocks), dim3(256), 0, b.stream, b.params, b.n_sets,
                       b.offsets, b.n_times, b.n_ss, b.t_exp, ctx->sc, ctx->seg_begin,
                       ctx->seg_len, ctx->chunk_off, ctx->ctr);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, b.stream, ctx->chunk_off, b.n_sets,
                       b.max_chunks, ctx->ctr);
    const int64_t fill_blocks = (b.max_chunks + 3) / 4;
    const int64_t cps = shared ? (b.n_times + kChunk - 1) / kChunk : 0;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)fill_blocks), dim3(256), 0, b.stream, b.times,
                       b.n_sets, shared, cps, ctx->sc, ctx->seg_begin, ctx->seg_len, ctx->chunk_off,
                       ctx->ctr, ctx->masks, ctx->chunk_set, b.out);
    const int64_t want = (int64_t)ctx->n_cu * ctx->waves_per_cu;
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(want, (b.max_chunks + kChunk - 1) / kChunk * 4 + 1));
    if (ev) GL_HIP(hipEventRecord(ev[1], b.stream), "hipEventRecord");
    ComputeFn fn = census ? k_compute<true> : k_compute<false>;
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(64), 0, b.stream, b.times, shared, ctx->sc,
                       ctx->seg_begin, ctx->chunk_off, ctx->ctr, ctx->masks, ctx->chunk_set, b.out);
    if (ev) GL_HIP(hipEventRecord(ev[2], b.stream), "hipEventRecord");
    GL_HIP(hipGetLastError(), "kernel launch");
    return GL_OK;
}

bool same_key(const gl_ctx::Key& a, const gl_ctx::Key& b)
{
    return std::memcmp(&a, &b, sizeof(a)) == 0;
}

}  // namespace

extern "C" {

gl_status gl_ctx_create(gl_ctx** out, int device)
{
    if (!out) return GL_ERR_NULL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return GL_ERR_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return GL_ERR_DEVICE;
    gl_ctx* ctx = new (std::nothrow) gl_ctx();
    if (!ctx) return GL_ERR_NOMEM;
    ctx->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        ctx->n_cu = prop.multiProcessorCount;
    if (hipMalloc(&ctx->ctr, sizeof(Counters)) != hipSuccess) {
        delete ctx;
        return GL_ERR_NOMEM;
    }
    if (hipMemset(ctx->ctr, 0, sizeof(Counters)) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(ctx->ctr);
        delete ctx;
        return GL_ERR_DEVICE;
    }
    *out = ctx;
    return GL_OK;
}

void free_timing(gl_ctx* ctx)
{
    for (int i = 0; i < 3 * ctx->t_slots; ++i) (void)hipEventDestroy(ctx->ev[i]);
    delete[] ctx->ev;
    ctx->ev = nullptr;
    ctx->t_slots = ctx->t_used = 0;
}

void gl_ctx_destroy(gl_ctx* ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    free_timing(ctx);
    drop_graph(ctx);
    free_ws(ctx);
    (void)hipFree(ctx->ctr);
    delete ctx;
}

gl_status gl_lightcurve_batch(gl_ctx* ctx, const double* params, int64_t n_sets,
                              const double* times, const int64_t* offsets, int64_t n_times,
                              const int32_t* n_ss, const double* t_exp, double* out,
                              void* stream)
{
    Batch b{params, n_sets, times, offsets, n_times, n_ss, t_exp, out, (hipStream_t)stream, 0};
    gl_status st = check_args(ctx, b);
    if (st != GL_OK) return st;
    GL_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    st = ensure_ws(ctx, n_sets, b.max_chunks);
    if (st != GL_OK) return st;
    // the legacy default stream cannot be captured, and timed launches record
    // events per launch: launch directly there
    if (!ctx->use_graph || stream == nullptr || ctx->t_slots > 0) return enqueue(ctx, b);
    gl_ctx::Key k{};
    k.params = params;
    k.n_sets = n_sets;
    k.times = times;
    k.offsets = offsets;
    k.n_times = n_times;
    k.n_ss = n_ss;
    k.t_exp = t_exp;
    k.out = out;
    k.stream = stream;
    k.waves = ctx->waves_per_cu;
    k.ws = ctx->masks;
    if (!ctx->have_graph || !same_key(k, ctx->key)) {
        drop_graph(ctx);
        GL_HIP(hipStreamBeginCapture(b.stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        gl_status est = enqueue(ctx, b);
        hipGraph_t g = nullptr;
        hipError_t ee = hipStreamEndCapture(b.stream, &g);
        if (est != GL_OK) {
            if (g) (void)hipGraphDestroy(g);
            return est;
        }
        if (ee != hipSuccess) return fail(ctx, GL_ERR_DEVICE, "hipStreamEndCapture", ee);
        hipGraphExec_t ex = nullptr;
        hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
            (void)hipGraphDestroy(g);
            return fail(ctx, GL_ERR_DEVICE, "hipGraphInstantiate", ie);
        }
        ctx->graph = g;
        ctx->gexec = ex;
        ctx->key = k;
        ctx->have_graph = true;
    }
    GL_HIP(hipGraphLaunch(ctx->gexec, b.stream), "hipGraphLaunch");
    return GL_OK;
}

gl_status gl_ctx_sync_status(gl_ctx* ctx)
{
    if (!ctx) return GL_ERR_NULL;
    GL_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    GL_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    unsigned int status = 0;
    GL_HIP(hipMemcpy(&status, &ctx->ctr->status, sizeof(status), hipMemcpyDeviceToHost), "hipMemcpy");
    if (status) {
        GL_HIP(hipMemset(&ctx->ctr->status, 0, sizeof(status)), "hipMemset");
        GL_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
        ctx->err.clear();
        if (status & 1u) ctx->err += "invalid parameter set; ";
        if (status & 2u) ctx->err += "invalid CSR segment; ";
        if (status & 4u) ctx->err += "non-finite time; ";
        return GL_ERR_DOMAIN;
    }
    return GL_OK;
}

const char* gl_ctx_last_error(const gl_ctx* ctx)
{
    return ctx ? ctx->err.c_str() : "null context";
}

gl_status gl_ctx_get_plan(const gl_ctx* ctx, int* waves_per_cu)
{
    if (!ctx) return GL_ERR_NULL;
    if (waves_per_cu) *waves_per_cu = ctx->waves_per_cu;
    return GL_OK;
}

gl_status gl_ctx_set_plan(gl_ctx* ctx, int waves_per_cu)
{
    if (!ctx) return GL_ERR_NULL;
    if (waves_per_cu < 1 || waves_per_cu > 32) return fail(ctx, GL_ERR_SIZE, "waves_per_cu in [1, 32]");
    ctx->waves_per_cu = waves_per_cu;
    return GL_OK;
}

gl_status gl_ctx_set_graph(gl_ctx* ctx, int on)
{
    if (!ctx) return GL_ERR_NULL;
    if (!on) drop_graph(ctx);
    ctx->use_graph = on != 0;
    return GL_OK;
}

gl_status gl_autotune(gl_ctx* ctx, const double* params, int64_t n_sets, const double* times,
                      const int64_t* offsets, int64_t n_times, const int32_t* n_ss,
                      const double* t_exp, double* out, void* stream)
{
    Batch b{params, n_sets, times, offsets, n_times, n_ss, t_exp, out, (hipStream_t)stream, 0};
    gl_status st = check_args(ctx, b);
    if (st != GL_OK) return st;
    GL_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    st = ensure_ws(ctx, n_sets, b.max_chunks);
    if (st != GL_OK) return st;
    const bool graph = ctx->use_graph;
    drop_graph(ctx);
    hipEvent_t e0, e1;
    GL_HIP(hipEventCreate(&e0), "hipEventCreate");
    GL_HIP(hipEventCreate(&e1), "hipEventCreate");
    const int cands[] = {2, 4, 8, 12, 16, 24, 32};
    int best = ctx->waves_per_cu;
    float best_ms = 1e30f;
    for (int w : cands) {
        ctx->waves_per_cu = w;
        st = enqueue(ctx, b);  // warm-up
        if (st != GL_OK) break;
        float tot = 0.0f;
        for (int r = 0; r < 3; ++r) {
            (void)hipEventRecord(e0, b.stream);
            st = enqueue(ctx, b);
            (void)hipEventRecord(e1, b.stream);
            (void)hipEventSynchronize(e1);
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            tot += ms;
        }
        if (tot < best_ms) {
            best_ms = tot;
            best = w;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->waves_per_cu = best;
    ctx->use_graph = graph;
    return st;
}

gl_status gl_ctx_set_timing(gl_ctx* ctx, int n_slots)
{
    if (!ctx) return GL_ERR_NULL;
    if (n_slots < 0 || n_slots > 100000) return fail(ctx, GL_ERR_SIZE, "n_slots in [0, 100000]");
    GL_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    GL_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    free_timing(ctx);
    if (n_slots == 0) return GL_OK;
    drop_graph(ctx);
    ctx->ev = new (std::nothrow) hipEvent_t[3 * n_slots];
    if (!ctx->ev) return fail(ctx, GL_ERR_NOMEM, "timing slots");
    for (int i = 0; i < 3 * n_slots; ++i) {
        if (hipEventCreate(&ctx->ev[i]) != hipSuccess) {
            for (int j = 0; j < i; ++j) (void)hipEventDestroy(ctx->ev[j]);
            delete[] ctx->ev;
            ctx->ev = nullptr;
            return fail(ctx, GL_ERR_DEVICE, "hipEventCreate");
        }
    }
    ctx->t_slots = n_slots;
    ctx->t_used = 0;
    return GL_OK;
}

gl_status gl_ctx_get_timing(gl_ctx* ctx, double* compute_ms, double* pipeline_ms, int* n)
{
    if (!ctx) return GL_ERR_NULL;
    double c = 0.0, p = 0.0;
    for (int i = 0; i < ctx->t_used; ++i) {
        hipEvent_t* ev = ctx->ev + 3 * i;
        GL_HIP(hipEventSynchronize(ev[2]), "hipEventSynchronize");
        float a = 0.0f, b = 0.0f;
        GL_HIP(hipEventElapsedTime(&a, ev[1], ev[2]), "hipEventElapsedTime");
        GL_HIP(hipEventElapsedTime(&b, ev[0], ev[2]), "hipEventElapsedTime");
        c += a;
        p += b;
    }
    if (compute_ms) *compute_ms = c;
    if (pipeline_ms) *pipeline_ms = p;
    if (n) *n = ctx->t_used;
    ctx->t_used = 0;
    return GL_OK;
}

gl_status gl_census(gl_ctx* ctx, const double* params, int64_t n_sets, const double* times,
                    const int64_t* offsets, int64_t n_times, const int32_t* n_ss,
                    const double* t_exp, double* out, void* stream, int64_t* counts)
{
    if (!counts) return GL_ERR_NULL;
    Batch b{params, n_sets, times, offsets, n_times, n_ss, t_exp, out, (hipStream_t)stream, 0};
    gl_status st = check_args(ctx, b);
    if (st != GL_OK) return st;
    GL_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    st = ensure_ws(ctx, n_sets, b.max_chunks);
    if (st != GL_OK) return st;
    st = enqueue(ctx, b, true);
    if (st != GL_OK) return st;
    GL_HIP(hipStreamSynchronize(b.stream), "hipStreamSynchronize");
    unsigned long long c[kCensus];
    GL_HIP(hipMemcpy(c, ctx->ctr->census, sizeof(c), hipMemcpyDeviceToHost), "hipMemcpy");
    for (int i = 0; i < kCensus; ++i) counts[i] = (int64_t)c[i];
    return GL_OK;
}

gl_status gl_flop_model(int64_t* per_item)
{
    if (!per_item) return GL_ERR_NULL;
    per_item[0] = gl::kFlopSample;
    per_item[1] = gl::kFlopWhole;
    per_item[2] = gl::kFlopPartial;
    per_item[3] = 0;
    per_item[4] = gl::kFlopTrapNode;
    per_item[5] = gl::kFlopGKPiece;
    per_item[6] = gl::kFlopIter;
    per_item[7] = gl::kFlopLimb;
    return GL_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- surrogate path
namespace {

// One sample per parameter set: features, scaled residual target
// (F_oblate - F_sphere) / scale, both fluxes, the scale and the bin.
__global__ void k_sur_samples(const double* __restrict__ params, int64_t n, const double* __restrict__ times,
                              float* __restrict__ feat, float* __restrict__ target, double* __restrict__ f_obl,
                              double* __restrict__ f_sph, double* __restrict__ scale_out,
                              int* __restrict__ bin_out, Counters* __restrict__ ctr)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double p[GL_NPARAM];
    for (int r = 0; r < GL_NPARAM; ++r) p[r] = params[(int64_t)r * n + i];
    gl::SetConst S;
    float fe[gl::kSurFeat];
    for (int r = 0; r < gl::kSurFeat; ++r) fe[r] = 0.f;
    double Fo = 1.0, Fs = 1.0, sc = 0.0;
    int bin = -1;
    if (!gl::make_set_const(p, 0.0, 1, S) || !gl::finite_d(times[i])) {
        atomicOr(&ctr->status, 1u);
        Fo = Fs = __builtin_nan("");
    } else {
        double x0, y0;
        if (gl::centre_at(S, times[i], x0, y0) && gl::sur_encode(S, x0, y0, fe, sc, bin)) {
            gl::NoCensus nc;
            Fo = 1.0 - gl::occulted<gl::NoCensus>(S, x0, y0, nullptr, nc);
            const gl::SetConst C = gl::sphere_of(S);
            Fs = 1.0 - gl::occulted<gl::NoCensus>(C, x0, y0, nullptr, nc);
        }
    }
    for (int r = 0; r < gl::kSurFeat; ++r) feat[i * gl::kSurFeat + r] = fe[r];
    target[i] = bin >= 0 ? (float)((Fo - Fs) / sc) : 0.f;
    if (f_obl) f_obl[i] = Fo;
    if (f_sph) f_sph[i] = Fs;
    if (scale_out) scale_out[i] = sc;
    if (bin_out) bin_out[i] = bin;
}

// table[bin] = max over samples of |(pred - target) * scale| (non-negative
// floats order like their bit patterns, so an integer max is exact)
__global__ void k_sur_bound(const float* __restrict__ pred, const float* __restrict__ target,
                            const double* __restrict__ scale, const int* __restrict__ bin, int64_t n,
                            float* __restrict__ table)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || bin[i] < 0) return;
    const float e = (float)(fabs((double)pred[i] - (double)target[i]) * scale[i]);
    atomicMax((unsigned int*)&table[bin[i]], __float_as_uint(e));
}

// sub-sample count per chunk: popcount(mask) * n_ss
__global__ void k_sub_count(const unsigned long long* __restrict__ masks, const int* __restrict__ chunk_set,
                            const gl::SetConst* __restrict__ sc, const Counters* __restrict__ ctr,
                            int64_t* __restrict__ cnt)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= (int64_t)ctr->total_chunks) return;
    const unsigned long long m = masks[c];
    cnt[c] = m ? (int64_t)__popcll(m) * sc[chunk_set[c]].n_ss : 0;
}

// exclusive scan of a[0..n) in place with a[n] = total, one workgroup
__global__ void __launch_bounds__(kScanThreads) k_scan_n(int64_t* __restrict__ a, const Counters* __restrict__ ctr)
{
    __shared__ int64_t part[kScanThreads];
    const int64_t n = (int64_t)ctr->total_chunks;
    const int tid = threadIdx.x;
    const int64_t per = (n + kScanThreads - 1) / kScanThreads;
    const int64_t lo = std::min<int64_t>(n, per * tid), hi = std::min<int64_t>(n, lo + per);
    int64_t sum = 0;
    for (int64_t i = lo; i < hi; ++i) sum += a[i];
    part[tid] = sum;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {
        const int64_t v = (tid >= d) ? part[tid - d] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int64_t run = part[tid] - sum;
    for (int64_t i = lo; i < hi; ++i) {
        const int64_t v = a[i];
        a[i] = run;
        run += v;
    }
    if (tid == kScanThreads - 1) a[n] = part[tid];
}

// one wavefront per chunk: sub-sample times, features, sphere flux
__global__ void __launch_bounds__(64)
k_sur_enum(const double* __restrict__ times, int shared_grid, const gl::SetConst* __restrict__ sc,
           const int64_t* __restrict__ seg_begin, const int64_t* __restrict__ chunk_off,
           const Counters* __restrict__ ctr, const unsigned long long* __restrict__ masks,
           const int* __restrict__ chunk_set, const int64_t* __restrict__ chunk_sub,
           float* __restrict__ feat, double* __restrict__ fsph, double* __restrict__ scale,
           double* __restrict__ tsub, double* __restrict__ F, int* __restrict__ bin, int* __restrict__ setid)
{
    __shared__ int lds_idx[kChunk];
    const int lane = threadIdx.x;
    const int64_t c = uniform64((int64_t)blockIdx.x);
    if (c >= (int64_t)ctr->total_chunks) return;
    const unsigned long long M = (unsigned long long)uniform64((int64_t)masks[c]);
    if (!M) return;
    const int64_t s = uniform64(chunk_set[c]);
    const gl::SetConst S = sc[s];
    const int64_t lc = c - chunk_off[s];
    const int64_t tb = shared_grid ? lc * kChunk : seg_begin[s] + lc * kChunk;
    if ((M >> lane) & 1ull) lds_idx[__popcll(M & ((1ull << lane) - 1ull))] = lane;
    __syncthreads();
    const int nss = S.n_ss;
    const int N = __popcll(M) * nss;
    const int64_t g0 = chunk_sub[c];
    for (int f = lane; f < N; f += kChunk) {
        const int o = f / nss, j = f - o * nss;
        const double t = times[tb + lds_idx[o]] + (((double)j + 0.5) / (double)nss - 0.5) * S.t_exp;
        const int64_t g = g0 + f;
        float fe[gl::kSurFeat];
        for (int r = 0; r < gl::kSurFeat; ++r) fe[r] = 0.f;
        double sc_ = 0.0, fs = 1.0, Fv = 1.0;
        int b = -1;
        double x0, y0;
        if (gl::centre_at(S, t, x0, y0) && gl::sur_encode(S, x0, y0, fe, sc_, b)) {
            gl::NoCensus nc;
            const gl::SetConst C = gl::sphere_of(S);
            fs = 1.0 - gl::occulted<gl::NoCensus>(C, x0, y0, nullptr, nc);
            Fv = __builtin_nan("");  // decided by the gate
        }
        for (int r = 0; r < gl::kSurFeat; ++r) feat[g * gl::kSurFeat + r] = fe[r];
        fsph[g] = fs;
        scale[g] = sc_;
        tsub[g] = t;
        F[g] = Fv;
        bin[g] = b;
        setid[g] = (int)s;
    }
}

// accept F = F_sphere + scale * pred where safety * table[bin] * ... <= tol,
// otherwise queue the sub-sample for the exact kernel
__global__ void k_sur_gate(const float* __restrict__ pred, const double* __restrict__ fsph,
                           const double* __restrict__ scale, const int* __restrict__ bin,
                           const float* __restrict__ table, double safety, double tol, int64_t n,
                           double* __restrict__ F, int64_t* __restrict__ fb, Counters* __restrict__ ctr)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool queue = false;
    if (g < n && bin[g] >= 0) {
        const float tb = table[bin[g]];
        const double bound = safety * (double)tb;
        if (tb >= 0.f && bound <= tol && gl::finite_d(bound)) F[g] = fsph[g] + scale[g] * (double)pred[g];
        else queue = true;
    }
    const unsigned long long qm = __ballot(queue);
    unsigned long long base = 0;
    const int lane = threadIdx.x & 63;
    if (lane == 0 && qm) base = atomicAdd(&ctr->head, (unsigned long long)__popcll(qm));
    base = (unsigned long long)uniform64((int64_t)base);
    if (queue) fb[base + __popcll(qm & ((1ull << lane) - 1ull))] = g;
}

// exact flux for the queued sub-samples (count in ctr->head)
__global__ void __launch_bounds__(64)
k_sur_exact(const int64_t* __restrict__ fb, const Counters* __restrict__ ctr, const double* __restrict__ tsub,
            const int* __restrict__ setid, const gl::SetConst* __restrict__ sc, double* __restrict__ F)
{
    const int64_t nq = (int64_t)ctr->head;
    for (int64_t k = (int64_t)blockIdx.x * 64 + threadIdx.x; k < nq; k += (int64_t)gridDim.x * 64) {
        const int64_t g = fb[k];
        F[g] = gl::flux_instant(sc[setid[g]], tsub[g]);
    }
}

// one wavefront per chunk: box average of each output's sub-samples in order
__global__ void __launch_bounds__(64)
k_sur_reduce(const gl::SetConst* __restrict__ sc, const int64_t* __restrict__ seg_begin,
             const int64_t* __restrict__ chunk_off, const Counters* __restrict__ ctr,
             const unsigned long long* __restrict__ masks, const int* __restrict__ chunk_set,
             const int64_t* __restrict__ chunk_sub, const double* __restrict__ F, double* __restrict__ out)
{
    __shared__ int lds_idx[kChunk];
    const int lane = threadIdx.x;
    const int64_t c = uniform64((int64_t)blockIdx.x);
    if (c >= (int64_t)ctr->total_chunks) return;
    const unsigned long long M = (unsigned long long)uniform64((int64_t)masks[c]);
    if (!M) return;
    const int64_t s = uniform64(chunk_set[c]);
    const int nss = sc[s].n_ss;
    const int64_t i0 = seg_begin[s] + (c - chunk_off[s]) * kChunk;
    if ((M >> lane) & 1ull) lds_idx[__popcll(M & ((1ull << lane) - 1ull))] = lane;
    __syncthreads();
    const int n_in = __popcll(M);
    const int64_t g0 = chunk_sub[c];
    for (int o = lane; o < n_in; o += kChunk) {
        double sum = 0.0;
        for (int j = 0; j < nss; ++j) sum += F[g0 + (int64_t)o * nss + j];
        out[i0 + lds_idx[o]] = sum / (double)nss;
    }
}

gl_status ensure_sur(gl_ctx* ctx, int64_t n_chunks, int64_t n_sub)
{
    if (n_chunks + 1 > ctx->cap_sub_chunks) {
        (void)hipFree(ctx->chunk_sub);
        ctx->chunk_sub = nullptr;
        ctx->cap_sub_chunks = 0;
        if (hipMalloc(&ctx->chunk_sub, sizeof(int64_t) * (n_chunks + 1)) != hipSuccess)
            return fail(ctx, GL_ERR_NOMEM, "surrogate workspace (chunks)");
        ctx->cap_sub_chunks = n_chunks + 1;
    }
    if (n_sub > ctx->cap_sub) {
        void* b[] = {ctx->s_feat, ctx->s_pred, ctx->s_fsph, ctx->s_scale, ctx->s_t,
                     ctx->s_F,    ctx->s_bin,  ctx->s_set,  ctx->s_fb};
        for (void* p : b) (void)hipFree(p);
        ctx->s_feat = ctx->s_pred = nullptr;
        ctx->s_fsph = ctx->s_scale = ctx->s_t = ctx->s_F = nullptr;
        ctx->s_bin = ctx->s_set = nullptr;
        ctx->s_fb = nullptr;
        ctx->cap_sub = 0;
        const int64_t cap = std::max<int64_t>(n_sub, 1 << 16);
        bool ok = hipMalloc(&ctx->s_feat, sizeof(float) * gl::kSurFeat * cap) == hipSuccess &&
                  hipMalloc(&ctx->s_pred, sizeof(float) * cap) == hipSuccess &&
                  hipMalloc(&ctx->s_fsph, sizeof(double) * cap) == hipSuccess &&
                  hipMalloc(&ctx->s_scale, sizeof(double) * cap) == hipSuccess &&
                  hipMalloc(&ctx->s_t, sizeof(double) * cap) == hipSuccess &&
                  hipMalloc(&ctx->s_F, sizeof(double) * cap) == hipSuccess &&
                  hipMalloc(&ctx->s_bin, sizeof(int) * cap) == hipSuccess &&
                  hipMalloc(&ctx->s_set, sizeof(int) * cap) == hipSuccess &&
                  hipMalloc(&ctx->s_fb, sizeof(int64_t) * cap) == hipSuccess;
        if (!ok) {
            free_sur(ctx);
            return fail(ctx, GL_ERR_NOMEM, "surrogate workspace (sub-samples)");
        }
        ctx->cap_sub = cap;
    }
    return GL_OK;
}

}  // namespace

extern "C" {

gl_status gl_surrogate_samples(gl_ctx* ctx, const double* params, const double* times, int64_t n,
                               float* feat, float* target, double* f_obl, double* f_sph,
                               double* scale, int32_t* bin, void* stream)
{
    if (!ctx) return GL_ERR_NULL;
    ctx->err.clear();
    if (!params || !times || !feat || !target) return fail(ctx, GL_ERR_NULL, "params, times, feat, target");
    if (n < 1) return fail(ctx, GL_ERR_SIZE, "n >= 1");
    GL_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    hipLaunchKernelGGL(k_sur_samples, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, (hipStream_t)stream,
                       params, n, times, feat, target, f_obl, f_sph, scale, bin, ctx->ctr);
    GL_HIP(hipGetLastError(), "kernel launch");
    return GL_OK;
}

gl_status gl_surrogate_bound(gl_ctx* ctx, const float* pred, const float* target, const double* scale,
                             const int32_t* bin, int64_t n, float* table, void* stream)
{
    if (!ctx) return GL_ERR_NULL;
    if (!pred || !target || !scale || !bin || !table) return fail(ctx, GL_ERR_NULL, "null argument");
    if (n < 1) return fail(ctx, GL_ERR_SIZE, "n >= 1");
    GL_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    hipLaunchKernelGGL(k_sur_bound, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       pred, target, scale, bin, n, table);
    GL_HIP(hipGetLastError(), "kernel launch");
    return GL_OK;
}

int gl_surrogate_num_bins(void) { return gl::kSurBins; }

gl_status gl_lightcurve_batch_surrogate(gl_ctx* ctx, gl_mlp* mlp, const float* table, double safety,
                                        double tol, const double* params, int64_t n_sets,
                                        const double* times, const int64_t* offsets, int64_t n_times,
                                        const int32_t* n_ss, const double* t_exp, double* out,
                                        void* stream, int64_t* n_sub_out, int64_t* n_fallback_out)
{
    Batch b{params, n_sets, times, offsets, n_times, n_ss, t_exp, out, (hipStream_t)stream, 0};
    gl_status st = check_args(ctx, b);
    if (st != GL_OK) return st;
    if (!mlp || !table) return fail(ctx, GL_ERR_NULL, "network and bound table are required");
    GL_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    st = ensure_ws(ctx, n_sets, b.max_chunks);
    if (st != GL_OK) return st;
    st = ensure_sur(ctx, b.max_chunks, 0);
    if (st != GL_OK) return st;
    hipStream_t s = b.stream;
    const int shared = b.offsets ? 0 : 1;
    const int64_t cps = shared ? (b.n_times + kChunk - 1) / kChunk : 0;
    hipLaunchKernelGGL(k_prep, dim3((unsigned)((n_sets + 255) / 256)), dim3(256), 0, s, params, n_sets,
                       offsets, n_times, n_ss, t_exp, ctx->sc, ctx->seg_begin, ctx->seg_len,
                       ctx->chunk_off, ctx->ctr);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, s, ctx->chunk_off, n_sets, b.max_chunks, ctx->ctr);
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((b.max_chunks + 3) / 4)), dim3(256), 0, s, times, n_sets,
                       shared, cps, ctx->sc, ctx->seg_begin, ctx->seg_len, ctx->chunk_off, ctx->ctr,
                       ctx->masks, ctx->chunk_set, out);
    hipLaunchKernelGGL(k_sub_count, dim3((unsigned)((b.max_chunks + 255) / 256)), dim3(256), 0, s, ctx->masks,
                       ctx->chunk_set, ctx->sc, ctx->ctr, ctx->chunk_sub);
    hipLaunchKernelGGL(k_scan_n, dim3(1), dim3(kScanThreads), 0, s, ctx->chunk_sub, ctx->ctr);
    GL_HIP(hipGetLastError(), "kernel launch");
    // the sub-sample count sizes the buffers: one synchronisation
    unsigned long long total_chunks = 0;
    GL_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    GL_HIP(hipMemcpy(&total_chunks, &ctx->ctr->total_chunks, sizeof(total_chunks), hipMemcpyDeviceToHost), "hipMemcpy");
    int64_t n_sub = 0;
    GL_HIP(hipMemcpy(&n_sub, ctx->chunk_sub + total_chunks, sizeof(n_sub), hipMemcpyDeviceToHost), "hipMemcpy");
    st = ensure_sur(ctx, b.max_chunks, n_sub);
    if (st != GL_OK) return st;
    if (n_sub > 0) {
        hipLaunchKernelGGL(k_sur_enum, dim3((unsigned)total_chunks), dim3(64), 0, s, times, shared, ctx->sc,
                           ctx->seg_begin, ctx->chunk_off, ctx->ctr, ctx->masks, ctx->chunk_set,
                           ctx->chunk_sub, ctx->s_feat, ctx->s_fsph, ctx->s_scale, ctx->s_t, ctx->s_F,
                           ctx->s_bin, ctx->s_set);
        st = gl_mlp_forward(mlp, ctx->s_feat, n_sub, ctx->s_pred, s);
        if (st != GL_OK) return fail(ctx, st, "surrogate network forward");
        hipLaunchKernelGGL(k_reset_head, dim3(1), dim3(1), 0, s, ctx->ctr);
        hipLaunchKernelGGL(k_sur_gate, dim3((unsigned)((n_sub + 255) / 256)), dim3(256), 0, s, ctx->s_pred,
                           ctx->s_fsph, ctx->s_scale, ctx->s_bin, table, safety, tol, n_sub, ctx->s_F,
                           ctx->s_fb, ctx->ctr);
        const int64_t grid = std::max<int64_t>(1, std::min<int64_t>((int64_t)ctx->n_cu * ctx->waves_per_cu,
                                                                    (n_sub + 63) / 64));
        hipLaunchKernelGGL(k_sur_exact, dim3((unsigned)grid), dim3(64), 0, s, ctx->s_fb, ctx->ctr, ctx->s_t,
                           ctx->s_set, ctx->sc, ctx->s_F);
        hipLaunchKernelGGL(k_sur_reduce, dim3((unsigned)total_chunks), dim3(64), 0, s, ctx->sc, ctx->seg_begin,
                           ctx->chunk_off, ctx->ctr, ctx->masks, ctx->chunk_set, ctx->chunk_sub, ctx->s_F, out);
        GL_HIP(hipGetLastError(), "kernel launch");
    }
    GL_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    unsigned long long nfb = 0;
    if (n_sub > 0) GL_HIP(hipMemcpy(&nfb, &ctx->ctr->head, sizeof(nfb), hipMemcpyDeviceToHost), "hipMemcpy");
    if (n_sub_out) *n_sub_out = n_sub;
    if (n_fallback_out) *n_fallback_out = (int64_t)nfb;
    return GL_OK;
}

const char* gl_version(void) { return "0.1.0"; }

}  // extern "C"
