// gl_lib.hip -- kernels and C ABI of the oblate transit light-curve library.
//
// Pipeline of one gl_lightcurve_batch call (all on the caller's stream):
//   k_prep      one thread per parameter set: domain checks, derived constants
//               (projected ellipse from eqs. dx, dy1, dy2, orbit, limb darkening),
//               CSR segment checks, number of 64-output chunks per set.
//   k_scan      one workgroup: exclusive scan of the chunk counts (CSR only).
//   k_window    one wavefront per 16 (shared grid) or 4 (CSR) chunks of 64
//               consecutive outputs of one set (k_window_grid / k_window):
//               outputs whose exposure cannot overlap the star are written as
//               1 (NaN for an invalid set); chunks with in-window outputs get
//               flux slots for their sub-samples, a work-chunk entry and one
//               group entry per 64 sub-samples.
//   k_classify  one wavefront per group: each sub-sample is classified by its
//               ellipse centre: off the disk (flux 1 now), whole ellipse well
//               inside (trapezoid list, with its rule order), hard (hard list).
//   k_trap      one thread per trapezoid entry (tiles counting-sorted by rule
//               order in LDS): mu integral of the whole ellipse.
//   k_hard      one thread per hard entry: intersection quartic, break points,
//               limb arcs in closed form, ellipse arcs appended to an arc list;
//               whole ellipses near the limb go to the nested-trapezoid list.
//   k_gk<L>     level L = 0, 1 of the self-checking arc rule: one thread per
//               Gauss-Kronrod piece (2^L pieces per arc, summed across lanes);
//               arcs whose error estimate is too large go on to level L + 1.
//   k_rare      the rare paths in one launch: one thread per in-place entry
//               (nested periodic trapezoid, or the whole boundary walk with the
//               arc rule in place), and one per arc that reached level 2 (the
//               rule from there on).
//   k_combine   one thread per hard entry: limb sums + its arcs -> flux.
//   k_average   one wavefront per listed chunk: box average of each output's
//               sub-samples in a fixed order (deterministic); its first
//               wavefront records the pass's work-list demand (sizes the next
//               batch).
//   k_compute   the fused per-lane evaluation, for chunks whose sub-samples
//               did not fit the work-list capacities (and the chunks of
//               tidally-locked sets); returns at once when none is queued.
// A batch too large for one pass runs the pipeline once per range of sets.
// Every list is appended through per-shard counters (see kShards).  The
// launches are captured once into a HIP graph and replayed while the
// arguments stay the same.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "gl.h"
#include "gl_device.h"
#include "gl_index.h"
#include "gl_internal.h"

namespace {

constexpr int kChunk = 64;
constexpr int kScanThreads = 1024;

constexpr int kCensus = 11;
constexpr int kLevels = gl::kArcMaxLevel + 1;

// Appended work lists are split into kShards shards, each with its own
// counter on its own 128-byte line and its own region of the list: a
// wavefront appends to shard (its workgroup index mod kShards), so the
// atomics spread over many L2 lines instead of serialising on one.
#ifndef GL_SHARDS
#define GL_SHARDS 64
#endif
constexpr int kShards = GL_SHARDS;  // a power of two, at most 64 (one lane per shard)
static_assert(kShards >= 2 && kShards <= 64 && (kShards & (kShards - 1)) == 0, "shard count");
enum : int {
    L_SUB = 0,   // sub-sample flux slots (reserved per chunk)
    L_WC,        // chunks evaluated through the lists
    L_GRP,       // groups of up to 64 sub-samples of one chunk
    L_TRAP,      // whole ellipses for the trapezoid stage
    L_HARD,      // hard samples
    L_NEST,      // whole ellipses near the limb for the nested trapezoid
    L_NET,       // surrogate batches: sub-samples whose residual the network predicts
    L_ARC,       // ellipse arcs (storage)
    L_LVL0,      // indices of the arcs at level 0 .. kArcMaxLevel of the arc rule
    kLists = L_LVL0 + gl::kArcMaxLevel + 1
};

// Work-list demand of the batches run on a context: `norm` is the largest
// per-shard demand of each list seen in one pass, times that batch's number of
// passes (what one pass over the whole batch would need); demand that a full
// upstream list hid (a chunk without flux slots is never classified) is
// estimated from the upstream list's ratio of demand to entries kept.
struct Demand {
    unsigned long long norm[kLists];
    double sub_per_slot;           // largest ratio of in-window sub-samples to output slots of a batch
    unsigned long long cur_sub;    // running sum over the passes of the current batch
};

struct alignas(128) LineCount {
    unsigned long long v;
    unsigned long long pad[15];
};

struct Counters {
    unsigned long long total_chunks;  // written by k_scan
    unsigned long long head;          // work head of the surrogate path
    unsigned int status;              // bit 0: invalid set, bit 1: bad CSR segment, bit 2: non-finite time
    unsigned int pad;
    unsigned long long n_fb;          // chunks queued for the fused kernel
    unsigned long long fb_head;       // work head of the fused kernel
    // arcs accepted at the arc rule's last level above its tolerance, summed
    // over every batch since gl_ctx_get_unconverged last read it
    unsigned long long unconverged;
    unsigned long long fused_batch;   // chunks of the latest batch evaluated by the fused kernel
    unsigned long long net_total;     // rows of the current pass's network batch
    double ll_norm;                   // likelihood batches on a shared grid: sum log(sigma) + (N/2) log(2 pi)
    Demand demand;                    // kept here; k_demand stores a copy to the host's record
    // work census (census launches only): in-window sub-samples, whole-on-star,
    // intersecting, in-window but off the star, trapezoid nodes of the rigorous
    // rule, Gauss-Kronrod pieces, Newton steps, limb arcs, nested-trapezoid
    // nodes, ellipse arcs, arcs accepted unconverged
    // tallies added by every wavefront of a launch go to the shard of its
    // workgroup (one address for all of them serialises the atomics at L2);
    // the host sums the shards
    LineCount census[kCensus][kShards];
    LineCount sur[3][kShards];        // surrogate batches: in-window sub-samples, of those
                                      // reaching the disk, of those accepted by the gate
    LineCount lc[kLists][kShards];    // shard counters (reset by k_prep)
};

// One sub-sample handed to the trapezoid or the hard stage.
struct Entry {
    double x0, y0;  // ellipse centre
    int set;        // -1: empty slot (its chunk overflowed a list)
    int sub;        // flux slot; trapezoid entries carry the rule order in bits 27..30
};
constexpr int kSubBits = 27;
constexpr int kSubMask = (1 << kSubBits) - 1;

// A chunk on the work lists and its first flux slot.
struct WorkChunk {
    int64_t c, base;          // base -1: empty slot
    unsigned long long mask;  // in-window outputs of the chunk
    int64_t i0;               // output index of the chunk's first output
    int nss, pad;
};

// Up to 64 consecutive sub-samples [f0, min(f0 + 64, cnt)) of chunk c, with
// what classifying them needs (no further index lookups).
struct Group {
    int64_t c, base;          // c -1: empty slot
    unsigned long long mask;  // in-window outputs of the chunk
    int64_t tb;               // index in `times` of the chunk's first output
    int f0, cnt;
    int set, pad;
};

// A hard sample after its boundary walk: the closed-form limb sums and its
// range in the arc list (what the final combination reads).  Its ellipse
// frame is kept beside it, in an array of its own indexed the same way.
struct HardRec {
    gl::Sums limb;
    int set, sub;
    int arc_begin, n_arcs;  // n_arcs = 0: the flux slot is already written
};

// One ellipse arc on the star (tau-rule description).
struct ArcRec {
    double cc, sc, h;
};

// Entry of a level list: an arc and the hard slot whose frame it uses, so
// that the two records load side by side.
struct ArcRef {
    int arc, hard;
};

// Device pointers and per-shard capacities of the work lists.
struct Pipe {
    double* fsub;          // sub-sample fluxes
    WorkChunk* wc;
    Group* grp;
    int64_t* fb_chunk;     // chunks for the fused kernel
    Entry* trap;
    Entry* hard;
    Entry* nest;
    HardRec* hrec;         // indexed like `hard`
    gl::Frame* hfr;        // indexed like `hard`: ellipse frame of a sample with arcs
    ArcRec* arcs;
    gl::Sums* arc_res;     // indexed like `arcs`
    ArcRef* lvl[kLevels];  // arcs evaluated at level L
    int64_t scap[kLists];  // entries per shard
    // surrogate batches (NULL otherwise): sub-samples the gate accepts are
    // integrated for the sphere of equal projected area (their entries carry
    // kSphBit in `set`) and, unless their bin takes the sphere alone, listed
    // for the network, whose prediction is added to the flux slot
    Entry* net;                  // L_NET list
    const gl::SetConst* sph;     // sphere constants per set
    const float* gate_table;     // calibrated scaled-error bound per bin (< 0: never accept)
    const uint8_t* gate_zero;    // per bin: 1 = the sphere alone (no network)
    double gate_k;               // safety / tolerance
    uint16_t* net_x;             // dense network rows (BF16 features)
    int64_t* net_slot;           // their flux slots
    double* net_scale;           // their residual scales
    float* net_y;                // network outputs
};

constexpr int kSphBit = 1 << 30;  // Entry::set flag: integrate the equal-area sphere

// set constants of a list entry: the parameter set's, or its sphere's
__device__ __forceinline__ const gl::SetConst& entry_set(const gl::SetConst* __restrict__ sc, const Pipe& P, int set)
{
    return (set & kSphBit) ? P.sph[set & (kSphBit - 1)] : sc[set];
}

// ---------------------------------------------------------------- kernels
// A batch runs as one or more passes over consecutive ranges of its
// parameter sets (the whole pipeline per pass); `ld` is the row stride of the
// parameter block, `first` / `last` mark the batch's first and last pass
// (census reset, CSR end checks).
// SHAPE 0: the oblate block (GL_NPARAM rows), 1: general ellipsoids, 2: MCMC
// walkers (converted to the oblate block); one instance per block kind.
template <int SHAPE>
__global__ void k_prep(const double* __restrict__ params, int64_t ld, int64_t n_sets,
                       const int64_t* __restrict__ offsets, int64_t n_times,
                       const int32_t* __restrict__ n_ss, const double* __restrict__ t_exp,
                       gl::SetConst* __restrict__ sc, int64_t* __restrict__ seg_begin,
                       int64_t* __restrict__ seg_len, int64_t* __restrict__ chunk_off,
                       Counters* __restrict__ ctr, int64_t cps_shared, int first, int last,
                       gl::SetConst* __restrict__ sph, const double* __restrict__ sigma,
                       int64_t n_sigma, double* __restrict__ norm)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s == 0) {
        ctr->head = 0ull;
        ctr->n_fb = ctr->fb_head = 0ull;
        if (first) {
            ctr->fused_batch = 0ull;
        }
    }
    for (int64_t i = s; i < (int64_t)kLists * kShards; i += (int64_t)gridDim.x * blockDim.x)
        ctr->lc[i / kShards][i % kShards].v = 0ull;
    if (first)
        for (int64_t i = s; i < (int64_t)(kCensus + 3) * kShards; i += (int64_t)gridDim.x * blockDim.x) {
            const int64_t r = i / kShards, j = i % kShards;
            (r < kCensus ? ctr->census[r][j] : ctr->sur[r - kCensus][j]).v = 0ull;
        }
    if (norm && blockIdx.x == gridDim.x - 1) {
        // the extra last workgroup: a shared grid's likelihood normalisation
        // sum log(sigma) + (N/2) log(2 pi), in a fixed order
        __shared__ double part[256 / 64];
        double acc = 0.0;
        for (int64_t i = threadIdx.x; i < n_sigma; i += blockDim.x) acc += log(sigma[i]);
        for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d);
        if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0)
            norm[0] = ((part[0] + part[1]) + (part[2] + part[3])) + 0.5 * (double)n_sigma * 1.8378770664093454836;
        return;
    }
    if (s >= n_sets) return;
    constexpr int rows = SHAPE == 1 ? gl::kEllParams : GL_NPARAM;
    double p[rows];
#pragma unroll
    for (int i = 0; i < rows; ++i) p[i] = params[(int64_t)i * ld + s];
    if (SHAPE == 2) {
        double w[gl::kWalkParams];
#pragma unroll
        for (int i = 0; i < gl::kWalkParams; ++i) w[i] = p[i];
        gl::walker_to_params(w, p);
    }
    const int nss = n_ss ? n_ss[s] : 1;
    const double te = t_exp ? t_exp[s] : 0.0;
    gl::SetConst c;
    bool ok;
    if constexpr (SHAPE == 1) ok = gl::make_set_const_ell(p, te, nss, c);
    else ok = gl::make_set_const(p, te, nss, c);
    int64_t b, e;
    unsigned int flag = ok ? 0u : 1u;
    if (offsets) {
        b = offsets[s];
        e = offsets[s + 1];
        bool seg_ok = (b >= 0) && (e >= b) && (e <= n_times);
        if (s == 0 && first) seg_ok = seg_ok && (b == 0);
        if (s == n_sets - 1 && last) seg_ok = seg_ok && (e == n_times);
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
    if (sph) sph[s] = gl::sphere_of(c);
    seg_begin[s] = b;
    seg_len[s] = e - b;
    if (cps_shared > 0) {
        // shared grid, every set has cps_shared chunks: the exclusive scan in
        // closed form (no k_scan launch)
        chunk_off[s] = s * cps_shared;
        if (s == n_sets - 1) {
            chunk_off[n_sets] = n_sets * cps_shared;
            ctr->total_chunks = (unsigned long long)(n_sets * cps_shared);
        }
    } else {
        chunk_off[s] = (e - b + kChunk - 1) / kChunk;
    }
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


__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const unsigned int lo = __builtin_amdgcn_readfirstlane((unsigned int)(v & 0xffffffffll));
    const unsigned int hi = __builtin_amdgcn_readfirstlane((unsigned int)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Occupancy requests of the list kernels (waves per SIMD; 0 = the compiler's
// choice), for launch-plan experiments at build time.
#ifndef GL_WAVES_TRAP
#define GL_WAVES_TRAP 0
#endif
#ifndef GL_WAVES_HARD
#define GL_WAVES_HARD 4  // measured: 4 waves/SIMD (a few spills) beats 3 (no spills) by ~10 %
#endif
#ifndef GL_WAVES_GK
#define GL_WAVES_GK 0
#endif
#define GL_WAVES(n) __attribute__((amdgpu_waves_per_eu((n) > 0 ? (n) : 1)))
// Issue priority (0-3) of the hard-sample chain's waves (hard samples, arc
// levels): the trapezoid kernel on the other stream shares SIMDs with them,
// and the chain is the longer branch of the step, so its waves issue first
// (on the walker batch 2 measured ~1.5 % faster per step than 0, and 3 no
// better than 2; the trapezoid launch stretches into its slack).
#ifndef GL_CHAIN_PRIO
#define GL_CHAIN_PRIO 2
#endif
// Where a surrogate batch evaluates its network: 0 after the join on the
// caller's stream; 1 on the second stream, before the trapezoid and the fused
// kernel; 2 on the second stream, with the trapezoid and the fused kernel
// after the hard chain on the caller's stream.
#ifndef GL_SUR_NET_SIDE
#define GL_SUR_NET_SIDE 2
#endif
// Default persistent grid of the trapezoid stage in wavefronts per CU.
#ifndef GL_TRAP_WAVES_PER_CU
#define GL_TRAP_WAVES_PER_CU 16
#endif
// Persistent grid of the classification in wavefronts per CU.
#ifndef GL_CLASSIFY_WAVES_PER_CU
#define GL_CLASSIFY_WAVES_PER_CU 24
#endif
// Persistent grid of the arc-rule levels in wavefronts per CU (0: the plan's);
// 20 = five per SIMD, what their register use allows (measured ~4 % faster
// than the plan's 16 on the arc stage).
#ifndef GL_GK_WAVES_PER_CU
#define GL_GK_WAVES_PER_CU 20
#endif

// ---------------------------------------------------------------- work-list helpers
// Set bits of m below the calling lane (mbcnt: no lane mask is kept live).
__device__ __forceinline__ int lanes_below(unsigned long long m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// Adds a wave's census counts (one atomic per counter).
__device__ __forceinline__ void census_add(Counters* ctr, int idx, unsigned long long v)
{
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(&ctr->census[idx][blockIdx.x % kShards].v, v);
}

// Adds a wave's count of unconverged arcs (and to the census in census launches).
__device__ __forceinline__ void unconverged_add(Counters* ctr, int v, bool census)
{
    unsigned long long u = (unsigned long long)v;
    for (int d = 32; d >= 1; d >>= 1) u += __shfl_xor(u, d);
    if ((threadIdx.x & 63) == 0 && u) {
        atomicAdd(&ctr->unconverged, u);
        if (census) atomicAdd(&ctr->census[10][blockIdx.x % kShards].v, u);
    }
}

// Reserves m slots of list l in shard j for the calling wavefront (called by
// every lane; lane 0 does the atomic): returns the position in the shard.
__device__ __forceinline__ int64_t reserve(Counters* ctr, int l, int j, unsigned long long m)
{
    unsigned long long p = 0;
    if ((threadIdx.x & 63) == 0 && m) p = atomicAdd(&ctr->lc[l][j].v, m);
    return uniform64((int64_t)p);
}

// Entries appended to shard j of list l.  The trapezoid and hard lists share
// one counter word per shard (low and high 32 bits), so that a classifying
// wavefront reserves in both with one atomic.
__device__ __forceinline__ int64_t list_count(const Counters* ctr, int l, int j)
{
    if (l == L_TRAP) return (int64_t)(ctr->lc[L_TRAP][j].v & 0xffffffffull);
    if (l == L_HARD) return (int64_t)(ctr->lc[L_TRAP][j].v >> 32);
    return (int64_t)ctr->lc[l][j].v;
}

// Wavefront view of a sharded list: lanes 0..kShards-1 hold the shard counts
// (clamped to the capacity) and their inclusive prefix sums.
struct ShardMap {
    int64_t incl;   // lane j < kShards: entries in shards 0..j (counts clamped to the capacity)
    int64_t total;  // wavefront-uniform
};

__device__ __forceinline__ ShardMap shard_map(const Counters* ctr, int l, int64_t scap)
{
    const int lane = threadIdx.x & 63;
    ShardMap m;
    m.incl = lane < kShards ? std::min<int64_t>(list_count(ctr, l, lane), scap) : 0;
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t v = __shfl_up(m.incl, d);
        if (lane >= d) m.incl += v;
    }
    m.total = uniform64(__shfl(m.incl, kShards - 1));
    return m;
}

// List slot of the g-th entry (0 <= g < total) in shard order; every lane of
// the wavefront must call it.
__device__ __forceinline__ int64_t shard_slot(const ShardMap& m, int64_t g, int64_t scap)
{
    int j = 0;
#pragma unroll
    for (int step = kShards / 2; step >= 1; step >>= 1) {
        const int64_t v = __shfl(m.incl, j + step - 1);
        if (v <= g) j += step;
    }
    const int64_t prev = __shfl(m.incl, j > 0 ? j - 1 : 0);  // entries before shard j
    return (int64_t)j * scap + (g - (j > 0 ? prev : 0));
}

// lane k's value v for a wave-uniform k (no LDS round trip)
__device__ __forceinline__ int64_t readlane64(int64_t v, int k)
{
    const unsigned int lo = __builtin_amdgcn_readlane((unsigned int)(v & 0xffffffffll), k);
    const unsigned int hi = __builtin_amdgcn_readlane((unsigned int)((uint64_t)v >> 32), k);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// shard_slot for a wavefront whose lanes that matter hold indices in the
// uniform range [g_first, g_last] (consecutive entries of the list): when the
// range lies in one shard (nearly always: a shard holds thousands of entries),
// every lane's slot follows from that shard's first index, found once for the
// wavefront; otherwise the per-lane search.  Lanes outside the range get a
// slot in bounds that they must not use.
__device__ __forceinline__ int64_t shard_slot_run(const ShardMap& m, int64_t g, int64_t g_first, int64_t g_last,
                                                  int64_t scap)
{
    g_first = uniform64(g_first);
    g_last = uniform64(g_last);
    int j = 0;  // wave-uniform: the shard holding g_first
#pragma unroll
    for (int step = kShards / 2; step >= 1; step >>= 1)
        if (readlane64(m.incl, j + step - 1) <= g_first) j += step;
    if (g_last < readlane64(m.incl, j)) {
        const int64_t o = g - (j > 0 ? readlane64(m.incl, j - 1) : 0);
        return (o >= 0 && o < scap) ? (int64_t)j * scap + o : 0;
    }
    return shard_slot(m, g, scap);
}

// shard_slot for a wave-uniform index g: the shard found with scalar reads of
// the prefix counts (no cross-lane shuffles).
__device__ __forceinline__ int64_t shard_slot_uniform(const ShardMap& m, int64_t g, int64_t scap)
{
    g = uniform64(g);
    int j = 0;
#pragma unroll
    for (int step = kShards / 2; step >= 1; step >>= 1)
        if (readlane64(m.incl, j + step - 1) <= g) j += step;
    const int64_t prev = j > 0 ? readlane64(m.incl, j - 1) : 0;
    return (int64_t)j * scap + (g - prev);
}

// Queues chunk c for the fused kernel once (the first caller wins).
__device__ __forceinline__ void to_fused(Counters* ctr, const Pipe& P, int* chunk_fb, int64_t c)
{
    if (atomicExch(&chunk_fb[c], 1) == 0) P.fb_chunk[atomicAdd(&ctr->n_fb, 1ull)] = c;
}

// Window test: outputs whose exposure cannot overlap the star are written as
// 1 (NaN for an invalid set or a non-finite time); a 64-bit mask of the others
// and the chunk's set are kept.  With `lists`, every chunk with in-window
// outputs gets its flux slots, a work-chunk entry and one group entry per 64
// sub-samples (one reservation per list for the wavefront); a chunk that does
// not fit is queued for the fused kernel.

// Appends the wavefront's chunks with in-window outputs to the lists: lane k
// describes chunk c_k (cnt_k sub-samples, 0 if none), positions come from
// wavefront scans, one reservation per list.
__device__ __forceinline__ void window_lists(Counters* ctr, const Pipe& P, int* chunk_fb, int shard,
                                             int64_t c_k, int cnt_k, unsigned long long mask_k,
                                             int64_t i0_k, int64_t tb_k, int nss_k, int set_k)
{
    const int lane = threadIdx.x & 63;
    const int ng_k = (cnt_k + kChunk - 1) / kChunk;
    // inclusive scans: sub-samples and (work chunks | groups << 16)
    int64_t isub = cnt_k;
    int iwg = (cnt_k > 0 ? 1 : 0) | (ng_k << 16);
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t v = __shfl_up(isub, d);
        const int u = __shfl_up(iwg, d);
        if (lane >= d) {
            isub += v;
            iwg += u;
        }
    }
    const int64_t tot_sub = __shfl(isub, 63);
    const int tot_wg = __shfl(iwg, 63);
    int64_t os = reserve(ctr, L_SUB, shard, (unsigned long long)tot_sub);
    int64_t ow = reserve(ctr, L_WC, shard, (unsigned long long)(tot_wg & 0xffff));
    int64_t og = reserve(ctr, L_GRP, shard, (unsigned long long)(tot_wg >> 16));
    if (cnt_k == 0) return;
    os += isub - cnt_k;
    ow += (iwg & 0xffff) - 1;
    og += (iwg >> 16) - ng_k;
    const int64_t scs = P.scap[L_SUB], scw = P.scap[L_WC], scg = P.scap[L_GRP];
    const bool ok = os + cnt_k <= scs && ow < scw && og + ng_k <= scg;
    const int64_t base = ok ? (int64_t)shard * scs + os : -1;
    chunk_fb[c_k] = 0;
    if (ow < scw) P.wc[(int64_t)shard * scw + ow] = WorkChunk{c_k, base, mask_k, i0_k, nss_k, 0};
    for (int j = 0; j < ng_k && og + j < scg; ++j)
        P.grp[(int64_t)shard * scg + og + j] = Group{ok ? c_k : -1, base, mask_k, tb_k, j * kChunk, cnt_k, set_k, 0};
    if (!ok) to_fused(ctr, P, chunk_fb, c_k);
}

// One time grid for every set: one wavefront per kWinGrid consecutive chunks
// of one set (bx = ceil(chunks per set / kWinGrid) wavefronts per set, set
// major);
// every time load is issued before the first test, and lane k keeps chunk k's
// mask for one store of all of them.
constexpr int kWinGrid = gl::kWinGridChunks;

__global__ void __launch_bounds__(64)
k_window_grid(const double* __restrict__ times, int64_t n_times, int64_t cps,
              const gl::SetConst* __restrict__ sc, Counters* __restrict__ ctr,
              unsigned long long* __restrict__ masks, int* __restrict__ chunk_set,
              double* __restrict__ out, int lists, Pipe P, int* __restrict__ chunk_fb)
{
    const int lane = threadIdx.x;
    int64_t s, lc0;  // the set and its first chunk here
    int nk;
    gl::window_grid_block(blockIdx.x, cps, kWinGrid, s, lc0, nk);
    const int64_t ob = s * n_times;  // the set's first output (its segment start)
    const gl::SetConst& S = sc[s];
    double t[kWinGrid];
#pragma unroll
    for (int k = 0; k < kWinGrid; ++k) {
        const int64_t pos = (lc0 + k) * kChunk + lane;
        t[k] = (k < nk && pos < n_times) ? times[pos] : 0.0;
    }
    const bool valid = S.valid;
    const double reach = S.half_win + 0.5 * S.t_exp;
    unsigned long long my_mask = 0ull, any = 0ull;
#pragma unroll
    for (int k = 0; k < kWinGrid; ++k) {
        const int64_t pos = (lc0 + k) * kChunk + lane;
        bool work = false;
        if (k < nk && pos < n_times) {
            if (!valid || !gl::finite_d(t[k])) {
                out[ob + pos] = __builtin_nan("");
                if (valid) atomicOr(&ctr->status, 4u);
            } else {
                work = fabs(gl::phase_time(S, t[k])) < reach;
                // streamed past the caches: the 1s are never read back, and
                // keeping them out of L2 leaves it to the work lists
                if (!work) __builtin_nontemporal_store(1.0, out + ob + pos);
            }
        }
        const unsigned long long m = __ballot(work);
        if (lane == k) my_mask = m;
        any |= m;
    }
    const int64_t c = s * cps + lc0 + lane;  // lane k: chunk k
    if (lane < nk) {
        masks[c] = my_mask;
        chunk_set[c] = (int)s;
    }
    if (!lists || !any) return;
    if (S.locked) {
        // a locked shadow changes per sample: the fused kernel evaluates it
        if (lane < nk && my_mask) {
            chunk_fb[c] = 0;
            to_fused(ctr, P, chunk_fb, c);
        }
        return;
    }
    const int cnt = lane < nk ? __popcll(my_mask) * S.n_ss : 0;
    const gl::ChunkPos cp = gl::chunk_pos(true, ob, lc0 + lane);
    const int shard = (int)(blockIdx.x % kShards);
    window_lists(ctr, P, chunk_fb, shard, c, cnt, my_mask, cp.out0, cp.time0, S.n_ss, (int)s);
}

// CSR segments: one wavefront per group of kWinChunks consecutive chunks (their
// memory operations overlap), the set of the first chunk found by binary
// search and stepped along from there.
constexpr int kWinChunks = gl::kWinCsrChunks;

__global__ void __launch_bounds__(256)
k_window(const double* __restrict__ times, int64_t n_sets,
         const gl::SetConst* __restrict__ sc, const int64_t* __restrict__ seg_begin,
         const int64_t* __restrict__ seg_len, const int64_t* __restrict__ chunk_off,
         Counters* __restrict__ ctr, unsigned long long* __restrict__ masks,
         int* __restrict__ chunk_set, double* __restrict__ out, int lists, Pipe P,
         int* __restrict__ chunk_fb)
{
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t total = (int64_t)ctr->total_chunks;
    const int64_t g = (int64_t)blockIdx.x * 4 + wv;
    const int64_t c_first = g * kWinChunks;
    int64_t s = 0;
    if (c_first < total) s = uniform64(gl::set_of_chunk(chunk_off, n_sets, c_first));
    // lane k (k < kWinChunks) collects chunk k's description for the lists
    int cnt_l = 0, nss_l = 0, set_l = 0, lock_l = 0;
    unsigned long long mask_l = 0ull, any = 0ull;
    int64_t i0_l = 0, t0_l = 0;
#pragma unroll
    for (int k = 0; k < kWinChunks; ++k) {
        const int64_t c = c_first + k;
        if (c >= total) continue;
        while (s + 1 < n_sets && chunk_off[s + 1] <= c) ++s;  // uniform
        const int64_t pos = (c - chunk_off[s]) * kChunk + lane;  // position in the segment
        const bool in_seg = pos < seg_len[s];
        const int64_t i = seg_begin[s] + pos;
        const gl::SetConst& S = sc[s];
        bool work = false;
        if (in_seg) {
            const double t = times[i];
            if (!S.valid || !gl::finite_d(t)) {
                out[i] = __builtin_nan("");
                if (S.valid) atomicOr(&ctr->status, 4u);
            } else {
                const double tau = gl::phase_time(S, t);
                work = fabs(tau) < S.half_win + 0.5 * S.t_exp;
                if (!work) __builtin_nontemporal_store(1.0, out + i);
            }
        }
        const unsigned long long m = __ballot(work);
        if (lane == 0) {
            masks[c] = m;
            chunk_set[c] = (int)s;
        }
        any |= m;
        if (lane == k) {
            mask_l = m;
            cnt_l = __popcll(m) * S.n_ss;
            nss_l = S.n_ss;
            set_l = (int)s;
            lock_l = S.locked;
            const gl::ChunkPos cp = gl::chunk_pos(false, seg_begin[s], c - chunk_off[s]);
            i0_l = cp.out0;
            t0_l = cp.time0;
        }
    }
    if (!lists || !any) return;
    // chunks of locked sets (per-sample shadow) go to the fused kernel
    window_lists(ctr, P, chunk_fb, (int)(g % kShards), c_first + lane, lock_l ? 0 : cnt_l, mask_l, i0_l, t0_l,
                 nss_l, set_l);
    if (lock_l && mask_l) {
        chunk_fb[c_first + lane] = 0;
        to_fused(ctr, P, chunk_fb, c_first + lane);
    }
}

// Classification: one wavefront per group of up to 64 sub-samples of one
// chunk, classified by the ellipse centre: off the disk (flux 1 now), whole
// ellipse provably well inside (trapezoid list with its rule order, in lane
// order: k_trap sorts its tiles by order), everything else (hard list).  A
// group that does not fit the lists sends its chunk to the fused kernel.
// SUR (surrogate batches): a sub-sample whose ellipse reaches the disk is
// first put to the gate; if accepted it is classified and listed for the
// sphere of equal projected area instead, and listed for the network unless
// its bin takes the sphere alone.
// Groups a wavefront classifies per list reservation (each reservation is a
// round trip to the shard's counter; two groups per round trip measured
// 1.5-2 us faster on the walker batch, four slower: their entries held over
// the reservation cost occupancy).
constexpr int kClsBatch = 2;

template <bool CENSUS, bool SUR>
__global__ void __launch_bounds__(64)
k_classify(const double* __restrict__ times, int shared_grid, const gl::SetConst* __restrict__ sc,
           const int64_t* __restrict__ seg_begin, const int64_t* __restrict__ chunk_off,
           Counters* __restrict__ ctr, Pipe P, const unsigned long long* __restrict__ masks,
           const int* __restrict__ chunk_set, int* __restrict__ chunk_fb)
{
    __shared__ double lds_t[kClsBatch][kChunk];  // times of each chunk's in-window outputs, compacted
    const int lane = threadIdx.x;
    const int shard = (int)(blockIdx.x % kShards);
    const int64_t gcap = P.scap[L_GRP];
    const ShardMap m = shard_map(ctr, L_GRP, gcap);
    unsigned long long c_in = 0, c_whole = 0, c_off = 0, c_sur_in = 0, c_sur_on = 0, c_sur_acc = 0;
    const int64_t gstride = gridDim.x;
    for (int64_t g0 = blockIdx.x; g0 < m.total; g0 += gstride * kClsBatch) {
        // the batch's group records, loaded together (their latencies overlap)
        Group G[kClsBatch];
#pragma unroll
        for (int b = 0; b < kClsBatch; ++b) {
            const int64_t gi = g0 + b * gstride;
            G[b] = Group{};  // a slot past the list's end: empty, every field defined
            G[b].c = -1;
            if (gi < m.total) G[b] = P.grp[shard_slot_uniform(m, gi, gcap)];
        }
#pragma unroll
        for (int b = 0; b < kClsBatch; ++b) {
            const unsigned long long M = (unsigned long long)uniform64((int64_t)G[b].mask);
            if (uniform64(G[b].c) >= 0 && ((M >> lane) & 1ull))
                lds_t[b][lanes_below(M)] = times[uniform64(G[b].tb) + lane];
        }
        __syncthreads();
        // each group's sub-samples classified, entries kept until the reservation
        double x0[kClsBatch], y0[kClsBatch];
        int cls[kClsBatch], eset[kClsBatch], sub[kClsBatch];
        bool to_net[kClsBatch];
        int64_t cb[kClsBatch];
        int64_t sb[kClsBatch];
#pragma unroll
        for (int b = 0; b < kClsBatch; ++b) {
            const int64_t c = uniform64(G[b].c);
            cb[b] = c;
            cls[b] = gl::kOffDisk - 1;  // no sample on this lane
            x0[b] = y0[b] = 0.0;
            to_net[b] = false;
            const int64_t s = __builtin_amdgcn_readfirstlane(G[b].set);
            sb[b] = s;
            eset[b] = (int)s;           // list entries' set (kSphBit: the sphere)
            // an empty group (c < 0: past the list's end, or a slot of an
            // overflowing chunk) has no sample on any lane, whatever its
            // other fields hold
            const bool grp = c >= 0;
            const int64_t base = grp ? uniform64(G[b].base) : 0;
            const int f0 = grp ? __builtin_amdgcn_readfirstlane(G[b].f0) : 0;
            const int cnt = grp ? __builtin_amdgcn_readfirstlane(G[b].cnt) : 0;
            const int f = f0 + lane;
            sub[b] = (int)(base + f);
            if (grp && f < cnt) {
                const gl::SetConst& S = sc[s];
                const int nss = S.n_ss;
                const double inv_nss = 1.0 / (double)nss;
                const float inv_nss_f = 1.0f / (float)nss;
                // f / nss for f < 4096, nss <= 64 from a float product (exact floor)
                const int o = (int)(((float)f + 0.5f) * inv_nss_f), j = f - o * nss;
                const double t = lds_t[b][o] + (((double)j + 0.5) * inv_nss - 0.5) * S.t_exp;
                double xx, yy;
                int k = gl::centre_at(S, t, xx, yy) ? gl::easy_class(S, xx, yy) : gl::kOffDisk;
                if (SUR) {
                    c_sur_in += 1;
                    float fe[gl::kSurFeat];
                    double scl;
                    int bin;
                    if (k != gl::kOffDisk && gl::sur_encode(S, xx, yy, fe, scl, bin)) {
                        c_sur_on += 1;
                        const float tb = P.gate_table[bin];
                        if (tb >= 0.f && P.gate_k * (double)tb * scl <= 1.0) {
                            c_sur_acc += 1;
                            eset[b] = (int)s | kSphBit;
                            to_net[b] = P.gate_zero[bin] == 0;
                            k = gl::easy_class(P.sph[s], xx, yy);
                        }
                    }
                }
                if (k == gl::kOffDisk) P.fsub[base + f] = 1.0;
                if (CENSUS) {
                    c_in += 1;
                    c_whole += k >= 0;
                    c_off += k == gl::kOffDisk;
                }
                cls[b] = k;
                x0[b] = xx;
                y0[b] = yy;
            }
        }
        unsigned long long mt[kClsBatch], mh[kClsBatch], mn[kClsBatch];
        unsigned long long nt = 0ull, nh = 0ull, nn = 0ull;
#pragma unroll
        for (int b = 0; b < kClsBatch; ++b) {
            mt[b] = __ballot(cls[b] >= 0);
            mh[b] = __ballot(cls[b] == gl::kHard);
            mn[b] = SUR ? __ballot(to_net[b]) : 0ull;
            nt += (unsigned long long)__popcll(mt[b]);
            nh += (unsigned long long)__popcll(mh[b]);
            nn += (unsigned long long)__popcll(mn[b]);
        }
        // one atomic reserves the batch's entries of both lists: trapezoid
        // count in the low half of the shard's counter word, hard count in
        // the high half; each group then takes its part in batch order
        const unsigned long long both = (unsigned long long)reserve(ctr, L_TRAP, shard, nt | (nh << 32));
        const int64_t np0 = (SUR && nn) ? reserve(ctr, L_NET, shard, nn) : 0;
        int64_t tp = (int64_t)(both & 0xffffffffull), hp = (int64_t)(both >> 32), np = np0;
        const int64_t tcap = P.scap[L_TRAP], hcap = P.scap[L_HARD];
        Entry* tl = P.trap + (int64_t)shard * tcap;
        Entry* hl = P.hard + (int64_t)shard * hcap;
#pragma unroll
        for (int b = 0; b < kClsBatch; ++b) {
            bool fb = false;
            if (mt[b]) {
                const int64_t slot = tp + lanes_below(mt[b]);
                if (tp + __popcll(mt[b]) > tcap) {
                    // slots reserved below the capacity are marked empty
                    if (cls[b] >= 0 && slot < tcap) tl[slot].set = -1;
                    fb = true;
                } else if (cls[b] >= 0) {
                    // in lane order: the trapezoid stage sorts its tiles by rule order
                    tl[slot] = Entry{x0[b], y0[b], eset[b], sub[b] | (cls[b] << kSubBits)};
                }
                tp += __popcll(mt[b]);
            }
            if (mh[b]) {
                const int64_t slot = hp + lanes_below(mh[b]);
                if (hp + __popcll(mh[b]) > hcap) {
                    if (cls[b] == gl::kHard && slot < hcap) hl[slot].set = -1;
                    fb = true;
                } else if (cls[b] == gl::kHard) {
                    hl[slot] = Entry{x0[b], y0[b], eset[b], sub[b]};
                }
                hp += __popcll(mh[b]);
            }
            if (SUR && mn[b]) {
                // the network's rows, in the shard of this workgroup
                const int64_t ncap = P.scap[L_NET];
                const int64_t slot = np + lanes_below(mn[b]);
                if (np + __popcll(mn[b]) > ncap) {
                    if (to_net[b] && slot < ncap) P.net[(int64_t)shard * ncap + slot].set = -1;
                    fb = true;
                } else if (to_net[b]) {
                    P.net[(int64_t)shard * ncap + slot] = Entry{x0[b], y0[b], (int)sb[b], sub[b]};
                }
                np += __popcll(mn[b]);
            }
            if (__ballot(fb) && lane == 0) to_fused(ctr, P, chunk_fb, cb[b]);
        }
        __syncthreads();
    }
    if (CENSUS) {
        census_add(ctr, 0, c_in);
        census_add(ctr, 1, c_whole);
        census_add(ctr, 3, c_off);
    }
    if (SUR) {
        unsigned long long a = c_sur_in, o = c_sur_on, b = c_sur_acc;
        for (int d = 32; d >= 1; d >>= 1) {
            a += __shfl_xor(a, d);
            o += __shfl_xor(o, d);
            b += __shfl_xor(b, d);
        }
        if (lane == 0) {
            const int j = (int)(blockIdx.x % kShards);
            if (a) atomicAdd(&ctr->sur[0][j].v, a);
            if (o) atomicAdd(&ctr->sur[1][j].v, o);
            if (b) atomicAdd(&ctr->sur[2][j].v, b);
        }
    }
}

// Whole ellipses well inside the disk, the trapezoid order chosen by
// k_classify from the singularity bound.  A workgroup takes kTrapRounds x
// kTrapThreads consecutive entries, sorts their list slots by rule order in
// LDS (counting sort, ranks from LDS atomics), then each thread integrates
// kTrapRounds of them in sorted order, so the lanes of a wavefront mostly run
// the same number of nodes.
// (1024-thread workgroups and four rounds: tiles of 4096 entries; beside the
// hard-sample chain they measured ~1 % faster per step than 512 x 8)
#ifndef GL_TRAP_THREADS
#define GL_TRAP_THREADS 1024
#endif
#ifndef GL_TRAP_ROUNDS
#define GL_TRAP_ROUNDS 4
#endif
constexpr int kTrapThreads = GL_TRAP_THREADS;
constexpr int kTrapWaves = kTrapThreads / 64;
constexpr int kTrapRounds = GL_TRAP_ROUNDS;
constexpr int kTrapBuckets = gl::kTrapOrders + 1;  // the last bucket holds empty slots

template <bool CENSUS>
__global__ void __launch_bounds__(kTrapThreads) GL_WAVES(GL_WAVES_TRAP)
k_trap(const gl::SetConst* __restrict__ sc, Counters* __restrict__ ctr, Pipe P)
{
    __shared__ int lds_slot[kTrapRounds * kTrapThreads];
    __shared__ int lds_cnt[kTrapBuckets];   // entries per rule order, then their first position
    const int tid = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t scap = P.scap[L_TRAP];
    const ShardMap m = shard_map(ctr, L_TRAP, scap);
    unsigned long long nodes = 0;
    constexpr int kBlock = kTrapRounds * kTrapThreads;
    for (int64_t b0 = (int64_t)blockIdx.x * kBlock; b0 < m.total; b0 += (int64_t)gridDim.x * kBlock) {
        if (tid < kTrapBuckets) lds_cnt[tid] = 0;
        __syncthreads();
        // counting sort by rule order: an entry's place within its order comes
        // from an LDS atomic (which thread integrates which entry may change
        // from run to run; every entry's value does not)
        int bucket[kTrapRounds], rank[kTrapRounds], slot[kTrapRounds];
#pragma unroll
        for (int r = 0; r < kTrapRounds; ++r) {
            const int64_t g = b0 + r * kTrapThreads + tid;
            const int64_t gw = b0 + r * kTrapThreads + 64 * wv;  // the wavefront's first entry
            const int64_t sl = shard_slot_run(m, g < m.total ? g : 0, gw, std::min(gw + 63, m.total - 1), scap);
            int k = gl::kTrapOrders;
            if (g < m.total) {
                const Entry& e = P.trap[sl];
                if (e.set >= 0) k = e.sub >> kSubBits;
            }
            bucket[r] = k;
            slot[r] = (int)sl;
            rank[r] = atomicAdd(&lds_cnt[k], 1);
        }
        __syncthreads();
        if (tid == 0) {
            int run = 0;
            for (int q = 0; q < kTrapBuckets; ++q) {
                const int v = lds_cnt[q];
                lds_cnt[q] = run;
                run += v;
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kTrapRounds; ++r) lds_slot[lds_cnt[bucket[r]] + rank[r]] = slot[r];
        const int n_valid = lds_cnt[gl::kTrapOrders];  // start of the empty bucket
        __syncthreads();
        for (int r = 0; r < kTrapRounds; ++r) {
            const int pos = r * kTrapThreads + tid;
            if (pos >= n_valid) break;
            const Entry e = P.trap[lds_slot[pos]];
            const int oi = e.sub >> kSubBits, sub = e.sub & kSubMask;
            const gl::SetConst& S = entry_set(sc, P, e.set);
            const double sl = gl::trap_lin_inl(S, e.x0, e.y0, oi);
            P.fsub[sub] = 1.0 - gl::whole_delta(S, e.x0, e.y0, sl);
            if (CENSUS) nodes += gl::kTrapN[oi];
        }
        __syncthreads();
    }
    if (CENSUS) census_add(ctr, 4, nodes);
}

// Hard entries: intersection quartic and break points per thread; one walk
// of the boundary sums the limb arcs in closed form and keeps up to kHardArcs
// ellipse arcs in LDS, which are then appended to the arc list (one
// reservation per wavefront, positions from a wavefront scan).  Samples off
// the disk get their flux here.  Whole ellipses near the limb with no cluster
// point, samples with more arcs than that and samples whose arcs do not fit
// the arc list go to the in-place list (pushed to the shard of their own hard
// slot, so that list never overflows and this kernel makes no calls).
constexpr int kInPlace = 1 << kSubBits;  // in-place entry flag: arcs integrated per lane
constexpr int kHardArcs = 4;             // ellipse arcs a hard sample keeps for the arc list

template <bool CENSUS>
__global__ void __launch_bounds__(64) GL_WAVES(GL_WAVES_HARD)
k_hard(const gl::SetConst* __restrict__ sc, Counters* __restrict__ ctr, Pipe P)
{
    __shared__ double lds_arc[kHardArcs][3][64];  // kept arcs (cc, sc, h) per lane
    if constexpr (GL_CHAIN_PRIO > 0) __builtin_amdgcn_s_setprio(GL_CHAIN_PRIO);
    const int lane = threadIdx.x;
    const int shard = (int)(blockIdx.x % kShards);
    const int64_t scap = P.scap[L_HARD], acap = P.scap[L_ARC], ncap = P.scap[L_NEST];
    const int64_t lcap = P.scap[L_LVL0];
    const ShardMap m = shard_map(ctr, L_HARD, scap);
    unsigned long long c_whole = 0, c_part = 0, c_off = 0, c_arcs = 0;
    gl::Census ct;
    gl::NoCensus nc;
    ArcRec* al = P.arcs + (int64_t)shard * acap;
    for (int64_t g0 = (int64_t)blockIdx.x * 64; g0 < m.total; g0 += (int64_t)gridDim.x * 64) {
        const int64_t g = g0 + lane;
        const int64_t slot = shard_slot_run(m, g < m.total ? g : 0, g0, std::min(g0 + 63, m.total - 1), scap);
        Entry e{0.0, 0.0, -1, 0};
        if (g < m.total) e = P.hard[slot];
        const bool valid = g < m.total && e.set >= 0;
        if (g < m.total && !valid) P.hrec[slot].n_arcs = 0;  // slot of an overflowing chunk
        gl::HardPrep H;
        gl::Frame F{};
        gl::Sums Sm{0.0, 0.0, 0.0};
        int na = 0, na1 = 0;  // ellipse arcs walked, of which starting at level 1
        unsigned lev1 = 0u;   // bit k: kept arc k starts at level 1
        bool open = false, to_list = false;
        int flag = 0;
        if (valid) {
            const gl::SetConst& S = entry_set(sc, P, e.set);
            if (CENSUS) gl::hard_prepare<gl::Census, true>(S, e.x0, e.y0, H, ct);
            else gl::hard_prepare<gl::NoCensus, true>(S, e.x0, e.y0, H, nc);
            const int cls = gl::hard_class(H);
            if (cls == gl::CLS_FULL && H.ntc == 0) to_list = true;
            else if (cls != gl::CLS_OUT) open = true;
            if (CENSUS) {
                c_off += cls == gl::CLS_OUT;
                c_whole += cls == gl::CLS_FULL;
                c_part += cls == gl::CLS_PARTIAL;
            }
            if (open) {
                // one walk: limb arcs summed in closed form, ellipse arcs kept
                // in this lane's LDS slots until their positions are reserved
                double bp[7];
                int kind[7];
                const int nb = gl::hard_breaks(H, bp, kind);
                gl::make_frame(S, e.x0, e.y0, H.c0a, H.s0a, F);
                auto keep = [&](double cc, double scv, double h, int lev) {
                    if (na < kHardArcs) {
                        lds_arc[na][0][lane] = cc;
                        lds_arc[na][1][lane] = scv;
                        lds_arc[na][2][lane] = h;
                        lev1 |= (unsigned)lev << na;
                    }
                    na1 += lev;
                    ++na;
                };
                if (CENSUS) gl::boundary_walk(H, F, bp, kind, nb, Sm, true, keep, ct);
                else gl::boundary_walk(H, F, bp, kind, nb, Sm, true, keep, nc);
                if (na > kHardArcs) {
                    // more arcs than slots (rare): the sample is integrated in place later
                    to_list = true;
                    flag = kInPlace;
                    open = false;
                    na = na1 = 0;
                    P.hrec[slot].n_arcs = 0;
                } else if (na == 0) {  // limb arcs only
                    P.fsub[e.sub] = 1.0 - gl::sums_delta(S, Sm);
                    P.hrec[slot].n_arcs = 0;
                    open = false;
                }
            } else {
                if (!to_list) P.fsub[e.sub] = 1.0;
                P.hrec[slot].n_arcs = 0;
            }
        }
        // positions in the arc list and in the level-0 / level-1 index lists:
        // inclusive wavefront scans (arcs, level-1 starts packed in one word)
        int incl = na | (na1 << 16);
        for (int d = 1; d < 64; d <<= 1) {
            const int v = __shfl_up(incl, d);
            if (lane >= d) incl += v;
        }
        const int wpack = __shfl(incl, 63);
        const int wtotal = wpack & 0xffff, wtot1 = wpack >> 16;
        const int incl0 = (incl & 0xffff) - (incl >> 16), incl1 = incl >> 16;  // level-0 and level-1 prefixes
        incl &= 0xffff;
        const int64_t ap = reserve(ctr, L_ARC, shard, (unsigned long long)wtotal);
        const bool over = ap + wtotal > acap;
        // index lists: reserved only when the arcs are stored
        const int64_t l0p = over ? 0 : reserve(ctr, L_LVL0, shard, (unsigned long long)(wtotal - wtot1));
        const int64_t l1p = over ? 0 : reserve(ctr, L_LVL0 + 1, shard, (unsigned long long)wtot1);
        if (open) {  // 1 <= na <= kHardArcs
            if (over) {
                // arcs do not fit: the whole sample is integrated in place later
                // (no index-list entry refers to this lane's reserved arc slots)
                P.hrec[slot].n_arcs = 0;
                to_list = true;
                flag = kInPlace;
            } else {
                // the kept arcs go to this lane's reserved range, their indices
                // to the index list of their starting level (same shard: never full)
                const int64_t first = ap + incl - na;
                int64_t k0 = l0p + incl0 - (na - na1), k1 = l1p + incl1 - na1;
#pragma unroll
                for (int k = 0; k < kHardArcs; ++k) {
                    if (k < na) {
                        al[first + k] = ArcRec{lds_arc[k][0][lane], lds_arc[k][1][lane], lds_arc[k][2][lane]};
                        const ArcRef r{(int)((int64_t)shard * acap + first + k), (int)slot};
                        if ((lev1 >> k) & 1u) P.lvl[1][(int64_t)shard * lcap + (k1++)] = r;
                        else P.lvl[0][(int64_t)shard * lcap + (k0++)] = r;
                    }
                }
                P.hrec[slot] = HardRec{Sm, e.set, e.sub, (int)((int64_t)shard * acap + first), na};
                P.hfr[slot] = F;
                if (CENSUS) c_arcs += na;
            }
        }
        // in-place list, in the shard of the entry's own hard slot
        const int hs = to_list ? (int)(slot / scap) : -1;
        unsigned long long pending = __ballot(to_list);
        while (pending) {
            const int j = __shfl(hs, __builtin_ctzll(pending));
            const unsigned long long mj = __ballot(to_list && hs == j);
            const int64_t np = reserve(ctr, L_NEST, j, (unsigned long long)__popcll(mj));
            if (to_list && hs == j)
                P.nest[(int64_t)j * ncap + np + lanes_below(mj)] = Entry{e.x0, e.y0, e.set, e.sub | flag};
            pending &= ~mj;
        }
    }
    if (CENSUS) {
        census_add(ctr, 1, c_whole);
        census_add(ctr, 2, c_part);
        census_add(ctr, 3, c_off);
        census_add(ctr, 6, (unsigned long long)ct.iters);
        census_add(ctr, 7, (unsigned long long)ct.limbs);
        census_add(ctr, 9, c_arcs);
    }
}

// In-place list: whole ellipses near the limb with no cluster point take the
// nested periodic trapezoid 8 -> 64 per thread (cluster arcs in place if it
// does not settle); samples whose arcs did not fit the arc list take the
// whole boundary walk with the arc rule in place.
// (workgroups bid of nb of the rare-path launch)
template <bool CENSUS>
__device__ __forceinline__ void nested_part(const gl::SetConst* __restrict__ sc, Counters* __restrict__ ctr,
                                            const Pipe& P, int64_t bid, int64_t nb)
{
    const int lane = threadIdx.x;
    const int64_t scap = P.scap[L_NEST];
    const ShardMap m = shard_map(ctr, L_NEST, scap);
    unsigned long long nodes = 0;
    gl::Census ct;
    gl::NoCensus nc;
    for (int64_t g0 = bid * 64; g0 < m.total; g0 += nb * 64) {
        const int64_t g = g0 + lane;
        const int64_t slot = shard_slot_run(m, g < m.total ? g : 0, g0, std::min(g0 + 63, m.total - 1), scap);
        if (g >= m.total) continue;
        const Entry e = P.nest[slot];
        const int sub = e.sub & kSubMask;
        const bool in_place = (e.sub & kInPlace) != 0;
        const gl::SetConst& S = entry_set(sc, P, e.set);
        if (!in_place) {
            double sl;
            int lev;
            const bool ok = gl::trap_lin_nested_inl(S, e.x0, e.y0, sl, lev);
            if (CENSUS) nodes += 8 << (lev - 1);
            if (ok) {
                P.fsub[sub] = 1.0 - gl::whole_delta(S, e.x0, e.y0, sl);
                continue;
            }
        }
        gl::HardPrep H;
        if (CENSUS) gl::hard_prepare(S, e.x0, e.y0, H, ct);
        else gl::hard_prepare(S, e.x0, e.y0, H, nc);
        if (!in_place) H.single_cluster(H.t_near);  // did not settle: cluster at the point nearest the limb
        double bp[7];
        int kind[7];
        const int nb = gl::hard_breaks(H, bp, kind);
        gl::Frame F;
        gl::make_frame(S, e.x0, e.y0, H.c0a, H.s0a, F);
        gl::Sums Sm{0.0, 0.0, 0.0};
        if (CENSUS)
            gl::boundary_walk(H, F, bp, kind, nb, Sm, true,
                              [&](double cc, double scv, double h, int lev) { gl::arc_gk(F, cc, scv, h, Sm, ct, lev); },
                              ct);
        else
            gl::boundary_walk(H, F, bp, kind, nb, Sm, true,
                              [&](double cc, double scv, double h, int lev) { gl::arc_gk(F, cc, scv, h, Sm, nc, lev); },
                              nc);
        P.fsub[sub] = 1.0 - gl::sums_delta(S, Sm);
    }
    if (CENSUS) {
        census_add(ctr, 8, nodes);
        census_add(ctr, 6, (unsigned long long)ct.iters);
        census_add(ctr, 7, (unsigned long long)ct.limbs);
        census_add(ctr, 5, (unsigned long long)ct.arcs);
    }
    unconverged_add(ctr, CENSUS ? ct.unconv : nc.unconv, CENSUS);
}

// Level L of the self-checking arc rule: arc tau in [-h, h] split into 2^L
// equal pieces, one clustered Gauss-Kronrod 10/21 piece per thread; the 2^L
// lanes of an arc sum their Kronrod sums and differences by a butterfly (same
// order on every lane).  Accepted when the summed difference is within the
// tolerance (or at the last level); otherwise the arc enters level L + 1.
template <int L, bool CENSUS>
__global__ void __launch_bounds__(64) GL_WAVES(GL_WAVES_GK)
k_gk(Counters* __restrict__ ctr, Pipe P)
{
    constexpr int np = 1 << L;
    constexpr int lin = L_LVL0 + L;                                          // input list
    constexpr int lout = (L < gl::kArcMaxLevel) ? L_LVL0 + L + 1 : L_LVL0;  // output list
    if constexpr (GL_CHAIN_PRIO > 0) __builtin_amdgcn_s_setprio(GL_CHAIN_PRIO);
    const int lane = threadIdx.x;
    const int64_t scap = P.scap[lin];
    const ShardMap m = shard_map(ctr, lin, scap);
    const int64_t n = m.total << L;
    unsigned long long pieces = 0;
    for (int64_t p0 = (int64_t)blockIdx.x * 64; p0 < n; p0 += (int64_t)gridDim.x * 64) {
        const int64_t p = p0 + lane;
        const bool valid = p < n;
        const int q = (int)(p & (np - 1));
        const int64_t slot = shard_slot_run(m, valid ? (p >> L) : 0, p0 >> L, std::min(p0 + 63, n - 1) >> L, scap);
        ArcRef r{-1, -1};
        gl::Sums K{0.0, 0.0, 0.0};
        double err = 0.0;
        if (valid) r = P.lvl[L][slot];
        const int a = r.arc;
        if (r.hard >= 0) {
            const ArcRec A = P.arcs[a];
            const gl::Frame F = P.hfr[r.hard];
            const double half = A.h / np;
            err = gl::gk_piece<true>(F, A.cc, A.sc, -A.h + (2 * q + 1) * half, half, K);
            if (CENSUS) pieces += 1;
        }
#pragma unroll
        for (int d = 1; d < np; d <<= 1) {
            K.flat += __shfl_xor(K.flat, d);
            K.lin += __shfl_xor(K.lin, d);
            K.quad += __shfl_xor(K.quad, d);
            err += __shfl_xor(err, d);
        }
        const bool lead = q == 0 && r.hard >= 0;
        const bool accept = err <= gl::kArcTol || L == gl::kArcMaxLevel;
        if (lead && accept) P.arc_res[a] = K;
        if (L < gl::kArcMaxLevel) {
            // an arc re-enters the shard of its home slot in the arc list, so a
            // level-list shard never holds more arcs than an arc-list shard
            const bool want = lead && !accept;
            const int64_t acap = P.scap[L_ARC];
            const int hs = want ? (int)(a / acap) : -1;
            unsigned long long pending = __ballot(want);
            while (pending) {
                const int j = __shfl(hs, __builtin_ctzll(pending));
                const unsigned long long mj = __ballot(want && hs == j);
                const int64_t op = reserve(ctr, lout, j, (unsigned long long)__popcll(mj));
                if (want && hs == j)
                    P.lvl[L + 1 < kLevels ? L + 1 : L][(int64_t)j * P.scap[lout] + op + lanes_below(mj)] = r;
                pending &= ~mj;
            }
        }
    }
    if (CENSUS) census_add(ctr, 5, pieces);
}

// Arcs that failed levels 0 and 1 (rare): one thread per arc runs the rule
// from level 2 on in place (workgroups bid of nb of the rare-path launch).
template <bool CENSUS>
__device__ __forceinline__ void gk_tail_part(Counters* __restrict__ ctr, const Pipe& P, int64_t bid, int64_t nb)
{
    const int lane = threadIdx.x;
    const int64_t scap = P.scap[L_LVL0 + 2];
    const ShardMap m = shard_map(ctr, L_LVL0 + 2, scap);
    gl::Census ct;
    gl::NoCensus nc;
    for (int64_t g0 = bid * 64; g0 < m.total; g0 += nb * 64) {
        const int64_t g = g0 + lane;
        const int64_t slot = shard_slot_run(m, g < m.total ? g : 0, g0, std::min(g0 + 63, m.total - 1), scap);
        if (g >= m.total) continue;
        const ArcRef r = P.lvl[2][slot];
        const ArcRec A = P.arcs[r.arc];
        const gl::Frame F = P.hfr[r.hard];
        gl::Sums K{0.0, 0.0, 0.0};
        if (CENSUS) gl::arc_gk(F, A.cc, A.sc, A.h, K, ct, 2);
        else gl::arc_gk(F, A.cc, A.sc, A.h, K, nc, 2);
        P.arc_res[r.arc] = K;
    }
    if (CENSUS) census_add(ctr, 5, (unsigned long long)ct.arcs);
    unconverged_add(ctr, CENSUS ? ct.unconv : nc.unconv, CENSUS);
}

// The two rare paths in one launch, after the arc levels: the in-place list
// (nested trapezoid, samples integrated in place; independent of the arc
// lists) on the first nb_nest workgroups, the arcs that reached level 2 on
// the rest.
template <bool CENSUS>
__global__ void __launch_bounds__(64)
k_rare(const gl::SetConst* __restrict__ sc, Counters* __restrict__ ctr, Pipe P, int nb_nest)
{
    if ((int)blockIdx.x < nb_nest) nested_part<CENSUS>(sc, ctr, P, blockIdx.x, nb_nest);
    else gk_tail_part<CENSUS>(ctr, P, (int64_t)blockIdx.x - nb_nest, (int64_t)gridDim.x - nb_nest);
}

// Hard samples with ellipse arcs: limb sums plus the accepted arc sums in
// list order -> flux.
__global__ void __launch_bounds__(256)
k_combine(const gl::SetConst* __restrict__ sc, const Counters* __restrict__ ctr, Pipe P)
{
    const int lane = threadIdx.x & 63;
    const int64_t scap = P.scap[L_HARD];
    const ShardMap m = shard_map(ctr, L_HARD, scap);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); g0 < m.total; g0 += stride) {
        const int64_t g = g0 + lane;
        const int64_t slot = shard_slot_run(m, g < m.total ? g : 0, g0, std::min(g0 + 63, m.total - 1), scap);
        if (g >= m.total) continue;
        const HardRec& R = P.hrec[slot];
        const int na = R.n_arcs;
        if (na <= 0) continue;
        gl::Sums S = R.limb;
        const int ab = R.arc_begin;
        for (int k0 = 0; k0 < na; k0 += 4) {  // four arcs per memory round trip, added in order
            gl::Sums B[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) B[k] = k0 + k < na ? P.arc_res[ab + k0 + k] : gl::Sums{0.0, 0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (k0 + k < na) {
                    S.flat += B[k].flat;
                    S.lin += B[k].lin;
                    S.quad += B[k].quad;
                }
        }
        P.fsub[R.sub] = 1.0 - gl::sums_delta(sc[R.set & (kSphBit - 1)], S);  // same law for the sphere
    }
}

// The paper's integrator over a batch, a workgroup per chunk of 64 outputs
// (wavefront w takes every fourth in-window output from the w-th on): the
// centres of an output's sub-samples are found one per lane, then each
// sub-sample that reaches the disk is integrated by the whole wavefront (node
// i on lane i mod 64, Simpson weight 4 on odd nodes: odd lanes, 2 on even),
// the three sums reduced across the lanes; outputs are box-averaged in FP64
// (the sub-samples off the disk first, then the others in order).  node_cs:
// cos and sin of 2 pi i / n_nodes.
constexpr int kSnapWaves = 4;

__global__ void __launch_bounds__(64 * kSnapWaves)
k_snap(const double* __restrict__ times, int shared_grid, const gl::SetConst* __restrict__ sc,
       const int64_t* __restrict__ seg_begin, const int64_t* __restrict__ chunk_off, const Counters* __restrict__ ctr,
       const unsigned long long* __restrict__ masks, const int* __restrict__ chunk_set, int n_nodes,
       const float2* __restrict__ node_cs, double* __restrict__ out)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t total = (int64_t)ctr->total_chunks;
    const float wt = (lane & 1) ? 4.0f : 2.0f;
    for (int64_t c = blockIdx.x; c < total; c += gridDim.x) {
        unsigned long long M = (unsigned long long)uniform64((int64_t)masks[c]);
        if (!M) continue;
        for (int w = 0; w < wv; ++w) M &= M - 1ull;  // this wavefront's outputs: the wv-th, wv+4-th, ...
        if (!M) continue;
        const int64_t s = uniform64(chunk_set[c]);
        const gl::SetConst& S = sc[s];
        const gl::ChunkPos cp = gl::chunk_pos(shared_grid != 0, seg_begin[s], c - chunk_off[s]);
        const int nss = S.n_ss;
        const double inv_nss = 1.0 / (double)nss;
        const float A = (float)S.A, B = (float)S.B, C = (float)S.C;
        const double reach2 = (1.0 + S.k) * (1.0 + S.k);
        const float k0 = (float)S.c0, k1 = (float)S.c1 * (2.0f / 3.0f), k2 = (float)S.c2;
        const float scale = (float)(gl::kTwoPi / 3.0) / (float)n_nodes * (float)S.inv_phi;
        while (M) {
            const int o = __builtin_ctzll(M);  // the output (a lane of the chunk)
            for (int w = 0; w < kSnapWaves && M; ++w) M &= M - 1ull;
            const double t = times[cp.time0 + o];
            // lane j: sub-sample j's centre and whether its ellipse can reach the disk
            double x0 = 0.0, y0 = 0.0;
            bool on = false;
            if (lane < nss) {
                on = gl::centre_at(S, t + (((double)lane + 0.5) * inv_nss - 0.5) * S.t_exp, x0, y0);
                on = on && x0 * x0 + y0 * y0 < reach2;
            }
            const unsigned long long todo = __ballot(on);
            double sum = (double)(nss - __popcll(todo));  // sub-samples off the disk: flux 1
            // then, in order of j, the flux of every sub-sample that reaches the disk
            for (int j = 0; j < nss; ++j) {
                if (!((todo >> j) & 1ull)) continue;
                const float xc = (float)__shfl(x0, j), yc = (float)__shfl(y0, j);
                float sf = 0.0f, sl = 0.0f, sq = 0.0f;
                for (int i = lane; i < n_nodes; i += 64) {
                    const float2 q = node_cs[i];
                    float ff, fl, fq;
                    gl::snap_node(A, B, C, xc, yc, q.x, q.y, ff, fl, fq);
                    sf += ff;
                    sl += fl;
                    sq += fq;
                }
                sf *= wt;
                sl *= wt;
                sq *= wt;
                for (int d = 32; d >= 1; d >>= 1) {
                    sf += __shfl_xor(sf, d);
                    sl += __shfl_xor(sl, d);
                    sq += __shfl_xor(sq, d);
                }
                sum += (double)(1.0f - (k0 * sf + k1 * sl + k2 * sq) * scale);
            }
            if (lane == 0) out[cp.out0 + o] = sum * inv_nss;
        }
    }
}

// cos and sin of 2 pi i / n, i < n (from the double-precision functions)
__global__ void k_snap_nodes(int n, float2* __restrict__ cs)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double sn, c;
    sincos(gl::kTwoPi * (double)i / (double)n, &sn, &c);
    cs[i] = float2{(float)c, (float)sn};
}

// Surrogate batches: the network's rows in list order, as dense arrays
// (features in BF16, flux slot, residual scale) and their count.
__global__ void __launch_bounds__(64)
k_net_gather(const gl::SetConst* __restrict__ sc, Counters* __restrict__ ctr, Pipe P)
{
    const int lane = threadIdx.x;
    const int64_t scap = P.scap[L_NET];
    const ShardMap m = shard_map(ctr, L_NET, scap);
    if (blockIdx.x == 0 && lane == 0) ctr->net_total = (unsigned long long)m.total;
    for (int64_t g0 = (int64_t)blockIdx.x * 64; g0 < m.total; g0 += (int64_t)gridDim.x * 64) {
        const int64_t g = g0 + lane;
        const int64_t slot = shard_slot_run(m, g < m.total ? g : 0, g0, std::min(g0 + 63, m.total - 1), scap);
        if (g >= m.total) continue;
        const Entry e = P.net[slot];
        float fe[gl::kSurFeat];
        double scl = 0.0;
        int bin = -1;
        unsigned int w[gl::kSurFeat / 2];
        if (e.set >= 0 && gl::sur_encode(sc[e.set], e.x0, e.y0, fe, scl, bin)) {
            for (int i = 0; i < gl::kSurFeat / 2; ++i)
                w[i] = (unsigned)gl::f2bf_rne(fe[2 * i]) | ((unsigned)gl::f2bf_rne(fe[2 * i + 1]) << 16);
        } else {
            for (int i = 0; i < gl::kSurFeat / 2; ++i) w[i] = 0u;
            scl = 0.0;  // an emptied slot (its chunk went to the fused kernel) adds nothing
        }
        uint4* dst = reinterpret_cast<uint4*>(P.net_x + g * gl::kSurFeat);
        dst[0] = uint4{w[0], w[1], w[2], w[3]};
        dst[1] = uint4{w[4], w[5], w[6], w[7]};
        P.net_slot[g] = e.set >= 0 ? (int64_t)e.sub : -1;
        P.net_scale[g] = scl;
    }
}

// flux slot += scale * predicted scaled residual
__global__ void k_net_add(const Counters* __restrict__ ctr, Pipe P)
{
    const int64_t n = (int64_t)ctr->net_total;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t slot = P.net_slot[g];
        if (slot >= 0) P.fsub[slot] += P.net_scale[g] * (double)P.net_y[g];
    }
}

// Updates the demand record at the end of every pass (in device memory) and
// stores a copy into the host's pinned record, which the host reads when it
// plans the next batch (a stale read only delays a resize).  Only stores
// cross to host memory: a load from there is a bus round trip.  Run by one
// wavefront of the pass's last launch, once the lists are complete.
struct DemandArgs {
    Demand* rec;  // NULL: no record
    int first, last, passes;
    double slots;
};

__device__ void demand_update(Counters* __restrict__ ctr, const Pipe& P, const DemandArgs& a)
{
    Demand* __restrict__ rec = a.rec;
    const int first = a.first, last = a.last, passes = a.passes;
    const double slots = a.slots;
    const int lane = threadIdx.x & 63;
    // every list's shard count at once (lane j: shard j), then the reductions
    unsigned long long raw[kLists];
#pragma unroll
    for (int l = 0; l < kLists; ++l) raw[l] = lane < kShards ? (unsigned long long)list_count(ctr, l, lane) : 0ull;
    Demand& D = ctr->demand;
    const unsigned long long n_fb = ctr->n_fb;
    const unsigned long long norm_l = lane < kLists ? D.norm[lane] : 0ull;
    const unsigned long long cur0 = D.cur_sub;
    const double spo0 = D.sub_per_slot;
    auto wsum = [](unsigned long long v) {
        for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
        return v;
    };
    auto wmax = [](unsigned long long v) {
        for (int d = 32; d >= 1; d >>= 1) v = std::max(v, (unsigned long long)__shfl_xor(v, d));
        return v;
    };
    const unsigned long long sub_raw = wsum(raw[L_SUB]);
    const unsigned long long sub_kept = wsum(std::min(raw[L_SUB], (unsigned long long)P.scap[L_SUB]));
    const unsigned long long hard_raw = wsum(raw[L_HARD]);
    const unsigned long long hard_kept = wsum(std::min(raw[L_HARD], (unsigned long long)P.scap[L_HARD]));
    const double r1 = (double)sub_raw / (double)std::max(1ull, sub_kept);
    const double r2 = r1 * (double)hard_raw / (double)std::max(1ull, hard_kept);
    unsigned long long mine = 0ull;  // lane l: the estimate of list l
#pragma unroll
    for (int l = 0; l < kLists; ++l) {
        const double r = (l == L_SUB || l == L_WC || l == L_GRP) ? 1.0 : (l == L_TRAP || l == L_HARD || l == L_NET) ? r1 : r2;
        const unsigned long long est = (unsigned long long)((double)wmax(raw[l]) * r * passes) + 1ull;
        if (lane == l) mine = est;
    }
    if (lane < kLists) {
        const unsigned long long nl = std::max(norm_l, mine);
        D.norm[lane] = nl;
        rec->norm[lane] = nl;
    }
    if (lane == 63) {
        const unsigned long long cur = (first ? 0ull : cur0) + sub_raw;
        const double spo = last ? std::max(spo0, (double)cur / slots) : spo0;
        D.cur_sub = cur;
        D.sub_per_slot = spo;
        rec->cur_sub = cur;
        rec->sub_per_slot = spo;
        ctr->fused_batch += n_fb;
    }
}

// One wavefront per listed chunk: each in-window output averages its
// sub-sample fluxes in order (loaded 16 at a time, so that one memory round
// trip serves up to 16 of them, then summed one by one).
__global__ void __launch_bounds__(64)
k_average(const gl::SetConst* __restrict__ sc, const int64_t* __restrict__ seg_begin,
          const int64_t* __restrict__ chunk_off, Counters* __restrict__ ctr, Pipe P,
          const unsigned long long* __restrict__ masks, const int* __restrict__ chunk_set,
          const int* __restrict__ chunk_fb, DemandArgs dem, double* __restrict__ out)
{
    // the pass's lists are complete here: the first wavefront records their demand
    if (blockIdx.x == 0 && dem.rec) demand_update(ctr, P, dem);
    const int lane = threadIdx.x;
    const int64_t wcap = P.scap[L_WC];
    const ShardMap m = shard_map(ctr, L_WC, wcap);
    WorkChunk Wn{};  // loaded one iteration ahead
    if ((int64_t)blockIdx.x < m.total) Wn = P.wc[shard_slot_uniform(m, blockIdx.x, wcap)];
    for (int64_t w = blockIdx.x; w < m.total; w += gridDim.x) {
        const WorkChunk W = Wn;
        if (w + gridDim.x < m.total) Wn = P.wc[shard_slot_uniform(m, w + gridDim.x, wcap)];
        const int64_t base = uniform64(W.base), c = uniform64(W.c);
        if (base < 0) continue;
        if (__builtin_amdgcn_readfirstlane(chunk_fb[c])) continue;  // evaluated by the fused kernel
        const unsigned long long M = (unsigned long long)uniform64((int64_t)W.mask);
        const int nss = __builtin_amdgcn_readfirstlane(W.nss);
        const int64_t i0 = uniform64(W.i0);
        if ((M >> lane) & 1ull) {
            const int64_t o = lanes_below(M);
            const double* f = P.fsub + base + o * nss;
            double sum = 0.0;
            for (int j0 = 0; j0 < nss; j0 += 16) {
                double v[16];
#pragma unroll
                for (int j = 0; j < 16; ++j) v[j] = j0 + j < nss ? f[j0 + j] : 0.0;
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    if (j0 + j < nss) sum += v[j];
            }
            out[i0 + lane] = sum / (double)nss;
        }
    }
}


// Sub-samples of one chunk kept in LDS by the three-phase path (n_ss <= 16).
constexpr int kMaxSubLds = kChunk * 16;

template <bool CENSUS>
struct Counter {
    unsigned long long v[kCensus];
    int unconv = 0;  // unconverged arcs (counted in every launch)
    __device__ void add_sample(int cls, const gl::Census& ct)
    {
        if (!CENSUS) return;
        v[0] += 1;
        v[cls == gl::CLS_FULL ? 1 : (cls == gl::CLS_PARTIAL ? 2 : 3)] += 1;
        v[4] += ct.trap_nodes;
        v[5] += ct.arcs;
        v[6] += ct.iters;
        v[7] += ct.limbs;
        unconv += ct.unconv;
    }
};

// Instantaneous flux, easy part only: returns false (and leaves F) when the
// sample needs the intersection machinery.
// LOCK: a tidally-locked set, whose shadow is rebuilt for the sample's phase.
template <bool CENSUS, bool LOCK>
__device__ __attribute__((noinline)) bool flux_easy(const gl::SetConst& S0, double t, double& F,
                                          Counter<CENSUS>& cnt)
{
    gl::SetConst Ls;
    if (LOCK) gl::lock_at(S0, t, Ls);
    const gl::SetConst& S = LOCK ? Ls : S0;
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

template <bool CENSUS, bool LOCK>
__device__ __attribute__((noinline)) double flux_hard(const gl::SetConst& S0, double t, Counter<CENSUS>& cnt)
{
    gl::SetConst Ls;
    if (LOCK) gl::lock_at(S0, t, Ls);
    const gl::SetConst& S = LOCK ? Ls : S0;
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
    const double d = gl::occulted_hard<gl::NoCensus>(S, x0, y0, nullptr, nc);
    cnt.unconv += nc.unconv;
    return 1.0 - d;
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

// ELL: batches of general ellipsoids, whose tidally-locked sets rebuild
// their shadow per sub-sample (lock_at); the oblate instance carries none of it.
template <bool CENSUS, bool ELL>
__global__ void GL_COMPUTE_ATTR
k_compute(const double* __restrict__ times, int shared_grid, const gl::SetConst* __restrict__ sc,
          const int64_t* __restrict__ seg_begin, const int64_t* __restrict__ chunk_off,
          Counters* __restrict__ ctr, const unsigned long long* __restrict__ masks,
          const int* __restrict__ chunk_set, Pipe P, double* __restrict__ out)
{
    if (ctr->n_fb == 0ull) return;  // nothing queued (the usual case): no work head to touch
    const int64_t* __restrict__ fb_chunk = P.fb_chunk;
    __shared__ double lds_f[kMaxSubLds];   // sub-sample fluxes of the chunk
    __shared__ short lds_def[kMaxSubLds];  // deferred (hard) sub-samples
    __shared__ int lds_idx[kChunk];        // chunk lanes with work, compacted
    const int lane = threadIdx.x;
    const int64_t n_fb = (int64_t)ctr->n_fb;
    Counter<CENSUS> cnt;
    for (int i = 0; i < kCensus; ++i) cnt.v[i] = 0ull;
    for (;;) {
        unsigned long long k = 0;
        if (lane == 0) k = atomicAdd(&ctr->fb_head, 1ull);
        k = (unsigned long long)uniform64((int64_t)k);  // lane 0's value
        if ((int64_t)k >= n_fb) break;
        {
            const int64_t c = uniform64(fb_chunk[k]);
            const unsigned long long M = (unsigned long long)uniform64((int64_t)masks[c]);
            const int64_t s = uniform64(chunk_set[c]);
            const gl::SetConst S = sc[s];
            const int64_t lc = c - chunk_off[s];
            const gl::ChunkPos cp = gl::chunk_pos(shared_grid != 0, seg_begin[s], lc);
            const int64_t i0 = cp.out0, tb = cp.time0;
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
                        hard = !((ELL && S.locked) ? flux_easy<CENSUS, ELL>(S, t, F, cnt)
                                                   : flux_easy<CENSUS, false>(S, t, F, cnt));
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
                        lds_f[f] = (ELL && S.locked) ? flux_hard<CENSUS, ELL>(S, t, cnt)
                                                     : flux_hard<CENSUS, false>(S, t, cnt);
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
                        if (ELL && S.locked) {
                            if (!flux_easy<CENSUS, ELL>(S, t, F, cnt)) F = flux_hard<CENSUS, ELL>(S, t, cnt);
                        } else if (!flux_easy<CENSUS, false>(S, t, F, cnt)) {
                            F = flux_hard<CENSUS, false>(S, t, cnt);
                        }
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
        for (int i = 0; i < 8; ++i) {
            unsigned long long v = cnt.v[i];
            for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
            if (lane == 0) atomicAdd(&ctr->census[i][blockIdx.x % kShards].v, v);
        }
    }
    unconverged_add(ctr, cnt.unconv, CENSUS);
}

}  // namespace

// ---------------------------------------------------------------- context
// Timing events of one pass: the caller's stream marks the start and the
// ends of set-up, window, classification, hard samples, arc levels, rare
// paths and averages (the pass's last stage: it waits for the second
// stream); the second stream marks its start (its wait on the
// classification met) and the ends of the trapezoid and fused stages.  Each
// stage is timed between two of them (kStageEv), on the stream it runs on.
enum {
    E_START, E_SETUP, E_WINDOW, E_CLASSIFY, E_SIDE, E_TRAP, E_FUSED, E_HARD, E_ARCS, E_RARE, E_AVERAGE, kEvPerPass
};
constexpr int kStageEv[GL_NSTAGES][2] = {
    {E_START, E_SETUP}, {E_SETUP, E_WINDOW}, {E_WINDOW, E_CLASSIFY}, {E_SIDE, E_TRAP}, {E_CLASSIFY, E_HARD},
    {E_HARD, E_ARCS},   {E_ARCS, E_RARE},    {E_RARE, E_AVERAGE},    {E_TRAP, E_FUSED}};

// Passes: a batch whose in-window sub-samples exceed what one pass should
// hold runs as up to kMaxPasses passes of the whole pipeline over equal
// ranges of its parameter sets.  Results do not depend on the split (every
// sub-sample and output is computed by itself), only the list sizes do.
constexpr int kMaxPasses = 8;
constexpr int64_t kPassSub = (int64_t)1 << 26;  // in-window sub-samples one pass aims at

struct gl_ctx {
    int device = 0;
    int n_cu = 256;
    int waves_per_cu = 16;  // persistent waves per CU of the hard-sample kernel
    int waves_trap = GL_TRAP_WAVES_PER_CU;          // of the trapezoid kernel
    int waves_classify = GL_CLASSIFY_WAVES_PER_CU;  // of the classification
    int waves_gk = GL_GK_WAVES_PER_CU;              // of the arc-rule levels
    bool use_graph = true;
    char err[256] = {};  // last host-side error (fixed buffer: error paths allocate nothing)
    // workspace
    gl::SetConst* sc = nullptr;
    gl::SetConst* sc_sph = nullptr;  // equal-area spheres (surrogate batches)
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
        int waves, waves_trap, waves_classify, waves_gk;
        void* ws;
        int passes;
        int shape;
        const double* data;
        const double* sigma;
        double* chi2;
        double* loglike;
    } key{};
    bool have_graph = false;
    // work lists of the exact path (capacities in entries; 0 = default)
    Pipe pipe{};
    bool have_pipe = false;
    int* chunk_fb = nullptr;  // per chunk: 1 = evaluated by the fused kernel
    int64_t pipe_chunks = 0;  // length of the per-chunk arrays
    int64_t want_sub = 0, want_hard = 0, want_arc = 0;
    bool want_net = false;  // lists and buffers of surrogate batches
    // the paper's integrator: cos / sin of its nodes (snap_n of them, room for snap_cap)
    float2* snap_cs = nullptr;
    int snap_cap = 0, snap_n = 0;
    // demand-driven sizing: the record k_demand writes (pinned host memory and
    // its device address), and the per-shard capacities it asked for
    Demand* rec = nullptr;
    Demand* rec_dev = nullptr;
    int64_t auto_scap[kLists] = {};
    int64_t mem_total = 0;
    int passes = 1;  // passes of the current batch (plan_passes)
    // timing of the next t_left batches: launched directly (the HIP runtime
    // a torch process loads rejects event records captured into a graph),
    // one set of stage events per pass, read right after the batch
    int t_left = 0, t_pass = 0, t_batches = 0;
    hipEvent_t* ev = nullptr;  // kEvPerPass x kMaxPasses
    double t_stage[GL_NSTAGES] = {};
    double t_comp = 0.0, t_pipe = 0.0;
    // a second stream for the trapezoid stage, which depends on the
    // classification only and runs beside the hard-sample chain
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

namespace {

gl_status fail(gl_ctx* ctx, gl_status st, const char* what, hipError_t e = hipSuccess)
{
    if (ctx) {
        if (e != hipSuccess) std::snprintf(ctx->err, sizeof(ctx->err), "%s: %s", what, hipGetErrorString(e));
        else std::snprintf(ctx->err, sizeof(ctx->err), "%s", what);
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

void free_pipe(gl_ctx* ctx)
{
    Pipe& P = ctx->pipe;
    void* b[] = {P.fsub, P.wc, P.grp, P.fb_chunk, P.trap, P.hard, P.nest, P.hrec, P.hfr, P.arcs,
                 P.arc_res, ctx->chunk_fb, P.net, P.net_x, P.net_slot, P.net_scale, P.net_y};
    for (void* q : b) (void)hipFree(q);
    ctx->chunk_fb = nullptr;
    for (int L = 0; L < kLevels; ++L) (void)hipFree(P.lvl[L]);
    P = Pipe{};
    ctx->have_pipe = false;
    ctx->pipe_chunks = 0;
}

void free_ws(gl_ctx* ctx)
{
    free_pipe(ctx);
    (void)hipFree(ctx->sc);
    (void)hipFree(ctx->sc_sph);
    (void)hipFree(ctx->seg_begin);
    (void)hipFree(ctx->seg_len);
    (void)hipFree(ctx->chunk_off);
    (void)hipFree(ctx->masks);
    (void)hipFree(ctx->chunk_set);
    ctx->sc = ctx->sc_sph = nullptr;
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
        (void)hipFree(ctx->sc_sph);
        (void)hipFree(ctx->seg_begin);
        (void)hipFree(ctx->seg_len);
        (void)hipFree(ctx->chunk_off);
        ctx->sc = ctx->sc_sph = nullptr;
        ctx->seg_begin = ctx->seg_len = ctx->chunk_off = nullptr;
        ctx->cap_sets = 0;
        const int64_t cap = std::max<int64_t>(n_sets, 1024);
        if (hipMalloc(&ctx->sc, sizeof(gl::SetConst) * cap) != hipSuccess ||
            hipMalloc(&ctx->sc_sph, sizeof(gl::SetConst) * cap) != hipSuccess ||
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

// Default work-list capacities: 16 Mi sub-samples (a chunk holds at most
// 64 outputs x 64 sub-samples), a quarter of that of hard samples, two arcs
// per hard sample, each split evenly over the shards.  About 1.5 GB of device
// memory at the defaults, less for small batches.
constexpr int64_t kDefSub = (int64_t)1 << 24;

gl_status ensure_pipe(gl_ctx* ctx, int64_t n_chunks)
{
    const int64_t per_chunk = (int64_t)kChunk * 64;
    int64_t cs = ctx->want_sub > 0 ? ctx->want_sub : std::min<int64_t>(kDefSub, n_chunks * per_chunk);
    cs = std::max<int64_t>(std::min<int64_t>(cs, kSubMask - kShards), kShards);
    int64_t ch = ctx->want_hard > 0 ? ctx->want_hard : std::max<int64_t>(cs / 4, kShards);
    int64_t ca = ctx->want_arc > 0 ? ctx->want_arc : 2 * ch;
    ch = std::max<int64_t>(std::min<int64_t>(ch, INT32_MAX / 2), kShards);
    ca = std::max<int64_t>(std::min<int64_t>(ca, INT32_MAX / 2), kShards);
    const int64_t nc = std::max<int64_t>(ctx->cap_chunks, n_chunks);
    int64_t sc_[kLists];
    sc_[L_SUB] = (cs + kShards - 1) / kShards;
    sc_[L_TRAP] = sc_[L_SUB];
    sc_[L_WC] = std::max<int64_t>(64, 2 * ((nc + kShards - 1) / kShards));
    sc_[L_HARD] = (ch + kShards - 1) / kShards;
    sc_[L_NEST] = sc_[L_HARD];
    sc_[L_ARC] = (ca + kShards - 1) / kShards;
    // lists without an explicit capacity grow to the demand of earlier batches
    const bool auto_sz = ctx->want_sub == 0 && ctx->want_hard == 0 && ctx->want_arc == 0;
    if (auto_sz) {
        const int64_t sub_max = (kSubMask - kShards) / kShards, ent_max = (INT32_MAX / 2) / kShards;
        sc_[L_SUB] = std::min(sub_max, std::max(sc_[L_SUB], ctx->auto_scap[L_SUB]));
        sc_[L_TRAP] = std::min(sub_max, std::max(sc_[L_SUB], ctx->auto_scap[L_TRAP]));
        sc_[L_HARD] = std::min(ent_max, std::max(sc_[L_HARD], ctx->auto_scap[L_HARD]));
        sc_[L_NEST] = std::min(ent_max, std::max(sc_[L_HARD], ctx->auto_scap[L_NEST]));
        int64_t arc = std::max(sc_[L_ARC], ctx->auto_scap[L_ARC]);
        for (int L = 0; L < kLevels; ++L) arc = std::max(arc, ctx->auto_scap[L_LVL0 + L]);
        sc_[L_ARC] = std::min(ent_max, arc);
    }
    sc_[L_GRP] = std::max<int64_t>(64, sc_[L_SUB] / kChunk + sc_[L_WC]);
    for (int L = 0; L < kLevels; ++L) sc_[L_LVL0 + L] = sc_[L_ARC];
    sc_[L_NET] = ctx->want_net ? std::max(sc_[L_SUB], auto_sz ? ctx->auto_scap[L_NET] : 0) : 0;
    Pipe& P = ctx->pipe;
    bool same = ctx->have_pipe && ctx->pipe_chunks >= n_chunks;
    for (int l = 0; l < kLists && same; ++l) same = P.scap[l] == sc_[l];
    if (same) return GL_OK;
    drop_graph(ctx);
    GL_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    free_pipe(ctx);
    const int64_t K = kShards;
    bool ok = hipMalloc(&P.fsub, sizeof(double) * K * sc_[L_SUB]) == hipSuccess &&
              hipMalloc(&P.wc, sizeof(WorkChunk) * K * sc_[L_WC]) == hipSuccess &&
              hipMalloc(&P.grp, sizeof(Group) * K * sc_[L_GRP]) == hipSuccess &&
              hipMalloc(&P.fb_chunk, sizeof(int64_t) * nc) == hipSuccess &&
              hipMalloc(&ctx->chunk_fb, sizeof(int) * nc) == hipSuccess &&
              hipMalloc(&P.trap, sizeof(Entry) * K * sc_[L_TRAP]) == hipSuccess &&
              hipMalloc(&P.hard, sizeof(Entry) * K * sc_[L_HARD]) == hipSuccess &&
              hipMalloc(&P.nest, sizeof(Entry) * K * sc_[L_NEST]) == hipSuccess &&
              hipMalloc(&P.hrec, sizeof(HardRec) * K * sc_[L_HARD]) == hipSuccess &&
              hipMalloc(&P.hfr, sizeof(gl::Frame) * K * sc_[L_HARD]) == hipSuccess &&
              hipMalloc(&P.arcs, sizeof(ArcRec) * K * sc_[L_ARC]) == hipSuccess &&
              hipMalloc(&P.arc_res, sizeof(gl::Sums) * K * sc_[L_ARC]) == hipSuccess;
    for (int L = 0; L < kLevels && ok; ++L)
        ok = hipMalloc(&P.lvl[L], sizeof(ArcRef) * K * sc_[L_ARC]) == hipSuccess;
    if (ok && sc_[L_NET] > 0) {
        const int64_t rows = K * sc_[L_NET];
        ok = hipMalloc(&P.net, sizeof(Entry) * rows) == hipSuccess &&
             hipMalloc(&P.net_x, sizeof(uint16_t) * gl::kSurFeat * rows) == hipSuccess &&
             hipMalloc(&P.net_slot, sizeof(int64_t) * rows) == hipSuccess &&
             hipMalloc(&P.net_scale, sizeof(double) * rows) == hipSuccess &&
             hipMalloc(&P.net_y, sizeof(float) * rows) == hipSuccess;
    }
    if (!ok) {
        free_pipe(ctx);
        return fail(ctx, GL_ERR_NOMEM, "work-list allocation");
    }
    for (int l = 0; l < kLists; ++l) P.scap[l] = sc_[l];
    ctx->pipe_chunks = nc;
    ctx->have_pipe = true;
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
    int64_t ld = 0;          // row stride of params (the whole batch's n_sets)
    int first = 1, last = 1;  // first / last pass of the batch
    int64_t slots = 0;       // output chunk slots of the whole batch, x 64
    // surrogate batches (net != NULL): the gate and the network
    gl_mlp* net = nullptr;
    const float* gate_table = nullptr;
    const uint8_t* gate_zero = nullptr;
    double gate_k = 0.0;
    int shape = 0;  // 0: oblate parameter block, 1: general ellipsoids, 2: MCMC walkers
    // MCMC glue (gl_loglike_batch): the per-walker likelihood of out against
    // data / sigma after the light curves
    const double* data = nullptr;
    const double* sigma = nullptr;
    double* chi2 = nullptr;
    double* loglike = nullptr;
};

// ctx may be NULL (no message is kept)
gl_status check_batch(gl_ctx* ctx, Batch& b)
{
    if (ctx) ctx->err[0] = 0;
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
        if ((cps + kWinGrid - 1) / kWinGrid * b.n_sets > (int64_t)INT32_MAX)
            return fail(ctx, GL_ERR_SIZE, "batch too large for one window launch");
    }
    if (b.max_chunks > ((int64_t)1 << 40)) return fail(ctx, GL_ERR_SIZE, "batch too large");
    b.ld = b.n_sets;
    b.slots = b.max_chunks * kChunk;
    return GL_OK;
}

gl_status check_args(gl_ctx* ctx, Batch& b)
{
    if (!ctx) return GL_ERR_NULL;
    return check_batch(ctx, b);
}

// Window test over all chunks (fills the out-of-window outputs, chunk masks).
void launch_window(gl_ctx* ctx, const Batch& b, hipStream_t st, int lists, const Pipe& P)
{
    if (!b.offsets) {
        const int64_t cps = (b.n_times + kChunk - 1) / kChunk;
        const int64_t bx = (cps + kWinGrid - 1) / kWinGrid;
        hipLaunchKernelGGL(k_window_grid, dim3((unsigned)(bx * b.n_sets)), dim3(64), 0, st, b.times,
                           b.n_times, cps, ctx->sc, ctx->ctr, ctx->masks, ctx->chunk_set, b.out, lists,
                           P, ctx->chunk_fb);
    } else {
        const int64_t groups = (b.max_chunks + kWinChunks - 1) / kWinChunks;
        hipLaunchKernelGGL(k_window, dim3((unsigned)((groups + 3) / 4)), dim3(256), 0, st, b.times,
                           b.n_sets, ctx->sc, ctx->seg_begin, ctx->seg_len, ctx->chunk_off,
                           ctx->ctr, ctx->masks, ctx->chunk_set, b.out, lists, P, ctx->chunk_fb);
    }
}

template <bool CENSUS>
void launch_arcs(gl_ctx* ctx, hipStream_t st, unsigned grid, const Pipe& P)
{
    hipLaunchKernelGGL((k_gk<0, CENSUS>), dim3(grid), dim3(64), 0, st, ctx->ctr, P);
    hipLaunchKernelGGL((k_gk<1, CENSUS>), dim3(grid), dim3(64), 0, st, ctx->ctr, P);
}

// few arcs reach the deeper levels and few samples take the in-place list:
// one launch finishes both, per lane
template <bool CENSUS>
void launch_rare(gl_ctx* ctx, hipStream_t st, unsigned arc_grid, const Pipe& P)
{
    const int nb_nest = (int)(ctx->n_cu * 4);
    const unsigned grid = (unsigned)nb_nest + std::max(1u, arc_grid / 16);
    hipLaunchKernelGGL((k_rare<CENSUS>), dim3(grid), dim3(64), 0, st, ctx->sc, ctx->ctr, P, nb_nest);
}

// A timing event (timed batches are launched directly, never captured); on
// failure the context's error names the pass and the event.
gl_status record_event(gl_ctx* ctx, hipEvent_t ev, hipStream_t s, int e)
{
    const hipError_t r = hipEventRecord(ev, s);
    if (r == hipSuccess) return GL_OK;
    char what[64];
    std::snprintf(what, sizeof(what), "timing event %d of pass %d", e, ctx->t_pass - 1);
    return fail(ctx, GL_ERR_DEVICE, what, r);
}

template <bool CENSUS>
gl_status enqueue_t(gl_ctx* ctx, const Batch& b)
{
    const int shared = b.offsets ? 0 : 1;
    hipStream_t st = b.stream;
    hipEvent_t* ev = nullptr;
    if (!CENSUS && ctx->t_left > 0 && ctx->ev && ctx->t_pass < kMaxPasses) {
        ev = ctx->ev + kEvPerPass * ctx->t_pass;
        ctx->t_pass++;
    }
#define GL_MARK(i, s)                                                     \
    do {                                                                  \
        if (ev) {                                                         \
            const gl_status r_ = record_event(ctx, ev[i], s, i);          \
            if (r_ != GL_OK) return r_;                                   \
        }                                                                 \
    } while (0)
    GL_MARK(E_START, st);
    Pipe P = ctx->pipe;
    const bool sur = b.net != nullptr;
    if (sur) {
        P.sph = ctx->sc_sph;
        P.gate_table = b.gate_table;
        P.gate_zero = b.gate_zero;
        P.gate_k = b.gate_k;
    }
    // with a likelihood on a shared grid, an extra workgroup of the first
    // pass forms its normalisation
    const bool norm = b.data && shared && b.first;
    const unsigned prep_blocks = (unsigned)((b.n_sets + 255) / 256) + (norm ? 1u : 0u);
    const int64_t cps_shared = shared ? (b.n_times + kChunk - 1) / kChunk : 0;
    auto prep = b.shape == 1 ? k_prep<1> : b.shape == 2 ? k_prep<2> : k_prep<0>;
    hipLaunchKernelGGL(prep, dim3(prep_blocks), dim3(256), 0, st, b.params, b.ld, b.n_sets,
                       b.offsets, b.n_times, b.n_ss, b.t_exp, ctx->sc, ctx->seg_begin,
                       ctx->seg_len, ctx->chunk_off, ctx->ctr, cps_shared, b.first, b.last,
                       sur ? ctx->sc_sph : nullptr, b.sigma, b.n_times, norm ? &ctx->ctr->ll_norm : nullptr);
    if (!shared)
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, st, ctx->chunk_off, b.n_sets,
                           b.max_chunks, ctx->ctr);
    GL_MARK(E_SETUP, st);
    const int64_t n_cu = ctx->n_cu;
    launch_window(ctx, b, st, 1, P);
    GL_MARK(E_WINDOW, st);
    const unsigned waves = (unsigned)std::max<int64_t>(4, n_cu * ctx->waves_per_cu);
    if (sur)
        hipLaunchKernelGGL((k_classify<false, true>), dim3((unsigned)(n_cu * ctx->waves_classify)), dim3(64), 0, st, b.times,
                           shared, ctx->sc, ctx->seg_begin, ctx->chunk_off, ctx->ctr, P, ctx->masks, ctx->chunk_set,
                           ctx->chunk_fb);
    else
        hipLaunchKernelGGL((k_classify<CENSUS, false>), dim3((unsigned)(n_cu * ctx->waves_classify)), dim3(64), 0, st,
                           b.times, shared, ctx->sc, ctx->seg_begin, ctx->chunk_off, ctx->ctr, P, ctx->masks,
                           ctx->chunk_set, ctx->chunk_fb);
    const unsigned twaves = (unsigned)std::max<int64_t>(4, n_cu * ctx->waves_trap);
    // whole ellipses (trapezoid) need nothing from the hard-sample chain and
    // write other sub-samples, so the two run side by side.  The hard chain
    // (hard samples, arc levels, rare paths, combine), the longer branch,
    // stays on the caller's stream and is enqueued first: a graph of the
    // batch keeps its first branch on the launching queue, so the chain
    // starts right after the classification and the averages follow it on
    // the same queue.  The trapezoid goes to the second stream after its
    // wait on the classification; its end is long past when the averages
    // wait for it.  Cross-queue waits cost ~10 us each on the critical path
    // in the opposite arrangement.
    const bool fork = ctx->side != nullptr;
    hipStream_t ts = fork ? ctx->side : st;
    if (fork) {
        GL_HIP(hipEventRecord(ctx->ev_fork, st), "hipEventRecord (fork)");
        GL_HIP(hipStreamWaitEvent(ts, ctx->ev_fork, 0), "hipStreamWaitEvent (fork)");
    }
    GL_MARK(E_CLASSIFY, st);  // after the fork record: the hard stage starts with its kernel
    hipLaunchKernelGGL(k_hard<CENSUS>, dim3(waves), dim3(64), 0, st, ctx->sc, ctx->ctr, P);
    GL_MARK(E_HARD, st);
    const unsigned arc_grid = ctx->waves_gk > 0 ? (unsigned)(n_cu * ctx->waves_gk) : waves;
    launch_arcs<CENSUS>(ctx, st, arc_grid, P);
    GL_MARK(E_ARCS, st);
    launch_rare<CENSUS>(ctx, st, arc_grid, P);
    GL_MARK(E_RARE, st);
    hipLaunchKernelGGL(k_combine, dim3((unsigned)(n_cu * 8)), dim3(256), 0, st, ctx->sc, ctx->ctr, P);
    // the network's rows (surrogate batches) need only the classification:
    // their features are gathered and the network evaluated on the second
    // stream, on the matrix cores beside the hard chain's FP64 work; the
    // residuals are added after the join
    auto net_rows = [&](hipStream_t s) {
        hipLaunchKernelGGL(k_net_gather, dim3((unsigned)(n_cu * 8)), dim3(64), 0, s, ctx->sc, ctx->ctr, P);
        gl_net::infer(b.net, P.net_x, (int64_t)kShards * P.scap[L_NET], &ctx->ctr->net_total, P.net_y, s);
    };
    const bool net_side = sur && GL_SUR_NET_SIDE >= 1;
    if (net_side) net_rows(ts);
    // the network's launch then makes the second stream the longer branch:
    // the trapezoid and the fused kernel follow the hard chain instead
    hipStream_t xs = (net_side && GL_SUR_NET_SIDE == 2) ? st : ts;
    GL_MARK(E_SIDE, xs);
    hipLaunchKernelGGL(k_trap<CENSUS>, dim3((twaves + kTrapWaves - 1) / kTrapWaves), dim3(kTrapThreads), 0, xs,
                       ctx->sc, ctx->ctr, P);
    GL_MARK(E_TRAP, xs);
    // the fused kernel takes the chunks the lists could not hold (few: a
    // quarter wave per CU; it returns at once when none is queued), and every
    // chunk of a tidally-locked set (general ellipsoids: a full grid at its
    // occupancy of two waves per SIMD).  Only the window and classification
    // queue chunks for it, and the averages skip those chunks, so it follows
    // the trapezoid, off the hard chain's path (on the caller's stream after
    // the chain in a surrogate batch)
    const unsigned fused_grid = b.shape == 1 ? (unsigned)(n_cu * 8) : (unsigned)std::max<int64_t>(1, n_cu / 4);
    auto fused = b.shape == 1 ? k_compute<CENSUS, true> : k_compute<CENSUS, false>;
    hipLaunchKernelGGL(fused, dim3(fused_grid), dim3(64), 0, xs, b.times, shared,
                       ctx->sc, ctx->seg_begin, ctx->chunk_off, ctx->ctr, ctx->masks, ctx->chunk_set,
                       P, b.out);
    GL_MARK(E_FUSED, xs);
    if (fork) {
        GL_HIP(hipEventRecord(ctx->ev_join, ts), "hipEventRecord (join)");
        GL_HIP(hipStreamWaitEvent(st, ctx->ev_join, 0), "hipStreamWaitEvent (join)");
    }
    if (sur) {
        // the network's residuals on the accepted sub-samples' sphere fluxes
        if (!net_side) net_rows(st);
        hipLaunchKernelGGL(k_net_add, dim3((unsigned)(n_cu * 8)), dim3(256), 0, st, ctx->ctr, P);
    }
    const DemandArgs dem{ctx->rec_dev, b.first, b.last, ctx->passes, (double)b.slots};
    hipLaunchKernelGGL(k_average, dim3((unsigned)(n_cu * 32)), dim3(64), 0, st, ctx->sc,
                       ctx->seg_begin, ctx->chunk_off, ctx->ctr, P, ctx->masks, ctx->chunk_set,
                       ctx->chunk_fb, dem, b.out);
    GL_MARK(E_AVERAGE, st);
#undef GL_MARK
    GL_HIP(hipGetLastError(), "kernel launch");
    return GL_OK;
}

// Bytes of the work lists at per-shard capacities c (entries).
int64_t pipe_bytes(const int64_t* c)
{
    const int64_t K = kShards;
    return K * (c[L_SUB] * 8 + c[L_TRAP] * (int64_t)sizeof(Entry) + c[L_GRP] * (int64_t)sizeof(Group) +
                c[L_WC] * (int64_t)sizeof(WorkChunk) +
                c[L_HARD] * (int64_t)(sizeof(Entry) + sizeof(HardRec) + sizeof(gl::Frame)) +
                c[L_NEST] * (int64_t)sizeof(Entry) +
                c[L_ARC] * (int64_t)(sizeof(ArcRec) + sizeof(gl::Sums) + kLevels * sizeof(ArcRef)));
}

// Number of passes for the batch, and the per-shard list capacities it asks
// for (ctx->auto_scap, only ever raised), from the demand record.  One pass
// with explicit capacities (gl_ctx_set_capacity) or no record yet.
int plan_passes(gl_ctx* ctx, const Batch& b)
{
    if (!ctx->rec || ctx->want_sub || ctx->want_hard || ctx->want_arc) return 1;
    const volatile Demand* r = ctx->rec;
    // expected in-window sub-samples of this batch at the densest ratio seen
    const int64_t bs = (int64_t)(r->sub_per_slot * (double)b.slots);
    if (bs == 0) return 1;
    int T = (int)std::min<int64_t>(kMaxPasses, (bs + bs / 8 + kPassSub - 1) / kPassSub);
    T = (int)std::max<int64_t>(1, std::min<int64_t>(T, b.n_sets));
    // the lists of one pass may take up to a third of the device memory
    const int64_t budget = ctx->mem_total / 3;
    int64_t need[kLists];
    for (;;) {
        for (int l = 0; l < kLists; ++l) {
            const int64_t n = (int64_t)r->norm[l];
            need[l] = std::max(ctx->auto_scap[l], n / T + n / (4 * T) + 64);
        }
        need[L_GRP] = need[L_SUB] / kChunk + need[L_WC];
        if (pipe_bytes(need) <= budget || T >= std::min<int64_t>(kMaxPasses, b.n_sets)) break;
        ++T;
    }
    for (int l = 0; l < kLists; ++l) ctx->auto_scap[l] = need[l];
    return T;
}

// Plans a batch's passes and sizes the workspace for them (may wait for the
// device and reallocate; never called inside a stream capture).
gl_status prepare_batch(gl_ctx* ctx, const Batch& b)
{
    ctx->passes = plan_passes(ctx, b);
    gl_status st = ensure_ws(ctx, b.n_sets, b.max_chunks);
    if (st != GL_OK) return st;
    return ensure_pipe(ctx, b.max_chunks);
}

// Enqueues every pass of a prepared batch (inside a stream capture when
// called from one).
gl_status run_batch(gl_ctx* ctx, const Batch& b, bool census)
{
    gl_status st = GL_OK;
    const int T = ctx->passes;
    ctx->t_pass = 0;
    for (int p = 0; p < T; ++p) {
        const int64_t a = b.n_sets * p / T, e = b.n_sets * (p + 1) / T;
        Batch q = b;
        q.params = b.params + a;
        q.n_sets = e - a;
        q.n_ss = b.n_ss ? b.n_ss + a : nullptr;
        q.t_exp = b.t_exp ? b.t_exp + a : nullptr;
        if (b.offsets) {
            q.offsets = b.offsets + a;
            q.max_chunks = b.n_times / kChunk + q.n_sets;
        } else {
            q.out = b.out + a * b.n_times;
            q.max_chunks = (b.n_times + kChunk - 1) / kChunk * q.n_sets;
        }
        q.first = p == 0;
        q.last = p == T - 1;
        st = census ? enqueue_t<true>(ctx, q) : enqueue_t<false>(ctx, q);
        if (st != GL_OK) return st;
    }
    return GL_OK;
}

gl_status enqueue(gl_ctx* ctx, const Batch& b, bool census = false)
{
    gl_status st = run_batch(ctx, b, census);
    if (st != GL_OK) return st;
    if (b.data) {
        // a shared grid's normalisation came from the first pass's k_prep
        const double* norm = b.offsets ? nullptr : &ctx->ctr->ll_norm;
        gl_mcmc::launch_loglike(b.out, b.n_sets, b.offsets, b.n_times, b.data, b.sigma, norm, b.chi2, b.loglike,
                                b.stream);
    }
    GL_HIP(hipGetLastError(), "kernel launch");
    return GL_OK;
}

// After a timed batch (t_pass passes recorded): waits for its stream and adds
// its stage times (kStageEv), the compute time (end of set-up to end of the
// averages, which wait for the second stream) and the pipeline time (start
// to end of the averages).
gl_status finish_timed(gl_ctx* ctx, hipStream_t s)
{
    if (ctx->t_left <= 0 || ctx->t_pass <= 0) return GL_OK;
    GL_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    for (int p = 0; p < ctx->t_pass; ++p) {
        hipEvent_t* ev = ctx->ev + kEvPerPass * p;
        for (int k = 0; k < GL_NSTAGES; ++k) {
            float ms = 0.0f;
            GL_HIP(hipEventElapsedTime(&ms, ev[kStageEv[k][0]], ev[kStageEv[k][1]]), "hipEventElapsedTime");
            ctx->t_stage[k] += ms;
        }
        float ms = 0.0f;
        GL_HIP(hipEventElapsedTime(&ms, ev[E_SETUP], ev[E_AVERAGE]), "hipEventElapsedTime");
        ctx->t_comp += ms;
        GL_HIP(hipEventElapsedTime(&ms, ev[E_START], ev[E_AVERAGE]), "hipEventElapsedTime");
        ctx->t_pipe += ms;
    }
    ctx->t_batches++;
    ctx->t_left--;
    ctx->t_pass = 0;
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
    hipDeviceProp_t prop{};
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        if (prop.multiProcessorCount > 0) ctx->n_cu = prop.multiProcessorCount;
        ctx->mem_total = (int64_t)prop.totalGlobalMem;
    }
    if (ctx->mem_total <= 0) ctx->mem_total = (int64_t)1 << 34;
    if (hipMalloc(&ctx->ctr, sizeof(Counters)) != hipSuccess) {
        delete ctx;
        return GL_ERR_NOMEM;
    }
    // the demand record lives in pinned host memory that k_demand writes
    if (hipHostMalloc((void**)&ctx->rec, sizeof(Demand), hipHostMallocMapped) != hipSuccess ||
        hipHostGetDevicePointer((void**)&ctx->rec_dev, ctx->rec, 0) != hipSuccess) {
        if (ctx->rec) (void)hipHostFree(ctx->rec);
        (void)hipFree(ctx->ctr);
        delete ctx;
        return GL_ERR_NOMEM;
    }
    std::memset(ctx->rec, 0, sizeof(Demand));
    if (hipMemset(ctx->ctr, 0, sizeof(Counters)) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(ctx->ctr);
        delete ctx;
        return GL_ERR_DEVICE;
    }
    // default priority, non-blocking (no implicit order with the legacy
    // default stream); without it every stage runs on the caller's stream
    if (hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming) != hipSuccess) {
        if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
        if (ctx->side) (void)hipStreamDestroy(ctx->side);
        ctx->side = nullptr;
        ctx->ev_fork = ctx->ev_join = nullptr;
    }
    *out = ctx;
    return GL_OK;
}

void free_timing(gl_ctx* ctx)
{
    if (ctx->ev)
        for (int i = 0; i < kEvPerPass * kMaxPasses; ++i) (void)hipEventDestroy(ctx->ev[i]);
    delete[] ctx->ev;
    ctx->ev = nullptr;
    ctx->t_left = ctx->t_pass = ctx->t_batches = 0;
    for (int k = 0; k < GL_NSTAGES; ++k) ctx->t_stage[k] = 0.0;
    ctx->t_comp = ctx->t_pipe = 0.0;
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
    (void)hipFree(ctx->snap_cs);
    if (ctx->rec) (void)hipHostFree(ctx->rec);
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    delete ctx;
}

}  // extern "C"

namespace {

// The exact path for either parameter block: plans and sizes the batch, then
// replays the captured pipeline (captured again when the arguments change).
gl_status lightcurve(gl_ctx* ctx, Batch& b)
{
    const double* params = b.params;
    const int64_t n_sets = b.n_sets;
    const double* times = b.times;
    const int64_t* offsets = b.offsets;
    const int64_t n_times = b.n_times;
    const int32_t* n_ss = b.n_ss;
    const double* t_exp = b.t_exp;
    double* out = b.out;
    void* stream = (void*)b.stream;
    gl_status st = check_args(ctx, b);
    if (st != GL_OK) return st;
    GL_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    st = prepare_batch(ctx, b);
    if (st != GL_OK) return st;
    // the legacy default stream cannot be captured: launch directly there,
    // as timed batches are (their events stay out of graphs)
    const bool timed = ctx->t_left > 0;
    if (!ctx->use_graph || stream == nullptr || timed) {
        st = enqueue(ctx, b);
        if (st != GL_OK) return st;
        return timed ? finish_timed(ctx, b.stream) : GL_OK;
    }
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
    k.waves_trap = ctx->waves_trap;
    k.waves_classify = ctx->waves_classify;
    k.waves_gk = ctx->waves_gk;
    k.ws = ctx->masks;
    k.passes = ctx->passes;
    k.shape = b.shape;
    k.data = b.data;
    k.sigma = b.sigma;
    k.chi2 = b.chi2;
    k.loglike = b.loglike;
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

}  // namespace

extern "C" {

gl_status gl_lightcurve_batch(gl_ctx* ctx, const double* params, int64_t n_sets,
                              const double* times, const int64_t* offsets, int64_t n_times,
                              const int32_t* n_ss, const double* t_exp, double* out,
                              void* stream)
{
    Batch b{params, n_sets, times, offsets, n_times, n_ss, t_exp, out, (hipStream_t)stream, 0};
    return lightcurve(ctx, b);
}

gl_status gl_lightcurve_batch_ellipsoid(gl_ctx* ctx, const double* params, int64_t n_sets,
                                        const double* times, const int64_t* offsets, int64_t n_times,
                                        const int32_t* n_ss, const double* t_exp, double* out,
                                        void* stream)
{
    Batch b{params, n_sets, times, offsets, n_times, n_ss, t_exp, out, (hipStream_t)stream, 0};
    b.shape = 1;
    return lightcurve(ctx, b);
}

gl_status gl_loglike_batch(gl_ctx* ctx, const double* walkers, int64_t n_walkers, const double* times,
                           const int64_t* offsets, int64_t n_times, const int32_t* n_ss, const double* t_exp,
                           const double* data, const double* sigma, double* model, double* chi2, double* loglike,
                           void* stream)
{
    if (!ctx) return GL_ERR_NULL;
    ctx->err[0] = 0;
    if (!walkers || !data || !sigma || !model || (!chi2 && !loglike))
        return fail(ctx, GL_ERR_NULL, "walkers, data, sigma, model and chi2 or loglike are required");
    Batch b{walkers, n_walkers, times, offsets, n_times, n_ss, t_exp, model, (hipStream_t)stream, 0};
    b.shape = 2;  // k_prep converts the walker block
    b.data = data;
    b.sigma = sigma;
    b.chi2 = chi2;
    b.loglike = loglike;
    return lightcurve(ctx, b);
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
        std::snprintf(ctx->err, sizeof(ctx->err), "%s%s%s", (status & 1u) ? "invalid parameter set; " : "",
                      (status & 2u) ? "invalid CSR segment; " : "", (status & 4u) ? "non-finite time; " : "");
        return GL_ERR_DOMAIN;
    }
    return GL_OK;
}

const char* gl_ctx_last_error(const gl_ctx* ctx)
{
    return ctx ? ctx->err : "null context";
}

gl_status gl_ctx_get_plan(const gl_ctx* ctx, int* waves_per_cu)
{
    if (!ctx) return GL_ERR_NULL;
    if (waves_per_cu) *waves_per_cu = ctx->waves_per_cu;
    return GL_OK;
}

gl_status gl_ctx_get_stage_plan(const gl_ctx* ctx, int* classify, int* hard, int* trap, int* gk)
{
    if (!ctx) return GL_ERR_NULL;
    if (classify) *classify = ctx->waves_classify;
    if (hard) *hard = ctx->waves_per_cu;
    if (trap) *trap = ctx->waves_trap;
    if (gk) *gk = ctx->waves_gk;
    return GL_OK;
}

gl_status gl_ctx_set_stage_plan(gl_ctx* ctx, int classify, int hard, int trap, int gk)
{
    if (!ctx) return GL_ERR_NULL;
    if (classify < 1 || classify > 64 || hard < 1 || hard > 64 || trap < 1 || trap > 64 || gk < 1 || gk > 64)
        return fail(ctx, GL_ERR_SIZE, "waves per CU in [1, 64]");
    ctx->waves_classify = classify;
    ctx->waves_per_cu = hard;
    ctx->waves_trap = trap;
    ctx->waves_gk = gk;
    drop_graph(ctx);
    return GL_OK;
}

gl_status gl_ctx_set_plan(gl_ctx* ctx, int waves_per_cu)
{
    if (!ctx) return GL_ERR_NULL;
    if (waves_per_cu < 1 || waves_per_cu > 64) return fail(ctx, GL_ERR_SIZE, "waves_per_cu in [1, 64]");
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

}  // extern "C"

namespace {

gl_status autotune(gl_ctx* ctx, Batch b)
{
    gl_status st = check_args(ctx, b);
    if (st != GL_OK) return st;
    GL_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    st = prepare_batch(ctx, b);
    if (st != GL_OK) return st;
    drop_graph(ctx);
    hipEvent_t e0, e1;
    GL_HIP(hipEventCreate(&e0), "hipEventCreate");
    GL_HIP(hipEventCreate(&e1), "hipEventCreate");
    // coordinate descent over the four grid sizes: hard-sample kernel,
    // trapezoid kernel (beside the hard chain, where a smaller grid can leave
    // the chain more of the chip), classification, arc levels; two sweeps.
    // Each candidate: one warm-up batch, then the median of seven timed ones.
    // Candidates run the way the batch call will run them: captured and
    // replayed as a graph where the caller's stream allows one (branches of a
    // graph and of direct launches overlap differently).
    auto time_plan = [&](float& ms_out) -> gl_status {
        Batch c = b;
        gl_status r = lightcurve(ctx, c);  // warm-up (and the capture)
        if (r != GL_OK) return r;
        constexpr int kReps = 7;
        float t[kReps];
        for (int rep = 0; rep < kReps; ++rep) {
            (void)hipEventRecord(e0, b.stream);
            c = b;
            r = lightcurve(ctx, c);
            (void)hipEventRecord(e1, b.stream);
            (void)hipEventSynchronize(e1);
            t[rep] = 0.0f;
            (void)hipEventElapsedTime(&t[rep], e0, e1);
            if (r != GL_OK) return r;
        }
        std::sort(t, t + kReps);
        ms_out = t[kReps / 2];
        return r;
    };
    struct Knob {
        int* v;
        std::vector<int> cands;
    };
    Knob knobs[4] = {{&ctx->waves_per_cu, {4, 8, 16, 24, 32, 48, 64}},
                     {&ctx->waves_trap, {4, 8, 16, 24, 32, 48, 64}},
                     {&ctx->waves_classify, {8, 16, 24, 32, 48, 64}},
                     {&ctx->waves_gk, {8, 12, 16, 20, 32, 48, 64}}};
    for (int sweep = 0; sweep < 2 && st == GL_OK; ++sweep) {
        for (Knob& kn : knobs) {
            int best = *kn.v;
            float best_ms = 1e30f;
            for (int w : kn.cands) {
                *kn.v = w;
                float ms = 0.0f;
                st = time_plan(ms);
                if (st != GL_OK) break;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = w;
                }
            }
            *kn.v = best;
            if (st != GL_OK) break;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    drop_graph(ctx);
    return st;
}

}  // namespace

extern "C" {

gl_status gl_autotune(gl_ctx* ctx, const double* params, int64_t n_sets, const double* times,
                      const int64_t* offsets, int64_t n_times, const int32_t* n_ss,
                      const double* t_exp, double* out, void* stream)
{
    Batch b{params, n_sets, times, offsets, n_times, n_ss, t_exp, out, (hipStream_t)stream, 0};
    return autotune(ctx, b);
}

gl_status gl_autotune_ellipsoid(gl_ctx* ctx, const double* params, int64_t n_sets, const double* times,
                                const int64_t* offsets, int64_t n_times, const int32_t* n_ss,
                                const double* t_exp, double* out, void* stream)
{
    Batch b{params, n_sets, times, offsets, n_times, n_ss, t_exp, out, (hipStream_t)stream, 0};
    b.shape = 1;
    return autotune(ctx, b);
}

gl_status gl_ctx_set_timing(gl_ctx* ctx, int n_slots)
{
    if (!ctx) return GL_ERR_NULL;
    if (n_slots < 0 || n_slots > 10000) return fail(ctx, GL_ERR_SIZE, "n_slots in [0, 10000]");
    GL_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    GL_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    free_timing(ctx);
    drop_graph(ctx);  // the next batch is captured with (or without) its timing events
    if (n_slots == 0) return GL_OK;
    // one event set per pass (a timed batch is read before the next one)
    ctx->ev = new (std::nothrow) hipEvent_t[kEvPerPass * kMaxPasses];
    if (!ctx->ev) return fail(ctx, GL_ERR_NOMEM, "timing events");
    for (int i = 0; i < kEvPerPass * kMaxPasses; ++i) {
        if (hipEventCreate(&ctx->ev[i]) != hipSuccess) {
            for (int j = 0; j < i; ++j) (void)hipEventDestroy(ctx->ev[j]);
            delete[] ctx->ev;
            ctx->ev = nullptr;
            return fail(ctx, GL_ERR_DEVICE, "hipEventCreate");
        }
    }
    ctx->t_left = n_slots;
    return GL_OK;
}

gl_status gl_ctx_get_stage_timing(gl_ctx* ctx, double* stage_ms, int* n)
{
    if (!ctx) return GL_ERR_NULL;
    if (stage_ms)
        for (int k = 0; k < GL_NSTAGES; ++k) stage_ms[k] = ctx->t_stage[k];
    if (n) *n = ctx->t_batches;
    for (int k = 0; k < GL_NSTAGES; ++k) ctx->t_stage[k] = 0.0;
    ctx->t_comp = ctx->t_pipe = 0.0;
    ctx->t_batches = 0;
    return GL_OK;
}

gl_status gl_ctx_get_timing(gl_ctx* ctx, double* compute_ms, double* pipeline_ms, int* n)
{
    if (!ctx) return GL_ERR_NULL;
    if (compute_ms) *compute_ms = ctx->t_comp;
    if (pipeline_ms) *pipeline_ms = ctx->t_pipe;
    if (n) *n = ctx->t_batches;
    for (int k = 0; k < GL_NSTAGES; ++k) ctx->t_stage[k] = 0.0;
    ctx->t_comp = ctx->t_pipe = 0.0;
    ctx->t_batches = 0;
    return GL_OK;
}

gl_status gl_ctx_set_capacity(gl_ctx* ctx, int64_t sub_samples, int64_t hard_samples, int64_t arcs)
{
    if (!ctx) return GL_ERR_NULL;
    if (sub_samples < 0 || hard_samples < 0 || arcs < 0 || sub_samples > kSubMask ||
        hard_samples > INT32_MAX / 2 || arcs > INT32_MAX / 2)
        return fail(ctx, GL_ERR_SIZE, "capacities: 0 (default) or sub <= 2^27 - 1, hard and arcs <= 2^30 - 1");
    GL_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    GL_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    ctx->want_sub = sub_samples;
    ctx->want_hard = hard_samples;
    ctx->want_arc = arcs;
    // sizing from demand starts over
    for (int l = 0; l < kLists; ++l) ctx->auto_scap[l] = 0;
    GL_HIP(hipMemset(&ctx->ctr->demand, 0, sizeof(Demand)), "hipMemset");
    GL_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    std::memset(ctx->rec, 0, sizeof(Demand));
    drop_graph(ctx);
    free_pipe(ctx);
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
    st = prepare_batch(ctx, b);
    if (st != GL_OK) return st;
    st = enqueue(ctx, b, true);
    if (st != GL_OK) return st;
    GL_HIP(hipStreamSynchronize(b.stream), "hipStreamSynchronize");
    std::vector<LineCount> c((size_t)kCensus * kShards);
    GL_HIP(hipMemcpy(c.data(), ctx->ctr->census, sizeof(LineCount) * c.size(), hipMemcpyDeviceToHost), "hipMemcpy");
    for (int i = 0; i < kCensus; ++i) {
        unsigned long long t = 0;
        for (int j = 0; j < kShards; ++j) t += c[(size_t)i * kShards + j].v;
        counts[i] = (int64_t)t;
    }
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
    per_item[8] = gl::kFlopTrapNode;
    per_item[9] = gl::kFlopArc;
    per_item[10] = 0;  // unconverged arcs: their pieces are already counted
    return GL_OK;
}

gl_status gl_lightcurve_batch_snap(gl_ctx* ctx, int n_nodes, const double* params, int64_t n_sets,
                                   const double* times, const int64_t* offsets, int64_t n_times,
                                   const int32_t* n_ss, const double* t_exp, double* out, void* stream)
{
    Batch b{params, n_sets, times, offsets, n_times, n_ss, t_exp, out, (hipStream_t)stream, 0};
    gl_status st = check_args(ctx, b);
    if (st != GL_OK) return st;
    if (n_nodes < 4 || n_nodes > (1 << 20) || n_nodes % 2) return fail(ctx, GL_ERR_SIZE, "n_nodes even in [4, 2^20]");
    GL_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    st = ensure_ws(ctx, n_sets, b.max_chunks);
    if (st != GL_OK) return st;
    st = ensure_pipe(ctx, b.max_chunks);  // the window kernel's arguments (its lists stay unused)
    if (st != GL_OK) return st;
    hipStream_t s = b.stream;
    const int shared = b.offsets ? 0 : 1;
    const int64_t cps_shared = shared ? (b.n_times + kChunk - 1) / kChunk : 0;
    hipLaunchKernelGGL(k_prep<0>, dim3((unsigned)((n_sets + 255) / 256)), dim3(256), 0, s, params, n_sets, n_sets,
                       offsets, n_times, n_ss, t_exp, ctx->sc, ctx->seg_begin, ctx->seg_len, ctx->chunk_off, ctx->ctr,
                       cps_shared, 1, 1, (gl::SetConst*)nullptr, (const double*)nullptr, (int64_t)0, (double*)nullptr);
    if (!shared)
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, s, ctx->chunk_off, n_sets, b.max_chunks, ctx->ctr);
    launch_window(ctx, b, s, 0, ctx->pipe);
    if (n_nodes > ctx->snap_cap) {
        GL_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
        (void)hipFree(ctx->snap_cs);
        ctx->snap_cs = nullptr;
        ctx->snap_cap = 0;
        if (hipMalloc(&ctx->snap_cs, sizeof(float2) * n_nodes) != hipSuccess) return fail(ctx, GL_ERR_NOMEM, "node table");
        ctx->snap_cap = n_nodes;
        ctx->snap_n = 0;
    }
    if (ctx->snap_n != n_nodes) {
        hipLaunchKernelGGL(k_snap_nodes, dim3((unsigned)((n_nodes + 255) / 256)), dim3(256), 0, s, n_nodes, ctx->snap_cs);
        ctx->snap_n = n_nodes;
    }
    // a workgroup per chunk (the dispatcher balances chunks of unequal work)
    const unsigned grid = (unsigned)std::min<int64_t>(b.max_chunks, (int64_t)INT32_MAX);
    hipLaunchKernelGGL(k_snap, dim3(grid), dim3(64 * kSnapWaves), 0, s, times, shared, ctx->sc, ctx->seg_begin,
                       ctx->chunk_off, ctx->ctr, ctx->masks, ctx->chunk_set, n_nodes, ctx->snap_cs, out);
    GL_HIP(hipGetLastError(), "kernel launch");
    return GL_OK;
}

gl_status gl_ctx_get_overflow(gl_ctx* ctx, int64_t* fused_chunks, int* passes)
{
    if (!ctx || !fused_chunks) return GL_ERR_NULL;
    GL_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    GL_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    unsigned long long f = 0;
    GL_HIP(hipMemcpy(&f, &ctx->ctr->fused_batch, sizeof(f), hipMemcpyDeviceToHost), "hipMemcpy");
    *fused_chunks = (int64_t)f;
    if (passes) *passes = ctx->passes;
    return GL_OK;
}

gl_status gl_ctx_get_unconverged(gl_ctx* ctx, int64_t* n_arcs)
{
    if (!ctx || !n_arcs) return GL_ERR_NULL;
    GL_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    GL_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    unsigned long long u = 0;
    GL_HIP(hipMemcpy(&u, &ctx->ctr->unconverged, sizeof(u), hipMemcpyDeviceToHost), "hipMemcpy");
    if (u) {
        GL_HIP(hipMemset(&ctx->ctr->unconverged, 0, sizeof(u)), "hipMemset");
        GL_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    }
    *n_arcs = (int64_t)u;
    return GL_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- allocation-free batch
// For callers that cannot allocate device memory (code under stream capture,
// tight serving loops): the whole exact pipeline with its workspace and work
// lists carved out of one file-scope device array, at fixed capacities.
// Chunks that do not fit the lists take the fused kernel, so results are those
// of gl_lightcurve_batch up to rounding.  Every call on a device shares that
// device's array: calls that overlap on one device race.
namespace {

constexpr int64_t kStaticSets = 16384;              // parameter sets per call
constexpr int64_t kStaticChunks = (int64_t)1 << 18;  // 64-output chunks per call (16.7 M outputs)
constexpr int64_t kStaticSub = (int64_t)1 << 19;     // sub-sample slots of the work lists
constexpr int64_t kStaticWC = (int64_t)1 << 16;      // chunks with in-window outputs on the lists

constexpr int64_t align256(int64_t x) { return (x + 255) / 256 * 256; }

// per-shard capacities of the lists
constexpr int64_t kSsub = kStaticSub / kShards;
constexpr int64_t kShard = kSsub / 4;
constexpr int64_t kSarc = 2 * kShard;
constexpr int64_t kSwc = kStaticWC / kShards;
constexpr int64_t kSgrp = kSsub / kChunk + kSwc;

// byte offsets of the parts of the array
constexpr int64_t kOffCtr = 0;
constexpr int64_t kOffSc = align256(kOffCtr + (int64_t)sizeof(Counters));
constexpr int64_t kOffSegB = align256(kOffSc + kStaticSets * (int64_t)sizeof(gl::SetConst));
constexpr int64_t kOffSegL = align256(kOffSegB + kStaticSets * 8);
constexpr int64_t kOffChOff = align256(kOffSegL + kStaticSets * 8);
constexpr int64_t kOffMasks = align256(kOffChOff + (kStaticSets + 1) * 8);
constexpr int64_t kOffChSet = align256(kOffMasks + kStaticChunks * 8);
constexpr int64_t kOffChFb = align256(kOffChSet + kStaticChunks * 4);
constexpr int64_t kOffFbCh = align256(kOffChFb + kStaticChunks * 4);
constexpr int64_t kOffFsub = align256(kOffFbCh + kStaticChunks * 8);
constexpr int64_t kOffWc = align256(kOffFsub + kShards * kSsub * 8);
constexpr int64_t kOffGrp = align256(kOffWc + kShards * kSwc * (int64_t)sizeof(WorkChunk));
constexpr int64_t kOffTrap = align256(kOffGrp + kShards * kSgrp * (int64_t)sizeof(Group));
constexpr int64_t kOffHard = align256(kOffTrap + kShards * kSsub * (int64_t)sizeof(Entry));
constexpr int64_t kOffNest = align256(kOffHard + kShards * kShard * (int64_t)sizeof(Entry));
constexpr int64_t kOffHrec = align256(kOffNest + kShards * kShard * (int64_t)sizeof(Entry));
constexpr int64_t kOffHfr = align256(kOffHrec + kShards * kShard * (int64_t)sizeof(HardRec));
constexpr int64_t kOffArcs = align256(kOffHfr + kShards * kShard * (int64_t)sizeof(gl::Frame));
constexpr int64_t kOffArcRes = align256(kOffArcs + kShards * kSarc * (int64_t)sizeof(ArcRec));
constexpr int64_t kOffLvl = align256(kOffArcRes + kShards * kSarc * (int64_t)sizeof(gl::Sums));
constexpr int64_t kLvlBytes = align256(kShards * kSarc * (int64_t)sizeof(ArcRef));
constexpr int64_t kScratchBytes = kOffLvl + kLevels * kLvlBytes;
static_assert(kScratchBytes <= ((int64_t)80 << 20), "allocation-free workspace above its stated 80 MiB");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` and CU count, per device (found once per
// device, with that device current, on the first call there).
constexpr int kMaxDevices = 64;
unsigned char* g_scratch_dev[kMaxDevices] = {};
int g_scratch_cu[kMaxDevices] = {};
std::mutex g_scratch_mu;

// counters that a batch reports and that must start from zero on every call
// (the ones of the work lists are reset by k_prep)
__global__ void k_clear_static(Counters* __restrict__ ctr)
{
    ctr->status = 0u;
    ctr->unconverged = 0ull;
    ctr->fused_batch = 0ull;
    ctr->total_chunks = 0ull;
}

}  // namespace

extern "C" gl_status gl_lightcurve_batch_noalloc(const double* params, int64_t n_sets, const double* times,
                                                 const int64_t* offsets, int64_t n_times, const int32_t* n_ss,
                                                 const double* t_exp, double* out, void* stream)
{
    Batch b{params, n_sets, times, offsets, n_times, n_ss, t_exp, out, (hipStream_t)stream, 0};
    gl_status st = check_batch(nullptr, b);
    if (st != GL_OK) return st;
    if (n_sets > kStaticSets || b.max_chunks > kStaticChunks) return GL_ERR_SIZE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GL_ERR_DEVICE;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_dev[dev]) {
            void* ptr = nullptr;
            if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return GL_ERR_DEVICE;
            int ncu = 0;
            if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
                ncu = 256;
            g_scratch_cu[dev] = ncu;
            g_scratch_dev[dev] = (unsigned char*)ptr;
        }
    }
    unsigned char* base = g_scratch_dev[dev];
    gl_ctx c;  // on the stack, pointing into this device's array only (it owns no memory)
    c.device = dev;
    c.n_cu = g_scratch_cu[dev];
    c.use_graph = false;
    c.ctr = (Counters*)(base + kOffCtr);
    c.sc = (gl::SetConst*)(base + kOffSc);
    c.seg_begin = (int64_t*)(base + kOffSegB);
    c.seg_len = (int64_t*)(base + kOffSegL);
    c.chunk_off = (int64_t*)(base + kOffChOff);
    c.cap_sets = kStaticSets;
    c.masks = (unsigned long long*)(base + kOffMasks);
    c.chunk_set = (int*)(base + kOffChSet);
    c.cap_chunks = kStaticChunks;
    c.chunk_fb = (int*)(base + kOffChFb);
    Pipe& P = c.pipe;
    P.fb_chunk = (int64_t*)(base + kOffFbCh);
    P.fsub = (double*)(base + kOffFsub);
    P.wc = (WorkChunk*)(base + kOffWc);
    P.grp = (Group*)(base + kOffGrp);
    P.trap = (Entry*)(base + kOffTrap);
    P.hard = (Entry*)(base + kOffHard);
    P.nest = (Entry*)(base + kOffNest);
    P.hrec = (HardRec*)(base + kOffHrec);
    P.hfr = (gl::Frame*)(base + kOffHfr);
    P.arcs = (ArcRec*)(base + kOffArcs);
    P.arc_res = (gl::Sums*)(base + kOffArcRes);
    for (int L = 0; L < kLevels; ++L) P.lvl[L] = (ArcRef*)(base + kOffLvl + L * kLvlBytes);
    P.scap[L_SUB] = P.scap[L_TRAP] = kSsub;
    P.scap[L_WC] = kSwc;
    P.scap[L_GRP] = kSgrp;
    P.scap[L_HARD] = P.scap[L_NEST] = kShard;
    P.scap[L_ARC] = kSarc;
    for (int L = 0; L < kLevels; ++L) P.scap[L_LVL0 + L] = kSarc;
    c.have_pipe = true;
    c.pipe_chunks = kStaticChunks;
    c.want_sub = kStaticSub;  // fixed capacities: one pass, no demand record
    c.passes = 1;
    hipLaunchKernelGGL(k_clear_static, dim3(1), dim3(1), 0, b.stream, c.ctr);
    return enqueue_t<false>(&c, b);
}

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
    gl::NoCensus nc;
    if (!gl::make_set_const(p, 0.0, 1, S) || !gl::finite_d(times[i])) {
        atomicOr(&ctr->status, 1u);
        Fo = Fs = __builtin_nan("");
    } else {
        double x0, y0;
        if (gl::centre_at(S, times[i], x0, y0) && gl::sur_encode(S, x0, y0, fe, sc, bin)) {
            Fo = 1.0 - gl::occulted<gl::NoCensus>(S, x0, y0, nullptr, nc);
            const gl::SetConst C = gl::sphere_of(S);
            Fs = 1.0 - gl::occulted<gl::NoCensus>(C, x0, y0, nullptr, nc);
        }
    }
    unconverged_add(ctr, nc.unconv, false);
    for (int r = 0; r < gl::kSurFeat; ++r) feat[i * gl::kSurFeat + r] = fe[r];
    target[i] = bin >= 0 ? (float)((Fo - Fs) / sc) : 0.f;
    if (f_obl) f_obl[i] = Fo;
    if (f_sph) f_sph[i] = Fs;
    if (scale_out) scale_out[i] = sc;
    if (bin_out) bin_out[i] = bin;
}

// Counter-based uniform draws in [0, 1): SplitMix64 of (seed, sample, column)
__device__ __forceinline__ double u01(uint64_t seed, int64_t i, int col)
{
    uint64_t z = seed ^ ((uint64_t)i * 0xd1342543de82ef95ull) ^ ((uint64_t)(col + 1) * 0x9e3779b97f4a7c15ull);
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-53;
}

// Training / calibration draws from the walker priors: k ~ U[0.05, 0.12],
// f ~ U[0, 0.9], theta ~ U[0, pi], phi ~ U[0, 2 pi), b ~ U[0, 0.9],
// a/R* ~ U[100, 300], q1, q2 ~ U[0, 1], P = 500 d, t0 = 0; one time per
// sample uniform in +-window * T14 (the transit duration of the sphere of
// radius k, T14 = (P / pi) asin(sqrt((1 + k)^2 - b^2) / (a/R* sin i)),
// sin i = sqrt(1 - (b / a/R*)^2)).
__global__ void k_sur_draw(uint64_t seed, int64_t n, double window, double* __restrict__ params,
                           double* __restrict__ times)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double k = 0.05 + 0.07 * u01(seed, i, 0);
    const double f = 0.9 * u01(seed, i, 1);
    const double th = gl::kPi * u01(seed, i, 2);
    const double ph = gl::kTwoPi * u01(seed, i, 3);
    const double b = 0.9 * u01(seed, i, 4);
    const double ars = 100.0 + 200.0 * u01(seed, i, 5);
    const double q1 = u01(seed, i, 6), q2 = u01(seed, i, 7);
    const double P = 500.0;
    const double sini = sqrt(1.0 - (b / ars) * (b / ars));
    const double t14 = P / gl::kPi * asin(fmin(1.0, sqrt((1.0 + k) * (1.0 + k) - b * b) / (ars * sini)));
    const double vals[GL_NPARAM] = {k, f, th, ph, b, ars, P, 0.0, q1, q2};
    for (int r = 0; r < GL_NPARAM; ++r) params[(int64_t)r * n + i] = vals[r];
    times[i] = (2.0 * u01(seed, i, 8) - 1.0) * window * t14;
}

constexpr int kKeepBlock = 1024;  // rows per block of the on-star compaction

// rows with bin >= 0 per block of kKeepBlock rows
__global__ void __launch_bounds__(256) k_keep_count(const int* __restrict__ bin, int64_t n, int64_t* __restrict__ cnt)
{
    __shared__ int red[4];
    const int64_t r0 = (int64_t)blockIdx.x * kKeepBlock;
    int c = 0;
    for (int k = threadIdx.x; k < kKeepBlock; k += 256)
        if (r0 + k < n && bin[r0 + k] >= 0) ++c;
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) cnt[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// exclusive scan of a[0..n) in place, a[n] = total (one workgroup)
__global__ void __launch_bounds__(kScanThreads) k_excl_scan(int64_t* __restrict__ a, int64_t n)
{
    __shared__ int64_t part[kScanThreads];
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

// the rows with bin >= 0, in order, as BF16 features and FP32 targets
__global__ void __launch_bounds__(256)
k_keep_write(const float* __restrict__ feat, const float* __restrict__ target, const int* __restrict__ bin, int64_t n,
             const int64_t* __restrict__ off, uint16_t* __restrict__ X, float* __restrict__ T)
{
    __shared__ int wsum[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * kKeepBlock;
    int64_t base = off[blockIdx.x];
    for (int k0 = 0; k0 < kKeepBlock; k0 += 256) {
        const int64_t r = r0 + k0 + threadIdx.x;
        const bool keep = r < n && bin[r] >= 0;
        const unsigned long long m = __ballot(keep);
        if (lane == 0) wsum[wv] = __popcll(m);
        __syncthreads();
        int before = 0;
        for (int w = 0; w < wv; ++w) before += wsum[w];
        if (keep) {
            const int64_t o = base + before + lanes_below(m);
            for (int f = 0; f < gl::kSurFeat; ++f) X[o * gl::kSurFeat + f] = gl::f2bf_rne(feat[r * gl::kSurFeat + f]);
            T[o] = target[r];
        }
        base += wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
    }
}

// Calibration: per bin the largest |prediction - target| of the network and
// of the zero predictor (float bits of non-negative values order like
// integers, so an integer maximum is exact and order-independent) and the
// sample count
__global__ void k_sur_calib(const float* __restrict__ pred, const float* __restrict__ target,
                            const int* __restrict__ bin, int64_t n, unsigned int* __restrict__ err_net,
                            unsigned int* __restrict__ err_zero, int* __restrict__ counts)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || bin[i] < 0) return;
    auto up = [](double e) {  // rounded up to float
        float x = (float)e;
        if ((double)x < e) x = __uint_as_float(__float_as_uint(x) + 1u);
        return __float_as_uint(x);
    };
    const double t = (double)target[i];
    atomicMax(&err_net[bin[i]], up(fabs((double)pred[i] - t)));
    atomicMax(&err_zero[bin[i]], up(fabs(t)));
    atomicAdd(&counts[bin[i]], 1);
}

// table[b] = the smaller calibrated bound of the two predictors (the zero
// predictor only, with zero_only), -1 where fewer than min_count samples
// fell; zero[b] = 1 where the sphere alone is taken
__global__ void k_sur_finalize(const unsigned int* __restrict__ err_net, const unsigned int* __restrict__ err_zero,
                               const int* __restrict__ counts, int min_count, int zero_only, float* __restrict__ table,
                               uint8_t* __restrict__ zero)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= gl::kSurBins) return;
    const float en = __uint_as_float(err_net[b]), ez = __uint_as_float(err_zero[b]);
    const bool z = zero_only || ez <= en;
    zero[b] = z ? 1 : 0;
    table[b] = counts[b] >= min_count ? (z ? ez : en) : -1.0f;
}

}  // namespace

struct gl_surrogate {
    int device = 0;
    gl_mlp* net = nullptr;
    float* table = nullptr;      // device [kSurBins]
    uint8_t* zero = nullptr;     // device [kSurBins]
    int32_t* counts = nullptr;   // device [kSurBins]
    gl_surrogate_config cfg{};
};

namespace {

void sur_free(gl_surrogate* s)
{
    if (!s) return;
    (void)hipSetDevice(s->device);
    (void)hipDeviceSynchronize();
    gl_mlp_destroy(s->net);
    (void)hipFree(s->table);
    (void)hipFree(s->zero);
    (void)hipFree(s->counts);
    delete s;
}

gl_status sur_alloc(gl_ctx* ctx, const gl_surrogate_config& cfg, gl_surrogate** out)
{
    gl_surrogate* s = new (std::nothrow) gl_surrogate();
    if (!s) return fail(ctx, GL_ERR_NOMEM, "surrogate");
    s->device = ctx->device;
    s->cfg = cfg;
    gl_status st = gl_mlp_create(&s->net, ctx->device, cfg.batch);
    if (st != GL_OK) {
        delete s;
        return fail(ctx, st, "surrogate network");
    }
    if (hipMalloc(&s->table, sizeof(float) * gl::kSurBins) != hipSuccess ||
        hipMalloc(&s->zero, gl::kSurBins) != hipSuccess ||
        hipMalloc(&s->counts, sizeof(int32_t) * gl::kSurBins) != hipSuccess) {
        sur_free(s);
        return fail(ctx, GL_ERR_NOMEM, "surrogate tables");
    }
    *out = s;
    return GL_OK;
}

// He-uniform initial weights, zero biases, from a seeded host generator
void init_weights(uint64_t seed, float* w)
{
    uint64_t z = seed * 0x2545f4914f6cdd1dull + 1ull;
    auto next = [&z]() {
        z += 0x9e3779b97f4a7c15ull;
        uint64_t x = z;
        x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
        x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
        return (double)((x ^ (x >> 31)) >> 11) * 0x1.0p-53;
    };
    const int dims[6] = {GL_MLP_DIN, GL_MLP_WIDTH, GL_MLP_WIDTH, GL_MLP_WIDTH, GL_MLP_WIDTH, 1};
    int64_t o = 0;
    for (int l = 0; l < 5; ++l) {
        const int a = dims[l], b = dims[l + 1];
        const double lim = b != 1 ? std::sqrt(6.0 / a) : std::sqrt(3.0 / a);
        for (int64_t e = 0; e < (int64_t)a * b; ++e) w[o++] = (float)((2.0 * next() - 1.0) * lim);
        for (int e = 0; e < b; ++e) w[o++] = 0.0f;
    }
}

}  // namespace

extern "C" {

void gl_surrogate_config_default(gl_surrogate_config* c)
{
    if (!c) return;
    c->n_train = 20000000;
    c->n_calib = 1000000;
    c->epochs = 4;
    c->batch = 8192;
    c->lr = 2e-3f;
    c->lr_final = 1e-4f;
    c->safety = 4.0;
    c->min_bin_count = 200;
    c->window = 0.6;
    c->seed = 5;
    c->zero_predictor = 0;
}

gl_status gl_surrogate_samples(gl_ctx* ctx, const double* params, const double* times, int64_t n,
                               float* feat, float* target, double* f_obl, double* f_sph,
                               double* scale, int32_t* bin, void* stream)
{
    if (!ctx) return GL_ERR_NULL;
    ctx->err[0] = 0;
    if (!params || !times || !feat || !target) return fail(ctx, GL_ERR_NULL, "params, times, feat, target");
    if (n < 1) return fail(ctx, GL_ERR_SIZE, "n >= 1");
    GL_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    hipLaunchKernelGGL(k_sur_samples, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, (hipStream_t)stream,
                       params, n, times, feat, target, f_obl, f_sph, scale, bin, ctx->ctr);
    GL_HIP(hipGetLastError(), "kernel launch");
    return GL_OK;
}

int gl_surrogate_num_bins(void) { return gl::kSurBins; }

gl_status gl_surrogate_train(gl_ctx* ctx, const gl_surrogate_config* cfg_in, gl_surrogate** out,
                             float* loss_history, void* stream)
{
    if (!ctx || !cfg_in || !out) return GL_ERR_NULL;
    *out = nullptr;
    ctx->err[0] = 0;
    const gl_surrogate_config cfg = *cfg_in;
    if (cfg.batch < 64 || cfg.batch % 64 || cfg.batch > (1 << 20) || cfg.epochs < 1 || cfg.epochs > 1000 ||
        cfg.n_train < cfg.batch || cfg.n_train > ((int64_t)1 << 31) || cfg.n_calib < 1 ||
        cfg.n_calib > ((int64_t)1 << 31) || !(cfg.lr > 0.f) || !(cfg.lr_final > 0.f) || !(cfg.safety > 0.0) ||
        cfg.min_bin_count < 1 || !(cfg.window > 0.0))
        return fail(ctx, GL_ERR_SIZE, "surrogate configuration out of range");
    GL_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t st = (hipStream_t)stream;
    gl_surrogate* s = nullptr;
    gl_status rs = sur_alloc(ctx, cfg, &s);
    if (rs != GL_OK) return rs;
    std::vector<float> w0(gl_mlp_num_params());
    init_weights(cfg.seed + 2, w0.data());
    if (cfg.zero_predictor) std::fill(w0.begin(), w0.end(), 0.0f);
    rs = gl_mlp_set_weights(s->net, w0.data(), (int64_t)w0.size());
    if (rs != GL_OK) {
        sur_free(s);
        return fail(ctx, rs, "surrogate weights");
    }
    // sample buffers, sized for the larger of the two draws
    const int64_t nmax = std::max(cfg.n_train, cfg.n_calib);
    const int64_t nblk = (nmax + kKeepBlock - 1) / kKeepBlock;
    double *prm = nullptr, *tms = nullptr, *scl = nullptr;
    float *feat = nullptr, *tgt = nullptr, *Tk = nullptr, *pred = nullptr, *hist = nullptr;
    int *bin = nullptr;
    int64_t* koff = nullptr;
    uint16_t* Xk = nullptr;
    unsigned int *en = nullptr, *ez = nullptr;
    bool ok = hipMalloc(&prm, sizeof(double) * GL_NPARAM * nmax) == hipSuccess &&
              hipMalloc(&tms, sizeof(double) * nmax) == hipSuccess &&
              hipMalloc(&scl, sizeof(double) * nmax) == hipSuccess &&
              hipMalloc(&feat, sizeof(float) * gl::kSurFeat * nmax) == hipSuccess &&
              hipMalloc(&tgt, sizeof(float) * nmax) == hipSuccess && hipMalloc(&Tk, sizeof(float) * nmax) == hipSuccess &&
              hipMalloc(&pred, sizeof(float) * nmax) == hipSuccess &&
              hipMalloc(&hist, sizeof(float) * cfg.epochs) == hipSuccess &&
              hipMalloc(&bin, sizeof(int) * nmax) == hipSuccess &&
              hipMalloc(&koff, sizeof(int64_t) * (nblk + 1)) == hipSuccess &&
              hipMalloc(&Xk, sizeof(uint16_t) * gl::kSurFeat * nmax) == hipSuccess &&
              hipMalloc(&en, sizeof(unsigned int) * gl::kSurBins) == hipSuccess &&
              hipMalloc(&ez, sizeof(unsigned int) * gl::kSurBins) == hipSuccess;
    auto release = [&]() {
        void* b[] = {prm, tms, scl, feat, tgt, Tk, pred, hist, bin, koff, Xk, en, ez};
        for (void* q : b) (void)hipFree(q);
    };
    if (!ok) {
        release();
        sur_free(s);
        return fail(ctx, GL_ERR_NOMEM, "surrogate sample buffers");
    }
    auto draw = [&](uint64_t seed, int64_t n) {
        hipLaunchKernelGGL(k_sur_draw, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, seed, n, cfg.window, prm, tms);
        hipLaunchKernelGGL(k_sur_samples, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, st, prm, n, tms, feat, tgt,
                           nullptr, nullptr, scl, bin, ctx->ctr);
    };
    // training: the samples on the star, compacted in order
    int64_t n_keep = 0;
    if (!cfg.zero_predictor) {
        draw(cfg.seed, cfg.n_train);
        const int64_t nb = (cfg.n_train + kKeepBlock - 1) / kKeepBlock;
        hipLaunchKernelGGL(k_keep_count, dim3((unsigned)nb), dim3(256), 0, st, bin, cfg.n_train, koff);
        hipLaunchKernelGGL(k_excl_scan, dim3(1), dim3(kScanThreads), 0, st, koff, nb);
        hipLaunchKernelGGL(k_keep_write, dim3((unsigned)nb), dim3(256), 0, st, feat, tgt, bin, cfg.n_train, koff, Xk, Tk);
        ok = hipMemcpyAsync(&n_keep, koff + nb, sizeof(int64_t), hipMemcpyDeviceToHost, st) == hipSuccess &&
             hipStreamSynchronize(st) == hipSuccess && hipMemsetAsync(hist, 0, sizeof(float) * cfg.epochs, st) == hipSuccess;
        if (ok && n_keep >= cfg.batch) {
            rs = gl_net::train_rows(s->net, Xk, Tk, n_keep, cfg.epochs, cfg.batch, cfg.lr, cfg.lr_final, cfg.seed, hist, st);
            if (rs != GL_OK) ok = false;
        } else if (ok) {
            rs = GL_ERR_SIZE;
            ok = false;
        }
    }
    // calibration on fresh draws: the network's and the zero predictor's
    // largest scaled error per bin, and the counts
    if (ok) {
        draw(cfg.seed + 1, cfg.n_calib);
        const int64_t nc = cfg.n_calib;
        ok = hipMemsetAsync(en, 0, sizeof(unsigned int) * gl::kSurBins, st) == hipSuccess &&
             hipMemsetAsync(ez, 0, sizeof(unsigned int) * gl::kSurBins, st) == hipSuccess &&
             hipMemsetAsync(s->counts, 0, sizeof(int32_t) * gl::kSurBins, st) == hipSuccess;
        if (ok) {
            rs = gl_mlp_forward(s->net, feat, nc, pred, st);
            if (rs != GL_OK) ok = false;
        }
        if (ok) {
            hipLaunchKernelGGL(k_sur_calib, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, pred, tgt, bin, nc, en, ez,
                               s->counts);
            hipLaunchKernelGGL(k_sur_finalize, dim3((gl::kSurBins + 255) / 256), dim3(256), 0, st, en, ez, s->counts,
                               cfg.min_bin_count, cfg.zero_predictor, s->table, s->zero);
            ok = hipGetLastError() == hipSuccess && hipStreamSynchronize(st) == hipSuccess;
            if (ok && loss_history) {
                if (cfg.zero_predictor) std::fill(loss_history, loss_history + cfg.epochs, 0.0f);
                else ok = hipMemcpy(loss_history, hist, sizeof(float) * cfg.epochs, hipMemcpyDeviceToHost) == hipSuccess;
            }
        }
    }
    release();
    if (!ok) {
        sur_free(s);
        return fail(ctx, rs != GL_OK ? rs : GL_ERR_DEVICE,
                    rs == GL_ERR_SIZE ? "too few training samples on the star for one batch" : "surrogate training");
    }
    *out = s;
    return GL_OK;
}

void gl_surrogate_destroy(gl_surrogate* s) { sur_free(s); }

gl_status gl_surrogate_get(const gl_surrogate* s, float* params, int64_t n_params, float* table, uint8_t* zero_bins,
                           int32_t* counts, int n_bins)
{
    if (!s) return GL_ERR_NULL;
    if (n_bins != gl::kSurBins || (params && n_params != gl_mlp_num_params())) return GL_ERR_SIZE;
    if (hipSetDevice(s->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return GL_ERR_DEVICE;
    if (params && gl_mlp_get_weights(s->net, params, n_params) != GL_OK) return GL_ERR_DEVICE;
    if (table && hipMemcpy(table, s->table, sizeof(float) * n_bins, hipMemcpyDeviceToHost) != hipSuccess)
        return GL_ERR_DEVICE;
    if (zero_bins && hipMemcpy(zero_bins, s->zero, n_bins, hipMemcpyDeviceToHost) != hipSuccess) return GL_ERR_DEVICE;
    if (counts && hipMemcpy(counts, s->counts, sizeof(int32_t) * n_bins, hipMemcpyDeviceToHost) != hipSuccess)
        return GL_ERR_DEVICE;
    return GL_OK;
}

gl_status gl_surrogate_config_of(const gl_surrogate* s, gl_surrogate_config* cfg)
{
    if (!s || !cfg) return GL_ERR_NULL;
    *cfg = s->cfg;
    return GL_OK;
}

gl_status gl_surrogate_save(const gl_surrogate* s, const char* path)
{
    if (!s || !path) return GL_ERR_NULL;
    const int np = gl_mlp_num_params();
    std::vector<float> w(np), m(np), v(np), table(gl::kSurBins);
    std::vector<uint8_t> zero(gl::kSurBins);
    std::vector<int32_t> counts(gl::kSurBins);
    int64_t step = 0;
    gl_status st = gl_surrogate_get(s, w.data(), np, table.data(), zero.data(), counts.data(), gl::kSurBins);
    if (st != GL_OK) return st;
    st = gl_net::get_state(s->net, m.data(), v.data(), &step);
    if (st != GL_OK) return st;
    return gl_surrogate_file_write(path, &s->cfg, w.data(), m.data(), v.data(), step, np, table.data(), zero.data(),
                                   counts.data(), gl::kSurBins);
}

gl_status gl_surrogate_load(gl_ctx* ctx, gl_surrogate** out, const char* path)
{
    if (!ctx || !out || !path) return GL_ERR_NULL;
    *out = nullptr;
    ctx->err[0] = 0;
    const int np = gl_mlp_num_params();
    std::vector<float> w(np), m(np), v(np), table(gl::kSurBins);
    std::vector<uint8_t> zero(gl::kSurBins);
    std::vector<int32_t> counts(gl::kSurBins);
    int64_t step = 0;
    gl_surrogate_config cfg{};
    gl_status st = gl_surrogate_file_read(path, &cfg, w.data(), m.data(), v.data(), &step, np, table.data(),
                                          zero.data(), counts.data(), gl::kSurBins);
    if (st != GL_OK) return fail(ctx, st, "surrogate file");
    GL_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    gl_surrogate* s = nullptr;
    st = sur_alloc(ctx, cfg, &s);
    if (st != GL_OK) return st;
    if (gl_mlp_set_weights(s->net, w.data(), np) != GL_OK || gl_net::set_state(s->net, m.data(), v.data(), step) != GL_OK ||
        hipMemcpy(s->table, table.data(), sizeof(float) * gl::kSurBins, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->zero, zero.data(), gl::kSurBins, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->counts, counts.data(), sizeof(int32_t) * gl::kSurBins, hipMemcpyHostToDevice) != hipSuccess) {
        sur_free(s);
        return fail(ctx, GL_ERR_DEVICE, "surrogate upload");
    }
    *out = s;
    return GL_OK;
}

gl_status gl_lightcurve_batch_surrogate(gl_ctx* ctx, const gl_surrogate* s, double tol, const double* params,
                                        int64_t n_sets, const double* times, const int64_t* offsets, int64_t n_times,
                                        const int32_t* n_ss, const double* t_exp, double* out, void* stream,
                                        int64_t* n_sub_out, int64_t* n_fallback_out)
{
    Batch b{params, n_sets, times, offsets, n_times, n_ss, t_exp, out, (hipStream_t)stream, 0};
    gl_status st = check_args(ctx, b);
    if (st != GL_OK) return st;
    if (!s) return fail(ctx, GL_ERR_NULL, "surrogate required");
    if (!(tol > 0.0)) return fail(ctx, GL_ERR_SIZE, "tol > 0");
    if (s->device != ctx->device) return fail(ctx, GL_ERR_STATE, "surrogate on another device");
    GL_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    b.net = s->net;
    b.gate_table = s->table;
    b.gate_zero = s->zero;
    b.gate_k = s->cfg.safety / tol;
    if (!ctx->want_net) {
        ctx->want_net = true;
        drop_graph(ctx);
        GL_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
        free_pipe(ctx);
    }
    st = prepare_batch(ctx, b);
    if (st != GL_OK) return st;
    st = run_batch(ctx, b, false);
    if (st != GL_OK) return st;
    st = finish_timed(ctx, b.stream);
    if (st != GL_OK) return st;
    if (n_sub_out || n_fallback_out) {
        unsigned long long c[3] = {0ull, 0ull, 0ull};  // in window, reaching the disk, accepted
        std::vector<LineCount> sh((size_t)3 * kShards);
        GL_HIP(hipStreamSynchronize(b.stream), "hipStreamSynchronize");
        GL_HIP(hipMemcpy(sh.data(), ctx->ctr->sur, sizeof(LineCount) * sh.size(), hipMemcpyDeviceToHost), "hipMemcpy");
        for (int r = 0; r < 3; ++r)
            for (int j = 0; j < kShards; ++j) c[r] += sh[(size_t)r * kShards + j].v;
        if (n_sub_out) *n_sub_out = (int64_t)c[0];
        if (n_fallback_out) *n_fallback_out = (int64_t)(c[1] - c[2]);
    }
    return GL_OK;
}

const char* gl_version(void) { return "0.1.0"; }

}  // extern "C"
