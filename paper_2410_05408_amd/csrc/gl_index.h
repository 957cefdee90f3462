// gl_index.h -- where the 64-output chunks of a batch live in the caller's
// arrays (host and device), shared by the kernels and the host check of
// their index arithmetic.
//
// A batch's outputs are cut, per parameter set, into chunks of 64 consecutive
// outputs.  On a shared time grid every set has the same cps chunks and set s
// owns outputs [s n_times, (s + 1) n_times) while its times are the whole grid
// [0, n_times): the index of a chunk's first output and of its first time
// differ for every set but the first.  With CSR segments both are the
// segment's own index.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gl {

constexpr int kChunkOuts = 64;
constexpr int kWinGridChunks = 16;  // chunks per wavefront of the shared-grid window launch
constexpr int kWinCsrChunks = 4;    // chunks per wavefront of the CSR window launch

struct ChunkPos {
    int64_t out0;   // index in `out` of the chunk's first output
    int64_t time0;  // index in `times` of the chunk's first time
};

// Chunk lc (within its set) of a set whose outputs start at seg_begin (k_prep
// sets s * n_times on a shared grid, the segment start with CSR).
__host__ __device__ __forceinline__ ChunkPos chunk_pos(bool shared_grid, int64_t seg_begin, int64_t lc)
{
    const int64_t o = lc * kChunkOuts;
    return ChunkPos{seg_begin + o, shared_grid ? o : seg_begin + o};
}

// Window launch over a shared grid: bx = ceil(cps / per) blocks per set, set
// major; block blk covers chunks lc0 .. lc0 + nk - 1 of set s.
__host__ __device__ __forceinline__ void window_grid_block(int64_t blk, int64_t cps, int per, int64_t& s,
                                                           int64_t& lc0, int& nk)
{
    const int64_t bx = (cps + per - 1) / per;
    s = blk / bx;
    lc0 = (blk - s * bx) * per;
    const int64_t left = cps - lc0;
    nk = (int)(left < per ? left : per);
}

// CSR: the set of chunk c, chunk_off[0..n_sets] being the exclusive scan of
// the sets' chunk counts (chunk_off[lo] <= c < chunk_off[lo + 1]).
__host__ __device__ __forceinline__ int64_t set_of_chunk(const int64_t* chunk_off, int64_t n_sets, int64_t c)
{
    int64_t lo = 0, hi = n_sets;
    while (hi - lo > 1) {
        const int64_t m = (lo + hi) >> 1;
        if (chunk_off[m] <= c) lo = m;
        else hi = m;
    }
    return lo;
}

}  // namespace gl
