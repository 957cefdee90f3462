// Host check of the index arithmetic the kernels use to place a batch's
// chunks in the caller's arrays (gl_index.h): every block of the window
// launch, every chunk and every output lane, for shared grids and CSR
// segments, with bounds assertions on every index the window, classification,
// averaging and fused kernels form from it.
//
//   gl_index_check shared N_SETS N_TIMES
//   gl_index_check csr LEN0 LEN1 ...        (segment lengths, in order)
//
// Prints "ok <outputs covered>" or the first violated bound and exits 1.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "gl_index.h"

static int fails = 0;
#define CHECK(cond, ...)                                      \
    do {                                                      \
        if (!(cond)) {                                        \
            if (fails++ == 0) {                               \
                std::printf("violated: %s: ", #cond);         \
                std::printf(__VA_ARGS__);                     \
                std::printf("\n");                            \
            }                                                 \
        }                                                     \
    } while (0)

static const int64_t K = gl::kChunkOuts;

// A shared grid: n_sets sets, all at the same n_times times.
static int64_t check_shared(int64_t n_sets, int64_t n_times)
{
    const int64_t cps = (n_times + K - 1) / K, max_chunks = cps * n_sets, n_out = n_sets * n_times;
    const int per = gl::kWinGridChunks;
    const int64_t blocks = (cps + per - 1) / per * n_sets;  // the launch's grid
    std::vector<unsigned char> written(n_out, 0), chunk_seen(max_chunks, 0);
    for (int64_t blk = 0; blk < blocks; ++blk) {
        int64_t s, lc0;
        int nk;
        gl::window_grid_block(blk, cps, per, s, lc0, nk);
        CHECK(s >= 0 && s < n_sets, "block %lld -> set %lld", (long long)blk, (long long)s);
        CHECK(lc0 >= 0 && lc0 < cps && nk >= 1 && nk <= per, "block %lld: lc0 %lld nk %d", (long long)blk,
              (long long)lc0, nk);
        const int64_t ob = s * n_times;  // what k_prep stores as the set's segment start
        for (int k = 0; k < nk; ++k)
            for (int lane = 0; lane < K; ++lane) {
                const int64_t pos = (lc0 + k) * K + lane;  // the window's time index
                if (pos >= n_times) continue;
                CHECK(ob + pos < n_out, "window output %lld", (long long)(ob + pos));
                if (ob + pos < n_out) written[ob + pos]++;
            }
        for (int lane = 0; lane < nk; ++lane) {
            const int64_t c = s * cps + lc0 + lane;  // the chunk a lane describes
            CHECK(c < max_chunks, "chunk %lld of %lld", (long long)c, (long long)max_chunks);
            if (c < max_chunks) chunk_seen[c]++;
            const gl::ChunkPos cp = gl::chunk_pos(true, ob, lc0 + lane);
            for (int j = 0; j < K; ++j) {
                if ((lc0 + lane) * K + j >= n_times) break;  // output j of the chunk does not exist
                CHECK(cp.time0 + j < n_times, "set %lld chunk %lld: time index %lld of %lld", (long long)s,
                      (long long)(lc0 + lane), (long long)(cp.time0 + j), (long long)n_times);
                CHECK(cp.out0 + j < n_out && cp.out0 + j == ob + (lc0 + lane) * K + j,
                      "set %lld: output index %lld", (long long)s, (long long)(cp.out0 + j));
            }
        }
    }
    // the fused kernel and the averages find a chunk's set and position from it
    for (int64_t c = 0; c < max_chunks; ++c) {
        CHECK(chunk_seen[c] == 1, "chunk %lld described %d times", (long long)c, chunk_seen[c]);
        const int64_t s = c / cps, lc = c - s * cps;
        const gl::ChunkPos cp = gl::chunk_pos(true, s * n_times, lc);
        CHECK(cp.time0 == lc * K && cp.out0 == s * n_times + lc * K, "chunk %lld position", (long long)c);
    }
    int64_t covered = 0;
    for (int64_t i = 0; i < n_out; ++i) {
        CHECK(written[i] == 1, "output %lld written %d times", (long long)i, written[i]);
        covered += written[i] == 1;
    }
    return covered;
}

// CSR segments of the given lengths.
static int64_t check_csr(const std::vector<int64_t>& lens)
{
    const int64_t n_sets = (int64_t)lens.size();
    std::vector<int64_t> off(n_sets + 1, 0), chunk_off(n_sets + 1, 0);
    for (int64_t s = 0; s < n_sets; ++s) {
        off[s + 1] = off[s] + lens[s];
        chunk_off[s + 1] = chunk_off[s] + (lens[s] + K - 1) / K;
    }
    const int64_t n_times = off[n_sets], total = chunk_off[n_sets];
    const int64_t max_chunks = n_times / K + n_sets;
    CHECK(total <= max_chunks, "chunks %lld above the bound %lld", (long long)total, (long long)max_chunks);
    const int per = gl::kWinCsrChunks;
    const int64_t waves = (max_chunks + per - 1) / per;
    std::vector<unsigned char> written(n_times, 0);
    for (int64_t g = 0; g < waves; ++g) {
        const int64_t c_first = g * per;
        int64_t s = c_first < total ? gl::set_of_chunk(chunk_off.data(), n_sets, c_first) : 0;
        for (int k = 0; k < per; ++k) {
            const int64_t c = c_first + k;
            if (c >= total) continue;
            while (s + 1 < n_sets && chunk_off[s + 1] <= c) ++s;
            CHECK(chunk_off[s] <= c && c < chunk_off[s + 1], "chunk %lld in set %lld", (long long)c, (long long)s);
            const gl::ChunkPos cp = gl::chunk_pos(false, off[s], c - chunk_off[s]);
            CHECK(cp.out0 == cp.time0, "CSR chunk %lld: output and time index differ", (long long)c);
            for (int lane = 0; lane < K; ++lane) {
                const int64_t pos = (c - chunk_off[s]) * K + lane;
                if (pos >= lens[s]) continue;
                CHECK(cp.out0 + lane < off[s + 1], "chunk %lld lane %d beyond its segment", (long long)c, lane);
                if (cp.out0 + lane < n_times) written[cp.out0 + lane]++;
            }
        }
    }
    int64_t covered = 0;
    for (int64_t i = 0; i < n_times; ++i) {
        CHECK(written[i] == 1, "output %lld written %d times", (long long)i, written[i]);
        covered += written[i] == 1;
    }
    return covered;
}

int main(int argc, char** argv)
{
    int64_t covered = -1;
    if (argc == 4 && std::strcmp(argv[1], "shared") == 0) {
        covered = check_shared(std::atoll(argv[2]), std::atoll(argv[3]));
    } else if (argc >= 3 && std::strcmp(argv[1], "csr") == 0) {
        std::vector<int64_t> lens;
        for (int i = 2; i < argc; ++i) lens.push_back(std::atoll(argv[i]));
        covered = check_csr(lens);
    } else {
        std::fprintf(stderr, "usage: gl_index_check shared N_SETS N_TIMES | csr LEN...\n");
        return 2;
    }
    if (fails) {
        std::printf("%d violations\n", fails);
        return 1;
    }
    std::printf("ok %lld\n", (long long)covered);
    return 0;
}
