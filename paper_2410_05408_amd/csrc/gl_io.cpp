// gl_io.cpp -- host-side file format of a trained surrogate: its training
// configuration, the network's packed FP32 parameters and Adam state, the
// calibrated per-bin error-bound table, the per-bin predictor choice and the
// calibration counts.  No device code: the file functions also run on a
// machine without a GPU.
//
// Layout (little-endian): a 32-byte header {magic "GLSURR02", version,
// input width, hidden width, parameter count, bin count, reserved}, a 64-byte
// configuration block, float32 parameters[n_params], float32 m[n_params],
// float32 v[n_params], int64 step, float32 table[n_bins], uint8
// zero_bins[n_bins], int32 counts[n_bins], then the 64-bit FNV-1a hash of
// everything before it.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "gl.h"

namespace {

constexpr char kMagic[8] = {'G', 'L', 'S', 'U', 'R', 'R', '0', '2'};
constexpr int32_t kVersion = 2;

struct Header {
    char magic[8];
    int32_t version, d_in, width, n_params, n_bins, reserved;
};
static_assert(sizeof(Header) == 32, "header layout");

// the configuration, field by field (no padding)
struct CfgBlock {
    int64_t n_train, n_calib;
    int32_t epochs, batch;
    float lr, lr_final;
    double safety, window;
    uint64_t seed;
    int32_t min_bin_count, zero_predictor;
};
static_assert(sizeof(CfgBlock) == 64, "configuration block layout");

uint64_t fnv1a(const unsigned char* p, size_t n, uint64_t h = 0xcbf29ce484222325ull)
{
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

size_t body_bytes(int64_t n_params, int n_bins)
{
    return sizeof(Header) + sizeof(CfgBlock) + 3 * sizeof(float) * (size_t)n_params + sizeof(int64_t) +
           (sizeof(float) + 1 + sizeof(int32_t)) * (size_t)n_bins;
}

}  // namespace

extern "C" {

gl_status gl_surrogate_file_write(const char* path, const gl_surrogate_config* cfg, const float* params,
                                  const float* m, const float* v, int64_t step, int64_t n_params,
                                  const float* table, const uint8_t* zero_bins, const int32_t* counts, int n_bins)
{
    if (!path || !cfg || !params || !m || !v || !table || !zero_bins || !counts) return GL_ERR_NULL;
    if (n_params != gl_mlp_num_params() || n_bins != gl_surrogate_num_bins()) return GL_ERR_SIZE;
    Header h{};
    std::memcpy(h.magic, kMagic, sizeof(kMagic));
    h.version = kVersion;
    h.d_in = GL_MLP_DIN;
    h.width = GL_MLP_WIDTH;
    h.n_params = (int32_t)n_params;
    h.n_bins = n_bins;
    const CfgBlock c{cfg->n_train, cfg->n_calib, cfg->epochs, cfg->batch, cfg->lr, cfg->lr_final,
                     cfg->safety, cfg->window, cfg->seed, cfg->min_bin_count, cfg->zero_predictor};
    std::vector<unsigned char> buf(body_bytes(n_params, n_bins));
    unsigned char* q = buf.data();
    auto put = [&q](const void* src, size_t n) {
        std::memcpy(q, src, n);
        q += n;
    };
    put(&h, sizeof(h));
    put(&c, sizeof(c));
    put(params, sizeof(float) * (size_t)n_params);
    put(m, sizeof(float) * (size_t)n_params);
    put(v, sizeof(float) * (size_t)n_params);
    put(&step, sizeof(step));
    put(table, sizeof(float) * (size_t)n_bins);
    put(zero_bins, (size_t)n_bins);
    put(counts, sizeof(int32_t) * (size_t)n_bins);
    const uint64_t sum = fnv1a(buf.data(), buf.size());
    FILE* f = std::fopen(path, "wb");
    if (!f) return GL_ERR_STATE;
    const bool ok = std::fwrite(buf.data(), 1, buf.size(), f) == buf.size() &&
                    std::fwrite(&sum, sizeof(sum), 1, f) == 1;
    const bool closed = std::fclose(f) == 0;
    return ok && closed ? GL_OK : GL_ERR_STATE;
}

gl_status gl_surrogate_file_read(const char* path, gl_surrogate_config* cfg, float* params, float* m, float* v,
                                 int64_t* step, int64_t n_params, float* table, uint8_t* zero_bins, int32_t* counts,
                                 int n_bins)
{
    if (!path || !cfg || !params || !m || !v || !step || !table || !zero_bins || !counts) return GL_ERR_NULL;
    if (n_params != gl_mlp_num_params() || n_bins != gl_surrogate_num_bins()) return GL_ERR_SIZE;
    FILE* f = std::fopen(path, "rb");
    if (!f) return GL_ERR_STATE;
    const size_t body = body_bytes(n_params, n_bins);
    std::vector<unsigned char> buf(body + sizeof(uint64_t) + 1);
    const size_t got = std::fread(buf.data(), 1, buf.size(), f);
    std::fclose(f);
    if (got < sizeof(Header)) return GL_ERR_STATE;
    Header h;
    std::memcpy(&h, buf.data(), sizeof(h));
    if (std::memcmp(h.magic, kMagic, sizeof(kMagic)) != 0 || h.version != kVersion) return GL_ERR_STATE;
    if (h.d_in != GL_MLP_DIN || h.width != GL_MLP_WIDTH || h.n_params != n_params || h.n_bins != n_bins)
        return GL_ERR_SIZE;
    if (got != body + sizeof(uint64_t)) return GL_ERR_STATE;  // truncated or trailing bytes
    uint64_t sum;
    std::memcpy(&sum, buf.data() + body, sizeof(sum));
    if (sum != fnv1a(buf.data(), body)) return GL_ERR_STATE;
    const unsigned char* q = buf.data() + sizeof(Header);
    auto get = [&q](void* dst, size_t n) {
        std::memcpy(dst, q, n);
        q += n;
    };
    CfgBlock c;
    get(&c, sizeof(c));
    get(params, sizeof(float) * (size_t)n_params);
    get(m, sizeof(float) * (size_t)n_params);
    get(v, sizeof(float) * (size_t)n_params);
    get(step, sizeof(*step));
    get(table, sizeof(float) * (size_t)n_bins);
    get(zero_bins, (size_t)n_bins);
    get(counts, sizeof(int32_t) * (size_t)n_bins);
    *cfg = gl_surrogate_config{c.n_train, c.n_calib, c.epochs, c.batch, c.lr, c.lr_final, c.safety,
                               c.min_bin_count, c.window, c.seed, c.zero_predictor};
    return GL_OK;
}

}  // extern "C"
