// gl_io.cpp -- host-side file format of a trained surrogate: the network's
// packed FP32 parameters, the calibrated per-bin error-bound table and the
// per-bin predictor choice.  No device code; the file functions can run on a
// machine without a GPU.
//
// Layout (little-endian): a 32-byte header {magic "GLSURR01", version,
// input width, hidden width, parameter count, bin count, reserved}, then
// float32 parameters[n_params], float32 table[n_bins], uint8 zero_bins[n_bins],
// then the 64-bit FNV-1a hash of everything before it.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "gl.h"

namespace {

constexpr char kMagic[8] = {'G', 'L', 'S', 'U', 'R', 'R', '0', '1'};
constexpr int32_t kVersion = 1;

struct Header {
    char magic[8];
    int32_t version, d_in, width, n_params, n_bins, reserved;
};
static_assert(sizeof(Header) == 32, "header layout");

uint64_t fnv1a(const unsigned char* p, size_t n, uint64_t h = 0xcbf29ce484222325ull)
{
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

}  // namespace

extern "C" {

gl_status gl_surrogate_save(const char* path, const float* params, int64_t n_params, const float* table,
                            const uint8_t* zero_bins, int n_bins)
{
    if (!path || !params || !table) return GL_ERR_NULL;
    if (n_params != gl_mlp_num_params() || n_bins != gl_surrogate_num_bins()) return GL_ERR_SIZE;
    Header h{};
    std::memcpy(h.magic, kMagic, sizeof(kMagic));
    h.version = kVersion;
    h.d_in = GL_MLP_DIN;
    h.width = GL_MLP_WIDTH;
    h.n_params = (int32_t)n_params;
    h.n_bins = n_bins;
    std::vector<unsigned char> buf(sizeof(Header) + sizeof(float) * (size_t)(n_params + n_bins) + (size_t)n_bins);
    unsigned char* q = buf.data();
    std::memcpy(q, &h, sizeof(h));
    q += sizeof(h);
    std::memcpy(q, params, sizeof(float) * (size_t)n_params);
    q += sizeof(float) * (size_t)n_params;
    std::memcpy(q, table, sizeof(float) * (size_t)n_bins);
    q += sizeof(float) * (size_t)n_bins;
    if (zero_bins) std::memcpy(q, zero_bins, (size_t)n_bins);
    else std::memset(q, 0, (size_t)n_bins);
    const uint64_t sum = fnv1a(buf.data(), buf.size());
    FILE* f = std::fopen(path, "wb");
    if (!f) return GL_ERR_STATE;
    const bool ok = std::fwrite(buf.data(), 1, buf.size(), f) == buf.size() &&
                    std::fwrite(&sum, sizeof(sum), 1, f) == 1;
    const bool closed = std::fclose(f) == 0;
    return ok && closed ? GL_OK : GL_ERR_STATE;
}

gl_status gl_surrogate_load(const char* path, float* params, int64_t n_params, float* table,
                            uint8_t* zero_bins, int n_bins)
{
    if (!path || !params || !table) return GL_ERR_NULL;
    if (n_params != gl_mlp_num_params() || n_bins != gl_surrogate_num_bins()) return GL_ERR_SIZE;
    FILE* f = std::fopen(path, "rb");
    if (!f) return GL_ERR_STATE;
    const size_t body = sizeof(Header) + sizeof(float) * (size_t)(n_params + n_bins) + (size_t)n_bins;
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
    std::memcpy(params, q, sizeof(float) * (size_t)n_params);
    q += sizeof(float) * (size_t)n_params;
    std::memcpy(table, q, sizeof(float) * (size_t)n_bins);
    q += sizeof(float) * (size_t)n_bins;
    if (zero_bins) std::memcpy(zero_bins, q, (size_t)n_bins);
    return GL_OK;
}

}  // extern "C"
