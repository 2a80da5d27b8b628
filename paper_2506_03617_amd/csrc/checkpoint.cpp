// The learned stage's checkpoint file, host side only (no HIP): the 8-byte
// tag below, int32 layer count, int32 channel counts (layers + 1), int64
// parameter count, int64 Adam step, then the parameters and the two Adam
// moments as float, all little-endian.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "mxp_internal.h"

namespace mxp {

static const char kCkptTag[8] = {'M', 'X', 'P', 'C', 'N', 'N', '0', '1'};

void write_checkpoint(const char* path, int32_t layers, const int32_t* channels, int64_t nparam, int64_t adam_t,
                      const std::vector<float>& buf) {
    if (!path) fail(MXP_ERR_INVALID_ARG, "path is NULL");
    if (nparam < 0 || buf.size() != 3 * size_t(nparam)) fail(MXP_ERR_INVALID_ARG, "checkpoint buffer size");
    std::unique_ptr<FILE, int (*)(FILE*)> f(std::fopen(path, "wb"), &std::fclose);
    if (!f) fail(MXP_ERR_INVALID_ARG, std::string("cannot open ") + path + " for writing");
    bool ok = std::fwrite(kCkptTag, 1, 8, f.get()) == 8 && std::fwrite(&layers, 4, 1, f.get()) == 1 &&
              std::fwrite(channels, 4, size_t(layers) + 1, f.get()) == size_t(layers) + 1 &&
              std::fwrite(&nparam, 8, 1, f.get()) == 1 && std::fwrite(&adam_t, 8, 1, f.get()) == 1 &&
              std::fwrite(buf.data(), 4, buf.size(), f.get()) == buf.size();
    ok = (std::fclose(f.release()) == 0) && ok;
    if (!ok) fail(MXP_ERR_INVALID_ARG, std::string("write to ") + path + " failed");
}

void read_checkpoint(const char* path, int32_t layers, const int32_t* channels, int64_t nparam, int64_t* adam_t,
                     std::vector<float>* buf) {
    if (!path || !adam_t || !buf) fail(MXP_ERR_INVALID_ARG, "NULL argument");
    std::unique_ptr<FILE, int (*)(FILE*)> f(std::fopen(path, "rb"), &std::fclose);
    if (!f) fail(MXP_ERR_INVALID_ARG, std::string("cannot open ") + path);
    char tag[8];
    int32_t got_layers = 0;
    int64_t np = 0, t = 0;
    if (std::fread(tag, 1, 8, f.get()) != 8 || std::memcmp(tag, kCkptTag, 8) != 0)
        fail(MXP_ERR_INVALID_ARG, "not a network checkpoint");
    if (std::fread(&got_layers, 4, 1, f.get()) != 1 || got_layers != layers)
        fail(MXP_ERR_INVALID_ARG, "checkpoint holds another architecture");
    std::vector<int32_t> ch(size_t(layers) + 1);
    if (std::fread(ch.data(), 4, ch.size(), f.get()) != ch.size() ||
        std::memcmp(ch.data(), channels, ch.size() * 4) != 0)
        fail(MXP_ERR_INVALID_ARG, "checkpoint holds another architecture");
    if (std::fread(&np, 8, 1, f.get()) != 1 || np != nparam || std::fread(&t, 8, 1, f.get()) != 1 || t < 0)
        fail(MXP_ERR_INVALID_ARG, "checkpoint header is inconsistent");
    const size_t n = size_t(np);
    std::vector<float> data(3 * n);
    if (std::fread(data.data(), 4, data.size(), f.get()) != data.size() || std::fgetc(f.get()) != EOF)
        fail(MXP_ERR_INVALID_ARG, "checkpoint has the wrong length");
    for (size_t k = 0; k < data.size(); ++k)
        if (!std::isfinite(data[k]) || (k >= 2 * n && data[k] < 0.0f))
            fail(MXP_ERR_NONFINITE, "checkpoint holds a non-finite parameter or moment");
    *adam_t = t;
    buf->swap(data);
}

}  // namespace mxp
