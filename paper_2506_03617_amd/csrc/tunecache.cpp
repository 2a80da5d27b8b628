// On-disk cache of autotuned tile configurations (host only).  The file is a
// JSON object whose members map a configuration key to [K, NX, Ly, us], the
// kernel shape and its measured microseconds per Clenshaw level:
//
//   {
//    "matexpre-mi355x 0.1.0|gfx950|2d 2048x2048x1|c64|D|pml": [4, 1, 25, 11.7],
//    ...
//   }
//
// Keys hold no quotes or backslashes.  A file that does not parse is treated
// as empty and never overwritten; an update rewrites the whole file through a
// temporary and a rename, so a reader never sees half a file.
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "mxp_internal.h"

namespace mxp {
namespace {

std::mutex g_cache_mu;

struct Entry {
    int v[3];
    double us;
};

bool read_file(const char* path, std::string* out, bool* missing) {
    *missing = false;
    FILE* f = std::fopen(path, "rb");
    if (!f) {
        *missing = (errno == ENOENT);
        return false;
    }
    char buf[4096];
    size_t k;
    out->clear();
    while ((k = std::fread(buf, 1, sizeof(buf), f)) > 0) {
        out->append(buf, k);
        if (out->size() > (size_t(16) << 20)) {  // not a cache this library wrote
            std::fclose(f);
            return false;
        }
    }
    const bool ok = !std::ferror(f);
    std::fclose(f);
    return ok;
}

// Parses the whole text; false on any deviation from the format above.
bool parse(const std::string& s, std::map<std::string, Entry>* out) {
    size_t i = 0;
    auto ws = [&]() {
        while (i < s.size() && (s[i] == ' ' || s[i] == '\n' || s[i] == '\r' || s[i] == '\t')) ++i;
    };
    auto number = [&](double* v) {
        ws();
        if (i >= s.size()) return false;
        const char* b = s.c_str() + i;
        char* e = nullptr;
        *v = std::strtod(b, &e);
        if (e == b) return false;
        i += size_t(e - b);
        return true;
    };
    ws();
    if (i >= s.size() || s[i] != '{') return false;
    ++i;
    ws();
    if (i < s.size() && s[i] == '}') return true;
    while (true) {
        ws();
        if (i >= s.size() || s[i] != '"') return false;
        const size_t q = s.find('"', i + 1);
        if (q == std::string::npos) return false;
        std::string key = s.substr(i + 1, q - i - 1);
        if (key.find('\\') != std::string::npos) return false;
        i = q + 1;
        ws();
        if (i >= s.size() || s[i] != ':') return false;
        ++i;
        ws();
        if (i >= s.size() || s[i] != '[') return false;
        ++i;
        double d[4];
        for (int k = 0; k < 4; ++k) {
            if (!number(&d[k])) return false;
            ws();
            if (i >= s.size() || s[i] != (k < 3 ? ',' : ']')) return false;
            ++i;
        }
        Entry e;
        for (int k = 0; k < 3; ++k) {
            if (!(d[k] >= -1e6 && d[k] <= 1e6) || d[k] != double(int(d[k]))) return false;
            e.v[k] = int(d[k]);
        }
        if (!(d[3] >= 0.0) || !(d[3] < 1e12)) return false;
        e.us = d[3];
        (*out)[key] = e;
        ws();
        if (i >= s.size()) return false;
        if (s[i] == ',') {
            ++i;
            continue;
        }
        if (s[i] != '}') return false;
        ++i;
        ws();
        return i == s.size();
    }
}

}  // namespace

bool tune_cache_get(const char* path, const std::string& key, int v[3], double* us) {
    if (!path || !*path) return false;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    std::string text;
    bool missing = false;
    if (!read_file(path, &text, &missing)) return false;
    std::map<std::string, Entry> m;
    if (!parse(text, &m)) return false;
    const auto it = m.find(key);
    if (it == m.end()) return false;
    for (int k = 0; k < 3; ++k) v[k] = it->second.v[k];
    *us = it->second.us;
    return true;
}

bool tune_cache_put(const char* path, const std::string& key, const int v[3], double us) {
    if (!path || !*path) return false;
    if (key.find('"') != std::string::npos || key.find('\\') != std::string::npos) return false;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    std::string text;
    bool missing = false;
    std::map<std::string, Entry> m;
    if (read_file(path, &text, &missing)) {
        if (!parse(text, &m)) return false;  // someone else's file: leave it alone
    } else if (!missing) {
        return false;
    }
    Entry e;
    for (int k = 0; k < 3; ++k) e.v[k] = v[k];
    e.us = us;
    m[key] = e;
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return false;
    bool ok = std::fputs("{\n", f) >= 0;
    size_t k = 0;
    for (const auto& kv : m) {
        ok = ok && std::fprintf(f, " \"%s\": [%d, %d, %d, %.6g]%s\n", kv.first.c_str(), kv.second.v[0],
                                kv.second.v[1], kv.second.v[2], kv.second.us, ++k < m.size() ? "," : "") > 0;
    }
    ok = ok && std::fputs("}\n", f) >= 0;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return false;
    }
    return true;
}

}  // namespace mxp
