// Host code of the library run under AddressSanitizer and UndefinedBehaviour
// Sanitizer (built by tests/test_host_sanitizers.py with g++, no GPU): the grid
// checks, the field-of-values box and schedule design for every absorber in
// both precisions, the psi_2 series, the dense exponential, the checkpoint
// reader on valid, truncated, corrupted and non-finite files, and the
// autotuner cache on round trips and on malformed files.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../paper_2506_03617_amd/csrc/mxp_internal.h"

using namespace mxp;

static int failures = 0;
#define CHECK(cond, what)                                                     \
    do {                                                                      \
        if (!(cond)) {                                                        \
            std::printf("FAILED: %s (line %d)\n", what, __LINE__);            \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

static mxp_grid_desc grid(int dim, int64_t n, int layer, int absorber) {
    mxp_grid_desc d;
    std::memset(&d, 0, sizeof(d));
    d.dim = dim;
    d.n[0] = n;
    d.n[1] = n - 3;
    d.n[2] = dim == 3 ? n - 5 : 1;
    d.h = 1.0 / double(n - 1);
    d.omega = 2.0 * M_PI / (8.0 * d.h);
    for (int a = 0; a < 3; ++a) d.layer[a][0] = d.layer[a][1] = (a < dim) ? layer : 0;
    d.pml_C = 20.0;
    d.pml_power = 2;
    d.c = nullptr;
    d.c_const = 1.0;
    d.absorber = absorber;
    if (absorber == MXP_ABSORB_ABC) d.hard[dim - 1][0] = 1;
    return d;
}

static mxp_status status_of(void (*fn)(const mxp_grid_desc*), const mxp_grid_desc* d) {
    try {
        fn(d);
        return MXP_OK;
    } catch (const Error& e) {
        return e.status;
    }
}

int main(int argc, char** argv) {
    const std::string dir = argc > 1 ? argv[1] : ".";
    // grid checks: every bound rejected before anything else happens
    {
        auto validate = [](const mxp_grid_desc* d) { (void)validate_grid(d); };
        mxp_grid_desc d = grid(2, 40, 6, MXP_ABSORB_PML);
        CHECK(status_of(validate, &d) == MXP_OK, "valid grid");
        d.n[0] = 2;
        CHECK(status_of(validate, &d) == MXP_ERR_INVALID_ARG, "short axis");
        d = grid(2, 40, 20, MXP_ABSORB_PML);
        CHECK(status_of(validate, &d) == MXP_ERR_INVALID_ARG, "layer too wide");
        d = grid(3, 40, 4, MXP_ABSORB_ABC);
        CHECK(status_of(validate, &d) == MXP_ERR_INVALID_ARG, "layer with boundary conditions");
        d = grid(2, 40, 6, 7);
        CHECK(status_of(validate, &d) == MXP_ERR_INVALID_ARG, "unknown absorber");
        d = grid(2, 40, 6, MXP_ABSORB_PML);
        d.h = -1.0;
        CHECK(status_of(validate, &d) == MXP_ERR_INVALID_ARG, "negative h");
        d = grid(2, 40, 6, MXP_ABSORB_PML);
        d.c_const = std::nan("");
        CHECK(status_of(validate, &d) == MXP_ERR_INVALID_ARG, "NaN speed");
        CHECK(status_of(validate, nullptr) == MXP_ERR_INVALID_ARG, "NULL description");
        std::vector<double> c(40 * 37, 1.5);
        c[17] = 0.0;
        double lo = 0, hi = 0;
        bool threw = false;
        try {
            speed_range_host(c.data(), MXP_F64, int64_t(c.size()), &lo, &hi);
        } catch (const Error&) {
            threw = true;
        }
        CHECK(threw, "zero speed rejected");
    }
    // schedules for every absorber, dimension and precision, and the psi_2 series
    for (int absorber : {MXP_ABSORB_PML, MXP_ABSORB_CAP, MXP_ABSORB_ABC}) {
        for (int dim : {2, 3}) {
            const int layer = absorber == MXP_ABSORB_ABC ? 0 : (absorber == MXP_ABSORB_CAP && dim == 2 ? 12 : 6);
            mxp_grid_desc d = grid(dim, dim == 2 ? 64 : 28, layer, absorber);
            GridInfo g = validate_grid(&d);
            for (mxp_precision prec : {MXP_PREC_FP64, MXP_PREC_MIXED}) {
                mxp_schedule sc;
                try {
                    design_schedule(g, 40.0 * d.h * d.h, 0.05, prec, &sc);
                } catch (const Error& e) {
                    // the potential in complex float may be refused (box too tall)
                    CHECK(absorber == MXP_ABSORB_CAP && e.status == MXP_ERR_UNSUPPORTED, e.what());
                    continue;
                }
                CHECK(sc.S > 0 && sc.m >= 3 && sc.m_psi >= 1, "schedule shape");
                CHECK(std::isfinite(sc.trunc_bound) && sc.box[0] < sc.box[1] && sc.box[2] <= sc.box[3], "box");
                std::vector<double> coef;
                int m2 = -1;
                design_psi2_series(sc, 40.0 * d.h * d.h, prec, &coef, &m2);
                CHECK(m2 >= 1 && coef.size() == 2 * size_t(m2 + 1), "psi_2 series");
            }
        }
    }
    // dense exponential: exp(A) exp(-A) = I for a random complex matrix
    {
        const int n = 24;
        std::vector<cd> A(n * n), B(n * n), P(n * n);
        unsigned s = 12345;
        for (auto& v : A) {
            s = s * 1103515245u + 12345u;
            const double re = double((s >> 8) & 0xffff) / 65536.0 - 0.5;
            s = s * 1103515245u + 12345u;
            const double im = double((s >> 8) & 0xffff) / 65536.0 - 0.5;
            v = cd(3.0 * re, 3.0 * im);
        }
        for (int i = 0; i < n * n; ++i) B[i] = -A[i];
        expm_dense(n, A);
        expm_dense(n, B);
        double err = 0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                cd acc = 0;
                for (int k = 0; k < n; ++k) acc += A[i * n + k] * B[k * n + j];
                err = std::max(err, std::abs(acc - (i == j ? 1.0 : 0.0)));
            }
        CHECK(err < 1e-10, "exp(A) exp(-A) = I");
    }
    // checkpoints
    {
        const int32_t layers = 3, ch[4] = {3, 8, 8, 2};
        const int64_t np = 50;
        std::vector<float> buf(3 * np);
        for (size_t k = 0; k < buf.size(); ++k) buf[k] = 0.25f * float(k % 17);
        const std::string path = dir + "/ck.bin";
        write_checkpoint(path.c_str(), layers, ch, np, 7, buf);
        std::vector<float> back;
        int64_t t = -1;
        read_checkpoint(path.c_str(), layers, ch, np, &t, &back);
        CHECK(t == 7 && back == buf, "round trip");
        auto expect_error = [&](const std::string& p, int32_t L, const int32_t* c, int64_t n, mxp_status want,
                                const char* what) {
            std::vector<float> b;
            int64_t tt = 0;
            mxp_status got = MXP_OK;
            try {
                read_checkpoint(p.c_str(), L, c, n, &tt, &b);
            } catch (const Error& e) {
                got = e.status;
            }
            CHECK(got == want, what);
        };
        const int32_t other[4] = {3, 8, 4, 2};
        expect_error(path, layers, other, np, MXP_ERR_INVALID_ARG, "other architecture");
        expect_error(path, layers, ch, np + 1, MXP_ERR_INVALID_ARG, "other parameter count");
        expect_error(dir + "/missing.bin", layers, ch, np, MXP_ERR_INVALID_ARG, "missing file");
        // truncated and overlong copies, a corrupted tag and a NaN parameter
        FILE* f = std::fopen(path.c_str(), "rb");
        std::vector<char> raw;
        for (int c; (c = std::fgetc(f)) != EOF;) raw.push_back(char(c));
        std::fclose(f);
        auto write_raw = [&](const std::string& p, const std::vector<char>& data) {
            FILE* g = std::fopen(p.c_str(), "wb");
            if (!data.empty()) std::fwrite(data.data(), 1, data.size(), g);
            std::fclose(g);
        };
        for (size_t cut : {size_t(0), size_t(5), size_t(12), size_t(40), raw.size() - 1}) {
            write_raw(dir + "/cut.bin", std::vector<char>(raw.begin(), raw.begin() + long(cut)));
            expect_error(dir + "/cut.bin", layers, ch, np, MXP_ERR_INVALID_ARG, "truncated file");
        }
        std::vector<char> longer = raw;
        longer.push_back('x');
        write_raw(dir + "/long.bin", longer);
        expect_error(dir + "/long.bin", layers, ch, np, MXP_ERR_INVALID_ARG, "overlong file");
        std::vector<char> tagged = raw;
        tagged[3] = 'Z';
        write_raw(dir + "/tag.bin", tagged);
        expect_error(dir + "/tag.bin", layers, ch, np, MXP_ERR_INVALID_ARG, "corrupted tag");
        std::vector<float> bad = buf;
        bad[9] = std::nanf("");
        write_checkpoint((dir + "/nan.bin").c_str(), layers, ch, np, 7, bad);
        expect_error(dir + "/nan.bin", layers, ch, np, MXP_ERR_NONFINITE, "NaN parameter");
    }
    // the autotuner's on-disk cache
    {
        const std::string path = dir + "/tiles.json";
        std::remove(path.c_str());
        int v[3] = {0, 0, 0};
        double us = 0.0;
        CHECK(!tune_cache_get(path.c_str(), "a", v, &us), "missing cache file reads as empty");
        CHECK(!tune_cache_get(nullptr, "a", v, &us) && !tune_cache_get("", "a", v, &us), "no cache path");
        const int a[3] = {4, 1, 25}, b[3] = {2, 1, 32}, c[3] = {6, 2, 8};
        CHECK(tune_cache_put(path.c_str(), "v|gfx950|2d 2048x2048x1|c64|D|absorber 0", a, 11.7), "first put");
        CHECK(tune_cache_put(path.c_str(), "v|gfx950|3d 256x256x256|c128|c|absorber 0", b, 171.8), "second put");
        CHECK(tune_cache_put(path.c_str(), "v|gfx950|2d 2048x2048x1|c64|D|absorber 0", c, 9.5), "replace");
        CHECK(!tune_cache_put(path.c_str(), "bad\"key", a, 1.0), "key with a quote refused");
        CHECK(tune_cache_get(path.c_str(), "v|gfx950|3d 256x256x256|c128|c|absorber 0", v, &us) && v[0] == 2 &&
                  v[1] == 1 && v[2] == 32 && std::fabs(us - 171.8) < 1e-9,
              "round trip");
        CHECK(tune_cache_get(path.c_str(), "v|gfx950|2d 2048x2048x1|c64|D|absorber 0", v, &us) && v[0] == 6 &&
                  v[1] == 2 && v[2] == 8,
              "replaced entry");
        CHECK(!tune_cache_get(path.c_str(), "absent", v, &us), "absent key");
        // malformed or foreign files: read as empty and never overwritten
        const char* bad[] = {"", "{", "[1, 2]", "{\"k\": [1, 2, 3]}", "{\"k\": [1, 2, 3, 4, 5]}",
                             "{\"k\": [1.5, 2, 3, 4]}", "{\"k\": [1, 2, 3, -4]}", "{\"k\": [1, 2, 3, 4]} x",
                             "{\"k\" [1, 2, 3, 4]}", "{\"k\": [1, 2, 3, 4],}", "{\"k\": [1, 2, 3, nan]}",
                             "{\"k\": [1e300, 2, 3, 4]}", "{\"k\\\": [1, 2, 3, 4]}"};
        for (const char* text : bad) {
            const std::string bp = dir + "/bad.json";
            FILE* f = std::fopen(bp.c_str(), "wb");
            if (f) {
                if (*text) std::fwrite(text, 1, std::strlen(text), f);
                std::fclose(f);
            }
            CHECK(!tune_cache_get(bp.c_str(), "k", v, &us), "malformed cache reads as empty");
            CHECK(!tune_cache_put(bp.c_str(), "k", a, 1.0), "malformed cache not overwritten");
            FILE* g = std::fopen(bp.c_str(), "rb");
            std::string back;
            if (g) {
                char chunk[256];
                size_t k;
                while ((k = std::fread(chunk, 1, sizeof(chunk), g)) > 0) back.append(chunk, k);
                std::fclose(g);
            }
            CHECK(back == text, "malformed cache left as it was");
        }
        {
            const std::string ep = dir + "/empty_obj.json";
            FILE* f = std::fopen(ep.c_str(), "wb");
            if (f) {
                std::fputs(" { } \n", f);
                std::fclose(f);
            }
            CHECK(!tune_cache_get(ep.c_str(), "k", v, &us), "empty object has no key");
            CHECK(tune_cache_put(ep.c_str(), "k", a, 2.5) && tune_cache_get(ep.c_str(), "k", v, &us) && v[2] == 25,
                  "empty object takes a first entry");
        }
    }
    if (failures == 0) std::printf("all host checks passed\n");
    return failures == 0 ? 0 : 1;
}
