// Set-up tables, Chebyshev schedules and the matrix-function actions
// exp(i t A_s) x, psi_1(i t A_s) x and psi_2(i t A_s) x (paper Section 3.1,
// Def. psi, eq. inverse-1), with the complex shift of Section 3.4.
//
//   t psi_1(i t A) r = sum_{k<S} exp(i k tau A) tau psi_1(i tau A) r, tau = t/S
// (semigroup property plus the variation-of-constants integral); every
// series is evaluated by the Clenshaw recurrence on stencil sweeps (3D) or
// temporally blocked passes (2D).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "engine.h"

namespace mxp {

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

size_t diag_table_bytes(const GridInfo& g) {
    const size_t total = size_t(g.n[0] + g.n[1] + g.n[2]);
    const size_t tot2 = g.dim == 2 ? 3 * size_t(g.n[0] + g.n[1]) : 0;
    return align256(total * sizeof(cpx<double>)) + align256(total * sizeof(cpx<float>)) +
           align256(tot2 * sizeof(cpx<double>)) + align256(tot2 * sizeof(cpx<float>));
}

// The diagonal tables of one (shift, centre) pair.  They go to buffers the
// tables own (ext == nullptr), or to `ext`, a device region of at least
// diag_table_bytes(P->g) bytes that the caller owns, uploaded on stream s.
void build_diag(mxp_problem* P, double shift, cd centre, DiagTables& dt, void* ext, hipStream_t s) {
    const GridInfo& g = P->g;
    size_t ext_off = 0;
    auto place = [&](DevMem& dm, const void* src, size_t bytes) -> void* {
        if (!ext) {
            dm.ensure(bytes);
            HIP_CHECK(hipMemcpy(dm.p, src, bytes, hipMemcpyHostToDevice));
            return dm.p;
        }
        void* p = static_cast<unsigned char*>(ext) + ext_off;
        ext_off += align256(bytes);
        HIP_CHECK(hipMemcpyAsync(p, src, bytes, hipMemcpyHostToDevice, s));
        return p;
    };
    const cd share = (cd(g.omega * g.omega, g.omega * g.omega * shift) * P->Dref - centre) / double(g.dim);
    size_t total = 0;
    for (int d = 0; d < 3; ++d) total += size_t(g.n[d]);
    std::vector<cpx<double>> h64(total);
    std::vector<cpx<float>> h32(total);
    size_t off = 0, offs[3];
    for (int d = 0; d < 3; ++d) {
        offs[d] = off;
        if (d < g.dim) {
            const AxisTables at = build_axis_tables(g.axis(d));
            for (int64_t i = 0; i < g.n[d]; ++i) {
                const cd v = at.gamma[i] + share;
                h64[off + i] = {v.real(), v.imag()};
                h32[off + i] = {float(v.real()), float(v.imag())};
            }
        } else {
            for (int64_t i = 0; i < g.n[d]; ++i) {
                h64[off + i] = {0.0, 0.0};
                h32[off + i] = {0.0f, 0.0f};
            }
        }
        off += g.n[d];
    }
    // Interior box: a node needs alpha = beta = 1/h^2 on its axis, i.e. the
    // stretch is 1 at the node and both half-nodes (everywhere with the
    // absorbing potential, which sits in the diagonal).  Nodes 0 and n-1 are
    // excluded so that every neighbour read stays inside the grid there.
    auto span = [&](int d, int64_t* lo, int64_t* hi) {
        const AxisLayer ax = g.axis(d);
        int64_t a0 = 1, a1 = g.n[d] - 1;
        while (a0 < a1 && (ax.stretch(a0 * g.h) != 0.0 || ax.stretch((a0 - 0.5) * g.h) != 0.0 ||
                           ax.stretch((a0 + 0.5) * g.h) != 0.0))
            ++a0;
        while (a1 > a0 && (ax.stretch((a1 - 1) * g.h) != 0.0 || ax.stretch((a1 - 0.5) * g.h) != 0.0 ||
                           ax.stretch((a1 - 1.5) * g.h) != 0.0))
            --a1;
        *lo = a0;
        *hi = a1;
    };
    if (g.dim == 2) {
        span(0, &dt.ix0, &dt.ix1);
        span(1, &dt.iy0, &dt.iy1);
        if (!(dt.ix0 < dt.ix1 && dt.iy0 < dt.iy1)) dt.ix0 = dt.ix1 = dt.iy0 = dt.iy1 = 0;
        const double h2 = g.h * g.h;
        const size_t tot2 = 3 * size_t(g.n[0] + g.n[1]);
        std::vector<cpx<double>> s64(tot2);
        std::vector<cpx<float>> s32(tot2);
        size_t o = 0, fo[2][3];
        for (int d = 0; d < 2; ++d) {
            const AxisTables at = build_axis_tables(g.axis(d));
            const std::vector<cd>* src[3] = {&at.alpha, &at.beta, &at.gamma};
            for (int q = 0; q < 3; ++q) {
                fo[d][q] = o;
                for (int64_t i = 0; i < g.n[d]; ++i) {
                    const cd v = ((*src[q])[i] + (q == 2 ? share : cd(0.0, 0.0))) * h2;
                    s64[o + i] = {v.real(), v.imag()};
                    s32[o + i] = {float(v.real()), float(v.imag())};
                }
                o += g.n[d];
            }
        }
        cpx<double>* f64 = static_cast<cpx<double>*>(place(dt.fmem64, s64.data(), tot2 * sizeof(cpx<double>)));
        cpx<float>* f32 = static_cast<cpx<float>*>(place(dt.fmem32, s32.data(), tot2 * sizeof(cpx<float>)));
        for (int d = 0; d < 2; ++d)
            for (int q = 0; q < 3; ++q) {
                dt.f64[d][q] = f64 + fo[d][q];
                dt.f32[d][q] = f32 + fo[d][q];
            }
    }
    cpx<double>* m64 = static_cast<cpx<double>*>(place(dt.mem64, h64.data(), total * sizeof(cpx<double>)));
    cpx<float>* m32 = static_cast<cpx<float>*>(place(dt.mem32, h32.data(), total * sizeof(cpx<float>)));
    for (int d = 0; d < 3; ++d) {
        dt.g64[d] = m64 + offs[d];
        dt.g32[d] = m32 + offs[d];
    }
    // the host tables go out of scope: the copies must have read them
    if (ext) HIP_CHECK(hipStreamSynchronize(s));
}

const DiagTables& plain_diag(mxp_problem* P, double shift) {
    auto it = P->plain_diag.find(shift);
    if (it != P->plain_diag.end()) return *it->second;
    auto dt = std::make_unique<DiagTables>();
    build_diag(P, shift, cd(0.0, 0.0), *dt, nullptr, nullptr);
    const DiagTables& ref = *dt;
    P->plain_diag.emplace(shift, std::move(dt));
    return ref;
}

const Sched& get_sched(mxp_problem* P, double t, double shift, mxp_precision prec,
                              int forceS, int forcem) {
    auto key = std::make_tuple(t, shift, int(prec), forceS, forcem);
    auto it = P->scheds.find(key);
    if (it != P->scheds.end()) return *it->second;
    auto sc = std::make_unique<Sched>();
    design_schedule(P->g, t, shift, prec, &sc->s, forceS, forcem);
    build_diag(P, shift, cd(sc->s.centre_re, sc->s.centre_im), sc->diag, nullptr, nullptr);
    sc->t = t;
    sc->prec = prec;
    const Sched& ref = *sc;
    P->scheds.emplace(key, std::move(sc));
    return ref;
}

template <typename R>
static StencilArgs<R> base_args(mxp_problem* P, double shift, const DiagTables& diag) {
    StencilArgs<R> a{};
    const GridInfo& g = P->g;
    a.dim = g.dim;
    a.n0 = g.n[0];
    a.n1 = g.n[1];
    a.n2 = g.n[2];
    const DevTables<R>* t;
    if constexpr (sizeof(R) == 8) t = &P->t64; else t = &P->t32;
    for (int d = 0; d < 3; ++d) {
        a.alpha[d] = t->alpha[d];
        a.beta[d] = t->beta[d];
        a.abc[d] = t->abc[d];
        if constexpr (sizeof(R) == 8) a.gamma[d] = diag.g64[d]; else a.gamma[d] = diag.g32[d];
    }
    if (g.homogeneous) {
        a.D = nullptr;
        a.Dconst = R(P->Dref);  // D - Dref is exactly zero
    } else {
        if constexpr (sizeof(R) == 8) a.D = P->D64.as<double>(); else a.D = P->D32.as<float>();
        a.Dconst = R(0);
    }
    a.Dref = R(P->Dref);
    // 3D sweeps: z segment length fixed by mxp_set_tiles (K = 1), else chosen per grid
    const TileCfg& tc = P->tiles[sizeof(R) == 4 ? 1 : 0];
    a.zc = (g.dim == 3 && tc.K == 1) ? tc.Ly : 0;
    const double w2 = g.omega * g.omega;
    a.kD = {R(w2), R(w2 * shift)};
    a.g = {R(1), R(0)};
    a.cx = a.e2 = a.e3 = {R(0), R(0)};
    return a;
}

static cd coef_at(const double* c, int k) { return cd(c[2 * k], c[2 * k + 1]); }

// bufA, bufB: scratch distinct from x, add and out.  out may equal x.
template <typename R>
static void cheb_series(const Emit<R>& em, const StencilArgs<R>& base, const mxp_schedule& sc,
                        const double* coef, int m, const cpx<R>* x, cpx<R>* out, cpx<R>* bufA,
                        cpx<R>* bufB, cd post, const cpx<R>* add, int64_t* steps) {
    const double hw = sc.half_width;
    StencilArgs<R> a = base;  // the centre is already folded into the diagonal tables
    a.x = x;
    // b_{m-1} = c_{m-1} x + 2 Ahat (c_m x)
    a.b1 = x;
    a.g = to_cpx<R>(coef_at(coef, m) * (2.0 / hw));
    a.cx = to_cpx<R>(coef_at(coef, m - 1));
    a.b2 = nullptr;
    a.b3 = nullptr;
    a.out = bufA;
    em.sweep(a);
    // b_{m-2} = c_{m-2} x + 2 Ahat b_{m-1} - c_m x
    a.b1 = bufA;
    a.g = to_cpx<R>(cd(2.0 / hw, 0.0));
    a.cx = to_cpx<R>(coef_at(coef, m - 2) - coef_at(coef, m));
    a.out = bufB;
    em.sweep(a);
    cpx<R>* cur = bufB;   // b_{k+1}
    cpx<R>* prev = bufA;  // b_{k+2}
    for (int k = m - 3; k >= 1; --k) {
        a.b1 = cur;
        a.b2 = prev;
        a.e2 = {R(-1), R(0)};
        a.cx = to_cpx<R>(coef_at(coef, k));
        a.out = prev;
        em.sweep(a);
        std::swap(cur, prev);
    }
    // out = post * (c_0 x + Ahat b_1 - b_2 + add)
    a.b1 = cur;
    a.b2 = prev;
    a.g = to_cpx<R>(post / hw);
    a.cx = to_cpx<R>(post * coef_at(coef, 0));
    a.e2 = to_cpx<R>(-post);
    a.b3 = add;
    a.e3 = to_cpx<R>(post);
    a.out = out;
    em.sweep(a);
    *steps += m;
}

// The same series on a 3D grid with two Clenshaw levels per pass: levels
// 0 .. m-1 in pairs (level q: c_{m-q} x + (q ? 2/hw : 0) S(L_{q-1}) - L_{q-2}),
// an odd one left over and the final level (post, add) as single sweeps.
// bufs: four scratch vectors distinct from x, add and out.
template <typename R>
static void cheb_series3d(const Emit<R>& em, const StencilArgs<R>& base, const mxp_schedule& sc, const double* coef,
                          int m, const cpx<R>* x, cpx<R>* out, cpx<R>* const bufs[4], cd post, const cpx<R>* add,
                          int64_t* steps, int zc, int levels) {
    const double hw = sc.half_width;
    ChebPass3DArgs<R> a{};
    a.n0 = base.n0;
    a.n1 = base.n1;
    a.n2 = base.n2;
    for (int d = 0; d < 3; ++d) {
        a.alpha[d] = base.alpha[d];
        a.beta[d] = base.beta[d];
        a.gamma[d] = base.gamma[d];
    }
    a.D = base.D;
    a.Dconst = base.Dconst;
    a.Dref = base.Dref;
    a.kD = base.kD;
    a.x = x;
    const cpx<R>* prevA = nullptr;  // L_{q-2}
    const cpx<R>* prevB = nullptr;  // L_{q-1}
    int q = 0, pair = 0;
    if (levels == 3) {
        // levels in triples: L_q, L_{q+1}, L_{q+2}, writing the last two
        ChebPass3DArgs<R> a3 = a;
        cheb3d3_geometry<R>(a3, zc);
        while (q + 2 <= m - 1) {
            a3.cx[0] = to_cpx<R>(coef_at(coef, m - q));
            a3.g[0] = R(q == 0 ? 0.0 : 2.0 / hw);
            a3.cx[1] = to_cpx<R>(coef_at(coef, m - q - 1));
            a3.g[1] = R(2.0 / hw);
            a3.cx[2] = to_cpx<R>(coef_at(coef, m - q - 2));
            a3.g[2] = R(2.0 / hw);
            a3.in0 = prevA;
            a3.in1 = prevB;
            a3.outA = bufs[2 * pair];
            a3.outB = bufs[2 * pair + 1];
            em.pass3d3(a3);
            prevA = a3.outA;
            prevB = a3.outB;
            pair ^= 1;
            q += 3;
        }
    }
    cheb3d_geometry<R>(a, zc);
    while (q + 1 <= m - 1) {
        a.cx[0] = to_cpx<R>(coef_at(coef, m - q));
        a.g[0] = R(q == 0 ? 0.0 : 2.0 / hw);
        a.cx[1] = to_cpx<R>(coef_at(coef, m - q - 1));
        a.g[1] = R(2.0 / hw);
        a.in0 = prevA;
        a.in1 = prevB;
        a.outA = bufs[2 * pair];
        a.outB = bufs[2 * pair + 1];
        em.pass3d(a);
        prevA = a.outA;
        prevB = a.outB;
        pair ^= 1;
        q += 2;
    }
    StencilArgs<R> st = base;
    st.x = x;
    if (q == m - 1) {
        // one more plain level: c_{m-q} x + (q ? 2/hw : 0) S(L_{q-1}) - L_{q-2}
        st.b1 = prevB ? prevB : x;
        st.g = to_cpx<R>(cd(q == 0 ? 0.0 : 2.0 / hw, 0.0));
        st.cx = to_cpx<R>(coef_at(coef, m - q));
        st.b2 = prevA;
        st.e2 = {R(-1), R(0)};
        st.b3 = nullptr;
        st.e3 = {R(0), R(0)};
        st.out = bufs[2 * pair];
        em.sweep(st);
        prevA = prevB;
        prevB = st.out;
    }
    // final level: post * (c_0 x + (1/hw) S(L_{m-1}) - L_{m-2}) + post * add
    st.b1 = prevB ? prevB : x;
    st.g = to_cpx<R>(prevB ? post / hw : cd(0.0, 0.0));
    st.cx = to_cpx<R>(post * coef_at(coef, 0));
    st.b2 = prevA;
    st.e2 = to_cpx<R>(-post);
    st.b3 = add;
    st.e3 = to_cpx<R>(post);
    st.out = out;
    em.sweep(st);
    *steps += m;
}

template <typename R>
static DevMem* act_buffers(Workspace& W) {
    if constexpr (sizeof(R) == 8) return W.act64; else return W.act32;
}

template <typename R>
static ChebPassArgs<R> pass_base(mxp_problem* P, const StencilArgs<R>& st, const DiagTables& dt) {
    ChebPassArgs<R> a{};
    a.n0 = st.n0;
    a.n1 = st.n1;
    cpx<R>* const(*f)[3];
    if constexpr (sizeof(R) == 8) f = dt.f64; else f = dt.f32;
    a.ax = f[0][0];
    a.bx = f[0][1];
    a.gx = f[0][2];
    a.ay = f[1][0];
    a.by = f[1][1];
    a.gy = f[1][2];
    a.D = st.D;
    a.Dconst = st.Dconst;
    a.Dref = st.Dref;
    const DevTables<R>* t;
    if constexpr (sizeof(R) == 8) t = &P->t64; else t = &P->t32;
    a.abx = t->abc_h2[0];
    a.aby = t->abc_h2[1];
    const double h2 = P->g.h * P->g.h;
    a.kD = {R(double(st.kD.re) * h2), R(double(st.kD.im) * h2)};
    a.ix0 = dt.ix0;
    a.ix1 = dt.ix1;
    a.iy0 = dt.iy0;
    a.iy1 = dt.iy1;
    return a;
}

// out = post * (sum_k c_k T_k(Ahat) x + add) by fused Clenshaw passes (2D).
// bufs: four scratch vectors distinct from x, add and out.
template <typename R>
static void cheb_series_fused(mxp_problem* P, const Emit<R>& em, const StencilArgs<R>& st, const DiagTables& dt,
                              const TileCfg& tc,
                              const mxp_schedule& sc, const double* coef, int m, const cpx<R>* x,
                              cpx<R>* out, cpx<R>* const bufs[4], cd post, const cpx<R>* add,
                              int64_t* steps) {
    ChebPassArgs<R> a = pass_base<R>(P, st, dt);
    a.x = x;
    if (post.imag() != 0.0) fail(MXP_ERR_INVALID_ARG, "series scaling must be real");
    const double inv_h2 = 1.0 / (P->g.h * P->g.h);
    a.post = R(post.real());
    a.e3 = add ? R(post.real()) : R(0);
    const R post_final = a.post, e3_final = a.e3;
    const cpx<R>* prevA = nullptr;
    const cpx<R>* prevB = nullptr;
    int pair = 0;
    int q0 = 0;
    while (q0 <= m) {
        const int nlev = std::min(tc.K, m + 1 - q0);
        const bool last = (q0 + nlev == m + 1);
        for (int l = 0; l < nlev; ++l) {
            // level q: b_{m-q} = c_{m-q} x + (2/hw) A_s-step - b_{m-q+2}; the final
            // level uses c_0 and 1/hw and is scaled by post in the kernel
            const int q = q0 + l;
            const cd cx = coef_at(coef, m - q);
            const double gq = (q == 0) ? 0.0 : (q == m ? 1.0 : 2.0) / sc.half_width;
            a.cx[l] = to_cpx<R>(cx);
            a.g[l] = R(gq * inv_h2);
        }
        a.final_pass = last ? 1 : 0;
        // non-final passes end on a plain level: unit scale, no addend
        a.post = last ? post_final : R(1);
        a.e3 = last ? e3_final : R(0);
        a.in0 = prevA;
        a.in1 = prevB;
        a.add = last ? add : nullptr;
        a.outA = last ? nullptr : bufs[2 * pair];
        a.outB = last ? out : bufs[2 * pair + 1];
        cheb2d_geometry<R>(a, nlev, tc.NX, tc.Ly);
        em.pass(a, nlev, tc.NX);
        prevA = a.outA;
        prevB = a.outB;
        pair ^= 1;
        q0 += nlev;
    }
    *steps += m;
}

// The on-disk tile cache named by MXP_AUTOTUNE_CACHE (empty: none), and the
// key of this problem's choice in it: library version, device architecture,
// grid shape, precision, medium (per-node D or constant) and absorber.
static const char* tile_cache_path() {
    const char* p = std::getenv("MXP_AUTOTUNE_CACHE");
    return (p && *p) ? p : nullptr;
}
static std::string tile_cache_key(const mxp_problem* P, bool dbl) {
    hipDeviceProp_t prop;
    HIP_CHECK(hipGetDeviceProperties(&prop, P->ctx->device));
    char buf[512];
    std::snprintf(buf, sizeof(buf), "%s|%s|%dd %lldx%lldx%lld|%s|%s|absorber %d%s", mxp_version(), prop.gcnArchName,
                  P->g.dim, (long long)P->g.n[0], (long long)P->g.n[1], (long long)P->g.n[2], dbl ? "c128" : "c64",
                  P->D64.p ? "D" : "c", int(P->g.absorber), P->g.abc_per_node() ? " per-node" : "");
    std::string k(buf);
    for (char& c : k)
        if (c == '"' || c == '\\') c = '_';
    return k;
}
// A cached choice this build can run on this problem.
static bool tiles_valid(const mxp_problem* P, bool dbl, const int v[3]) {
    const int K = v[0], NX = v[1], Ly = v[2];
    if (P->g.dim == 2)
        return K >= 1 && K <= kMaxFused && (NX == 1 || NX == 2) && Ly >= 1 && NX * 64 - 2 * K > 0 &&
               !(dbl && NX == 2 && K > 3);
    return Ly >= 0 && NX == 1 && (K == 1 || ((K == 2 || K == 3) && !P->g.abc_per_node()));
}
template <typename R>
static bool tiles_from_cache(mxp_problem* P) {
    const char* path = tile_cache_path();
    if (!path) return false;
    int v[3];
    double us = 0.0;
    const bool dbl = sizeof(R) == 8;
    if (!tune_cache_get(path, tile_cache_key(P, dbl), v, &us) || !tiles_valid(P, dbl, v)) return false;
    TileCfg t;
    t.K = v[0];
    t.NX = v[1];
    t.Ly = v[2];
    t.us_per_level = us;
    P->tiles[dbl ? 0 : 1] = t;
    if (P->ctx->verbose)
        std::fprintf(stderr, "[mxp] tiles from %s: K=%d NX=%d Ly=%d (%.3f us/level)\n", path, t.K, t.NX, t.Ly, us);
    return true;
}
template <typename R>
static void tiles_to_cache(const mxp_problem* P) {
    const char* path = tile_cache_path();
    if (!path) return;
    const bool dbl = sizeof(R) == 8;
    const TileCfg& t = P->tiles[dbl ? 0 : 1];
    const int v[3] = {t.K, t.NX, t.Ly};
    if (!tune_cache_put(path, tile_cache_key(P, dbl), v, t.us_per_level) && P->ctx->verbose)
        std::fprintf(stderr, "[mxp] tile cache %s not updated (unreadable or not a tile cache)\n", path);
}

template <typename R>
static void tune_tiles(mxp_problem* P, Workspace& ws, const Sched& sd, hipStream_t s);
template <typename R>
static void tune_3d(mxp_problem* P, Workspace& ws, const Sched& sd, hipStream_t s);

// Device buffers of one action.
template <typename R>
struct ActBufs {
    cpx<R>* w[6];
    cpx<R>* pbuf;
    cpx<R>* y1;
};

// y = exp(i t A_s) x, psi_1(i t A_s) x or psi_2(i t A_s) x (fn), precision R,
// on the device buffers B (w[0..5] always, pbuf for psi_1 and psi_2, y1 for
// psi_2), with the 2D pass tiles tc.  x and y: distinct device vectors of
// precision R, neither of them one of B's buffers.
template <typename R>
static void action_on(mxp_problem* P, const ActBufs<R>& B, const TileCfg& tc, const Emit<R>& em, const Sched& sd,
                      double t, double shift, int fn, const cpx<R>* x, cpx<R>* y, int64_t* steps) {
    if (fn < ACT_EXP || fn > ACT_PSI2) fail(MXP_ERR_INVALID_ARG, "unknown matrix function");
    const bool psi = fn == ACT_PSI1;
    const mxp_schedule& sc = sd.s;
    cpx<R>* const* w = B.w;
    cpx<R>* pbuf = B.pbuf;
    const StencilArgs<R> base = base_args<R>(P, shift, sd.diag);
    const bool fused = (P->g.dim == 2);
    const int S = sc.S;
    // Scratch for one series: five buffers other than its input (four for the
    // passes, one for the output); the unfused path uses two of them.
    auto pick = [&](const cpx<R>* cur, cpx<R>** b, cpx<R>** o) {
        int k = 0;
        for (int q = 0; q < 6 && k < 5; ++q)
            if (w[q] != cur) {
                if (k < 4) b[k] = w[q]; else *o = w[q];
                ++k;
            }
    };
    auto series = [&](const double* coef, int m, const cpx<R>* xin, cpx<R>* out, cd post,
                      const cpx<R>* add) {
        cpx<R>* b[4];
        cpx<R>* spare;
        pick(xin, b, &spare);
        if (fused) {
            cheb_series_fused<R>(P, em, base, sd.diag, tc, sc, coef, m, xin, out, b, post, add, steps);
        } else if (P->g.dim == 3 && (tc.K == 2 || tc.K == 3) && !P->g.abc_per_node()) {
            cheb_series3d<R>(em, base, sc, coef, m, xin, out, b, post, add, steps, tc.Ly, tc.K);
        } else {
            cheb_series<R>(em, base, sc, coef, m, xin, out, b[0], b[1], post, add, steps);
        }
    };
    auto substep_out = [&](const cpx<R>* xin) {
        cpx<R>* b[4];
        cpx<R>* spare = nullptr;
        pick(xin, b, &spare);
        return spare;
    };
    if (fn == ACT_PSI2) {
        // With tau = t/S, E = exp(i tau A_s) and F = tau psi_1(i tau A_s):
        //   t^2 psi_2(i t A_s) x = S y_1 + F (g_1 + ... + g_{S-1}),
        // y_1 = tau^2 psi_2(i tau A_s) x, g_1 = F x, g_{k+1} = E g_k + g_1
        // (split the double time integral at the substeps).  The running sum
        // G_k = g_1 + ... + g_k obeys G_{k+1} = E G_k + (k+1) g_1, so its mean
        // H_k = G_k / k obeys H_{k+1} = (k/(k+1)) E H_k + g_1: one exp series
        // with scaled coefficients per substep, and no extra vector update.
        if (sd.m_psi2 < 0) design_psi2_series(sc, sd.t, sd.prec, &sd.coef_psi2, &sd.m_psi2);
        const double it2 = 1.0 / (t * t);
        if (S == 1) {
            series(sd.coef_psi2.data(), sd.m_psi2, x, y, cd(it2, 0.0), nullptr);
            return;
        }
        cpx<R>* y1 = B.y1;
        series(sd.coef_psi2.data(), sd.m_psi2, x, y1, cd(1.0, 0.0), nullptr);
        series(sc.coef_psi, sc.m_psi, x, pbuf, cd(1.0, 0.0), nullptr);  // g_1 = H_1
        const cpx<R>* hk = pbuf;
        std::vector<double> scaled(2 * size_t(std::max(sc.m, sc.m_psi) + 1));
        for (int k = 1; k <= S - 2; ++k) {
            const double f = double(k) / double(k + 1);
            for (int i = 0; i < 2 * (sc.m + 1); ++i) scaled[i] = f * sc.coef[i];
            cpx<R>* out = substep_out(hk);
            series(scaled.data(), sc.m, hk, out, cd(1.0, 0.0), pbuf);
            hk = out;
        }
        // t^2 psi_2 x = S (((S-1)/S) F H_{S-1} + y_1)
        const double f = double(S - 1) / double(S);
        for (int i = 0; i < 2 * (sc.m_psi + 1); ++i) scaled[i] = f * sc.coef_psi[i];
        series(scaled.data(), sc.m_psi, hk, y, cd(double(S) * it2, 0.0), y1);
        return;
    }
    const cpx<R>* xcur = x;
    int first = 0;
    const cpx<R>* add = nullptr;
    if (psi) {
        // p = tau psi_1(i tau A_s) x; with S == 1 the answer is p / t.
        if (S == 1) {
            series(sc.coef_psi, sc.m_psi, x, y, cd(1.0 / t, 0.0), nullptr);
            return;
        }
        series(sc.coef_psi, sc.m_psi, x, pbuf, cd(1.0, 0.0), nullptr);
        xcur = pbuf;
        add = pbuf;
        first = 1;
    }
    for (int sub = first; sub < S; ++sub) {
        const bool last = (sub == S - 1);
        cpx<R>* out = last ? y : substep_out(xcur);
        const cd post = (psi && last) ? cd(1.0 / t, 0.0) : cd(1.0, 0.0);
        series(sc.coef, sc.m, xcur, out, post, add);
        xcur = out;
    }
}

// The same action with buffers from workspace ws (the 2D tiles are tuned at
// the problem's first action).
template <typename R>
static void action(mxp_problem* P, Workspace& ws, const Emit<R>& em, const Sched& sd, double t, double shift,
                   int fn, const cpx<R>* x, cpx<R>* y, int64_t* steps) {
    const int64_t n = npts(P);
    DevMem* W = act_buffers<R>(ws);
    for (int q = 0; q < 7; ++q) W[q].ensure(size_t(n) * sizeof(cpx<R>));
    if (fn == ACT_PSI2) W[9].ensure(size_t(n) * sizeof(cpx<R>));
    ActBufs<R> B;
    for (int q = 0; q < 6; ++q) B.w[q] = W[q].as<cpx<R>>();
    B.pbuf = W[6].as<cpx<R>>();
    B.y1 = W[9].as<cpx<R>>();
    TileCfg& slot = P->tiles[sizeof(R) == 4 ? 1 : 0];
    if (slot.K == 0) {
        if (em.rec) fail(MXP_ERR_HIP, "tiles must be tuned before a batched action");
        if (P->g.dim == 2)
            tune_tiles<R>(P, ws, sd, em.s);
        else
            tune_3d<R>(P, ws, sd, em.s);
    }
    const TileCfg tc = slot;
    action_on<R>(P, B, tc, em, sd, t, shift, fn, x, y, steps);
}

// Times candidate tile configurations of the fused 2D pass on this problem's
// own buffers (HIP events on the context stream) and keeps the fastest per
// Clenshaw level.
template <typename R>
static void tune_tiles(mxp_problem* P, Workspace& ws, const Sched& sd, hipStream_t s) {
    Range range("tile tuning 2D");
    if (tiles_from_cache<R>(P)) return;
    const int64_t n = npts(P);
    DevMem* W = act_buffers<R>(ws);
    for (int q = 0; q < 7; ++q) {
        W[q].ensure(size_t(n) * sizeof(cpx<R>));
        launch_zero<R>(W[q].as<cpx<R>>(), n, s);
    }
    const StencilArgs<R> st = base_args<R>(P, 0.0, sd.diag);
    ChebPassArgs<R> a = pass_base<R>(P, st, sd.diag);
    a.x = W[0].as<cpx<R>>();
    a.in0 = W[1].as<cpx<R>>();
    a.in1 = W[2].as<cpx<R>>();
    a.outA = W[3].as<cpx<R>>();
    a.outB = W[4].as<cpx<R>>();
    for (int l = 0; l < kMaxFused; ++l) {
        a.cx[l] = {R(0.1), R(0)};
        a.g[l] = R(0.1);
    }
    a.post = R(1);
    a.e3 = R(0);
    a.final_pass = 0;
    TileCfg best;
    best.us_per_level = 1e300;
    hipEvent_t e0, e1;
    HIP_CHECK(hipEventCreate(&e0));
    HIP_CHECK(hipEventCreate(&e1));
    // short segments and single levels give small grids enough wavefronts
    const int Ks[] = {1, 2, 3, 4, 6, 8};
    // Every workgroup (4 wavefronts) is resident at once, so the compute units
    // holding one more of them than the others set the time.  Besides the
    // fixed lengths, each (K, NX) tries the segment lengths whose workgroup
    // count is just below c times the CU count, c = 1..6.
    const int Lys[] = {4, 8, 12, 16, 20, 24, 28, 32, 40, 48, 64, 96, 128};
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        fail(MXP_ERR_HIP, "cannot query the compute-unit count");
    for (int NX = 1; NX <= 2; ++NX) {
        for (int K : Ks) {
            if (sizeof(R) == 8 && NX == 2 && K > 3) continue;  // register-limited
            const int64_t W = int64_t(NX) * 64 - 2 * K;
            const int64_t strips = (P->g.n[0] + W - 1) / W;
            std::vector<int> lys(std::begin(Lys), std::end(Lys));
            for (int c = 1; c <= 6; ++c) {
                const int64_t segs = (4 * int64_t(c) * cus) / strips;  // waves <= 4 c CUs
                if (segs < 1) continue;
                const int64_t ly = (P->g.n[1] + segs - 1) / segs;
                if (ly >= 2 && ly <= 256) lys.push_back(int(ly));
            }
            std::sort(lys.begin(), lys.end());
            lys.erase(std::unique(lys.begin(), lys.end()), lys.end());
            for (int Ly : lys) {
                // segments longer than the grid only repeat the one-segment case
                if (Ly != lys.front() && Ly / 2 >= P->g.n[1]) continue;
                cheb2d_geometry<R>(a, K, NX, Ly);
                if (a.W <= 0) continue;
                launch_cheb2d<R>(a, K, NX, s);  // warm
                HIP_CHECK(hipEventRecord(e0, s));
                const int reps = 3;
                for (int r = 0; r < reps; ++r) launch_cheb2d<R>(a, K, NX, s);
                HIP_CHECK(hipEventRecord(e1, s));
                HIP_CHECK(hipEventSynchronize(e1));
                float ms = 0;
                HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
                const double us = 1e3 * ms / (reps * K);
                if (P->ctx->verbose) {
                    std::fprintf(stderr, "[mxp] tune %s K=%d NX=%d Ly=%d: %.3f us/level\n",
                                 sizeof(R) == 4 ? "c64" : "c128", K, NX, Ly, us);
                }
                if (us < best.us_per_level) {
                    best.K = K;
                    best.NX = NX;
                    best.Ly = Ly;
                    best.us_per_level = us;
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best.K == 0) fail(MXP_ERR_HIP, "tile autotuning measured no candidate");
    P->tiles[sizeof(R) == 4 ? 1 : 0] = best;
    tiles_to_cache<R>(P);
}

// y = exp, psi_1 or psi_2 action (fn) on complex-double vectors, in the requested
// precision, enqueued on stream s with workspace ws, or recorded into
// rec64 / rec32 when given (the caller then launches the records and, for
// the mixed form, the cast back).  The mixed form casts at the boundary.
void action64_on(mxp_problem* P, Workspace& ws, hipStream_t s, const Sched& sc, double t, double shift,
                        int fn, mxp_precision prec, const cpx<double>* x, cpx<double>* y, int64_t* steps,
                        std::vector<StepRec<double>>* rec64, std::vector<StepRec<float>>* rec32) {
    Range range(fn == ACT_EXP ? "exp action" : (fn == ACT_PSI1 ? "psi1 action" : "psi2 action"));
    if (prec == MXP_PREC_FP64) {
        action<double>(P, ws, Emit<double>{s, rec64}, sc, t, shift, fn, x, y, steps);
        return;
    }
    const int64_t n = npts(P);
    ws.act32[7].ensure(size_t(n) * sizeof(cpx<float>));
    ws.act32[8].ensure(size_t(n) * sizeof(cpx<float>));
    cpx<float>* xs = ws.act32[7].as<cpx<float>>();
    cpx<float>* ys = ws.act32[8].as<cpx<float>>();
    launch_to_c64(x, xs, n, s);
    action<float>(P, ws, Emit<float>{s, rec32}, sc, t, shift, fn, xs, ys, steps);
    if (!rec32) launch_to_c128(ys, y, n, s);
}


// The same action from a captured HIP graph.  The graph reads a fixed input
// buffer and writes a fixed output buffer of the workspace (the mixed form's
// cast buffers, or two complex-double staging buffers), so one capture per
// (schedule, function, precision) serves every call: the input is staged, the
// graph replays on the workspace's stream (ordered after and before the
// caller's stream by events) and the output is copied out.  The first use of
// a key runs eagerly (it allocates the buffers and tunes the tiles), the
// second captures.  Kernels only: nothing in an action is a memset or a copy.
void action64_graph(mxp_problem* P, Workspace& ws, hipStream_t s, const Sched& sc, double t, double shift,
                           int fn, mxp_precision prec, const cpx<double>* x, cpx<double>* y, int64_t* steps) {
    const int64_t n = npts(P);
    const bool f32 = prec != MXP_PREC_FP64;
    DevMem* in = f32 ? &ws.act32[7] : &ws.act64[7];
    DevMem* out = f32 ? &ws.act32[8] : &ws.act64[8];
    const size_t bytes = size_t(n) * (f32 ? sizeof(cpx<float>) : sizeof(cpx<double>));
    in->ensure(bytes);
    out->ensure(bytes);
    if (f32) launch_to_c64(x, in->as<cpx<float>>(), n, s);
    else launch_scale({1.0, 0.0}, x, in->as<cpx<double>>(), n, s);
    auto run_action = [&](hipStream_t st, int64_t* cnt) {
        if (f32)
            action<float>(P, ws, Emit<float>{st, nullptr}, sc, t, shift, fn, in->as<cpx<float>>(),
                          out->as<cpx<float>>(), cnt);
        else
            action<double>(P, ws, Emit<double>{st, nullptr}, sc, t, shift, fn, in->as<cpx<double>>(),
                           out->as<cpx<double>>(), cnt);
    };
    GraphEntry& ge = ws.graphs[std::make_tuple(static_cast<const void*>(&sc), fn, int(prec))];
    if (ge.uses++ == 0) {
        run_action(s, steps);
    } else {
        if (!ws.gstream) {
            HIP_CHECK(hipStreamCreateWithFlags(&ws.gstream, hipStreamNonBlocking));
            HIP_CHECK(hipEventCreateWithFlags(&ws.gev[0], hipEventDisableTiming));
            HIP_CHECK(hipEventCreateWithFlags(&ws.gev[1], hipEventDisableTiming));
        }
        HIP_CHECK(hipEventRecord(ws.gev[0], s));
        HIP_CHECK(hipStreamWaitEvent(ws.gstream, ws.gev[0], 0));
        if (!ge.exec) {
            int64_t cnt = 0;
            HIP_CHECK(hipStreamBeginCapture(ws.gstream, hipStreamCaptureModeThreadLocal));
            try {
                run_action(ws.gstream, &cnt);
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(ws.gstream, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            HIP_CHECK(hipStreamEndCapture(ws.gstream, &ge.graph));
            HIP_CHECK(hipGraphInstantiate(&ge.exec, ge.graph, nullptr, nullptr, 0));
            ge.steps = cnt;
        }
        HIP_CHECK(hipGraphLaunch(ge.exec, ws.gstream));
        *steps += ge.steps;
        HIP_CHECK(hipEventRecord(ws.gev[1], ws.gstream));
        HIP_CHECK(hipStreamWaitEvent(s, ws.gev[1], 0));
    }
    if (f32) launch_to_c128(out->as<cpx<float>>(), y, n, s);
    else launch_scale({1.0, 0.0}, out->as<cpx<double>>(), y, n, s);
}

void apply_A64(mxp_problem* P, hipStream_t s, double shift, const cpx<double>* x, cpx<double>* y,
                      double g, const cpx<double>* add, double eadd) {
    StencilArgs<double> a = base_args<double>(P, shift, plain_diag(P, shift));
    a.g = {g, 0.0};
    a.b1 = x;
    a.b2 = add;
    a.e2 = {eadd, 0.0};
    a.out = y;
    launch_stencil(a, s);
}

// f(i t A_s) x with f = exp or psi_1 from one Arnoldi basis, the route the
// paper takes for its matrix functions (a Krylov method, Section 4

// Chooses the 3D Clenshaw kernel of this problem and precision: times a
// single-level sweep (a middle step: x, b_{k+1}, b_{k+2}) against two- and
// three-level passes (x, in0, in1) on the problem's own buffers (HIP events on
// the context stream) and keeps the fastest per Clenshaw level: K = 2 or 3
// for the multi-level passes (Ly: the best z-chunk of 16, 32, 64 and, for
// three levels, 128 planes) when they beat the sweep by more than 3%, else K = 1 with
// Ly = 0 (automatic z-chunk) for sweeps.  Grids whose
// absorbing faces carry a per-node term take sweeps (the two-level pass does
// not carry that term).
template <typename R>
static void tune_3d(mxp_problem* P, Workspace& ws, const Sched& sd, hipStream_t s) {
    Range range("tile tuning 3D");
    if (tiles_from_cache<R>(P)) return;
    TileCfg& slot = P->tiles[sizeof(R) == 4 ? 1 : 0];
    TileCfg sweep;
    sweep.K = 1;
    sweep.NX = 1;
    sweep.Ly = 0;
    if (P->g.abc_per_node()) {
        slot = sweep;
        return;
    }
    const int64_t n = npts(P);
    DevMem* W = act_buffers<R>(ws);
    for (int q = 0; q < 5; ++q) {
        W[q].ensure(size_t(n) * sizeof(cpx<R>));
        launch_zero<R>(W[q].as<cpx<R>>(), n, s);
    }
    StencilArgs<R> st = base_args<R>(P, 0.0, sd.diag);
    st.x = W[0].as<cpx<R>>();
    st.b1 = W[1].as<cpx<R>>();
    st.b2 = W[2].as<cpx<R>>();
    st.b3 = nullptr;
    st.g = {R(0.1), R(0)};
    st.cx = {R(0.1), R(0)};
    st.e2 = {R(-1), R(0)};
    st.e3 = {R(0), R(0)};
    st.out = W[3].as<cpx<R>>();
    ChebPass3DArgs<R> a{};
    a.n0 = st.n0;
    a.n1 = st.n1;
    a.n2 = st.n2;
    for (int d = 0; d < 3; ++d) {
        a.alpha[d] = st.alpha[d];
        a.beta[d] = st.beta[d];
        a.gamma[d] = st.gamma[d];
    }
    a.D = st.D;
    a.Dconst = st.Dconst;
    a.Dref = st.Dref;
    a.kD = st.kD;
    a.x = W[0].as<cpx<R>>();
    a.in0 = W[1].as<cpx<R>>();
    a.in1 = W[2].as<cpx<R>>();
    a.outA = W[3].as<cpx<R>>();
    a.outB = W[4].as<cpx<R>>();
    for (int l = 0; l < 2; ++l) {
        a.cx[l] = {R(0.1), R(0)};
        a.g[l] = R(0.1);
    }
    hipEvent_t e0, e1;
    HIP_CHECK(hipEventCreate(&e0));
    HIP_CHECK(hipEventCreate(&e1));
    auto time_us = [&](auto&& launch, int levels) {
        launch();  // warm
        const int reps = 5;
        HIP_CHECK(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r) launch();
        HIP_CHECK(hipEventRecord(e1, s));
        HIP_CHECK(hipEventSynchronize(e1));
        float ms = 0;
        HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
        return 1e3 * ms / (reps * levels);
    };
    const double us_sweep = time_us([&] { launch_stencil(st, s); }, 1);
    // two-level passes with z-chunks of 16, 32 and 64 planes and three-level
    // passes with 16, 32, 64 and 128 (no longer than the grid; at 256^3 the
    // long chunks win although they leave compute units idle: their z-halo
    // is smaller)
    double us_pass = 1e300;
    int best_zc = 0, best_k = 2;
    for (int levels : {2, 3}) {
        for (int zc : {16, 32, 64, 128}) {
            if (zc > 16 && zc / 2 >= P->g.n[2]) continue;
            if (levels == 2 && zc > 64) continue;
            double us;
            if (levels == 2) {
                cheb3d_geometry<R>(a, zc);
                us = time_us([&] { launch_cheb3d<R>(a, s); }, 2);
            } else {
                ChebPass3DArgs<R> a3 = a;
                a3.cx[2] = {R(0.1), R(0)};
                a3.g[2] = R(0.1);
                cheb3d3_geometry<R>(a3, zc);
                us = time_us([&] { launch_cheb3d3<R>(a3, s); }, 3);
            }
            if (P->ctx->verbose)
                std::fprintf(stderr, "[mxp] tune 3D %s: %d-level pass, %d-plane chunks: %.3f us/level\n",
                             sizeof(R) == 4 ? "c64" : "c128", levels, zc, us);
            if (us < us_pass) {
                us_pass = us;
                best_zc = zc;
                best_k = levels;
            }
        }
    }
    HIP_CHECK(hipEventDestroy(e0));
    HIP_CHECK(hipEventDestroy(e1));
    if (P->ctx->verbose)
        std::fprintf(stderr, "[mxp] tune 3D %s: sweep %.3f us/level, best %d-level pass %.3f us/level\n",
                     sizeof(R) == 4 ? "c64" : "c128", us_sweep, best_k, us_pass);
    // a multi-level pass must win by a margin larger than the timing noise
    // of single launches, else the simpler sweep stays
    if (us_pass < 0.97 * us_sweep) {
        TileCfg two;
        two.K = best_k;
        two.NX = 1;
        two.Ly = best_zc;
        two.us_per_level = us_pass;
        slot = two;
    } else {
        sweep.us_per_level = us_sweep;
        slot = sweep;
    }
    tiles_to_cache<R>(P);
}

void reserve_action(mxp_problem* P, Workspace& ws, const Sched& sd, bool psi2, bool graphs, hipStream_t s) {
    const size_t n = size_t(npts(P));
    if (sd.prec == MXP_PREC_FP64) {
        // [0..5] pass and substep buffers, [6] the psi addend, [7..8] graph
        // staging, [9] the psi_2 action's first-substep term
        for (int q = 0; q < 7; ++q) ws.act64[q].ensure(n * sizeof(cpx<double>));
        if (graphs) {
            ws.act64[7].ensure(n * sizeof(cpx<double>));
            ws.act64[8].ensure(n * sizeof(cpx<double>));
        }
        if (psi2) ws.act64[9].ensure(n * sizeof(cpx<double>));
    } else {
        // as above, with [7..8] the casts of complex-double arguments
        for (int q = 0; q < 9; ++q) ws.act32[q].ensure(n * sizeof(cpx<float>));
        if (psi2) ws.act32[9].ensure(n * sizeof(cpx<float>));
    }
    if (psi2 && sd.m_psi2 < 0) design_psi2_series(sd.s, sd.t, sd.prec, &sd.coef_psi2, &sd.m_psi2);
    ensure_tiles(P, ws, sd, s);
}

void ensure_tiles(mxp_problem* P, Workspace& ws, const Sched& sd, hipStream_t s) {
    const bool dbl = sd.prec == MXP_PREC_FP64;
    if (P->tiles[dbl ? 0 : 1].K != 0) return;
    if (P->g.dim == 2) {
        if (dbl) tune_tiles<double>(P, ws, sd, s); else tune_tiles<float>(P, ws, sd, s);
    } else {
        if (dbl) tune_3d<double>(P, ws, sd, s); else tune_3d<float>(P, ws, sd, s);
    }
}

void apply_A(mxp_problem* P, hipStream_t s, double shift, mxp_dtype dtype, const void* x, void* y) {
    if (dtype == MXP_C128) {
        apply_A64(P, s, shift, static_cast<const cpx<double>*>(x), static_cast<cpx<double>*>(y), 1.0, nullptr, 0.0);
    } else if (dtype == MXP_C64) {
        StencilArgs<float> a = base_args<float>(P, shift, plain_diag(P, shift));
        a.b1 = static_cast<const cpx<float>*>(x);
        a.out = static_cast<cpx<float>*>(y);
        launch_stencil(a, s);
    } else {
        fail(MXP_ERR_INVALID_ARG, "dtype must be MXP_C64 or MXP_C128");
    }
}

void apply_action_on(mxp_problem* P, void* const bufs[6], const TileCfg& tc, hipStream_t s, const Sched& sd,
                     double t, double shift, mxp_dtype dtype, const void* x, void* y, int64_t* steps) {
    if (dtype == MXP_C128) {
        ActBufs<double> B{};
        for (int q = 0; q < 6; ++q) B.w[q] = static_cast<cpx<double>*>(bufs[q]);
        action_on<double>(P, B, tc, Emit<double>{s, nullptr}, sd, t, shift, ACT_EXP,
                          static_cast<const cpx<double>*>(x), static_cast<cpx<double>*>(y), steps);
    } else if (dtype == MXP_C64) {
        ActBufs<float> B{};
        for (int q = 0; q < 6; ++q) B.w[q] = static_cast<cpx<float>*>(bufs[q]);
        action_on<float>(P, B, tc, Emit<float>{s, nullptr}, sd, t, shift, ACT_EXP,
                         static_cast<const cpx<float>*>(x), static_cast<cpx<float>*>(y), steps);
    } else {
        fail(MXP_ERR_INVALID_ARG, "dtype must be MXP_C64 or MXP_C128");
    }
}

void apply_action(mxp_problem* P, Workspace& ws, hipStream_t s, const Sched& sd, double t, double shift, int fn,
                  mxp_dtype dtype, const void* x, void* y, int64_t* steps) {
    if (dtype == MXP_C128)
        action<double>(P, ws, Emit<double>{s, nullptr}, sd, t, shift, fn, static_cast<const cpx<double>*>(x),
                       static_cast<cpx<double>*>(y), steps);
    else if (dtype == MXP_C64)
        action<float>(P, ws, Emit<float>{s, nullptr}, sd, t, shift, fn, static_cast<const cpx<float>*>(x),
                      static_cast<cpx<float>*>(y), steps);
    else
        fail(MXP_ERR_INVALID_ARG, "dtype must be MXP_C64 or MXP_C128");
}

}  // namespace mxp
