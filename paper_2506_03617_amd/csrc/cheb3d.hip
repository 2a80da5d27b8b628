// Two Clenshaw levels per HBM pass on 3D grids (gfx950).
//
//   L_0 = cx0 x + g0 S(in1) - in0,   L_1 = cx1 x + g1 S(L_0) - in1
//
// A workgroup of sixteen wavefronts owns a tile of 62 x 14 output nodes (x, y)
// and marches along z over a chunk of planes.  Wavefront w holds grid row
// y0 - 1 + w (rows 0 and 15 are halo rows) and its 64 lanes hold columns
// x0 - 1 .. x0 + 62 (lanes 0 and 63 are halo columns).  At step k:
//  * every wavefront computes L_0 on plane k for its row (in1's z-window of
//    three planes is carried in registers; x-neighbours come from the
//    adjacent lanes through DPP, the two edge lanes load theirs);
//  * L_0 is written to a three-plane LDS ring and the workgroup synchronises
//    once;
//  * wavefronts 1..14 compute L_1 on plane k - 1: x-neighbours by DPP,
//    y-neighbours from the ring, z-neighbours from the L_0 planes the
//    wavefront carries; lanes 1..62 store both levels.
// Ghost nodes (outside the grid) hold zero, as in the single-level sweep.
// One pass reads in0, in1, x (and D) and writes two levels: 40-44 bytes per
// node for two levels instead of 64-72 for two single-level sweeps.
#include <hip/hip_runtime.h>

#include <string>
#include <utility>

#include "cheb3d.h"
#include "devmem.h"
#include "kernels.h"
#include "mxp_internal.h"

namespace mxp {

namespace {

constexpr int TY = 14;          // output rows per workgroup (16 wavefronts: 4 per SIMD at one workgroup per CU)
constexpr int NW = TY + 2;      // wavefronts: one per row, plus a halo row each side
constexpr int TXO = 62;         // output columns per 64-lane wavefront
constexpr int kZChunk = 32;  // default z-chunk (planes)
// three-level pass: NW3 wavefronts hold rows y0 - 2 .. y0 + TY3 + 1
constexpr int NW3 = 16;
constexpr int TY3 = NW3 - 4;
constexpr int TXO3 = 60;

template <typename R>
__device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cpx<R> cadd(cpx<R> a, cpx<R> b) {
    return {a.re + b.re, a.im + b.im};
}
template <typename R>
__device__ __forceinline__ cpx<R> cfma(cpx<R> a, cpx<R> b, cpx<R> c) {
    return {fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im))};
}
template <typename R>
__device__ __forceinline__ cpx<R> cscale(R s, cpx<R> a) {
    return {s * a.re, s * a.im};
}
template <typename R>
__device__ __forceinline__ cpx<R> keep_if(bool c, cpx<R> v) {
    return {c ? v.re : R(0), c ? v.im : R(0)};
}

__device__ __forceinline__ float dpp_f(float v, bool below) {
    const int iv = __builtin_bit_cast(int, v);
    const int r = below ? __builtin_amdgcn_mov_dpp(iv, 0x138, 0xf, 0xf, true)
                        : __builtin_amdgcn_mov_dpp(iv, 0x130, 0xf, 0xf, true);
    return __builtin_bit_cast(float, r);
}
__device__ __forceinline__ double dpp_d(double v, bool below) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = int(b & 0xffffffffll), hi = int(b >> 32);
    int rlo, rhi;
    if (below) {
        rlo = __builtin_amdgcn_mov_dpp(lo, 0x138, 0xf, 0xf, true);
        rhi = __builtin_amdgcn_mov_dpp(hi, 0x138, 0xf, 0xf, true);
    } else {
        rlo = __builtin_amdgcn_mov_dpp(lo, 0x130, 0xf, 0xf, true);
        rhi = __builtin_amdgcn_mov_dpp(hi, 0x130, 0xf, 0xf, true);
    }
    const long long r = (long long)(unsigned(rlo)) | ((long long)rhi << 32);
    return __builtin_bit_cast(double, r);
}
// lane l receives lane l - 1 (below) or l + 1 (above)
template <typename R>
__device__ __forceinline__ cpx<R> from_below(cpx<R> v) {
    if constexpr (sizeof(R) == 4) return {dpp_f(v.re, true), dpp_f(v.im, true)};
    else return {dpp_d(v.re, true), dpp_d(v.im, true)};
}
template <typename R>
__device__ __forceinline__ cpx<R> from_above(cpx<R> v) {
    if constexpr (sizeof(R) == 4) return {dpp_f(v.re, false), dpp_f(v.im, false)};
    else return {dpp_d(v.re, false), dpp_d(v.im, false)};
}

template <typename R>
struct vec2_of;
template <>
struct vec2_of<float> {
    typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct vec2_of<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};
template <typename R>
__device__ __forceinline__ cpx<R> gload(const cpx<R>* p, int64_t i) {
    typedef typename vec2_of<R>::type V;
    const V v = ((const __attribute__((address_space(1))) V*)(p))[i];
    return {v.x, v.y};
}
template <typename R>
__device__ __forceinline__ R gload(const R* p, int64_t i) {
    return ((const __attribute__((address_space(1))) R*)(p))[i];
}
template <typename R>
__device__ __forceinline__ void gstore(cpx<R>* p, int64_t i, cpx<R> c) {
    typedef typename vec2_of<R>::type V;
    V v;
    v.x = c.re;
    v.y = c.im;
    ((__attribute__((address_space(1))) V*)(p))[i] = v;
}
template <typename R>
__device__ __forceinline__ cpx<R> sload(const cpx<R>* p, int64_t idx) {
    const __attribute__((address_space(4))) R* q = (const __attribute__((address_space(4))) R*)(p);
    return {q[2 * idx], q[2 * idx + 1]};
}
template <class T>
__device__ __forceinline__ T sload_words(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "dword-sized struct expected");
    const __attribute__((address_space(4))) uint32_t* q = (const __attribute__((address_space(4))) uint32_t*)(p);
    uint32_t w[sizeof(T) / 4];
#pragma unroll
    for (unsigned i = 0; i < sizeof(T) / 4; ++i) w[i] = q[i];
    return __builtin_bit_cast(T, w);
}

// VAR: 1 D present, 2 in0 present, 4 in1 present
template <typename R, int VAR>
__device__ __forceinline__ void cheb3d_body(const ChebPass3DArgs<R>& a, int tile, cpx<R> (*ring)[NW][64]) {
    constexpr bool HD = VAR & 1, IN0 = VAR & 2, IN1 = VAR & 4;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tx = tile % a.tiles_x;
    const int rest = tile / a.tiles_x;
    const int ty = rest % a.tiles_y;
    const int tz = rest / a.tiles_y;
    const int64_t n0 = a.n0, n1 = a.n1, n2 = a.n2;
    const int64_t sy = n0, sz = n0 * n1;
    const int64_t gx = int64_t(tx) * TXO - 1 + lane;
    const int64_t gy = int64_t(ty) * TY - 1 + w;
    const int64_t z0 = int64_t(tz) * a.zc;
    const int64_t z1 = z0 + a.zc < n2 ? z0 + a.zc : n2;
    const bool xin = gx >= 0 && gx < n0, yin = gy >= 0 && gy < n1;
    const bool live = xin && yin;
    const int64_t cxl = gx < 0 ? 0 : (gx >= n0 ? n0 - 1 : gx);
    const int64_t cyl = gy < 0 ? 0 : (gy >= n1 ? n1 - 1 : gy);
    const int64_t cym = gy - 1 < 0 ? 0 : (gy - 1 >= n1 ? n1 - 1 : gy - 1);
    const int64_t cyp = gy + 1 < 0 ? 0 : (gy + 1 >= n1 ? n1 - 1 : gy + 1);
    // the edge lanes' own outer x-neighbour (other lanes get theirs by DPP)
    const int64_t ex = lane == 0 ? gx - 1 : (lane == 63 ? gx + 1 : gx);
    const int64_t cex = ex < 0 ? 0 : (ex >= n0 ? n0 - 1 : ex);
    const cpx<R> wxm = keep_if(xin && gx > 0, gload(a.alpha[0], cxl));
    const cpx<R> wxp = keep_if(xin && gx < n0 - 1, gload(a.beta[0], cxl));
    const cpx<R> wym = keep_if(yin && gy > 0, gload(a.alpha[1], cyl));
    const cpx<R> wyp = keep_if(yin && gy < n1 - 1, gload(a.beta[1], cyl));
    const cpx<R> gxy = cadd(gload(a.gamma[0], cxl), gload(a.gamma[1], cyl));
    const cpx<R> zero{R(0), R(0)};
    const int64_t prow = cxl + sy * cyl;  // this lane's node in plane 0
    auto in1_at = [&](int64_t k, int64_t off) -> cpx<R> {
        if constexpr (!IN1) return zero;
        const bool ok = k >= 0 && k < n2;
        const cpx<R> v = gload(a.in1, off + sz * (ok ? k : 0));
        return keep_if(ok, v);
    };
    // Operands of plane k for L_0, loaded one step ahead (software pipeline:
    // the loads of plane k + 1 are in flight while plane k is computed).
    struct PlaneIn {
        cpx<R> x, in0, ym, yp, e, zp;  // zp: in1 on plane k + 1
        R D;
    };
    auto load_plane = [&](int64_t k) -> PlaneIn {
        PlaneIn q;
        const bool kin = k >= 0 && k < n2;
        const int64_t kc = kin ? k : 0;
        const int64_t pk = prow + sz * kc;
        q.x = gload(a.x, pk);
        q.in0 = zero;
        if constexpr (IN0) q.in0 = gload(a.in0, pk);
        q.D = a.Dconst;
        if constexpr (HD) q.D = gload(a.D, pk);
        q.ym = q.yp = q.e = zero;
        if constexpr (IN1) {
            q.ym = gload(a.in1, cxl + sy * cym + sz * kc);
            q.yp = gload(a.in1, cxl + sy * cyp + sz * kc);
            q.e = gload(a.in1, cex + sy * cyl + sz * kc);
        }
        // in1 on plane k + 1 as loaded (a clamped plane past the grid): it is
        // masked where it is used, one step later, so that no wait for this
        // load (and, loads returning in order, for the whole prefetch) lands
        // in the step that issues it
        q.zp = zero;
        if constexpr (IN1) q.zp = gload(a.in1, prow + sz * (k + 1 >= 0 && k + 1 < n2 ? k + 1 : 0));
        return q;
    };
    cpx<R> a_m = in1_at(z0 - 2, prow);
    cpx<R> a_c = in1_at(z0 - 1, prow);
    cpx<R> l0_m2 = zero, l0_m1 = zero, x_m1 = zero;
    R D_m1 = a.Dconst;
    // one plane step: L_0 on plane k from `cur` (its operands, loaded one
    // step earlier), L_1 on plane k - 1
    auto step = [&](int64_t k, const PlaneIn& cur) {
        const cpx<R> zp = keep_if(k + 1 >= 0 && k + 1 < n2, cur.zp);
        // ---- L_0 on plane k (every row of the workgroup, halo included)
        const bool kin = k >= 0 && k < n2;  // uniform
        const int64_t kc = kin ? k : 0;
        cpx<R> left = from_below(a_c), right = from_above(a_c);
        if (lane == 0) left = cur.e;
        if (lane == 63) right = cur.e;
        cpx<R> diag = cadd(gxy, sload(a.gamma[2], kc));
        diag = cadd(diag, cscale(cur.D - a.Dref, a.kD));
        cpx<R> s = cmul(diag, a_c);
        s = cfma(wxm, left, s);
        s = cfma(wxp, right, s);
        s = cfma(wym, cur.ym, s);
        s = cfma(wyp, cur.yp, s);
        s = cfma(sload(a.alpha[2], kc), a_m, s);
        s = cfma(sload(a.beta[2], kc), zp, s);
        cpx<R> l0 = cscale(a.g[0], s);
        l0 = cfma(a.cx[0], cur.x, l0);
        l0 = {l0.re - cur.in0.re, l0.im - cur.in0.im};
        l0 = keep_if(live && kin, l0);
        const int slot = int(((k % 3) + 3) % 3);
        ring[slot][w][lane] = l0;
        // LDS writes complete, then the barrier; the global loads of the next
        // plane stay in flight across it
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0), vmcnt and expcnt left free
        __builtin_amdgcn_s_barrier();
        // ---- L_1 on plane k - 1 (rows 1..TY of the workgroup)
        const int64_t kb = k - 1;
        if (kb >= z0 && kb < z1 && w >= 1 && w <= TY) {
            const int sb = int(((kb % 3) + 3) % 3);
            const cpx<R> ym = ring[sb][w - 1][lane];
            const cpx<R> yp = ring[sb][w + 1][lane];
            const cpx<R> lx = from_below(l0_m1), rx = from_above(l0_m1);
            cpx<R> db = cadd(gxy, sload(a.gamma[2], kb));
            db = cadd(db, cscale(D_m1 - a.Dref, a.kD));
            cpx<R> t = cmul(db, l0_m1);
            t = cfma(wxm, lx, t);
            t = cfma(wxp, rx, t);
            t = cfma(wym, ym, t);
            t = cfma(wyp, yp, t);
            t = cfma(sload(a.alpha[2], kb), l0_m2, t);
            t = cfma(sload(a.beta[2], kb), l0, t);
            cpx<R> l1 = cscale(a.g[1], t);
            l1 = cfma(a.cx[1], x_m1, l1);
            l1 = {l1.re - a_m.re, l1.im - a_m.im};
            if (live && lane >= 1 && lane <= TXO) {
                const int64_t pb = prow + sz * kb;
                gstore(a.outA, pb, l0_m1);
                gstore(a.outB, pb, l1);
            }
        }
        l0_m2 = l0_m1;
        l0_m1 = l0;
        a_m = a_c;
        a_c = zp;
        x_m1 = cur.x;
        D_m1 = cur.D;
    };
    // The loads of plane k + 1 are issued before plane k is computed.  In
    // complex float the loop is unrolled by two, as in the three-level pass
    // below, so that no loaded value is copied across the back edge; in
    // complex double the unrolled loop measured slower (167.9 against 160.2
    // us per level at 256^3) and the operands are copied.  Planes past the
    // chunk read clamped, in-bounds nodes.
    if constexpr (sizeof(R) == 4) {
        PlaneIn pa = load_plane(z0 - 1);
        PlaneIn pb;
        for (int64_t k = z0 - 1; k <= z1; k += 2) {
            pb = load_plane(k + 1);
            step(k, pa);
            if (k + 1 > z1) break;
            pa = load_plane(k + 2);
            step(k + 1, pb);
        }
    } else {
        PlaneIn cur = load_plane(z0 - 1);
        for (int64_t k = z0 - 1; k <= z1; ++k) {
            const PlaneIn nxt = load_plane(k + 1);
            step(k, cur);
            cur = nxt;
        }
    }
}

template <typename R, int VAR>
__global__ __launch_bounds__(NW * 64) void k_cheb3d(ChebPass3DArgs<R> a) {
    __shared__ cpx<R> ring[3][NW][64];
    cheb3d_body<R, VAR>(a, blockIdx.x, ring);
}

// Three levels per pass.  Wavefront w holds grid row y0 - 2 + w and its
// lanes columns x0 - 2 .. x0 + 61.  At step k: every wavefront computes L_0
// on plane k and writes it to ring0, then the workgroup synchronises once;
// rows 1 .. NW3 - 2 compute L_1 on plane k - 1 (y-neighbours from ring0) and
// write it to ring1; rows 2 .. NW3 - 3 compute L_2 on plane k - 2, with the
// y-neighbours of L_1 from ring1 as written in step k - 1, i.e. before this
// step's barrier, so one barrier per plane orders every ring access (a slot
// is rewritten three steps after it was written, after every wavefront has
// passed the two barriers in between).  Lanes 2..61 of those rows store L_1
// and L_2.  Levels outside the grid are zero.
template <typename R, int VAR>
__device__ __forceinline__ void cheb3d3_body(const ChebPass3DArgs<R>& a, int tile, cpx<R> (*ring0)[NW3][64],
                                             cpx<R> (*ring1)[NW3][64]) {
    constexpr bool HD = VAR & 1, IN0 = VAR & 2, IN1 = VAR & 4;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tx = tile % a.tiles_x;
    const int rest = tile / a.tiles_x;
    const int ty = rest % a.tiles_y;
    const int tz = rest / a.tiles_y;
    const int64_t n0 = a.n0, n1 = a.n1, n2 = a.n2;
    const int64_t sy = n0, sz = n0 * n1;
    const int64_t gx = int64_t(tx) * TXO3 - 2 + lane;
    const int64_t gy = int64_t(ty) * TY3 - 2 + w;
    const int64_t z0 = int64_t(tz) * a.zc;
    const int64_t z1 = z0 + a.zc < n2 ? z0 + a.zc : n2;
    const bool xin = gx >= 0 && gx < n0, yin = gy >= 0 && gy < n1;
    const bool live = xin && yin;
    const int64_t cxl = gx < 0 ? 0 : (gx >= n0 ? n0 - 1 : gx);
    const int64_t cyl = gy < 0 ? 0 : (gy >= n1 ? n1 - 1 : gy);
    const int64_t cym = gy - 1 < 0 ? 0 : (gy - 1 >= n1 ? n1 - 1 : gy - 1);
    const int64_t cyp = gy + 1 < 0 ? 0 : (gy + 1 >= n1 ? n1 - 1 : gy + 1);
    const int64_t ex = lane == 0 ? gx - 1 : (lane == 63 ? gx + 1 : gx);
    const int64_t cex = ex < 0 ? 0 : (ex >= n0 ? n0 - 1 : ex);
    const cpx<R> wxm = keep_if(xin && gx > 0, gload(a.alpha[0], cxl));
    const cpx<R> wxp = keep_if(xin && gx < n0 - 1, gload(a.beta[0], cxl));
    const cpx<R> wym = keep_if(yin && gy > 0, gload(a.alpha[1], cyl));
    const cpx<R> wyp = keep_if(yin && gy < n1 - 1, gload(a.beta[1], cyl));
    const cpx<R> gxy = cadd(gload(a.gamma[0], cxl), gload(a.gamma[1], cyl));
    const cpx<R> zero{R(0), R(0)};
    const int64_t prow = cxl + sy * cyl;
    auto in1_at = [&](int64_t k, int64_t off) -> cpx<R> {
        if constexpr (!IN1) return zero;
        const bool ok = k >= 0 && k < n2;
        const cpx<R> v = gload(a.in1, off + sz * (ok ? k : 0));
        return keep_if(ok, v);
    };
    struct PlaneIn {
        cpx<R> x, in0, ym, yp, e, zp;
        R D;
    };
    auto load_plane = [&](int64_t k) -> PlaneIn {
        PlaneIn q;
        const bool kin = k >= 0 && k < n2;
        const int64_t kc = kin ? k : 0;
        const int64_t pk = prow + sz * kc;
        q.x = gload(a.x, pk);
        q.in0 = zero;
        if constexpr (IN0) q.in0 = gload(a.in0, pk);
        q.D = a.Dconst;
        if constexpr (HD) q.D = gload(a.D, pk);
        q.ym = q.yp = q.e = zero;
        if constexpr (IN1) {
            q.ym = gload(a.in1, cxl + sy * cym + sz * kc);
            q.yp = gload(a.in1, cxl + sy * cyp + sz * kc);
            q.e = gload(a.in1, cex + sy * cyl + sz * kc);
        }
        // in1 on plane k + 1 as loaded (a clamped plane past the grid): it is
        // masked where it is used, one step later, so that no wait for this
        // load (and, loads returning in order, for the whole prefetch) lands
        // in the step that issues it
        q.zp = zero;
        if constexpr (IN1) q.zp = gload(a.in1, prow + sz * (k + 1 >= 0 && k + 1 < n2 ? k + 1 : 0));
        return q;
    };
    auto diag_at = [&](int64_t k, R D) {
        cpx<R> d = cadd(gxy, sload(a.gamma[2], k));
        return cadd(d, cscale(D - a.Dref, a.kD));
    };
    cpx<R> a_m = in1_at(z0 - 3, prow);  // in1 on plane k - 1
    cpx<R> a_c = in1_at(z0 - 2, prow);  // in1 on plane k
    cpx<R> l0_m2 = zero, l0_m1 = zero;  // L_0 on planes k - 2, k - 1
    cpx<R> l1_m2 = zero, l1_m1 = zero;  // L_1 on planes k - 3, k - 2
    cpx<R> x_m1 = zero, x_m2 = zero;
    R D_m1 = a.Dconst, D_m2 = a.Dconst;
    // one plane step: L_0 on plane k from `cur` (its operands, loaded one or
    // two steps ahead, see below), L_1 on plane k - 1, L_2 on plane k - 2;
    // after_l0 runs once L_0 has read `cur` (complex double reloads it there)
    auto step = [&](int64_t k, const PlaneIn& cur, auto&& after_l0) {
        const cpx<R> zp = keep_if(k + 1 >= 0 && k + 1 < n2, cur.zp);
        // ---- L_0 on plane k (every row)
        const bool kin = k >= 0 && k < n2;  // uniform
        const int64_t kc = kin ? k : 0;
        cpx<R> left = from_below(a_c), right = from_above(a_c);
        if (lane == 0) left = cur.e;
        if (lane == 63) right = cur.e;
        cpx<R> s = cmul(diag_at(kc, cur.D), a_c);
        s = cfma(wxm, left, s);
        s = cfma(wxp, right, s);
        s = cfma(wym, cur.ym, s);
        s = cfma(wyp, cur.yp, s);
        s = cfma(sload(a.alpha[2], kc), a_m, s);
        s = cfma(sload(a.beta[2], kc), zp, s);
        cpx<R> l0 = cscale(a.g[0], s);
        l0 = cfma(a.cx[0], cur.x, l0);
        l0 = {l0.re - cur.in0.re, l0.im - cur.in0.im};
        l0 = keep_if(live && kin, l0);
        ring0[int(((k % 3) + 3) % 3)][w][lane] = l0;
        // the plane's operands are dead past L_0 but for x and D
        const cpx<R> xk = cur.x;
        const R Dk = cur.D;
        after_l0();
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0), vmcnt and expcnt left free
        __builtin_amdgcn_s_barrier();
        // ---- L_1 on plane k - 1 (rows 1 .. NW3 - 2)
        const int64_t k1 = k - 1;
        const bool k1in = k1 >= 0 && k1 < n2;
        const int64_t k1c = k1in ? k1 : 0;
        cpx<R> l1 = zero;
        if (k1 >= z0 - 1 && k1 <= z1 && w >= 1 && w <= NW3 - 2) {
            const int sb = int(((k1 % 3) + 3) % 3);
            const cpx<R> ym = ring0[sb][w - 1][lane];
            const cpx<R> yp = ring0[sb][w + 1][lane];
            const cpx<R> lx = from_below(l0_m1), rx = from_above(l0_m1);
            cpx<R> t = cmul(diag_at(k1c, D_m1), l0_m1);
            t = cfma(wxm, lx, t);
            t = cfma(wxp, rx, t);
            t = cfma(wym, ym, t);
            t = cfma(wyp, yp, t);
            t = cfma(sload(a.alpha[2], k1c), l0_m2, t);
            t = cfma(sload(a.beta[2], k1c), l0, t);
            l1 = cscale(a.g[1], t);
            l1 = cfma(a.cx[1], x_m1, l1);
            l1 = {l1.re - a_m.re, l1.im - a_m.im};
            l1 = keep_if(live && k1in, l1);
            ring1[sb][w][lane] = l1;
        }
        // ---- L_2 on plane k - 2 (rows 2 .. NW3 - 3); ring1's plane k - 2 was
        // written in step k - 1
        const int64_t k2 = k - 2;
        if (k2 >= z0 && k2 < z1 && w >= 2 && w <= NW3 - 3) {
            const int sb = int(((k2 % 3) + 3) % 3);
            const cpx<R> ym = ring1[sb][w - 1][lane];
            const cpx<R> yp = ring1[sb][w + 1][lane];
            const cpx<R> lx = from_below(l1_m1), rx = from_above(l1_m1);
            cpx<R> t = cmul(diag_at(k2, D_m2), l1_m1);
            t = cfma(wxm, lx, t);
            t = cfma(wxp, rx, t);
            t = cfma(wym, ym, t);
            t = cfma(wyp, yp, t);
            t = cfma(sload(a.alpha[2], k2), l1_m2, t);
            t = cfma(sload(a.beta[2], k2), l1, t);
            cpx<R> l2 = cscale(a.g[2], t);
            l2 = cfma(a.cx[2], x_m2, l2);
            l2 = {l2.re - l0_m2.re, l2.im - l0_m2.im};
            if (live && lane >= 2 && lane <= TXO3 + 1) {
                const int64_t pb = prow + sz * k2;
                gstore(a.outA, pb, l1_m1);
                gstore(a.outB, pb, l2);
            }
        }
        l0_m2 = l0_m1;
        l0_m1 = l0;
        l1_m2 = l1_m1;
        l1_m1 = l1;
        a_m = a_c;
        a_c = zp;
        x_m2 = x_m1;
        x_m1 = xk;
        D_m2 = D_m1;
        D_m1 = Dk;
    };
    // Software pipeline.  In complex float the operands of plane k + 2 are
    // loaded before plane k is computed, and the loop is unrolled by three so
    // that the three operand sets rotate through pa, pb and pc: no loaded
    // value is copied across the back edge (a copy waits for every load in
    // flight, loads returning in order).  With one plane in flight and a copy
    // per step the pass took 105.6 us per level at 256^3, unrolled by two
    // 95.3, with two planes 85.8.  In complex double an unrolled loop needs
    // more than the 128 registers of four wavefronts per SIMD (it spills), so
    // one operand set serves: the loads of plane k + 1 go into it as soon as
    // L_0 of plane k has read it, and stay in flight across the barrier, L_1
    // and L_2.  Planes past the chunk read clamped, in-bounds nodes.
    if constexpr (sizeof(R) == 4) {
        PlaneIn pa = load_plane(z0 - 2);
        PlaneIn pb = load_plane(z0 - 1);
        PlaneIn pc;
        for (int64_t k = z0 - 2; k <= z1 + 1; k += 3) {
            pc = load_plane(k + 2);
            step(k, pa, [] {});
            if (k + 1 > z1 + 1) break;
            pa = load_plane(k + 3);
            step(k + 1, pb, [] {});
            if (k + 2 > z1 + 1) break;
            pb = load_plane(k + 4);
            step(k + 2, pc, [] {});
        }
    } else {
        PlaneIn cur = load_plane(z0 - 2);
        for (int64_t k = z0 - 2; k <= z1 + 1; ++k) step(k, cur, [&] { cur = load_plane(k + 1); });
    }
}

template <typename R, int VAR>
__global__ __launch_bounds__(NW3 * 64) void k_cheb3d3(ChebPass3DArgs<R> a) {
    __shared__ cpx<R> ring0[3][NW3][64];
    __shared__ cpx<R> ring1[3][NW3][64];
    cheb3d3_body<R, VAR>(a, blockIdx.x, ring0, ring1);
}

// Batched form over grids of different sizes: a persistent grid of resident
// workgroups strides over the concatenated tile ranges of the jobs (job of
// index w from the lookup table, one entry per 64 indices, read through the
// scalar cache).  Every wavefront of a workgroup works on the same tile, so
// the per-plane barriers stay uniform; one more barrier after each tile keeps
// the next tile's first ring writes behind the last reads of this one.
template <typename R, int VAR>
__global__ __launch_bounds__(NW * 64) void k_cheb3d_batch(const Cheb3DJob<R>* jobs, const uint32_t* lut, int total) {
    __shared__ cpx<R> ring[3][NW][64];
    const __attribute__((address_space(4))) uint32_t* lq = (const __attribute__((address_space(4))) uint32_t*)(lut);
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        const uint32_t q = lq[b >> 6];
        const Cheb3DJob<R> job = sload_words(jobs + q);
        const int local = b - int(job.block0);
        if (local >= int(job.blocks)) continue;  // uniform: the whole workgroup skips
        cheb3d_body<R, VAR>(job.a, local, ring);
        __syncthreads();
    }
}

// Batched three-level passes: one workgroup per tile of the concatenated
// tile ranges (job from the lookup table as in k_cheb3d_batch), not
// persistent: a tile's z-march is long enough to amortise the launch, and the
// persistent loop's state pushed the complex-double kernel past its 128
// registers (40 bytes of spill per lane; a batch of one right-hand side took
// 4.09 s against 2.94 s for the single solve at 256^3).
template <typename R, int VAR>
__global__ __launch_bounds__(NW3 * 64) void k_cheb3d3_batch(const Cheb3DJob<R>* jobs, const uint32_t* lut, int total) {
    __shared__ cpx<R> ring0[3][NW3][64];
    __shared__ cpx<R> ring1[3][NW3][64];
    const __attribute__((address_space(4))) uint32_t* lq = (const __attribute__((address_space(4))) uint32_t*)(lut);
    const int b = blockIdx.x;
    if (b >= total) return;
    const uint32_t q = lq[b >> 6];
    const Cheb3DJob<R> job = sload_words(jobs + q);
    const int local = b - int(job.block0);
    if (local >= int(job.blocks)) return;  // uniform: padding of the job's range
    cheb3d3_body<R, VAR>(job.a, local, ring0, ring1);
}

template <typename R, int V>
void launch_one(const ChebPass3DArgs<R>& a, unsigned nb, hipStream_t s) {
    hipLaunchKernelGGL((k_cheb3d<R, V>), dim3(nb), dim3(NW * 64), 0, s, a);
}
template <typename R, int V>
void launch_one_batch(const Cheb3DJob<R>* jobs, const uint32_t* lut, unsigned nb, hipStream_t s) {
    // resident workgroups: occupancy (asked once per instantiation) times the
    // compute units, at most the total
    static int per_cu = 0;
    if (per_cu == 0) {
        int n = 0;
        HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, reinterpret_cast<const void*>(k_cheb3d_batch<R, V>), NW * 64, 0));
        per_cu = n > 0 ? n : 1;
    }
    int dev = 0, cus = 0;
    HIP_CHECK(hipGetDevice(&dev));
    HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int64_t g = int64_t(per_cu) * (cus > 0 ? cus : 1);
    if (g > int64_t(nb)) g = nb;
    hipLaunchKernelGGL((k_cheb3d_batch<R, V>), dim3(unsigned(g)), dim3(NW * 64), 0, s, jobs, lut, int(nb));
}
template <typename R, int... V>
void launch_var(const ChebPass3DArgs<R>& a, unsigned nb, int var, hipStream_t s, std::integer_sequence<int, V...>) {
    ((var == V ? launch_one<R, V>(a, nb, s) : void()), ...);
}
template <typename R, int V>
void launch_one3(const ChebPass3DArgs<R>& a, unsigned nb, hipStream_t s) {
    hipLaunchKernelGGL((k_cheb3d3<R, V>), dim3(nb), dim3(NW3 * 64), 0, s, a);
}
template <typename R, int... V>
void launch_var3(const ChebPass3DArgs<R>& a, unsigned nb, int var, hipStream_t s, std::integer_sequence<int, V...>) {
    ((var == V ? launch_one3<R, V>(a, nb, s) : void()), ...);
}
template <typename R, int V>
void launch_one3_batch(const Cheb3DJob<R>* jobs, const uint32_t* lut, unsigned nb, hipStream_t s) {
    hipLaunchKernelGGL((k_cheb3d3_batch<R, V>), dim3(nb), dim3(NW3 * 64), 0, s, jobs, lut, int(nb));
}
template <typename R, int... V>
void launch_var3_batch(const Cheb3DJob<R>* jobs, const uint32_t* lut, unsigned nb, int var, hipStream_t s,
                       std::integer_sequence<int, V...>) {
    ((var == V ? launch_one3_batch<R, V>(jobs, lut, nb, s) : void()), ...);
}
template <typename R, int... V>
void launch_var_batch(const Cheb3DJob<R>* jobs, const uint32_t* lut, unsigned nb, int var, hipStream_t s,
                      std::integer_sequence<int, V...>) {
    ((var == V ? launch_one_batch<R, V>(jobs, lut, nb, s) : void()), ...);
}

inline void check_launch(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(MXP_ERR_HIP, std::string("kernel launch failed (") + what + "): " + hipGetErrorString(e));
}

}  // namespace

template <typename R>
void cheb3d_geometry(ChebPass3DArgs<R>& a, int zc) {
    a.tiles_x = int((a.n0 + TXO - 1) / TXO);
    a.tiles_y = int((a.n1 + TY - 1) / TY);
    a.zc = zc > 0 ? zc : kZChunk;
    a.zchunks = int((a.n2 + a.zc - 1) / a.zc);
}

template <typename R>
void cheb3d3_geometry(ChebPass3DArgs<R>& a, int zc) {
    a.tiles_x = int((a.n0 + TXO3 - 1) / TXO3);
    a.tiles_y = int((a.n1 + TY3 - 1) / TY3);
    a.zc = zc > 0 ? zc : kZChunk;
    a.zchunks = int((a.n2 + a.zc - 1) / a.zc);
}

template <typename R>
int cheb3d_variant(const ChebPass3DArgs<R>& a) {
    return (a.D ? 1 : 0) | (a.in0 ? 2 : 0) | (a.in1 ? 4 : 0);
}

template <typename R>
void launch_cheb3d(const ChebPass3DArgs<R>& a, hipStream_t s) {
    const int64_t nb = int64_t(a.tiles_x) * a.tiles_y * a.zchunks;
    if (nb <= 0 || a.tiles_x <= 0) fail(MXP_ERR_INVALID_ARG, "3D pass geometry not set");
    if (nb > 0x7fffffff) fail(MXP_ERR_UNSUPPORTED, "grid too large for the 3D pass");
    if (!a.x || !a.outA || !a.outB) fail(MXP_ERR_INVALID_ARG, "3D pass needs x and both outputs");
    launch_var<R>(a, unsigned(nb), cheb3d_variant(a), s, std::make_integer_sequence<int, 8>{});
    check_launch("3D Clenshaw pass");
}

template <typename R>
void launch_cheb3d3(const ChebPass3DArgs<R>& a, hipStream_t s) {
    const int64_t nb = int64_t(a.tiles_x) * a.tiles_y * a.zchunks;
    if (nb <= 0 || a.tiles_x <= 0) fail(MXP_ERR_INVALID_ARG, "3D pass geometry not set");
    if (nb > 0x7fffffff) fail(MXP_ERR_UNSUPPORTED, "grid too large for the 3D pass");
    if (!a.x || !a.outA || !a.outB) fail(MXP_ERR_INVALID_ARG, "3D pass needs x and both outputs");
    launch_var3<R>(a, unsigned(nb), cheb3d_variant(a), s, std::make_integer_sequence<int, 8>{});
    check_launch("3D three-level Clenshaw pass");
}

template <typename R>
void launch_cheb3d3_batch(const Cheb3DJob<R>* jobs, const uint32_t* lut, int64_t total_blocks, int variant,
                          hipStream_t s) {
    if (total_blocks <= 0) return;
    if (total_blocks > 0x7fffffff) fail(MXP_ERR_UNSUPPORTED, "batched 3D pass too large");
    launch_var3_batch<R>(jobs, lut, unsigned(total_blocks), variant, s, std::make_integer_sequence<int, 8>{});
    check_launch("batched 3D three-level Clenshaw pass");
}

template <typename R>
void launch_cheb3d_batch(const Cheb3DJob<R>* jobs, const uint32_t* lut, int64_t total_blocks, int variant,
                         hipStream_t s) {
    if (total_blocks <= 0) return;
    if (total_blocks > 0x7fffffff) fail(MXP_ERR_UNSUPPORTED, "batched 3D pass too large");
    launch_var_batch<R>(jobs, lut, unsigned(total_blocks), variant, s, std::make_integer_sequence<int, 8>{});
    check_launch("batched 3D Clenshaw pass");
}

template void cheb3d_geometry<float>(ChebPass3DArgs<float>&, int);
template void cheb3d_geometry<double>(ChebPass3DArgs<double>&, int);
template void cheb3d3_geometry<float>(ChebPass3DArgs<float>&, int);
template void cheb3d3_geometry<double>(ChebPass3DArgs<double>&, int);
template void launch_cheb3d3<float>(const ChebPass3DArgs<float>&, hipStream_t);
template void launch_cheb3d3<double>(const ChebPass3DArgs<double>&, hipStream_t);
template void launch_cheb3d3_batch<float>(const Cheb3DJob<float>*, const uint32_t*, int64_t, int, hipStream_t);
template void launch_cheb3d3_batch<double>(const Cheb3DJob<double>*, const uint32_t*, int64_t, int, hipStream_t);
template int cheb3d_variant<float>(const ChebPass3DArgs<float>&);
template int cheb3d_variant<double>(const ChebPass3DArgs<double>&);
template void launch_cheb3d<float>(const ChebPass3DArgs<float>&, hipStream_t);
template void launch_cheb3d<double>(const ChebPass3DArgs<double>&, hipStream_t);
template void launch_cheb3d_batch<float>(const Cheb3DJob<float>*, const uint32_t*, int64_t, int, hipStream_t);
template void launch_cheb3d_batch<double>(const Cheb3DJob<double>*, const uint32_t*, int64_t, int, hipStream_t);

}  // namespace mxp
