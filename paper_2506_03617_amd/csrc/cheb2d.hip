// Temporally blocked Clenshaw passes for 2D grids (gfx950).
//
// One pass computes K consecutive levels of the Clenshaw recurrence
//
//   L_l = cx_l x + g_l S(L_{l-1}) - L_{l-2},   last level of a final pass:
//   L   = post * (cx x + g S(L_prev) - L_prevprev) + e3 add
//
// where S is the shifted stencil operator scaled by h^2 (so that an interior
// node has unit neighbour weights) and L_{-2}, L_{-1} are the pass inputs (two
// levels of the previous pass, or zero for the first pass of a series).  Each
// HBM pass reads the two input levels, x and D once and writes only the last
// two levels, so K Clenshaw steps cost about one step's traffic.
//
// Work decomposition: every 64-wide wavefront owns a strip of NX*64 columns
// (W output columns plus K halo columns on each side, recomputed by the
// neighbouring strip) and a segment of Ly output rows, and marches along y.
// Row r of level l is computed when row r + l - 1 of the inputs arrives:
//  * each level keeps a three-row register window (the row loop is unrolled by
//    three, so window slots are compile-time and rotate by renaming);
//  * x and the per-node diagonal of the last K+1 rows sit in a per-lane LDS
//    ring (each lane reads only what it wrote: no barriers);
//  * x-neighbours come from the adjacent lane through DPP wavefront shifts;
//  * row j+1 is fetched while the levels of row j are computed;
//  * a level is skipped on rows no output depends on;
//  * the per-row diagonal term goes through the scalar cache: in complex
//    double the three rows of a group are loaded together at the start of
//    the group (one wait per group instead of one per row: 8% faster
//    there, 6% slower in complex float, which loads it per row).
// Waves are independent.
#include <hip/hip_runtime.h>

#include <utility>

#include "devmem.h"
#include "kernels.h"
#include "mxp_internal.h"

namespace mxp {

namespace {

template <typename R>
__device__ __forceinline__ cpx<R> csel(bool c, cpx<R> a, cpx<R> b) {
    return {c ? a.re : b.re, c ? a.im : b.im};
}

// DPP wavefront shifts: lane l receives lane l-1 (from_below) or lane l+1
// (from_above); with bound_ctrl set, lanes without a source read 0.
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

// 32-bit byte offsets from a uniform base: the loads use the SGPR-base +
// VGPR-offset form (launch_cheb2d guarantees vectors below 4 GiB).
template <typename T>
__device__ __forceinline__ T ld(const T* base, uint32_t byte_off) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <typename T>
__device__ __forceinline__ void st(T* base, uint32_t byte_off, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off) = v;
}

// Wave-uniform table reads through the constant address space, so they become
// scalar loads (their own counter: they never wait on the row loads).
template <typename R>
__device__ __forceinline__ cpx<R> sload(const cpx<R>* p, int idx) {
    const __attribute__((address_space(4))) R* q = (const __attribute__((address_space(4))) R*)(p);
    return {q[2 * idx], q[2 * idx + 1]};
}
template <typename R>
__device__ __forceinline__ R sload_r(const R* p, int idx) {
    return ((const __attribute__((address_space(4))) R*)(p))[idx];
}
// A whole uniform struct through the scalar cache, one dword at a time.
template <class T>
__device__ __forceinline__ T sload_words(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "dword-sized struct expected");
    const __attribute__((address_space(4))) uint32_t* q = (const __attribute__((address_space(4))) uint32_t*)(p);
    uint32_t w[sizeof(T) / 4];
#pragma unroll
    for (unsigned i = 0; i < sizeof(T) / 4; ++i) w[i] = q[i];
    return __builtin_bit_cast(T, w);
}

// The fields of ChebPassArgs a pass reads, copied out of the kernel argument
// (holding a reference to the argument would force it into scratch memory).
template <typename R, int K>
struct PassParams {
    int n0, n1;
    const cpx<R>* ay;
    const cpx<R>* by;
    const cpx<R>* gy;
    const R* D;
    const R* aby;  // absorbing faces: h^2-scaled y weights (nullptr when absent)
    R Dconst, Dref, e3, post;
    cpx<R> kD;
    const cpx<R>* x;
    const cpx<R>* in0;
    const cpx<R>* in1;
    const cpx<R>* add;
    cpx<R>* outA;
    cpx<R>* outB;
    cpx<R> cx[K];
    R g[K];
    int iy0, iy1;
    int in0_zero, in1_zero, D_const, final_pass;
    __device__ __forceinline__ void from(const ChebPassArgs<R>& s) {
        n0 = int(s.n0);
        n1 = int(s.n1);
        ay = s.ay;
        by = s.by;
        gy = s.gy;
        D = s.D;
        aby = s.aby;
        Dconst = s.Dconst;
        Dref = s.Dref;
        e3 = s.e3;
        post = s.post;
        kD = s.kD;
        x = s.x;
        in0 = s.in0;
        in1 = s.in1;
        add = s.add;
        outA = s.outA;
        outB = s.outB;
#pragma unroll
        for (int l = 0; l < K; ++l) {
            cx[l] = s.cx[l];
            g[l] = s.g[l];
        }
        iy0 = int(s.iy0);
        iy1 = int(s.iy1);
        in0_zero = s.in0_zero;
        in1_zero = s.in1_zero;
        D_const = s.D_const;
        final_pass = s.final_pass;
    }
};

// Rows of x / diagonal history kept in LDS: a power of two >= K + 1, so the
// ring slot of row r is r & (ring - 1).
template <int K>
constexpr int ring_rows() { return K + 1 <= 2 ? 2 : (K + 1 <= 4 ? 4 : (K + 1 <= 8 ? 8 : 16)); }

template <typename R, int K, int NX>
struct Pass2D {
    static constexpr int M = ring_rows<K>();
    using Params = PassParams<R, K>;
    int cbase, Y0, Y1, jstart, lane;
    bool cin[NX], cout[NX];
    uint32_t ccl[NX];                 // clamped column of each element
    cpx<R> axv[NX], bxv[NX], gxv[NX];
    R abxv[NX];                       // absorbing faces: h^2-scaled x weights
    bool x_interior;
    cpx<R> Lw[K + 2][3][NX];          // level windows, slot = row mod 3
    cpx<R> P0[NX], P1[NX], PX[NX];    // row j+1, fetched one step ahead
    R PD[NX];
    cpx<R> PA[NX];                    // addend at row (j+1) - K, fetched one step ahead

    // Issues the loads of row `row` (clamped into the grid; masked when used).
    __device__ __forceinline__ void fetch(const Params& a, int row) {
        const int rcl = row < 0 ? 0 : (row >= a.n1 ? a.n1 - 1 : row);
        const uint32_t rbase = uint32_t(rcl) * uint32_t(a.n0);
#pragma unroll
        for (int e = 0; e < NX; ++e) {
            const uint32_t idx = rbase + ccl[e];
            P0[e] = ld(a.in0, idx * uint32_t(sizeof(cpx<R>)));
            P1[e] = ld(a.in1, idx * uint32_t(sizeof(cpx<R>)));
            PX[e] = ld(a.x, idx * uint32_t(sizeof(cpx<R>)));
            PD[e] = ld(a.D, idx * uint32_t(sizeof(R)));
        }
        const int ra = row - K;
        const int racl = ra < 0 ? 0 : (ra >= a.n1 ? a.n1 - 1 : ra);
#pragma unroll
        for (int e = 0; e < NX; ++e)
            PA[e] = ld(a.add, (uint32_t(racl) * uint32_t(a.n0) + ccl[e]) * uint32_t(sizeof(cpx<R>)));
    }

    // Level l (2..K+1) at row r = j - l + 1; every window slot is compile-time.
    // FAST: every level of this step is interior and needed (the steady state).
    template <int PH, int l, bool FAST>
    __device__ __forceinline__ void level(const Params& a, const cpx<R> (&xr)[K][NX],
                                          const cpx<R> (&dr)[K][NX], int j, const cpx<R>* addv) {
        constexpr int i = l - 2;                          // level index within the pass
        constexpr int s_up = ((PH - l + 2) % 3 + 3) % 3;  // row r+1 of level l-1
        constexpr int s_c = ((PH - l + 1) % 3 + 3) % 3;   // row r
        constexpr int s_dn = ((PH - l) % 3 + 3) % 3;      // row r-1
        const int r = j - l + 1;
        // rows this level must provide: the outputs' dependency cone
        if (!FAST && (r < Y0 - (K - 1 - i) || r >= Y1 + (K - 1 - i))) return;
        const cpx<R> zero{R(0), R(0)};
        const bool rv = FAST || (r >= 0 && r < a.n1);
        const cpx<R> cxl = a.cx[i];
        const R gl = a.g[i];
        const bool interior = FAST || (x_interior && (r >= a.iy0) && (r < a.iy1));
        cpx<R> v[NX + 2];
#pragma unroll
        for (int e = 0; e < NX; ++e) v[e + 1] = Lw[l - 1][s_c][e];
        v[0] = from_below(Lw[l - 1][s_c][NX - 1]);
        v[NX + 1] = from_above(Lw[l - 1][s_c][0]);
        cpx<R> nw[NX];
        if (interior) {
#pragma unroll
            for (int e = 0; e < NX; ++e) {
                const cpx<R> xv = xr[i][e];
                const cpx<R> dv = dr[i][e];
                const cpx<R> up = Lw[l - 1][s_up][e], dn = Lw[l - 1][s_dn][e];
                const cpx<R> c = v[e + 1], prev2 = Lw[l - 2][s_c][e];
                // s = (L + R + U + D) + diag * c   (unit neighbour weights)
                cpx<R> s = {(v[e].re + v[e + 2].re) + (up.re + dn.re), (v[e].im + v[e + 2].im) + (up.im + dn.im)};
                s.re = fma(dv.re, c.re, fma(-dv.im, c.im, s.re));
                s.im = fma(dv.re, c.im, fma(dv.im, c.re, s.im));
                // val = g s - prev2 + cx x
                cpx<R> val = {fma(gl, s.re, -prev2.re), fma(gl, s.im, -prev2.im)};
                val.re = fma(cxl.re, xv.re, fma(-cxl.im, xv.im, val.re));
                val.im = fma(cxl.re, xv.im, fma(cxl.im, xv.re, val.im));
                nw[e] = val;
            }
        } else {
            const int rc = __builtin_amdgcn_readfirstlane(rv ? r : 0);
            const cpx<R> ayr = sload(a.ay, rc), byr = sload(a.by, rc);
#pragma unroll
            for (int e = 0; e < NX; ++e) {
                const cpx<R> xv = xr[i][e];
                const cpx<R> dv = dr[i][e];
                const cpx<R> up = Lw[l - 1][s_up][e], dn = Lw[l - 1][s_dn][e];
                const cpx<R> c = v[e + 1], prev2 = Lw[l - 2][s_c][e];
                cpx<R> s;
                s.re = fma(dv.re, c.re, -dv.im * c.im);
                s.im = fma(dv.re, c.im, dv.im * c.re);
                s.re = fma(axv[e].re, v[e].re, fma(-axv[e].im, v[e].im, s.re));
                s.im = fma(axv[e].re, v[e].im, fma(axv[e].im, v[e].re, s.im));
                s.re = fma(bxv[e].re, v[e + 2].re, fma(-bxv[e].im, v[e + 2].im, s.re));
                s.im = fma(bxv[e].re, v[e + 2].im, fma(bxv[e].im, v[e + 2].re, s.im));
                s.re = fma(ayr.re, dn.re, fma(-ayr.im, dn.im, s.re));
                s.im = fma(ayr.re, dn.im, fma(ayr.im, dn.re, s.im));
                s.re = fma(byr.re, up.re, fma(-byr.im, up.im, s.re));
                s.im = fma(byr.re, up.im, fma(byr.im, up.re, s.im));
                cpx<R> val = {fma(gl, s.re, -prev2.re), fma(gl, s.im, -prev2.im)};
                val.re = fma(cxl.re, xv.re, fma(-cxl.im, xv.im, val.re));
                val.im = fma(cxl.re, xv.im, fma(cxl.im, xv.re, val.im));
                nw[e] = csel(rv && cin[e], val, zero);
            }
        }
        if (l == K + 1) {
            // last level: post * value + e3 * add (post = 1, e3 = 0 unless this
            // pass ends the series; branch-free to keep the row group one block)
#pragma unroll
            for (int e = 0; e < NX; ++e) {
                const R e3 = (FAST || (rv && cin[e])) ? a.e3 : R(0);
                nw[e].re = fma(e3, addv[e].re, a.post * nw[e].re);
                nw[e].im = fma(e3, addv[e].im, a.post * nw[e].im);
            }
        }
#pragma unroll
        for (int e = 0; e < NX; ++e) Lw[l][s_c][e] = nw[e];
    }

    template <int PH, bool FAST, int... Ls>
    __device__ __forceinline__ void levels(const Params& a, const cpx<R> (&xr)[K][NX],
                                           const cpx<R> (&dr)[K][NX], int j, const cpx<R>* addv,
                                           std::integer_sequence<int, Ls...>) {
        (level<PH, Ls + 2, FAST>(a, xr, dr, j, addv), ...);
    }

    // One row step at iteration j (PH = (j - jstart) mod 3).
    template <int PH, bool FAST>
    __device__ __forceinline__ void step_impl(const Params& a, cpx<R>* __restrict__ xs, cpx<R>* __restrict__ dg,
                                              const cpx<R> (&gyg)[3], int j) {
        const cpx<R> zero{R(0), R(0)};
        const bool rin = (j >= 0 && j < a.n1);
        const int slot_j = j & (M - 1);
        constexpr int sj = PH;
        // row j (fetched during the previous step) into the windows and the ring
        cpx<R> gyj;
        if constexpr (sizeof(R) == 8) {
            gyj = gyg[PH];
        } else {
            const int rj = __builtin_amdgcn_readfirstlane(rin ? j : 0);
            gyj = sload(a.gy, rj);
        }
#pragma unroll
        for (int e = 0; e < NX; ++e) {
            const bool ok = rin && cin[e];
            Lw[0][sj][e] = csel(ok && !a.in0_zero, P0[e], zero);
            Lw[1][sj][e] = csel(ok && !a.in1_zero, P1[e], zero);
            xs[slot_j * 64 * NX + lane * NX + e] = csel(ok, PX[e], zero);
            const R dd = (a.D_const ? a.Dconst : PD[e]) - a.Dref;
            cpx<R> dgv = {gxv[e].re + gyj.re + a.kD.re * dd, gxv[e].im + gyj.im + a.kD.im * dd};
            if (a.aby) {  // absorbing faces: 2 i omega h sqrt(D_p) per face of the node
                const R w = abxv[e] + sload_r(a.aby, __builtin_amdgcn_readfirstlane(rin ? j : 0));
                if (w != R(0)) dgv.im += w * sqrt(PD[e]);
            }
            dg[slot_j * 64 * NX + lane * NX + e] = dgv;
        }
        cpx<R> addv[NX];
#pragma unroll
        for (int e = 0; e < NX; ++e) addv[e] = PA[e];
        // x and the diagonal of rows j-1 .. j-K (level i works on row j-1-i),
        // read from the ring together so one wait covers them
        cpx<R> xr[K][NX], dr[K][NX];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int sl = (j - 1 - i) & (M - 1);
#pragma unroll
            for (int e = 0; e < NX; ++e) {
                xr[i][e] = xs[sl * 64 * NX + lane * NX + e];
                dr[i][e] = dg[sl * 64 * NX + lane * NX + e];
            }
        }
        fetch(a, j + 1);
        levels<PH, FAST>(a, xr, dr, j, addv, std::make_integer_sequence<int, K>{});
    }

    // Outputs of the row group starting at j0: level K+1 rows j0-K .. j0-K+2
    // (outB) and level K rows j0-K+1 .. j0-K+3 (outA), all still in the windows.
    template <int PH>
    __device__ __forceinline__ void store_row(const Params& a, int j) {
        const int rB = j - K;
        constexpr int sB = ((PH - K) % 3 + 3) % 3;
        if (rB >= Y0 && rB < Y1) {
#pragma unroll
            for (int e = 0; e < NX; ++e)
                if (cout[e])
                    st(a.outB, (uint32_t(rB) * uint32_t(a.n0) + ccl[e]) * uint32_t(sizeof(cpx<R>)),
                       Lw[K + 1][sB][e]);
        }
        if (!a.final_pass) {
            const int rA = j - K + 1;
            constexpr int sA = ((PH - K + 1) % 3 + 3) % 3;
            if (rA >= Y0 && rA < Y1) {
#pragma unroll
                for (int e = 0; e < NX; ++e)
                    if (cout[e])
                        st(a.outA, (uint32_t(rA) * uint32_t(a.n0) + ccl[e]) * uint32_t(sizeof(cpx<R>)),
                           Lw[K][sA][e]);
            }
        }
    }

    // Three row steps j0, j0+1, j0+2.  In the steady state (every level row of
    // the group needed and interior) one uniform test selects a body free of
    // branches, so the scheduler can overlap the level chains of the rows.
    // Scalar loads of the y diagonal term of rows j .. j+2 (clamped rows are
    // never used unmasked).
    __device__ __forceinline__ void load_gy(const Params& a, int j, cpx<R> (&g)[3]) const {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int r = j + q;
            g[q] = sload(a.gy, __builtin_amdgcn_readfirstlane(r >= 0 && r < a.n1 ? r : 0));
        }
    }

    __device__ __forceinline__ void group(const Params& a, cpx<R>* __restrict__ xs, cpx<R>* __restrict__ dg,
                                          int j0) {
        cpx<R> gyg[3] = {};
        if constexpr (sizeof(R) == 8) load_gy(a, j0, gyg);
        const bool fast = x_interior && (j0 >= Y0 + K) && (j0 - K >= a.iy0) && (j0 + 1 < a.iy1);
        if (fast) {
            step_impl<0, true>(a, xs, dg, gyg, j0);
            step_impl<1, true>(a, xs, dg, gyg, j0 + 1);
            step_impl<2, true>(a, xs, dg, gyg, j0 + 2);
        } else {
            step_impl<0, false>(a, xs, dg, gyg, j0);
            step_impl<1, false>(a, xs, dg, gyg, j0 + 1);
            step_impl<2, false>(a, xs, dg, gyg, j0 + 2);
        }
        store_row<0>(a, j0);
        store_row<1>(a, j0 + 1);
        store_row<2>(a, j0 + 2);
    }
};

// One wavefront's share of a pass: strip and row segment number wv of the
// grid (strips vary fastest), with its LDS ring rows xs and dg.
template <typename R, int K, int NX>
__device__ __forceinline__ void pass2d(const ChebPassArgs<R>& a, int wv, cpx<R>* xs, cpx<R>* dg) {
    const int lane = threadIdx.x & 63;
    const int strip = wv % a.strips;
    const int seg = wv / a.strips;
    PassParams<R, K> pp;
    pp.from(a);
    Pass2D<R, K, NX> ps;
    ps.Y0 = seg * a.Ly;
    if (ps.Y0 >= pp.n1) return;  // the whole wavefront leaves together
    ps.Y1 = (ps.Y0 + a.Ly < pp.n1) ? ps.Y0 + a.Ly : pp.n1;
    const int X0 = strip * a.W;
    ps.cbase = X0 - K + lane * NX;
    ps.lane = lane;
    const cpx<R> zero{R(0), R(0)};
#pragma unroll
    for (int e = 0; e < NX; ++e) {
        const int c = ps.cbase + e;
        ps.cin[e] = (c >= 0 && c < pp.n0);
        ps.cout[e] = ps.cin[e] && c >= X0 && c < X0 + a.W;
        ps.ccl[e] = uint32_t(c < 0 ? 0 : (c >= pp.n0 ? pp.n0 - 1 : c));
        ps.axv[e] = csel(ps.cin[e], a.ax[ps.ccl[e]], zero);
        ps.bxv[e] = csel(ps.cin[e], a.bx[ps.ccl[e]], zero);
        ps.gxv[e] = csel(ps.cin[e], a.gx[ps.ccl[e]], zero);
        ps.abxv[e] = (a.abx && ps.cin[e]) ? a.abx[ps.ccl[e]] : R(0);
    }
    // interior strip: every column has unit neighbour weights
    ps.x_interior = (X0 - K >= a.ix0) && (X0 - K + 64 * NX <= a.ix1);
#pragma unroll
    for (int l = 0; l < K + 2; ++l)
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int e = 0; e < NX; ++e) ps.Lw[l][q][e] = zero;
    ps.jstart = ps.Y0 - K;
    ps.fetch(pp, ps.jstart);
    const int jend = ps.Y1 + K;  // iterations past jend only touch rows outside [Y0, Y1)
    for (int j = ps.jstart; j < jend; j += 3) ps.group(pp, xs, dg, j);
}

template <typename R, int K, int NX>
__global__ __launch_bounds__(256) void k_cheb2d(ChebPassArgs<R> a) {
    constexpr int M = ring_rows<K>();
    __shared__ cpx<R> xs_all[4][M * 64 * NX];
    __shared__ cpx<R> dg_all[4][M * 64 * NX];
    const int wid = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    pass2d<R, K, NX>(a, int(blockIdx.x) * 4 + wid, xs_all[wid], dg_all[wid]);
}

// Batched form over the passes of many grids (one K, NX): a persistent grid
// of resident workgroups strides over the concatenated workgroup ranges of
// the jobs.  The job of range index w comes from a lookup table with one
// entry per 64 indices, and its description is read through the scalar
// cache (uniform across the workgroup).  The wavefronts of a workgroup share
// no data, so each leaves a job's range on its own.
template <typename R, int K, int NX>
__device__ __forceinline__ void cheb2d_batch_body(const Cheb2DJob<R>* jobs, const uint32_t* lut, int total) {
    constexpr int M = ring_rows<K>();
    __shared__ cpx<R> xs_all[4][M * 64 * NX];
    __shared__ cpx<R> dg_all[4][M * 64 * NX];
    const int wid = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const __attribute__((address_space(4))) uint32_t* lq = (const __attribute__((address_space(4))) uint32_t*)(lut);
    for (int w = blockIdx.x; w < total; w += gridDim.x) {
        const uint32_t q = lq[w >> 6];
        const Cheb2DJob<R> job = sload_words(jobs + q);
        const int local = w - int(job.block0);
        if (local >= int(job.blocks)) continue;
        pass2d<R, K, NX>(job.a, local * 4 + wid, xs_all[wid], dg_all[wid]);
    }
}

template <typename R, int K, int NX>
__global__ __launch_bounds__(256) void k_cheb2d_batch(const Cheb2DJob<R>* jobs, const uint32_t* lut, int total) {
    cheb2d_batch_body<R, K, NX>(jobs, lut, total);
}
// The same, held to two wavefronts per SIMD: for the shapes whose
// single-grid pass fits two and whose loop state would otherwise tip the
// register count past 256 (complex double, K = 6, NX = 1).
template <typename R, int K, int NX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_cheb2d_batch_w2(
    const Cheb2DJob<R>* jobs, const uint32_t* lut, int total) {
    cheb2d_batch_body<R, K, NX>(jobs, lut, total);
}

template <typename R, int K, int NX>
void launch_k(const ChebPassArgs<R>& a, hipStream_t s) {
    if constexpr (sizeof(R) == 8 && NX == 2 && K > 3) {
        // register- and LDS-limited shape: not built
        (void)a;
        (void)s;
        fail(MXP_ERR_UNSUPPORTED, "complex-double passes with NX = 2 support K <= 3");
    } else {
        const int waves = a.strips * a.segs;
        const int blocks = (waves + 3) / 4;
        hipLaunchKernelGGL((k_cheb2d<R, K, NX>), dim3(blocks), dim3(256), 0, s, a);
    }
}

// Resident workgroups of a batched kernel: its occupancy per compute unit
// (asked once per instantiation) times the device's compute units, at most
// `total`.
template <typename Kern>
int64_t persistent_grid(Kern kern, int64_t total) {
    static int per_cu = 0;
    if (per_cu == 0) {
        int n = 0;
        HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(kern), 256, 0));
        per_cu = n > 0 ? n : 1;
    }
    int dev = 0, cus = 0;
    HIP_CHECK(hipGetDevice(&dev));
    HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int64_t slots = int64_t(per_cu) * (cus > 0 ? cus : 1);
    return total < slots ? total : slots;
}

template <typename R, int K, int NX>
void launch_k_batch(const Cheb2DJob<R>* jobs, const uint32_t* lut, int64_t total, hipStream_t s) {
    if constexpr (sizeof(R) == 8 && NX == 2 && K > 3) {
        (void)jobs;
        (void)lut;
        (void)total;
        (void)s;
        fail(MXP_ERR_UNSUPPORTED, "complex-double passes with NX = 2 support K <= 3");
    } else {
        if constexpr (sizeof(R) == 8 && K == 6 && NX == 1) {
            const int64_t g = persistent_grid(k_cheb2d_batch_w2<R, K, NX>, total);
            hipLaunchKernelGGL((k_cheb2d_batch_w2<R, K, NX>), dim3(unsigned(g)), dim3(256), 0, s, jobs, lut,
                               int(total));
        } else {
            const int64_t g = persistent_grid(k_cheb2d_batch<R, K, NX>, total);
            hipLaunchKernelGGL((k_cheb2d_batch<R, K, NX>), dim3(unsigned(g)), dim3(256), 0, s, jobs, lut,
                               int(total));
        }
    }
}

template <typename R, int NX>
void launch_nx_batch(const Cheb2DJob<R>* jobs, const uint32_t* lut, int64_t total, int K, hipStream_t s) {
    switch (K) {
        case 1: launch_k_batch<R, 1, NX>(jobs, lut, total, s); break;
        case 2: launch_k_batch<R, 2, NX>(jobs, lut, total, s); break;
        case 3: launch_k_batch<R, 3, NX>(jobs, lut, total, s); break;
        case 4: launch_k_batch<R, 4, NX>(jobs, lut, total, s); break;
        case 5: launch_k_batch<R, 5, NX>(jobs, lut, total, s); break;
        case 6: launch_k_batch<R, 6, NX>(jobs, lut, total, s); break;
        case 7: launch_k_batch<R, 7, NX>(jobs, lut, total, s); break;
        case 8: launch_k_batch<R, 8, NX>(jobs, lut, total, s); break;
        default: fail(MXP_ERR_INVALID_ARG, "fused level count must be 1..8");
    }
}

template <typename R, int NX>
void launch_nx(const ChebPassArgs<R>& a, int K, hipStream_t s) {
    switch (K) {
        case 1: launch_k<R, 1, NX>(a, s); break;
        case 2: launch_k<R, 2, NX>(a, s); break;
        case 3: launch_k<R, 3, NX>(a, s); break;
        case 4: launch_k<R, 4, NX>(a, s); break;
        case 5: launch_k<R, 5, NX>(a, s); break;
        case 6: launch_k<R, 6, NX>(a, s); break;
        case 7: launch_k<R, 7, NX>(a, s); break;
        case 8: launch_k<R, 8, NX>(a, s); break;
        default: fail(MXP_ERR_INVALID_ARG, "fused level count must be 1..8");
    }
}

}  // namespace

template <typename R>
void cheb2d_geometry(ChebPassArgs<R>& a, int K, int NX, int Ly) {
    a.W = NX * 64 - 2 * K;
    a.strips = int((a.n0 + a.W - 1) / a.W);
    a.Ly = Ly;
    a.segs = int((a.n1 + Ly - 1) / Ly);
}
template void cheb2d_geometry<float>(ChebPassArgs<float>&, int, int, int);
template void cheb2d_geometry<double>(ChebPassArgs<double>&, int, int, int);

template <typename R>
ChebPassArgs<R> prepare_cheb2d(const ChebPassArgs<R>& in, int K, int NX) {
    if (K < 1 || K > kMaxFused) fail(MXP_ERR_INVALID_ARG, "fused level count out of range");
    if (NX != 1 && NX != 2) fail(MXP_ERR_INVALID_ARG, "NX must be 1 or 2");
    if (uint64_t(in.n0) * uint64_t(in.n1) * sizeof(cpx<R>) >= (uint64_t(1) << 32))
        fail(MXP_ERR_UNSUPPORTED, "fused 2D passes need vectors below 4 GiB");
    if (in.W != NX * 64 - 2 * K || in.W <= 0) fail(MXP_ERR_INVALID_ARG, "pass geometry does not match K, NX");
    // every pointer the kernel reads must be valid: absent operands read x and are ignored
    ChebPassArgs<R> a = in;
    a.in0_zero = (a.in0 == nullptr);
    a.in1_zero = (a.in1 == nullptr);
    if (!a.in0) a.in0 = a.x;
    if (!a.in1) a.in1 = a.x;
    a.D_const = (a.D == nullptr);
    if (!a.D) a.D = reinterpret_cast<const R*>(a.x);  // read as reals within x's bytes
    if (!a.add) {
        a.add = a.x;
        a.e3 = R(0);
    }
    if (!a.final_pass && !a.outA) fail(MXP_ERR_INVALID_ARG, "a non-final pass writes two levels");
    return a;
}

template <typename R>
int64_t cheb2d_blocks(const ChebPassArgs<R>& a) {
    return (int64_t(a.strips) * a.segs + 3) / 4;
}

template <typename R>
void launch_cheb2d(const ChebPassArgs<R>& in, int K, int NX, hipStream_t s) {
    const ChebPassArgs<R> a = prepare_cheb2d(in, K, NX);
    if (NX == 1)
        launch_nx<R, 1>(a, K, s);
    else
        launch_nx<R, 2>(a, K, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(MXP_ERR_HIP, std::string("cheb2d launch failed: ") + hipGetErrorString(e));
}

template <typename R>
void launch_cheb2d_batch(const Cheb2DJob<R>* jobs, const uint32_t* lut, int64_t total_blocks, int K, int NX,
                         hipStream_t s) {
    if (total_blocks <= 0) return;
    if (total_blocks > 0x7fffffff) fail(MXP_ERR_UNSUPPORTED, "batched 2D pass too large");
    if (NX == 1)
        launch_nx_batch<R, 1>(jobs, lut, total_blocks, K, s);
    else if (NX == 2)
        launch_nx_batch<R, 2>(jobs, lut, total_blocks, K, s);
    else
        fail(MXP_ERR_INVALID_ARG, "NX must be 1 or 2");
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(MXP_ERR_HIP, std::string("batched cheb2d launch failed: ") + hipGetErrorString(e));
}
template ChebPassArgs<float> prepare_cheb2d<float>(const ChebPassArgs<float>&, int, int);
template ChebPassArgs<double> prepare_cheb2d<double>(const ChebPassArgs<double>&, int, int);
template int64_t cheb2d_blocks<float>(const ChebPassArgs<float>&);
template int64_t cheb2d_blocks<double>(const ChebPassArgs<double>&);
template void launch_cheb2d_batch<float>(const Cheb2DJob<float>*, const uint32_t*, int64_t, int, int, hipStream_t);
template void launch_cheb2d_batch<double>(const Cheb2DJob<double>*, const uint32_t*, int64_t, int, int, hipStream_t);
template void launch_cheb2d<float>(const ChebPassArgs<float>&, int, int, hipStream_t);
template void launch_cheb2d<double>(const ChebPassArgs<double>&, int, int, hipStream_t);

}  // namespace mxp
