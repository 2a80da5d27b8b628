// HIP kernels of the MatExPre library for gfx950 (MI355X).
//
// All kernels stream interleaved complex vectors (x fastest).  Workgroups are
// 256 work-items (four 64-wide wavefronts).  Reductions are two-pass and
// deterministic: wavefront butterfly (__shfl_xor over 64 lanes) -> LDS across
// the four wavefronts -> one partial per workgroup -> a second kernel sums the
// partials in a fixed order.
#include <hip/hip_runtime.h>

#include <utility>

#include "devmem.h"
#include "kernels.h"
#include "mxp_internal.h"

namespace mxp {

namespace {

template <typename R>
__device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cpx<R> cadd(cpx<R> a, cpx<R> b) {
    return {a.re + b.re, a.im + b.im};
}
// a*b + c
template <typename R>
__device__ __forceinline__ cpx<R> cfma(cpx<R> a, cpx<R> b, cpx<R> c) {
    return {fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im))};
}
template <typename R>
__device__ __forceinline__ cpx<R> cscale(R s, cpx<R> a) {
    return {s * a.re, s * a.im};
}

constexpr int kBX = 64;
constexpr int kBY = 4;
constexpr int kSweepW = 256;  // columns of a 3D sweep tile (four wavefronts)


// 2D sweep: one work-item per node, 64 x 4 workgroups.
template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_stencil(StencilArgs<R> a) {
    const int64_t i = int64_t(blockIdx.x) * kBX + threadIdx.x;
    const int64_t j = int64_t(blockIdx.y) * kBY + threadIdx.y;
    const int64_t k = blockIdx.z;
    if (i >= a.n0 || j >= a.n1) return;
    const int64_t sy = a.n0;
    const int64_t sz = a.n0 * a.n1;
    const int64_t p = i + sy * j + sz * k;
    const cpx<R>* __restrict__ v = a.b1;
    const cpx<R> c = v[p];
    cpx<R> diag = cadd(a.gamma[0][i], a.gamma[1][j]);
    if (DIM == 3) diag = cadd(diag, a.gamma[2][k]);
    const R Draw = a.D ? a.D[p] : a.Dconst;
    diag = cadd(diag, cscale(Draw - a.Dref, a.kD));
    if (a.abc[0]) {  // absorbing faces: 2 i omega sqrt(D_p)/h per face the node lies on
        R w = a.abc[0][i] + a.abc[1][j];
        if (DIM == 3) w += a.abc[2][k];
        if (w != R(0)) diag.im += w * sqrt(Draw);
    }
    cpx<R> s = cmul(diag, c);
    if (i > 0) s = cfma(a.alpha[0][i], v[p - 1], s);
    if (i < a.n0 - 1) s = cfma(a.beta[0][i], v[p + 1], s);
    if (j > 0) s = cfma(a.alpha[1][j], v[p - sy], s);
    if (j < a.n1 - 1) s = cfma(a.beta[1][j], v[p + sy], s);
    if (DIM == 3) {
        if (k > 0) s = cfma(a.alpha[2][k], v[p - sz], s);
        if (k < a.n2 - 1) s = cfma(a.beta[2][k], v[p + sz], s);
    }
    cpx<R> o = cmul(a.g, s);
    if (a.x) o = cfma(a.cx, a.x[p], o);
    if (a.b2) o = cfma(a.e2, a.b2[p], o);
    if (a.b3) o = cfma(a.e3, a.b3[p], o);
    a.out[p] = o;
}

template <typename R>
__device__ __forceinline__ cpx<R> keep_if(bool c, cpx<R> v) {
    return {c ? v.re : R(0), c ? v.im : R(0)};
}

// Uniform table entry through the scalar cache (constant address space): the
// z tables are indexed by the plane, the same for every work-item.
template <typename R>
__device__ __forceinline__ cpx<R> sload(const cpx<R>* p, int64_t idx) {
    const __attribute__((address_space(4))) R* q = (const __attribute__((address_space(4))) R*)(p);
    return {q[2 * idx], q[2 * idx + 1]};
}
template <typename R>
__device__ __forceinline__ R sload_r(const R* p, int64_t idx) {
    return ((const __attribute__((address_space(4))) R*)(p))[idx];
}

// Loads and stores through the global address space.  Pointers read from
// memory (the batched job table) are generic to the compiler, which would
// otherwise emit flat accesses that also count against the LDS counter.
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
template <typename R>
__device__ __forceinline__ cpx<R> csel(bool c, cpx<R> a, cpx<R> b) {
    return {c ? a.re : b.re, c ? a.im : b.im};
}

// Tile of workgroup `b` among `tiles` tiles padded to `padded` (a multiple of
// eight): consecutive workgroups go round-robin to the eight XCDs, each with
// its own L2, so XCD q is given the q-th contiguous eighth of the tiles.  Tiles
// are numbered y fastest, so the rows one tile reads beyond its own edges were
// loaded by a tile on the same XCD.  Returns -1 for padding.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t tiles, int64_t padded) {
    const int64_t t = (b & 7) * (padded >> 3) + (b >> 3);
    return t < tiles ? t : -1;
}

// 3D sweep marching along z.  A workgroup's four wavefronts lie side by side
// along x: work-item c owns column c of a tile of kSweepW columns and TY rows
// and keeps those TY values of v for planes k-1 .. k+2 in registers.  So per
// plane v is loaded once for the tile's rows plus one halo row on either
// side; y-neighbours inside the tile come from the work-item's own registers
// and x-neighbours from the adjacent lanes by DPP wavefront shifts (lanes 0
// and 63 load theirs: it lies in the neighbouring wavefront, or tile).  The
// loop is software-pipelined: the step for plane k first issues the loads of
// plane k+2 of v and of plane k+1's other operands, then computes plane k
// from registers loaded one step earlier, so a wavefront's loads are in
// flight while it computes.  It is unrolled by four so that the four plane
// slots and the two operand sets rotate by renaming.  The x weights are
// loop-invariant per lane, the y and z tables are uniform (scalar cache);
// ghost neighbours get weight zero and planes outside the grid clamped
// addresses (no branch around a load).  OPS marks the operands present (1: x,
// 2: b2, 4: b3, 8: D), so absent ones cost no load.
template <typename R, int OPS, int TY>
struct PipeOps {
    cpx<R> xe[TY], xv[TY], b2v[TY], b3v[TY];
    R Dv[TY];
    cpx<R> hm, hp;
};

template <typename R, int OPS, int TY>
__device__ __forceinline__ void sweep3d(const StencilArgs<R>& a, const Sweep3DGeom& m, int64_t tile) {
    constexpr bool HX = OPS & 1, H2 = OPS & 2, H3 = OPS & 4, HD = OPS & 8;
    const int64_t ty = tile % m.tiles_y;
    const int64_t rest = tile / m.tiles_y;
    const int64_t tz = rest % m.zchunks;
    const int64_t tx = rest / m.zchunks;
    const int lane = threadIdx.x & 63;
    const int64_t i = tx * kSweepW + threadIdx.x;
    const bool col_ok = i < a.n0;
    const int64_t ic = col_ok ? i : a.n0 - 1;  // clamped column for loads
    const int64_t j0 = ty * TY;
    const int64_t z0 = tz * m.zc;
    const int64_t z1 = z0 + m.zc < a.n2 ? z0 + m.zc : a.n2;
    const int64_t sy = a.n0;
    const int64_t sz = a.n0 * a.n1;
    const cpx<R>* __restrict__ v = a.b1;
    // x weights (zero for ghosts and for columns beyond the grid)
    const cpx<R> wxm = keep_if(col_ok && i > 0, gload(a.alpha[0], ic));
    const cpx<R> wxp = keep_if(col_ok && i < a.n0 - 1, gload(a.beta[0], ic));
    const cpx<R> gx = gload(a.gamma[0], ic);
    const bool abc_on = a.abc[0] != nullptr;
    const R abx = abc_on ? gload(a.abc[0], ic) : R(0);
    const int64_t eoff = (lane == 0 && ic > 0) ? -1 : ((lane == 63 && ic < a.n0 - 1) ? 1 : 0);
    int64_t roff[TY];
#pragma unroll
    for (int r = 0; r < TY; ++r) roff[r] = sy * (j0 + r < a.n1 ? j0 + r : a.n1 - 1);
    const int64_t hlo = sy * (j0 > 0 ? j0 - 1 : 0);
    const int64_t hhi = sy * (j0 + TY < a.n1 ? j0 + TY : a.n1 - 1);
    const bool has_lo = j0 > 0, has_hi = j0 + TY < a.n1;
    // plane k clamped into the grid
    auto zcl = [&](int64_t k) { return k < 0 ? int64_t(0) : (k >= a.n2 ? a.n2 - 1 : k); };
    auto load_v = [&](int64_t k, cpx<R>(&dst)[TY]) {
        const int64_t pk = ic + sz * zcl(k);
#pragma unroll
        for (int r = 0; r < TY; ++r) dst[r] = gload(v, pk + roff[r]);
    };
    auto load_ops = [&](int64_t k, PipeOps<R, OPS, TY>& o) {
        const int64_t pk = ic + sz * zcl(k);
        o.hm = gload(v, pk + hlo);
#pragma unroll
        for (int r = 0; r < TY; ++r) {
            o.xe[r] = gload(v, pk + roff[r] + eoff);
            if constexpr (HX) o.xv[r] = gload(a.x, pk + roff[r]);
            if constexpr (H2) o.b2v[r] = gload(a.b2, pk + roff[r]);
            if constexpr (H3) o.b3v[r] = gload(a.b3, pk + roff[r]);
            if constexpr (HD) o.Dv[r] = gload(a.D, pk + roff[r]);
        }
        o.hp = gload(v, pk + hhi);
    };
    auto compute = [&](int64_t k, const cpx<R>(&prev)[TY], const cpx<R>(&cur)[TY], const cpx<R>(&next)[TY],
                       const PipeOps<R, OPS, TY>& o) {
        const int64_t pk = ic + sz * k;
        const bool dn = k > 0, up = k + 1 < a.n2;
        const cpx<R> hm = keep_if(has_lo, o.hm), hp = keep_if(has_hi, o.hp);
        const cpx<R> az = sload(a.alpha[2], k), bz = sload(a.beta[2], k);
        const cpx<R> gxz = cadd(gx, sload(a.gamma[2], k));
        const R abxz = abc_on ? abx + sload_r(a.abc[2], k) : R(0);
#pragma unroll
        for (int r = 0; r < TY; ++r) {
            const int64_t j = j0 + r;
            if (j >= a.n1) break;  // uniform: rows beyond the grid
            cpx<R> xm = from_below(cur[r]), xp = from_above(cur[r]);
            xm = csel(lane == 0, o.xe[r], xm);
            xp = csel(lane == 63, o.xe[r], xp);
            const cpx<R> ym = r > 0 ? cur[r - 1] : hm;
            const cpx<R> yp = r < TY - 1 ? cur[r + 1] : hp;
            const cpx<R> wym = keep_if(j > 0, sload(a.alpha[1], j));
            const cpx<R> wyp = keep_if(j < a.n1 - 1, sload(a.beta[1], j));
            R Draw = a.Dconst;
            if constexpr (HD) Draw = o.Dv[r];
            cpx<R> diag = cadd(gxz, sload(a.gamma[1], j));
            diag = cadd(diag, cscale(Draw - a.Dref, a.kD));
            if (abc_on) {  // 2 i omega sqrt(D_p)/h per absorbing face of the node
                const R w = abxz + sload_r(a.abc[1], j);
                if (w != R(0)) diag.im += w * sqrt(Draw);
            }
            cpx<R> s = cmul(diag, cur[r]);
            s = cfma(wxm, xm, s);
            s = cfma(wxp, xp, s);
            s = cfma(wym, ym, s);
            s = cfma(wyp, yp, s);
            s = cfma(az, keep_if(dn, prev[r]), s);
            s = cfma(bz, keep_if(up, next[r]), s);
            cpx<R> o2 = cmul(a.g, s);
            if constexpr (HX) o2 = cfma(a.cx, o.xv[r], o2);
            if constexpr (H2) o2 = cfma(a.e2, o.b2v[r], o2);
            if constexpr (H3) o2 = cfma(a.e3, o.b3v[r], o2);
            if (col_ok) gstore(a.out, pk + roff[r], o2);
        }
    };
    cpx<R> V0[TY], V1[TY], V2[TY], V3[TY];
    PipeOps<R, OPS, TY> O0, O1;
    load_v(z0 - 1, V0);
    load_v(z0, V1);
    load_v(z0 + 1, V2);
    load_ops(z0, O0);
    // step for plane k: slots (k-1, k, k+1, k+2) and operands (k, k+1)
#define MXP_PIPE_STEP(A, B, C, Dn, OC, ON)        \
    {                                             \
        load_v(k + 2, Dn);                        \
        if (k + 1 < z1) load_ops(k + 1, ON);      \
        compute(k, A, B, C, OC);                  \
        if (++k >= z1) break;                     \
    }
    int64_t k = z0;
    while (true) {
        MXP_PIPE_STEP(V0, V1, V2, V3, O0, O1)
        MXP_PIPE_STEP(V1, V2, V3, V0, O1, O0)
        MXP_PIPE_STEP(V2, V3, V0, V1, O0, O1)
        MXP_PIPE_STEP(V3, V0, V1, V2, O1, O0)
    }
#undef MXP_PIPE_STEP
}

// rows per work-item: complex float 4, complex double 2 (the pipelined loop
// holds two planes of operands in registers)
template <typename R>
constexpr int sweep_rows() { return sizeof(R) == 4 ? 4 : 2; }

template <typename R, int OPS>
__global__ __launch_bounds__(256) void k_stencil3d(StencilArgs<R> a, Sweep3DGeom m) {
    const int64_t t = xcd_tile(blockIdx.x, m.tiles, m.blocks);
    if (t < 0) return;
    sweep3d<R, OPS, sweep_rows<R>()>(a, m, t);
}

// Batched form over grids of different sizes: a persistent grid of resident
// workgroups (a multiple of eight, so that index w keeps the XCD of w mod 8)
// strides over the concatenated workgroup ranges of the jobs.  The job of
// range index w comes from a lookup table with one entry per 64 indices, and
// its description is read through the scalar cache (uniform across the
// workgroup).  The wavefronts of a workgroup share no data.
template <typename R, int OPS>
__global__ __launch_bounds__(256) void k_stencil3d_batch(const Sweep3DJob<R>* jobs, const uint32_t* lut, int total) {
    const __attribute__((address_space(4))) uint32_t* lq = (const __attribute__((address_space(4))) uint32_t*)(lut);
    for (int w = blockIdx.x; w < total; w += gridDim.x) {
        const uint32_t q = lq[w >> 6];
        const Sweep3DJob<R> job = sload_words(jobs + q);
        const int local = w - int(job.block0);
        if (local >= int(job.geom.blocks)) continue;
        const int64_t t = xcd_tile(local, job.geom.tiles, job.geom.blocks);
        if (t < 0) continue;
        sweep3d<R, OPS, sweep_rows<R>()>(job.a, job.geom, t);
    }
}

template <typename R, int OPS>
void launch_3d_ops(const StencilArgs<R>& a, const Sweep3DGeom& m, unsigned nb, hipStream_t s) {
    hipLaunchKernelGGL((k_stencil3d<R, OPS>), dim3(nb), dim3(kSweepW, 1, 1), 0, s, a, m);
}

template <typename R, int... OPS>
void launch_3d(const StencilArgs<R>& a, const Sweep3DGeom& m, unsigned nb, int ops, hipStream_t s,
               std::integer_sequence<int, OPS...>) {
    ((ops == OPS ? launch_3d_ops<R, OPS>(a, m, nb, s) : void()), ...);
}

template <typename R, int OPS>
void launch_3d_batch_ops(const Sweep3DJob<R>* jobs, const uint32_t* lut, int64_t total, hipStream_t s) {
    // resident workgroups: occupancy (asked once per instantiation) times the
    // compute units, rounded down to a multiple of eight, at most the total
    static int per_cu = 0;
    if (per_cu == 0) {
        int n = 0;
        HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, reinterpret_cast<const void*>(k_stencil3d_batch<R, OPS>), kSweepW, 0));
        per_cu = n > 0 ? n : 1;
    }
    int dev = 0, cus = 0;
    HIP_CHECK(hipGetDevice(&dev));
    HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int64_t g = int64_t(per_cu) * (cus > 0 ? cus : 1);
    g = g >= 8 ? g / 8 * 8 : g;
    if (g > total) g = total;
    hipLaunchKernelGGL((k_stencil3d_batch<R, OPS>), dim3(unsigned(g)), dim3(kSweepW, 1, 1), 0, s, jobs, lut,
                       int(total));
}

template <typename R, int... OPS>
void launch_3d_batch(const Sweep3DJob<R>* jobs, const uint32_t* lut, int64_t total, int ops, hipStream_t s,
                     std::integer_sequence<int, OPS...>) {
    ((ops == OPS ? launch_3d_batch_ops<R, OPS>(jobs, lut, total, s) : void()), ...);
}

// ---------------------------------------------------------------- reductions

__device__ __forceinline__ cpx<double> wave_sum(cpx<double> v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        v.re += __shfl_xor(v.re, off, 64);
        v.im += __shfl_xor(v.im, off, 64);
    }
    return v;
}

// Sum over the 256 work-items of a workgroup; result valid in thread 0.
__device__ __forceinline__ cpx<double> block_sum(cpx<double> v) {
    __shared__ cpx<double> red[4];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    cpx<double> r{0.0, 0.0};
    if (threadIdx.x == 0) {
        r = red[0];
        for (int w = 1; w < 4; ++w) r = cadd(r, red[w]);
    }
    __syncthreads();
    return r;
}

constexpr int kRedThreads = 256;
constexpr int kMaxBlocks = 1024;

// A basis vector entry in double (a complex-float basis is widened exactly).
__device__ __forceinline__ cpx<double> widen(cpx<double> v) { return v; }
__device__ __forceinline__ cpx<double> widen(cpx<float> v) { return {double(v.re), double(v.im)}; }

// Partial sums of conj(V_q) . w for a group of up to kDotGroup basis
// vectors q = blockIdx.y * kDotGroup + i: each work-item loads w[p] once for
// the whole group and accumulates one sum per vector, so w is read once per
// group instead of once per vector.  Every sum is accumulated in the same
// order as a one-vector kernel would (grid-stride p, then the wavefront
// butterfly, then the four wavefronts in order), so the result does not
// depend on the grouping.  TV: the basis' element type (complex double, or
// complex float for the inner GMRES of the mixed form); w and all arithmetic
// are complex double.
constexpr int kDotGroup = 8;

template <typename TV>
__global__ __launch_bounds__(256) void k_mdot_partial(const TV* __restrict__ V, int64_t ld, int nv,
                                                      const cpx<double>* __restrict__ w, int64_t n,
                                                      cpx<double>* __restrict__ partial) {
    __shared__ cpx<double> red[4][kDotGroup];
    const int q0 = int(blockIdx.y) * kDotGroup;
    const int g = nv - q0 < kDotGroup ? nv - q0 : kDotGroup;  // uniform
    cpx<double> acc[kDotGroup];
#pragma unroll
    for (int i = 0; i < kDotGroup; ++i) acc[i] = {0.0, 0.0};
    const int64_t stride = int64_t(gridDim.x) * kRedThreads;
    for (int64_t p = int64_t(blockIdx.x) * kRedThreads + threadIdx.x; p < n; p += stride) {
        const cpx<double> b = w[p];
#pragma unroll
        for (int i = 0; i < kDotGroup; ++i) {
            if (i < g) {
                const cpx<double> a = widen(V[int64_t(q0 + i) * ld + p]);
                // conj(a) * b
                acc[i].re = fma(a.re, b.re, fma(a.im, b.im, acc[i].re));
                acc[i].im = fma(a.re, b.im, fma(-a.im, b.re, acc[i].im));
            }
        }
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < kDotGroup; ++i) {
        const cpx<double> v = wave_sum(acc[i]);
        if (lane == 0) red[wid][i] = v;
    }
    __syncthreads();
    if (threadIdx.x < g) {
        const int i = threadIdx.x;
        cpx<double> r = red[0][i];
        for (int k = 1; k < 4; ++k) r = cadd(r, red[k][i]);
        partial[int64_t(q0 + i) * gridDim.x + blockIdx.x] = r;
    }
}

__global__ __launch_bounds__(256) void k_nrm2_partial(const cpx<double>* __restrict__ w, int64_t n,
                                                      cpx<double>* __restrict__ partial) {
    cpx<double> acc{0.0, 0.0};
    const int64_t stride = int64_t(gridDim.x) * kRedThreads;
    for (int64_t p = int64_t(blockIdx.x) * kRedThreads + threadIdx.x; p < n; p += stride) {
        const cpx<double> b = w[p];
        acc.re = fma(b.re, b.re, fma(b.im, b.im, acc.re));
    }
    const cpx<double> s = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// out[i] = sum_b partial[i*nb + b] in a fixed order.
__global__ __launch_bounds__(256) void k_partial_sum(const cpx<double>* __restrict__ partial, int nb,
                                                     cpx<double>* __restrict__ out) {
    const int vi = blockIdx.x;
    cpx<double> acc{0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += kRedThreads) acc = cadd(acc, partial[int64_t(vi) * nb + b]);
    const cpx<double> s = block_sum(acc);
    if (threadIdx.x == 0) out[vi] = s;
}

constexpr int kMaxVec = 256;

template <typename TV, bool kSub>
__global__ __launch_bounds__(256) void k_mupdate(cpx<double>* __restrict__ w,
                                                 const TV* __restrict__ V, int64_t ld, int nv,
                                                 const cpx<double>* __restrict__ h, int64_t n) {
    __shared__ cpx<double> hs[kMaxVec];
    for (int q = threadIdx.x; q < nv; q += blockDim.x) hs[q] = h[q];
    __syncthreads();
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n; p += stride) {
        cpx<double> acc{0.0, 0.0};
        for (int q = 0; q < nv; ++q) acc = cfma(hs[q], widen(V[int64_t(q) * ld + p]), acc);
        cpx<double> o = w[p];
        if (kSub) {
            o.re -= acc.re;
            o.im -= acc.im;
        } else {
            o.re += acc.re;
            o.im += acc.im;
        }
        w[p] = o;
    }
}

__global__ __launch_bounds__(256) void k_axpby(cpx<double> a, const cpx<double>* __restrict__ x,
                                               cpx<double> b, cpx<double>* __restrict__ y, int64_t n) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n; p += stride)
        y[p] = cfma(a, x[p], cmul(b, y[p]));
}

__global__ __launch_bounds__(256) void k_scale(cpx<double> a, const cpx<double>* __restrict__ x,
                                               cpx<double>* __restrict__ y, int64_t n) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n; p += stride)
        y[p] = cmul(a, x[p]);
}

__global__ __launch_bounds__(256) void k_scale_to_c64(cpx<double> a, const cpx<double>* __restrict__ x,
                                                      cpx<float>* __restrict__ y, int64_t n) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n; p += stride) {
        const cpx<double> v = cmul(a, x[p]);
        y[p] = {float(v.re), float(v.im)};
    }
}

__global__ __launch_bounds__(256) void k_to_c64(const cpx<double>* __restrict__ x,
                                                cpx<float>* __restrict__ y, int64_t n) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n; p += stride)
        y[p] = {float(x[p].re), float(x[p].im)};
}

__global__ __launch_bounds__(256) void k_to_c128(const cpx<float>* __restrict__ x,
                                                 cpx<double>* __restrict__ y, int64_t n) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n; p += stride)
        y[p] = {double(x[p].re), double(x[p].im)};
}

__global__ __launch_bounds__(256) void k_inv_c2(const void* __restrict__ c, int is_f32,
                                                double* __restrict__ D64, float* __restrict__ D32,
                                                int64_t n) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n; p += stride) {
        const double v = is_f32 ? double(static_cast<const float*>(c)[p]) : static_cast<const double*>(c)[p];
        const double d = 1.0 / (v * v);
        D64[p] = d;
        D32[p] = float(d);
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_zero(cpx<R>* __restrict__ y, int64_t n) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n; p += stride) y[p] = {R(0), R(0)};
}

inline unsigned stream_blocks(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return unsigned(b < 8192 ? (b < 1 ? 1 : b) : 8192);
}

inline void check_launch(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(MXP_ERR_HIP, std::string("kernel launch failed (") + what + "): " + hipGetErrorString(e));
}

}  // namespace

template <typename R>
void launch_stencil(const StencilArgs<R>& a, hipStream_t s) {
    const dim3 block(kBX, kBY, 1);
    if (a.dim == 3) {
        const Sweep3DGeom m = sweep3d_geometry(a);
        if (m.blocks > 0x7fffffff) fail(MXP_ERR_UNSUPPORTED, "grid too large for the 3D sweep");
        launch_3d<R>(a, m, unsigned(m.blocks), sweep_ops(a), s, std::make_integer_sequence<int, 16>{});
    } else {
        const dim3 grid(unsigned((a.n0 + kBX - 1) / kBX), unsigned((a.n1 + kBY - 1) / kBY), 1);
        hipLaunchKernelGGL((k_stencil<R, 2>), grid, block, 0, s, a);
    }
    check_launch("stencil");
}
template void launch_stencil<double>(const StencilArgs<double>&, hipStream_t);

template <typename R>
Sweep3DGeom sweep3d_geometry(const StencilArgs<R>& a) {
    Sweep3DGeom m;
    constexpr int TY = sweep_rows<R>();
    m.rows = TY;
    m.tiles_x = int((a.n0 + kSweepW - 1) / kSweepW);
    m.tiles_y = int((a.n1 + TY - 1) / TY);
    // z segments: the caller's length, else about four workgroups per compute
    // unit of a 256-CU device, in 8..32 planes
    int zc = a.zc;
    if (zc <= 0) {
        const int64_t cols = int64_t(m.tiles_x) * m.tiles_y;
        const int64_t want = (4 * 256 + cols - 1) / cols;  // segments wanted
        zc = int((a.n2 + want - 1) / want);
        zc = zc < 8 ? 8 : (zc > 32 ? 32 : zc);
    }
    m.zc = zc;
    m.zchunks = int((a.n2 + m.zc - 1) / m.zc);
    m.tiles = int64_t(m.tiles_x) * m.tiles_y * m.zchunks;
    m.blocks = (m.tiles + 7) / 8 * 8;
    return m;
}
template Sweep3DGeom sweep3d_geometry<double>(const StencilArgs<double>&);
template Sweep3DGeom sweep3d_geometry<float>(const StencilArgs<float>&);

template <typename R>
void launch_stencil3d_batch(const Sweep3DJob<R>* jobs, const uint32_t* lut, int64_t total_blocks, int ops,
                            hipStream_t s) {
    if (total_blocks <= 0) return;
    if (total_blocks > 0x7fffffff) fail(MXP_ERR_UNSUPPORTED, "batched 3D sweep too large");
    launch_3d_batch<R>(jobs, lut, total_blocks, ops, s, std::make_integer_sequence<int, 16>{});
    check_launch("batched 3D sweep");
}
template void launch_stencil3d_batch<double>(const Sweep3DJob<double>*, const uint32_t*, int64_t, int, hipStream_t);
template void launch_stencil3d_batch<float>(const Sweep3DJob<float>*, const uint32_t*, int64_t, int, hipStream_t);
template void launch_stencil<float>(const StencilArgs<float>&, hipStream_t);

int reduce_blocks(int64_t n) {
    const int64_t b = (n + 4 * kRedThreads - 1) / (4 * kRedThreads);
    return int(b < 1 ? 1 : (b > kMaxBlocks ? kMaxBlocks : b));
}

template <typename TV>
void launch_mdot(const TV* V, int64_t ld, int nv, const cpx<double>* w, int64_t n,
                 cpx<double>* partial, cpx<double>* out, hipStream_t s) {
    const int nb = reduce_blocks(n);
    const int groups = (nv + kDotGroup - 1) / kDotGroup;
    hipLaunchKernelGGL(k_mdot_partial<TV>, dim3(nb, groups), dim3(kRedThreads), 0, s, V, ld, nv, w, n, partial);
    hipLaunchKernelGGL(k_partial_sum, dim3(nv), dim3(kRedThreads), 0, s, partial, nb, out);
    check_launch("mdot");
}
template void launch_mdot<cpx<double>>(const cpx<double>*, int64_t, int, const cpx<double>*, int64_t,
                                       cpx<double>*, cpx<double>*, hipStream_t);
template void launch_mdot<cpx<float>>(const cpx<float>*, int64_t, int, const cpx<double>*, int64_t,
                                      cpx<double>*, cpx<double>*, hipStream_t);

template <typename TV>
void launch_mupdate(cpx<double>* w, const TV* V, int64_t ld, int nv, const cpx<double>* h,
                    int64_t n, hipStream_t s) {
    if (nv > kMaxVec) fail(MXP_ERR_INVALID_ARG, "too many basis vectors");
    hipLaunchKernelGGL((k_mupdate<TV, true>), dim3(stream_blocks(n)), dim3(256), 0, s, w, V, ld, nv, h, n);
    check_launch("mupdate");
}
template void launch_mupdate<cpx<double>>(cpx<double>*, const cpx<double>*, int64_t, int, const cpx<double>*,
                                          int64_t, hipStream_t);
template void launch_mupdate<cpx<float>>(cpx<double>*, const cpx<float>*, int64_t, int, const cpx<double>*,
                                         int64_t, hipStream_t);

template <typename TV>
void launch_mcombine(cpx<double>* w, const TV* V, int64_t ld, int nv, const cpx<double>* y,
                     int64_t n, hipStream_t s) {
    if (nv > kMaxVec) fail(MXP_ERR_INVALID_ARG, "too many basis vectors");
    hipLaunchKernelGGL((k_mupdate<TV, false>), dim3(stream_blocks(n)), dim3(256), 0, s, w, V, ld, nv, y, n);
    check_launch("mcombine");
}
template void launch_mcombine<cpx<double>>(cpx<double>*, const cpx<double>*, int64_t, int, const cpx<double>*,
                                           int64_t, hipStream_t);
template void launch_mcombine<cpx<float>>(cpx<double>*, const cpx<float>*, int64_t, int, const cpx<double>*,
                                          int64_t, hipStream_t);

void launch_scale_to_c64(cpx<double> a, const cpx<double>* x, cpx<float>* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_to_c64, dim3(stream_blocks(n)), dim3(256), 0, s, a, x, y, n);
    check_launch("scale_to_c64");
}

void launch_nrm2sq(const cpx<double>* w, int64_t n, cpx<double>* partial, cpx<double>* out,
                   hipStream_t s) {
    const int nb = reduce_blocks(n);
    hipLaunchKernelGGL(k_nrm2_partial, dim3(nb), dim3(kRedThreads), 0, s, w, n, partial);
    hipLaunchKernelGGL(k_partial_sum, dim3(1), dim3(kRedThreads), 0, s, partial, nb, out);
    check_launch("nrm2");
}

void launch_axpby(cpx<double> a, const cpx<double>* x, cpx<double> b, cpx<double>* y, int64_t n,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_axpby, dim3(stream_blocks(n)), dim3(256), 0, s, a, x, b, y, n);
    check_launch("axpby");
}

void launch_scale(cpx<double> a, const cpx<double>* x, cpx<double>* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_scale, dim3(stream_blocks(n)), dim3(256), 0, s, a, x, y, n);
    check_launch("scale");
}

void launch_to_c64(const cpx<double>* x, cpx<float>* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_to_c64, dim3(stream_blocks(n)), dim3(256), 0, s, x, y, n);
    check_launch("to_c64");
}

void launch_to_c128(const cpx<float>* x, cpx<double>* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_to_c128, dim3(stream_blocks(n)), dim3(256), 0, s, x, y, n);
    check_launch("to_c128");
}

void launch_inv_c2(const void* c, int is_f32, double* D64, float* D32, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_inv_c2, dim3(stream_blocks(n)), dim3(256), 0, s, c, is_f32, D64, D32, n);
    check_launch("inv_c2");
}

template <typename R>
void launch_zero(cpx<R>* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero<R>, dim3(stream_blocks(n)), dim3(256), 0, s, y, n);
    check_launch("zero");
}
template void launch_zero<double>(cpx<double>*, int64_t, hipStream_t);
template void launch_zero<float>(cpx<float>*, int64_t, hipStream_t);

}  // namespace mxp
