// HIP kernels of the MatExPre library for gfx950 (MI355X).
//
// All kernels stream interleaved complex vectors (x fastest).  Workgroups are
// 256 work-items (four 64-wide wavefronts).  Reductions are two-pass and
// deterministic: wavefront butterfly (__shfl_xor over 64 lanes) -> LDS across
// the four wavefronts -> one partial per workgroup -> a second kernel sums the
// partials in a fixed order.
#include <hip/hip_runtime.h>

#include <utility>

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
    const R Dp = (a.D ? a.D[p] : a.Dconst) - a.Dref;
    diag = cadd(diag, cscale(Dp, a.kD));
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

// 3D sweep marching along z.  A workgroup owns a 64 x 4 column tile and a
// chunk of zc planes.  Each work-item carries v at planes k-1 and k in
// registers and loads plane k+1, so v is fetched about once per chunk and
// the x/y neighbours come from the caches.  The x/y weights are
// loop-invariant: a ghost neighbour gets weight zero and a clamped offset (no
// branch around a load); the z boundary and the z tables are uniform.  OPS
// marks the operands present (1: x, 2: b2, 4: b3, 8: D), so absent ones cost
// no load.  Measured on 256^3: 64 x 4 tiles with chunks of 16 planes in plain
// workgroup order (taller tiles, 8-plane chunks and an XCD-contiguous
// renumbering were as fast or slower: the halo rows are served by L1 and the
// last-level cache, not a shared L2).
// (at most four wavefronts per SIMD: with the default target of eight the
// compiler serialises the complex-double loads to save registers)
template <typename R, int OPS>
__device__ __forceinline__ void sweep3d(const StencilArgs<R>& a, const Sweep3DGeom& m, int tile) {
    constexpr bool HX = OPS & 1, H2 = OPS & 2, H3 = OPS & 4, HD = OPS & 8;
    const int tx = tile % m.tiles_x;
    const int rest = tile / m.tiles_x;
    const int ty = rest % m.tiles_y;
    const int tz = rest / m.tiles_y;
    const int64_t i = int64_t(tx) * kBX + threadIdx.x;
    const int64_t j = int64_t(ty) * kBY + threadIdx.y;
    if (i >= a.n0 || j >= a.n1) return;
    const int64_t z0 = int64_t(tz) * m.zc;
    const int64_t z1 = z0 + m.zc < a.n2 ? z0 + m.zc : a.n2;
    const int64_t sy = a.n0;
    const int64_t sz = a.n0 * a.n1;
    const cpx<R>* __restrict__ v = a.b1;
    const cpx<R> zero{R(0), R(0)};
    const int64_t oxm = i > 0 ? -1 : 0, oxp = i < a.n0 - 1 ? 1 : 0;
    const int64_t oym = j > 0 ? -sy : 0, oyp = j < a.n1 - 1 ? sy : 0;
    const cpx<R> wxm = keep_if(i > 0, gload(a.alpha[0], i));
    const cpx<R> wxp = keep_if(i < a.n0 - 1, gload(a.beta[0], i));
    const cpx<R> wym = keep_if(j > 0, gload(a.alpha[1], j));
    const cpx<R> wyp = keep_if(j < a.n1 - 1, gload(a.beta[1], j));
    const cpx<R> gxy = cadd(gload(a.gamma[0], i), gload(a.gamma[1], j));
    int64_t p = i + sy * j + sz * z0;
    cpx<R> vm = gload(v, z0 > 0 ? p - sz : p);
    if (z0 == 0) vm = zero;
    cpx<R> vc = gload(v, p);
    for (int64_t k = z0; k < z1; ++k, p += sz) {
        const bool up = k + 1 < a.n2;
        cpx<R> vp = gload(v, up ? p + sz : p);
        const cpx<R> vxm = gload(v, p + oxm), vxp = gload(v, p + oxp);
        const cpx<R> vym = gload(v, p + oym), vyp = gload(v, p + oyp);
        R Draw = a.Dconst;
        if constexpr (HD) Draw = gload(a.D, p);
        cpx<R> xv = zero, b2v = zero, b3v = zero;
        if constexpr (HX) xv = gload(a.x, p);
        if constexpr (H2) b2v = gload(a.b2, p);
        if constexpr (H3) b3v = gload(a.b3, p);
        vp = keep_if(up, vp);
        cpx<R> diag = cadd(gxy, sload(a.gamma[2], k));
        diag = cadd(diag, cscale(Draw - a.Dref, a.kD));
        cpx<R> s = cmul(diag, vc);
        s = cfma(wxm, vxm, s);
        s = cfma(wxp, vxp, s);
        s = cfma(wym, vym, s);
        s = cfma(wyp, vyp, s);
        s = cfma(sload(a.alpha[2], k), vm, s);
        s = cfma(sload(a.beta[2], k), vp, s);
        cpx<R> o = cmul(a.g, s);
        if constexpr (HX) o = cfma(a.cx, xv, o);
        if constexpr (H2) o = cfma(a.e2, b2v, o);
        if constexpr (H3) o = cfma(a.e3, b3v, o);
        gstore(a.out, p, o);
        vm = vc;
        vc = vp;
    }
}

template <typename R, int OPS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_stencil3d(StencilArgs<R> a,
                                                                                             Sweep3DGeom m) {
    sweep3d<R, OPS>(a, m, blockIdx.x);
}

// Batched form: the job of a workgroup comes from a lookup table with one
// entry per 64 workgroups, and its description is read through the scalar
// cache (uniform across the workgroup).
template <typename R, int OPS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_stencil3d_batch(
    const Sweep3DJob<R>* jobs, const uint32_t* lut) {
    const int b = blockIdx.x;
    const __attribute__((address_space(4))) uint32_t* lq = (const __attribute__((address_space(4))) uint32_t*)(lut);
    const int q = lq[b >> 6];
    const Sweep3DJob<R> job = sload_words(jobs + q);
    const int64_t local = int64_t(b) - job.block0;
    if (local >= job.blocks) return;
    sweep3d<R, OPS>(job.a, job.geom, int(local));
}

template <typename R, int OPS>
void launch_3d_ops(const StencilArgs<R>& a, const Sweep3DGeom& m, unsigned nb, hipStream_t s) {
    hipLaunchKernelGGL((k_stencil3d<R, OPS>), dim3(nb), dim3(kBX, kBY, 1), 0, s, a, m);
}

template <typename R, int... OPS>
void launch_3d(const StencilArgs<R>& a, const Sweep3DGeom& m, unsigned nb, int ops, hipStream_t s,
               std::integer_sequence<int, OPS...>) {
    ((ops == OPS ? launch_3d_ops<R, OPS>(a, m, nb, s) : void()), ...);
}

template <typename R, int OPS>
void launch_3d_batch_ops(const Sweep3DJob<R>* jobs, const uint32_t* lut, unsigned nb, hipStream_t s) {
    hipLaunchKernelGGL((k_stencil3d_batch<R, OPS>), dim3(nb), dim3(kBX, kBY, 1), 0, s, jobs, lut);
}

template <typename R, int... OPS>
void launch_3d_batch(const Sweep3DJob<R>* jobs, const uint32_t* lut, unsigned nb, int ops, hipStream_t s,
                     std::integer_sequence<int, OPS...>) {
    ((ops == OPS ? launch_3d_batch_ops<R, OPS>(jobs, lut, nb, s) : void()), ...);
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

// TV: the basis' element type (complex double, or complex float for the
// inner GMRES of the mixed form); w and all arithmetic are complex double.
template <typename TV>
__global__ __launch_bounds__(256) void k_mdot_partial(const TV* __restrict__ V, int64_t ld,
                                                      const cpx<double>* __restrict__ w, int64_t n,
                                                      cpx<double>* __restrict__ partial) {
    const int vi = blockIdx.y;
    const TV* __restrict__ Vi = V + int64_t(vi) * ld;
    cpx<double> acc{0.0, 0.0};
    const int64_t stride = int64_t(gridDim.x) * kRedThreads;
    for (int64_t p = int64_t(blockIdx.x) * kRedThreads + threadIdx.x; p < n; p += stride) {
        const cpx<double> a = widen(Vi[p]), b = w[p];
        // conj(a) * b
        acc.re = fma(a.re, b.re, fma(a.im, b.im, acc.re));
        acc.im = fma(a.re, b.im, fma(-a.im, b.re, acc.im));
    }
    const cpx<double> s = block_sum(acc);
    if (threadIdx.x == 0) partial[int64_t(vi) * gridDim.x + blockIdx.x] = s;
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
        const int64_t nb = int64_t(m.tiles_x) * m.tiles_y * m.zchunks;
        if (nb > 0x7fffffff) fail(MXP_ERR_UNSUPPORTED, "grid too large for the 3D sweep");
        launch_3d<R>(a, m, unsigned(nb), sweep_ops(a), s, std::make_integer_sequence<int, 16>{});
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
    m.tiles_x = int((a.n0 + kBX - 1) / kBX);
    m.tiles_y = int((a.n1 + kBY - 1) / kBY);
    m.zc = 16;
    m.zchunks = int((a.n2 + m.zc - 1) / m.zc);
    return m;
}
template Sweep3DGeom sweep3d_geometry<double>(const StencilArgs<double>&);
template Sweep3DGeom sweep3d_geometry<float>(const StencilArgs<float>&);

template <typename R>
void launch_stencil3d_batch(const Sweep3DJob<R>* jobs, const uint32_t* lut, int64_t total_blocks, int ops,
                            hipStream_t s) {
    if (total_blocks <= 0) return;
    if (total_blocks > 0x7fffffff) fail(MXP_ERR_UNSUPPORTED, "batched 3D sweep too large");
    launch_3d_batch<R>(jobs, lut, unsigned(total_blocks), ops, s, std::make_integer_sequence<int, 16>{});
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
    hipLaunchKernelGGL(k_mdot_partial<TV>, dim3(nb, nv), dim3(kRedThreads), 0, s, V, ld, w, n, partial);
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
