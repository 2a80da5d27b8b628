// HIP kernels of the MatExPre library for gfx950 (MI355X).
//
// All kernels stream interleaved complex vectors (x fastest).  Workgroups are
// 256 work-items (four 64-wide wavefronts).  Reductions are two-pass and
// deterministic: wavefront butterfly (__shfl_xor over 64 lanes) -> LDS across
// the four wavefronts -> one partial per workgroup -> a second kernel sums the
// partials in a fixed order.
#include <hip/hip_runtime.h>

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

__global__ __launch_bounds__(256) void k_mdot_partial(const cpx<double>* __restrict__ V, int64_t ld,
                                                      const cpx<double>* __restrict__ w, int64_t n,
                                                      cpx<double>* __restrict__ partial) {
    const int vi = blockIdx.y;
    const cpx<double>* __restrict__ Vi = V + int64_t(vi) * ld;
    cpx<double> acc{0.0, 0.0};
    const int64_t stride = int64_t(gridDim.x) * kRedThreads;
    for (int64_t p = int64_t(blockIdx.x) * kRedThreads + threadIdx.x; p < n; p += stride) {
        const cpx<double> a = Vi[p], b = w[p];
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

template <bool kSub>
__global__ __launch_bounds__(256) void k_mupdate(cpx<double>* __restrict__ w,
                                                 const cpx<double>* __restrict__ V, int64_t ld, int nv,
                                                 const cpx<double>* __restrict__ h, int64_t n) {
    __shared__ cpx<double> hs[kMaxVec];
    for (int q = threadIdx.x; q < nv; q += blockDim.x) hs[q] = h[q];
    __syncthreads();
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n; p += stride) {
        cpx<double> acc{0.0, 0.0};
        for (int q = 0; q < nv; ++q) acc = cfma(hs[q], V[int64_t(q) * ld + p], acc);
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
    const dim3 grid(unsigned((a.n0 + kBX - 1) / kBX), unsigned((a.n1 + kBY - 1) / kBY),
                    unsigned(a.dim == 3 ? a.n2 : 1));
    if (a.dim == 3)
        hipLaunchKernelGGL((k_stencil<R, 3>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((k_stencil<R, 2>), grid, block, 0, s, a);
    check_launch("stencil");
}
template void launch_stencil<double>(const StencilArgs<double>&, hipStream_t);
template void launch_stencil<float>(const StencilArgs<float>&, hipStream_t);

int reduce_blocks(int64_t n) {
    const int64_t b = (n + 4 * kRedThreads - 1) / (4 * kRedThreads);
    return int(b < 1 ? 1 : (b > kMaxBlocks ? kMaxBlocks : b));
}

void launch_mdot(const cpx<double>* V, int64_t ld, int nv, const cpx<double>* w, int64_t n,
                 cpx<double>* partial, cpx<double>* out, hipStream_t s) {
    const int nb = reduce_blocks(n);
    hipLaunchKernelGGL(k_mdot_partial, dim3(nb, nv), dim3(kRedThreads), 0, s, V, ld, w, n, partial);
    hipLaunchKernelGGL(k_partial_sum, dim3(nv), dim3(kRedThreads), 0, s, partial, nb, out);
    check_launch("mdot");
}

void launch_mupdate(cpx<double>* w, const cpx<double>* V, int64_t ld, int nv, const cpx<double>* h,
                    int64_t n, hipStream_t s) {
    if (nv > kMaxVec) fail(MXP_ERR_INVALID_ARG, "too many basis vectors");
    hipLaunchKernelGGL(k_mupdate<true>, dim3(stream_blocks(n)), dim3(256), 0, s, w, V, ld, nv, h, n);
    check_launch("mupdate");
}

void launch_mcombine(cpx<double>* w, const cpx<double>* V, int64_t ld, int nv, const cpx<double>* y,
                     int64_t n, hipStream_t s) {
    if (nv > kMaxVec) fail(MXP_ERR_INVALID_ARG, "too many basis vectors");
    hipLaunchKernelGGL(k_mupdate<false>, dim3(stream_blocks(n)), dim3(256), 0, s, w, V, ld, nv, y, n);
    check_launch("mcombine");
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
