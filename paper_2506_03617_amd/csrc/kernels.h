// Device-kernel launch interface of the MatExPre library (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mxp {

template <typename R>
struct alignas(2 * sizeof(R)) cpx {
    R re, im;
};

// One fused sweep of the shifted stencil operator with affine extras:
//
//   out[p] = g * ( sum_d [alpha_d v[p-e_d] + beta_d v[p+e_d] + gamma_d v[p]]
//                  + kD * (D[p] - Dref) * v[p] )
//            + cx * x[p] + e2 * b2[p] + e3 * b3[p]
//
// with v = b1 (the stencil input), per-axis three-point tables alpha/beta of
// the stretched second difference (zero Dirichlet ghosts), D = 1/c^2 per node
// (or the constant Dconst when D == nullptr).  The diagonal tables gamma_d
// carry -(alpha_d + beta_d) plus an equal share of every constant diagonal
// term (kD * Dref - centre), summed in double on the host: summing the large
// axis terms and the shift in the working precision would cancel badly.  Any of
// x, b2, b3 may be nullptr (term omitted).  out may alias x, b2 or b3 (each
// point is read before it is written by the same thread) but not b1.
//
// Used for:  y = A_s x                         (g = 1, kD = omega^2(1+is))
//            r = -A u - f                      (g = -1, e2 = -1, b2 = f)
//            Clenshaw step b_k = c_k x + 2 Ahat b_{k+1} - b_{k+2},
//            Ahat = (A_s - centre)/half_width  (g = 2/half_width, centre in gamma)
template <typename R>
struct StencilArgs {
    int dim;
    int64_t n0, n1, n2;
    const cpx<R>* alpha[3];
    const cpx<R>* beta[3];
    const cpx<R>* gamma[3];
    const R* D;
    R Dconst, Dref;
    cpx<R> g, kD, cx, e2, e3;
    const cpx<R>* x;
    const cpx<R>* b1;
    const cpx<R>* b2;
    const cpx<R>* b3;
    cpx<R>* out;
    int zc;  // 3D sweeps: z segment length (0 = chosen from the grid)
    // first-order absorbing faces with a varying speed: per-axis weights
    // 2 omega/h at the absorbing end nodes (0 elsewhere); the diagonal gains
    // i (abc_x + abc_y + abc_z) sqrt(D_p).  nullptr when absent.
    const R* abc[3];
};

template <typename R>
void launch_stencil(const StencilArgs<R>& a, hipStream_t s);

// Geometry of the 3D sweep: tiles of 256 columns x `rows` rows, segments of
// zc planes; `tiles` tiles launched as `blocks` workgroups (padded to a
// multiple of eight for the XCD-aware tile order).
struct Sweep3DGeom {
    int tiles_x, tiles_y, zchunks, zc, rows;
    int64_t tiles, blocks;
};
template <typename R>
Sweep3DGeom sweep3d_geometry(const StencilArgs<R>& a);
// Operands present in a sweep: 1 x, 2 b2, 4 b3, 8 D.
template <typename R>
int sweep_ops(const StencilArgs<R>& a) {
    return (a.x ? 1 : 0) | (a.b2 ? 2 : 0) | (a.b3 ? 4 : 0) | (a.D ? 8 : 0);
}

// One 3D sweep inside a batched launch over grids of different sizes.  Job q
// owns workgroups [block0, block0 + blocks); block0 is a multiple of 64 and
// lut[b / 64] (uint32) names the job of workgroup b.
template <typename R>
struct Sweep3DJob {
    StencilArgs<R> a;
    Sweep3DGeom geom;
    int64_t block0, blocks;
};
// jobs, lut: device arrays; every job has operand set `ops`; total_blocks
// covers the last job's padded range.
template <typename R>
void launch_stencil3d_batch(const Sweep3DJob<R>* jobs, const uint32_t* lut, int64_t total_blocks, int ops,
                            hipStream_t s);

// One temporally blocked Clenshaw pass on a 2D grid (vectors below 4 GiB):
// K consecutive levels
//   L_l = cx_l x + g_l S(L_{l-1}) - L_{l-2}
// with S the h^2-scaled stencil (tables ax/bx/gx, ay/by/gy multiplied by h^2,
// kD likewise, so interior nodes have unit neighbour weights), inputs
// in0 = L_{-2}, in1 = L_{-1} (nullptr = zero).  A non-final pass writes its
// second-to-last level to outA and its last to outB; a final pass writes
// post * L_last + e3 * add to outB only.  Outputs must not alias any input:
// neighbouring strips and segments read input halos concurrently.
constexpr int kMaxFused = 8;
template <typename R>
struct ChebPassArgs {
    int64_t n0, n1;
    const cpx<R>* ax;
    const cpx<R>* bx;
    const cpx<R>* gx;
    const cpx<R>* ay;
    const cpx<R>* by;
    const cpx<R>* gy;
    const R* D;
    R Dconst, Dref;
    cpx<R> kD;
    // absorbing faces with a varying speed: h^2-scaled per-axis weights (2 omega h
    // at absorbing end nodes), the diagonal gains i (abx + aby) sqrt(D_p); nullptr
    // when absent (D must then be given)
    const R* abx;
    const R* aby;
    const cpx<R>* x;
    const cpx<R>* in0;
    const cpx<R>* in1;
    const cpx<R>* add;
    cpx<R>* outA;
    cpx<R>* outB;
    cpx<R> cx[kMaxFused];
    R g[kMaxFused];
    R post, e3;
    int final_pass;
    // interior box: columns [ix0, ix1) and rows [iy0, iy1) have unit
    // neighbour weights on both axes (outside the layers and the end nodes)
    int64_t ix0, ix1, iy0, iy1;
    // set by launch_cheb2d: every pointer is valid, these flags mark absent operands
    int in0_zero, in1_zero, D_const;
    // geometry (cheb2d_geometry): strips of W output columns, segments of Ly rows
    int W, strips, Ly, segs;
};
template <typename R>
void cheb2d_geometry(ChebPassArgs<R>& a, int K, int NX, int Ly);
template <typename R>
void launch_cheb2d(const ChebPassArgs<R>& a, int K, int NX, hipStream_t s);
// Checks a pass against K, NX and points absent operands at x with their
// flags set, as launch_cheb2d does before a launch.
template <typename R>
ChebPassArgs<R> prepare_cheb2d(const ChebPassArgs<R>& a, int K, int NX);
// Workgroups of one pass (four wavefronts each, one strip segment per wavefront).
template <typename R>
int64_t cheb2d_blocks(const ChebPassArgs<R>& a);
// Batched form over the passes of grids of different sizes with one K, NX:
// each job holds prepared arguments and its range [block0, block0 + blocks)
// of workgroup indices (block0 a multiple of 64); lut maps each 64 indices
// to their job.  A persistent grid of resident workgroups covers
// total_blocks indices.
template <typename R>
struct Cheb2DJob {
    ChebPassArgs<R> a;
    int64_t block0, blocks;
};
template <typename R>
void launch_cheb2d_batch(const Cheb2DJob<R>* jobs, const uint32_t* lut, int64_t total_blocks, int K, int NX,
                         hipStream_t s);

// Complex-double BLAS-1 and deterministic reductions.  Vectors have length n;
// a "block" V holds nv vectors of length n back to back (stride ld >= n).
// Reductions write per-workgroup partial sums to `partial` and a second
// kernel sums them in a fixed order, so results are bitwise reproducible.
int reduce_blocks(int64_t n);  // number of partial sums used for length n

// TV, the basis' element type: cpx<double>, or cpx<float> for a complex-float
// basis (widened exactly; w and the sums stay complex double).
// out[i] = sum_p conj(V_i[p]) * w[p], i < nv   (out on device)
template <typename TV>
void launch_mdot(const TV* V, int64_t ld, int nv, const cpx<double>* w, int64_t n,
                 cpx<double>* partial, cpx<double>* out, hipStream_t s);
// w[p] -= sum_i h[i] * V_i[p]   (h on device)
template <typename TV>
void launch_mupdate(cpx<double>* w, const TV* V, int64_t ld, int nv,
                    const cpx<double>* h, int64_t n, hipStream_t s);
// w[p] += sum_i y[i] * V_i[p]   (y on device)
template <typename TV>
void launch_mcombine(cpx<double>* w, const TV* V, int64_t ld, int nv,
                     const cpx<double>* y, int64_t n, hipStream_t s);
// y = a*x rounded to complex float
void launch_scale_to_c64(cpx<double> a, const cpx<double>* x, cpx<float>* y, int64_t n, hipStream_t s);
// out[0].re = sum_p |w[p]|^2
void launch_nrm2sq(const cpx<double>* w, int64_t n, cpx<double>* partial, cpx<double>* out,
                   hipStream_t s);
// y = a*x + b*y
void launch_axpby(cpx<double> a, const cpx<double>* x, cpx<double> b, cpx<double>* y, int64_t n,
                  hipStream_t s);
// y = a*x
void launch_scale(cpx<double> a, const cpx<double>* x, cpx<double>* y, int64_t n, hipStream_t s);
// conversions between complex double and complex float
void launch_to_c64(const cpx<double>* x, cpx<float>* y, int64_t n, hipStream_t s);
void launch_to_c128(const cpx<float>* x, cpx<double>* y, int64_t n, hipStream_t s);
// D = 1/c^2 in double and float from a device speed array
void launch_inv_c2(const void* c, int is_f32, double* D64, float* D32, int64_t n, hipStream_t s);
// y = 0
template <typename R>
void launch_zero(cpx<R>* y, int64_t n, hipStream_t s);

}  // namespace mxp
