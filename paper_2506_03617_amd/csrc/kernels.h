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
};

template <typename R>
void launch_stencil(const StencilArgs<R>& a, hipStream_t s);

// Complex-double BLAS-1 and deterministic reductions.  Vectors have length n;
// a "block" V holds nv vectors of length n back to back (stride ld >= n).
// Reductions write per-workgroup partial sums to `partial` and a second
// kernel sums them in a fixed order, so results are bitwise reproducible.
int reduce_blocks(int64_t n);  // number of partial sums used for length n

// out[i] = sum_p conj(V_i[p]) * w[p], i < nv   (complex double, out on device)
void launch_mdot(const cpx<double>* V, int64_t ld, int nv, const cpx<double>* w, int64_t n,
                 cpx<double>* partial, cpx<double>* out, hipStream_t s);
// w[p] -= sum_i h[i] * V_i[p]   (h on device)
void launch_mupdate(cpx<double>* w, const cpx<double>* V, int64_t ld, int nv,
                    const cpx<double>* h, int64_t n, hipStream_t s);
// w[p] += sum_i y[i] * V_i[p]   (y on device)
void launch_mcombine(cpx<double>* w, const cpx<double>* V, int64_t ld, int nv,
                     const cpx<double>* y, int64_t n, hipStream_t s);
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
