// Two-level Clenshaw passes on 3D grids (internal).
#pragma once

#include "kernels.h"

namespace mxp {

// Two consecutive Clenshaw levels in one pass over a 3D grid:
//   L_0 = cx[0] x + g[0] S(in1) - in0,   L_1 = cx[1] x + g[1] S(L_0) - in1,
// S the stencil of StencilArgs (unscaled tables, the centre folded into
// gamma, kD (D - Dref) per node); in0 / in1 = nullptr read as zero.  Writes
// L_0 to outA and L_1 to outB; outputs must not alias any input.  Geometry
// (cheb3d_geometry): tiles of 62 x 14 output columns x rows, chunks of zc
// planes; a workgroup of sixteen wavefronts also recomputes L_0 on a one-node
// halo in x and y and one plane in z on each side.
template <typename R>
struct ChebPass3DArgs {
    int64_t n0, n1, n2;
    const cpx<R>* alpha[3];
    const cpx<R>* beta[3];
    const cpx<R>* gamma[3];
    const R* D;
    R Dconst, Dref;
    cpx<R> kD;
    const cpx<R>* x;
    const cpx<R>* in0;
    const cpx<R>* in1;
    cpx<R>* outA;
    cpx<R>* outB;
    cpx<R> cx[3];  // the two-level pass reads [0..1], the three-level pass [0..2]
    R g[3];
    int tiles_x, tiles_y, zchunks, zc;
};
template <typename R>
void cheb3d_geometry(ChebPass3DArgs<R>& a, int zc);  // zc: planes per z-chunk, 0 for 32
template <typename R>
int cheb3d_variant(const ChebPass3DArgs<R>& a);  // 1: D present, 2: in0, 4: in1
template <typename R>
void launch_cheb3d(const ChebPass3DArgs<R>& a, hipStream_t s);
// Three consecutive levels in one pass over a 3D grid:
//   L_0 = cx[0] x + g[0] S(in1) - in0,   L_1 = cx[1] x + g[1] S(L_0) - in1,
//   L_2 = cx[2] x + g[2] S(L_1) - L_0;
// writes L_1 to outA and L_2 to outB (the two levels the next pass reads).
// Geometry (cheb3d3_geometry): tiles of 60 columns and the workgroup's output
// rows, chunks of zc planes (0: 32); L_0 is recomputed on a two-node halo and
// L_1 on a one-node halo in x, y and z.
template <typename R>
void cheb3d3_geometry(ChebPass3DArgs<R>& a, int zc);
template <typename R>
void launch_cheb3d3(const ChebPass3DArgs<R>& a, hipStream_t s);
// Batched form over grids of different sizes (same variant): as Sweep3DJob.
template <typename R>
struct Cheb3DJob {
    ChebPass3DArgs<R> a;
    int64_t block0, blocks;
};
template <typename R>
void launch_cheb3d_batch(const Cheb3DJob<R>* jobs, const uint32_t* lut, int64_t total_blocks, int variant,
                         hipStream_t s);
// The same for three-level passes (jobs set up by cheb3d3_geometry).
template <typename R>
void launch_cheb3d3_batch(const Cheb3DJob<R>* jobs, const uint32_t* lut, int64_t total_blocks, int variant,
                          hipStream_t s);

}  // namespace mxp
