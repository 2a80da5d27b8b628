// Device kernels of the learned preconditioner stage (internal).
//
// The network: six 3x3x3 convolutions with zero padding, channels
// 3 -> 32 -> 32 -> 32 -> 32 -> 32 -> 2, bias on every layer, ReLU after the
// first five.  Tensors are channels-last bfloat16, [voxel][C] with the voxel
// index x fastest, C = 8 for the network input (3 used) and the last layer's
// gradient (2 used), C = 32 otherwise.  The output is float [voxel][2].  A
// batch is nb volumes of nz x ny x nx voxels stored one after another; each
// volume is zero-padded on its own.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mxp {

struct ConvShape {
    int nb, nz, ny, nx;
    int64_t voxels() const { return int64_t(nb) * nz * ny * nx; }
};

// Epilogues of the implicit-GEMM convolution.
enum ConvMode {
    CONV_BIAS_RELU = 0,  // out bf16 [V][32] = relu(conv + bias)
    CONV_BIAS_F32 = 1,   // out float [V][2] = conv + bias (output channels 0, 1)
    CONV_MASK = 2,       // out bf16 [V][32] = conv * (mask > 0), mask bf16 [V][32]
};

// out = conv(in, w) with the chosen epilogue.  cin: 8 or 32 (channels of in);
// w: bf16 [27][32][cin] (tap-major, output channel, input channel; taps
// ordered dz, dy, dx with dx fastest; unused rows zero).
void launch_conv(int cin, ConvMode mode, const uint16_t* in, const uint16_t* w, const float* bias,
                 const uint16_t* mask, void* out, const ConvShape& s, hipStream_t st);

// Weight gradient partial sums: partial[g][tap][co][ci] over the bricks
// workgroup g handles, for gW[co][ci][tap] = sum_v G[v][co] H[v + tap - 1][ci].
// cg: channels of G (8 or 32), ch: channels of H (8 or 32).  Returns the
// number of workgroups (partials) used; partial must hold that many
// 27 * 32 * 32 floats (at most conv_wgrad_max_groups()).
int conv_wgrad_max_groups();
int launch_conv_wgrad(int cg, int ch, const uint16_t* G, const uint16_t* H, float* partial, const ConvShape& s,
                      hipStream_t st);
// gW (float [cout][cin][27], the master layout) = sum over groups of partial.
void launch_wgrad_reduce(const float* partial, int groups, int cout, int cin, float* gW, hipStream_t st);
// gb[co] = sum_v G[v][co], co < cout (G has cg channels); partial: >= 1024 * 32 floats.
void launch_bias_grad(const uint16_t* G, int cg, int cout, int64_t V, float* partial, float* gb, hipStream_t st);

// Mean squared error of out (float [V][2]) against target (float [V][2]):
// gout bf16 [V][8] = 2 (out - target) / (2 V) in channels 0, 1 (zeros after),
// lsum[0] = sum (out - target)^2 in double (deterministic two passes;
// partial: >= 1024 doubles).
void launch_mse(const float* out, const float* target, int64_t V, uint16_t* gout, double* partial, double* lsum,
                hipStream_t st);
// gout bf16 [V][8] from a float [V][2] output gradient.
void launch_grad_to_bf16(const float* g, int64_t V, uint16_t* gout, hipStream_t st);

// Adam update of n parameters (float), bias corrections given.
void launch_adam(float* w, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2, float eps,
                 float bc1, float bc2, hipStream_t st);
// bf16 layouts of one layer from the master weights W [cout][cin][27]:
// wf [27][32][cinp] (forward) and, when wb != nullptr, wb [27][32][coutp]
// with wb[t][ci][co] = W[co][ci][26 - t] (the data gradient's correlation).
void launch_pack_weights(const float* W, int cout, int cin, int cinp, int coutp, uint16_t* wf, uint16_t* wb,
                         hipStream_t st);

// Network input from a complex residual: channels (Re r, Im r) * scale[0]
// and D = 1/c^2 (or the constant Dc when D == nullptr), zeros after;
// scale: device double.  r: complex double [V].
void launch_cnn_input(const void* r, const float* D, float Dc, const double* scale, int64_t V, uint16_t* in,
                      hipStream_t st);
// z (complex double [V]) = scale[0] * (out[v][0] + i out[v][1]).
void launch_cnn_output(const float* out, const double* scale, int64_t V, void* z, hipStream_t st);
// Training sample from a (residual, preconditioned residual) pair on a grid
// of g0 x g1 x g2 nodes: the crop of c0 x c1 x c2 nodes at offset (o0, o1,
// o2): in bf16 [crop][8] as launch_cnn_input with scale rs, target float
// [crop][2] = zs * z.
void launch_cnn_crop(const void* r, const void* z, const float* D, float Dc, int64_t g0, int64_t g1, int o0,
                     int o1, int o2, int c0, int c1, int c2, double rs, double zs, uint16_t* in, float* target,
                     hipStream_t st);

}  // namespace mxp
