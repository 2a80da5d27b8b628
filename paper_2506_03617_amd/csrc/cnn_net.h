// The learned stage's network object (internal): parameters, Adam state,
// bf16 weight layouts and activation workspace on one device.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "cnn.h"
#include "devmem.h"

namespace mxp {

constexpr int kLayers = 6;
constexpr int kChannels[kLayers + 1] = {3, 32, 32, 32, 32, 32, 2};

}  // namespace mxp

struct mxp_cnn {
    int device;
    hipStream_t stream;
    mxp::Allocator alloc;  // the context's device-memory hooks
    // master parameters, gradients and Adam moments (float), flattened layer
    // by layer: W [cout][cin][27] then b [cout]
    mxp::DevMem params, grads, adam_m, adam_v;
    int64_t offW[mxp::kLayers], offB[mxp::kLayers], nparam;
    int64_t adam_t = 0;
    mxp::DevMem wf[mxp::kLayers], wb[mxp::kLayers];  // bf16 forward / data-gradient layouts
    bool packed = false;
    // activation workspace (voxels of the last shape used)
    mxp::DevMem act[mxp::kLayers];  // act[1..5]: bf16 [V][32]; act[0] unused (the input is the caller's)
    int64_t kept_voxels = 0;        // V of the last forward that kept every activation
    mxp::DevMem out;                // float [V][2]
    mxp::DevMem g6, gA, gB;         // bf16 gradients
    mxp::DevMem wpart, bpart, lpart, lsum;
    mxp::DevMem io_in, io_scale;    // solver inference: bf16 input, two scales
};

namespace mxp {

// Device, stream and allocator of a context (defined with the context).
void context_info(const mxp_context* ctx, int* device, hipStream_t* stream);
const Allocator& context_alloc(const mxp_context* ctx);
// Reserves the network's inference buffers for volumes of `s`.
void cnn_reserve(mxp_cnn* net, const ConvShape& s, hipStream_t st);

// Network forward; with keep = true every activation is kept for backward,
// else two buffers alternate.  in: bf16 [V][8] device; out: float [V][2], or
// nullptr for the network's own output buffer (allocated here first).
void cnn_forward(mxp_cnn* net, const ConvShape& s, const uint16_t* in, float* out, bool keep, hipStream_t st);
// z = net applied to the residual v (complex double, one volume nz x ny x nx):
// input (v * rs, D), output scaled by out_scale.  D: float per node or nullptr
// with the constant Dc.
void cnn_apply(mxp_cnn* net, const ConvShape& s, const void* v, const float* D, float Dc, double rs,
               double out_scale, void* z, hipStream_t st);

}  // namespace mxp
