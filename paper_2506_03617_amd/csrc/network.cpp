// The learned stage's network: parameters, forward and backward passes, one
// Adam training step, and the C ABI around them.  Every layer runs on the
// bf16 matrix-core kernels of cnn.hip; the master weights, gradients and Adam
// moments are float.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <optional>
#include <random>
#include <vector>

#include "cnn_net.h"
#include "mxp_internal.h"

namespace mxp {

extern thread_local std::string g_last_error;

namespace {

int cin_pad(int l) { return l == 0 ? 8 : 32; }        // channels of layer l's input tensor
int gout_ch(int l) { return l == kLayers - 1 ? 8 : 32; }  // channels of layer l's output gradient

// keep: training shapes (every activation and the gradient buffers);
// otherwise the two alternating activation buffers of inference.  Work still
// queued on the stream may use a buffer that has to grow, so the stream is
// drained before any reallocation.
void ensure_shape(mxp_cnn* net, int64_t V, bool keep, hipStream_t st) {
    const size_t a32 = size_t(V) * 32 * 2, o2 = size_t(V) * 2 * 4, g8 = size_t(V) * 8 * 2;
    bool grow = net->out.bytes < o2;
    for (int l = 1; l < (keep ? kLayers : 3); ++l) grow = grow || net->act[l].bytes < a32;
    if (keep) grow = grow || net->g6.bytes < g8 || net->gA.bytes < a32 || net->gB.bytes < a32;
    if (grow) HIP_CHECK(hipStreamSynchronize(st));
    for (int l = 1; l < (keep ? kLayers : 3); ++l) net->act[l].ensure(a32);
    net->out.ensure(o2);
    if (!keep) return;
    net->g6.ensure(g8);
    net->gA.ensure(a32);
    net->gB.ensure(a32);
    net->wpart.ensure(size_t(conv_wgrad_max_groups()) * 27 * 32 * 32 * 4);
    net->bpart.ensure(size_t(1024) * 32 * 4);
    net->lpart.ensure(size_t(1024) * 8);
    net->lsum.ensure(8);
}

void pack(mxp_cnn* net, hipStream_t st) {
    for (int l = 0; l < kLayers; ++l) {
        net->wf[l].ensure(size_t(27) * 32 * cin_pad(l) * 2);
        if (l > 0) net->wb[l].ensure(size_t(27) * 32 * gout_ch(l) * 2);
        launch_pack_weights(net->params.as<float>() + net->offW[l], kChannels[l + 1], kChannels[l], cin_pad(l),
                            gout_ch(l), net->wf[l].as<uint16_t>(), l > 0 ? net->wb[l].as<uint16_t>() : nullptr, st);
    }
    net->packed = true;
}

void check_shape(const ConvShape& s) {
    if (s.nb < 1 || s.nz < 1 || s.ny < 1 || s.nx < 1) fail(MXP_ERR_INVALID_ARG, "network shape must be positive");
}

// Gradients of every parameter for output gradient g6 (bf16 [V][8]), with the
// activations of the preceding forward pass (input `in`).
void backward(mxp_cnn* net, const ConvShape& s, const uint16_t* in, hipStream_t st) {
    const int64_t V = s.voxels();
    const uint16_t* g = net->g6.as<uint16_t>();
    uint16_t* bufs[2] = {net->gA.as<uint16_t>(), net->gB.as<uint16_t>()};
    int which = 0;
    for (int l = kLayers - 1; l >= 0; --l) {
        const uint16_t* H = l == 0 ? in : net->act[l].as<uint16_t>();
        const int groups = launch_conv_wgrad(gout_ch(l), cin_pad(l), g, H, net->wpart.as<float>(), s, st);
        launch_wgrad_reduce(net->wpart.as<float>(), groups, kChannels[l + 1], kChannels[l],
                            net->grads.as<float>() + net->offW[l], st);
        launch_bias_grad(g, gout_ch(l), kChannels[l + 1], V, net->bpart.as<float>(),
                         net->grads.as<float>() + net->offB[l], st);
        if (l > 0) {
            // gradient of act[l] through the transposed convolution, masked by
            // the ReLU that produced act[l]
            uint16_t* next = bufs[which];
            which ^= 1;
            launch_conv(gout_ch(l), CONV_MASK, g, net->wb[l].as<uint16_t>(), nullptr, net->act[l].as<uint16_t>(),
                        next, s, st);
            g = next;
        }
    }
}

}  // namespace

void cnn_forward(mxp_cnn* net, const ConvShape& s, const uint16_t* in, float* out, bool keep, hipStream_t st) {
    check_shape(s);
    if (!net->packed) pack(net, st);
    // workspace first: every internal pointer is taken after it is allocated
    ensure_shape(net, s.voxels(), keep, st);
    net->kept_voxels = keep ? s.voxels() : 0;
    if (!out) out = net->out.as<float>();
    const uint16_t* x = in;
    for (int l = 0; l < kLayers; ++l) {
        const float* b = net->params.as<float>() + net->offB[l];
        if (l == kLayers - 1) {
            launch_conv(cin_pad(l), CONV_BIAS_F32, x, net->wf[l].as<uint16_t>(), b, nullptr, out, s, st);
        } else {
            uint16_t* y = keep ? net->act[l + 1].as<uint16_t>() : net->act[1 + (l & 1)].as<uint16_t>();
            launch_conv(cin_pad(l), CONV_BIAS_RELU, x, net->wf[l].as<uint16_t>(), b, nullptr, y, s, st);
            x = y;
        }
    }
}

void cnn_reserve(mxp_cnn* net, const ConvShape& s, hipStream_t st) {
    check_shape(s);
    if (!net->packed) pack(net, st);
    ensure_shape(net, s.voxels(), false, st);
    net->io_in.ensure(size_t(s.voxels()) * 8 * 2);
    net->io_scale.ensure(2 * sizeof(double));
}

void cnn_apply(mxp_cnn* net, const ConvShape& s, const void* v, const float* D, float Dc, double rs,
               double out_scale, void* z, hipStream_t st) {
    const int64_t V = s.voxels();
    if (net->io_in.bytes < size_t(V) * 8 * 2) HIP_CHECK(hipStreamSynchronize(st));
    net->io_in.ensure(size_t(V) * 8 * 2);
    net->io_scale.ensure(2 * sizeof(double));
    const double sc[2] = {rs, out_scale};
    HIP_CHECK(hipMemcpyAsync(net->io_scale.p, sc, sizeof(sc), hipMemcpyHostToDevice, st));
    const double* dsc = net->io_scale.as<double>();
    launch_cnn_input(v, D, Dc, dsc, V, net->io_in.as<uint16_t>(), st);
    cnn_forward(net, s, net->io_in.as<uint16_t>(), nullptr, false, st);
    launch_cnn_output(net->out.as<float>(), dsc + 1, V, z, st);
    // the scales live in a host array that goes out of scope
    HIP_CHECK(hipStreamSynchronize(st));
}

template <class F>
static mxp_status cnn_guard(const Allocator* al, F&& fn) {
    try {
        g_last_error.clear();
        std::optional<AllocScope> scope;
        if (al) scope.emplace(*al);
        return fn();
    } catch (const Error& e) {
        g_last_error = e.what();
        return e.status;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return MXP_ERR_OOM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return MXP_ERR_HIP;
    }
}

}  // namespace mxp

using namespace mxp;

extern "C" {

int64_t mxp_cnn_num_params(void) {
    int64_t n = 0;
    for (int l = 0; l < kLayers; ++l) n += int64_t(kChannels[l + 1]) * (kChannels[l] * 27 + 1);
    return n;
}

mxp_status mxp_cnn_create(mxp_context* ctx, uint64_t seed, mxp_cnn** out) {
    return cnn_guard(nullptr, [&]() {
        if (!ctx || !out) fail(MXP_ERR_INVALID_ARG, "context or out is NULL");
        AllocScope scope(context_alloc(ctx));
        *out = nullptr;
        int dev = 0;
        hipStream_t st = nullptr;
        context_info(ctx, &dev, &st);
        HIP_CHECK(hipSetDevice(dev));
        auto net = std::make_unique<mxp_cnn>();
        net->device = dev;
        net->stream = st;
        net->alloc = context_alloc(ctx);
        int64_t off = 0;
        for (int l = 0; l < kLayers; ++l) {
            net->offW[l] = off;
            off += int64_t(kChannels[l + 1]) * kChannels[l] * 27;
            net->offB[l] = off;
            off += kChannels[l + 1];
        }
        net->nparam = off;
        // He-normal weights (standard deviation sqrt(2 / fan_in)), zero biases
        std::vector<float> host(size_t(off), 0.0f);
        std::mt19937_64 gen(seed);
        std::normal_distribution<double> nd(0.0, 1.0);
        for (int l = 0; l < kLayers; ++l) {
            const double sd = std::sqrt(2.0 / (kChannels[l] * 27));
            for (int64_t k = 0; k < int64_t(kChannels[l + 1]) * kChannels[l] * 27; ++k)
                host[size_t(net->offW[l] + k)] = float(nd(gen) * sd);
        }
        const size_t bytes = size_t(off) * 4;
        net->params.ensure(bytes);
        net->grads.ensure(bytes);
        net->adam_m.ensure(bytes);
        net->adam_v.ensure(bytes);
        HIP_CHECK(hipMemcpy(net->params.p, host.data(), bytes, hipMemcpyHostToDevice));
        HIP_CHECK(hipMemset(net->grads.p, 0, bytes));
        HIP_CHECK(hipMemset(net->adam_m.p, 0, bytes));
        HIP_CHECK(hipMemset(net->adam_v.p, 0, bytes));
        *out = net.release();
        return MXP_OK;
    });
}

void mxp_cnn_destroy(mxp_cnn* net) {
    if (!net) return;
    (void)hipSetDevice(net->device);
    (void)hipStreamSynchronize(net->stream);
    delete net;
}

mxp_status mxp_cnn_get_params(const mxp_cnn* net, float* host) {
    return cnn_guard(net ? &net->alloc : nullptr, [&]() {
        if (!net || !host) fail(MXP_ERR_INVALID_ARG, "network or buffer is NULL");
        HIP_CHECK(hipSetDevice(net->device));
        HIP_CHECK(hipStreamSynchronize(net->stream));
        HIP_CHECK(hipMemcpy(host, net->params.p, size_t(net->nparam) * 4, hipMemcpyDeviceToHost));
        return MXP_OK;
    });
}

mxp_status mxp_cnn_set_params(mxp_cnn* net, const float* host) {
    return cnn_guard(net ? &net->alloc : nullptr, [&]() {
        if (!net || !host) fail(MXP_ERR_INVALID_ARG, "network or buffer is NULL");
        for (int64_t k = 0; k < net->nparam; ++k)
            if (!std::isfinite(host[k])) fail(MXP_ERR_NONFINITE, "non-finite parameter");
        HIP_CHECK(hipSetDevice(net->device));
        HIP_CHECK(hipStreamSynchronize(net->stream));
        const size_t bytes = size_t(net->nparam) * 4;
        HIP_CHECK(hipMemcpy(net->params.p, host, bytes, hipMemcpyHostToDevice));
        HIP_CHECK(hipMemset(net->adam_m.p, 0, bytes));
        HIP_CHECK(hipMemset(net->adam_v.p, 0, bytes));
        net->adam_t = 0;
        net->packed = false;
        return MXP_OK;
    });
}

mxp_status mxp_cnn_get_grads(const mxp_cnn* net, float* host) {
    return cnn_guard(net ? &net->alloc : nullptr, [&]() {
        if (!net || !host) fail(MXP_ERR_INVALID_ARG, "network or buffer is NULL");
        HIP_CHECK(hipSetDevice(net->device));
        HIP_CHECK(hipStreamSynchronize(net->stream));
        HIP_CHECK(hipMemcpy(host, net->grads.p, size_t(net->nparam) * 4, hipMemcpyDeviceToHost));
        return MXP_OK;
    });
}

mxp_status mxp_cnn_save(const mxp_cnn* net, const char* path) {
    return cnn_guard(net ? &net->alloc : nullptr, [&]() {
        if (!net || !path) fail(MXP_ERR_INVALID_ARG, "network or path is NULL");
        HIP_CHECK(hipSetDevice(net->device));
        HIP_CHECK(hipStreamSynchronize(net->stream));
        const size_t n = size_t(net->nparam);
        std::vector<float> buf(3 * n);
        HIP_CHECK(hipMemcpy(buf.data(), net->params.p, n * 4, hipMemcpyDeviceToHost));
        HIP_CHECK(hipMemcpy(buf.data() + n, net->adam_m.p, n * 4, hipMemcpyDeviceToHost));
        HIP_CHECK(hipMemcpy(buf.data() + 2 * n, net->adam_v.p, n * 4, hipMemcpyDeviceToHost));
        write_checkpoint(path, kLayers, kChannels, net->nparam, net->adam_t, buf);
        return MXP_OK;
    });
}

mxp_status mxp_cnn_load(mxp_cnn* net, const char* path) {
    return cnn_guard(net ? &net->alloc : nullptr, [&]() {
        if (!net || !path) fail(MXP_ERR_INVALID_ARG, "network or path is NULL");
        std::vector<float> buf;
        int64_t t = 0;
        read_checkpoint(path, kLayers, kChannels, net->nparam, &t, &buf);
        const size_t n = size_t(net->nparam);
        HIP_CHECK(hipSetDevice(net->device));
        HIP_CHECK(hipStreamSynchronize(net->stream));
        HIP_CHECK(hipMemcpy(net->params.p, buf.data(), n * 4, hipMemcpyHostToDevice));
        HIP_CHECK(hipMemcpy(net->adam_m.p, buf.data() + n, n * 4, hipMemcpyHostToDevice));
        HIP_CHECK(hipMemcpy(net->adam_v.p, buf.data() + 2 * n, n * 4, hipMemcpyHostToDevice));
        net->adam_t = t;
        net->packed = false;
        return MXP_OK;
    });
}

mxp_status mxp_cnn_forward(mxp_cnn* net, int32_t nb, int32_t nz, int32_t ny, int32_t nx, const void* in,
                           float* out) {
    return cnn_guard(net ? &net->alloc : nullptr, [&]() {
        if (!net || !in || !out) fail(MXP_ERR_INVALID_ARG, "network, input or output is NULL");
        HIP_CHECK(hipSetDevice(net->device));
        const ConvShape s{nb, nz, ny, nx};
        cnn_forward(net, s, static_cast<const uint16_t*>(in), out, false, net->stream);
        HIP_CHECK(hipStreamSynchronize(net->stream));
        return MXP_OK;
    });
}

mxp_status mxp_cnn_backward(mxp_cnn* net, int32_t nb, int32_t nz, int32_t ny, int32_t nx, const void* in,
                            const float* gout) {
    return cnn_guard(net ? &net->alloc : nullptr, [&]() {
        if (!net || !in || !gout) fail(MXP_ERR_INVALID_ARG, "network, input or gradient is NULL");
        HIP_CHECK(hipSetDevice(net->device));
        const ConvShape s{nb, nz, ny, nx};
        const uint16_t* x = static_cast<const uint16_t*>(in);
        cnn_forward(net, s, x, nullptr, true, net->stream);
        launch_grad_to_bf16(gout, s.voxels(), net->g6.as<uint16_t>(), net->stream);
        backward(net, s, x, net->stream);
        HIP_CHECK(hipStreamSynchronize(net->stream));
        return MXP_OK;
    });
}

mxp_status mxp_cnn_get_activations(const mxp_cnn* net, int32_t layer, int64_t voxels, uint16_t* host) {
    return cnn_guard(net ? &net->alloc : nullptr, [&]() {
        if (!net || !host) fail(MXP_ERR_INVALID_ARG, "network or buffer is NULL");
        if (layer < 1 || layer >= kLayers) fail(MXP_ERR_INVALID_ARG, "layer must be 1..5");
        if (voxels <= 0 || voxels != net->kept_voxels)
            fail(MXP_ERR_INVALID_ARG, "voxels must be those of the last backward or training step");
        HIP_CHECK(hipSetDevice(net->device));
        HIP_CHECK(hipStreamSynchronize(net->stream));
        HIP_CHECK(hipMemcpy(host, net->act[layer].p, size_t(voxels) * 32 * 2, hipMemcpyDeviceToHost));
        return MXP_OK;
    });
}

mxp_status mxp_cnn_train_step(mxp_cnn* net, int32_t nb, int32_t nz, int32_t ny, int32_t nx, const void* in,
                              const float* target, float lr, double* loss) {
    return cnn_guard(net ? &net->alloc : nullptr, [&]() {
        if (!net || !in || !target) fail(MXP_ERR_INVALID_ARG, "network, input or target is NULL");
        if (!(lr > 0) || !std::isfinite(lr)) fail(MXP_ERR_INVALID_ARG, "learning rate must be positive");
        HIP_CHECK(hipSetDevice(net->device));
        const ConvShape s{nb, nz, ny, nx};
        hipStream_t st = net->stream;
        const uint16_t* x = static_cast<const uint16_t*>(in);
        cnn_forward(net, s, x, nullptr, true, st);
        launch_mse(net->out.as<float>(), target, s.voxels(), net->g6.as<uint16_t>(), net->lpart.as<double>(),
                   net->lsum.as<double>(), st);
        backward(net, s, x, st);
        net->adam_t += 1;
        const float b1 = 0.9f, b2 = 0.999f;
        const float bc1 = float(1.0 - std::pow(0.9, double(net->adam_t)));
        const float bc2 = float(1.0 - std::pow(0.999, double(net->adam_t)));
        launch_adam(net->params.as<float>(), net->adam_m.as<float>(), net->adam_v.as<float>(),
                    net->grads.as<float>(), net->nparam, lr, b1, b2, 1e-8f, bc1, bc2, st);
        pack(net, st);
        double l = 0.0;
        HIP_CHECK(hipMemcpyAsync(&l, net->lsum.p, sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_CHECK(hipStreamSynchronize(st));
        if (loss) *loss = l / double(2 * s.voxels());
        if (!std::isfinite(l)) fail(MXP_ERR_NONFINITE, "non-finite training loss");
        return MXP_OK;
    });
}

}  // extern "C"
