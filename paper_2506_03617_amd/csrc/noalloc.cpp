// The exponential action without any device allocation, for callers that
// cannot allocate (code under HIP graph capture, tight serving loops,
// harnesses that forbid it).  Its Clenshaw buffers and the schedule's
// diagonal tables live in one fixed device array, `scratch`, which every GPU
// the library runs on holds until the process ends.  Calls on one GPU share
// that array: calls that overlap on a GPU (several host threads) race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "engine.h"

namespace mxp {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be the current device,
// looked up once per device: each GPU holds its own copy of the array at its
// own address.
void* scratch_on(int device) {
    if (device < 0 || device >= kMaxDevices) fail(MXP_ERR_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) fail(MXP_ERR_HIP, "no device address for the scratch array");
        g_scratch_ptr[device] = p;
    }
    return g_scratch_ptr[device];
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace
}  // namespace mxp

using namespace mxp;

extern "C" mxp_status mxp_apply_exp_noalloc(mxp_problem* prob, double t, double shift, mxp_dtype dtype,
                                            const void* x, void* y) {
    return guard([&]() {
        check_problem(prob);
        if (!x || !y || x == y) fail(MXP_ERR_INVALID_ARG, "x and y must be distinct non-NULL pointers");
        if (dtype != MXP_C128 && dtype != MXP_C64) fail(MXP_ERR_INVALID_ARG, "dtype must be MXP_C64 or MXP_C128");
        if (!(t > 0) || !std::isfinite(t)) fail(MXP_ERR_INVALID_ARG, "t must be positive and finite");
        if (!(shift >= 0) || !std::isfinite(shift)) fail(MXP_ERR_INVALID_ARG, "shift must be >= 0");
        const size_t vec = align256(size_t(npts(prob)) * (dtype == MXP_C128 ? 16 : 8));
        const size_t need = 6 * vec + diag_table_bytes(prob->g);
        if (need > kScratchBytes)
            fail(MXP_ERR_INVALID_ARG, "the action needs " + std::to_string(need) + " bytes of scratch, more than the " +
                                          std::to_string(kScratchBytes) + " bytes of the no-allocation path");
        // check_problem made the problem's device current: the address is that device's copy
        unsigned char* base = static_cast<unsigned char*>(scratch_on(prob->ctx->device));
        hipStream_t s = prob->ctx->stream;
        const mxp_precision prec = dtype == MXP_C128 ? MXP_PREC_FP64 : MXP_PREC_MIXED;
        // the schedule, designed on the host; its diagonal tables follow the six vectors
        Sched sd;
        design_schedule(prob->g, t, shift, prec, &sd.s);
        sd.t = t;
        sd.prec = prec;
        build_diag(prob, shift, cd(sd.s.centre_re, sd.s.centre_im), sd.diag, base + 6 * vec, s);
        // 2D passes: the problem's tuned tiles, else six levels per pass (no tuning here)
        TileCfg tc = prob->tiles[prec == MXP_PREC_MIXED ? 1 : 0];
        if (prob->g.dim == 2 && tc.K == 0) {
            tc.K = 6;
            tc.NX = 1;
            tc.Ly = 32;
        }
        void* bufs[6];
        for (int q = 0; q < 6; ++q) bufs[q] = base + q * vec;
        int64_t steps = 0;
        apply_action_on(prob, bufs, tc, s, sd, t, shift, dtype, x, y, &steps);
        HIP_CHECK(hipStreamSynchronize(s));
        return MXP_OK;
    });
}
