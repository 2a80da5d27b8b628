// Learned preconditioner stage: 3x3x3 convolutions on the bf16 matrix cores
// of gfx950 (v_mfma_f32_32x32x16_bf16, float accumulation), and the small
// kernels of training (loss, bias gradient, Adam, weight packing) and of
// moving residuals in and out of the network.
//
// Convolution as an implicit GEMM over (tap, input channel), marching along z
// (k_conv_zm below).  MFMA lane layout (checked on the device): A row i =
// lane % 32 with k = 8 (lane / 32) .. +7, B column j = lane % 32 with the
// same k, result register r holds row 8 (r / 4) + 4 (lane / 32) + r % 4 of
// column lane % 32.
#include <hip/hip_runtime.h>

#include <string>

#include "cnn.h"
#include "mxp_internal.h"

namespace mxp {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ bf16x8 ld8(const uint16_t* p) {
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}
__device__ __forceinline__ uint16_t bf16_bits(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf16_value(uint16_t h) { return __builtin_bit_cast(float, uint32_t(h) << 16); }
__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

inline void check_launch(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(MXP_ERR_HIP, std::string("kernel launch failed (") + what + "): " + hipGetErrorString(e));
}

// ------------------------------------------------- z-marching convolution
//
// A workgroup of four wavefronts owns a column of 32 x 8 output voxels (x, y)
// over a segment of z planes and marches along z.  Input plane p, with a
// one-voxel halo in x and y (34 x 10 voxels), is staged in LDS, double
// buffered: the next plane's loads are issued before the current plane's
// products and written to the other buffer after them.  Input plane p feeds
// output planes p + 1, p and p - 1 (taps dz = 0, 1, 2), held in three
// accumulators that rotate with the plane (the plane loop is unrolled by
// three, so the rotation is compile-time); after plane p, output plane p - 1
// is complete.  Wavefront w computes output rows 2w and 2w + 1, one 32 x 32
// tile each (output channels x voxels): the weights are the MFMA A operand
// and the activations B.  Per plane it reads its 24 activation fragments
// (input rows 2w .. 2w + 3, three x shifts, two 16-channel halves) once and
// streams the 54 weight fragments, each used for both rows, so the LDS
// operand traffic is 78 reads per 108 products.  With eight input channels
// (the first layer, and the data gradient of the last) one product covers two
// taps of the same dz: half-wavefront kh takes tap 2q + kh of the nine, the
// ninth paired with zero weights, so a plane costs 30 products from 10
// activation and 15 weight reads per wavefront.  The weights (27 x 32 x cin)
// stay in LDS for all the segments a (persistent) workgroup visits.
//
// The last layer has two output channels, so a 32-channel tile would waste
// 30 of its rows.  There the (dz, dy) taps go into the rows instead: row
// i = 8 g + 4 h + q stands for output channel h and tap pair t = 4 g + q
// (dz = t / 3, dy = t % 3; rows with t >= 9 have zero weights), and K runs
// over (dx, input channel).  One input row then needs six products (three dx
// times two channel halves) whose result register t of half-wavefront h is
// the partial sum of channel h for output plane p + 1 - dz and row hy - dy;
// each lane adds it to one of six running sums (three planes, two rows).  That
// is 24 products per plane instead of 108, with the weights (six fragments)
// held in registers.
constexpr int ZX = 32, ZY = 8;                  // output voxels per column
constexpr int ZHX = ZX + 2, ZHY = ZY + 2;       // staged plane with halo

template <int CIN>
struct ZLayout {
    static constexpr int CS = CIN == 32 ? 40 : 8;         // channel stride (bf16), padded for 32
    static constexpr int CH = CIN / 8;                    // 16-byte chunks per voxel
    static constexpr int PLANE = ZHX * ZHY * CS;          // bf16 per staged plane
    static constexpr int CHUNKS = ZHX * ZHY * CH;         // 16-byte chunks per plane
    static constexpr int LOADS = (CHUNKS + 255) / 256;    // chunks per thread
};

struct ZMarch {
    int tx, ty, zsegs, Lz;  // columns in x and y, segments per volume, planes per segment
};

template <int CIN, int MODE>
struct ZConv {
    using L = ZLayout<CIN>;
    static constexpr int ZCS = L::CS, ZPLANE = L::PLANE, ZCHUNKS = L::CHUNKS, ZLOADS = L::LOADS;
    static constexpr bool LAST = MODE == CONV_BIAS_F32;  // two output channels
    static_assert(!LAST || CIN == 32, "the two-channel layer reads 32 channels");
    const uint16_t* in;
    ConvShape s;
    int x0, y0, vol, za, zb;
    int64_t vbase;
    int lane, wv, j, kh;
    f32x16 acc[2][3];
    float oacc[3][2];    // last layer: running sums, [plane slot][row], channel kh
    bf16x8 wl[3][2];     // last layer: weight fragments per (dx, channel half)
    uint4 stg[ZLOADS];

    // Loads of input plane p (zero outside the volume); every address is
    // clamped into the volume, so the loads are unconditional.
    __device__ __forceinline__ void issue(int p, int tid) {
        const bool pin = p >= 0 && p < s.nz;
        const int pc = p < 0 ? 0 : (p >= s.nz ? s.nz - 1 : p);
#pragma unroll
        for (int q = 0; q < ZLOADS; ++q) {
            const int c = tid + 256 * q;
            const int cc = c < ZCHUNKS ? c : ZCHUNKS - 1;
            const int ch = cc % L::CH, v = cc / L::CH;
            const int hx = v % ZHX, hy = v / ZHX;
            const int gx = x0 - 1 + hx, gy = y0 - 1 + hy;
            const bool ok = pin && gx >= 0 && gx < s.nx && gy >= 0 && gy < s.ny;
            const int gxc = gx < 0 ? 0 : (gx >= s.nx ? s.nx - 1 : gx);
            const int gyc = gy < 0 ? 0 : (gy >= s.ny ? s.ny - 1 : gy);
            const uint4 val =
                *reinterpret_cast<const uint4*>(in + (vbase + (int64_t(pc) * s.ny + gyc) * s.nx + gxc) * CIN + ch * 8);
            stg[q] = ok ? val : make_uint4(0u, 0u, 0u, 0u);
        }
    }
    __device__ __forceinline__ void commit(uint16_t* slot, int tid) {
#pragma unroll
        for (int q = 0; q < ZLOADS; ++q) {
            const int c = tid + 256 * q;
            if (c < ZCHUNKS) {
                const int ch = c % L::CH, v = c / L::CH;
                *reinterpret_cast<uint4*>(&slot[v * ZCS + ch * 8]) = stg[q];
            }
        }
    }

    // Products of one tap plane dz with the staged activations B: output
    // plane p + 1 - dz, accumulator slot (PH - dz) mod 3.
    template <int PH, int DZ>
    __device__ __forceinline__ void tap_plane(const bf16x8 (&B)[4][3][2], const uint16_t* s_w) {
        constexpr int SL = (PH - DZ + 3) % 3;
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                for (int kb = 0; kb < 2; ++kb) {
                    const int tap = DZ * 9 + dy * 3 + dx;
                    const bf16x8 a = ld8(s_w + (tap * 32 + j) * ZCS + 16 * kb + 8 * kh);
                    acc[0][SL] = mfma(a, B[dy][dx][kb], acc[0][SL]);
                    acc[1][SL] = mfma(a, B[dy + 1][dx][kb], acc[1][SL]);
                }
    }

    // Eight input channels: tap pairs (2q, 2q + 1) of one dz.
    template <int PH, int DZ>
    __device__ __forceinline__ void tap_pairs(const bf16x8 (&B)[5][2], const uint16_t* s_w) {
        constexpr int SL = (PH - DZ + 3) % 3;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const int t9 = 2 * q + kh;  // tap of this half-wavefront within the dz plane
            bf16x8 a = ld8(s_w + ((DZ * 9 + (t9 < 9 ? t9 : 8)) * 32 + j) * 8);
            if (t9 >= 9) a = bf16x8{};
            acc[0][SL] = mfma(a, B[q][0], acc[0][SL]);
            acc[1][SL] = mfma(a, B[q][1], acc[1][SL]);
        }
    }

    // Last layer: the products of input row hr of the staged plane.
    template <int PH, int HR>
    __device__ __forceinline__ void last_row(const uint16_t* slot) {
        f32x16 d = {};
#pragma unroll
        for (int dx = 0; dx < 3; ++dx)
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
                d = mfma(wl[dx][kb], ld8(slot + ((2 * wv + HR) * ZHX + j + dx) * ZCS + 16 * kb + 8 * kh), d);
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int dz = t / 3, dy = t % 3, rr = HR - dy;
            if (rr >= 0 && rr <= 1) oacc[(PH - dz + 3) % 3][rr] += d[t];
        }
    }

    // Products of the staged plane in `slot` (phase PH of the rotation).
    template <int PH>
    __device__ __forceinline__ void products(const uint16_t* slot, const uint16_t* s_w) {
        if constexpr (LAST) {
            last_row<PH, 0>(slot);
            last_row<PH, 1>(slot);
            last_row<PH, 2>(slot);
            last_row<PH, 3>(slot);
        } else if constexpr (CIN == 8) {
            bf16x8 B[5][2];
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                const int t9 = 2 * q + kh < 9 ? 2 * q + kh : 8;
                const int dy = t9 / 3, dx = t9 % 3;
#pragma unroll
                for (int rr = 0; rr < 2; ++rr) B[q][rr] = ld8(slot + ((2 * wv + rr + dy) * ZHX + j + dx) * ZCS);
            }
            tap_pairs<PH, 0>(B, s_w);
            tap_pairs<PH, 1>(B, s_w);
            tap_pairs<PH, 2>(B, s_w);
        } else {
            bf16x8 B[4][3][2];
#pragma unroll
            for (int hr = 0; hr < 4; ++hr)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                    for (int kb = 0; kb < 2; ++kb)
                        B[hr][dx][kb] = ld8(slot + ((2 * wv + hr) * ZHX + j + dx) * ZCS + 16 * kb + 8 * kh);
            tap_plane<PH, 0>(B, s_w);
            tap_plane<PH, 1>(B, s_w);
            tap_plane<PH, 2>(B, s_w);
        }
    }

    // Output plane z from accumulator slot SL, then the slot is cleared.
    template <int SL>
    __device__ __forceinline__ void emit(int z, const float (&bco)[16], const uint16_t* mask, void* out) {
        if constexpr (LAST) {
            if (z >= za && z < zb) {
#pragma unroll
                for (int rr = 0; rr < 2; ++rr) {
                    const int y = y0 + 2 * wv + rr, x = x0 + j;
                    if (y < s.ny && x < s.nx) {
                        const int64_t vox = vbase + (int64_t(z) * s.ny + y) * s.nx + x;
                        static_cast<float*>(out)[vox * 2 + kh] = oacc[SL][rr] + bco[0];
                    }
                }
            }
            oacc[SL][0] = 0.0f;
            oacc[SL][1] = 0.0f;
        } else {
            if (z >= za && z < zb) {
#pragma unroll
                for (int rr = 0; rr < 2; ++rr) {
                    const int y = y0 + 2 * wv + rr, x = x0 + j;
                    if (y < s.ny && x < s.nx) {
                        const int64_t vox = vbase + (int64_t(z) * s.ny + y) * s.nx + x;
                        const f32x16& a = acc[rr][SL];
#pragma unroll
                        for (int g = 0; g < 4; ++g) {
                            const int64_t off = vox * 32 + 8 * g + 4 * kh;
                            uint16_t h[4];
                            if constexpr (MODE == CONV_BIAS_RELU) {
#pragma unroll
                                for (int e = 0; e < 4; ++e) {
                                    const float v = a[4 * g + e] + bco[4 * g + e];
                                    h[e] = bf16_bits(v > 0.0f ? v : 0.0f);
                                }
                            } else {
                                const uint2 mk = *reinterpret_cast<const uint2*>(mask + off);
                                const uint16_t m[4] = {uint16_t(mk.x & 0xffffu), uint16_t(mk.x >> 16),
                                                       uint16_t(mk.y & 0xffffu), uint16_t(mk.y >> 16)};
#pragma unroll
                                for (int e = 0; e < 4; ++e)
                                    h[e] = bf16_bits(bf16_value(m[e]) > 0.0f ? a[4 * g + e] : 0.0f);
                            }
                            uint2 pk;
                            pk.x = uint32_t(h[0]) | (uint32_t(h[1]) << 16);
                            pk.y = uint32_t(h[2]) | (uint32_t(h[3]) << 16);
                            *reinterpret_cast<uint2*>(static_cast<uint16_t*>(out) + off) = pk;
                        }
                    }
                }
            }
            acc[0][SL] = f32x16{};
            acc[1][SL] = f32x16{};
        }
    }

    // Input plane p = za - 1 + t (phase PH = t mod 3): issue the next plane's
    // loads, take the products, emit output plane p - 1, stage the next plane.
    template <int PH>
    __device__ __forceinline__ void plane(int t, int T, uint16_t* s_in, const uint16_t* s_w, const float (&bco)[16],
                                          const uint16_t* mask, void* out, int tid) {
        const int p = za - 1 + t;
        const bool more = t + 1 < T;
        if (more) issue(p + 1, tid);
        products<PH>(s_in + (t & 1) * ZPLANE, s_w);
        emit<(PH + 1) % 3>(p - 1, bco, mask, out);
        if (more) commit(s_in + ((t + 1) & 1) * ZPLANE, tid);
        __syncthreads();
    }
};

// (32 input channels: one wavefront per SIMD, its registers hold the
// activation fragments and three accumulator pairs; 8 input channels and the
// two-channel layer: two per SIMD)
template <int CIN, int MODE>
__global__ __launch_bounds__(256) __attribute__((
    amdgpu_waves_per_eu(CIN == 32 && MODE != CONV_BIAS_F32 ? 1 : 2, CIN == 32 && MODE != CONV_BIAS_F32 ? 1 : 2))) void
k_conv_zm(const uint16_t* __restrict__ in, const uint16_t* __restrict__ w, const float* __restrict__ bias,
          const uint16_t* __restrict__ mask, void* __restrict__ out, ConvShape s, ZMarch zm, int nseg) {
    using L = ZLayout<CIN>;
    constexpr bool LAST = ZConv<CIN, MODE>::LAST;
    __shared__ __attribute__((aligned(16))) uint16_t s_w[LAST ? 8 : 27 * 32 * L::CS];
    __shared__ __attribute__((aligned(16))) uint16_t s_in[2 * L::PLANE];
    const int tid = threadIdx.x;
    ZConv<CIN, MODE> zc;
    zc.in = in;
    zc.s = s;
    zc.lane = tid & 63;
    zc.wv = tid >> 6;
    zc.j = zc.lane & 31;
    zc.kh = zc.lane >> 5;
    float bco[16];
    if constexpr (LAST) {
        // A row i = lane % 32: output channel (i / 4) % 2, tap pair t = 4 (i / 8) + i % 4
        const int i = zc.lane & 31;
        const int co = (i >> 2) & 1, t = 4 * (i >> 3) + (i & 3);
        const int dz = t / 3, dy = t % 3;
#pragma unroll
        for (int dx = 0; dx < 3; ++dx)
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) {
                const int tap = t < 9 ? dz * 9 + dy * 3 + dx : 0;
                const bf16x8 v = ld8(w + (int64_t(tap) * 32 + co) * 32 + 16 * kb + 8 * zc.kh);
                zc.wl[dx][kb] = t < 9 ? v : bf16x8{};
            }
#pragma unroll
        for (int r = 0; r < 16; ++r) bco[r] = 0.0f;
        bco[0] = bias[zc.kh];  // this half-wavefront's output channel
    } else {
        for (int c = tid; c < 27 * 32 * L::CH; c += 256) {
            const int ch = c % L::CH, row = c / L::CH;
            *reinterpret_cast<uint4*>(&s_w[row * L::CS + ch * 8]) =
                *reinterpret_cast<const uint4*>(w + int64_t(row) * CIN + ch * 8);
        }
        // bias of the output channels this lane holds, 8 (r / 4) + 4 kh + r % 4
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int co = 8 * (r >> 2) + 4 * zc.kh + (r & 3);
            bco[r] = 0.0f;
            if constexpr (MODE == CONV_BIAS_RELU) bco[r] = bias[co];
        }
    }
    for (int seg = blockIdx.x; seg < nseg; seg += gridDim.x) {
        int b = seg;
        const int bx = b % zm.tx;
        b /= zm.tx;
        const int by = b % zm.ty;
        b /= zm.ty;
        const int zs = b % zm.zsegs;
        zc.vol = b / zm.zsegs;
        zc.x0 = bx * ZX;
        zc.y0 = by * ZY;
        zc.za = zs * zm.Lz;
        zc.zb = zc.za + zm.Lz < s.nz ? zc.za + zm.Lz : s.nz;
        zc.vbase = int64_t(zc.vol) * s.nz * s.ny * s.nx;
#pragma unroll
        for (int rr = 0; rr < 2; ++rr)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                if constexpr (LAST) zc.oacc[q][rr] = 0.0f;
                else zc.acc[rr][q] = f32x16{};
            }
        // input planes za - 1 .. zb
        const int T = zc.zb - zc.za + 2;
        zc.issue(zc.za - 1, tid);
        zc.commit(s_in, tid);
        __syncthreads();
        for (int t = 0; t < T; t += 3) {
            zc.template plane<0>(t, T, s_in, s_w, bco, mask, out, tid);
            if (t + 1 >= T) break;
            zc.template plane<1>(t + 1, T, s_in, s_w, bco, mask, out, tid);
            if (t + 2 >= T) break;
            zc.template plane<2>(t + 2, T, s_in, s_w, bco, mask, out, tid);
        }
    }
}

// ---------------------------------------------------------- weight gradient

// Brick counts of a volume batch along x, y and z.
struct Bricks {
    int bx, by, bz;
};

constexpr int WX = 32, WY = 2, WZ = 2;
constexpr int WROWS_H = (WZ + 2) * (WY + 2);  // halo rows of H per brick
constexpr int WROWS_G = WZ * WY;
constexpr int SG_STRIDE = WROWS_G * WX + 8;   // per output channel (odd multiple of 16 bytes)
constexpr int SH_STRIDE = WROWS_H * WX + 8;   // per input channel
constexpr int kWgradGroups = 512;

// H transposed into x-contiguous rows, one copy per x shift dx so that every
// 8-voxel operand read is 16-byte aligned; G transposed likewise.  Each
// wavefront accumulates the taps tap = wave + 4j in registers over all the
// bricks its workgroup visits, then writes its partial sums.
template <int CG, int CHN>
__global__ __launch_bounds__(256) void k_conv_wgrad(const uint16_t* __restrict__ G, const uint16_t* __restrict__ H,
                                                   float* __restrict__ partial, ConvShape s, Bricks nbk,
                                                   int nbricks) {
    __shared__ __attribute__((aligned(16))) uint16_t s_g[32 * SG_STRIDE];
    __shared__ __attribute__((aligned(16))) uint16_t s_h[3 * 32 * SH_STRIDE];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const int i = lane & 31;
    const int kh = lane >> 5;
    // channels past CG / CHN stay zero for the whole kernel
    for (int c = tid; c < 32 * SG_STRIDE; c += 256) s_g[c] = 0;
    for (int c = tid; c < 3 * 32 * SH_STRIDE; c += 256) s_h[c] = 0;
    f32x16 acc[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) acc[j] = f32x16{};
    for (int brick = blockIdx.x; brick < nbricks; brick += gridDim.x) {
        int b = brick;
        const int bxi = b % nbk.bx;
        b /= nbk.bx;
        const int byi = b % nbk.by;
        b /= nbk.by;
        const int bzi = b % nbk.bz;
        const int vol = b / nbk.bz;
        const int x0 = bxi * WX, y0 = byi * WY, z0 = bzi * WZ;
        const int64_t vbase = int64_t(vol) * s.nz * s.ny * s.nx;
        __syncthreads();  // the previous brick's operands are consumed
        // G rows: (z, y) in the brick, x0 .. x0 + 31
        for (int c = tid; c < WROWS_G * WX * (CG / 8); c += 256) {
            const int ch = c % (CG / 8);
            int v = c / (CG / 8);
            const int xi = v % WX;
            const int row = v / WX;  // z * WY + y
            const int gx = x0 + xi, gy = y0 + row % WY, gz = z0 + row / WY;
            uint4 val = make_uint4(0u, 0u, 0u, 0u);
            if (gx < s.nx && gy < s.ny && gz < s.nz)
                val = *reinterpret_cast<const uint4*>(G + (vbase + (int64_t(gz) * s.ny + gy) * s.nx + gx) * CG +
                                                      ch * 8);
            const uint16_t* e = reinterpret_cast<const uint16_t*>(&val);
#pragma unroll
            for (int q = 0; q < 8; ++q) s_g[(ch * 8 + q) * SG_STRIDE + row * WX + xi] = e[q];
        }
        // H halo rows: (z, y) in -1 .. brick + 1, x0 - 1 .. x0 + 32, stored
        // for every dx whose window holds the voxel
        for (int c = tid; c < WROWS_H * (WX + 2) * (CHN / 8); c += 256) {
            const int ch = c % (CHN / 8);
            int v = c / (CHN / 8);
            const int hx = v % (WX + 2);
            const int row = v / (WX + 2);  // hz * (WY + 2) + hy
            const int gx = x0 - 1 + hx, gy = y0 - 1 + row % (WY + 2), gz = z0 - 1 + row / (WY + 2);
            uint4 val = make_uint4(0u, 0u, 0u, 0u);
            if (gx >= 0 && gx < s.nx && gy >= 0 && gy < s.ny && gz >= 0 && gz < s.nz)
                val = *reinterpret_cast<const uint4*>(H + (vbase + (int64_t(gz) * s.ny + gy) * s.nx + gx) * CHN +
                                                      ch * 8);
            const uint16_t* e = reinterpret_cast<const uint16_t*>(&val);
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int xi = hx - dx;
                if (xi < 0 || xi >= WX) continue;
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    s_h[(dx * 32 + ch * 8 + q) * SH_STRIDE + row * WX + xi] = e[q];
            }
        }
        __syncthreads();
        // A operands (G^T: output channel x 8 voxels) for the 4 rows x 2 x-halves
        bf16x8 ga[WROWS_G][2];
#pragma unroll
        for (int row = 0; row < WROWS_G; ++row)
#pragma unroll
            for (int xb = 0; xb < 2; ++xb) ga[row][xb] = ld8(&s_g[i * SG_STRIDE + row * WX + 16 * xb + 8 * kh]);
#pragma unroll
        for (int j = 0; j < 7; ++j) {
            const int tap = wv + 4 * j;
            if (tap >= 27) break;
            const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap - 3 * (tap / 3);
            const uint16_t* hb = &s_h[(dx * 32 + i) * SH_STRIDE + 8 * kh];
#pragma unroll
            for (int zz = 0; zz < WZ; ++zz)
#pragma unroll
                for (int yy = 0; yy < WY; ++yy) {
                    const int hrow = (zz + dz) * (WY + 2) + (yy + dy);
#pragma unroll
                    for (int xb = 0; xb < 2; ++xb)
                        acc[j] = mfma(ga[zz * WY + yy][xb], ld8(hb + hrow * WX + 16 * xb), acc[j]);
                }
        }
    }
    // partial[group][tap][co][ci]: register r is output channel co = 8 (r/4) + 4 kh + r%4, input channel i
    float* pg = partial + int64_t(blockIdx.x) * 27 * 32 * 32;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        const int tap = wv + 4 * j;
        if (tap >= 27) break;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int co = 8 * (r >> 2) + 4 * kh + (r & 3);
            pg[(tap * 32 + co) * 32 + i] = acc[j][r];
        }
    }
}

// gW = sum over groups of the partials, in a fixed order: eight interleaved
// double partial sums per element (independent loads in flight), combined
// in order.
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* __restrict__ partial, int groups, int cout,
                                                      int cin, float* __restrict__ gW) {
    const int idx = blockIdx.x * 256 + threadIdx.x;  // (co, ci, tap) in the master layout
    if (idx >= cout * cin * 27) return;
    const int tap = idx % 27;
    const int ci = (idx / 27) % cin;
    const int co = idx / (27 * cin);
    const int64_t off = (int64_t(tap) * 32 + co) * 32 + ci;
    const int64_t stride = int64_t(27) * 32 * 32;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int g = 0;
    for (; g + 8 <= groups; g += 8) {
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] += partial[(g + q) * stride + off];
    }
    for (int q = 0; g + q < groups; ++q) acc[q] += partial[(g + q) * stride + off];
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) t += acc[q];
    gW[idx] = float(t);
}

// ------------------------------------------------------ small training kernels

constexpr int kRedGroups = 1024;

__global__ __launch_bounds__(256) void k_bias_partial(const uint16_t* __restrict__ G, int cg, int64_t V,
                                                     float* __restrict__ partial) {
    __shared__ float red[8][32];
    const int co = threadIdx.x & 31;
    const int sub = threadIdx.x >> 5;  // 8 voxel lanes per channel
    float acc = 0.0f;
    if (co < cg)
        for (int64_t v = int64_t(blockIdx.x) * 8 + sub; v < V; v += int64_t(gridDim.x) * 8)
            acc += bf16_value(G[v * cg + co]);
    red[sub][co] = acc;
    __syncthreads();
    if (threadIdx.x < 32) {
        float t = 0.0f;
        for (int q = 0; q < 8; ++q) t += red[q][threadIdx.x];
        partial[blockIdx.x * 32 + threadIdx.x] = t;
    }
}

// gb[co] = sum over groups of the partials: one workgroup per channel, a
// fixed-order tree over 256 strided partial sums.
__global__ __launch_bounds__(256) void k_bias_reduce(const float* __restrict__ partial, int groups, int cout,
                                                     float* __restrict__ gb) {
    __shared__ double red[256];
    const int co = blockIdx.x;
    double acc = 0.0;
    for (int g = threadIdx.x; g < groups; g += 256) acc += partial[g * 32 + co];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0 && co < cout) gb[co] = float(red[0]);
}

__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ out, const float* __restrict__ target,
                                            int64_t V, float scale, uint16_t* __restrict__ gout,
                                            double* __restrict__ partial) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t v = int64_t(blockIdx.x) * 256 + threadIdx.x; v < V; v += int64_t(gridDim.x) * 256) {
        const float d0 = out[2 * v] - target[2 * v];
        const float d1 = out[2 * v + 1] - target[2 * v + 1];
        acc += double(d0) * d0 + double(d1) * d1;
        uint4 g = make_uint4(0u, 0u, 0u, 0u);
        g.x = uint32_t(bf16_bits(scale * d0)) | (uint32_t(bf16_bits(scale * d1)) << 16);
        reinterpret_cast<uint4*>(gout)[v] = g;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_sum_doubles(const double* __restrict__ partial, int n, double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double acc = 0.0;
    for (int g = 0; g < n; ++g) acc += partial[g];
    out[0] = acc;
}

__global__ __launch_bounds__(256) void k_grad_to_bf16(const float* __restrict__ g, int64_t V,
                                                     uint16_t* __restrict__ gout) {
    const int64_t v = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (v >= V) return;
    uint4 o = make_uint4(0u, 0u, 0u, 0u);
    o.x = uint32_t(bf16_bits(g[2 * v])) | (uint32_t(bf16_bits(g[2 * v + 1])) << 16);
    reinterpret_cast<uint4*>(gout)[v] = o;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                                             const float* __restrict__ g, int64_t n, float lr, float b1, float b2,
                                             float eps, float bc1, float bc2) {
    const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (k >= n) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    w[k] -= lr * (mk / bc1) / (sqrtf(vk / bc2) + eps);
}

__global__ __launch_bounds__(256) void k_pack_weights(const float* __restrict__ W, int cout, int cin, int cinp,
                                                     int coutp, uint16_t* __restrict__ wf, uint16_t* __restrict__ wb) {
    // wf: [27][32][cinp]; wb: [27][32][coutp]
    const int idx = blockIdx.x * 256 + threadIdx.x;
    const int nf = 27 * 32 * cinp;
    if (idx < nf) {
        const int ci = idx % cinp;
        const int co = (idx / cinp) % 32;
        const int tap = idx / (cinp * 32);
        const float val = (co < cout && ci < cin) ? W[(co * cin + ci) * 27 + tap] : 0.0f;
        wf[idx] = bf16_bits(val);
    }
    if (wb && idx < 27 * 32 * coutp) {
        const int co = idx % coutp;
        const int ci = (idx / coutp) % 32;
        const int tap = idx / (coutp * 32);
        const float val = (co < cout && ci < cin) ? W[(co * cin + ci) * 27 + (26 - tap)] : 0.0f;
        wb[idx] = bf16_bits(val);
    }
}

struct cd2 {
    double re, im;
};

__global__ __launch_bounds__(256) void k_cnn_input(const cd2* __restrict__ r, const float* __restrict__ D, float Dc,
                                                  const double* __restrict__ scale, int64_t V,
                                                  uint16_t* __restrict__ in) {
    const int64_t v = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (v >= V) return;
    const double sc = scale[0];
    const cd2 x = r[v];
    const float d = D ? D[v] : Dc;
    uint4 o = make_uint4(0u, 0u, 0u, 0u);
    o.x = uint32_t(bf16_bits(float(x.re * sc))) | (uint32_t(bf16_bits(float(x.im * sc))) << 16);
    o.y = uint32_t(bf16_bits(d));
    reinterpret_cast<uint4*>(in)[v] = o;
}

__global__ __launch_bounds__(256) void k_cnn_output(const float* __restrict__ out, const double* __restrict__ scale,
                                                   int64_t V, cd2* __restrict__ z) {
    const int64_t v = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (v >= V) return;
    const double sc = scale[0];
    z[v] = {sc * out[2 * v], sc * out[2 * v + 1]};
}

__global__ __launch_bounds__(256) void k_cnn_crop(const cd2* __restrict__ r, const cd2* __restrict__ zv,
                                                 const float* __restrict__ D, float Dc, int64_t g0, int64_t g1,
                                                 int o0, int o1, int o2, int c0, int c1, int c2, double rs, double zs,
                                                 uint16_t* __restrict__ in, float* __restrict__ target) {
    const int64_t q = int64_t(blockIdx.x) * 256 + threadIdx.x;
    const int64_t n = int64_t(c0) * c1 * c2;
    if (q >= n) return;
    const int i0 = int(q % c0), i1 = int((q / c0) % c1), i2 = int(q / (int64_t(c0) * c1));
    const int64_t p = (o0 + i0) + g0 * ((o1 + i1) + g1 * int64_t(o2 + i2));
    const cd2 x = r[p];
    const float d = D ? D[p] : Dc;
    uint4 o = make_uint4(0u, 0u, 0u, 0u);
    o.x = uint32_t(bf16_bits(float(x.re * rs))) | (uint32_t(bf16_bits(float(x.im * rs))) << 16);
    o.y = uint32_t(bf16_bits(d));
    reinterpret_cast<uint4*>(in)[q] = o;
    const cd2 t = zv[p];
    target[2 * q] = float(t.re * zs);
    target[2 * q + 1] = float(t.im * zs);
}

inline unsigned grid_for(int64_t n) { return unsigned((n + 255) / 256); }

}  // namespace

// Resident workgroups of the persistent convolution: one per CU (its LDS
// footprint allows no more), a few rounds so that uneven brick costs even out.
static int conv_groups() {
    static int cached = 0;
    if (!cached) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
            (void)hipGetLastError();
            cus = 256;
        }
        cached = 2 * cus;
    }
    return cached;
}

// Columns of 32 x 8 voxels, each split along z into as few segments as give
// every workgroup slot one (one workgroup per compute unit with 32 input
// channels, two with 8).
static void launch_conv_zm(int cin, ConvMode mode, const uint16_t* in, const uint16_t* w, const float* bias, const uint16_t* mask,
                           void* out, const ConvShape& s, hipStream_t st) {
    ZMarch zm;
    zm.tx = (s.nx + ZX - 1) / ZX;
    zm.ty = (s.ny + ZY - 1) / ZY;
    const int64_t cols = int64_t(zm.tx) * zm.ty * s.nb;
    if (cols <= 0 || s.nz <= 0) return;
    const int units = cin == 32 && mode != CONV_BIAS_F32 ? conv_groups() / 2 : conv_groups();
    int64_t zsegs = (units + cols - 1) / cols;
    const int64_t zmax = (s.nz + 3) / 4;  // at least four planes per segment
    if (zsegs > zmax) zsegs = zmax;
    if (zsegs < 1) zsegs = 1;
    zm.Lz = int((s.nz + zsegs - 1) / zsegs);
    zm.zsegs = (s.nz + zm.Lz - 1) / zm.Lz;
    const int64_t nseg = cols * zm.zsegs;
    if (nseg > 0x7fffffff) fail(MXP_ERR_UNSUPPORTED, "convolution grid too large");
    const dim3 grid(unsigned(nseg < units ? nseg : units)), block(256);
    const int ns = int(nseg);
#define MXP_ZM(C, M) hipLaunchKernelGGL((k_conv_zm<C, M>), grid, block, 0, st, in, w, bias, mask, out, s, zm, ns)
    if (cin == 32) {
        if (mode == CONV_BIAS_RELU) MXP_ZM(32, CONV_BIAS_RELU);
        else if (mode == CONV_BIAS_F32) MXP_ZM(32, CONV_BIAS_F32);
        else MXP_ZM(32, CONV_MASK);
    } else {
        if (mode == CONV_BIAS_RELU) MXP_ZM(8, CONV_BIAS_RELU);
        else if (mode == CONV_MASK) MXP_ZM(8, CONV_MASK);
        else fail(MXP_ERR_INVALID_ARG, "the two-channel output layer reads 32 channels");
    }
#undef MXP_ZM
}

void launch_conv(int cin, ConvMode mode, const uint16_t* in, const uint16_t* w, const float* bias,
                 const uint16_t* mask, void* out, const ConvShape& s, hipStream_t st) {
    if (cin != 32 && cin != 8) fail(MXP_ERR_INVALID_ARG, "convolution input channels must be 8 or 32");
    launch_conv_zm(cin, mode, in, w, bias, mask, out, s, st);
    check_launch("conv");
}

int conv_wgrad_max_groups() { return kWgradGroups; }

int launch_conv_wgrad(int cg, int ch, const uint16_t* G, const uint16_t* H, float* partial, const ConvShape& s,
                      hipStream_t st) {
    Bricks nbk{(s.nx + WX - 1) / WX, (s.ny + WY - 1) / WY, (s.nz + WZ - 1) / WZ};
    const int64_t nbr = int64_t(nbk.bx) * nbk.by * nbk.bz * s.nb;
    if (nbr <= 0) return 0;
    if (nbr > 0x7fffffff) fail(MXP_ERR_UNSUPPORTED, "weight-gradient grid too large");
    const int groups = int(nbr < kWgradGroups ? nbr : kWgradGroups);
    const dim3 grid(groups), block(256);
#define MXP_WG(A, B) hipLaunchKernelGGL((k_conv_wgrad<A, B>), grid, block, 0, st, G, H, partial, s, nbk, int(nbr))
    if (cg == 32 && ch == 32) MXP_WG(32, 32);
    else if (cg == 32 && ch == 8) MXP_WG(32, 8);
    else if (cg == 8 && ch == 32) MXP_WG(8, 32);
    else if (cg == 8 && ch == 8) MXP_WG(8, 8);
    else fail(MXP_ERR_INVALID_ARG, "weight gradient channels must be 8 or 32");
#undef MXP_WG
    check_launch("conv weight gradient");
    return groups;
}

void launch_wgrad_reduce(const float* partial, int groups, int cout, int cin, float* gW, hipStream_t st) {
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(grid_for(int64_t(cout) * cin * 27)), dim3(256), 0, st, partial, groups,
                       cout, cin, gW);
    check_launch("weight gradient reduction");
}

void launch_bias_grad(const uint16_t* G, int cg, int cout, int64_t V, float* partial, float* gb, hipStream_t st) {
    const int groups = int(V / 8 + 1 < kRedGroups ? V / 8 + 1 : kRedGroups);
    hipLaunchKernelGGL(k_bias_partial, dim3(groups), dim3(256), 0, st, G, cg, V, partial);
    hipLaunchKernelGGL(k_bias_reduce, dim3(cout), dim3(256), 0, st, partial, groups, cout, gb);
    check_launch("bias gradient");
}

void launch_mse(const float* out, const float* target, int64_t V, uint16_t* gout, double* partial, double* lsum,
                hipStream_t st) {
    const int groups = int(V / 256 + 1 < kRedGroups ? V / 256 + 1 : kRedGroups);
    const float scale = float(2.0 / (2.0 * double(V)));
    hipLaunchKernelGGL(k_mse, dim3(groups), dim3(256), 0, st, out, target, V, scale, gout, partial);
    hipLaunchKernelGGL(k_sum_doubles, dim3(1), dim3(1), 0, st, partial, groups, lsum);
    check_launch("mse");
}

void launch_grad_to_bf16(const float* g, int64_t V, uint16_t* gout, hipStream_t st) {
    hipLaunchKernelGGL(k_grad_to_bf16, dim3(grid_for(V)), dim3(256), 0, st, g, V, gout);
    check_launch("gradient cast");
}

void launch_adam(float* w, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2, float eps,
                 float bc1, float bc2, hipStream_t st) {
    hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, st, w, m, v, g, n, lr, b1, b2, eps, bc1, bc2);
    check_launch("adam");
}

void launch_pack_weights(const float* W, int cout, int cin, int cinp, int coutp, uint16_t* wf, uint16_t* wb,
                         hipStream_t st) {
    const int64_t n = 27 * 32 * int64_t(cinp > coutp ? cinp : coutp);
    hipLaunchKernelGGL(k_pack_weights, dim3(grid_for(n)), dim3(256), 0, st, W, cout, cin, cinp, coutp, wf, wb);
    check_launch("pack weights");
}

void launch_cnn_input(const void* r, const float* D, float Dc, const double* scale, int64_t V, uint16_t* in,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_cnn_input, dim3(grid_for(V)), dim3(256), 0, st, static_cast<const cd2*>(r), D, Dc, scale, V,
                       in);
    check_launch("network input");
}

void launch_cnn_output(const float* out, const double* scale, int64_t V, void* z, hipStream_t st) {
    hipLaunchKernelGGL(k_cnn_output, dim3(grid_for(V)), dim3(256), 0, st, out, scale, V, static_cast<cd2*>(z));
    check_launch("network output");
}

void launch_cnn_crop(const void* r, const void* z, const float* D, float Dc, int64_t g0, int64_t g1, int o0, int o1,
                     int o2, int c0, int c1, int c2, double rs, double zs, uint16_t* in, float* target,
                     hipStream_t st) {
    const int64_t n = int64_t(c0) * c1 * c2;
    hipLaunchKernelGGL(k_cnn_crop, dim3(grid_for(n)), dim3(256), 0, st, static_cast<const cd2*>(r),
                       static_cast<const cd2*>(z), D, Dc, g0, g1, o0, o1, o2, c0, c1, c2, rs, zs, in, target);
    check_launch("training crop");
}

}  // namespace mxp
