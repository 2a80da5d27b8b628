// Internal declarations of the MatExPre library (not part of the C ABI).
#pragma once

#include <cmath>
#include <complex>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/matexpre.h"

namespace mxp {

using cd = std::complex<double>;

// Error carried from the depths of the library to the ABI boundary, where it
// becomes an mxp_status plus a thread-local message.
struct Error : std::runtime_error {
    mxp_status status;
    Error(mxp_status s, const std::string& msg) : std::runtime_error(msg), status(s) {}
};

[[noreturn]] inline void fail(mxp_status s, const std::string& msg) { throw Error(s, msg); }

// Absorbing-layer stretch along one axis (Section 3.3, eq. pml-1d-s): the
// imaginary part sigma(x) of s(x) = 1 + i sigma(x).  Nodes x_i = i h, the low
// face has `lo` layer cells (inner edge at lo*h, delta = lo*h), the high face
// `hi` cells (inner edge at (n-1-hi)*h, delta = hi*h).
struct AxisLayer {
    int64_t n;
    int32_t lo, hi;
    double h, omega, C;
    int32_t power;
    int32_t absorber;  // MXP_ABSORB_PML, MXP_ABSORB_CAP or MXP_ABSORB_ABC
    // MXP_ABSORB_ABC: the end faces that absorb (the others are sound-hard),
    // and omega/c when c is constant (the absorbing term is then per axis), else 0
    bool abs_lo = false, abs_hi = false;
    double kc = 0.0;
    // the layer profile sigma(x) = C/(delta omega) (dist/delta)^power
    double sigma(double x) const;
    // imaginary part of the coordinate stretch (zero for the potential)
    double stretch(double x) const { return absorber == MXP_ABSORB_PML ? sigma(x) : 0.0; }
};

// Per-axis three-point coefficients of (1/s) d/dx((1/s) du/dx), or with
// MXP_ABSORB_ABC of the second difference with ghost-point end rows (weight
// 2/h^2 on the inner neighbour, none outside, and with constant c the
// absorbing term 2 i omega/(c h) of an absorbing end in gamma):
//   (L u)_i = alpha_i u_{i-1} + beta_i u_{i+1} + gamma_i u_i,
//   alpha_i = 1/(s_i s_{i-1/2} h^2), beta_i = 1/(s_i s_{i+1/2} h^2),
//   gamma_i = -(alpha_i + beta_i) + i 2 omega^2 sigma(x_i) (the last term
//   only with the absorbing potential, where every stretch is 1).
struct AxisTables {
    std::vector<cd> alpha, beta, gamma;
};
AxisTables build_axis_tables(const AxisLayer& ax);

// Validated copy of a grid description plus derived host-side facts.
struct GridInfo {
    int dim;
    int64_t n[3];
    double h, omega, pml_C;
    int32_t pml_power;
    int32_t absorber;
    int32_t layer[3][2];
    int32_t hard[3][2];  // MXP_ABSORB_ABC: sound-hard faces
    bool homogeneous;
    double c_const;
    double dmin, dmax;  // range of D = 1/c^2
    int64_t npts() const { return n[0] * n[1] * n[2]; }
    AxisLayer axis(int d) const {
        AxisLayer a{n[d], layer[d][0], layer[d][1], h, omega, pml_C, pml_power, absorber};
        if (absorber == MXP_ABSORB_ABC) {
            a.abs_lo = hard[d][0] == 0;
            a.abs_hi = hard[d][1] == 0;
            a.kc = homogeneous ? omega / c_const : 0.0;
        }
        return a;
    }
    // MXP_ABSORB_ABC with a varying c: the absorbing term 2 i omega sqrt(D_p)/h
    // is per node and the kernels add it from per-axis tables
    bool abc_per_node() const { return absorber == MXP_ABSORB_ABC && !homogeneous; }
    // condition number of the diagonal similarity that symmetrises the ghost rows
    double similarity_cond() const { return absorber == MXP_ABSORB_ABC ? std::pow(std::sqrt(2.0), dim) : 1.0; }
};

// Checks the description; fills everything except dmin/dmax when c is given.
GridInfo validate_grid(const mxp_grid_desc* desc);

// Range of D = 1/c^2 over a host array of `count` speeds; fails on c <= 0 or
// non-finite values.
void speed_range_host(const void* c, mxp_dtype dt, int64_t count, double* dmin, double* dmax);

// Field-of-values box of A_s (re_min, re_max, im_min, im_max).
void fov_box(const GridInfo& g, double shift, double box[4]);

// Substepped Chebyshev schedule for exp(i t A_s) and psi_1(i t A_s).
// forceS / forcem > 0 fix the substep count / series degree (0 = designed).
void design_schedule(const GridInfo& g, double t, double shift, mxp_precision prec,
                     mxp_schedule* out, int forceS = 0, int forcem = 0);

// Scalar psi_1(z) = (e^z - 1)/z with the power series near 0.
cd psi1_scalar(cd z);

// Scalar psi_2(z) = (e^z - 1 - z)/z^2 with the power series near 0.
cd psi2_scalar(cd z);

// exp(A) in place for a small dense n x n row-major matrix (scaling and
// squaring with the [13/13] Pade approximant).
void expm_dense(int n, std::vector<cd>& A);

// Chebyshev series of tau^2 psi_2(i tau z), tau = t / sc.S, on the segment of
// schedule sc: coef holds (re, im) pairs, m the degree.
void design_psi2_series(const mxp_schedule& sc, double t, mxp_precision prec, std::vector<double>* coef,
                        int* m);

// The learned stage's checkpoint file (host only): write the parameters and
// both Adam moments (buf: 3 * nparam floats) with the architecture header, or
// read them back after checking the architecture, length and finiteness.
void write_checkpoint(const char* path, int32_t layers, const int32_t* channels, int64_t nparam, int64_t adam_t,
                      const std::vector<float>& buf);
void read_checkpoint(const char* path, int32_t layers, const int32_t* channels, int64_t nparam, int64_t* adam_t,
                     std::vector<float>* buf);

// On-disk cache of autotuned tiles (host only): the JSON file at `path` maps
// a configuration key to (K, NX, Ly) and the measured microseconds per level.
// get: false if the path is empty, the file is missing or does not parse, or
// the key is absent.  put: adds or replaces the key and rewrites the file
// through a temporary and a rename; false (file untouched) if the path is
// empty, the file exists but does not parse, or writing fails.  Calls within
// a process are serialised.
bool tune_cache_get(const char* path, const std::string& key, int v[3], double* us);
bool tune_cache_put(const char* path, const std::string& key, const int v[3], double us);

}  // namespace mxp
