// Host-side problem set-up: absorbing-layer tables (coordinate stretch, or the
// complex absorbing potential of Section 2.1), field-of-values bounds, the
// design of the substepped Chebyshev schedule for exp(i t A_s), psi_1(i t A_s)
// and psi_2(i t A_s), and a small dense matrix exponential for the Arnoldi
// route.  Nothing here touches the GPU.
//
// Matrix-function evaluation scheme (the library's own choice; the paper uses
// a restarted Krylov method for the same actions, Section 4 introduction):
//   exp(i t A_s) = (exp(i tau A_s))^S,  tau = t/S,
//   exp(i tau z) ~ sum_{k<=m} c_k T_k((z - centre)/half_width),
// a Chebyshev expansion on a horizontal segment.  With W(A_s) the field of
// values, Crouzeix--Palencia gives ||f(A) - p(A)|| <= (1+sqrt 2) max_{W(A)}|f-p|,
// and W(A_s) lies in a rectangle computed exactly from per-axis Hermitian and
// skew-Hermitian parts (A_s is a Kronecker sum of axis operators plus a
// diagonal).  The design picks (S, segment, m) of least total cost S*m whose
// truncation bound S*(1+sqrt 2)*max_box|f-p| meets the tolerance, subject to
// a cap on the rounding amplification max_box sum_k |c_k T_k|.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

#include "mxp_internal.h"

namespace mxp {

double AxisLayer::sigma(double x) const {
    if (lo > 0) {
        const double xa = lo * h;
        if (x < xa) {
            const double delta = lo * h;
            return C / (delta * omega) * std::pow((xa - x) / delta, power);
        }
    }
    if (hi > 0) {
        const double xb = (n - 1 - hi) * h;
        if (x > xb) {
            const double delta = hi * h;
            return C / (delta * omega) * std::pow((x - xb) / delta, power);
        }
    }
    return 0.0;
}

AxisTables build_axis_tables(const AxisLayer& ax) {
    AxisTables t;
    t.alpha.resize(ax.n);
    t.beta.resize(ax.n);
    t.gamma.resize(ax.n);
    const double h2 = ax.h * ax.h;
    if (ax.absorber == MXP_ABSORB_ABC) {
        // ghost-point end rows (Section 4.3.4): u_ghost = u_inner + 2 h q u_end
        // with q = i omega/c (absorbing) or 0 (sound-hard)
        for (int64_t i = 0; i < ax.n; ++i) {
            t.alpha[i] = i == 0 ? 0.0 : (i == ax.n - 1 ? 2.0 : 1.0) / h2;
            t.beta[i] = i == ax.n - 1 ? 0.0 : (i == 0 ? 2.0 : 1.0) / h2;
            t.gamma[i] = -2.0 / h2;
        }
        if (ax.abs_lo) t.gamma[0] += cd(0.0, 2.0 * ax.kc / ax.h);
        if (ax.abs_hi) t.gamma[ax.n - 1] += cd(0.0, 2.0 * ax.kc / ax.h);
        return t;
    }
    for (int64_t i = 0; i < ax.n; ++i) {
        const double x = i * ax.h;
        const cd s0(1.0, ax.stretch(x));
        const cd sl(1.0, ax.stretch(x - 0.5 * ax.h));
        const cd sr(1.0, ax.stretch(x + 0.5 * ax.h));
        t.alpha[i] = 1.0 / (s0 * sl * h2);
        t.beta[i] = 1.0 / (s0 * sr * h2);
        t.gamma[i] = -(t.alpha[i] + t.beta[i]);
        if (ax.absorber == MXP_ABSORB_CAP) t.gamma[i] += cd(0.0, 2.0 * ax.omega * ax.omega * ax.sigma(x));
    }
    return t;
}

GridInfo validate_grid(const mxp_grid_desc* d) {
    if (!d) fail(MXP_ERR_INVALID_ARG, "grid description is NULL");
    GridInfo g{};
    if (d->dim != 2 && d->dim != 3) fail(MXP_ERR_INVALID_ARG, "dim must be 2 or 3");
    g.dim = d->dim;
    for (int a = 0; a < 3; ++a) g.n[a] = d->n[a];
    if (g.dim == 2) g.n[2] = 1;
    for (int a = 0; a < g.dim; ++a) {
        if (g.n[a] < 3) fail(MXP_ERR_INVALID_ARG, "every axis needs at least 3 nodes");
        if (g.n[a] > (int64_t(1) << 24)) fail(MXP_ERR_INVALID_ARG, "axis too long");
    }
    if (g.dim == 3 && g.n[2] < 3) fail(MXP_ERR_INVALID_ARG, "every axis needs at least 3 nodes");
    // launch-grid limits of the stencil sweep (y in blocks of 4 rows, z one per block)
    if (g.n[1] > 4 * 65535 || g.n[2] > 65535) fail(MXP_ERR_INVALID_ARG, "axis too long for the launch grid");
    if (!(d->h > 0) || !std::isfinite(d->h)) fail(MXP_ERR_INVALID_ARG, "h must be positive and finite");
    if (!(d->omega > 0) || !std::isfinite(d->omega))
        fail(MXP_ERR_INVALID_ARG, "omega must be positive and finite");
    if (!(d->pml_C >= 0) || !std::isfinite(d->pml_C)) fail(MXP_ERR_INVALID_ARG, "pml_C must be >= 0");
    if (d->pml_power < 1 || d->pml_power > 8) fail(MXP_ERR_INVALID_ARG, "pml_power must be in 1..8");
    if (d->absorber != MXP_ABSORB_PML && d->absorber != MXP_ABSORB_CAP && d->absorber != MXP_ABSORB_ABC)
        fail(MXP_ERR_INVALID_ARG, "absorber must be MXP_ABSORB_PML, MXP_ABSORB_CAP or MXP_ABSORB_ABC");
    g.h = d->h;
    g.omega = d->omega;
    g.pml_C = d->pml_C;
    g.pml_power = d->pml_power;
    g.absorber = d->absorber;
    for (int a = 0; a < 3; ++a) {
        for (int s = 0; s < 2; ++s) {
            int32_t L = (a < g.dim) ? d->layer[a][s] : 0;
            if (L < 0 || (a < g.dim && 2 * int64_t(L) >= g.n[a]))
                fail(MXP_ERR_INVALID_ARG, "layer widths must satisfy 0 <= layer < n/2");
            if (g.absorber == MXP_ABSORB_ABC && L != 0)
                fail(MXP_ERR_INVALID_ARG, "MXP_ABSORB_ABC takes no layer: every layer width must be 0");
            g.layer[a][s] = L;
            g.hard[a][s] = (g.absorber == MXP_ABSORB_ABC && a < g.dim && d->hard[a][s] != 0) ? 1 : 0;
        }
    }
    const double npts = double(g.n[0]) * double(g.n[1]) * double(g.n[2]);
    if (npts > 4.0e9) fail(MXP_ERR_INVALID_ARG, "grid too large");
    if (d->c == nullptr) {
        if (!(d->c_const > 0) || !std::isfinite(d->c_const))
            fail(MXP_ERR_INVALID_ARG, "c_const must be positive and finite");
        g.homogeneous = true;
        g.c_const = d->c_const;
        g.dmin = g.dmax = 1.0 / (d->c_const * d->c_const);
    } else {
        if (d->c_dtype != MXP_F32 && d->c_dtype != MXP_F64)
            fail(MXP_ERR_INVALID_ARG, "c_dtype must be MXP_F32 or MXP_F64");
        g.homogeneous = false;
        g.c_const = 0.0;
        g.dmin = g.dmax = 0.0;
    }
    return g;
}

void speed_range_host(const void* c, mxp_dtype dt, int64_t count, double* dmin, double* dmax) {
    double lo = std::numeric_limits<double>::infinity(), hi = 0.0;
    for (int64_t i = 0; i < count; ++i) {
        const double v = (dt == MXP_F32) ? double(static_cast<const float*>(c)[i])
                                         : static_cast<const double*>(c)[i];
        if (!(v > 0) || !std::isfinite(v))
            fail(MXP_ERR_INVALID_ARG, "wave speed must be positive and finite at every node");
        const double dd = 1.0 / (v * v);
        lo = std::min(lo, dd);
        hi = std::max(hi, dd);
    }
    *dmin = lo;
    *dmax = hi;
}

// Extreme eigenvalues of a Hermitian tridiagonal matrix with real diagonal a
// and off-diagonal moduli e (a diagonal unitary similarity removes the phases),
// by Sturm-sequence bisection.
static int sturm_count(const std::vector<double>& a, const std::vector<double>& e2, double x) {
    int cnt = 0;
    double q = a[0] - x;
    if (q < 0) ++cnt;
    for (size_t i = 1; i < a.size(); ++i) {
        if (q == 0.0) q = 1e-300;
        q = (a[i] - x) - e2[i - 1] / q;
        if (q < 0) ++cnt;
    }
    return cnt;
}

static void herm_tridiag_extremes(const std::vector<double>& a, const std::vector<double>& e,
                                  double* lmin, double* lmax) {
    const size_t n = a.size();
    std::vector<double> e2(e.size());
    double lo = std::numeric_limits<double>::infinity(), hi = -lo;
    for (size_t i = 0; i < n; ++i) {
        double r = 0;
        if (i > 0) r += e[i - 1];
        if (i + 1 < n) r += e[i];
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    for (size_t i = 0; i < e.size(); ++i) e2[i] = e[i] * e[i];
    const double span = std::max(hi - lo, 1e-300);
    lo -= 1e-12 * span;
    hi += 1e-12 * span;
    // smallest: largest x with count(x) == 0
    double l = lo, r = hi;
    for (int it = 0; it < 200 && r - l > 1e-15 * span; ++it) {
        const double mid = 0.5 * (l + r);
        if (sturm_count(a, e2, mid) >= 1) r = mid; else l = mid;
    }
    *lmin = l;
    l = lo;
    r = hi;
    for (int it = 0; it < 200 && r - l > 1e-15 * span; ++it) {
        const double mid = 0.5 * (l + r);
        if (sturm_count(a, e2, mid) >= int(n)) r = mid; else l = mid;
    }
    *lmax = r;
}

void fov_box(const GridInfo& g, double shift, double box[4]) {
    // With ghost-point end rows (MXP_ABSORB_ABC) the box bounds the field of
    // values of W^{1/2} A_s W^{-1/2}, w = 1/2 at each axis' end nodes, which
    // makes the second difference symmetric; the schedule's error bound
    // carries the similarity's condition number.  The absorbing term
    // 2 i omega sqrt(D_p)/h of a varying c lies between its values at
    // D_min and D_max.
    double re0 = 0, re1 = 0, im0 = 0, im1 = 0;
    for (int d = 0; d < g.dim; ++d) {
        const AxisLayer ax = g.axis(d);
        const AxisTables t = build_axis_tables(ax);
        const size_t n = t.gamma.size();
        const bool ghost = g.absorber == MXP_ABSORB_ABC;
        std::vector<double> ha(n), ka(n), kb(n), he(n - 1), ke(n - 1);
        for (size_t i = 0; i < n; ++i) {
            ha[i] = t.gamma[i].real();
            ka[i] = kb[i] = t.gamma[i].imag();
        }
        if (g.abc_per_node()) {
            const double a = 2.0 * g.omega / g.h;
            if (ax.abs_lo) {
                ka[0] += a * std::sqrt(g.dmin);
                kb[0] += a * std::sqrt(g.dmax);
            }
            if (ax.abs_hi) {
                ka[n - 1] += a * std::sqrt(g.dmin);
                kb[n - 1] += a * std::sqrt(g.dmax);
            }
        }
        auto w = [&](size_t i) { return ghost && (i == 0 || i == n - 1) ? 0.5 : 1.0; };
        for (size_t i = 0; i + 1 < n; ++i) {
            // entry (i, i+1) is beta_i, entry (i+1, i) is alpha_{i+1}
            const double r = std::sqrt(w(i) / w(i + 1));
            const cd up = t.beta[i] * r, dn = t.alpha[i + 1] / r;
            he[i] = std::abs(0.5 * (up + std::conj(dn)));
            ke[i] = std::abs((up - std::conj(dn)) / cd(0.0, 2.0));
        }
        double a0, a1, b0, b1, c0, c1;
        herm_tridiag_extremes(ha, he, &a0, &a1);
        herm_tridiag_extremes(ka, ke, &b0, &b1);
        herm_tridiag_extremes(kb, ke, &c0, &c1);
        re0 += a0;
        re1 += a1;
        im0 += std::min(b0, c0);
        im1 += std::max(b1, c1);
    }
    const double w2 = g.omega * g.omega;
    box[0] = re0 + w2 * g.dmin;
    box[1] = re1 + w2 * g.dmax;
    box[2] = im0 + w2 * shift * g.dmin;
    box[3] = im1 + w2 * shift * g.dmax;
}

cd psi2_scalar(cd z) {
    if (std::abs(z) < 1.0) {
        cd sum = 0.0, term = 0.5;
        for (int k = 1; k < 40; ++k) {
            sum += term;
            term *= z / double(k + 2);
            if (std::abs(term) < 1e-19 * std::abs(sum)) break;
        }
        return sum;
    }
    return (std::exp(z) - 1.0 - z) / (z * z);
}

cd psi1_scalar(cd z) {
    if (std::abs(z) < 0.5) {
        cd sum = 0.0, term = 1.0;
        for (int k = 1; k < 40; ++k) {
            sum += term;
            term *= z / double(k + 1);
            if (std::abs(term) < 1e-19 * std::abs(sum)) break;
        }
        return sum;
    }
    return (std::exp(z) - 1.0) / z;
}

// J_k(a), k = 0..kmax, real a >= 0, by Miller's backward recurrence normalised
// with J_0 + 2 sum J_{2k} = 1.
static void bessel_j(double a, int kmax, std::vector<double>& J) {
    J.assign(kmax + 1, 0.0);
    if (a == 0.0) {
        J[0] = 1.0;
        return;
    }
    int start = std::max(kmax, int(a)) + 40 + int(std::sqrt(40.0 * std::max(a, 1.0)));
    if (start % 2) ++start;
    double jp1 = 0.0, j = 1e-300, norm = 0.0;
    std::vector<double> tmp(start + 1, 0.0);
    for (int k = start; k >= 0; --k) {
        tmp[k] = j;
        if (k % 2 == 0) norm += (k == 0 ? 1.0 : 2.0) * j;
        const double jm1 = (k > 0) ? (2.0 * k / a) * j - jp1 : 0.0;
        jp1 = j;
        j = jm1;
        if (std::abs(j) > 1e250) {  // rescale to avoid overflow
            for (int q = k; q <= start; ++q) tmp[q] *= 1e-250;
            jp1 *= 1e-250;
            j *= 1e-250;
            norm *= 1e-250;
        }
    }
    for (int k = 0; k <= kmax; ++k) J[k] = tmp[k] / norm;
}

namespace {

struct Boundary {
    std::vector<cd> z;
};

Boundary box_boundary(const double box[4]) {
    Boundary b;
    const int nh = 160, nv = 24;
    for (int i = 0; i <= nh; ++i) {
        const double x = box[0] + (box[1] - box[0]) * i / nh;
        b.z.emplace_back(x, box[2]);
        b.z.emplace_back(x, box[3]);
    }
    for (int i = 1; i < nv; ++i) {
        const double y = box[2] + (box[3] - box[2]) * i / nv;
        b.z.emplace_back(box[0], y);
        b.z.emplace_back(box[1], y);
    }
    return b;
}

// Smallest degree m (>= 3) of the series `coef` on segment (c0, hw) whose error
// against f on the boundary points meets `err_tol` and whose amplification
// stays <= amp_max; returns -1 if none below `m_cap`.
int min_degree(const std::vector<cd>& coef, cd c0, double hw, const Boundary& bd,
               const std::vector<cd>& fval, double err_tol, double amp_max, int m_cap,
               double* err_out, double* amp_out, int exact_m = 0) {
    // Long double keeps the evaluation noise (growing like max|T_k| on the box)
    // far below the tolerances being tested.
    using ld = long double;
    using cl = std::complex<ld>;
    const size_t np = bd.z.size();
    std::vector<cl> xi(np), t0(np), t1(np), acc(np), fv(np);
    std::vector<ld> amp(np);
    for (size_t q = 0; q < np; ++q) {
        const cd x = (bd.z[q] - c0) / hw;
        xi[q] = cl(x.real(), x.imag());
        fv[q] = cl(fval[q].real(), fval[q].imag());
        const cl c0l(coef[0].real(), coef[0].imag()), c1l(coef[1].real(), coef[1].imag());
        t0[q] = 1.0L;
        t1[q] = xi[q];
        acc[q] = c0l + c1l * xi[q];
        amp[q] = std::max(std::abs(c0l), std::abs(c1l * xi[q]));
    }
    for (int k = 2; k <= m_cap && k < int(coef.size()); ++k) {
        const cl ck(coef[k].real(), coef[k].imag());
        ld err = 0.0L, am = 0.0L;
        for (size_t q = 0; q < np; ++q) {
            const cl t2 = 2.0L * xi[q] * t1[q] - t0[q];
            t0[q] = t1[q];
            t1[q] = t2;
            const cl term = ck * t2;
            acc[q] += term;
            amp[q] = std::max(amp[q], std::abs(term));
            err = std::max(err, std::abs(acc[q] - fv[q]));
            am = std::max(am, amp[q]);
        }
        if ((exact_m > 0 && k == exact_m) ||
            (exact_m == 0 && k >= 3 && err <= err_tol && am <= amp_max)) {
            *err_out = double(err);
            *amp_out = double(am);
            return k;
        }
    }
    return -1;
}

// Gauss--Legendre nodes and weights on [-1, 1] (Newton on P_n).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            const double dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::abs(dz) < 1e-16) {
                w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
                break;
            }
            w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
        }
        x[i] = z;
    }
}

// Chebyshev coefficients on the segment c0 + hw*[-1, 1] of
//   q(z) = tau psi_1(i tau z) = int_0^tau exp(i sigma z) d sigma,
// from the Jacobi--Anger expansion of the integrand:
//   q_k = (2 - delta_k0) i^k int_0^tau exp(i sigma c0) J_k(sigma hw) d sigma,
// integrated by composite Gauss--Legendre.  Every q_k keeps its relative
// accuracy, so the super-exponential decay of the series survives.
// With `second` set, the integrand carries the weight (tau - sigma), giving
//   tau^2 psi_2(i tau z) = int_0^tau (tau - sigma) exp(i sigma z) d sigma.
std::vector<cd> psi1_coefficients(cd c0, double hw, double tau, int kmax, bool second = false) {
    std::vector<cd> q(kmax + 1, cd(0.0, 0.0));
    std::vector<double> gx, gw, J;
    gauss_legendre(32, gx, gw);
    const double osc = tau * (std::abs(c0) + hw);
    const int panels = std::max(4, int(osc / 4.0) + 1);
    for (int pnl = 0; pnl < panels; ++pnl) {
        const double a = tau * pnl / panels, b = tau * (pnl + 1) / panels;
        for (size_t j = 0; j < gx.size(); ++j) {
            const double sig = 0.5 * (b - a) * gx[j] + 0.5 * (a + b);
            const double wt = 0.5 * (b - a) * gw[j] * (second ? tau - sig : 1.0);
            bessel_j(sig * hw, kmax, J);
            const cd e = std::exp(cd(0.0, sig) * c0) * wt;
            for (int k = 0; k <= kmax; ++k) q[k] += e * J[k];
        }
    }
    cd ik = 1.0;
    for (int k = 0; k <= kmax; ++k) {
        q[k] *= (k == 0 ? 1.0 : 2.0) * ik;
        ik *= cd(0.0, 1.0);
    }
    return q;
}

}  // namespace

void design_schedule(const GridInfo& g, double t, double shift, mxp_precision prec,
                     mxp_schedule* out, int forceS, int forcem) {
    if (forceS < 0 || forceS > 4096 || forcem < 0 || forcem > 500 || (forcem > 0 && forcem < 3))
        fail(MXP_ERR_INVALID_ARG, "forced schedule out of range (S <= 4096, 3 <= m <= 500)");
    if (!(t > 0) || !std::isfinite(t)) fail(MXP_ERR_INVALID_ARG, "t must be positive and finite");
    if (!(shift >= 0) || !std::isfinite(shift)) fail(MXP_ERR_INVALID_ARG, "shift must be >= 0");
    std::memset(out, 0, sizeof(*out));
    double box[4];
    fov_box(g, shift, box);
    const bool fp64 = (prec == MXP_PREC_FP64);
    // Rounding errors of the Clenshaw recurrence grow like the Chebyshev
    // polynomials of the second kind at the operator's eigenvalues, which is
    // fast when the box is tall against the segment.  Replayed in complex
    // float on the CPU, the absorbing potential's boxes gave errors <= 4e-6 up
    // to height/width 1.03, 1e-4..1e-3 at 1.5 and no digits at 2.0; layer
    // boxes stay below 0.6.  Complex-float stepping is refused beyond 1.25.
    const double aspect = (box[3] - box[2]) / std::max(box[1] - box[0], 1e-300);
    if (!fp64 && aspect > 1.25)
        fail(MXP_ERR_UNSUPPORTED,
             "complex-float stepping is unstable for this operator (field-of-values box taller than 1.25 "
             "times its width, e.g. a strong absorbing potential in a thin layer); use MXP_PREC_FP64");
    const double tol = fp64 ? 1e-12 : 1e-6;     // truncation bound of one action
    const double amp_max = fp64 ? 1e3 : 8.0;    // rounding amplification cap
    // Crouzeix-Palencia, times the similarity's condition number with ghost rows
    const double crouzeix = (1.0 + std::sqrt(2.0)) * g.similarity_cond();
    const int m_cap = 500;
    const Boundary bd = box_boundary(box);
    const double width = std::max(box[1] - box[0], 1e-300);
    const double fis[2] = {0.5, 0.4};
    const double scs[3] = {1.1, 1.2, 1.3};

    long best_cost = std::numeric_limits<long>::max();
    int bS = 0, bm = 0;
    double bfi = 0.5, bsc = 1.2, berr = 0, bamp = 0;
    std::vector<cd> fval(bd.z.size());
    std::vector<double> J;
    const int S_lo = forceS > 0 ? forceS : 1;
    const int S_hi = forceS > 0 ? forceS : 256;
    for (int S = S_lo; S <= S_hi; ++S) {
        if (forceS == 0 && long(S) * 3 >= best_cost) break;
        const double tau = t / S;
        for (size_t q = 0; q < bd.z.size(); ++q) fval[q] = std::exp(cd(0.0, tau) * bd.z[q]);
        for (double fi : fis) {
            for (double sc : scs) {
                const cd c0(0.5 * (box[0] + box[1]), box[2] + fi * (box[3] - box[2]));
                const double hw = sc * 0.5 * width;
                const double a = tau * hw;
                const int mlim = forcem > 0 ? forcem
                                            : int(std::min<long>(m_cap, (best_cost - 1) / S));
                if (mlim < 3) continue;
                bessel_j(a, mlim, J);
                std::vector<cd> coef(mlim + 1);
                const cd pre = std::exp(cd(0.0, tau) * c0);
                cd ik = 1.0;
                for (int k = 0; k <= mlim; ++k) {
                    coef[k] = pre * (k == 0 ? 1.0 : 2.0) * ik * J[k];
                    ik *= cd(0.0, 1.0);
                }
                double err, amp;
                // a forced degree accepts any error: the bound is only reported
                const int m = min_degree(coef, c0, hw, bd, fval,
                                         forcem > 0 ? 1e300 : tol / (crouzeix * S),
                                         forcem > 0 ? 1e300 : amp_max, mlim, &err, &amp,
                                         forcem);
                if (m > 0 && long(S) * m < best_cost) {
                    best_cost = long(S) * m;
                    bS = S;
                    bm = m;
                    bfi = fi;
                    bsc = sc;
                    berr = err;
                    bamp = amp;
                }
            }
        }
    }
    if (bS == 0) fail(MXP_ERR_UNSUPPORTED, "no Chebyshev schedule within 500 terms per substep");

    const double tau = t / bS;
    const cd c0(0.5 * (box[0] + box[1]), box[2] + bfi * (box[3] - box[2]));
    const double hw = bsc * 0.5 * width;
    // exp series from the closed form: exp(i a x) = sum (2 - delta_k0) i^k J_k(a) T_k(x)
    bessel_j(tau * hw, bm, J);
    const cd pre = std::exp(cd(0.0, tau) * c0);
    cd ik = 1.0;
    for (int k = 0; k <= bm; ++k) {
        const cd ck = pre * (k == 0 ? 1.0 : 2.0) * ik * J[k];
        out->coef[2 * k] = ck.real();
        out->coef[2 * k + 1] = ck.imag();
        ik *= cd(0.0, 1.0);
    }
    // psi_1 series: q(z) = tau psi_1(i tau z); degree chosen so that
    // its error on the box is below tol*tau/(1+sqrt 2).
    const int kmax = std::min(511, bm + 60);
    auto g_fun = [tau](cd z) { return tau * psi1_scalar(cd(0.0, tau) * z); };
    std::vector<cd> qc = psi1_coefficients(c0, hw, tau, kmax);
    for (size_t q = 0; q < bd.z.size(); ++q) fval[q] = g_fun(bd.z[q]);
    double qerr = 0, qamp = 0;
    int mq = min_degree(qc, c0, hw, bd, fval, tol * tau / crouzeix, amp_max * tau, kmax,
                        &qerr, &qamp);
    if (mq < 0) fail(MXP_ERR_UNSUPPORTED, "no psi_1 series within the term limit");
    for (int k = 0; k <= mq; ++k) {
        out->coef_psi[2 * k] = qc[k].real();
        out->coef_psi[2 * k + 1] = qc[k].imag();
    }
    out->S = bS;
    out->m = bm;
    out->m_psi = mq;
    out->centre_re = c0.real();
    out->centre_im = c0.imag();
    out->half_width = hw;
    for (int i = 0; i < 4; ++i) out->box[i] = box[i];
    out->trunc_bound = crouzeix * bS * berr;
    out->similarity_cond = g.similarity_cond();
    out->amplification = bamp;
}

namespace {

// C = A B, n x n row-major complex.  The products are written out in real
// arithmetic: std::complex multiplication keeps the full IEEE inf/NaN
// treatment, several times slower, and nothing here is infinite.
void matmul(int n, const std::vector<cd>& A, const std::vector<cd>& B, std::vector<cd>& C) {
    C.assign(size_t(n) * n, cd(0.0, 0.0));
    for (int i = 0; i < n; ++i) {
        double* c = reinterpret_cast<double*>(&C[size_t(i) * n]);
        for (int k = 0; k < n; ++k) {
            const double ar = A[size_t(i) * n + k].real(), ai = A[size_t(i) * n + k].imag();
            if (ar == 0.0 && ai == 0.0) continue;
            const double* b = reinterpret_cast<const double*>(&B[size_t(k) * n]);
            for (int j = 0; j < n; ++j) {
                const double br = b[2 * j], bi = b[2 * j + 1];
                c[2 * j] += ar * br - ai * bi;
                c[2 * j + 1] += ar * bi + ai * br;
            }
        }
    }
}

// X = D^{-1} N by Gaussian elimination with partial pivoting (N overwritten).
void solve_in_place(int n, std::vector<cd> D, std::vector<cd>& N) {
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::abs(D[size_t(r) * n + c]) > std::abs(D[size_t(piv) * n + c])) piv = r;
        if (D[size_t(piv) * n + c] == cd(0.0, 0.0)) fail(MXP_ERR_BREAKDOWN, "singular Pade denominator");
        if (piv != c)
            for (int j = 0; j < n; ++j) {
                std::swap(D[size_t(piv) * n + j], D[size_t(c) * n + j]);
                std::swap(N[size_t(piv) * n + j], N[size_t(c) * n + j]);
            }
        const cd inv = 1.0 / D[size_t(c) * n + c];
        for (int r = c + 1; r < n; ++r) {
            const cd f = D[size_t(r) * n + c] * inv;
            if (f == cd(0.0, 0.0)) continue;
            for (int j = c; j < n; ++j) D[size_t(r) * n + j] -= f * D[size_t(c) * n + j];
            for (int j = 0; j < n; ++j) N[size_t(r) * n + j] -= f * N[size_t(c) * n + j];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        const cd inv = 1.0 / D[size_t(c) * n + c];
        for (int j = 0; j < n; ++j) {
            cd v = N[size_t(c) * n + j];
            for (int k = c + 1; k < n; ++k) v -= D[size_t(c) * n + k] * N[size_t(k) * n + j];
            N[size_t(c) * n + j] = v * inv;
        }
    }
}

}  // namespace

// exp(A) of a small dense matrix by scaling and squaring with the diagonal
// [13/13] Pade approximant (Higham, SIAM J. Matrix Anal. Appl. 26, 2005):
// A is scaled by 2^-s so that its 1-norm is at most 5.37, and the
// approximant's coefficients are (26-j)! 13! / (26! j! (13-j)!).
void expm_dense(int n, std::vector<cd>& A) {
    double norm1 = 0.0;
    for (int j = 0; j < n; ++j) {
        double col = 0.0;
        for (int i = 0; i < n; ++i) col += std::abs(A[size_t(i) * n + j]);
        norm1 = std::max(norm1, col);
    }
    if (!std::isfinite(norm1)) fail(MXP_ERR_NONFINITE, "non-finite matrix in expm");
    const int s = norm1 > 5.37 ? int(std::ceil(std::log2(norm1 / 5.37))) : 0;
    const double scale = std::ldexp(1.0, -s);
    for (cd& a : A) a *= scale;
    double c[14];
    c[0] = 1.0;
    for (int j = 1; j <= 13; ++j) c[j] = c[j - 1] * double(13 - j + 1) / (double(j) * double(26 - j + 1));
    const size_t nn = size_t(n) * n;
    std::vector<cd> I(nn, cd(0.0, 0.0)), B2, B4, B6, T, U, V, W;
    for (int i = 0; i < n; ++i) I[size_t(i) * n + i] = 1.0;
    matmul(n, A, A, B2);
    matmul(n, B2, B2, B4);
    matmul(n, B2, B4, B6);
    // U = A [B6 (c13 B6 + c11 B4 + c9 B2) + c7 B6 + c5 B4 + c3 B2 + c1 I]
    T.assign(nn, 0.0);
    for (size_t q = 0; q < nn; ++q) T[q] = c[13] * B6[q] + c[11] * B4[q] + c[9] * B2[q];
    matmul(n, B6, T, W);
    for (size_t q = 0; q < nn; ++q) W[q] += c[7] * B6[q] + c[5] * B4[q] + c[3] * B2[q] + c[1] * I[q];
    matmul(n, A, W, U);
    // V = B6 (c12 B6 + c10 B4 + c8 B2) + c6 B6 + c4 B4 + c2 B2 + c0 I
    for (size_t q = 0; q < nn; ++q) T[q] = c[12] * B6[q] + c[10] * B4[q] + c[8] * B2[q];
    matmul(n, B6, T, V);
    for (size_t q = 0; q < nn; ++q) V[q] += c[6] * B6[q] + c[4] * B4[q] + c[2] * B2[q] + c[0] * I[q];
    std::vector<cd> Nm(nn), Dm(nn);
    for (size_t q = 0; q < nn; ++q) {
        Nm[q] = V[q] + U[q];
        Dm[q] = V[q] - U[q];
    }
    solve_in_place(n, Dm, Nm);
    for (int k = 0; k < s; ++k) {
        matmul(n, Nm, Nm, T);
        Nm.swap(T);
    }
    A.swap(Nm);
}

void design_psi2_series(const mxp_schedule& sc, double t, mxp_precision prec, std::vector<double>* coef,
                        int* m) {
    const bool fp64 = (prec == MXP_PREC_FP64);
    const double tol = fp64 ? 1e-12 : 1e-6;
    const double amp_max = fp64 ? 1e3 : 8.0;
    const double crouzeix = (1.0 + std::sqrt(2.0)) * (sc.similarity_cond > 1.0 ? sc.similarity_cond : 1.0);
    const double tau = t / sc.S;
    const cd c0(sc.centre_re, sc.centre_im);
    const double hw = sc.half_width;
    const Boundary bd = box_boundary(sc.box);
    const int kmax = std::min(511, sc.m + 60);
    const std::vector<cd> qc = psi1_coefficients(c0, hw, tau, kmax, true);
    std::vector<cd> fval(bd.z.size());
    for (size_t q = 0; q < bd.z.size(); ++q) fval[q] = tau * tau * psi2_scalar(cd(0.0, tau) * bd.z[q]);
    double err = 0, amp = 0;
    // the series enters the action once, scaled by S / t^2: an error below
    // tol tau^2 / (1 + sqrt 2) adds at most tol / ((1 + sqrt 2) S) to psi_2
    const int mq = min_degree(qc, c0, hw, bd, fval, tol * tau * tau / crouzeix, amp_max * tau * tau, kmax,
                              &err, &amp);
    if (mq < 0) fail(MXP_ERR_UNSUPPORTED, "no psi_2 series within the term limit");
    coef->assign(2 * size_t(mq + 1), 0.0);
    for (int k = 0; k <= mq; ++k) {
        (*coef)[2 * k] = qc[k].real();
        (*coef)[2 * k + 1] = qc[k].imag();
    }
    *m = mq;
}

}  // namespace mxp
