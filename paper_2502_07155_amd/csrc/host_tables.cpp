// Host-side FP64 tables: window transforms (deconvolution factors), default beta,
// twiddle factors and FFT factorisations.
#include <cmath>
#include <cstdint>
#include <vector>

#include "blnfft_internal.h"

namespace bl {

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

// sin(pi t) with the argument reduced exactly to |r| <= 1/2.
double sin_pi(double t) {
    double n = std::nearbyint(t);
    double r = t - n;
    double s = std::sin(kPi * r);
    return (std::fmod(std::fabs(n), 2.0) == 0.0) ? s : -s;
}

double cos_pi(double t) {
    double n = std::nearbyint(t);
    double r = t - n;
    double c = std::cos(kPi * r);
    return (std::fmod(std::fabs(n), 2.0) == 0.0) ? c : -c;
}

// Modified Bessel function I0 by its power series sum (x/2)^{2k} / (k!)^2; every term
// is positive, so the sum is accurate for the arguments used here (|x| < 100).
double bessel_i0(double x) {
    double q = 0.25 * x * x, term = 1.0, sum = 1.0;
    for (int k = 1; k < 500; ++k) {
        term *= q / (double(k) * double(k));
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return sum;
}

// Window in grid units (t = L u) on |t| <= m, given e = m - |t| >= 0 computed without
// cancellation.  Returns phi_g(t).
double window_g(bl_window win, int m, double beta, double t_abs, double e) {
    // 1 - (t/m)^2 = (m - |t|)(m + |t|) / m^2
    double one_minus_q2 = e * (double(m) + t_abs) / (double(m) * double(m));
    if (one_minus_q2 <= 0.0) return 0.0;
    double s = std::sqrt(one_minus_q2);
    if (win == BL_WIN_SINH) return std::sinh(beta * s) / std::sinh(beta);
    return (bessel_i0(beta * s) - 1.0) / (bessel_i0(beta) - 1.0);
}

}  // namespace

double default_beta(int64_t M, int64_t L, int m, bl_method method) {
    if (method == BL_SHANNON) return kPi * m * double(L - M) / double(L);
    return 2.0 * kPi * m * (1.0 - double(M) / (2.0 * double(L)));
}

// hat(v) = (2/L) int_0^m g(t) cos(2 pi v t / L) dt, g = sinc(pi t) phi_g(t) (psi, eq. (4.2))
// or g = phi_g(t).  Double-exponential (tanh-sinh) quadrature on [0, m]:
//   t = m / (1 + e^{-2a}),  m - t = m / (1 + e^{2a}),  a = (pi/2) sinh(tau),
//   dt/dtau = m (pi/2) cosh(tau) / (2 cosh(a)^2).
// The rule handles the (m - t)^{1/2} behaviour of the window at the edge of its support.
double window_transform(bl_window win, bl_method method, int64_t L, int m, double beta, double v) {
    const double h = 1.0 / 64.0;
    const int K = 220;  // |tau| <= 3.44: weights below 1e-40 beyond
    double sum = 0.0;
    for (int k = -K; k <= K; ++k) {
        double tau = k * h;
        double a = 0.5 * kPi * std::sinh(tau);
        if (std::fabs(a) > 350.0) continue;
        double ea = std::exp(2.0 * a);
        double t = m * ea / (1.0 + ea);          // m / (1 + e^{-2a})
        double e = m / (1.0 + ea);               // m - t
        double ca = std::cosh(a);
        double w = double(m) * 0.5 * kPi * std::cosh(tau) / (2.0 * ca * ca);
        if (w == 0.0) continue;
        double g = window_g(win, m, beta, t, e);
        if (method == BL_SHANNON) g *= (t == 0.0) ? 1.0 : sin_pi(t) / (kPi * t);
        g *= cos_pi(2.0 * v * t / double(L));
        sum += w * g;
    }
    return (2.0 / double(L)) * h * sum;
}

// e^{2 pi i n / L}: the angle 2 pi n / L = (pi/4)(o + r/L) with octant o = floor(8n/L) and
// remainder r in [0, L) is formed in integers, and odd octants use the reflected remainder
// L - r, so sin and cos are only evaluated on [0, pi/4].
void twiddles(int64_t L, std::vector<double>* out) {
    out->assign(2 * L, 0.0);
    for (int64_t n = 0; n < L; ++n) {
        int64_t n8 = 8 * n;
        int64_t o = n8 / L;
        int64_t r = n8 - o * L;
        bool odd = (o & 1) != 0;
        double frac = odd ? double(L - r) / double(L) : double(r) / double(L);
        double th = 0.25 * kPi * frac;
        double s = std::sin(th), c = std::cos(th);
        // angle within the quadrant q = o / 2: phi = th (even octant) or pi/2 - th (odd)
        double cq = odd ? s : c;   // cos(phi)
        double sq = odd ? c : s;   // sin(phi)
        double re, im;
        switch (o >> 1) {
            case 0: re = cq; im = sq; break;
            case 1: re = -sq; im = cq; break;
            case 2: re = -cq; im = -sq; break;
            default: re = sq; im = -cq; break;
        }
        (*out)[2 * n] = re;
        (*out)[2 * n + 1] = im;
    }
}

// Radices 16, 8, 4, 2 for powers of two (the compiled Stockham stages).
bool factor_length(int L, FftFactors* out) {
    out->L = L;
    out->nstages = 0;
    if (L < 2 || (L & (L - 1)) != 0) return false;
    int rem = L;
    while (rem > 1) {
        int r = (rem % 16 == 0) ? 16 : (rem % 8 == 0) ? 8 : (rem % 4 == 0) ? 4 : 2;
        if (out->nstages >= kMaxStages) return false;
        out->radix[out->nstages++] = r;
        rem /= r;
    }
    return true;
}

}  // namespace bl
