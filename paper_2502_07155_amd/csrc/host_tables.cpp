// Host-side FP64 tables: window transforms (deconvolution factors), default beta,
// twiddle factors and FFT factorisations.
#include <algorithm>
#include <cmath>
#include <complex>
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

// Modified Bessel function I1 by its power series sum (x/2)^{2k+1} / (k! (k+1)!), positive
// terms as for I0.
double bessel_i1(double x) {
    double q = 0.25 * x * x, term = 0.5 * x, sum = term;
    for (int k = 1; k < 500; ++k) {
        term *= q / (double(k) * double(k + 1));
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

// window_transform at v = 0, 1, ..., K-1 with the same quadrature nodes.  Per node the
// factor cos(2 pi v t / L) is advanced by the rotation e^{2 pi i t / L} and recomputed
// directly every 32 steps, which keeps its error near 32 roundings.
void window_transform_ints(bl_window win, bl_method method, int64_t L, int m, double beta, int64_t K,
                           double* out) {
    const double h = 1.0 / 64.0;
    const int Q = 220;
    for (int64_t v = 0; v < K; ++v) out[v] = 0.0;
    for (int k = -Q; k <= Q; ++k) {
        double tau = k * h;
        double a = 0.5 * kPi * std::sinh(tau);
        if (std::fabs(a) > 350.0) continue;
        double ea = std::exp(2.0 * a);
        double t = m * ea / (1.0 + ea);
        double e = m / (1.0 + ea);
        double ca = std::cosh(a);
        double w = double(m) * 0.5 * kPi * std::cosh(tau) / (2.0 * ca * ca);
        if (w == 0.0) continue;
        double g = window_g(win, m, beta, t, e);
        if (method == BL_SHANNON) g *= (t == 0.0) ? 1.0 : sin_pi(t) / (kPi * t);
        const double wg = (2.0 / double(L)) * h * w * g;
        if (wg == 0.0) continue;
        const double step = 2.0 * t / double(L);
        const double cr = cos_pi(step), sr = sin_pi(step);
        double c = 1.0, s = 0.0;
        for (int64_t v = 0; v < K; ++v) {
            if ((v & 31) == 0) {
                c = cos_pi(step * double(v));
                s = sin_pi(step * double(v));
            }
            out[v] += wg * c;
            const double cn = c * cr - s * sr;
            s = s * cr + c * sr;
            c = cn;
        }
    }
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

// In-place radix-2 DFT (FP64) of a power-of-two length, sign -1: X_q = sum x_n e^{-2 pi i n q/P};
// root[k] = e^{2 pi i k / P}, k < P/2.
void host_dft(std::vector<std::complex<double>>& x, const std::vector<std::complex<double>>& root) {
    const size_t n = x.size();
    for (size_t i = 1, j = 0; i < n; ++i) {
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(x[i], x[j]);
    }
    for (size_t len = 2; len <= n; len <<= 1) {
        const size_t step = n / len;
        for (size_t i = 0; i < n; i += len)
            for (size_t k = 0; k < len / 2; ++k) {
                const std::complex<double> w = std::conj(root[k * step]);
                const std::complex<double> u = x[i + k], v = x[i + k + len / 2] * w;
                x[i + k] = u + v;
                x[i + k + len / 2] = u - v;
            }
    }
}

std::complex<double> chirp(int64_t q, int64_t L, const std::vector<double>& tw2L) {
    int64_t r = q % (2 * L);
    if (r < 0) r += 2 * L;
    return {tw2L[2 * r], tw2L[2 * r + 1]};
}

std::vector<std::complex<double>> chirp_spectrum(int64_t L, int64_t M, int64_t P) {
    std::vector<double> tw2L;
    twiddles(2 * L, &tw2L);
    std::vector<std::complex<double>> h(P, 0.0);
    const int64_t J = (L + M) / 2;
    for (int64_t j = -J + 1; j < J; ++j) h[(j % P + P) % P] = std::conj(chirp(j * j, L, tw2L));
    std::vector<double> twp;
    twiddles(P, &twp);
    std::vector<std::complex<double>> root(P / 2);
    for (int64_t k = 0; k < P / 2; ++k) root[k] = {twp[2 * k], twp[2 * k + 1]};
    host_dft(h, root);
    for (auto& v : h) v /= double(P);
    return h;
}

// Regularized sinc psi_g(u) (shannon) or window phi_g(u) (nfft) in grid units, u = L x - l.
double window_value(bl_window win, bl_method method, int m, double beta, double u) {
    const double a = std::fabs(u);
    if (a >= double(m)) return 0.0;
    double v = window_g(win, m, beta, a, double(m) - a);
    if (method == BL_SHANNON) v *= (u == 0.0) ? 1.0 : sin_pi(u) / (kPi * u);
    return v;
}

// d/du of window_value: phi_g'(u) = phi'(s) ds/du with s = sqrt(1 - (u/m)^2),
// ds/du = -u / (m^2 s), and sinh(beta s)' = beta cosh(beta s), (I0(beta s))' = beta I1(beta s);
// for BL_SHANNON times sinc plus sinc'(u) = (cos(pi u) - sinc(u)) / u times the window.
// At |u| -> m the sinh-type window's derivative is unbounded; callers stay inside.
double window_deriv_value(bl_window win, bl_method method, int m, double beta, double u) {
    const double a = std::fabs(u);
    if (a >= double(m)) return 0.0;
    const double e = double(m) - a;
    const double omq = e * (double(m) + a) / (double(m) * double(m));
    const double s = std::sqrt(omq);
    const double dsdu = -u / (double(m) * double(m) * s);
    double phi, dphi;
    if (win == BL_WIN_SINH) {
        phi = std::sinh(beta * s) / std::sinh(beta);
        dphi = beta * std::cosh(beta * s) / std::sinh(beta) * dsdu;
    } else {
        const double den = bessel_i0(beta) - 1.0;
        phi = (bessel_i0(beta * s) - 1.0) / den;
        // beta I1(beta s) ds/du = -beta^2 u / m^2 * I1(beta s) / (beta s): finite at s = 0
        const double bs = beta * s;
        const double i1_over = bs > 1e-8 ? bessel_i1(bs) / bs : 0.5;
        dphi = -beta * beta * u / (double(m) * double(m)) * i1_over / den;
    }
    if (method != BL_SHANNON) return dphi;
    if (std::fabs(u) < 1e-2) {   // Taylor: sinc and sinc' without the cancellation below
        const double z2 = kPi * kPi * u * u;
        const double sc = 1.0 - z2 * (1.0 / 6.0 - z2 / 120.0);
        const double dsc = -(kPi * kPi * u / 3.0) * (1.0 - z2 * (0.1 - z2 / 280.0));
        return dsc * phi + sc * dphi;
    }
    const double sc = sin_pi(u) / (kPi * u);
    const double dsc = (cos_pi(u) - sc) / u;
    return dsc * phi + sc * dphi;
}

// Edge exponent k of the weight polynomials: the edge pair is sqrt(1 - k theta) K(theta)
// and sqrt(k theta + 1 - k) K(1 - theta).  The sinh-type window behaves like a square
// root at the end of its support (k = 1); the continuous Kaiser-Bessel window like
// 1 - q^2, which is smooth (k = 0: no factor).
double edge_exponent(bl_window win) { return win == BL_WIN_SINH ? 1.0 : 0.0; }

// Polynomials for the float short-sum weights.  Offset o carries u = theta + m - 1 - o,
// theta in [0, 1].  For o = 1..m-1 the weight itself, for o = 0 the factor
// K(theta) = w_0(theta) / sqrt(1 - k theta) (for the sinh window the square-root
// behaviour at |u| = m is taken out).  Each is interpolated at nc Chebyshev points of theta in
// [0, 1], converted to monomials in t = theta - 1/2 and stored as nc/2 even then nc/2
// odd coefficients (the kernel uses w_{2m-1-o}(theta) = w_o(1 - theta)).  Returns the
// largest deviation of the resulting weights from the exact ones, all 2m offsets, in
// double.
double fit_weight_polys(bl_window win, bl_method method, int m, double beta, int nc,
                        std::vector<double>* coef) {
    const int n = nc;
    coef->assign(size_t(m) * nc, 0.0);
    std::vector<std::vector<double>> T(n, std::vector<double>(n, 0.0));
    T[0][0] = 1.0;
    if (n > 1) T[1][1] = 1.0;
    for (int k = 1; k + 1 < n; ++k)
        for (int j = 0; j < n; ++j) {
            double v = -T[k - 1][j];
            if (j > 0) v += 2.0 * T[k][j - 1];
            T[k + 1][j] = v;
        }
    const double k = edge_exponent(win);
    auto target = [&](int o, double th) {
        const double w = window_value(win, method, m, beta, th + (m - 1 - o));
        return o == 0 ? w / std::sqrt(1.0 - k * th) : w;
    };
    double worst = 0.0;
    std::vector<double> mono(n);
    for (int o = 0; o < m; ++o) {
        std::vector<double> f(n), b(n, 0.0), d(n, 0.0);
        for (int i = 0; i < n; ++i) f[i] = target(o, 0.5 * (std::cos(kPi * (i + 0.5) / n) + 1.0));
        for (int k = 0; k < n; ++k) {
            double s = 0.0;
            for (int i = 0; i < n; ++i) s += f[i] * std::cos(kPi * k * (i + 0.5) / n);
            b[k] = (k == 0 ? 1.0 : 2.0) * s / n;
        }
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j) d[j] += b[k] * T[k][j];
        double p2 = 1.0;
        for (int j = 0; j < n; ++j) {
            mono[j] = d[j] * p2;   // x = 2t
            p2 *= 2.0;
        }
        for (int j = 0; j < n; ++j)
            (*coef)[size_t(o) * nc + (j % 2 == 0 ? j / 2 : n / 2 + j / 2)] = mono[j];
        for (int qi = 0; qi <= 512; ++qi) {
            const double th = qi / 512.0;
            for (int side = 0; side < 2; ++side) {
                const double t = side == 0 ? th - 0.5 : 0.5 - th;
                double acc = 0.0;
                for (int j = n - 1; j >= 0; --j) acc = acc * t + mono[j];
                double wv;
                if (o == 0) wv = acc * std::sqrt(side == 0 ? 1.0 - k * th : k * th + 1.0 - k);
                else wv = acc;
                const int oo = side == 0 ? o : 2 * m - 1 - o;
                worst = std::max(worst, std::fabs(wv - window_value(win, method, m, beta, th + (m - 1 - oo))));
            }
        }
    }
    return worst;
}

// Largest deviation of the derivatives d w_o / d theta of the fitted weights (coefficients
// as fit_weight_polys stores them, nc per offset) from the exact ones, relative to the
// largest exact derivative, over all 2m offsets on a grid of theta in [0, 1].  The sinh
// window's edge factor has an unbounded derivative at the support end; the check is meant
// for windows with edge exponent 0.
double weight_deriv_fit_error(bl_window win, bl_method method, int m, double beta, int nc,
                              const std::vector<double>& coef) {
    const int n = nc;
    const double k = edge_exponent(win);
    double worst = 0.0, scale = 0.0;
    std::vector<double> mono(n);
    for (int o = 0; o < m; ++o) {
        for (int j = 0; j < n; ++j) mono[j] = coef[size_t(o) * nc + (j % 2 == 0 ? j / 2 : n / 2 + j / 2)];
        for (int qi = 1; qi < 512; ++qi) {
            const double th = qi / 512.0;
            for (int side = 0; side < 2; ++side) {
                // w_o(theta) = P(theta - 1/2), w_{2m-1-o}(theta) = P(1/2 - theta) (times the
                // edge factor for o = 0)
                const double t = side == 0 ? th - 0.5 : 0.5 - th;
                const double sgn = side == 0 ? 1.0 : -1.0;
                double P = 0.0, dP = 0.0;
                for (int j = n - 1; j >= 0; --j) {
                    dP = dP * t + P;
                    P = P * t + mono[j];
                }
                double dw = sgn * dP;
                if (o == 0 && k != 0.0) {
                    const double f = side == 0 ? 1.0 - k * th : k * th + 1.0 - k;
                    const double sf = std::sqrt(f);
                    dw = sf * dw + (side == 0 ? -k : k) * P / (2.0 * sf);
                }
                const int oo = side == 0 ? o : 2 * m - 1 - o;
                const double ex = window_deriv_value(win, method, m, beta, th + (m - 1 - oo));
                worst = std::max(worst, std::fabs(dw - ex));
                scale = std::max(scale, std::fabs(ex));
            }
        }
    }
    return scale > 0.0 ? worst / scale : worst;
}

// Per-stage twiddles w^{r k} = e^{2 pi i r k / (Ns R)}, laid out [k][r-1] for each stage
// so that the R-1 values a butterfly needs are contiguous.  Stage s starts at off[s].
void stage_twiddles(const FftFactors& fac, const std::vector<double>& tw, std::vector<double>* out,
                    int* off) {
    out->clear();
    const int64_t L = fac.L;
    int64_t Ns = 1;
    for (int s = 0; s < fac.nstages; ++s) {
        const int R = fac.radix[s];
        off[s] = int(out->size() / 2);
        if (Ns > 1) {
            for (int64_t k = 0; k < Ns; ++k)
                for (int r = 1; r < R; ++r) {
                    const int64_t idx = (int64_t(r) * k * (L / (Ns * R))) % L;
                    out->push_back(tw[2 * idx]);
                    out->push_back(tw[2 * idx + 1]);
                }
        }
        Ns *= R;
    }
}

// Powers of two L >= 16: stages of the main radix E followed by at most one smaller power
// of two (the stage plan the pass kernel is compiled for).
bool factor_length(int L, int E, FftFactors* out) {
    out->L = L;
    out->nstages = 0;
    if (L < 16 || (L & (L - 1)) != 0) return false;
    int rem = L;
    while (rem % E == 0 && rem > 1) {
        if (out->nstages >= kMaxStages) return false;
        out->radix[out->nstages++] = E;
        rem /= E;
    }
    if (rem > 1) out->radix[out->nstages++] = rem;
    return true;
}

}  // namespace bl
