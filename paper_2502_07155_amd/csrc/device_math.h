// Device helpers shared by the short-sum, spreading and gradient kernels: complex
// values, the node-to-cell split, the window and regularized-sinc weights and the
// accumulators.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace bl {
namespace dev {

template <typename R>
struct Cx {
    R re, im;
};

// ---------------------------------------------------------------- math helpers
__device__ __forceinline__ double dev_sinpi(double r) { return sinpi(r); }
__device__ __forceinline__ float dev_sinpi(float r) { return sinpif(r); }
__device__ __forceinline__ double dev_exp(double v) { return exp(v); }
__device__ __forceinline__ float dev_exp(float v) { return expf(v); }
__device__ __forceinline__ double dev_sqrt(double v) { return sqrt(v); }
__device__ __forceinline__ float dev_sqrt(float v) { return sqrtf(v); }
__device__ __forceinline__ double dev_rcp(double v) { return 1.0 / v; }
__device__ __forceinline__ float dev_rcp(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double dev_fma(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float dev_fma(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double dev_cospi(double r) { return cospi(r); }
__device__ __forceinline__ float dev_cospi(float r) { return cospif(r); }
__device__ __forceinline__ double dev_floor(double v) { return floor(v); }
__device__ __forceinline__ float dev_floor(float v) { return floorf(v); }

// L x = n + theta with theta in [0, 1]: p = fl(L x), e = L x - p exactly (fma), so the
// offset keeps full precision also when L is not a power of two.  n is clamped to the
// grid [-L/2, L/2 - 1] (x = 1/2 - tiny can round L x up to L/2).
template <typename R>
__device__ __forceinline__ void cell_of(R x, int L, int& n, R& theta) {
    R Lr = R(L);
    R p = Lr * x;
    R e = dev_fma(Lr, x, -p);
    R c = dev_floor(p);
    R th = (p - c) + e;
    if (th < R(0)) { th += R(1); c -= R(1); }
    if (th >= R(1)) { th -= R(1); c += R(1); }
    int ni = int(c);
    if (ni > L / 2 - 1) { th += R(ni - (L / 2 - 1)); ni = L / 2 - 1; }
    if (ni < -L / 2) { ni = -L / 2; th = R(0); }
    n = ni;
    theta = th;
}

// Window phi_g(u) (grid units) at u = theta + m - 1 - o, for |u| < m; 0 otherwise.
// phi = sinh(beta s)/sinh(beta) = e^{beta (s-1)} (1 - e^{-2 beta s}) / (1 - e^{-2 beta}),
// s = sqrt(1 - (u/m)^2), with beta (s - 1) = -beta q^2 / (1 + s) free of cancellation and
// 1 - q^2 = (m - u)(m + u)/m^2 formed from (o + 1 - theta) and (theta + 2m - 1 - o).
template <typename R>
__device__ __forceinline__ R window_at(R theta, int o, int m, R beta, R cb, R inv_m2) {
    R u = theta + R(m - 1 - o);
    R a = R(o + 1) - theta;              // m - u
    R b = theta + R(2 * m - 1 - o);      // m + u
    R omq = a * b * inv_m2;
    if (!(omq > R(0))) return R(0);
    R s = dev_sqrt(omq);
    R q2 = u * u * inv_m2;
    R x1 = -beta * q2 * dev_rcp(R(1) + s);
    return dev_exp(x1) * (R(1) - dev_exp(R(-2) * beta * s)) * cb;
}

// The 2m weights of one coordinate.  METHOD 0: psi_g = sinc(pi u) phi_g(u); 1: phi_g(u).
template <typename R, int M2, int METHOD>
__device__ __forceinline__ void weights(R theta, R beta, R cb, R inv_m2, R* w) {
    constexpr int m = M2 / 2;
    R S = R(0);
    if (METHOD == 0) {
        R r = theta < R(0.5) ? theta : R(1) - theta;
        S = dev_sinpi(r) * R(0.31830988618379067154);   // sin(pi theta) / pi
    }
#pragma unroll
    for (int o = 0; o < M2; ++o) {
        R ph = window_at<R>(theta, o, m, beta, cb, inv_m2);
        if (METHOD == 0) {
            R u = theta + R(m - 1 - o);
            R sg = ((m - 1 - o) & 1) ? R(-1) : R(1);
            R sc = (u == R(0)) ? R(1) : sg * S * dev_rcp(u);
            w[o] = sc * ph;
        } else {
            w[o] = ph;
        }
    }
}

// psi_g(u) and d psi_g / du at u = theta + m - 1 - o (grid units), for the node gradient:
//   d/du sinc(pi u) = (cos(pi u) - sinc(pi u)) / u, with a Taylor branch near u = 0;
//   d/du phi_g(u)  = -beta cosh(beta s)/sinh(beta) * u / (m^2 s),
// cosh(beta s)/sinh(beta) = e^{beta (s-1)} (1 + e^{-2 beta s}) / (1 - e^{-2 beta}).
// At |u| >= m both are 0 (psi is C^1 at the edge of its support).
template <typename R, int M2>
__device__ __forceinline__ void weights_and_derivs(R theta, R beta, R cb, R inv_m2, R* w, R* dw) {
    constexpr int m = M2 / 2;
    constexpr R kPi = R(3.14159265358979323846);
    constexpr R kInvPi = R(0.31830988618379067154);
    constexpr R small = sizeof(R) == 8 ? R(1e-3) : R(0.05);
    const R r = theta < R(0.5) ? theta : R(1) - theta;
    const R sp = dev_sinpi(r);
    const R cp = dev_cospi(theta);
#pragma unroll
    for (int o = 0; o < M2; ++o) {
        const int k = m - 1 - o;
        const R u = theta + R(k);
        const R sg = (k & 1) ? R(-1) : R(1);
        const R a = R(o + 1) - theta;
        const R b = theta + R(2 * m - 1 - o);
        const R omq = a * b * inv_m2;
        R ph = R(0), dph = R(0);
        if (omq > R(0)) {
            const R s = dev_sqrt(omq);
            const R q2 = u * u * inv_m2;
            const R x1 = -beta * q2 * dev_rcp(R(1) + s);
            const R e1 = dev_exp(x1), e2 = dev_exp(R(-2) * beta * s);
            ph = e1 * (R(1) - e2) * cb;
            dph = -beta * cb * e1 * (R(1) + e2) * u * inv_m2 * dev_rcp(s);
        }
        R sc, dsc;
        if (u < small && u > -small) {
            const R z2 = kPi * kPi * u * u;
            sc = R(1) - z2 * (R(1) / R(6) - z2 / R(120));
            dsc = -(kPi * kPi * u / R(3)) * (R(1) - z2 * (R(0.1) - z2 / R(280)));
        } else {
            const R iu = dev_rcp(u);
            sc = sg * sp * kInvPi * iu;
            dsc = (sg * cp - sc) * iu;
        }
        w[o] = sc * ph;
        dw[o] = dsc * ph + sc * dph;
    }
}

// ---------------------------------------------------------------- accumulators
template <typename R>
struct Plain {
    R re = R(0), im = R(0);
    __device__ __forceinline__ void add(R w, Cx<R> v) {
        re = dev_fma(w, v.re, re);
        im = dev_fma(w, v.im, im);
    }
    __device__ __forceinline__ Cx<R> value() const { return {re, im}; }
};

// Compensated dot product (error-free product by fma, two-sum accumulation): the running
// sum s and a correction c collecting every rounding error of products and sums.
template <typename R>
struct TwoSumAcc {
    R s_re = R(0), c_re = R(0), s_im = R(0), c_im = R(0);
    __device__ __forceinline__ static void step(R w, R v, R& s, R& c) {
        R p = w * v;
        R pe = dev_fma(w, v, -p);
        R t = s + p;
        R z = t - s;
        R se = (s - (t - z)) + (p - z);
        s = t;
        c += pe + se;
    }
    __device__ __forceinline__ void add(R w, Cx<R> v) {
        step(w, v.re, s_re, c_re);
        step(w, v.im, s_im, c_im);
    }
    // weight given as the unevaluated sum w + wl (wl: rounding error of a weight product)
    __device__ __forceinline__ void add2(R w, R wl, Cx<R> v) {
        step(w, v.re, s_re, c_re);
        step(w, v.im, s_im, c_im);
        c_re = dev_fma(wl, v.re, c_re);
        c_im = dev_fma(wl, v.im, c_im);
    }
    __device__ __forceinline__ Cx<R> value() const { return {s_re + c_re, s_im + c_im}; }
};


}  // namespace dev
}  // namespace bl
