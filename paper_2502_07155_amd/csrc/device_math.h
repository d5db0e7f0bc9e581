// Device helpers shared by the short-sum, spreading and gradient kernels: complex
// values, the node-to-cell split, the window and regularized-sinc weights and the
// accumulators.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace bl {
namespace dev {

template <typename R>
struct alignas(2 * sizeof(R)) Cx {
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
    // p - c must use the rounded product p: a contraction into fma(L, x, -c) would count
    // the residual e twice.
#pragma clang fp contract(off)
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

// FP32 weights on the hardware transcendentals (v_sqrt_f32, v_exp_f32 = 2^x, v_rcp_f32):
//   phi = e^{beta (s - 1)} (1 - e^{-2 beta s}) / (1 - e^{-2 beta}),  s = sqrt(1 - (u/m)^2),
// with beta (s - 1) = -beta q^2 / (1 + s), q = u/m.  This form matters in float: the
// window's sensitivity to a rounding of s is beta s ds/s in e^{beta s}, but only
// beta q^2/(1+s)^2 ds in e^{-beta q^2/(1+s)}, which is small where the weights are large.
// For the regularized sinc, psi = (-1)^k sin(pi theta)/(pi u) phi with k = m - 1 - o, and
// one reciprocal 1/((1 + s) u) yields both 1/(1 + s) and 1/u.
struct WinF32 {
    float b2;         // beta * log2(e)
    float cb;         // 1 / (1 - e^{-2 beta})
    float inv_m2;     // 1 / m^2
};

// One float weight at offset o, from the exact formula (used for the two edge offsets,
// where the (m - |u|)^{1/2} behaviour of the window defeats polynomials).  sc is
// sin(pi theta)/pi/(1 - e^{-2 beta}) for the regularized sinc.
template <int M2, int METHOD>
__device__ __forceinline__ float weight_f32_exact(float theta, int o, float sc, const WinF32& wp) {
    constexpr int m = M2 / 2;
    const float u = theta + float(m - 1 - o);
    const float a = float(o + 1) - theta;          // m - u
    const float b = theta + float(2 * m - 1 - o);  // m + u
    const float omq = a * b * wp.inv_m2;           // 1 - (u/m)^2 >= 0
    const float s = __builtin_amdgcn_sqrtf(omq);
    const float q2 = u * u * wp.inv_m2;
    const float e2 = __builtin_amdgcn_exp2f(-2.0f * wp.b2 * s);
    if (METHOD == 0) {
        const float onep = 1.0f + s;
        const float rden = __builtin_amdgcn_rcpf(onep * u);
        const float e1 = __builtin_amdgcn_exp2f(-wp.b2 * q2 * (u * rden));
        const float sg = ((m - 1 - o) & 1) ? -sc : sc;
        const float v = sg * e1 * (1.0f - e2) * (onep * rden);
        return (u == 0.0f) ? 1.0f : v;
    }
    const float e1 = __builtin_amdgcn_exp2f(-wp.b2 * q2 * __builtin_amdgcn_rcpf(1.0f + s));
    return e1 * (1.0f - e2) * wp.cb;
}

template <int M2, int METHOD>
__device__ __forceinline__ float edge_scale(float theta, const WinF32& wp) {
    if (METHOD != 0) return 0.0f;
    constexpr float kInvPi = 0.31830988618379067154f;
    const float r = theta < 0.5f ? theta : 1.0f - theta;
    return sinpif(r) * kInvPi * wp.cb;
}

template <int M2, int METHOD>
__device__ __forceinline__ void weights_f32(float theta, const WinF32& wp, float* w) {
    const float sc = edge_scale<M2, METHOD>(theta, wp);
#pragma unroll
    for (int o = 0; o < M2; ++o) w[o] = weight_f32_exact<M2, METHOD>(theta, o, sc, wp);
}

// Float weights of D coordinates from polynomials (coefficients fitted on the host in
// double).  psi is even, so offset 2m-1-o at theta equals offset o at 1 - theta, i.e. at
// -t with t = theta - 1/2: one polynomial P_o(t) = E_o(t^2) + t O_o(t^2) gives both,
// w[o] = E + t O and w[2m-1-o] = E - t O.  At the edge offsets the sinh-type window has a
// square-root factor, psi(theta + m - 1) = sqrt(1 - theta) K(theta) with K analytic, so
// P_0 fits K and w[0] = sqrt(1 - theta) P_0(t), w[2m-1] = sqrt(theta) P_0(-t).  The
// factors are written sqrt(1 - ek theta) and sqrt(ek theta + 1 - ek): ek = 1 for that
// window, ek = 0 (no factor) for the continuous Kaiser-Bessel window, which is smooth
// there.  coef: per o, NC/2 even then NC/2 odd coefficients.
template <int D, int M2, int NC>
__device__ __forceinline__ void weights_poly(const float* theta, const float* coef,
                                             float (*w)[M2], float ek) {
    constexpr int m = M2 / 2;
    constexpr int NE = NC / 2;
    static_assert(NC % 8 == 4 || NC % 8 == 0, "coefficients are read as float4");
    float t[D], t2[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        t[d] = theta[d] - 0.5f;
        t2[d] = t[d] * t[d];
    }
#pragma unroll
    for (int o = 0; o < m; ++o) {
        float c[NC];
#pragma unroll
        for (int q = 0; q < NC / 4; ++q) {
            const float4 v = reinterpret_cast<const float4*>(coef + o * NC)[q];
            c[4 * q] = v.x;
            c[4 * q + 1] = v.y;
            c[4 * q + 2] = v.z;
            c[4 * q + 3] = v.w;
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
            float E = c[NE - 1], Od = c[NC - 1];
#pragma unroll
            for (int k = NE - 2; k >= 0; --k) {
                E = fmaf(E, t2[d], c[k]);
                Od = fmaf(Od, t2[d], c[NE + k]);
            }
            const float tO = t[d] * Od;
            const float p = E + tO, q = E - tO;
            if (o == 0) {
                w[d][0] = __builtin_amdgcn_sqrtf(fmaf(-ek, theta[d], 1.0f)) * p;
                w[d][M2 - 1] = __builtin_amdgcn_sqrtf(fmaf(ek, theta[d], 1.0f - ek)) * q;
            } else {
                w[d][o] = p;
                w[d][M2 - 1 - o] = q;
            }
        }
    }
}

// Weights and their theta-derivatives from the polynomials of weights_poly: the derivative
// of the approximant itself (for the edge pair, of sqrt(1 - ek theta) K(theta) and
// sqrt(ek theta + 1 - ek) K(1 - theta); with ek = 1 these grow like 1 / sqrt at the
// support end).  Where the square root is zero the edge derivative is taken as zero: the
// window's support ends there.
template <int D, int M2, int NC>
__device__ __forceinline__ void weights_poly_deriv(const float* theta, const float* coef,
                                                   float (*w)[M2], float (*dw)[M2], float ek) {
    constexpr int m = M2 / 2;
    constexpr int NE = NC / 2;
    static_assert(NC % 8 == 4 || NC % 8 == 0, "coefficients are read as float4");
    float t[D], t2[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        t[d] = theta[d] - 0.5f;
        t2[d] = t[d] * t[d];
    }
#pragma unroll
    for (int o = 0; o < m; ++o) {
        float c[NC];
#pragma unroll
        for (int q = 0; q < NC / 4; ++q) {
            const float4 v = reinterpret_cast<const float4*>(coef + o * NC)[q];
            c[4 * q] = v.x;
            c[4 * q + 1] = v.y;
            c[4 * q + 2] = v.z;
            c[4 * q + 3] = v.w;
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
            // E(t^2), O(t^2) and their derivatives in t^2 by Horner
            float E = c[NE - 1], Od = c[NC - 1], dE = 0.0f, dO = 0.0f;
#pragma unroll
            for (int k = NE - 2; k >= 0; --k) {
                dE = fmaf(dE, t2[d], E);
                E = fmaf(E, t2[d], c[k]);
                dO = fmaf(dO, t2[d], Od);
                Od = fmaf(Od, t2[d], c[NE + k]);
            }
            // p(t) = E + t O, q(t) = p(-t); dp/dtheta = A + B, dq/dtheta = A - B
            const float tO = t[d] * Od;
            const float A = 2.0f * t[d] * dE, B = fmaf(2.0f * t2[d], dO, Od);
            const float p = E + tO, q = E - tO, dp = A + B, dq = A - B;
            if (o == 0) {
                const float s1 = __builtin_amdgcn_sqrtf(fmaf(-ek, theta[d], 1.0f));
                const float s0 = __builtin_amdgcn_sqrtf(fmaf(ek, theta[d], 1.0f - ek));
                w[d][0] = s1 * p;
                dw[d][0] = fmaf(s1, dp, -0.5f * ek * p * __builtin_amdgcn_rcpf(s1));
                w[d][M2 - 1] = s0 * q;
                dw[d][M2 - 1] = s0 > 0.0f ? fmaf(s0, dq, 0.5f * ek * q * __builtin_amdgcn_rcpf(s0)) : 0.0f;
            } else {
                w[d][o] = p;
                w[d][M2 - 1 - o] = q;
                dw[d][o] = dp;
                dw[d][M2 - 1 - o] = dq;
            }
        }
    }
}

// Double weights from polynomials in the same even/odd layout as weights_poly (NC/2 even
// then NC/2 odd coefficients per offset pair, read from LDS as uniform double2 loads).
template <int D, int M2, int NC>
__device__ __forceinline__ void weights_poly64(const double* theta, const double* coef,
                                               double (*w)[M2], double ek) {
    constexpr int m = M2 / 2;
    constexpr int NE = NC / 2;
    static_assert(NC % 2 == 0 && NE % 2 == 0, "coefficients are read as double2");
    // dimension-major, so that only one offset's coefficients are live at a time
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const double t = theta[d] - 0.5, t2 = t * t;
#pragma unroll
        for (int o = 0; o < m; ++o) {
            const double2* c2 = reinterpret_cast<const double2*>(coef + o * NC);
            double2 top = c2[NE / 2 - 1], topo = c2[NC / 2 - 1];
            double E = top.y, Od = topo.y;
            E = fma(E, t2, top.x);
            Od = fma(Od, t2, topo.x);
#pragma unroll
            for (int q = NE / 2 - 2; q >= 0; --q) {
                const double2 ce = c2[q], co = c2[NE / 2 + q];
                E = fma(fma(E, t2, ce.y), t2, ce.x);
                Od = fma(fma(Od, t2, co.y), t2, co.x);
            }
            const double tO = t * Od;
            const double p = E + tO, q = E - tO;
            if (o == 0) {
                w[d][0] = sqrt(fma(-ek, theta[d], 1.0)) * p;
                w[d][M2 - 1] = sqrt(fma(ek, theta[d], 1.0 - ek)) * q;
            } else {
                w[d][o] = p;
                w[d][M2 - 1 - o] = q;
            }
            // keep each polynomial's coefficient loads next to their use (bounded
            // register pressure)
            __builtin_amdgcn_sched_barrier(0);
        }
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

// Wide accumulation of float terms: each product of two floats is exact in double, and the
// running sum is kept in double, so the only rounding of the sum is the final one to the
// working precision.  For double data it is the plain FMA sum.
template <typename R>
struct WideAcc {
    double re = 0.0, im = 0.0;
    __device__ __forceinline__ void add(R w, Cx<R> v) {
        const double wd = double(w);
        re = fma(wd, double(v.re), re);
        im = fma(wd, double(v.im), im);
    }
    __device__ __forceinline__ Cx<R> value() const { return {R(re), R(im)}; }
};

// Compensated accumulation of float terms: each product w v is rounded once, and every
// addition to the running sum is made error-free by Knuth's two-sum (s + t = s' + e exactly,
// e formed from s, t and s' in six float operations); the errors are summed separately and
// added once at the end.  For double data it is the plain FMA sum.
template <typename R>
struct TwoSumAcc {
    R re = R(0), im = R(0), cre = R(0), cim = R(0);
    __device__ __forceinline__ static void two_sum(R& s, R t, R& c) {
        const R s1 = s + t;
        const R bp = s1 - s;
        const R ap = s1 - bp;
        c += (s - ap) + (t - bp);
        s = s1;
    }
    __device__ __forceinline__ void add(R w, Cx<R> v) {
        if constexpr (std::is_same<R, double>::value) {
            re = dev_fma(w, v.re, re);
            im = dev_fma(w, v.im, im);
        } else {
            two_sum(re, w * v.re, cre);
            two_sum(im, w * v.im, cim);
        }
    }
    __device__ __forceinline__ Cx<R> value() const { return {re + cre, im + cim}; }
};

// Accumulator of the outermost short-sum loop: 0 plain FMA sums, 1 double (WideAcc),
// 2 two-sum compensated (TwoSumAcc).
template <typename R, int ACC>
using OuterAcc = typename std::conditional<ACC == 1, WideAcc<R>,
                 typename std::conditional<ACC == 2, TwoSumAcc<R>, Plain<R>>::type>::type;

}  // namespace dev
}  // namespace bl
