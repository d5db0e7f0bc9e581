// Small DFT kernels (radix 2, 4, 8, 16) on complex values held in registers, shared by
// the FFT pass kernels and the batched transforms.  DIR = +1 computes
// X_q = sum_p a_p e^{+2 pi i p q / R}, DIR = -1 the same with e^{-...}.
#pragma once

#include <hip/hip_runtime.h>

namespace bl {
namespace stockham {

template <typename R>
struct alignas(2 * sizeof(R)) Cx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ Cx<R> cadd(Cx<R> a, Cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ Cx<R> csub(Cx<R> a, Cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ Cx<R> cmul(Cx<R> a, Cx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// v * w in the precision of w (double twiddles: the product is formed in double and rounded
// once to R).
template <typename R, typename TW>
__device__ __forceinline__ Cx<R> mulw(Cx<R> v, Cx<TW> w) {
    const TW re = TW(v.re) * w.re - TW(v.im) * w.im;
    const TW im = TW(v.re) * w.im + TW(v.im) * w.re;
    return {R(re), R(im)};
}
// a * (dir * i)
template <typename R, int DIR>
__device__ __forceinline__ Cx<R> rot(Cx<R> a) {
    return DIR > 0 ? Cx<R>{-a.im, a.re} : Cx<R>{a.im, -a.re};
}
// a * e^{dir * 2 pi i j / 16} for the constant angles of the radix-16 split
template <typename R, int DIR, int J>
__device__ __forceinline__ Cx<R> w16(Cx<R> a) {
    constexpr double c1 = 0.92387953251128675613;  // cos(pi/8)
    constexpr double s1 = 0.38268343236508977173;  // sin(pi/8)
    constexpr double h = 0.70710678118654752440;   // cos(pi/4)
    constexpr int j = J & 15;
    constexpr double cr = j == 0 ? 1.0 : j == 1 ? c1 : j == 2 ? h : j == 3 ? s1 : j == 4 ? 0.0
                        : j == 6 ? -h : j == 9 ? -c1 : 0.0;
    constexpr double si = j == 0 ? 0.0 : j == 1 ? s1 : j == 2 ? h : j == 3 ? c1 : j == 4 ? 1.0
                        : j == 6 ? h : j == 9 ? -s1 : 0.0;
    if constexpr (j == 0) {
        return a;
    } else if constexpr (j == 4) {
        return rot<R, DIR>(a);
    } else {
        Cx<R> w{R(cr), R(DIR * si)};
        return cmul(a, w);
    }
}

template <typename R, int DIR>
__device__ __forceinline__ void dft2(Cx<R>* a) {
    Cx<R> t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
}

// 4-point DFT with kernel e^{dir 2 pi i pq/4} on a[0], a[s], a[2s], a[3s] (in place).
template <typename R, int DIR, int S = 1>
__device__ __forceinline__ void dft4(Cx<R>* a) {
    Cx<R> t0 = cadd(a[0], a[2 * S]);
    Cx<R> t1 = csub(a[0], a[2 * S]);
    Cx<R> t2 = cadd(a[S], a[3 * S]);
    Cx<R> t3 = rot<R, DIR>(csub(a[S], a[3 * S]));
    a[0] = cadd(t0, t2);
    a[2 * S] = csub(t0, t2);
    a[S] = cadd(t1, t3);
    a[3 * S] = csub(t1, t3);
}

template <typename R, int DIR>
__device__ __forceinline__ void dft8(Cx<R>* a) {
    Cx<R> e[4] = {a[0], a[2], a[4], a[6]};
    Cx<R> o[4] = {a[1], a[3], a[5], a[7]};
    dft4<R, DIR>(e);
    dft4<R, DIR>(o);
    constexpr double h = 0.70710678118654752440;
    Cx<R> o1 = cmul(o[1], Cx<R>{R(h), R(DIR * h)});
    Cx<R> o2 = rot<R, DIR>(o[2]);
    Cx<R> o3 = cmul(o[3], Cx<R>{R(-h), R(DIR * h)});
    a[0] = cadd(e[0], o[0]);
    a[4] = csub(e[0], o[0]);
    a[1] = cadd(e[1], o1);
    a[5] = csub(e[1], o1);
    a[2] = cadd(e[2], o2);
    a[6] = csub(e[2], o2);
    a[3] = cadd(e[3], o3);
    a[7] = csub(e[3], o3);
}

// 16 = 4 x 4: p = 4 p1 + p2, q = q1 + 4 q2;
// X[q1 + 4 q2] = sum_p2 w4^{p2 q2} w16^{p2 q1} sum_p1 w4^{p1 q1} a[4 p1 + p2].
template <typename R, int DIR>
__device__ __forceinline__ void dft16(Cx<R>* a) {
    // inner 4-point DFTs over p1 for each p2 (stride-4 subsequences, in place)
    dft4<R, DIR, 4>(a + 0);
    dft4<R, DIR, 4>(a + 1);
    dft4<R, DIR, 4>(a + 2);
    dft4<R, DIR, 4>(a + 3);
    // now a[4 q1 + p2] = Y[p2][q1]; twiddle by w16^{p2 q1}
    a[5] = w16<R, DIR, 1>(a[5]);
    a[6] = w16<R, DIR, 2>(a[6]);
    a[7] = w16<R, DIR, 3>(a[7]);
    a[9] = w16<R, DIR, 2>(a[9]);
    a[10] = w16<R, DIR, 4>(a[10]);
    a[11] = w16<R, DIR, 6>(a[11]);
    a[13] = w16<R, DIR, 3>(a[13]);
    a[14] = w16<R, DIR, 6>(a[14]);
    a[15] = w16<R, DIR, 9>(a[15]);
    // outer 4-point DFTs over p2 for each q1 (contiguous groups)
    dft4<R, DIR>(a + 0);
    dft4<R, DIR>(a + 4);
    dft4<R, DIR>(a + 8);
    dft4<R, DIR>(a + 12);
    // now a[4 q1 + q2] = X[q1 + 4 q2]; out_slot<16> maps output index to register
}

// Register holding output X[r] after dft<RAD>: radix 16 leaves its 4x4 digits transposed.
template <int RAD>
__host__ __device__ constexpr int out_slot(int r) {
    return RAD == 16 ? 4 * (r & 3) + (r >> 2) : r;
}

template <typename R, int DIR, int RAD>
__device__ __forceinline__ void dft(Cx<R>* a) {
    if constexpr (RAD == 2) dft2<R, DIR>(a);
    else if constexpr (RAD == 4) dft4<R, DIR>(a);
    else if constexpr (RAD == 8) dft8<R, DIR>(a);
    else dft16<R, DIR>(a);
}

__host__ __device__ __forceinline__ int padpos(int pos) { return pos + (pos >> 4); }


}  // namespace stockham
}  // namespace bl
