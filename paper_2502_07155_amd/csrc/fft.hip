// Steps 1-2 of Algorithm 4.2 (and of Algorithm 2.1): deconvolution, zero-padding and the
// d-variate oversampled iFFT (4.7), as one pruned HBM pass per dimension.  Also the
// adjoint direction (forward DFT, truncation to I_M, deconvolution) used by bl_adjoint.
//
// Each pass transforms one axis of a row-major array.  A workgroup owns B lines of that
// axis, stages them in LDS (interleaved: element (b, pos) at P(pos)*B + b, with one pad
// slot every 16 positions), runs radix-16/8/4/2 Stockham stages with every thread holding
// E = 16 complex values in registers per stage, and writes the lines back.
//  * Forward pass (dir +1): the M band samples of a line are placed at FFT position
//    k mod L (k = i - M/2) after multiplication by the FP64 factor 1/(L psihat1(k)); the
//    other L - M positions are zero.  Output position q (l = q or q - L) is stored at
//    centred index (q + L/2) mod L.  Axes not yet transformed keep extent M (pruning).
//  * Adjoint pass (dir -1): input in centred order, output the M band entries times the
//    factor.  Axes already transformed have extent M.
//  * Precision: BL_F64 and BL_F32 compute and store in their own type.  BL_F32C reads
//    float, computes in double (LDS and registers; FP64 runs at the FP32 vector rate on
//    this GPU when packed FP32 is not used), keeps the pass intermediates in double and
//    rounds once, when the grid of samples (or the output band) is stored as float.
#include "blnfft_internal.h"

namespace bl {
namespace {

constexpr int kE = 16;  // complex values per thread per stage

template <typename R>
struct Cx {
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

struct PassArgs {
    const void* in;
    void* out;
    const double* factor;   // M entries (band side), or nullptr
    const void* tw;         // L complex twiddles e^{+2 pi i n / L}
    int64_t outer, inner;
    int Min, Mout, L, M;
    int lgB;                // log2 of lines per workgroup
    int nstages;
    int radix[kMaxStages];
};

// One Stockham stage of radix RAD on B interleaved lines in LDS.
template <typename R, int DIR, int RAD>
__device__ __forceinline__ void stage(Cx<R>* lds, Cx<R>* reg, const Cx<R>* __restrict__ tw,
                                      int L, int lgB, int Ns, int tid, int NT) {
    constexpr int NB = kE / RAD;
    const int B = 1 << lgB;
    const int LR = L / RAD;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        int g = tid + u * NT;
        int b = g & (B - 1);
        int j = g >> lgB;
#pragma unroll
        for (int r = 0; r < RAD; ++r) reg[u * RAD + r] = lds[padpos(j + r * LR) * B + b];
    }
    __syncthreads();
    const int stride = L / (Ns * RAD);
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        int g = tid + u * NT;
        int b = g & (B - 1);
        int j = g >> lgB;
        int k = j % Ns;
        Cx<R>* a = reg + u * RAD;
        if (Ns > 1) {
#pragma unroll
            for (int r = 1; r < RAD; ++r) {
                Cx<R> w = tw[r * k * stride];
                if (DIR < 0) w.im = -w.im;
                a[r] = cmul(a[r], w);
            }
        }
        dft<R, DIR, RAD>(a);
        int base = (j - k) * RAD + k;
#pragma unroll
        for (int r = 0; r < RAD; ++r) lds[padpos(base + r * Ns) * B + b] = a[out_slot<RAD>(r)];
    }
    __syncthreads();
}

template <typename R>
__device__ __forceinline__ Cx<R> scale(Cx<R> v, double f) {
    return {R(double(v.re) * f), R(double(v.im) * f)};
}

// DIR +1: forward transform pass (band in, centred full out).
// DIR -1: adjoint pass (centred full in, band out).
template <typename R>
constexpr int max_threads() { return sizeof(R) == 8 ? 512 : 1024; }

// TI: input element type, R: LDS / arithmetic type, TO: output element type.
template <typename TI, typename R, typename TO, int DIR>
__global__ void __launch_bounds__(max_threads<R>()) k_fft_pass(PassArgs a) {
    extern __shared__ unsigned char smem_raw[];
    Cx<R>* lds = reinterpret_cast<Cx<R>*>(smem_raw);
    const Cx<TI>* __restrict__ in = static_cast<const Cx<TI>*>(a.in);
    Cx<TO>* __restrict__ out = static_cast<Cx<TO>*>(a.out);
    const Cx<R>* __restrict__ tw = static_cast<const Cx<R>*>(a.tw);
    const int tid = threadIdx.x;
    const int NT = blockDim.x;
    const int B = 1 << a.lgB;
    const int L = a.L;
    const int Lp = padpos(L - 1) + 1;

    // line block -> (o0, i0): contiguous lines (inner == 1) group B consecutive outer
    // indices; strided lines group B consecutive inner indices.
    int64_t o0, i0;
    const bool contiguous = (a.inner == 1);
    if (contiguous) {
        o0 = int64_t(blockIdx.x) * B;
        i0 = 0;
    } else {
        int64_t iblocks = (a.inner + B - 1) / B;
        o0 = int64_t(blockIdx.x) / iblocks;
        i0 = (int64_t(blockIdx.x) % iblocks) * B;
    }

    for (int e = tid; e < B * Lp; e += NT) lds[e] = Cx<R>{R(0), R(0)};
    __syncthreads();

    // ---- load
    const int half_in = (DIR > 0) ? a.M / 2 : L / 2;
    const int nin = B * a.Min;
    for (int e = tid; e < nin; e += NT) {
        int b, k;
        if (contiguous) { b = e / a.Min; k = e - b * a.Min; }
        else { b = e & (B - 1); k = e >> a.lgB; }
        int64_t o = contiguous ? o0 + b : o0;
        int64_t i = contiguous ? 0 : i0 + b;
        if (o >= a.outer || i >= a.inner) continue;
        const Cx<TI> vi = in[(o * a.Min + k) * a.inner + i];
        Cx<R> v{R(vi.re), R(vi.im)};
        if (DIR > 0 && a.factor) v = scale(v, a.factor[k]);
        int pos = k - half_in;
        pos += (pos < 0) ? L : 0;
        lds[padpos(pos) * B + b] = v;
    }
    __syncthreads();

    // ---- Stockham stages
    Cx<R> reg[kE];
    int Ns = 1;
    for (int s = 0; s < a.nstages; ++s) {
        int rad = a.radix[s];
        if (rad == 16) stage<R, DIR, 16>(lds, reg, tw, L, a.lgB, Ns, tid, NT);
        else if (rad == 8) stage<R, DIR, 8>(lds, reg, tw, L, a.lgB, Ns, tid, NT);
        else if (rad == 4) stage<R, DIR, 4>(lds, reg, tw, L, a.lgB, Ns, tid, NT);
        else stage<R, DIR, 2>(lds, reg, tw, L, a.lgB, Ns, tid, NT);
        Ns *= rad;
    }

    // ---- store
    const int half_out = (DIR > 0) ? L / 2 : a.M / 2;
    const int nout = B * a.Mout;
    for (int e = tid; e < nout; e += NT) {
        int b, q;
        if (contiguous) { b = e / a.Mout; q = e - b * a.Mout; }
        else { b = e & (B - 1); q = e >> a.lgB; }
        int64_t o = contiguous ? o0 + b : o0;
        int64_t i = contiguous ? 0 : i0 + b;
        if (o >= a.outer || i >= a.inner) continue;
        // output index q holds frequency / grid point q - half_out, FFT position mod L
        int pos = q - half_out;
        pos += (pos < 0) ? L : 0;
        Cx<R> v = lds[padpos(pos) * B + b];
        if (DIR < 0 && a.factor) v = scale(v, a.factor[q]);
        out[(o * a.Mout + q) * a.inner + i] = Cx<TO>{TO(v.re), TO(v.im)};
    }
}

int ilog2(int v) {
    int l = 0;
    while ((1 << (l + 1)) <= v) ++l;
    return l;
}

// Lines per workgroup: enough to coalesce strided accesses, threads B*L/E <= 1024, and
// LDS within `lds_cap` bytes.
int choose_lines(const Plan& p, size_t c) {
    const int L = int(p.L);
    const int bmax = (c == 16) ? 8 : 16;
    const int tmax = (c == 16) ? 512 : 1024;
    int b = 1;
    while (b * 2 <= bmax && (int64_t(b) * 2 * L) / kE <= tmax &&
           size_t(b) * 2 * size_t(padpos(L - 1) + 1) * c <= 96 * 1024)
        b *= 2;
    // at least E values per... B*L must be a multiple of E and give >= 1 wave
    while ((int64_t(b) * L) % kE != 0 || (int64_t(b) * L) / kE < 64) {
        if (b >= 1024) break;
        b *= 2;
    }
    return b;
}

template <typename TI, typename R, typename TO, int DIR>
bl_status run_pass(Plan& p, const PassArgs& a0) {
    PassArgs a = a0;
    const bool contiguous = (a.inner == 1);
    int B = choose_lines(p, sizeof(Cx<R>));
    a.lgB = ilog2(B);
    const int L = a.L;
    const int NT = int((int64_t(B) * L) / kE);
    const size_t lds = size_t(B) * size_t(padpos(L - 1) + 1) * sizeof(Cx<R>);
    if (NT > max_threads<R>() || lds > 160 * 1024) {
        set_error("FFT length too large for the LDS pass kernel");
        return BL_EUNSUPPORTED;
    }
    int64_t nblocks = contiguous ? (a.outer + B - 1) / B : a.outer * ((a.inner + B - 1) / B);
    if (nblocks == 0) return BL_OK;
    if (nblocks > 0x7fffffffLL) {
        set_error("FFT pass grid too large");
        return BL_EUNSUPPORTED;
    }
    auto kern = k_fft_pass<TI, R, TO, DIR>;
    if (lds > 64 * 1024)
        BL_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   int(lds)));
    hipLaunchKernelGGL(kern, dim3(unsigned(nblocks)), dim3(NT), lds, p.stream, a);
    BL_HIP(hipGetLastError());
    return BL_OK;
}

// Element types of one pass.  F64: all double.  F32: all float.  F32C: float input and
// output at the ends of the chain, double arithmetic in LDS and double intermediates
// between passes (a single rounding to float, at the final store).
struct PassTypes {
    bool in64, comp64, out64;
};

PassTypes pass_types(const Plan& p, bool first, bool last) {
    if (p.prec == BL_F64) return {true, true, true};
    if (p.prec == BL_F32) return {false, false, false};
    return {!first, true, !last};
}

template <int DIR>
bl_status dispatch_pass(Plan& p, const PassArgs& a, PassTypes t) {
    if (t.comp64) {
        if (t.in64 && t.out64) return run_pass<double, double, double, DIR>(p, a);
        if (!t.in64 && t.out64) return run_pass<float, double, double, DIR>(p, a);
        if (t.in64 && !t.out64) return run_pass<double, double, float, DIR>(p, a);
        return run_pass<float, double, float, DIR>(p, a);
    }
    return run_pass<float, float, float, DIR>(p, a);
}

void fill_common(const Plan& p, PassArgs& a, bool comp64) {
    a.factor = p.d_deconv;
    a.tw = comp64 ? p.d_tw64 : p.d_tw32;
    a.L = int(p.L);
    a.M = int(p.M);
    a.nstages = p.fac.nstages;
    for (int s = 0; s < p.fac.nstages; ++s) a.radix[s] = p.fac.radix[s];
}

// Forward: f̂ (M^d) -> grid (L^d).  Axis d-1 first; after the pass over axis a, axes
// a..d-1 have extent L and axes before a still extent M.
bl_status forward_fft(Plan& p, const void* fhat) {
    const int d = p.d;
    const void* src = fhat;
    for (int axis = d - 1; axis >= 0; --axis) {
        const PassTypes t = pass_types(p, axis == d - 1, axis == 0);
        PassArgs a{};
        a.in = src;
        void* dst = (axis == 0) ? p.d_grid : ((axis == d - 1) ? p.d_bufA : p.d_bufB);
        a.out = dst;
        fill_common(p, a, t.comp64);
        a.outer = 1;
        for (int k = 0; k < axis; ++k) a.outer *= p.M;
        a.inner = 1;
        for (int k = axis + 1; k < d; ++k) a.inner *= p.L;
        a.Min = int(p.M);
        a.Mout = int(p.L);
        BL_TRY(dispatch_pass<+1>(p, a, t));
        src = dst;
    }
    return BL_OK;
}

// Adjoint: grid (L^d, centred) -> f̂ (M^d), e^{-2 pi i k l / L}, truncation to I_M and
// the real factors.  Axis d-1 first; after it, axes a..d-1 have extent M.
bl_status adjoint_fft(Plan& p, const void* grid, void* fhat_out) {
    const int d = p.d;
    const void* src = grid;
    for (int axis = d - 1; axis >= 0; --axis) {
        const PassTypes t = pass_types(p, axis == d - 1, axis == 0);
        PassArgs a{};
        a.in = src;
        void* dst = (axis == 0) ? fhat_out : ((axis == d - 1) ? p.d_bufA : p.d_bufB);
        a.out = dst;
        fill_common(p, a, t.comp64);
        a.outer = 1;
        for (int k = 0; k < axis; ++k) a.outer *= p.L;
        a.inner = 1;
        for (int k = axis + 1; k < d; ++k) a.inner *= p.M;
        a.Min = int(p.L);
        a.Mout = int(p.M);
        BL_TRY(dispatch_pass<-1>(p, a, t));
        src = dst;
    }
    return BL_OK;
}

}  // namespace

bl_status launch_forward_fft(Plan& p, const void* fhat) { return forward_fft(p, fhat); }

bl_status launch_adjoint_fft(Plan& p, const void* grid, void* fhat_out) {
    return adjoint_fft(p, grid, fhat_out);
}

}  // namespace bl
