// Step 2 of Algorithm 4.2 (and of Algorithm 2.1) and the adjoint transform for any even L,
// by the chirp-z (Bluestein) form of the length-L DFT along each axis.  With u = e^{i pi/L}
// and 2 k l = k^2 + l^2 - (l - k)^2, the forward line transform (4.7)
//   theta_l = sum_{k in I_M} a_k e^{2 pi i k l / L} = u^{l^2} sum_k (a_k u^{k^2}) u^{-(l-k)^2}
// is a linear convolution over the lags |l - k| < (L + M)/2, evaluated as a cyclic one of
// power-of-two size P >= L + M - 1:
//   z = IDFT_P( DFT_P(b) H ),   b at position k mod P,   H = DFT_P(h) / P,
//   h_j = u^{-j^2} at position j mod P,   theta_l = u^{l^2} z[l mod P].
// The adjoint line transform sum_l g_l e^{-2 pi i k l / L} is the same with every chirp
// conjugated (h is even in j, so its spectrum becomes conj(H)).  In both directions a line
// reads Min values in centred order (index i <-> i - Min/2, placed at position
// (i - Min/2) mod P) and writes Mout values in centred order.  The chirps u^{k^2} (times the
// deconvolution factor 1/(L psihat1(k)) of step 1, applied on every axis) and u^{l^2} are
// FP64 tables formed on the host from k^2 mod 2L in integers; H is an FP64 host table.
//
// A workgroup holds B lines of P points in LDS (line-major, one pad slot per 16 points) and
// runs both P-point transforms there with radix-16 Stockham stages (a last radix-2/4/8
// stage) and twiddles from two small LDS root tables.  One d = 1 line too long for LDS is
// split into R = P / S pieces of S points by a radix-R decimation in frequency through
// global scratch (k_czt_dif), each piece transformed, multiplied and transformed back in
// LDS by its own workgroup (k_czt_piece), and the pieces recombined per output
// (k_czt_combine):
//   DFT_P(b)[R q + h] = DFT_S(y_h)[q],   y_h[n] = w^{-h n} sum_r b[n + r S] e^{-2 pi i r h/R},
//   z[p] = sum_h w^{h p} E_h[p mod S],   E_h = IDFT_S( Z[R . + h] ),   w = e^{2 pi i / P}.
//
// Precision: R is the arithmetic and LDS type, TW the type of the root, chirp and H tables
// and of their products (double for FP64 plans and for float plans that keep FP64 twiddles;
// the product is then formed in double and rounded once to R).
#include <algorithm>
#include <cstdlib>

#include "blnfft_internal.h"
#include "stockham.h"

namespace bl {
namespace {

using namespace stockham;

constexpr int kRootLo = 128;   // roots e^{2 pi i n / P} = hi[n >> 7] * lo[n & 127]

template <typename TW>
struct Roots {
    const Cx<TW>* hi;
    const Cx<TW>* lo;
    __device__ __forceinline__ Cx<TW> operator()(int n) const { return cmul(hi[n >> 7], lo[n & (kRootLo - 1)]); }
};

// Stage the root tables of the S-th roots root_S(n) = rootsP[n * rs] (rootsP: P-th roots)
// into LDS at `lds` (nhi + nlo entries).
template <typename TW>
__device__ __forceinline__ Roots<TW> stage_roots(Cx<TW>* lds, const Cx<TW>* __restrict__ rootsP, int S,
                                                 int rs, int tid, int NT) {
    const int nlo = S < kRootLo ? S : kRootLo;
    const int nhi = S / nlo;
    Cx<TW>* hi = lds;
    Cx<TW>* lo = lds + nhi;
    for (int e = tid; e < nhi; e += NT) hi[e] = rootsP[size_t(e) * kRootLo * rs];
    for (int e = tid; e < nlo; e += NT) lo[e] = rootsP[size_t(e) * rs];
    return Roots<TW>{hi, lo};
}

template <typename TW>
__host__ __device__ constexpr int root_entries(int S) {
    return (S < kRootLo ? 1 : S / kRootLo) + (S < kRootLo ? S : kRootLo);
}

template <int RAD>
constexpr int lg_of() { return RAD == 2 ? 1 : RAD == 4 ? 2 : RAD == 8 ? 3 : 4; }

// One in-place Stockham stage of radix RAD over B lines of S points in LDS (line stride Sp,
// positions through padpos).  Every butterfly of the stage is read into registers before
// any is written (at most 16 values per thread: NT * 16 >= B * S).
template <typename R, typename TW, int DIR, int RAD>
__device__ __forceinline__ void lds_stage(Cx<R>* buf, int B, int lgS, int Sp, int Ns, const Roots<TW>& rt,
                                          int tid, int NT) {
    constexpr int NB = 16 / RAD;
    const int lgSR = lgS - lg_of<RAD>();
    const int nper = 1 << lgSR;          // butterflies per line
    const int nbf = B << lgSR;
    const int stride = (1 << lgS) / (Ns * RAD);
    Cx<R> reg[16];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int g = tid + u * NT;
        if (g < nbf) {
            const int b = g >> lgSR, j = g & (nper - 1);
            const Cx<R>* line = buf + b * Sp;
#pragma unroll
            for (int r = 0; r < RAD; ++r) reg[u * RAD + r] = line[padpos(j + r * nper)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int g = tid + u * NT;
        if (g < nbf) {
            const int b = g >> lgSR, j = g & (nper - 1);
            const int k = j & (Ns - 1);
            Cx<R>* a = reg + u * RAD;
            if (Ns > 1) {
#pragma unroll
                for (int r = 1; r < RAD; ++r) {
                    Cx<TW> w = rt(r * k * stride);
                    if (DIR < 0) w.im = -w.im;
                    a[r] = mulw<R, TW>(a[r], w);
                }
            }
            dft<R, DIR, RAD>(a);
            const int base = (j - k) * RAD + k;
            Cx<R>* line = buf + b * Sp;
#pragma unroll
            for (int r = 0; r < RAD; ++r) line[padpos(base + r * Ns)] = a[out_slot<RAD>(r)];
        }
    }
    __syncthreads();
}

// DFT of S = 2^lgS points (DIR -1: kernel e^{-2 pi i n q/S}; +1: e^{+...}) on B lines in LDS.
template <typename R, typename TW, int DIR>
__device__ void lds_dft(Cx<R>* buf, int B, int lgS, int Sp, const Roots<TW>& rt, int tid, int NT) {
    int Ns = 1, lg = lgS;
    while (lg >= 4) {
        lds_stage<R, TW, DIR, 16>(buf, B, lgS, Sp, Ns, rt, tid, NT);
        Ns *= 16;
        lg -= 4;
    }
    if (lg == 3) lds_stage<R, TW, DIR, 8>(buf, B, lgS, Sp, Ns, rt, tid, NT);
    else if (lg == 2) lds_stage<R, TW, DIR, 4>(buf, B, lgS, Sp, Ns, rt, tid, NT);
    else if (lg == 1) lds_stage<R, TW, DIR, 2>(buf, B, lgS, Sp, Ns, rt, tid, NT);
}

struct CztArgs {
    const void* in;
    void* out;
    const void* pre;      // Min TW-complex factors of the input (chirp, times deconvolution)
    const void* post;     // Mout TW-complex factors of the output
    const void* H;        // P TW-complex (conjugated in the kernel for DIR = -1)
    const void* roots;    // P TW-complex roots e^{2 pi i n / P}
    void* scr;            // split path: P R-complex
    int outer, inner;     // lines: outer x inner
    int Min, Mout;
    int P, lgP;
    int lgB;              // log2 of lines per workgroup
    int R, lgS;           // split path: pieces and log2 of their length
    int lines;            // lines per workgroup chosen by the autotuner (0: heuristic)
};

// Global index of element i of line b (base offsets of the workgroup's first line o0, i0).
struct Lines {
    int o0, i0, inner, outer, B;
    bool contig;
    __device__ __forceinline__ bool valid(int b) const {
        return contig ? (o0 + b < outer) : (i0 + b < inner);
    }
    __device__ __forceinline__ unsigned index(int b, int i, int len) const {
        const int o = contig ? o0 + b : o0;
        const int ii = contig ? 0 : i0 + b;
        return unsigned(o) * unsigned(len) * unsigned(inner) + unsigned(ii) + unsigned(i) * unsigned(inner);
    }
};

__device__ __forceinline__ int cyc(int c, int P) { return c < 0 ? c + P : c; }

// One workgroup: B lines of one pass.  TI/TO: element types in HBM.
template <typename TI, typename R, typename TO, typename TW, int DIR, int NTMAX>
__global__ void __launch_bounds__(NTMAX) k_czt_pass(CztArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int tid = threadIdx.x, NT = blockDim.x;
    const int B = 1 << a.lgB, P = a.P;
    const int Pp = padpos(P - 1) + 1;
    Cx<R>* buf = reinterpret_cast<Cx<R>*>(smem_raw);
    Cx<TW>* rlds = reinterpret_cast<Cx<TW>*>(smem_raw + ((size_t(B) * Pp * sizeof(Cx<R>) + 15) & ~size_t(15)));
    const int blk = xcd_block(int(blockIdx.x), int(gridDim.x));
    Lines ln;
    ln.contig = a.inner == 1;
    ln.inner = a.inner;
    ln.outer = a.outer;
    ln.B = B;
    if (ln.contig) {
        ln.o0 = blk * B;
        ln.i0 = 0;
    } else {
        const int iblocks = (a.inner + B - 1) / B;
        ln.o0 = blk / iblocks;
        ln.i0 = (blk % iblocks) * B;
    }
    const Cx<TI>* __restrict__ in = static_cast<const Cx<TI>*>(a.in);
    Cx<TO>* __restrict__ out = static_cast<Cx<TO>*>(a.out);
    const Cx<TW>* __restrict__ pre = static_cast<const Cx<TW>*>(a.pre);
    const Cx<TW>* __restrict__ post = static_cast<const Cx<TW>*>(a.post);
    const Cx<TW>* __restrict__ H = static_cast<const Cx<TW>*>(a.H);

    // zero the lines, then place the chirped inputs (strided passes: consecutive threads
    // take consecutive lines, contiguous ones consecutive elements of a line)
    for (int e = tid; e < B * Pp; e += NT) buf[e] = Cx<R>{R(0), R(0)};
    const Roots<TW> rt = stage_roots<TW>(rlds, static_cast<const Cx<TW>*>(a.roots), P, 1, tid, NT);
    __syncthreads();
    const int nin = B * a.Min;
    constexpr int U = 4;
    for (int e0 = tid; e0 < nin; e0 += U * NT) {
        Cx<TI> v[U];
        Cx<TW> f[U];
        int slot[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * NT;
            slot[u] = -1;
            if (e < nin) {
                const int b = ln.contig ? e / a.Min : e % B;
                const int i = ln.contig ? e % a.Min : e / B;
                if (ln.valid(b)) {
                    v[u] = in[ln.index(b, i, a.Min)];
                    f[u] = pre[i];
                    if (DIR < 0) f[u].im = -f[u].im;
                    slot[u] = b * Pp + padpos(cyc(i - a.Min / 2, P));
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (slot[u] >= 0) buf[slot[u]] = mulw<R, TW>(Cx<R>{R(v[u].re), R(v[u].im)}, f[u]);
    }
    __syncthreads();
    lds_dft<R, TW, -1>(buf, B, a.lgP, Pp, rt, tid, NT);
    for (int e = tid; e < B * P; e += NT) {
        const int b = e >> a.lgP, q = e & (P - 1);
        Cx<TW> h = H[q];
        if (DIR < 0) h.im = -h.im;
        const int s = b * Pp + padpos(q);
        buf[s] = mulw<R, TW>(buf[s], h);
    }
    __syncthreads();
    lds_dft<R, TW, +1>(buf, B, a.lgP, Pp, rt, tid, NT);
    const int nout = B * a.Mout;
    for (int e = tid; e < nout; e += NT) {
        const int b = ln.contig ? e / a.Mout : e % B;
        const int o = ln.contig ? e % a.Mout : e / B;
        if (!ln.valid(b)) continue;
        Cx<TW> f = post[o];
        if (DIR < 0) f.im = -f.im;
        const Cx<R> z = mulw<R, TW>(buf[b * Pp + padpos(cyc(o - a.Mout / 2, P))], f);
        out[ln.index(b, o, a.Mout)] = Cx<TO>{TO(z.re), TO(z.im)};
    }
}

// ---- split path (one line, d = 1)

// y_h[n] for every piece h, one thread per n < S.
template <typename TI, typename R, typename TW, int DIR, int RR>
__device__ __forceinline__ void dif_point(const CztArgs& a, int n) {
    const int S = 1 << a.lgS, P = a.P;
    const Cx<TI>* __restrict__ in = static_cast<const Cx<TI>*>(a.in);
    const Cx<TW>* __restrict__ pre = static_cast<const Cx<TW>*>(a.pre);
    const Cx<TW>* __restrict__ roots = static_cast<const Cx<TW>*>(a.roots);
    Cx<R>* __restrict__ scr = static_cast<Cx<R>*>(a.scr);
    Cx<R> v[RR];
#pragma unroll
    for (int r = 0; r < RR; ++r) {
        const int pos = n + r * S;
        // position -> input index: pos = (i - Min/2) mod P
        int i = -1;
        if (pos < a.Min / 2) i = pos + a.Min / 2;
        else if (pos >= P - a.Min / 2) i = pos - P + a.Min / 2;
        v[r] = Cx<R>{R(0), R(0)};
        if (i >= 0) {
            const Cx<TI> x = in[i];
            Cx<TW> f = pre[i];
            if (DIR < 0) f.im = -f.im;
            v[r] = mulw<R, TW>(Cx<R>{R(x.re), R(x.im)}, f);
        }
    }
    dft<R, -1, RR>(v);
#pragma unroll
    for (int h = 0; h < RR; ++h) {
        Cx<TW> w = roots[(h * n) & (P - 1)];
        w.im = -w.im;
        scr[h * S + n] = mulw<R, TW>(v[out_slot<RR>(h)], w);
    }
}

template <typename TI, typename R, typename TW, int DIR>
__global__ void __launch_bounds__(256) k_czt_dif(CztArgs a) {
    const int n = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (n >= (1 << a.lgS)) return;
    switch (a.R) {
        case 2: dif_point<TI, R, TW, DIR, 2>(a, n); break;
        case 4: dif_point<TI, R, TW, DIR, 4>(a, n); break;
        default: dif_point<TI, R, TW, DIR, 8>(a, n); break;
    }
}

// Piece h (blockIdx.x): E_h = IDFT_S( DFT_S(y_h) H[R . + h] ), in place in scratch.
template <typename R, typename TW, int DIR, int NTMAX>
__global__ void __launch_bounds__(NTMAX) k_czt_piece(CztArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int tid = threadIdx.x, NT = blockDim.x;
    const int h = blockIdx.x, S = 1 << a.lgS;
    const int Sp = padpos(S - 1) + 1;
    Cx<R>* buf = reinterpret_cast<Cx<R>*>(smem_raw);
    Cx<TW>* rlds = reinterpret_cast<Cx<TW>*>(smem_raw + ((size_t(Sp) * sizeof(Cx<R>) + 15) & ~size_t(15)));
    Cx<R>* __restrict__ scr = static_cast<Cx<R>*>(a.scr) + size_t(h) * S;
    const Cx<TW>* __restrict__ H = static_cast<const Cx<TW>*>(a.H);
    const Roots<TW> rt = stage_roots<TW>(rlds, static_cast<const Cx<TW>*>(a.roots), S, a.R, tid, NT);
    for (int n = tid; n < S; n += NT) buf[padpos(n)] = scr[n];
    __syncthreads();
    lds_dft<R, TW, -1>(buf, 1, a.lgS, Sp, rt, tid, NT);
    for (int q = tid; q < S; q += NT) {
        Cx<TW> hv = H[q * a.R + h];
        if (DIR < 0) hv.im = -hv.im;
        buf[padpos(q)] = mulw<R, TW>(buf[padpos(q)], hv);
    }
    __syncthreads();
    lds_dft<R, TW, +1>(buf, 1, a.lgS, Sp, rt, tid, NT);
    for (int n = tid; n < S; n += NT) scr[n] = buf[padpos(n)];
}

// Output o: z[p] = sum_h w^{h p} E_h[p mod S] at p = (o - Mout/2) mod P, times its factor.
template <typename R, typename TO, typename TW, int DIR, int RR>
__device__ __forceinline__ void combine_point(const CztArgs& a, int o) {
    const int S = 1 << a.lgS, P = a.P;
    const Cx<R>* __restrict__ scr = static_cast<const Cx<R>*>(a.scr);
    const Cx<TW>* __restrict__ roots = static_cast<const Cx<TW>*>(a.roots);
    const Cx<TW>* __restrict__ post = static_cast<const Cx<TW>*>(a.post);
    const int p = cyc(o - a.Mout / 2, P);
    const int n = p & (S - 1);
    Cx<R> e[RR];
    Cx<TW> w[RR];
#pragma unroll
    for (int h = 0; h < RR; ++h) {
        e[h] = scr[h * S + n];
        w[h] = roots[(h * p) & (P - 1)];
    }
    Cx<TW> z{TW(0), TW(0)};
#pragma unroll
    for (int h = 0; h < RR; ++h) {
        z.re += TW(e[h].re) * w[h].re - TW(e[h].im) * w[h].im;
        z.im += TW(e[h].re) * w[h].im + TW(e[h].im) * w[h].re;
    }
    Cx<TW> f = post[o];
    if (DIR < 0) f.im = -f.im;
    const TW re = z.re * f.re - z.im * f.im, im = z.re * f.im + z.im * f.re;
    static_cast<Cx<TO>*>(a.out)[o] = Cx<TO>{TO(re), TO(im)};
}

template <typename R, typename TO, typename TW, int DIR>
__global__ void __launch_bounds__(256) k_czt_combine(CztArgs a) {
    const int o = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (o >= a.Mout) return;
    switch (a.R) {
        case 2: combine_point<R, TO, TW, DIR, 2>(a, o); break;
        case 4: combine_point<R, TO, TW, DIR, 4>(a, o); break;
        default: combine_point<R, TO, TW, DIR, 8>(a, o); break;
    }
}

int ilog2c(int64_t v) {
    int l = 0;
    while ((int64_t(1) << (l + 1)) <= v) ++l;
    return l;
}

template <typename R>
constexpr int ntmax() { return sizeof(R) == 8 ? 512 : 1024; }

template <typename TI, typename R, typename TO, typename TW, int DIR>
bl_status run_czt(Plan& p, CztArgs a) {
    const CztTables& t = p.czt;
    a.P = int(t.P);
    a.lgP = ilog2c(t.P);
    const bool tw64 = sizeof(TW) == 8;
    a.roots = tw64 ? t.d_roots64 : t.d_roots32;
    a.H = tw64 ? t.d_H64 : t.d_H32;
    if (!t.split) {
        const int64_t lines = int64_t(a.outer) * a.inner;
        const int64_t cap = int64_t(kCztLdsPoints<R>()) / t.P;   // lines per workgroup
        int B = 1;
        while (int64_t(B) * 2 <= cap && B * 2 <= 16 && B * 2 <= lines) B *= 2;
        if (a.lines > 0) {   // measured at plan creation (autotune.cpp)
            if (a.lines > cap) {
                set_error("chirp-z lines per workgroup above the LDS size");
                return BL_EUNSUPPORTED;
            }
            B = a.lines;
        }
        if (const char* e = std::getenv("BL_CZT_LINES")) {   // tuning override
            const int v = std::atoi(e);
            if (v >= 1 && v <= cap && (v & (v - 1)) == 0) B = v;
        }
        a.lgB = ilog2c(B);
        const int NT = int(std::max<int64_t>(64, int64_t(B) * t.P / 16));
        const int Pp = stockham::padpos(int(t.P) - 1) + 1;
        const size_t lds = ((size_t(B) * Pp * sizeof(Cx<R>) + 15) & ~size_t(15)) +
                           size_t(root_entries<TW>(int(t.P))) * sizeof(Cx<TW>);
        if (NT > ntmax<R>() || lds > 160 * 1024) {
            set_error("chirp-z line too long for the LDS kernel");
            return BL_EUNSUPPORTED;
        }
        const int64_t nblocks = a.inner == 1 ? (a.outer + B - 1) / B
                                             : int64_t(a.outer) * ((int64_t(a.inner) + B - 1) / B);
        if (nblocks == 0) return BL_OK;
        auto kern = k_czt_pass<TI, R, TO, TW, DIR, ntmax<R>()>;
        if (lds > 64 * 1024)
            BL_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
        hipLaunchKernelGGL(kern, dim3(unsigned(nblocks)), dim3(NT), lds, p.stream, a);
        BL_HIP(hipGetLastError());
        return BL_OK;
    }
    // one line too long for LDS (d = 1): decimation into R pieces of S points
    if (a.outer != 1 || a.inner != 1) {
        set_error("internal: split chirp-z pass on more than one line");
        return BL_EUNSUPPORTED;
    }
    a.R = t.R;
    a.lgS = ilog2c(t.P / t.R);
    a.scr = t.d_scr;
    const int S = 1 << a.lgS;
    const int NT = std::max(64, S / 16);
    const int Sp = stockham::padpos(S - 1) + 1;
    const size_t lds = ((size_t(Sp) * sizeof(Cx<R>) + 15) & ~size_t(15)) + size_t(root_entries<TW>(S)) * sizeof(Cx<TW>);
    if (NT > ntmax<R>() || lds > 160 * 1024) {
        set_error("internal: chirp-z piece too long for the LDS kernel");
        return BL_EUNSUPPORTED;
    }
    hipLaunchKernelGGL((k_czt_dif<TI, R, TW, DIR>), dim3(unsigned((S + 255) / 256)), dim3(256), 0, p.stream, a);
    BL_HIP(hipGetLastError());
    auto piece = k_czt_piece<R, TW, DIR, ntmax<R>()>;
    if (lds > 64 * 1024)
        BL_HIP(hipFuncSetAttribute((const void*)piece, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    hipLaunchKernelGGL(piece, dim3(unsigned(a.R)), dim3(NT), lds, p.stream, a);
    BL_HIP(hipGetLastError());
    hipLaunchKernelGGL((k_czt_combine<R, TO, TW, DIR>), dim3(unsigned((a.Mout + 255) / 256)), dim3(256), 0,
                       p.stream, a);
    BL_HIP(hipGetLastError());
    return BL_OK;
}

template <int DIR>
bl_status czt_dispatch(Plan& p, CztArgs a, PassTypes t) {
    if (t.comp64) {
        if (t.in64 && t.out64) return run_czt<double, double, double, double, DIR>(p, a);
        if (!t.in64 && t.out64) return run_czt<float, double, double, double, DIR>(p, a);
        if (t.in64 && !t.out64) return run_czt<double, double, float, double, DIR>(p, a);
        return run_czt<float, double, float, double, DIR>(p, a);
    }
    if (t.tw64) return run_czt<float, float, float, double, DIR>(p, a);
    return run_czt<float, float, float, float, DIR>(p, a);
}

}  // namespace

bl_status launch_czt_pass(Plan& p, int dir, const void* in, void* out, int outer, int inner, int Min,
                          int Mout, PassTypes t, int lines) {
    CztArgs a{};
    a.lines = lines;
    a.in = in;
    a.out = out;
    a.outer = outer;
    a.inner = inner;
    a.Min = Min;
    a.Mout = Mout;
    // forward: band chirp (with deconvolution) in, grid chirp out; adjoint: the reverse
    const bool tw64 = t.comp64 || t.tw64;
    const void* band = tw64 ? p.czt.d_band64 : p.czt.d_band32;
    const void* grid = tw64 ? p.czt.d_grid64 : p.czt.d_grid32;
    a.pre = dir > 0 ? band : grid;
    a.post = dir > 0 ? grid : band;
    return dir > 0 ? czt_dispatch<+1>(p, a, t) : czt_dispatch<-1>(p, a, t);
}

}  // namespace bl
