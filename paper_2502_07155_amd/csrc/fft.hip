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
//  * Precision: BL_F64 and BL_F32 compute and store in their own type.  BL_F32C computes
//    and stores in float but keeps the twiddles in FP64: each twiddle product is formed in
//    double and rounded once (as the deconvolution factors are for every precision).
//    BL_F32D reads float, computes in double (LDS and registers; FP64 runs at the FP32
//    vector rate on this GPU when packed FP32 is not used), keeps the pass intermediates
//    in double and rounds once, when the grid of samples (or the output band) is stored.
//  * L that is not a power of two (or a d = 1 line longer than the LDS pass takes) runs
//    the chirp-z passes of czt.hip instead, with the same layouts and factors.
#include <cstdio>
#include <cstdlib>

#include "blnfft_internal.h"
#include "stockham.h"

namespace bl {
namespace {


using namespace stockham;

struct PassArgs {
    const void* in;
    void* out;
    const double* factor;   // M entries (band side), or nullptr
    const void* tw;         // per-stage twiddles, [k][r-1] per stage (tw_off)
    int outer, inner;       // lines: outer x inner (L^d < 2^31, so 32-bit offsets suffice)
    int Min, Mout, L, M;
    int lgB;                // log2 of lines per workgroup
    int lgL;                // log2 of L
    int tw_in_lds;          // stage the twiddle table in LDS
    int tw_len;             // complex entries in the twiddle table
    int nmain;              // stages of the main radix E (the plan is E, ..., E, rlast)
    int rlast;              // trailing radix (2, 4 or 8 for E = 16; 2 for E = 4), 1 for none
    int tw_off[kMaxStages];
    int lines;              // lines per workgroup chosen by the autotuner (0: heuristic)
    int radix;              // values per thread (4 or 16) chosen by the autotuner (0: heuristic)
};

// Butterfly g of a stage -> (line b, butterfly index j within the line).  Contiguous
// lines map consecutive threads to consecutive j (unit stride along the line, which is
// unit stride in HBM and in the line-major LDS layout); strided lines map consecutive
// threads to consecutive lines (unit stride in HBM and in the interleaved LDS layout).
template <bool CONTIG>
__device__ __forceinline__ void map_butterfly(int g, int lgB, int lgLR, int& b, int& j) {
    if (CONTIG) {
        j = g & ((1 << lgLR) - 1);
        b = g >> lgLR;
    } else {
        b = g & ((1 << lgB) - 1);
        j = g >> lgB;
    }
}

template <bool CONTIG>
__device__ __forceinline__ int lds_index(int b, int pos, int lgB, int Lp) {
    return CONTIG ? b * Lp + padpos(pos) : padpos(pos) * (1 << lgB) + b;
}

template <typename R>
__device__ __forceinline__ Cx<R> scale(Cx<R> v, double f) {
    return {R(double(v.re) * f), R(double(v.im) * f)};
}

// Global-memory view of one workgroup's B lines.
template <typename TI, typename R, typename TO, int DIR, bool CONTIG>
struct LineIO {
    using In = TI;
    const Cx<TI>* __restrict__ in;
    Cx<TO>* __restrict__ out;
    const double* __restrict__ factor;
    int o0, i0, outer, inner;
    int Min, Mout, L, M;

    __device__ __forceinline__ bool line(int b, unsigned& base_in, unsigned& base_out) const {
        const int o = CONTIG ? o0 + b : o0;
        const int i = CONTIG ? 0 : i0 + b;
        base_in = unsigned(o) * unsigned(Min) * unsigned(inner) + unsigned(i);
        base_out = unsigned(o) * unsigned(Mout) * unsigned(inner) + unsigned(i);
        return o < outer && i < inner;
    }
    // FFT input position pos of line b.  Forward: the band sample k with k - M/2 = pos
    // (mod L), times its factor; other positions are zero.  Adjoint: the centred sample
    // (pos + L/2) mod L.
    // Loads of FFT input position pos of line b, split from their use so that a thread's
    // loads of one stage are all in flight together: fetch() issues the (predicated) loads
    // of the value and, with FAC, of its factor; finish() forms the value.
    template <bool FAC>
    __device__ __forceinline__ bool fetch(int b, int pos, Cx<TI>& raw, double& fac) const {
        unsigned bi, bo;
        bool ok = line(b, bi, bo);
        int k;
        if (DIR > 0) {
            k = pos + M / 2;
            if (k >= L) k -= L;
            ok = ok && k < Min;
        } else {
            k = pos + L / 2;
            if (k >= L) k -= L;
        }
        if (ok) {
            raw = in[bi + unsigned(k) * unsigned(inner)];
            if (DIR > 0 && FAC) fac = factor[k];
        }
        return ok;
    }
    template <bool FAC>
    __device__ __forceinline__ Cx<R> finish(bool ok, Cx<TI> raw, double fac) const {
        if (!ok) return Cx<R>{R(0), R(0)};
        const Cx<R> r{R(raw.re), R(raw.im)};
        return (DIR > 0 && FAC) ? scale(r, fac) : r;
    }
    // FFT output position q of line b.  Forward: centred index (q + L/2) mod L.  Adjoint:
    // the band entry k with k - M/2 = q (mod L), times its factor; other q are dropped.
    __device__ __forceinline__ void store(int b, int q, Cx<R> v) const {
        unsigned bi, bo;
        if (!line(b, bi, bo)) return;
        int k;
        if (DIR > 0) {
            k = q + L / 2;
            if (k >= L) k -= L;
        } else {
            k = q + M / 2;
            if (k >= L) k -= L;
            if (k >= Mout) return;
            if (factor) v = scale(v, factor[k]);
        }
        out[bo + unsigned(k) * unsigned(inner)] = Cx<TO>{TO(v.re), TO(v.im)};
    }
};

// One Stockham stage of radix RAD over the workgroup's B lines, split in its read half
// and its compute/write half so a caller can overlap the first stage's HBM reads with
// other work.  Butterfly j of a line reads positions j + r L/RAD, twiddles by w^{r k},
// k = j mod Ns, w = e^{dir 2 pi i/(Ns RAD)} (tw holds this stage's w^{r k} at
// k (RAD-1) + r - 1), and writes positions (j - k) RAD + k + r Ns.
// SRC/DST: 0 = LDS, 1 = global (the first stage reads HBM, the last writes HBM).
template <typename R, int E, int RAD, bool CONTIG, int SRC, typename IO, bool FAC = false>
__device__ __forceinline__ void stage_read(Cx<R>* reg, const Cx<R>* lds, const IO& io, int lgL,
                                           int lgB, int Lp, int tid, int NT) {
    constexpr int NB = E / RAD;
    constexpr int lgR = RAD == 2 ? 1 : RAD == 4 ? 2 : RAD == 8 ? 3 : 4;
    const int lgLR = lgL - lgR;
    const int LR = 1 << lgLR;
    if constexpr (SRC == 0) {
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            int b, j;
            map_butterfly<CONTIG>(tid + u * NT, lgB, lgLR, b, j);
#pragma unroll
            for (int r = 0; r < RAD; ++r) reg[u * RAD + r] = lds[lds_index<CONTIG>(b, j + r * LR, lgB, Lp)];
        }
    } else {
        Cx<typename IO::In> raw[NB * RAD];
        double fac[NB * RAD];
        bool ok[NB * RAD];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            int b, j;
            map_butterfly<CONTIG>(tid + u * NT, lgB, lgLR, b, j);
#pragma unroll
            for (int r = 0; r < RAD; ++r)
                ok[u * RAD + r] = io.template fetch<FAC>(b, j + r * LR, raw[u * RAD + r], fac[u * RAD + r]);
        }
#pragma unroll
        for (int q = 0; q < NB * RAD; ++q) reg[q] = io.template finish<FAC>(ok[q], raw[q], fac[q]);
    }
}

template <typename R, typename TW, int E, int DIR, int RAD, bool CONTIG, int DST, typename IO>
__device__ __forceinline__ void stage_write(Cx<R>* reg, Cx<R>* lds, const Cx<TW>* __restrict__ tw,
                                            const IO& io, int lgL, int lgB, int Lp, int Ns,
                                            int tid, int NT) {
    constexpr int NB = E / RAD;
    constexpr int lgR = RAD == 2 ? 1 : RAD == 4 ? 2 : RAD == 8 ? 3 : 4;
    const int lgLR = lgL - lgR;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        int b, j;
        map_butterfly<CONTIG>(tid + u * NT, lgB, lgLR, b, j);
        const int k = j & (Ns - 1);
        Cx<R>* a = reg + u * RAD;
        if (Ns > 1) {
            const Cx<TW>* wk = tw + k * (RAD - 1);
#pragma unroll
            for (int r = 1; r < RAD; ++r) {
                Cx<TW> w = wk[r - 1];
                if (DIR < 0) w.im = -w.im;
                a[r] = mulw<R, TW>(a[r], w);
            }
        }
        dft<R, DIR, RAD>(a);
        const int base = (j - k) * RAD + k;
#pragma unroll
        for (int r = 0; r < RAD; ++r) {
            const int pos = base + r * Ns;
            if (DST == 0) lds[lds_index<CONTIG>(b, pos, lgB, Lp)] = a[out_slot<RAD>(r)];
            else io.store(b, pos, a[out_slot<RAD>(r)]);
        }
    }
}

// Last stage (LDS -> HBM) of radix RAD.
template <typename R, typename TW, int E, int DIR, int RAD, bool CONTIG, typename IO>
__device__ __forceinline__ void last_stage(Cx<R>* reg, Cx<R>* lds, const Cx<TW>* tw, const IO& io,
                                           int lgL, int lgB, int Lp, int Ns, int tid, int NT) {
    stage_read<R, E, RAD, CONTIG, 0>(reg, lds, io, lgL, lgB, Lp, tid, NT);
    stage_write<R, TW, E, DIR, RAD, CONTIG, 1>(reg, lds, tw, io, lgL, lgB, Lp, Ns, tid, NT);
}

// Threads per workgroup: 1024 with four values per thread, 512 with sixteen (register
// pressure of the radix-16 butterflies in double).
template <int E>
constexpr int max_threads() { return E == 4 ? 1024 : 512; }

// TI: input element type, R: LDS / arithmetic type, TO: output element type, TW: twiddle
// type (products formed in it), E: values per thread (= the main radix: 16, or 4 when the
// pass has few lines and needs more threads).
template <typename TI, typename R, typename TO, typename TW, int DIR, bool CONTIG, int E>
__global__ void __launch_bounds__(max_threads<E>()) k_fft_pass(PassArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int tid = threadIdx.x;
    const int NT = blockDim.x;
    const int B = 1 << a.lgB;
    const int L = a.L;
    const int Lp = padpos(L - 1) + 1;
    Cx<R>* lds = reinterpret_cast<Cx<R>*>(smem_raw);
    const Cx<TW>* tw = static_cast<const Cx<TW>*>(a.tw);
    const int blk = xcd_block(int(blockIdx.x), int(gridDim.x));

    LineIO<TI, R, TO, DIR, CONTIG> io;
    io.in = static_cast<const Cx<TI>*>(a.in);
    io.out = static_cast<Cx<TO>*>(a.out);
    io.factor = a.factor;
    io.outer = a.outer;
    io.inner = a.inner;
    io.Min = a.Min;
    io.Mout = a.Mout;
    io.L = L;
    io.M = a.M;
    if (CONTIG) {
        io.o0 = blk * B;
        io.i0 = 0;
    } else {
        const int iblocks = (a.inner + B - 1) / B;
        io.o0 = blk / iblocks;
        io.i0 = (blk % iblocks) * B;
    }

    // First stage: radix E, Ns = 1 (no twiddles).  Its HBM reads are issued before the
    // twiddle table is staged, so the two latencies overlap.
    Cx<R> reg[E];
    if (a.factor) stage_read<R, E, E, CONTIG, 1, decltype(io), true>(reg, lds, io, a.lgL, a.lgB, Lp, tid, NT);
    else stage_read<R, E, E, CONTIG, 1, decltype(io), false>(reg, lds, io, a.lgL, a.lgB, Lp, tid, NT);
    if (a.tw_in_lds) {
        Cx<TW>* twl = reinterpret_cast<Cx<TW>*>(lds + size_t(B) * Lp);
        for (int e0 = tid; e0 < a.tw_len; e0 += 4 * NT) {
            Cx<TW> v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = tw[min(e0 + u * NT, a.tw_len - 1)];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (e0 + u * NT < a.tw_len) twl[e0 + u * NT] = v[u];
        }
        tw = twl;
    }
    const int nstages = a.nmain + (a.rlast > 1 ? 1 : 0);
    if (nstages == 1) {
        stage_write<R, TW, E, DIR, E, CONTIG, 1>(reg, lds, tw, io, a.lgL, a.lgB, Lp, 1, tid, NT);
        return;
    }
    stage_write<R, TW, E, DIR, E, CONTIG, 0>(reg, lds, tw, io, a.lgL, a.lgB, Lp, 1, tid, NT);
    __syncthreads();
    int Ns = E;
    // middle radix-E stages, LDS -> LDS in place
    const int nmid = a.nmain - 1 - (a.rlast > 1 ? 0 : 1);
    for (int s = 1; s <= nmid; ++s) {
        stage_read<R, E, E, CONTIG, 0>(reg, lds, io, a.lgL, a.lgB, Lp, tid, NT);
        __syncthreads();
        stage_write<R, TW, E, DIR, E, CONTIG, 0>(reg, lds, tw + a.tw_off[s], io, a.lgL, a.lgB, Lp, Ns, tid, NT);
        __syncthreads();
        Ns *= E;
    }
    const Cx<TW>* twl = tw + a.tw_off[nstages - 1];
    if constexpr (E == 16) {
        switch (a.rlast) {
            case 2: last_stage<R, TW, E, DIR, 2, CONTIG>(reg, lds, twl, io, a.lgL, a.lgB, Lp, Ns, tid, NT); break;
            case 4: last_stage<R, TW, E, DIR, 4, CONTIG>(reg, lds, twl, io, a.lgL, a.lgB, Lp, Ns, tid, NT); break;
            case 8: last_stage<R, TW, E, DIR, 8, CONTIG>(reg, lds, twl, io, a.lgL, a.lgB, Lp, Ns, tid, NT); break;
            default: last_stage<R, TW, E, DIR, 16, CONTIG>(reg, lds, twl, io, a.lgL, a.lgB, Lp, Ns, tid, NT); break;
        }
    } else {
        if (a.rlast == 2) last_stage<R, TW, E, DIR, 2, CONTIG>(reg, lds, twl, io, a.lgL, a.lgB, Lp, Ns, tid, NT);
        else last_stage<R, TW, E, DIR, E, CONTIG>(reg, lds, twl, io, a.lgL, a.lgB, Lp, Ns, tid, NT);
    }
}

int ilog2(int v) {
    int l = 0;
    while ((1 << (l + 1)) <= v) ++l;
    return l;
}

// Lines per workgroup: enough to coalesce strided accesses, threads B*L/E within
// max_threads, and LDS within 96 KB.  Contiguous passes need no line grouping for
// coalescing, so there B is halved while the pass would have fewer workgroups than CUs
// (measured: 512 lines of 1024 points run faster as 256 workgroups of 2 than 128 of 4).
int choose_lines(const Plan& p, size_t c, int E, bool contiguous, int64_t lines, int tuned) {
    const int L = int(p.L);
    const int bmax = (c == 16) ? 8 : 16;
    const int tmax = E == 4 ? 1024 : 512;
    int b = 1;
    while (b * 2 <= bmax && (int64_t(b) * 2 * L) / E <= tmax &&
           size_t(b) * 2 * size_t(padpos(L - 1) + 1) * c <= 96 * 1024)
        b *= 2;
    constexpr int64_t kCUs = 256;
    if (contiguous)
        while (b > 1 && (lines + b - 1) / b < kCUs) b /= 2;
    if (tuned > 0) b = tuned;   // measured at plan creation (autotune.cpp)
    if (const char* e = std::getenv("BL_FFT_LINES")) {   // tuning override
        const int v = std::atoi(e);
        if (v >= 1 && v <= 64 && (v & (v - 1)) == 0) b = v;
    }
    // B*L must be a multiple of E and give at least one wave
    while ((int64_t(b) * L) % E != 0 || (int64_t(b) * L) / E < 64) {
        if (b >= 1024) break;
        b *= 2;
    }
    return b;
}

// Values per thread.  Radix-4 stages (four values per thread) measured faster than
// radix-16 ones at every size used here: the passes are latency-bound, and four times the
// threads hide more of it than the fewer LDS round trips of radix 16 save.
// Lengths above 4 * 512 need radix 16 to keep one line within a 512-thread workgroup.
int choose_radix(const Plan& p, int64_t lines) {
    (void)lines;
    if (p.L / 4 > 512) return 16;
    if (const char* e = std::getenv("BL_FFT_RADIX")) {   // tuning override
        const int v = std::atoi(e);
        if (v == 4 || v == 16) return v;
    }
    return 4;
}

template <typename TI, typename R, typename TO, typename TW, int DIR, int E>
bl_status run_pass_e(Plan& p, PassArgs a) {
    const bool contiguous = (a.inner == 1);
    const int B = choose_lines(p, sizeof(Cx<R>), E, contiguous, int64_t(a.outer) * a.inner, a.lines);
    a.lgB = ilog2(B);
    a.lgL = ilog2(a.L);
    const int L = a.L;
    const int NT = int((int64_t(B) * L) / E);
    const size_t data = size_t(B) * size_t(padpos(L - 1) + 1) * sizeof(Cx<R>);
    const size_t twb = size_t(a.tw_len) * sizeof(Cx<TW>);
    a.tw_in_lds = (twb <= 32 * 1024 && data + twb <= 160 * 1024) ? 1 : 0;
    const size_t lds = data + (a.tw_in_lds ? twb : 0);
    if (NT > max_threads<E>() || lds > 160 * 1024) {
        set_error("FFT length too large for the LDS pass kernel");
        return BL_EUNSUPPORTED;
    }
    int64_t nblocks = contiguous ? (int64_t(a.outer) + B - 1) / B
                                 : int64_t(a.outer) * ((int64_t(a.inner) + B - 1) / B);
    if (nblocks == 0) return BL_OK;
    if (nblocks > 0x7fffffffLL) {
        set_error("FFT pass grid too large");
        return BL_EUNSUPPORTED;
    }
    auto kern = contiguous ? k_fft_pass<TI, R, TO, TW, DIR, true, E> : k_fft_pass<TI, R, TO, TW, DIR, false, E>;
    if (lds > 64 * 1024)
        BL_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   int(lds)));
    hipLaunchKernelGGL(kern, dim3(unsigned(nblocks)), dim3(NT), lds, p.stream, a);
    BL_HIP(hipGetLastError());
    return BL_OK;
}

template <typename TI, typename R, typename TO, typename TW, int DIR>
bl_status run_pass(Plan& p, PassArgs a) {
    const int64_t lines = int64_t(a.outer) * a.inner;
    int E = choose_radix(p, lines);
    if (a.radix == 4 || a.radix == 16) E = a.radix;
    if (E == 4 && p.L / 4 > 512) {
        set_error("radix-4 passes take lines of at most 2048 points");
        return BL_EUNSUPPORTED;
    }
    const FftStages& st = E == 16 ? p.st16 : p.st4;
    a.nmain = st.nmain;
    a.rlast = st.rlast;
    for (int s = 0; s < kMaxStages; ++s) a.tw_off[s] = st.tw_off[s];
    a.tw = sizeof(TW) == 8 ? st.d_tw64 : st.d_tw32;
    a.tw_len = st.tw_len;
    if (E == 16) return run_pass_e<TI, R, TO, TW, DIR, 16>(p, a);
    return run_pass_e<TI, R, TO, TW, DIR, 4>(p, a);
}

// Element types of one pass.  F64: all double.  F32: all float.  F32C: float data and
// arithmetic, FP64 twiddles.  F32D: float input and output at the ends of the chain,
// double arithmetic in LDS and double intermediates between passes (a single rounding to
// float, at the final store).
PassTypes pass_types(const Plan& p, bool first, bool last) {
    if (p.prec == BL_F64) return {true, true, true, true};
    if (p.prec == BL_F32) return {false, false, false, false};
    if (p.prec == BL_F32C) return {false, false, false, true};
    return {!first, true, !last, true};
}

template <int DIR>
bl_status dispatch_pass(Plan& p, const PassArgs& a, PassTypes t) {
    if (p.czt.on)
        return launch_czt_pass(p, DIR, a.in, a.out, a.outer, a.inner, a.Min, a.Mout, t, a.lines);
    if (t.comp64) {
        if (t.in64 && t.out64) return run_pass<double, double, double, double, DIR>(p, a);
        if (!t.in64 && t.out64) return run_pass<float, double, double, double, DIR>(p, a);
        if (t.in64 && !t.out64) return run_pass<double, double, float, double, DIR>(p, a);
        return run_pass<float, double, float, double, DIR>(p, a);
    }
    if (t.tw64) return run_pass<float, float, float, double, DIR>(p, a);
    return run_pass<float, float, float, float, DIR>(p, a);
}

void fill_common(const Plan& p, PassArgs& a) {
    a.factor = p.d_deconv;
    a.L = int(p.L);
    a.M = int(p.M);
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
        fill_common(p, a);
        a.outer = 1;
        for (int k = 0; k < axis; ++k) a.outer *= int(p.M);
        a.inner = 1;
        for (int k = axis + 1; k < d; ++k) a.inner *= int(p.L);
        a.Min = int(p.M);
        a.Mout = int(p.L);
        a.lines = p.fft_lines[0][axis];
        a.radix = p.fft_radix[0][axis];
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
        fill_common(p, a);
        a.outer = 1;
        for (int k = 0; k < axis; ++k) a.outer *= int(p.L);
        a.inner = 1;
        for (int k = axis + 1; k < d; ++k) a.inner *= int(p.M);
        a.Min = int(p.L);
        a.Mout = int(p.M);
        a.lines = p.fft_lines[1][axis];
        a.radix = p.fft_radix[1][axis];
        BL_TRY(dispatch_pass<-1>(p, a, t));
        src = dst;
    }
    return BL_OK;
}

// Average time (ms) of `reps` launches of one pass with `lines` lines per workgroup; a
// negative value when that line count is not valid for the pass.
template <int DIR>
double time_pass(Plan& p, PassArgs a, PassTypes t, int lines, int radix, int reps, hipEvent_t e0, hipEvent_t e1) {
    a.lines = lines;
    a.radix = radix;
    if (dispatch_pass<DIR>(p, a, t) != BL_OK) return -1.0;   // warm-up (and validity)
    if (hipEventRecord(e0, p.stream) != hipSuccess) return -1.0;
    for (int r = 0; r < reps; ++r)
        if (dispatch_pass<DIR>(p, a, t) != BL_OK) return -1.0;
    if (hipEventRecord(e1, p.stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -1.0;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0;
    return double(ms) / reps;
}

}  // namespace

bl_status tune_fft_lines(Plan& p, void* buf_in, void* buf_out) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    BL_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        set_error("hipEventCreate failed");
        return BL_EDEVICE;
    }
    const int d = p.d;
    for (int dir = 0; dir < 2; ++dir) {
        for (int axis = d - 1; axis >= 0; --axis) {
            const PassTypes t = pass_types(p, axis == d - 1, axis == 0);
            PassArgs a{};
            a.in = buf_in;
            a.out = buf_out;
            fill_common(p, a);
            a.outer = 1;
            a.inner = 1;
            for (int k = 0; k < axis; ++k) a.outer *= int(dir == 0 ? p.M : p.L);
            for (int k = axis + 1; k < d; ++k) a.inner *= int(dir == 0 ? p.L : p.M);
            a.Min = int(dir == 0 ? p.M : p.L);
            a.Mout = int(dir == 0 ? p.L : p.M);
            int best = 0, best_radix = 0;
            double best_ms = 0.0;
            // the chirp-z passes have one radix (16); the Stockham passes try 4 and 16
            for (int radix : {4, 16}) {
                if (p.czt.on && radix == 4) continue;
                for (int lines = 1; lines <= 64; lines *= 2) {
                    const double ms = dir == 0 ? time_pass<+1>(p, a, t, lines, radix, 5, e0, e1)
                                               : time_pass<-1>(p, a, t, lines, radix, 5, e0, e1);
                    if (ms > 0.0 && std::getenv("BL_TUNE_VERBOSE"))
                        std::fprintf(stderr, "blnfft tune fft: %s axis %d lines=%d radix=%d: %.2f us\n",
                                     dir == 0 ? "forward" : "adjoint", axis, lines, radix, ms * 1e3);
                    if (ms > 0.0 && (best == 0 || ms < best_ms)) {
                        best = lines;
                        best_radix = p.czt.on ? 0 : radix;
                        best_ms = ms;
                    }
                }
            }
            (void)hipGetLastError();
            p.fft_lines[dir][axis] = best;
            p.fft_radix[dir][axis] = best_radix;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    set_error("");
    return BL_OK;
}

bl_status launch_forward_fft(Plan& p, const void* fhat) { return forward_fft(p, fhat); }

bl_status launch_adjoint_fft(Plan& p, const void* grid, void* fhat_out) {
    return adjoint_fft(p, grid, fhat_out);
}

}  // namespace bl
