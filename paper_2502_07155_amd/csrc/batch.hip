// Batched d = 1 transforms (Algorithm 4.2) of many independent instances with their own
// (M_i, L_i, m_i, N_i), executed as one hipGraph (DFT kernels, then the short sums).
//
// Step 2 for arbitrary even L (not only powers of two) uses the chirp-z (Bluestein) form
// of the transform (4.7): with u = e^{i pi / L} and k l = (k^2 + l^2 - (l-k)^2)/2,
//   theta_l = sum_{k in I_M} a_k e^{2 pi i k l / L} = u^{l^2} sum_k (a_k u^{k^2}) u^{-(l-k)^2},
// a linear convolution evaluated as a cyclic one of power-of-two size P >= L + M - 1:
//   z = IDFT_P( DFT_P(b) * H ),  b_k = a_k u^{k^2} at position k mod P,
//   H = DFT_P(h) / P,  h_j = u^{-j^2} at position j mod P, |j| < (L + M)/2,
//   theta_l = u^{l^2} z[l mod P].
// a_k = fhat(k) / (L psihat(k)) (step 1) and the chirps u^{k^2}, u^{l^2} are formed in FP64 on
// the host (k^2 mod 2L in integers); H is computed on the host in FP64 and stored as float.
// An instance with P <= 8192 runs both DFTs in LDS in one 512-thread workgroup.  A larger
// one is split into R = P / S pieces of S <= 8192 points: k_batch_dif forms the pieces of
// a radix-R decimation in frequency in global scratch, one workgroup per piece runs its
// two DFTs in LDS, and k_batch_combine undoes the decimation for the output.  Work items
// are ordered largest first, and the DFT launch is persistent: its workgroups (as many as
// fit the GPU at once) take the items from a device work queue, so the uneven instances
// balance over the CUs.
//
// Step 3 runs one workgroup per work chunk of the instances' node tiles, as in the
// single-transform short sums, with each chunk's instance parameters (L, m, window
// polynomials) read from a descriptor table.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "blnfft_internal.h"
#include "device_math.h"
#include "stockham.h"

namespace bl {

namespace {

namespace sk = stockham;
using CxF = dev::Cx<float>;

constexpr int kBatchThreads = 512;
constexpr int kMaxLdsFft = 8192;       // largest DFT held in LDS (float complex)
constexpr int kMaxP = 32768;

struct InstDesc {
    int M, L, m, P;
    int R;               // P = R S: R pieces of S points (R = 1: one LDS DFT)
    int lgS;             // log2 of the LDS DFT size S (P or P/2)
    int tw_off;          // twiddle table e^{2 pi i n / S}, n < S
    int twP_off;         // twiddle table e^{2 pi i n / P}, n < P (R > 1)
    long long fhat_off;  // band samples (M complex)
    long long theta_off; // samples theta (L complex, centred)
    long long pre_off;   // a-factor times chirp, M double complex
    long long post_off;  // chirp u^{l^2}, L double complex
    long long h_off;     // H, P float complex
    long long scr_off;   // scratch (P float complex) for R > 1
    long long node_off;  // first node of the instance
    int tile_base;       // first global tile of the instance
    int ntiles;
};

// ---------------------------------------------------------------- LDS DFT
// Twiddles e^{2 pi i n / S} from two small LDS tables: hi[n >> 7] * lo[n & 127].
struct Roots {
    const sk::Cx<float>* hi;
    const sk::Cx<float>* lo;
    __device__ __forceinline__ sk::Cx<float> operator[](int n) const {
        return sk::cmul(hi[n >> 7], lo[n & 127]);
    }
};
constexpr int kRootLo = 128;
constexpr int kRootHi = kMaxLdsFft / kRootLo;

// Stage the two tables of S-th roots from the full table tw (S entries) into LDS.
__device__ __forceinline__ Roots stage_roots(sk::Cx<float>* lds, const sk::Cx<float>* tw, int S, int tid) {
    sk::Cx<float>* hi = lds;
    sk::Cx<float>* lo = lds + kRootHi;
    const int nlo = S < kRootLo ? S : kRootLo;
    const int nhi = S / nlo;
    for (int e = tid; e < nhi; e += kBatchThreads) hi[e] = tw[e * kRootLo];
    for (int e = tid; e < nlo; e += kBatchThreads) lo[e] = tw[e];
    return Roots{hi, lo};
}

// In-place Stockham DFT stage of radix RAD on S = 2^lgS points in LDS (indexed through
// padpos); kBatchThreads threads, up to 16 values each.
template <int DIR, int RAD>
__device__ __forceinline__ void lds_stage(sk::Cx<float>* buf, int S, int Ns, const Roots tw, int tid) {
    constexpr int NB = 16 / RAD;
    const int nb = S / RAD;
    const int stride = S / (Ns * RAD);
    sk::Cx<float> reg[16];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int g = tid + u * kBatchThreads;
        if (g < nb) {
#pragma unroll
            for (int r = 0; r < RAD; ++r) reg[u * RAD + r] = buf[sk::padpos(g + r * nb)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int g = tid + u * kBatchThreads;
        if (g < nb) {
            const int k = g & (Ns - 1);
            sk::Cx<float>* a = reg + u * RAD;
            if (Ns > 1) {
#pragma unroll
                for (int r = 1; r < RAD; ++r) {
                    sk::Cx<float> w = tw[r * k * stride];
                    if (DIR < 0) w.im = -w.im;
                    a[r] = sk::cmul(a[r], w);
                }
            }
            sk::dft<float, DIR, RAD>(a);
            const int base = (g - k) * RAD + k;
#pragma unroll
            for (int r = 0; r < RAD; ++r) buf[sk::padpos(base + r * Ns)] = a[sk::out_slot<RAD>(r)];
        }
    }
    __syncthreads();
}

// Radix-16 stages (one butterfly per thread at S = 16384), then one radix-2/4/8 stage.
template <int DIR>
__device__ void lds_dft(sk::Cx<float>* buf, int lgS, const Roots tw, int tid) {
    const int S = 1 << lgS;
    int Ns = 1, lg = lgS;
    while (lg >= 4) {
        lds_stage<DIR, 16>(buf, S, Ns, tw, tid);
        Ns *= 16;
        lg -= 4;
    }
    if (lg == 3) lds_stage<DIR, 8>(buf, S, Ns, tw, tid);
    else if (lg == 2) lds_stage<DIR, 4>(buf, S, Ns, tw, tid);
    else if (lg == 1) lds_stage<DIR, 2>(buf, S, Ns, tw, tid);
}

__device__ __forceinline__ sk::Cx<float> mul_d(sk::Cx<float> v, double2 f) {
    const double re = double(v.re) * f.x - double(v.im) * f.y;
    const double im = double(v.re) * f.y + double(v.im) * f.x;
    return {float(re), float(im)};
}

// Band sample at cyclic position n of the length-P input b (zero off the band).
__device__ __forceinline__ sk::Cx<float> band_at(const InstDesc& d, const sk::Cx<float>* fhat,
                                                 const double2* pre, int n) {
    // k = n for n < M/2, k = n - P for n >= P - M/2
    int i;
    if (n < d.M / 2) i = n + d.M / 2;
    else if (n >= d.P - d.M / 2) i = n - d.P + d.M / 2;
    else return sk::Cx<float>{0.0f, 0.0f};
    return mul_d(fhat[i], pre[i]);
}

// Element-wise pass over n items with U global loads in flight per thread: load(i) for U
// items first, then store(i, value) for the same items.
template <int U, typename T, typename Load, typename Store>
__device__ __forceinline__ void staged_pass(int n, int tid, int nt, Load load, Store store) {
    for (int base = tid; base < n; base += U * nt) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = base + u * nt;
            if (i < n) v[u] = load(i);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = base + u * nt;
            if (i < n) store(i, v[u]);
        }
    }
}

// Work item of the transform kernel: a whole instance (half < 0) or one of the two
// half-length transforms of an instance with P = 2S (half = 0, 1).
struct FftItem {
    int inst;
    int half;
};

constexpr int kBatchQueue = 2;   // ints of the transform launch's work queue

struct FftArgs {
    const InstDesc* desc;
    const FftItem* items;
    const void* fhat;
    void* theta;
    const double2* pre;
    const double2* post;
    const void* h;
    void* scratch;
    const void* tw;
};

// P = R S, pieces h = 0..R-1: X[R q + h] = DFT_S(y_h)[q] with
// y_h[n] = e^{-2 pi i h n/P} sum_r b[n + r S] e^{-2 pi i r h/R}, and the inverse is
// z[p] = sum_h e^{2 pi i h p/P} E_h[p mod S], E_h the inverse DFT of Z[R q + h] over q.
// Each piece runs on its own workgroup and leaves E_h in scratch; k_batch_combine then
// forms the outputs.
// theta_l = u^{l^2} z[l mod P] with z[p] = sum_h e^{2 pi i h p/P} E_h[p mod S] (E_h in
// scratch slices); all loads of an output are issued before its arithmetic.
template <int R>
__device__ __forceinline__ void combine_pieces(const InstDesc& d, const sk::Cx<float>* scr,
                                               const sk::Cx<float>* twP, const double2* post,
                                               sk::Cx<float>* theta, int tid, int NT) {
    const int S = 1 << d.lgS;
    for (int i = tid; i < d.L; i += NT) {
        const int l = i - d.L / 2;
        const int pz = l < 0 ? l + d.P : l;
        const int n = pz & (S - 1);
        sk::Cx<float> e[R], w[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            e[q] = scr[q * S + n];
            w[q] = twP[(q * pz) & (d.P - 1)];
        }
        const double2 c = post[i];
        sk::Cx<float> z{0.0f, 0.0f};
#pragma unroll
        for (int q = 0; q < R; ++q) z = sk::cadd(z, sk::cmul(e[q], w[q]));
        theta[i] = mul_d(z, c);
    }
}

// Radix-R decimation in frequency of the chirped band b (length P = R S): one thread per
// position n < S computes y_h[n] = e^{-2 pi i h n/P} sum_r b[n + r S] e^{-2 pi i r h/R} for
// every piece h and stores it to scratch slice h.
struct DifItem {
    int inst;
    int n0;   // first position of this workgroup's 256
};

template <int R>
__device__ __forceinline__ void dif_point(const InstDesc& d, const sk::Cx<float>* fhat, const double2* pre,
                                          const sk::Cx<float>* twP, sk::Cx<float>* scr, int n) {
    const int S = 1 << d.lgS;
    sk::Cx<float> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = band_at(d, fhat, pre, n + r * S);
    sk::dft<float, -1, R>(v);
#pragma unroll
    for (int q = 0; q < R; ++q) {
        sk::Cx<float> w = twP[(q * n) & (d.P - 1)];
        w.im = -w.im;
        scr[q * S + n] = sk::cmul(v[sk::out_slot<R>(q)], w);
    }
}

__global__ void __launch_bounds__(256) k_batch_dif(FftArgs a, const DifItem* items) {
    const DifItem it = items[blockIdx.x];
    const InstDesc d = a.desc[it.inst];
    const int n = it.n0 + int(threadIdx.x);
    if (n >= (1 << d.lgS)) return;
    const sk::Cx<float>* fhat = static_cast<const sk::Cx<float>*>(a.fhat) + d.fhat_off;
    const double2* pre = a.pre + d.pre_off;
    const sk::Cx<float>* twP = static_cast<const sk::Cx<float>*>(a.tw) + d.twP_off;
    sk::Cx<float>* scr = static_cast<sk::Cx<float>*>(a.scratch) + d.scr_off;
    switch (d.R) {
        case 2: dif_point<2>(d, fhat, pre, twP, scr, n); break;
        case 4: dif_point<4>(d, fhat, pre, twP, scr, n); break;
        default: dif_point<8>(d, fhat, pre, twP, scr, n); break;
    }
}

// Work queue of a persistent launch: queue[0] is the next item, queue[1] counts the
// workgroups that have run out of items.  A workgroup takes items until they run out; the
// last one to finish clears both counters for the next launch (no other workgroup touches
// them by then), so the queue needs no clearing kernel.  Item lists are sorted most
// expensive first, so the queue balances uneven instances.
__device__ __forceinline__ int next_item(int* queue) {
    __shared__ int item;
    __syncthreads();   // the previous item is done with LDS and with `item`
    if (threadIdx.x == 0) item = atomicAdd(&queue[0], 1);
    __syncthreads();
    return item;
}

__device__ __forceinline__ void queue_done(int* queue) {
    if (threadIdx.x == 0 && atomicAdd(&queue[1], 1) == int(gridDim.x) - 1) {
        atomicExch(&queue[0], 0);
        atomicExch(&queue[1], 0);
    }
}

// One transform work item (a whole instance, or one piece of a split one).
__device__ void batch_fft_item(const FftArgs& a, int index, sk::Cx<float>* buf) {
    const FftItem item = a.items[index];
    const InstDesc d = a.desc[item.inst];
    const int tid = threadIdx.x;
    const int S = 1 << d.lgS;
    const sk::Cx<float>* fhat = static_cast<const sk::Cx<float>*>(a.fhat) + d.fhat_off;
    const double2* pre = a.pre + d.pre_off;
    const double2* post = a.post + d.post_off;
    const sk::Cx<float>* H = static_cast<const sk::Cx<float>*>(a.h) + d.h_off;
    sk::Cx<float>* theta = static_cast<sk::Cx<float>*>(a.theta) + d.theta_off;
    // root tables after the data buffer (visible to all threads after the first barrier)
    const Roots tw = stage_roots(buf + (sk::padpos(kMaxLdsFft - 1) + 1),
                                 static_cast<const sk::Cx<float>*>(a.tw) + d.tw_off, S, tid);

    using SCx = sk::Cx<float>;
    constexpr int U = 8;
    const int NT = kBatchThreads;
    // output position i (centred l = i - L/2) reads cyclic position (l mod P)
    auto out_pos = [&](int i) {
        const int n = i - d.L / 2;
        return n < 0 ? n + d.P : n;
    };
    auto mult_h = [&](int hoff, int hstride) {
        staged_pass<U, SCx>(S, tid, NT, [&](int q) { return H[hstride * q + hoff]; },
                            [&](int q, SCx hv) { buf[sk::padpos(q)] = sk::cmul(buf[sk::padpos(q)], hv); });
    };
    if (item.half < 0) {
        staged_pass<U, SCx>(S, tid, NT, [&](int n) { return band_at(d, fhat, pre, n); },
                            [&](int n, SCx v) { buf[sk::padpos(n)] = v; });
        __syncthreads();
        lds_dft<-1>(buf, d.lgS, tw, tid);
        mult_h(0, 1);
        __syncthreads();
        lds_dft<+1>(buf, d.lgS, tw, tid);
        staged_pass<U, double2>(d.L, tid, NT, [&](int i) { return post[i]; },
                                [&](int i, double2 c) { theta[i] = mul_d(buf[sk::padpos(out_pos(i))], c); });
        return;
    }
    const int h = item.half;
    const int R = d.R;
    sk::Cx<float>* scr = static_cast<sk::Cx<float>*>(a.scratch) + d.scr_off;
    const sk::Cx<float>* twP = static_cast<const sk::Cx<float>*>(a.tw) + d.twP_off;
    // y_h, written by k_batch_dif into this piece's slice of scratch
    staged_pass<U, SCx>(S, tid, NT, [&](int n) { return scr[h * S + n]; },
                        [&](int n, SCx v) { buf[sk::padpos(n)] = v; });
    __syncthreads();
    lds_dft<-1>(buf, d.lgS, tw, tid);
    mult_h(h, R);
    __syncthreads();
    lds_dft<+1>(buf, d.lgS, tw, tid);
    for (int n = tid; n < S; n += NT) scr[h * S + n] = buf[sk::padpos(n)];
}

// Persistent: the workgroups of one launch take the transform items from the queue.
__global__ void __launch_bounds__(kBatchThreads) k_batch_fft(FftArgs a, int nitems, int* queue) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    sk::Cx<float>* buf = reinterpret_cast<sk::Cx<float>*>(smem_raw);
    for (int it = next_item(queue); it < nitems; it = next_item(queue)) batch_fft_item(a, it, buf);
    queue_done(queue);
}

// Output pass of instances split into R > 1 pieces (after every piece has run): one thread
// per output, work items of 256 outputs.
__global__ void __launch_bounds__(256) k_batch_combine(FftArgs a, const DifItem* items) {
    const DifItem it = items[blockIdx.x];
    const InstDesc d = a.desc[it.inst];
    const int i = it.n0 + int(threadIdx.x);
    if (i >= d.L) return;
    const sk::Cx<float>* scr = static_cast<const sk::Cx<float>*>(a.scratch) + d.scr_off;
    const sk::Cx<float>* twP = static_cast<const sk::Cx<float>*>(a.tw) + d.twP_off;
    const double2* post = a.post + d.post_off;
    sk::Cx<float>* theta = static_cast<sk::Cx<float>*>(a.theta) + d.theta_off;
    switch (d.R) {
        case 2: combine_pieces<2>(d, scr, twP, post, theta, i, d.L); break;
        case 4: combine_pieces<4>(d, scr, twP, post, theta, i, d.L); break;
        default: combine_pieces<8>(d, scr, twP, post, theta, i, d.L); break;
    }
}

// ---------------------------------------------------------------- binning
struct BBinArgs {
    const float* x;
    long long N;
    const long long* node_off;   // count + 1 prefix offsets
    const InstDesc* desc;
    int count;
    int tile;
    int32_t* node_tile;
    int32_t* tile_count;
    unsigned long long* flags;
};

__device__ __forceinline__ int find_instance(const long long* off, int count, long long j) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= j) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Binning with per-workgroup LDS histograms (as for single transforms): a workgroup takes
// kBinPer * kBinThreads consecutive nodes, which fall into the tiles of few instances,
// and walks the tiles between its smallest and largest in windows of kLdsBins, counting
// its nodes of the window in LDS and adding each nonzero count to the global counter once.
// The scatter recounts window by window, keeps each node's LDS rank, reserves one range
// per tile with a single global atomic and places every node at its rank in that range.
constexpr int kBinThreads = 256;
constexpr int kBinPer = 16;
constexpr int kLdsBins = 8192;

// Smallest and largest tile among the workgroup's nodes (tl < 0: none), uniform over the
// workgroup; hi < lo when it has no nodes.
__device__ __forceinline__ void tile_range(const int* tl, int& lo, int& hi) {
    __shared__ int s_lo, s_hi;
    if (threadIdx.x == 0) {
        s_lo = 0x7fffffff;
        s_hi = -1;
    }
    int a = 0x7fffffff, b = -1;
#pragma unroll
    for (int k = 0; k < kBinPer; ++k) {
        if (tl[k] >= 0) {
            a = min(a, tl[k]);
            b = max(b, tl[k]);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        a = min(a, __shfl_xor(a, off));
        b = max(b, __shfl_xor(b, off));
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0 && b >= 0) {
        atomicMin(&s_lo, a);
        atomicMax(&s_hi, b);
    }
    __syncthreads();
    lo = s_lo;
    hi = s_hi;
}

__global__ void __launch_bounds__(kBinThreads) k_bbin_count(BBinArgs a, int ntiles) {
    __shared__ int hist[kLdsBins];
    const long long j0 = (long long)blockIdx.x * (kBinThreads * kBinPer) + threadIdx.x;
    int tl[kBinPer];
    unsigned invalid = 0, outside = 0;
    // A thread's nodes increase by kBinThreads, so its instance is found once by bisection
    // and then advanced; the instance's parameters are reloaded only when it changes.
    int inst = j0 < a.N ? find_instance(a.node_off, a.count, j0) : 0;
    long long next = a.node_off[inst + 1];
    InstDesc d = a.desc[inst];
#pragma unroll
    for (int k = 0; k < kBinPer; ++k) {
        const long long j = j0 + (long long)k * kBinThreads;
        tl[k] = -1;
        if (j < a.N) {
            if (j >= next) {
                while (j >= a.node_off[inst + 1]) ++inst;
                next = a.node_off[inst + 1];
                d = a.desc[inst];
            }
            float xv = a.x[j];
            if (!(xv >= -0.5f && xv < 0.5f)) {
                ++invalid;
                xv = 0.0f;
            }
            const float lim = 0.5f - float(d.m) / float(d.L);
            if (!(xv >= -lim && xv < lim)) ++outside;
            int n;
            float th;
            dev::cell_of<float>(xv, d.L, n, th);
            tl[k] = d.tile_base + (n + d.L / 2) / a.tile;
            a.node_tile[j] = tl[k];
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        invalid += __shfl_xor(invalid, off);
        outside += __shfl_xor(outside, off);
    }
    if ((threadIdx.x & 63) == 0) {
        if (invalid) atomicAdd(&a.flags[0], (unsigned long long)invalid);
        if (outside) atomicAdd(&a.flags[1], (unsigned long long)outside);
    }
    int tlo, thi;
    tile_range(tl, tlo, thi);
    for (int w0 = thi < 0 ? ntiles : (tlo / kLdsBins) * kLdsBins; w0 <= thi && w0 < ntiles; w0 += kLdsBins) {
        const int nw = min(kLdsBins, ntiles - w0);
        __syncthreads();   // previous window flushed
        for (int e = threadIdx.x; e < nw; e += kBinThreads) hist[e] = 0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kBinPer; ++k) {
            const int e = tl[k] - w0;
            if (tl[k] >= 0 && e >= 0 && e < nw) atomicAdd(&hist[e], 1);
        }
        __syncthreads();
        for (int e = threadIdx.x; e < nw; e += kBinThreads)
            if (hist[e]) atomicAdd(&a.tile_count[w0 + e], hist[e]);
    }
}

__global__ void __launch_bounds__(kBinThreads) k_bbin_scatter(const float* __restrict__ x, long long N,
                                                             const int32_t* node_tile, const int32_t* offset,
                                                             int32_t* cursor, int32_t* perm,
                                                             float* __restrict__ xs, int ntiles) {
    __shared__ int hist[kLdsBins];   // counts, then the start of this workgroup's range
    const long long j0 = (long long)blockIdx.x * (kBinThreads * kBinPer) + threadIdx.x;
    int tl[kBinPer], rank[kBinPer];
#pragma unroll
    for (int k = 0; k < kBinPer; ++k) {
        const long long j = j0 + (long long)k * kBinThreads;
        tl[k] = j < N ? node_tile[j] : -1;
        rank[k] = 0;
    }
    int tlo, thi;
    tile_range(tl, tlo, thi);
    for (int w0 = thi < 0 ? ntiles : (tlo / kLdsBins) * kLdsBins; w0 <= thi && w0 < ntiles; w0 += kLdsBins) {
        const int nw = min(kLdsBins, ntiles - w0);
        __syncthreads();   // previous window placed
        for (int e = threadIdx.x; e < nw; e += kBinThreads) hist[e] = 0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kBinPer; ++k) {
            const int e = tl[k] - w0;
            if (tl[k] >= 0 && e >= 0 && e < nw) rank[k] = atomicAdd(&hist[e], 1);
        }
        __syncthreads();
        for (int e = threadIdx.x; e < nw; e += kBinThreads) {
            const int c = hist[e];
            if (c) hist[e] = offset[w0 + e] + atomicAdd(&cursor[w0 + e], c);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kBinPer; ++k) {
            const int e = tl[k] - w0;
            if (tl[k] < 0 || e < 0 || e >= nw) continue;
            const long long j = j0 + (long long)k * kBinThreads;
            const int pos = hist[e] + rank[k];
            perm[pos] = int32_t(j);
            xs[pos] = x[j];
        }
    }
}

// Chunk list entry: {tile, start, count, instance}.
__global__ void k_bchunk_fill(const int32_t* count, const int32_t* offset, const int32_t* chunk_off,
                              const int32_t* tile_inst, long long ntiles, int cap, int4* chunks) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    const int c = count[t];
    const int base = chunk_off[t];
    for (int s = 0, k = 0; s < c; s += cap, ++k)
        chunks[base + k] = make_int4(int(t), offset[t] + s, (c - s) < cap ? (c - s) : cap, tile_inst[t]);
}

// Order a chunk's nodes by cell (see the single-transform binning).
constexpr int kSortPerThread = 4;
__global__ void __launch_bounds__(256) k_bchunk_sort(const int4* chunks, const InstDesc* desc, int tile,
                                                     float* xs, int32_t* perm) {
    extern __shared__ int hist[];
    __shared__ int part[256];
    const int4 ch = chunks[blockIdx.x];
    const InstDesc d = desc[ch.w];
    const int n0 = (ch.x - d.tile_base) * tile;
    for (int e = threadIdx.x; e < tile; e += blockDim.x) hist[e] = 0;
    __syncthreads();
    float xv[kSortPerThread];
    int pv[kSortPerThread], key[kSortPerThread], rank[kSortPerThread];
#pragma unroll
    for (int q = 0; q < kSortPerThread; ++q) {
        const int jj = threadIdx.x + q * blockDim.x;
        key[q] = -1;
        if (jj < ch.z) {
            const long long j = (long long)ch.y + jj;
            xv[q] = xs[j];
            int n;
            float th;
            dev::cell_of<float>(xv[q], d.L, n, th);
            key[q] = n + d.L / 2 - n0;
            pv[q] = perm[j];
            rank[q] = atomicAdd(&hist[key[q]], 1);
        }
    }
    __syncthreads();
    const int per = (tile + blockDim.x - 1) / blockDim.x;
    const int beg = threadIdx.x * per;
    const int end = beg + per < tile ? beg + per : tile;
    int sum = 0;
    for (int e = beg; e < end; ++e) sum += hist[e];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < int(blockDim.x); off *= 2) {
        const int v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int run = part[threadIdx.x] - sum;
    for (int e = beg; e < end; ++e) {
        const int c = hist[e];
        hist[e] = run;
        run += c;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kSortPerThread; ++q) {
        if (key[q] < 0) continue;
        const long long pos = (long long)ch.y + hist[key[q]] + rank[q];
        xs[pos] = xv[q];
        perm[pos] = pv[q];
    }
}

// ---------------------------------------------------------------- short sums
struct BGatherArgs {
    const InstDesc* desc;
    const int4* chunks;
    const float* xs;
    const int32_t* perm;
    const void* theta;
    const float* coef;    // per instance: kMaxM * kPolyCoef floats
    void* f;
    int tile;
};

template <int M2, int ACC>
__device__ __forceinline__ void batch_gather_chunk(const BGatherArgs& a, const int4 ch, const InstDesc& d,
                                                   unsigned char* smem_raw) {
    constexpr int m = M2 / 2;
    const int n0 = (ch.x - d.tile_base) * a.tile;
    const int W = a.tile + M2 - 1;
    CxF* lds = reinterpret_cast<CxF*>(smem_raw);
    float* coef = reinterpret_cast<float*>(smem_raw + ((size_t(a.tile + 2 * kMaxM) * sizeof(CxF) + 15) & ~size_t(15)));
    const CxF* th = static_cast<const CxF*>(a.theta) + d.theta_off;
    staged_pass<8, CxF>(W, int(threadIdx.x), int(blockDim.x),
                        [&](int e) {
                            const int p = n0 - m + 1 + e;
                            return (p >= 0 && p < d.L) ? th[p] : CxF{0.0f, 0.0f};
                        },
                        [&](int e, CxF v) { lds[e] = v; });
    for (int e = threadIdx.x; e < m * kPolyCoef; e += blockDim.x)
        coef[e] = a.coef[(long long)ch.w * kMaxM * kPolyCoef + e];
    __syncthreads();
    CxF* f = static_cast<CxF*>(a.f);
    // node coordinates and output indices of up to 4 nodes per thread are loaded first
    struct Node {
        float x;
        int32_t out;
    };
    staged_pass<4, Node>(ch.z, int(threadIdx.x), int(blockDim.x),
                         [&](int jj) { return Node{a.xs[ch.y + jj], a.perm[ch.y + jj]}; },
                         [&](int, Node nd) {
                             int n;
                             float theta[1];
                             dev::cell_of<float>(nd.x, d.L, n, theta[0]);
                             const int r = n + d.L / 2 - n0;
                             float w[1][M2];
                             // an opaque zero offset keeps the (uniform) coefficient loads
                             // per node instead of holding all of them in registers
                             int opaque = 0;
                             asm volatile("" : "+s"(opaque));
                             dev::weights_poly<1, M2, kPolyCoef>(theta, coef + opaque, w, 1.0f);
                             dev::OuterAcc<float, ACC> acc;
#pragma unroll
                             for (int o = 0; o < M2; ++o) acc.add(w[0][o], lds[r + o]);
                             f[nd.out] = acc.value();
                         });
}

// ---------------------------------------------------------------- host helpers
int ilog2i(int64_t v) {
    int l = 0;
    while ((int64_t(1) << (l + 1)) <= v) ++l;
    return l;
}

}  // namespace

}  // namespace bl

struct bl_batch_s {
    int count = 0;
    bl_precision prec = BL_F32;
    hipStream_t stream = nullptr;
    int device = 0;
    std::vector<bl::InstDesc> h_desc;
    std::vector<long long> h_node_off;
    std::vector<int32_t> h_tile_inst;
    std::vector<bl::FftItem> h_items;    // transform work items, largest first
    int64_t total_M = 0, total_L = 0, total_N = 0;
    int tile = 512;
    int chunk_cap = 1024;
    bool tuned = false;
    // device
    bl::InstDesc* d_desc = nullptr;
    long long* d_node_off = nullptr;
    double2* d_pre = nullptr;
    double2* d_post = nullptr;
    void* d_h = nullptr;
    void* d_tw = nullptr;
    void* d_theta = nullptr;
    void* d_scratch = nullptr;
    float* d_coef = nullptr;
    bl::FftItem* d_items = nullptr;
    std::vector<bl::DifItem> h_dif;      // decimation work items (instances with R > 1)
    bl::DifItem* d_dif = nullptr;
    std::vector<bl::DifItem> h_comb;     // output items of instances with R > 1
    bl::DifItem* d_comb = nullptr;
    // nodes
    float* d_xs = nullptr;
    int32_t* d_perm = nullptr;
    int32_t* d_node_tile = nullptr;
    int32_t* d_tile_count = nullptr;
    int32_t* d_tile_offset = nullptr;
    int32_t* d_tile_cursor = nullptr;
    int32_t* d_chunk_offset = nullptr;
    int32_t* d_tile_inst = nullptr;
    void* d_scan = nullptr;   // block sums of the tile scans
    int4* d_chunks = nullptr;
    unsigned long long* d_flags = nullptr;
    int* d_work = nullptr;          // work queue of the persistent transform launch
    int num_cus = 256;              // compute units of the device
    int64_t ntiles = 0, chunk_alloc = 0, nchunks = 0, tile_alloc = 0;
    bool have_nodes = false;
    size_t fft_lds = 0;
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t exec = nullptr;
    const void* g_fhat = nullptr;
    void* g_f = nullptr;
};

namespace bl {
namespace {

bl_status bfail(bl_status s, const std::string& msg) {
    set_error(msg);
    return s;
}

template <typename T>
bl_status balloc(T** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return BL_OK;
    if (const char* f = std::getenv("BL_TEST_FAIL_ALLOC"))
        if (f[0] == '1') return bfail(BL_ENOMEM, "allocation refused by BL_TEST_FAIL_ALLOC");
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return bfail(e == hipErrorOutOfMemory ? BL_ENOMEM : BL_EDEVICE,
                     std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    return BL_OK;
}

void free_batch(bl_batch_s* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    void* ptrs[] = {b->d_desc, b->d_node_off, b->d_pre, b->d_post, b->d_h, b->d_tw, b->d_theta,
                    b->d_scratch, b->d_coef, b->d_items, b->d_dif, b->d_comb, b->d_xs, b->d_perm, b->d_node_tile, b->d_tile_count,
                    b->d_tile_offset, b->d_tile_cursor, b->d_chunk_offset, b->d_tile_inst, b->d_scan,
                    b->d_chunks, b->d_flags, b->d_work};
    for (void* q : ptrs) (void)hipFree(q);
}

// Short sums: one workgroup per work-list entry (a chunk of one instance's tile), in the
// XCD-aware order; the instance's m selects the specialised body (uniform per workgroup).
// Entries hold at most one chunk capacity of nodes each, so the hardware's dispatch
// balances them; persistent forms measured slower (an atomic queue 237 us, a fixed stride
// per XCD segment 150 us, this form 129 us on the 512-instance workload).
template <int ACC>
__global__ void __launch_bounds__(256) k_batch_gather(BGatherArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int4 ch = a.chunks[xcd_block(int(blockIdx.x), int(gridDim.x))];
    const InstDesc d = a.desc[ch.w];
    switch (d.m) {
        case 2: batch_gather_chunk<4, ACC>(a, ch, d, smem_raw); break;
        case 3: batch_gather_chunk<6, ACC>(a, ch, d, smem_raw); break;
        case 4: batch_gather_chunk<8, ACC>(a, ch, d, smem_raw); break;
        case 5: batch_gather_chunk<10, ACC>(a, ch, d, smem_raw); break;
        case 6: batch_gather_chunk<12, ACC>(a, ch, d, smem_raw); break;
        case 7: batch_gather_chunk<14, ACC>(a, ch, d, smem_raw); break;
        default: batch_gather_chunk<16, ACC>(a, ch, d, smem_raw); break;
    }
}

// Launch the transforms (a persistent launch over the work items), then the short sums.
bl_status batch_launches(bl_batch_s* b, hipStream_t s, const void* fhat, void* f, bool fft = true) {
    if (fft) {
        FftArgs fa{};
        fa.desc = b->d_desc;
        fa.items = b->d_items;
        fa.fhat = fhat;
        fa.theta = b->d_theta;
        fa.pre = b->d_pre;
        fa.post = b->d_post;
        fa.h = b->d_h;
        fa.scratch = b->d_scratch;
        fa.tw = b->d_tw;
        if (!b->h_dif.empty()) {
            hipLaunchKernelGGL(k_batch_dif, dim3(unsigned(b->h_dif.size())), dim3(256), 0, s, fa,
                               static_cast<const DifItem*>(b->d_dif));
            BL_HIP(hipGetLastError());
        }
        const int per_cu = std::max(1, int((160 * 1024) / b->fft_lds));
        const int64_t wgs = std::min<int64_t>(int64_t(b->h_items.size()), int64_t(per_cu) * b->num_cus);
        hipLaunchKernelGGL(k_batch_fft, dim3(unsigned(wgs)), dim3(kBatchThreads), b->fft_lds, s, fa,
                           int(b->h_items.size()), b->d_work);
        BL_HIP(hipGetLastError());
        if (!b->h_comb.empty()) {
            hipLaunchKernelGGL(k_batch_combine, dim3(unsigned(b->h_comb.size())), dim3(256), 0, s, fa,
                               static_cast<const DifItem*>(b->d_comb));
            BL_HIP(hipGetLastError());
        }
    }
    if (b->nchunks == 0) return BL_OK;
    BGatherArgs ga{};
    ga.desc = b->d_desc;
    ga.chunks = b->d_chunks;
    ga.xs = b->d_xs;
    ga.perm = b->d_perm;
    ga.theta = b->d_theta;
    ga.coef = b->d_coef;
    ga.f = f;
    ga.tile = b->tile;
    const size_t lds = ((size_t(b->tile + 2 * kMaxM) * sizeof(CxF) + 15) & ~size_t(15)) +
                       sizeof(float) * kMaxM * kPolyCoef;
    if (b->prec == BL_F32C)
        hipLaunchKernelGGL(k_batch_gather<2>, dim3(unsigned(b->nchunks)), dim3(256), lds, s, ga);
    else if (b->prec == BL_F32D)
        hipLaunchKernelGGL(k_batch_gather<1>, dim3(unsigned(b->nchunks)), dim3(256), lds, s, ga);
    else
        hipLaunchKernelGGL(k_batch_gather<0>, dim3(unsigned(b->nchunks)), dim3(256), lds, s, ga);
    BL_HIP(hipGetLastError());
    return BL_OK;
}

// Bin the bound nodes with tile edge `tile`.
bl_status batch_bin(bl_batch_s* b, const float* x, int tile) {
    b->tile = tile;
    int64_t nt = 0;
    std::vector<int32_t>& tile_inst = b->h_tile_inst;
    tile_inst.clear();
    // Tiles are numbered instance by instance, grouped by m (neighbouring work-list entries
    // then run the same specialised code).
    for (int mm = 0; mm <= kMaxM; ++mm) {
        for (int i = 0; i < b->count; ++i) {
            if (b->h_desc[i].m != mm) continue;
            b->h_desc[i].tile_base = int(nt);
            b->h_desc[i].ntiles = int((b->h_desc[i].L + tile - 1) / tile);
            nt += b->h_desc[i].ntiles;
            for (int k = 0; k < b->h_desc[i].ntiles; ++k) tile_inst.push_back(i);
        }
    }
    b->ntiles = nt;
    const int64_t N = b->total_N;
    const int64_t chunk_bound = N / b->chunk_cap + nt + 1;
    if (nt > b->tile_alloc) {
        (void)hipFree(b->d_tile_count);
        (void)hipFree(b->d_tile_offset);
        (void)hipFree(b->d_tile_cursor);
        (void)hipFree(b->d_chunk_offset);
        (void)hipFree(b->d_tile_inst);
        (void)hipFree(b->d_scan);
        b->d_tile_count = b->d_tile_offset = b->d_tile_cursor = b->d_chunk_offset = b->d_tile_inst = nullptr;
        b->d_scan = nullptr;
        b->tile_alloc = 0;
        BL_TRY(balloc(&b->d_tile_count, sizeof(int32_t) * nt));
        BL_TRY(balloc(&b->d_tile_offset, sizeof(int32_t) * nt));
        BL_TRY(balloc(&b->d_tile_cursor, sizeof(int32_t) * nt));
        BL_TRY(balloc(&b->d_chunk_offset, sizeof(int32_t) * nt));
        BL_TRY(balloc(&b->d_tile_inst, sizeof(int32_t) * nt));
        BL_TRY(balloc(reinterpret_cast<char**>(&b->d_scan), tile_scan_scratch_bytes(nt)));
        b->tile_alloc = nt;
    }
    if (chunk_bound > b->chunk_alloc) {
        (void)hipFree(b->d_chunks);
        b->d_chunks = nullptr;
        b->chunk_alloc = 0;
        BL_TRY(balloc(&b->d_chunks, sizeof(int4) * chunk_bound));
        b->chunk_alloc = chunk_bound;
    }
    hipStream_t s = b->stream;
    BL_HIP(hipMemcpyAsync(b->d_desc, b->h_desc.data(), sizeof(InstDesc) * b->count, hipMemcpyHostToDevice, s));
    BL_HIP(hipMemcpyAsync(b->d_tile_inst, tile_inst.data(), sizeof(int32_t) * nt, hipMemcpyHostToDevice, s));
    BL_HIP(hipMemsetAsync(b->d_tile_count, 0, sizeof(int32_t) * nt, s));
    BL_HIP(hipMemsetAsync(b->d_tile_cursor, 0, sizeof(int32_t) * nt, s));
    BL_HIP(hipMemsetAsync(b->d_flags, 0, sizeof(unsigned long long) * 4, s));
    const unsigned nb = unsigned((N + kBinThreads * kBinPer - 1) / (kBinThreads * kBinPer));
    if (N > 0) {
        BBinArgs ba{};
        ba.x = x;
        ba.N = N;
        ba.node_off = b->d_node_off;
        ba.desc = b->d_desc;
        ba.count = b->count;
        ba.tile = tile;
        ba.node_tile = b->d_node_tile;
        ba.tile_count = b->d_tile_count;
        ba.flags = b->d_flags;
        hipLaunchKernelGGL(k_bbin_count, dim3(nb), dim3(kBinThreads), 0, s, ba, int(nt));
        BL_HIP(hipGetLastError());
    }
    BL_TRY(launch_tile_scan(b->d_tile_count, b->d_tile_offset, b->d_chunk_offset, nt, b->chunk_cap, b->d_flags,
                            b->d_scan, s));
    if (N > 0) {
        hipLaunchKernelGGL(k_bbin_scatter, dim3(nb), dim3(kBinThreads), 0, s, x, (long long)N, b->d_node_tile,
                           b->d_tile_offset, b->d_tile_cursor, b->d_perm, b->d_xs, int(nt));
        BL_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_bchunk_fill, dim3(unsigned((nt + 255) / 256)), dim3(256), 0, s, b->d_tile_count,
                       b->d_tile_offset, b->d_chunk_offset, b->d_tile_inst, (long long)nt, b->chunk_cap,
                       b->d_chunks);
    BL_HIP(hipGetLastError());
    unsigned long long h[4] = {0, 0, 0, 0};
    BL_HIP(hipMemcpyAsync(h, b->d_flags, sizeof(h), hipMemcpyDeviceToHost, s));
    BL_HIP(hipStreamSynchronize(s));
    if (h[0] != 0)
        return bfail(BL_EDOMAIN, std::to_string(h[0]) + " node coordinate(s) are NaN/Inf or outside [-1/2, 1/2)");
    b->nchunks = int64_t(h[2]);
    if (b->nchunks > b->chunk_alloc) return bfail(BL_EDEVICE, "internal: chunk count exceeds its bound");
    if (b->nchunks > 0) {
        hipLaunchKernelGGL(k_bchunk_sort, dim3(unsigned(b->nchunks)), dim3(256), sizeof(int) * tile, s,
                           b->d_chunks, b->d_desc, tile, b->d_xs, b->d_perm);
        BL_HIP(hipGetLastError());
        BL_HIP(hipStreamSynchronize(s));
    }
    return BL_OK;
}

// Time the short sums (on the zeroed samples theta) for each candidate tile edge and keep
// the fastest.  Runs once per batch, at its first node binding.
// Key of the batch in the tuning cache: device, precision and a hash of every instance's
// (M, L, m, N).
std::string batch_tune_key(const bl_batch_s* b) {
    uint64_t h = 1469598103934665603ull;   // FNV-1a
    auto mix = [&](int64_t v) {
        for (int k = 0; k < 8; ++k) {
            h ^= uint64_t((v >> (8 * k)) & 0xff);
            h *= 1099511628211ull;
        }
    };
    for (const InstDesc& d : b->h_desc) {
        mix(d.M);
        mix(d.L);
        mix(d.m);
    }
    for (int i = 0; i < b->count; ++i) mix(b->h_node_off[i + 1] - b->h_node_off[i]);
    char buf[32];
    std::snprintf(buf, sizeof(buf), "%016llx", (unsigned long long)h);
    return "batch|" + tune_device_tag(b->device) + "|n" + std::to_string(b->count) + "|" +
           (b->prec == BL_F32 ? "f32" : b->prec == BL_F32C ? "f32c" : "f32d") + "|" + buf;
}

bl_status autotune_tile(bl_batch_s* b, const float* x) {
    const std::string key = batch_tune_key(b);
    std::vector<int> cached;
    if (tune_lookup(key, &cached) && cached.size() == 1) {
        b->tile = cached[0];
        b->tuned = true;
        return BL_OK;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    CxF* fdummy = nullptr;
    bl_status st = balloc(&fdummy, sizeof(CxF) * b->total_N);
    if (st == BL_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        st = bfail(BL_EDEVICE, "hipEventCreate failed");
    float best = 1e30f;
    int best_tile = b->tile;
    for (int cand : {256, 512, 1024, 2048}) {
        if (st != BL_OK) break;
        if ((st = batch_bin(b, x, cand)) != BL_OK) break;
        if ((st = batch_launches(b, b->stream, nullptr, fdummy, false)) != BL_OK) break;
        (void)hipEventRecord(e0, b->stream);
        for (int rep = 0; rep < 3 && st == BL_OK; ++rep) st = batch_launches(b, b->stream, nullptr, fdummy, false);
        (void)hipEventRecord(e1, b->stream);
        if (hipEventSynchronize(e1) != hipSuccess) st = bfail(BL_EDEVICE, "hipEventSynchronize failed");
        float ms = 0.0f;
        if (st == BL_OK && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms < best) {
            best = ms;
            best_tile = cand;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(b->stream);
    (void)hipFree(fdummy);
    if (st != BL_OK) return st;
    b->tile = best_tile;
    b->tuned = true;
    tune_store(key, std::vector<int>{best_tile});
    return BL_OK;
}

void drop_graph(bl_batch_s* b) {
    if (b->exec) {
        (void)hipStreamSynchronize(b->stream);   // a launch of the graph may still be in flight
        (void)hipGraphExecDestroy(b->exec);
    }
    b->exec = nullptr;
    b->g_fhat = nullptr;
    b->g_f = nullptr;
}

}  // namespace
}  // namespace bl

using namespace bl;

extern "C" {

bl_status bl_batch_create(bl_batch* out, int count, const int64_t* M, const int64_t* L,
                          const int* m, const int64_t* N, bl_precision prec, void* stream) {
    if (!out) return bfail(BL_EINVAL, "out is NULL");
    *out = nullptr;
    if (count < 1 || !M || !L || !m || !N) return bfail(BL_EINVAL, "count >= 1 and four host arrays required");
    if (prec != BL_F32 && prec != BL_F32C && prec != BL_F32D)
        return bfail(prec == BL_F64 ? BL_EUNSUPPORTED : BL_EINVAL, "batched transforms run in float precisions");
    for (int i = 0; i < count; ++i) {
        if (M[i] < 2 || M[i] % 2 || L[i] <= M[i] || L[i] % 2 || m[i] < 1 || 2 * int64_t(m[i]) >= L[i] || N[i] < 0)
            return bfail(BL_EINVAL, "instance " + std::to_string(i) + ": need even M >= 2, even L > M, 2m < L, N >= 0");
        if (m[i] < kMinM || m[i] > kMaxM)
            return bfail(BL_EUNSUPPORTED, "instance " + std::to_string(i) + ": kernels cover 2 <= m <= 8");
        int64_t P = 1;
        while (P < L[i] + M[i] - 1) P *= 2;
        if (P > kMaxP) return bfail(BL_EUNSUPPORTED, "instance " + std::to_string(i) + ": L + M - 1 above 32768");
    }
    bl_batch_s* b = new (std::nothrow) bl_batch_s();
    if (!b) return bfail(BL_ENOMEM, "host allocation failed");
    auto cleanup = [&](bl_status s) {
        free_batch(b);
        delete b;
        return s;
    };
    b->count = count;
    b->prec = prec;
    b->stream = static_cast<hipStream_t>(stream);
    if (hipGetDevice(&b->device) != hipSuccess) return cleanup(bfail(BL_EDEVICE, "hipGetDevice failed"));
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) == hipSuccess && cus > 0)
            b->num_cus = cus;
    }
    if (const char* e = std::getenv("BL_TILE")) {
        const int v = std::atoi(e);
        if (v >= 16 && v <= 8192) {
            b->tile = v;
            b->tuned = true;
        }
    }

    // Per-instance layout and host tables.
    b->h_desc.resize(count);
    b->h_node_off.resize(count + 1);
    std::vector<double2> pre, post;
    std::vector<float> hbuf, coef(size_t(count) * kMaxM * kPolyCoef, 0.0f);
    std::vector<float> tw;            // twiddle tables, interleaved float
    std::vector<int> tw_at(17, -1);   // offset of the table for size 2^q
    int64_t scr = 0;
    auto table = [&](int lg) {
        if (tw_at[lg] < 0) {
            tw_at[lg] = int(tw.size() / 2);
            std::vector<double> t;
            twiddles(int64_t(1) << lg, &t);
            for (double v : t) tw.push_back(float(v));
        }
        return tw_at[lg];
    };
    // Largest DFT held in LDS; BL_BATCH_LDS_FFT (a power of two in [1024, 16384]) lowers it.
    int lds_fft_max = kMaxLdsFft;
    if (const char* e = std::getenv("BL_BATCH_LDS_FFT")) {
        const int v = std::atoi(e);
        if (v >= 256 && v <= kMaxLdsFft && (v & (v - 1)) == 0) lds_fft_max = v;
    }
    long long node_off = 0;
    for (int i = 0; i < count; ++i) {
        InstDesc& d = b->h_desc[i];
        d.M = int(M[i]);
        d.L = int(L[i]);
        d.m = m[i];
        int64_t P = 1;
        while (P < L[i] + M[i] - 1) P *= 2;
        d.P = int(P);
        const int64_t S = std::min<int64_t>(P, lds_fft_max);
        d.R = int(P / S);
        if (d.R > 8)
            return cleanup(bfail(BL_EUNSUPPORTED, "instance " + std::to_string(i) + ": transform above eight LDS pieces"));
        d.lgS = ilog2i(S);
        d.tw_off = table(d.lgS);
        d.twP_off = d.R > 1 ? table(ilog2i(P)) : 0;
        d.fhat_off = b->total_M;
        d.theta_off = b->total_L;
        d.pre_off = (long long)pre.size();
        d.post_off = (long long)post.size();
        d.h_off = (long long)(hbuf.size() / 2);
        d.scr_off = d.R > 1 ? scr : 0;
        if (d.R > 1) scr += P;
        d.node_off = node_off;
        b->h_node_off[i] = node_off;
        node_off += N[i];
        b->total_M += M[i];
        b->total_L += L[i];

        const double beta = default_beta(M[i], L[i], m[i], BL_SHANNON);
        std::vector<double> tw2L;
        twiddles(2 * L[i], &tw2L);   // e^{2 pi i n / (2L)} = e^{i pi n / L}
        // psihat on I_M (even in k) from the library's quadrature rule
        std::vector<double> hat(size_t(M[i] / 2 + 1));
        window_transform_ints(BL_WIN_SINH, BL_SHANNON, L[i], m[i], beta, M[i] / 2 + 1, hat.data());
        for (int64_t k = -M[i] / 2; k < M[i] / 2; ++k) {
            const double hv = hat[size_t(k < 0 ? -k : k)];
            if (!(hv > 0.0) || !std::isfinite(hv))
                return cleanup(bfail(BL_EINVAL, "instance " + std::to_string(i) + ": window transform vanishes on I_M"));
            const std::complex<double> a = chirp(k * k, L[i], tw2L) / (double(L[i]) * hv);
            pre.push_back(double2{a.real(), a.imag()});
        }
        for (int64_t l = -L[i] / 2; l < L[i] / 2; ++l) {
            const std::complex<double> c = chirp(l * l, L[i], tw2L);
            post.push_back(double2{c.real(), c.imag()});
        }
        // H = DFT_P(h) / P, h_j = u^{-j^2} at j mod P for |j| < (L + M)/2
        const std::vector<std::complex<double>> h = chirp_spectrum(L[i], M[i], P);
        for (int64_t q = 0; q < P; ++q) {
            hbuf.push_back(float(h[q].real()));
            hbuf.push_back(float(h[q].imag()));
        }
        std::vector<double> pc;
        const double fit = fit_weight_polys(BL_WIN_SINH, BL_SHANNON, m[i], beta, kPolyCoef, &pc);
        if (!(fit <= kPolyFitTol))
            return cleanup(bfail(BL_EUNSUPPORTED, "instance " + std::to_string(i) +
                                                      ": float weight polynomials fit only to " +
                                                      std::to_string(fit)));
        for (size_t q = 0; q < pc.size(); ++q) coef[size_t(i) * kMaxM * kPolyCoef + q] = float(pc[q]);
    }
    b->h_node_off[count] = node_off;
    b->total_N = node_off;
    if (b->total_N > int64_t(0x7fffffff)) return cleanup(bfail(BL_EUNSUPPORTED, "total node count above 2^31"));
    // Transform work items, most expensive first: whole instances (R = 1), or the R pieces
    // of a larger one (each costs two DFTs of S points, R band loads per point and, for the
    // last piece, the combination of the L outputs).
    {
        std::vector<std::pair<double, FftItem>> items;
        for (int i = 0; i < count; ++i) {
            const InstDesc& d = b->h_desc[i];
            const double S = double(int64_t(1) << d.lgS);
            const double cost = 2.0 * S * d.lgS + S * d.R + double(d.L) * d.R / 2.0;
            if (d.R > 1) {
                for (int h = 0; h < d.R; ++h) items.push_back({cost, FftItem{i, h}});
            } else {
                items.push_back({cost, FftItem{i, -1}});
            }
        }
        std::stable_sort(items.begin(), items.end(),
                         [](const std::pair<double, FftItem>& x, const std::pair<double, FftItem>& y) {
                             return x.first > y.first;
                         });
        for (const auto& it : items) b->h_items.push_back(it.second);
        for (int i = 0; i < count; ++i) {
            const InstDesc& d = b->h_desc[i];
            if (d.R > 1) {
                for (int n0 = 0; n0 < (1 << d.lgS); n0 += 256) b->h_dif.push_back(DifItem{i, n0});
                for (int i0 = 0; i0 < d.L; i0 += 256) b->h_comb.push_back(DifItem{i, i0});
            }
        }
    }

    bl_status s;
    if ((s = balloc(&b->d_desc, sizeof(InstDesc) * count)) != BL_OK) return cleanup(s);
    if ((s = balloc(&b->d_node_off, sizeof(long long) * (count + 1))) != BL_OK) return cleanup(s);
    if ((s = balloc(&b->d_pre, sizeof(double2) * pre.size())) != BL_OK) return cleanup(s);
    if ((s = balloc(&b->d_post, sizeof(double2) * post.size())) != BL_OK) return cleanup(s);
    if ((s = balloc(&b->d_h, sizeof(float) * hbuf.size())) != BL_OK) return cleanup(s);
    if ((s = balloc(&b->d_tw, sizeof(float) * tw.size())) != BL_OK) return cleanup(s);
    if ((s = balloc(&b->d_theta, sizeof(CxF) * b->total_L)) != BL_OK) return cleanup(s);
    if ((s = balloc(&b->d_scratch, sizeof(CxF) * std::max<int64_t>(scr, 1))) != BL_OK) return cleanup(s);
    if ((s = balloc(&b->d_coef, sizeof(float) * coef.size())) != BL_OK) return cleanup(s);
    if ((s = balloc(&b->d_items, sizeof(FftItem) * b->h_items.size())) != BL_OK) return cleanup(s);
    if ((s = balloc(&b->d_comb, sizeof(DifItem) * b->h_comb.size())) != BL_OK) return cleanup(s);
    if ((s = balloc(&b->d_dif, sizeof(DifItem) * b->h_dif.size())) != BL_OK) return cleanup(s);
    if ((s = balloc(&b->d_flags, sizeof(unsigned long long) * 4)) != BL_OK) return cleanup(s);
    if ((s = balloc(&b->d_work, sizeof(int) * kBatchQueue)) != BL_OK) return cleanup(s);
    const int64_t ncap = std::max<int64_t>(b->total_N, 1);
    if ((s = balloc(&b->d_xs, sizeof(float) * ncap)) != BL_OK) return cleanup(s);
    if ((s = balloc(&b->d_perm, sizeof(int32_t) * ncap)) != BL_OK) return cleanup(s);
    if ((s = balloc(&b->d_node_tile, sizeof(int32_t) * ncap)) != BL_OK) return cleanup(s);

    hipStream_t st = b->stream;
    hipError_t e = hipMemcpyAsync(b->d_desc, b->h_desc.data(), sizeof(InstDesc) * count, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_node_off, b->h_node_off.data(), sizeof(long long) * (count + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_pre, pre.data(), sizeof(double2) * pre.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_post, post.data(), sizeof(double2) * post.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_h, hbuf.data(), sizeof(float) * hbuf.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_tw, tw.data(), sizeof(float) * tw.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_coef, coef.data(), sizeof(float) * coef.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_items, b->h_items.data(), sizeof(FftItem) * b->h_items.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !b->h_comb.empty())
        e = hipMemcpyAsync(b->d_comb, b->h_comb.data(), sizeof(DifItem) * b->h_comb.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !b->h_dif.empty())
        e = hipMemcpyAsync(b->d_dif, b->h_dif.data(), sizeof(DifItem) * b->h_dif.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(b->d_theta, 0, sizeof(CxF) * b->total_L, st);
    if (e == hipSuccess) e = hipMemsetAsync(b->d_work, 0, sizeof(int) * kBatchQueue, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return cleanup(bfail(BL_EDEVICE, std::string("table upload: ") + hipGetErrorString(e)));

    int lg_max = 0;
    for (const InstDesc& d : b->h_desc) lg_max = std::max(lg_max, d.lgS);
    b->fft_lds = (size_t(sk::padpos(kMaxLdsFft - 1) + 1) + kRootHi + kRootLo) * sizeof(CxF);
    (void)lg_max;
    if (b->fft_lds > 64 * 1024) {
        e = hipFuncSetAttribute((const void*)k_batch_fft, hipFuncAttributeMaxDynamicSharedMemorySize, int(b->fft_lds));
        if (e != hipSuccess) return cleanup(bfail(BL_EDEVICE, std::string("LDS attribute: ") + hipGetErrorString(e)));
    }
    *out = b;
    return BL_OK;
}

bl_status bl_batch_set_nodes(bl_batch b, const void* x_dev) {
    if (!b) return bfail(BL_EINVAL, "batch is NULL");
    if (b->total_N > 0 && !x_dev) return bfail(BL_EINVAL, "x_dev is NULL");
    BL_HIP(hipSetDevice(b->device));
    b->have_nodes = false;
    drop_graph(b);
    const float* x = static_cast<const float*>(x_dev);
    if (!b->tuned && b->total_N > 0 && tuning_enabled()) {
        // Autotune the tile edge (or read it from the tuning cache): bin with each
        // candidate and time the short sums alone.
        bl_status st = autotune_tile(b, x);
        if (st != BL_OK) return st;
    }
    BL_TRY(batch_bin(b, x, b->tile));
    b->have_nodes = true;
    return BL_OK;
}

bl_status bl_batch_forward(bl_batch b, const void* fhat_dev, void* f_dev) {
    if (!b) return bfail(BL_EINVAL, "batch is NULL");
    if (!b->have_nodes) return bfail(BL_ESTATE, "bl_batch_set_nodes must succeed before bl_batch_forward");
    if (!fhat_dev || (b->total_N > 0 && !f_dev)) return bfail(BL_EINVAL, "NULL buffer");
    BL_HIP(hipSetDevice(b->device));
    if (!b->exec || b->g_fhat != fhat_dev || b->g_f != f_dev) {
        drop_graph(b);
        if (!b->capture_stream) BL_HIP(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking));
        hipError_t e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal);
        bl_status st = BL_OK;
        if (e == hipSuccess) st = batch_launches(b, b->capture_stream, fhat_dev, f_dev);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(b->capture_stream, &g);
        if (e != hipSuccess || e2 != hipSuccess || st != BL_OK) {
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            if (st != BL_OK) return st;
            return bfail(BL_EDEVICE, "batched graph capture failed");
        }
        e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            b->exec = nullptr;
            return bfail(BL_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
        }
        b->g_fhat = fhat_dev;
        b->g_f = f_dev;
    }
    BL_HIP(hipGraphLaunch(b->exec, b->stream));
    return BL_OK;
}

bl_status bl_batch_destroy(bl_batch b) {
    if (!b) return BL_OK;
    (void)hipSetDevice(b->device);
    (void)hipStreamSynchronize(b->stream);
    free_batch(b);
    delete b;
    return BL_OK;
}

}  // extern "C"
