// Batched d = 1 transforms (Algorithm 4.2) of many independent instances with their own
// (M_i, L_i, m_i, N_i), executed as one hipGraph of two kernels.
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
// One workgroup per instance runs its two DFTs in LDS (size P <= 16384); for P = 32768 one
// radix-2 split through global scratch reduces them to four LDS DFTs of P/2.
//
// Step 3 runs one workgroup per work chunk of the instances' node tiles, as in the
// single-transform short sums, with each chunk's instance parameters (L, m, window
// polynomials) read from a descriptor table.
#include <algorithm>
#include <cmath>
#include <complex>
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

constexpr int kBatchThreads = 1024;
constexpr int kMaxLdsFft = 16384;      // largest DFT held in LDS (float complex)
constexpr int kMaxP = 32768;

struct InstDesc {
    int M, L, m, P;
    int split;           // 1: P = 2 S, one radix-2 split through scratch
    int lgS;             // log2 of the LDS DFT size S (P or P/2)
    int tw_off;          // twiddle table e^{2 pi i n / S}, n < S
    int twP_off;         // twiddle table e^{2 pi i n / P}, n < P (split instances)
    long long fhat_off;  // band samples (M complex)
    long long theta_off; // samples theta (L complex, centred)
    long long pre_off;   // a-factor times chirp, M double complex
    long long post_off;  // chirp u^{l^2}, L double complex
    long long h_off;     // H, P float complex
    long long scr_off;   // scratch (P float complex) for split instances
    long long node_off;  // first node of the instance
    int tile_base;       // first global tile of the instance
    int ntiles;
};

// ---------------------------------------------------------------- LDS DFT
// In-place radix-4 (+ a final radix-2) Stockham DFT of size S = 2^lgS on an LDS buffer
// indexed through padpos; kBatchThreads threads, up to 16 values each per stage.
template <int DIR, int RAD>
__device__ __forceinline__ void lds_stage(sk::Cx<float>* buf, int S, int Ns,
                                          const sk::Cx<float>* __restrict__ tw, int tid) {
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

template <int DIR>
__device__ void lds_dft(sk::Cx<float>* buf, int lgS, const sk::Cx<float>* __restrict__ tw, int tid) {
    const int S = 1 << lgS;
    int Ns = 1, lg = lgS;
    while (lg >= 2) {
        lds_stage<DIR, 4>(buf, S, Ns, tw, tid);
        Ns *= 4;
        lg -= 2;
    }
    if (lg == 1) lds_stage<DIR, 2>(buf, S, Ns, tw, tid);
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

struct FftArgs {
    const InstDesc* desc;
    const void* fhat;
    void* theta;
    const double2* pre;
    const double2* post;
    const void* h;
    void* scratch;
    const void* tw;
};

__global__ void __launch_bounds__(kBatchThreads) k_batch_fft(FftArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    sk::Cx<float>* buf = reinterpret_cast<sk::Cx<float>*>(smem_raw);
    const InstDesc d = a.desc[blockIdx.x];
    const int tid = threadIdx.x;
    const int S = 1 << d.lgS;
    const sk::Cx<float>* fhat = static_cast<const sk::Cx<float>*>(a.fhat) + d.fhat_off;
    const double2* pre = a.pre + d.pre_off;
    const double2* post = a.post + d.post_off;
    const sk::Cx<float>* H = static_cast<const sk::Cx<float>*>(a.h) + d.h_off;
    const sk::Cx<float>* tw = static_cast<const sk::Cx<float>*>(a.tw) + d.tw_off;
    sk::Cx<float>* theta = static_cast<sk::Cx<float>*>(a.theta) + d.theta_off;

    if (!d.split) {
        for (int n = tid; n < S; n += kBatchThreads) buf[sk::padpos(n)] = band_at(d, fhat, pre, n);
        __syncthreads();
        lds_dft<-1>(buf, d.lgS, tw, tid);
        for (int q = tid; q < S; q += kBatchThreads) buf[sk::padpos(q)] = sk::cmul(buf[sk::padpos(q)], H[q]);
        __syncthreads();
        lds_dft<+1>(buf, d.lgS, tw, tid);
        for (int i = tid; i < d.L; i += kBatchThreads) {
            int n = i - d.L / 2;
            n += (n < 0) ? d.P : 0;
            theta[i] = mul_d(buf[sk::padpos(n)], post[i]);
        }
        return;
    }
    // P = 2S: X[2q + h] = DFT_S(y_h)[q] with y_0[n] = b[n] + b[n+S],
    // y_1[n] = (b[n] - b[n+S]) e^{-2 pi i n/P}; the inverse is z[n] = E[n] + e^{2 pi i n/P} O[n]
    // and z[n + S] = E[n] - e^{2 pi i n/P} O[n] with E, O the inverse DFTs of the halves.
    sk::Cx<float>* scr = static_cast<sk::Cx<float>*>(a.scratch) + d.scr_off;
    const sk::Cx<float>* twP = static_cast<const sk::Cx<float>*>(a.tw) + d.twP_off;
    for (int n = tid; n < S; n += kBatchThreads) {
        const sk::Cx<float> lo = band_at(d, fhat, pre, n), hi = band_at(d, fhat, pre, n + S);
        sk::Cx<float> w = twP[n];
        w.im = -w.im;
        scr[n] = sk::cadd(lo, hi);
        scr[S + n] = sk::cmul(sk::csub(lo, hi), w);
    }
    __syncthreads();
    for (int h = 0; h < 2; ++h) {
        for (int n = tid; n < S; n += kBatchThreads) buf[sk::padpos(n)] = scr[h * S + n];
        __syncthreads();
        lds_dft<-1>(buf, d.lgS, tw, tid);
        for (int q = tid; q < S; q += kBatchThreads)
            buf[sk::padpos(q)] = sk::cmul(buf[sk::padpos(q)], H[2 * q + h]);
        __syncthreads();
        lds_dft<+1>(buf, d.lgS, tw, tid);
        for (int n = tid; n < S; n += kBatchThreads) scr[h * S + n] = buf[sk::padpos(n)];
        __syncthreads();
    }
    for (int i = tid; i < d.L; i += kBatchThreads) {
        int n = i - d.L / 2;
        n += (n < 0) ? d.P : 0;
        const int nn = n < S ? n : n - S;
        const sk::Cx<float> e = scr[nn], o = scr[S + nn];
        const sk::Cx<float> wo = sk::cmul(o, twP[nn]);
        const sk::Cx<float> z = n < S ? sk::cadd(e, wo) : sk::csub(e, wo);
        theta[i] = mul_d(z, post[i]);
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

__global__ void k_bbin_count(BBinArgs a) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.N) return;
    const int i = find_instance(a.node_off, a.count, j);
    const InstDesc d = a.desc[i];
    float xv = a.x[j];
    if (!(xv >= -0.5f && xv < 0.5f)) {
        atomicAdd(&a.flags[0], 1ull);
        xv = 0.0f;
    }
    const float lim = 0.5f - float(d.m) / float(d.L);
    if (!(xv >= -lim && xv < lim)) atomicAdd(&a.flags[1], 1ull);
    int n;
    float th;
    dev::cell_of<float>(xv, d.L, n, th);
    const int tile = d.tile_base + (n + d.L / 2) / a.tile;
    a.node_tile[j] = tile;
    atomicAdd(&a.tile_count[tile], 1);
}

__global__ void k_bbin_scatter(const float* __restrict__ x, long long N, const int32_t* node_tile,
                               const int32_t* offset, int32_t* cursor, int32_t* perm,
                               float* __restrict__ xs) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const int tile = node_tile[j];
    const int pos = offset[tile] + atomicAdd(&cursor[tile], 1);
    perm[pos] = int32_t(j);
    xs[pos] = x[j];
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
__device__ __forceinline__ void bgather_nodes(const BGatherArgs& a, const int4& ch, const InstDesc& d,
                                              const CxF* lds, const float* coef, int n0) {
    CxF* f = static_cast<CxF*>(a.f);
    for (int jj = threadIdx.x; jj < ch.z; jj += blockDim.x) {
        const long long j = (long long)ch.y + jj;
        int n;
        float theta[1];
        dev::cell_of<float>(a.xs[j], d.L, n, theta[0]);
        const int r = n + d.L / 2 - n0;
        float w[1][M2];
        dev::weights_poly<1, M2, kPolyCoef>(theta, coef, w);
        typename std::conditional<ACC == 1, dev::WideAcc<float>, dev::Plain<float>>::type acc;
#pragma unroll
        for (int o = 0; o < M2; ++o) acc.add(w[0][o], lds[r + o]);
        f[a.perm[j]] = acc.value();
    }
}

template <int ACC>
__global__ void __launch_bounds__(256) k_batch_gather(BGatherArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int4 ch = a.chunks[blockIdx.x];
    const InstDesc d = a.desc[ch.w];
    const int n0 = (ch.x - d.tile_base) * a.tile;
    const int W = a.tile + 2 * d.m - 1;
    CxF* lds = reinterpret_cast<CxF*>(smem_raw);
    float* coef = reinterpret_cast<float*>(smem_raw + ((size_t(a.tile + 2 * kMaxM) * sizeof(CxF) + 15) & ~size_t(15)));
    const CxF* th = static_cast<const CxF*>(a.theta) + d.theta_off;
    for (int e = threadIdx.x; e < W; e += blockDim.x) {
        const int p = n0 - d.m + 1 + e;
        lds[e] = (p >= 0 && p < d.L) ? th[p] : CxF{0.0f, 0.0f};
    }
    for (int e = threadIdx.x; e < d.m * kPolyCoef; e += blockDim.x)
        coef[e] = a.coef[(long long)ch.w * kMaxM * kPolyCoef + e];
    __syncthreads();
    switch (d.m) {
        case 2: bgather_nodes<4, ACC>(a, ch, d, lds, coef, n0); break;
        case 3: bgather_nodes<6, ACC>(a, ch, d, lds, coef, n0); break;
        case 4: bgather_nodes<8, ACC>(a, ch, d, lds, coef, n0); break;
        case 5: bgather_nodes<10, ACC>(a, ch, d, lds, coef, n0); break;
        case 6: bgather_nodes<12, ACC>(a, ch, d, lds, coef, n0); break;
        case 7: bgather_nodes<14, ACC>(a, ch, d, lds, coef, n0); break;
        default: bgather_nodes<16, ACC>(a, ch, d, lds, coef, n0); break;
    }
}

__global__ void k_tile_scan_b(const int32_t* count, int32_t* offset, int32_t* chunk_off,
                              long long ntiles, int cap, unsigned long long* flags) {
    __shared__ long long s1[1024];
    __shared__ long long s2[1024];
    const int tid = threadIdx.x, NT = blockDim.x;
    const long long per = (ntiles + NT - 1) / NT;
    const long long beg = tid * per, end = beg + per < ntiles ? beg + per : ntiles;
    long long x = 0, y = 0;
    for (long long i = beg; i < end; ++i) {
        x += count[i];
        y += (count[i] + cap - 1) / cap;
    }
    s1[tid] = x;
    s2[tid] = y;
    __syncthreads();
    for (int off = 1; off < NT; off *= 2) {
        const long long va = tid >= off ? s1[tid - off] : 0, vb = tid >= off ? s2[tid - off] : 0;
        __syncthreads();
        s1[tid] += va;
        s2[tid] += vb;
        __syncthreads();
    }
    long long ea = s1[tid] - x, eb = s2[tid] - y;
    for (long long i = beg; i < end; ++i) {
        offset[i] = int32_t(ea);
        chunk_off[i] = int32_t(eb);
        ea += count[i];
        eb += (count[i] + cap - 1) / cap;
    }
    if (tid == NT - 1) flags[2] = (unsigned long long)s2[NT - 1];
}

// ---------------------------------------------------------------- host helpers
// In-place radix-2 DFT (FP64) of a power-of-two length, sign -1: X_q = sum x_n e^{-2 pi i n q/P}.
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

// e^{i pi q / L} for integer q (reduced mod 2L in integers, then the twiddle table).
std::complex<double> chirp(int64_t q, int64_t L, const std::vector<double>& tw2L) {
    int64_t r = q % (2 * L);
    if (r < 0) r += 2 * L;
    return {tw2L[2 * r], tw2L[2 * r + 1]};
}

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
    // nodes
    float* d_xs = nullptr;
    int32_t* d_perm = nullptr;
    int32_t* d_node_tile = nullptr;
    int32_t* d_tile_count = nullptr;
    int32_t* d_tile_offset = nullptr;
    int32_t* d_tile_cursor = nullptr;
    int32_t* d_chunk_offset = nullptr;
    int32_t* d_tile_inst = nullptr;
    int4* d_chunks = nullptr;
    unsigned long long* d_flags = nullptr;
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
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->capture_stream) hipStreamDestroy(b->capture_stream);
    void* ptrs[] = {b->d_desc, b->d_node_off, b->d_pre, b->d_post, b->d_h, b->d_tw, b->d_theta,
                    b->d_scratch, b->d_coef, b->d_xs, b->d_perm, b->d_node_tile, b->d_tile_count,
                    b->d_tile_offset, b->d_tile_cursor, b->d_chunk_offset, b->d_tile_inst,
                    b->d_chunks, b->d_flags};
    for (void* q : ptrs) hipFree(q);
}

// Launch the transforms: one workgroup per instance, then the short sums.
bl_status batch_launches(bl_batch_s* b, hipStream_t s, const void* fhat, void* f, bool fft = true) {
    if (fft) {
    FftArgs fa{};
    fa.desc = b->d_desc;
    fa.fhat = fhat;
    fa.theta = b->d_theta;
    fa.pre = b->d_pre;
    fa.post = b->d_post;
    fa.h = b->d_h;
    fa.scratch = b->d_scratch;
    fa.tw = b->d_tw;
    hipLaunchKernelGGL(k_batch_fft, dim3(unsigned(b->count)), dim3(kBatchThreads), b->fft_lds, s, fa);
    BL_HIP(hipGetLastError());
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
    for (int i = 0; i < b->count; ++i) {
        b->h_desc[i].tile_base = int(nt);
        b->h_desc[i].ntiles = int((b->h_desc[i].L + tile - 1) / tile);
        nt += b->h_desc[i].ntiles;
        for (int k = 0; k < b->h_desc[i].ntiles; ++k) tile_inst.push_back(i);
    }
    b->ntiles = nt;
    const int64_t N = b->total_N;
    const int64_t chunk_bound = N / b->chunk_cap + nt + 1;
    if (nt > b->tile_alloc) {
        hipFree(b->d_tile_count);
        hipFree(b->d_tile_offset);
        hipFree(b->d_tile_cursor);
        hipFree(b->d_chunk_offset);
        hipFree(b->d_tile_inst);
        b->d_tile_count = b->d_tile_offset = b->d_tile_cursor = b->d_chunk_offset = b->d_tile_inst = nullptr;
        b->tile_alloc = 0;
        BL_TRY(balloc(&b->d_tile_count, sizeof(int32_t) * nt));
        BL_TRY(balloc(&b->d_tile_offset, sizeof(int32_t) * nt));
        BL_TRY(balloc(&b->d_tile_cursor, sizeof(int32_t) * nt));
        BL_TRY(balloc(&b->d_chunk_offset, sizeof(int32_t) * nt));
        BL_TRY(balloc(&b->d_tile_inst, sizeof(int32_t) * nt));
        b->tile_alloc = nt;
    }
    if (chunk_bound > b->chunk_alloc) {
        hipFree(b->d_chunks);
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
    const unsigned nb = unsigned((N + 255) / 256);
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
        hipLaunchKernelGGL(k_bbin_count, dim3(nb), dim3(256), 0, s, ba);
        BL_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_tile_scan_b, dim3(1), dim3(1024), 0, s, b->d_tile_count, b->d_tile_offset,
                       b->d_chunk_offset, (long long)nt, b->chunk_cap, b->d_flags);
    BL_HIP(hipGetLastError());
    if (N > 0) {
        hipLaunchKernelGGL(k_bbin_scatter, dim3(nb), dim3(256), 0, s, x, (long long)N, b->d_node_tile,
                           b->d_tile_offset, b->d_tile_cursor, b->d_perm, b->d_xs);
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
bl_status autotune_tile(bl_batch_s* b, const float* x) {
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
        hipEventRecord(e0, b->stream);
        for (int rep = 0; rep < 3 && st == BL_OK; ++rep) st = batch_launches(b, b->stream, nullptr, fdummy, false);
        hipEventRecord(e1, b->stream);
        if (hipEventSynchronize(e1) != hipSuccess) st = bfail(BL_EDEVICE, "hipEventSynchronize failed");
        float ms = 0.0f;
        if (st == BL_OK && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms < best) {
            best = ms;
            best_tile = cand;
        }
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipStreamSynchronize(b->stream);
    hipFree(fdummy);
    if (st != BL_OK) return st;
    b->tile = best_tile;
    b->tuned = true;
    return BL_OK;
}

void drop_graph(bl_batch_s* b) {
    if (b->exec) {
        hipStreamSynchronize(b->stream);   // a launch of the graph may still be in flight
        hipGraphExecDestroy(b->exec);
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
    if (prec != BL_F32 && prec != BL_F32C)
        return bfail(prec == BL_F64 ? BL_EUNSUPPORTED : BL_EINVAL, "batched transforms run in BL_F32 or BL_F32C");
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
        if (v >= 1024 && v <= kMaxLdsFft && (v & (v - 1)) == 0) lds_fft_max = v;
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
        d.split = P > lds_fft_max ? 1 : 0;
        if (P > 2 * int64_t(lds_fft_max))
            return cleanup(bfail(BL_EUNSUPPORTED, "instance " + std::to_string(i) + ": transform above twice the LDS size"));
        const int64_t S = d.split ? P / 2 : P;
        d.lgS = ilog2i(S);
        d.tw_off = table(d.lgS);
        d.twP_off = d.split ? table(ilog2i(P)) : 0;
        d.fhat_off = b->total_M;
        d.theta_off = b->total_L;
        d.pre_off = (long long)pre.size();
        d.post_off = (long long)post.size();
        d.h_off = (long long)(hbuf.size() / 2);
        d.scr_off = d.split ? scr : 0;
        if (d.split) scr += P;
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
        std::vector<std::complex<double>> h(P, 0.0);
        const int64_t J = (L[i] + M[i]) / 2;
        for (int64_t j = -J + 1; j < J; ++j) h[(j % P + P) % P] = std::conj(chirp(j * j, L[i], tw2L));
        std::vector<double> twp;
        twiddles(P, &twp);
        std::vector<std::complex<double>> root(P / 2);
        for (int64_t k = 0; k < P / 2; ++k) root[k] = {twp[2 * k], twp[2 * k + 1]};
        host_dft(h, root);
        for (int64_t q = 0; q < P; ++q) {
            hbuf.push_back(float(h[q].real() / double(P)));
            hbuf.push_back(float(h[q].imag() / double(P)));
        }
        std::vector<double> pc;
        fit_weight_polys(BL_WIN_SINH, BL_SHANNON, m[i], beta, kPolyCoef, &pc);
        for (size_t q = 0; q < pc.size(); ++q) coef[size_t(i) * kMaxM * kPolyCoef + q] = float(pc[q]);
    }
    b->h_node_off[count] = node_off;
    b->total_N = node_off;
    if (b->total_N > int64_t(0x7fffffff)) return cleanup(bfail(BL_EUNSUPPORTED, "total node count above 2^31"));

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
    if ((s = balloc(&b->d_flags, sizeof(unsigned long long) * 4)) != BL_OK) return cleanup(s);
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
    if (e == hipSuccess) e = hipMemsetAsync(b->d_theta, 0, sizeof(CxF) * b->total_L, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return cleanup(bfail(BL_EDEVICE, std::string("table upload: ") + hipGetErrorString(e)));

    int lg_max = 0;
    for (const InstDesc& d : b->h_desc) lg_max = std::max(lg_max, d.lgS);
    b->fft_lds = size_t(sk::padpos((1 << lg_max) - 1) + 1) * sizeof(CxF);
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
    if (!b->tuned && b->total_N > 0) {
        // Autotune the tile edge: bin with each candidate and time the short sums alone.
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
            if (g) hipGraphDestroy(g);
            (void)hipGetLastError();
            if (st != BL_OK) return st;
            return bfail(BL_EDEVICE, "batched graph capture failed");
        }
        e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
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
    hipSetDevice(b->device);
    hipStreamSynchronize(b->stream);
    free_batch(b);
    delete b;
    return BL_OK;
}

}  // extern "C"
