// Step 3 of Algorithm 4.2 (short sums of the regularized Shannon formula, (4.8)) and of
// Algorithm 2.1 (periodic window sums over I_{L,m}(x_j), (2.5)), plus the node binning
// that realises step 0b.
//
// Binning sorts nodes by grid tile (counting sort: histogram, one-workgroup scan,
// scatter) and cuts every tile into work chunks of at most `cap` nodes.  The short-sum
// kernel runs one workgroup per chunk: it stages the tile's samples theta plus a halo of
// m-1 cells below and m above in LDS, then each thread evaluates its nodes.
//
// For a node with L x = n + theta (n integer, theta in [0, 1)) the 2m grid points
// l = n - m + 1 + o, o = 0..2m-1, carry every nonzero weight: the end points of
// J_{L,m}(x) have sinc(+-m pi) phi(+-m/L) = 0.  The offset u = L x - l = theta + m - 1 - o,
// and sin(pi u) = (-1)^{m-1-o} sin(pi theta), so one sin per node and dimension serves all
// 2m weights; sin(pi theta) is reduced to [0, 1/2] by reflection.
#include <algorithm>
#include <cstdlib>

#include "blnfft_internal.h"
#include "device_math.h"

namespace bl {
namespace {

using namespace dev;

// ---------------------------------------------------------------- binning kernels
struct BinArgs {
    const void* x;
    int64_t N;
    int d, L, m;
    int tile[3];
    int tpd[3];              // tiles per dimension
    int32_t* node_tile;
    int32_t* tile_count;
    unsigned long long* flags;   // [0] invalid, [1] outside truncated domain
};

// Tile of node j (row-major over tiles), with the domain checks: bad = non-finite or outside
// [-1/2, 1/2) (evaluated as 0), outside = outside the truncated domain.
template <typename R, int D>
__device__ __forceinline__ int node_tile_of(const BinArgs& a, const R* x, int64_t j, bool& bad,
                                            bool& outside) {
    int tile = 0;
    bad = false;
    outside = false;
    const R lim = R(0.5) - R(a.m) / R(a.L);
#pragma unroll
    for (int t = 0; t < D; ++t) {
        R xt = x[j * D + t];
        if (!(xt >= R(-0.5) && xt < R(0.5))) { bad = true; xt = R(0); }
        if (!(xt >= -lim && xt < lim)) outside = true;
        int n;
        R th;
        cell_of<R>(xt, a.L, n, th);
        int cell = n + a.L / 2;
        tile = tile * a.tpd[t] + cell / a.tile[t];
    }
    return tile;
}

// Binning with per-workgroup LDS histograms.  A workgroup takes kBinPer * kBinThreads
// consecutive nodes (their tiles stay in registers) and walks the tiles between its
// smallest and largest in windows of kLdsBins: it counts its nodes of the window in LDS, then adds each nonzero count to the
// global counter once, instead of one contended global atomic per node.  The domain flags
// are summed per wave first.  The scatter recounts the same nodes window by window, keeping
// each node's LDS rank, reserves one range per tile with a single global atomic and places
// every node at its rank in that range.
constexpr int kLdsBins = 8192;
constexpr int kBinThreads = 256;
constexpr int kBinPer = 16;

// Smallest and largest tile among the workgroup's nodes (tl < 0: no node); the windows
// of kLdsBins tiles outside [lo, hi] hold none of them and are skipped.  Uniform over the
// workgroup (read from LDS after a barrier); hi < lo when the workgroup has no nodes.
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

template <typename R, int D>
__global__ void __launch_bounds__(kBinThreads) k_bin_count(BinArgs a, int ntiles) {
    __shared__ int hist[kLdsBins];
    const R* x = static_cast<const R*>(a.x);
    const int64_t j0 = int64_t(blockIdx.x) * (kBinThreads * kBinPer) + threadIdx.x;
    int tl[kBinPer];
    int nbad = 0, nout = 0;
#pragma unroll
    for (int k = 0; k < kBinPer; ++k) {
        const int64_t j = j0 + int64_t(k) * kBinThreads;
        tl[k] = -1;
        if (j < a.N) {
            bool bad, outside;
            tl[k] = node_tile_of<R, D>(a, x, j, bad, outside);
            nbad += bad ? 1 : 0;
            nout += outside ? 1 : 0;
            a.node_tile[j] = tl[k];
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        nbad += __shfl_xor(nbad, off);
        nout += __shfl_xor(nout, off);
    }
    if ((threadIdx.x & 63) == 0) {
        if (nbad) atomicAdd(&a.flags[0], (unsigned long long)nbad);
        if (nout) atomicAdd(&a.flags[1], (unsigned long long)nout);
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

}  // namespace

// ---------------------------------------------------------------- tile scans
// Exclusive scans of the node counts and of the chunk counts ceil(count / cap) per tile,
// device-wide in three kernels: per-block sums over kScanBlock tiles, one workgroup
// scanning the block sums (and storing the total chunk count in flags[2]), and the
// per-block scans offset by their block's prefix.
constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;
constexpr int kScanBlock = kScanThreads * kScanPer;

namespace {

// Inclusive scan of v over the workgroup (Hillis-Steele in LDS); returns the total in tot.
template <int NT>
__device__ __forceinline__ long long block_scan(long long v, long long* sh, long long& tot) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < NT; off *= 2) {
        const long long u = int(threadIdx.x) >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += u;
        __syncthreads();
    }
    const long long r = sh[threadIdx.x];
    tot = sh[NT - 1];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_partial(const int32_t* count, int64_t ntiles, int cap,
                                                               long long* bsum) {
    __shared__ long long sa[kScanThreads], sb[kScanThreads];
    const int64_t t0 = int64_t(blockIdx.x) * kScanBlock + int64_t(threadIdx.x) * kScanPer;
    long long a = 0, b = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (t0 + k < ntiles) {
            const int c = count[t0 + k];
            a += c;
            b += (c + cap - 1) / cap;
        }
    }
    long long ta, tb;
    block_scan<kScanThreads>(a, sa, ta);
    block_scan<kScanThreads>(b, sb, tb);
    if (threadIdx.x == 0) {
        bsum[2 * blockIdx.x] = ta;
        bsum[2 * blockIdx.x + 1] = tb;
    }
}

__global__ void __launch_bounds__(1024) k_scan_blocks(long long* bsum, int64_t nb, unsigned long long* flags) {
    __shared__ long long sa[1024], sb[1024];
    const int64_t per = (nb + 1023) / 1024;
    const int64_t beg = int64_t(threadIdx.x) * per, end = min(beg + per, nb);
    long long a = 0, b = 0;
    for (int64_t i = beg; i < end; ++i) {
        a += bsum[2 * i];
        b += bsum[2 * i + 1];
    }
    long long ta, tb;
    long long ea = block_scan<1024>(a, sa, ta) - a, eb = block_scan<1024>(b, sb, tb) - b;
    for (int64_t i = beg; i < end; ++i) {
        const long long va = bsum[2 * i], vb = bsum[2 * i + 1];
        bsum[2 * i] = ea;
        bsum[2 * i + 1] = eb;
        ea += va;
        eb += vb;
    }
    if (threadIdx.x == 0) flags[2] = (unsigned long long)tb;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_final(const int32_t* count, int64_t ntiles, int cap,
                                                             const long long* bsum, int32_t* offset,
                                                             int32_t* chunk_off) {
    __shared__ long long sa[kScanThreads], sb[kScanThreads];
    const int64_t t0 = int64_t(blockIdx.x) * kScanBlock + int64_t(threadIdx.x) * kScanPer;
    int c[kScanPer];
    long long a = 0, b = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        c[k] = t0 + k < ntiles ? count[t0 + k] : 0;
        a += c[k];
        b += (c[k] + cap - 1) / cap;
    }
    long long ta, tb;
    long long ea = block_scan<kScanThreads>(a, sa, ta) - a + bsum[2 * blockIdx.x];
    long long eb = block_scan<kScanThreads>(b, sb, tb) - b + bsum[2 * blockIdx.x + 1];
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (t0 + k < ntiles) {
            offset[t0 + k] = int32_t(ea);
            chunk_off[t0 + k] = int32_t(eb);
        }
        ea += c[k];
        eb += (c[k] + cap - 1) / cap;
    }
}

}  // namespace

size_t tile_scan_scratch_bytes(int64_t ntiles) {
    return size_t(2 * ((ntiles + kScanBlock - 1) / kScanBlock + 1)) * sizeof(long long);
}

bl_status launch_tile_scan(const int32_t* count, int32_t* offset, int32_t* chunk_off, int64_t ntiles, int cap,
                           unsigned long long* flags, void* scratch, hipStream_t stream) {
    const int64_t nb = std::max<int64_t>(1, (ntiles + kScanBlock - 1) / kScanBlock);
    long long* bsum = static_cast<long long*>(scratch);
    hipLaunchKernelGGL(k_scan_partial, dim3(unsigned(nb)), dim3(kScanThreads), 0, stream, count, ntiles, cap, bsum);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, stream, bsum, nb, flags);
    hipLaunchKernelGGL(k_scan_final, dim3(unsigned(nb)), dim3(kScanThreads), 0, stream, count, ntiles, cap,
                       static_cast<const long long*>(bsum), offset, chunk_off);
    BL_HIP(hipGetLastError());
    return BL_OK;
}

namespace {

template <typename R, int D>
__global__ void __launch_bounds__(kBinThreads) k_bin_scatter(const R* __restrict__ x, int64_t N,
                                                             const int32_t* node_tile,
                                                             const int32_t* offset, int32_t* cursor,
                                                             int32_t* perm, R* __restrict__ xs,
                                                             int ntiles) {
    __shared__ int hist[kLdsBins];   // counts, then the start of this workgroup's range
    const int64_t j0 = int64_t(blockIdx.x) * (kBinThreads * kBinPer) + threadIdx.x;
    int tl[kBinPer], rank[kBinPer];
#pragma unroll
    for (int k = 0; k < kBinPer; ++k) {
        const int64_t j = j0 + int64_t(k) * kBinThreads;
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
            const int64_t j = j0 + int64_t(k) * kBinThreads;
            const int pos = hist[e] + rank[k];
            perm[pos] = int32_t(j);
#pragma unroll
            for (int t = 0; t < D; ++t) xs[int64_t(pos) * D + t] = x[j * D + t];
        }
    }
}

__global__ void k_chunk_fill(const int32_t* count, const int32_t* offset,
                             const int32_t* chunk_off, int64_t ntiles, int cap, int4* chunks) {
    int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    int c = count[t];
    int base = chunk_off[t];
    for (int s = 0, k = 0; s < c; s += cap, ++k) {
        int cnt = (c - s) < cap ? (c - s) : cap;
        chunks[base + k] = make_int4(int(t), offset[t] + s, cnt, 0);
    }
}

// Within one chunk, order the nodes by their cell inside the tile (row-major), so that
// neighbouring lanes of the short-sum kernel read neighbouring samples from LDS, and the
// nodes of one cell by their index in the caller's order: the order inside a chunk then
// depends only on the chunk's nodes, not on the order the binning scatter left them in.
// LDS counting sort over the tile's cells, then each node's rank among its cell's nodes
// from their caller indices; the chunk's sorted nodes and permutation are rewritten in
// place (all reads complete before the first write).
constexpr int kSortPerThread = 4;   // chunk_cap / 256

struct SortArgs {
    const int4* chunks;
    void* xs;
    int32_t* perm;
    int L;
    int tile[3];
    int tpd[3];
};

template <typename R, int D>
__global__ void __launch_bounds__(256) k_chunk_sort(SortArgs a) {
    extern __shared__ int hist[];
    __shared__ int part[256];
    const int4 ch = a.chunks[blockIdx.x];
    int n0[3] = {0, 0, 0};
    int tvol = 1;
    {
        int tt = ch.x;
#pragma unroll
        for (int t = D - 1; t >= 0; --t) {
            n0[t] = (tt % a.tpd[t]) * a.tile[t];
            tt /= a.tpd[t];
            tvol *= a.tile[t];
        }
    }
    for (int e = threadIdx.x; e < tvol; e += blockDim.x) hist[e] = 0;
    __syncthreads();
    R* xs = static_cast<R*>(a.xs);
    R xv[kSortPerThread][D];
    int pv[kSortPerThread], key[kSortPerThread], rank[kSortPerThread];
#pragma unroll
    for (int q = 0; q < kSortPerThread; ++q) {
        const int jj = threadIdx.x + q * blockDim.x;
        key[q] = -1;
        if (jj < ch.z) {
            const int64_t j = int64_t(ch.y) + jj;
            int k = 0;
#pragma unroll
            for (int t = 0; t < D; ++t) {
                xv[q][t] = xs[j * D + t];
                int n;
                R th;
                cell_of<R>(xv[q][t], a.L, n, th);
                k = k * a.tile[t] + (n + a.L / 2 - n0[t]);
            }
            pv[q] = a.perm[j];
            key[q] = k;
            rank[q] = atomicAdd(&hist[k], 1);
        }
    }
    __syncthreads();
    // exclusive scan of hist[0..tvol)
    const int per = (tvol + blockDim.x - 1) / blockDim.x;
    const int beg = threadIdx.x * per;
    const int end = beg + per < tvol ? beg + per : tvol;
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
    // the caller indices of each cell's nodes, in arrival order, then every node's rank
    // among them by caller index (caller indices are distinct)
    __shared__ int bucket[kSortPerThread * 256];
#pragma unroll
    for (int q = 0; q < kSortPerThread; ++q)
        if (key[q] >= 0) bucket[hist[key[q]] + rank[q]] = pv[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kSortPerThread; ++q) {
        if (key[q] < 0) continue;
        const int s0 = hist[key[q]], s1 = key[q] + 1 < tvol ? hist[key[q] + 1] : ch.z;
        int r = 0;
        for (int e = s0; e < s1; ++e) r += bucket[e] < pv[q] ? 1 : 0;
        rank[q] = r;
    }
#pragma unroll
    for (int q = 0; q < kSortPerThread; ++q) {
        if (key[q] < 0) continue;
        const int64_t pos = int64_t(ch.y) + hist[key[q]] + rank[q];
#pragma unroll
        for (int t = 0; t < D; ++t) xs[pos * D + t] = xv[q][t];
        a.perm[pos] = pv[q];
    }
}

// ---------------------------------------------------------------- short sums
struct GatherArgs {
    const void* theta;     // L^d complex, centred
    const void* xs;        // sorted nodes
    const int32_t* perm;
    const int4* chunks;
    void* f;
    int L;
    int tile[3];
    int tpd[3];
    int pitch[3];          // LDS pitch (elements) of each tile dimension
    uint32_t wdiv[3];      // floor(2^20 / W) + 1 for each box extent W = tile + 2m - 1
    double beta, cb;
    WinF32 wf;             // float window constants
    alignas(16) float poly[kMaxM * kPolyCoef];   // float weight polynomials (see weights_poly)
    alignas(16) double poly64[kMaxM * kPolyCoef64];   // double ones (see weights_poly64)
    int use_poly64;
    float edge_k;   // edge exponent of the weight polynomials
    const void* wpre;   // PRE: weights of node j (binned order) at [j][t][o], d x 2m each
    int64_t N;          // k_weights: bound nodes
};

// Weights of node j (binned order), per dimension, as the short-sum kernel evaluates them.
template <typename R, int D, int M2, int METHOD>
__device__ __forceinline__ void node_weights(const GatherArgs& a, const R* theta, const float* coef,
                                             const double* coef64, R (*w)[M2]) {
    constexpr int m = M2 / 2;
    if constexpr (std::is_same<R, float>::value) {
        weights_poly<D, M2, kPolyCoef>(theta, coef, w, a.edge_k);
    } else if (a.use_poly64) {
        weights_poly64<D, M2, kPolyCoef64>(theta, coef64, w, double(a.edge_k));
    } else {
#pragma unroll
        for (int t = 0; t < D; ++t)
            weights<R, M2, METHOD>(theta[t], R(a.beta), R(a.cb), R(1) / R(m * m), w[t]);
    }
}

// Algorithm 4.2, step 0b in precomputed form: the d x 2m weights of every bound node,
// stored in binned order for the PRE short-sum kernels (one thread per node).
template <typename R, int D, int M2>
__global__ void __launch_bounds__(256) k_weights(GatherArgs a) {
    const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= a.N) return;
    const R* __restrict__ xs = static_cast<const R*>(a.xs);
    R theta[D];
#pragma unroll
    for (int t = 0; t < D; ++t) {
        int n;
        cell_of<R>(xs[j * D + t], a.L, n, theta[t]);
    }
    R w[D][M2];
    node_weights<R, D, M2, 0>(a, theta, a.poly, a.poly64, w);
    R* __restrict__ out = static_cast<R*>(const_cast<void*>(a.wpre)) + j * (D * M2);
#pragma unroll
    for (int t = 0; t < D; ++t)
#pragma unroll
        for (int o = 0; o < M2; ++o) out[t * M2 + o] = w[t][o];
}

// PRE: the weights come from a.wpre (bl_precompute_weights) instead of being evaluated.
// EXACT (double only): the closed-form weights instead of the double polynomials; a
// separate instantiation, so that the polynomial kernel's registers are not sized for
// the closed form.
template <typename R, int D, int M2, int ACC, int METHOD, bool PRE = false, bool EXACT = false>
__global__ void __launch_bounds__(256) k_gather(GatherArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Cx<R>* lds = reinterpret_cast<Cx<R>*>(smem_raw);
    constexpr int m = M2 / 2;
    // Chunks are in tile order, so an XCD's consecutive chunks are neighbouring tiles whose
    // halos overlap in its L2 (measured: 1-2 us less for d = 2, FP32C; 4 us for FP64).
    const int4 ch = a.chunks[xcd_block(int(blockIdx.x), int(gridDim.x))];
    const int L = a.L;
    // tile origin (cell index in [0, L)) and LDS extents
    int n0[3] = {0, 0, 0}, W[3] = {1, 1, 1};
    {
        int tt = ch.x;
#pragma unroll
        for (int t = D - 1; t >= 0; --t) {
            int tc = tt % a.tpd[t];
            tt /= a.tpd[t];
            n0[t] = tc * a.tile[t];
            W[t] = a.tile[t] + M2 - 1;
        }
    }
    // LDS strides: dimension t advances by S[t] elements; the innermost row is padded to
    // a.pitch[D-1] elements.
    int S[3] = {1, 1, 1};
    if (D >= 2) S[D - 2] = a.pitch[D - 1];
    if (D >= 3) S[0] = S[1] * W[1];
    // d = 2, 3 float tiles are stored twice, the second copy shifted by one element, so
    // that every node's rows start 16-byte aligned in one of them and are read with
    // 128-bit loads (the row pitch is even).
    constexpr bool dual = dual_tiles_for(D, M2 / 2, std::is_same<R, float>::value);
    const int one_copy = dual ? ((S[0] * W[0] + 1) & ~1) : S[0] * W[0];
    const int lds_elems = dual ? 2 * one_copy : one_copy;
    Cx<R>* ldsB = lds + one_copy;
    const Cx<R>* __restrict__ th = static_cast<const Cx<R>*>(a.theta);
    // float weight polynomials after the tile in LDS, 16-byte aligned
    float* coef = reinterpret_cast<float*>(smem_raw + ((size_t(lds_elems) * sizeof(Cx<R>) + 15) & ~size_t(15)));
    if constexpr (std::is_same<R, float>::value && M2 > 12) {
        for (int e = threadIdx.x; e < m * kPolyCoef; e += blockDim.x) coef[e] = a.poly[e];
    }
    double* coef64 = reinterpret_cast<double*>(coef);
    if constexpr (std::is_same<R, double>::value && !EXACT && !PRE) {
        for (int e = threadIdx.x; e < m * kPolyCoef64; e += blockDim.x) coef64[e] = a.poly64[e];
    }
    // Stage the tile plus halo.  Element e of the box is split into per-dimension
    // coordinates by multiplying with wdiv[t] = floor(2^20 / W[t]) + 1 (exact division
    // while e * W[t] < 2^20, which the 64 KB tile budget guarantees).  Grid indices fit in
    // 32 bits (L^d <= 2^31).
    // Loads are issued kStage at a time per thread before their LDS writes, so that
    // several are in flight at once.
    constexpr int kStage = 4;
    const int total = W[0] * W[1] * W[2];
    for (int e0 = threadIdx.x; e0 < total; e0 += kStage * blockDim.x) {
        Cx<R> v[kStage];
        int lis[kStage];
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int e = e0 + u * int(blockDim.x);
            lis[u] = -1;
            v[u] = Cx<R>{R(0), R(0)};
            if (e < total) {
                uint32_t rem = uint32_t(e);
                int li = 0;
                uint32_t gidx = 0, gstride = 1;
                bool ingrid = true;
#pragma unroll
                for (int t = D - 1; t >= 0; --t) {
                    int ct;
                    if (t > 0) {
                        const uint32_t q = uint32_t((uint64_t(rem) * a.wdiv[t]) >> 20);
                        ct = int(rem - q * uint32_t(W[t]));
                        rem = q;
                    } else {
                        ct = int(rem);
                    }
                    li += ct * S[t];
                    int p = n0[t] - m + 1 + ct;   // cell index of this grid point
                    if (METHOD == 1) {
                        // periodic: p lies in [-m, 2L + m) (tile start < L, tile <= L, m < L)
                        p += p < 0 ? L : 0;
                        p -= p >= L ? L : 0;
                        p -= p >= L ? L : 0;
                    } else if (p < 0 || p >= L) {
                        ingrid = false;
                    }
                    gidx += uint32_t(p) * gstride;   // the last dimension is the fastest
                    gstride *= uint32_t(L);
                }
                lis[u] = li;
                if (ingrid) v[u] = th[gidx];
            }
        }
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            if (lis[u] < 0) continue;
            lds[lis[u]] = v[u];
            if (dual && lis[u] > 0) ldsB[lis[u] - 1] = v[u];
        }
    }
    __syncthreads();

    const R* __restrict__ xs = static_cast<const R*>(a.xs);
    Cx<R>* __restrict__ f = static_cast<Cx<R>*>(a.f);
    for (int jj = threadIdx.x; jj < ch.z; jj += blockDim.x) {
        const int64_t j = int64_t(ch.y) + jj;
        R w[D][M2];
        R theta[D];
        int r[3] = {0, 0, 0};
#pragma unroll
        for (int t = 0; t < D; ++t) {
            int n;
            cell_of<R>(xs[j * D + t], L, n, theta[t]);
            r[t] = n + L / 2 - n0[t];
        }
        if constexpr (PRE) {
            const R* __restrict__ wp = static_cast<const R*>(a.wpre) + j * (D * M2);
#pragma unroll
            for (int t = 0; t < D; ++t)
#pragma unroll
                for (int o = 0; o < M2; ++o) w[t][o] = wp[t * M2 + o];
        } else if constexpr (std::is_same<R, float>::value) {
            // m <= 6: coefficients straight from the kernel arguments (SGPRs); larger m
            // would spill SGPRs, so those read them from LDS (broadcast).
            if constexpr (M2 <= 12) weights_poly<D, M2, kPolyCoef>(theta, a.poly, w, a.edge_k);
            else weights_poly<D, M2, kPolyCoef>(theta, coef, w, a.edge_k);
        } else if constexpr (!EXACT) {
            // An opaque zero offset keeps the (uniform, LDS) coefficient loads inside the
            // node loop instead of holding every coefficient in registers.
            int opaque = 0;
            asm volatile("" : "+s"(opaque));
            weights_poly64<D, M2, kPolyCoef64>(theta, coef64 + opaque, w, double(a.edge_k));
        } else {
#pragma unroll
            for (int t = 0; t < D; ++t)
                weights<R, M2, METHOD>(theta[t], R(a.beta), R(a.cb), R(1) / R(m * m), w[t]);
        }
        // Separable contraction: plain FMA sums along the last dimension(s); the outermost
        // sum is plain (ACC 0), accumulated in double (ACC 1: float products are exact
        // there) or compensated by two-sums (ACC 2).
        using Outer = OuterAcc<R, ACC>;
        Cx<R> res;
        if constexpr (D == 1) {
            Outer acc;
#pragma unroll
            for (int o = 0; o < M2; ++o) acc.add(w[0][o], lds[r[0] + o]);
            res = acc.value();
        } else if constexpr (D == 2) {
            const int base = r[0] * S[0] + r[1];
            Outer acc;
            if constexpr (dual) {
                const Cx<R>* src = (base & 1) ? ldsB + (base - 1) : lds + base;
#pragma unroll
                for (int o0 = 0; o0 < M2; ++o0) {
                    const float4* row = reinterpret_cast<const float4*>(src + o0 * S[0]);
                    Plain<R> racc;
#pragma unroll
                    for (int q = 0; q < M2 / 2; ++q) {
                        const float4 v = row[q];
                        racc.add(w[1][2 * q], Cx<R>{v.x, v.y});
                        racc.add(w[1][2 * q + 1], Cx<R>{v.z, v.w});
                    }
                    acc.add(w[0][o0], racc.value());
                }
            } else {
#pragma unroll
                for (int o0 = 0; o0 < M2; ++o0) {
                    const Cx<R>* row = lds + base + o0 * S[0];
                    Plain<R> racc;
#pragma unroll
                    for (int o1 = 0; o1 < M2; ++o1) racc.add(w[1][o1], row[o1]);
                    acc.add(w[0][o0], racc.value());
                }
            }
            res = acc.value();
        } else {
            const int base = r[0] * S[0] + r[1] * S[1] + r[2];
            Outer acc;
            // The o0 loop stays rolled (code size); its weight is taken from the front of
            // a register array shifted each iteration, not by a dynamic index (which
            // would place the array in scratch memory).
#pragma unroll 1
            for (int o0 = 0; o0 < M2; ++o0) {
                const R w0 = w[0][0];
#pragma unroll
                for (int k = 0; k + 1 < M2; ++k) w[0][k] = w[0][k + 1];
                Plain<R> pacc;
#pragma unroll
                for (int o1 = 0; o1 < M2; ++o1) {
                    Plain<R> racc;
                    if constexpr (dual) {
                        const Cx<R>* src = (base & 1) ? ldsB + (base - 1) : lds + base;
                        const float4* row = reinterpret_cast<const float4*>(src + o0 * S[0] + o1 * S[1]);
#pragma unroll
                        for (int q = 0; q < M2 / 2; ++q) {
                            const float4 v = row[q];
                            racc.add(w[2][2 * q], Cx<R>{v.x, v.y});
                            racc.add(w[2][2 * q + 1], Cx<R>{v.z, v.w});
                        }
                    } else {
                        const Cx<R>* row = lds + base + o0 * S[0] + o1 * S[1];
#pragma unroll
                        for (int o2 = 0; o2 < M2; ++o2) racc.add(w[2][o2], row[o2]);
                    }
                    pacc.add(w[1][o1], racc.value());
                }
                acc.add(w0, pacc.value());
            }
            res = acc.value();
        }
        f[a.perm[j]] = res;
    }
}

using GatherFn = void (*)(GatherArgs);

template <typename R, int D, int ACC, int METHOD, bool PRE, bool EXACT>
GatherFn pick_m(int m) {
    switch (m) {
        case 2: return k_gather<R, D, 4, ACC, METHOD, PRE, EXACT>;
        case 3: return k_gather<R, D, 6, ACC, METHOD, PRE, EXACT>;
        case 4: return k_gather<R, D, 8, ACC, METHOD, PRE, EXACT>;
        case 5: return k_gather<R, D, 10, ACC, METHOD, PRE, EXACT>;
        case 6: return k_gather<R, D, 12, ACC, METHOD, PRE, EXACT>;
        case 7: return k_gather<R, D, 14, ACC, METHOD, PRE, EXACT>;
        case 8: return k_gather<R, D, 16, ACC, METHOD, PRE, EXACT>;
        default: return nullptr;
    }
}

template <typename R, int ACC, int METHOD, bool PRE = false, bool EXACT = false>
GatherFn pick_d(int d, int m) {
    switch (d) {
        case 1: return pick_m<R, 1, ACC, METHOD, PRE, EXACT>(m);
        case 2: return pick_m<R, 2, ACC, METHOD, PRE, EXACT>(m);
        case 3: return pick_m<R, 3, ACC, METHOD, PRE, EXACT>(m);
        default: return nullptr;
    }
}

GatherFn pick_gather(const Plan& p) {
    const int M = p.method == BL_NFFT ? 1 : 0;
    if (p.use_wpre && !M) {   // precomputed weights: Algorithm 4.2 only
        if (p.prec == BL_F64) return pick_d<double, 0, 0, true>(p.d, p.m);
        if (p.prec == BL_F32) return pick_d<float, 0, 0, true>(p.d, p.m);
        if (p.prec == BL_F32C) return pick_d<float, 2, 0, true>(p.d, p.m);
        return pick_d<float, 1, 0, true>(p.d, p.m);
    }
    if (p.prec == BL_F64) {
        if (p.use_poly64) return M ? pick_d<double, 0, 1>(p.d, p.m) : pick_d<double, 0, 0>(p.d, p.m);
        return M ? pick_d<double, 0, 1, false, true>(p.d, p.m) : pick_d<double, 0, 0, false, true>(p.d, p.m);
    }
    if (p.prec == BL_F32)
        return M ? pick_d<float, 0, 1>(p.d, p.m) : pick_d<float, 0, 0>(p.d, p.m);
    if (p.prec == BL_F32C)
        return M ? pick_d<float, 2, 1>(p.d, p.m) : pick_d<float, 2, 0>(p.d, p.m);
    return M ? pick_d<float, 1, 1>(p.d, p.m) : pick_d<float, 1, 0>(p.d, p.m);
}

using WeightsFn = void (*)(GatherArgs);

template <typename R, int D>
WeightsFn pick_weights_m(int m) {
    switch (m) {
        case 2: return k_weights<R, D, 4>;
        case 3: return k_weights<R, D, 6>;
        case 4: return k_weights<R, D, 8>;
        case 5: return k_weights<R, D, 10>;
        case 6: return k_weights<R, D, 12>;
        case 7: return k_weights<R, D, 14>;
        case 8: return k_weights<R, D, 16>;
        default: return nullptr;
    }
}

template <typename R>
WeightsFn pick_weights(int d, int m) {
    switch (d) {
        case 1: return pick_weights_m<R, 1>(m);
        case 2: return pick_weights_m<R, 2>(m);
        case 3: return pick_weights_m<R, 3>(m);
        default: return nullptr;
    }
}

}  // namespace

dev::WinF32 make_win_f32(const Plan& p) {
    dev::WinF32 w;
    w.b2 = float(p.beta * 1.44269504088896340736);   // beta log2(e)
    w.cb = float(1.0 / (-std::expm1(-2.0 * p.beta)));
    w.inv_m2 = float(1.0 / (double(p.m) * double(p.m)));
    return w;
}

// LDS pitch (elements) of the staged tile's innermost row.  Rows are padded so that a
// row step moves by half of the 64 LDS banks: lanes reading neighbouring tile rows then
// fall on disjoint banks.
bool dual_tile(const Plan& p) { return p.dual_tiles; }

int tile_pitch(const Plan& p) {
    const int w = p.tile[p.d - 1] + 2 * p.m - 1;
    int mode = 1;
    if (const char* e = std::getenv("BL_PITCH")) mode = std::atoi(e);   // tuning override
    int q = w;
    if (p.d == 1 || mode == 0) {
        q = w;
    } else if (mode == 2) {
        q = w | 1;
    } else if (p.d == 2) {   // measured: padding helps d = 2 tiles, not d = 3
        const int words = int(p.cplx_size() / 4);   // 32-bit banks per element
        for (int c = w; c < w + 64; ++c)
            if ((c * words) % 64 == 32) {
                q = c;
                break;
            }
    }
    if (dual_tile(p)) q = (q + 1) & ~1;   // 128-bit row reads need an even pitch
    return q;
}

// LDS bytes of the staged tile (both copies for dual tiles), 16-byte multiple.
size_t gather_lds_bytes(const Plan& p) {
    size_t e = size_t(tile_pitch(p));
    for (int t = 0; t + 1 < p.d; ++t) e *= size_t(p.tile[t] + 2 * p.m - 1);
    if (dual_tile(p)) e = 2 * ((e + 1) & ~size_t(1));
    return (e * p.cplx_size() + 15) & ~size_t(15);
}

bl_status launch_binning(Plan& p, const void* x, int64_t N) {
    BL_HIP(hipMemsetAsync(p.d_tile_count, 0, sizeof(int32_t) * p.ntiles, p.stream));
    BL_HIP(hipMemsetAsync(p.d_tile_cursor, 0, sizeof(int32_t) * p.ntiles, p.stream));
    BL_HIP(hipMemsetAsync(p.d_flags, 0, sizeof(unsigned long long) * 4, p.stream));
    BinArgs a{};
    a.x = x;
    a.N = N;
    a.d = p.d;
    a.L = int(p.L);
    a.m = p.m;
    for (int t = 0; t < 3; ++t) {
        a.tile[t] = p.tile[t];
        a.tpd[t] = p.tiles_per_dim[t];
    }
    a.node_tile = p.d_node_tile;
    a.tile_count = p.d_tile_count;
    a.flags = p.d_flags;
    const bool dbl = p.prec == BL_F64;
    const unsigned nbl = unsigned((N + kBinThreads * kBinPer - 1) / (kBinThreads * kBinPer));
    const int nt = int(p.ntiles);
    if (N > 0) {
        if (dbl) {
            if (p.d == 1) hipLaunchKernelGGL((k_bin_count<double, 1>), dim3(nbl), dim3(kBinThreads), 0, p.stream, a, nt);
            if (p.d == 2) hipLaunchKernelGGL((k_bin_count<double, 2>), dim3(nbl), dim3(kBinThreads), 0, p.stream, a, nt);
            if (p.d == 3) hipLaunchKernelGGL((k_bin_count<double, 3>), dim3(nbl), dim3(kBinThreads), 0, p.stream, a, nt);
        } else {
            if (p.d == 1) hipLaunchKernelGGL((k_bin_count<float, 1>), dim3(nbl), dim3(kBinThreads), 0, p.stream, a, nt);
            if (p.d == 2) hipLaunchKernelGGL((k_bin_count<float, 2>), dim3(nbl), dim3(kBinThreads), 0, p.stream, a, nt);
            if (p.d == 3) hipLaunchKernelGGL((k_bin_count<float, 3>), dim3(nbl), dim3(kBinThreads), 0, p.stream, a, nt);
        }
        BL_HIP(hipGetLastError());
    }
    BL_TRY(launch_tile_scan(p.d_tile_count, p.d_tile_offset, p.d_chunk_offset, p.ntiles, p.chunk_cap, p.d_flags,
                            p.d_scan, p.stream));
    if (N > 0) {
        if (dbl) {
            const double* xd = static_cast<const double*>(x);
            double* xs = static_cast<double*>(p.d_xs);
            if (p.d == 1) hipLaunchKernelGGL((k_bin_scatter<double, 1>), dim3(nbl), dim3(kBinThreads), 0, p.stream, xd, N, p.d_node_tile, p.d_tile_offset, p.d_tile_cursor, p.d_perm, xs, nt);
            if (p.d == 2) hipLaunchKernelGGL((k_bin_scatter<double, 2>), dim3(nbl), dim3(kBinThreads), 0, p.stream, xd, N, p.d_node_tile, p.d_tile_offset, p.d_tile_cursor, p.d_perm, xs, nt);
            if (p.d == 3) hipLaunchKernelGGL((k_bin_scatter<double, 3>), dim3(nbl), dim3(kBinThreads), 0, p.stream, xd, N, p.d_node_tile, p.d_tile_offset, p.d_tile_cursor, p.d_perm, xs, nt);
        } else {
            const float* xf = static_cast<const float*>(x);
            float* xs = static_cast<float*>(p.d_xs);
            if (p.d == 1) hipLaunchKernelGGL((k_bin_scatter<float, 1>), dim3(nbl), dim3(kBinThreads), 0, p.stream, xf, N, p.d_node_tile, p.d_tile_offset, p.d_tile_cursor, p.d_perm, xs, nt);
            if (p.d == 2) hipLaunchKernelGGL((k_bin_scatter<float, 2>), dim3(nbl), dim3(kBinThreads), 0, p.stream, xf, N, p.d_node_tile, p.d_tile_offset, p.d_tile_cursor, p.d_perm, xs, nt);
            if (p.d == 3) hipLaunchKernelGGL((k_bin_scatter<float, 3>), dim3(nbl), dim3(kBinThreads), 0, p.stream, xf, N, p.d_node_tile, p.d_tile_offset, p.d_tile_cursor, p.d_perm, xs, nt);
        }
        BL_HIP(hipGetLastError());
    }
    const unsigned tb = unsigned((p.ntiles + 255) / 256);
    hipLaunchKernelGGL(k_chunk_fill, dim3(tb), dim3(256), 0, p.stream, p.d_tile_count,
                       p.d_tile_offset, p.d_chunk_offset, p.ntiles, p.chunk_cap, p.d_chunks);
    BL_HIP(hipGetLastError());
    unsigned long long h[4] = {0, 0, 0, 0};
    BL_HIP(hipMemcpyAsync(h, p.d_flags, sizeof(h), hipMemcpyDeviceToHost, p.stream));
    BL_HIP(hipStreamSynchronize(p.stream));
    if (h[0] != 0) {
        set_error(std::to_string(h[0]) + " node coordinate(s) are NaN/Inf or outside [-1/2, 1/2)");
        return BL_EDOMAIN;
    }
    p.n_outside = int64_t(h[1]);
    p.nchunks = int64_t(h[2]);
    if (p.nchunks > p.chunk_alloc) {
        set_error("internal: chunk count exceeds its bound");
        return BL_EDEVICE;
    }
    if (p.nchunks > 0) {
        if (p.chunk_cap > 256 * kSortPerThread) {
            set_error("internal: chunk capacity above the sort kernel's");
            return BL_EDEVICE;
        }
        SortArgs s{};
        s.chunks = p.d_chunks;
        s.xs = p.d_xs;
        s.perm = p.d_perm;
        s.L = int(p.L);
        int tvol = 1;
        for (int t = 0; t < 3; ++t) {
            s.tile[t] = p.tile[t];
            s.tpd[t] = p.tiles_per_dim[t];
            tvol *= p.tile[t];
        }
        const size_t sh = sizeof(int) * size_t(tvol);
        const dim3 grid(unsigned(p.nchunks)), blk(256);
        if (dbl) {
            if (p.d == 1) hipLaunchKernelGGL((k_chunk_sort<double, 1>), grid, blk, sh, p.stream, s);
            if (p.d == 2) hipLaunchKernelGGL((k_chunk_sort<double, 2>), grid, blk, sh, p.stream, s);
            if (p.d == 3) hipLaunchKernelGGL((k_chunk_sort<double, 3>), grid, blk, sh, p.stream, s);
        } else {
            if (p.d == 1) hipLaunchKernelGGL((k_chunk_sort<float, 1>), grid, blk, sh, p.stream, s);
            if (p.d == 2) hipLaunchKernelGGL((k_chunk_sort<float, 2>), grid, blk, sh, p.stream, s);
            if (p.d == 3) hipLaunchKernelGGL((k_chunk_sort<float, 3>), grid, blk, sh, p.stream, s);
        }
        BL_HIP(hipGetLastError());
        BL_HIP(hipStreamSynchronize(p.stream));
    }
    return BL_OK;
}

bl_status launch_gather(Plan& p, const void* theta, void* f) {
    if (p.N == 0 || p.nchunks == 0) return BL_OK;
    GatherFn fn = pick_gather(p);
    if (!fn) {
        set_error("no short-sum kernel for this (d, m)");
        return BL_EUNSUPPORTED;
    }
    GatherArgs a{};
    a.theta = theta;
    a.xs = p.d_xs;
    a.perm = p.d_perm;
    a.chunks = p.d_chunks;
    a.f = f;
    a.L = int(p.L);
    for (int t = 0; t < 3; ++t) {
        a.tile[t] = p.tile[t];
        a.tpd[t] = p.tiles_per_dim[t];
        a.pitch[t] = (t == p.d - 1) ? tile_pitch(p) : (t < p.d ? p.tile[t] + 2 * p.m - 1 : 1);
        a.wdiv[t] = (1u << 20) / uint32_t(p.tile[t] + 2 * p.m - 1) + 1u;
    }
    a.beta = p.beta;
    a.cb = 1.0 / (-std::expm1(-2.0 * p.beta));
    a.wf = make_win_f32(p);
    for (size_t i = 0; i < p.poly.size() && i < size_t(kMaxM * kPolyCoef); ++i) a.poly[i] = p.poly[i];
    for (size_t i = 0; i < p.poly64.size() && i < size_t(kMaxM * kPolyCoef64); ++i) a.poly64[i] = p.poly64[i];
    a.use_poly64 = p.use_poly64 ? 1 : 0;
    a.edge_k = float(p.edge_k);
    a.wpre = p.use_wpre ? p.d_wpre : nullptr;
    const size_t lds = gather_lds_bytes(p) + 16 + sizeof(double) * kMaxM * kPolyCoef64;
    if (lds > 64 * 1024)
        BL_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    hipLaunchKernelGGL(fn, dim3(unsigned(p.nchunks)), dim3(256), lds, p.stream, a);
    BL_HIP(hipGetLastError());
    return BL_OK;
}

bl_status launch_weights(Plan& p) {
    if (p.N == 0) return BL_OK;
    WeightsFn fn = p.prec == BL_F64 ? pick_weights<double>(p.d, p.m) : pick_weights<float>(p.d, p.m);
    if (!fn) {
        set_error("no weight kernel for this (d, m)");
        return BL_EUNSUPPORTED;
    }
    GatherArgs a{};
    a.xs = p.d_xs;
    a.L = int(p.L);
    a.beta = p.beta;
    a.cb = 1.0 / (-std::expm1(-2.0 * p.beta));
    for (size_t i = 0; i < p.poly.size() && i < size_t(kMaxM * kPolyCoef); ++i) a.poly[i] = p.poly[i];
    for (size_t i = 0; i < p.poly64.size() && i < size_t(kMaxM * kPolyCoef64); ++i) a.poly64[i] = p.poly64[i];
    a.use_poly64 = p.use_poly64 ? 1 : 0;
    a.edge_k = float(p.edge_k);
    a.wpre = p.d_wpre;
    a.N = p.N;
    hipLaunchKernelGGL(fn, dim3(unsigned((p.N + 255) / 256)), dim3(256), 0, p.stream, a);
    BL_HIP(hipGetLastError());
    return BL_OK;
}

}  // namespace bl
