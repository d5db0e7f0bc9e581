// Adjoint spreading (Psi^T g of the factorisation (4.11), or B^T g for Algorithm 2.1) and
// the node gradient d f_j / d x_jt of the short sums (4.8).
//
// Spreading runs one workgroup per binning chunk (all its nodes share one tile): the
// contributions g_j psi(x_j - l/L) of the chunk's nodes to the (2m)^d cells around each of
// them are accumulated over the chunk's box (tile plus halo) and the box is written to the
// chunk's slot of a box buffer.  A merge kernel then forms every grid point as the sum of
// the box entries that cover it, visiting tiles, and the chunks of each tile, in a fixed
// order: no float atomics reach HBM, and for one node binding repeated adjoints are
// bitwise equal.  Box cells outside I_L are dropped (Psi has columns l in I_L only) or
// wrapped (periodic B).
//
// The gradient kernel mirrors the short-sum kernel, with psi' in one dimension:
//   d f_j / d x_jt = L sum_l theta_l psi_g'(u_t) prod_{s != t} psi_g(u_s).
#include <cstdlib>
#include <mutex>
#include <string>

#include "blnfft_internal.h"
#include "device_math.h"

namespace bl {

// LDS bytes of one unpadded tile-plus-halo box of the plan's complex type, 16-byte multiple.
size_t box_bytes(const Plan& p) {
    size_t e = 1;
    for (int t = 0; t < p.d; ++t) e *= size_t(p.tile[t] + 2 * p.m - 1);
    return (e * p.cplx_size() + 15) & ~size_t(15);
}
dev::WinF32 make_win_f32(const Plan& p);

namespace {

using namespace dev;

struct SpreadArgs {
    const void* g;          // N complex, caller order
    const void* xs;
    const int32_t* perm;
    const int4* chunks;
    void* grid;             // L^d complex, centred
    void* gx;               // gradient output (N x d real)
    int L;
    int tile[3];
    int tpd[3];
    double beta, cb;
    WinF32 wf;
    float poly[kMaxM * kPolyCoef];
    alignas(16) double poly64[kMaxM * kPolyCoef64];   // double weight polynomials
    int use_poly64;          // double kernels: weights from poly64 instead of the exact form
    float edge_k;            // edge exponent of the weight polynomials
    void* boxes;             // spreading: one box (prod_t (tile_t + 2m - 1) complex) per chunk
    int64_t box_vol;         // complex entries per box
};

__device__ __forceinline__ void lds_add(float* p, float v) { atomicAdd(p, v); }
__device__ __forceinline__ void lds_add(double* p, double v) { atomicAdd(p, v); }
// Entry e (row-major over the box extents) of the box of chunk ci.
template <typename R>
__device__ __forceinline__ void box_store(const SpreadArgs& a, int ci, int e, Cx<R> v) {
    static_cast<Cx<R>*>(a.boxes)[int64_t(ci) * a.box_vol + e] = v;
}

template <int D>
__device__ __forceinline__ void tile_geometry(const int4& ch, const int* tpd, const int* tile,
                                              int M2, int* n0, int* W) {
    int tt = ch.x;
#pragma unroll
    for (int t = D - 1; t >= 0; --t) {
        int tc = tt % tpd[t];
        tt /= tpd[t];
        n0[t] = tc * tile[t];
        W[t] = tile[t] + M2 - 1;
    }
}

template <typename R, int D, int M2, int METHOD>
__global__ void __launch_bounds__(256) k_spread(SpreadArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    R* acc = reinterpret_cast<R*>(smem_raw);   // interleaved re, im
    constexpr int m = M2 / 2;
    const int4 ch = a.chunks[xcd_block(int(blockIdx.x), int(gridDim.x))];
    const int L = a.L;
    int n0[3] = {0, 0, 0}, W[3] = {1, 1, 1};
    tile_geometry<D>(ch, a.tpd, a.tile, M2, n0, W);
    const int total = W[0] * W[1] * W[2];
    for (int e = threadIdx.x; e < 2 * total; e += blockDim.x) acc[e] = R(0);
    float* coef = reinterpret_cast<float*>(smem_raw + ((size_t(total) * 2 * sizeof(R) + 15) & ~size_t(15)));
    if constexpr (std::is_same<R, float>::value) {
        for (int e = threadIdx.x; e < m * kPolyCoef; e += blockDim.x) coef[e] = a.poly[e];
    }
    __syncthreads();

    const R* __restrict__ xs = static_cast<const R*>(a.xs);
    const Cx<R>* __restrict__ g = static_cast<const Cx<R>*>(a.g);
    const R beta = R(a.beta), cb = R(a.cb), inv_m2 = R(1) / R(m * m);
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
        if constexpr (std::is_same<R, float>::value) {
            weights_poly<D, M2, kPolyCoef>(theta, coef, w, a.edge_k);
        } else if (a.use_poly64) {
            weights_poly64<D, M2, kPolyCoef64>(theta, a.poly64, w, double(a.edge_k));
        } else {
#pragma unroll
            for (int t = 0; t < D; ++t) weights<R, M2, METHOD>(theta[t], beta, cb, inv_m2, w[t]);
        }
        const Cx<R> gj = g[a.perm[j]];
        if constexpr (D == 1) {
#pragma unroll
            for (int o0 = 0; o0 < M2; ++o0) {
                R* c = acc + 2 * (r[0] + o0);
                lds_add(c, w[0][o0] * gj.re);
                lds_add(c + 1, w[0][o0] * gj.im);
            }
        } else if constexpr (D == 2) {
#pragma unroll
            for (int o0 = 0; o0 < M2; ++o0) {
                const R are = w[0][o0] * gj.re, aim = w[0][o0] * gj.im;
                R* row = acc + 2 * ((r[0] + o0) * W[1] + r[1]);
#pragma unroll
                for (int o1 = 0; o1 < M2; ++o1) {
                    lds_add(row + 2 * o1, w[1][o1] * are);
                    lds_add(row + 2 * o1 + 1, w[1][o1] * aim);
                }
            }
        } else {
#pragma unroll 1
            for (int o0 = 0; o0 < M2; ++o0) {
#pragma unroll
                for (int o1 = 0; o1 < M2; ++o1) {
                    const R w01 = w[0][o0] * w[1][o1];
                    const R are = w01 * gj.re, aim = w01 * gj.im;
                    R* row = acc + 2 * (((r[0] + o0) * W[1] + r[1] + o1) * W[2] + r[2]);
#pragma unroll
                    for (int o2 = 0; o2 < M2; ++o2) {
                        lds_add(row + 2 * o2, w[2][o2] * are);
                        lds_add(row + 2 * o2 + 1, w[2][o2] * aim);
                    }
                }
            }
        }
    }
    __syncthreads();

    const int ci = xcd_block(int(blockIdx.x), int(gridDim.x));
    for (int e = threadIdx.x; e < total; e += blockDim.x) box_store<R>(a, ci, e, Cx<R>{acc[2 * e], acc[2 * e + 1]});
}

// Output-stationary spreading (LDS float atomics are slow on this GPU): each thread owns
// grid points of the chunk's box (tile plus halo) and accumulates, in registers, the
// contributions of the nodes whose window covers them.  The chunk's nodes are processed in
// batches of kOsBatch: their cells, weights and values go to LDS, then for a grid point the
// contributing nodes of each tile row in reach form a contiguous range of the cell-sorted
// batch (found from a per-cell start table), so no node outside the window is visited.
constexpr int kOsThreads = 256;
constexpr int kOsBatch = 256;
template <int D>
constexpr int os_points() { return D == 1 ? 4 : D == 2 ? 8 : 20; }   // box points per thread

template <typename R, int D, int M2, int METHOD>
__global__ void __launch_bounds__(kOsThreads) k_spread_os(SpreadArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int m = M2 / 2;
    constexpr int KP = os_points<D>();
    const int4 ch = a.chunks[xcd_block(int(blockIdx.x), int(gridDim.x))];
    const int L = a.L;
    const int tid = threadIdx.x;
    int n0[3] = {0, 0, 0}, W[3] = {1, 1, 1}, T[3] = {1, 1, 1};
    tile_geometry<D>(ch, a.tpd, a.tile, M2, n0, W);
#pragma unroll
    for (int t = 0; t < D; ++t) T[t] = a.tile[t];
    const int total = W[0] * W[1] * W[2];
    const int ncell = T[0] * T[1] * T[2];
    // LDS: weights [D][M2][kOsBatch], values [kOsBatch], cells [kOsBatch], starts [ncell+1], coef
    R* wts = reinterpret_cast<R*>(smem_raw);
    Cx<R>* gv = reinterpret_cast<Cx<R>*>(wts + D * M2 * kOsBatch);
    int* key = reinterpret_cast<int*>(gv + kOsBatch);
    int* start = key + kOsBatch;
    float* coef = reinterpret_cast<float*>(smem_raw + ((size_t(reinterpret_cast<unsigned char*>(start + ncell + 1) - smem_raw) + 15) & ~size_t(15)));
    if constexpr (std::is_same<R, float>::value) {
        for (int e = tid; e < m * kPolyCoef; e += kOsThreads) coef[e] = a.poly[e];
    }
    Cx<R> acc[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) acc[k] = Cx<R>{R(0), R(0)};

    const R* __restrict__ xs = static_cast<const R*>(a.xs);
    const Cx<R>* __restrict__ g = static_cast<const Cx<R>*>(a.g);
    const R beta = R(a.beta), cb = R(a.cb), inv_m2 = R(1) / R(m * m);
    for (int b0 = 0; b0 < ch.z; b0 += kOsBatch) {
        const int nb = min(kOsBatch, ch.z - b0);
        __syncthreads();   // coefficients staged / previous batch consumed
        if (tid < nb) {
            const int64_t j = int64_t(ch.y) + b0 + tid;
            R theta[D];
            int kc = 0;
#pragma unroll
            for (int t = 0; t < D; ++t) {
                int nc;
                cell_of<R>(xs[j * D + t], L, nc, theta[t]);
                kc = kc * T[t] + (nc + L / 2 - n0[t]);
            }
            R w[D][M2];
            if constexpr (std::is_same<R, float>::value) {
                weights_poly<D, M2, kPolyCoef>(theta, coef, w, a.edge_k);
            } else if (a.use_poly64) {
                weights_poly64<D, M2, kPolyCoef64>(theta, a.poly64, w, double(a.edge_k));
            } else {
#pragma unroll
                for (int t = 0; t < D; ++t) weights<R, M2, METHOD>(theta[t], beta, cb, inv_m2, w[t]);
            }
#pragma unroll
            for (int t = 0; t < D; ++t)
#pragma unroll
                for (int o = 0; o < M2; ++o) wts[(t * M2 + o) * kOsBatch + tid] = w[t][o];
            gv[tid] = g[a.perm[j]];
            key[tid] = kc;
        }
        __syncthreads();
        // start[c] = first batch position with cell >= c (the batch is sorted by cell)
        for (int c = tid; c <= ncell; c += kOsThreads) {
            int lo = 0, hi = nb;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (key[mid] < c) lo = mid + 1;
                else hi = mid;
            }
            start[c] = lo;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            const int e = tid + k * kOsThreads;
            if (e >= total) break;
            int c[3] = {0, 0, 0};
            {
                int rem = e;
#pragma unroll
                for (int t = D - 1; t >= 0; --t) {
                    c[t] = rem % W[t];
                    rem /= W[t];
                }
            }
            // tile cells in reach of box point c along t: r in [c - M2 + 1, c] within [0, T)
            int lo[3], hi[3];
#pragma unroll
            for (int t = 0; t < D; ++t) {
                lo[t] = max(0, c[t] - M2 + 1);
                hi[t] = min(T[t] - 1, c[t]);
            }
            Cx<R> sum = acc[k];
            auto visit = [&](int rowkey, int wprod_off0, R wpre) {
                // contiguous cells rowkey + lo..hi along the last dimension
                const int jb = start[rowkey + lo[D - 1]], je = start[rowkey + hi[D - 1] + 1];
                for (int j = jb; j < je; ++j) {
                    const int rl = key[j] - rowkey;   // cell along the last dimension
                    const R wl = wts[((D - 1) * M2 + (c[D - 1] - rl)) * kOsBatch + j];
                    R wv = wl * wpre;
                    if (wprod_off0 >= 0) wv *= wts[wprod_off0 + j];
                    const Cx<R> gj = gv[j];
                    sum.re = dev_fma(wv, gj.re, sum.re);
                    sum.im = dev_fma(wv, gj.im, sum.im);
                }
            };
            if constexpr (D == 1) {
                if (lo[0] <= hi[0]) visit(0, -1, R(1));
            } else if constexpr (D == 2) {
                if (lo[1] <= hi[1])
                    for (int r0 = lo[0]; r0 <= hi[0]; ++r0)
                        visit(r0 * T[1], (0 * M2 + (c[0] - r0)) * kOsBatch, R(1));
            } else {
                if (lo[2] <= hi[2])
                    for (int r0 = lo[0]; r0 <= hi[0]; ++r0)
                        for (int r1 = lo[1]; r1 <= hi[1]; ++r1) {
                            // the node's w0 and w1 both vary per node: w0 folded in per node
                            const int rowkey = (r0 * T[1] + r1) * T[2];
                            const int jb = start[rowkey + lo[2]], je = start[rowkey + hi[2] + 1];
                            const int off0 = (0 * M2 + (c[0] - r0)) * kOsBatch;
                            const int off1 = (1 * M2 + (c[1] - r1)) * kOsBatch;
                            for (int j = jb; j < je; ++j) {
                                const int r2 = key[j] - rowkey;
                                const R wv = wts[off0 + j] * wts[off1 + j] *
                                             wts[(2 * M2 + (c[2] - r2)) * kOsBatch + j];
                                const Cx<R> gj = gv[j];
                                sum.re = dev_fma(wv, gj.re, sum.re);
                                sum.im = dev_fma(wv, gj.im, sum.im);
                            }
                        }
            }
            acc[k] = sum;
        }
    }

    const int ci = xcd_block(int(blockIdx.x), int(gridDim.x));
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        const int e = tid + k * kOsThreads;
        if (e < total) box_store<R>(a, ci, e, acc[k]);
    }
}

// d = 2 spreading by tile rows.  Lane l of wave w owns the box column c1 = l mod 32 and
// the four box rows c0 = 8w + 4 (l div 32) + k, k < 4, so a box of at most 32 x 32 points
// is covered by 256 threads.  For a batch of the chunk's nodes, LDS holds both dimensions'
// weights of every node at their absolute box coordinates (zero elsewhere): a lane reads
// the weight of any node at its own row and column without knowing the node's cell, and
// a wave walks its nodes in groups of 16 bytes per load (the node values and first-
// dimension weights are broadcast reads).  A wave visits only the nodes of the tile rows
// that reach its eight box rows; others contribute zero and are harmless at group ends.
template <typename R>
constexpr int rows_batch() { return std::is_same<R, float>::value ? 128 : 64; }
template <typename R>
constexpr int rows_pitch() { return rows_batch<R>() + 16 / int(sizeof(R)); }   // spreads the banks
template <typename R>
constexpr size_t rows_lds_bytes() {
    return sizeof(R) * 64 * rows_pitch<R>() + sizeof(Cx<R>) * rows_batch<R>() +
           sizeof(int) * (48 + rows_batch<R>()) + sizeof(float) * kMaxM * kPolyCoef;
}

// RPL box rows per lane: 4 (256 threads, waves of 8 rows) or 8 (128 threads, waves of 16
// rows: more FMAs per broadcast LDS load, fewer waves visiting each node).
template <typename R, int M2, int METHOD, bool EXACT, int RPL = 4>
__global__ void __launch_bounds__(1024 / RPL) k_spread_rows(SpreadArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int m = M2 / 2;
    constexpr int NB = rows_batch<R>();
    constexpr int P = rows_pitch<R>();
    constexpr int VEC = 16 / int(sizeof(R));   // nodes per 16-byte load
    typedef R vec_t __attribute__((ext_vector_type(VEC)));
    R* w0s = reinterpret_cast<R*>(smem_raw);     // [32][P]: first-dimension weight at box row
    R* w1s = w0s + 32 * P;                       // [32][P]: last-dimension weight at box column
    Cx<R>* gv = reinterpret_cast<Cx<R>*>(w1s + 32 * P);   // [NB]
    int* rowstart = reinterpret_cast<int*>(gv + NB);      // [T0 + 1], T0 <= 32
    int* key = rowstart + 48;                             // [NB]
    float* coef = reinterpret_cast<float*>(key + NB);

    const int4 ch = a.chunks[xcd_block(int(blockIdx.x), int(gridDim.x))];
    const int L = a.L;
    const int tid = threadIdx.x;
    int n0[3] = {0, 0, 0}, W[3] = {1, 1, 1};
    tile_geometry<2>(ch, a.tpd, a.tile, M2, n0, W);
    const int T0 = a.tile[0], T1 = a.tile[1];
    if constexpr (std::is_same<R, float>::value) {
        for (int e = tid; e < m * kPolyCoef; e += blockDim.x) coef[e] = a.poly[e];
    }
    constexpr int RW = 2 * RPL;   // box rows per wave
    const int lane = tid & 63, wv = tid >> 6;
    const int c1 = lane & 31;
    const int cb = RW * wv + RPL * (lane >> 5);
    // tile rows whose nodes reach box rows [RW wv, RW wv + RW)
    const int rlo = max(0, RW * wv - M2 + 1), rhi = min(T0 - 1, RW * wv + RW - 1);
    Cx<R> acc[RPL];
#pragma unroll
    for (int k = 0; k < RPL; ++k) acc[k] = Cx<R>{R(0), R(0)};

    const R* __restrict__ xs = static_cast<const R*>(a.xs);
    const Cx<R>* __restrict__ g = static_cast<const Cx<R>*>(a.g);
    const R beta = R(a.beta), cbeta = R(a.cb), inv_m2 = R(1) / R(m * m);
    for (int b0 = 0; b0 < ch.z; b0 += NB) {
        const int nb = min(NB, ch.z - b0);
        __syncthreads();   // coefficients staged / previous batch consumed
        {
            vec_t* z = reinterpret_cast<vec_t*>(w0s);
            for (int e = tid; e < 64 * P / VEC; e += blockDim.x) z[e] = vec_t(R(0));
        }
        __syncthreads();
        if (tid < nb) {
            {
                const int64_t j = int64_t(ch.y) + b0 + tid;
                R theta[2];
                int r[2];
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    int nc;
                    cell_of<R>(xs[j * 2 + t], L, nc, theta[t]);
                    r[t] = nc + L / 2 - n0[t];
                }
                R w[2][M2];
                if constexpr (std::is_same<R, float>::value) {
                    weights_poly<2, M2, kPolyCoef>(theta, coef, w, a.edge_k);
                } else if constexpr (!EXACT) {
                    weights_poly64<2, M2, kPolyCoef64>(theta, a.poly64, w, double(a.edge_k));
                } else {
#pragma unroll
                    for (int t = 0; t < 2; ++t) weights<R, M2, METHOD>(theta[t], beta, cbeta, inv_m2, w[t]);
                }
#pragma unroll
                for (int o = 0; o < M2; ++o) {
                    w0s[(r[0] + o) * P + tid] = w[0][o];
                    w1s[(r[1] + o) * P + tid] = w[1][o];
                }
                gv[tid] = g[a.perm[j]];
                key[tid] = r[0] * T1 + r[1];
            }
        } else if (tid < NB) {
            gv[tid] = Cx<R>{R(0), R(0)};   // past the batch: group ends read it
        }
        __syncthreads();
        // rowstart[r] = first batch position in tile row r or later (the batch is sorted)
        if (tid <= T0) {
            const int c = tid * T1;
            int lo = 0, hi = nb;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (key[mid] < c) lo = mid + 1;
                else hi = mid;
            }
            rowstart[tid] = lo;
        }
        __syncthreads();
        const int js = rlo <= rhi ? rowstart[rlo] & ~(VEC - 1) : 0;
        const int je = rlo <= rhi ? rowstart[rhi + 1] : 0;
        const R* w1p = w1s + c1 * P;
        const R* w0p = w0s + cb * P;
#pragma unroll 2
        for (int j = js; j < je; j += VEC) {
            const vec_t wl = *reinterpret_cast<const vec_t*>(w1p + j);
            vec_t w0[RPL];
#pragma unroll
            for (int k = 0; k < RPL; ++k) w0[k] = *reinterpret_cast<const vec_t*>(w0p + k * P + j);
            Cx<R> gq[VEC];
#pragma unroll
            for (int q = 0; q < VEC; ++q) gq[q] = gv[j + q];
#pragma unroll
            for (int q = 0; q < VEC; ++q) {
                const R are = wl[q] * gq[q].re, aim = wl[q] * gq[q].im;
#pragma unroll
                for (int k = 0; k < RPL; ++k) {
                    acc[k].re = dev_fma(w0[k][q], are, acc[k].re);
                    acc[k].im = dev_fma(w0[k][q], aim, acc[k].im);
                }
            }
        }
    }

    if (c1 >= W[1]) return;
    const int ci = xcd_block(int(blockIdx.x), int(gridDim.x));
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
        const int c0 = cb + k;
        if (c0 < W[0]) box_store<R>(a, ci, c0 * W[1] + c1, acc[k]);
    }
}

// d = 2 spreading on the matrix cores (float).  For one batch of a chunk's nodes the box
// is B[r][c] = sum_j (g_j w0_j(r)) w1_j(c), the product of a (rows x nodes) and a (nodes x
// columns) matrix that are mostly zero.  The box (at most 32 x 32) is covered by two bands
// of 16 rows, [0, 16) and [S, S + 16) with S = W0 - 16 (band 1 alone when W0 <= 16), and
// two blocks of 16 columns; each band-block product is a chain of 16x16x4 FP32 MFMAs, four
// nodes per instruction.  Band 1 takes the nodes whose rows reach row 16; rows below 16 of
// a node that starts below row S are band 0's (masked out of band 1), and band 0 takes no
// node that starts at row S or later.  The batch is sorted by cell, so band 0's nodes are a
// prefix of the batch and band 1's a suffix.  Waves take the (band, group of 16 nodes)
// items in turn; at the end the four waves' accumulators are summed through LDS in a fixed
// order (waves 0..3, band 0 then band 1), so a box does not depend on timing.
//
// One workgroup per chunk.  A staging thread owns one column of one weight table (node jj,
// dimension dim), so it clears the entries it wrote for the previous batch before writing
// the next: the tables are cleared in full only once.  The loads run one batch ahead
// (coordinates and node indices of batch b + 1, values of batch b in flight while batch
// b - 1 is on the matrix cores), in straight-line code and in two slots that take turns,
// so that nothing waits for a load before its use.
typedef float mfma_f4 __attribute__((ext_vector_type(4)));
constexpr int kMfmaBatch = 128;                 // nodes per batch (two staging threads each)
constexpr int kMfmaPitch = kMfmaBatch + 4;      // LDS row pitch of the weight tables
constexpr int kMfmaFar = 1 << 20;               // first row of the empty slots past a batch
constexpr size_t mfma2_lds_bytes() {
    return sizeof(float) * 64 * kMfmaPitch + sizeof(Cx<float>) * kMfmaBatch + sizeof(int) * kMfmaBatch +
           sizeof(float) * kMaxM * kPolyCoef;
}

// One item: 16 nodes from j0 into the band's accumulators acc[column block][re, im].
template <int BAND>
__device__ __forceinline__ void mfma2_item(const float* ws, const Cx<float>* gv, const int* rrow, int j0,
                                           int S, mfma_f4 (&acc)[2][2]) {
    constexpr int P = kMfmaPitch;
    const int lane = threadIdx.x & 63, kq = lane >> 4, i = lane & 15;
    const int jb = j0 + 4 * kq;            // this lane's four nodes: k slot kq of four MFMAs
    const int rho = BAND ? S + i : i;      // box row of the A operand (row i of the band)
    const mfma_f4 av = *reinterpret_cast<const mfma_f4*>(ws + rho * P + jb);
    const int4 rr = *reinterpret_cast<const int4*>(rrow + jb);
    const mfma_f4 b0 = *reinterpret_cast<const mfma_f4*>(ws + (32 + i) * P + jb);
    const mfma_f4 b1 = *reinterpret_cast<const mfma_f4*>(ws + (48 + i) * P + jb);
    const mfma_f4 gA = *reinterpret_cast<const mfma_f4*>(gv + jb);
    const mfma_f4 gB = *reinterpret_cast<const mfma_f4*>(gv + jb + 2);
    const float gre[4] = {gA[0], gA[2], gB[0], gB[2]};
    const float gim[4] = {gA[1], gA[3], gB[1], gB[3]};
    const int rq[4] = {rr.x, rr.y, rr.z, rr.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const bool keep = BAND ? (rho >= 16 || rq[q] >= S) : (rq[q] < S);
        const float aq = keep ? av[q] : 0.0f;
        const float are = aq * gre[q], aim = aq * gim[q];
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(are, b0[q], acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(aim, b0[q], acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(are, b1[q], acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(aim, b1[q], acc[1][1], 0, 0, 0);
    }
}

template <int M2>
__global__ void __launch_bounds__(256) k_spread_mfma2(SpreadArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int NB = kMfmaBatch;
    constexpr int P = kMfmaPitch;
    // ws rows 0..31: first-dimension weight of each batch node at its box row; rows 32..63:
    // last-dimension weight at its box column (zero outside the node's window)
    float* ws = reinterpret_cast<float*>(smem_raw);
    Cx<float>* gv = reinterpret_cast<Cx<float>*>(ws + 64 * P);   // [NB] node values
    int* rrow = reinterpret_cast<int*>(gv + NB);                   // [NB] first box row of each node
    float* coef = reinterpret_cast<float*>(rrow + NB);
    __shared__ int cnt[2][2];   // per staging wave: batch nodes starting below S, below r1lo

    const int ci = xcd_block(int(blockIdx.x), int(gridDim.x));
    const int4 ch = a.chunks[ci];
    const int L = a.L;
    const int tid = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave index (uniform)
    int n0[3] = {0, 0, 0}, W[3] = {1, 1, 1};
    tile_geometry<2>(ch, a.tpd, a.tile, M2, n0, W);
    for (int e = tid; e < (M2 / 2) * kPolyCoef; e += blockDim.x) coef[e] = a.poly[e];
    {
        mfma_f4* z = reinterpret_cast<mfma_f4*>(ws);
        for (int e = tid; e < 64 * P / 4; e += blockDim.x) z[e] = mfma_f4{0.0f, 0.0f, 0.0f, 0.0f};
    }
    const int S = W[0] > 16 ? W[0] - 16 : 0;
    const int r1lo = min(S, max(0, 17 - M2));   // first box row from which a window reaches row 16
    mfma_f4 acc0[2][2], acc1[2][2];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            acc0[b][c] = mfma_f4{0.0f, 0.0f, 0.0f, 0.0f};
            acc1[b][c] = mfma_f4{0.0f, 0.0f, 0.0f, 0.0f};
        }

    const float* __restrict__ xs = static_cast<const float*>(a.xs);
    const Cx<float>* __restrict__ g = static_cast<const Cx<float>*>(a.g);
    const int jj = tid & (NB - 1), dim = tid >> 7;   // staging: node jj, dimension dim
    const int nbatch = (ch.z + NB - 1) / NB;
    // node of slot jj in batch b (slots past the chunk read its last node and are not used)
    auto node = [&](int b) { return int64_t(ch.y) + min(b * NB + jj, ch.z - 1); };
    struct Slot {
        float x;
        int p;
        Cx<float> gq;
    };
    Slot sa, sb;
    sa.x = xs[node(0) * 2 + dim];
    sa.p = a.perm[node(0)];
    sb.x = xs[node(1) * 2 + dim];
    sb.p = a.perm[node(1)];
    sa.gq = g[sa.p];
    int prev_r = -1;   // first table row this thread wrote for the previous batch (-1: none)
    // batch b from slot `use` (coordinate and value loaded); then the value of batch b + 1
    // into `other` and the coordinate and index of batch b + 2 into `use`
    auto batch = [&](int b, Slot& use, Slot& other) {
        const int nb = min(NB, ch.z - b * NB);
        __syncthreads();   // tables cleared / previous batch consumed
        int r = kMfmaFar;
        {
            float* wd = ws + dim * 32 * P + jj;   // this thread's column
            if (prev_r >= 0) {
#pragma unroll
                for (int o = 0; o < M2; ++o) wd[(prev_r + o) * P] = 0.0f;
            }
            prev_r = -1;
            if (jj < nb) {
                int nc;
                float th;
                cell_of<float>(use.x, L, nc, th);
                r = nc + L / 2 - n0[dim];
                float w[1][M2];
                weights_poly<1, M2, kPolyCoef>(&th, coef, w, a.edge_k);
#pragma unroll
                for (int o = 0; o < M2; ++o) wd[(r + o) * P] = w[0][o];
                prev_r = r;
            }
        }
        if (dim == 0) {
            gv[jj] = jj < nb ? use.gq : Cx<float>{0.0f, 0.0f};   // zero past the batch
            rrow[jj] = r;
            // the batch is sorted by box row: the counts below a row are prefix lengths
            const int below_s = __popcll(__ballot(r < S));
            const int below_r1 = __popcll(__ballot(r < r1lo));
            if ((tid & 63) == 0) {
                cnt[wv][0] = below_s;
                cnt[wv][1] = below_r1;
            }
        }
        other.gq = g[other.p];
        use.x = xs[node(b + 2) * 2 + dim];
        use.p = a.perm[node(b + 2)];
        __syncthreads();
        const int n0g = (cnt[0][0] + cnt[1][0] + 15) >> 4;   // band 0: nodes [0, #rows < S)
        const int s1 = (cnt[0][1] + cnt[1][1]) & ~15;         // band 1: nodes [s1, nb)
        const int n1g = (nb - s1 + 15) >> 4;
        for (int it = wv; it < n0g; it += 4) mfma2_item<0>(ws, gv, rrow, 16 * it, S, acc0);
        for (int it = n0g + ((wv - n0g) % 4 + 4) % 4; it < n0g + n1g; it += 4)
            mfma2_item<1>(ws, gv, rrow, s1 + 16 * (it - n0g), S, acc1);
    };
    for (int b = 0; b < nbatch; b += 2) {
        batch(b, sa, sb);
        if (b + 1 < nbatch) batch(b + 1, sb, sa);
    }

    // Sum the waves' accumulators in a fixed order.  red[w][band][re, im][row][column]
    // (16 x 32 per band) reuses the weight tables.
    __syncthreads();
    float* red = ws;
    {
        const int lane = tid & 63, kq = lane >> 4, i = lane & 15;
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int part = 0; part < 2; ++part)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int rc = (4 * kq + v) * 32 + 16 * bj + i;
                    red[((wv * 2 + 0) * 2 + part) * 512 + rc] = acc0[bj][part][v];
                    red[((wv * 2 + 1) * 2 + part) * 512 + rc] = acc1[bj][part][v];
                }
    }
    __syncthreads();
    const int vol = W[0] * W[1];
    for (int e = tid; e < vol; e += blockDim.x) {
        const int rho = e / W[1], c = e - rho * W[1];
        float re = 0.0f, im = 0.0f;
        if (rho < 16) {
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                re += red[((w * 2 + 0) * 2 + 0) * 512 + rho * 32 + c];
                im += red[((w * 2 + 0) * 2 + 1) * 512 + rho * 32 + c];
            }
        }
        if (rho >= S) {
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                re += red[((w * 2 + 1) * 2 + 0) * 512 + (rho - S) * 32 + c];
                im += red[((w * 2 + 1) * 2 + 1) * 512 + (rho - S) * 32 + c];
            }
        }
        box_store<float>(a, ci, e, Cx<float>{re, im});
    }
}

// d = 3 spreading by box columns.  Thread t owns the box column (c1, c2) = (t div 16,
// t mod 16) with every c0 in registers, so boxes of at most 16^3 points are covered by 256
// threads; wave w holds c1 in [4w, 4w + 4).  For a batch of the chunk's nodes, LDS holds
// the second and last dimensions' weights at absolute box coordinates (zero elsewhere) and
// the first dimension's weights by offset.  The batch is sorted by cell, so for each tile
// row r0 the nodes whose windows reach the wave's c1 range are one contiguous range; they
// add to c0 in [r0, r0 + 2m), fixed accumulator registers because r0 is a compile-time
// constant in each unrolled pass.  Nodes at the ends of a 16-byte group outside that range are masked.
// f(std::integral_constant<int, I>) for I = 0 .. N-1, each with I a constant expression.
template <int N, int I = 0, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<N, I + 1>(f);
    }
}

constexpr int kRows3Box = 16;                                // box extent bound per dimension
constexpr int kRows3Starts = kRows3Box * (kRows3Box + 1);    // [r0][r1] start table
template <typename R>
constexpr size_t rows3_lds_bytes(int M2) {
    return sizeof(R) * size_t(M2 + 2 * kRows3Box) * rows_pitch<R>() + sizeof(Cx<R>) * rows_batch<R>() +
           sizeof(int) * (rows_batch<R>() + kRows3Starts) + sizeof(float) * kMaxM * kPolyCoef;
}

template <typename R, int M2, int METHOD, bool EXACT>
__global__ void __launch_bounds__(256) k_spread_rows3(SpreadArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int m = M2 / 2;
    constexpr int NB = rows_batch<R>();
    constexpr int P = rows_pitch<R>();
    constexpr int VEC = 16 / int(sizeof(R));   // nodes per 16-byte load
    constexpr int C = kRows3Box;
    constexpr int R0 = C - M2 + 1;              // tile rows along the first dimension
    typedef R vec_t __attribute__((ext_vector_type(VEC)));
    R* w0s = reinterpret_cast<R*>(smem_raw);   // [M2][P]: first-dimension weight by offset
    R* w1s = w0s + M2 * P;                     // [C][P]: second-dimension weight at box c1
    R* w2s = w1s + C * P;                      // [C][P]: last-dimension weight at box c2
    Cx<R>* gv = reinterpret_cast<Cx<R>*>(w2s + C * P);   // [NB]
    int* key = reinterpret_cast<int*>(gv + NB);          // [NB]
    int* cstart = key + NB;                              // [r0 (C + 1) + r1]
    float* coef = reinterpret_cast<float*>(cstart + kRows3Starts);

    const int4 ch = a.chunks[xcd_block(int(blockIdx.x), int(gridDim.x))];
    const int L = a.L;
    const int tid = threadIdx.x;
    int n0[3] = {0, 0, 0}, W[3] = {1, 1, 1};
    tile_geometry<3>(ch, a.tpd, a.tile, M2, n0, W);
    const int T0 = a.tile[0], T1 = a.tile[1], T2 = a.tile[2];
    if constexpr (std::is_same<R, float>::value) {
        for (int e = tid; e < m * kPolyCoef; e += blockDim.x) coef[e] = a.poly[e];
    }
    const int wv = tid >> 6;
    const int c1 = tid >> 4, c2 = tid & (C - 1);
    // tile rows along the second dimension whose nodes reach box rows [4 wv, 4 wv + 4)
    const int r1lo = max(0, 4 * wv - M2 + 1), r1hi = min(T1 - 1, 4 * wv + 3);
    Cx<R> acc[C];
#pragma unroll
    for (int k = 0; k < C; ++k) acc[k] = Cx<R>{R(0), R(0)};

    const R* __restrict__ xs = static_cast<const R*>(a.xs);
    const Cx<R>* __restrict__ g = static_cast<const Cx<R>*>(a.g);
    const R beta = R(a.beta), cbeta = R(a.cb), inv_m2 = R(1) / R(m * m);
    for (int b0 = 0; b0 < ch.z; b0 += NB) {
        const int nb = min(NB, ch.z - b0);
        __syncthreads();   // coefficients staged / previous batch consumed
        {
            vec_t* z = reinterpret_cast<vec_t*>(w1s);
            for (int e = tid; e < 2 * C * P / VEC; e += blockDim.x) z[e] = vec_t(R(0));
        }
        __syncthreads();
        if (tid < nb) {
            const int64_t j = int64_t(ch.y) + b0 + tid;
            R theta[3];
            int r[3];
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                int nc;
                cell_of<R>(xs[j * 3 + t], L, nc, theta[t]);
                r[t] = nc + L / 2 - n0[t];
            }
            R w[3][M2];
            if constexpr (std::is_same<R, float>::value) {
                weights_poly<3, M2, kPolyCoef>(theta, coef, w, a.edge_k);
            } else if constexpr (!EXACT) {
                weights_poly64<3, M2, kPolyCoef64>(theta, a.poly64, w, double(a.edge_k));
            } else {
#pragma unroll
                for (int t = 0; t < 3; ++t) weights<R, M2, METHOD>(theta[t], beta, cbeta, inv_m2, w[t]);
            }
#pragma unroll
            for (int o = 0; o < M2; ++o) {
                w0s[o * P + tid] = w[0][o];
                w1s[(r[1] + o) * P + tid] = w[1][o];
                w2s[(r[2] + o) * P + tid] = w[2][o];
            }
            gv[tid] = g[a.perm[j]];
            key[tid] = (r[0] * T1 + r[1]) * T2 + r[2];
        } else if (tid < NB) {
            // past the batch (read at group ends, masked): finite zeros
#pragma unroll
            for (int o = 0; o < M2; ++o) w0s[o * P + tid] = R(0);
            gv[tid] = Cx<R>{R(0), R(0)};
        }
        __syncthreads();
        // cstart[r0 (C + 1) + r1] = first batch position in cell row (r0, r1) or later
        for (int e = tid; e < T0 * (T1 + 1); e += blockDim.x) {
            const int r0 = e / (T1 + 1), r1 = e - r0 * (T1 + 1);
            const int c = (r0 * T1 + r1) * T2;
            int lo = 0, hi = nb;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (key[mid] < c) lo = mid + 1;
                else hi = mid;
            }
            cstart[r0 * (C + 1) + r1] = lo;
        }
        __syncthreads();
        if (r1lo > r1hi) continue;
        const R* w1p = w1s + c1 * P;
        const R* w2p = w2s + c2 * P;
        static_for<R0>([&](auto r0c) __attribute__((always_inline)) {
            constexpr int r0 = decltype(r0c)::value;
            if (r0 >= T0) return;
            const int jb = cstart[r0 * (C + 1) + r1lo], je = cstart[r0 * (C + 1) + r1hi + 1];
            for (int j = jb & ~(VEC - 1); j < je; j += VEC) {
                const vec_t v1 = *reinterpret_cast<const vec_t*>(w1p + j);
                const vec_t v2 = *reinterpret_cast<const vec_t*>(w2p + j);
                vec_t v0[M2];
#pragma unroll
                for (int o = 0; o < M2; ++o) v0[o] = *reinterpret_cast<const vec_t*>(w0s + o * P + j);
#pragma unroll
                for (int q = 0; q < VEC; ++q) {
                    const Cx<R> gq = gv[j + q];
                    const bool in = j + q >= jb && j + q < je;
                    const R s = in ? v1[q] * v2[q] : R(0);
                    const R are = s * gq.re, aim = s * gq.im;
#pragma unroll
                    for (int o = 0; o < M2; ++o) {
                        acc[r0 + o].re = dev_fma(v0[o][q], are, acc[r0 + o].re);
                        acc[r0 + o].im = dev_fma(v0[o][q], aim, acc[r0 + o].im);
                    }
                }
            }
        });
    }

    if (c1 >= W[1] || c2 >= W[2]) return;
    const int ci = xcd_block(int(blockIdx.x), int(gridDim.x));
    static_for<C>([&](auto c0c) __attribute__((always_inline)) {
        constexpr int c0 = decltype(c0c)::value;
        if (c0 < W[0]) box_store<R>(a, ci, (c0 * W[1] + c1) * W[2] + c2, acc[c0]);
    });
}

// Double weights and their theta-derivatives from the double weight polynomials (layout
// of weights_poly64: per offset o, even then odd monomial coefficients in t = theta - 1/2;
// w_o = P_o(t), w_{2m-1-o} = P_o(-t), the edge pair times sqrt(1 - k theta) and
// sqrt(k theta + 1 - k)).  Used for windows without an exact device formula.
template <int D, int M2, int NC>
__device__ __forceinline__ void weights_poly64_deriv(const double* theta, const double* coef,
                                                     double (*w)[M2], double (*dw)[M2], double ek) {
    constexpr int m = M2 / 2;
    constexpr int NE = NC / 2;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const double t = theta[d] - 0.5, t2 = t * t;
#pragma unroll
        for (int o = 0; o < m; ++o) {
            const double* c = coef + o * NC;
            double E = c[NE - 1], Od = c[NC - 1], dE = 0.0, dO = 0.0;
#pragma unroll
            for (int k = NE - 2; k >= 0; --k) {
                dE = fma(dE, t2, E);
                E = fma(E, t2, c[k]);
                dO = fma(dO, t2, Od);
                Od = fma(Od, t2, c[NE + k]);
            }
            // p(t) = E + t O, q(t) = p(-t); dp/dtheta = A + B, dq/dtheta = A - B
            const double tO = t * Od;
            const double A = 2.0 * t * dE, B = fma(2.0 * t2, dO, Od);
            const double p = E + tO, q = E - tO, dp = A + B, dq = A - B;
            if (o == 0) {
                const double s1 = sqrt(fma(-ek, theta[d], 1.0));
                const double s0 = sqrt(fma(ek, theta[d], 1.0 - ek));
                w[d][0] = s1 * p;
                dw[d][0] = ek != 0.0 ? fma(s1, dp, -0.5 * ek * p / s1) : dp;
                w[d][M2 - 1] = s0 * q;
                dw[d][M2 - 1] = ek != 0.0 ? (s0 > 0.0 ? fma(s0, dq, 0.5 * ek * q / s0) : 0.0) : dq;
            } else {
                w[d][o] = p;
                w[d][M2 - 1 - o] = q;
                dw[d][o] = dp;
                dw[d][M2 - 1 - o] = dq;
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// DPOLY (double only): weights and derivatives from the double weight polynomials
// (windows without an exact device formula) instead of the sinh window's closed form.
template <typename R, int D, int M2, bool DPOLY>
__global__ void __launch_bounds__(256) k_grad_x(SpreadArgs a) {
    extern __shared__ unsigned char smem_raw[];
    Cx<R>* lds = reinterpret_cast<Cx<R>*>(smem_raw);
    constexpr int m = M2 / 2;
    const int4 ch = a.chunks[xcd_block(int(blockIdx.x), int(gridDim.x))];
    const int L = a.L;
    int n0[3] = {0, 0, 0}, W[3] = {1, 1, 1};
    tile_geometry<D>(ch, a.tpd, a.tile, M2, n0, W);
    const int total = W[0] * W[1] * W[2];
    const Cx<R>* __restrict__ th = static_cast<const Cx<R>*>(a.grid);
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        int rem = e;
        int64_t gidx = 0;
        bool ok = true;
#pragma unroll
        for (int t = D - 1; t >= 0; --t) {
            int ct = rem % W[t];
            rem /= W[t];
            int p = n0[t] - m + 1 + ct;
            if (p < 0 || p >= L) ok = false;
            int64_t st = 1;
            for (int s = t + 1; s < D; ++s) st *= L;
            gidx += int64_t(p) * st;
        }
        lds[e] = ok ? th[gidx] : Cx<R>{R(0), R(0)};
    }
    float* coef = reinterpret_cast<float*>(smem_raw + ((size_t(total) * sizeof(Cx<R>) + 15) & ~size_t(15)));
    if constexpr (std::is_same<R, float>::value) {
        for (int e = threadIdx.x; e < m * kPolyCoef; e += blockDim.x) coef[e] = a.poly[e];
    }
    __syncthreads();

    const R* __restrict__ xs = static_cast<const R*>(a.xs);
    const Cx<R>* __restrict__ g = static_cast<const Cx<R>*>(a.g);
    R* __restrict__ gx = static_cast<R*>(a.gx);
    const R beta = R(a.beta), cb = R(a.cb), inv_m2 = R(1) / R(m * m);
    for (int jj = threadIdx.x; jj < ch.z; jj += blockDim.x) {
        const int64_t j = int64_t(ch.y) + jj;
        R w[D][M2], dw[D][M2];
        R theta[D];
        int r[3] = {0, 0, 0};
#pragma unroll
        for (int t = 0; t < D; ++t) {
            int n;
            cell_of<R>(xs[j * D + t], L, n, theta[t]);
            r[t] = n + L / 2 - n0[t];
        }
        if constexpr (std::is_same<R, float>::value) {
            weights_poly_deriv<D, M2, kPolyCoef>(theta, coef, w, dw, a.edge_k);
        } else if constexpr (DPOLY) {
            weights_poly64_deriv<D, M2, kPolyCoef64>(theta, a.poly64, w, dw, double(a.edge_k));
        } else {
#pragma unroll
            for (int t = 0; t < D; ++t) weights_and_derivs<R, M2>(theta[t], beta, cb, inv_m2, w[t], dw[t]);
        }
        Cx<R> der[3];
        if constexpr (D == 1) {
            Plain<R> d0;
#pragma unroll
            for (int o = 0; o < M2; ++o) d0.add(dw[0][o], lds[r[0] + o]);
            der[0] = d0.value();
        } else if constexpr (D == 2) {
            Plain<R> d0, d1;
            const int base = r[0] * W[1] + r[1];
#pragma unroll
            for (int o0 = 0; o0 < M2; ++o0) {
                const Cx<R>* row = lds + base + o0 * W[1];
                Plain<R> ra, rd;
#pragma unroll
                for (int o1 = 0; o1 < M2; ++o1) {
                    ra.add(w[1][o1], row[o1]);
                    rd.add(dw[1][o1], row[o1]);
                }
                d0.add(dw[0][o0], ra.value());
                d1.add(w[0][o0], rd.value());
            }
            der[0] = d0.value();
            der[1] = d1.value();
        } else {
            Plain<R> d0, d1, d2;
            const int base = (r[0] * W[1] + r[1]) * W[2] + r[2];
            // first-dimension weights shifted down each step (no dynamic register index)
            R w0v[M2], dw0v[M2];
#pragma unroll
            for (int o = 0; o < M2; ++o) {
                w0v[o] = w[0][o];
                dw0v[o] = dw[0][o];
            }
#pragma unroll 1
            for (int o0 = 0; o0 < M2; ++o0) {
                Plain<R> pa, p1, p2;
#pragma unroll
                for (int o1 = 0; o1 < M2; ++o1) {
                    const Cx<R>* row = lds + base + (o0 * W[1] + o1) * W[2];
                    Plain<R> ra, rd;
#pragma unroll
                    for (int o2 = 0; o2 < M2; ++o2) {
                        ra.add(w[2][o2], row[o2]);
                        rd.add(dw[2][o2], row[o2]);
                    }
                    pa.add(w[1][o1], ra.value());
                    p1.add(dw[1][o1], ra.value());
                    p2.add(w[1][o1], rd.value());
                }
                d0.add(dw0v[0], pa.value());
                d1.add(w0v[0], p1.value());
                d2.add(w0v[0], p2.value());
#pragma unroll
                for (int o = 0; o + 1 < M2; ++o) {
                    w0v[o] = w0v[o + 1];
                    dw0v[o] = dw0v[o + 1];
                }
            }
            der[0] = d0.value();
            der[1] = d1.value();
            der[2] = d2.value();
        }
        const int32_t pj = a.perm[j];
        const Cx<R> gj = g[pj];
        const R Lr = R(L);
#pragma unroll
        for (int t = 0; t < D; ++t)
            gx[int64_t(pj) * D + t] = Lr * (gj.re * der[t].re + gj.im * der[t].im);
    }
}

using KFn = void (*)(SpreadArgs);

template <typename R, int D, int METHOD>
KFn spread_m(int m) {
    switch (m) {
        case 2: return k_spread<R, D, 4, METHOD>;
        case 3: return k_spread<R, D, 6, METHOD>;
        case 4: return k_spread<R, D, 8, METHOD>;
        case 5: return k_spread<R, D, 10, METHOD>;
        case 6: return k_spread<R, D, 12, METHOD>;
        case 7: return k_spread<R, D, 14, METHOD>;
        case 8: return k_spread<R, D, 16, METHOD>;
        default: return nullptr;
    }
}

template <typename R, int D, bool DPOLY>
KFn grad_m(int m) {
    switch (m) {
        case 2: return k_grad_x<R, D, 4, DPOLY>;
        case 3: return k_grad_x<R, D, 6, DPOLY>;
        case 4: return k_grad_x<R, D, 8, DPOLY>;
        case 5: return k_grad_x<R, D, 10, DPOLY>;
        case 6: return k_grad_x<R, D, 12, DPOLY>;
        case 7: return k_grad_x<R, D, 14, DPOLY>;
        case 8: return k_grad_x<R, D, 16, DPOLY>;
        default: return nullptr;
    }
}

template <typename R, int D, int METHOD>
KFn spread_os_m(int m) {
    switch (m) {
        case 2: return k_spread_os<R, D, 4, METHOD>;
        case 3: return k_spread_os<R, D, 6, METHOD>;
        case 4: return k_spread_os<R, D, 8, METHOD>;
        case 5: return k_spread_os<R, D, 10, METHOD>;
        case 6: return k_spread_os<R, D, 12, METHOD>;
        case 7: return k_spread_os<R, D, 14, METHOD>;
        case 8: return k_spread_os<R, D, 16, METHOD>;
        default: return nullptr;
    }
}

template <typename R, int METHOD, bool EXACT>
KFn spread_rows_m(int m, int rpl) {
    if (rpl == 8) {
        switch (m) {
            case 2: return k_spread_rows<R, 4, METHOD, EXACT, 8>;
            case 3: return k_spread_rows<R, 6, METHOD, EXACT, 8>;
            case 4: return k_spread_rows<R, 8, METHOD, EXACT, 8>;
            case 5: return k_spread_rows<R, 10, METHOD, EXACT, 8>;
            case 6: return k_spread_rows<R, 12, METHOD, EXACT, 8>;
            case 7: return k_spread_rows<R, 14, METHOD, EXACT, 8>;
            case 8: return k_spread_rows<R, 16, METHOD, EXACT, 8>;
            default: return nullptr;
        }
    }
    switch (m) {
        case 2: return k_spread_rows<R, 4, METHOD, EXACT>;
        case 3: return k_spread_rows<R, 6, METHOD, EXACT>;
        case 4: return k_spread_rows<R, 8, METHOD, EXACT>;
        case 5: return k_spread_rows<R, 10, METHOD, EXACT>;
        case 6: return k_spread_rows<R, 12, METHOD, EXACT>;
        case 7: return k_spread_rows<R, 14, METHOD, EXACT>;
        case 8: return k_spread_rows<R, 16, METHOD, EXACT>;
        default: return nullptr;
    }
}

KFn spread_mfma2_m(int m) {
    switch (m) {
        case 2: return k_spread_mfma2<4>;
        case 3: return k_spread_mfma2<6>;
        case 4: return k_spread_mfma2<8>;
        case 5: return k_spread_mfma2<10>;
        case 6: return k_spread_mfma2<12>;
        case 7: return k_spread_mfma2<14>;
        case 8: return k_spread_mfma2<16>;
        default: return nullptr;
    }
}

template <typename R, int METHOD, bool EXACT>
KFn spread_rows3_m(int m) {
    switch (m) {
        case 2: return k_spread_rows3<R, 4, METHOD, EXACT>;
        case 3: return k_spread_rows3<R, 6, METHOD, EXACT>;
        case 4: return k_spread_rows3<R, 8, METHOD, EXACT>;
        case 5: return k_spread_rows3<R, 10, METHOD, EXACT>;
        case 6: return k_spread_rows3<R, 12, METHOD, EXACT>;
        case 7: return k_spread_rows3<R, 14, METHOD, EXACT>;
        default: return nullptr;
    }
}

template <typename R, int METHOD>
KFn spread_os_d(int d, int m) {
    if (d == 1) return spread_os_m<R, 1, METHOD>(m);
    if (d == 2) return spread_os_m<R, 2, METHOD>(m);
    if (d == 3) return spread_os_m<R, 3, METHOD>(m);
    return nullptr;
}

template <typename R, int METHOD>
KFn spread_d(int d, int m) {
    if (d == 1) return spread_m<R, 1, METHOD>(m);
    if (d == 2) return spread_m<R, 2, METHOD>(m);
    if (d == 3) return spread_m<R, 3, METHOD>(m);
    return nullptr;
}

template <typename R, bool DPOLY>
KFn grad_d(int d, int m) {
    if (d == 1) return grad_m<R, 1, DPOLY>(m);
    if (d == 2) return grad_m<R, 2, DPOLY>(m);
    if (d == 3) return grad_m<R, 3, DPOLY>(m);
    return nullptr;
}

// ---------------------------------------------------------------- box merge
struct MergeArgs {
    const void* boxes;
    void* grid;
    const int32_t* tile_count;   // nodes per tile
    const int32_t* chunk_off;    // first chunk of each tile
    const int* cov;              // coverage table, kCovRow ints per coordinate (or null):
                                 // tile of p, count, (tile offset, box position) pairs
    int periodic;                // tile offsets wrap (Algorithm 2.1)
    int prezeroed;               // the grid was zero-filled before the merge
    const unsigned char* reach;  // per tile: some non-empty box covers it (null: not marked)
    int64_t box_vol, n;
    int L, m, cap;
    int tile[3], tpd[3], W[3];
};
using KFnM = void (*)(MergeArgs);

__device__ __forceinline__ int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// Calls f(tc, c) for every tile tc (of tpd, edge T) whose box covers grid coordinate p along
// one dimension, c being p's position in that box: box points n0 - m + 1 + c, c < W, with
// n0 = tc T, reach p itself (zero-extended sums) or p + s L (periodic sums, boxes wrap).
template <int METHOD, typename F>
__device__ __forceinline__ void covering(int p, int L, int T, int tpd, int m, int W, F&& f) {
    constexpr int s_lo = METHOD == 1 ? -1 : 0, s_hi = METHOD == 1 ? 2 : 0;
#pragma unroll
    for (int s = s_lo; s <= s_hi; ++s) {
        const int q = p + s * L;
        const int lo = max(0, floor_div(q + m - W + T - 1, T));   // ceil((q + m - W) / T)
        const int hi = min(tpd - 1, floor_div(q + m - 1, T));
        for (int tc = lo; tc <= hi; ++tc) f(tc, q + m - 1 - tc * T);
    }
}

// One thread per grid point: the sum of the covering boxes' entries, over tiles in row-major
// order (and s), and over each tile's chunks in order.  Every grid point is written.  This general form derives the covering tiles by division;
// k_box_merge_tiles below reads them from per-coordinate tables and is used whenever those
// fit.
template <typename R, int D, int METHOD>
__global__ void __launch_bounds__(256) k_box_merge(MergeArgs a) {
    int p[3] = {0, 0, 0};
    p[D - 1] = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (p[D - 1] >= a.L) return;
    if (D >= 2) p[D - 2] = int(blockIdx.y);
    if (D == 3) p[0] = int(blockIdx.z);
    int64_t gi = 0;
#pragma unroll
    for (int t = 0; t < D; ++t) gi = gi * a.L + p[t];
    const Cx<R>* __restrict__ boxes = static_cast<const Cx<R>*>(a.boxes);
    R re = R(0), im = R(0);
    auto add_tile = [&](int tile, int e) {   // the tile's chunks in order
        const int cnt = a.tile_count[tile];
        if (cnt == 0) return;
        const int nch = (cnt + a.cap - 1) / a.cap;
        const int64_t base = int64_t(a.chunk_off[tile]) * a.box_vol + e;
        for (int k = 0; k < nch; ++k) {
            const Cx<R> v = boxes[base + int64_t(k) * a.box_vol];
            re += v.re;
            im += v.im;
        }
    };
    if constexpr (D == 1) {
        covering<METHOD>(p[0], a.L, a.tile[0], a.tpd[0], a.m, a.W[0], [&](int t0, int c0) { add_tile(t0, c0); });
    } else if constexpr (D == 2) {
        covering<METHOD>(p[0], a.L, a.tile[0], a.tpd[0], a.m, a.W[0], [&](int t0, int c0) {
            covering<METHOD>(p[1], a.L, a.tile[1], a.tpd[1], a.m, a.W[1], [&](int t1, int c1) {
                add_tile(t0 * a.tpd[1] + t1, c0 * a.W[1] + c1);
            });
        });
    } else {
        covering<METHOD>(p[0], a.L, a.tile[0], a.tpd[0], a.m, a.W[0], [&](int t0, int c0) {
            covering<METHOD>(p[1], a.L, a.tile[1], a.tpd[1], a.m, a.W[1], [&](int t1, int c1) {
                covering<METHOD>(p[2], a.L, a.tile[2], a.tpd[2], a.m, a.W[2], [&](int t2, int c2) {
                    add_tile((t0 * a.tpd[1] + t1) * a.tpd[2] + t2, (c0 * a.W[1] + c1) * a.W[2] + c2);
                });
            });
        });
    }
    static_cast<Cx<R>*>(a.grid)[gi] = Cx<R>{re, im};
}

// Per-tile flag (d = 3): does the box of some non-empty tile cover a point of this tile?  Cleared,
// then marked from the non-empty tiles: tile t spans box coordinates t T - m + 1 ...
// t T + T + m - 2 per dimension (wrapped for the periodic sums), and every tile holding
// one of them is marked (the same value from every writer).  Launched over the tiles as a
// 3-D grid (last dimension in x), so no index is divided.
constexpr int kReachList = 8;
__global__ void k_reach_clear(unsigned char* reach, int64_t ntiles) {
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t < ntiles) reach[t] = 0;
}

template <int D, int METHOD>
__global__ void __launch_bounds__(256) k_reach_mark(MergeArgs a, unsigned char* reach) {
    int tc[3] = {0, 0, 0};
    tc[D - 1] = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (tc[D - 1] >= a.tpd[D - 1]) return;
    if (D >= 2) tc[D - 2] = int(blockIdx.y);
    if (D == 3) tc[0] = int(blockIdx.z);
    int t = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) t = t * a.tpd[k] + tc[k];
    if (a.tile_count[t] == 0) return;
    int list[3][kReachList], n[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const int T = a.tile[k];
        const int c0 = tc[k] * T - a.m + 1, c1 = tc[k] * T + T + a.m - 2;
        int last = -1;
        for (int c = c0; c <= c1; ++c) {
            int q = c;
            if (METHOD == 1) q = ((q % a.L) + a.L) % a.L;
            else if (q < 0 || q >= a.L) continue;
            const int tt = q / T;
            if (tt == last) continue;
            last = tt;
            bool seen = false;
            for (int e = 0; e < n[k]; ++e) seen = seen || list[k][e] == tt;
            if (!seen && n[k] < kReachList) list[k][n[k]++] = tt;
        }
    }
    if constexpr (D == 1) {
        for (int i = 0; i < n[0]; ++i) reach[list[0][i]] = 1;
    } else if constexpr (D == 2) {
        for (int i = 0; i < n[0]; ++i)
            for (int j = 0; j < n[1]; ++j) reach[list[0][i] * a.tpd[1] + list[1][j]] = 1;
    } else {
        for (int i = 0; i < n[0]; ++i)
            for (int j = 0; j < n[1]; ++j)
                for (int k = 0; k < n[2]; ++k) reach[(list[0][i] * a.tpd[1] + list[1][j]) * a.tpd[2] + list[2][k]] = 1;
    }
}

// Zero fill of the spreading grid (16-byte stores; n16 of them).
__global__ void __launch_bounds__(256) k_grid_zero(uint4* g, int64_t n16) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < n16) g[i] = make_uint4(0u, 0u, 0u, 0u);
}

// The merge, one workgroup per tile.  The workgroup first stages, for every neighbour offset
// (dt_0, ..., dt_{d-1}) in [-kNbR, kNbR]^d, the first chunk box of that neighbour and its
// chunk count (-1 for an empty or absent tile).  A tile that no non-empty box reaches is
// written with zeros, or left as it is when the grid was zero-filled before (d = 3, where
// most tiles of clustered nodes are such tiles and a streaming fill writes them faster than
// tile by tile); otherwise every point of the tile is
// the sum over the (offset, box position) pairs of its coordinates' coverage rows, in
// row-major order of the pairs and chunk order within a tile (each chunk-box entry is read
// exactly once, by the one grid point it covers).
template <typename R, int D>
__global__ void __launch_bounds__(256) k_box_merge_tiles(MergeArgs a) {
    constexpr int NB = 2 * kNbR + 1;
    constexpr int NBV = D == 1 ? NB : D == 2 ? NB * NB : NB * NB * NB;
    __shared__ long long nb[NBV];    // first box of the neighbour tile (-1: none)
    __shared__ int nbc[NBV];         // its chunk count
    // d <= 2: each XCD takes a contiguous run of tiles, so that neighbouring tiles, which
    // read the same cache lines of their common boxes, share that XCD's L2 (d = 2 headline
    // merge 15.5 -> 14.1 us).  Not for d = 3, whose clustered nodes would put the dense
    // tiles on a few XCDs (122 -> 145 us).
    const int t = D <= 2 ? xcd_block(int(blockIdx.x), int(gridDim.x)) : int(blockIdx.x);
    if (a.reach && !a.reach[t]) return;   // marked unreached on a zero-filled grid
    int tc[3] = {0, 0, 0}, n0[3] = {0, 0, 0}, ext[3] = {1, 1, 1};
    {
        int r = t;
#pragma unroll
        for (int k = D - 1; k >= 0; --k) {
            tc[k] = r % a.tpd[k];
            r /= a.tpd[k];
            n0[k] = tc[k] * a.tile[k];
            ext[k] = min(a.tile[k], a.L - n0[k]);
        }
    }
    int reached = 0;   // some neighbour within reach has nodes
    for (int q = threadIdx.x; q < NBV; q += blockDim.x) {
        int rem = q, tt = 0;
        bool ok = true;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const int stride = D - 1 - k == 2 ? NB * NB : D - 1 - k == 1 ? NB : 1;
            const int dk = rem / stride - kNbR;
            rem %= stride;
            int u = tc[k] + dk;
            if (a.periodic) u = ((u % a.tpd[k]) + a.tpd[k]) % a.tpd[k];
            else ok = ok && u >= 0 && u < a.tpd[k];
            tt = tt * a.tpd[k] + (u < 0 ? 0 : u);
        }
        const int cnt = ok ? a.tile_count[tt] : 0;
        nb[q] = cnt > 0 ? (long long)a.chunk_off[tt] * a.box_vol : -1;
        nbc[q] = (cnt + a.cap - 1) / a.cap;
        reached = reached || cnt > 0;
    }
    reached = __syncthreads_or(reached);   // also the barrier after the tables
    const Cx<R>* __restrict__ boxes = static_cast<const Cx<R>*>(a.boxes);
    Cx<R>* __restrict__ grid = static_cast<Cx<R>*>(a.grid);
    const int vol = ext[0] * ext[1] * ext[2];
    if (!reached) {
        if (a.prezeroed) return;
        for (int e = threadIdx.x; e < vol; e += blockDim.x) {
            int r = e;
            int64_t gi = 0, stride = 1;
#pragma unroll
            for (int k = D - 1; k >= 0; --k) {
                gi += (n0[k] + r % ext[k]) * stride;
                r /= ext[k];
                stride *= a.L;
            }
            grid[gi] = Cx<R>{R(0), R(0)};
        }
        return;
    }
    for (int e = threadIdx.x; e < vol; e += blockDim.x) {
        int p[3] = {0, 0, 0};
        {
            int r = e;
#pragma unroll
            for (int k = D - 1; k >= 0; --k) {
                p[k] = n0[k] + r % ext[k];
                r /= ext[k];
            }
        }
        const int* r0 = a.cov + p[0] * kCovRow;
        const int* r1 = a.cov + p[D >= 2 ? 1 : 0] * kCovRow;
        const int* r2 = a.cov + p[D == 3 ? 2 : 0] * kCovRow;
        const int n0c = r0[1], n1c = D >= 2 ? r1[1] : 1, n2c = D == 3 ? r2[1] : 1;
        R re = R(0), im = R(0);
        // At most two covering boxes per coordinate, none of a tile with several chunks
        // (decided from the staged tables before any box is read): every read is issued
        // before the first add, and the terms are summed in the order of the general loop
        // below (an absent term adds +0, which changes no sum that starts at +0), so both
        // forms give the same bits.
        bool done = false;
        if (n0c <= 2 && n1c <= 2 && n2c <= 2) {
            constexpr int K1 = D >= 2 ? 2 : 1, K2 = D == 3 ? 2 : 1, K = 2 * K1 * K2;
            int slot[K], be[K];
            bool single = true;   // every present covering tile has one chunk
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < K1; ++j)
#pragma unroll
                    for (int k = 0; k < K2; ++k) {
                        const int q = (i * K1 + j) * K2 + k;
                        slot[q] = -1;
                        be[q] = 0;
                        if (i < n0c && j < n1c && k < n2c) {
                            const int o0 = r0[2 + 2 * i] + kNbR, c0 = r0[3 + 2 * i];
                            const int o1 = D >= 2 ? r1[2 + 2 * j] + kNbR : 0, c1 = D >= 2 ? r1[3 + 2 * j] : 0;
                            const int o2 = D == 3 ? r2[2 + 2 * k] + kNbR : 0, c2 = D == 3 ? r2[3 + 2 * k] : 0;
                            slot[q] = D == 1 ? o0 : D == 2 ? o0 * NB + o1 : (o0 * NB + o1) * NB + o2;
                            be[q] = D == 1 ? c0 : D == 2 ? c0 * a.W[1] + c1 : (c0 * a.W[1] + c1) * a.W[2] + c2;
                            single = single && nbc[slot[q]] <= 1;
                        }
                    }
            if (single) {
                Cx<R> v[K];
#pragma unroll
                for (int q = 0; q < K; ++q) {
                    v[q] = Cx<R>{R(0), R(0)};
                    const long long base = slot[q] >= 0 ? nb[slot[q]] : -1;
                    if (base >= 0) v[q] = boxes[base + be[q]];
                }
#pragma unroll
                for (int q = 0; q < K; ++q) {
                    re += v[q].re;
                    im += v[q].im;
                }
                done = true;
            }
        }
        for (int i = 0; i < (done ? 0 : n0c); ++i) {
            const int o0 = r0[2 + 2 * i] + kNbR, c0 = r0[3 + 2 * i];
            for (int j = 0; j < n1c; ++j) {
                const int o1 = D >= 2 ? r1[2 + 2 * j] + kNbR : 0, c1 = D >= 2 ? r1[3 + 2 * j] : 0;
#pragma unroll 4
                for (int k = 0; k < n2c; ++k) {
                    const int o2 = D == 3 ? r2[2 + 2 * k] + kNbR : 0, c2 = D == 3 ? r2[3 + 2 * k] : 0;
                    const int slot = D == 1 ? o0 : D == 2 ? o0 * NB + o1 : (o0 * NB + o1) * NB + o2;
                    const int be = D == 1 ? c0 : D == 2 ? c0 * a.W[1] + c1 : (c0 * a.W[1] + c1) * a.W[2] + c2;
                    const long long base = nb[slot];
                    if (base >= 0) {
                        const int nch = nbc[slot];
#pragma unroll 4
                        for (int c = 0; c < nch; ++c) {   // the tile's chunks in order
                            const Cx<R> v = boxes[base + int64_t(c) * a.box_vol + be];
                            re += v.re;
                            im += v.im;
                        }
                    }
                }
            }
        }
        int64_t gi = p[0];
        if (D >= 2) gi = gi * a.L + p[1];
        if (D == 3) gi = gi * a.L + p[2];
        grid[gi] = Cx<R>{re, im};
    }
}

template <typename R, int METHOD>
KFnM merge_d(int d) {
    if (d == 1) return k_box_merge<R, 1, METHOD>;
    if (d == 2) return k_box_merge<R, 2, METHOD>;
    return k_box_merge<R, 3, METHOD>;
}

template <typename R>
KFnM merge_tiles_d(int d) {
    if (d == 1) return k_box_merge_tiles<R, 1>;
    if (d == 2) return k_box_merge_tiles<R, 2>;
    return k_box_merge_tiles<R, 3>;
}

SpreadArgs make_args(const Plan& p) {
    SpreadArgs a{};
    a.xs = p.d_xs;
    a.perm = p.d_perm;
    a.chunks = p.d_chunks;
    a.L = int(p.L);
    for (int t = 0; t < 3; ++t) {
        a.tile[t] = p.tile[t];
        a.tpd[t] = p.tiles_per_dim[t];
    }
    a.beta = p.beta;
    a.cb = 1.0 / (-std::expm1(-2.0 * p.beta));
    a.wf = make_win_f32(p);
    for (size_t i = 0; i < p.poly.size() && i < size_t(kMaxM * kPolyCoef); ++i) a.poly[i] = p.poly[i];
    for (size_t i = 0; i < p.poly64.size() && i < size_t(kMaxM * kPolyCoef64); ++i) a.poly64[i] = p.poly64[i];
    a.use_poly64 = p.use_poly64 ? 1 : 0;
    a.edge_k = float(p.edge_k);
    return a;
}

}  // namespace

int64_t spread_box_vol(const Plan& p) {
    int64_t v = 1;
    for (int t = 0; t < p.d; ++t) v *= p.tile[t] + 2 * p.m - 1;
    return v;
}

size_t spread_boxes_bytes(const Plan& p) {
    return size_t(std::max<int64_t>(p.nchunks, 1)) * size_t(spread_box_vol(p)) * p.cplx_size();
}

bl_status launch_spread(Plan& p, const void* g, void* grid, void* boxes) {
    SpreadArgs a = make_args(p);
    a.g = g;
    a.grid = grid;
    a.boxes = boxes;
    a.box_vol = spread_box_vol(p);
    MergeArgs ma{};
    ma.boxes = boxes;
    ma.grid = grid;
    ma.tile_count = p.d_tile_count;
    ma.chunk_off = p.d_chunk_offset;
    ma.box_vol = a.box_vol;
    ma.n = p.grid_elems();
    ma.L = int(p.L);
    ma.m = p.m;
    ma.cap = p.chunk_cap;
    for (int t = 0; t < 3; ++t) {
        ma.tile[t] = p.tile[t];
        ma.tpd[t] = p.tiles_per_dim[t];
        ma.W[t] = p.tile[t] + 2 * p.m - 1;
    }
    ma.cov = p.d_cov;
    ma.periodic = p.method == BL_NFFT ? 1 : 0;
    auto merge = [&]() -> bl_status {
        KFnM mf;
        if (p.d_cov) {
            if (p.d == 3 && p.d_reach) {
                // clustered d = 3 nodes leave most tiles unreached: mark the reached ones from
                // the non-empty tiles and zero-fill the grid first
                hipLaunchKernelGGL(k_reach_clear, dim3(unsigned((p.ntiles + 255) / 256)), dim3(256), 0, p.stream,
                                   p.d_reach, p.ntiles);
                const dim3 tg(unsigned((p.tiles_per_dim[2] + 255) / 256), unsigned(p.tiles_per_dim[1]),
                              unsigned(p.tiles_per_dim[0]));
                void (*rf)(MergeArgs, unsigned char*) = p.method == BL_NFFT ? k_reach_mark<3, 1> : k_reach_mark<3, 0>;
                hipLaunchKernelGGL(rf, tg, dim3(256), 0, p.stream, ma, p.d_reach);
                const int64_t bytes = p.grid_elems() * int64_t(p.cplx_size());   // a multiple of 16 (L even)
                hipLaunchKernelGGL(k_grid_zero, dim3(unsigned((bytes / 16 + 255) / 256)), dim3(256), 0, p.stream,
                                   static_cast<uint4*>(grid), bytes / 16);
                ma.prezeroed = 1;
                ma.reach = p.d_reach;
            }
            mf = p.prec == BL_F64 ? merge_tiles_d<double>(p.d) : merge_tiles_d<float>(p.d);
            // d = 2: two points per thread (128 threads for a 16 x 16 tile), so that every
            // tile of a CU's share is resident at once
            const unsigned nt = p.d == 2 ? 128u : 256u;
            hipLaunchKernelGGL(mf, dim3(unsigned(p.ntiles)), dim3(nt), 0, p.stream, ma);
            BL_HIP(hipGetLastError());
            return BL_OK;
        } else {
            mf = p.prec == BL_F64 ? (p.method == BL_NFFT ? merge_d<double, 1>(p.d) : merge_d<double, 0>(p.d))
                                  : (p.method == BL_NFFT ? merge_d<float, 1>(p.d) : merge_d<float, 0>(p.d));
        }
        const dim3 g(unsigned((p.L + 255) / 256), p.d >= 2 ? unsigned(p.L) : 1u, p.d == 3 ? unsigned(p.L) : 1u);
        hipLaunchKernelGGL(mf, g, dim3(256), 0, p.stream, ma);
        BL_HIP(hipGetLastError());
        return BL_OK;
    };
    if (p.N == 0 || p.nchunks == 0) return merge();   // every tile empty: zeros
    // Row kernels (d = 2: box edges <= 32; d = 3: <= 16); otherwise the output-stationary
    // kernel when the box fits its points per thread and its LDS fits; otherwise the
    // LDS-atomic kernel.  BL_SPREAD_OS / BL_SPREAD_ATOMIC force the latter two.
    int64_t box = 1, ncell = 1;
    for (int t = 0; t < p.d; ++t) {
        box *= p.tile[t] + 2 * p.m - 1;
        ncell *= p.tile[t];
    }
    const int kp = p.d == 1 ? os_points<1>() : p.d == 2 ? os_points<2>() : os_points<3>();
    const size_t rs = p.prec == BL_F64 ? 8 : 4;
    const size_t os_lds = ((rs * p.d * 2 * p.m * kOsBatch + 2 * rs * kOsBatch + 4 * kOsBatch +
                            4 * size_t(ncell + 1) + 15) & ~size_t(15)) + sizeof(float) * kMaxM * kPolyCoef;
    const bool by_rows = std::getenv("BL_SPREAD_ATOMIC") == nullptr && std::getenv("BL_SPREAD_OS") == nullptr;
    const bool use_rows = by_rows && p.d == 2 && p.tile[0] + 2 * p.m - 1 <= 32 && p.tile[1] + 2 * p.m - 1 <= 32;
    bool use_rows3 = by_rows && p.d == 3 && p.m <= 7;
    for (int t = 0; t < 3 && use_rows3; ++t) use_rows3 = p.tile[t] + 2 * p.m - 1 <= kRows3Box;
    const bool use_os = !use_rows && !use_rows3 && box <= int64_t(kp) * kOsThreads && os_lds <= 160 * 1024 &&
                        std::getenv("BL_SPREAD_ATOMIC") == nullptr;
    KFn fn;
    // d = 2 row kernel: box rows per lane, 4 (eight rows per lane measured slower;
    // BL_SPREAD_RPL=8 selects them)
    int rpl = 4;
    if (const char* e = std::getenv("BL_SPREAD_RPL")) rpl = std::atoi(e) == 8 ? 8 : 4;
    // Double row kernels with closed-form weights are separate instantiations, so that the
    // polynomial ones are not register-sized for them.
    const bool exact = p.prec == BL_F64 && !p.use_poly64;
    // float d = 2 boxes run on the matrix cores unless BL_SPREAD_ROWS asks for the row kernel
    const bool use_mfma2 = use_rows && p.prec != BL_F64 && std::getenv("BL_SPREAD_ROWS") == nullptr;
    if (use_mfma2) {
        const KFn fp = spread_mfma2_m(p.m);
        if (!fp) {
            set_error("no spreading kernel for this (d, m)");
            return BL_EUNSUPPORTED;
        }
        hipLaunchKernelGGL(fp, dim3(unsigned(p.nchunks)), dim3(256), mfma2_lds_bytes(), p.stream, a);
        BL_HIP(hipGetLastError());
        return merge();
    }
    if (use_rows) {
        if (p.prec != BL_F64) fn = p.method == BL_NFFT ? spread_rows_m<float, 1, false>(p.m, rpl) : spread_rows_m<float, 0, false>(p.m, rpl);
        else if (exact) fn = p.method == BL_NFFT ? spread_rows_m<double, 1, true>(p.m, rpl) : spread_rows_m<double, 0, true>(p.m, rpl);
        else fn = p.method == BL_NFFT ? spread_rows_m<double, 1, false>(p.m, rpl) : spread_rows_m<double, 0, false>(p.m, rpl);
    } else if (use_rows3) {
        if (p.prec != BL_F64) fn = p.method == BL_NFFT ? spread_rows3_m<float, 1, false>(p.m) : spread_rows3_m<float, 0, false>(p.m);
        else if (exact) fn = p.method == BL_NFFT ? spread_rows3_m<double, 1, true>(p.m) : spread_rows3_m<double, 0, true>(p.m);
        else fn = p.method == BL_NFFT ? spread_rows3_m<double, 1, false>(p.m) : spread_rows3_m<double, 0, false>(p.m);
    } else if (use_os) {
        if (p.prec == BL_F64) fn = p.method == BL_NFFT ? spread_os_d<double, 1>(p.d, p.m) : spread_os_d<double, 0>(p.d, p.m);
        else fn = p.method == BL_NFFT ? spread_os_d<float, 1>(p.d, p.m) : spread_os_d<float, 0>(p.d, p.m);
    } else {
        if (p.prec == BL_F64) fn = p.method == BL_NFFT ? spread_d<double, 1>(p.d, p.m) : spread_d<double, 0>(p.d, p.m);
        else fn = p.method == BL_NFFT ? spread_d<float, 1>(p.d, p.m) : spread_d<float, 0>(p.d, p.m);
    }
    if (!fn) {
        set_error("no spreading kernel for this (d, m)");
        return BL_EUNSUPPORTED;
    }
    const size_t lds = use_rows ? (p.prec == BL_F64 ? rows_lds_bytes<double>() : rows_lds_bytes<float>())
                       : use_rows3 ? (p.prec == BL_F64 ? rows3_lds_bytes<double>(2 * p.m) : rows3_lds_bytes<float>(2 * p.m))
                       : use_os ? os_lds : box_bytes(p) + 16 + sizeof(float) * kMaxM * kPolyCoef;
    if (lds > 64 * 1024)
        BL_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    const unsigned threads = use_rows ? unsigned(1024 / rpl) : 256u;
    hipLaunchKernelGGL(fn, dim3(unsigned(p.nchunks)), dim3(threads), lds, p.stream, a);
    BL_HIP(hipGetLastError());
    return merge();
}

// ---------------------------------------------------------------- allocation-free adjoint
// Spreading target of bl_adjoint_noalloc: a file-scope device array instead of plan memory,
// for callers that cannot allocate (code under stream capture, serving loops).  Every GPU
// the library runs on holds one copy until the process ends; all calls on one GPU share it,
// so such calls that overlap in time on one GPU race.  In host code `scratch` is only a
// stand-in for the symbol: its device address comes from hipGetSymbolAddress, looked up
// once per device with that device current, and only that address is passed to kernels.
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
constexpr int kNoallocMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoallocMaxDevices] = {};

// Device address of `scratch` on the current device (which must be `device`).
bl_status scratch_address(int device, void** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= kNoallocMaxDevices) {
        set_error("device index above the allocation-free entry point's table");
        return BL_EUNSUPPORTED;
    }
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr) {
            set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return BL_EDEVICE;
        }
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return BL_OK;
}
}  // namespace

size_t noalloc_scratch_bytes() { return kNoallocScratchBytes; }

bl_status launch_adjoint_noalloc(Plan& p, const void* g, void* fhat_out) {
    const size_t grid_bytes = (size_t(p.grid_elems()) * p.cplx_size() + 255) & ~size_t(255);
    const size_t need = grid_bytes + spread_boxes_bytes(p);
    if (need > kNoallocScratchBytes) {
        set_error("bl_adjoint_noalloc: the spreading grid and chunk boxes (" + std::to_string(need) +
                  " bytes) exceed its fixed device scratch of " + std::to_string(kNoallocScratchBytes) +
                  " bytes; use bl_adjoint");
        return BL_EUNSUPPORTED;
    }
    void* base = nullptr;
    BL_TRY(scratch_address(p.device, &base));
    // grid first, then the chunk boxes; every box entry and every grid point is written
    // before it is read, so the array's contents from an earlier call never show
    void* grid = base;
    void* boxes = static_cast<unsigned char*>(base) + grid_bytes;
    BL_TRY(launch_spread(p, g, grid, boxes));
    return launch_adjoint_fft(p, grid, fhat_out);
}

bl_status launch_grad_x(Plan& p, const void* g, void* gx) {
    if (p.N == 0 || p.nchunks == 0) return BL_OK;
    // FP64: the sinh window's closed form, else (checked at bl_grad_x) the polynomials'
    KFn fn = p.prec != BL_F64 ? grad_d<float, false>(p.d, p.m)
             : p.win == BL_WIN_SINH ? grad_d<double, false>(p.d, p.m) : grad_d<double, true>(p.d, p.m);
    if (!fn) {
        set_error("no gradient kernel for this (d, m)");
        return BL_EUNSUPPORTED;
    }
    SpreadArgs a = make_args(p);
    a.g = g;
    a.grid = p.d_grid;
    a.gx = gx;
    const size_t lds = box_bytes(p) + 16 + sizeof(float) * kMaxM * kPolyCoef;
    if (lds > 64 * 1024)
        BL_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    hipLaunchKernelGGL(fn, dim3(unsigned(p.nchunks)), dim3(256), lds, p.stream, a);
    BL_HIP(hipGetLastError());
    return BL_OK;
}

}  // namespace bl
