// Adjoint spreading (Psi^T g of the factorisation (4.11), or B^T g for Algorithm 2.1) and
// the node gradient d f_j / d x_jt of the short sums (4.8).
//
// Spreading runs one workgroup per binning chunk (all its nodes share one tile): each
// node adds g_j psi(x_j - l/L) to the (2m)^d cells around it in an LDS copy of the tile
// plus halo (LDS atomics), and the workgroup then adds that copy to the grid in HBM with
// hardware float atomics.  Cells outside I_L are dropped (Psi has columns l in I_L only)
// or wrapped (periodic B).  Summation order across threads is not fixed, so results can
// differ in the last bits between runs.
//
// The gradient kernel mirrors the short-sum kernel, with psi' in one dimension:
//   d f_j / d x_jt = L sum_l theta_l psi_g'(u_t) prod_{s != t} psi_g(u_s).
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
};

template <typename R>
__global__ void k_zero(Cx<R>* p, int64_t n) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = Cx<R>{R(0), R(0)};
}

__device__ __forceinline__ void lds_add(float* p, float v) { atomicAdd(p, v); }
__device__ __forceinline__ void lds_add(double* p, double v) { atomicAdd(p, v); }
__device__ __forceinline__ void hbm_add(float* p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void hbm_add(double* p, double v) { unsafeAtomicAdd(p, v); }

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
    const int4 ch = a.chunks[blockIdx.x];
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
            weights_poly<D, M2, kPolyCoef>(theta, coef, w);
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

    R* __restrict__ grid = static_cast<R*>(a.grid);
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const R vre = acc[2 * e], vim = acc[2 * e + 1];
        if (vre == R(0) && vim == R(0)) continue;
        int rem = e;
        int64_t gidx = 0;
        bool ok = true;
#pragma unroll
        for (int t = D - 1; t >= 0; --t) {
            int ct = rem % W[t];
            rem /= W[t];
            int p = n0[t] - m + 1 + ct;
            if (METHOD == 1) {
                p = (p % L + L) % L;
            } else if (p < 0 || p >= L) {
                ok = false;
            }
            int64_t st = 1;
            for (int s = t + 1; s < D; ++s) st *= L;
            gidx += int64_t(p) * st;
        }
        if (!ok) continue;
        hbm_add(grid + 2 * gidx, vre);
        hbm_add(grid + 2 * gidx + 1, vim);
    }
}

template <typename R, int D, int M2>
__global__ void __launch_bounds__(256) k_grad_x(SpreadArgs a) {
    extern __shared__ unsigned char smem_raw[];
    Cx<R>* lds = reinterpret_cast<Cx<R>*>(smem_raw);
    constexpr int m = M2 / 2;
    const int4 ch = a.chunks[blockIdx.x];
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
    __syncthreads();

    const R* __restrict__ xs = static_cast<const R*>(a.xs);
    const Cx<R>* __restrict__ g = static_cast<const Cx<R>*>(a.g);
    R* __restrict__ gx = static_cast<R*>(a.gx);
    const R beta = R(a.beta), cb = R(a.cb), inv_m2 = R(1) / R(m * m);
    for (int jj = threadIdx.x; jj < ch.z; jj += blockDim.x) {
        const int64_t j = int64_t(ch.y) + jj;
        R w[D][M2], dw[D][M2];
        int r[3] = {0, 0, 0};
#pragma unroll
        for (int t = 0; t < D; ++t) {
            int n;
            R theta;
            cell_of<R>(xs[j * D + t], L, n, theta);
            r[t] = n + L / 2 - n0[t];
            weights_and_derivs<R, M2>(theta, beta, cb, inv_m2, w[t], dw[t]);
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
                d0.add(dw[0][o0], pa.value());
                d1.add(w[0][o0], p1.value());
                d2.add(w[0][o0], p2.value());
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

template <typename R, int D>
KFn grad_m(int m) {
    switch (m) {
        case 2: return k_grad_x<R, D, 4>;
        case 3: return k_grad_x<R, D, 6>;
        case 4: return k_grad_x<R, D, 8>;
        case 5: return k_grad_x<R, D, 10>;
        case 6: return k_grad_x<R, D, 12>;
        case 7: return k_grad_x<R, D, 14>;
        case 8: return k_grad_x<R, D, 16>;
        default: return nullptr;
    }
}

template <typename R, int METHOD>
KFn spread_d(int d, int m) {
    if (d == 1) return spread_m<R, 1, METHOD>(m);
    if (d == 2) return spread_m<R, 2, METHOD>(m);
    if (d == 3) return spread_m<R, 3, METHOD>(m);
    return nullptr;
}

template <typename R>
KFn grad_d(int d, int m) {
    if (d == 1) return grad_m<R, 1>(m);
    if (d == 2) return grad_m<R, 2>(m);
    if (d == 3) return grad_m<R, 3>(m);
    return nullptr;
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
    return a;
}

}  // namespace

bl_status launch_spread(Plan& p, const void* g, void* grid) {
    const int64_t n = p.grid_elems();
    const unsigned zb = unsigned((n + 255) / 256);
    if (p.prec == BL_F64)
        hipLaunchKernelGGL(k_zero<double>, dim3(zb), dim3(256), 0, p.stream, static_cast<Cx<double>*>(grid), n);
    else
        hipLaunchKernelGGL(k_zero<float>, dim3(zb), dim3(256), 0, p.stream, static_cast<Cx<float>*>(grid), n);
    BL_HIP(hipGetLastError());
    if (p.N == 0 || p.nchunks == 0) return BL_OK;
    KFn fn;
    if (p.prec == BL_F64) fn = p.method == BL_NFFT ? spread_d<double, 1>(p.d, p.m) : spread_d<double, 0>(p.d, p.m);
    else fn = p.method == BL_NFFT ? spread_d<float, 1>(p.d, p.m) : spread_d<float, 0>(p.d, p.m);
    if (!fn) {
        set_error("no spreading kernel for this (d, m)");
        return BL_EUNSUPPORTED;
    }
    SpreadArgs a = make_args(p);
    a.g = g;
    a.grid = grid;
    const size_t lds = box_bytes(p) + 16 + sizeof(float) * kMaxM * kPolyCoef;
    if (lds > 64 * 1024)
        BL_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    hipLaunchKernelGGL(fn, dim3(unsigned(p.nchunks)), dim3(256), lds, p.stream, a);
    BL_HIP(hipGetLastError());
    return BL_OK;
}

bl_status launch_grad_x(Plan& p, const void* g, void* gx) {
    if (p.N == 0 || p.nchunks == 0) return BL_OK;
    KFn fn = (p.prec == BL_F64) ? grad_d<double>(p.d, p.m) : grad_d<float>(p.d, p.m);
    if (!fn) {
        set_error("no gradient kernel for this (d, m)");
        return BL_EUNSUPPORTED;
    }
    SpreadArgs a = make_args(p);
    a.g = g;
    a.grid = p.d_grid;
    a.gx = gx;
    const size_t lds = box_bytes(p);
    if (lds > 64 * 1024)
        BL_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    hipLaunchKernelGGL(fn, dim3(unsigned(p.nchunks)), dim3(256), lds, p.stream, a);
    BL_HIP(hipGetLastError());
    return BL_OK;
}

}  // namespace bl
