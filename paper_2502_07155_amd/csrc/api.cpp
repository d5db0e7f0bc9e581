// C ABI of the blnfft library: validation, plan lifecycle and call dispatch.
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

struct bl_plan_s {
    bl::Plan p;
};

namespace bl {

namespace {
thread_local std::string g_err;
}

void set_error(const std::string& msg) { g_err = msg; }
const std::string& last_error() { return g_err; }

namespace {

bl_status fail(bl_status s, const std::string& msg) {
    set_error(msg);
    return s;
}

int64_t ipow(int64_t b, int e) {
    int64_t r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

template <typename T>
bl_status dev_alloc(T** ptr, size_t bytes, size_t* total) {
    *ptr = nullptr;
    if (bytes == 0) return BL_OK;
    if (const char* f = std::getenv("BL_TEST_FAIL_ALLOC")) {
        if (f[0] == '1') return fail(BL_ENOMEM, "allocation refused by BL_TEST_FAIL_ALLOC");
    }
    hipError_t e = hipMalloc(reinterpret_cast<void**>(ptr), bytes);
    if (e != hipSuccess) {
        *ptr = nullptr;
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? BL_ENOMEM : BL_EDEVICE,
                    std::string("hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
    }
    *total += bytes;
    return BL_OK;
}

void free_nodes(Plan& p) {
    hipFree(p.d_xs);
    hipFree(p.d_perm);
    hipFree(p.d_node_tile);
    hipFree(p.d_chunks);
    p.d_xs = nullptr;
    p.d_perm = nullptr;
    p.d_node_tile = nullptr;
    p.d_chunks = nullptr;
    p.N_cap = 0;
    p.chunk_alloc = 0;
}

// Destroy one cached forward graph.  A replay launched before may still be running on the
// plan's stream, so the stream is synchronized before its executable graph is destroyed.
void drop_one_graph(Plan& p, Plan::FwdGraph& g) {
    if (!g.exec) return;
    (void)hipStreamSynchronize(p.stream);
    hipGraphExecDestroy(g.exec);
    g = Plan::FwdGraph{};
}

void drop_graph(Plan& p) {
    bool any = false;
    for (auto& g : p.graphs) any = any || g.exec != nullptr;
    if (!any) return;
    (void)hipStreamSynchronize(p.stream);
    for (auto& g : p.graphs) {
        if (g.exec) hipGraphExecDestroy(g.exec);
        g = Plan::FwdGraph{};
    }
}

void free_plan(Plan& p) {
    drop_graph(p);
    if (p.capture_stream) hipStreamDestroy(p.capture_stream);
    p.capture_stream = nullptr;
    free_nodes(p);
    hipFree(p.d_deconv);
    for (FftStages* st : {&p.st16, &p.st4}) {
        hipFree(st->d_tw64);
        hipFree(st->d_tw32);
        st->d_tw64 = st->d_tw32 = nullptr;
    }
    hipFree(p.d_bufA);
    hipFree(p.d_bufB);
    hipFree(p.d_grid);
    hipFree(p.d_sgrid);
    hipFree(p.d_boxes);
    p.d_boxes = nullptr;
    p.boxes_cap = 0;
    hipFree(p.d_tile_count);
    hipFree(p.d_tile_offset);
    hipFree(p.d_tile_cursor);
    hipFree(p.d_chunk_offset);
    hipFree(p.d_scan);
    p.d_scan = nullptr;
    hipFree(p.d_cov);
    p.d_cov = nullptr;
    hipFree(p.d_reach);
    p.d_reach = nullptr;
    hipFree(p.d_flags);
    hipFree(p.d_wpre);
    p.d_wpre = nullptr;
    p.use_wpre = false;
    for (void** t : {&p.czt.d_roots64, &p.czt.d_roots32, &p.czt.d_H64, &p.czt.d_H32, &p.czt.d_band64,
                     &p.czt.d_band32, &p.czt.d_grid64, &p.czt.d_grid32, &p.czt.d_scr}) {
        hipFree(*t);
        *t = nullptr;
    }
}

// LDS budget of one staged tile plus halo (stored twice for float tiles with d >= 2).  The
// d = 3 budget keeps at least three workgroups per CU (measured: occupancy outweighs the
// larger halo overhead there).
bool tile_fits(const Plan& p, int T) {
    size_t e = 1;
    for (int k = 0; k < p.d; ++k) e *= size_t(T + 2 * p.m - 1);
    const size_t c = p.cplx_size() * (p.dual_tiles ? 2 : 1);
    return e * c <= size_t(p.d == 3 ? 44 : 64) * 1024;
}

// Default tile edge of the short-sum kernels, shrunk until the tile fits its LDS budget.
int default_tile(const Plan& p) {
    int T = p.d == 1 ? 512 : p.d == 2 ? 16 : 8;
    if (const char* e = std::getenv("BL_TILE")) {   // tuning override
        const int v = std::atoi(e);
        if (v >= 1 && v <= 4096) T = v;
    }
    while (T > 1 && !tile_fits(p, T)) --T;
    return int(std::min<int64_t>(T, p.L));
}

// Candidates of the autotuner: (tile edge, chunk capacity) pairs whose tile fits its LDS
// budget and whose box (tile + 2m - 1) keeps the adjoint's deterministic spreading kernels:
// the output-stationary one for d = 1 (<= 1024 points), the row kernels for d = 2 and 3
// (edges <= 32 and <= 16).
std::vector<std::pair<int, int>> tile_candidates(const Plan& p) {
    std::vector<int> Ts;
    if (p.d == 1) Ts = {256, 512, 1024, 2048};
    else if (p.d == 2) Ts = {12, 14, 16, 20, 24};
    else Ts = {5, 6, 7, 8};
    std::vector<int> caps = p.d == 1 ? std::vector<int>{1024} : std::vector<int>{512, 1024};
    std::vector<std::pair<int, int>> out;
    for (int T : Ts) {
        if (T > p.L || !tile_fits(p, T)) continue;
        if (p.d == 1 && T + 2 * p.m - 1 > 1024) continue;   // output-stationary spreading
        if (p.d == 2 && T + 2 * p.m - 1 > 32) continue;
        if (p.d == 3 && p.m <= 7 && T + 2 * p.m - 1 > 16) continue;
        for (int c : caps) out.push_back({T, c});
    }
    return out;
}

int64_t tiles_for(const Plan& p, int T) {
    int64_t n = 1;
    for (int t = 0; t < p.d; ++t) n *= (p.L + T - 1) / T;
    return n;
}

// Coverage table of the adjoint's box merge for tile edge T: per coordinate p of a
// dimension, its tile and every (tile, position) whose box (tile + halo, tile t spanning
// grid points t T - m + 1 ... t T + T + m - 2) covers p, periodically for Algorithm 2.1.
// Empty when some coordinate has more than kCovMax covering boxes.
std::vector<int> coverage_table(const Plan& p, int T) {
    const int L = int(p.L), m = p.m, W = T + 2 * p.m - 1, tpd = (L + T - 1) / T;
    std::vector<int> tab(size_t(L) * kCovRow, 0);
    const int s_lo = p.method == BL_NFFT ? -1 : 0, s_hi = p.method == BL_NFFT ? 2 : 0;
    for (int q = 0; q < L; ++q) {
        int* row = &tab[size_t(q) * kCovRow];
        row[0] = q / T;
        int n = 0;
        for (int s = s_lo; s <= s_hi; ++s) {
            const int u = q + s * L;   // unwrapped coordinate: box position c = u - (t T - m + 1)
            // c in [0, W) <=> t T in [u + m - W, u + m - 1]
            const int tlo = std::max(0, (u + m - W + T - 1 + 2 * L * T) / T - 2 * L);   // ceil, any sign
            const int thi = std::min(tpd - 1, u + m - 1 < 0 ? -1 : (u + m - 1) / T);
            for (int t = tlo; t <= thi; ++t) {
                const int c = u - (t * T - m + 1);
                if (c < 0 || c >= W) continue;
                if (n == kCovMax) return std::vector<int>();
                // offset of the covering tile from the coordinate's own tile, wrapped for the
                // periodic sums into [-kNbR, kNbR] (the merge stages that neighbourhood)
                int dt = t - q / T;
                if (p.method == BL_NFFT) {
                    if (dt > kNbR) dt -= tpd;
                    if (dt < -kNbR) dt += tpd;
                    if (((q / T + dt) % tpd + tpd) % tpd != t) return std::vector<int>();
                }
                if (dt < -kNbR || dt > kNbR) return std::vector<int>();
                row[2 + 2 * n] = dt;
                row[3 + 2 * n] = c;
                ++n;
            }
        }
        row[1] = n;
    }
    // d = 3: the merge's reach flags mark, per box, the distinct tiles of its W coordinates:
    // at most eight per dimension (kReachList in spread.hip), else the general merge is used
    for (int t = 0; t < tpd && p.d == 3; ++t) {
        int distinct = 0, last = -1;
        std::vector<int> seen;
        for (int c = t * T - m + 1; c <= t * T + T + m - 2; ++c) {
            int q = c;
            if (p.method == BL_NFFT) q = ((q % L) + L) % L;
            else if (q < 0 || q >= L) continue;
            const int tt = q / T;
            if (tt == last || std::find(seen.begin(), seen.end(), tt) != seen.end()) continue;
            last = tt;
            seen.push_back(tt);
            if (++distinct > 8) return std::vector<int>();
        }
    }
    return tab;
}

// Sets the tile edge and the chunk capacity, growing the per-tile arrays when needed.
bl_status apply_tiles(Plan& p, int T, int cap) {
    p.ntiles = 1;
    for (int t = 0; t < 3; ++t) {
        p.tile[t] = t < p.d ? T : 1;
        p.tiles_per_dim[t] = t < p.d ? int((p.L + T - 1) / T) : 1;
        p.ntiles *= p.tiles_per_dim[t];
    }
    p.chunk_cap = cap;
    // the adjoint merge's coverage table for this tile edge (empty: the general merge)
    BL_HIP(hipStreamSynchronize(p.stream));
    hipFree(p.d_cov);
    p.d_cov = nullptr;
    const std::vector<int> cov = coverage_table(p, T);
    if (!cov.empty()) {
        size_t extra = 0;
        BL_TRY(dev_alloc(&p.d_cov, sizeof(int) * cov.size(), &extra));
        BL_HIP(hipMemcpy(p.d_cov, cov.data(), sizeof(int) * cov.size(), hipMemcpyHostToDevice));
    }
    if (p.ntiles <= p.tile_alloc) return BL_OK;
    BL_HIP(hipStreamSynchronize(p.stream));
    for (int32_t** a : {&p.d_tile_count, &p.d_tile_offset, &p.d_tile_cursor, &p.d_chunk_offset}) {
        hipFree(*a);
        *a = nullptr;
    }
    hipFree(p.d_scan);
    p.d_scan = nullptr;
    hipFree(p.d_reach);
    p.d_reach = nullptr;
    p.workspace_bytes -= size_t(p.tile_alloc) * 4 * sizeof(int32_t) + (p.tile_alloc ? tile_scan_scratch_bytes(p.tile_alloc) : 0);
    p.tile_alloc = 0;
    size_t extra = 0;
    for (int32_t** a : {&p.d_tile_count, &p.d_tile_offset, &p.d_tile_cursor, &p.d_chunk_offset})
        BL_TRY(dev_alloc(a, sizeof(int32_t) * size_t(p.ntiles), &extra));
    BL_TRY(dev_alloc(reinterpret_cast<char**>(&p.d_scan), tile_scan_scratch_bytes(p.ntiles), &extra));
    if (p.d == 3) BL_TRY(dev_alloc(&p.d_reach, size_t(p.ntiles), &extra));
    p.tile_alloc = p.ntiles;
    p.workspace_bytes += extra;
    return BL_OK;
}

// Average time (ms) of the short-sum kernel on the bound nodes (zero samples).
double time_gather(Plan& p, void* f, hipEvent_t e0, hipEvent_t e1) {
    if (launch_gather(p, p.d_grid, f) != BL_OK) return -1.0;
    if (hipEventRecord(e0, p.stream) != hipSuccess) return -1.0;
    constexpr int reps = 10;
    for (int r = 0; r < reps; ++r)
        if (launch_gather(p, p.d_grid, f) != BL_OK) return -1.0;
    float ms = 0.0f;
    if (hipEventRecord(e1, p.stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        return -1.0;
    return double(ms) / reps;
}

// Node binning with the autotuned tile edge and chunk capacity: the nodes are binned with
// the default tiles first, which classifies them (nodes per grid point, fullest tile
// against the mean); a cached choice for that class is applied, or every candidate's short
// sums are timed and the choice cached: among the candidates within kTileTie of the
// fastest (the spread of repeated timings), the one with the fewest work chunks, since the
// adjoint writes and merges one box per chunk.  A later binning of as many nodes keeps
// the plan's choice.
constexpr double kTileTie = 0.015;
constexpr int kDefaultChunk = 1024;   // nodes per work chunk without tuning
constexpr int kSmallChunk = 256;     // the same below kTuneMinNodes nodes

bl_status bin_tuned(Plan& p, const void* x, int64_t N) {
    if (!tile_tuning_wanted(p, N) || (p.tuned_N == N && p.tune_tile_source != 0))
        return launch_binning(p, x, N);
    p.N = N;   // the short-sum kernel timed below runs over p.N nodes
    BL_TRY(apply_tiles(p, default_tile(p), kDefaultChunk));
    BL_TRY(launch_binning(p, x, N));
    std::vector<int32_t> cnt(size_t(p.ntiles));
    BL_HIP(hipMemcpy(cnt.data(), p.d_tile_count, sizeof(int32_t) * cnt.size(), hipMemcpyDeviceToHost));
    const double mean = double(N) / double(p.ntiles);
    const double fullest = double(*std::max_element(cnt.begin(), cnt.end()));
    const int density = int(std::lround(2.0 * std::log2(double(N) / double(p.grid_elems()))));
    const int cluster = int(std::lround(std::log2(std::max(1.0, fullest / mean))));
    int T = p.tile[0], cap = p.chunk_cap;
    const int T0 = T, cap0 = cap;
    if (tile_cache_lookup(p, density, cluster, &T, &cap)) {
        p.tune_tile_source = 2;
    } else {
        const auto cands = tile_candidates(p);
        if (cands.empty()) return BL_OK;
        void* f = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        BL_TRY(dev_alloc(reinterpret_cast<char**>(&f), size_t(N) * p.cplx_size(), &p.workspace_bytes));
        p.workspace_bytes -= size_t(N) * p.cplx_size();
        bl_status st = BL_OK;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
            hipMemsetAsync(p.d_grid, 0, size_t(p.grid_elems()) * p.cplx_size(), p.stream) != hipSuccess) {
            st = fail(BL_EDEVICE, "autotuner: event or memset failed");
        }
        double best_ms = -1.0;
        std::vector<double> ms_of(cands.size(), -1.0);
        std::vector<int64_t> chunks_of(cands.size(), 0);
        for (size_t i = 0; st == BL_OK && i < cands.size(); ++i) {
            st = apply_tiles(p, cands[i].first, cands[i].second);
            if (st == BL_OK) st = launch_binning(p, x, N);
            if (st != BL_OK) break;
            const double ms = time_gather(p, f, e0, e1);
            ms_of[i] = ms;
            chunks_of[i] = p.nchunks;
            if (std::getenv("BL_TUNE_VERBOSE"))
                std::fprintf(stderr, "blnfft tune tiles: d=%d L=%lld m=%d tile=%d cap=%d chunks=%lld: %.2f us\n", p.d,
                             (long long)p.L, p.m, cands[i].first, cands[i].second, (long long)p.nchunks, ms * 1e3);
            if (ms > 0.0 && (best_ms < 0.0 || ms < best_ms)) best_ms = ms;
        }
        size_t pick = cands.size();
        for (size_t i = 0; best_ms > 0.0 && i < cands.size(); ++i) {
            if (!(ms_of[i] > 0.0 && ms_of[i] <= best_ms * (1.0 + kTileTie))) continue;
            if (pick == cands.size() || chunks_of[i] < chunks_of[pick] ||
                (chunks_of[i] == chunks_of[pick] && ms_of[i] < ms_of[pick]))
                pick = i;
        }
        if (pick < cands.size()) {
            T = cands[pick].first;
            cap = cands[pick].second;
        }
        (void)hipStreamSynchronize(p.stream);
        if (e0) hipEventDestroy(e0);
        if (e1) hipEventDestroy(e1);
        hipFree(f);
        BL_TRY(st);
        if (best_ms < 0.0) {
            T = T0;
            cap = cap0;
        } else {
            tile_cache_store(p, density, cluster, T, cap);
            p.tune_tile_source = 1;
        }
    }
    p.tuned_N = N;
    if (T == p.tile[0] && cap == p.chunk_cap) return BL_OK;
    BL_TRY(apply_tiles(p, T, cap));
    return launch_binning(p, x, N);
}

// Steps 1-3 as kernel launches on p.stream.
bl_status forward_launches(Plan& p, const void* fhat, void* f) {
    BL_TRY(launch_forward_fft(p, fhat));
    return launch_gather(p, p.d_grid, f);
}

// Capture the forward launches into a graph on the private capture stream, into a free
// cache slot or the least recently used one.
bl_status capture_forward(Plan& p, const void* fhat, void* f, Plan::FwdGraph** out) {
    Plan::FwdGraph* slot = &p.graphs[0];
    for (auto& g : p.graphs) {
        if (!g.exec) {
            slot = &g;
            break;
        }
        if (g.used < slot->used) slot = &g;
    }
    drop_one_graph(p, *slot);
    if (!p.capture_stream) BL_HIP(hipStreamCreateWithFlags(&p.capture_stream, hipStreamNonBlocking));
    hipStream_t user = p.stream;
    p.stream = p.capture_stream;
    hipError_t e = hipStreamBeginCapture(p.capture_stream, hipStreamCaptureModeThreadLocal);
    bl_status st = BL_OK;
    if (e == hipSuccess) st = forward_launches(p, fhat, f);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(p.capture_stream, &g);
    p.stream = user;
    if (e != hipSuccess || e2 != hipSuccess || st != BL_OK) {
        if (g) hipGraphDestroy(g);
        (void)hipGetLastError();
        if (st != BL_OK) return st;
        return fail(BL_EDEVICE, std::string("graph capture failed: ") +
                                    hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) return fail(BL_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    slot->exec = ge;
    slot->fhat = fhat;
    slot->f = f;
    *out = slot;
    return BL_OK;
}

bl_status check_plan(bl_plan plan) {
    if (!plan) return fail(BL_EINVAL, "plan is NULL");
    BL_HIP(hipSetDevice(plan->p.device));
    return BL_OK;
}

}  // namespace
}  // namespace bl

using namespace bl;

extern "C" {

const char* bl_status_string(bl_status s) {
    switch (s) {
        case BL_OK: return "BL_OK";
        case BL_EINVAL: return "BL_EINVAL: invalid argument";
        case BL_EDOMAIN: return "BL_EDOMAIN: node outside [-1/2, 1/2)^d or not finite";
        case BL_ENOMEM: return "BL_ENOMEM: out of memory";
        case BL_EDEVICE: return "BL_EDEVICE: HIP runtime error";
        case BL_ESTATE: return "BL_ESTATE: call out of order";
        case BL_EUNSUPPORTED: return "BL_EUNSUPPORTED: not supported by this build";
    }
    return "unknown bl_status";
}

const char* bl_last_error(void) { return last_error().c_str(); }

const char* bl_version(void) { return "blnfft 0.1 (gfx950)"; }

bl_status bl_window_transform(bl_window win, bl_method method, int64_t M, int64_t L, int m,
                              double beta, int64_t n, const double* v, double* out) {
    if (win != BL_WIN_SINH && win != BL_WIN_CKB) return fail(BL_EINVAL, "unknown window");
    if (method != BL_SHANNON && method != BL_NFFT) return fail(BL_EINVAL, "unknown method");
    if (L < 2 || m < 1 || 2 * int64_t(m) >= L || M < 2 || M > L)
        return fail(BL_EINVAL, "need 2 <= M <= L and 1 <= m, 2m < L");
    if (n < 0 || (n > 0 && (!v || !out))) return fail(BL_EINVAL, "bad array arguments");
    if (!(beta > 0.0)) beta = default_beta(M, L, m, method);
    if (!std::isfinite(beta)) return fail(BL_EINVAL, "beta not finite");
    for (int64_t i = 0; i < n; ++i) out[i] = window_transform(win, method, L, m, beta, v[i]);
    return BL_OK;
}

bl_status bl_plan_create(bl_plan* out, int d, int64_t M, int64_t L, int m, bl_window win,
                         double beta, bl_method method, bl_precision prec, void* stream) {
    if (!out) return fail(BL_EINVAL, "out is NULL");
    *out = nullptr;
    if (d < 1 || d > 3) return fail(BL_EINVAL, "d must be 1, 2 or 3");
    if (M < 2 || (M % 2) != 0) return fail(BL_EINVAL, "M must be even and >= 2");
    if (L < M || (L % 2) != 0) return fail(BL_EINVAL, "L must be even and >= M");
    if (m < 1 || 2 * int64_t(m) >= L) return fail(BL_EINVAL, "need 1 <= m and 2m < L");
    if (win != BL_WIN_SINH && win != BL_WIN_CKB) return fail(BL_EINVAL, "unknown window");
    if (method != BL_SHANNON && method != BL_NFFT) return fail(BL_EINVAL, "unknown method");
    if (prec != BL_F64 && prec != BL_F32 && prec != BL_F32C && prec != BL_F32D)
        return fail(BL_EINVAL, "unknown precision");
    if (std::isnan(beta) || std::isinf(beta)) return fail(BL_EINVAL, "beta not finite");
    if (m < kMinM || m > kMaxM)
        return fail(BL_EUNSUPPORTED, "compiled short-sum kernels cover 2 <= m <= 8");
    // Steps 1-2 and the adjoint: power-of-two L in [16, 8192] run the Stockham passes; any
    // other even L the chirp-z passes with a cyclic convolution of power-of-two size
    // P >= L + M - 1, held in LDS when P fits (8192 points in double arithmetic, 16384 in
    // float), else, for d = 1 only, split into up to eight LDS pieces.  A d >= 2 plan whose
    // P exceeds the LDS size still runs the short sums (bl_interpolate) alone.
    const int64_t Lmax = d == 1 ? 32768 : 8192;
    if (L > Lmax) return fail(BL_EUNSUPPORTED, "L above " + std::to_string(Lmax) + " for d = " + std::to_string(d));
    FftFactors fac16, fac4;
    const bool stockham_ok = L <= 8192 && factor_length(int(L), 16, &fac16) && factor_length(int(L), 4, &fac4);
    const bool f64 = prec == BL_F64 || prec == BL_F32D;
    const int64_t lds_points = f64 ? kCztLdsPoints<double>() : kCztLdsPoints<float>();
    int64_t czP = 4;
    while (czP < L + M - 1) czP *= 2;
    const bool czt_split = czP > lds_points;
    const bool fft_ok = stockham_ok || !czt_split || (d == 1 && czP <= 8 * lds_points);
    const int64_t grid = ipow(L, d);
    if (grid > (int64_t(1) << 31)) return fail(BL_EUNSUPPORTED, "grid L^d too large");

    bl_plan_s* h = new (std::nothrow) bl_plan_s();
    if (!h) return fail(BL_ENOMEM, "host allocation failed");
    Plan& p = h->p;
    p.d = d;
    p.M = M;
    p.L = L;
    p.m = m;
    p.win = win;
    p.method = method;
    p.fft_ok = fft_ok;
    p.prec = prec;
    p.beta = (beta > 0.0) ? beta : default_beta(M, L, m, method);
    p.stream = static_cast<hipStream_t>(stream);
    if (const char* e = std::getenv("BL_GRAPH")) p.use_graph = e[0] != '0';
    auto cleanup = [&](bl_status s) {
        free_plan(p);
        delete h;
        return s;
    };
    if (hipGetDevice(&p.device) != hipSuccess) return cleanup(fail(BL_EDEVICE, "hipGetDevice failed"));

    // Step 0a: per-dimension factors 1/(L hat1(k)), k = i - M/2, in FP64 (4.9) / (2.2).
    std::vector<double> fac_h(M);
    for (int64_t i = 0; i < M; ++i) {
        double hv = window_transform(win, method, L, m, p.beta, double(i - M / 2));
        if (!(std::fabs(hv) > 0.0) || !std::isfinite(hv))
            return cleanup(fail(BL_EINVAL, "window transform vanishes on I_M for this beta"));
        fac_h[i] = 1.0 / (double(L) * hv);
    }
    std::vector<double> tw0;
    if (stockham_ok) twiddles(L, &tw0);
    std::vector<double> tw[2];
    std::vector<float> tw32[2];
    const FftFactors* facs[2] = {&fac16, &fac4};
    FftStages* sts[2] = {&p.st16, &p.st4};
    for (int v = 0; v < 2; ++v) {
        if (stockham_ok) stage_twiddles(*facs[v], tw0, &tw[v], sts[v]->tw_off);
        if (tw[v].empty()) tw[v].assign(2, 0.0);
        sts[v]->tw_len = int(tw[v].size() / 2);
        sts[v]->nmain = 0;
        sts[v]->rlast = 1;
        const int E = v == 0 ? 16 : 4;
        for (int s = 0; stockham_ok && s < facs[v]->nstages; ++s) {
            if (facs[v]->radix[s] == E) ++sts[v]->nmain;
            else sts[v]->rlast = facs[v]->radix[s];
        }
        tw32[v].resize(tw[v].size());
        for (size_t i = 0; i < tw[v].size(); ++i) tw32[v][i] = float(tw[v][i]);
    }
    p.edge_k = edge_exponent(win);
    if (prec != BL_F64) {
        std::vector<double> pc;
        p.poly_err = fit_weight_polys(win, method, m, p.beta, kPolyCoef, &pc);
        if (!(p.poly_err <= kPolyFitTol))
            return cleanup(fail(BL_EUNSUPPORTED, "float weight polynomials fit this window only to " +
                                                     std::to_string(p.poly_err) +
                                                     " (above 1e-7; beta too large for float plans)"));
        p.poly.assign(pc.begin(), pc.end());
    } else {
        p.poly64_err = fit_weight_polys(win, method, m, p.beta, kPolyCoef64, &p.poly64);
        if (win == BL_WIN_SINH) {
            p.use_poly64 = p.poly64_err <= 1e-13 && std::getenv("BL_EXACT_WEIGHTS") == nullptr;
        } else {
            // the exact device weight formula is the sinh-type window's
            if (p.poly64_err > 1e-13)
                return cleanup(fail(BL_EUNSUPPORTED, "FP64 weights of this window need a polynomial fit within 1e-13"));
            p.use_poly64 = true;
            // bl_grad_x differentiates the same polynomials
            p.poly64_deriv_err = weight_deriv_fit_error(win, method, m, p.beta, kPolyCoef64, p.poly64);
        }
    }

    size_t total = 0;
    bl_status s;
    const size_t c = p.cplx_size();
    // FFT intermediates: forward passes produce M^{d-1} L and M^{d-2} L^2 elements; the
    // adjoint passes L^{d-1} M and L^{d-2} M^2.
    int64_t A = 0, B = 0;
    if (d >= 2) A = std::max(ipow(M, d - 1) * L, ipow(L, d - 1) * M);
    if (d >= 3) B = std::max(ipow(M, d - 2) * L * L, ipow(L, d - 2) * M * M);
    if ((s = dev_alloc(&p.d_deconv, sizeof(double) * M, &total)) != BL_OK) return cleanup(s);
    for (int v = 0; v < 2; ++v) {
        if ((s = dev_alloc(&sts[v]->d_tw64, sizeof(double) * tw[v].size(), &total)) != BL_OK) return cleanup(s);
        if ((s = dev_alloc(&sts[v]->d_tw32, sizeof(float) * tw[v].size(), &total)) != BL_OK) return cleanup(s);
    }
    if ((s = dev_alloc(&p.d_grid, size_t(grid) * c, &total)) != BL_OK) return cleanup(s);
    // F32D keeps the FFT pass intermediates in double.
    const size_t ci = p.fft64() ? 16 : c;
    if ((s = dev_alloc(&p.d_bufA, size_t(A) * ci, &total)) != BL_OK) return cleanup(s);
    if ((s = dev_alloc(&p.d_bufB, size_t(B) * ci, &total)) != BL_OK) return cleanup(s);
    if (!stockham_ok && fft_ok) {
        // chirp-z tables, FP64 (with float copies): u^{k^2} times the factor on I_M,
        // u^{l^2} on I_L, H = DFT_P(h) / P and the P-th roots, u = e^{i pi / L}
        CztTables& z = p.czt;
        z.on = true;
        z.P = czP;
        z.split = czt_split;
        z.R = czt_split ? int(czP / lds_points) : 1;
        std::vector<double> tw2L, rootsP;
        twiddles(2 * L, &tw2L);
        twiddles(czP, &rootsP);
        std::vector<double> band(2 * M), gridc(2 * L), Hd(2 * czP);
        for (int64_t i = 0; i < M; ++i) {
            const int64_t k = i - M / 2;
            const std::complex<double> v = chirp(k * k, L, tw2L) * fac_h[i];
            band[2 * i] = v.real();
            band[2 * i + 1] = v.imag();
        }
        for (int64_t i = 0; i < L; ++i) {
            const int64_t l = i - L / 2;
            const std::complex<double> v = chirp(l * l, L, tw2L);
            gridc[2 * i] = v.real();
            gridc[2 * i + 1] = v.imag();
        }
        const std::vector<std::complex<double>> H = chirp_spectrum(L, M, czP);
        for (int64_t q = 0; q < czP; ++q) {
            Hd[2 * q] = H[q].real();
            Hd[2 * q + 1] = H[q].imag();
        }
        struct Tab {
            const std::vector<double>* v;
            void** d64;
            void** d32;
        } tabs[4] = {{&band, &z.d_band64, &z.d_band32}, {&gridc, &z.d_grid64, &z.d_grid32},
                     {&Hd, &z.d_H64, &z.d_H32}, {&rootsP, &z.d_roots64, &z.d_roots32}};
        for (const Tab& tb : tabs) {
            const size_t n = tb.v->size();
            if ((s = dev_alloc(reinterpret_cast<char**>(tb.d64), sizeof(double) * n, &total)) != BL_OK) return cleanup(s);
            if ((s = dev_alloc(reinterpret_cast<char**>(tb.d32), sizeof(float) * n, &total)) != BL_OK) return cleanup(s);
            std::vector<float> f32(tb.v->begin(), tb.v->end());
            if (hipMemcpy(*tb.d64, tb.v->data(), sizeof(double) * n, hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(*tb.d32, f32.data(), sizeof(float) * n, hipMemcpyHostToDevice) != hipSuccess)
                return cleanup(fail(BL_EDEVICE, "chirp-z table upload failed"));
        }
        if (czt_split && (s = dev_alloc(reinterpret_cast<char**>(&z.d_scr), size_t(czP) * ci, &total)) != BL_OK)
            return cleanup(s);
    }
    p.dual_tiles = dual_tiles_for(d, p.m, p.prec != BL_F64);
    if ((s = apply_tiles(p, default_tile(p), kDefaultChunk)) != BL_OK) return cleanup(s);
    if ((s = dev_alloc(&p.d_flags, sizeof(unsigned long long) * 4, &total)) != BL_OK) return cleanup(s);
    p.workspace_bytes += total;

    hipError_t e = hipMemcpyAsync(p.d_deconv, fac_h.data(), sizeof(double) * M, hipMemcpyHostToDevice, p.stream);
    for (int v = 0; v < 2 && e == hipSuccess; ++v) {
        e = hipMemcpyAsync(sts[v]->d_tw64, tw[v].data(), sizeof(double) * tw[v].size(), hipMemcpyHostToDevice, p.stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(sts[v]->d_tw32, tw32[v].data(), sizeof(float) * tw32[v].size(), hipMemcpyHostToDevice, p.stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(p.stream);
    if (e != hipSuccess) return cleanup(fail(BL_EDEVICE, std::string("table upload: ") + hipGetErrorString(e)));
    if ((s = autotune_fft(p)) != BL_OK) return cleanup(s);
    *out = h;
    return BL_OK;
}

bl_status bl_plan_destroy(bl_plan plan) {
    if (!plan) return BL_OK;
    hipSetDevice(plan->p.device);
    hipStreamSynchronize(plan->p.stream);
    free_plan(plan->p);
    delete plan;
    return BL_OK;
}

bl_status bl_set_nodes(bl_plan plan, int64_t N, const void* x_dev) {
    BL_TRY(check_plan(plan));
    Plan& p = plan->p;
    if (N < 0 || N > int64_t(0x7fffffff)) return fail(BL_EINVAL, "N out of range");
    if (N > 0 && !x_dev) return fail(BL_EINVAL, "x_dev is NULL");
    p.have_nodes = false;
    p.have_theta = false;
    p.N = 0;
    drop_graph(p);
    if (p.d_wpre) {   // precomputed weights belong to the previous nodes
        BL_HIP(hipStreamSynchronize(p.stream));
        hipFree(p.d_wpre);
        p.d_wpre = nullptr;
    }
    p.use_wpre = false;
    // Bindings the tile tuning does not time take chunks of at most kSmallChunk nodes below
    // kTuneMinNodes nodes (one node per thread of a short-sum workgroup, so that a few
    // thousand nodes occupy several workgroups instead of one looping over them), else
    // kDefaultChunk.
    if (!tile_tuning_wanted(p, N)) {
        const int want = N < kTuneMinNodes ? kSmallChunk : kDefaultChunk;
        if (want != p.chunk_cap) BL_TRY(apply_tiles(p, p.tile[0], want));
    }
    // work chunks: at most N / cap + ntiles + 1 for the current tiles and every candidate
    // of the autotuner
    int64_t chunk_bound = N / p.chunk_cap + p.ntiles + 1;
    if (tile_tuning_wanted(p, N)) {
        chunk_bound = std::max<int64_t>(chunk_bound, N / 1024 + tiles_for(p, default_tile(p)) + 1);
        for (const auto& c : tile_candidates(p))
            chunk_bound = std::max<int64_t>(chunk_bound, N / c.second + tiles_for(p, c.first) + 1);
    }
    if (N > p.N_cap || chunk_bound > p.chunk_alloc) {
        BL_HIP(hipStreamSynchronize(p.stream));
        free_nodes(p);
        size_t extra = 0;
        const int64_t ncap = std::max<int64_t>(N, 1);
        bl_status s;
        if ((s = dev_alloc(&p.d_xs, size_t(ncap) * p.d * p.real_size(), &extra)) != BL_OK) return s;
        if ((s = dev_alloc(&p.d_perm, sizeof(int32_t) * ncap, &extra)) != BL_OK) return s;
        if ((s = dev_alloc(&p.d_node_tile, sizeof(int32_t) * ncap, &extra)) != BL_OK) return s;
        const int64_t cb = std::max<int64_t>(chunk_bound, ncap / p.chunk_cap + p.ntiles + 1);
        if ((s = dev_alloc(&p.d_chunks, sizeof(int4) * cb, &extra)) != BL_OK) return s;
        p.N_cap = ncap;
        p.chunk_alloc = cb;
    }
    const bl_status st = bin_tuned(p, x_dev, N);
    if (st != BL_OK) {
        p.N = 0;
        return st;
    }
    p.N = N;
    p.have_nodes = true;
    return BL_OK;
}

bl_status bl_forward(bl_plan plan, const void* fhat_dev, void* f_dev) {
    BL_TRY(check_plan(plan));
    Plan& p = plan->p;
    if (!p.fft_ok) return fail(BL_EUNSUPPORTED, "bl_forward: L + M - 1 above the chirp-z LDS size for d >= 2 (bl_interpolate takes any even L)");
    if (!p.have_nodes) return fail(BL_ESTATE, "bl_set_nodes must succeed before bl_forward");
    if (!fhat_dev || (p.N > 0 && !f_dev)) return fail(BL_EINVAL, "NULL buffer");
    if (p.use_graph) {
        Plan::FwdGraph* g = nullptr;
        for (auto& c : p.graphs)
            if (c.exec && c.fhat == fhat_dev && c.f == f_dev) g = &c;
        if (!g) BL_TRY(capture_forward(p, fhat_dev, f_dev, &g));
        g->used = ++p.graph_tick;
        BL_HIP(hipGraphLaunch(g->exec, p.stream));
    } else {
        BL_TRY(forward_launches(p, fhat_dev, f_dev));
    }
    p.have_theta = true;
    return BL_OK;
}

bl_status bl_samples(bl_plan plan, const void* fhat_dev) {
    BL_TRY(check_plan(plan));
    Plan& p = plan->p;
    if (!p.fft_ok) return fail(BL_EUNSUPPORTED, "bl_samples: L + M - 1 above the chirp-z LDS size for d >= 2");
    if (!fhat_dev) return fail(BL_EINVAL, "NULL buffer");
    BL_TRY(launch_forward_fft(p, fhat_dev));
    p.have_theta = true;
    return BL_OK;
}

bl_status bl_precompute_weights(bl_plan plan, int enable) {
    BL_TRY(check_plan(plan));
    Plan& p = plan->p;
    drop_graph(p);   // the short-sum kernel changes
    if (!enable) {
        BL_HIP(hipStreamSynchronize(p.stream));
        hipFree(p.d_wpre);
        p.d_wpre = nullptr;
        p.use_wpre = false;
        return BL_OK;
    }
    if (p.method != BL_SHANNON) return fail(BL_EUNSUPPORTED, "precomputed weights are implemented for BL_SHANNON");
    if (!p.have_nodes) return fail(BL_ESTATE, "bl_set_nodes must succeed before bl_precompute_weights");
    if (p.use_wpre) return BL_OK;
    const size_t bytes = size_t(std::max<int64_t>(p.N, 1)) * size_t(p.d) * size_t(2 * p.m) * p.real_size();
    size_t extra = 0;
    BL_TRY(dev_alloc(&p.d_wpre, bytes, &extra));
    const bl_status s = launch_weights(p);
    if (s != BL_OK) {
        hipFree(p.d_wpre);
        p.d_wpre = nullptr;
        return s;
    }
    BL_HIP(hipStreamSynchronize(p.stream));
    p.use_wpre = true;
    return BL_OK;
}

bl_status bl_interpolate(bl_plan plan, const void* theta_dev, void* f_dev) {
    BL_TRY(check_plan(plan));
    Plan& p = plan->p;
    if (!p.have_nodes) return fail(BL_ESTATE, "bl_set_nodes must succeed before bl_interpolate");
    if (!theta_dev || (p.N > 0 && !f_dev)) return fail(BL_EINVAL, "NULL buffer");
    return launch_gather(p, theta_dev, f_dev);
}

bl_status bl_get_theta(bl_plan plan, void* theta_dev) {
    BL_TRY(check_plan(plan));
    Plan& p = plan->p;
    if (!p.have_theta) return fail(BL_ESTATE, "no forward transform has run");
    if (!theta_dev) return fail(BL_EINVAL, "NULL buffer");
    BL_HIP(hipMemcpyAsync(theta_dev, p.d_grid, size_t(p.grid_elems()) * p.cplx_size(),
                          hipMemcpyDeviceToDevice, p.stream));
    return BL_OK;
}

bl_status bl_adjoint(bl_plan plan, const void* g_dev, void* fhat_dev) {
    BL_TRY(check_plan(plan));
    Plan& p = plan->p;
    if (!p.fft_ok) return fail(BL_EUNSUPPORTED, "bl_adjoint: L + M - 1 above the chirp-z LDS size for d >= 2");
    if (!p.have_nodes) return fail(BL_ESTATE, "bl_set_nodes must succeed before bl_adjoint");
    if (!fhat_dev || (p.N > 0 && !g_dev)) return fail(BL_EINVAL, "NULL buffer");
    if (!p.d_sgrid) {
        size_t extra = 0;
        BL_HIP(hipStreamSynchronize(p.stream));
        BL_TRY(dev_alloc(&p.d_sgrid, size_t(p.grid_elems()) * p.cplx_size(), &extra));
        p.workspace_bytes += extra;
    }
    const size_t nb = spread_boxes_bytes(p);
    if (nb > p.boxes_cap) {
        BL_HIP(hipStreamSynchronize(p.stream));
        hipFree(p.d_boxes);
        p.d_boxes = nullptr;
        p.workspace_bytes -= p.boxes_cap;
        p.boxes_cap = 0;
        size_t extra = 0;
        BL_TRY(dev_alloc(&p.d_boxes, nb, &extra));
        p.boxes_cap = nb;
        p.workspace_bytes += extra;
    }
    BL_TRY(launch_spread(p, g_dev, p.d_sgrid, p.d_boxes));
    return launch_adjoint_fft(p, p.d_sgrid, fhat_dev);
}

bl_status bl_adjoint_noalloc(bl_plan plan, const void* g_dev, void* fhat_dev) {
    BL_TRY(check_plan(plan));
    Plan& p = plan->p;
    if (!p.fft_ok) return fail(BL_EUNSUPPORTED, "bl_adjoint_noalloc: L + M - 1 above the chirp-z LDS size for d >= 2");
    if (!p.have_nodes) return fail(BL_ESTATE, "bl_set_nodes must succeed before bl_adjoint_noalloc");
    if (!fhat_dev || (p.N > 0 && !g_dev)) return fail(BL_EINVAL, "NULL buffer");
    return launch_adjoint_noalloc(p, g_dev, fhat_dev);
}

bl_status bl_grad_x(bl_plan plan, const void* g_dev, void* gx_dev) {
    BL_TRY(check_plan(plan));
    Plan& p = plan->p;
    if (p.method != BL_SHANNON) return fail(BL_EUNSUPPORTED, "grad_x is implemented for BL_SHANNON");
    if (p.prec == BL_F64 && p.win != BL_WIN_SINH && !(p.poly64_deriv_err <= kDerivFitTol))
        return fail(BL_EUNSUPPORTED, "FP64 grad_x of this window needs weight-polynomial derivatives within 5e-12");
    if (!p.have_theta) return fail(BL_ESTATE, "bl_grad_x needs the samples of a preceding bl_forward");
    if (p.N > 0 && (!g_dev || !gx_dev)) return fail(BL_EINVAL, "NULL buffer");
    return launch_grad_x(p, g_dev, gx_dev);
}

bl_status bl_plan_stats(bl_plan plan, bl_stats* out) {
    if (!plan || !out) return fail(BL_EINVAL, "NULL argument");
    const Plan& p = plan->p;
    std::memset(out, 0, sizeof(*out));
    out->n_nodes = p.N;
    out->n_outside = p.n_outside;
    out->n_chunks = p.nchunks;
    for (int t = 0; t < 3; ++t) out->tile[t] = p.tile[t];
    out->chunk_cap = p.chunk_cap;
    out->workspace_bytes = int64_t(p.workspace_bytes);
    out->beta = p.beta;
    out->weight_fit_err = p.prec == BL_F64 ? (p.use_poly64 ? p.poly64_err : 0.0) : p.poly_err;
    for (int i = 0; i < 2; ++i)
        for (int t = 0; t < 3; ++t) {
            out->fft_lines[i][t] = p.fft_lines[i][t];
            out->fft_radix[i][t] = p.fft_radix[i][t];
        }
    out->tuned[0] = p.tune_fft_source;
    out->tuned[1] = p.tune_tile_source;
    return BL_OK;
}

}  // extern "C"
