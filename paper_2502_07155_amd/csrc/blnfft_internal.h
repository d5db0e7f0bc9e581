// Internal declarations of the blnfft library (host side and kernel launchers).
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "blnfft.h"

namespace bl {

// Thread-local error text for bl_last_error().
void set_error(const std::string& msg);
const std::string& last_error();

// Return BL_EDEVICE (with the failing call's text) if a HIP call failed.
#define BL_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            ::bl::set_error(std::string(#call) + ": " + hipGetErrorString(e_));        \
            return e_ == hipErrorOutOfMemory ? BL_ENOMEM : BL_EDEVICE;                \
        }                                                                             \
    } while (0)

#define BL_TRY(expr)                         \
    do {                                     \
        bl_status s_ = (expr);               \
        if (s_ != BL_OK) return s_;          \
    } while (0)

constexpr int kMaxStages = 16;
constexpr int kCovMax = 4;                    // covering boxes per coordinate in the merge table
constexpr int kCovRow = 2 + 2 * kCovMax;      // tile, count, (tile offset, box position) pairs
constexpr int kNbR = 2;                       // largest tile offset of a covering box per dimension
constexpr int kMinM = 2;    // truncation range of the compiled short-sum kernels
constexpr int kMaxM = 8;
constexpr int kPolyCoef = 12;   // coefficients of the float weight polynomials (degree 11)
constexpr int kPolyCoef64 = 16; // coefficients of the double weight polynomials (degree 15)
constexpr double kDerivFitTol = 5e-12;   // FP64 grad_x from differentiated polynomials (relative)
constexpr double kPolyFitTol = 1e-7;     // float weight polynomials (relative to the largest weight)
// Float tiles of the short sums are staged twice (shifted copies, for 128-bit row reads)
// when the doubled tile still leaves room for several workgroups per CU.
constexpr bool dual_tiles_for(int d, int m, bool is_float) {
    return is_float && (d == 2 || (d == 3 && m <= 5));
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.  Maps the
// hardware block index p (of n) to a logical one so that each XCD runs one contiguous
// range of logical blocks: neighbouring work items (strided FFT lines, adjacent tiles
// with overlapping halos, entries of one batched instance) then share an L2.  A
// bijection of [0, n).
__device__ __forceinline__ int xcd_block(int p, int n) {
    constexpr int X = 8;
    const int x = p % X;
    const int q = n / X, r = n % X;
    const int start = x * q + (x < r ? x : r);
    return start + p / X;
}

// Factorisation of one FFT length into Stockham stages.
struct FftFactors {
    int L = 0;
    int nstages = 0;
    int radix[kMaxStages] = {0};
};
// Powers of two L >= 16 as main-radix stages E, ..., E followed by at most one smaller
// power of two; false otherwise.
bool factor_length(int L, int E, FftFactors* out);

// Device twiddles of one stage plan: w^{r k} per stage, laid out [k][r-1].
struct FftStages {
    int nmain = 0, rlast = 1;
    int tw_off[kMaxStages] = {0};
    int tw_len = 0;
    void* d_tw64 = nullptr;
    void* d_tw32 = nullptr;
};

// One pass of the pruned multi-dimensional iFFT: transforms axis `axis` of an array
// whose axes before `axis` have extent M (still in frequency), `axis` has Min inputs
// (M) and L outputs, and axes after it have extent L (already transformed).
struct PassShape {
    int64_t outer = 1;   // M^axis
    int64_t inner = 1;   // L^(d-1-axis)
    int Min = 0;         // inputs per line (M)
    int L = 0;           // FFT length and outputs per line
};

// Element types of one FFT pass: input in double, arithmetic in double, output in double,
// twiddle (and chirp) tables in double with their products formed in double.
struct PassTypes {
    bool in64, comp64, out64, tw64;
};

// Largest chirp-z transform held in LDS by one workgroup (points of the arithmetic type).
template <typename R>
constexpr int64_t kCztLdsPoints() { return sizeof(R) == 8 ? 8192 : 16384; }

// Chirp-z (Bluestein) form of the per-axis transforms, for L that the power-of-two passes
// do not take: cyclic convolutions of power-of-two size P >= L + M - 1.
struct CztTables {
    bool on = false;       // the plan's passes use the chirp-z kernels
    int64_t P = 0;
    bool split = false;    // one d = 1 line above the LDS size: R pieces of P / R points
    int R = 1;
    void* d_roots64 = nullptr;   // e^{2 pi i n / P}, n < P
    void* d_roots32 = nullptr;
    void* d_H64 = nullptr;       // H = DFT_P(h) / P
    void* d_H32 = nullptr;
    void* d_band64 = nullptr;    // 1/(L psihat1(k)) e^{i pi k^2 / L}, k = i - M/2 (M entries)
    void* d_band32 = nullptr;
    void* d_grid64 = nullptr;    // e^{i pi l^2 / L}, l = i - L/2 (L entries)
    void* d_grid32 = nullptr;
    void* d_scr = nullptr;       // split path: P complex of the arithmetic type
};

// Device tables and buffers owned by a plan.
struct Plan {
    int d = 0;
    int64_t M = 0, L = 0;
    int m = 0;
    bl_window win = BL_WIN_SINH;
    bl_method method = BL_SHANNON;
    bl_precision prec = BL_F64;
    double beta = 0.0;
    hipStream_t stream = nullptr;
    int device = 0;

    // Per-dimension deconvolution factor 1/(L * hat1(k)), k = i - M/2 (FP64, M entries).
    double* d_deconv = nullptr;
    // Stage plans with main radix 16 and 4 and their twiddles.
    FftStages st16, st4;
    // Float weight polynomials, [m][kPolyCoef] (even then odd coefficients), and the
    // largest deviation of the fitted weights from the exact ones.
    std::vector<float> poly;
    double poly_err = 0.0;         // refused above kPolyFitTol for float plans
    // The same in double with kPolyCoef64 coefficients (BL_F64 plans), used when the fit
    // is within 1e-13 of the exact weights; otherwise the kernels evaluate them exactly.
    std::vector<double> poly64;
    double poly64_err = 0.0;
    double poly64_deriv_err = 1.0;  // relative error of the polynomials' theta-derivatives
    bool use_poly64 = false;
    double edge_k = 1.0;           // edge exponent of the weight polynomials (edge_exponent)
    bool fft_ok = true;            // steps 1-2 and the adjoint available for this L
    int fft_lines[2][3] = {{0, 0, 0}, {0, 0, 0}};   // [forward, adjoint][axis]: tuned lines per workgroup
    int fft_radix[2][3] = {{0, 0, 0}, {0, 0, 0}};   // the same for the values per thread (4 or 16)
    int tune_fft_source = 0;       // 0 heuristic (or override), 1 measured, 2 from the tuning cache
    int tune_tile_source = 0;      // the same for the short-sum tiles and chunk capacity
    int64_t tuned_N = -1;          // node count the tiles were tuned (or looked up) for
    CztTables czt;                 // chirp-z passes (L not a power of two, or too long)
    void* d_wpre = nullptr;        // precomputed weights (bl_precompute_weights), binned order
    bool use_wpre = false;
    // Inverse-direction twiddles for the adjoint are the conjugates; computed in kernel.

    // FFT ping-pong buffers and the grid of theta (L^d complex).
    void* d_bufA = nullptr;
    void* d_bufB = nullptr;
    void* d_grid = nullptr;
    void* d_sgrid = nullptr;   // adjoint spreading target (allocated on first bl_adjoint)
    void* d_boxes = nullptr;   // adjoint: one tile-plus-halo box per chunk (first bl_adjoint)
    size_t boxes_cap = 0;
    size_t bytes_grid = 0, bytes_A = 0, bytes_B = 0;

    // Nodes, sorted by tile.
    int64_t N = 0;
    int64_t N_cap = 0;
    void* d_xs = nullptr;          // N x d sorted copy
    int32_t* d_perm = nullptr;     // sorted position -> caller index
    int32_t* d_node_tile = nullptr;
    int tile[3] = {1, 1, 1};       // cells per tile edge
    int tiles_per_dim[3] = {1, 1, 1};
    int64_t ntiles = 0;
    int chunk_cap = 1024;
    // float tiles of d >= 2 staged twice (shifted copies) for 128-bit row reads
    bool dual_tiles = false;
    int64_t tile_alloc = 0;        // entries of the four per-tile arrays
    int32_t* d_tile_count = nullptr;
    int32_t* d_tile_offset = nullptr;
    int32_t* d_tile_cursor = nullptr;
    int32_t* d_chunk_offset = nullptr;
    void* d_scan = nullptr;        // block sums of the tile scans (tile_scan_scratch_bytes)
    // Adjoint merge table: per grid coordinate (shared by the dimensions) its tile and the
    // (tile offset, box position) pairs of the boxes that cover it (kCovRow ints, up to
    // kCovMax pairs with offsets within kNbR; null otherwise), and for d = 3 one reach flag
    // per tile.
    int* d_cov = nullptr;
    unsigned char* d_reach = nullptr;
    int4* d_chunks = nullptr;      // {tile, start, count, 0}
    int64_t chunk_alloc = 0;
    int64_t nchunks = 0;
    unsigned long long* d_flags = nullptr;  // [0]: invalid nodes, [1]: outside truncated domain, [2]: chunks
    int64_t n_outside = 0;

    bool have_nodes = false;
    bool have_theta = false;
    size_t workspace_bytes = 0;

    // Forward transform captured as hipGraphs (on a private stream) and replayed on
    // `stream`: one executable graph per (fhat, f) pointer pair, up to kGraphCache of
    // them (least recently used evicted), all valid for one node binding.
    static constexpr int kGraphCache = 4;
    struct FwdGraph {
        hipGraphExec_t exec = nullptr;
        const void* fhat = nullptr;
        void* f = nullptr;
        uint64_t used = 0;
    };
    bool use_graph = false;   // BL_GRAPH=1: forward transforms replay a captured graph
    hipStream_t capture_stream = nullptr;
    FwdGraph graphs[kGraphCache];
    uint64_t graph_tick = 0;

    size_t real_size() const { return prec == BL_F64 ? 8 : 4; }
    // FFT arithmetic in double (F64, and F32D's float data with double passes)
    bool fft64() const { return prec == BL_F64 || prec == BL_F32D; }
    size_t cplx_size() const { return 2 * real_size(); }
    int64_t grid_elems() const {
        int64_t g = 1;
        for (int t = 0; t < d; ++t) g *= L;
        return g;
    }
    int64_t band_elems() const {
        int64_t g = 1;
        for (int t = 0; t < d; ++t) g *= M;
        return g;
    }
};

// ---- host tables (host_tables.cpp)
double default_beta(int64_t M, int64_t L, int m, bl_method method);
// Univariate transform of psi (shannon) or phi (nfft) at v, by the library's own
// double-exponential quadrature.
double window_transform(bl_window win, bl_method method, int64_t L, int m, double beta, double v);
// The same at v = 0, 1, ..., K-1 (out has K entries).
void window_transform_ints(bl_window win, bl_method method, int64_t L, int m, double beta, int64_t K,
                           double* out);
// e^{2 pi i n / L} for n in [0, L), correctly reduced; interleaved (re, im).
void twiddles(int64_t L, std::vector<double>* out);
bool factor_length(int L, int E, FftFactors* out);
// In-place FP64 radix-2 DFT with kernel e^{-2 pi i n q / P} (root[k] = e^{2 pi i k/P}, k < P/2).
void host_dft(std::vector<std::complex<double>>& x, const std::vector<std::complex<double>>& root);
// e^{i pi q / L} for integer q, reduced mod 2L in integers (tw2L = twiddles(2L)).
std::complex<double> chirp(int64_t q, int64_t L, const std::vector<double>& tw2L);
// Chirp-z convolution kernel spectrum H = DFT_P(h) / P of h_j = e^{-i pi j^2 / L} at cyclic
// position j mod P, |j| < (L + M)/2 (zero elsewhere), FP64; P >= L + M - 1, a power of two.
std::vector<std::complex<double>> chirp_spectrum(int64_t L, int64_t M, int64_t P);
void stage_twiddles(const FftFactors& fac, const std::vector<double>& tw, std::vector<double>* out,
                    int* off);
double window_value(bl_window win, bl_method method, int m, double beta, double u);
double edge_exponent(bl_window win);
double window_deriv_value(bl_window win, bl_method method, int m, double beta, double u);
double weight_deriv_fit_error(bl_window win, bl_method method, int m, double beta, int nc,
                              const std::vector<double>& coef);
double fit_weight_polys(bl_window win, bl_method method, int m, double beta, int nc,
                        std::vector<double>* coef);

// ---- kernel launchers (fft.hip, gather.hip, bin.hip)
// Steps 1-2: deconvolve + zero-pad + iFFT, f̂ (M^d) -> grid (L^d).  `sign` = +1 forward
// transform (inverse DFT); the adjoint path uses launch_fft_adjoint.
bl_status launch_forward_fft(Plan& p, const void* fhat);
// Adjoint FFT: grid (L^d, centred) -> fhat (M^d) with e^{-2 pi i k l/L} and D.
bl_status launch_adjoint_fft(Plan& p, const void* grid, void* fhat_out);
// Step 3 on the plan's grid (or a given theta).
bl_status launch_gather(Plan& p, const void* theta, void* f);
// Evaluate the weights of every bound node into p.d_wpre (Algorithm 4.2, step 0b).
bl_status launch_weights(Plan& p);
// Binning of nodes.
bl_status launch_binning(Plan& p, const void* x, int64_t N);
// Device-wide exclusive scans of per-tile node counts and chunk counts ceil(count / cap);
// flags[2] receives the total chunk count.  scratch: tile_scan_scratch_bytes(ntiles).
bl_status launch_tile_scan(const int32_t* count, int32_t* offset, int32_t* chunk_off, int64_t ntiles, int cap,
                           unsigned long long* flags, void* scratch, hipStream_t stream);
size_t tile_scan_scratch_bytes(int64_t ntiles);
// Adjoint spreading Psi^T g (or B^T g) onto `grid` (L^d, centred), which it overwrites:
// per-chunk boxes into `boxes` (spread_boxes_bytes), then their fixed-order merge.
bl_status launch_spread(Plan& p, const void* g, void* grid, void* boxes);
size_t spread_boxes_bytes(const Plan& p);
// bl_adjoint with the spreading grid and chunk boxes in the library's fixed device scratch
// (no allocation); BL_EUNSUPPORTED when they exceed it.
bl_status launch_adjoint_noalloc(Plan& p, const void* g, void* fhat_out);
size_t noalloc_scratch_bytes();
// One chirp-z pass (czt.hip): lines outer x inner, Min inputs and Mout outputs per line in
// centred order; dir +1 forward (band -> grid), -1 adjoint (grid -> band).
bl_status launch_czt_pass(Plan& p, int dir, const void* in, void* out, int outer, int inner, int Min,
                          int Mout, PassTypes t, int lines);
// Autotuner (fft.hip): time every forward and adjoint pass of the plan for 1, 2, ..., 64
// lines per workgroup and 4 or 16 values per thread on the given scratch buffers (each >= L^d complex of the pass type)
// and keep the fastest in p.fft_lines.
bl_status tune_fft_lines(Plan& p, void* buf_in, void* buf_out);
// autotune.cpp: FFT lines per workgroup at plan creation (cached), and the cache of the
// short-sum tile edge and chunk capacity measured at the first large node binding.
constexpr int64_t kTuneMinNodes = int64_t(1) << 16;
bool tuning_enabled();
bool tune_lookup(const std::string& key, std::vector<int>* vals);
void tune_store(const std::string& key, const std::vector<int>& vals);
std::string tune_device_tag(int device);   // architecture and compute-unit count
bl_status autotune_fft(Plan& p);
bool tile_tuning_wanted(const Plan& p, int64_t N);
bool tile_cache_lookup(const Plan& p, int density, int cluster, int* T, int* cap);
void tile_cache_store(const Plan& p, int density, int cluster, int T, int cap);
// Node gradient from the plan's grid.
bl_status launch_grad_x(Plan& p, const void* g, void* gx);

}  // namespace bl
