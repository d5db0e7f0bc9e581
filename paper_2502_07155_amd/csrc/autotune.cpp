// Autotuner of the per-plan launch shapes, with a persistent cache.
//
// Measured on the plan's own device and stream, never guessed:
//  * FFT passes (at plan creation): lines per workgroup (1, 2, ..., 64, as far as the
//    pass's LDS and thread limits allow) and values per thread (4 or 16) of every forward
//    and adjoint pass, timed with HIP events on scratch buffers (tune_fft_lines, fft.hip);
//  * short sums (at the first node binding with at least kTuneMinNodes nodes): the tile
//    edge of the node binning and the work-chunk capacity, timed by binning the nodes with
//    each candidate and running the short-sum kernel on zero samples.
// Results are cached per process and in a JSON file (one object of "key": [values]),
// keyed by device (architecture and compute-unit count), dimension, M, L, m, precision,
// method and, for the short sums, the node-density class (nodes per grid point and the
// fullest tile against the mean, both on a log2 scale).  BL_AUTOTUNE=0 turns the tuner
// off; BL_TUNE_CACHE names the cache file ("off": this process only; default
// $XDG_CACHE_HOME/blnfft/tune.json or ~/.cache/blnfft/tune.json).  BL_TILE and
// BL_FFT_LINES override the tuner.
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "blnfft_internal.h"

namespace bl {
namespace {

std::mutex g_mu;
std::map<std::string, std::vector<int>> g_cache;   // entries of the file g_path
bool g_loaded = false;
std::string g_path;


std::string cache_path() {
    if (const char* e = std::getenv("BL_TUNE_CACHE")) return std::string(e) == "off" ? std::string() : std::string(e);
    if (const char* x = std::getenv("XDG_CACHE_HOME")) return std::string(x) + "/blnfft/tune.json";
    if (const char* h = std::getenv("HOME")) return std::string(h) + "/.cache/blnfft/tune.json";
    return std::string();
}

// Entries "key": [v, v, ...] of the flat JSON object written by save_cache.
void load_cache_locked() {
    const std::string path = cache_path();
    if (g_loaded && path == g_path) return;
    g_loaded = true;
    g_path = path;
    g_cache.clear();
    if (path.empty()) return;
    std::ifstream in(path);
    if (!in) return;
    std::stringstream ss;
    ss << in.rdbuf();
    const std::string text = ss.str();
    size_t pos = 0;
    while ((pos = text.find('"', pos)) != std::string::npos) {
        const size_t end = text.find('"', pos + 1);
        if (end == std::string::npos) break;
        const std::string key = text.substr(pos + 1, end - pos - 1);
        const size_t lb = text.find('[', end), rb = text.find(']', end);
        if (lb == std::string::npos || rb == std::string::npos || rb < lb) break;
        std::vector<int> vals;
        std::stringstream vs(text.substr(lb + 1, rb - lb - 1));
        std::string tok;
        while (std::getline(vs, tok, ',')) {
            if (tok.find_first_of("0123456789") != std::string::npos) vals.push_back(std::atoi(tok.c_str()));
        }
        if (!key.empty()) g_cache[key] = vals;
        pos = rb + 1;
    }
}

void make_dirs(const std::string& path) {
    for (size_t i = 1; i < path.size(); ++i)
        if (path[i] == '/') mkdir(path.substr(0, i).c_str(), 0755);
}

// Rewrites the whole file (write to a temporary name, then rename): a failed write leaves
// the old cache in place, and the in-process cache keeps working without a file.
void save_cache_locked() {
    const std::string& path = g_path;
    if (path.empty()) return;
    make_dirs(path);
    const std::string tmp = path + ".tmp" + std::to_string(long(getpid()));
    {
        std::ofstream out(tmp);
        if (!out) return;
        out << "{\n";
        size_t n = 0;
        for (const auto& kv : g_cache) {
            out << "  \"" << kv.first << "\": [";
            for (size_t i = 0; i < kv.second.size(); ++i) out << (i ? ", " : "") << kv.second[i];
            out << "]" << (++n < g_cache.size() ? "," : "") << "\n";
        }
        out << "}\n";
        if (!out) return;
    }
    std::rename(tmp.c_str(), path.c_str());
}

}  // namespace

bool tuning_enabled() {
    const char* e = std::getenv("BL_AUTOTUNE");
    return !(e && e[0] == '0');
}

bool tune_lookup(const std::string& key, std::vector<int>* vals) {
    std::lock_guard<std::mutex> lock(g_mu);
    load_cache_locked();
    auto it = g_cache.find(key);
    if (it == g_cache.end()) return false;
    *vals = it->second;
    return true;
}

void tune_store(const std::string& key, const std::vector<int>& vals) {
    std::lock_guard<std::mutex> lock(g_mu);
    load_cache_locked();
    g_cache[key] = vals;
    save_cache_locked();
}

std::string tune_device_tag(int device) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
    std::string arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    return arch + "x" + std::to_string(prop.multiProcessorCount);
}

namespace {

const char* prec_name(bl_precision p) {
    switch (p) {
        case BL_F64: return "f64";
        case BL_F32: return "f32";
        case BL_F32C: return "f32c";
        default: return "f32d";
    }
}

std::string plan_key(const Plan& p, const char* what) {
    std::ostringstream k;
    k << what << "|" << tune_device_tag(p.device) << "|d" << p.d << "|M" << p.M << "|L" << p.L << "|m" << p.m << "|"
      << prec_name(p.prec) << "|" << (p.method == BL_NFFT ? "nfft" : "shannon") << "|"
      << (p.czt.on ? "czt" : "pow2");
    return k.str();
}

}  // namespace

bl_status autotune_fft(Plan& p) {
    if (!p.fft_ok || !tuning_enabled() || std::getenv("BL_FFT_LINES") || std::getenv("BL_CZT_LINES")) return BL_OK;
    const std::string key = plan_key(p, "fft");
    std::vector<int> v;
    if (tune_lookup(key, &v) && v.size() == 12) {
        for (int i = 0; i < 6; ++i) {
            p.fft_lines[i / 3][i % 3] = v[i];
            p.fft_radix[i / 3][i % 3] = v[6 + i];
        }
        p.tune_fft_source = 2;
        return BL_OK;
    }
    // two scratch grids of the widest pass element (double for F64 and F32D passes)
    const size_t bytes = size_t(p.grid_elems()) * (p.fft64() ? 16 : 8);
    void* a = nullptr;
    void* b = nullptr;
    if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) {
        (void)hipGetLastError();
        hipFree(a);
        return BL_OK;   // tuning is an optimisation: keep the heuristic
    }
    bl_status st = BL_OK;
    if (hipMemsetAsync(a, 0, bytes, p.stream) == hipSuccess) st = tune_fft_lines(p, a, b);
    (void)hipStreamSynchronize(p.stream);
    hipFree(a);
    hipFree(b);
    if (st != BL_OK) {
        for (int i = 0; i < 6; ++i) p.fft_lines[i / 3][i % 3] = p.fft_radix[i / 3][i % 3] = 0;
        set_error("");
        return BL_OK;
    }
    v.assign(12, 0);
    for (int i = 0; i < 6; ++i) {
        v[i] = p.fft_lines[i / 3][i % 3];
        v[6 + i] = p.fft_radix[i / 3][i % 3];
    }
    tune_store(key, v);
    p.tune_fft_source = 1;
    return BL_OK;
}

std::string tile_key(const Plan& p, int density, int cluster) {
    return plan_key(p, "tiles") + "|n" + std::to_string(density) + "|c" + std::to_string(cluster);
}

bool tile_tuning_wanted(const Plan& p, int64_t N) {
    return tuning_enabled() && std::getenv("BL_TILE") == nullptr && N >= kTuneMinNodes && p.d >= 1;
}

bool tile_cache_lookup(const Plan& p, int density, int cluster, int* T, int* cap) {
    std::vector<int> v;
    if (!tune_lookup(tile_key(p, density, cluster), &v) || v.size() != 2) return false;
    *T = v[0];
    *cap = v[1];
    return true;
}

void tile_cache_store(const Plan& p, int density, int cluster, int T, int cap) {
    tune_store(tile_key(p, density, cluster), std::vector<int>{T, cap});
}

}  // namespace bl
