// swe_tune.hip - tile-variant autotuner.
//
// For a grid size the tuner times every compiled tile variant of the stage
// kernel on a synthetic wet problem of that size (a sloping bed under a
// Gaussian surface hump with momentum, so every WENO weight is exercised) and
// keeps the fastest.  Results live in a process-wide table consulted by
// default_variant() and, optionally, in a JSON file keyed by
// "<arch>:<nx>x<ny>".  Tile shape does not change results.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "swe_internal.hpp"

namespace swe {

static std::mutex g_tune_mu;

// First variant with this tile shape (0 if none: every variant is correct).
static int variant_by_shape(int tx, int ty, int r)
{
    for (int i = 0; i < variant_count(); ++i) {
        const Variant &v = variant(i);
        if (v.tx == tx && v.ty == ty && v.r == r) return i;
    }
    return 0;
}
static std::map<std::pair<int, int>, int> g_tuned;

// Built-in choice when nothing was tuned for this size.  With 256 or more
// 128x16 tiles (about one per CU and more) that tile (256 threads, 8 cells per
// thread per sweep) measured fastest on MI355X (1024x512 to 4096^2).  Smaller
// grids leave most CUs idle and a stage lasts one block's critical path,
// which tiles with fewer cells per thread shorten: 64x16 with 4 cells per
// thread from 64 tiles (512^2: 4.95e9 vs 4.20e9 cell-updates/s), 32x16 with 2
// below (256^2: 1.74e9 vs 1.09e9).
int default_variant(int nx, int ny)
{
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find({nx, ny});
        if (it != g_tuned.end()) return it->second;
    }
    const long long tiles = (long long)((nx + 127) / 128) * ((ny + 15) / 16);
    if (tiles >= 256) return variant_by_shape(128, 16, 8);
    return tiles >= 64 ? variant_by_shape(64, 16, 4) : variant_by_shape(32, 16, 2);
}

// Variant of a launch over several scenarios (a batch run or a server
// segment).  Once their 128x16 tiles number 256 or more together, the GPU is
// full whatever each grid's size, and the 128x16 tile with 8 cells per
// thread (the fewest instructions per cell) is the fastest for the mix: the
// size a grid alone would be tuned to only matters when the launch cannot
// fill the GPU.  Otherwise the largest scenario's own choice.
int batch_variant_for(const std::vector<std::pair<int, int>> &sizes)
{
    long long tiles = 0;
    size_t big = 0;
    int nx = 0, ny = 0;
    for (const auto &s : sizes) {
        tiles += (long long)((s.first + 127) / 128) * ((s.second + 15) / 16);
        if ((size_t)s.first * s.second > big) {
            big = (size_t)s.first * s.second;
            nx = s.first;
            ny = s.second;
        }
    }
    if (tiles >= 256) return variant_by_shape(128, 16, 8);
    return default_variant(nx, ny);
}

static std::string arch_name()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

static std::string read_file(const char *path)
{
    std::string s;
    FILE *f = std::fopen(path, "rb");
    if (!f) return s;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, n);
    std::fclose(f);
    return s;
}

// Entries of the cache: "key": {"tile": T, "ms_per_step": M}
static std::map<std::string, std::pair<int, double>> parse_cache(const std::string &s)
{
    std::map<std::string, std::pair<int, double>> out;
    size_t pos = 0;
    while ((pos = s.find('"', pos)) != std::string::npos) {
        const size_t end = s.find('"', pos + 1);
        if (end == std::string::npos) break;
        const std::string key = s.substr(pos + 1, end - pos - 1);
        pos = end + 1;
        if (key == "tile" || key == "ms_per_step") continue;
        const size_t t = s.find("\"tile\"", pos), m = s.find("\"ms_per_step\"", pos);
        const size_t close = s.find('}', pos);
        if (t == std::string::npos || m == std::string::npos || close == std::string::npos || t > close ||
            m > close)
            continue;
        int tile = -1;
        double ms = 0;
        if (std::sscanf(s.c_str() + s.find(':', t) + 1, "%d", &tile) == 1 &&
            std::sscanf(s.c_str() + s.find(':', m) + 1, "%lf", &ms) == 1 && tile >= 0 && tile < variant_count())
            out[key] = {tile, ms};
        pos = close + 1;
    }
    return out;
}

static void write_cache(const char *path, const std::map<std::string, std::pair<int, double>> &m)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return;
    std::fprintf(f, "{\n");
    size_t i = 0;
    for (const auto &kv : m)
        std::fprintf(f, " \"%s\": {\"tile\": %d, \"ms_per_step\": %.6f}%s\n", kv.first.c_str(), kv.second.first,
                     kv.second.second, ++i < m.size() ? "," : "");
    std::fprintf(f, "}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

}  // namespace swe

using namespace swe;

extern "C" int swe_autotune(int32_t nx, int32_t ny, const char *cache_path, int32_t *best_tile,
                            double *best_ms_per_step)
{
    if (nx < 3 || ny < 3 || !best_tile) return SWE_EINVAL;
    char keybuf[128];
    std::snprintf(keybuf, sizeof keybuf, "%s:%dx%d", arch_name().c_str(), nx, ny);
    const std::string key = keybuf;
    std::map<std::string, std::pair<int, double>> cache;
    if (cache_path) {
        cache = parse_cache(read_file(cache_path));
        auto it = cache.find(key);
        if (it != cache.end()) {
            *best_tile = it->second.first;
            if (best_ms_per_step) *best_ms_per_step = it->second.second;
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tuned[{nx, ny}] = it->second.first;
            return SWE_OK;
        }
    }
    // synthetic wet problem
    const size_t N = (size_t)nx * ny;
    std::vector<float> b(N), n(N, 0.03f), h(N), hu(N), hv(N);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const double x = (i + 0.5) / nx, y = (j + 0.5) / ny;
            const double bed = -20.0 + 10.0 * x + std::sin(6.0 * y);
            const double eta = 2.0 * std::exp(-((x - 0.3) * (x - 0.3) + (y - 0.5) * (y - 0.5)) / 0.01);
            const size_t k = (size_t)j * nx + i;
            b[k] = (float)bed;
            h[k] = (float)std::max(eta - bed, 0.0);
            hu[k] = (float)(0.5 * h[k] * std::sin(3.0 * y));
            hv[k] = (float)(0.3 * h[k] * std::cos(2.0 * x));
        }
    swe_params p{};
    p.nx = nx;
    p.ny = ny;
    p.dx = p.dy = 2.0;
    p.g = 9.81;
    p.cfl = 0.4;
    p.h_dry = 1e-3;
    p.weno_eps = 1e-6;
    p.kappa_cap = 1.0;
    swe_ctx *c = nullptr;
    int rc = swe_create(&p, b.data(), n.data(), h.data(), hu.data(), hv.data(), nullptr, &c);
    if (rc) return rc;
    int best = -1;
    double best_ms = 1e300;
    const int reps = N >= (1u << 22) ? 3 : 10;
    for (int vi = 0; vi < variant_count() && !rc; ++vi) {
        rc = swe_set_option(c, SWE_OPT_TILE, vi);
        double ms[3];
        if (!rc) rc = swe_time_stages(c, 2, ms);  // warm-up
        if (!rc) rc = swe_time_stages(c, reps, ms);
        if (!rc && ms[0] + ms[1] + ms[2] < best_ms) {
            best_ms = ms[0] + ms[1] + ms[2];
            best = vi;
        }
    }
    swe_destroy(c);
    if (rc) return rc;
    *best_tile = best;
    if (best_ms_per_step) *best_ms_per_step = best_ms;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[{nx, ny}] = best;
    }
    if (cache_path) {
        cache[key] = {best, best_ms};
        write_cache(cache_path, cache);
    }
    return SWE_OK;
}
