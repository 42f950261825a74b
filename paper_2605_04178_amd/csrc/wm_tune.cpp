// wm_tune.cpp -- launch-configuration registry: defaults, tuned entries keyed
// by (GPU architecture, compute units, op, floor(log2 n)), and an optional
// JSON-lines cache file named by the WAVEMODEL_TUNE_CACHE environment
// variable (read once, appended to by every persisted tuning result).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "wm_launch.hpp"

namespace wm {
namespace {

typedef std::tuple<std::string, int, int, int> Key;  // arch, CUs, op, bucket

std::mutex g_mu;
std::map<Key, LaunchCfg> g_cfg;
bool g_loaded = false;
std::vector<std::pair<std::string, int>> g_dev;  // per device index: arch, CUs

int bucket_of(int64_t n)
{
    int b = 0;
    while (b < 62 && ((int64_t)1 << (b + 1)) <= n) ++b;
    return n <= 0 ? 0 : b;
}

int canonical_op(int op) { return op == kOpCalibrate ? kOpLossGrad : op; }

// caller holds g_mu
bool device_id(std::string& arch, int& cus)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return false;
    if ((int)g_dev.size() <= dev) g_dev.resize(dev + 1, std::make_pair(std::string(), 0));
    if (g_dev[dev].first.empty()) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
        std::string a(prop.gcnArchName);
        const size_t colon = a.find(':');
        if (colon != std::string::npos) a = a.substr(0, colon);
        g_dev[dev] = std::make_pair(a, prop.multiProcessorCount);
    }
    arch = g_dev[dev].first;
    cus = g_dev[dev].second;
    return true;
}

bool get_int(const char* line, const char* key, long long* out)
{
    const char* p = std::strstr(line, key);
    if (!p) return false;
    p = std::strchr(p + std::strlen(key), ':');
    if (!p) return false;
    return std::sscanf(p + 1, " %lld", out) == 1;
}

bool get_str(const char* line, const char* key, std::string* out)
{
    const char* p = std::strstr(line, key);
    if (!p) return false;
    p = std::strchr(p + std::strlen(key), ':');
    if (!p) return false;
    p = std::strchr(p, '"');
    if (!p) return false;
    const char* q = std::strchr(p + 1, '"');
    if (!q) return false;
    out->assign(p + 1, q);
    return true;
}

// caller holds g_mu
void load_cache()
{
    if (g_loaded) return;
    g_loaded = true;
    const char* path = std::getenv("WAVEMODEL_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof(line), f)) {
        std::string arch;
        long long cus, op, bucket, block, vec, gm, chunk;
        if (!get_str(line, "\"arch\"", &arch) || !get_int(line, "\"cus\"", &cus) ||
            !get_int(line, "\"op\"", &op) || !get_int(line, "\"bucket\"", &bucket) ||
            !get_int(line, "\"block\"", &block) || !get_int(line, "\"vec\"", &vec) ||
            !get_int(line, "\"grid_mult\"", &gm) || !get_int(line, "\"chunk\"", &chunk))
            continue;
        LaunchCfg c;
        c.block = (int32_t)block;
        c.vec = (int32_t)vec;
        c.grid_mult = (int32_t)gm;
        c.chunk = (int32_t)chunk;
        if (!cfg_valid((int)op, c)) continue;
        g_cfg[Key(arch, (int)cus, canonical_op((int)op), (int)bucket)] = c;
    }
    std::fclose(f);
}

bool pow2_in(int64_t x, int64_t lo, int64_t hi)
{
    return x >= lo && x <= hi && (x & (x - 1)) == 0;
}

}  // namespace

LaunchCfg default_cfg(int op)
{
    LaunchCfg c;
    c.block = 256;
    c.vec = 1;
    c.grid_mult = 1;
    c.chunk = 0;
    switch (canonical_op(op)) {
    case kOpPredict: c.vec = 4; break;
    case kOpCalibrateBatched: c.chunk = 2048; break;
    default: break;
    }
    return c;
}

bool cfg_valid(int op, const LaunchCfg& c)
{
    const bool blk = c.block == 64 || c.block == 128 || c.block == 256 || c.block == 512;
    switch (canonical_op(op)) {
    case kOpPredict:
        return blk && (c.vec == 1 || c.vec == 2 || c.vec == 4 || c.vec == 8);
    case kOpVjp:
    case kOpLossGrad:
    case kOpSelectTile:
    case kOpPredictApps:
    case kOpAppsLossGrad:
        return blk && c.grid_mult >= 1 && c.grid_mult <= 8;
    case kOpCalibrateBatched:
        return c.block == 256 && c.grid_mult >= 1 && c.grid_mult <= 8 &&
               pow2_in(c.chunk, kMinChunk, 65536);
    default:
        return false;
    }
}

LaunchCfg launch_cfg(int op, int64_t n)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_cache();
    std::string arch;
    int cus = 0;
    if (device_id(arch, cus)) {
        auto it = g_cfg.find(Key(arch, cus, canonical_op(op), bucket_of(n)));
        if (it != g_cfg.end()) return it->second;
    }
    return default_cfg(op);
}

void store_cfg(int op, int64_t n, const LaunchCfg& c, double us, bool persist)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_cache();
    std::string arch;
    int cus = 0;
    if (!device_id(arch, cus)) return;
    const int b = bucket_of(n);
    g_cfg[Key(arch, cus, canonical_op(op), b)] = c;
    const char* path = std::getenv("WAVEMODEL_TUNE_CACHE");
    if (!persist || !path || !*path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f,
                 "{\"arch\": \"%s\", \"cus\": %d, \"op\": %d, \"bucket\": %d, \"block\": %d, "
                 "\"vec\": %d, \"grid_mult\": %d, \"chunk\": %d, \"us\": %.3f}\n",
                 arch.c_str(), cus, canonical_op(op), b, c.block, c.vec, c.grid_mult, c.chunk, us);
    std::fclose(f);
}

}  // namespace wm
