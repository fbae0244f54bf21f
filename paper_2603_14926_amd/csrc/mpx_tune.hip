// mpx_tune.hip -- persistent cache of autotuned launch choices (host code).
//
// The GEMM tilings and the root solver's launch variants give identical bits,
// so a tuned choice is pure performance state.  It is kept per process and,
// when MPX_TUNE_CACHE names a file, in that file as well, so later processes
// start from the tuned choice instead of the size heuristic.
//
// File format: one entry per line, whitespace-separated
//     <gfx arch> <op> <key...> <choice>
// e.g. "gfx950 gemm 4 0 0 11 11 11 qd_2x2_k8" (precision, transposes, log2
// size buckets, tiling name) or "gfx950 dk 4 12 9 6" (precision, log2 batch
// and largest-degree buckets, variant index).  Lines for other GPUs are kept
// untouched; a later entry for the same (arch, op, key) replaces an earlier
// one.  The file is read on first use (and by mpx_tune_reload) and rewritten
// whole after every autotune; a missing or unreadable file is an empty cache.
//
// Environment:
//   MPX_TUNE_CACHE=<path>      use this cache file (unset: in-process only);
//   MPX_TUNE=off               ignore tuned choices from the file and from
//                              this process (the size heuristic / plan default);
//   MPX_GEMM_VARIANT=<names>   comma-separated tiling names; a GEMM of a
//                              precision whose tilings include one of them
//                              uses it, whatever was tuned;
//   MPX_DK_VARIANT=<index>     every root-solver plan starts on this variant.
#include "mpx_internal.hpp"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <iterator>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

namespace mpx {

namespace {

struct TuneCache {
    std::mutex mu;
    bool loaded = false;
    std::string arch;                        // current device, e.g. "gfx950"
    std::map<std::string, std::string> own;  // "op key" -> choice, this arch
    std::vector<std::string> foreign;        // lines for other archs, kept as read
};

TuneCache& cache() {
    static TuneCache c;
    return c;
}

std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');  // drop feature suffixes (":sramecc+:xnack-")
    return colon == std::string::npos ? a : a.substr(0, colon);
}

const char* cache_path() {
    const char* p = std::getenv("MPX_TUNE_CACHE");
    return (p && *p) ? p : nullptr;
}

// Load under c.mu.
void load_locked(TuneCache& c) {
    c.loaded = true;
    c.arch = device_arch();
    c.own.clear();
    c.foreign.clear();
    const char* path = cache_path();
    if (!path) return;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        std::istringstream ss(line);
        std::vector<std::string> f;
        std::string w;
        while (ss >> w) f.push_back(w);
        if (f.size() < 3) continue;  // not an entry
        if (f[0] != c.arch) {
            c.foreign.push_back(line);
            continue;
        }
        std::string key = f[1];
        for (size_t i = 2; i + 1 < f.size(); ++i) key += " " + f[i];
        c.own[key] = f.back();
    }
}

void save_locked(const TuneCache& c) {
    const char* path = cache_path();
    if (!path) return;
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream out(tmp, std::ios::trunc);
        if (!out) return;
        for (const std::string& l : c.foreign) out << l << "\n";
        for (const auto& kv : c.own) out << c.arch << " " << kv.first << " " << kv.second << "\n";
        if (!out) return;
    }
    std::rename(tmp.c_str(), path);
}

}  // namespace

bool tune_disabled() {
    const char* t = std::getenv("MPX_TUNE");
    return t && std::strcmp(t, "off") == 0;
}

bool tune_lookup(const std::string& op_key, std::string& choice) {
    if (tune_disabled()) return false;
    TuneCache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    if (!c.loaded) load_locked(c);
    auto it = c.own.find(op_key);
    if (it == c.own.end()) return false;
    choice = it->second;
    return true;
}

void tune_forget(const std::string& op) {
    TuneCache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    if (!c.loaded) load_locked(c);
    for (auto it = c.own.begin(); it != c.own.end();)
        it = it->first.compare(0, op.size() + 1, op + " ") == 0 ? c.own.erase(it) : std::next(it);
}

void tune_store(const std::string& op_key, const std::string& choice) {
    TuneCache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    if (!c.loaded) load_locked(c);
    c.own[op_key] = choice;
    save_locked(c);
}

}  // namespace mpx

// Re-read the environment's cache file (forgetting this process's entries
// that the file does not hold).
extern "C" int mpx_tune_reload(void) {
    mpx::TuneCache& c = mpx::cache();
    std::lock_guard<std::mutex> lk(c.mu);
    mpx::load_locked(c);
    return MPX_OK;
}
