// re_tune.cpp -- the autotuner.  For a workload (keyed by its size
// classes), it times short runs on throwaway contexts of the same workload:
// first every batched engine (lockstep or persistent) with every force
// lanes-per-atom count (and, for the lockstep engine, two block sizes), the
// same for every replica; then, when the replicas fall into more than one
// replica size class (floor(log2 N)), a pass over the classes, largest
// first, that tries every other lanes-per-atom count for that class alone
// and keeps it when the whole workload runs faster.  Choices are kept
// in-process and, when a cache path is given, in a small JSON file.
#include "re_tune.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

namespace re {

static std::mutex g_mu;
static std::map<std::string, TuneChoice> g_mem;

// Size class: device, precision, exchange mode, thermostat, replica count, the median
// and the spread of the atom counts (log2 bins), the mean density (0.05
// bins), r_c and the list radius.
std::string tune_key(int R, const int32_t* N, const double* rho_r, double rho, double rc, double skin, int prec,
                     int xmode, int thermo)
{
    std::vector<int32_t> n(N, N + R);
    std::sort(n.begin(), n.end());
    const int med = n[R / 2];
    double rs = 0;
    for (int r = 0; r < R; ++r) rs += rho_r ? rho_r[r] : rho;
    rs /= R;
    char arch[64] = "gpu";
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        std::snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
        for (char* p = arch; *p; ++p)
            if (*p == ':') *p = '+';
    }
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s|p%d|x%d|t%d|R%d|N%d|S%d|rho%.2f|rc%.3f|rl%.3f", arch, prec, xmode, thermo, R,
                  (int)std::lround(std::log2((double)med) * 2.0),
                  (int)std::lround(std::log2((double)n[R - 1] / (double)n[0])), std::round(rs * 20.0) / 20.0, rc,
                  rc + skin);
    return buf;
}

int tune_class(int32_t N)
{
    int k = 0;
    while (k + 1 < kTuneClasses && ((int64_t)2 << k) <= (int64_t)N) ++k;
    return k;
}

static std::string classes_str(const TuneChoice& c)
{
    std::string out;
    for (int k = 0; k < kTuneClasses; ++k)
        if (c.cls_tpa[k]) {
            if (!out.empty()) out += ",";
            out += std::to_string(k) + ":" + std::to_string(c.cls_tpa[k]);
        }
    return out;
}

static void parse_classes(const std::string& s, TuneChoice& c)
{
    size_t p = 0;
    while (p < s.size()) {
        int k = 0, t = 0;
        if (std::sscanf(s.c_str() + p, "%d:%d", &k, &t) == 2 && k >= 0 && k < kTuneClasses) c.cls_tpa[k] = t;
        const size_t q = s.find(',', p);
        if (q == std::string::npos) break;
        p = q + 1;
    }
}

// The cache file: {"<key>": {"engine": E, "tpa": T, "block": B, "ms_per_step": M,
// "classes": "k:t,..."}, ...}
static std::map<std::string, TuneChoice> read_cache(const char* path)
{
    std::map<std::string, TuneChoice> out;
    std::ifstream f(path);
    if (!f) return out;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t p = 0;
    for (;;) {
        const size_t k0 = s.find('"', p);
        if (k0 == std::string::npos) break;
        const size_t k1 = s.find('"', k0 + 1);
        if (k1 == std::string::npos) break;
        const std::string key = s.substr(k0 + 1, k1 - k0 - 1);
        const size_t b0 = s.find('{', k1), b1 = s.find('}', k1);
        if (b0 == std::string::npos || b1 == std::string::npos || b0 > b1) break;
        const std::string body = s.substr(b0, b1 - b0);
        TuneChoice c{};
        int ok = 0;
        size_t q;
        if ((q = body.find("\"engine\"")) != std::string::npos) ok += std::sscanf(body.c_str() + body.find(':', q) + 1, "%d", &c.engine);
        if ((q = body.find("\"tpa\"")) != std::string::npos) ok += std::sscanf(body.c_str() + body.find(':', q) + 1, "%d", &c.tpa);
        if ((q = body.find("\"ms_per_step\"")) != std::string::npos)
            ok += std::sscanf(body.c_str() + body.find(':', q) + 1, "%lf", &c.ms);
        if ((q = body.find("\"block\"")) != std::string::npos)
            std::sscanf(body.c_str() + body.find(':', q) + 1, "%d", &c.block);
        if ((q = body.find("\"classes\"")) != std::string::npos) {
            const size_t a = body.find('"', body.find(':', q) + 1), e = body.find('"', a + 1);
            if (a != std::string::npos && e != std::string::npos) parse_classes(body.substr(a + 1, e - a - 1), c);
        }
        if (ok == 3) out[key] = c;
        p = b1 + 1;
    }
    return out;
}

static void write_cache(const char* path, const std::map<std::string, TuneChoice>& m)
{
    const std::string tmp = std::string(path) + ".tmp";
    std::ofstream f(tmp);
    if (!f) return;
    f << "{\n";
    size_t i = 0;
    for (const auto& kv : m) {
        f << "  \"" << kv.first << "\": {\"engine\": " << kv.second.engine << ", \"tpa\": " << kv.second.tpa
          << ", \"block\": " << kv.second.block << ", \"ms_per_step\": " << kv.second.ms << ", \"classes\": \""
          << classes_str(kv.second) << "\"}" << (++i < m.size() ? "," : "") << "\n";
    }
    f << "}\n";
    f.close();
    std::rename(tmp.c_str(), path);
}

bool tune_lookup(const char* path, const std::string& key, TuneChoice& out)
{
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_mem.find(key);
    if (it != g_mem.end()) {
        out = it->second;
        return true;
    }
    if (path) {
        auto m = read_cache(path);
        auto jt = m.find(key);
        if (jt != m.end()) {
            g_mem[key] = jt->second;
            out = jt->second;
            return true;
        }
    }
    return false;
}

void tune_store(const char* path, const std::string& key, const TuneChoice& c)
{
    std::lock_guard<std::mutex> g(g_mu);
    g_mem[key] = c;
    if (path) {
        auto m = read_cache(path);
        m[key] = c;
        write_cache(path, m);
    }
}

// Milliseconds per step of one candidate on a throwaway context of the
// workload (1e300 when it cannot run): about 0.1 s of warm-up past the
// melting of the start lattice, whose list updates come at another rate,
// then about half a second timed.
static double time_candidate(int R, const int32_t* N, const double* T, double rho, double rc, double skin, double dt,
                             int Nx, uint64_t seed, const re_options& o, int* err)
{
    re_ctx* c = nullptr;
    const int rc0 = re_create(&c, R, N, T, rho, rc, skin, dt, Nx, seed, &o);
    if (rc0 != RE_OK) {
        *err = rc0;
        return 1e300;
    }
    using clk = std::chrono::steady_clock;
    std::vector<double> Uq(R);  // a query synchronises the context's stream
    double ms = 1e300;
    bool ok = re_step(c, 4) == RE_OK;
    auto t0 = clk::now();
    ok = ok && re_step(c, 4) == RE_OK && re_query_energies(c, Uq.data()) == RE_OK;
    const double est = std::max(std::chrono::duration<double, std::milli>(clk::now() - t0).count() / 4.0, 1e-3);
    if (ok) {
        const int warm = std::max(20, std::min(1000, (int)(100.0 / est)));
        ok = re_step(c, warm) == RE_OK && re_query_energies(c, Uq.data()) == RE_OK;
    }
    if (ok) {
        const int k = std::max(8, std::min(4000, (int)(500.0 / est)));
        t0 = clk::now();
        ok = re_step(c, k) == RE_OK && re_query_energies(c, Uq.data()) == RE_OK;
        ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count() / k;
    }
    re_destroy(c);
    return ok ? ms : 1e300;
}

int tune_run(int R, const int32_t* N, const double* T, double rho, double rc, double skin, double dt, int Nx,
             uint64_t seed, const re_options& base, TuneChoice& best)
{
    std::vector<int> engines;
    if (base.exchange_mode == RE_ASYNC)
        engines = {RE_PERSISTENT};
    else
        engines = {RE_LOCKSTEP, RE_PERSISTENT};
    best = TuneChoice{};
    int last_err = RE_OK;
    re_options o = base;
    o.autotune = 0;
    o.tune_cache = nullptr;
    o.log_capacity = 1 << 12;
    o.threads_per_atom_per_replica = nullptr;
    // (1) one lanes-per-atom count for every replica
    for (int eng : engines)
        for (int blk : (eng == RE_LOCKSTEP ? std::vector<int>{128, 256} : std::vector<int>{0}))
            for (int tpa : {1, 2, 4, 8}) {
                o.batched_engine = eng;
                o.threads_per_atom = tpa;
                o.block_size = blk;
                const double ms = time_candidate(R, N, T, rho, rc, skin, dt, Nx, seed, o, &last_err);
                if (ms < best.ms) {
                    best = TuneChoice{};
                    best.engine = eng;
                    best.tpa = tpa;
                    best.block = blk;
                    best.ms = ms;
                }
            }
    if (best.engine < 0) return last_err ? last_err : RE_EDEVICE;
    // (2) per size class, largest class (by atoms) first: another count for
    // that class alone, kept when the workload runs at least 2 % faster
    std::vector<int64_t> atoms(kTuneClasses, 0);
    for (int r = 0; r < R; ++r) atoms[tune_class(N[r])] += N[r];
    std::vector<int> cls;
    for (int k = 0; k < kTuneClasses; ++k)
        if (atoms[k] > 0) cls.push_back(k);
    if (cls.size() < 2) return RE_OK;
    std::stable_sort(cls.begin(), cls.end(), [&](int a, int b) { return atoms[a] > atoms[b]; });
    o.batched_engine = best.engine;
    o.block_size = best.block;
    o.threads_per_atom = best.tpa;
    std::vector<int32_t> per(R);
    for (int k : cls) {
        int keep = 0;
        for (int tpa : {1, 2, 4, 8}) {
            const int cur = best.cls_tpa[k] ? best.cls_tpa[k] : best.tpa;
            if (tpa == cur) continue;
            for (int r = 0; r < R; ++r) {
                const int kr = tune_class(N[r]);
                per[r] = kr == k ? tpa : (best.cls_tpa[kr] ? best.cls_tpa[kr] : best.tpa);
            }
            o.threads_per_atom_per_replica = per.data();
            const double ms = time_candidate(R, N, T, rho, rc, skin, dt, Nx, seed, o, &last_err);
            if (ms < 0.98 * best.ms) {
                best.ms = ms;
                keep = tpa;
            }
        }
        if (keep) best.cls_tpa[k] = keep;
    }
    return RE_OK;
}

}  // namespace re
