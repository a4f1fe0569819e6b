// Autotuner of launch shapes (host side): times the candidate shapes of a kernel on the
// problem it will run, once per key (kernel, d, m, method, precision, size class), and
// keeps the fastest in a process-wide cache.  With HW_TUNE_CACHE=<file> the cache is read
// from and appended to that text file (one "kernel d m method fp64 size choice us" line
// per key), so later processes reuse the choices; HW_AUTOTUNE=0 turns the timing off
// (every kernel then takes its default shape); HW_TUNE_FORCE="kernel=choice,..." imposes
// a choice for the named kernels (tests use it to run every variant); HW_TUNE_LOG=1 prints
// every candidate's time to stderr as it is measured.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "hw_kernels.h"

namespace {

using Key = std::tuple<std::string, int, int, int, int, int>;
struct Entry {
    int choice;
    double us;
};

std::mutex g_mu;
std::map<Key, Entry> g_cache;
bool g_loaded = false;

const char* cache_file()
{
    const char* f = std::getenv("HW_TUNE_CACHE");
    return (f && *f) ? f : nullptr;
}

void load_locked()
{
    if (g_loaded) return;
    g_loaded = true;
    const char* f = cache_file();
    if (!f) return;
    FILE* fp = std::fopen(f, "r");
    if (!fp) return;
    char name[64];
    int d, m, meth, fp64, size, choice;
    double us;
    while (std::fscanf(fp, "%63s %d %d %d %d %d %d %lf", name, &d, &m, &meth, &fp64, &size, &choice, &us) == 8)
        g_cache[Key(name, d, m, meth, fp64, size)] = Entry{choice, us};
    std::fclose(fp);
}

// the choice HW_TUNE_FORCE imposes on `kernel`, if any
bool forced_choice(const char* kernel, int& choice)
{
    const char* f = std::getenv("HW_TUNE_FORCE");
    if (!f) return false;
    const std::string spec(f), name(kernel);
    size_t pos = 0;
    while (pos < spec.size()) {
        size_t end = spec.find(',', pos);
        if (end == std::string::npos) end = spec.size();
        const std::string item = spec.substr(pos, end - pos);
        const size_t eq = item.find('=');
        if (eq != std::string::npos && item.substr(0, eq) == name) {
            char* rest = nullptr;
            const long v = std::strtol(item.c_str() + eq + 1, &rest, 10);
            if (rest && *rest == '\0' && rest != item.c_str() + eq + 1) {
                choice = (int)v;
                return true;
            }
        }
        pos = end + 1;
    }
    return false;
}

} // namespace

bool hw_tune_forced(const char* kernel, int& choice) { return forced_choice(kernel, choice); }

bool hw_tune_enabled()
{
    const char* e = std::getenv("HW_AUTOTUNE");
    return !(e && std::strcmp(e, "0") == 0);
}

int hw_tune_size_class(int64_t cells)
{
    // coarse classes of the work per launch: < 2^14, < 2^17, < 2^20, larger
    if (cells < (1 << 14)) return 0;
    if (cells < (1 << 17)) return 1;
    if (cells < (1 << 20)) return 2;
    return 3;
}

int hw_tune_choose(const char* kernel, int d, int m, int method, bool fp64, int size_class,
                   const std::vector<int>& candidates, const std::function<double(int)>& time_us)
{
    const Key key(kernel, d, m, method, fp64 ? 1 : 0, size_class);
    int forced = 0;
    if (forced_choice(kernel, forced)) return forced;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        load_locked();
        auto it = g_cache.find(key);
        if (it != g_cache.end()) return it->second.choice;
    }
    int best = candidates.empty() ? 0 : candidates[0];
    double best_us = 1e300;
    const char* lg = std::getenv("HW_TUNE_LOG");
    const bool log = lg && std::strcmp(lg, "0") != 0;
    for (int c : candidates) {
        const double t = time_us(c);
        if (log)
            std::fprintf(stderr, "[tune] %s d=%d m=%d method=%d fp64=%d size=%d choice %d: %.3f us\n", kernel, d, m,
                         method, fp64 ? 1 : 0, size_class, c, t);
        if (t > 0.0 && t < best_us) {
            best_us = t;
            best = c;
        }
    }
    std::lock_guard<std::mutex> lock(g_mu);
    g_cache[key] = Entry{best, best_us};
    if (const char* f = cache_file()) {
        if (FILE* fp = std::fopen(f, "a")) {
            std::fprintf(fp, "%s %d %d %d %d %d %d %.3f\n", kernel, d, m, method, fp64 ? 1 : 0, size_class, best,
                         best_us);
            std::fclose(fp);
        }
    }
    return best;
}

std::string hw_tune_report_text()
{
    std::lock_guard<std::mutex> lock(g_mu);
    std::string out;
    char line[160];
    for (const auto& kv : g_cache) {
        std::snprintf(line, sizeof line, "%s d=%d m=%d method=%d fp64=%d size_class=%d -> %d (%.1f us)\n",
                      std::get<0>(kv.first).c_str(), std::get<1>(kv.first), std::get<2>(kv.first),
                      std::get<3>(kv.first), std::get<4>(kv.first), std::get<5>(kv.first), kv.second.choice,
                      kv.second.us);
        out += line;
    }
    return out;
}
