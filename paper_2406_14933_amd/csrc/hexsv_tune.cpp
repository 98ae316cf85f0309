// hexsv_tune.cpp — the autotuner's result cache (a flat JSON object).
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <fstream>
#include <map>
#include <sstream>
#include <string>

#include "hexsv_host.h"

static std::string tune_key(const char *kernel, int prec, int64_t cells) {
    const int bucket = cells > 0 ? (int)lround(log2((double)cells)) : 0;
    char buf[128];
    snprintf(buf, sizeof buf, "gfx950/%s/%s/2^%d", kernel, prec == HEXSV_FP64 ? "fp64" : "fp32", bucket);
    return buf;
}

// Parse {"key": {...}, ...} into key -> raw value text (values are objects
// without nested braces, as written below).
static std::map<std::string, std::string> read_cache(const char *path) {
    std::map<std::string, std::string> m;
    std::ifstream f(path);
    if (!f) return m;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string t = ss.str();
    size_t i = 0;
    while (true) {
        const size_t k0 = t.find('"', i);
        if (k0 == std::string::npos) break;
        const size_t k1 = t.find('"', k0 + 1);
        if (k1 == std::string::npos) break;
        const size_t b0 = t.find('{', k1);
        const size_t b1 = t.find('}', b0 == std::string::npos ? k1 : b0);
        if (b0 == std::string::npos || b1 == std::string::npos) break;
        m[t.substr(k0 + 1, k1 - k0 - 1)] = t.substr(b0, b1 - b0 + 1);
        i = b1 + 1;
    }
    return m;
}

int tune_cache_store(const char *path, const char *kernel, int prec, int64_t cells, int tile,
                     double ms, const double *all_ms, int nvar) {
    std::map<std::string, std::string> m = read_cache(path);
    std::ostringstream v;
    v.precision(6);
    v << "{\"tile\": " << tile << ", \"us\": " << ms * 1e3 << ", \"all_us\": [";
    for (int i = 0; i < nvar; ++i) v << (i ? ", " : "") << all_ms[i] * 1e3;
    v << "]}";
    m[tune_key(kernel, prec, cells)] = v.str();
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return hexsv_fail(HEXSV_EINVAL, "autotune: cannot write %s", tmp.c_str());
        f << "{\n";
        size_t k = 0;
        for (auto &kv : m) f << "  \"" << kv.first << "\": " << kv.second << (++k < m.size() ? ",\n" : "\n");
        f << "}\n";
    }
    if (rename(tmp.c_str(), path) != 0) return hexsv_fail(HEXSV_EINVAL, "autotune: cannot replace %s", path);
    return HEXSV_OK;
}

int tuned_tile(const char *kernel, int prec, int64_t cells, int fallback) {
    const char *path = getenv("HEXSV_TUNE_CACHE");
    if (!path || !*path) return fallback;
    std::map<std::string, std::string> m = read_cache(path);
    auto it = m.find(tune_key(kernel, prec, cells));
    if (it == m.end()) return fallback;
    const size_t p = it->second.find("\"tile\":");
    if (p == std::string::npos) return fallback;
    const int v = atoi(it->second.c_str() + p + 7);
    return v >= 0 ? v : fallback;
}
