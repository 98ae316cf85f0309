// tune_check.cpp — drives the autotuner's JSON cache (csrc/hexsv_tune.cpp) under
// the address and undefined-behaviour sanitizers on the CPU: stores, reads back,
// overwrites and reads malformed or truncated cache files.  Test infrastructure,
// compiled and run by tests/test_sanitizers.py (host code only; no GPU call).
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <string>

#include "hexsv_host.h"

int hexsv_fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vfprintf(stderr, fmt, ap);
    va_end(ap);
    fprintf(stderr, "\n");
    return code;
}

static int failures = 0;
#define CHECK(c, msg)                                 \
    do {                                              \
        if (!(c)) {                                   \
            fprintf(stderr, "FAIL: %s\n", msg);       \
            ++failures;                               \
        }                                             \
    } while (0)

int main(int argc, char **argv) {
    if (argc < 2) return 2;
    const std::string path = std::string(argv[1]) + "/tune.json";
    setenv("HEXSV_TUNE_CACHE", path.c_str(), 1);
    const double all[3] = {0.2, 0.1, 0.3};
    CHECK(tuned_tile("k_step", HEXSV_FP32, 1 << 20, 7) == 7, "missing file gives the fallback");
    CHECK(tune_cache_store(path.c_str(), "k_step", HEXSV_FP32, 1 << 20, 1, 0.1, all, 3) == 0,
          "store");
    CHECK(tune_cache_store(path.c_str(), "k_step", HEXSV_FP64, 1 << 24, 4, 0.2, all, 3) == 0,
          "second key");
    CHECK(tune_cache_store(path.c_str(), "k_step", HEXSV_FP32, 1 << 20, 2, 0.05, all, 3) == 0,
          "overwrite");
    CHECK(tuned_tile("k_step", HEXSV_FP32, 1 << 20, 7) == 2, "read back the overwritten key");
    CHECK(tuned_tile("k_step", HEXSV_FP64, 1 << 24, 7) == 4, "read back the second key");
    CHECK(tuned_tile("k_ens_step", HEXSV_FP32, 1 << 20, 7) == 7, "unknown kernel");
    // malformed and truncated files must give the fallback without reading past the text
    const char *bad[] = {"", "{", "{\"", "{\"gfx950/k_step/fp32/2^20\": {\"tile\": ",
                         "\"gfx950/k_step/fp32/2^20\"", "{\"a\": {\"tile\": -3}}",
                         "{\"gfx950/k_step/fp32/2^20\": {\"tile\": -3}}", "}}}}{{{{\"\"\""};
    for (const char *t : bad) {
        FILE *f = fopen(path.c_str(), "w");
        if (!f) return 2;
        fputs(t, f);
        fclose(f);
        const int v = tuned_tile("k_step", HEXSV_FP32, 1 << 20, 7);
        CHECK(v == 7, t);
    }
    printf("%s\n", failures ? "FAILED" : "OK");
    return failures ? 1 : 0;
}
