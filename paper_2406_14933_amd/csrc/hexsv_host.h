// hexsv_host.h — host-side helpers shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "hexsv.h"
#include "hexsv_device.h"
#include "hexsv_nn.h"

// Record a thread-local message (read by hexsv_last_error) and return code.
int hexsv_fail(int code, const char *fmt, ...);
#define fail hexsv_fail

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(HEXSV_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));         \
    } while (0)

// The raster handle (shared by the single-domain and ensemble APIs).
struct hexsv_grid {
    hexsv::KGrid kg;
    double edge;
    int64_t n, n_active, n_dirichlet;  // n_dirichlet: boundary cells (Dirichlet or given flux)
    uint8_t *d_active;  // per cell 0 / 1 / 2 / 3 (outside, updated, Dirichlet, given flux);
                        // nullptr when all are 1
};

// Geometry constants of a raster of edge a (regular hexagon area, CFL bound).
inline void hexsv_geometry(double a, double cfl, double *sigma, double *cfl_phi) {
    const double S3H = 0.86602540378443864676;
    *sigma = 6.0 * (0.5 * a * (S3H * a));
    *cfl_phi = cfl * (*sigma / (6.0 * a));
}

// ---------------------------------------------------------- tuning cache
// A small JSON object keyed by "gfx950/<kernel>/<precision>/<size bucket>"
// (size bucket = round(log2(cells))) whose values are {"tile": v, "us": t,
// "all_us": [...]}.  The cache path comes from the caller or from the
// HEXSV_TUNE_CACHE environment variable.
int tune_cache_store(const char *path, const char *kernel, int prec, int64_t cells, int tile,
                     double ms, const double *all_ms, int nvar);
// Tile recorded for this key in $HEXSV_TUNE_CACHE, else `fallback`.
int tuned_tile(const char *kernel, int prec, int64_t cells, int fallback);

// ------------------------------------------------ surrogate for the solver
// Workspace of the surrogate for one nq x nr sample: the packed bf16 input
// (nn::FEATURES channels per cell) and the FP32 output (nn::OUT_STRIDE per
// cell); gen changes whenever those buffers move (graphs that captured them
// must be rebuilt).
int sur_window_bind(hexsv_surrogate *s, int nq, int nr, void **x0, const float **out,
                    uint64_t *gen);
// Network forward over the bound input into the bound output (stream-ordered),
// taps following the grid's neighbour rule (periodic sides, domain mask); the
// layers do nothing when *live (device, nullable) is 0.
int sur_forward_x0(hexsv_surrogate *s, const hexsv_grid *grid, hipStream_t st,
                   const int32_t *live);
// The layers before the last one, as sur_forward_x0 runs them; *last receives
// the last layer's input (32 channels per cell), forward weights and bias, for a
// kernel that applies the last layer itself.  EUNSUPPORTED when the forward runs
// fused (hexsv_surrogate_set_fused): the caller then uses sur_forward_x0.
struct SurLast {
    const __bf16 *x;
    const __bf16 *wm;
    const float *bias;
    hexsv::nn::ConvMask cm;
};
int sur_forward_hidden(hexsv_surrogate *s, const hexsv_grid *grid, hipStream_t st,
                       const int32_t *live, SurLast *last);
