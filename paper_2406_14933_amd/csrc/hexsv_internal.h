// hexsv_internal.h — interface between the host library and the per-precision
// kernel translation units (FP64 built without contraction, FP32 with it).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hexsv_device.h"
#include "hexsv_nn.h"

namespace hexsv {

struct TileShape {
    int tq, tr, nt;
};

// Tile variants the step kernels are built for (the autotuner picks one).
constexpr TileShape TILES[] = {
    {64, 4, 256}, {64, 8, 256}, {64, 16, 256}, {128, 4, 256},
    {128, 8, 256}, {128, 8, 512}, {64, 32, 256}, {64, 8, 512},
};
constexpr int NUM_TILES = sizeof(TILES) / sizeof(TILES[0]);
#define HEXSV_TILE_SWITCH(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7)

// Tile variants of the persistent ensemble kernel (one 1024-thread workgroup
// sweeps a whole scenario).
constexpr TileShape ENS_TILES[] = {{64, 16, 1024}, {64, 32, 1024}, {128, 16, 1024}};
constexpr int NUM_ENS_TILES = sizeof(ENS_TILES) / sizeof(ENS_TILES[0]);

struct EnsScen;
struct EnsTile;
// Batched-step mode of the ensemble: the tile kernel over the tiles of all
// scenarios (one workgroup each) followed by the per-scenario finalize.
// Tile t loads the buffers of parity par_hint ^ tpar[t] first (tpar: the
// scenarios' parities relative to the launch hint).
template <typename T>
hipError_t launch_ens_step(int variant, bool visc, bool bc, const KDom<T> &base,
                           const EnsScen *scen, const EnsTile *tiles, const uint8_t *tpar,
                           Ctl *ctl, Part *part, int ntiles_total, int nscen, int par_hint,
                           hipStream_t stream);
hipError_t launch_ens_finalize(const EnsScen *scen, Ctl *ctl, const Part *part, int nscen,
                               hipStream_t stream);
// Reset the ensemble's scenario queue (a one-thread kernel, safe inside graphs).
hipError_t launch_queue_reset(uint32_t *queue, hipStream_t stream);
// One launch of the persistent ensemble kernel: nwg workgroups take the
// scenarios in `order` from the queue and advance each by up to ksteps steps.
template <typename T>
hipError_t launch_ensemble(int variant, const KDom<T> &base, const EnsScen *scen, Ctl *ctl,
                           const int32_t *order, int nscen, uint32_t *queue, int ksteps, int nwg,
                           hipStream_t stream);
constexpr int DEFAULT_TILE = 2;
// Step tile of a single domain when the tuning cache has no entry: in FP32, 128 x 8
// cells (256 threads) for rasters at least 2048 cells wide, whose long row
// segments it streams fastest; else the tallest of 64 x 16, 64 x 8 and 64 x 4
// (variants 2, 1, 0) that still makes 512 workgroups, two per CU (on smaller
// rasters a step is bound by latency, which more workgroups in flight hide),
// and 64 x 4 below that.
constexpr int WIDE_TILE = 4;
inline int default_step_tile(int nq, int nr, bool fp32) {
    if (fp32 && nq >= 2048) return WIDE_TILE;
    for (int v = DEFAULT_TILE; v > 0; --v) {
        const int64_t n = (int64_t)((nq + TILES[v].tq - 1) / TILES[v].tq) *
                          ((nr + TILES[v].tr - 1) / TILES[v].tr);
        if (n >= 512) return v;
    }
    return 0;
}

// Number of tiles covering an nq x nr raster with variant v.
inline void tile_grid(int v, int nq, int nr, int *ntq, int *ntiles) {
    const TileShape s = TILES[v];
    *ntq = (nq + s.tq - 1) / s.tq;
    *ntiles = *ntq * ((nr + s.tr - 1) / s.tr);
}

// One step launch (nwg == ntiles workgroups): closes the step of the
// previous launch and starts the next (see k_step, Ctl and KClose).  ctl
// points at the two control slots; `in` is the slot this launch reads and
// `set` its accumulator set (launch k after a fold: in = k % 2, set = k % 3).
// par_hint: the buffer parity the step is expected to read (its loads start
// before the control block is read; a wrong hint only costs a reload).
template <typename T>
hipError_t launch_step(int variant, const KDom<T> &d, const KGrid &g, const KConst &kc,
                       const KRain &rn, Ctl *ctl, const KClose &cl, int ntq, int ntiles, int nwg,
                       int par_hint, int in, int set, hipStream_t stream);

// After a run of `launches` step launches since the previous fold, the last of
// which read slot `in` with accumulator set `set`: close its pending step, add
// the books of every closed step in the ring to ctl[0] in step order, empty the
// ring and clear the accumulators (one workgroup per ring slot the run can have
// filled, at most `launches`: the first launch after a fold has nothing to close,
// then one wave).
hipError_t launch_fold(Ctl *ctl, const KClose &cl, int ntiles, const KConst &kc, const KRain &rn,
                       int in, int set, int launches, hipStream_t stream);
// Close a priming pass over nparts partial records: tau (and, with
// reset_books, the initial books) of the current state.
hipError_t launch_prime_finalize(Ctl *ctl, const Part *part, int nparts, const KConst &kc,
                                 int reset_books, hipStream_t stream);
constexpr int PRIME_BLOCKS = 1024;

template <typename T>
hipError_t launch_prime(const KDom<T> &d, int64_t n, const KConst &kc, Ctl *ctl, Part *part,
                        int nblocks, int reset_books, hipStream_t stream);

// FP64 caller arrays -> internal precision (theta forced to 0 outside the mask).
// nq, pitch: the internal rows are `pitch` cells apart (0: the caller's layout).
template <typename T>
hipError_t launch_import(const double *src, T *dst, const uint8_t *active, int zero_inactive,
                         int64_t n, hipStream_t stream, int64_t nq = 0, int64_t pitch = 0);
// internal state -> FP64 caller arrays (each output nullable); nq, pitch as above.
template <typename T>
hipError_t launch_export(const KDom<T> &d, int par, int64_t n, double *h, double *v1,
                         double *v2, double *q1, double *q2, hipStream_t stream,
                         int64_t nq = 0, int64_t pitch = 0);

// Validation of caller inputs: counts offending active cells and records the
// lowest offending index in chk[0] (count) / chk[1] (index) / chk[2] (reason).
hipError_t launch_check_fields(const double *z, const double *th, const double *ap,
                               const uint8_t *active, int64_t n, int32_t *chk,
                               hipStream_t stream);
hipError_t launch_check_state(const double *h, const double *v1, const double *v2,
                              const uint8_t *active, int64_t n, double g, int32_t *chk,
                              hipStream_t stream);

// ------------------------------------------------------ surrogate windows
//
// A window advances the state by a fixed span with one network call; it is
// kept only if the predicted state keeps the water balance.  Everything of a
// window runs on the device (so windows chain inside a graph); the host only
// reads this record after a chain.
struct alignas(64) SurWin {
    double t_stop, window, tol;     // set by the host for a run
    double depth, R, t0, S0, rho;   // of the current window
    int32_t k;                      // rain sub-steps of a window
    int32_t live;                   // the current window runs
    int32_t alive;                  // every window of this chain so far was accepted
    int32_t rejected;               // a window of this chain was refused
    int32_t accepted;               // windows accepted in this chain
    int32_t project;                // 1: rescale an accepted state onto the balance
    int32_t scale_live;             // the current state waits for its rescaling by `scale`:
                                    // the windows of a chain read it scaled, and one
                                    // k_win_scale after the chain stores it
    int32_t perr, perr_cell;        // non-finite value met by a probe step
    double scale;                   // factor of that rescaling
    double c0;                      // reference c_max: of the last state the solver made
                                    // (run start, end of a refused span); < 0: take it
                                    // from the next window's start state
    int32_t why;                    // reason of the last refusal: 1 residual, 2 wave speed, 4 non-finite
    int32_t pad2;
};

constexpr int FEATURES = nn::FEATURES;
constexpr int WIN_PARTS = 1024;  // partial records of the window reductions

// Feature scales: H (depth), Q (discharge), Z (elevation), S (slope), and the
// window changes of depth and discharge dH, dQ.
struct FeatScale {
    float H, Q, Z, S, dH, dQ;
};

hipError_t launch_win_reset(SurWin *sw, hipStream_t stream);
// Gate of a window: part holds n_part records of the predicted state, op0 the
// probe's n_op0 records of the start state's outflow rate.
hipError_t launch_win_gate(Ctl *ctl, SurWin *sw, const Part *part, int n_part, const Part *op0,
                           int n_op0, const KConst &kc, hipStream_t stream);
// Window kernels on the current state (buffer ctl->parity), each a no-op unless sw->live
// (which the probe, the first of them, decides).
// scr holds 3 x cells values of T (the probe step's h, v1, v2).  The probe also
// writes the network's features of the current state into fout (feat 1: packed
// bf16; 2: FP32; 0: none) and one record per probe tile of the current state's
// outflow rate into op0[].stored (win_probe_tiles of them).
template <typename T>
hipError_t launch_win_probe(const KDom<T> &d, const KGrid &g, const KConst &kc, const KRain &rn,
                            const Ctl *ctl, SurWin *sw, T *scr, double dt_max,
                            const float2 *slope, FeatScale fs, int feat, void *fout, Part *op0,
                            hipStream_t stream);
// Tile of a window's probe launch: 64 x 4 cells, one per thread, so that the
// features the probe writes are spread over four times the workgroups of the
// step's default tile (a 512 x 512 raster: 1024).
constexpr int PROBE_TILE = 0;
// Workgroups (tiles) of a window's probe launch on an nq x nr raster.
inline int win_probe_tiles(int nq, int nr) {
    int ntq, ntiles;
    tile_grid(PROBE_TILE, nq, nr, &ntq, &ntiles);
    return ntiles;
}
// Terrain slope of every cell (float2), static for a simulation.
template <typename T>
hipError_t launch_win_slope(const KDom<T> &d, const KGrid &g, double a, float2 *slope,
                            hipStream_t stream);
// Predicted state into the other buffer, with its reductions (WIN_PARTS partials
// {c_max, stored, outflow rate, non-finite count}).
template <typename T>
hipError_t launch_win_apply(const KDom<T> &d, const KGrid &g, double l, const KConst &kc,
                            const Ctl *ctl, const SurWin *sw, const T *scr, double dt_max,
                            const float *out, int out_stride, float dH, float dQ, double m_min,
                            Part *part, hipStream_t stream);
// The network's last layer (input x: 32 channels per cell, weights wm, bias) with
// the predicted state as its epilogue, as launch_win_apply computes it from the
// stored network output; one record per conv tile (nn::conv_tiles of them) in part.
template <typename T>
hipError_t launch_win_last(const __bf16 *x, const __bf16 *wm, const float *bias,
                           const nn::ConvMask &cm, const KDom<T> &d, const KGrid &g, double l,
                           const KConst &kc, const Ctl *ctl, const SurWin *sw, const T *scr,
                           double dt_max, float dH, float dQ, double m_min, Part *part,
                           hipStream_t stream);
// Rescaling of the current state onto the water balance (no-op unless sw->scale_live),
// once after a chain of windows; the next chain's reset clears the flag.
template <typename T>
hipError_t launch_win_scale(const KDom<T> &d, int64_t n, const Ctl *ctl, const SurWin *sw,
                            hipStream_t stream);
// Neighbour and edge-code tables and the axial index arrays (each output nullable).
hipError_t launch_tables(const KGrid &g, const uint8_t *active, int32_t *nbr, uint8_t *code,
                         int32_t *q, int32_t *r, hipStream_t stream);

}  // namespace hexsv
