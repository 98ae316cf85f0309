// hexsv_internal.h — interface between the host library and the per-precision
// kernel translation units (FP64 built without contraction, FP32 with it).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hexsv_device.h"

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
// Batched-step mode of the ensemble: the tile kernel over the tiles of all
// scenarios (one workgroup each) followed by the per-scenario finalize.
template <typename T>
hipError_t launch_ens_step(int variant, const KDom<T> &base, const EnsScen *scen,
                           const int32_t *tile_scen, Ctl *ctl, Part *part, int ntiles_total,
                           int nscen, hipStream_t stream);
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

// Number of tiles covering an nq x nr raster with variant v.
inline void tile_grid(int v, int nq, int nr, int *ntq, int *ntiles) {
    const TileShape s = TILES[v];
    *ntq = (nq + s.tq - 1) / s.tq;
    *ntiles = *ntq * ((nr + s.tr - 1) / s.tr);
}

// One step: the tile kernel (nwg == ntiles workgroups, one record per tile
// in part) followed by the single-workgroup finalize kernel.
template <typename T>
hipError_t launch_step(int variant, const KDom<T> &d, const KGrid &g, const KConst &kc,
                       const KRain &rn, Ctl *ctl, Part *part, int ntq, int ntiles, int nwg,
                       hipStream_t stream);


// The tile kernel alone (no finalize): used to time the kernel in isolation.
template <typename T>
hipError_t launch_step_only(int variant, const KDom<T> &d, const KGrid &g, const KConst &kc,
                            const KRain &rn, Ctl *ctl, Part *part, int ntq, int ntiles, int nwg,
                            hipStream_t stream);

// Close a step from the per-tile records (single workgroup).
hipError_t launch_finalize(Ctl *ctl, const Part *part, int ntiles, const KConst &kc,
                           const KRain &rn, hipStream_t stream);
// Close a priming pass over nparts partial records: tau (and, with
// reset_books, the initial books) of the current state.
hipError_t launch_prime_finalize(Ctl *ctl, const Part *part, int nparts, const KConst &kc,
                                 int reset_books, hipStream_t stream);
constexpr int PRIME_BLOCKS = 1024;

template <typename T>
hipError_t launch_prime(const KDom<T> &d, int64_t n, const KConst &kc, Ctl *ctl, Part *part,
                        int nblocks, int reset_books, hipStream_t stream);

// FP64 caller arrays -> internal precision (theta forced to 0 outside the mask).
template <typename T>
hipError_t launch_import(const double *src, T *dst, const uint8_t *active, int zero_inactive,
                         int64_t n, hipStream_t stream);
// internal state -> FP64 caller arrays (each output nullable).
template <typename T>
hipError_t launch_export(const KDom<T> &d, int par, int64_t n, double *h, double *v1,
                         double *v2, double *q1, double *q2, hipStream_t stream);

// Validation of caller inputs: counts offending active cells and records the
// lowest offending index in chk[0] (count) / chk[1] (index) / chk[2] (reason).
hipError_t launch_check_fields(const double *z, const double *th, const double *ap,
                               const uint8_t *active, int64_t n, int32_t *chk,
                               hipStream_t stream);
hipError_t launch_check_state(const double *h, const double *v1, const double *v2,
                              const uint8_t *active, int64_t n, int32_t *chk, hipStream_t stream);

// Surrogate glue (see hexsv_kernels.h).
template <typename S>
hipError_t launch_features(int64_t n, const S *h, const S *v1, const S *v2, const S *z,
                           const S *th, double rain_depth, float H, float Q, float Z, float *f,
                           hipStream_t stream);
template <typename T>
hipError_t launch_apply_surrogate(const KDom<T> &d, int par, int64_t n, const float *out,
                                  float dH, float dQ, double m_min, hipStream_t stream);
template <typename T>
hipError_t launch_outflow_rate(const KDom<T> &d, int par, const KGrid &g, double l, double *part,
                               int nparts, hipStream_t stream);

hipError_t launch_tables(const KGrid &g, const uint8_t *active, int32_t *nbr, uint8_t *code,
                         hipStream_t stream);

}  // namespace hexsv
