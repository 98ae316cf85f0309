// hexsv_ensemble.h — persistent kernel that advances a batch of independent
// catchments (uneven raster sizes, each with its own time step, rain and
// books) in one launch.
//
// One workgroup owns one scenario at a time and sweeps all of its tiles for
// every step, so all synchronisation of a step (tiles done before the next
// step reads them, reduction of c_max and of the FP64 books, the new dt) is
// inside one workgroup: a barrier with workgroup-scope fences.  Workgroups
// take scenarios from a queue ordered largest first and advance each by up to
// `ksteps` steps per launch.  Within a workgroup the loads of the next tile
// are issued before the arithmetic of the current tile (two register sets),
// so every CU keeps HBM requests in flight while it computes.
//
// Cross-workgroup coordination is avoided on purpose: on gfx950 each of the
// 8 XCDs has its own L2, and an agent-scope release per tile (needed for a
// step barrier shared by several workgroups) writes back the whole L2.
#pragma once

#include "hexsv_internal.h"
#include "hexsv_tile.h"

namespace hexsv {

// One scenario of the batch: where its cells live in the concatenated
// arrays and its raster, constants and rain.
struct EnsScen {
    int64_t off;
    KGrid g;
    KConst kc;
    KRain rn;
    int32_t ntq, ntiles;          // persistent mode tiling
    int32_t bntq, bntiles, bbase;  // batched-step mode tiling and first global tile
};

// One tile of the batched-step mode: everything its loads need (where the
// scenario's cells start, its raster size and periodic sides, the tile's
// position), so that a workgroup issues its tile loads before it reads the
// scenario's control block and constants.
struct alignas(16) EnsTile {
    int64_t off;
    int32_t nq, nr, pitch;
    int32_t tq, tr;
    int32_t s;
    int32_t wrap;  // bit 0: periodic in q, bit 1: periodic in r
};

// The domain of the scenario at `off`, with its buffers ordered so that
// parity 0 is the current state (a run-time parity index into a local copy of
// the struct would place it in scratch memory).
template <typename T>
__device__ inline KDom<T> dom_at(const KDom<T> &base, int64_t off, int par) {
    KDom<T> d;
    for (int f = 0; f < 3; ++f) {
        d.st[0][f] = (par ? base.st[1][f] : base.st[0][f]) + off;
        d.st[1][f] = (par ? base.st[0][f] : base.st[1][f]) + off;
    }
    d.z = base.z + off;
    d.th = base.th + off;
    d.ap = base.ap + off;
    return d;
}

template <typename T, int TQ, int TR, int NT>
__global__ __launch_bounds__(NT) void k_ensemble(KDom<T> base, const EnsScen *__restrict__ scen,
                                                 Ctl *__restrict__ ctl,
                                                 const int32_t *__restrict__ order, int nscen,
                                                 uint32_t *queue, int ksteps) {
    __shared__ TileLDS<T, TQ, TR> L;
    __shared__ Ctl sc;
    __shared__ int s_next;
    for (;;) {
        if (threadIdx.x == 0) s_next = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int qi = s_next;
        if (qi >= nscen) break;
        const int s = order[qi];
        // by reference: the segment tables are indexed dynamically, and a local
        // copy of them would live in scratch memory
        const KGrid &g = scen[s].g;
        const KConst &kc = scen[s].kc;
        const KRain &rn = scen[s].rn;
        const int ntq = scen[s].ntq, ntiles = scen[s].ntiles;
        const int64_t off = scen[s].off;
        if (threadIdx.x == 0) sc = ctl[s];
        __syncthreads();
        for (int step = 0; step < ksteps; ++step) {
            const StepTime st = step_time(&sc);
            if (!st.live) break;
            const double r_next = rain_rate(rn, st.t_next);
            const KDom<T> d = dom_at(base, off, sc.parity);
            const int par = 0;
            Acc acc{0.0, 0.0, 0.0, 0.0};
            TileRegs<T, TQ, TR, NT> R0, R1;
            tile_load<T, TQ, TR, NT>(R0, d, g, par, 0, 0);
            for (int t = 0; t < ntiles; t += 2) {
                {
                    const int tr = t / ntq, tq = t - tr * ntq;
                    const bool bad = tile_stage<T, TQ, TR, NT>(L, R0, g, kc, tq, tr);
                    const bool inner = tile_inner(g, tq * TQ, tr * TR, TQ, TR);
                    const bool general = __syncthreads_or((!inner) || bad) != 0;
                    if (t + 1 < ntiles) {
                        const int tr1 = (t + 1) / ntq, tq1 = (t + 1) - tr1 * ntq;
                        tile_load<T, TQ, TR, NT>(R1, d, g, par, tq1, tr1);
                    }
                    tile_compute<T, TQ, TR, NT, false>(L, R0, general, d, g, kc, par, tq, tr,
                                                       st.dt, r_next, acc, &ctl[s].err,
                                                       &ctl[s].err_cell);
                    __syncthreads();
                }
                if (t + 1 >= ntiles) break;
                {
                    const int tr = (t + 1) / ntq, tq = (t + 1) - tr * ntq;
                    const bool bad = tile_stage<T, TQ, TR, NT>(L, R1, g, kc, tq, tr);
                    const bool inner = tile_inner(g, tq * TQ, tr * TR, TQ, TR);
                    const bool general = __syncthreads_or((!inner) || bad) != 0;
                    if (t + 2 < ntiles) {
                        const int tr2 = (t + 2) / ntq, tq2 = (t + 2) - tr2 * ntq;
                        tile_load<T, TQ, TR, NT>(R0, d, g, par, tq2, tr2);
                    }
                    tile_compute<T, TQ, TR, NT, false>(L, R1, general, d, g, kc, par, tq, tr,
                                                       st.dt, r_next, acc, &ctl[s].err,
                                                       &ctl[s].err_cell);
                    __syncthreads();
                }
            }
            Part p = block_reduce<NT>(acc.c, acc.s, acc.o, acc.cl);
            if (p.cmax < kc.c_floor) p.cmax = kc.c_floor;  // the Dirichlet cells' wave speed
            if (threadIdx.x == 0) {
                close_step(&sc, p, st, kc, r_next);
                sc.err = ctl[s].err;
            }
            // the new state must be visible to every thread of the workgroup
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __syncthreads();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
        if (threadIdx.x == 0) {
            const int32_t err = ctl[s].err, cell = ctl[s].err_cell;
            ctl[s] = sc;
            ctl[s].err = err;
            ctl[s].err_cell = cell;
        }
        __syncthreads();
    }
}

// Batched-step mode: one launch advances every live scenario by one step.
// The tiles of all scenarios form one index space (one workgroup per tile,
// XCD-banded).  A workgroup reads its tile descriptor and issues the tile's
// loads from the buffers of the parity the launcher expects, par_hint XOR the
// tile's offset tpar[t] (live scenarios step together, so each keeps its
// parity relative to the others; the offsets record it for scenarios that
// stopped at different step counts), then reads the scenario's control block;
// a scenario of the other parity reloads (a cost, never a wrong result).  It writes one partial record; k_ens_finalize (one
// workgroup per scenario) then closes each scenario's step.  Kernel
// boundaries order the steps.
// V: the augmented momentum flux with artificial viscosity (set_viscosity);
// EXT: the extended scheme (some scenario holds Dirichlet or given-flux cells).
template <typename T, int TQ, int TR, int NT, bool V, bool EXT>
__global__ __launch_bounds__(NT) void k_ens_step(KDom<T> base, const EnsScen *__restrict__ scen,
                                                 const EnsTile *__restrict__ tiles,
                                                 const uint8_t *__restrict__ tpar,
                                                 Ctl *__restrict__ ctl, Part *__restrict__ part,
                                                 int ntiles_total, int par_hint) {
    const int t = xcd_tile(blockIdx.x, gridDim.x, ntiles_total, 0);
    if (t < 0) return;
    const EnsTile tl = tiles[t];
    const int hint = par_hint ^ (int)tpar[t];
    // what tile_load reads of the raster: its size and periodic sides
    KGrid gl;
    gl.nq = tl.nq;
    gl.nr = tl.nr;
    gl.pitch = tl.pitch;
    gl.perq = tl.wrap & 1;
    gl.perr = (tl.wrap >> 1) & 1;
    TileRegs<T, TQ, TR, NT> R;
    tile_load<T, TQ, TR, NT>(R, dom_at(base, tl.off, hint), gl, 0, tl.tq, tl.tr);
    const int s = tl.s;
    const StepTime st = step_time(&ctl[s]);
    if (!st.live) return;
    const int par = ctl[s].parity;
    const KDom<T> d = dom_at(base, tl.off, par);
    if (par != hint) tile_load<T, TQ, TR, NT>(R, d, gl, 0, tl.tq, tl.tr);
    const KGrid &g = scen[s].g;  // by reference (see k_ensemble)
    const KConst &kc = scen[s].kc;
    const double r_next = rain_rate(scen[s].rn, st.t_next);
    __shared__ TileLDS<T, TQ, TR, V> L;
    const bool bad = tile_stage<T, TQ, TR, NT, EXT>(L, R, g, kc, tl.tq, tl.tr);
    const bool inner = tile_inner(g, tl.tq * TQ, tl.tr * TR, TQ, TR);
    const bool general = __syncthreads_or((!inner) || bad) != 0;
    Acc acc{0.0, 0.0, 0.0, 0.0};
    tile_compute<T, TQ, TR, NT, true, V, EXT>(L, R, general, d, g, kc, 0, tl.tq, tl.tr, st.dt,
                                             r_next, acc, &ctl[s].err, &ctl[s].err_cell);
    const Part p = block_reduce<NT>(acc.c, acc.s, acc.o, acc.cl);
    if (threadIdx.x == 0) part[t] = p;
}

template <typename T, int TQ, int TR, int NT>
static hipError_t launch_ens_step_v(bool visc, bool bc, const KDom<T> &base,
                                    const EnsScen *scen, const EnsTile *tiles,
                                    const uint8_t *tpar, Ctl *ctl, Part *part, int ntiles_total,
                                    int nscen, int par_hint, hipStream_t stream) {
    if (visc)
        hipLaunchKernelGGL((k_ens_step<T, TQ, TR, NT, true, true>), dim3(ntiles_total), dim3(NT),
                           0, stream, base, scen, tiles, tpar, ctl, part, ntiles_total, par_hint);
    else if (bc)
        hipLaunchKernelGGL((k_ens_step<T, TQ, TR, NT, false, true>), dim3(ntiles_total), dim3(NT),
                           0, stream, base, scen, tiles, tpar, ctl, part, ntiles_total, par_hint);
    else
        hipLaunchKernelGGL((k_ens_step<T, TQ, TR, NT, false, false>), dim3(ntiles_total),
                           dim3(NT), 0, stream, base, scen, tiles, tpar, ctl, part, ntiles_total,
                           par_hint);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_ens_finalize(scen, ctl, part, nscen, stream);
}

template <typename T>
hipError_t launch_ens_step(int variant, bool visc, bool bc, const KDom<T> &base,
                           const EnsScen *scen, const EnsTile *tiles, const uint8_t *tpar,
                           Ctl *ctl, Part *part, int ntiles_total, int nscen, int par_hint,
                           hipStream_t stream) {
    switch (variant) {
#define HEXSV_CASE(V)                                                                          \
    case V:                                                                                    \
        return launch_ens_step_v<T, TILES[V].tq, TILES[V].tr, TILES[V].nt>(                    \
            visc, bc, base, scen, tiles, tpar, ctl, part, ntiles_total, nscen, par_hint, stream);
        HEXSV_TILE_SWITCH(HEXSV_CASE)
#undef HEXSV_CASE
        default:
            return hipErrorInvalidValue;
    }
}

template <typename T, int TQ, int TR, int NT>
static hipError_t launch_ensemble_v(const KDom<T> &base, const EnsScen *scen, Ctl *ctl,
                                    const int32_t *order, int nscen, uint32_t *queue, int ksteps,
                                    int nwg, hipStream_t stream) {
    hipError_t e = launch_queue_reset(queue, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_ensemble<T, TQ, TR, NT>), dim3(nwg), dim3(NT), 0, stream, base, scen, ctl,
                       order, nscen, queue, ksteps);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ensemble(int variant, const KDom<T> &base, const EnsScen *scen, Ctl *ctl,
                           const int32_t *order, int nscen, uint32_t *queue, int ksteps, int nwg,
                           hipStream_t stream) {
    switch (variant) {
#define HEXSV_CASE(V)                                                                        \
    case V:                                                                                  \
        return launch_ensemble_v<T, ENS_TILES[V].tq, ENS_TILES[V].tr, ENS_TILES[V].nt>(      \
            base, scen, ctl, order, nscen, queue, ksteps, nwg, stream);
        HEXSV_CASE(0)
        HEXSV_CASE(1)
        HEXSV_CASE(2)
#undef HEXSV_CASE
        default:
            return hipErrorInvalidValue;
    }
}

#define HEXSV_INSTANTIATE_ENSEMBLE(T)                                                         \
    template hipError_t launch_ensemble<T>(int, const KDom<T> &, const EnsScen *, Ctl *,      \
                                           const int32_t *, int, uint32_t *, int, int,        \
                                           hipStream_t);                                      \
    template hipError_t launch_ens_step<T>(int, bool, bool, const KDom<T> &, const EnsScen *, \
                                           const EnsTile *, const uint8_t *, Ctl *, Part *,   \
                                           int, int, int, hipStream_t);

}  // namespace hexsv
