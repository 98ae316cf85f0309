// hexsv_kernels.h — step, finalize and state-transfer kernels, templated on
// the state precision T.  Included by one translation unit per precision.
#pragma once

#include <math.h>

#include "hexsv_internal.h"
#include "hexsv_tile.h"

namespace hexsv {

// One explicit step of one tile (see tile_step).  Every workgroup first
// recomputes the step's dt from the control block; a step past t_end or
// past the step limit does nothing, so a captured graph of many steps can
// overrun the end of a run safely.
// One explicit step over the raster, one workgroup per tile (tiles mapped to
// XCD bands, see xcd_tile); every workgroup writes its tile's partial record
// and the single-workgroup finalize kernel launched right after folds the
// records into the control block, so the next step sees the new dt.
template <typename T, int TQ, int TR, int NT>
__global__ __launch_bounds__(NT) void k_step(KDom<T> d, KGrid g, KConst kc, KRain rn, Ctl *ctl,
                                             Part *part, int ntq, int ntiles) {
    const StepTime st = step_time(ctl);
    if (!st.live) return;
    __shared__ TileLDS<T, TQ, TR> L;
    const double r_next = rain_rate(rn, st.t_next);
    const int tile = xcd_tile(blockIdx.x, gridDim.x, ntiles, 0);
    const int tr = tile / ntq, tq = tile - tr * ntq;
    Acc acc{0.0, 0.0, 0.0, 0.0};
    tile_step<T, TQ, TR, NT, true>(L, d, g, kc, ctl->parity, tq, tr, st.dt, r_next, acc,
                                   &ctl->err, &ctl->err_cell);
    const Part p = block_reduce<NT>(acc.c, acc.s, acc.o, acc.cl);
    if (threadIdx.x == 0) part[tile] = p;
}

template <typename T, int TQ, int TR, int NT>
static hipError_t launch_step_v(const KDom<T> &d, const KGrid &g, const KConst &kc,
                                const KRain &rn, Ctl *ctl, Part *part, int ntq, int ntiles,
                                int nwg, bool finalize, hipStream_t stream) {
    hipLaunchKernelGGL((k_step<T, TQ, TR, NT>), dim3(nwg), dim3(NT), 0, stream, d, g, kc, rn, ctl,
                       part, ntq, ntiles);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !finalize) return e;
    return launch_finalize(ctl, part, nwg, kc, rn, stream);
}

template <typename T>
static hipError_t launch_step_any(int variant, const KDom<T> &d, const KGrid &g,
                                  const KConst &kc, const KRain &rn, Ctl *ctl, Part *part,
                                  int ntq, int ntiles, int nwg, bool finalize,
                                  hipStream_t stream) {
    switch (variant) {
#define HEXSV_CASE(V)                                                                          \
    case V:                                                                                    \
        return launch_step_v<T, TILES[V].tq, TILES[V].tr, TILES[V].nt>(                        \
            d, g, kc, rn, ctl, part, ntq, ntiles, nwg, finalize, stream);
        HEXSV_TILE_SWITCH(HEXSV_CASE)
#undef HEXSV_CASE
        default:
            return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_step(int variant, const KDom<T> &d, const KGrid &g, const KConst &kc,
                       const KRain &rn, Ctl *ctl, Part *part, int ntq, int ntiles, int nwg,
                       hipStream_t stream) {
    return launch_step_any<T>(variant, d, g, kc, rn, ctl, part, ntq, ntiles, nwg, true, stream);
}

template <typename T>
hipError_t launch_step_only(int variant, const KDom<T> &d, const KGrid &g, const KConst &kc,
                            const KRain &rn, Ctl *ctl, Part *part, int ntq, int ntiles, int nwg,
                            hipStream_t stream) {
    return launch_step_any<T>(variant, d, g, kc, rn, ctl, part, ntq, ntiles, nwg, false, stream);
}

// Initial c_max and stored volume of the current buffer.
template <typename T>
__global__ __launch_bounds__(256) void k_prime(KDom<T> d, int64_t n, KConst kc, Ctl *ctl,
                                               Part *part) {
    const int par = ctl->parity;
    const T *h = d.buf(par, 0), *v1 = d.buf(par, 1), *v2 = d.buf(par, 2);
    double c = 0.0, s = 0.0;
    const T G = (T)kc.g;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const T th = d.th[i];
        if (!(th > T(0))) continue;
        const T cc = p_sqrt(v1[i] * v1[i] + v2[i] * v2[i]) + p_sqrt(G * h[i]);
        c = (double)cc > c ? (double)cc : c;
        s += kc.sigma * ((double)th * (double)h[i]);
    }
    const Part p = block_reduce<256>(c, s, 0.0, 0.0);
    if (threadIdx.x == 0) part[blockIdx.x] = p;
}

template <typename T>
hipError_t launch_prime(const KDom<T> &d, int64_t n, const KConst &kc, Ctl *ctl, Part *part,
                        int nblocks, int reset_books, hipStream_t stream) {
    hipLaunchKernelGGL((k_prime<T>), dim3(nblocks), dim3(256), 0, stream, d, n, kc, ctl, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_prime_finalize(ctl, part, nblocks, kc, reset_books, stream);
}

template <typename T>
__global__ void k_import(const double *src, T *dst, const uint8_t *active, int zero_inactive,
                         int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const bool act = active ? active[i] != 0 : true;
        dst[i] = (zero_inactive && !act) ? T(0) : (T)src[i];
    }
}

template <typename T>
hipError_t launch_import(const double *src, T *dst, const uint8_t *active, int zero_inactive,
                         int64_t n, hipStream_t stream) {
    const int nb = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    hipLaunchKernelGGL((k_import<T>), dim3(nb > 0 ? nb : 1), dim3(256), 0, stream, src, dst,
                       active, zero_inactive, n);
    return hipGetLastError();
}

template <typename T>
__global__ void k_export(KDom<T> d, int par, int64_t n, double *h, double *v1, double *v2,
                         double *q1, double *q2) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double hh = (double)d.buf(par, 0)[i];
        const double a = (double)d.buf(par, 1)[i];
        const double b = (double)d.buf(par, 2)[i];
        const double th = (double)d.th[i];
        if (h) h[i] = hh;
        if (v1) v1[i] = a;
        if (v2) v2[i] = b;
        if (q1) q1[i] = th * hh * a;
        if (q2) q2[i] = th * hh * b;
    }
}

template <typename T>
hipError_t launch_export(const KDom<T> &d, int par, int64_t n, double *h, double *v1,
                         double *v2, double *q1, double *q2, hipStream_t stream) {
    const int nb = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    hipLaunchKernelGGL((k_export<T>), dim3(nb > 0 ? nb : 1), dim3(256), 0, stream, d, par, n,
                       h, v1, v2, q1, q2);
    return hipGetLastError();
}

#define HEXSV_INSTANTIATE(T)                                                                  \
    template hipError_t launch_step<T>(int, const KDom<T> &, const KGrid &, const KConst &,   \
                                       const KRain &, Ctl *, Part *, int, int, int,           \
                                       hipStream_t);                                          \
    template hipError_t launch_step_only<T>(int, const KDom<T> &, const KGrid &, const KConst &, \
                                            const KRain &, Ctl *, Part *, int, int, int,      \
                                            hipStream_t);                                     \
    template hipError_t launch_prime<T>(const KDom<T> &, int64_t, const KConst &, Ctl *, Part *, \
                                        int, int, hipStream_t);                               \
    template hipError_t launch_import<T>(const double *, T *, const uint8_t *, int, int64_t,  \
                                         hipStream_t);                                        \
    template hipError_t launch_export<T>(const KDom<T> &, int, int64_t, double *, double *,   \
                                         double *, double *, double *, hipStream_t);

}  // namespace hexsv
