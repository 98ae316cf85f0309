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

// ------------------------------------------------------------ surrogate glue

// Surrogate input features of every cell (scales {H, Q, Z}):
// h/H, theta h v1/Q, theta h v2/Q, z/Z, theta, rain_depth/H (0 outside the domain).
template <typename S>
__global__ void k_features(int64_t n, const S *h, const S *v1, const S *v2, const S *z,
                           const S *th, double rain_depth, float H, float Q, float Z,
                           float *__restrict__ f) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float t = (float)th[i];
        const float hh = (float)h[i];
        const bool act = t > 0.f;
        f[i * 6 + 0] = act ? hh / H : 0.f;
        f[i * 6 + 1] = act ? t * hh * (float)v1[i] / Q : 0.f;
        f[i * 6 + 2] = act ? t * hh * (float)v2[i] / Q : 0.f;
        f[i * 6 + 3] = act ? (float)z[i] / Z : 0.f;
        f[i * 6 + 4] = t;
        f[i * 6 + 5] = act ? (float)(rain_depth / H) : 0.f;
    }
}

template <typename S>
hipError_t launch_features(int64_t n, const S *h, const S *v1, const S *v2, const S *z,
                           const S *th, double rain_depth, float H, float Q, float Z, float *f,
                           hipStream_t stream) {
    const int nb = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    hipLaunchKernelGGL((k_features<S>), dim3(nb > 0 ? nb : 1), dim3(256), 0, stream, n, h, v1, v2, z,
                       th, rain_depth, H, Q, Z, f);
    return hipGetLastError();
}

// Apply a predicted window change to state buffer `par` into buffer par^1:
// h' = max(h + dH*out0, 0), q' = theta h v + dQ*(out1, out2), v' = q' / (theta h')
// (0 where theta h' <= m_min).  Inactive cells are copied.
template <typename T>
__global__ void k_apply_surrogate(KDom<T> d, int par, int64_t n, const float *__restrict__ out,
                                  float dH, float dQ, double m_min) {
    const T *h = d.buf(par, 0), *v1 = d.buf(par, 1), *v2 = d.buf(par, 2);
    T *ho = d.buf(par ^ 1, 0), *v1o = d.buf(par ^ 1, 1), *v2o = d.buf(par ^ 1, 2);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const T th = d.th[i];
        if (!(th > T(0))) {
            ho[i] = h[i];
            v1o[i] = v1[i];
            v2o[i] = v2[i];
            continue;
        }
        const T m = th * h[i];
        T hn = h[i] + (T)dH * (T)out[i * 4 + 0];
        hn = hn > T(0) ? hn : T(0);
        const T q1 = m * v1[i] + (T)dQ * (T)out[i * 4 + 1];
        const T q2 = m * v2[i] + (T)dQ * (T)out[i * 4 + 2];
        const T mn = th * hn;
        ho[i] = hn;
        v1o[i] = mn > (T)m_min ? q1 / mn : T(0);
        v2o[i] = mn > (T)m_min ? q2 / mn : T(0);
    }
}

template <typename T>
hipError_t launch_apply_surrogate(const KDom<T> &d, int par, int64_t n, const float *out,
                                  float dH, float dQ, double m_min, hipStream_t stream) {
    const int nb = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    hipLaunchKernelGGL((k_apply_surrogate<T>), dim3(nb > 0 ? nb : 1), dim3(256), 0, stream, d, par,
                       n, out, dH, dQ, m_min);
    return hipGetLastError();
}

// Instantaneous volume flux through the OUTFLOW edges of state buffer `par`:
// with the free-outflow ghost (the cell's own h, v, theta) an edge carries
// l * theta h * (v . n_k) whatever its sign.  One FP64 partial per workgroup.
template <typename T>
__global__ __launch_bounds__(256) void k_outflow_rate(KDom<T> d, int par, KGrid g, double l,
                                                      double *__restrict__ part) {
    const T *h = d.buf(par, 0), *v1 = d.buf(par, 1), *v2 = d.buf(par, 2);
    const double S3 = 0.86602540378443864676;
    const double NX[6] = {1.0, 0.5, -0.5, -1.0, -0.5, 0.5};
    const double NY[6] = {0.0, S3, S3, 0.0, -S3, -S3};
    double acc = 0.0;
    const int64_t n = (int64_t)g.nq * g.nr;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        if (!(d.th[i] > T(0))) continue;
        const int r = (int)(i / g.nq), q = (int)(i - (int64_t)r * g.nq);
        for (int k = 0; k < 6; ++k) {
            int qn = q + dq_of(k), rn = r + dr_of(k);
            int cd;
            if (wrap_pos(g, qn, rn)) cd = d.th[(int64_t)rn * g.nq + qn] > T(0) ? CODE_INTERIOR : g.mask_bc;
            else cd = side_code(g, qn, rn);
            if (cd != CODE_OUTFLOW) continue;
            const double m = (double)d.th[i] * (double)h[i];
            acc += l * m * ((double)v1[i] * NX[k] + (double)v2[i] * NY[k]);
        }
    }
    const Part p = block_reduce<256>(0.0, acc, 0.0, 0.0);
    if (threadIdx.x == 0) part[blockIdx.x] = p.stored;
}

template <typename T>
hipError_t launch_outflow_rate(const KDom<T> &d, int par, const KGrid &g, double l, double *part,
                               int nparts, hipStream_t stream) {
    hipLaunchKernelGGL((k_outflow_rate<T>), dim3(nparts), dim3(256), 0, stream, d, par, g, l, part);
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
    template hipError_t launch_features<T>(int64_t, const T *, const T *, const T *, const T *, \
                                           const T *, double, float, float, float, float *,   \
                                           hipStream_t);                                      \
    template hipError_t launch_apply_surrogate<T>(const KDom<T> &, int, int64_t, const float *, \
                                                  float, float, double, hipStream_t);         \
    template hipError_t launch_outflow_rate<T>(const KDom<T> &, int, const KGrid &, double,   \
                                               double *, int, hipStream_t);                   \
    template hipError_t launch_import<T>(const double *, T *, const uint8_t *, int, int64_t,  \
                                         hipStream_t);                                        \
    template hipError_t launch_export<T>(const KDom<T> &, int, int64_t, double *, double *,   \
                                         double *, double *, double *, hipStream_t);

}  // namespace hexsv
