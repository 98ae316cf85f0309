// hexsv_kernels.h — step, priming and state-transfer kernels, templated on
// the state precision T.  Included by one translation unit per precision.
#pragma once

#include <math.h>

#include "hexsv_conv.h"
#include "hexsv_internal.h"
#include "hexsv_tile.h"

namespace hexsv {

// One explicit step over the raster, one workgroup per tile (tiles mapped to
// XCD bands, see xcd_tile).  Every workgroup first closes the step the
// previous launch started (from control slot `in` and the wave-speed maximum
// that launch accumulated, see open_step) and derives this step's dt from it;
// workgroup 0 also writes the control slot the next launch reads.  A step
// past t_end or past the step limit computes nothing, so a captured graph of
// many steps can overrun the end of a run safely.  Each tile adds its wave
// speed to the launch's accumulator set and its water books to the step ring.
//
// par_hint is the buffer parity the launcher expects this step to read (a
// graph of consecutive live steps alternates it).  The launcher passes the
// buffers of that parity as d.st[0], so the tile's loads use fixed argument
// offsets and are issued before the control block has arrived; the kernel
// works in parities relative to the hint.  A wrong hint (never for a live
// step of a graph replayed from the parity it was captured for) only costs a
// reload.
//
// VISC: the momentum flux is the augmented J^v with artificial viscosity
// (eqs. eq_artif_visc, eq_visc1), an instance of its own so that the plain
// scheme pays nothing for it.  EXT: the extended scheme (Dirichlet or given-flux
// cells, infiltration), likewise an instance of its own.
template <typename T, int TQ, int TR, int NT, bool VISC, bool EXT>
__global__ __launch_bounds__(NT) void k_step(KDom<T> d, KGrid g, KConst kc, KRain rn, Ctl *ctl,
                                             KClose cl, int ntq, int ntiles, int par_hint, int in,
                                             int set) {
    __shared__ TileLDS<T, TQ, TR, VISC> L;
    const int tile = xcd_tile(blockIdx.x, gridDim.x, ntiles, 0);
    const int tr = tile / ntq, tq = tile - tr * ntq;
    TileRegs<T, TQ, TR, NT> R;
    tile_load<T, TQ, TR, NT>(R, d, g, 0, tq, tr);
    const OpenStep o = open_step(ctl, in, cl.acc + ((set + 2) % ACC_SETS) * ACC_SET_WORDS, kc);
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) write_slot(ctl + (in ^ 1), ctl + in, o, kc, rn, true);
        unsigned long long *next = cl.acc + ((set + 1) % ACC_SETS) * ACC_SET_WORDS;
        if (threadIdx.x < ACC_SLOTS)
            __hip_atomic_store(next + threadIdx.x * ACC_STRIDE, 0ull, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!o.live) return;
    const int rel = o.parity ^ par_hint;  // buffer parity relative to d
    if (rel) tile_load<T, TQ, TR, NT>(R, d, g, 1, tq, tr);
    const double r_next = rain_rate(rn, o.t_next);
    const bool bad = tile_stage<T, TQ, TR, NT, EXT>(L, R, g, kc, tq, tr);
    const bool inner = tile_inner(g, tq * TQ, tr * TR, TQ, TR);
    const bool general = __syncthreads_or((!inner) || bad) != 0;
    Acc acc{0.0, 0.0, 0.0, 0.0};
    tile_compute<T, TQ, TR, NT, true, VISC, EXT>(L, R, general, d, g, kc, rel, tq, tr, o.dt, r_next,
                                                acc, &ctl->err, &ctl->err_cell);
    const Part p = block_reduce<NT>(acc.c, acc.s, acc.o, acc.cl);
    if (threadIdx.x == 0) {
        // the host folds the ring before it fills; the clamp only keeps a
        // broken invariant from writing out of bounds
        const int s = (unsigned)o.open < (unsigned)cl.ring_len ? o.open : cl.ring_len - 1;
        cl.ring[(size_t)s * ntiles + tile] = p;
        atomicMax(cl.acc + set * ACC_SET_WORDS + (tile % ACC_SLOTS) * ACC_STRIDE,
                  (unsigned long long)__double_as_longlong(p.cmax));
    }
}

template <typename T, int TQ, int TR, int NT>
static hipError_t launch_step_v(const KDom<T> &d, const KGrid &g, const KConst &kc,
                                const KRain &rn, Ctl *ctl, const KClose &cl, int ntq, int ntiles,
                                int nwg, int par_hint, int in, int set, hipStream_t stream) {
    KDom<T> dh = d;  // buffers of the hinted parity first
    if (par_hint & 1)
        for (int f = 0; f < 3; ++f) {
            dh.st[0][f] = d.st[1][f];
            dh.st[1][f] = d.st[0][f];
        }
    // instances: plain, extended, viscosity (which takes the extended scheme as well)
    if (kc.visc)
        hipLaunchKernelGGL((k_step<T, TQ, TR, NT, true, true>), dim3(nwg), dim3(NT), 0, stream,
                           dh, g, kc, rn, ctl, cl, ntq, ntiles, par_hint & 1, in, set);
    else if (kc.ext)
        hipLaunchKernelGGL((k_step<T, TQ, TR, NT, false, true>), dim3(nwg), dim3(NT), 0, stream,
                           dh, g, kc, rn, ctl, cl, ntq, ntiles, par_hint & 1, in, set);
    else
        hipLaunchKernelGGL((k_step<T, TQ, TR, NT, false, false>), dim3(nwg), dim3(NT), 0, stream,
                           dh, g, kc, rn, ctl, cl, ntq, ntiles, par_hint & 1, in, set);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_step_any(int variant, const KDom<T> &d, const KGrid &g,
                                  const KConst &kc, const KRain &rn, Ctl *ctl, const KClose &cl,
                                  int ntq, int ntiles, int nwg, int par_hint, int in, int set,
                                  hipStream_t stream) {
    switch (variant) {
#define HEXSV_CASE(V)                                                                          \
    case V:                                                                                    \
        return launch_step_v<T, TILES[V].tq, TILES[V].tr, TILES[V].nt>(                        \
            d, g, kc, rn, ctl, cl, ntq, ntiles, nwg, par_hint, in, set, stream);
        HEXSV_TILE_SWITCH(HEXSV_CASE)
#undef HEXSV_CASE
        default:
            return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_step(int variant, const KDom<T> &d, const KGrid &g, const KConst &kc,
                       const KRain &rn, Ctl *ctl, const KClose &cl, int ntq, int ntiles, int nwg,
                       int par_hint, int in, int set, hipStream_t stream) {
    return launch_step_any<T>(variant, d, g, kc, rn, ctl, cl, ntq, ntiles, nwg, par_hint, in, set,
                              stream);
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

// Cell i of a row-major raster of nq columns sits at element (i / nq) pitch + i % nq
// of an array whose rows are `pitch` apart (pitch == nq: the same index).
__device__ inline int64_t pitched(int64_t i, int64_t nq, int64_t pitch) {
    return pitch == nq ? i : (i / nq) * pitch + (i % nq);
}

// zero_inactive: 0 copies, 1 writes zero outside the domain, 2 also negates the
// value on Dirichlet cells and writes -2 on flux cells (theta: the step kernel tells
// such cells by theta < 0 and theta < -1.5).
template <typename T>
__global__ void k_import(const double *src, T *dst, const uint8_t *active, int zero_inactive,
                         int64_t n, int64_t nq, int64_t pitch) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint8_t a = active ? active[i] : (uint8_t)1;
        T v = (zero_inactive && a == 0) ? T(0) : (T)src[i];
        if (zero_inactive == 2 && a == 2) v = -v;
        if (zero_inactive == 2 && a == 3) v = T(-2);
        dst[pitched(i, nq, pitch)] = v;
    }
}

template <typename T>
hipError_t launch_import(const double *src, T *dst, const uint8_t *active, int zero_inactive,
                         int64_t n, hipStream_t stream, int64_t nq, int64_t pitch) {
    const int nb = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    if (nq <= 0 || pitch < nq) nq = pitch = 1;
    hipLaunchKernelGGL((k_import<T>), dim3(nb > 0 ? nb : 1), dim3(256), 0, stream, src, dst,
                       active, zero_inactive, n, nq, pitch);
    return hipGetLastError();
}

template <typename T>
__global__ void k_export(KDom<T> d, int par, int64_t n, double *h, double *v1, double *v2,
                         double *q1, double *q2, int64_t nq, int64_t pitch) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = pitched(i, nq, pitch);
        const double hh = (double)d.buf(par, 0)[j];
        const double a = (double)d.buf(par, 1)[j];
        const double b = (double)d.buf(par, 2)[j];
        // Dirichlet cells hold -theta; flux cells hold -2 and carry the discharge h v
        const double ts = (double)d.th[j];
        const double th = ts < -1.5 ? 1.0 : __builtin_fabs(ts);
        if (h) h[i] = hh;
        if (v1) v1[i] = a;
        if (v2) v2[i] = b;
        if (q1) q1[i] = th * hh * a;
        if (q2) q2[i] = th * hh * b;
    }
}

template <typename T>
hipError_t launch_export(const KDom<T> &d, int par, int64_t n, double *h, double *v1,
                         double *v2, double *q1, double *q2, hipStream_t stream, int64_t nq,
                         int64_t pitch) {
    const int nb = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    if (nq <= 0 || pitch < nq) nq = pitch = 1;
    hipLaunchKernelGGL((k_export<T>), dim3(nb > 0 ? nb : 1), dim3(256), 0, stream, d, par, n,
                       h, v1, v2, q1, q2, nq, pitch);
    return hipGetLastError();
}

// ------------------------------------------------------------ surrogate windows
//
// The learned surrogate is not part of the paper's method: a window replaces
// the explicit steps over a fixed span by one network call and is kept only
// if the predicted state keeps the water balance of the scheme (stored =
// initial + rain - outflow - clamped).

// Is the neighbour of (q, r) in direction k an active raster cell?  (The
// INTERIOR edge of the tables; periodic sides wrap.)  Sets j to its index.
template <typename S>
__device__ inline bool active_nbr(const KGrid &g, const S *th, const uint8_t *active, int q, int r,
                                  int k, int64_t &j) {
    int qn = q + dq_of(k), rn = r + dr_of(k);
    if (!wrap_pos(g, qn, rn)) return false;
    j = (int64_t)rn * g.nq + qn;
    if (active && !active[j]) return false;
    return th[j] > S(0);
}

// Terrain slope of cell i = (q, r): along each axis k < 3 of the hexagon the
// estimate d_k = D_k / (2 sqrt(3) a) with D_k the central difference of the
// two neighbours (twice the one-sided one if only one is active); the slope
// is the least-squares (minimum-norm) fit of n_k . grad z = d_k over the axes
// present.  Exact for a plane whenever two axes are present.
template <typename S>
__device__ inline void terrain_slope(const KGrid &g, double a, const S *z, const S *th,
                                     const uint8_t *active, int q, int r, int64_t i, double &sx,
                                     double &sy) {
    const double S3 = 0.86602540378443864676;
    const double NX[3] = {1.0, 0.5, -0.5}, NY[3] = {0.0, S3, S3};
    const double inv = 1.0 / (2.0 * 1.7320508075688772935 * a);
    double m00 = 0.0, m01 = 0.0, m11 = 0.0, b0 = 0.0, b1 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        int64_t j = 0, m = 0;
        const bool pj = active_nbr(g, th, active, q, r, k, j);
        const bool pm = active_nbr(g, th, active, q, r, k + 3, m);
        double D;
        if (pj && pm) D = (double)z[j] - (double)z[m];
        else if (pj) D = 2.0 * ((double)z[j] - (double)z[i]);
        else if (pm) D = 2.0 * ((double)z[i] - (double)z[m]);
        else continue;
        m00 += NX[k] * NX[k];
        m01 += NX[k] * NY[k];
        m11 += NY[k] * NY[k];
        b0 += NX[k] * D * inv;
        b1 += NY[k] * D * inv;
    }
    const double det = m00 * m11 - m01 * m01;
    if (det > 1e-9) {  // two or three axes: M^-1 b
        sx = (m11 * b0 - m01 * b1) / det;
        sy = (m00 * b1 - m01 * b0) / det;
    } else {  // one axis (M = n n^T, b along n: the minimum-norm fit is b) or none
        sx = b0;
        sy = b1;
    }
}

// Time step of a window's probe step: the solver's next step (CFL bound of
// the current state, at most dt_max).
__device__ inline double win_probe_dt(const Ctl *ctl, double dt_max) {
    const double tau = ctl->tau;
    return tau < dt_max ? tau : dt_max;
}

// Terrain slope of every cell (static: computed once per run of windows).
template <typename T>
__global__ __launch_bounds__(256) void k_win_slope(KDom<T> d, KGrid g, double a,
                                                   float2 *__restrict__ slope) {
    const int n = g.nq * g.nr;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const int r = i / g.nq, q = i - r * g.nq;
        double sx = 0.0, sy = 0.0;
        if (d.th[i] > T(0)) terrain_slope<T>(g, a, d.z, d.th, nullptr, q, r, i, sx, sy);
        slope[i] = make_float2((float)sx, (float)sy);
    }
}

template <typename T>
hipError_t launch_win_slope(const KDom<T> &d, const KGrid &g, double a, float2 *slope,
                            hipStream_t stream) {
    const int64_t n = (int64_t)g.nq * g.nr;
    const int nb = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    hipLaunchKernelGGL((k_win_slope<T>), dim3(nb), dim3(256), 0, stream, d, g, a, slope);
    return hipGetLastError();
}

// Volume flux (m^3/s) out of cell (q, r) through its OUTFLOW edges: the ghost
// carries the cell's own h, v and theta, so each such edge passes
// l * theta h * (v . n_k) whatever its sign.
// hscale: a factor the stored depths still wait for (1: none).
template <typename T>
__device__ inline double cell_outflow(const KGrid &g, double l, const T *h, const T *v1,
                                      const T *v2, const T *th, int q, int r, int64_t i,
                                      T hscale = T(1)) {
    const double S3 = 0.86602540378443864676;
    const double NX[6] = {1.0, 0.5, -0.5, -1.0, -0.5, 0.5};
    const double NY[6] = {0.0, S3, S3, 0.0, -S3, -S3};
    if (!(th[i] > T(0))) return 0.0;
    double acc = 0.0;
    for (int k = 0; k < 6; ++k) {
        int qn = q + dq_of(k), rn = r + dr_of(k);
        int cd;
        if (wrap_pos(g, qn, rn)) cd = th[(int64_t)rn * g.nq + qn] > T(0) ? CODE_INTERIOR : g.mask_bc;
        else cd = side_code(g, qn, rn);
        if (cd != CODE_OUTFLOW) continue;
        const double m = (double)th[i] * (double)(hscale == T(1) ? h[i] : h[i] * hscale);
        acc += l * m * ((double)v1[i] * NX[k] + (double)v2[i] * NY[k]);
    }
    return acc;
}

// Can cell (q, r) have an OUTFLOW edge?  Without an active mask only the rim can.
__device__ inline bool may_outflow(const KGrid &g, int q, int r) {
    return g.has_mask || q == 0 || r == 0 || q == g.nq - 1 || r == g.nr - 1;
}

// The network inputs of one cell (all but theta zero on inactive cells):
//   h/H, theta h v1/Q, theta h v2/Q, z/Z, theta, depth/H, slope/S (2),
//   and the probe step's change scaled by xs = window/dt: x_h/dH, x_q1/dQ, x_q2/dQ.
template <typename T>
__device__ inline void win_feature_vec(T h, T v1, T v2, T z, T th, T hs, T v1s, T v2s, float2 sl,
                                       double depth, double xs, const FeatScale &sc,
                                       float f[FEATURES]) {
#pragma unroll
    for (int c = 0; c < FEATURES; ++c) f[c] = 0.f;
    if (!(th > T(0))) return;
    const T q1 = th * h * v1, q2 = th * h * v2;
    f[0] = (float)h / sc.H;
    f[1] = (float)q1 / sc.Q;
    f[2] = (float)q2 / sc.Q;
    f[3] = (float)z / sc.Z;
    f[4] = (float)th;
    f[5] = (float)(depth / sc.H);
    f[6] = sl.x / sc.S;
    f[7] = sl.y / sc.S;
    f[8] = (float)(xs * (double)(hs - h)) / sc.dH;
    f[9] = (float)(xs * (double)(th * hs * v1s - q1)) / sc.dQ;
    f[10] = (float)(xs * (double)(th * hs * v2s - q2)) / sc.dQ;
}

// Probe step of a window, with the network's features: one explicit step of the
// scheme (rain included) from the current state into the scratch buffers, with
// the control block untouched; its change, scaled to the window, is the
// extrapolation the network corrects.  In the same launch every cell's features
// are formed from the start state (still in the tile's registers) and the probe
// state (the values this thread just stored) and written as the network's input
// (FEAT 1: bf16, FEATURES_PAD channels per cell; FEAT 2: FP32, FEATURES
// channels), and each workgroup sums the start state's outflow rate over its
// cells into op0[tile].stored.
//
// The probe also starts the window: every workgroup decides (identically)
// whether it runs -- the chain is alive and the span fits before t_stop -- and
// workgroup 0 records that and the window's rain depth (k equal sub-steps,
// each at the rate of its end: the solver's right-endpoint rule), rain volume,
// start time, stored volume and c_max for the kernels that follow.
template <typename T, int TQ, int TR, int NT, int FEAT>
__global__ __launch_bounds__(NT) void k_win_probe(KDom<T> d, KGrid g, KConst kc, KRain rn,
                                                  const Ctl *ctl, SurWin *sw, T *scr, int ntq,
                                                  int ntiles, double dt_max,
                                                  const float2 *__restrict__ slope, FeatScale fs,
                                                  void *fout, Part *op0) {
    const double t0 = ctl->t;
    const bool live = sw->alive && !ctl->err && t0 + sw->window <= sw->t_stop;
    // the window's rain depth over k equal sub-steps (every workgroup forms the same sum)
    const double dts = sw->window / sw->k;
    double depth = 0.0;
    for (int j = 1; j <= sw->k; ++j) depth += dts * rain_rate(rn, t0 + j * dts);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sw->live = live ? 1 : 0;
        if (live) {
            sw->depth = depth;
            sw->R = kc.area_active * depth;
            sw->t0 = t0;
            sw->S0 = ctl->stored;
            if (!(sw->c0 >= 0.0)) sw->c0 = ctl->last_cmax;
        }
    }
    if (!live) return;
    const int tile = blockIdx.x;
    if (tile >= ntiles) return;
    const int par = ctl->parity;
    const int64_t n = (int64_t)g.nq * g.nr;
    KDom<T> e;
    for (int f = 0; f < 3; ++f) {
        e.st[0][f] = par ? d.st[1][f] : d.st[0][f];
        e.st[1][f] = scr + f * n;
    }
    e.z = d.z;
    e.th = d.th;
    e.ap = d.ap;
    const double dt = win_probe_dt(ctl, dt_max);
    const double r_next = rain_rate(rn, ctl->t + dt);
    __shared__ TileLDS<T, TQ, TR> L;
    Acc acc{0.0, 0.0, 0.0, 0.0};
    const int tr = tile / ntq, tq = tile - tr * ntq;
    TileRegs<T, TQ, TR, NT> R;
    tile_load<T, TQ, TR, NT>(R, e, g, 0, tq, tr);
    // the depths of an accepted, projected window wait for their rescaling until the
    // chain ends: read them scaled (the product the rescaling stores)
    const bool sc_live = sw->scale_live != 0;
    const T hf = (T)sw->scale;
    if (sc_live) {
        using Regs = TileRegs<T, TQ, TR, NT>;
#pragma unroll
        for (int k = 0; k < Regs::CPT; ++k) R.h[k] = R.h[k] * hf;
#pragma unroll
        for (int k = 0; k < Regs::RPT; ++k) R.rh[k] = R.rh[k] * hf;
    }
    const bool bad = tile_stage<T, TQ, TR, NT>(L, R, g, kc, tq, tr);
    const bool inner = tile_inner(g, tq * TQ, tr * TR, TQ, TR);
    const bool general = __syncthreads_or((!inner) || bad) != 0;
    tile_compute<T, TQ, TR, NT, false, false>(L, R, general, e, g, kc, 0, tq, tr, dt, r_next, acc,
                                              &sw->perr, &sw->perr_cell);
    if constexpr (FEAT != 0) {
        using Regs = TileRegs<T, TQ, TR, NT>;
        typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
        const double xs = sw->window / dt;
        const T *h0 = e.st[0][0], *v10 = e.st[0][1], *v20 = e.st[0][2];
        double o = 0.0;
#pragma unroll
        for (int k = 0; k < Regs::CPT; ++k) {
            if (R.pos[k] != POS_OWN) continue;
            const int cc = threadIdx.x + k * NT;
            const int lr = cc / TQ, lq = cc - lr * TQ;
            const int q = tq * TQ + lq, r = tr * TR + lr;
            const uint32_t i = (uint32_t)(r * g.pitch + q);
            // the probe state of this cell: this thread's own stores above (unwritten, and
            // unused, on cells outside the domain)
            float f[FEATURES];
            win_feature_vec<T>(R.h[k], R.v1[k], R.v2[k], R.z[k], R.th[k], e.st[1][0][i],
                               e.st[1][1][i], e.st[1][2][i], slope[i], depth, xs, fs, f);
            if constexpr (FEAT == 1) {
                bf16x8 v[nn::FEATURES_PAD / 8];
#pragma unroll
                for (int c = 0; c < nn::FEATURES_PAD; ++c)
                    v[c / 8][c % 8] = c < FEATURES ? (__bf16)f[c] : (__bf16)0.f;
#pragma unroll
                for (int u = 0; u < nn::FEATURES_PAD / 8; ++u)
                    reinterpret_cast<bf16x8 *>((__bf16 *)fout + (size_t)i * nn::FEATURES_PAD)[u] = v[u];
            } else {
#pragma unroll
                for (int c = 0; c < FEATURES; ++c) ((float *)fout)[(size_t)i * FEATURES + c] = f[c];
            }
            if (may_outflow(g, q, r))
                o += cell_outflow<T>(g, kc.a, h0, v10, v20, d.th, q, r, i, sc_live ? hf : T(1));
        }
        const Part p = block_reduce<NT>(0.0, o, 0.0, 0.0);
        if (threadIdx.x == 0) op0[tile] = p;
    }
}

template <typename T>
hipError_t launch_win_probe(const KDom<T> &d, const KGrid &g, const KConst &kc, const KRain &rn,
                            const Ctl *ctl, SurWin *sw, T *scr, double dt_max,
                            const float2 *slope, FeatScale fs, int feat, void *fout, Part *op0,
                            hipStream_t stream) {
    constexpr TileShape S = TILES[PROBE_TILE];
    int ntq, ntiles;
    tile_grid(PROBE_TILE, g.nq, g.nr, &ntq, &ntiles);
#define HEXSV_PROBE(F)                                                                          \
    hipLaunchKernelGGL((k_win_probe<T, S.tq, S.tr, S.nt, F>), dim3(ntiles), dim3(S.nt), 0, stream, \
                       d, g, kc, rn, ctl, sw, scr, ntq, ntiles, dt_max, slope, fs, fout, op0)
    if (feat == 1) HEXSV_PROBE(1);
    else if (feat == 2) HEXSV_PROBE(2);
    else HEXSV_PROBE(0);
#undef HEXSV_PROBE
    return hipGetLastError();
}

// Predicted state of the window into buffer parity^1, with x the probe's
// change scaled to the window:
//   h' = max(h + x_h + dH out0, 0),  q' = theta h v + x_q + dQ (out1, out2),
//   v' = q' / (theta h') (0 where theta h' <= m_min).  Inactive cells are copied.
// Also reduces, per workgroup (WIN_PARTS workgroups), the predicted state's
// c_max, stored volume sum sigma theta h', outflow rate and count of
// non-finite wave speeds into part[b] = {cmax, stored, outflow, bad}.
template <typename T>
__global__ __launch_bounds__(256) void k_win_apply(KDom<T> d, KGrid g, double l, KConst kc,
                                                   const Ctl *ctl, const SurWin *sw, const T *scr,
                                                   double dt_max, const float *__restrict__ out,
                                                   int os, float dH, float dQ, double m_min,
                                                   Part *part) {
    if (!sw->live) return;
    const int par = ctl->parity;
    const int n = g.nq * g.nr;  // 32-bit cell indices: creation limits a field to 4 GiB
    const double xs = sw->window / win_probe_dt(ctl, dt_max);
    const T *h = par ? d.st[1][0] : d.st[0][0];
    const T *v1 = par ? d.st[1][1] : d.st[0][1];
    const T *v2 = par ? d.st[1][2] : d.st[0][2];
    T *ho = par ? d.st[0][0] : d.st[1][0];
    T *v1o = par ? d.st[0][1] : d.st[1][1];
    T *v2o = par ? d.st[0][2] : d.st[1][2];
    const T *hs = scr, *v1s = scr + n, *v2s = scr + 2 * (size_t)n;  // 2 n can pass 2^31
    const T G = (T)kc.g;
    const bool sc_live = sw->scale_live != 0;  // the start state's depths await a factor
    const T hf = (T)sw->scale;
    double c = 0.0, s = 0.0, o = 0.0, bad = 0.0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const T th = d.th[i];
        const T hi = sc_live ? h[i] * hf : h[i];
        if (!(th > T(0))) {
            ho[i] = hi;
            v1o[i] = v1[i];
            v2o[i] = v2[i];
            continue;
        }
        const T q1 = th * hi * v1[i], q2 = th * hi * v2[i];
        const double xh = xs * (double)(hs[i] - hi);
        const double xq1 = xs * (double)(th * hs[i] * v1s[i] - q1);
        const double xq2 = xs * (double)(th * hs[i] * v2s[i] - q2);
        double hn = (double)hi + xh + (double)dH * (double)out[(size_t)i * os + 0];
        hn = hn > 0.0 ? hn : 0.0;
        const double p1 = (double)q1 + xq1 + (double)dQ * (double)out[(size_t)i * os + 1];
        const double p2 = (double)q2 + xq2 + (double)dQ * (double)out[(size_t)i * os + 2];
        const double mn = (double)th * hn;
        const T hT = (T)hn;
        const T a1 = mn > m_min ? (T)(p1 / mn) : T(0);
        const T a2 = mn > m_min ? (T)(p2 / mn) : T(0);
        ho[i] = hT;
        v1o[i] = a1;
        v2o[i] = a2;
        const double cc = (double)(p_sqrt(a1 * a1 + a2 * a2) + p_sqrt(G * hT));
        if (__builtin_isfinite(cc)) c = cc > c ? cc : c;
        else bad += 1.0;  // the gate refuses such a window
        s += kc.sigma * ((double)th * (double)hT);
        const int r = i / g.nq, q = i - r * g.nq;
        if (may_outflow(g, q, r)) o += cell_outflow<T>(g, l, ho, v1o, v2o, d.th, q, r, i);
    }
    const Part p = block_reduce<256>(c, s, o, bad);
    if (threadIdx.x == 0) part[blockIdx.x] = p;
}

template <typename T>
hipError_t launch_win_apply(const KDom<T> &d, const KGrid &g, double l, const KConst &kc,
                            const Ctl *ctl, const SurWin *sw, const T *scr, double dt_max,
                            const float *out, int out_stride, float dH, float dQ, double m_min,
                            Part *part, hipStream_t stream) {
    hipLaunchKernelGGL((k_win_apply<T>), dim3(WIN_PARTS), dim3(256), 0, stream, d, g, l, kc, ctl, sw,
                       scr, dt_max, out, out_stride, dH, dQ, m_min, part);
    return hipGetLastError();
}

// The network's last layer (32 -> 3 channels) with the window's predicted state
// as its epilogue: the tile's MFMA accumulators plus bias are the network's
// outputs (the values k_hexconv would store), and the lanes holding channels
// 0..2 of a cell apply k_win_apply's arithmetic to them directly.  One record
// per tile of the predicted state's {c_max, stored, outflow rate, non-finite
// count} in part[tile].
template <typename T>
__global__ __launch_bounds__(nn::NT) void k_win_last(const __bf16 *__restrict__ x,
                                                     const __bf16 *__restrict__ wm,
                                                     const float *__restrict__ bias,
                                                     nn::ConvMask cm, KDom<T> d, KGrid g,
                                                     double l, KConst kc, const Ctl *ctl,
                                                     const SurWin *sw, const T *scr,
                                                     double dt_max, float dH, float dQ,
                                                     double m_min, Part *part, int ntiles) {
    using namespace nn;
    __shared__ uint4 lds[NSLOT * 4];
    __shared__ uint8_t fl[NSLOT];
    if (!sw->live) return;
    const int nq = g.nq, nr = g.nr;
    const int ntq = (nq + TQ - 1) / TQ, ntr = (nr + TR - 1) / TR;
    const int tile = xcd_tile(blockIdx.x, gridDim.x, ntiles, 0);
    if (tile < 0) return;
    int b, q0, r0;
    tile_of(tile, ntq, ntr, b, q0, r0);
    stage_act<32>(lds, fl, x, nq, nr, 0, q0, r0, cm);
    __syncthreads();
    f32x4 acc[1][4];
    conv_acc<32, 16>(lds, fl, cm.active != nullptr, wm, acc);
    // the network's outputs of the tile's cells, through LDS to one cell per thread
    static_assert(TQ * TR == NT, "one cell of the tile per thread");
    __shared__ float net[TQ * TR][3];
    {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        if ((lane >> 4) == 0) {  // lanes holding output channels 0..3
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                const int c = w * TQ + nb * 16 + (lane & 15);
#pragma unroll
                for (int j = 0; j < 3; ++j) net[c][j] = acc[0][nb][j] + bias[j];
            }
        }
    }
    __syncthreads();
    const int par = ctl->parity;
    const int n = nq * nr;  // 32-bit cell indices: creation limits a field to 4 GiB
    const double xs = sw->window / win_probe_dt(ctl, dt_max);
    const T *h = par ? d.st[1][0] : d.st[0][0];
    const T *v1 = par ? d.st[1][1] : d.st[0][1];
    const T *v2 = par ? d.st[1][2] : d.st[0][2];
    T *ho = par ? d.st[0][0] : d.st[1][0];
    T *v1o = par ? d.st[0][1] : d.st[1][1];
    T *v2o = par ? d.st[0][2] : d.st[1][2];
    const T *hs = scr, *v1s = scr + n, *v2s = scr + 2 * (size_t)n;  // 2 n can pass 2^31
    const T G = (T)kc.g;
    const bool sc_live = sw->scale_live != 0;  // the start state's depths await a factor
    const T hf = (T)sw->scale;
    double c = 0.0, s = 0.0, o = 0.0, bad = 0.0;
    const int lr = threadIdx.x / TQ, lq = threadIdx.x - lr * TQ;
    const int q = q0 + lq, r = r0 + lr;
    if (q < nq && r < nr) {
        const int i = r * g.pitch + q;
        const T th = d.th[i];
        const T hi = sc_live ? h[i] * hf : h[i];
        if (!(th > T(0))) {
            ho[i] = hi;
            v1o[i] = v1[i];
            v2o[i] = v2[i];
        } else {
            const T q1 = th * hi * v1[i], q2 = th * hi * v2[i];
            const double xh = xs * (double)(hs[i] - hi);
            const double xq1 = xs * (double)(th * hs[i] * v1s[i] - q1);
            const double xq2 = xs * (double)(th * hs[i] * v2s[i] - q2);
            double hn = (double)hi + xh + (double)dH * (double)net[threadIdx.x][0];
            hn = hn > 0.0 ? hn : 0.0;
            const double p1 = (double)q1 + xq1 + (double)dQ * (double)net[threadIdx.x][1];
            const double p2 = (double)q2 + xq2 + (double)dQ * (double)net[threadIdx.x][2];
            const double mn = (double)th * hn;
            const T hT = (T)hn;
            const T a1 = mn > m_min ? (T)(p1 / mn) : T(0);
            const T a2 = mn > m_min ? (T)(p2 / mn) : T(0);
            ho[i] = hT;
            v1o[i] = a1;
            v2o[i] = a2;
            const double cc = (double)(p_sqrt(a1 * a1 + a2 * a2) + p_sqrt(G * hT));
            if (__builtin_isfinite(cc)) c = cc > c ? cc : c;
            else bad += 1.0;  // the gate refuses such a window
            s += kc.sigma * ((double)th * (double)hT);
            if (may_outflow(g, q, r)) o += cell_outflow<T>(g, l, ho, v1o, v2o, d.th, q, r, i);
        }
    }
    const Part p = block_reduce<NT>(c, s, o, bad);
    if (threadIdx.x == 0) part[tile] = p;
}

template <typename T>
hipError_t launch_win_last(const __bf16 *x, const __bf16 *wm, const float *bias,
                           const nn::ConvMask &cm, const KDom<T> &d, const KGrid &g, double l,
                           const KConst &kc, const Ctl *ctl, const SurWin *sw, const T *scr,
                           double dt_max, float dH, float dQ, double m_min, Part *part,
                           hipStream_t stream) {
    const int nt = nn::conv_tiles(g.nq, g.nr, 1);
    hipLaunchKernelGGL((k_win_last<T>), dim3(nt), dim3(nn::NT), 0, stream, x, wm, bias, cm, d, g,
                       l, kc, ctl, sw, scr, dt_max, dH, dQ, m_min, part, nt);
    return hipGetLastError();
}

// h *= scale on the state an accepted window produced (its velocities kept).
template <typename T>
__global__ __launch_bounds__(256) void k_win_scale(KDom<T> d, int64_t n, const Ctl *ctl,
                                                   const SurWin *sw) {
    if (!sw->scale_live) return;
    const int par = ctl->parity;
    const T f = (T)sw->scale;
    T *h = d.buf(par, 0);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        h[i] = h[i] * f;
}

template <typename T>
hipError_t launch_win_scale(const KDom<T> &d, int64_t n, const Ctl *ctl, const SurWin *sw,
                            hipStream_t stream) {
    const int nb = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    hipLaunchKernelGGL((k_win_scale<T>), dim3(nb), dim3(256), 0, stream, d, n, ctl, sw);
    return hipGetLastError();
}

#define HEXSV_INSTANTIATE(T)                                                                  \
    template hipError_t launch_step<T>(int, const KDom<T> &, const KGrid &, const KConst &,   \
                                       const KRain &, Ctl *, const KClose &, int, int, int,   \
                                       int, int, int, hipStream_t);                           \
    template hipError_t launch_prime<T>(const KDom<T> &, int64_t, const KConst &, Ctl *, Part *, \
                                        int, int, hipStream_t);                               \
    template hipError_t launch_win_probe<T>(const KDom<T> &, const KGrid &, const KConst &,   \
                                            const KRain &, const Ctl *, SurWin *, T *, double, \
                                            const float2 *, FeatScale, int, void *, Part *,   \
                                            hipStream_t);                                     \
    template hipError_t launch_win_slope<T>(const KDom<T> &, const KGrid &, double, float2 *, \
                                            hipStream_t);                                     \
    template hipError_t launch_win_apply<T>(const KDom<T> &, const KGrid &, double,           \
                                            const KConst &, const Ctl *, const SurWin *,      \
                                            const T *, double, const float *, int, float,     \
                                            float, double, Part *, hipStream_t);              \
    template hipError_t launch_win_last<T>(const __bf16 *, const __bf16 *, const float *,    \
                                           const nn::ConvMask &, const KDom<T> &, const KGrid &, \
                                           double, const KConst &, const Ctl *, const SurWin *, \
                                           const T *, double, float, float, double, Part *,   \
                                           hipStream_t);                                      \
    template hipError_t launch_win_scale<T>(const KDom<T> &, int64_t, const Ctl *,            \
                                            const SurWin *, hipStream_t);                     \
    template hipError_t launch_import<T>(const double *, T *, const uint8_t *, int, int64_t,  \
                                         hipStream_t, int64_t, int64_t);                      \
    template hipError_t launch_export<T>(const KDom<T> &, int, int64_t, double *, double *,   \
                                         double *, double *, double *, hipStream_t, int64_t,  \
                                         int64_t);

}  // namespace hexsv
