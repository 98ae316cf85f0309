// hexsv_device.h — device-side data structures and the per-tile step of the
// porous Saint-Venant scheme on a hexagonal raster (gfx950, wave64).
//
// One workgroup advances one TQ x TR tile of cells by one time step:
//   1. stage the tile plus a one-cell halo of (h, v1, v2, z, theta) and the
//      edge code of every staged position in LDS (one coalesced HBM read per
//      field per cell; halo rows come from L2/MALL);
//   2. per cell, sum the six edge terms L, J, S (Sec. 2.2 (c), eqs.
//      fvm_2D_eq.04-.06 and fvm_2D_eq_frac.01), update theta*h with the rain
//      at t^{n+1} and clamp at zero (eq. fvm_2D_eq_frac.05-1/.06-1), then solve
//      the implicit friction step in closed form (Appendix A, miu-formula);
//   3. reduce c = |v| + sqrt(g h) (max) and the FP64 volume books (sums) over
//      the workgroup into one partial record per tile.
// The arithmetic follows the order of the equations; the FP64 build keeps
// contraction off so each operation rounds as written.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hexsv {

enum { CODE_INTERIOR = 0, CODE_WALL = 1, CODE_OUTFLOW = 2, CODE_PERIODIC = 3 };
enum { SIDE_S = 0, SIDE_E = 1, SIDE_N = 2, SIDE_W = 3 };

constexpr int MAX_SEG = 8;

// Raster description as the kernels see it (passed by value).
struct KGrid {
    int32_t nq, nr;
    int32_t perq, perr;
    int32_t side[4];
    int32_t nseg;
    int32_t mask_bc;
    int32_t seg_side[MAX_SEG], seg_lo[MAX_SEG], seg_hi[MAX_SEG], seg_code[MAX_SEG];
};

struct KRain {
    int32_t kind;
    double i_a, t_a, T_d;
};

// Device-resident control block: time, CFL bound, step counters, the buffer
// parity and the FP64 books.  Read by every step kernel, written only by the
// single-workgroup finalize kernel that closes each step.
struct alignas(128) Ctl {
    double t, tau, t_end, dt_max;
    int64_t steps, step_limit;
    int32_t parity, err;
    int32_t err_cell, pad0;
    double initial, stored, rain, outflow, clamp, dt_min, dt_max_seen, last_cmax;
};
static_assert(sizeof(Ctl) == 128, "control block is 128 bytes");

// Per-tile partial results of one step.
struct alignas(32) Part {
    double cmax, stored, outflow, clamp;
};

// Static geometry and parameters of one domain.
struct KConst {
    double g, a, sigma, cfl_phi, h_dry, alpha_s;
    double area_active;  // sigma * number of active cells
};

template <typename T>
struct KDom {
    T *st[2][3];      // state buffers [parity][h, v1, v2]
    const T *z, *th, *ap;
};

// ------------------------------------------------------------- helpers

__device__ __host__ inline int dq_of(int k) {
    return k == 0 ? 1 : (k == 1 ? 0 : (k == 2 ? -1 : (k == 3 ? -1 : (k == 4 ? 0 : 1))));
}
__device__ __host__ inline int dr_of(int k) {
    return k == 0 ? 0 : (k == 1 ? 1 : (k == 2 ? 1 : (k == 3 ? 0 : (k == 4 ? -1 : -1))));
}

// Apply periodic wraps; true if (q, r) is then inside the raster.
__device__ inline bool wrap_pos(const KGrid &g, int &q, int &r) {
    if (g.perq) {
        if (q < 0) q += g.nq;
        else if (q >= g.nq) q -= g.nq;
    }
    if (g.perr) {
        if (r < 0) r += g.nr;
        else if (r >= g.nr) r -= g.nr;
    }
    return q >= 0 && q < g.nq && r >= 0 && r < g.nr;
}

// Code of a boundary edge whose outside neighbour sits at (q, r) (after wraps,
// outside the raster): S/N when r is out of range, else E/W; a segment of
// that side containing the position along the side overrides the side code.
__device__ inline int side_code(const KGrid &g, int q, int r) {
    int side, pos;
    if (r < 0) { side = SIDE_S; pos = q; }
    else if (r >= g.nr) { side = SIDE_N; pos = q; }
    else if (q < 0) { side = SIDE_W; pos = r; }
    else { side = SIDE_E; pos = r; }
    for (int s = 0; s < g.nseg; ++s)
        if (g.seg_side[s] == side && pos >= g.seg_lo[s] && pos < g.seg_hi[s]) return g.seg_code[s];
    return g.side[side];
}

__device__ inline double rain_rate(const KRain &rn, double t) {
    if (rn.kind == 0) return (t >= 0.0 && t <= rn.T_d) ? rn.i_a : 0.0;
    double gamma = rn.t_a / rn.T_d;
    if (t >= 0.0 && t <= rn.t_a) return rn.i_a * (t / rn.t_a);
    if (t > rn.t_a && t <= rn.T_d) return rn.i_a * ((1.0 - t / rn.T_d) / (1.0 - gamma));
    return 0.0;
}

// Time step of the step that starts from ctl (Appendix A, eq. .12): the same
// scalar is computed by every workgroup and by the finalize kernel.
struct StepTime {
    double dt, t_next;
    bool live;
};
__device__ inline StepTime step_time(const Ctl *ctl) {
    StepTime s;
    double t = ctl->t, t_end = ctl->t_end;
    double dt = ctl->dt_max;
    if (ctl->tau < dt) dt = ctl->tau;
    if (t_end - t < dt) dt = t_end - t;
    s.dt = dt;
    s.live = (dt > 0.0) && (ctl->steps < ctl->step_limit) && (ctl->err == 0);
    s.t_next = (dt == t_end - t) ? t_end : t + dt;
    return s;
}

// Precision-specific primitives: FP64 uses correctly rounded sqrt and
// division (same results as the CPU reference); FP32 uses the hardware
// square root and reciprocal (about 1 ulp).
__device__ inline float p_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline double p_sqrt(double x) { return __builtin_sqrt(x); }
__device__ inline float p_div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ inline double p_div(double a, double b) { return a / b; }

template <typename T>
__device__ inline T wave_max(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T u = __shfl_xor(v, o, 64);
        v = u > v ? u : v;
    }
    return v;
}
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Reduce (cmax, stored, outflow, clamp) over the workgroup; thread 0 returns it.
template <int NT>
__device__ inline Part block_reduce(double c, double s, double o, double cl) {
    constexpr int NW = NT / 64;
    __shared__ double red[4][NW];
    c = wave_max(c);
    s = wave_sum(s);
    o = wave_sum(o);
    cl = wave_sum(cl);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][w] = c;
        red[1][w] = s;
        red[2][w] = o;
        red[3][w] = cl;
    }
    __syncthreads();
    Part p{0.0, 0.0, 0.0, 0.0};
    if (threadIdx.x == 0) {
        p.cmax = red[0][0];
        p.stored = red[1][0];
        p.outflow = red[2][0];
        p.clamp = red[3][0];
        for (int i = 1; i < NW; ++i) {
            p.cmax = red[0][i] > p.cmax ? red[0][i] : p.cmax;
            p.stored += red[1][i];
            p.outflow += red[2][i];
            p.clamp += red[3][i];
        }
    }
    return p;
}

// Close one step on the device (Appendix A, eqs. .12-.13 for the next bound):
// FP64 books, t^{n+1}, step count, buffer parity and tau = CFL*phi_min/c_max.
__device__ inline void close_step(Ctl *ctl, const Part &p, const StepTime &st, const KConst &kc,
                                  double r_next) {
    ctl->stored = p.stored;
    ctl->outflow += p.outflow;
    ctl->clamp += p.clamp;
    ctl->rain += kc.area_active * st.dt * r_next;
    ctl->t = st.t_next;
    ctl->steps += 1;
    if (st.dt < ctl->dt_min) ctl->dt_min = st.dt;
    if (st.dt > ctl->dt_max_seen) ctl->dt_max_seen = st.dt;
    ctl->last_cmax = p.cmax;
    ctl->tau = p.cmax > 0.0 ? kc.cfl_phi / p.cmax : __builtin_inf();
    ctl->parity ^= 1;
}

// Reduce n (<= 64) partial records with one wave in a fixed order; lane 0
// holds the result.
__device__ inline Part wave_reduce_parts(const Part *part, int n) {
    const int lane = threadIdx.x & 63;
    Part p{0.0, 0.0, 0.0, 0.0};
    if (lane < n) p = part[lane];
    p.cmax = wave_max(p.cmax);
    p.stored = wave_sum(p.stored);
    p.outflow = wave_sum(p.outflow);
    p.clamp = wave_sum(p.clamp);
    return p;
}

constexpr int GROUP = 64;  // tiles per first-level group of the step reduction

// Two-level "last workgroup closes" reduction of the per-tile records of one
// step: the last tile of each group of 64 folds the group into gpart, the
// last group folds the groups and closes the step.  Deterministic: every sum
// is taken in tile order regardless of which workgroup finishes last.
// ctr[0] counts groups, ctr[1+g] counts tiles of group g; closers reset them.
template <int NT>
__device__ inline void finish_tile(const Part &p, int tile, int ntiles, Part *part, Part *gpart,
                                   uint32_t *ctr, Ctl *ctl, const StepTime &st, const KConst &kc,
                                   double r_next) {
    __shared__ int s_close;
    const int grp = tile / GROUP;
    const int ngroups = (ntiles + GROUP - 1) / GROUP;
    if (threadIdx.x == 0) {
        part[tile] = p;
        const int gsize = (ntiles - grp * GROUP) < GROUP ? (ntiles - grp * GROUP) : GROUP;
        const uint32_t prev =
            __hip_atomic_fetch_add(&ctr[1 + grp], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        s_close = (prev == (uint32_t)(gsize - 1)) ? 1 : 0;
    }
    __syncthreads();
    if (!s_close) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (threadIdx.x < 64) {
        const int base = grp * GROUP;
        const int gsize = (ntiles - base) < GROUP ? (ntiles - base) : GROUP;
        const Part g = wave_reduce_parts(part + base, gsize);
        if (threadIdx.x == 0) {
            gpart[grp] = g;
            ctr[1 + grp] = 0u;
            const uint32_t prev =
                __hip_atomic_fetch_add(&ctr[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            s_close = (prev == (uint32_t)(ngroups - 1)) ? 2 : 0;
        }
    }
    __syncthreads();
    if (s_close != 2) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    // fold the groups: fixed strided assignment, then the workgroup reduction
    double c = 0.0, s = 0.0, o = 0.0, cl = 0.0;
    for (int i = threadIdx.x; i < ngroups; i += NT) {
        const Part g = gpart[i];
        c = g.cmax > c ? g.cmax : c;
        s += g.stored;
        o += g.outflow;
        cl += g.clamp;
    }
    const Part tot = block_reduce<NT>(c, s, o, cl);
    if (threadIdx.x == 0) {
        close_step(ctl, tot, st, kc, r_next);
        ctr[0] = 0u;
    }
}

// Logical tile of hardware workgroup b: workgroups are dispatched round-robin
// over the 8 XCDs, so give each XCD a contiguous band of tiles (its L2 then
// holds the halo rows shared by vertically adjacent tiles).
__device__ inline int xcd_tile(int b, int ntiles) {
    const int per = ntiles >> 3, rem = ntiles & 7;
    const int x = b & 7, j = b >> 3;
    return x * per + (x < rem ? x : rem) + j;
}

// ------------------------------------------------------------ tile step

template <typename T, int TQ, int TR>
struct TileLDS {
    static constexpr int W = TQ + 2, H = TR + 2, NS = W * H;
    T h[NS], v1[NS], v2[NS], z[NS], th[NS];
    uint8_t code[NS];
};

// Advance tile (tq, tr) of domain d by one step: reads buffer `par`, writes
// buffer par^1.  Returns the tile's partial record in thread 0.
template <typename T, int TQ, int TR, int NT>
__device__ inline Part tile_step(TileLDS<T, TQ, TR> &L, const KDom<T> &d, const KGrid &g,
                                 const KConst &kc, int par, int tq, int tr, double dt,
                                 double r_next, int32_t *err_flag, int32_t *err_cell) {
    constexpr int W = TQ + 2;
    constexpr int NS = (TQ + 2) * (TR + 2);
    const int q0 = tq * TQ, r0 = tr * TR;
    const T *__restrict__ hin = d.st[par][0];
    const T *__restrict__ v1in = d.st[par][1];
    const T *__restrict__ v2in = d.st[par][2];
    T *__restrict__ hout = d.st[par ^ 1][0];
    T *__restrict__ v1out = d.st[par ^ 1][1];
    T *__restrict__ v2out = d.st[par ^ 1][2];

    // 1. stage tile + halo
    for (int s = threadIdx.x; s < NS; s += NT) {
        const int lr = s / W, lq = s - lr * W;
        int q = q0 + lq - 1, r = r0 + lr - 1;
        if (wrap_pos(g, q, r)) {
            const int64_t i = (int64_t)r * g.nq + q;
            const T th = d.th[i];
            L.h[s] = hin[i];
            L.v1[s] = v1in[i];
            L.v2[s] = v2in[i];
            L.z[s] = d.z[i];
            L.th[s] = th;
            L.code[s] = th > T(0) ? (uint8_t)CODE_INTERIOR : (uint8_t)g.mask_bc;
        } else {
            L.h[s] = T(0);
            L.v1[s] = T(0);
            L.v2[s] = T(0);
            L.z[s] = T(0);
            L.th[s] = T(0);
            L.code[s] = (uint8_t)side_code(g, q, r);
        }
    }
    __syncthreads();

    const T G = (T)kc.g;
    const T l = (T)kc.a;
    const T half_l = (T)(0.5 * kc.a);
    const T dtT = (T)dt;
    const T dts = (T)(dt / kc.sigma);
    const T rT = (T)r_next;
    const T alpha_s = (T)kc.alpha_s;
    const T h_dry = (T)kc.h_dry;
    const T S3H = (T)0.86602540378443864676;
    const T NX[6] = {T(1), T(0.5), T(-0.5), T(-1), T(-0.5), T(0.5)};
    const T NY[6] = {T(0), S3H, S3H, T(0), -S3H, -S3H};
    constexpr int OFF[6] = {1, W, W - 1, -1, -W, -W + 1};

    double c_loc = 0.0, s_loc = 0.0, o_loc = 0.0, cl_loc = 0.0;

    for (int c = threadIdx.x; c < TQ * TR; c += NT) {
        const int lr = c / TQ, lq = c - lr * TQ;
        const int q = q0 + lq, r = r0 + lr;
        if (q >= g.nq || r >= g.nr) continue;
        const int s = (lr + 1) * W + (lq + 1);
        if (L.code[s] != CODE_INTERIOR) continue;  // cell outside the domain
        const T hi = L.h[s], v1i = L.v1[s], v2i = L.v2[s], zi = L.z[s], thi = L.th[s];
        const T mi = thi * hi;
        const T wi = G * (zi + hi);
        T Ls = T(0), J1 = T(0), J2 = T(0), S1 = T(0), S2 = T(0), Fout = T(0);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int sn = s + OFF[k];
            const int cd = L.code[sn];
            if (cd == CODE_WALL) continue;
            T hj, v1j, v2j, zj, thj;
            if (cd == CODE_INTERIOR) {
                hj = L.h[sn];
                v1j = L.v1[sn];
                v2j = L.v2[sn];
                zj = L.z[sn];
                thj = L.th[sn];
            } else {  // free outflow ghost
                const int so = s - OFF[k];
                hj = hi;
                v1j = v1i;
                v2j = v2i;
                thj = thi;
                zj = (L.code[so] == CODE_INTERIOR) ? T(2) * zi - L.z[so] : zi;
            }
            const T mj = thj * hj;
            const T wj = G * (zj + hj);
            const T vb1 = (v1i + v1j) * T(0.5);
            const T vb2 = (v2i + v2j) * T(0.5);
            const T vn = vb1 * NX[k] + vb2 * NY[k];
            const T mup = vn > T(0) ? mi : (vn < T(0) ? mj : T(0));
            const T mhat = vn != T(0) ? mup : (wi > wj ? mi : mj);
            const T F = l * mup * vn;
            Ls -= F;
            J1 -= F * vb1;
            J2 -= F * vb2;
            const T P = half_l * (wj - wi) * mhat;
            S1 -= P * NX[k];
            S2 -= P * NY[k];
            if (cd == CODE_OUTFLOW) Fout += F;
        }
        // mass: eq. fvm_2D_eq_frac.05-1 then .06-1 (rain at t^{n+1})
        const T ms = mi + dts * Ls;
        T m1 = ms + dtT * rT;
        if (m1 < T(0)) {
            cl_loc += kc.sigma * (-(double)m1);
            m1 = T(0);
        }
        const T h1 = p_div(m1, thi);
        // momentum: (theta h v)^* of eq. .05-2, friction of eq. .06-2 solved in closed form
        const T g1 = mi * v1i + dts * (J1 + S1);
        const T g2 = mi * v2i + dts * (J2 + S2);
        const int64_t i = (int64_t)r * g.nq + q;
        const T K = d.ap[i] * h1 * (T(1) - thi) + thi * alpha_s;
        const T beta = dtT * K;
        const T Gm = p_sqrt(g1 * g1 + g2 * g2);
        const T D = m1 + p_sqrt(m1 * m1 + T(4) * beta * Gm);
        T mu = (D == T(0)) ? T(0) : p_div(T(2), D);
        if (h_dry > T(0) && h1 < h_dry) mu = T(0);
        const T v1n = mu * g1, v2n = mu * g2;
        hout[i] = h1;
        v1out[i] = v1n;
        v2out[i] = v2n;
        const T cc = p_sqrt(v1n * v1n + v2n * v2n) + p_sqrt(G * h1);
        c_loc = (double)cc > c_loc ? (double)cc : c_loc;
        s_loc += kc.sigma * ((double)thi * (double)h1);
        o_loc += dt * (double)Fout;
        if (!__builtin_isfinite(h1) || !__builtin_isfinite(v1n) || !__builtin_isfinite(v2n)) {
            if (atomicOr(err_flag, 1) == 0) *err_cell = (int32_t)i;
        }
    }
    return block_reduce<NT>(c_loc, s_loc, o_loc, cl_loc);
}

}  // namespace hexsv
