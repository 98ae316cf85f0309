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

// CODE_DIRICHLET: the neighbour is a cell held at a prescribed state (inflow of
// Sec. 3.2.1, eq. numerics-bc); it is read like a cell, the edge carries its velocity
// and the flux across is booked with the outflow.  CODE_FLUX: the neighbour prescribes
// the discharge h v across the edge (given mass flux); the pressure term sees the cell's
// own depth over the neighbour's bed.  Both kinds hold theta negated (flux cells: -2).
enum {
    CODE_INTERIOR = 0, CODE_WALL = 1, CODE_OUTFLOW = 2, CODE_PERIODIC = 3, CODE_DIRICHLET = 4,
    CODE_FLUX = 5
};
enum { SIDE_S = 0, SIDE_E = 1, SIDE_N = 2, SIDE_W = 3 };

constexpr int MAX_SEG = 8;

// Raster description as the kernels see it (passed by value).
struct KGrid {
    int32_t nq, nr;
    int32_t pitch;  // row stride of the cell arrays (nq, or more for aligned rows)
    int32_t perq, perr;
    int32_t side[4];
    int32_t nseg;
    int32_t mask_bc;
    int32_t has_mask;  // some cells are outside the domain
    int32_t seg_side[MAX_SEG], seg_lo[MAX_SEG], seg_hi[MAX_SEG], seg_code[MAX_SEG];
};

struct KRain {
    int32_t kind;
    double i_a, t_a, T_d;
};

// Device-resident control block: time, CFL bound, step counters, the buffer
// parity and the FP64 books.
//
// A single domain keeps two of them.  ctl[0] is the one the host and every
// other kernel see between graph replays; inside a run of step launches the
// two alternate: a launch reads slot `in` and its workgroup 0 writes slot
// in ^ 1 for the next launch.  The step a launch starts is closed by the next
// launch (its wave-speed maximum is only complete once the launch has ended),
// so a slot carries that pending step (p_live, p_dt, p_tnext) beside the state
// after the last closed one; a fold kernel closes the last pending step and
// brings ctl[0] up to date.  err and err_cell are only used in ctl[0].
// The ensemble keeps one block per scenario and closes each step at once.
struct alignas(128) Ctl {
    double t, tau, t_end, dt_max;
    int64_t steps, step_limit;
    int32_t parity, err;
    int32_t err_cell;
    int32_t open;  // closed steps whose water books still wait in the step ring
    double initial, stored, rain, outflow, clamp, dt_min, dt_max_seen, last_cmax;
    double p_dt, p_tnext;  // the pending step's dt and end time
    int32_t p_live, pad0;  // a step was started and is not closed yet
};
static_assert(sizeof(Ctl) == 256, "control block is 256 bytes");

// Per-tile partial results of one step.
struct alignas(32) Part {
    double cmax, stored, outflow, clamp;
};

// Where the tile kernel of a single-domain step leaves its results: the
// largest wave speed goes into one of ACC_SLOTS accumulators of the launch's
// set (an atomic maximum over the bit patterns of non-negative doubles, which
// order like the values; tile t uses slot t % ACC_SLOTS, ACC_STRIDE words
// apart, so that the atomics of concurrent tiles do not queue on one
// address), the tile's water books into slot `open` of the ring
// (ring[slot * ntiles + tile]).  Launch k of a run accumulates into set k % 3,
// reads set (k - 1) % 3 to close the previous step and clears set (k + 1) % 3
// for the next launch.  The fold kernels add the ring's records to the books,
// step by step in order, every ring_len steps at most.
constexpr int ACC_SLOTS = 16;
constexpr int ACC_STRIDE = 32;  // 256 bytes
constexpr int ACC_SETS = 3;
constexpr int ACC_SET_WORDS = ACC_SLOTS * ACC_STRIDE;
struct KClose {
    Part *ring;
    Part *slots;  // per-slot totals (fold scratch)
    unsigned long long *acc;
    int ring_len;
};

// Static geometry and parameters of one domain.
struct KConst {
    double g, a, sigma, cfl_phi, h_dry, alpha_s;
    double area_active;  // sigma * number of active cells
    double tau_lin;      // linear soil resistance -tau h v (Thacker test), 1/s; 0: off
    double c_floor;      // largest |v| + sqrt(g h) of the Dirichlet cells (fixed), 0 if none
    double f_inf, h_inf; // infiltration i(h) = f_inf h / (h + h_inf) at h^{n+1}; f_inf 0: off
    int32_t visc;        // 1: augmented momentum flux with artificial viscosity
    int32_t ext;         // 1: Dirichlet or given-flux cells, or infiltration (extended instance)
};

template <typename T>
struct KDom {
    T *st[2][3];      // state buffers [parity][h, v1, v2]
    const T *z, *th, *ap;
    const T *as = nullptr;  // soil coefficient per cell (eq_tsa_darcy), read by the
                            // extended instance only; null: the scalar KConst::alpha_s
    __device__ __host__ T *buf(int p, int f) const { return st[p][f]; }
};

// ------------------------------------------------------------- helpers

// Element i of a field through a 32-bit byte offset from the field's base
// (a uniform register pair), so each access needs no 64-bit address
// arithmetic.  Valid while a field holds less than 4 GiB, which sim and
// ensemble creation check.
template <typename T>
__device__ inline T ld(const T *p, uint32_t i) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(p) + i * (uint32_t)sizeof(T));
}
// The same with the nontemporal (streaming) hint, for data read once per step.
template <typename T>
__device__ inline T ld_stream(const T *p, uint32_t i) {
    return __builtin_nontemporal_load(
        reinterpret_cast<const T *>(reinterpret_cast<const char *>(p) + i * (uint32_t)sizeof(T)));
}
template <typename T>
__device__ inline T *at(T *p, uint32_t i) {
    return reinterpret_cast<T *>(reinterpret_cast<char *>(p) + i * (uint32_t)sizeof(T));
}

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
    // FP64 time and books: rounded as written in every translation unit, whatever its
    // contraction setting, so all kernels that close steps agree bit for bit
#pragma clang fp contract(off)
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
    // FP64 time and books: rounded as written in every translation unit, whatever its
    // contraction setting, so all kernels that close steps agree bit for bit
#pragma clang fp contract(off)
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
// Largest wave speed in one accumulator set (see KClose).  The addresses are
// uniform and nothing is stored before, so these are scalar loads, which do
// not wait for the tile's vector loads.  The set was last written by the
// previous launch: the kernel boundary makes it visible, as it does for the
// control slots.
__device__ inline double acc_max(const unsigned long long *set) {
    unsigned long long m = 0;
#pragma unroll
    for (int i = 0; i < ACC_SLOTS; ++i) {
        const unsigned long long v = set[i * ACC_STRIDE];
        m = v > m ? v : m;
    }
    return __longlong_as_double((long long)m);
}

// A launch's view of the run: control slot `in` with its pending step
// closed (when there is one and no error was flagged), and the step this
// launch starts from there.
struct OpenStep {
    double t, tau, cmax;  // after the close (cmax: of the closed step)
    double dt, t_next;    // of the step this launch starts
    int64_t steps;
    int parity, open;
    bool closed, live;
};

// prev_set: the accumulator set the pending step of slot `in` accumulated
// into (read whether or not a step is pending, so the loads start at once).
__device__ inline OpenStep open_step(const Ctl *ctl, int in, const unsigned long long *prev_set,
                                     const KConst &kc) {
    // FP64 time and books: rounded as written in every translation unit, whatever its
    // contraction setting, so all kernels that close steps agree bit for bit
#pragma clang fp contract(off)
    const double prev_max = acc_max(prev_set);
    const Ctl *c = ctl + in;
    const int err = ctl[0].err;
    OpenStep o;
    o.closed = c->p_live != 0 && err == 0;
    o.t = c->t;
    o.tau = c->tau;
    o.steps = c->steps;
    o.parity = c->parity;
    o.open = c->open;
    o.cmax = 0.0;
    if (o.closed) {
        // c_max of eq. .12 over the updated cells and the Dirichlet cells, whose
        // prescribed states enter the fluxes of their neighbours as well
        o.cmax = prev_max > kc.c_floor ? prev_max : kc.c_floor;
        o.t = c->p_tnext;
        o.tau = o.cmax > 0.0 ? kc.cfl_phi / o.cmax : __builtin_inf();
        o.steps += 1;
        o.parity ^= 1;
        o.open += 1;
    }
    const double t_end = c->t_end;
    double dt = c->dt_max;
    if (o.tau < dt) dt = o.tau;
    if (t_end - o.t < dt) dt = t_end - o.t;
    o.dt = dt;
    o.live = (dt > 0.0) && (o.steps < c->step_limit) && (err == 0);
    o.t_next = (dt == t_end - o.t) ? t_end : o.t + dt;
    return o;
}

// Slot `out` of the control block from slot `in` and the launch's view: the
// pending step of `in` closed (time, counters, CFL bound, rain book, dt range)
// and the launch's own step pending.  err and err_cell are left alone.
__device__ inline void write_slot(Ctl *out, const Ctl *in, const OpenStep o, const KConst &kc,
                                  const KRain &rn, bool pending) {
    // FP64 time and books: rounded as written in every translation unit, whatever its
    // contraction setting, so all kernels that close steps agree bit for bit
#pragma clang fp contract(off)
    double rain = in->rain, dmin = in->dt_min, dmax = in->dt_max_seen, lc = in->last_cmax;
    if (o.closed) {
        const double pdt = in->p_dt;
        rain += kc.area_active * pdt * rain_rate(rn, in->p_tnext);
        if (pdt < dmin) dmin = pdt;
        if (pdt > dmax) dmax = pdt;
        lc = o.cmax;
    }
    const double t_end = in->t_end, dt_max = in->dt_max, initial = in->initial;
    const double stored = in->stored, outflow = in->outflow, clamp = in->clamp;
    const int64_t limit = in->step_limit;
    out->t = o.t;
    out->tau = o.tau;
    out->t_end = t_end;
    out->dt_max = dt_max;
    out->steps = o.steps;
    out->step_limit = limit;
    out->parity = o.parity;
    out->open = o.open;
    out->initial = initial;
    out->stored = stored;
    out->rain = rain;
    out->outflow = outflow;
    out->clamp = clamp;
    out->dt_min = dmin;
    out->dt_max_seen = dmax;
    out->last_cmax = lc;
    out->p_live = pending && o.live ? 1 : 0;
    out->p_dt = o.dt;
    out->p_tnext = o.t_next;
}

__device__ inline void close_step(Ctl *ctl, const Part &p, const StepTime &st, const KConst &kc,
                                  double r_next) {
    // FP64 time and books: rounded as written in every translation unit, whatever its
    // contraction setting, so all kernels that close steps agree bit for bit
#pragma clang fp contract(off)
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

// Tile schedule of a grid-stride launch of G workgroups over ntiles tiles.
// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on
// XCD b % 8), so each XCD gets a contiguous band of tiles and its workgroups
// sweep the band together: concurrently processed tiles are neighbours and
// their shared halo rows stay in that XCD's L2.  Returns -1 past the end.
__device__ inline int xcd_tile(int b, int G, int ntiles, int k) {
    const int x = b & 7;
    const int gx = (G >> 3) + (x < (G & 7) ? 1 : 0);  // workgroups on XCD x
    const int j = b >> 3;                               // rank among them
    const int per = ntiles >> 3, rem = ntiles & 7;
    const int cnt = per + (x < rem ? 1 : 0);            // tiles of XCD x
    const int start = x * per + (x < rem ? x : rem);
    const int t = j + k * gx;
    return t < cnt ? start + t : -1;
}

}  // namespace hexsv
