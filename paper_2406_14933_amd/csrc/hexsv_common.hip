// hexsv_common.hip — precision-independent kernels: the single-workgroup
// finalize that closes each step (FP64 books, time, CFL bound), the priming
// pass after set_state, input validation and the neighbour/edge-code tables.
#include <math.h>

#include "hexsv_ensemble.h"
#include "hexsv_internal.h"

namespace hexsv {

// Deterministic reduction of partial records: fixed strided assignment to
// threads (eight independent loads in flight per thread), xor-butterfly within
// waves, fixed order across waves.
template <int NT>
__device__ inline Part reduce_parts(const Part *part, int nparts) {
    double c = 0.0, s = 0.0, o = 0.0, cl = 0.0;
    constexpr int U = 8;
    for (int base = 0; base < nparts; base += NT * U) {
        Part p[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = base + u * NT + threadIdx.x;
            p[u] = i < nparts ? part[i] : Part{0.0, 0.0, 0.0, 0.0};
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            c = p[u].cmax > c ? p[u].cmax : c;
            s += p[u].stored;
            o += p[u].outflow;
            cl += p[u].clamp;
        }
    }
    return block_reduce<NT>(c, s, o, cl);
}

// Totals of one ring slot (one closed step) over its tile records, in the
// same order as a whole-domain reduction of that step.  The slots in use are
// the closed steps of slot `in` plus its pending step.
__global__ __launch_bounds__(1024) void k_fold_slots(const Ctl *ctl, KClose cl, int ntiles,
                                                     int in) {
    const int j = blockIdx.x;
    const Ctl *c = ctl + in;
    const int n = c->open + ((c->p_live != 0 && ctl[0].err == 0) ? 1 : 0);
    if (j >= n) return;
    const Part p = reduce_parts<1024>(cl.ring + (size_t)j * ntiles, ntiles);
    if (threadIdx.x == 0) cl.slots[j] = p;
}

// The pending step of slot `in` closed into ctl[0], the slots' books added in
// step order, the ring emptied and every accumulator cleared.  One wave.
__global__ __launch_bounds__(64) void k_fold_close(Ctl *ctl, KClose cl, KConst kc, KRain rn,
                                                   int in, int set) {
    const OpenStep o = open_step(ctl, in, cl.acc + set * ACC_SET_WORDS, kc);
    if (threadIdx.x == 0) {
        write_slot(ctl, ctl + in, o, kc, rn, false);
        const int n = o.open < cl.ring_len ? o.open : cl.ring_len;
        // in registers: stores to ctl inside the loop would serialise its loads
        double stored = ctl->stored, outflow = ctl->outflow, clamp = ctl->clamp;
        for (int j = 0; j < n; ++j) {
            const Part p = cl.slots[j];
            stored = p.stored;
            outflow += p.outflow;
            clamp += p.clamp;
        }
        ctl->stored = stored;
        ctl->outflow = outflow;
        ctl->clamp = clamp;
        ctl->open = 0;
    }
    for (int i = threadIdx.x; i < ACC_SETS * ACC_SLOTS; i += 64)
        __hip_atomic_store(cl.acc + i * ACC_STRIDE, 0ull, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

hipError_t launch_fold(Ctl *ctl, const KClose &cl, int ntiles, const KConst &kc, const KRain &rn,
                       int in, int set, int launches, hipStream_t stream) {
    const int slots = launches < 1 ? 1 : (launches < cl.ring_len ? launches : cl.ring_len);
    hipLaunchKernelGGL(k_fold_slots, dim3(slots), dim3(1024), 0, stream, ctl, cl, ntiles, in);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fold_close, dim3(1), dim3(64), 0, stream, ctl, cl, kc, rn, in, set);
    return hipGetLastError();
}

__global__ __launch_bounds__(1024) void k_prime_finalize(Ctl *ctl, const Part *part, int nparts,
                                                         KConst kc, int reset_books) {
    const Part p = reduce_parts<1024>(part, nparts);
    if (threadIdx.x == 0) {
        const double cm = p.cmax > kc.c_floor ? p.cmax : kc.c_floor;  // Dirichlet cells too
        ctl->last_cmax = cm;
        ctl->tau = cm > 0.0 ? kc.cfl_phi / cm : INFINITY;
        ctl->stored = p.stored;
        if (reset_books) {
            ctl->initial = p.stored;
            ctl->rain = 0.0;
            ctl->outflow = 0.0;
            ctl->clamp = 0.0;
            ctl->steps = 0;
            ctl->dt_min = INFINITY;
            ctl->dt_max_seen = 0.0;
        }
        ctl->err = 0;
        ctl->err_cell = -1;
    }
}

hipError_t launch_prime_finalize(Ctl *ctl, const Part *part, int nparts, const KConst &kc,
                                 int reset_books, hipStream_t stream) {
    hipLaunchKernelGGL(k_prime_finalize, dim3(1), dim3(1024), 0, stream, ctl, part, nparts, kc,
                       reset_books);
    return hipGetLastError();
}

// chk[0] = number of offending active cells, chk[1] = lowest offending index,
// chk[2] = reason of that cell (bit mask); chk[4..5] (8-byte aligned) = bits of the
// largest |v| + sqrt(g h) over valid Dirichlet and flux cells (state check only).
__device__ inline void flag_bad(int32_t *chk, int64_t i, int reason) {
    atomicAdd(&chk[0], 1);
    atomicMin(&chk[1], (int32_t)i);
    atomicOr(&chk[2], reason);
}

__global__ void k_check_fields(const double *z, const double *th, const double *ap,
                               const uint8_t *active, int64_t n, int32_t *chk) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (active && !active[i]) continue;
        int reason = 0;
        if (!(th[i] > 0.0 && th[i] <= 1.0)) reason |= 1;
        if (!(ap[i] >= 0.0) || !__builtin_isfinite(ap[i])) reason |= 2;
        if (!__builtin_isfinite(z[i])) reason |= 4;
        if (reason) flag_bad(chk, i, reason);
    }
}

__global__ void k_check_state(const double *h, const double *v1, const double *v2,
                              const uint8_t *active, int64_t n, double g, int32_t *chk) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (active && !active[i]) continue;
        int reason = 0;
        if (!(h[i] >= 0.0) || !__builtin_isfinite(h[i])) reason |= 1;
        if (!__builtin_isfinite(v1[i]) || !__builtin_isfinite(v2[i])) reason |= 2;
        if (reason) {
            flag_bad(chk, i, reason);
        } else if (active && active[i] >= 2) {
            // non-negative doubles order like their bit patterns
            const double c = __builtin_sqrt(v1[i] * v1[i] + v2[i] * v2[i]) + __builtin_sqrt(g * h[i]);
            atomicMax((unsigned long long *)(chk + 4), (unsigned long long)__double_as_longlong(c));
        }
    }
}

static int grid_blocks(int64_t n) {
    const int64_t nb = (n + 255) / 256;
    return (int)(nb < 1 ? 1 : (nb > 65536 ? 65536 : nb));
}

hipError_t launch_check_fields(const double *z, const double *th, const double *ap,
                               const uint8_t *active, int64_t n, int32_t *chk,
                               hipStream_t stream) {
    hipLaunchKernelGGL(k_check_fields, dim3(grid_blocks(n)), dim3(256), 0, stream, z, th, ap,
                       active, n, chk);
    return hipGetLastError();
}

hipError_t launch_check_state(const double *h, const double *v1, const double *v2,
                              const uint8_t *active, int64_t n, double g, int32_t *chk,
                              hipStream_t stream) {
    hipLaunchKernelGGL(k_check_state, dim3(grid_blocks(n)), dim3(256), 0, stream, h, v1, v2,
                       active, n, g, chk);
    return hipGetLastError();
}

// Neighbour / edge-code tables, one thread per cell, with the same target
// rules the step kernel applies to its staged halo.
__global__ void k_tables(KGrid g, const uint8_t *active, int32_t *nbr, uint8_t *code,
                         int32_t *qa, int32_t *ra) {
    const int64_t n = (int64_t)g.nq * g.nr;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(i / g.nq), q = (int)(i - (int64_t)r * g.nq);
        if (qa) qa[i] = q;
        if (ra) ra[i] = r;
        if (!nbr && !code) continue;
        const bool act = active ? active[i] != 0 : true;
        for (int k = 0; k < 6; ++k) {
            int qn = q + dq_of(k), rn = r + dr_of(k);
            int32_t j = -1;
            int cd;
            if (!act) {
                cd = CODE_WALL;
            } else if (wrap_pos(g, qn, rn)) {
                const int64_t jj = (int64_t)rn * g.nq + qn;
                const int aj = active ? (int)active[jj] : 1;
                cd = aj == 0   ? g.mask_bc
                     : aj == 2 ? (int)CODE_DIRICHLET
                     : aj == 3 ? (int)CODE_FLUX
                               : (int)CODE_INTERIOR;
                j = aj == 0 ? -1 : (int32_t)jj;
            } else {
                cd = side_code(g, qn, rn);
            }
            if (nbr) nbr[i * 6 + k] = j;
            if (code) code[i * 6 + k] = (uint8_t)cd;
        }
    }
}

// Per-scenario close of a batched step: workgroup s folds the records of
// scenario s's tiles (same order as the single-catchment finalize).
__global__ __launch_bounds__(1024) void k_ens_finalize(const EnsScen *scen, Ctl *ctl,
                                                       const Part *part) {
    const int s = blockIdx.x;
    const StepTime st = step_time(&ctl[s]);
    if (!st.live) return;
    Part p = reduce_parts<1024>(part + scen[s].bbase, scen[s].bntiles);
    const KConst &kc = scen[s].kc;
    if (p.cmax < kc.c_floor) p.cmax = kc.c_floor;  // the Dirichlet cells' wave speed
    if (threadIdx.x == 0) close_step(&ctl[s], p, st, kc, rain_rate(scen[s].rn, st.t_next));
}

hipError_t launch_ens_finalize(const EnsScen *scen, Ctl *ctl, const Part *part, int nscen,
                               hipStream_t stream) {
    hipLaunchKernelGGL(k_ens_finalize, dim3(nscen), dim3(1024), 0, stream, scen, ctl, part);
    return hipGetLastError();
}

// ------------------------------------------------------ surrogate windows

__global__ void k_win_reset(SurWin *sw) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        sw->live = 0;
        sw->alive = 1;
        sw->rejected = 0;
        sw->accepted = 0;
        sw->scale_live = 0;
    }
}

hipError_t launch_win_reset(SurWin *sw, hipStream_t stream) {
    hipLaunchKernelGGL(k_win_reset, dim3(1), dim3(64), 0, stream, sw);
    return hipGetLastError();
}

// Water-balance gate of a window.  With S0, S1 the stored volumes at both
// ends, R the rain volume and O the outflow volume by the trapezoid rule on
// the outflow rates of both states, rho = |S1 - S0 - (R - O)| / max(S0 + R,
// tiny).  Accepted (finite and rho <= tol): the predicted buffer becomes the
// state and time, books and CFL bound advance; with `project` the depths are
// then rescaled (k_win_scale) so that the stored volume is S0 + R - O
// exactly, which keeps the accepted residuals from adding up over many
// windows.  A window is also refused if its fastest wave speed more than
// doubles.  Refused: the chain stops and the state at t0 is untouched.
// The predicted state's records and the start state's outflow records reduced in
// one pass (their loads in flight together), each in reduce_parts' order.
__device__ inline void reduce_window_parts(const Part *part, int n_part, const Part *op0,
                                           int n_op0, Part &p, double &o0) {
    constexpr int NT = 1024;
    double c = 0.0, s = 0.0, o = 0.0, cl = 0.0, s0 = 0.0;
    const int n = n_part > n_op0 ? n_part : n_op0;
    for (int base = 0; base < n; base += NT * 4) {
        Part a[4];
        double b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = base + u * NT + threadIdx.x;
            a[u] = i < n_part ? part[i] : Part{0.0, 0.0, 0.0, 0.0};
            b[u] = i < n_op0 ? op0[i].stored : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            c = a[u].cmax > c ? a[u].cmax : c;
            s += a[u].stored;
            o += a[u].outflow;
            cl += a[u].clamp;
            s0 += b[u];
        }
    }
    __shared__ double red[5][NT / 64];
    c = wave_max(c);
    s = wave_sum(s);
    o = wave_sum(o);
    cl = wave_sum(cl);
    s0 = wave_sum(s0);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][w] = c;
        red[1][w] = s;
        red[2][w] = o;
        red[3][w] = cl;
        red[4][w] = s0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        p = Part{red[0][0], red[1][0], red[2][0], red[3][0]};
        o0 = red[4][0];
        for (int i = 1; i < NT / 64; ++i) {
            p.cmax = red[0][i] > p.cmax ? red[0][i] : p.cmax;
            p.stored += red[1][i];
            p.outflow += red[2][i];
            p.clamp += red[3][i];
            o0 += red[4][i];
        }
    }
}

__global__ __launch_bounds__(1024) void k_win_gate(Ctl *ctl, SurWin *sw, const Part *part,
                                                   int n_part, const Part *op0, int n_op0,
                                                   KConst kc) {
    if (!sw->live) return;
    // the window's record and the books it updates, loaded while the partial sums
    // are reduced (nothing else writes them during this launch)
    double window = 0.0, S0 = 0.0, R = 0.0, c0 = 0.0, tol = 0.0, t0 = 0.0, rain = 0.0,
           outflow = 0.0;
    int project = 0, parity = 0;
    if (threadIdx.x == 0) {
        window = sw->window;
        S0 = sw->S0;
        R = sw->R;
        c0 = sw->c0;
        tol = sw->tol;
        t0 = sw->t0;
        project = sw->project;
        rain = ctl->rain;
        outflow = ctl->outflow;
        parity = ctl->parity;
    }
    Part p{0.0, 0.0, 0.0, 0.0};
    double o0_stored = 0.0;
    reduce_window_parts(part, n_part, op0, n_op0, p, o0_stored);
    if (threadIdx.x != 0) return;
    const double Ow = 0.5 * (o0_stored + p.outflow) * window;
    double ref = S0 + R;
    if (ref < 1e-300) ref = 1e-300;
    const double rho = fabs(p.stored - S0 - (R - Ow)) / ref;
    sw->rho = rho;
    // also refused: a prediction whose fastest wave more than doubles within the
    // window (it would shrink the solver's next steps for no physical reason)
    // (an infinite tolerance keeps every finite window)
    const bool calm = !(c0 > 0.0) || p.cmax <= 2.0 * c0 || isinf(tol);
    const bool ok = p.clamp == 0.0 && isfinite(p.stored) && isfinite(Ow) && rho <= tol && calm;
    if (ok) {
        const double target = S0 + R - Ow;
        double stored = p.stored;
        // the new state waits for its projection factor (applied by the next window's
        // loads and once after the chain); the start state's factor is spent
        sw->scale_live = 0;
        if (project && p.stored > 0.0 && target > 0.0) {
            sw->scale = target / p.stored;
            sw->scale_live = 1;
            stored = target;
        }
        ctl->t = t0 + window;
        ctl->parity = parity ^ 1;
        ctl->stored = stored;
        ctl->rain = rain + R;
        ctl->outflow = outflow + Ow;
        ctl->last_cmax = p.cmax;
        ctl->tau = p.cmax > 0.0 ? kc.cfl_phi / p.cmax : INFINITY;
        sw->accepted += 1;
    } else {
        sw->alive = 0;
        sw->rejected = 1;
        const bool finite = p.clamp == 0.0 && isfinite(p.stored) && isfinite(Ow);
        sw->why = !finite ? 4 : (rho > tol ? 1 : 2);
    }
    sw->live = 0;
}

hipError_t launch_win_gate(Ctl *ctl, SurWin *sw, const Part *part, int n_part, const Part *op0,
                           int n_op0, const KConst &kc, hipStream_t stream) {
    hipLaunchKernelGGL(k_win_gate, dim3(1), dim3(1024), 0, stream, ctl, sw, part, n_part, op0,
                       n_op0, kc);
    return hipGetLastError();
}

__global__ void k_queue_reset(uint32_t *queue) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *queue = 0u;
}

hipError_t launch_queue_reset(uint32_t *queue, hipStream_t stream) {
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, stream, queue);
    return hipGetLastError();
}

hipError_t launch_tables(const KGrid &g, const uint8_t *active, int32_t *nbr, uint8_t *code,
                         int32_t *q, int32_t *r, hipStream_t stream) {
    hipLaunchKernelGGL(k_tables, dim3(grid_blocks((int64_t)g.nq * g.nr)), dim3(256), 0, stream, g,
                       active, nbr, code, q, r);
    return hipGetLastError();
}

}  // namespace hexsv
