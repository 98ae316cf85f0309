// hexsv_tile.h — one explicit step of one TQ x TR tile of the raster.
//
// A tile step has three phases, kept apart so that a persistent kernel can
// overlap the loads of the next tile with the arithmetic of the current one:
//   load:    every thread loads (h, v1, v2, z, theta, alpha_p) of the cells it
//            owns (coalesced rows of the tile) and the halo slots of the tile
//            rim it is responsible for, into registers;
//   stage:   registers -> one 4-word LDS record per staged position,
//              {mass, w = g (z + h), v1/2, v2/2},
//            with mass = theta*h (FP64) or l*theta*h (FP32), plus an edge
//            code per position when the tile touches the raster boundary or
//            an inactive cell.  Interface velocities of eq. fvm_2D_eq.04 are
//            then one add (v_i/2 + v_j/2 equals (v_i + v_j)/2 exactly) and a
//            neighbour is one 16-byte LDS read;
//   compute: per owned cell, the six edge terms of eq. fvm_2D_eq_frac.01 with
//            the interface rules of eqs. fvm_2D_eq.05-.06, the mass update
//            with rain at t^{n+1} and clamping (eqs. .05-1/.06-1), and the
//            closed-form friction solve (Appendix A, miu-formula).
//
// FP64 evaluates the equations operation for operation as the CPU reference
// (contraction off); FP32 regroups them (J + S in one accumulator, l folded
// into the staged mass, depth updated by its increment) to save instructions
// and keep still water exactly still.
#pragma once

#include <type_traits>

#include "hexsv_device.h"

namespace hexsv {

template <typename T>
struct Rec;
template <>
struct Rec<float> {
    using type = float4;
};
template <>
struct Rec<double> {
    using type = double4;
};

// V: the step adds the artificial viscosity of the augmented momentum flux
// (eqs. eq_artif_visc, eq_visc1), which needs c = |v| + sqrt(g h) of every
// staged position as well.
template <typename T, int TQ, int TR, bool V = false>
struct TileLDS {
    static constexpr int W = TQ + 2, H = TR + 2, NS = W * H;
    typename Rec<T>::type rec[NS];
    uint8_t code[NS];
    T c[V ? NS : 1];
};

// Map ring index t (0 <= t < 2*(TQ+2) + 2*TR) to a halo slot (lq, lr) in
// staged coordinates (the tile's cells occupy lq in [1,TQ], lr in [1,TR]).
template <int TQ, int TR>
__device__ inline void ring_slot(int t, int &lq, int &lr) {
    constexpr int W = TQ + 2;
    if (t < W) { lq = t; lr = 0; }
    else if (t < 2 * W) { lq = t - W; lr = TR + 1; }
    else if (t < 2 * W + TR) { lq = 0; lr = 1 + (t - 2 * W); }
    else { lq = TQ + 1; lr = 1 + (t - 2 * W - TR); }
}

// Where a staged position lies: a cell of the tile, a raster cell reached
// through the halo (or a periodic wrap), or outside the raster.
enum : uint8_t { POS_OWN = 0, POS_NEIGHBOUR = 1, POS_OUTSIDE = 2 };

template <typename T, int TQ, int TR, int NT>
struct TileRegs {
    static constexpr int CPT = (TQ * TR) / NT;
    static constexpr int NRING = 2 * (TQ + 2) + 2 * TR;
    static constexpr int RPT = (NRING + NT - 1) / NT;
    static_assert(CPT * NT == TQ * TR, "tile must be a multiple of the workgroup");
    T h[CPT], th[CPT], ap[CPT], z[CPT], v1[CPT], v2[CPT];
    uint8_t pos[CPT];
    T rh[RPT], rth[RPT], rz[RPT], rv1[RPT], rv2[RPT];
    uint8_t rpos[RPT];
};

template <typename T>
__device__ inline typename Rec<T>::type make_rec(T m_or_M, T w, T vh1, T vh2) {
    typename Rec<T>::type r;
    r.x = m_or_M;
    r.y = w;
    r.z = vh1;
    r.w = vh2;
    return r;
}

template <typename T, bool NT_STORE>
__device__ inline void put(T *p, T v) {
    if constexpr (NT_STORE) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Per-thread accumulators of the step's reductions (c_max and FP64 books).
struct Acc {
    double c, s, o, cl;
};

__device__ inline bool tile_inner(const KGrid &g, int q0, int r0, int TQ, int TR) {
    return q0 >= 1 && q0 + TQ + 1 <= g.nq && r0 >= 1 && r0 + TR + 1 <= g.nr;
}

// ------------------------------------------------------------------ load

template <typename T, int TQ, int TR, int NT>
__device__ inline void tile_load(TileRegs<T, TQ, TR, NT> &R, const KDom<T> &d, const KGrid &g,
                                 int par, int tq, int tr) {
    using Regs = TileRegs<T, TQ, TR, NT>;
    const int q0 = tq * TQ, r0 = tr * TR;
    const T *__restrict__ hin = d.buf(par, 0);
    const T *__restrict__ v1in = d.buf(par, 1);
    const T *__restrict__ v2in = d.buf(par, 2);
    const bool inner = tile_inner(g, q0, r0, TQ, TR);
    // The state is read once per step.  Tiles 128 cells wide read their own cells with
    // streaming loads, which leave the L2 to the halo reads of neighbouring tiles; on
    // narrower tiles a larger share of each row is a neighbour's halo, and the ordinary
    // policy keeps those lines for it.
    constexpr bool STREAM = TQ >= 128;
#pragma unroll
    for (int k = 0; k < Regs::CPT; ++k) {
        const int cc = threadIdx.x + k * NT;
        const int lr = cc / TQ, lq = cc - lr * TQ;
        int q = q0 + lq, r = r0 + lr;
        uint8_t pos = POS_OWN;
        if (!(inner || (q < g.nq && r < g.nr)))
            pos = wrap_pos(g, q, r) ? POS_NEIGHBOUR : POS_OUTSIDE;
        R.pos[k] = pos;
        if (pos != POS_OUTSIDE) {
            const uint32_t i = (uint32_t)(r * g.pitch + q);
            // the static fields always use the ordinary cache policy
            R.h[k] = STREAM ? ld_stream(hin, i) : ld(hin, i);
            R.th[k] = ld(d.th, i);
            R.ap[k] = ld(d.ap, i);
            R.z[k] = ld(d.z, i);
            R.v1[k] = STREAM ? ld_stream(v1in, i) : ld(v1in, i);
            R.v2[k] = STREAM ? ld_stream(v2in, i) : ld(v2in, i);
        }
    }
#pragma unroll
    for (int k = 0; k < Regs::RPT; ++k) {
        const int t = threadIdx.x + k * NT;
        R.rpos[k] = POS_OUTSIDE;
        if (t < Regs::NRING) {
            int lq, lr;
            ring_slot<TQ, TR>(t, lq, lr);
            int q = q0 + lq - 1, r = r0 + lr - 1;
            if (inner || wrap_pos(g, q, r)) {
                R.rpos[k] = POS_NEIGHBOUR;
                const uint32_t i = (uint32_t)(r * g.pitch + q);
                R.rh[k] = ld(hin, i);
                R.rth[k] = ld(d.th, i);
                R.rz[k] = ld(d.z, i);
                R.rv1[k] = ld(v1in, i);
                R.rv2[k] = ld(v2in, i);
            }
        }
    }
}

// ----------------------------------------------------------------- stage

// Write the LDS records; returns true if a staged raster cell is inactive.
// EXT: the extended scheme: the raster may hold Dirichlet or given-flux cells
// (theta < 0), and the mass source may lose infiltration; the plain instance keeps
// the plain records and mass update.
template <typename T, int TQ, int TR, int NT, bool EXT = false, bool V>
__device__ inline bool tile_stage(TileLDS<T, TQ, TR, V> &L, const TileRegs<T, TQ, TR, NT> &R,
                                  const KGrid &g, const KConst &kc, int tq, int tr) {
    using Regs = TileRegs<T, TQ, TR, NT>;
    constexpr int W = TQ + 2;
    constexpr bool F32 = sizeof(T) == 4;
    const int q0 = tq * TQ, r0 = tr * TR;
    const bool inner = tile_inner(g, q0, r0, TQ, TR);
    const bool need_codes = !inner || g.has_mask;
    const T G = (T)kc.g;
    const T mscale = F32 ? (T)kc.a : T(1);
    bool bad = false;
#pragma unroll
    for (int k = 0; k < Regs::CPT; ++k) {
        const int cc = threadIdx.x + k * NT;
        const int lr = cc / TQ, lq = cc - lr * TQ;
        const int s = (lr + 1) * W + (lq + 1);
        if (R.pos[k] != POS_OUTSIDE) {
            const bool act = R.th[k] > T(0);
            if constexpr (EXT) {
                // boundary cells: Dirichlet (-theta: |theta| h) or given flux (-2: the
                // discharge's depth, and the bed only, as the edge adds the cell's depth)
                const bool fl = R.th[k] < T(-1.5);
                const T m = fl ? R.h[k] : __builtin_fabs(R.th[k]) * R.h[k];
                const T w = fl ? R.z[k] : G * (R.z[k] + R.h[k]);
                L.rec[s] = make_rec<T>(mscale * m, w, R.v1[k] * T(0.5), R.v2[k] * T(0.5));
                if (need_codes)
                    L.code[s] = act ? (uint8_t)CODE_INTERIOR
                                    : (fl ? (uint8_t)CODE_FLUX
                                          : R.th[k] < T(0) ? (uint8_t)CODE_DIRICHLET
                                                           : (uint8_t)g.mask_bc);
            } else {
                const T m = R.th[k] * R.h[k];
                L.rec[s] = make_rec<T>(mscale * m, G * (R.z[k] + R.h[k]), R.v1[k] * T(0.5),
                                       R.v2[k] * T(0.5));
                if (need_codes) L.code[s] = act ? (uint8_t)CODE_INTERIOR : (uint8_t)g.mask_bc;
            }
            if constexpr (V)
                L.c[s] = p_sqrt(R.v1[k] * R.v1[k] + R.v2[k] * R.v2[k]) + p_sqrt(G * R.h[k]);
            bad |= !act;
        } else {
            int q = q0 + lq, r = r0 + lr;
            wrap_pos(g, q, r);
            L.rec[s] = make_rec<T>(T(0), T(0), T(0), T(0));
            if constexpr (V) L.c[s] = T(0);
            L.code[s] = (uint8_t)side_code(g, q, r);
        }
    }
#pragma unroll
    for (int k = 0; k < Regs::RPT; ++k) {
        const int t = threadIdx.x + k * NT;
        if (t >= Regs::NRING) continue;
        int lq, lr;
        ring_slot<TQ, TR>(t, lq, lr);
        const int s = lr * W + lq;
        if (R.rpos[k] != POS_OUTSIDE) {
            const bool act = R.rth[k] > T(0);
            if constexpr (EXT) {
                const bool fl = R.rth[k] < T(-1.5);
                const T m = fl ? R.rh[k] : __builtin_fabs(R.rth[k]) * R.rh[k];
                const T w = fl ? R.rz[k] : G * (R.rz[k] + R.rh[k]);
                L.rec[s] = make_rec<T>(mscale * m, w, R.rv1[k] * T(0.5), R.rv2[k] * T(0.5));
                if (need_codes)
                    L.code[s] = act ? (uint8_t)CODE_INTERIOR
                                    : (fl ? (uint8_t)CODE_FLUX
                                          : R.rth[k] < T(0) ? (uint8_t)CODE_DIRICHLET
                                                            : (uint8_t)g.mask_bc);
            } else {
                const T m = R.rth[k] * R.rh[k];
                L.rec[s] = make_rec<T>(mscale * m, G * (R.rz[k] + R.rh[k]), R.rv1[k] * T(0.5),
                                       R.rv2[k] * T(0.5));
                if (need_codes) L.code[s] = act ? (uint8_t)CODE_INTERIOR : (uint8_t)g.mask_bc;
            }
            if constexpr (V)
                L.c[s] = p_sqrt(R.rv1[k] * R.rv1[k] + R.rv2[k] * R.rv2[k]) + p_sqrt(G * R.rh[k]);
            bad |= !act;
        } else {
            int q = q0 + lq - 1, r = r0 + lr - 1;
            wrap_pos(g, q, r);
            L.rec[s] = make_rec<T>(T(0), T(0), T(0), T(0));
            if constexpr (V) L.c[s] = T(0);
            L.code[s] = (uint8_t)side_code(g, q, r);
        }
    }
    return bad;
}

// --------------------------------------------------------------- compute

template <typename T, int TQ, int TR, int NT, bool NT_STORE, bool V, bool EXT = false>
__device__ inline void tile_compute(const TileLDS<T, TQ, TR, V> &L, const TileRegs<T, TQ, TR, NT> &R,
                                    bool general, const KDom<T> &d, const KGrid &g,
                                    const KConst &kc, int par, int tq, int tr, double dt,
                                    double r_next, Acc &acc, int32_t *err_flag,
                                    int32_t *err_cell) {
    using Regs = TileRegs<T, TQ, TR, NT>;
    constexpr int W = TQ + 2;
    constexpr bool F32 = sizeof(T) == 4;
    const int q0 = tq * TQ, r0 = tr * TR;
    T *__restrict__ hout = d.buf(par ^ 1, 0);
    T *__restrict__ v1out = d.buf(par ^ 1, 1);
    T *__restrict__ v2out = d.buf(par ^ 1, 2);
    const T G = (T)kc.g;
    const T mscale = F32 ? (T)kc.a : T(1);
    const T l = (T)kc.a;
    const T half_l = (T)(0.5 * kc.a);
    const T dtT = (T)dt;
    const T dts = (T)(dt / kc.sigma);
    const T rT = (T)r_next;
    const T alpha_s = (T)kc.alpha_s;
    // linear soil resistance theta tau h v, implicit in v^{n+1}: the coefficient of
    // v is m^{n+1} + dt tau m^{n+1} = m^{n+1} (1 + dt tau) (exactly m^{n+1} at tau = 0)
    const bool lin = kc.tau_lin != 0.0;
    const T ftau = T(1) + dtT * (T)kc.tau_lin;
    const T h_dry = (T)kc.h_dry;
    const T S3H = (T)0.86602540378443864676;
    const T NX[6] = {T(1), T(0.5), T(-0.5), T(-1), T(-0.5), T(0.5)};
    const T NY[6] = {T(0), S3H, S3H, T(0), -S3H, -S3H};
    const T NXh[6] = {T(0.5), T(0.25), T(-0.25), T(-0.5), T(-0.25), T(0.25)};
    const T NYh[6] = {T(0), T(0.5) * S3H, T(0.5) * S3H, T(0), -T(0.5) * S3H, -T(0.5) * S3H};
    constexpr int OFF[6] = {1, W, W - 1, -1, -W, -W + 1};

    float cmax32 = 0.f, m32 = 0.f;  // FP32 path: c_max and sum theta h of this thread's cells
    float wsum = 0.f;
    auto cell = [&](int k, auto gen_tag) {
        constexpr bool GEN = decltype(gen_tag)::value;
        const int cc = threadIdx.x + k * NT;
        const int lr = cc / TQ, lq = cc - lr * TQ;
        const int s = (lr + 1) * W + (lq + 1);
        const int q = q0 + lq, r = r0 + lr;
        const T hi = R.h[k], thi = R.th[k];
        const T mi = thi * hi;
        // the cell's own staged record (the values its neighbours see, formed by the same
        // operations), so that the bed register is free after staging; FP32 also takes
        // its velocity as twice the staged half, FP64 keeps the loaded one
        const typename Rec<T>::type me = L.rec[s];
        const T Mi = me.x, wi = me.y, vh1i = me.z, vh2i = me.w;
        T Ls = T(0), A1 = T(0), A2 = T(0), S1 = T(0), S2 = T(0), Fout = T(0);
        T V1 = T(0), V2 = T(0);  // viscous part of J^v (V only)
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            const int sn = s + OFF[e];
            T mj, wj, vh1j, vh2j;
            int cd = CODE_INTERIOR;
            if constexpr (GEN) {
                cd = L.code[sn];
                if (cd == CODE_WALL) continue;
            }
            // a cell: interior (or, EXT, a Dirichlet or flux cell)
            if (!GEN || (EXT ? cd != CODE_OUTFLOW : cd == CODE_INTERIOR)) {
                const typename Rec<T>::type nb = L.rec[sn];
                mj = nb.x;
                wj = nb.y;
                vh1j = nb.z;
                vh2j = nb.w;
            } else {
                // free outflow ghost: the cell's h, v, theta; terrain extrapolated linearly
                // through the opposite neighbour (read from memory: rim cells only)
                wj = wi;
                if (L.code[s - OFF[e]] == CODE_INTERIOR) {
                    int qo = q - dq_of(e), ro = r - dr_of(e);
                    wrap_pos(g, qo, ro);
                    const T zi = ld(d.z, (uint32_t)(r * g.pitch + q));
                    const T zg = T(2) * zi - d.z[(int64_t)ro * g.pitch + qo];
                    wj = G * (zg + hi);
                }
                mj = Mi;
                vh1j = vh1i;
                vh2j = vh2i;
            }
            // interface velocity; an edge to a Dirichlet or flux cell carries the prescribed one
            T vb1 = vh1i + vh1j;
            T vb2 = vh2i + vh2j;
            if (EXT && GEN && cd >= CODE_DIRICHLET) {
                vb1 = vh1j + vh1j;
                vb2 = vh2j + vh2j;
            }
            if (EXT && GEN && cd == CODE_FLUX) {
                // given mass flux: the discharge h_j v_j crosses the edge whatever the cell
                // holds; the pressure term sees the cell's own depth over the neighbour's
                // bed (wj holds that bed level)
                const T vn = vb1 * NX[e] + vb2 * NY[e];
                if constexpr (F32) {
                    const T F = mj * vn;  // mj holds l h_j
                    Ls -= F;
                    A1 -= F * vb1;
                    A2 -= F * vb2;
                    const T Q = (G * (wj + hi) - wi) * Mi;
                    A1 -= Q * NXh[e];
                    A2 -= Q * NYh[e];
                    Fout += F;
                } else {
                    const T F = l * mj * vn;
                    Ls -= F;
                    A1 -= F * vb1;
                    A2 -= F * vb2;
                    const T P = half_l * (G * (wj + hi) - wi) * mi;
                    S1 -= P * NX[e];
                    S2 -= P * NY[e];
                    Fout += F;
                }
                continue;
            }
            if constexpr (F32) {
                // mj holds l*theta_j*h_j
                const T vn = (e == 0) ? vb1 : ((e == 3) ? -vb1 : vb1 * NX[e] + vb2 * NY[e]);
                const T dw = wj - wi;
                // one selected mass serves both terms: the upwind mass of the flux
                // (at vn = 0 the flux vanishes whatever it is) and the pressure mass,
                // which at vn = 0 follows the free-surface tie rule
                const T key = (vn != T(0)) ? vn : -dw;  // w_i > w_j decides at vn = 0
                const T msel = key > T(0) ? Mi : mj;
                const T F = msel * vn;
                Ls -= F;
                A1 -= F * vb1;
                A2 -= F * vb2;
                const T Q = dw * msel;
                A1 -= Q * NXh[e];
                if (e != 0 && e != 3) A2 -= Q * NYh[e];
                if (GEN && (EXT ? cd != CODE_INTERIOR : cd == CODE_OUTFLOW))
                    Fout += F;  // outflow or Dirichlet edge
            } else {
                const T vn = vb1 * NX[e] + vb2 * NY[e];
                const T mup = vn > T(0) ? mi : (vn < T(0) ? mj : T(0));
                const T mhat = vn != T(0) ? mup : (wi > wj ? mi : mj);
                const T F = l * mup * vn;
                Ls -= F;
                A1 -= F * vb1;
                A2 -= F * vb2;
                const T P = half_l * (wj - wi) * mhat;
                S1 -= P * NX[e];
                S2 -= P * NY[e];
                if (GEN && (EXT ? cd != CODE_INTERIOR : cd == CODE_OUTFLOW))
                    Fout += F;  // outflow or Dirichlet edge
            }
            if constexpr (V) {
                // artificial viscosity l c_ij mu_ij (v_j - v_i) of an interior edge (an
                // outflow ghost carries the cell's own velocity); (v_j - v_i) is twice the
                // difference of the staged halves, exactly.  FP32 masses carry the l.
                if (!GEN || cd == CODE_INTERIOR) {
                    const T ci = L.c[s], cj = L.c[sn];
                    const T cij = ci > cj ? ci : cj;
                    const T ms = Mi + mj;
                    const T mu = ms > T(0) ? p_div(T(2) * Mi * mj, ms) : T(0);
                    const T lc = F32 ? cij : l * cij;
                    V1 += lc * mu * (T(2) * (vh1j - vh1i));
                    V2 += lc * mu * (T(2) * (vh2j - vh2i));
                }
            }
        }
        const T v1i = F32 ? vh1i + vh1i : R.v1[k], v2i = F32 ? vh2i + vh2i : R.v2[k];
        T m1, h1, g1, g2;
        if constexpr (F32) {
            const T dm = dts * Ls + dtT * rT;
            m1 = mi + dm;
            if (m1 < T(0)) {
                acc.cl += kc.sigma * (-(double)m1);
                m1 = T(0);
                h1 = T(0);
            } else {
                h1 = hi + p_div(dm, thi);
                h1 = h1 > T(0) ? h1 : T(0);
            }
            if constexpr (V) {
                g1 = mi * v1i + dts * (A1 + V1);
                g2 = mi * v2i + dts * (A2 + V2);
            } else {
                g1 = mi * v1i + dts * A1;
                g2 = mi * v2i + dts * A2;
            }
        } else {
            const T ms = mi + dts * Ls;
            m1 = ms + dtT * rT;
            if (m1 < T(0)) {
                acc.cl += kc.sigma * (-(double)m1);
                m1 = T(0);
            }
            h1 = p_div(m1, thi);
            if constexpr (V) {  // J^v = J + viscous sums, then the pressure part
                g1 = mi * v1i + dts * ((A1 + V1) + S1);
                g2 = mi * v2i + dts * ((A2 + V2) + S2);
            } else {
                g1 = mi * v1i + dts * (A1 + S1);
                g2 = mi * v2i + dts * (A2 + S2);
            }
        }
        if constexpr (EXT) {
            if (kc.f_inf > 0.0 && m1 > T(0)) {
                // the mass source r - i(h^{n+1}) with i(h) = f h / (h + c) turns the mass
                // update into theta x + dt f x / (x + c) = m1 for x = h^{n+1}.  With
                // x = h1 - e (h1: the depth without infiltration, which FP32 keeps as an
                // increment) the loss e is the smaller root of theta e^2 - P e + dt f h1,
                // P = theta (h1 + c) + dt f; the soil's water is booked with the outflow
                const T c = (T)kc.h_inf, fd = dtT * (T)kc.f_inf, hs = h1;
                const T P = thi * (hs + c) + fd;
                const T Q = thi * (hs + c) - fd;
                const T Dq = Q * Q + T(4) * thi * fd * c;
                const T e = p_div(T(2) * fd * hs, P + p_sqrt(Dq));
                const T x = hs - e;
                const T mx = thi * x;
                acc.o += kc.sigma * (double)(m1 - mx);
                m1 = mx;
                h1 = x;
            }
        }
        const uint32_t i = (uint32_t)(r * g.pitch + q);
        T as_i = alpha_s;
        if constexpr (EXT) {
            if (d.as) as_i = ld(d.as, i);  // a soil coefficient per cell
        }
        const T K = R.ap[k] * h1 * (T(1) - thi) + thi * as_i;
        const T beta = dtT * K;
        const T Gm = p_sqrt(g1 * g1 + g2 * g2);
        T alpha = m1;
        if (lin) alpha = m1 * ftau;
        const T D = alpha + p_sqrt(alpha * alpha + T(4) * beta * Gm);
        T mu = (D == T(0)) ? T(0) : p_div(T(2), D);
        if (h_dry > T(0) && h1 < h_dry) mu = T(0);
        const T v1n = mu * g1, v2n = mu * g2;
        put<T, NT_STORE>(at(hout, i), h1);
        put<T, NT_STORE>(at(v1out, i), v1n);
        put<T, NT_STORE>(at(v2out, i), v2n);
        // wave speed of the new state (eq. fvm_2D_eq_frac.13); FP32 takes |v^{n+1}| as
        // mu |gamma| (the same value up to rounding), FP64 the oracle's sqrt(v1^2 + v2^2)
        const T vabs = F32 ? mu * Gm : p_sqrt(v1n * v1n + v2n * v2n);
        const T cc2 = vabs + p_sqrt(G * h1);
        if constexpr (F32) {
            // FP32 partials over this thread's cells, folded into the FP64 books below;
            // wsum carries any non-finite h or v of the thread's cells to one check
            cmax32 = cc2 > cmax32 ? cc2 : cmax32;
            m32 += thi * h1;
            wsum += cc2;
        } else {
            acc.c = (double)cc2 > acc.c ? (double)cc2 : acc.c;
            acc.s += kc.sigma * ((double)thi * (double)h1);
            if (!__builtin_isfinite(h1) || !__builtin_isfinite(v1n) || !__builtin_isfinite(v2n)) {
                if (atomicOr(err_flag, 1) == 0) *err_cell = (int32_t)i;
            }
        }
        if (GEN) acc.o += dt * (double)Fout;
    };

    if (general) {
#pragma unroll
        for (int k = 0; k < Regs::CPT; ++k)
            if (R.pos[k] == POS_OWN && R.th[k] > T(0)) cell(k, std::true_type{});
    } else {
#pragma unroll
        for (int k = 0; k < Regs::CPT; ++k) cell(k, std::false_type{});
    }
    if constexpr (F32) {
        acc.c = (double)cmax32 > acc.c ? (double)cmax32 : acc.c;
        acc.s += kc.sigma * (double)m32;
        if (!__builtin_isfinite(m32 + wsum)) {
            // rare: find the offending cell among the values this thread just stored
#pragma unroll
            for (int k = 0; k < Regs::CPT; ++k) {
                if (R.pos[k] != POS_OWN) continue;
                const int cc = threadIdx.x + k * NT;
                const int lr = cc / TQ, lq = cc - lr * TQ;
                const uint32_t i = (uint32_t)((r0 + lr) * g.pitch + q0 + lq);
                if (!__builtin_isfinite(ld(hout, i)) || !__builtin_isfinite(ld(v1out, i)) ||
                    !__builtin_isfinite(ld(v2out, i))) {
                    if (atomicOr(err_flag, 1) == 0) *err_cell = (int32_t)i;
                }
            }
        }
    }
}

// All three phases for one tile (the caller separates consecutive tiles on
// the same LDS with a barrier).
template <typename T, int TQ, int TR, int NT, bool NT_STORE, bool V = false, bool EXT = false>
__device__ inline void tile_step(TileLDS<T, TQ, TR, V> &L, const KDom<T> &d, const KGrid &g,
                                 const KConst &kc, int par, int tq, int tr, double dt,
                                 double r_next, Acc &acc, int32_t *err_flag, int32_t *err_cell) {
    TileRegs<T, TQ, TR, NT> R;
    tile_load<T, TQ, TR, NT>(R, d, g, par, tq, tr);
    const bool bad = tile_stage<T, TQ, TR, NT, EXT>(L, R, g, kc, tq, tr);
    const bool inner = tile_inner(g, tq * TQ, tr * TR, TQ, TR);
    const bool general = __syncthreads_or((!inner) || bad) != 0;
    tile_compute<T, TQ, TR, NT, NT_STORE, V, EXT>(L, R, general, d, g, kc, par, tq, tr, dt, r_next,
                                             acc, err_flag, err_cell);
}

}  // namespace hexsv
