// hexsv_tile.h — one explicit step of one TQ x TR tile of the raster.
//
// Staging: every thread loads the (h, v1, v2, z, theta, alpha_p) of the cells
// it owns (coalesced rows of the tile) and one-cell halo slots along the tile
// rim, and writes a 4-word record per staged position to LDS:
//   {mass, w = g (z + h), v1/2, v2/2}
// with mass = theta*h (FP64) or l*theta*h (FP32).  Interface velocities of
// eq. fvm_2D_eq.04 are then a single add (v_i/2 + v_j/2 equals
// (v_i + v_j)/2 exactly), and each neighbour is one 16-byte LDS read.
//
// Tiles whose halo lies inside the raster and holds no inactive cell take
// the interior path (no edge codes); the others read an edge code per staged
// position (INTERIOR, WALL, OUTFLOW).
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

template <typename T, int TQ, int TR>
struct TileLDS {
    static constexpr int W = TQ + 2, H = TR + 2, NS = W * H;
    typename Rec<T>::type rec[NS];
    uint8_t code[NS];
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

template <typename T>
struct CellRegs {
    T h, th, ap, z, m, w, vh1, vh2;
    bool ok;
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

// Advance tile (tq, tr) by one step: reads state buffer `par`, writes par^1.
// Returns the tile's partial record in thread 0.
template <typename T, int TQ, int TR, int NT, bool NT_STORE>
__device__ inline Part tile_step(TileLDS<T, TQ, TR> &L, const KDom<T> &d, const KGrid &g,
                                 const KConst &kc, int par, int tq, int tr, double dt,
                                 double r_next, int32_t *err_flag, int32_t *err_cell) {
    constexpr int W = TQ + 2;
    constexpr int CPT = (TQ * TR) / NT;
    static_assert(CPT * NT == TQ * TR, "tile must be a multiple of the workgroup");
    constexpr int NRING = 2 * (TQ + 2) + 2 * TR;
    const int q0 = tq * TQ, r0 = tr * TR;
    const T *__restrict__ hin = d.st[par][0];
    const T *__restrict__ v1in = d.st[par][1];
    const T *__restrict__ v2in = d.st[par][2];
    T *__restrict__ hout = d.st[par ^ 1][0];
    T *__restrict__ v1out = d.st[par ^ 1][1];
    T *__restrict__ v2out = d.st[par ^ 1][2];
    const T G = (T)kc.g;
    constexpr bool F32 = sizeof(T) == 4;
    // FP32 stages l*theta*h; FP64 stages theta*h
    const T mscale = F32 ? (T)kc.a : T(1);

    const bool inner = q0 >= 1 && q0 + TQ + 1 <= g.nq && r0 >= 1 && r0 + TR + 1 <= g.nr;
    const bool need_codes = !inner || g.has_mask;
    bool bad = false;

    // ---- stage owned cells (positions past the raster edge of a ragged tile
    //      are staged like halo slots: wrapped neighbour or boundary code)
    CellRegs<T> c[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        const int cc = threadIdx.x + k * NT;
        const int lr = cc / TQ, lq = cc - lr * TQ;
        int q = q0 + lq, r = r0 + lr;
        const int s = (lr + 1) * W + (lq + 1);
        c[k].ok = false;
        if (q < g.nq && r < g.nr) {
            const int64_t i = (int64_t)r * g.nq + q;
            c[k].h = hin[i];
            c[k].th = d.th[i];
            c[k].ap = d.ap[i];
            c[k].z = d.z[i];
            const T v1 = v1in[i], v2 = v2in[i];
            c[k].m = c[k].th * c[k].h;
            c[k].w = G * (c[k].z + c[k].h);
            c[k].vh1 = v1 * T(0.5);
            c[k].vh2 = v2 * T(0.5);
            L.rec[s] = make_rec<T>(mscale * c[k].m, c[k].w, c[k].vh1, c[k].vh2);
            const bool act = c[k].th > T(0);
            c[k].ok = act;
            bad |= !act;
            if (need_codes) L.code[s] = act ? (uint8_t)CODE_INTERIOR : (uint8_t)g.mask_bc;
        } else if (wrap_pos(g, q, r)) {
            const int64_t i = (int64_t)r * g.nq + q;
            const T h = hin[i], th = d.th[i], z = d.z[i];
            L.rec[s] = make_rec<T>(mscale * (th * h), G * (z + h), v1in[i] * T(0.5),
                                   v2in[i] * T(0.5));
            L.code[s] = th > T(0) ? (uint8_t)CODE_INTERIOR : (uint8_t)g.mask_bc;
        } else {
            L.rec[s] = make_rec<T>(T(0), T(0), T(0), T(0));
            L.code[s] = (uint8_t)side_code(g, q, r);
        }
    }
    // ---- stage the halo ring
    for (int t = threadIdx.x; t < NRING; t += NT) {
        int lq, lr;
        ring_slot<TQ, TR>(t, lq, lr);
        int q = q0 + lq - 1, r = r0 + lr - 1;
        const int s = lr * W + lq;
        const bool in = inner ? true : wrap_pos(g, q, r);
        if (in) {
            const int64_t i = (int64_t)r * g.nq + q;
            const T h = hin[i], th = d.th[i], z = d.z[i];
            L.rec[s] = make_rec<T>(mscale * (th * h), G * (z + h), v1in[i] * T(0.5),
                                   v2in[i] * T(0.5));
            const bool act = th > T(0);
            bad |= !act;
            if (need_codes) L.code[s] = act ? (uint8_t)CODE_INTERIOR : (uint8_t)g.mask_bc;
        } else {
            L.rec[s] = make_rec<T>(T(0), T(0), T(0), T(0));
            L.code[s] = (uint8_t)side_code(g, q, r);
        }
    }
    const bool general = __syncthreads_or((!inner) || bad) != 0;

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
    const T NXh[6] = {T(0.5), T(0.25), T(-0.25), T(-0.5), T(-0.25), T(0.25)};
    const T NYh[6] = {T(0), T(0.5) * S3H, T(0.5) * S3H, T(0), -T(0.5) * S3H, -T(0.5) * S3H};
    constexpr int OFF[6] = {1, W, W - 1, -1, -W, -W + 1};

    double c_loc = 0.0, s_loc = 0.0, o_loc = 0.0, cl_loc = 0.0;

    auto cell = [&](const CellRegs<T> &cr, int lq, int lr, auto gen_tag) {
        constexpr bool GEN = decltype(gen_tag)::value;
        const int s = (lr + 1) * W + (lq + 1);
        const int q = q0 + lq, r = r0 + lr;
        const T mi = cr.m, wi = cr.w, vh1i = cr.vh1, vh2i = cr.vh2;
        const T Mi = mscale * mi;
        T Ls = T(0), A1 = T(0), A2 = T(0), S1 = T(0), S2 = T(0), Fout = T(0);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int sn = s + OFF[k];
            T mj, wj, vh1j, vh2j;
            int cd = CODE_INTERIOR;
            if constexpr (GEN) {
                cd = L.code[sn];
                if (cd == CODE_WALL) continue;
            }
            if (!GEN || cd == CODE_INTERIOR) {
                const typename Rec<T>::type nb = L.rec[sn];
                mj = nb.x;
                wj = nb.y;
                vh1j = nb.z;
                vh2j = nb.w;
            } else {
                // free outflow ghost: the cell's h, v, theta; terrain extrapolated linearly
                // through the opposite neighbour (read from memory: rim cells only)
                T zg = cr.z;
                if (L.code[s - OFF[k]] == CODE_INTERIOR) {
                    int qo = q - dq_of(k), ro = r - dr_of(k);
                    wrap_pos(g, qo, ro);
                    zg = T(2) * cr.z - d.z[(int64_t)ro * g.nq + qo];
                }
                mj = Mi;
                wj = G * (zg + cr.h);
                vh1j = vh1i;
                vh2j = vh2i;
            }
            const T vb1 = vh1i + vh1j;
            const T vb2 = vh2i + vh2j;
            if constexpr (F32) {
                // mj holds l*theta_j*h_j
                const T vn = (k == 0) ? vb1 : ((k == 3) ? -vb1 : vb1 * NX[k] + vb2 * NY[k]);
                const bool up = vn > T(0);
                const T F = (up ? Mi : mj) * vn;
                Ls -= F;
                A1 -= F * vb1;
                A2 -= F * vb2;
                const T dw = wj - wi;
                const bool take_i = up || (vn == T(0) && dw < T(0));
                const T Q = dw * (take_i ? Mi : mj);
                A1 -= Q * NXh[k];
                if (k != 0 && k != 3) A2 -= Q * NYh[k];
                if (GEN && cd == CODE_OUTFLOW) Fout += F;
            } else {
                const T vn = vb1 * NX[k] + vb2 * NY[k];
                const T mup = vn > T(0) ? mi : (vn < T(0) ? mj : T(0));
                const T mhat = vn != T(0) ? mup : (wi > wj ? mi : mj);
                const T F = l * mup * vn;
                Ls -= F;
                A1 -= F * vb1;
                A2 -= F * vb2;
                const T P = half_l * (wj - wi) * mhat;
                S1 -= P * NX[k];
                S2 -= P * NY[k];
                if (GEN && cd == CODE_OUTFLOW) Fout += F;
            }
        }
        const T thi = cr.th, hi = cr.h;
        const T v1i = vh1i * T(2), v2i = vh2i * T(2);
        T m1, h1, g1, g2;
        if constexpr (F32) {
            const T dm = dts * Ls + dtT * rT;
            m1 = mi + dm;
            if (m1 < T(0)) {
                cl_loc += kc.sigma * (-(double)m1);
                m1 = T(0);
                h1 = T(0);
            } else {
                h1 = hi + p_div(dm, thi);
                h1 = h1 > T(0) ? h1 : T(0);
            }
            g1 = mi * v1i + dts * A1;
            g2 = mi * v2i + dts * A2;
        } else {
            const T ms = mi + dts * Ls;
            m1 = ms + dtT * rT;
            if (m1 < T(0)) {
                cl_loc += kc.sigma * (-(double)m1);
                m1 = T(0);
            }
            h1 = p_div(m1, thi);
            g1 = mi * v1i + dts * (A1 + S1);
            g2 = mi * v2i + dts * (A2 + S2);
        }
        const T K = cr.ap * h1 * (T(1) - thi) + thi * alpha_s;
        const T beta = dtT * K;
        const T Gm = p_sqrt(g1 * g1 + g2 * g2);
        const T D = m1 + p_sqrt(m1 * m1 + T(4) * beta * Gm);
        T mu = (D == T(0)) ? T(0) : p_div(T(2), D);
        if (h_dry > T(0) && h1 < h_dry) mu = T(0);
        const T v1n = mu * g1, v2n = mu * g2;
        const int64_t i = (int64_t)r * g.nq + q;
        put<T, NT_STORE>(hout + i, h1);
        put<T, NT_STORE>(v1out + i, v1n);
        put<T, NT_STORE>(v2out + i, v2n);
        const T cc = p_sqrt(v1n * v1n + v2n * v2n) + p_sqrt(G * h1);
        c_loc = (double)cc > c_loc ? (double)cc : c_loc;
        s_loc += kc.sigma * ((double)thi * (double)h1);
        if (GEN) o_loc += dt * (double)Fout;
        if (!__builtin_isfinite(h1) || !__builtin_isfinite(v1n) || !__builtin_isfinite(v2n)) {
            if (atomicOr(err_flag, 1) == 0) *err_cell = (int32_t)i;
        }
    };

    if (general) {
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int cc = threadIdx.x + k * NT;
            const int lr = cc / TQ, lq = cc - lr * TQ;
            if (c[k].ok) cell(c[k], lq, lr, std::true_type{});
        }
    } else {
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int cc = threadIdx.x + k * NT;
            const int lr = cc / TQ, lq = cc - lr * TQ;
            cell(c[k], lq, lr, std::false_type{});
        }
    }
    return block_reduce<NT>(c_loc, s_loc, o_loc, cl_loc);
}

}  // namespace hexsv
