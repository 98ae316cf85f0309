// hexsv_nn.hip — kernels of the learned hex-convolution surrogate: BF16 MFMA
// forward / data-gradient / weight-gradient hex convolutions with FP32
// accumulation (the tile's staging and MFMA mapping are in hexsv_conv.h), the
// fused 4-layer forward, the L1 loss, Adam, and the weight-layout preparation.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hexsv_conv.h"
#include "hexsv_device.h"
#include "hexsv_nn.h"

namespace hexsv {
namespace nn {

// ---------------------------------------------------------------- conv

// out[i][co] for the tile; EPI selects the epilogue:
//   EPI_RELU:  bf16 out = max(acc + b, 0)           (hidden layers, forward)
//   EPI_LIN:   f32 out[i][co < cout_real] = acc + b  (last layer, forward)
//   EPI_MASK:  bf16 out = acc * (mask[i][co] > 0)    (data gradient through ReLU)
template <int CIN, int COUT, int EPI>
__global__ __launch_bounds__(NT) void k_hexconv(const __bf16 *__restrict__ x,
                                                const __bf16 *__restrict__ wm,
                                                const float *__restrict__ bias, void *out,
                                                const __bf16 *__restrict__ mask, int nq, int nr,
                                                int ntiles_total, int cout_real,
                                                const int32_t *live, ConvMask cm) {
    constexpr int CH = CIN / 8;
    constexpr int MB = COUT / 16;                 // output-channel blocks
    __shared__ uint4 lds[NSLOT * CH];
    __shared__ uint8_t fl[NSLOT];
    const int ntq = (nq + TQ - 1) / TQ, ntr = (nr + TR - 1) / TR;
    // XCD-banded tile order: every layer gives a tile to the same XCD, so the
    // activations a layer writes are mostly read back from that XCD's L2
    const int tile = xcd_tile(blockIdx.x, gridDim.x, ntiles_total, 0);
    if (tile < 0) return;
    if (live && !*live) return;  // a surrogate window that does not run
    int b, q0, r0;
    tile_of(tile, ntq, ntr, b, q0, r0);
    const int64_t soff = (int64_t)b * nq * nr;
    stage_act<CIN>(lds, fl, x, nq, nr, soff, q0, r0, cm);
    __syncthreads();
    const bool masked = cm.active != nullptr;

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;  // wave w: tile row w
    const int g = lane >> 4, l16 = lane & 15;
    f32x4 acc[MB][4];
    conv_acc<CIN, COUT>(lds, fl, masked, wm, acc);
    // epilogue: lane holds channels co = m*16 + 4g + j of cell n*16 + l16
    const int r = r0 + w;
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const int q = q0 + n * 16 + l16;
        if (q >= nq || r >= nr) continue;
        const int64_t i = soff + (int64_t)r * nq + q;
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            const int co = m * 16 + 4 * g;
            float v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = acc[m][n][j];
            if constexpr (EPI == EPI_RELU || EPI == EPI_LIN) {
#pragma unroll
                for (int j = 0; j < 4; ++j) v[j] += bias[co + j];
            }
            if constexpr (EPI == EPI_LIN) {
                float *o = reinterpret_cast<float *>(out) + i * OUT_STRIDE;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (co + j < cout_real) o[co + j] = v[j];
            } else {
                if constexpr (EPI == EPI_RELU) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) v[j] = v[j] > 0.f ? v[j] : 0.f;
                }
                if constexpr (EPI == EPI_MASK) {
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (!((float)mask[i * COUT + co + j] > 0.f)) v[j] = 0.f;
                }
                __bf16 *o = reinterpret_cast<__bf16 *>(out) + i * COUT + co;
                typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
                bf16x4 pk;
#pragma unroll
                for (int j = 0; j < 4; ++j) pk[j] = (__bf16)v[j];
                *reinterpret_cast<bf16x4 *>(o) = pk;
            }
        }
    }
}

// ------------------------------------------------------- fused 4-layer forward
//
// The whole 4-layer network (16 -> 32 -> 32 -> 32 -> 16 channels) for a 16 x 16
// tile of output cells in one workgroup.  The packed input features of the tile
// and a 4-cell margin (24 x 24 positions) are staged once; layer l is evaluated on
// the tile grown by 3 - l cells on each side and its activations stay in LDS for
// layer l + 1, so hidden activations never leave the CU.  Each layer's arithmetic
// is that of k_hexconv (the same MFMA, the same K order, bias and ReLU, the same
// bf16 rounding of hidden activations), so the output equals the layer-by-layer
// chain's bit for bit.  fl[p] is 1 where staged position p holds a cell of the
// domain (wrapped through periodic sides); a tap t >= 1 reads its neighbour only
// when the centre and the neighbour both are, which also zeroes every position
// outside the raster, as the chain's zero staging does.
namespace f4 {
constexpr int OT = 16;        // output tile edge
constexpr int WI = OT + 8;    // staged input frame edge (margin 4)
constexpr int NG = 4;         // 16-cell column groups per wave pass
}

// One layer over a WO x WO frame.  taps_all: every staged position of the tile is
// a domain cell (an interior tile of an unmasked raster), so no tap is cut.
// SSTR: 16-byte chunks between consecutive source cells; DSTR: bf16 values
// between consecutive destination cells (hidden activations are padded from 64
// to 80 bytes per cell, so that the 16 cells of an MFMA column fall on distinct
// LDS banks when gathered and when written).
template <int CIN, int COUT, int EPI, int WO, int SSTR, int DSTR>
__device__ inline void net_layer(const uint4 *src, uint4 *dst, const uint8_t *fl,
                                 const __bf16 *__restrict__ wm, const float *__restrict__ bias,
                                 float *__restrict__ out, int nq, int nr, int64_t soff, int q0,
                                 int r0, int cout_real, bool taps_all) {
    using namespace f4;
    constexpr int CH = CIN / 8;            // 16-byte chunks per source cell
    constexpr int MB = COUT / 16;
    constexpr int TPK = 32 / CIN;
    constexpr int KSTEPS = (7 + TPK - 1) / TPK;
    constexpr int WS = WO + 2;             // source frame edge
    constexpr int OI = (WI - WO) / 2;      // this frame's origin in the staged frame
    constexpr int NCELL = WO * WO;
    constexpr int NGRP = (NCELL + 15) / 16;
    constexpr int NCHUNK = (NGRP + NG - 1) / NG;
    constexpr int OFF_S[7] = {0, 1, WS, WS - 1, -1, -WS, -WS + 1};
    constexpr int OFF_I[7] = {0, 1, WI, WI - 1, -1, -WI, -WI + 1};
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane >> 4, l16 = lane & 15;
    // this lane's weight fragments for every K step, loaded once per layer
    bf16x8 av[KSTEPS][MB];
#pragma unroll
    for (int ks = 0; ks < KSTEPS; ++ks) {
        const int tap = ks * TPK + g / CH;
        const int c0 = (g % CH) * 8;
#pragma unroll
        for (int m = 0; m < MB; ++m)
            av[ks][m] = tap < 7 ? *reinterpret_cast<const bf16x8 *>(
                                      wm + ((int64_t)(tap * COUT + m * 16 + l16)) * CIN + c0)
                                : bf16x8{};
    }
    for (int chunk = w; chunk < NCHUNK; chunk += 4) {
        f32x4 acc[MB][NG];
        int sslot[NG], islot[NG], cell[NG];
#pragma unroll
        for (int n = 0; n < NG; ++n) {
#pragma unroll
            for (int m = 0; m < MB; ++m) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
            int c = (chunk * NG + n) * 16 + l16;
            cell[n] = c;
            c = c < NCELL ? c : NCELL - 1;  // lanes past the frame compute a copy, never stored
            const int b = c / WO, a = c - b * WO;
            sslot[n] = (b + 1) * WS + (a + 1);
            islot[n] = (b + OI) * WI + (a + OI);
        }
#pragma unroll
        for (int ks = 0; ks < KSTEPS; ++ks) {
            const int tap = ks * TPK + g / CH;
            const int c0 = (g % CH) * 8;
#pragma unroll
            for (int n = 0; n < NG; ++n) {
                if ((chunk * NG + n) >= NGRP) break;  // uniform over the wave
                bf16x8 bv = bf16x8{};
                if (tap < 7) {
                    uint4 raw = src[(sslot[n] + OFF_S[tap]) * SSTR + c0 / 8];
                    if (!taps_all && tap > 0 && !(fl[islot[n]] & fl[islot[n] + OFF_I[tap]]))
                        raw = make_uint4(0u, 0u, 0u, 0u);
                    bv = *reinterpret_cast<const bf16x8 *>(&raw);
                }
#pragma unroll
                for (int m = 0; m < MB; ++m)
                    acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[ks][m], bv, acc[m][n], 0, 0, 0);
            }
        }
        // epilogue: lane holds channels co = m*16 + 4g + j of cell[n]
#pragma unroll
        for (int n = 0; n < NG; ++n) {
            const int c = cell[n];
            if ((chunk * NG + n) >= NGRP || c >= NCELL) continue;
            const int b = c / WO, a = c - b * WO;
#pragma unroll
            for (int m = 0; m < MB; ++m) {
                const int co = m * 16 + 4 * g;
                float v[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) v[j] = acc[m][n][j] + bias[co + j];
                if constexpr (EPI == EPI_LIN) {
                    const int q = q0 + a, r = r0 + b;
                    if (q < nq && r < nr) {
                        float *o = out + (soff + (int64_t)r * nq + q) * OUT_STRIDE;
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            if (co + j < cout_real) o[co + j] = v[j];
                    }
                } else {
                    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
                    bf16x4 pk;
#pragma unroll
                    for (int j = 0; j < 4; ++j) pk[j] = (__bf16)(v[j] > 0.f ? v[j] : 0.f);
                    *reinterpret_cast<bf16x4 *>(reinterpret_cast<__bf16 *>(dst) + c * DSTR + co) = pk;
                }
            }
        }
    }
}

__global__ __launch_bounds__(NT) void k_hexnet4(const __bf16 *__restrict__ x, Net4 nw,
                                                float *__restrict__ out, int nq, int nr,
                                                int ntiles_total, int cout_real,
                                                const int32_t *live, ConvMask cm) {
    using namespace f4;
    constexpr int W0 = OT + 6, W1 = OT + 4;
    constexpr int AS = 5;  // 16-byte chunks per cell of hidden activations (32 channels + pad)
    __shared__ uint4 bufA[W0 * W0 * AS];  // layer 0 and layer 2 activations
    __shared__ uint4 bufB[W1 * W1 * AS];  // the staged input (16 channels), then layer 1
    __shared__ uint8_t fl[WI * WI];
    static_assert(WI * WI * 2 <= W1 * W1 * AS, "staged input fits the layer-1 buffer");
    const int ntq = (nq + OT - 1) / OT, ntr = (nr + OT - 1) / OT;
    const int tile = xcd_tile(blockIdx.x, gridDim.x, ntiles_total, 0);
    if (tile < 0) return;
    if (live && !*live) return;  // a surrogate window that does not run
    const int per = ntq * ntr;
    const int bs = tile / per, lt = tile - bs * per;
    const int tr = lt / ntq;
    const int q0 = (lt - tr * ntq) * OT, r0 = tr * OT;
    const int64_t soff = (int64_t)bs * nq * nr;
    // stage the 24 x 24 input frame: two 16-byte chunks per position, loads first
    constexpr int NE = WI * WI * 2;
    constexpr int ITERS = (NE + NT - 1) / NT;
    uint4 v[ITERS];
    uint8_t a[ITERS];
#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
        const int e = threadIdx.x + it * NT;
        const int p = e >> 1, ch = e & 1;
        const int pb = p / WI, pa = p - pb * WI;
        int q = q0 - 4 + pa, r = r0 - 4 + pb;
        if (cm.perq) q = ((q % nq) + nq) % nq;
        if (cm.perr) r = ((r % nr) + nr) % nr;
        v[it] = make_uint4(0u, 0u, 0u, 0u);
        a[it] = 0;
        if (e < NE && q >= 0 && q < nq && r >= 0 && r < nr) {
            const int64_t i = soff + (int64_t)r * nq + q;
            v[it] = reinterpret_cast<const uint4 *>(x + i * FEATURES_PAD)[ch];
            a[it] = cm.active ? (uint8_t)(cm.active[(int64_t)r * nq + q] != 0) : (uint8_t)1;
        }
    }
#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
        const int e = threadIdx.x + it * NT;
        if (e < NE) {
            bufB[e] = v[it];
            if ((e & 1) == 0) fl[e >> 1] = a[it];
        }
    }
    __syncthreads();
    // the staged frame lies inside an unmasked raster: no tap is cut
    const bool all = !cm.active && q0 >= 4 && q0 + OT + 4 <= nq && r0 >= 4 && r0 + OT + 4 <= nr;
    net_layer<16, 32, EPI_RELU, OT + 6, 2, 8 * AS>(bufB, bufA, fl, nw.wm[0], nw.bias[0], nullptr,
                                                   nq, nr, soff, q0, r0, 32, all);
    __syncthreads();
    net_layer<32, 32, EPI_RELU, OT + 4, AS, 8 * AS>(bufA, bufB, fl, nw.wm[1], nw.bias[1], nullptr,
                                                    nq, nr, soff, q0, r0, 32, all);
    __syncthreads();
    net_layer<32, 32, EPI_RELU, OT + 2, AS, 8 * AS>(bufB, bufA, fl, nw.wm[2], nw.bias[2], nullptr,
                                                    nq, nr, soff, q0, r0, 32, all);
    __syncthreads();
    net_layer<32, 16, EPI_LIN, OT, AS, 0>(bufA, nullptr, fl, nw.wm[3], nw.bias[3], out, nq, nr,
                                          soff, q0, r0, cout_real, all);
}

// ------------------------------------------------------------ weight grad

// Per-tile partial dW[t][co][ci] = sum_cells dy[cell][co] x[nbr_t(cell)][ci] and
// db[co] = sum_cells dy[cell][co], in FP32; wave w handles taps w and w+4.
// A = dy^T (16 channels x 32 cells), B = x_t (32 cells x 16 channels).
template <int CIN, int COUT>
__global__ __launch_bounds__(NT) void k_hexconv_wgrad(const __bf16 *__restrict__ x,
                                                      const __bf16 *__restrict__ dy,
                                                      float *__restrict__ part, int nq, int nr,
                                                      int ntiles_total, ConvMask cm) {
    constexpr int CH = CIN / 8;
    constexpr int MB = COUT / 16;
    constexpr int NB = CIN == 32 ? 2 : 1;
    constexpr int PSZ = 7 * COUT * CIN + COUT;
    __shared__ uint4 lds[NSLOT * CH];
    __shared__ uint8_t fl[NSLOT];
    __shared__ __bf16 sdy[TQ * TR * COUT];
    const int ntq = (nq + TQ - 1) / TQ, ntr = (nr + TR - 1) / TR;
    const int tile = xcd_tile(blockIdx.x, gridDim.x, ntiles_total, 0);
    if (tile < 0) return;
    float *P = part + (int64_t)tile * PSZ;
    int b, q0, r0;
    tile_of(tile, ntq, ntr, b, q0, r0);
    const int64_t soff = (int64_t)b * nq * nr;
    stage_act<CIN>(lds, fl, x, nq, nr, soff, q0, r0, cm);
    const bool masked = cm.active != nullptr;
    // dy of the tile's cells (zero outside the raster), channels-last; loads first
    constexpr int DITERS = (TQ * TR * COUT / 8 + NT - 1) / NT;
    uint4 dv[DITERS];
#pragma unroll
    for (int it = 0; it < DITERS; ++it) {
        const int e = threadIdx.x + it * NT;
        const int c = e / (COUT / 8), ch = e - c * (COUT / 8);
        const int lr = c / TQ, lq = c - lr * TQ;
        const int q = q0 + lq, r = r0 + lr;
        dv[it] = make_uint4(0u, 0u, 0u, 0u);
        if (e < TQ * TR * COUT / 8 && q < nq && r < nr)
            dv[it] = reinterpret_cast<const uint4 *>(dy + (soff + (int64_t)r * nq + q) * COUT)[ch];
    }
#pragma unroll
    for (int it = 0; it < DITERS; ++it) {
        const int e = threadIdx.x + it * NT;
        if (e < TQ * TR * COUT / 8) reinterpret_cast<uint4 *>(sdy)[e] = dv[it];
    }
    __syncthreads();
    const uint16_t *sx16 = reinterpret_cast<const uint16_t *>(lds);
    const uint16_t *sdy16 = reinterpret_cast<const uint16_t *>(sdy);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane >> 4, l16 = lane & 15;
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
        const int tap = w + 4 * tt;
        if (tap >= 7) break;
        f32x4 acc[MB][NB];
#pragma unroll
        for (int m = 0; m < MB; ++m)
#pragma unroll
            for (int n = 0; n < NB; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
        // K = 256 cells in 8 steps of 32; a group of 8 consecutive cells stays in one row
#pragma unroll 2
        for (int ks = 0; ks < (TQ * TR) / 32; ++ks) {
            const int c0 = ks * 32 + 8 * g;  // first of this lane's 8 cells
            const int lr = c0 / TQ, lq0 = c0 - lr * TQ;
            bf16x8 a[MB], bv[NB];
#pragma unroll
            for (int m = 0; m < MB; ++m) {
                const int co = m * 16 + l16;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const uint16_t u = sdy16[(c0 + j) * COUT + co];
                    a[m][j] = __builtin_bit_cast(__bf16, u);
                }
            }
#pragma unroll
            for (int n = 0; n < NB; ++n) {
                const int ci = n * 16 + l16;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int sc = (lr + 1) * SW + (lq0 + j + 1);
                    const int s = sc + OFFS[tap];
                    uint16_t u = ci < CIN ? sx16[s * CIN + ci] : (uint16_t)0;
                    if (masked && tap > 0 && !(fl[sc] & fl[s])) u = 0;
                    bv[n][j] = __builtin_bit_cast(__bf16, u);
                }
            }
#pragma unroll
            for (int m = 0; m < MB; ++m)
#pragma unroll
                for (int n = 0; n < NB; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], bv[n], acc[m][n], 0, 0, 0);
        }
        // lane holds dW rows co = m*16 + 4g + j, column ci = n*16 + l16
#pragma unroll
        for (int m = 0; m < MB; ++m)
#pragma unroll
            for (int n = 0; n < NB; ++n) {
                const int ci = n * 16 + l16;
                if (ci >= CIN) continue;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int co = m * 16 + 4 * g + j;
                    P[(tap * COUT + co) * CIN + ci] = acc[m][n][j];
                }
            }
    }
    // bias gradient: thread co sums its channel over the tile in cell order
    if (threadIdx.x < COUT) {
        float s = 0.f;
        for (int c = 0; c < TQ * TR; ++c) s += (float)sdy[c * COUT + threadIdx.x];
        P[7 * COUT * CIN + threadIdx.x] = s;
    }
}

// Sum the per-tile partials in tile order (deterministic) and scatter them
// into the flat parameter-gradient layout W[o][c][t] (o < cout, c < cin), b[o].
__global__ void k_wgrad_reduce(const float *__restrict__ part, int ntiles, int cinp, int coutp,
                               int cin, int cout, float *__restrict__ grad) {
    const int psz = 7 * coutp * cinp + coutp;
    const int nw = cout * cin * 7;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nw + cout; e += gridDim.x * blockDim.x) {
        int src;
        if (e < nw) {
            const int o = e / (cin * 7), rem = e - o * cin * 7, c = rem / 7, t = rem - c * 7;
            src = (t * coutp + o) * cinp + c;
        } else {
            src = 7 * coutp * cinp + (e - nw);
        }
        float s = 0.f;
        for (int k = 0; k < ntiles; ++k) s += part[(int64_t)k * psz + src];
        grad[e] = s;
    }
}

// ------------------------------------------------------------ parameters

// From the flat FP32 parameters of one layer (W[o][c][t], b[o]) build the
// bf16 MFMA weights: forward wm[t][co][ci] = W[co][ci][t]; data gradient
// wt[t][ci][co] = W[co][ci][opp(t)] (the transposed, mirrored stencil).
// Padded channels are zero.
__global__ void k_prepare_weights(const float *__restrict__ p, int cin, int cout, int cinp,
                                  int coutp, __bf16 *__restrict__ wm, __bf16 *__restrict__ wt,
                                  float *__restrict__ bias) {
    const int n = 7 * coutp * cinp;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const int t = e / (coutp * cinp), rem = e - t * coutp * cinp;
        const int co = rem / cinp, ci = rem - co * cinp;
        const float v = (co < cout && ci < cin) ? p[(co * cin + ci) * 7 + t] : 0.f;
        wm[e] = (__bf16)v;
        // wt is [t][ci][co] with cinp/coutp swapped roles
        const float vt = (co < cout && ci < cin) ? p[(co * cin + ci) * 7 + OPP[t]] : 0.f;
        wt[(t * cinp + ci) * coutp + co] = (__bf16)vt;
    }
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < coutp; e += gridDim.x * blockDim.x)
        bias[e] = e < cout ? p[cout * cin * 7 + e] : 0.f;
}

__global__ void k_adam(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// ------------------------------------------------------------ loss, pack

// L1 loss of pred (OUT_STRIDE floats per cell, 3 used) against target (3 per
// cell): per-workgroup FP64 partial sums and dy = sign(diff)/count as bf16
// in the 16-channel layout of the last layer.
__global__ __launch_bounds__(256) void k_l1_loss(const float *__restrict__ pred,
                                                 const float *__restrict__ target, int64_t ncell,
                                                 double inv_count, __bf16 *__restrict__ dy,
                                                 double *__restrict__ part) {
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ncell;
         i += (int64_t)gridDim.x * blockDim.x) {
        typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
        bf16x4 d0 = bf16x4{}, d1 = bf16x4{}, d2 = bf16x4{}, d3 = bf16x4{};
        for (int c = 0; c < 3; ++c) {
            const float df = pred[i * OUT_STRIDE + c] - target[i * 3 + c];
            s += fabs((double)df);
            const float gs = df > 0.f ? (float)inv_count : (df < 0.f ? -(float)inv_count : 0.f);
            d0[c] = (__bf16)gs;
        }
        bf16x4 *o = reinterpret_cast<bf16x4 *>(dy + i * 16);
        o[0] = d0;
        o[1] = d1;
        o[2] = d2;
        o[3] = d3;
    }
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// FP32 features (6 per cell) -> bf16 activations (8 channels, 2 zero).
__global__ void k_pack_features(const float *__restrict__ f, int64_t ncell,
                                __bf16 *__restrict__ x) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ncell;
         i += (int64_t)gridDim.x * blockDim.x) {
        bf16x8 v[FEATURES_PAD / 8];
#pragma unroll
        for (int c = 0; c < FEATURES_PAD; ++c)
            v[c / 8][c % 8] = c < FEATURES ? (__bf16)f[i * FEATURES + c] : (__bf16)0.f;
#pragma unroll
        for (int u = 0; u < FEATURES_PAD / 8; ++u)
            reinterpret_cast<bf16x8 *>(x + i * FEATURES_PAD)[u] = v[u];
    }
}

// ------------------------------------------------------------- launchers

static int blocks_for(int64_t n, int per = 256) {
    const int64_t b = (n + per - 1) / per;
    return (int)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

int conv_tiles(int nq, int nr, int batch) {
    return ((nq + TQ - 1) / TQ) * ((nr + TR - 1) / TR) * batch;
}

hipError_t launch_conv(int cinp, int coutp, int epi, const __bf16 *x, const __bf16 *wm,
                       const float *bias, void *out, const __bf16 *mask, int nq, int nr,
                       int batch, int cout_real, const ConvMask &cm, hipStream_t st,
                       const int32_t *live) {
    const int nt = conv_tiles(nq, nr, batch);
#define HEXSV_CONV(CI, CO, E)                                                                   \
    if (cinp == CI && coutp == CO && epi == E) {                                                \
        hipLaunchKernelGGL((k_hexconv<CI, CO, E>), dim3(nt), dim3(NT), 0, st, x, wm, bias, out, \
                           mask, nq, nr, nt, cout_real, live, cm);                              \
        return hipGetLastError();                                                               \
    }
    HEXSV_CONV(16, 32, EPI_RELU)
    HEXSV_CONV(32, 32, EPI_RELU)
    HEXSV_CONV(32, 16, EPI_LIN)
    HEXSV_CONV(16, 32, EPI_MASK)
    HEXSV_CONV(32, 32, EPI_MASK)
#undef HEXSV_CONV
    return hipErrorInvalidValue;
}

int net4_tiles(int nq, int nr, int batch) {
    return ((nq + f4::OT - 1) / f4::OT) * ((nr + f4::OT - 1) / f4::OT) * batch;
}

hipError_t launch_net4(const __bf16 *x, const Net4 &nw, float *out, int nq, int nr, int batch,
                       int cout_real, const ConvMask &cm, hipStream_t st, const int32_t *live) {
    const int nt = net4_tiles(nq, nr, batch);
    hipLaunchKernelGGL(k_hexnet4, dim3(nt), dim3(NT), 0, st, x, nw, out, nq, nr, nt, cout_real,
                       live, cm);
    return hipGetLastError();
}

hipError_t launch_wgrad(int cinp, int coutp, const __bf16 *x, const __bf16 *dy, float *part,
                        int nq, int nr, int batch, const ConvMask &cm, hipStream_t st) {
    const int nt = conv_tiles(nq, nr, batch);
#define HEXSV_WG(CI, CO)                                                                       \
    if (cinp == CI && coutp == CO) {                                                           \
        hipLaunchKernelGGL((k_hexconv_wgrad<CI, CO>), dim3(nt), dim3(NT), 0, st, x, dy, part, nq, \
                           nr, nt, cm);                                                        \
        return hipGetLastError();                                                              \
    }
    HEXSV_WG(16, 32)
    HEXSV_WG(32, 32)
    HEXSV_WG(32, 16)
#undef HEXSV_WG
    return hipErrorInvalidValue;
}

hipError_t launch_wgrad_reduce(const float *part, int ntiles, int cinp, int coutp, int cin,
                               int cout, float *grad, hipStream_t st) {
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(blocks_for(7 * cin * cout + cout)), dim3(256), 0, st,
                       part, ntiles, cinp, coutp, cin, cout, grad);
    return hipGetLastError();
}

hipError_t launch_prepare_weights(const float *p, int cin, int cout, int cinp, int coutp,
                                  __bf16 *wm, __bf16 *wt, float *bias, hipStream_t st) {
    hipLaunchKernelGGL(k_prepare_weights, dim3(blocks_for(7 * cinp * coutp)), dim3(256), 0, st, p,
                       cin, cout, cinp, coutp, wm, wt, bias);
    return hipGetLastError();
}

hipError_t launch_adam(float *p, float *m, float *v, const float *g, int64_t n, float lr,
                       int step, hipStream_t st) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(n)), dim3(256), 0, st, p, m, v, g, n, lr, b1, b2,
                       1e-8f, c1, c2);
    return hipGetLastError();
}

hipError_t launch_l1_loss(const float *pred, const float *target, int64_t ncell, double inv_count,
                          __bf16 *dy, double *part, int nparts, hipStream_t st) {
    hipLaunchKernelGGL(k_l1_loss, dim3(nparts), dim3(256), 0, st, pred, target, ncell, inv_count,
                       dy, part);
    return hipGetLastError();
}

hipError_t launch_pack_features(const float *f, int64_t ncell, __bf16 *x, hipStream_t st) {
    hipLaunchKernelGGL(k_pack_features, dim3(blocks_for(ncell)), dim3(256), 0, st, f, ncell, x);
    return hipGetLastError();
}

}  // namespace nn
}  // namespace hexsv
