// hexsv_conv.h — the hex-convolution tile of the surrogate's BF16 MFMA kernels:
// halo staging into LDS and the MFMA accumulation of one 64 x 4 tile, shared by
// the convolution kernels (hexsv_nn.hip) and the window kernel that applies the
// network's last layer to the state (hexsv_kernels.h).
//
// Hex convolution on an nq x nr raster (per sample of a batch):
//   y[i][o] = b[o] + sum_{t<7, c} W[o][c][t] * x[nbr_t(i)][c]
// tap 0 is the cell, tap 1+k its neighbour in direction k: the neighbour of
// the scheme's tables (periodic sides wrap; zero outside the raster and, on a
// masked raster, unless both cells are in the domain; see ConvMask).
// Activations are channels-last bfloat16 (x[cell][c], C = 16 or 32).
//
// MFMA mapping (v_mfma_f32_16x16x32_bf16): the output block is 16 output
// channels x 16 cells, A = weights (16 channels x 32 K), B = gathered
// activations (32 K x 16 cells), K = the 32 input channels of one tap (or
// two taps of 16 channels for the 16-channel input layer).  A lane holds the
// 8 consecutive K values of its row/column, i.e. 16 contiguous bytes of a
// weight row or of one neighbour's channel vector in LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hexsv_device.h"
#include "hexsv_nn.h"

namespace hexsv {
namespace nn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int TQ = 64, TR = 4, NT = 256;  // 256 cells per workgroup, one row per wave
constexpr int SW = TQ + 2, SH = TR + 2, NSLOT = SW * SH;
constexpr int OFFS[7] = {0, 1, SW, SW - 1, -1, -SW, -SW + 1};  // tap -> LDS slot offset
constexpr int OPP[7] = {0, 4, 5, 6, 1, 2, 3};                   // tap of the opposite direction

__device__ inline int tile_of(int tile, int ntq, int ntr, int &b, int &q0, int &r0) {
    const int per = ntq * ntr;
    b = tile / per;
    const int lt = tile - b * per;
    const int tr = lt / ntq;
    q0 = (lt - tr * ntq) * TQ;
    r0 = tr * TR;
    return lt;
}

// Stage the (TQ+2) x (TR+2) halo of channels-last bf16 activations of one
// sample into LDS as 16-byte chunks, with periodic wraps; positions outside the
// raster are zero.  fl[slot] is 1 where the slot holds a cell of the domain
// (written only on masked rasters, where the taps test it).  All of a thread's
// loads are issued before any LDS store, so the staging costs one memory
// latency rather than one per chunk.
template <int C>
__device__ inline void stage_act(uint4 *lds, uint8_t *fl, const __bf16 *__restrict__ x, int nq,
                                 int nr, int64_t sample_off, int q0, int r0, const ConvMask &cm) {
    constexpr int CH = C / 8;  // 16-byte chunks per cell
    constexpr int ITERS = (NSLOT * CH + NT - 1) / NT;
    uint4 v[ITERS];
    uint8_t a[ITERS];
#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
        const int e = threadIdx.x + it * NT;
        const int s = e / CH, ch = e - s * CH;
        const int lr = s / SW, lq = s - lr * SW;
        int q = q0 + lq - 1, r = r0 + lr - 1;
        if (cm.perq) q = q < 0 ? q + nq : (q >= nq ? q - nq : q);
        if (cm.perr) r = r < 0 ? r + nr : (r >= nr ? r - nr : r);
        v[it] = make_uint4(0u, 0u, 0u, 0u);
        a[it] = 0;
        if (e < NSLOT * CH && q >= 0 && q < nq && r >= 0 && r < nr) {
            const int64_t i = sample_off + (int64_t)r * nq + q;
            v[it] = reinterpret_cast<const uint4 *>(x + i * C)[ch];
            if (cm.active && ch == 0) a[it] = cm.active[(int64_t)r * nq + q] != 0;
        }
    }
#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
        const int e = threadIdx.x + it * NT;
        if (e < NSLOT * CH) {
            lds[e] = v[it];
            if (cm.active && (e % CH) == 0) fl[e / CH] = a[it];
        }
    }
}

// Accumulators of the tile staged in lds (CIN channels per cell): lane (g, l16)
// of wave w ends holding output channels co = m*16 + 4g + j (j < 4) of cell
// (n*16 + l16, w) of the tile in acc[m][n][j].  Weights wm[t][COUT][CIN].
template <int CIN, int COUT>
__device__ inline void conv_acc(const uint4 *lds, const uint8_t *fl, bool masked,
                                const __bf16 *__restrict__ wm, f32x4 (&acc)[COUT / 16][4]) {
    constexpr int CH = CIN / 8;
    constexpr int MB = COUT / 16;                 // output-channel blocks
    constexpr int TPK = 32 / CIN;                 // taps per K step of 32
    constexpr int KSTEPS = (7 + TPK - 1) / TPK;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;  // wave w: tile row w
    const int g = lane >> 4, l16 = lane & 15;
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};

#pragma unroll
    for (int ks = 0; ks < KSTEPS; ++ks) {
        // tap and channel offset of this lane's 8 K values
        const int tap = ks * TPK + g / CH;
        const int c0 = (g % CH) * 8;
        bf16x8 a[MB];
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            if (tap < 7) {
                a[m] = *reinterpret_cast<const bf16x8 *>(wm + ((int64_t)(tap * COUT + m * 16 + l16)) * CIN + c0);
            } else {
                a[m] = bf16x8{};
            }
        }
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            const int lq = n * 16 + l16;             // cell column in the tile
            const int s = (w + 1) * SW + (lq + 1);   // its staged slot
            bf16x8 bv = bf16x8{};
            if (tap < 7) {
                uint4 raw = lds[(s + OFFS[tap]) * CH + c0 / 8];
                // masked raster: a neighbour tap needs both cells in the domain
                if (masked && tap > 0 && !(fl[s] & fl[s + OFFS[tap]]))
                    raw = make_uint4(0u, 0u, 0u, 0u);
                bv = *reinterpret_cast<const bf16x8 *>(&raw);
            }
#pragma unroll
            for (int m = 0; m < MB; ++m)
                acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], bv, acc[m][n], 0, 0, 0);
        }
    }
}

}  // namespace nn
}  // namespace hexsv
