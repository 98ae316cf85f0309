// hexsv_nn.h — launchers of the surrogate's kernels (hexsv_nn.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hexsv {
namespace nn {

enum { EPI_RELU = 0, EPI_LIN = 1, EPI_MASK = 2 };
constexpr int OUT_STRIDE = 4;  // floats per cell of the network output (3 used)
constexpr int FEATURES = 11;     // network input channels
constexpr int FEATURES_PAD = 16; // stored input channels per cell (bf16, zero padded)

// Which raster positions a tap may reach, as in the neighbour table of the
// scheme: periodic sides wrap (perq: q, perr: r), positions outside the raster
// are zero, and with an active mask (per raster cell, nonzero = in the domain;
// nullable: every cell) a tap t >= 1 reads its neighbour only when both the cell
// and the neighbour are in the domain (tap 0, the cell itself, is always read).
// The rule is symmetric, so the transposed stencil of the data gradient uses it
// unchanged.
struct ConvMask {
    const uint8_t *active;
    int perq, perr;
};

// Workgroups (tiles of 64 x 4 cells) of one conv launch over a batch.
int conv_tiles(int nq, int nr, int batch);

// Hex convolution of channels-last bf16 x (cinp channels) with the MFMA
// weight layout wm[t][coutp][cinp]; epilogue per EPI_* (see hexsv_nn.hip).
// Built for (cinp, coutp, epi) in {(16,32,RELU), (32,32,RELU), (32,16,LIN),
// (16,32,MASK), (32,32,MASK)}.
// live (nullable, device): the launch does nothing unless *live != 0.
hipError_t launch_conv(int cinp, int coutp, int epi, const __bf16 *x, const __bf16 *wm,
                       const float *bias, void *out, const __bf16 *mask, int nq, int nr,
                       int batch, int cout_real, const ConvMask &cm, hipStream_t st,
                       const int32_t *live = nullptr);
// The 4-layer network with 32 hidden channels in one launch (k_hexnet4): weights
// and biases of each layer as for launch_conv (layer 0: 16 -> 32, layers 1-2:
// 32 -> 32, layer 3: 32 -> 16 with cout_real outputs written, FP32, OUT_STRIDE
// per cell); the output equals the layer-by-layer launch_conv chain bit for bit.
struct Net4 {
    const __bf16 *wm[4];
    const float *bias[4];
};
int net4_tiles(int nq, int nr, int batch);
hipError_t launch_net4(const __bf16 *x, const Net4 &nw, float *out, int nq, int nr, int batch,
                       int cout_real, const ConvMask &cm, hipStream_t st,
                       const int32_t *live = nullptr);
// Per-tile weight-gradient partials (7*coutp*cinp + coutp floats per tile).
hipError_t launch_wgrad(int cinp, int coutp, const __bf16 *x, const __bf16 *dy, float *part,
                        int nq, int nr, int batch, const ConvMask &cm, hipStream_t st);
hipError_t launch_wgrad_reduce(const float *part, int ntiles, int cinp, int coutp, int cin,
                               int cout, float *grad, hipStream_t st);
hipError_t launch_prepare_weights(const float *p, int cin, int cout, int cinp, int coutp,
                                  __bf16 *wm, __bf16 *wt, float *bias, hipStream_t st);
hipError_t launch_adam(float *p, float *m, float *v, const float *g, int64_t n, float lr,
                       int step, hipStream_t st);
hipError_t launch_l1_loss(const float *pred, const float *target, int64_t ncell, double inv_count,
                          __bf16 *dy, double *part, int nparts, hipStream_t st);
hipError_t launch_pack_features(const float *f, int64_t ncell, __bf16 *x, hipStream_t st);

}  // namespace nn
}  // namespace hexsv
