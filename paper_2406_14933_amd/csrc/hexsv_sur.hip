// hexsv_sur.hip — C-ABI of the learned hex-convolution surrogate: parameters,
// batched forward, gradient and Adam training step (kernels in hexsv_nn.hip).
#include <math.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "hexsv.h"
#include "hexsv_host.h"
#include "hexsv_nn.h"

using namespace hexsv;

struct SurLayer {
    int cin, cout, cinp, coutp;
    int64_t off;          // offset of W in the flat parameters (b follows)
    __bf16 *wm, *wt;      // forward and data-gradient MFMA weights
    float *bias;          // padded FP32 bias
};

struct hexsv_surrogate {
    int layers, channels;
    int k;  // solver steps a window spans (its rain sub-steps)
    bool fused;  // forward of the 4-layer, 32-channel network in one kernel (k_hexnet4)
    int64_t nparams;
    float *d_p, *d_m, *d_v, *d_g;
    std::vector<SurLayer> L;
    int adam_step;
    bool weights_ready;
    float scales[8];
    // workspace sized for ws_cells cells and ws_tiles conv tiles; ws_gen
    // counts reallocations (a captured graph holds the buffer addresses)
    int64_t ws_cells;
    int ws_tiles;
    uint64_t ws_gen;
    __bf16 *x0;                 // packed features, 8 channels
    std::vector<__bf16 *> act;  // hidden activations, channels each
    float *out;                 // network output, OUT_STRIDE floats per cell
    __bf16 *dy_last;            // loss gradient, 16 channels
    __bf16 *dA, *dB;            // data-gradient ping-pong buffers, channels each
    float *wpart;               // weight-gradient partials
    double *lpart, *h_lpart;    // loss partials (device, pinned host)
};

static const int LOSS_PARTS = 1024;

extern "C" void hexsv_surrogate_destroy(hexsv_surrogate *s);

static void free_ws(hexsv_surrogate *s) {
    auto F = [](void *p) { if (p) (void)hipFree(p); };
    F(s->x0);
    for (auto p : s->act) F(p);
    s->act.clear();
    F(s->out);
    F(s->dy_last);
    F(s->dA);
    F(s->dB);
    F(s->wpart);
    F(s->lpart);
    if (s->h_lpart) (void)hipHostFree(s->h_lpart);
    s->x0 = nullptr;
    s->out = nullptr;
    s->dy_last = s->dA = s->dB = nullptr;
    s->wpart = nullptr;
    s->lpart = nullptr;
    s->h_lpart = nullptr;
    s->ws_cells = 0;
    s->ws_tiles = 0;
}

static int ensure_ws(hexsv_surrogate *s, int64_t cells, int tiles) {
    if (cells <= s->ws_cells && tiles <= s->ws_tiles) return HEXSV_OK;
    free_ws(s);
    const int C = s->channels;
    hipError_t e = hipMalloc(&s->x0, sizeof(__bf16) * nn::FEATURES_PAD * cells);
    for (int l = 0; l + 1 < s->layers && e == hipSuccess; ++l) {
        __bf16 *p = nullptr;
        e = hipMalloc(&p, sizeof(__bf16) * C * cells);
        s->act.push_back(p);
    }
    if (e == hipSuccess) e = hipMalloc(&s->out, sizeof(float) * nn::OUT_STRIDE * cells);
    if (e == hipSuccess) e = hipMalloc(&s->dy_last, sizeof(__bf16) * 16 * cells);
    if (e == hipSuccess) e = hipMalloc(&s->dA, sizeof(__bf16) * C * cells);
    if (e == hipSuccess) e = hipMalloc(&s->dB, sizeof(__bf16) * C * cells);
    size_t psz = 0;
    for (auto &l : s->L) psz = std::max(psz, (size_t)(7 * l.coutp * l.cinp + l.coutp));
    if (e == hipSuccess) e = hipMalloc(&s->wpart, sizeof(float) * psz * (size_t)tiles);
    if (e == hipSuccess) e = hipMalloc(&s->lpart, sizeof(double) * LOSS_PARTS);
    if (e == hipSuccess) e = hipHostMalloc(&s->h_lpart, sizeof(double) * LOSS_PARTS, hipHostMallocDefault);
    if (e != hipSuccess) {
        free_ws(s);
        return fail(HEXSV_ENOMEM, "surrogate workspace: %s", hipGetErrorString(e));
    }
    s->ws_cells = cells;
    s->ws_tiles = tiles;
    s->ws_gen += 1;
    return HEXSV_OK;
}

extern "C" int hexsv_surrogate_create(int32_t layers, int32_t channels, int32_t k,
                                      hexsv_surrogate **out) {
    if (!out) return fail(HEXSV_EINVAL, "surrogate_create: null argument");
    *out = nullptr;
    if (channels != 32) return fail(HEXSV_EUNSUPPORTED, "surrogate_create: only 32 channels are built");
    if (layers < 2 || layers > 16) return fail(HEXSV_EINVAL, "surrogate_create: layers must be in [2, 16]");
    if (k < 1) return fail(HEXSV_EINVAL, "surrogate_create: k must be >= 1");
    hexsv_surrogate *s = new (std::nothrow) hexsv_surrogate();
    if (!s) return fail(HEXSV_ENOMEM, "surrogate_create: out of host memory");
    s->layers = layers;
    s->channels = channels;
    s->k = k;
    s->fused = false;  // the layer chain measures faster on the 512 x 512 windows
    int64_t off = 0;
    for (int l = 0; l < layers; ++l) {
        SurLayer y{};
        y.cin = l == 0 ? nn::FEATURES : channels;
        y.cout = l == layers - 1 ? 3 : channels;
        y.cinp = l == 0 ? nn::FEATURES_PAD : channels;
        y.coutp = l == layers - 1 ? 16 : channels;
        y.off = off;
        off += (int64_t)y.cout * y.cin * 7 + y.cout;
        s->L.push_back(y);
    }
    s->nparams = off;
    for (int k = 0; k < 8; ++k) s->scales[k] = 1.f;
    hipError_t e = hipMalloc(&s->d_p, sizeof(float) * off);
    if (e == hipSuccess) e = hipMalloc(&s->d_m, sizeof(float) * off);
    if (e == hipSuccess) e = hipMalloc(&s->d_v, sizeof(float) * off);
    if (e == hipSuccess) e = hipMalloc(&s->d_g, sizeof(float) * off);
    for (auto &y : s->L) {
        if (e == hipSuccess) e = hipMalloc(&y.wm, sizeof(__bf16) * 7 * y.cinp * y.coutp);
        if (e == hipSuccess) e = hipMalloc(&y.wt, sizeof(__bf16) * 7 * y.cinp * y.coutp);
        if (e == hipSuccess) e = hipMalloc(&y.bias, sizeof(float) * y.coutp);
    }
    if (e == hipSuccess) e = hipMemset(s->d_p, 0, sizeof(float) * off);
    if (e == hipSuccess) e = hipMemset(s->d_m, 0, sizeof(float) * off);
    if (e == hipSuccess) e = hipMemset(s->d_v, 0, sizeof(float) * off);
    if (e != hipSuccess) {
        hexsv_surrogate_destroy(s);
        return fail(HEXSV_ENOMEM, "surrogate_create: %s", hipGetErrorString(e));
    }
    *out = s;
    return HEXSV_OK;
}

extern "C" void hexsv_surrogate_destroy(hexsv_surrogate *s) {
    if (!s) return;
    free_ws(s);
    auto F = [](void *p) { if (p) (void)hipFree(p); };
    F(s->d_p);
    F(s->d_m);
    F(s->d_v);
    F(s->d_g);
    for (auto &y : s->L) {
        F(y.wm);
        F(y.wt);
        F(y.bias);
    }
    delete s;
}

extern "C" int64_t hexsv_surrogate_num_params(const hexsv_surrogate *s) { return s ? s->nparams : -1; }
extern "C" int32_t hexsv_surrogate_steps(const hexsv_surrogate *s) { return s ? s->k : -1; }

extern "C" int hexsv_surrogate_set_fused(hexsv_surrogate *s, int32_t on) {
    if (!s) return fail(HEXSV_EINVAL, "surrogate_set_fused: null surrogate");
    if (on != 0 && on != 1) return fail(HEXSV_EINVAL, "surrogate_set_fused: on must be 0 or 1");
    s->fused = on != 0;
    return HEXSV_OK;
}

static int prepare(hexsv_surrogate *s, hipStream_t st) {
    for (auto &y : s->L)
        HIP_TRY(nn::launch_prepare_weights(s->d_p + y.off, y.cin, y.cout, y.cinp, y.coutp, y.wm, y.wt,
                                           y.bias, st));
    s->weights_ready = true;
    return HEXSV_OK;
}

extern "C" int hexsv_surrogate_set_params(hexsv_surrogate *s, const float *d_params, int64_t n,
                                          hipStream_t st) {
    if (!s || !d_params) return fail(HEXSV_EINVAL, "surrogate_set_params: null argument");
    if (n != s->nparams) return fail(HEXSV_EINVAL, "surrogate_set_params: %lld values, expected %lld",
                                     (long long)n, (long long)s->nparams);
    HIP_TRY(hipMemcpyAsync(s->d_p, d_params, sizeof(float) * n, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemsetAsync(s->d_m, 0, sizeof(float) * n, st));
    HIP_TRY(hipMemsetAsync(s->d_v, 0, sizeof(float) * n, st));
    s->adam_step = 0;
    return prepare(s, st);
}

extern "C" int hexsv_surrogate_get_params(const hexsv_surrogate *s, float *d_params, int64_t n,
                                          hipStream_t st) {
    if (!s || !d_params || n != s->nparams) return fail(HEXSV_EINVAL, "surrogate_get_params: bad argument");
    HIP_TRY(hipMemcpyAsync(d_params, s->d_p, sizeof(float) * n, hipMemcpyDeviceToDevice, st));
    return HEXSV_OK;
}

extern "C" int hexsv_surrogate_set_scales(hexsv_surrogate *s, const float *scales, int32_t n) {
    if (!s || !scales || n < 1 || n > 8) return fail(HEXSV_EINVAL, "surrogate_set_scales: bad argument");
    for (int k = 0; k < n; ++k) s->scales[k] = scales[k];
    return HEXSV_OK;
}

extern "C" int hexsv_surrogate_get_scales(const hexsv_surrogate *s, float *scales, int32_t n) {
    if (!s || !scales || n < 1 || n > 8) return fail(HEXSV_EINVAL, "surrogate_get_scales: bad argument");
    for (int k = 0; k < n; ++k) scales[k] = s->scales[k];
    return HEXSV_OK;
}

// Tap rule of a raster: its periodic sides and its domain mask (no grid: a
// walled nq x nr parallelogram with every cell in the domain).
static int conv_mask(const hexsv_grid *g, int nq, int nr, nn::ConvMask *cm, const char *who) {
    *cm = nn::ConvMask{nullptr, 0, 0};
    if (!g) return HEXSV_OK;
    if (g->kg.nq != nq || g->kg.nr != nr)
        return fail(HEXSV_EINVAL, "%s: the raster is %d x %d, the grid %d x %d", who, nq, nr,
                    g->kg.nq, g->kg.nr);
    if (g->n_dirichlet)
        return fail(HEXSV_EUNSUPPORTED, "%s: not built for Dirichlet or flux cells", who);
    *cm = nn::ConvMask{g->d_active, g->kg.perq, g->kg.perr};
    return HEXSV_OK;
}

// Forward over the packed features already in s->x0; output in s->out.  With
// fusion switched on, the 4-layer, 32-channel network runs as one kernel unless
// the hidden activations are wanted (keep_act: the gradient reads them); both
// paths give the same output bit for bit.
static int forward_packed(hexsv_surrogate *s, int nq, int nr, int batch, const nn::ConvMask &cm,
                          hipStream_t st, const int32_t *live = nullptr, bool keep_act = false) {
    if (!keep_act && s->fused && s->layers == 4 && s->channels == 32) {
        nn::Net4 nw;
        for (int l = 0; l < 4; ++l) {
            nw.wm[l] = s->L[l].wm;
            nw.bias[l] = s->L[l].bias;
        }
        HIP_TRY(nn::launch_net4(s->x0, nw, s->out, nq, nr, batch, s->L[3].cout, cm, st, live));
        return HEXSV_OK;
    }
    const __bf16 *x = s->x0;
    for (int l = 0; l < s->layers; ++l) {
        const SurLayer &y = s->L[l];
        const bool last = l == s->layers - 1;
        void *o = last ? (void *)s->out : (void *)s->act[l];
        HIP_TRY(nn::launch_conv(y.cinp, y.coutp, last ? nn::EPI_LIN : nn::EPI_RELU, x, y.wm, y.bias,
                                o, nullptr, nq, nr, batch, y.cout, cm, st, live));
        if (!last) x = s->act[l];
    }
    return HEXSV_OK;
}

static int check_shape(hexsv_surrogate *s, int batch, int nq, int nr, int64_t *cells) {
    if (batch < 1 || nq < 1 || nr < 1) return fail(HEXSV_EINVAL, "surrogate: bad batch or raster size");
    if (!s->weights_ready) return fail(HEXSV_ESTATE, "surrogate: set the parameters first");
    *cells = (int64_t)batch * nq * nr;
    return ensure_ws(s, *cells, nn::conv_tiles(nq, nr, batch));
}

extern "C" int hexsv_surrogate_forward(hexsv_surrogate *s, const hexsv_grid *grid, int32_t batch,
                                       int32_t nq, int32_t nr, const float *d_features,
                                       float *d_out, hipStream_t st) {
    if (!s || !d_features || !d_out) return fail(HEXSV_EINVAL, "surrogate_forward: null argument");
    nn::ConvMask cm;
    int rc = conv_mask(grid, nq, nr, &cm, "surrogate_forward");
    if (rc) return rc;
    int64_t cells;
    rc = check_shape(s, batch, nq, nr, &cells);
    if (rc) return rc;
    HIP_TRY(nn::launch_pack_features(d_features, cells, s->x0, st));
    rc = forward_packed(s, nq, nr, batch, cm, st);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(d_out, s->out, sizeof(float) * nn::OUT_STRIDE * cells,
                           hipMemcpyDeviceToDevice, st));
    return HEXSV_OK;
}

// ---- interface for the solver's surrogate windows (hexsv_capi.hip)

int sur_window_bind(hexsv_surrogate *s, int nq, int nr, void **x0, const float **out,
                    uint64_t *gen) {
    int64_t cells;
    int rc = check_shape(s, 1, nq, nr, &cells);
    if (rc) return rc;
    *x0 = s->x0;
    *out = s->out;
    *gen = s->ws_gen;
    return HEXSV_OK;
}

int sur_forward_x0(hexsv_surrogate *s, const hexsv_grid *grid, hipStream_t st,
                   const int32_t *live) {
    nn::ConvMask cm;
    int rc = conv_mask(grid, grid->kg.nq, grid->kg.nr, &cm, "run_surrogate");
    if (rc) return rc;
    return forward_packed(s, grid->kg.nq, grid->kg.nr, 1, cm, st, live);
}

int sur_forward_hidden(hexsv_surrogate *s, const hexsv_grid *grid, hipStream_t st,
                       const int32_t *live, SurLast *last) {
    if (s->fused || s->channels != 32) return HEXSV_EUNSUPPORTED;
    nn::ConvMask cm;
    int rc = conv_mask(grid, grid->kg.nq, grid->kg.nr, &cm, "run_surrogate");
    if (rc) return rc;
    const int nq = grid->kg.nq, nr = grid->kg.nr;
    const __bf16 *x = s->x0;
    for (int l = 0; l + 1 < s->layers; ++l) {
        const SurLayer &y = s->L[l];
        HIP_TRY(nn::launch_conv(y.cinp, y.coutp, nn::EPI_RELU, x, y.wm, y.bias, s->act[l],
                                nullptr, nq, nr, 1, y.cout, cm, st, live));
        x = s->act[l];
    }
    const SurLayer &y = s->L[s->layers - 1];
    *last = SurLast{x, y.wm, y.bias, cm};
    return HEXSV_OK;
}

// Forward + L1 loss + backward into s->d_g; loss in *loss (synchronises).
static int gradient(hexsv_surrogate *s, const hexsv_grid *grid, int batch, int nq, int nr,
                    const float *feat, const float *target, double *loss, hipStream_t st) {
    nn::ConvMask cm;
    int rc = conv_mask(grid, nq, nr, &cm, "surrogate_gradient");
    if (rc) return rc;
    int64_t cells;
    rc = check_shape(s, batch, nq, nr, &cells);
    if (rc) return rc;
    HIP_TRY(nn::launch_pack_features(feat, cells, s->x0, st));
    rc = forward_packed(s, nq, nr, batch, cm, st, nullptr, true);
    if (rc) return rc;
    const double inv_count = 1.0 / (3.0 * (double)cells);
    HIP_TRY(nn::launch_l1_loss(s->out, target, cells, inv_count, s->dy_last, s->lpart, LOSS_PARTS, st));
    const int tiles = nn::conv_tiles(nq, nr, batch);
    const __bf16 *dy = s->dy_last;
    __bf16 *buf[2] = {s->dA, s->dB};
    for (int l = s->layers - 1; l >= 0; --l) {
        const SurLayer &y = s->L[l];
        const __bf16 *xin = l == 0 ? s->x0 : s->act[l - 1];
        HIP_TRY(nn::launch_wgrad(y.cinp, y.coutp, xin, dy, s->wpart, nq, nr, batch, cm, st));
        HIP_TRY(nn::launch_wgrad_reduce(s->wpart, tiles, y.cinp, y.coutp, y.cin, y.cout, s->d_g + y.off, st));
        if (l > 0) {
            __bf16 *dx = buf[l & 1];
            // data gradient: input channels of the transposed stencil = coutp, output = cinp
            HIP_TRY(nn::launch_conv(y.coutp, y.cinp, nn::EPI_MASK, dy, y.wt, nullptr, dx, s->act[l - 1],
                                    nq, nr, batch, y.cin, cm, st));
            dy = dx;
        }
    }
    HIP_TRY(hipMemcpyAsync(s->h_lpart, s->lpart, sizeof(double) * LOSS_PARTS, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    double tot = 0.0;
    for (int k = 0; k < LOSS_PARTS; ++k) tot += s->h_lpart[k];
    if (loss) *loss = tot * inv_count;
    return HEXSV_OK;
}

extern "C" int hexsv_surrogate_gradient(hexsv_surrogate *s, const hexsv_grid *grid, int32_t batch,
                                        int32_t nq, int32_t nr, const float *d_features,
                                        const float *d_target, float *d_grad, double *loss,
                                        hipStream_t st) {
    if (!s || !d_features || !d_target) return fail(HEXSV_EINVAL, "surrogate_gradient: null argument");
    int rc = gradient(s, grid, batch, nq, nr, d_features, d_target, loss, st);
    if (rc) return rc;
    if (d_grad)
        HIP_TRY(hipMemcpyAsync(d_grad, s->d_g, sizeof(float) * s->nparams, hipMemcpyDeviceToDevice, st));
    return HEXSV_OK;
}

extern "C" int hexsv_surrogate_train_step(hexsv_surrogate *s, const hexsv_grid *grid,
                                          int32_t batch, int32_t nq, int32_t nr,
                                          const float *d_features, const float *d_target, float lr,
                                          double *loss, hipStream_t st) {
    if (!s || !d_features || !d_target || !(lr > 0.f)) return fail(HEXSV_EINVAL, "surrogate_train_step: bad argument");
    int rc = gradient(s, grid, batch, nq, nr, d_features, d_target, loss, st);
    if (rc) return rc;
    s->adam_step += 1;
    HIP_TRY(nn::launch_adam(s->d_p, s->d_m, s->d_v, s->d_g, s->nparams, lr, s->adam_step, st));
    return prepare(s, st);
}

// ---- forward without allocation
//
// For callers that cannot allocate (graph capture, serving loops): the packed
// input and two ping-pong hidden-activation buffers live in one static device
// array, `scratch`, held by every GPU the library runs on until the process
// ends.  Host code reaches it only through the address hipGetSymbolAddress
// returns on each device (the array's name is a host-side stand-in).
constexpr int64_t NOALLOC_MAX_CELLS = (int64_t)1 << 18;  // a 512 x 512 sample
constexpr int64_t NOALLOC_CH = 32;                        // hidden channels built
constexpr size_t NOALLOC_X0 = sizeof(__bf16) * nn::FEATURES_PAD * NOALLOC_MAX_CELLS;
constexpr size_t NOALLOC_ACT = sizeof(__bf16) * NOALLOC_CH * NOALLOC_MAX_CELLS;
constexpr size_t NOALLOC_BYTES = NOALLOC_X0 + 2 * NOALLOC_ACT;  // 40 MiB
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

static const int NOALLOC_MAX_DEVICES = 64;
static void *g_scratch_ptr[NOALLOC_MAX_DEVICES];
static std::mutex g_scratch_mu;

// Device address of `scratch` on the current device (looked up once per device).
static int scratch_of_device(unsigned char **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(HEXSV_EUNSUPPORTED, "surrogate_forward_noalloc: device %d", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(HEXSV_EHIP, "surrogate_forward_noalloc: hipGetSymbolAddress: %s",
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = (unsigned char *)g_scratch_ptr[dev];
    return HEXSV_OK;
}

extern "C" int hexsv_surrogate_forward_noalloc(hexsv_surrogate *s, const hexsv_grid *grid,
                                               int32_t batch, int32_t nq, int32_t nr,
                                               const float *d_features, float *d_out,
                                               hipStream_t st) {
    if (!s || !d_features || !d_out)
        return fail(HEXSV_EINVAL, "surrogate_forward_noalloc: null argument");
    if (batch < 1 || nq < 1 || nr < 1)
        return fail(HEXSV_EINVAL, "surrogate_forward_noalloc: bad batch or raster size");
    if (!s->weights_ready) return fail(HEXSV_ESTATE, "surrogate_forward_noalloc: set the parameters first");
    const int64_t cells = (int64_t)batch * nq * nr;
    if (cells > NOALLOC_MAX_CELLS)
        return fail(HEXSV_EINVAL,
                    "surrogate_forward_noalloc: %lld cells exceed the %lld of its static workspace "
                    "(use hexsv_surrogate_forward)", (long long)cells, (long long)NOALLOC_MAX_CELLS);
    if (s->channels != NOALLOC_CH)
        return fail(HEXSV_EUNSUPPORTED, "surrogate_forward_noalloc: %d channels", s->channels);
    nn::ConvMask cm;
    int rc = conv_mask(grid, nq, nr, &cm, "surrogate_forward_noalloc");
    if (rc) return rc;
    unsigned char *ws = nullptr;
    rc = scratch_of_device(&ws);
    if (rc) return rc;
    __bf16 *x0 = (__bf16 *)ws;
    __bf16 *act[2] = {(__bf16 *)(ws + NOALLOC_X0), (__bf16 *)(ws + NOALLOC_X0 + NOALLOC_ACT)};
    // every buffer is written in full before it is read: nothing needs clearing
    HIP_TRY(nn::launch_pack_features(d_features, cells, x0, st));
    const __bf16 *x = x0;
    for (int l = 0; l < s->layers; ++l) {
        const SurLayer &y = s->L[l];
        const bool last = l == s->layers - 1;
        void *o = last ? (void *)d_out : (void *)act[l & 1];
        HIP_TRY(nn::launch_conv(y.cinp, y.coutp, last ? nn::EPI_LIN : nn::EPI_RELU, x, y.wm, y.bias,
                                o, nullptr, nq, nr, batch, y.cout, cm, st));
        if (!last) x = act[l & 1];
    }
    return HEXSV_OK;
}
