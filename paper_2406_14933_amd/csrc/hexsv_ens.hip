// hexsv_ens.hip — C-ABI of the batched ensemble: many independent catchments
// of uneven raster sizes advanced together by the persistent kernel.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "hexsv.h"
#include "hexsv_ensemble.h"
#include "hexsv_host.h"
#include "hexsv_internal.h"

using namespace hexsv;

struct hexsv_ensemble {
    int n;
    int prec;
    size_t esz;
    int tile, ksteps, nwg;
    int mode;                   // HEXSV_ENS_PERSISTENT or HEXSV_ENS_BATCHED
    int visc;                   // 1: artificial viscosity (batched mode only)
    int bc;                     // 1: a scenario holds Dirichlet or flux cells (batched mode only)
    int btile, btotal;          // batched mode: tile variant and total tiles
    EnsTile *d_tiles;           // batched mode: descriptor of every global tile
    Part *d_bpart;              // batched mode: one record per global tile
    uint8_t *d_tpar;            // batched mode: parity offset of every global tile
    std::vector<uint8_t> h_tpar;  // what d_tpar holds (empty: not set)
    double dt_max;
    std::vector<const hexsv_grid *> grids;
    std::vector<EnsScen> scen;  // host copy
    std::vector<int64_t> active;
    int64_t total;
    void *buf;                  // [h0 v10 v20 h1 v11 v21 z th ap], total elements each;
                                // scenario s at scen[s].off, rows scen[s].g.pitch apart
    EnsScen *d_scen;
    Ctl *d_ctl;
    Ctl *h_ctl;                 // pinned mirror, n entries
    Part *d_part;
    int32_t *d_chk, *h_chk;
    int32_t *d_order;
    uint32_t *d_queue;
    std::vector<char> ready;
    hipStream_t cap;
    hipGraph_t graph[2];        // ksteps launches, live scenarios starting at parity 0 / 1
    hipGraphExec_t gexec[2];
    bool timing;
    hipEvent_t ev0, ev1;
    double timed_ms;
    int64_t timed_updates, timed_launches;
};

// Row stride of a scenario's arrays: nq rounded up to 16 cells, so that every row
// starts on a 64-byte boundary (128 in FP64) and a row's stores cover whole cache
// lines instead of sharing a line with the next row.  The padding cells stay zero.
static int ens_pitch(int nq) { return (nq + 15) / 16 * 16; }

template <typename T>
static KDom<T> ens_base(const hexsv_ensemble *e) {
    KDom<T> d;
    T *b = (T *)e->buf;
    for (int p = 0; p < 2; ++p)
        for (int f = 0; f < 3; ++f) d.st[p][f] = b + (int64_t)(3 * p + f) * e->total;
    d.z = b + 6 * e->total;
    d.th = b + 7 * e->total;
    d.ap = b + 8 * e->total;
    return d;
}

template <typename T>
static KDom<T> ens_dom(const hexsv_ensemble *e, int s) {
    KDom<T> b = ens_base<T>(e), d;
    const int64_t off = e->scen[s].off;
    for (int p = 0; p < 2; ++p)
        for (int f = 0; f < 3; ++f) d.st[p][f] = b.st[p][f] + off;
    d.z = b.z + off;
    d.th = b.th + off;
    d.ap = b.ap + off;
    return d;
}

static void ens_drop_graph(hexsv_ensemble *e) {
    for (int p = 0; p < 2; ++p) {
        if (e->gexec[p]) (void)hipGraphExecDestroy(e->gexec[p]);
        if (e->graph[p]) (void)hipGraphDestroy(e->graph[p]);
        e->gexec[p] = nullptr;
        e->graph[p] = nullptr;
    }
}

static void ens_set_tile(hexsv_ensemble *e, int v) {
    e->tile = v;
    const TileShape ts = ENS_TILES[v];
    for (int s = 0; s < e->n; ++s) {
        EnsScen &sc = e->scen[s];
        sc.ntq = (sc.g.nq + ts.tq - 1) / ts.tq;
        sc.ntiles = sc.ntq * ((sc.g.nr + ts.tr - 1) / ts.tr);
    }
    ens_drop_graph(e);
}

// Batched-mode tiling: tile shape TILES[v] per scenario, global tile order
// scenario by scenario; rebuilds the tile -> scenario table on the device.
static int ens_set_btile(hexsv_ensemble *e, int v) {
    e->btile = v;
    int base = 0;
    std::vector<EnsTile> map;
    for (int s = 0; s < e->n; ++s) {
        EnsScen &sc = e->scen[s];
        int ntq, nt;
        tile_grid(v, sc.g.nq, sc.g.nr, &ntq, &nt);
        sc.bntq = ntq;
        sc.bntiles = nt;
        sc.bbase = base;
        base += nt;
        for (int lt = 0; lt < nt; ++lt) {
            EnsTile tl;
            tl.off = sc.off;
            tl.nq = sc.g.nq;
            tl.nr = sc.g.nr;
            tl.pitch = sc.g.pitch;
            tl.tr = lt / ntq;
            tl.tq = lt - tl.tr * ntq;
            tl.s = s;
            tl.wrap = (sc.g.perq ? 1 : 0) | (sc.g.perr ? 2 : 0);
            map.push_back(tl);
        }
    }
    e->btotal = base;
    e->h_tpar.clear();
    ens_drop_graph(e);
    if (e->d_tiles) HIP_TRY(hipMemcpy(e->d_tiles, map.data(), sizeof(EnsTile) * map.size(),
                                      hipMemcpyHostToDevice));
    return HEXSV_OK;
}

extern "C" void hexsv_ensemble_destroy(hexsv_ensemble *e) {
    if (!e) return;
    ens_drop_graph(e);
    if (e->cap) (void)hipStreamDestroy(e->cap);
    if (e->ev0) (void)hipEventDestroy(e->ev0);
    if (e->ev1) (void)hipEventDestroy(e->ev1);
    if (e->buf) (void)hipFree(e->buf);
    if (e->d_scen) (void)hipFree(e->d_scen);
    if (e->d_ctl) (void)hipFree(e->d_ctl);
    if (e->d_part) (void)hipFree(e->d_part);
    if (e->d_chk) (void)hipFree(e->d_chk);
    if (e->d_order) (void)hipFree(e->d_order);
    if (e->d_queue) (void)hipFree(e->d_queue);
    if (e->d_tiles) (void)hipFree(e->d_tiles);
    if (e->d_bpart) (void)hipFree(e->d_bpart);
    if (e->d_tpar) (void)hipFree(e->d_tpar);
    if (e->h_ctl) (void)hipHostFree(e->h_ctl);
    if (e->h_chk) (void)hipHostFree(e->h_chk);
    delete e;
}

extern "C" int hexsv_ensemble_create(int32_t n, const hexsv_grid *const *grids,
                                     const hexsv_params *params, hexsv_ensemble **out) {
    if (!grids || !params || !out || n < 1) return fail(HEXSV_EINVAL, "ensemble_create: bad argument");
    *out = nullptr;
    const hexsv_params &p = *params;
    if (!(p.g > 0.0) || !(p.cfl > 0.0 && p.cfl < 1.0) || !(p.dt_max > 0.0) || !(p.h_dry >= 0.0))
        return fail(HEXSV_EDOMAIN, "ensemble_create: g, cfl, dt_max or h_dry out of range");
    if (p.precision != HEXSV_FP64 && p.precision != HEXSV_FP32)
        return fail(HEXSV_EINVAL, "ensemble_create: precision %d unknown", p.precision);
    if (p.ensemble_mode < HEXSV_ENS_AUTO || p.ensemble_mode > HEXSV_ENS_BATCHED)
        return fail(HEXSV_EINVAL, "ensemble_create: mode %d unknown", p.ensemble_mode);
    for (int s = 0; s < n; ++s) {
        if (!grids[s]) return fail(HEXSV_EINVAL, "ensemble_create: grid %d is null", s);
        if ((uint64_t)grids[s]->kg.nr * ens_pitch(grids[s]->kg.nq) *
                (p.precision == HEXSV_FP64 ? 8u : 4u) >= (1ull << 32))
            return fail(HEXSV_EUNSUPPORTED, "ensemble_create: scenario %d exceeds 4 GiB per field", s);
    }
    hexsv_ensemble *e = new (std::nothrow) hexsv_ensemble();
    if (!e) return fail(HEXSV_ENOMEM, "ensemble_create: out of host memory");
    e->n = n;
    e->visc = 0;
    e->bc = 0;
    for (int s = 0; s < n; ++s)
        if (grids[s]->n_dirichlet) e->bc = 1;
    e->prec = p.precision;
    e->esz = p.precision == HEXSV_FP64 ? sizeof(double) : sizeof(float);
    e->tile = 0;
    e->ksteps = p.steps_per_graph > 0 ? p.steps_per_graph : 50;
    e->dt_max = p.dt_max;
    e->grids.assign(grids, grids + n);
    e->scen.resize(n);
    e->active.resize(n);
    e->ready.assign(n, 0);
    int64_t off = 0;
    for (int s = 0; s < n; ++s) {
        EnsScen &sc = e->scen[s];
        memset(&sc, 0, sizeof sc);
        sc.off = off;
        sc.g = grids[s]->kg;
        sc.g.pitch = ens_pitch(sc.g.nq);
        const double a = grids[s]->edge;
        sc.kc.g = p.g;
        sc.kc.a = a;
        hexsv_geometry(a, p.cfl, &sc.kc.sigma, &sc.kc.cfl_phi);
        sc.kc.h_dry = p.h_dry;
        sc.kc.area_active = sc.kc.sigma * (double)grids[s]->n_active;
        sc.rn.kind = 0;
        sc.rn.T_d = INFINITY;
        e->active[s] = grids[s]->n_active;
        off += (int64_t)sc.g.nr * sc.g.pitch;
        off = (off + 63) / 64 * 64;  // keep every scenario 64 cells aligned
    }
    e->total = off;
    // mode and tile: explicit, else from the tuning cache (encoded as
    // 100 * mode + tile), else batched steps with the default step tile
    {
        int64_t cells = 0;
        for (int s = 0; s < n; ++s) cells += grids[s]->n_active;
        const int tuned = tuned_tile("ensemble", p.precision, cells, 100 * HEXSV_ENS_BATCHED + DEFAULT_TILE);
        e->mode = p.ensemble_mode == HEXSV_ENS_AUTO ? tuned / 100 : p.ensemble_mode;
        if (e->mode != HEXSV_ENS_PERSISTENT && e->mode != HEXSV_ENS_BATCHED) e->mode = HEXSV_ENS_BATCHED;
        int v = p.tile >= 0 ? p.tile : (p.ensemble_mode == HEXSV_ENS_AUTO ? tuned % 100 : 0);
        if (p.tile < 0 && p.ensemble_mode == HEXSV_ENS_BATCHED) v = DEFAULT_TILE;
        const int lim = e->mode == HEXSV_ENS_PERSISTENT ? NUM_ENS_TILES : NUM_TILES;
        if (v < 0 || v >= lim) {
            delete e;
            return fail(HEXSV_EINVAL, "ensemble_create: tile %d not built for this mode", v);
        }
        ens_set_tile(e, e->mode == HEXSV_ENS_PERSISTENT ? v : 0);
        ens_set_btile(e, e->mode == HEXSV_ENS_BATCHED ? v : DEFAULT_TILE);
        // the persistent kernel is not built for Dirichlet or flux cells
        if (e->bc) e->mode = HEXSV_ENS_BATCHED;
    }
    // largest scenarios first: they bound the length of every launch
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t y) { return grids[x]->n > grids[y]->n; });
    int dev = 0, ncu = 1;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    e->nwg = std::min(n, std::max(ncu, 1));
    hipError_t err = hipMalloc(&e->buf, e->esz * 9 * (size_t)e->total);
    if (err == hipSuccess) err = hipMalloc(&e->d_scen, sizeof(EnsScen) * n);
    if (err == hipSuccess) err = hipMalloc(&e->d_ctl, sizeof(Ctl) * n);
    if (err == hipSuccess) err = hipMalloc(&e->d_part, sizeof(Part) * PRIME_BLOCKS);
    if (err == hipSuccess) err = hipMalloc(&e->d_chk, 8 * sizeof(int32_t));
    if (err == hipSuccess) err = hipMalloc(&e->d_order, sizeof(int32_t) * n);
    if (err == hipSuccess) err = hipMalloc(&e->d_queue, sizeof(uint32_t));
    // records for the batched tile variant with the most tiles
    int maxtiles = 0;
    for (int v = 0; v < NUM_TILES; ++v) {
        int tot = 0;
        for (int s = 0; s < n; ++s) {
            int ntq, nt;
            tile_grid(v, grids[s]->kg.nq, grids[s]->kg.nr, &ntq, &nt);
            tot += nt;
        }
        maxtiles = std::max(maxtiles, tot);
    }
    if (err == hipSuccess) err = hipMalloc(&e->d_bpart, sizeof(Part) * (size_t)maxtiles);
    if (err == hipSuccess) err = hipMalloc(&e->d_tiles, sizeof(EnsTile) * (size_t)maxtiles);
    if (err == hipSuccess) err = hipMalloc(&e->d_tpar, (size_t)maxtiles);
    if (err == hipSuccess) err = hipMemset(e->d_tpar, 0, (size_t)maxtiles);
    if (err == hipSuccess) err = hipHostMalloc(&e->h_ctl, sizeof(Ctl) * n, hipHostMallocDefault);
    if (err == hipSuccess) err = hipHostMalloc(&e->h_chk, 8 * sizeof(int32_t), hipHostMallocDefault);
    if (err == hipSuccess) err = hipStreamCreateWithFlags(&e->cap, hipStreamNonBlocking);
    if (err == hipSuccess) err = hipMemcpy(e->d_scen, e->scen.data(), sizeof(EnsScen) * n, hipMemcpyHostToDevice);
    if (err == hipSuccess) err = hipMemcpy(e->d_order, order.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice);
    if (err == hipSuccess) err = hipMemset(e->buf, 0, e->esz * 9 * (size_t)e->total);
    if (err == hipSuccess && ens_set_btile(e, e->btile) != HEXSV_OK) err = hipErrorUnknown;
    if (err != hipSuccess) {
        hexsv_ensemble_destroy(e);
        return fail(HEXSV_ENOMEM, "ensemble_create: allocation failed: %s", hipGetErrorString(err));
    }
    memset(e->h_ctl, 0, sizeof(Ctl) * n);
    for (int s = 0; s < n; ++s) e->h_ctl[s].err_cell = -1;
    *out = e;
    return HEXSV_OK;
}

static int ens_check(hexsv_ensemble *e, int s, bool fields, const double *a, const double *b,
                     const double *c, hipStream_t stream, int32_t *cnt, int32_t *first, int32_t *why,
                     double *c_dirichlet = nullptr) {
    const int32_t init[8] = {0, 0x7fffffff, 0, 0, 0, 0, 0, 0};
    memcpy(e->h_chk, init, sizeof init);
    HIP_TRY(hipMemcpyAsync(e->d_chk, e->h_chk, sizeof init, hipMemcpyHostToDevice, stream));
    const hexsv_grid *g = e->grids[s];
    if (fields) HIP_TRY(launch_check_fields(a, b, c, g->d_active, g->n, e->d_chk, stream));
    else HIP_TRY(launch_check_state(a, b, c, g->d_active, g->n, e->scen[s].kc.g, e->d_chk, stream));
    HIP_TRY(hipMemcpyAsync(e->h_chk, e->d_chk, sizeof init, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    *cnt = e->h_chk[0];
    *first = e->h_chk[1];
    *why = e->h_chk[2];
    if (c_dirichlet) memcpy(c_dirichlet, e->h_chk + 4, sizeof(double));
    return HEXSV_OK;
}

template <typename T>
static int ens_import(hexsv_ensemble *e, int s, const double *z, const double *th, const double *ap,
                      const double *h, const double *v1, const double *v2, hipStream_t stream) {
    const KDom<T> d = ens_dom<T>(e, s);
    const hexsv_grid *g = e->grids[s];
    // rows land at the scenario's pitch; the padding cells stay zero (theta 0: outside)
    const int nq = g->kg.nq, pitch = e->scen[s].g.pitch;
    HIP_TRY(launch_import<T>(z, (T *)d.z, g->d_active, 0, g->n, stream, nq, pitch));
    HIP_TRY(launch_import<T>(th, (T *)d.th, g->d_active, 2, g->n, stream, nq, pitch));
    HIP_TRY(launch_import<T>(ap, (T *)d.ap, g->d_active, 0, g->n, stream, nq, pitch));
    for (int p = 0; p < 2; ++p) {
        HIP_TRY(launch_import<T>(h, d.st[p][0], g->d_active, 1, g->n, stream, nq, pitch));
        HIP_TRY(launch_import<T>(v1, d.st[p][1], g->d_active, 1, g->n, stream, nq, pitch));
        HIP_TRY(launch_import<T>(v2, d.st[p][2], g->d_active, 1, g->n, stream, nq, pitch));
    }
    HIP_TRY(launch_prime<T>(d, (int64_t)g->kg.nr * pitch, e->scen[s].kc, e->d_ctl + s, e->d_part,
                            PRIME_BLOCKS, 1, stream));
    return HEXSV_OK;
}

extern "C" int hexsv_ensemble_set_scenario(hexsv_ensemble *e, int32_t s, const double *d_z,
                                           const double *d_theta, const double *d_alpha_p,
                                           double alpha_s, const hexsv_rain *rain, double t0,
                                           const double *d_h, const double *d_v1,
                                           const double *d_v2, hipStream_t stream) {
    if (!e || s < 0 || s >= e->n || !d_z || !d_theta || !d_alpha_p || !rain || !d_h || !d_v1 || !d_v2)
        return fail(HEXSV_EINVAL, "ensemble_set_scenario: bad argument");
    if (!(alpha_s >= 0.0) || !isfinite(alpha_s) || !isfinite(t0))
        return fail(HEXSV_EDOMAIN, "ensemble_set_scenario: alpha_s or t0 out of range");
    if ((rain->kind != 0 && rain->kind != 1) || !(rain->i_a >= 0.0) ||
        (rain->kind == 1 && !(rain->t_a > 0.0 && rain->T_d > rain->t_a && isfinite(rain->T_d))))
        return fail(HEXSV_EDOMAIN, "ensemble_set_scenario: rain parameters out of range");
    int32_t cnt, first, why;
    int rc = ens_check(e, s, true, d_z, d_theta, d_alpha_p, stream, &cnt, &first, &why);
    if (rc) return rc;
    if (cnt) return fail(HEXSV_EDOMAIN, "ensemble_set_scenario %d: %d invalid cells; first cell %d", s, cnt, first);
    double c_dirichlet = 0.0;
    rc = ens_check(e, s, false, d_h, d_v1, d_v2, stream, &cnt, &first, &why, &c_dirichlet);
    if (rc) return rc;
    if (cnt) return fail(HEXSV_EDOMAIN, "ensemble_set_scenario %d: %d invalid state cells; first cell %d", s, cnt, first);
    EnsScen &sc = e->scen[s];
    sc.kc.alpha_s = alpha_s;
    sc.kc.c_floor = c_dirichlet;  // read by the kernels from the device copy below
    sc.rn.kind = rain->kind;
    sc.rn.i_a = rain->i_a;
    sc.rn.t_a = rain->t_a;
    sc.rn.T_d = rain->T_d;
    HIP_TRY(hipMemcpyAsync(e->d_scen + s, &sc, sizeof(EnsScen), hipMemcpyHostToDevice, stream));
    Ctl &c = e->h_ctl[s];
    memset(&c, 0, sizeof c);
    c.t = t0;
    c.t_end = t0;
    c.dt_max = e->dt_max;
    c.err_cell = -1;
    HIP_TRY(hipMemcpyAsync(e->d_ctl + s, &c, sizeof(Ctl), hipMemcpyHostToDevice, stream));
    rc = e->prec == HEXSV_FP64 ? ens_import<double>(e, s, d_z, d_theta, d_alpha_p, d_h, d_v1, d_v2, stream)
                               : ens_import<float>(e, s, d_z, d_theta, d_alpha_p, d_h, d_v1, d_v2, stream);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(e->h_ctl + s, e->d_ctl + s, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    e->ready[s] = 1;
    return HEXSV_OK;
}

// One persistent launch of ksteps steps, or ksteps batched steps whose live
// scenarios start from buffer parity p0 (launch k reads parity (p0 + k) & 1).
static hipError_t ens_launch(hexsv_ensemble *e, int mode, int v, int ksteps, int p0,
                             hipStream_t st) {
    if (mode == HEXSV_ENS_PERSISTENT)
        return e->prec == HEXSV_FP64
                   ? launch_ensemble<double>(v, ens_base<double>(e), e->d_scen, e->d_ctl, e->d_order,
                                             e->n, e->d_queue, ksteps, e->nwg, st)
                   : launch_ensemble<float>(v, ens_base<float>(e), e->d_scen, e->d_ctl, e->d_order,
                                            e->n, e->d_queue, ksteps, e->nwg, st);
    hipError_t err = hipSuccess;
    for (int k = 0; k < ksteps && err == hipSuccess; ++k)
        err = e->prec == HEXSV_FP64
                  ? launch_ens_step<double>(v, e->visc != 0, e->bc != 0, ens_base<double>(e),
                                            e->d_scen, e->d_tiles, e->d_tpar, e->d_ctl,
                                            e->d_bpart, e->btotal, e->n, (p0 + k) & 1, st)
                  : launch_ens_step<float>(v, e->visc != 0, e->bc != 0, ens_base<float>(e),
                                           e->d_scen, e->d_tiles, e->d_tpar, e->d_ctl,
                                           e->d_bpart, e->btotal, e->n, (p0 + k) & 1, st);
    return err;
}

static int ens_capture(hexsv_ensemble *e) {
    ens_drop_graph(e);
    for (int p0 = 0; p0 < 2; ++p0) {
        HIP_TRY(hipStreamBeginCapture(e->cap, hipStreamCaptureModeThreadLocal));
        hipError_t err = ens_launch(e, e->mode,
                                    e->mode == HEXSV_ENS_PERSISTENT ? e->tile : e->btile,
                                    e->ksteps, p0, e->cap);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(e->cap, &g);
        if (err != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(HEXSV_EHIP, "ensemble graph capture failed: %s",
                        hipGetErrorString(err != hipSuccess ? err : e2));
        }
        e->graph[p0] = g;
        HIP_TRY(hipGraphInstantiate(&e->gexec[p0], g, nullptr, nullptr, 0));
    }
    return HEXSV_OK;
}

// The batched launches' load hints: every tile of scenario s gets the offset
// c[s].parity, so that launch k after this call hints parity k & 1 to all tiles
// and every scenario that is live then reads the buffers of its own parity
// (scenarios stopped at different step counts by runs to their own t_end keep
// their relative parities while they step together).  Uploads only a change.
static hipError_t ens_set_parities(hexsv_ensemble *e, const Ctl *c, hipStream_t st) {
    std::vector<uint8_t> tp((size_t)e->btotal);
    for (int s = 0; s < e->n; ++s)
        std::fill(tp.begin() + e->scen[s].bbase, tp.begin() + e->scen[s].bbase + e->scen[s].bntiles,
                  (uint8_t)(c[s].parity & 1));
    if (tp == e->h_tpar) return hipSuccess;
    // ordered before the launches that read it: the stream's pending work first, then a
    // copy that has finished when it returns
    hipError_t err = hipStreamSynchronize(st);
    if (err == hipSuccess) err = hipMemcpy(e->d_tpar, tp.data(), tp.size(), hipMemcpyHostToDevice);
    if (err == hipSuccess) e->h_tpar.swap(tp);
    return err;
}

static bool ens_done(const Ctl &c) { return c.err || c.t >= c.t_end || c.steps >= c.step_limit; }

extern "C" int hexsv_ensemble_run(hexsv_ensemble *e, const double *t_end, int64_t max_steps,
                                  hipStream_t stream) {
    if (!e || !t_end) return fail(HEXSV_EINVAL, "ensemble_run: bad argument");
    for (int s = 0; s < e->n; ++s)
        if (!e->ready[s]) return fail(HEXSV_ESTATE, "ensemble_run: scenario %d has no state", s);
    HIP_TRY(hipMemcpyAsync(e->h_ctl, e->d_ctl, sizeof(Ctl) * e->n, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    std::vector<int64_t> steps0(e->n);
    for (int s = 0; s < e->n; ++s) {
        Ctl &c = e->h_ctl[s];
        if (!(t_end[s] >= c.t)) return fail(HEXSV_EDOMAIN, "ensemble_run: t_end[%d]=%g before t=%g", s, t_end[s], c.t);
        c.t_end = t_end[s];
        c.dt_max = e->dt_max;
        c.step_limit = max_steps > 0 ? c.steps + max_steps : INT64_MAX;
        steps0[s] = c.steps;
    }
    HIP_TRY(hipMemcpyAsync(e->d_ctl, e->h_ctl, sizeof(Ctl) * e->n, hipMemcpyHostToDevice, stream));
    if (!e->gexec[0]) {
        int rc = ens_capture(e);
        if (rc) return rc;
    }
    if (e->mode == HEXSV_ENS_BATCHED) HIP_TRY(ens_set_parities(e, e->h_ctl, stream));
    int64_t launched = 0;  // batched launches since the parities were set
    for (;;) {
        if (e->timing) HIP_TRY(hipEventRecord(e->ev0, stream));
        HIP_TRY(hipGraphLaunch(e->gexec[launched & 1], stream));
        launched += e->ksteps;
        if (e->timing) HIP_TRY(hipEventRecord(e->ev1, stream));
        HIP_TRY(hipMemcpyAsync(e->h_ctl, e->d_ctl, sizeof(Ctl) * e->n, hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        if (e->timing) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, e->ev0, e->ev1));
            e->timed_ms += ms;
            e->timed_launches += 1;
        }
        bool all = true;
        for (int s = 0; s < e->n; ++s) {
            if (e->h_ctl[s].err)
                return fail(HEXSV_ENUMERIC, "ensemble_run: non-finite value in scenario %d at cell %d",
                            s, e->h_ctl[s].err_cell);
            all = all && ens_done(e->h_ctl[s]);
        }
        if (all) break;
    }
    if (e->timing)
        for (int s = 0; s < e->n; ++s) e->timed_updates += (e->h_ctl[s].steps - steps0[s]) * e->active[s];
    return HEXSV_OK;
}

extern "C" int hexsv_ensemble_get_state(const hexsv_ensemble *ec, int32_t s, double *d_h,
                                        double *d_v1, double *d_v2, double *d_q1, double *d_q2,
                                        hipStream_t stream) {
    hexsv_ensemble *e = const_cast<hexsv_ensemble *>(ec);
    if (!e || s < 0 || s >= e->n) return fail(HEXSV_EINVAL, "ensemble_get_state: bad argument");
    if (!e->ready[s]) return fail(HEXSV_ESTATE, "ensemble_get_state: scenario %d has no state", s);
    HIP_TRY(hipMemcpyAsync(e->h_ctl + s, e->d_ctl + s, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    const int par = e->h_ctl[s].parity;
    const int64_t n = e->grids[s]->n;
    const int nq = e->grids[s]->kg.nq, pitch = e->scen[s].g.pitch;
    if (e->prec == HEXSV_FP64)
        HIP_TRY(launch_export<double>(ens_dom<double>(e, s), par, n, d_h, d_v1, d_v2, d_q1, d_q2, stream,
                                      nq, pitch));
    else
        HIP_TRY(launch_export<float>(ens_dom<float>(e, s), par, n, d_h, d_v1, d_v2, d_q1, d_q2, stream,
                                     nq, pitch));
    return HEXSV_OK;
}

extern "C" int hexsv_ensemble_get_books(hexsv_ensemble *e, int32_t s, hexsv_books *out,
                                        hipStream_t stream) {
    if (!e || !out || s < 0 || s >= e->n) return fail(HEXSV_EINVAL, "ensemble_get_books: bad argument");
    HIP_TRY(hipMemcpyAsync(e->h_ctl + s, e->d_ctl + s, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    const Ctl &c = e->h_ctl[s];
    out->t = c.t;
    out->initial = c.initial;
    out->stored = c.stored;
    out->rain = c.rain;
    out->outflow = c.outflow;
    out->clamp = c.clamp;
    // water supplied: initial, rain and any net inflow through Dirichlet edges
    double ref = c.initial + c.rain + (c.outflow < 0.0 ? -c.outflow : 0.0);
    if (ref < 1e-300) ref = 1e-300;
    out->residual = fabs(c.stored - (c.initial + c.rain - c.outflow + c.clamp)) / ref;
    out->steps = c.steps;
    out->dt_min = c.dt_min;
    out->dt_max_seen = c.dt_max_seen;
    return HEXSV_OK;
}

extern "C" int hexsv_ensemble_set_viscosity(hexsv_ensemble *e, int32_t on) {
    if (!e) return fail(HEXSV_EINVAL, "ensemble_set_viscosity: null ensemble");
    if (on != 0 && on != 1) return fail(HEXSV_EINVAL, "ensemble_set_viscosity: on must be 0 or 1");
    e->visc = on;
    if (on && e->mode == HEXSV_ENS_PERSISTENT) e->mode = HEXSV_ENS_BATCHED;
    ens_drop_graph(e);
    return HEXSV_OK;
}

extern "C" int hexsv_ensemble_timing(hexsv_ensemble *e, int32_t enable, double *gpu_ms,
                                     int64_t *cell_updates, int64_t *launches) {
    if (!e) return fail(HEXSV_EINVAL, "ensemble_timing: null ensemble");
    if (gpu_ms) *gpu_ms = e->timed_ms;
    if (cell_updates) *cell_updates = e->timed_updates;
    if (launches) *launches = e->timed_launches;
    if (enable >= 0) {
        if (enable && !e->ev0) {
            HIP_TRY(hipEventCreate(&e->ev0));
            HIP_TRY(hipEventCreate(&e->ev1));
        }
        e->timing = enable != 0;
        e->timed_ms = 0.0;
        e->timed_updates = 0;
        e->timed_launches = 0;
    }
    return HEXSV_OK;
}

extern "C" int hexsv_ensemble_autotune(hexsv_ensemble *e, int32_t ksteps, const char *cache_path,
                                       int32_t *best_tile, double *best_ms, hipStream_t stream) {
    if (!e || ksteps < 1) return fail(HEXSV_EINVAL, "ensemble_autotune: bad argument");
    for (int s = 0; s < e->n; ++s)
        if (!e->ready[s]) return fail(HEXSV_ESTATE, "ensemble_autotune: scenario %d has no state", s);
    // save state and control blocks; every variant runs from the same start
    const size_t sbytes = e->esz * 6 * (size_t)e->total;
    void *save = nullptr;
    HIP_TRY(hipMalloc(&save, sbytes));
    std::vector<Ctl> c0(e->n);
    int rc = HEXSV_OK;
    hipError_t he = hipMemcpyAsync(save, e->buf, sbytes, hipMemcpyDeviceToDevice, stream);
    if (he == hipSuccess) he = hipMemcpyAsync(c0.data(), e->d_ctl, sizeof(Ctl) * e->n, hipMemcpyDeviceToHost, stream);
    if (he == hipSuccess) he = hipStreamSynchronize(stream);
    const int nvar = NUM_ENS_TILES + NUM_TILES;  // persistent variants, then batched ones
    std::vector<double> times(nvar, INFINITY);
    int best = -1;
    double bms = INFINITY;
    hipEvent_t a = nullptr, b = nullptr;
    if (he == hipSuccess) he = hipEventCreate(&a);
    if (he == hipSuccess) he = hipEventCreate(&b);
    for (int c = 0; c < nvar && he == hipSuccess; ++c) {
        const int mode = c < NUM_ENS_TILES ? HEXSV_ENS_PERSISTENT : HEXSV_ENS_BATCHED;
        const int v = c < NUM_ENS_TILES ? c : c - NUM_ENS_TILES;
        // the persistent kernel is built without viscosity and boundary cells
        if ((e->visc || e->bc) && mode == HEXSV_ENS_PERSISTENT) continue;
        if (mode == HEXSV_ENS_PERSISTENT) ens_set_tile(e, v);
        else if (ens_set_btile(e, v) != HEXSV_OK) he = hipErrorUnknown;
        std::vector<Ctl> cc = c0;
        for (auto &x : cc) {
            x.t_end = INFINITY;
            x.step_limit = x.steps + ksteps;
        }
        if (he == hipSuccess) he = hipMemcpyAsync(e->d_scen, e->scen.data(), sizeof(EnsScen) * e->n, hipMemcpyHostToDevice, stream);
        if (he == hipSuccess) he = hipMemcpyAsync(e->d_ctl, cc.data(), sizeof(Ctl) * e->n, hipMemcpyHostToDevice, stream);
        if (he == hipSuccess && mode == HEXSV_ENS_BATCHED) he = ens_set_parities(e, cc.data(), stream);
        if (he == hipSuccess) he = hipEventRecord(a, stream);
        if (he == hipSuccess) he = ens_launch(e, mode, v, ksteps, 0, stream);
        if (he == hipSuccess) he = hipEventRecord(b, stream);
        if (he == hipSuccess) he = hipEventSynchronize(b);
        float ms = 0.f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, a, b);
        if (he == hipSuccess) {
            times[c] = ms;
            if (ms < bms) { bms = ms; best = c; }
        }
        if (he == hipSuccess) he = hipMemcpyAsync(e->buf, save, sbytes, hipMemcpyDeviceToDevice, stream);
    }
    if (he == hipSuccess) he = hipMemcpyAsync(e->d_ctl, c0.data(), sizeof(Ctl) * e->n, hipMemcpyHostToDevice, stream);
    if (he == hipSuccess) he = hipStreamSynchronize(stream);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    (void)hipFree(save);
    if (he != hipSuccess) return fail(HEXSV_EHIP, "ensemble_autotune: %s", hipGetErrorString(he));
    // the default (batched steps, DEFAULT_TILE) unless a variant beats it by more than 3 %:
    // trial launches of a few steps differ by about that much from run to run
    const int def = NUM_ENS_TILES + DEFAULT_TILE;
    if (best >= 0 && times[def] <= 1.03 * bms) {
        best = def;
        bms = times[def];
    }
    if (best < NUM_ENS_TILES) {
        e->mode = HEXSV_ENS_PERSISTENT;
        ens_set_tile(e, best);
    } else {
        e->mode = HEXSV_ENS_BATCHED;
        if (ens_set_btile(e, best - NUM_ENS_TILES) != HEXSV_OK) return HEXSV_EHIP;
    }
    HIP_TRY(hipMemcpy(e->d_scen, e->scen.data(), sizeof(EnsScen) * e->n, hipMemcpyHostToDevice));
    ens_drop_graph(e);
    const int code = e->mode == HEXSV_ENS_PERSISTENT ? 100 * HEXSV_ENS_PERSISTENT + e->tile
                                                      : 100 * HEXSV_ENS_BATCHED + e->btile;
    if (best_tile) *best_tile = code;
    if (best_ms) *best_ms = bms;
    int64_t cells = 0;
    for (int s = 0; s < e->n; ++s) cells += e->active[s];
    if (cache_path && *cache_path)
        rc = tune_cache_store(cache_path, "ensemble", e->prec, cells, code, bms, times.data(), nvar);
    return rc;
}

extern "C" int hexsv_ensemble_info(const hexsv_ensemble *e, int32_t *workgroups, int32_t *tile,
                                   int64_t *cells, int32_t *steps_per_launch, int32_t *mode) {
    if (!e) return fail(HEXSV_EINVAL, "ensemble_info: null ensemble");
    if (workgroups) *workgroups = e->mode == HEXSV_ENS_PERSISTENT ? e->nwg : e->btotal;
    if (tile) *tile = e->mode == HEXSV_ENS_PERSISTENT ? e->tile : e->btile;
    if (mode) *mode = e->mode;
    if (cells) {
        int64_t c = 0;
        for (int s = 0; s < e->n; ++s) c += e->active[s];
        *cells = c;
    }
    if (steps_per_launch) *steps_per_launch = e->ksteps;
    return HEXSV_OK;
}
