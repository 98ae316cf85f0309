/*
 * hexsv.h — C-ABI of the MI355X (gfx950) time stepper for the porous
 * Saint-Venant model on a regular hexagonal raster.
 *
 * Method: Ion, Marinescu, Cruceanu, "ASTERIX: Module for modelling the water
 * flow on vegetated hillslopes" (arXiv 2406.14933).  Model: Sec. 2.1,
 * eq. swe_vegm_rm.02 with the Darcy-Weisbach soil friction (eq_tsa_darcy), the
 * plant drag (eq_tpa) and their sum K(h, theta) (eq_K_h_theta).  Scheme:
 * Sec. 2.2, eqs. fvm_2D_eq.04-.06 (interface values), fvm_2D_eq_frac.01
 * (operators L, J, S) and fvm_2D_eq_frac.07 (full step), solved as in
 * Appendix A (fractional steps .05/.06, CFL time step .12/.13, closed-form
 * friction solve miu-formula).  Rain: constant or the triangular hyetograph
 * of Appendix C.
 *
 * Conventions
 *  - Units SI (m, s, m/s).  g defaults to 9.81 m/s^2.
 *  - Raster: nq x nr axial parallelogram of pointy-top hexagons of edge a
 *    (the paper's "cell radius"), cell (q, r) at index i = r*nq + q, centre
 *    (a*sqrt(3)*(q + r/2), 1.5*a*r).  Direction k in 0..5 points at k*60
 *    degrees: (dq,dr) = (+1,0),(0,+1),(-1,+1),(-1,0),(0,-1),(+1,-1).
 *  - Sides: S is r = -1, E is q = nq, N is r = nr, W is q = -1.  An edge that
 *    leaves the raster (after periodic wraps) takes the code of the side its
 *    outside neighbour lies on (S/N when r is out of range, else E/W), or of
 *    a segment of that side containing the outside neighbour's position
 *    along the side (q for S/N, r for E/W).  Edges into inactive cells take
 *    mask_bc.  WALL edges carry no flux or pressure term; OUTFLOW edges see a
 *    ghost with the cell's h, v, theta and the terrain extrapolated linearly
 *    through the opposite neighbour.
 *  - Dirichlet cells (active == 2; the prescribed inflow state of Sec. 3.2.1,
 *    eq. numerics-bc): a band of cells outside the domain held at the state
 *    set_state gives them.  They are never updated and are not in the books
 *    or c_max.  An edge from an updated cell into one (code DIRICHLET) reads
 *    it like a neighbour, but the interface velocity is the prescribed
 *    velocity itself rather than the mean of eq. fvm_2D_eq.04, so the inflow
 *    flux is l h_D (v_D . n); that flux enters the books as negative outflow.
 *    Viscous sums (set_viscosity) run over INTERIOR edges only.
 *  - Given-flux cells (active == 3; the given mass flux of Sec. 2.2's boundary
 *    conditions, e.g. the flume inflow u h = q_L of Sec. 3.3.2): held like
 *    Dirichlet cells, but what they prescribe is the discharge h v across the
 *    edge (their theta is not used).  An edge into one (code FLUX) carries the
 *    mass flux l h_F (v_F . n) and momentum flux l h_F (v_F . n) v_F, and its
 *    pressure term sees the updated cell's own depth over the flux cell's bed:
 *    0.5 l g (z_F + h_i - z_i - h_i) theta_i h_i.  The flux is booked with the
 *    outflow.
 *  - The wave speeds |v| + sqrt(g h) of Dirichlet and flux cells enter c_max
 *    (eq. .12).  Surrogate windows refuse grids with either kind; an ensemble
 *    holding either kind runs in the batched-step mode.
 *  - Every d_* pointer is caller-owned device memory (e.g. a torch tensor's
 *    data_ptr()), read or written only during the call (stream-ordered on
 *    `stream`); the library copies inputs into its own buffers and never frees
 *    caller memory.  Handles are library-owned; *_destroy frees them.  A
 *    handle is not thread-safe; distinct handles are independent.
 *  - Every int-returning call returns HEXSV_OK (0) or a negative hexsv_status
 *    and sets a thread-local message readable with hexsv_last_error().  No
 *    call aborts or throws.
 */
#ifndef HEXSV_H
#define HEXSV_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HEXSV_OK = 0,
    HEXSV_EINVAL = -1,      /* malformed argument (null handle, bad size, ...) */
    HEXSV_EDOMAIN = -2,     /* a field or parameter outside the model's domain */
    HEXSV_ENOMEM = -3,      /* device or host allocation failed */
    HEXSV_EHIP = -4,        /* a HIP runtime call failed (message has hipGetErrorString) */
    HEXSV_ENUMERIC = -5,    /* a non-finite value appeared during a run */
    HEXSV_ESTATE = -6,      /* call out of order (e.g. run before set_state) */
    HEXSV_EUNSUPPORTED = -7 /* option not built */
} hexsv_status;

typedef enum { HEXSV_FP64 = 0, HEXSV_FP32 = 1 } hexsv_precision;

/* edge codes and side kinds */
enum { HEXSV_INTERIOR = 0, HEXSV_WALL = 1, HEXSV_OUTFLOW = 2, HEXSV_PERIODIC = 3,
       HEXSV_DIRICHLET = 4, /* edge codes only: the neighbour is a Dirichlet cell */
       HEXSV_FLUX = 5       /* edge codes only: the neighbour is a given-flux cell */ };
/* sides */
enum { HEXSV_S = 0, HEXSV_E = 1, HEXSV_N = 2, HEXSV_W = 3 };

#define HEXSV_MAX_SEGMENTS 8

/* Part [lo, hi) of a side whose boundary edges take `code` (WALL or OUTFLOW). */
typedef struct {
    int32_t side, lo, hi, code;
} hexsv_segment;

/* Raster and boundary description (Sec. 2.2 (a) cell decomposition; boundary
 * kinds of Sec. 3 "Boundary conditions": free discharge and impermeable wall). */
typedef struct {
    int32_t nq, nr;          /* cells along q and r, each >= 1 */
    double edge;             /* hexagon edge length a > 0 (m) */
    int32_t side_bc[4];      /* WALL, OUTFLOW or PERIODIC per side S,E,N,W;
                                E/W (and S/N) must agree on PERIODIC */
    int32_t nseg;            /* number of valid entries in seg (<= 8) */
    hexsv_segment seg[HEXSV_MAX_SEGMENTS];
    const uint8_t *active;   /* host, nq*nr, nullable (all 1): 0 = outside the domain,
                                1 = in the domain, 2 = Dirichlet cell, 3 = given-flux
                                cell; other values EINVAL */
    int32_t mask_bc;         /* code of edges into inactive cells: WALL or OUTFLOW */
} hexsv_grid_desc;

/* Scheme parameters (Appendix A; control parameters listed in Sec. 3). */
typedef struct {
    double g;                /* gravitational acceleration, > 0 */
    double cfl;              /* Courant number in (0, 1) (Appendix A, eq. .12) */
    double dt_max;           /* maximum time step, > 0 */
    double h_dry;            /* >= 0; cells with h^{n+1} < h_dry get v = 0 (0: off) */
    int32_t precision;       /* hexsv_precision */
    int32_t steps_per_graph; /* steps captured per graph replay (0: default 100) */
    int32_t tile;            /* tile variant index (< 0: tuned or default) */
    int32_t wg_per_cu;       /* must be 0 (one workgroup per tile) */
    int32_t ensemble_mode;   /* ensembles only: HEXSV_ENS_* */
    int32_t reserved;
} hexsv_params;

/* Ensemble execution modes: the persistent kernel (one workgroup sweeps one
 * scenario, all scenarios in one launch), or batched steps (each launch moves
 * every live scenario one step, one workgroup per tile of any scenario). */
enum { HEXSV_ENS_AUTO = 0, HEXSV_ENS_PERSISTENT = 1, HEXSV_ENS_BATCHED = 2 };

/* Rain source of the mass equation (Sec. 2.1 (c), Appendix C).
 * kind 0: r = i_a for 0 <= t <= T_d (T_d may be +inf), else 0.
 * kind 1: triangular hyetograph: i_a t/t_a on [0, t_a], i_a (1 - t/T_d)/(1 - t_a/T_d)
 *         on (t_a, T_d], 0 otherwise.  r is evaluated at t^{n+1}. */
typedef struct {
    int32_t kind;
    double i_a;              /* m/s */
    double t_a, T_d;         /* s */
} hexsv_rain;

/* Volume books (the rainfall / water out / water left table of the paper's
 * Susita experiment), all FP64, in m^3. */
typedef struct {
    double t;         /* current time */
    double initial;   /* sum sigma*theta*h at set_state */
    double stored;    /* sum sigma*theta*h now */
    double rain;      /* rain volume added */
    double outflow;   /* volume that left the surface: through OUTFLOW edges, into
                         the soil (infiltration), and through Dirichlet and flux
                         edges, where inflow counts negative */
    double clamp;     /* volume added by clamping negative theta*h to zero */
    double residual;  /* |stored - (initial + rain - outflow + clamp)| /
                         (initial + rain + max(-outflow, 0)) */
    int64_t steps;    /* steps taken since set_state */
    double dt_min, dt_max_seen;
} hexsv_books;

typedef struct hexsv_grid hexsv_grid;
typedef struct hexsv_sim hexsv_sim;
typedef struct hexsv_ensemble hexsv_ensemble;
typedef struct hexsv_surrogate hexsv_surrogate;

/* Library version and the thread-local message of the last failed call. */
const char *hexsv_version(void);
const char *hexsv_last_error(void);

/* ---------------------------------------------------------------- raster */

/* Validate `desc` and build a raster handle (copies `active`).
 * EINVAL: sizes, codes or segments malformed.  ENOMEM. */
int hexsv_grid_create(const hexsv_grid_desc *desc, hexsv_grid **out);
void hexsv_grid_destroy(hexsv_grid *grid);
/* Number of cells nq*nr and of updated cells (active == 1). */
int hexsv_grid_counts(const hexsv_grid *grid, int64_t *cells, int64_t *active);

/* Neighbour, edge-code and index tables of the raster (Sec. 2.2 (a): the cell
 * decomposition and the neighbour set N(i) of each cell), computed on the device
 * by one kernel (one thread per cell):
 *   nbr[i*6+k]  index of the neighbour across edge k for INTERIOR (periodic
 *               wraps included), DIRICHLET and FLUX edges, -1 otherwise;
 *   code[i*6+k] edge code; cells outside the domain (active == 0) get six WALL;
 *   q[i], r[i]  axial coordinates of cell i = r*nq + q.
 * The step kernels do not read these tables (they derive neighbours and codes
 * from (q, r) on the fly); they are for export and validation.
 * hexsv_grid_tables_device writes caller-allocated device arrays (nq*nr*6 int32,
 * nq*nr*6 uint8, nq*nr int32, nq*nr int32; each nullable), stream-ordered.
 * hexsv_grid_tables writes caller-allocated host arrays of the same sizes (each
 * nullable); it stages them in a temporary device buffer, runs the same kernel
 * and synchronises the device.  ENOMEM / EHIP on allocation or copy failure. */
int hexsv_grid_tables_device(const hexsv_grid *grid, int32_t *d_nbr, uint8_t *d_code,
                             int32_t *d_q, int32_t *d_r, hipStream_t stream);
int hexsv_grid_tables(const hexsv_grid *grid, int32_t *nbr, uint8_t *code, int32_t *q,
                      int32_t *r);

/* ------------------------------------------------------ single catchment */

/* Create a simulation on `grid` (the grid must outlive it).  Allocates the
 * double-buffered state and static fields in the chosen precision.
 * EDOMAIN: cfl not in (0,1), dt_max <= 0, g <= 0, h_dry < 0. */
int hexsv_sim_create(const hexsv_grid *grid, const hexsv_params *params, hexsv_sim **out);
void hexsv_sim_destroy(hexsv_sim *sim);

/* Static fields (Sec. 2.1 (a), (b), (f), (e)): terrain z, porosity theta and
 * plant coefficient alpha_p per cell (device FP64 arrays of nq*nr), and the
 * Darcy-Weisbach soil coefficient of eq_tsa_darcy: per cell in d_alpha_s
 * (device FP64, nq*nr; the step kernel then reads it as a seventh field, in the
 * extended instance) or, when d_alpha_s is null, the one value alpha_s.
 * EDOMAIN (after a device check, synchronising `stream`): theta not in (0,1] on
 * an active cell, alpha_p < 0, non-finite z, alpha_s < 0 or non-finite (the
 * scalar, or any active cell of the field).  The message names the first
 * offending cell.  Surrogate windows refuse a simulation with a soil field. */
int hexsv_sim_set_fields(hexsv_sim *sim, const double *d_z, const double *d_theta,
                         const double *d_alpha_p, const double *d_alpha_s, double alpha_s,
                         hipStream_t stream);

/* Rain forcing.  EDOMAIN: i_a < 0, kind 1 with t_a <= 0 or T_d <= t_a. */
int hexsv_sim_set_rain(hexsv_sim *sim, const hexsv_rain *rain);

/* Momentum flux with artificial viscosity (on = 1), for shocks and the
 * Riemann problem (Sec. 3.2.3, Appendix A, eqs. eq_artif_visc and eq_visc1):
 * J^v_a,i = J_a,i + sum over the interior edges of l c_ij mu_ij ((v_a)_j -
 * (v_a)_i), c_ij = max(c_i, c_j), c = |v| + sqrt(g h), mu_ij =
 * 2 m_i m_j / (m_i + m_j), m = theta*h; explicit, like J.  Off (0) by default.
 * Takes effect from the next run; surrogate windows refuse a viscous sim
 * (EUNSUPPORTED).  EINVAL: on not 0 or 1. */
int hexsv_sim_set_viscosity(hexsv_sim *sim, int32_t on);

/* Linear soil resistance -tau*h*v (1/s), the law of the Thacker test
 * (Sec. 3.2.2, Appendix B), added to the friction terms of the momentum step
 * and, like them, implicit in v^{n+1} (weighted by theta like the soil term):
 * the coefficient of v becomes m^{n+1} (1 + dt*tau), m = theta*h.  tau = 0
 * (the default) leaves the paper's Darcy-Weisbach scheme unchanged bit for bit.
 * Takes effect from the next run.  EDOMAIN: tau < 0 or non-finite. */
int hexsv_sim_set_linear_friction(hexsv_sim *sim, double tau);

/* Infiltration in the mass source (the paper's future extension of the source
 * term by an algebraic law, Sec. 4; the scalar equation for h^{n+1} of
 * Appendix A): the source r(t) loses i(h) = f_inf h / (h + h_inf), taken at
 * h^{n+1} (m/s; i rises from 0 on a dry cell to f_inf under deep water, half
 * of it at depth h_inf).  The update theta x + dt i(x) = (theta h)^n + dt/sigma
 * L + dt r is solved exactly for x = h^{n+1}: x = h_s - e with h_s the depth
 * without infiltration and e the smaller root of a quadratic; the water that
 * enters the soil is booked with the outflow.
 * f_inf = 0 (the default) turns it off; the kernel used then is the plain one.
 * Takes effect from the next run; surrogate windows refuse it.  EDOMAIN:
 * f_inf < 0 or non-finite, or f_inf > 0 with h_inf <= 0. */
int hexsv_sim_set_infiltration(hexsv_sim *sim, double f_inf, double h_inf);

/* Initial state (the paper's "initial water layer", Sec. 3) at time t0:
 * h, v1, v2 per cell (device FP64 arrays of nq*nr).  Resets the books and
 * the step count, and computes the first CFL bound.  EDOMAIN: h < 0 or a
 * non-finite value on an active cell.  ESTATE: set_fields not called. */
int hexsv_sim_set_state(hexsv_sim *sim, double t0, const double *d_h, const double *d_v1,
                        const double *d_v2, hipStream_t stream);

/* Advance to t_end, or until max_steps more steps were taken (max_steps <= 0:
 * no limit).  Each step: dt = min(dt_max, CFL*phi_min/c_max, t_end - t),
 * then eq. fvm_2D_eq_frac.07 on every active cell, then c_max and the FP64
 * books of the new state; the last step lands on t_end exactly.  Runs as
 * replays of captured graphs of steps_per_graph (and of 8) steps on `stream`,
 * batched by the steps expected to remain, reading the 256-byte control block
 * back after each batch.  EDOMAIN: t_end < t.
 * ENUMERIC: a non-finite value appeared (state left at the failing step). */
int hexsv_sim_run(hexsv_sim *sim, double t_end, int64_t max_steps, hipStream_t stream);

/* Current state as FP64 device arrays (each nullable): h, v1, v2 and the
 * discharges q_a = theta*h*v_a. */
int hexsv_sim_get_state(const hexsv_sim *sim, double *d_h, double *d_v1, double *d_v2,
                        double *d_q1, double *d_q2, hipStream_t stream);

/* Books of the current state (synchronises `stream`). */
int hexsv_sim_get_books(hexsv_sim *sim, hexsv_books *out, hipStream_t stream);
/* Restore books saved with get_books after set_state of the saved state
 * (checkpoint/resume).  The time t and step count are restored too. */
int hexsv_sim_set_books(hexsv_sim *sim, const hexsv_books *books, hipStream_t stream);

/* Device timing of run(): while enabled, run() brackets every graph replay
 * with hipEvents on its stream and accumulates the replays' GPU time and the
 * steps they took.  Reads the totals since the last reset; enable >= 0
 * switches timing on (1) or off (0) and resets the totals, enable < 0 only
 * reads.  Each step is one kernel launch, so gpu_ms/steps is the step
 * kernel's average duration including launch gaps inside the graph. */
int hexsv_sim_timing(hexsv_sim *sim, int32_t enable, double *gpu_ms, int64_t *steps,
                     int64_t *replays);

/* Average duration of the step kernel alone: nlaunch back-to-back launches of
 * the tile kernel (without the finalize kernel) between two hipEvents on
 * `stream`.  Every launch recomputes the next step from the current state,
 * so the state, time and books are unchanged afterwards. */
int hexsv_sim_time_kernel(hexsv_sim *sim, int32_t nlaunch, double *avg_ms, hipStream_t stream);

/* Autotuner: time every tile variant of the step kernel on this simulation's
 * raster and current state (nlaunch launches each, as hexsv_sim_time_kernel,
 * leaving state and books unchanged), switch the simulation to the fastest
 * and, if cache_path is non-null, record the result there (JSON keyed by
 * architecture, kernel, precision and size bucket).  hexsv_sim_create
 * consults the file named by $HEXSV_TUNE_CACHE when params->tile < 0. */
int hexsv_sim_autotune(hexsv_sim *sim, int32_t nlaunch, const char *cache_path,
                       int32_t *best_tile, double *best_ms, hipStream_t stream);

/* Launch/tile statistics of the step kernel: number of workgroups, tile
 * variant in use and its shape (tq x tr cells, threads). */
int hexsv_sim_info(const hexsv_sim *sim, int32_t *workgroups, int32_t *tile, int32_t *tq,
                   int32_t *tr, int32_t *threads);

/* ---------------------------------------------------- batched ensemble */

/* An ensemble of n independent catchments on rasters of any sizes, advanced
 * together (each scenario with its own CFL time step, rain and books; same
 * g, cfl, dt_max, h_dry and precision).  params->ensemble_mode picks the
 * persistent kernel (one workgroup sweeps one scenario at a time, scenarios
 * taken largest first, params->steps_per_graph steps per scenario per launch,
 * 0: 50) or batched steps (a graph of steps_per_graph steps, each a tile
 * kernel over the tiles of every live scenario plus a per-scenario close);
 * AUTO means batched unless the tuning cache says otherwise.  params->tile
 * selects the tile variant of the chosen mode (< 0: tuned or default).  The
 * grids must outlive the ensemble. */
int hexsv_ensemble_create(int32_t n, const hexsv_grid *const *grids, const hexsv_params *params,
                          hexsv_ensemble **out);
void hexsv_ensemble_destroy(hexsv_ensemble *ens);

/* Fields, rain and initial state of scenario s (device FP64 arrays sized for
 * its raster), with the same validation as the single-catchment calls;
 * resets the scenario's books.  Synchronises `stream`. */
int hexsv_ensemble_set_scenario(hexsv_ensemble *ens, int32_t s, const double *d_z,
                                const double *d_theta, const double *d_alpha_p, double alpha_s,
                                const hexsv_rain *rain, double t0, const double *d_h,
                                const double *d_v1, const double *d_v2, hipStream_t stream);

/* The momentum flux with artificial viscosity (eqs. eq_artif_visc, eq_visc1;
 * as hexsv_sim_set_viscosity) for every scenario: on = 1 or 0 (EINVAL
 * otherwise).  It is built for the batched-step mode only: turning it on
 * switches a persistent ensemble to batched steps, and the autotuner then
 * times batched variants only. */
int hexsv_ensemble_set_viscosity(hexsv_ensemble *ens, int32_t on);

/* Advance every scenario s to t_end[s] (host array of n), or by at most
 * max_steps steps (<= 0: no limit).  Replays a captured graph of one
 * persistent launch until every scenario is done.  EDOMAIN: t_end[s] before
 * the scenario's time.  ENUMERIC: a non-finite value appeared. */
int hexsv_ensemble_run(hexsv_ensemble *ens, const double *t_end, int64_t max_steps,
                       hipStream_t stream);

/* State (FP64 device arrays sized for scenario s, each nullable) and books. */
int hexsv_ensemble_get_state(const hexsv_ensemble *ens, int32_t s, double *d_h, double *d_v1,
                             double *d_v2, double *d_q1, double *d_q2, hipStream_t stream);
int hexsv_ensemble_get_books(hexsv_ensemble *ens, int32_t s, hexsv_books *out, hipStream_t stream);

/* Device timing of ensemble runs (as hexsv_sim_timing): GPU time of the
 * launches, cell-updates they performed (sum over scenarios of active cells
 * times steps taken) and number of launches. */
int hexsv_ensemble_timing(hexsv_ensemble *ens, int32_t enable, double *gpu_ms,
                          int64_t *cell_updates, int64_t *launches);
/* Autotuner of the ensemble: ksteps steps of every tile variant of both modes
 * from the current state (state and books are restored afterwards); switch
 * to the fastest mode and variant; record it in cache_path when non-null. */
int hexsv_ensemble_autotune(hexsv_ensemble *ens, int32_t ksteps, const char *cache_path,
                            int32_t *best_tile, double *best_ms, hipStream_t stream);
int hexsv_ensemble_info(const hexsv_ensemble *ens, int32_t *workgroups, int32_t *tile,
                        int64_t *cells, int32_t *steps_per_launch, int32_t *mode);

/* Standalone autotuner (no caller workload needed): builds the tuner's own
 * workload of about cells_hint cells in `precision` (a planar 5 % slope under a
 * flowing 5 cm sheet, every cell wet: the arithmetic of a wet catchment), times
 * every tile variant as hexsv_sim_autotune (kernel HEXSV_TUNE_STEP: one square
 * raster) or hexsv_ensemble_autotune (HEXSV_TUNE_ENSEMBLE: 8 equal square
 * scenarios of cells_hint / 8 cells each, both modes) do, and records the
 * fastest in the JSON cache at cache_path (keyed by architecture, kernel,
 * precision and size bucket), where hexsv_sim_create / hexsv_ensemble_create
 * find it through $HEXSV_TUNE_CACHE.  Everything it allocates is freed before it
 * returns; synchronises `stream`.  best_tile / best_ms (nullable) receive the
 * choice and its time per launch (or per ensemble step).
 * EINVAL: no cache path, unknown kernel or precision, cells_hint outside
 * [64, 2^30]. */
enum { HEXSV_TUNE_STEP = 0, HEXSV_TUNE_ENSEMBLE = 1 };
int hexsv_autotune(const char *cache_path, int32_t kernel, int32_t precision, int64_t cells_hint,
                   int32_t *best_tile, double *best_ms, hipStream_t stream);

/* ------------------------------------------------------ learned surrogate */

/* A hex-convolution residual network that predicts the change of the state
 * over a window of k solver steps (not part of the paper's method; the
 * solver stays its fallback and the reference for its error).  Layers: hex_conv(11 -> C), ReLU,
 * (layers - 2) x [hex_conv(C -> C), ReLU], hex_conv(C -> 3), where
 * hex_conv(x)[i][o] = b[o] + sum_{t<7, c} W[o][c][t] x[nbr_t(i)][c], tap 0
 * the cell, tap 1+k its neighbour in direction k as the raster's neighbour
 * table defines it (the INTERIOR edges of hexsv_grid_tables: periodic sides
 * wrap; a tap t >= 1 is zero across a WALL or OUTFLOW side and, on a masked
 * raster, unless both cells are in the domain).
 * Operands are bfloat16 with FP32 accumulation (MFMA); parameters are an FP32
 * master vector laid out per layer as W[o][c][t] then b[o].  Inputs are 11
 * FP32 features per cell (see hexsv_sim_surrogate_features), outputs 4 FP32 per cell (3 used), for a batch of
 * samples on one nq x nr raster (cell (b, r, q) at b*nq*nr + r*nq + q).
 * Only C = 32 is built (EUNSUPPORTED otherwise); 2 <= layers <= 16; k >= 1 is
 * the number of solver steps a window spans (the k of hexsv_sim_run_surrogate). */
int hexsv_surrogate_create(int32_t layers, int32_t channels, int32_t k, hexsv_surrogate **out);
void hexsv_surrogate_destroy(hexsv_surrogate *sur);
int64_t hexsv_surrogate_num_params(const hexsv_surrogate *sur);
/* k of create: the solver steps one window spans (EINVAL at create if k < 1).
 * The window calls below take it when their own k is <= 0.  -1 for a null handle. */
int32_t hexsv_surrogate_steps(const hexsv_surrogate *sur);
/* Forward of the 4-layer, 32-channel network as one fused kernel (on = 1:
 * activations stay on chip, 16 x 16 output cells per workgroup with a 4-cell
 * halo, 1.46x the MFMA work for the recomputed halo) or one launch per layer
 * (on = 0, the default, which measures faster on 512 x 512 rasters).  Both give
 * the same outputs bit for bit; other depths always run per layer.  EINVAL:
 * null handle or on not 0/1. */
int hexsv_surrogate_set_fused(hexsv_surrogate *sur, int32_t on);
/* Copy parameters in (device FP32, n == num_params; resets Adam) or out. */
int hexsv_surrogate_set_params(hexsv_surrogate *sur, const float *d_params, int64_t n,
                               hipStream_t stream);
int hexsv_surrogate_get_params(const hexsv_surrogate *sur, float *d_params, int64_t n,
                               hipStream_t stream);
/* Normalisation scales used when the surrogate advances a simulation:
 * {H, Q, Z, dH, dQ, S}: input depth, discharge, elevation, output depth and
 * discharge, input slope (1 <= n <= 8; unset scales are 1). */
int hexsv_surrogate_set_scales(hexsv_surrogate *sur, const float *scales, int32_t n);
int hexsv_surrogate_get_scales(const hexsv_surrogate *sur, float *scales, int32_t n);
/* Batched forward: d_features (batch*nq*nr x 11) -> d_out (batch*nq*nr x 4).
 * grid (nullable): the raster whose neighbour rule the taps follow (its nq x nr
 * must match; EUNSUPPORTED if it holds Dirichlet or flux cells); null means a
 * walled nq x nr parallelogram with every cell in the domain.  Every cell gets
 * an output, cells outside the domain included (their tap 0 reads their own
 * input). */
int hexsv_surrogate_forward(hexsv_surrogate *sur, const hexsv_grid *grid, int32_t batch,
                            int32_t nq, int32_t nr, const float *d_features, float *d_out,
                            hipStream_t stream);
/* hexsv_surrogate_forward for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and result (outputs 0..2 of each cell; the fourth float of d_out is
 * not written), with the packed input and the hidden activations in a static
 * device workspace of 40 MiB that every GPU the library runs on holds until the
 * process ends, instead of the surrogate's own workspace.  It calls no
 * hipMalloc, hipFree or allocating library routine.  The caller passes inputs
 * and outputs as for hexsv_surrogate_forward.  Every call on one GPU shares
 * that GPU's workspace: calls that overlap on one GPU (other streams or host
 * threads) race; calls on one stream are ordered.  EINVAL: batch*nq*nr above
 * 262144 cells (one 512 x 512 sample), or the arguments hexsv_surrogate_forward
 * refuses.  EUNSUPPORTED: a device index above 63.  EHIP: the workspace's device
 * address could not be looked up. */
int hexsv_surrogate_forward_noalloc(hexsv_surrogate *sur, const hexsv_grid *grid, int32_t batch,
                                    int32_t nq, int32_t nr, const float *d_features,
                                    float *d_out, hipStream_t stream);
/* Mean L1 loss over every cell and the 3 outputs against d_target
 * (batch*nq*nr x 3) and its parameter gradient (d_grad nullable, num_params
 * floats); grid as for forward; synchronises `stream`. */
int hexsv_surrogate_gradient(hexsv_surrogate *sur, const hexsv_grid *grid, int32_t batch,
                             int32_t nq, int32_t nr, const float *d_features,
                             const float *d_target, float *d_grad, double *loss,
                             hipStream_t stream);
/* gradient + one Adam step (beta1 0.9, beta2 0.999, eps 1e-8) at rate lr. */
int hexsv_surrogate_train_step(hexsv_surrogate *sur, const hexsv_grid *grid, int32_t batch,
                               int32_t nq, int32_t nr, const float *d_features,
                               const float *d_target, float lr, double *loss,
                               hipStream_t stream);

/* Network inputs of a window starting at the simulation's current state,
 * n x 11 FP32 into d_features (scales from set_scales):
 *   h/H, theta h v1/Q, theta h v2/Q, z/Z, theta, rain_depth/H, (dz/dx)/S,
 *   (dz/dy)/S, x_h/dH, x_q1/dQ, x_q2/dQ,
 * all but theta zero on inactive cells.  rain_depth is the window's rain (k
 * equal sub-steps, each at the rate of its end; k <= 0: the surrogate's k).  The slope of a cell is the
 * least-squares fit of the elevation differences along the three axes of its
 * hexagon (central differences of the two active neighbours on an axis,
 * one-sided with one), exact for a plane.  x is the change of one probe step
 * of the scheme (rain included; dt = min(dt_max, CFL bound of the state))
 * scaled by window/dt.  The state and books are not changed.  These are the
 * inputs run_surrogate feeds the network; training pairs use them too.
 * EUNSUPPORTED: the sim has Dirichlet or flux cells, the viscous flux,
 * infiltration or a soil field (the probe step runs the plain scheme). */
int hexsv_sim_surrogate_features(hexsv_sim *sim, hexsv_surrogate *sur, double window, int32_t k,
                                 float *d_features, hipStream_t stream);

/* Advance a simulation to t_end in windows of `window` seconds predicted by
 * the surrogate (trained on windows of that span).  A window runs entirely on
 * the device: the probe step and features of the state (see
 * hexsv_sim_surrogate_features), the network, the predicted state
 *   h' = max(h + x_h + dH out0, 0),  theta h' v' = theta h v + x_q + dQ (out1, out2)
 * (v' = 0 where theta h' <= 1e-6), and the FP64 water-balance residual
 *   rho = |S' - S - (R - O)| / max(S + R, 1e-300)
 * (S, S' stored volume sum sigma theta h at both ends, R = rain volume of the
 * window as k equal sub-steps each taking the rate at its end, O the outflow
 * volume by the trapezoid rule on the outflow rates of both states).  A
 * finite window with rho <= residual_tol whose largest wave speed
 * |v| + sqrt(g h) is at most twice that of its start state is kept (time,
 * rain and outflow books and the CFL bound advance; steps does not; an
 * infinite residual_tol keeps every finite window); with project != 0 its
 * depths are then scaled by (S + R - O) / S' so that the kept state closes
 * the balance exactly (small residuals would otherwise add up over many
 * windows).  A refused window is discarded and the plain solver advances
 * that span (ENUMERIC if it stalls); after n >= 2 refusals in a row it also
 * advances the next min(2^(n-1), 8) whole spans before a window is tried
 * again, each span to its own end (hexsv_sim_set_surrogate_backoff).  A last span shorter than `window` is
 * always solved.  k <= 0 takes the surrogate's k.  Windows are chained
 * several to a graph launch (after a refusal the next chain is as long as the
 * run of kept windows before it plus one; a chain kept whole is followed by
 * one at least twice as long); the host synchronises once per chain.  Counts
 * of kept windows and of spans the solver advanced are returned.  The
 * surrogate must not be used by another simulation while this runs (its
 * workspace is shared). */
int hexsv_sim_run_surrogate(hexsv_sim *sim, hexsv_surrogate *sur, double t_end, double window,
                            int32_t k, double residual_tol, int32_t project, int64_t *n_accepted,
                            int64_t *n_fallback, hipStream_t stream);

/* The back-off of hexsv_sim_run_surrogate: after n >= 2 refusals in a row the
 * solver also advances min(2^(n-1), max_spans) whole spans before the next
 * window (default 8; 0 turns the back-off off, so that every whole span is
 * tried).  EINVAL: null sim or max_spans < 0. */
int hexsv_sim_set_surrogate_backoff(hexsv_sim *sim, int32_t max_spans);

/* Window counts of every run_surrogate call on this simulation so far:
 * counts[0] kept, counts[1] refused for the water-balance residual, counts[2]
 * refused for the wave-speed growth, counts[3] refused as non-finite. */
int hexsv_sim_surrogate_stats(const hexsv_sim *sim, int64_t *counts);

/* Number of tile variants built, and the shape of variant v. */
int hexsv_tile_count(void);
int hexsv_tile_shape(int32_t v, int32_t *tq, int32_t *tr, int32_t *threads);

#ifdef __cplusplus
}
#endif
#endif
