/*
 * hexsv_oracle.h — TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 CPU oracle for the porous Saint-Venant finite-volume
 * scheme on a regular hexagonal raster (Ion, Marinescu, Cruceanu, "ASTERIX:
 * Module for modelling the water flow on vegetated hillslopes", arXiv
 * 2406.14933): model of Sec. 2.1 (eq. swe_vegm_rm.02 with eq_tsa_darcy,
 * eq_tpa, eq_K_h_theta), scheme of Sec. 2.2 (eqs. fvm_2D_eq.04-.06,
 * fvm_2D_eq_frac.01, fvm_2D_eq_frac.07) solved as in Appendix A
 * (eqs. fvm_2D_eq_frac.05/.06, .12, .13, miu-formula), rain of Appendix C.
 *
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no source with the GPU path.
 * Every array is a plain host array; every index is i = r*nq + q.  Cells
 * outside the domain are marked by theta == 0 in the field arrays (and by
 * the active mask given to ref_tables).
 */
#ifndef HEXSV_ORACLE_H
#define HEXSV_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* edge codes */
#define REF_INTERIOR 0
#define REF_WALL 1
#define REF_OUTFLOW 2
#define REF_PERIODIC 3 /* side kind only; a wrapped edge is INTERIOR */
#define REF_DIRICHLET 4 /* edge to a boundary cell whose state is held fixed (Sec. 2.2,
                           boundary conditions: Dirichlet); its flux is booked as outflow */
#define REF_FLUX 5      /* edge to a boundary cell prescribing the mass flux h v (given
                           mass flux); its flux is booked as outflow */

/* sides */
#define REF_S 0 /* r < 0   */
#define REF_E 1 /* q >= nq */
#define REF_N 2 /* r >= nr */
#define REF_W 3 /* q < 0   */

/* Geometry of the regular hexagon of edge length a (= circumradius):
 * out[0] = area sigma, out[1] = edge length l, out[2] = phi_min of
 * eq. fvm_2D_eq_frac.13 for a cell with six flux-carrying edges. */
void ref_geometry(double a, double out[3]);

/* Unit normal of direction k (k*60 degrees counter-clockwise from +x). */
void ref_normal(int k, double n[2]);

/* Neighbour and edge-code tables of an nq x nr axial parallelogram.
 * side[4]: WALL/OUTFLOW/PERIODIC per side (S,E,N,W); opposite sides must
 * agree on PERIODIC.  segs: nseg rows of (side, lo, hi, code) overriding the
 * side's code for boundary edges whose outside position along the side lies
 * in [lo,hi).  active: nullable, 1 = cell belongs to the domain.  mask_code:
 * code of an edge from an active cell to an inactive one.
 * nbr[i*6+k] = neighbour index for INTERIOR edges, -1 otherwise;
 * code[i*6+k] = edge code (inactive cells: all WALL).
 * Returns 0, or -1 on invalid arguments. */
int ref_tables(int32_t nq, int32_t nr, const int32_t side[4], int32_t nseg,
               const int32_t *segs, const uint8_t *active, int32_t mask_code,
               int32_t *nbr, uint8_t *code);

/* Instantaneous rain intensity r(t) in m/s.  kind 0: i_a on [0, T_d], else 0.
 * kind 1: triangular hyetograph of Appendix C (peak i_a at t_a, ends at T_d). */
double ref_rain_rate(int32_t kind, double i_a, double t_a, double T_d, double t);

/* Closed-form implicit friction solve (Appendix A, miu-formula):
 * alpha*v + beta*|v|*v = gamma.  Returns mu with v = mu*gamma (0 if D = 0).
 * alpha is the new mass m = theta*h^{n+1}, times (1 + dt*tau) when a linear
 * soil resistance theta*tau*h*v is on (it is implicit in v like the quadratic
 * terms). */
double ref_mu(double alpha, double beta, double g1, double g2);

typedef struct {
    double g;      /* gravitational acceleration */
    double cfl;    /* Courant number, in (0,1) */
    double dt_max; /* maximum time step */
    double h_dry;  /* depth below which v is set to 0 (0 disables) */
    double alpha_s;/* Darcy-Weisbach soil coefficient (uniform) */
    double tau_lin;/* linear soil resistance -tau*h*v of the Thacker test (Sec. 3.2.2,
                      Appendix B), in 1/s; 0 for the paper's Darcy-Weisbach runs */
    int32_t visc;  /* 1: augmented momentum flux J^v with artificial viscosity
                      (eqs. eq_artif_visc, eq_visc1), for shocks */
    double f_inf;  /* infiltration: the mass source loses i(h) = f_inf h / (h + h_inf)
                      (m/s), taken at h^{n+1}; 0 disables (Sec. 4, future extensions) */
    double h_inf;  /* depth at which i(h) reaches half of f_inf (m), > 0 when f_inf > 0 */
    const double *alpha_s_cell; /* nullable: Darcy-Weisbach coefficient per cell (N values),
                                   replacing alpha_s (eq_tsa_darcy with a soil that varies) */
} ref_params;

typedef struct {
    int32_t kind;
    double i_a, t_a, T_d;
} ref_rain;

typedef struct {
    double t;        /* current time */
    double initial;  /* sum sigma*theta*h at the start */
    double stored;   /* sum sigma*theta*h now */
    double rain;     /* rain volume added */
    double outflow;  /* volume that left the surface: OUTFLOW edges, the soil, and
                        Dirichlet / flux edges (inflow counts negative) */
    double clamp;    /* volume added by clamping negative theta*h to 0 */
    double residual; /* |stored - (initial + rain - outflow + clamp)| /
                        (initial + rain + max(-outflow, 0)) */
    int64_t steps;
    double dt_min, dt_max_seen;
} ref_books;

/* The per-cell sums of eq. fvm_2D_eq_frac.01 for cell i at state (h,v1,v2):
 * out = {L, J1, J2, S1, S2, F_out} with F_out the volume flux leaving through
 * OUTFLOW edges of the cell. */
void ref_cell_sums(int32_t N, const int32_t *nbr, const uint8_t *code, double a,
                   double g, const double *z, const double *theta,
                   const double *h, const double *v1, const double *v2,
                   int32_t i, double out[6]);

/* The artificial-viscosity part of the augmented flux J^v (eq. eq_artif_visc):
 * out = sum over the INTERIOR edges of cell i, in direction order, of
 * l * c_ij * mu_ij * ((v_a)_j - (v_a)_i) (eq. eq_visc1), with c_ij the larger
 * of c = |v| + sqrt(g h) of the two cells and mu_ij = 2 m_i m_j / (m_i + m_j),
 * m = theta*h (0 when both are dry).  OUTFLOW ghosts carry the cell's own
 * velocity and WALL edges carry nothing, so neither contributes. */
void ref_visc_sums(int32_t N, const int32_t *nbr, const uint8_t *code, double a,
                   double g, const double *theta, const double *h, const double *v1,
                   const double *v2, int32_t i, double out[2]);

/* Largest c_i = |v_i| + sqrt(g h_i) over active cells (eq. fvm_2D_eq_frac.13). */
double ref_cmax(int32_t N, const double *theta, double g, const double *h,
                const double *v1, const double *v2);

/* Time step for the step starting at t (eqs. fvm_2D_eq_frac.12-13):
 * min(dt_max, CFL*phi_min/c_max, t_end - t); c_max = 0 gives dt_max. */
double ref_dt(double a, const ref_params *p, double cmax, double t, double t_end);

/* One step n -> n+1 of eq. fvm_2D_eq_frac.07 for the listed cells only,
 * given dt and t^{n+1}.  Writes hn/v1n/v2n[c] for cells[c].  add[3] (nullable)
 * receives the cells' {outflow volume, clamp volume, rain volume}. */
void ref_step_cells(int32_t N, const int32_t *nbr, const uint8_t *code, double a,
                    const double *z, const double *theta, const double *alpha_p,
                    const ref_params *p, const ref_rain *rain, double dt,
                    double t_next, const double *h, const double *v1,
                    const double *v2, int32_t ncells, const int32_t *cells,
                    double *hn, double *v1n, double *v2n, double add[3]);

/* Start the books from state h. */
void ref_books_init(int32_t N, double a, const double *theta, const double *h,
                    double t0, ref_books *b);

/* Advance (h,v1,v2) in place from b->t to t_end or until max_steps steps
 * have been taken in this call.  dt_log (nullable, max_steps long) receives
 * each step's dt.  Returns the number of steps taken, or -1 on bad input,
 * -2 if a non-finite value appears. */
int64_t ref_run(int32_t N, const int32_t *nbr, const uint8_t *code, double a,
                const double *z, const double *theta, const double *alpha_p,
                const ref_params *p, const ref_rain *rain, double t_end,
                int64_t max_steps, double *h, double *v1, double *v2,
                ref_books *b, double *dt_log, int32_t nthreads);

/* Hex convolution (test oracle of the learned surrogate).  Tap 0 is the cell
 * itself, tap 1+k its neighbour in direction k; taps without an INTERIOR
 * neighbour read zero.  x[c*N+i], W[(o*cin+c)*7+t], y[o*N+i]. */
void ref_hexconv_fwd(int32_t N, const int32_t *nbr, int32_t cin, int32_t cout,
                     const double *x, const double *W, const double *b, double *y);
/* Gradients of the above: dx (nullable) += ..., dW += ..., db += ... */
void ref_hexconv_bwd(int32_t N, const int32_t *nbr, int32_t cin, int32_t cout,
                     const double *x, const double *W, const double *dy,
                     double *dx, double *dW, double *db);

#ifdef __cplusplus
}
#endif
#endif
