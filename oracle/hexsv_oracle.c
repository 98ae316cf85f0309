/*
 * hexsv_oracle.c — TEST INFRASTRUCTURE ONLY (see hexsv_oracle.h).
 *
 * A plain FP64 CPU implementation of the time stepper of the porous
 * Saint-Venant model on a regular hexagonal raster, written to be checked by
 * eye against the paper.  Nothing here is blocked, fused or reordered beyond
 * what the equations state: each step computes c_max and the time step, then
 * for every cell the six edge terms, the mass update with rain, and the
 * closed-form friction solve.  Build with -O2 -fno-fast-math
 * -ffp-contract=off so that every operation is a correctly rounded IEEE
 * double operation in the order written.
 *
 * Readings of points the paper leaves open (all binding on the GPU path too):
 *  - "cell radius" = edge length a = circumradius; sigma = (3 sqrt3 / 2) a^2,
 *    every interface has l = a, phi_min = sigma / (6 a).
 *  - raster = axial parallelogram, pointy-top hexagons, centre
 *    (a sqrt3 (q + r/2), 1.5 a r); direction k points at k*60 degrees with
 *    (dq,dr) = (+1,0),(0,+1),(-1,+1),(-1,0),(0,-1),(+1,-1).
 *  - the upwind mass of eq. fvm_2D_eq.06 at v_n = 0 is 0 (it multiplies 0).
 *  - WALL edges carry no term (a mirror ghost gives exactly zero terms).
 *  - OUTFLOW edges use a ghost with the cell's h, v, theta and the terrain
 *    extrapolated linearly through the opposite neighbour.
 *  - rain is evaluated at t^{n+1} (as in eq. fvm_2D_eq_frac.07); a negative
 *    theta*h after the update is clamped to 0 and the added volume booked.
 *  - a cell whose denominator D of the miu-formula is 0 gets v = 0.
 */
#include "hexsv_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* sqrt(3)/2 rounded once to double */
static const double S3H = 0.86602540378443864676;

static const int DQ[6] = {+1, 0, -1, -1, 0, +1};
static const int DR[6] = {0, +1, +1, 0, -1, -1};

void ref_geometry(double a, double out[3]) {
    /* Area of a regular hexagon with edge a: six equilateral triangles. */
    double sigma = 6.0 * (0.5 * a * (S3H * a));
    out[0] = sigma;
    out[1] = a;
    /* eq. fvm_2D_eq_frac.13: sigma_i / sum_j l_(i,j) with six edges of length a */
    out[2] = sigma / (6.0 * a);
}

void ref_normal(int k, double n[2]) {
    /* cos/sin of k*60 degrees, written out exactly; n_{k+3} = -n_k */
    static const double NX[6] = {1.0, 0.5, -0.5, -1.0, -0.5, 0.5};
    static const double NY[6] = {0.0, S3H, S3H, 0.0, -S3H, -S3H};
    n[0] = NX[k];
    n[1] = NY[k];
}

/* ---------------------------------------------------------------- tables */

static int side_code_at(int32_t side, int32_t pos, const int32_t sidebc[4],
                        int32_t nseg, const int32_t *segs) {
    for (int s = 0; s < nseg; ++s) {
        if (segs[4 * s + 0] == side && pos >= segs[4 * s + 1] && pos < segs[4 * s + 2])
            return segs[4 * s + 3];
    }
    return sidebc[side];
}

int ref_tables(int32_t nq, int32_t nr, const int32_t side[4], int32_t nseg,
               const int32_t *segs, const uint8_t *active, int32_t mask_code,
               int32_t *nbr, uint8_t *code) {
    if (nq <= 0 || nr <= 0) return -1;
    int perq = side[REF_E] == REF_PERIODIC;
    int perr = side[REF_S] == REF_PERIODIC;
    if (perq != (side[REF_W] == REF_PERIODIC)) return -1;
    if (perr != (side[REF_N] == REF_PERIODIC)) return -1;
    for (int32_t r = 0; r < nr; ++r) {
        for (int32_t q = 0; q < nq; ++q) {
            int64_t i = (int64_t)r * nq + q;
            int is_active = active ? active[i] != 0 : 1;
            for (int k = 0; k < 6; ++k) {
                nbr[i * 6 + k] = -1;
                if (!is_active) { code[i * 6 + k] = REF_WALL; continue; }
                int32_t qn = q + DQ[k], rn = r + DR[k];
                /* periodic wraps first */
                if (perq) qn = (qn + nq) % nq;
                if (perr) rn = (rn + nr) % nr;
                if (rn < 0) {
                    code[i * 6 + k] = (uint8_t)side_code_at(REF_S, qn, side, nseg, segs);
                } else if (rn >= nr) {
                    code[i * 6 + k] = (uint8_t)side_code_at(REF_N, qn, side, nseg, segs);
                } else if (qn < 0) {
                    code[i * 6 + k] = (uint8_t)side_code_at(REF_W, rn, side, nseg, segs);
                } else if (qn >= nq) {
                    code[i * 6 + k] = (uint8_t)side_code_at(REF_E, rn, side, nseg, segs);
                } else {
                    int64_t j = (int64_t)rn * nq + qn;
                    if (active && !active[j]) {
                        code[i * 6 + k] = (uint8_t)mask_code;
                    } else if (active && active[j] == 2) {
                        code[i * 6 + k] = REF_DIRICHLET;
                        nbr[i * 6 + k] = (int32_t)j;
                    } else if (active && active[j] == 3) {
                        code[i * 6 + k] = REF_FLUX;
                        nbr[i * 6 + k] = (int32_t)j;
                    } else {
                        code[i * 6 + k] = REF_INTERIOR;
                        nbr[i * 6 + k] = (int32_t)j;
                    }
                }
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ rain */

double ref_rain_rate(int32_t kind, double i_a, double t_a, double T_d, double t) {
    if (kind == 0) {
        return (t >= 0.0 && t <= T_d) ? i_a : 0.0;
    }
    /* Appendix C: triangle of base T_d and height i_a, peak at t_a */
    double gamma = t_a / T_d;
    if (t >= 0.0 && t <= t_a) return i_a * (t / t_a);
    if (t > t_a && t <= T_d) return i_a * ((1.0 - t / T_d) / (1.0 - gamma));
    return 0.0;
}

/* -------------------------------------------------------------- friction */

double ref_mu(double alpha, double beta, double g1, double g2) {
    /* Appendix A, miu-formula: mu = 2 / (alpha + sqrt(alpha^2 + 4 beta |gamma|)) */
    double G = sqrt(g1 * g1 + g2 * g2);
    double D = alpha + sqrt(alpha * alpha + 4.0 * beta * G);
    if (D == 0.0) return 0.0;
    return 2.0 / D;
}

/* ------------------------------------------------------------ edge sums */

void ref_cell_sums(int32_t N, const int32_t *nbr, const uint8_t *code, double a,
                   double g, const double *z, const double *theta,
                   const double *h, const double *v1, const double *v2,
                   int32_t i, double out[6]) {
    (void)N;
    double l = a;
    double L = 0.0, J1 = 0.0, J2 = 0.0, S1 = 0.0, S2 = 0.0, Fout = 0.0;
    double mi = theta[i] * h[i];
    double wi = g * (z[i] + h[i]);
    for (int k = 0; k < 6; ++k) {
        int c = code[(int64_t)i * 6 + k];
        if (c == REF_WALL) continue; /* impermeable wall: no flux, no pressure term */
        double hj, v1j, v2j, zj, thj;
        if (c == REF_FLUX) {
            /* given mass flux: the neighbour prescribes the discharge h_j v_j across the
             * edge; the depth seen by the pressure term is the cell's own (zero gradient) */
            int32_t j = nbr[(int64_t)i * 6 + k];
            double n[2];
            ref_normal(k, n);
            double vn = v1[j] * n[0] + v2[j] * n[1];
            double F = l * h[j] * vn;
            L -= F;
            J1 -= F * v1[j];
            J2 -= F * v2[j];
            double wg = g * (z[j] + h[i]);
            double P = 0.5 * l * (wg - wi) * mi;
            S1 -= P * n[0];
            S2 -= P * n[1];
            Fout += F;
            continue;
        }
        if (c == REF_INTERIOR || c == REF_DIRICHLET) {
            int32_t j = nbr[(int64_t)i * 6 + k];
            hj = h[j];
            v1j = v1[j];
            v2j = v2[j];
            zj = z[j];
            /* a Dirichlet cell carries its porosity negated (it is not updated) */
            thj = c == REF_DIRICHLET ? -theta[j] : theta[j];
        } else { /* OUTFLOW: zero-gradient ghost, terrain extrapolated linearly */
            int ko = (k + 3) % 6;
            hj = h[i];
            v1j = v1[i];
            v2j = v2[i];
            thj = theta[i];
            if (code[(int64_t)i * 6 + ko] == REF_INTERIOR)
                zj = 2.0 * z[i] - z[nbr[(int64_t)i * 6 + ko]];
            else
                zj = z[i];
        }
        double n[2];
        ref_normal(k, n);
        double mj = thj * hj;
        double wj = g * (zj + hj);
        /* eq. fvm_2D_eq.04: interface velocity and its normal component; on an edge
         * to a Dirichlet cell the edge carries the prescribed velocity itself */
        double vb1 = c == REF_DIRICHLET ? v1j : (v1[i] + v1j) * 0.5;
        double vb2 = c == REF_DIRICHLET ? v2j : (v2[i] + v2j) * 0.5;
        double vn = vb1 * n[0] + vb2 * n[1];
        /* eq. fvm_2D_eq.06: upwind theta*h */
        double mup;
        if (vn > 0.0) mup = mi;
        else if (vn < 0.0) mup = mj;
        else mup = 0.0;
        /* eq. fvm_2D_eq.05: theta*h of the pressure term */
        double mhat;
        if (vn != 0.0) mhat = mup;
        else if (wi > wj) mhat = mi;
        else mhat = mj;
        /* eq. fvm_2D_eq_frac.01 */
        double F = l * mup * vn;
        L -= F;
        J1 -= F * vb1;
        J2 -= F * vb2;
        double P = 0.5 * l * (wj - wi) * mhat;
        S1 -= P * n[0];
        S2 -= P * n[1];
        if (c == REF_OUTFLOW || c == REF_DIRICHLET) Fout += F;
    }
    out[0] = L;
    out[1] = J1;
    out[2] = J2;
    out[3] = S1;
    out[4] = S2;
    out[5] = Fout;
}

void ref_visc_sums(int32_t N, const int32_t *nbr, const uint8_t *code, double a,
                   double g, const double *theta, const double *h, const double *v1,
                   const double *v2, int32_t i, double out[2]) {
    (void)N;
    double l = a;
    double V1 = 0.0, V2 = 0.0;
    double mi = theta[i] * h[i];
    double ci = sqrt(v1[i] * v1[i] + v2[i] * v2[i]) + sqrt(g * h[i]);
    for (int k = 0; k < 6; ++k) {
        if (code[(int64_t)i * 6 + k] != REF_INTERIOR) continue;
        int32_t j = nbr[(int64_t)i * 6 + k];
        double mj = theta[j] * h[j];
        double cj = sqrt(v1[j] * v1[j] + v2[j] * v2[j]) + sqrt(g * h[j]);
        double c = ci > cj ? ci : cj;
        double ms = mi + mj;
        double mu = ms > 0.0 ? 2.0 * mi * mj / ms : 0.0;
        V1 += l * c * mu * (v1[j] - v1[i]);
        V2 += l * c * mu * (v2[j] - v2[i]);
    }
    out[0] = V1;
    out[1] = V2;
}

/* Cells outside the domain carry theta == 0; theta of a cell of the domain
 * lies in (0,1] (eq. eq_theta, and theta*h must determine h). */
static int is_active_cell(const double *theta, int64_t i) { return theta[i] > 0.0; }

/* The wave speeds of eq. .12 run over the updated cells and the Dirichlet cells
 * (theta < 0): a prescribed state enters its neighbours' fluxes as well. */
static int enters_cfl(const double *theta, int64_t i) { return theta[i] != 0.0; }

double ref_cmax(int32_t N, const double *theta, double g, const double *h,
                const double *v1, const double *v2) {
    double cmax = 0.0;
    for (int32_t i = 0; i < N; ++i) {
        if (!enters_cfl(theta, i)) continue;
        double c = sqrt(v1[i] * v1[i] + v2[i] * v2[i]) + sqrt(g * h[i]);
        if (c > cmax) cmax = c;
    }
    return cmax;
}

double ref_dt(double a, const ref_params *p, double cmax, double t, double t_end) {
    double geo[3];
    ref_geometry(a, geo);
    double tau = (cmax > 0.0) ? p->cfl * geo[2] / cmax : INFINITY;
    double dt = p->dt_max;
    if (tau < dt) dt = tau;
    if (t_end - t < dt) dt = t_end - t;
    return dt;
}

/* One cell of eq. fvm_2D_eq_frac.07 (Appendix A: mass, then velocity). */
static void step_one(const int32_t *nbr, const uint8_t *code, double a,
                     const double *z, const double *theta, const double *alpha_p,
                     const ref_params *p, double r_next, double dt,
                     const double *h, const double *v1, const double *v2, int32_t i,
                     double *hn, double *v1n, double *v2n, double add[3]) {
    double geo[3];
    ref_geometry(a, geo);
    double sigma = geo[0];
    double s[6];
    ref_cell_sums(0, nbr, code, a, p->g, z, theta, h, v1, v2, i, s);
    double th = theta[i];
    double mi = th * h[i];
    double dts = dt / sigma;
    /* eq. fvm_2D_eq_frac.05-1 then .06-1 with rain at t^{n+1} */
    double ms = mi + dts * s[0];
    double m1 = ms + dt * r_next;
    double clamp = 0.0;
    if (m1 < 0.0) {
        clamp = sigma * (-m1);
        m1 = 0.0;
    }
    double h1 = m1 / th;
    double infil = 0.0;
    if (p->f_inf > 0.0 && m1 > 0.0) {
        /* the mass source r - i(h^{n+1}) with i(h) = f h / (h + c) makes .05-1/.06-1 the
         * scalar equation theta x + dt f x / (x + c) = m1 for x = h^{n+1}.  With
         * x = hs - e (hs = m1 / theta, the depth without infiltration) the loss e is the
         * smaller root of theta e^2 - P e + dt f hs = 0, P = theta (hs + c) + dt f, whose
         * discriminant is (theta (hs + c) - dt f)^2 + 4 theta dt f c */
        double c = p->h_inf, fd = dt * p->f_inf, hs = h1;
        double P = th * (hs + c) + fd;
        double Q = th * (hs + c) - fd;
        double D = Q * Q + 4.0 * th * fd * c;
        double e = (2.0 * fd * hs) / (P + sqrt(D));
        double x = hs - e;
        double mx = th * x;
        infil = sigma * (m1 - mx); /* the water that went into the soil this step */
        m1 = mx;
        h1 = x;
    }
    /* eq. fvm_2D_eq_frac.05-2: (theta h v)^*, with J^v = J + viscous sums when on */
    double g1, g2;
    if (p->visc) {
        double vs[2];
        ref_visc_sums(0, nbr, code, a, p->g, theta, h, v1, v2, i, vs);
        g1 = mi * v1[i] + dts * ((s[1] + vs[0]) + s[3]);
        g2 = mi * v2[i] + dts * ((s[2] + vs[1]) + s[4]);
    } else {
        g1 = mi * v1[i] + dts * (s[1] + s[3]);
        g2 = mi * v2[i] + dts * (s[2] + s[4]);
    }
    /* eq. fvm_2D_eq_frac.06-2 solved by the miu-formula, with eq_K_h_theta */
    /* eq_tsa_darcy: alpha_s of the soil under cell i (one value, or a field) */
    double as = p->alpha_s_cell ? p->alpha_s_cell[i] : p->alpha_s;
    double K = alpha_p[i] * h1 * (1.0 - th) + th * as;
    double beta = dt * K;
    /* the linear soil term theta*tau*h*v (Thacker test), implicit in v^{n+1}:
     * it adds dt*tau*theta*h^{n+1} = dt*tau*m^{n+1} to the coefficient of v */
    double alpha = m1 * (1.0 + dt * p->tau_lin);
    double mu = ref_mu(alpha, beta, g1, g2);
    if (p->h_dry > 0.0 && h1 < p->h_dry) mu = 0.0;
    *hn = h1;
    *v1n = mu * g1;
    *v2n = mu * g2;
    if (add) {
        add[0] = dt * s[5] + infil; /* water leaving the surface: open edges, soil */
        add[1] = clamp;
        add[2] = sigma * dt * r_next;
    }
}

void ref_step_cells(int32_t N, const int32_t *nbr, const uint8_t *code, double a,
                    const double *z, const double *theta, const double *alpha_p,
                    const ref_params *p, const ref_rain *rain, double dt,
                    double t_next, const double *h, const double *v1,
                    const double *v2, int32_t ncells, const int32_t *cells,
                    double *hn, double *v1n, double *v2n, double add[3]) {
    (void)N;
    double r_next = ref_rain_rate(rain->kind, rain->i_a, rain->t_a, rain->T_d, t_next);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int32_t c = 0; c < ncells; ++c) {
        int32_t i = cells[c];
        double one[3];
        step_one(nbr, code, a, z, theta, alpha_p, p, r_next, dt, h, v1, v2, i,
                 &hn[c], &v1n[c], &v2n[c], one);
        acc[0] += one[0];
        acc[1] += one[1];
        acc[2] += one[2];
    }
    if (add) {
        add[0] = acc[0];
        add[1] = acc[1];
        add[2] = acc[2];
    }
}

void ref_books_init(int32_t N, double a, const double *theta, const double *h,
                    double t0, ref_books *b) {
    double geo[3];
    ref_geometry(a, geo);
    double S = 0.0;
    for (int32_t i = 0; i < N; ++i)
        if (is_active_cell(theta, i)) S += geo[0] * (theta[i] * h[i]);
    memset(b, 0, sizeof(*b));
    b->t = t0;
    b->initial = S;
    b->stored = S;
    b->dt_min = INFINITY;
    b->dt_max_seen = 0.0;
}

int64_t ref_run(int32_t N, const int32_t *nbr, const uint8_t *code, double a,
                const double *z, const double *theta, const double *alpha_p,
                const ref_params *p, const ref_rain *rain, double t_end,
                int64_t max_steps, double *h, double *v1, double *v2,
                ref_books *b, double *dt_log, int32_t nthreads) {
    if (N <= 0 || !(p->cfl > 0.0 && p->cfl < 1.0) || !(p->dt_max > 0.0)) return -1;
    if (t_end < b->t) return -1;
    double geo[3];
    ref_geometry(a, geo);
    double sigma = geo[0];
    double *hn = malloc(sizeof(double) * (size_t)N);
    double *v1n = malloc(sizeof(double) * (size_t)N);
    double *v2n = malloc(sizeof(double) * (size_t)N);
    double *outf = malloc(sizeof(double) * (size_t)N);
    double *clmp = malloc(sizeof(double) * (size_t)N);
    if (!hn || !v1n || !v2n || !outf || !clmp) {
        free(hn); free(v1n); free(v2n); free(outf); free(clmp);
        return -1;
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int64_t taken = 0;
    int64_t status = 0;
    while (taken < max_steps) {
        /* eqs. fvm_2D_eq_frac.12-13 over the updated and the Dirichlet cells */
        double cmax = 0.0;
        for (int32_t i = 0; i < N; ++i) {
            if (!enters_cfl(theta, i)) continue;
            double c = sqrt(v1[i] * v1[i] + v2[i] * v2[i]) + sqrt(p->g * h[i]);
            if (c > cmax) cmax = c;
        }
        double dt = ref_dt(a, p, cmax, b->t, t_end);
        if (!(dt > 0.0)) break;
        double t_next = (dt == t_end - b->t) ? t_end : b->t + dt;
        double r_next = ref_rain_rate(rain->kind, rain->i_a, rain->t_a, rain->T_d, t_next);
        /* every cell reads state n only, so cells are independent */
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < N; ++i) {
            if (!is_active_cell(theta, i)) {
                hn[i] = h[i];
                v1n[i] = v1[i];
                v2n[i] = v2[i];
                outf[i] = 0.0;
                clmp[i] = 0.0;
                continue;
            }
            double add[3];
            step_one(nbr, code, a, z, theta, alpha_p, p, r_next, dt, h, v1, v2, i,
                     &hn[i], &v1n[i], &v2n[i], add);
            outf[i] = add[0];
            clmp[i] = add[1];
        }
        /* books, summed serially in index order */
        double S = 0.0, O = 0.0, C = 0.0, R = 0.0;
        int nonfinite = 0;
        for (int32_t i = 0; i < N; ++i) {
            if (!is_active_cell(theta, i)) continue;
            S += sigma * (theta[i] * hn[i]);
            O += outf[i];
            C += clmp[i];
            R += sigma * dt * r_next;
            if (!isfinite(hn[i]) || !isfinite(v1n[i]) || !isfinite(v2n[i])) nonfinite = 1;
        }
        memcpy(h, hn, sizeof(double) * (size_t)N);
        memcpy(v1, v1n, sizeof(double) * (size_t)N);
        memcpy(v2, v2n, sizeof(double) * (size_t)N);
        b->stored = S;
        b->outflow += O;
        b->clamp += C;
        b->rain += R;
        b->t = t_next;
        b->steps += 1;
        if (dt < b->dt_min) b->dt_min = dt;
        if (dt > b->dt_max_seen) b->dt_max_seen = dt;
        /* water supplied: initial, rain and any net inflow (Dirichlet edges) */
        double ref = b->initial + b->rain + (b->outflow < 0.0 ? -b->outflow : 0.0);
        if (ref < 1e-300) ref = 1e-300;
        b->residual = fabs(S - (b->initial + b->rain - b->outflow + b->clamp)) / ref;
        if (dt_log) dt_log[taken] = dt;
        ++taken;
        if (nonfinite) { status = -2; break; }
    }
    free(hn); free(v1n); free(v2n); free(outf); free(clmp);
    return status ? status : taken;
}

/* -------------------------------------------------------------- hex conv */

void ref_hexconv_fwd(int32_t N, const int32_t *nbr, int32_t cin, int32_t cout,
                     const double *x, const double *W, const double *b, double *y) {
    for (int32_t o = 0; o < cout; ++o) {
        for (int32_t i = 0; i < N; ++i) {
            double acc = b ? b[o] : 0.0;
            for (int32_t c = 0; c < cin; ++c) {
                for (int t = 0; t < 7; ++t) {
                    int32_t j = (t == 0) ? i : nbr[(int64_t)i * 6 + (t - 1)];
                    if (j < 0) continue;
                    acc += W[((int64_t)o * cin + c) * 7 + t] * x[(int64_t)c * N + j];
                }
            }
            y[(int64_t)o * N + i] = acc;
        }
    }
}

void ref_hexconv_bwd(int32_t N, const int32_t *nbr, int32_t cin, int32_t cout,
                     const double *x, const double *W, const double *dy,
                     double *dx, double *dW, double *db) {
    for (int32_t o = 0; o < cout; ++o) {
        for (int32_t i = 0; i < N; ++i) {
            double g = dy[(int64_t)o * N + i];
            if (db) db[o] += g;
            for (int32_t c = 0; c < cin; ++c) {
                for (int t = 0; t < 7; ++t) {
                    int32_t j = (t == 0) ? i : nbr[(int64_t)i * 6 + (t - 1)];
                    if (j < 0) continue;
                    dW[((int64_t)o * cin + c) * 7 + t] += g * x[(int64_t)c * N + j];
                    if (dx) dx[(int64_t)c * N + j] += W[((int64_t)o * cin + c) * 7 + t] * g;
                }
            }
        }
    }
}
