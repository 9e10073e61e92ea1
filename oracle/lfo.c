/*
 * lfo.c -- plain FP64 CPU oracle of the second-order Lagrange-flux scheme
 * (arXiv:1607.08710).  TEST INFRASTRUCTURE ONLY: loaded by the tests, the
 * smoke check and the CPU-baseline leg of the benchmark, never by the
 * product path.  It shares no code with the GPU library.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math -shared -fPIC.
 *
 * Each function cites the passage of the paper it restates.  Section
 * numbers follow the paper: Sec. 3 (Lagrange step, Euler system and EOS),
 * Sec. 5 (derivation of the second-order Lagrange-flux scheme: eq. (11),
 * eq. (12), eq. (sweby), the Heun predictor-corrector list), Sec. 5.1
 * (Lagrangian HLL solver, eqs. (13)-(14)).
 */
#include "lfo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Pointwise physics                                                        */
/* ------------------------------------------------------------------------ */

/* Sec. 3: U = (rho, rho u, rho v, rho E) with E the specific total energy;
 * perfect gas p = (gamma - 1) rho (E - |u|^2 / 2). */
void lfo_cons_to_prim(double gamma, const double U[4], double w[4])
{
    double rho = U[0];
    double u = U[1] / rho;
    double v = U[2] / rho;
    double E = U[3] / rho;
    w[0] = rho;
    w[1] = u;
    w[2] = v;
    w[3] = (gamma - 1.0) * rho * (E - 0.5 * (u * u + v * v));
}

static double sgn(double a) { return a > 0.0 ? 1.0 : (a < 0.0 ? -1.0 : 0.0); }

/* eq. (sweby): phi(a,b) = (ab > 0) sign(a) max(min(|a|, beta|b|), min(beta|a|, |b|)). */
double lfo_sweby(double a, double b, double beta)
{
    if (!(a * b > 0.0))
        return 0.0;
    return sgn(a) * fmax(fmin(fabs(a), beta * fabs(b)), fmin(beta * fabs(a), fabs(b)));
}

/* Partial derivatives of eq. (sweby) with fixed conventions at its kinks:
 * zero when ab <= 0; min(x, y) follows x when x <= y; max(m1, m2) follows
 * m1 when m1 >= m2.  Since a and b share their sign when ab > 0,
 * d phi/da = dM/d|a| and d phi/db = dM/d|b| with M the max-min term. */
static void sweby_partials(double a, double b, double beta, double *da, double *db)
{
    *da = 0.0;
    *db = 0.0;
    if (!(a * b > 0.0))
        return;
    double aa = fabs(a), ab = fabs(b);
    double m1 = fmin(aa, beta * ab);
    double m2 = fmin(beta * aa, ab);
    double m1a, m1b, m2a, m2b;
    if (aa <= beta * ab) { m1a = 1.0; m1b = 0.0; } else { m1a = 0.0; m1b = beta; }
    if (beta * aa <= ab) { m2a = beta; m2b = 0.0; } else { m2a = 0.0; m2b = 1.0; }
    if (m1 >= m2) { *da = m1a; *db = m1b; } else { *da = m2a; *db = m2b; }
}

/* Sec. 5.1, eqs. (13)-(14): contact pressure and normal contact velocity
 * of the Lagrangian HLL solver with the single sound speed max(c_L, c_R);
 * c = sqrt(gamma p / rho) (Sec. 3). */
void lfo_acoustic_solve(double gamma,
                        double rho_l, double u_l, double p_l,
                        double rho_r, double u_r, double p_r,
                        double *u_star, double *p_star)
{
    double c_l = sqrt(gamma * p_l / rho_l);
    double c_r = sqrt(gamma * p_r / rho_r);
    double a = fmax(c_l, c_r);
    double S = rho_l + rho_r;
    *p_star = (rho_r * p_l + rho_l * p_r) / S - (rho_l * rho_r / S) * a * (u_r - u_l);
    *u_star = (rho_l * u_l + rho_r * u_r) / S - (1.0 / S) * (p_r - p_l) / a;
}

/* eq. (12) in the face frame: Phi_l = (U_l)_A (u_A . nu) + (pi_l)_A . nu
 * with (u_A . nu) = u*, pi_1 = 0, pi_2 . nu = p*, pi_3 . nu = 0 (tangential),
 * pi_4 . nu = p* u*.  (U_l)_A is taken from the upwind side of u*
 * (Sec. 5: "upwind process according to the sign of the normal velocity"):
 * the left state when u* > 0, the right state otherwise.  The upwind
 * conservative vector is that of the reconstructed primitive state. */
void lfo_face_flux(double gamma, const double wl[4], const double wr[4], double phi[4])
{
    double us, ps;
    lfo_acoustic_solve(gamma, wl[0], wl[1], wl[3], wr[0], wr[1], wr[3], &us, &ps);
    const double *wa = (us > 0.0) ? wl : wr;
    double rho = wa[0], un = wa[1], ut = wa[2], p = wa[3];
    double E = p / (gamma - 1.0) + 0.5 * rho * (un * un + ut * ut); /* rho E */
    phi[0] = rho * us;
    phi[1] = rho * un * us + ps;
    phi[2] = rho * ut * us;
    phi[3] = (E + ps) * us;
}

/* Jacobian of the face flux w.r.t. (wl, wr) = (rho_l, un_l, ut_l, p_l,
 * rho_r, un_r, ut_r, p_r), differentiating eqs. (12)-(14) by hand.  At the
 * kinks: max(c_l, c_r) follows c_l when c_l >= c_r; the upwind switch
 * follows the same rule as the value (left when u* > 0). */
static void face_flux_jacobian(double g, const double wl[4], const double wr[4],
                               double phi[4], double J[4][8])
{
    lfo_face_flux(g, wl, wr, phi);

    double rl = wl[0], ul = wl[1], pl = wl[3];
    double rr = wr[0], ur = wr[1], pr = wr[3];
    double cl = sqrt(g * pl / rl), cr = sqrt(g * pr / rr);
    int a_left = (cl >= cr);
    double a = a_left ? cl : cr;
    double S = rl + rr, S2 = S * S;
    double Z = rl * rr / S;
    double du = ur - ul, dp = pr - pl;
    double us, ps;
    lfo_acoustic_solve(g, rl, ul, pl, rr, ur, pr, &us, &ps);

    /* da/d(rho_l, p_l, rho_r, p_r): c = sqrt(g p / rho) -> dc/dp = c/(2p),
     * dc/drho = -c/(2 rho). */
    double da_rl = a_left ? -a / (2.0 * rl) : 0.0;
    double da_pl = a_left ? a / (2.0 * pl) : 0.0;
    double da_rr = a_left ? 0.0 : -a / (2.0 * rr);
    double da_pr = a_left ? 0.0 : a / (2.0 * pr);

    double dps_da = -Z * du;
    double dus_da = dp / (S * a * a);

    /* d p*, d u* w.r.t. the 8 inputs (ut does not enter eqs. (13)-(14)). */
    double dps[8], dus[8];
    dps[0] = rr * dp / S2 - (rr * rr / S2) * a * du + dps_da * da_rl;
    dps[1] = Z * a;
    dps[2] = 0.0;
    dps[3] = rr / S + dps_da * da_pl;
    dps[4] = -rl * dp / S2 - (rl * rl / S2) * a * du + dps_da * da_rr;
    dps[5] = -Z * a;
    dps[6] = 0.0;
    dps[7] = rl / S + dps_da * da_pr;

    dus[0] = -rr * du / S2 + dp / (S2 * a) + dus_da * da_rl;
    dus[1] = rl / S;
    dus[2] = 0.0;
    dus[3] = 1.0 / (S * a) + dus_da * da_pl;
    dus[4] = rl * du / S2 + dp / (S2 * a) + dus_da * da_rr;
    dus[5] = rr / S;
    dus[6] = 0.0;
    dus[7] = -1.0 / (S * a) + dus_da * da_pr;

    int off = (us > 0.0) ? 0 : 4;
    const double *wa = (us > 0.0) ? wl : wr;
    double rho = wa[0], un = wa[1], ut = wa[2], p = wa[3];
    double E = p / (g - 1.0) + 0.5 * rho * (un * un + ut * ut);

    double dphi_dus[4] = {rho, rho * un, rho * ut, E + ps};
    double dphi_dps[4] = {0.0, 1.0, 0.0, us};
    double dphi_dside[4][4] = {
        /* d/d rho_A */ {us, un * us, ut * us, 0.5 * (un * un + ut * ut) * us},
        /* d/d un_A  */ {0.0, rho * us, 0.0, rho * un * us},
        /* d/d ut_A  */ {0.0, 0.0, rho * us, rho * ut * us},
        /* d/d p_A   */ {0.0, 0.0, 0.0, us / (g - 1.0)},
    };
    for (int c = 0; c < 4; ++c) {
        for (int k = 0; k < 8; ++k)
            J[c][k] = dphi_dus[c] * dus[k] + dphi_dps[c] * dps[k];
        for (int k = 0; k < 4; ++k)
            J[c][off + k] += dphi_dside[k][c];
    }
}

/* ------------------------------------------------------------------------ */
/* One face from its four-cell stencil                                      */
/* ------------------------------------------------------------------------ */

/* W[k] = primitive state of cells m-1, m, m+1, m+2 along the face normal,
 * in the face frame (rho, u_n, u_t, p).  MUSCL reconstruction (Sec. 5):
 * slope sigma_m = phi(w_m - w_{m-1}, w_{m+1} - w_m) per variable,
 * w^L = w_m + sigma_m / 2, w^R = w_{m+1} - sigma_{m+1} / 2, then eq. (12).
 * If Jl is not NULL it receives d phi / d W (4 x 16, column 4k+v for cell
 * k, variable v). */
static void stencil_face(double gamma, double beta, const double W[4][4],
                         double phi[4], double Jl[4][16])
{
    double wl[4], wr[4];
    double dl[4][3], dr[4][3]; /* d w^L/d W[0..2], d w^R/d W[1..3] per var */
    for (int v = 0; v < 4; ++v) {
        double a1 = W[1][v] - W[0][v], b1 = W[2][v] - W[1][v];
        double a2 = W[2][v] - W[1][v], b2 = W[3][v] - W[2][v];
        double s1 = lfo_sweby(a1, b1, beta);
        double s2 = lfo_sweby(a2, b2, beta);
        wl[v] = W[1][v] + 0.5 * s1;
        wr[v] = W[2][v] - 0.5 * s2;
        if (Jl) {
            double pa, pb;
            sweby_partials(a1, b1, beta, &pa, &pb);
            dl[v][0] = -0.5 * pa;
            dl[v][1] = 1.0 + 0.5 * (pa - pb);
            dl[v][2] = 0.5 * pb;
            sweby_partials(a2, b2, beta, &pa, &pb);
            dr[v][0] = 0.5 * pa;
            dr[v][1] = 1.0 - 0.5 * (pa - pb);
            dr[v][2] = -0.5 * pb;
        }
    }
    if (!Jl) {
        lfo_face_flux(gamma, wl, wr, phi);
        return;
    }
    double Jf[4][8];
    face_flux_jacobian(gamma, wl, wr, phi, Jf);
    for (int c = 0; c < 4; ++c) {
        for (int k = 0; k < 16; ++k)
            Jl[c][k] = 0.0;
        for (int v = 0; v < 4; ++v) {
            for (int k = 0; k < 3; ++k) {
                Jl[c][4 * k + v] += Jf[c][v] * dl[v][k];           /* w^L: cells 0..2 */
                Jl[c][4 * (k + 1) + v] += Jf[c][4 + v] * dr[v][k]; /* w^R: cells 1..3 */
            }
        }
    }
}

/* The conservative-variable reconstruction (an alternative to the primitive
 * one of Sec. 5): Q[k] = face-frame conservative state (rho, rho u_n,
 * rho u_t, rho E) of cells m-1 .. m+2; the limited slopes of eq. (sweby)
 * act on Q, the two face states are converted to primitive variables for
 * the acoustic solve of eqs. (13)-(14), and eq. (12) takes the
 * reconstructed conservative vector of the upwind side. */
static void stencil_face_cons(double gamma, double beta, const double Q[4][4], double phi[4])
{
    double ql[4], qr[4], wl[4], wr[4];
    for (int v = 0; v < 4; ++v) {
        ql[v] = Q[1][v] + 0.5 * lfo_sweby(Q[1][v] - Q[0][v], Q[2][v] - Q[1][v], beta);
        qr[v] = Q[2][v] - 0.5 * lfo_sweby(Q[2][v] - Q[1][v], Q[3][v] - Q[2][v], beta);
    }
    lfo_cons_to_prim(gamma, ql, wl);
    lfo_cons_to_prim(gamma, qr, wr);
    double us, ps;
    lfo_acoustic_solve(gamma, wl[0], wl[1], wl[3], wr[0], wr[1], wr[3], &us, &ps);
    const double *qa = (us > 0.0) ? ql : qr;
    phi[0] = qa[0] * us;
    phi[1] = qa[1] * us + ps;
    phi[2] = qa[2] * us;
    phi[3] = (qa[3] + ps) * us;
}

/* Flux of rho y_k under the conservative reconstruction: rho y_k itself is
 * reconstructed, and crosses the face from the upwind side of u* (the same
 * u* as stencil_face_cons). */
static double species_face_flux_cons(double gamma, double beta, const double Q[4][4],
                                     const double Y[4])
{
    double ql[4], qr[4], wl[4], wr[4];
    for (int v = 0; v < 4; ++v) {
        ql[v] = Q[1][v] + 0.5 * lfo_sweby(Q[1][v] - Q[0][v], Q[2][v] - Q[1][v], beta);
        qr[v] = Q[2][v] - 0.5 * lfo_sweby(Q[2][v] - Q[1][v], Q[3][v] - Q[2][v], beta);
    }
    lfo_cons_to_prim(gamma, ql, wl);
    lfo_cons_to_prim(gamma, qr, wr);
    double us, ps;
    lfo_acoustic_solve(gamma, wl[0], wl[1], wl[3], wr[0], wr[1], wr[3], &us, &ps);
    double yl = Y[1] + 0.5 * lfo_sweby(Y[1] - Y[0], Y[2] - Y[1], beta);
    double yr = Y[2] - 0.5 * lfo_sweby(Y[2] - Y[1], Y[3] - Y[2], beta);
    return ((us > 0.0) ? yl : yr) * us;
}

/* ------------------------------------------------------------------------ */
/* Grid helpers                                                             */
/* ------------------------------------------------------------------------ */

/* Boundary index mapping: periodic wraps, transmissive clamps (ghost cells
 * copy the edge cell). */
static int map_index(int k, int n, int bc)
{
    if (bc == LFO_BC_PERIODIC) {
        k %= n;
        return k < 0 ? k + n : k;
    }
    return k < 0 ? 0 : (k >= n ? n - 1 : k);
}

static int check_params(const lfo_params *P)
{
    if (!P || P->nx < 1 || P->ny < 1) return 0;
    if (!(P->dx > 0.0) || !(P->dy > 0.0)) return 0;
    if (!(P->gamma > 1.0 && P->gamma <= 3.0)) return 0;
    if (!(P->beta >= 0.0 && P->beta <= 2.0)) return 0;
    if (!(P->cfl > 0.0)) return 0;
    if (P->ns < 0 || P->ns > LFO_MAX_SPECIES) return 0;
    if (P->recon != LFO_RECON_PRIMITIVE && P->recon != LFO_RECON_CONSERVATIVE) return 0;
    if ((P->bc_x != LFO_BC_PERIODIC && P->bc_x != LFO_BC_TRANSMISSIVE) ||
        (P->bc_y != LFO_BC_PERIODIC && P->bc_y != LFO_BC_TRANSMISSIVE))
        return 0;
    return 1;
}

/* Primitive variables of every cell, layout w[v][j][i]: (rho, u, v, p)
 * followed by the mass fractions y_k = (rho y_k) / rho. */
static void all_prims(const lfo_params *P, const double *U, double *w)
{
    const int64_t N = (int64_t)P->nx * P->ny;
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < N; ++q) {
        double Uq[4] = {U[q], U[N + q], U[2 * N + q], U[3 * N + q]};
        double wq[4];
        lfo_cons_to_prim(P->gamma, Uq, wq);
        for (int v = 0; v < 4; ++v)
            w[v * N + q] = wq[v];
        for (int k = 0; k < P->ns; ++k)
            w[(4 + k) * N + q] = U[(4 + k) * N + q] / U[q];
    }
}

/* Flux of rho y_k through one face (Sec. 7, conservative form of the mass
 * fraction transport, discretised like the mass flux of eq. (12)).  W is
 * the face-frame Euler stencil of stencil_face() and Y the mass fraction
 * of the same four cells.  Both y and the Euler variables are
 * reconstructed with the limited slopes of Sec. 5; the acoustic solve of
 * eqs. (13)-(14) on the reconstructed states gives u*, the upwind side A
 * is the left one when u* > 0, and the flux is (rho_A y_A) u*. */
static double species_face_flux(double gamma, double beta, const double W[4][4],
                                const double Y[4])
{
    double wl[4], wr[4];
    for (int v = 0; v < 4; ++v) {
        wl[v] = W[1][v] + 0.5 * lfo_sweby(W[1][v] - W[0][v], W[2][v] - W[1][v], beta);
        wr[v] = W[2][v] - 0.5 * lfo_sweby(W[2][v] - W[1][v], W[3][v] - W[2][v], beta);
    }
    double yl = Y[1] + 0.5 * lfo_sweby(Y[1] - Y[0], Y[2] - Y[1], beta);
    double yr = Y[2] - 0.5 * lfo_sweby(Y[2] - Y[1], Y[3] - Y[2], beta);
    double us, ps;
    lfo_acoustic_solve(gamma, wl[0], wl[1], wl[3], wr[0], wr[1], wr[3], &us, &ps);
    if (us > 0.0)
        return (wl[0] * yl) * us;
    return (wr[0] * yr) * us;
}

/* Face-frame stencil of x-face k (between cells k-1 and k of row j):
 * cells k-2 .. k+1, frame (rho, u, v, p).  Returns the mapped cell ids. */
static void gather_x(const lfo_params *P, const double *w, int j, int k,
                     double W[4][4], int64_t cell[4])
{
    const int64_t N = (int64_t)P->nx * P->ny;
    for (int s = 0; s < 4; ++s) {
        int i = map_index(k - 2 + s, P->nx, P->bc_x);
        int64_t q = (int64_t)j * P->nx + i;
        cell[s] = q;
        W[s][0] = w[q];
        W[s][1] = w[N + q];
        W[s][2] = w[2 * N + q];
        W[s][3] = w[3 * N + q];
    }
}

/* y-face k (between cells k-1 and k of column i): frame (rho, v, u, p). */
static void gather_y(const lfo_params *P, const double *w, int i, int k,
                     double W[4][4], int64_t cell[4])
{
    const int64_t N = (int64_t)P->nx * P->ny;
    for (int s = 0; s < 4; ++s) {
        int j = map_index(k - 2 + s, P->ny, P->bc_y);
        int64_t q = (int64_t)j * P->nx + i;
        cell[s] = q;
        W[s][0] = w[q];
        W[s][1] = w[2 * N + q];
        W[s][2] = w[N + q];
        W[s][3] = w[3 * N + q];
    }
}

/* Frame component c of a face flux -> conservative field index. */
static const int XFIELD[4] = {0, 1, 2, 3};
static const int YFIELD[4] = {0, 2, 1, 3};

/* ------------------------------------------------------------------------ */
/* Residual, eq. (11): R_K = (1/|K|) sum_A |A| Phi_A                         */
/* ------------------------------------------------------------------------ */

int lfo_residual(const lfo_params *P, const double *U, double *R)
{
    if (!check_params(P) || !U || !R) return LFO_ERR_ARG;
    const int nx = P->nx, ny = P->ny, nf = 4 + P->ns;
    const int64_t N = (int64_t)nx * ny;
    double *w = (double *)malloc(sizeof(double) * nf * N);
    /* Fx[c][j][k], k = 0..nx: x-face between cells k-1 and k.
     * Gy[c][k][i], k = 0..ny: y-face between cells k-1 and k. */
    const int64_t NFx = (int64_t)ny * (nx + 1), NGy = (int64_t)(ny + 1) * nx;
    double *Fx = (double *)malloc(sizeof(double) * nf * NFx);
    double *Gy = (double *)malloc(sizeof(double) * nf * NGy);
    if (!w || !Fx || !Gy) { free(w); free(Fx); free(Gy); return LFO_ERR_ARG; }

    all_prims(P, U, w);

#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
        for (int k = 0; k <= nx; ++k) {
            double W[4][4], phi[4];
            int64_t cell[4];
            gather_x(P, w, j, k, W, cell);
            double Q[4][4];
            if (P->recon == LFO_RECON_CONSERVATIVE) {
                for (int t = 0; t < 4; ++t)
                    for (int c = 0; c < 4; ++c)
                        Q[t][c] = U[XFIELD[c] * N + cell[t]];
                stencil_face_cons(P->gamma, P->beta, Q, phi);
            } else {
                stencil_face(P->gamma, P->beta, W, phi, NULL);
            }
            for (int c = 0; c < 4; ++c)
                Fx[XFIELD[c] * NFx + (int64_t)j * (nx + 1) + k] = phi[c];
            for (int sp = 0; sp < P->ns; ++sp) {
                double Y[4];
                const int cons = P->recon == LFO_RECON_CONSERVATIVE;
                for (int t = 0; t < 4; ++t)
                    Y[t] = cons ? U[(4 + sp) * N + cell[t]] : w[(4 + sp) * N + cell[t]];
                Fx[(4 + sp) * NFx + (int64_t)j * (nx + 1) + k] =
                    cons ? species_face_flux_cons(P->gamma, P->beta, Q, Y)
                         : species_face_flux(P->gamma, P->beta, W, Y);
            }
        }
    }
#pragma omp parallel for schedule(static)
    for (int k = 0; k <= ny; ++k) {
        for (int i = 0; i < nx; ++i) {
            double W[4][4], phi[4];
            int64_t cell[4];
            gather_y(P, w, i, k, W, cell);
            double Q[4][4];
            if (P->recon == LFO_RECON_CONSERVATIVE) {
                for (int t = 0; t < 4; ++t)
                    for (int c = 0; c < 4; ++c)
                        Q[t][c] = U[YFIELD[c] * N + cell[t]];
                stencil_face_cons(P->gamma, P->beta, Q, phi);
            } else {
                stencil_face(P->gamma, P->beta, W, phi, NULL);
            }
            for (int c = 0; c < 4; ++c)
                Gy[YFIELD[c] * NGy + (int64_t)k * nx + i] = phi[c];
            for (int sp = 0; sp < P->ns; ++sp) {
                double Y[4];
                const int cons = P->recon == LFO_RECON_CONSERVATIVE;
                for (int t = 0; t < 4; ++t)
                    Y[t] = cons ? U[(4 + sp) * N + cell[t]] : w[(4 + sp) * N + cell[t]];
                Gy[(4 + sp) * NGy + (int64_t)k * nx + i] =
                    cons ? species_face_flux_cons(P->gamma, P->beta, Q, Y)
                         : species_face_flux(P->gamma, P->beta, W, Y);
            }
        }
    }
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            for (int f = 0; f < nf; ++f) {
                double fe = Fx[f * NFx + (int64_t)j * (nx + 1) + i + 1];
                double fw = Fx[f * NFx + (int64_t)j * (nx + 1) + i];
                double gn = Gy[f * NGy + (int64_t)(j + 1) * nx + i];
                double gs = Gy[f * NGy + (int64_t)j * nx + i];
                R[f * N + (int64_t)j * nx + i] = (fe - fw) / P->dx + (gn - gs) / P->dy;
            }
        }
    }
    free(w);
    free(Fx);
    free(Gy);
    return LFO_OK;
}

/* ------------------------------------------------------------------------ */
/* Time step (Heun list, item 1: "compute dt subject to some CFL condition") */
/* ------------------------------------------------------------------------ */

int lfo_dt(const lfo_params *P, const double *U, double *dt)
{
    if (!check_params(P) || !U || !dt) return LFO_ERR_ARG;
    const int64_t N = (int64_t)P->nx * P->ny;
    double smax = 0.0;
    int bad = 0;
#pragma omp parallel for reduction(max : smax) reduction(| : bad) schedule(static)
    for (int64_t q = 0; q < N; ++q) {
        double Uq[4] = {U[q], U[N + q], U[2 * N + q], U[3 * N + q]};
        double w[4];
        lfo_cons_to_prim(P->gamma, Uq, w);
        double c = sqrt(P->gamma * w[3] / w[0]);
        double s = (fabs(w[1]) + c) / P->dx + (fabs(w[2]) + c) / P->dy;
        if (!(w[0] > 0.0) || !(w[3] > 0.0) || !isfinite(s) || !isfinite(Uq[0]) ||
            !isfinite(Uq[1]) || !isfinite(Uq[2]) || !isfinite(Uq[3])) {
            bad = 1;
        } else if (s > smax) {
            smax = s;
        }
    }
    if (bad || !(smax > 0.0)) {
        *dt = 0.0;
        return LFO_ERR_NONPHYSICAL;
    }
    *dt = P->cfl / smax;
    return LFO_OK;
}

/* ------------------------------------------------------------------------ */
/* Heun step (Sec. 5, predictor-corrector list, items 2-11)                 */
/* ------------------------------------------------------------------------ */

int lfo_step(const lfo_params *P, const double *Un, double dt, double *Unp1)
{
    if (!check_params(P) || !Un || !Unp1) return LFO_ERR_ARG;
    const int64_t M = (4 + P->ns) * (int64_t)P->nx * P->ny;
    double *Rn = (double *)malloc(sizeof(double) * M);
    double *Us = (double *)malloc(sizeof(double) * M);
    double *Rs = (double *)malloc(sizeof(double) * M);
    if (!Rn || !Us || !Rs) { free(Rn); free(Us); free(Rs); return LFO_ERR_ARG; }

    /* items 2-6: predictor U* = U^n - dt R(U^n) */
    lfo_residual(P, Un, Rn);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < M; ++q)
        Us[q] = Un[q] - dt * Rn[q];
    /* items 7-11: corrector with the mean of both fluxes */
    lfo_residual(P, Us, Rs);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < M; ++q)
        Unp1[q] = Un[q] - dt * (0.5 * (Rn[q] + Rs[q]));

    free(Rn);
    free(Us);
    free(Rs);
    return LFO_OK;
}

int lfo_advance(const lfo_params *P, double *U, double t0, double t_end,
                int64_t max_steps, double *t_out, int64_t *steps_out, double *dts)
{
    if (!check_params(P) || !U) return LFO_ERR_ARG;
    const int64_t M = (4 + P->ns) * (int64_t)P->nx * P->ny;
    double *Unew = (double *)malloc(sizeof(double) * M);
    if (!Unew) return LFO_ERR_ARG;
    double t = t0;
    int64_t steps = 0;
    int rc = LFO_OK;
    while (t < t_end && steps < max_steps) {
        double dt;
        rc = lfo_dt(P, U, &dt);
        if (rc != LFO_OK) break;
        int last = 0;
        if (dt >= t_end - t) {
            dt = t_end - t;
            last = 1;
        }
        lfo_step(P, U, dt, Unew);
        memcpy(U, Unew, sizeof(double) * M);
        t = last ? t_end : t + dt;
        if (dts) dts[steps] = dt;
        ++steps;
    }
    if (rc == LFO_OK) {
        double dt_end;
        rc = lfo_dt(P, U, &dt_end); /* the final state must be physical too */
    }
    free(Unew);
    if (t_out) *t_out = t;
    if (steps_out) *steps_out = steps;
    return rc;
}

void lfo_totals(const lfo_params *P, const double *U, double *out)
{
    const int64_t N = (int64_t)P->nx * P->ny;
    for (int f = 0; f < 4 + P->ns; ++f) {
        double s = 0.0, comp = 0.0; /* Neumaier compensated sum */
        for (int64_t q = 0; q < N; ++q) {
            double x = U[f * N + q];
            double t = s + x;
            if (fabs(s) >= fabs(x))
                comp += (s - t) + x;
            else
                comp += (x - t) + s;
            s = t;
        }
        out[f] = (s + comp) * P->dx * P->dy;
    }
}

/* ------------------------------------------------------------------------ */
/* Linearisation at frozen dt                                               */
/* ------------------------------------------------------------------------ */

/* d w / d U of lfo_cons_to_prim at one cell (row v = primitive variable). */
static void prim_jacobian(double gamma, const double U[4], double D[4][4])
{
    double w[4];
    lfo_cons_to_prim(gamma, U, w);
    double rho = w[0], u = w[1], v = w[2];
    double gm = gamma - 1.0;
    double D0[4][4] = {
        {1.0, 0.0, 0.0, 0.0},
        {-u / rho, 1.0 / rho, 0.0, 0.0},
        {-v / rho, 0.0, 1.0 / rho, 0.0},
        {gm * 0.5 * (u * u + v * v), -gm * u, -gm * v, gm},
    };
    memcpy(D, D0, sizeof(D0));
}

/* Tangent of every primitive variable: dw = (dw/dU) dU per cell. */
static void prim_tangent(const lfo_params *P, const double *U, const double *dU, double *dw)
{
    const int64_t N = (int64_t)P->nx * P->ny;
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < N; ++q) {
        double Uq[4] = {U[q], U[N + q], U[2 * N + q], U[3 * N + q]};
        double D[4][4];
        prim_jacobian(P->gamma, Uq, D);
        for (int v = 0; v < 4; ++v) {
            double s = 0.0;
            for (int f = 0; f < 4; ++f)
                s += D[v][f] * dU[f * N + q];
            dw[v * N + q] = s;
        }
    }
}

int lfo_residual_jvp(const lfo_params *P, const double *U, const double *dU, double *out)
{
    if (!check_params(P) || !U || !dU || !out) return LFO_ERR_ARG;
    if (P->ns != 0 || P->recon != LFO_RECON_PRIMITIVE) return LFO_ERR_ARG; /* Euler fields, Sec. 5 reconstruction */
    const int nx = P->nx, ny = P->ny;
    const int64_t N = (int64_t)nx * ny;
    const int64_t NFx = (int64_t)ny * (nx + 1), NGy = (int64_t)(ny + 1) * nx;
    double *w = (double *)malloc(sizeof(double) * 4 * N);
    double *dw = (double *)malloc(sizeof(double) * 4 * N);
    double *dFx = (double *)malloc(sizeof(double) * 4 * NFx);
    double *dGy = (double *)malloc(sizeof(double) * 4 * NGy);
    if (!w || !dw || !dFx || !dGy) { free(w); free(dw); free(dFx); free(dGy); return LFO_ERR_ARG; }
    all_prims(P, U, w);
    prim_tangent(P, U, dU, dw);

#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
        for (int k = 0; k <= nx; ++k) {
            double W[4][4], dW[4][4], phi[4], Jl[4][16];
            int64_t cell[4];
            gather_x(P, w, j, k, W, cell);
            gather_x(P, dw, j, k, dW, cell);
            stencil_face(P->gamma, P->beta, W, phi, Jl);
            for (int c = 0; c < 4; ++c) {
                double s = 0.0;
                for (int m = 0; m < 16; ++m)
                    s += Jl[c][m] * dW[m / 4][m % 4];
                dFx[XFIELD[c] * NFx + (int64_t)j * (nx + 1) + k] = s;
            }
        }
    }
#pragma omp parallel for schedule(static)
    for (int k = 0; k <= ny; ++k) {
        for (int i = 0; i < nx; ++i) {
            double W[4][4], dW[4][4], phi[4], Jl[4][16];
            int64_t cell[4];
            gather_y(P, w, i, k, W, cell);
            gather_y(P, dw, i, k, dW, cell);
            stencil_face(P->gamma, P->beta, W, phi, Jl);
            for (int c = 0; c < 4; ++c) {
                double s = 0.0;
                for (int m = 0; m < 16; ++m)
                    s += Jl[c][m] * dW[m / 4][m % 4];
                dGy[YFIELD[c] * NGy + (int64_t)k * nx + i] = s;
            }
        }
    }
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            for (int f = 0; f < 4; ++f)
                out[f * N + (int64_t)j * nx + i] =
                    (dFx[f * NFx + (int64_t)j * (nx + 1) + i + 1] - dFx[f * NFx + (int64_t)j * (nx + 1) + i]) / P->dx +
                    (dGy[f * NGy + (int64_t)(j + 1) * nx + i] - dGy[f * NGy + (int64_t)j * nx + i]) / P->dy;
    free(w);
    free(dw);
    free(dFx);
    free(dGy);
    return LFO_OK;
}

/* Transpose of lfo_residual_jvp.  Face k of a row carries +Phi/dx into
 * cell k-1 and -Phi/dx into cell k (those that exist), so its cotangent is
 * (g_{k-1} - g_k)/dx; it is pulled back through the face's local Jacobian
 * onto the primitive variables of its four (mapped) stencil cells, then
 * through d w / d U. */
int lfo_residual_vjp(const lfo_params *P, const double *U, const double *g, double *out)
{
    if (!check_params(P) || !U || !g || !out) return LFO_ERR_ARG;
    if (P->ns != 0 || P->recon != LFO_RECON_PRIMITIVE) return LFO_ERR_ARG; /* Euler fields, Sec. 5 reconstruction */
    const int nx = P->nx, ny = P->ny;
    const int64_t N = (int64_t)nx * ny;
    double *w = (double *)malloc(sizeof(double) * 4 * N);
    double *wbar = (double *)calloc(4 * N, sizeof(double));
    if (!w || !wbar) { free(w); free(wbar); return LFO_ERR_ARG; }
    all_prims(P, U, w);

    /* x-faces: every stencil cell of a row-j face lies in row j, so rows
     * are independent. */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
        for (int k = 0; k <= nx; ++k) {
            double W[4][4], phi[4], Jl[4][16];
            int64_t cell[4];
            gather_x(P, w, j, k, W, cell);
            stencil_face(P->gamma, P->beta, W, phi, Jl);
            double pbar[4];
            for (int c = 0; c < 4; ++c) {
                int f = XFIELD[c];
                double gl = (k - 1 >= 0) ? g[f * N + (int64_t)j * nx + k - 1] : 0.0;
                double gr = (k < nx) ? g[f * N + (int64_t)j * nx + k] : 0.0;
                pbar[c] = (gl - gr) / P->dx;
            }
            for (int m = 0; m < 16; ++m) {
                double s = 0.0;
                for (int c = 0; c < 4; ++c)
                    s += Jl[c][m] * pbar[c];
                int fv = m % 4; /* frame var -> primitive index (rho,u,v,p) */
                int pv = fv;    /* x frame is (rho, u, v, p) */
                wbar[pv * N + cell[m / 4]] += s;
            }
        }
    }
    /* y-faces: columns are independent. */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nx; ++i) {
        for (int k = 0; k <= ny; ++k) {
            double W[4][4], phi[4], Jl[4][16];
            int64_t cell[4];
            gather_y(P, w, i, k, W, cell);
            stencil_face(P->gamma, P->beta, W, phi, Jl);
            double pbar[4];
            for (int c = 0; c < 4; ++c) {
                int f = YFIELD[c];
                double gl = (k - 1 >= 0) ? g[f * N + (int64_t)(k - 1) * nx + i] : 0.0;
                double gr = (k < ny) ? g[f * N + (int64_t)k * nx + i] : 0.0;
                pbar[c] = (gl - gr) / P->dy;
            }
            for (int m = 0; m < 16; ++m) {
                double s = 0.0;
                for (int c = 0; c < 4; ++c)
                    s += Jl[c][m] * pbar[c];
                static const int YPRIM[4] = {0, 2, 1, 3}; /* frame (rho,v,u,p) */
                wbar[YPRIM[m % 4] * N + cell[m / 4]] += s;
            }
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < N; ++q) {
        double Uq[4] = {U[q], U[N + q], U[2 * N + q], U[3 * N + q]};
        double D[4][4];
        prim_jacobian(P->gamma, Uq, D);
        for (int f = 0; f < 4; ++f) {
            double s = 0.0;
            for (int v = 0; v < 4; ++v)
                s += D[v][f] * wbar[v * N + q];
            out[f * N + q] = s;
        }
    }
    free(w);
    free(wbar);
    return LFO_OK;
}

/* Tangent of U^{n+1} = U^n - dt (R(U^n) + R(U*))/2, U* = U^n - dt R(U^n). */
int lfo_tlm_step(const lfo_params *P, const double *Un, double dt,
                 const double *dUn, double *dUnp1)
{
    if (!check_params(P) || !Un || !dUn || !dUnp1) return LFO_ERR_ARG;
    if (P->ns != 0 || P->recon != LFO_RECON_PRIMITIVE) return LFO_ERR_ARG; /* Euler fields, Sec. 5 reconstruction */
    const int64_t M = 4 * (int64_t)P->nx * P->ny;
    double *Rn = (double *)malloc(sizeof(double) * M);
    double *Us = (double *)malloc(sizeof(double) * M);
    double *dRn = (double *)malloc(sizeof(double) * M);
    double *dUs = (double *)malloc(sizeof(double) * M);
    double *dRs = (double *)malloc(sizeof(double) * M);
    if (!Rn || !Us || !dRn || !dUs || !dRs) {
        free(Rn); free(Us); free(dRn); free(dUs); free(dRs);
        return LFO_ERR_ARG;
    }
    lfo_residual(P, Un, Rn);
    for (int64_t q = 0; q < M; ++q)
        Us[q] = Un[q] - dt * Rn[q];
    lfo_residual_jvp(P, Un, dUn, dRn);
    for (int64_t q = 0; q < M; ++q)
        dUs[q] = dUn[q] - dt * dRn[q];
    lfo_residual_jvp(P, Us, dUs, dRs);
    for (int64_t q = 0; q < M; ++q)
        dUnp1[q] = dUn[q] - dt * (0.5 * (dRn[q] + dRs[q]));
    free(Rn); free(Us); free(dRn); free(dUs); free(dRs);
    return LFO_OK;
}

/* Reverse mode of the same step:
 *   cotangent of U*  : mu  = -(dt/2) J_R(U*)^T lam
 *   cotangent of R^n : rb  = -(dt/2) lam - dt mu
 *   lam^n            = lam + mu + J_R(U^n)^T rb.                         */
int lfo_adjoint_step(const lfo_params *P, const double *Un, double dt,
                     const double *lam_np1, double *lam_n)
{
    if (!check_params(P) || !Un || !lam_np1 || !lam_n) return LFO_ERR_ARG;
    if (P->ns != 0 || P->recon != LFO_RECON_PRIMITIVE) return LFO_ERR_ARG; /* Euler fields, Sec. 5 reconstruction */
    const int64_t M = 4 * (int64_t)P->nx * P->ny;
    double *Rn = (double *)malloc(sizeof(double) * M);
    double *Us = (double *)malloc(sizeof(double) * M);
    double *mu = (double *)malloc(sizeof(double) * M);
    double *rb = (double *)malloc(sizeof(double) * M);
    double *tmp = (double *)malloc(sizeof(double) * M);
    if (!Rn || !Us || !mu || !rb || !tmp) {
        free(Rn); free(Us); free(mu); free(rb); free(tmp);
        return LFO_ERR_ARG;
    }
    lfo_residual(P, Un, Rn);
    for (int64_t q = 0; q < M; ++q)
        Us[q] = Un[q] - dt * Rn[q];
    lfo_residual_vjp(P, Us, lam_np1, tmp);
    for (int64_t q = 0; q < M; ++q) {
        mu[q] = -(0.5 * dt) * tmp[q];
        rb[q] = -(0.5 * dt) * lam_np1[q] - dt * mu[q];
    }
    lfo_residual_vjp(P, Un, rb, tmp);
    for (int64_t q = 0; q < M; ++q)
        lam_n[q] = lam_np1[q] + mu[q] + tmp[q];
    free(Rn); free(Us); free(mu); free(rb); free(tmp);
    return LFO_OK;
}

/* ------------------------------------------------------------------------ */
/* Exact Riemann solver (ideal gas), by the pressure-function method of     */
/* Toro, "Riemann Solvers and Numerical Methods for Fluid Dynamics", ch. 4, */
/* the textbook the paper compares its shock tubes against.                 */
/* ------------------------------------------------------------------------ */

/* Pressure function f_K(p) of one side and its derivative: shock branch
 * for p > p_K (Rankine-Hugoniot), rarefaction branch otherwise
 * (isentropic). */
static void pressure_function(double g, double p, double rk, double pk, double ck,
                              double *f, double *fd)
{
    if (p > pk) {
        double A = 2.0 / ((g + 1.0) * rk);
        double B = (g - 1.0) / (g + 1.0) * pk;
        double q = sqrt(A / (p + B));
        *f = (p - pk) * q;
        *fd = q * (1.0 - 0.5 * (p - pk) / (B + p));
    } else {
        double r = p / pk;
        *f = 2.0 * ck / (g - 1.0) * (pow(r, (g - 1.0) / (2.0 * g)) - 1.0);
        *fd = 1.0 / (rk * ck) * pow(r, -(g + 1.0) / (2.0 * g));
    }
}

int lfo_exact_riemann(double g,
                      double rl, double ul, double pl,
                      double rr, double ur, double pr,
                      int64_t n, const double *xi,
                      double *rho, double *u, double *p,
                      double *p_star, double *u_star)
{
    double cl = sqrt(g * pl / rl), cr = sqrt(g * pr / rr);
    if (2.0 / (g - 1.0) * (cl + cr) <= ur - ul)
        return LFO_ERR_VACUUM; /* the data generate vacuum */

    /* Newton iteration on f_L(p) + f_R(p) + (u_R - u_L) = 0, started from
     * the two-rarefaction approximation (exact when both waves are
     * rarefactions). */
    double z = (g - 1.0) / (2.0 * g);
    double ps = pow((cl + cr - 0.5 * (g - 1.0) * (ur - ul)) /
                        (cl / pow(pl, z) + cr / pow(pr, z)), 1.0 / z);
    if (!(ps > 0.0)) ps = 1e-12;
    for (int it = 0; it < 200; ++it) {
        double fl, fdl, fr, fdr;
        pressure_function(g, ps, rl, pl, cl, &fl, &fdl);
        pressure_function(g, ps, rr, pr, cr, &fr, &fdr);
        double pn = ps - (fl + fr + ur - ul) / (fdl + fdr);
        if (pn <= 0.0) pn = 0.5 * ps;
        double change = fabs(pn - ps) / (0.5 * (pn + ps));
        ps = pn;
        if (change < 1e-15) break;
    }
    double fl, fdl, fr, fdr;
    pressure_function(g, ps, rl, pl, cl, &fl, &fdl);
    pressure_function(g, ps, rr, pr, cr, &fr, &fdr);
    double us = 0.5 * (ul + ur) + 0.5 * (fr - fl);
    if (p_star) *p_star = ps;
    if (u_star) *u_star = us;

    double gp = (g + 1.0) / (2.0 * g), gm = (g - 1.0) / (2.0 * g);
    double g6 = (g - 1.0) / (g + 1.0);
    for (int64_t k = 0; k < n; ++k) {
        double S = xi[k];
        double R, V, Pp;
        if (S <= us) { /* left of the contact */
            if (ps > pl) { /* left shock */
                double SL = ul - cl * sqrt(gp * ps / pl + gm);
                if (S <= SL) { R = rl; V = ul; Pp = pl; }
                else { R = rl * (ps / pl + g6) / (g6 * ps / pl + 1.0); V = us; Pp = ps; }
            } else { /* left rarefaction */
                double SHL = ul - cl;
                double cml = cl * pow(ps / pl, gm);
                double STL = us - cml;
                if (S <= SHL) { R = rl; V = ul; Pp = pl; }
                else if (S > STL) { R = rl * pow(ps / pl, 1.0 / g); V = us; Pp = ps; }
                else {
                    V = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + S);
                    double c = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * (ul - S));
                    R = rl * pow(c / cl, 2.0 / (g - 1.0));
                    Pp = pl * pow(c / cl, 2.0 * g / (g - 1.0));
                }
            }
        } else { /* right of the contact */
            if (ps > pr) { /* right shock */
                double SR = ur + cr * sqrt(gp * ps / pr + gm);
                if (S >= SR) { R = rr; V = ur; Pp = pr; }
                else { R = rr * (ps / pr + g6) / (g6 * ps / pr + 1.0); V = us; Pp = ps; }
            } else { /* right rarefaction */
                double SHR = ur + cr;
                double cmr = cr * pow(ps / pr, gm);
                double STR = us + cmr;
                if (S >= SHR) { R = rr; V = ur; Pp = pr; }
                else if (S < STR) { R = rr * pow(ps / pr, 1.0 / g); V = us; Pp = ps; }
                else {
                    V = 2.0 / (g + 1.0) * (-cr + 0.5 * (g - 1.0) * ur + S);
                    double c = 2.0 / (g + 1.0) * (cr - 0.5 * (g - 1.0) * (ur - S));
                    R = rr * pow(c / cr, 2.0 / (g - 1.0));
                    Pp = pr * pow(c / cr, 2.0 * g / (g - 1.0));
                }
            }
        }
        if (rho) rho[k] = R;
        if (u) u[k] = V;
        if (p) p[k] = Pp;
    }
    return LFO_OK;
}
