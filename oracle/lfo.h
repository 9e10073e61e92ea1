/*
 * lfo.h -- plain FP64 CPU oracle of the second-order Lagrange-flux scheme
 * (De Vuyst, Gasc, Motte, Peybernes, Poncet, "Lagrange-flux schemes:
 * reformulating second-order accurate Lagrange-remap schemes for better
 * node-based HPC performance", arXiv:1607.08710).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or helper with
 * the GPU library, and the GPU library never calls it.
 *
 * Everything is IEEE double, compiled without floating-point contraction
 * or fast-math, and written as the plainest loop that states the
 * definition: every face flux is computed from its own four-cell stencil,
 * fluxes are stored on the faces, then differenced.  No blocking, fusion
 * or reordering beyond the paper's own algorithm (Sec. 5, the Heun list).
 *
 * State layout: structure of arrays U[f][j][i], f = 0..3 for
 * (rho, rho*u, rho*v, rho*E), i the x index (fastest), j the y index.
 * Primitive layout: w = (rho, u, v, p).
 *
 * Readings of the paper taken here (where it is silent):
 *  - MUSCL reconstruction of the primitive variables (rho, u, v, p),
 *    dimension by dimension; the upwind interface state is the
 *    conservative vector of the reconstructed upwind primitive state.
 *    The conservative-variable reconstruction (recon = 1) is an ablation:
 *    it limits (rho, rho u, rho v, rho E) instead, converts the face
 *    states to primitive variables for the acoustic solve and upwinds the
 *    reconstructed conservative vector.
 *  - The CFL time step is dt = cfl / max_K[(|u|+c)/dx + (|v|+c)/dy].
 *  - Boundary conditions per axis: periodic (index wrap) or transmissive
 *    (index clamp: ghost cells copy the edge cell).
 *  - Upwind side: left when u* > 0, right otherwise.
 *  - Passive mass fractions (the conservative transport equations of
 *    rho y_k, Sec. 7): y_k = (rho y_k) / rho is reconstructed like the other
 *    primitive variables, and the flux through a face is (rho_A y_k,A) u*
 *    with A the same upwind side and rho_A the reconstructed density of
 *    that side.  A single gamma for the mixture (the paper gives no mixture
 *    law).
 */
#ifndef LFO_H
#define LFO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { LFO_BC_PERIODIC = 0, LFO_BC_TRANSMISSIVE = 1 };

/* Return codes. */
enum { LFO_OK = 0, LFO_ERR_ARG = 1, LFO_ERR_NONPHYSICAL = 3, LFO_ERR_VACUUM = 5 };

typedef struct {
    int32_t nx, ny;      /* cells along x and y, >= 1                        */
    double dx, dy;       /* uniform cell sizes, > 0                          */
    double gamma;        /* ratio of specific heats, in (1, 3]               */
    double cfl;          /* CFL number used by lfo_dt, > 0                   */
    double beta;         /* Sweby limiter coefficient, in [0, 2]             */
    int32_t bc_x, bc_y;  /* LFO_BC_PERIODIC or LFO_BC_TRANSMISSIVE          */
    int32_t ns;          /* passive mass fractions, 0..LFO_MAX_SPECIES: the
                            state then holds 4 + ns fields, field 4 + k
                            being rho y_k                                    */
    int32_t recon;       /* LFO_RECON_PRIMITIVE (Sec. 5: rho, u, v, p and
                            y_k) or LFO_RECON_CONSERVATIVE (rho, rho u,
                            rho v, rho E and rho y_k; the ablation)           */
} lfo_params;

enum { LFO_RECON_PRIMITIVE = 0, LFO_RECON_CONSERVATIVE = 1 };

#define LFO_MAX_SPECIES 8

/* ---- pointwise pieces (Sec. 3 EOS; eq. (sweby); eqs. (13)-(14); eq. (12)) */

/* Conservative -> primitive, perfect-gas law of Sec. 3. */
void lfo_cons_to_prim(double gamma, const double U[4], double w[4]);

/* Sweby limiter phi(a, b) of eq. (sweby); zero when a*b <= 0. */
double lfo_sweby(double a, double b, double beta);

/* Lagrangian HLL (acoustic) interface solve, eqs. (13)-(14). */
void lfo_acoustic_solve(double gamma,
                        double rho_l, double u_l, double p_l,
                        double rho_r, double u_r, double p_r,
                        double *u_star, double *p_star);

/* Face flux of eq. (12) in the face frame.  wl, wr = (rho, u_n, u_t, p)
 * with u_n the velocity along the face normal (pointing from the left cell
 * to the right cell) and u_t the tangential velocity.  phi = (mass, normal
 * momentum, tangential momentum, energy) flux through the face. */
void lfo_face_flux(double gamma, const double wl[4], const double wr[4],
                   double phi[4]);

/* ---- grid operators ----------------------------------------------------- */

/* R(U) = (F_{i+1/2} - F_{i-1/2})/dx + (G_{j+1/2} - G_{j-1/2})/dy, i.e.
 * (1/|K|) sum_A |A| Phi_A of the semi-discrete scheme (eq. (11)). */
int lfo_residual(const lfo_params *P, const double *U, double *R);

/* CFL time step from state U.  Returns LFO_ERR_NONPHYSICAL (and dt = 0)
 * if any cell has rho <= 0, p <= 0 or a non-finite value. */
int lfo_dt(const lfo_params *P, const double *U, double *dt);

/* One Heun step at a given dt (Sec. 5, the predictor-corrector list):
 *   U*      = U^n - dt R(U^n)
 *   U^{n+1} = U^n - dt (R(U^n) + R(U*)) / 2.                               */
int lfo_step(const lfo_params *P, const double *Un, double dt, double *Unp1);

/* Steps U in place from t0 to t_end (or max_steps).  Each step takes
 * dt = min(lfo_dt(U), t_end - t); when that clamp is active the step lands
 * exactly on t_end.  dts (nullable) receives the dt of every step.  Returns
 * LFO_ERR_NONPHYSICAL if a state goes non-physical. */
int lfo_advance(const lfo_params *P, double *U, double t0, double t_end,
                int64_t max_steps, double *t_out, int64_t *steps_out,
                double *dts);

/* Compensated (Neumaier) sums of each of the 4 + ns fields times dx*dy. */
void lfo_totals(const lfo_params *P, const double *U, double *out);

/* ---- linearisation of the step at frozen dt ----------------------------- */

/* Jacobian-vector product J_R(U) dU, and vector-Jacobian product
 * J_R(U)^T g, of the residual R.  These and the tangent-linear and adjoint
 * steps below cover the Euler fields with primitive reconstruction only:
 * LFO_ERR_ARG when ns > 0 or recon != LFO_RECON_PRIMITIVE. */
int lfo_residual_jvp(const lfo_params *P, const double *U, const double *dU,
                     double *out);
int lfo_residual_vjp(const lfo_params *P, const double *U, const double *g,
                     double *out);

/* Tangent-linear and adjoint of one Heun step at frozen dt. */
int lfo_tlm_step(const lfo_params *P, const double *Un, double dt,
                 const double *dUn, double *dUnp1);
int lfo_adjoint_step(const lfo_params *P, const double *Un, double dt,
                     const double *lam_np1, double *lam_n);

/* ---- exact Riemann solution (test reference for shock tubes) ------------ */

/* Exact solution of the 1D Riemann problem for the ideal gas, sampled at
 * the self-similar coordinates xi[k] = (x - x0)/t.  Writes rho, u, p at
 * each xi and the star-region pressure and velocity.  Returns
 * LFO_ERR_VACUUM if the data generate vacuum. */
int lfo_exact_riemann(double gamma,
                      double rho_l, double u_l, double p_l,
                      double rho_r, double u_r, double p_r,
                      int64_t n, const double *xi,
                      double *rho, double *u, double *p,
                      double *p_star, double *u_star);

#ifdef __cplusplus
}
#endif
#endif /* LFO_H */
