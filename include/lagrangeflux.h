/*
 * lagrangeflux.h -- C ABI of the MI355X (gfx950) Lagrange-flux library.
 *
 * The library advances the 2D compressible Euler equations of an ideal
 * gas (Sec. 3 of De Vuyst, Gasc, Motte, Peybernes, Poncet, "Lagrange-flux
 * schemes", arXiv:1607.08710) with the second-order Lagrange-flux scheme of
 * Sec. 5: per face, MUSCL reconstruction of the primitive variables with
 * the Sweby limiter (eq. (sweby)), the Lagrangian HLL acoustic solve for
 * (u*, p*) (eqs. (13)-(14)), upwinding on the sign of u* and the flux of
 * eq. (12); per cell, the conservative update of eq. (11) inside the Heun
 * predictor-corrector of Sec. 5, with dt from a global CFL reduction.
 *
 * A state may also carry passive mass fractions y_k (the conservative
 * transport of rho y_k that the paper prefers for multimaterial flow,
 * Sec. 7): each y_k is reconstructed like the primitive variables and
 * crosses a face with the face mass flux of its upwind side, (rho_A u*)
 * y_k,A, so a uniform fraction stays uniform and every rho y_k is
 * conserved.  One gamma holds for the whole mixture.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - State arrays are DEVICE pointers owned by the caller, contiguous, in
 *    structure-of-arrays layout U[f][j][i]: f = 0..3 for (rho, rho*u, rho*v,
 *    rho*E), then f = 4..3+n_species for rho*y_k; j = 0..ny-1 the y index,
 *    i = 0..nx-1 the x index (fastest).  Element type is double (LF_F64) or
 *    float (LF_F32), per the context.  The adjoint entry points take the 4
 *    Euler fields only and require n_species == 0 and the primitive
 *    reconstruction.
 *  - ws is a DEVICE workspace of at least the size lf_init reports, owned
 *    by the caller, 256-byte aligned.  It holds the predictor state U*, the
 *    adjoint intermediate, the reduction cells and the device-side dt / t /
 *    step counters.  One workspace must not be used by two calls that run
 *    concurrently.
 *  - stream is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued on it; "async" calls return before it runs.
 *  - The library never allocates device memory and never frees caller
 *    memory.
 *  - Every call returns an lf_status.  Argument errors are detected on the
 *    host before anything is enqueued.  A context is not thread-safe;
 *    distinct contexts are independent.
 */
#ifndef LAGRANGEFLUX_H
#define LAGRANGEFLUX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lf_ctx lf_ctx; /* opaque, host memory only */

typedef enum {
    LF_OK = 0,
    LF_ERR_ARG = 1,          /* invalid argument (null, size, range, aliasing) */
    LF_ERR_HIP = 2,          /* a HIP runtime call failed                       */
    LF_ERR_NONPHYSICAL = 3,  /* a state with rho <= 0, p <= 0 or a non-finite
                                value was detected                             */
    LF_ERR_STATE = 4,        /* misuse of the context (e.g. dtype mismatch)     */
    LF_ERR_TOO_LARGE = 5     /* the grid does not fit the fixed scratch of
                                lf_adjoint_step_noalloc                        */
} lf_status;

typedef enum { LF_F64 = 0, LF_F32 = 1 } lf_dtype;

#define LF_MAX_SPECIES 4
/* Rows a strip of a larger grid needs beyond each of its ends for one
 * step (lf_step_halo): two for each of the step's two stages. */
#define LF_GHOST_ROWS 4

typedef enum { LF_RECON_PRIMITIVE = 0, LF_RECON_CONSERVATIVE = 1 } lf_recon;
typedef enum { LF_BC_PERIODIC = 0, LF_BC_TRANSMISSIVE = 1 } lf_bc;

typedef struct {
    int32_t nx, ny;   /* cells along x and y; 1 <= nx, ny; nx*ny < 2^31        */
    double dx, dy;    /* uniform cell sizes, > 0                                */
    double gamma;     /* ratio of specific heats, in (1, 3] (Sec. 3)            */
    double cfl;       /* CFL number, > 0 (Heun list, item 1)                    */
    double beta;      /* Sweby coefficient: 1 <= beta <= 2, the paper's range
                         for second order (eq. (sweby)), or 0 for the
                         first-order scheme; other values are LF_ERR_ARG    */
    int32_t bc_x;     /* lf_bc along x: periodic wraps the index, transmissive
                         clamps it (ghost cells copy the edge cell)             */
    int32_t bc_y;     /* lf_bc along y                                          */
    int32_t dtype;    /* lf_dtype of every state / adjoint array                */
    int32_t n_species; /* passive mass fractions carried after the Euler
                         fields, 0 <= n_species <= LF_MAX_SPECIES            */
    int32_t reconstruction; /* lf_recon: LF_RECON_PRIMITIVE, the paper's
                         limited reconstruction of (rho, u, v, p) (Sec. 5),
                         or LF_RECON_CONSERVATIVE, an ablation that limits
                         (rho, rho u, rho v, rho E), converts the face states
                         to primitive variables for eqs. (13)-(14) and
                         upwinds the reconstructed conservative vector; the
                         latter requires n_species == 0                     */
} lf_params;

/* Validates *params, creates a context and reports the workspace size in
 * bytes.  Makes no HIP call.  LF_ERR_ARG on a null pointer or an
 * out-of-range parameter.  The context is released by lf_destroy. */
int lf_init(const lf_params *params, lf_ctx **out, size_t *workspace_bytes);

/* Releases a context (NULL is accepted). */
void lf_destroy(lf_ctx *ctx);

/* Static English text for an lf_status value. */
const char *lf_status_string(int status);

/* CFL time step of state U (Heun list, item 1):
 *   dt = cfl / max_K [ (|u|+c)/dx + (|v|+c)/dy ],  c = sqrt(gamma p / rho),
 * reduced in FP64.  Synchronises the stream and writes *dt_out.  Returns
 * LF_ERR_NONPHYSICAL (and *dt_out = 0) if any cell has rho <= 0, p <= 0
 * or a non-finite value. */
int lf_dt(lf_ctx *ctx, const void *U, void *ws, void *stream, double *dt_out);

/* One Heun step at the caller's dt (Sec. 5, items 2-11), async:
 *   U*      = U^n - dt R(U^n)
 *   U^{n+1} = (U^n + U* - dt R(U*)) / 2,
 * algebraically the paper's U^n - dt (R(U^n) + R(U*)) / 2.  R(U) is the
 * flux balance of eq. (11).  Unp1 may equal Un (in-place update); any other
 * overlap is LF_ERR_ARG.  dt must be finite and >= 0.  In the FP32 context
 * the states are float, the flux arithmetic is float and every stage
 * update is formed in FP64 and rounded once.  With Unp1 != Un the step is
 * one single-pass kernel (U* never leaves the chip); in place, U* goes
 * through the workspace.  Either way the result is bitwise that of
 * lf_stage(1) followed by lf_stage(2). */
int lf_step(lf_ctx *ctx, const void *Un, void *Unp1, double dt, void *ws, void *stream);

/* lf_step into a separate buffer that also writes the predictor state
 * U* = U^n - dt R(U^n) of the step (items 2-6) into Ustar, async: for
 * checkpoint-and-recompute rollouts, which keep U* for
 * lf_adjoint_step_ustar instead of recomputing it there.  Unp1 is bitwise
 * that of lf_step and Ustar that of lf_stage(1).  Un, Unp1, Ustar and ws
 * must not overlap each other (LF_ERR_ARG). */
int lf_step_save(lf_ctx *ctx, const void *Un, void *Unp1, void *Ustar, double dt, void *ws,
                 void *stream);

/* One lf_step of a horizontal strip of a larger grid, async: the unit of
 * work of one GPU when the grid is split into strips of rows (Sec. 5,
 * items 2-11 on the strip).  The context describes the strip (ny = its
 * rows; bc_x applies, bc_y is not used).  The LF_GHOST_ROWS rows below
 * row 0 and above row ny-1 are read from ghost_lo and ghost_hi, each
 * [4 + n_species][LF_GHOST_ROWS][nx] in the context's dtype (ghost_lo row
 * k is strip row k - LF_GHOST_ROWS, ghost_hi row k is strip row ny + k),
 * which the caller fills from the neighbouring strips' U^n before the
 * call (across GPUs, by the halo exchange).  Every strip of a grid
 * stepped with its neighbours' rows (taken across the wrap for a periodic
 * y) gives, together, lf_step of the whole grid bit for bit.  Single
 * pass.  The inputs (Un and the ghost rows) may overlap each other; Unp1
 * and ws must not overlap any input or each other (LF_ERR_ARG). */
int lf_step_halo(lf_ctx *ctx, const void *Un, const void *ghost_lo, const void *ghost_hi,
                 void *Unp1, double dt, void *ws, void *stream);

/* One stage of the Heun step at the caller's dt, async (the two kernels
 * lf_step chains, exposed for callers that schedule stages themselves):
 *   stage 1 (predictor, items 2-6):  out = in - dt R(in)
 *   stage 2 (corrector, items 7-11): out = (base + in - dt R(in)) / 2
 * base is read for stage 2 only and may equal out; in must not overlap out.
 * With reduce != 0, stage 2 also reduces the CFL wave speed of out into
 * the workspace (as lf_advance does); the result is not returned. */
int lf_stage(lf_ctx *ctx, int stage, const void *in, const void *base, void *out, double dt,
             int reduce, void *ws, void *stream);

/* Advances U in place from t0 until t_end or max_steps steps, each step
 * with dt = min(CFL dt of the current state, t_end - t); the step that is
 * clamped lands exactly on t_end.  dt and t stay on the device; the host
 * synchronises once per batch of steps.  Writes the final time, the step
 * count, and (if dts_out != NULL) the dt of the first min(steps,
 * dts_capacity) steps into the host array dts_out.  Returns
 * LF_ERR_NONPHYSICAL if the initial state or any state produced is
 * non-physical (the state of that step is left in U).  Every step, with
 * or without mass fractions, is the single-pass kernel of lf_step,
 * alternating between U and the workspace's U* buffer; an odd step count
 * ends with one device copy back into U. */
int lf_advance(lf_ctx *ctx, void *U, double t0, double t_end, int64_t max_steps,
               void *ws, void *stream, double *t_out, int64_t *steps_out,
               double *dts_out, int64_t dts_capacity);

/* Residual R(U) of eq. (11), (F_{i+1/2} - F_{i-1/2})/dx + (G_{j+1/2} -
 * G_{j-1/2})/dy, written to R (same layout and dtype as U), async.  R must
 * not overlap U. */
int lf_residual(lf_ctx *ctx, const void *U, void *R, void *ws, void *stream);

/* Vector-Jacobian product out = J_R(U)^T g of the residual, async
 * (contexts without mass fractions and with the primitive reconstruction;
 * LF_ERR_ARG otherwise).  The
 * derivative conventions at the non-differentiable points are: limiter
 * derivative zero when ab <= 0, min follows its first argument on ties,
 * max(m1, m2) follows m1 on ties, max(c_L, c_R) follows c_L on ties, the
 * upwind side is left iff u* > 0.  out must not overlap U or g. */
int lf_residual_vjp(lf_ctx *ctx, const void *U, const void *g, void *out, void *ws,
                    void *stream);

/* Adjoint of one lf_step at the frozen dt, async (contexts without mass
 * fractions and with the primitive reconstruction; LF_ERR_ARG otherwise):
 * given lam_np1 =
 * dJ/dU^{n+1}, writes lam_n = dJ/dU^n, recomputing U* from Un:
 *   mu    = (lam_np1 - dt J_R(U*)^T lam_np1) / 2
 *   lam_n = lam_np1 / 2 + mu - dt J_R(U^n)^T mu.
 * lam_n must not overlap Un or lam_np1. */
int lf_adjoint_step(lf_ctx *ctx, const void *Un, double dt, const void *lam_np1,
                    void *lam_n, void *ws, void *stream);

/* lf_adjoint_step with the step's predictor state U* supplied by the
 * caller (as lf_step_save wrote it) instead of recomputed: the same two
 * adjoint stages, bitwise the same result, one predictor pass less.  Same
 * context restrictions; lam_n must not overlap Un, Ustar or lam_np1. */
int lf_adjoint_step_ustar(lf_ctx *ctx, const void *Un, const void *Ustar, double dt,
                          const void *lam_np1, void *lam_n, void *ws, void *stream);

/* Bytes of the library's fixed device scratch used by
 * lf_adjoint_step_noalloc (64 MiB; one copy per GPU the library runs on,
 * held until the process ends). */
#define LF_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* lf_adjoint_step for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments without the workspace, same kernels, bitwise
 * the same lam_n as lf_adjoint_step, async.  U* and mu live in a scratch
 * array of LF_NOALLOC_SCRATCH_BYTES that the library holds in device
 * memory (a static device array, not an allocation): nothing is allocated
 * or freed by the call.  Limit: U* and mu (4 planes each, 256-byte
 * aligned) must fit the scratch, i.e. nx*ny <= 1048576 cells in FP64 and
 * <= 2097152 in FP32; larger grids return LF_ERR_TOO_LARGE before any HIP
 * call.  Same context restrictions as lf_adjoint_step (LF_ERR_ARG);
 * lam_n must not overlap Un or lam_np1.  stream must belong to the
 * current device (LF_ERR_ARG otherwise).  The first call on a device
 * resolves the scratch's device address (hipGetSymbolAddress), which may
 * load the library's device code there: make that first call outside
 * stream capture.  All calls on one GPU share its scratch, which keeps
 * the last call's contents (each call writes U* and mu in full before it
 * reads them, so nothing needs clearing): calls that may overlap in time
 * on one GPU -- on different streams, from different threads or contexts
 * -- race and give undefined results; order them, e.g. on one stream. */
int lf_adjoint_step_noalloc(lf_ctx *ctx, const void *Un, double dt, const void *lam_np1,
                            void *lam_n, void *stream);

/* Conservation totals: out[f] = dx*dy * sum_K U_f(K) for the 4 + n_species
 * fields (out has that many entries), summed in FP64 with compensation in
 * a fixed order (deterministic).  Synchronises. */
int lf_totals(lf_ctx *ctx, const void *U, void *ws, void *stream, double *out);

#ifdef __cplusplus
}
#endif
#endif /* LAGRANGEFLUX_H */
