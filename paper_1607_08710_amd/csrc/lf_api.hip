// lf_api.hip -- the C ABI declared in include/lagrangeflux.h.
//
// Host-side argument validation, workspace layout and launch sequencing.
// The library owns no device memory: states, adjoint vectors and the
// workspace are caller pointers.  Validation happens before any HIP call.
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <mutex>
#include <new>

#include "lagrangeflux.h"
#include "lf_internal.h"

static_assert(LF_MAX_SPECIES == lf::kMaxSpecies, "species cap of the ABI and the kernels");
static_assert(LF_GHOST_ROWS == lf::kGhostRows, "ghost rows of a strip");

struct lf_ctx {
  lf::Grid g;
  lf::Layout L;
  size_t state_bytes;
};

namespace {

bool params_ok(const lf_params* p) {
  if (!p) return false;
  if (p->nx < 1 || p->ny < 1) return false;
  if ((long long)p->nx * (long long)p->ny >= (1LL << 31)) return false;
  if (!(p->dx > 0.0) || !(p->dy > 0.0) || !isfinite(p->dx) || !isfinite(p->dy)) return false;
  if (!(p->gamma > 1.0 && p->gamma <= 3.0)) return false;
  if (!(p->beta == 0.0 || (p->beta >= 1.0 && p->beta <= 2.0))) return false;
  if (!(p->cfl > 0.0) || !isfinite(p->cfl)) return false;
  if (p->bc_x != LF_BC_PERIODIC && p->bc_x != LF_BC_TRANSMISSIVE) return false;
  if (p->bc_y != LF_BC_PERIODIC && p->bc_y != LF_BC_TRANSMISSIVE) return false;
  if (p->dtype != LF_F64 && p->dtype != LF_F32) return false;
  if (p->n_species < 0 || p->n_species > LF_MAX_SPECIES) return false;
  if (p->reconstruction != LF_RECON_PRIMITIVE && p->reconstruction != LF_RECON_CONSERVATIVE) return false;
  if (p->reconstruction == LF_RECON_CONSERVATIVE && p->n_species != 0) return false;
  return true;
}

// Do the byte ranges [a, a+na) and [b, b+nb) intersect?
bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + nb && y < x + na;
}

int hip_status(hipError_t e) { return e == hipSuccess ? LF_OK : LF_ERR_HIP; }

lf::Ctl* ctl_of(const lf_ctx* c, void* ws) {
  return reinterpret_cast<lf::Ctl*>(static_cast<char*>(ws) + c->L.ctl);
}
void* ustar_of(const lf_ctx* c, void* ws) { return static_cast<char*>(ws) + c->L.ustar; }
void* mu_of(const lf_ctx* c, void* ws) { return static_cast<char*>(ws) + c->L.mu; }

constexpr size_t kCtlHeader = offsetof(lf::Ctl, dt_hist);

// ---- scratch of lf_adjoint_step_noalloc ------------------------------------
//
// The predictor state U* and the adjoint intermediate mu of that entry point
// live in this array instead of a caller workspace.  Every GPU the library
// runs on holds its own copy from the module's load until the process ends.
// In host code the name stands for a host-side handle, not a device
// address: its address on a device comes from hipGetSymbolAddress (with
// that device current), once per device, and only that address is passed
// to kernels.
constexpr size_t kNoAllocScratch = LF_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratch];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices];  // device address of scratch, per device

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

// Device address of scratch on device dev (resolved on first use, with dev
// current).
int scratch_on(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return LF_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LF_ERR_HIP;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return LF_OK;
}

int read_ctl(lf::Ctl* dev, lf::Ctl* host, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(host, dev, kCtlHeader, hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return LF_ERR_HIP;
  return hip_status(hipStreamSynchronize(s));
}

}  // namespace

extern "C" {

int lf_init(const lf_params* params, lf_ctx** out, size_t* workspace_bytes) {
  if (!out || !workspace_bytes || !params_ok(params)) return LF_ERR_ARG;
  lf_ctx* c = new (std::nothrow) lf_ctx;
  if (!c) return LF_ERR_ARG;
  c->g = lf::make_grid(params->nx, params->ny, params->dx, params->dy, params->gamma, params->cfl,
                       params->beta, params->bc_x, params->bc_y, params->dtype, params->n_species,
                       params->reconstruction);
  c->L = lf::make_layout(c->g);
  c->state_bytes = (size_t)(4 + params->n_species) * (size_t)params->nx * (size_t)params->ny *
                   (params->dtype == LF_F64 ? sizeof(double) : sizeof(float));
  *out = c;
  *workspace_bytes = c->L.total;
  return LF_OK;
}

void lf_destroy(lf_ctx* ctx) { delete ctx; }

const char* lf_status_string(int status) {
  switch (status) {
    case LF_OK: return "ok";
    case LF_ERR_ARG: return "invalid argument";
    case LF_ERR_HIP: return "HIP runtime error";
    case LF_ERR_NONPHYSICAL: return "non-physical state (rho <= 0, p <= 0 or non-finite)";
    case LF_ERR_STATE: return "invalid context state";
    case LF_ERR_TOO_LARGE: return "grid too large for the no-allocation scratch (LF_NOALLOC_SCRATCH_BYTES)";
    default: return "unknown status";
  }
}

int lf_dt(lf_ctx* ctx, const void* U, void* ws, void* stream, double* dt_out) {
  if (!ctx || !U || !ws || !dt_out) return LF_ERR_ARG;
  if (overlap(U, ctx->state_bytes, ws, ctx->L.total)) return LF_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  lf::Ctl* ctl = ctl_of(ctx, ws);
  hipError_t e = lf::launch_ctl_init(ctl, 0.0, INFINITY, 1, ctx->g.cfl, s);
  if (e == hipSuccess) e = lf::launch_wavespeed(ctx->g, U, ctl, s);
  if (e == hipSuccess) e = lf::launch_ctl_first(ctl, s);
  if (e != hipSuccess) return LF_ERR_HIP;
  lf::Ctl h;
  int rc = read_ctl(ctl, &h, s);
  if (rc != LF_OK) return rc;
  if (h.flag) {
    *dt_out = 0.0;
    return LF_ERR_NONPHYSICAL;
  }
  *dt_out = h.dt;
  return LF_OK;
}

int lf_step(lf_ctx* ctx, const void* Un, void* Unp1, double dt, void* ws, void* stream) {
  if (!ctx || !Un || !Unp1 || !ws) return LF_ERR_ARG;
  if (!(dt >= 0.0) || !isfinite(dt)) return LF_ERR_ARG;
  const size_t n = ctx->state_bytes;
  if (Un != Unp1 && overlap(Un, n, Unp1, n)) return LF_ERR_ARG;
  if (overlap(Un, n, ws, ctx->L.total) || overlap(Unp1, n, ws, ctx->L.total)) return LF_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // single pass when the output is a separate buffer; in place the two
  // stages, through U* in the workspace
  if (Un != Unp1)
    return hip_status(lf::launch_fused_step(ctx->g, Un, Unp1, nullptr, dt, nullptr, false, false, s));
  void* us = ustar_of(ctx, ws);
  hipError_t e = lf::launch_stage(ctx->g, lf::kPredictor, Un, nullptr, us, dt, nullptr, false, false, s);
  if (e == hipSuccess)
    e = lf::launch_stage(ctx->g, lf::kCorrector, us, Un, Unp1, dt, nullptr, false, false, s);
  return hip_status(e);
}

int lf_step_save(lf_ctx* ctx, const void* Un, void* Unp1, void* Ustar, double dt, void* ws, void* stream) {
  if (!ctx || !Un || !Unp1 || !Ustar || !ws) return LF_ERR_ARG;
  if (!(dt >= 0.0) || !isfinite(dt)) return LF_ERR_ARG;
  const size_t n = ctx->state_bytes, w = ctx->L.total;
  if (overlap(Un, n, Unp1, n) || overlap(Un, n, Ustar, n) || overlap(Unp1, n, Ustar, n)) return LF_ERR_ARG;
  if (overlap(Un, n, ws, w) || overlap(Unp1, n, ws, w) || overlap(Ustar, n, ws, w)) return LF_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return hip_status(lf::launch_fused_step(ctx->g, Un, Unp1, Ustar, dt, nullptr, false, false, s));
}

int lf_step_halo(lf_ctx* ctx, const void* Un, const void* ghost_lo, const void* ghost_hi, void* Unp1, double dt,
                 void* ws, void* stream) {
  if (!ctx || !Un || !ghost_lo || !ghost_hi || !Unp1 || !ws) return LF_ERR_ARG;
  if (!(dt >= 0.0) || !isfinite(dt)) return LF_ERR_ARG;
  const size_t n = ctx->state_bytes, w = ctx->L.total;
  const size_t gb = ctx->state_bytes / (size_t)ctx->g.ny * LF_GHOST_ROWS;  // [fields][4][nx]
  if (overlap(Unp1, n, Un, n) || overlap(Unp1, n, ghost_lo, gb) || overlap(Unp1, n, ghost_hi, gb) ||
      overlap(Unp1, n, ws, w))
    return LF_ERR_ARG;
  if (overlap(Un, n, ws, w) || overlap(ghost_lo, gb, ws, w) || overlap(ghost_hi, gb, ws, w)) return LF_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  lf::GhostRows gh;
  gh.lo = ghost_lo;
  gh.hi = ghost_hi;
  return hip_status(lf::launch_fused_step(ctx->g, Un, Unp1, nullptr, dt, nullptr, false, false, s, gh));
}

int lf_stage(lf_ctx* ctx, int stage, const void* in, const void* base, void* out, double dt, int reduce,
             void* ws, void* stream) {
  if (!ctx || !in || !out || !ws || (stage != 1 && stage != 2)) return LF_ERR_ARG;
  if (stage == 2 && !base) return LF_ERR_ARG;
  if (!(dt >= 0.0) || !isfinite(dt)) return LF_ERR_ARG;
  const size_t n = ctx->state_bytes, w = ctx->L.total;
  if (overlap(in, n, out, n) || overlap(in, n, ws, w) || overlap(out, n, ws, w)) return LF_ERR_ARG;
  if (stage == 2 && base != out && (overlap(base, n, out, n) || overlap(base, n, ws, w))) return LF_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  lf::Ctl* ctl = ctl_of(ctx, ws);
  const bool red = stage == 2 && reduce != 0;
  return hip_status(lf::launch_stage(ctx->g, stage == 1 ? lf::kPredictor : lf::kCorrector, in,
                                     stage == 2 ? base : nullptr, out, dt, red ? ctl : nullptr, false, red, s));
}

int lf_advance(lf_ctx* ctx, void* U, double t0, double t_end, int64_t max_steps, void* ws, void* stream,
               double* t_out, int64_t* steps_out, double* dts_out, int64_t dts_capacity) {
  if (!ctx || !U || !ws || !t_out || !steps_out) return LF_ERR_ARG;
  if (!isfinite(t0) || isnan(t_end) || max_steps < 0 || dts_capacity < 0) return LF_ERR_ARG;
  if (dts_out == nullptr && dts_capacity != 0) return LF_ERR_ARG;
  if (overlap(U, ctx->state_bytes, ws, ctx->L.total)) return LF_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  lf::Ctl* ctl = ctl_of(ctx, ws);
  void* us = ustar_of(ctx, ws);

  hipError_t e = lf::launch_ctl_init(ctl, t0, t_end, (long long)max_steps, ctx->g.cfl, s);
  if (e == hipSuccess) e = lf::launch_wavespeed(ctx->g, U, ctl, s);
  if (e == hipSuccess) e = lf::launch_ctl_first(ctl, s);
  if (e != hipSuccess) return LF_ERR_HIP;
  lf::Ctl h;
  int rc = read_ctl(ctl, &h, s);
  if (rc != LF_OK) return rc;

  // Each step is one single-pass launch that alternates between U and the
  // U* buffer of the workspace (launch j reads buffer j % 2); launches after
  // the device marks the loop done return at once, so the result is in
  // buffer (steps % 2) and is copied back to U at the end when that is the
  // workspace.
  void* buf[2] = {U, us};
  long long launched = 0;
  long long done_steps = 0;
  while (!h.done) {
    // Size the next batch from the current dt; steps launched after the
    // device marks the loop done return at once.
    double est = (h.dt > 0.0) ? (h.t_end - h.t) / h.dt : 1.0;
    long long batch = isfinite(est) ? (long long)(est * 1.05) + 2 : (long long)lf::kDtHist;
    if (batch > lf::kDtHist) batch = lf::kDtHist;
    if (batch > (long long)max_steps - done_steps) batch = (long long)max_steps - done_steps;
    if (batch < 1) batch = 1;
    for (long long k = 0; k < batch && e == hipSuccess; ++k) {
      e = lf::launch_fused_step(ctx->g, buf[launched & 1], buf[(launched + 1) & 1], nullptr, 0.0, ctl, true,
                                true, s);
      ++launched;
      if (e == hipSuccess) e = lf::launch_ctl_step(ctl, s);
    }
    if (e != hipSuccess) return LF_ERR_HIP;
    rc = read_ctl(ctl, &h, s);
    if (rc != LF_OK) return rc;
    // copy the dt records of the steps completed in this batch (the batch
    // never exceeds the ring, so its records form at most two runs)
    if (dts_out) {
      long long k0 = done_steps, k1 = h.step < dts_capacity ? h.step : dts_capacity;
      while (k0 < k1) {
        const long long slot = k0 % lf::kDtHist;
        long long run = lf::kDtHist - slot;
        if (run > k1 - k0) run = k1 - k0;
        e = hipMemcpyAsync(dts_out + k0, &ctl->dt_hist[slot], (size_t)run * sizeof(double),
                           hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return LF_ERR_HIP;
        k0 += run;
      }
      e = hipStreamSynchronize(s);
      if (e != hipSuccess) return LF_ERR_HIP;
    }
    done_steps = h.step;
  }
  if (h.step & 1) {
    e = hipMemcpyAsync(U, us, ctx->state_bytes, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return LF_ERR_HIP;
  }
  *t_out = h.t;
  *steps_out = h.step;
  return h.flag ? LF_ERR_NONPHYSICAL : LF_OK;
}

int lf_residual(lf_ctx* ctx, const void* U, void* R, void* ws, void* stream) {
  if (!ctx || !U || !R || !ws) return LF_ERR_ARG;
  const size_t n = ctx->state_bytes;
  if (overlap(U, n, R, n) || overlap(R, n, ws, ctx->L.total)) return LF_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return hip_status(lf::launch_stage(ctx->g, lf::kResidual, U, nullptr, R, 0.0, nullptr, false, false, s));
}

int lf_residual_vjp(lf_ctx* ctx, const void* U, const void* g, void* out, void* ws, void* stream) {
  if (!ctx || !U || !g || !out || !ws || ctx->g.ns != 0 || ctx->g.recon != 0) return LF_ERR_ARG;
  const size_t n = ctx->state_bytes;
  if (overlap(out, n, U, n) || overlap(out, n, g, n) || overlap(out, n, ws, ctx->L.total))
    return LF_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return hip_status(lf::launch_adjoint(ctx->g, lf::kVjp, U, g, nullptr, out, 0.0, s));
}

int lf_adjoint_step(lf_ctx* ctx, const void* Un, double dt, const void* lam_np1, void* lam_n, void* ws,
                    void* stream) {
  if (!ctx || !Un || !lam_np1 || !lam_n || !ws || ctx->g.ns != 0 || ctx->g.recon != 0) return LF_ERR_ARG;
  if (!(dt >= 0.0) || !isfinite(dt)) return LF_ERR_ARG;
  const size_t n = ctx->state_bytes, w = ctx->L.total;
  if (overlap(lam_n, n, Un, n) || overlap(lam_n, n, lam_np1, n)) return LF_ERR_ARG;
  if (overlap(Un, n, ws, w) || overlap(lam_np1, n, ws, w) || overlap(lam_n, n, ws, w)) return LF_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  void* us = ustar_of(ctx, ws);
  void* mu = mu_of(ctx, ws);
  hipError_t e = lf::launch_stage(ctx->g, lf::kPredictor, Un, nullptr, us, dt, nullptr, false, false, s);
  if (e == hipSuccess) e = lf::launch_adjoint(ctx->g, lf::kAdjCorr, us, lam_np1, nullptr, mu, dt, s);
  if (e == hipSuccess) e = lf::launch_adjoint(ctx->g, lf::kAdjPred, Un, mu, lam_np1, lam_n, dt, s);
  return hip_status(e);
}

int lf_adjoint_step_ustar(lf_ctx* ctx, const void* Un, const void* Ustar, double dt, const void* lam_np1,
                          void* lam_n, void* ws, void* stream) {
  if (!ctx || !Un || !Ustar || !lam_np1 || !lam_n || !ws || ctx->g.ns != 0 || ctx->g.recon != 0) return LF_ERR_ARG;
  if (!(dt >= 0.0) || !isfinite(dt)) return LF_ERR_ARG;
  const size_t n = ctx->state_bytes, w = ctx->L.total;
  if (overlap(lam_n, n, Un, n) || overlap(lam_n, n, lam_np1, n) || overlap(lam_n, n, Ustar, n)) return LF_ERR_ARG;
  if (overlap(Un, n, ws, w) || overlap(Ustar, n, ws, w) || overlap(lam_np1, n, ws, w) || overlap(lam_n, n, ws, w))
    return LF_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  void* mu = mu_of(ctx, ws);
  hipError_t e = lf::launch_adjoint(ctx->g, lf::kAdjCorr, Ustar, lam_np1, nullptr, mu, dt, s);
  if (e == hipSuccess) e = lf::launch_adjoint(ctx->g, lf::kAdjPred, Un, mu, lam_np1, lam_n, dt, s);
  return hip_status(e);
}

int lf_adjoint_step_noalloc(lf_ctx* ctx, const void* Un, double dt, const void* lam_np1, void* lam_n,
                            void* stream) {
  if (!ctx || !Un || !lam_np1 || !lam_n || ctx->g.ns != 0 || ctx->g.recon != 0) return LF_ERR_ARG;
  if (!(dt >= 0.0) || !isfinite(dt)) return LF_ERR_ARG;
  const size_t n = ctx->state_bytes;
  if (overlap(lam_n, n, Un, n) || overlap(lam_n, n, lam_np1, n)) return LF_ERR_ARG;
  // U* and mu, each 256-byte aligned, must fit the scratch
  const size_t half = align256(n);
  if (2 * half > kNoAllocScratch) return LF_ERR_TOO_LARGE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the scratch of the device the stream belongs to, which must be the
  // current device (the address is resolved with it current)
  int cur = 0;
  hipDevice_t sdev = 0;
  if (hipGetDevice(&cur) != hipSuccess || hipStreamGetDevice(s, &sdev) != hipSuccess) return LF_ERR_HIP;
  if (sdev != cur) return LF_ERR_ARG;
  void* base = nullptr;
  const int rc = scratch_on(cur, &base);
  if (rc != LF_OK) return rc;
  if (overlap(Un, n, base, kNoAllocScratch) || overlap(lam_np1, n, base, kNoAllocScratch) ||
      overlap(lam_n, n, base, kNoAllocScratch))
    return LF_ERR_ARG;
  void* us = base;
  void* mu = static_cast<char*>(base) + half;
  // U* and mu are written in full before they are read: nothing in the
  // scratch needs clearing between calls
  hipError_t e = lf::launch_stage(ctx->g, lf::kPredictor, Un, nullptr, us, dt, nullptr, false, false, s);
  if (e == hipSuccess) e = lf::launch_adjoint(ctx->g, lf::kAdjCorr, us, lam_np1, nullptr, mu, dt, s);
  if (e == hipSuccess) e = lf::launch_adjoint(ctx->g, lf::kAdjPred, Un, mu, lam_np1, lam_n, dt, s);
  return hip_status(e);
}

int lf_totals(lf_ctx* ctx, const void* U, void* ws, void* stream, double* out) {
  if (!ctx || !U || !ws || !out) return LF_ERR_ARG;
  if (overlap(U, ctx->state_bytes, ws, ctx->L.total)) return LF_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  lf::Ctl* ctl = ctl_of(ctx, ws);
  hipError_t e = lf::launch_totals(ctx->g, ctx->L, U, ws, s);
  if (e != hipSuccess) return LF_ERR_HIP;
  e = hipMemcpyAsync(out, ctl->totals, (size_t)(4 + ctx->g.ns) * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return LF_ERR_HIP;
  return hip_status(hipStreamSynchronize(s));
}

}  // extern "C"
