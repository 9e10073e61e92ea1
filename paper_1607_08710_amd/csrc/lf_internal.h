// lf_internal.h -- host-side interface between the C ABI (lf_api.hip) and
// the kernel launchers (lf_forward.hip, lf_adjoint.hip).  Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "lf_device.h"

namespace lf {

// Geometry and physics of one context, plus the derived launch shape.
struct Grid {
  int nx, ny;
  double dx, dy, gamma, cfl, beta;
  int bc_x, bc_y;
  int dtype;            // 0 = double, 1 = float
  int ns;               // passive mass fractions carried after the 4 Euler fields
  int recon;            // 0: primitive reconstruction (Sec. 5), 1: conservative
  int tiles_x, tiles_y; // wave tiles of kTileW columns x rows_per_wave rows
  int rows_per_wave;
  int wpb;              // waves per stage block (a block is wpb adjacent tiles)
  int blocks_x;         // blocks per row band: ceil(tiles_x / wpb)
  int blocks, blocks_pad;
};

// Workspace layout (byte offsets from ws, all 256-byte aligned).
struct Layout {
  size_t ustar;     // predictor state U* (4 + ns planes of the context dtype)
  size_t mu;        // adjoint intermediate (4 planes)
  size_t ctl;       // Ctl
  size_t partials;  // totals: per-block (sum, compensation) pairs
  size_t total;
  int totals_blocks;
};

Grid make_grid(int nx, int ny, double dx, double dy, double gamma, double cfl, double beta,
               int bc_x, int bc_y, int dtype, int ns, int recon);
Layout make_layout(const Grid& g);


// in: stencil input; base: U^n for the corrector (may equal out); out.
// dt_dev != nullptr: read dt from the control block and honour its done flag.
// reduce: corrector only, reduce the wave speed of the output into ctl.
hipError_t launch_stage(const Grid& g, int mode, const void* in, const void* base, void* out,
                        double dt, Ctl* ctl, bool dt_dev, bool reduce, hipStream_t s);
// Ghost rows of a strip of a larger grid: kGhostRows rows below row 0
// (lo) and above row ny-1 (hi), [fields][kGhostRows][nx] each.
struct GhostRows {
  const void* lo = nullptr;
  const void* hi = nullptr;
};
// One whole Heun step in a single pass, out = step(in); in and out must
// not overlap.  ustar (nullable) receives the predictor state U*.  With
// ghost rows, rows beyond the grid's ends are read from them instead of
// following bc_y.
hipError_t launch_fused_step(const Grid& g, const void* in, void* out, void* ustar, double dt, Ctl* ctl,
                             bool dt_dev, bool reduce, hipStream_t s, GhostRows gh = GhostRows());
hipError_t launch_wavespeed(const Grid& g, const void* U, Ctl* ctl, hipStream_t s);
hipError_t launch_ctl_init(Ctl* ctl, double t0, double t_end, long long max_steps, double cfl,
                           hipStream_t s);
hipError_t launch_ctl_first(Ctl* ctl, hipStream_t s);
hipError_t launch_ctl_step(Ctl* ctl, hipStream_t s);
hipError_t launch_totals(const Grid& g, const Layout& L, const void* U, void* ws, hipStream_t s);

// Adjoint modes: out = v (kVjp); out = (g - dt v)/2 (kAdjCorr, g = lam);
// out = lam/2 + g - dt v (kAdjPred, g = mu), where v = J_R(U)^T g.
enum AdjMode : int { kVjp = 0, kAdjCorr = 1, kAdjPred = 2 };
hipError_t launch_adjoint(const Grid& g, int mode, const void* U, const void* gvec,
                          const void* lam, void* out, double dt, hipStream_t s);

}  // namespace lf
