// lf_fused.hip -- one whole Heun step (Sec. 5, items 2-11) in a single pass
// over the state, for states without mass fractions.
//
// The two-stage path writes the predictor state U* to memory and reads it
// back (160 B per FP64 cell and step).  Here a wave runs both stages on the
// same strip: the predictor works two rows ahead of the corrector, U* never
// leaves the chip, and only U^n is read and U^{n+1} written (64 B per cell
// plus the halos).  The arithmetic is that of the stage kernels, term for
// term, so U^{n+1} is bitwise the two-stage result.
//
// Layout.  A wave owns 64 consecutive columns and produces the middle 56:
// the corrector reads U* two lanes to each side of its outputs, and U* is
// valid two lanes inside the loaded U^n.  The wave marches up a strip of
// rows: each row it takes U^n row o+4, the predictor produces U* row o+2,
// and the corrector finishes row o.  Waves are independent (no block
// barrier); a block is WPB adjacent waves only for the tile numbering.
//
// Boundaries.  Periodic: stencil rows and columns wrap, and U* of a wrapped
// row or column is computed from the wrapped data (what the two-stage path
// would read).  Transmissive: the corrector sees ghost rows and columns of
// U* as copies of the edge row or column, as the two-stage path does when
// it reads U* with clamped indices; the predictor never computes ghost rows,
// and a ghost lane reads U* from the lane of the edge column.
#include <stdlib.h>

#include "lf_internal.h"

namespace lf {

constexpr int kFHalo = 4;
constexpr int kFTileW = kWave - 2 * kFHalo;  // 56 output columns per wave

template <typename T>
struct FusedArgs {
  const T* in;  // U^n
  T* out;       // U^{n+1}, must not overlap in
  Ctl* ctl;
  int nx, ny, rows;
  int blocks_x, blocks, blocks_pad;
  long long plane;
  T gamma, gm1, inv_gm1, beta, idx, idy, kxy;
  double dt;
  int dt_dev, reduce;
};

// y-window of one stage: primitive rows a and a+1, the y-slope of row a and
// the flux through face a-1/2.
template <typename T>
struct Win {
  Prim<T> w0, w1, s0;
  Flux<T> g;
};

// Window of row a from the primitive rows a-2 .. a+1.
template <bool CONS, typename T>
__device__ __forceinline__ Win<T> prime_window(const Prim<T>& wa, const Prim<T>& wb, const Prim<T>& w0,
                                               const Prim<T>& w1, T beta, T gam, T gm1, T igm1) {
  Win<T> W;
  const Prim<T> d_mid = sub(w0, wb);
  const Prim<T> s_b = slope(sub(wb, wa), d_mid, beta);
  W.s0 = slope(d_mid, sub(w1, w0), beta);
  W.g = face_flux(face_prim<CONS>(face_plus<T, true>(wb, s_b), gm1),
                  face_prim<CONS>(face_minus<T, true>(w0, W.s0), gm1), gam, igm1);
  W.w0 = w0;
  W.w1 = w1;
  return W;
}

// Residual of eq. (11) for row a of the window (every lane; valid two lanes
// inside the valid input), given primitive row a+2; slides the window by a
// row.  Same arithmetic, in the same order, as the stage kernel's row.
template <bool CONS, typename T>
__device__ __forceinline__ void window_row(Win<T>& W, const Prim<T>& wn, T beta, T gam, T gm1, T igm1, T kxy,
                                           T idx, T (&r)[4]) {
  const Prim<T> s1 = slope(sub(W.w1, W.w0), sub(wn, W.w1), beta);
  const Flux<T> G = face_flux(face_prim<CONS>(face_plus<T, true>(W.w0, W.s0), gm1),
                              face_prim<CONS>(face_minus<T, true>(W.w1, s1), gm1), gam, igm1);
  const Prim<T> wr1 = shl1(W.w0);
  const Prim<T> dxp = sub(wr1, W.w0);
  const Prim<T> dxm = shr1(dxp);
  const Prim<T> sx = slope(dxm, dxp, beta);
  const Prim<T> sx1 = shl1(sx);
  const Flux<T> F = face_flux(face_prim<CONS>(face_plus<T, false>(W.w0, sx), gm1),
                              face_prim<CONS>(face_minus<T, false>(wr1, sx1), gm1), gam, igm1);
  const Flux<T> Fm = shr1(F);
  r[0] = fma(G.f0 - W.g.f0, kxy, F.f0 - Fm.f0) * idx;
  r[1] = fma(G.f2 - W.g.f2, kxy, F.f1 - Fm.f1) * idx;
  r[2] = fma(G.f1 - W.g.f1, kxy, F.f2 - Fm.f2) * idx;
  r[3] = fma(G.f3 - W.g.f3, kxy, F.f3 - Fm.f3) * idx;
  W.w0 = W.w1;
  W.w1 = wn;
  W.s0 = s1;
  W.g = G;
}

// The kernel is bound by arithmetic, not by memory (it moves 64 B per FP64
// cell and step), so its LDS footprint is kept small for occupancy: U^n of
// the rows still to be combined waits in a per-wave LDS ring, U* of the two
// rows waiting for the corrector's combination stays in registers, and one
// LDS row of U* serves the reads across lanes.  Results are stored straight
// from the lanes (no staging, no block barrier).
template <typename T, int BCX, int BCY, bool CONS>
__global__ __launch_bounds__(kWave * waves_per_block<T>())
void fused_step_kernel(FusedArgs<T> a) {
  constexpr int WPB = waves_per_block<T>();
  constexpr bool XT = BCX == kBcTransmissive;
  constexpr bool YT = BCY == kBcTransmissive;
  if (a.dt_dev && a.ctl->done) return;
  const int lb = xcd_block(blockIdx.x, a.blocks_pad);
  if (lb >= a.blocks) return;  // whole block
  const int by = lb / a.blocks_x;
  const int bx = lb - by * a.blocks_x;
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & (kWave - 1);
  const int nx = a.nx, ny = a.ny;
  const int c = (bx * WPB + w) * kFTileW - kFHalo + lane;  // unwrapped column of this lane
  const int cm = map_index<BCX>(c, nx);
  // transmissive: a ghost lane reads U* of the edge column, held by the lane
  // lane + (cm - c) of the same wave (columns 0 and nx-1 are output columns
  // of the wave whose halo holds their ghosts); clamped to the wave for the
  // waves of the last block that lie wholly past the edge and store nothing
  const int src = XT ? min(max(lane + (cm - c), 0), kWave - 1) : lane;
  const bool out_lane = lane >= kFHalo && lane < kWave - kFHalo && c < nx;
  const int y0 = by * a.rows;
  const int y1 = min(y0 + a.rows, ny);
  const long long P = a.plane;
  const double dt = a.dt_dev ? a.ctl->dt : a.dt;
  const T gm1 = a.gm1, gam = a.gamma, igm1 = a.inv_gm1, beta = a.beta, kxy = a.kxy, idx = a.idx;

  const T* __restrict__ I0 = a.in;
  auto load_row = [&](int row, T (&q)[4]) {
    const int off = map_index<BCY>(row, ny) * nx + cm;
    q[0] = I0[off];
    q[1] = I0[P + off];
    q[2] = I0[2 * P + off];
    q[3] = I0[3 * P + off];
  };

  // U^n ring (rows o .. o+4 are alive while row o is finished) and the
  // U* row exchanged across lanes.
  __shared__ T nring[WPB][5][4][kWave];
  __shared__ T srow[WPB][4][kWave];
  T(*my_n)[4][kWave] = nring[w];
  T(*my_s)[kWave] = srow[w];
  auto nslot = [](int r) { return (r % 5 + 5) % 5; };
  auto put_n = [&](int r, const T (&q)[4]) {
    const int sl = nslot(r);
    my_n[sl][0][lane] = q[0];
    my_n[sl][1][lane] = q[1];
    my_n[sl][2][lane] = q[2];
    my_n[sl][3][lane] = q[3];
  };
  // U* row r as the corrector sees it: transmissive ghost rows are the edge
  // row
  auto rmap = [&](int r) { return YT ? min(max(r, 0), ny - 1) : r; };

  // Rows of U* the corrector needs: y0-2 .. y1+1; the predictor produces
  // the ones that are not transmissive ghosts.
  const int plo = YT ? max(y0 - 2, 0) : y0 - 2;
  const int phi = YT ? min(y1 + 1, ny - 1) : y1 + 1;
  const int nlast = phi + 2;  // last U^n row the predictor reads

  // ---- predictor: window of row plo, U^n rows plo+2 and plo+3 in flight ----
  T QA[4], QB[4] = {T(0), T(0), T(0), T(0)};
  Win<T> PW;
  {
    T qa[4], qb[4], q0[4], q1[4];
    load_row(plo - 2, qa);
    load_row(plo - 1, qb);
    load_row(plo, q0);
    load_row(plo + 1, q1);
    load_row(plo + 2, QA);
    if (plo + 3 <= nlast) load_row(plo + 3, QB);
    put_n(plo, q0);
    put_n(plo + 1, q1);
    PW = prime_window<CONS>(rec_vars<CONS>(qa[0], qa[1], qa[2], qa[3], gm1),
                            rec_vars<CONS>(qb[0], qb[1], qb[2], qb[3], gm1),
                            rec_vars<CONS>(q0[0], q0[1], q0[2], q0[3], gm1),
                            rec_vars<CONS>(q1[0], q1[1], q1[2], q1[3], gm1), beta, gam, gm1, igm1);
  }
  int pr = plo;  // next U* row to produce
  // U* of the last two rows produced (conservative, this lane's column):
  // S1 = row pr-1, S0 = row pr-2
  T S0[4] = {T(0), T(0), T(0), T(0)}, S1[4] = {T(0), T(0), T(0), T(0)};
  // U* row pr = U^n - dt R(U^n); it goes to S1 (S1 moves to S0) and to the
  // LDS row read across lanes
  auto produce = [&]() {
    const Prim<T> wn = rec_vars<CONS>(QA[0], QA[1], QA[2], QA[3], gm1);  // U^n row pr+2
    put_n(pr + 2, QA);
#pragma unroll
    for (int f = 0; f < 4; ++f) QA[f] = QB[f];
    if (pr + 4 <= nlast) load_row(pr + 4, QB);
    T res[4];
    window_row<CONS>(PW, wn, beta, gam, gm1, igm1, kxy, idx, res);
    const int sn = nslot(pr);
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      S0[f] = S1[f];
      S1[f] = combine<kPredictor>(my_n[sn][f][lane], T(0), res[f], dt);
      my_s[f][lane] = S1[f];
    }
    ++pr;
  };
  // primitive U* of the newest row produced, at this lane's column (ghost
  // lanes: the edge column)
  auto star_prim = [&]() {
    __builtin_amdgcn_wave_barrier();
    return rec_vars<CONS>(my_s[0][src], my_s[1][src], my_s[2][src], my_s[3][src], gm1);
  };

  // ---- corrector: window of row y0 from U* rows y0-2 .. y0+1 ----
  // Each needed row is read as soon as it is the newest one produced
  // (transmissive ghost rows reuse the edge row).
  Prim<T> cw[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = rmap(y0 - 2 + k);
    while (pr <= r) produce();
    cw[k] = star_prim();
  }
  Win<T> CW = prime_window<CONS>(cw[0], cw[1], cw[2], cw[3], beta, gam, gm1, igm1);
  // U* (conservative) of the rows the corrector combines next: row o in C0,
  // row o+1 in C1
  T C0[4], C1[4];
  {
    // rows y0 and y0+1 were the last ones produced, unless the strip ends
    // at a transmissive top (then row y0 is the newest: y0 == ny - 1)
    const bool two = pr - 1 >= y0 + 1;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      C0[f] = two ? S0[f] : S1[f];
      C1[f] = S1[f];
    }
  }

  double smax = 0.0;
  bool bad = false;

#pragma unroll 1
  for (int o = y0; o < y1; ++o) {
    const bool fresh = o + 2 <= phi;
    if (fresh) produce();
    const Prim<T> wn = star_prim();  // U* row rmap(o+2), the newest produced
    T res[4];
    window_row<CONS>(CW, wn, beta, gam, gm1, igm1, kxy, idx, res);
    const int sn = nslot(o);
    T u[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) u[f] = combine<kCorrector>(C0[f], my_n[sn][f][lane], res[f], dt);
    if (out_lane) {
      const long long so = (long long)o * nx + c;
      a.out[so] = u[0];
      a.out[P + so] = u[1];
      a.out[2 * P + so] = u[2];
      a.out[3 * P + so] = u[3];
    }
    // next row's U*: row o+1 (C1), and row o+2 (just produced, S1) behind it
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      C0[f] = C1[f];
      C1[f] = fresh ? S1[f] : C1[f];
    }
    if (a.reduce) {
      // CFL wave speed of the new state, (|u|+c)/dx + (|v|+c)/dy
      const T ir = rcp(u[0]);
      const T uu = u[1] * ir, vv = u[2] * ir;
      const T pp = gm1 * (u[3] - T(0.5) * (u[1] * uu + u[2] * vv));
      const T c2 = gam * pp * ir;
      const T cs = c2 * rsq(c2);
      const T sp = (fabs(uu) + cs) * a.idx + (fabs(vv) + cs) * a.idy;
      const bool ok = (u[0] > T(0)) && (pp > T(0)) && (sp <= T(3.0e38));
      if (out_lane) {
        if (ok) smax = fmax(smax, double(sp));
        else bad = true;
      }
    }
  }

  if (a.reduce) {
    unsigned long long m = wave_max_u64((unsigned long long)__double_as_longlong(smax));
    unsigned long long anybad = __ballot(bad);
    if (lane == 0) {
      if (m) atomicMax(&a.ctl->smax, m);
      if (anybad) atomicOr(&a.ctl->flag, 1u);
    }
  }
}

// Strip height of the fused kernel: 64 rows (each strip recomputes 4 rows
// of U* for its halo; measured on MI355X at 16384^2, 64 and 128 rows are
// best in FP64, 64 in FP32), halved (down to 8) until at least ~8k waves
// exist; LF_FUSED_ROWS (a power of two, 4..4096) overrides it.  The launch
// shape never changes the result.
static int fused_rows(int nx, int ny) {
  const int tiles_x = (nx + kFTileW - 1) / kFTileW;
  int r = 64;
  while (r > 8 && (long long)tiles_x * ((ny + r - 1) / r) < 8192) r /= 2;
  if (const char* env = getenv("LF_FUSED_ROWS")) {
    const int v = atoi(env);
    if (v >= 4 && v <= 4096 && (v & (v - 1)) == 0) r = v;
  }
  return r > ny ? ny : r;
}

template <typename T, int BCX, int BCY, bool CONS>
static hipError_t launch_fused_t(const Grid& g, const void* in, void* out, double dt, Ctl* ctl, bool dt_dev,
                                 bool reduce, hipStream_t s) {
  constexpr int WPB = waves_per_block<T>();
  FusedArgs<T> a;
  a.in = static_cast<const T*>(in);
  a.out = static_cast<T*>(out);
  a.ctl = ctl;
  a.nx = g.nx;
  a.ny = g.ny;
  a.rows = fused_rows(g.nx, g.ny);
  const int tiles_x = (g.nx + kFTileW - 1) / kFTileW;
  const int tiles_y = (g.ny + a.rows - 1) / a.rows;
  a.blocks_x = (tiles_x + WPB - 1) / WPB;
  a.blocks = a.blocks_x * tiles_y;
  a.blocks_pad = (a.blocks + kXcds - 1) / kXcds * kXcds;
  a.plane = (long long)g.nx * g.ny;
  a.gamma = T(g.gamma);
  a.gm1 = T(g.gamma - 1.0);
  a.inv_gm1 = T(1.0 / (g.gamma - 1.0));
  a.beta = T(g.beta);
  a.idx = T(1.0 / g.dx);
  a.idy = T(1.0 / g.dy);
  a.kxy = T(g.dx / g.dy);
  a.dt = dt;
  a.dt_dev = dt_dev ? 1 : 0;
  a.reduce = reduce ? 1 : 0;
  hipLaunchKernelGGL((fused_step_kernel<T, BCX, BCY, CONS>), dim3(a.blocks_pad), dim3(kWave * WPB), 0, s, a);
  return hipGetLastError();
}

template <typename T, bool CONS>
static hipError_t launch_fused_bc(const Grid& g, const void* in, void* out, double dt, Ctl* ctl, bool dt_dev,
                                  bool reduce, hipStream_t s) {
  if (g.bc_x == kBcPeriodic) {
    if (g.bc_y == kBcPeriodic)
      return launch_fused_t<T, kBcPeriodic, kBcPeriodic, CONS>(g, in, out, dt, ctl, dt_dev, reduce, s);
    return launch_fused_t<T, kBcPeriodic, kBcTransmissive, CONS>(g, in, out, dt, ctl, dt_dev, reduce, s);
  }
  if (g.bc_y == kBcPeriodic)
    return launch_fused_t<T, kBcTransmissive, kBcPeriodic, CONS>(g, in, out, dt, ctl, dt_dev, reduce, s);
  return launch_fused_t<T, kBcTransmissive, kBcTransmissive, CONS>(g, in, out, dt, ctl, dt_dev, reduce, s);
}

hipError_t launch_fused_step(const Grid& g, const void* in, void* out, double dt, Ctl* ctl, bool dt_dev,
                             bool reduce, hipStream_t s) {
  if (g.ns != 0) return hipErrorInvalidValue;  // states with mass fractions take the two-stage path
  if (g.dtype == 0)
    return g.recon ? launch_fused_bc<double, true>(g, in, out, dt, ctl, dt_dev, reduce, s)
                   : launch_fused_bc<double, false>(g, in, out, dt, ctl, dt_dev, reduce, s);
  return g.recon ? launch_fused_bc<float, true>(g, in, out, dt, ctl, dt_dev, reduce, s)
                 : launch_fused_bc<float, false>(g, in, out, dt, ctl, dt_dev, reduce, s);
}

}  // namespace lf
