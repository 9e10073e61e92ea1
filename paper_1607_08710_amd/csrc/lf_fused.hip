// lf_fused.hip -- one whole Heun step (Sec. 5, items 2-11) in a single pass
// over the state, mass fractions included.
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
// and a ghost lane reads U* from the lane of the edge column.  Ghost rows
// (a strip of a larger grid, lf_step_halo): the 4 rows beyond each end of
// the strip come from caller buffers, and U* of the rows beyond the ends is
// computed from them as a periodic strip computes it from wrapped rows.
#include <stdlib.h>

#include "lf_internal.h"

namespace lf {

constexpr int kFHalo = 4;
constexpr int kFTileW = kWave - 2 * kFHalo;  // 56 output columns per wave
// Waves per block, both precisions (the waves are independent; a block
// only numbers adjacent tiles).  Measured at 16384^2: FP32 runs 2.5%
// faster than with 8; FP64 runs as fast as with 2 and 12-28% faster than
// with 6.
constexpr int kFusedWaves = 4;

template <typename T>
struct FusedArgs {
  const T* in;  // U^n
  T* out;       // U^{n+1}, must not overlap in
  T* ustar;     // nullable: receives the predictor state U* of every cell
  const T* ghost_lo;  // BCY == kBcGhost: rows -4 .. -1, [NF][4][nx]
  const T* ghost_hi;  // BCY == kBcGhost: rows ny .. ny+3, [NF][4][nx]
  Ctl* ctl;
  int nx, ny, rows;
  int blocks_x, blocks, blocks_pad;
  long long plane;
  T gamma, gm1, inv_gm1, beta, idx, idy, kxy;
  T h;         // weight of a slope in a face value: 1/2, or 0 for beta = 0
  double rdx;  // 1 / dx, for dt / dx
  double dt;
  int dt_dev, reduce;
};

// FP64 with two or more mass fractions is short of registers (more than
// 256 VGPRs would leave one wave per SIMD): it recomputes the window's row
// difference instead of carrying it, and runs one row per loop trip.
template <typename T, int NS>
constexpr bool regs_to_spare() { return !(sizeof(T) == 8 && NS >= 2); }

// FP64 without mass fractions, periodic in x, periodic or ghost-row in y,
// with the primitive reconstruction: with one row of U^n in flight ahead
// of the predictor instead of two it needs 167 VGPRs, which leaves three
// waves per SIMD instead of two (1.5% faster at 16384^2).  The variants
// that stay at two waves keep two rows in flight (one row is up to 3%
// slower there).
template <typename T, int BCX, int BCY, int NS, bool CONS>
constexpr bool fp64_three_waves() {
  return sizeof(T) == 8 && NS == 0 && !CONS && BCX == kBcPeriodic && BCY != kBcTransmissive;
}

// Waves per SIMD the compiler must leave room for.  FP32 without mass
// fractions, periodic in x and periodic or ghost-row in y, with the
// primitive reconstruction, fits five (96 VGPRs without a spill), which
// runs 2% faster than the four its unconstrained 97-register allocation
// allows; the other variants would spill at 96 and take what their
// registers allow.  FP64: three where fp64_three_waves() holds.
template <typename T, int BCX, int BCY, int NS, bool CONS>
constexpr int fused_min_waves() {
  if constexpr (sizeof(T) == 4)
    return NS == 0 && !CONS && BCX == kBcPeriodic && BCY != kBcTransmissive ? 5 : 1;
  else
    return fp64_three_waves<T, BCX, BCY, NS, CONS>() ? 3 : 1;
}

// Rows of U^n in flight ahead of the predictor: one or two.
template <typename T, int BCX, int BCY, int NS, bool CONS>
constexpr int fused_ahead() { return fp64_three_waves<T, BCX, BCY, NS, CONS>() ? 1 : 2; }

// Reconstruction variables of one row: the Euler part (primitive, or
// conservative under CONS) and the mass fractions y_k = (rho y_k) / rho.
template <typename T, int NS>
struct RowV {
  Prim<T> w;
  Frac<T, NS> y;
};

template <bool CONS, int NS, typename T, int NF>
__device__ __forceinline__ RowV<T, NS> row_vars(const T (&q)[NF], T gm1) {
  RowV<T, NS> r;
  r.w = rec_vars<CONS>(q[0], q[1], q[2], q[3], gm1);
  if constexpr (NS > 0) {
    const T ir = rcp(q[0]);
#pragma unroll
    for (int s = 0; s < NS; ++s) r.y.v[s] = q[4 + s] * ir;
  }
  return r;
}

// y-window of one stage: rows a and a+1, their difference, the y-slopes
// of row a and the fluxes through face a-1/2, for the Euler variables and
// the fractions.
template <typename T, int NS>
struct Win {
  Prim<T> w0, w1, d1, s0;
  Flux<T> g;
  Frac<T, NS> y0, y1, sy0, gy;
};

// Window of row a from the rows a-2 .. a+1.
template <bool CONS, int NS, typename T>
__device__ __forceinline__ Win<T, NS> prime_window(const RowV<T, NS>& ra, const RowV<T, NS>& rb,
                                                   const RowV<T, NS>& r0, const RowV<T, NS>& r1, T beta, T h,
                                                   T gam, T gm1, T igm1) {
  Win<T, NS> W;
  const Prim<T> d_mid = sub(r0.w, rb.w);
  const Prim<T> s_b = slope(sub(rb.w, ra.w), d_mid, beta);
  W.d1 = sub(r1.w, r0.w);
  W.s0 = slope(d_mid, W.d1, beta);
  bool gl;
  W.g = face_flux(face_prim<CONS>(face_plus<T, true>(rb.w, s_b, h), gm1),
                  face_prim<CONS>(face_minus<T, true>(r0.w, W.s0, h), gm1), gam, igm1, gl);
  W.w0 = r0.w;
  W.w1 = r1.w;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const T sb = sweby(r0.y.v[s] - rb.y.v[s], rb.y.v[s] - ra.y.v[s], beta);
    W.sy0.v[s] = sweby(r1.y.v[s] - r0.y.v[s], r0.y.v[s] - rb.y.v[s], beta);
    W.gy.v[s] = W.g.f0 * fma(gl ? h : -h, gl ? sb : W.sy0.v[s], gl ? rb.y.v[s] : r0.y.v[s]);
  }
  W.y0 = r0.y;
  W.y1 = r1.y;
  return W;
}

// Flux balance (dx times the residual of eq. (11)) of row a of the window
// (every lane; valid two lanes inside the valid input), given row a+2;
// slides the window by a row.  Same arithmetic, in the same order, as the
// stage kernel's row, mass fractions included (their face value is one fma
// on the operands of the upwind side, so no lane shift is left to a
// branch).  The difference w1 - w0 is the one formed a row earlier (the
// same value, when it is recomputed).
template <bool CONS, int NS, typename T>
__device__ __forceinline__ void window_row(Win<T, NS>& W, const RowV<T, NS>& rn, T beta, T h, T gam, T gm1, T igm1,
                                           T kxy, T (&r)[4 + NS]) {
  const Prim<T> dn = sub(rn.w, W.w1);
  Prim<T> d1;
  if constexpr (regs_to_spare<T, NS>()) d1 = W.d1;
  else d1 = sub(W.w1, W.w0);
  const Prim<T> s1 = slope(d1, dn, beta);
  bool gl, fl;
  const Flux<T> G = face_flux(face_prim<CONS>(face_plus<T, true>(W.w0, W.s0, h), gm1),
                              face_prim<CONS>(face_minus<T, true>(W.w1, s1, h), gm1), gam, igm1, gl);
  const Prim<T> wr1 = shl1(W.w0);
  const Prim<T> dxp = sub(wr1, W.w0);
  const Prim<T> dxm = shr1(dxp);
  const Prim<T> sx = slope(dxm, dxp, beta);
  const Prim<T> sx1 = shl1(sx);
  const Flux<T> F = face_flux(face_prim<CONS>(face_plus<T, false>(W.w0, sx, h), gm1),
                              face_prim<CONS>(face_minus<T, false>(wr1, sx1, h), gm1), gam, igm1, fl);
  const Flux<T> Fm = shr1(F);
  r[0] = fma(G.f0 - W.g.f0, kxy, F.f0 - Fm.f0);
  r[1] = fma(G.f2 - W.g.f2, kxy, F.f1 - Fm.f1);
  r[2] = fma(G.f1 - W.g.f1, kxy, F.f2 - Fm.f2);
  r[3] = fma(G.f3 - W.g.f3, kxy, F.f3 - Fm.f3);
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const T sy1 = sweby(rn.y.v[s] - W.y1.v[s], W.y1.v[s] - W.y0.v[s], beta);
    const T gy = G.f0 * fma(gl ? h : -h, gl ? W.sy0.v[s] : sy1, gl ? W.y0.v[s] : W.y1.v[s]);
    const T yr1 = shl1(W.y0.v[s]);
    const T dp = yr1 - W.y0.v[s];
    const T sxs = sweby(dp, shr1(dp), beta);
    const T sxs1 = shl1(sxs);
    const T fy = F.f0 * fma(fl ? h : -h, fl ? sxs : sxs1, fl ? W.y0.v[s] : yr1);
    r[4 + s] = fma(gy - W.gy.v[s], kxy, fy - shr1(fy));
    W.sy0.v[s] = sy1;
    W.gy.v[s] = gy;
  }
  W.w0 = W.w1;
  W.w1 = rn.w;
  W.d1 = dn;
  W.s0 = s1;
  W.g = G;
  W.y0 = W.y1;
  W.y1 = rn.y;
}

// The kernel is bound by arithmetic, not by memory (it moves 64 B per FP64
// cell and step without fractions), so its LDS footprint is kept small for
// occupancy: U^n of the rows still to be combined waits in a per-wave LDS
// ring, U* of the two rows waiting for the corrector's combination stays in
// registers, and one LDS row of U* serves the reads across lanes where they
// are needed (transmissive x) and in FP32 (where the round trip through LDS
// saves the registers that a fifth wave per SIMD needs).  Results are
// stored straight from the lanes (no staging, no block barrier).
template <typename T, int BCX, int BCY, int NS, bool CONS>
__global__ __launch_bounds__(kWave * kFusedWaves) __attribute__((amdgpu_waves_per_eu(fused_min_waves<T, BCX, BCY, NS, CONS>())))
void fused_step_kernel(FusedArgs<T> a) {
  static_assert(!CONS || NS == 0, "the conservative reconstruction is built without mass fractions");
  constexpr int NF = 4 + NS;  // conservative fields: Euler, then rho*y_k
  constexpr int WPB = kFusedWaves;
  constexpr bool XT = BCX == kBcTransmissive;
  constexpr bool YT = BCY == kBcTransmissive;
  constexpr bool SROW = XT || sizeof(T) == 4;  // U* rows pass through LDS
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
  const double dtx = dt * a.rdx;
  const T gm1 = a.gm1, gam = a.gamma, igm1 = a.inv_gm1, beta = a.beta, h = a.h, kxy = a.kxy, idx = a.idx;

  const T* __restrict__ I0 = a.in;
  // byte offsets of this lane's column in a row: loads (cm) and stores (c,
  // stored only where it lies in the grid)
  const unsigned lboff = unsigned(cm) * sizeof(T), sboff = unsigned(c) * sizeof(T);
  auto load_row = [&](int row, T (&q)[NF]) {
    if constexpr (BCY == kBcGhost) {
      // the strip's rows, or the ghost rows beyond its ends (every row
      // read lies in -kGhostRows .. ny+kGhostRows-1: see nlast below)
      const T* src = I0;
      long long pl = P;
      int r = row;
      if (row < 0) {
        src = a.ghost_lo;
        pl = (long long)kGhostRows * nx;
        r = row + kGhostRows;
      } else if (row >= ny) {
        src = a.ghost_hi;
        pl = (long long)kGhostRows * nx;
        r = row - ny;
      }
      const T* rp = src + (long long)r * nx;
      const unsigned bo = lane_offset(rp, lboff);
#pragma unroll
      for (int f = 0; f < NF; ++f) q[f] = ld_lane(rp + f * pl, bo);
    } else {
      const T* rp = I0 + (long long)map_index<BCY>(row, ny) * nx;
      const unsigned bo = lane_offset(rp, lboff);
#pragma unroll
      for (int f = 0; f < NF; ++f) q[f] = ld_lane(rp + f * P, bo);
    }
  };

  // U^n ring (rows o .. o+4 are alive while row o is finished) and the
  // U* row exchanged across lanes.
  __shared__ T nring[WPB][5][NF][kWave];
  __shared__ T srow[WPB][NF][SROW ? kWave : 1];
  T(*my_n)[NF][kWave] = nring[w];
  T(*my_s)[SROW ? kWave : 1] = srow[w];
  auto nslot = [](int r) { return (r % 5 + 5) % 5; };
  auto put_n = [&](int r, const T (&q)[NF]) {
    const int sl = nslot(r);
#pragma unroll
    for (int f = 0; f < NF; ++f) my_n[sl][f][lane] = q[f];
  };
  // U* row r as the corrector sees it: transmissive ghost rows are the edge
  // row
  auto rmap = [&](int r) { return YT ? min(max(r, 0), ny - 1) : r; };

  // Rows of U* the corrector needs: y0-2 .. y1+1; the predictor produces
  // the ones that are not transmissive ghosts, reading U^n rows plo-2 ..
  // nlast (y0-4 .. y1+3 unless transmissive: within the ghost rows).
  const int plo = YT ? max(y0 - 2, 0) : y0 - 2;
  const int phi = YT ? min(y1 + 1, ny - 1) : y1 + 1;
  const int nlast = phi + 2;  // last U^n row the predictor reads

  // ---- predictor: window of row plo, U^n row plo+2 (and plo+3) in flight ----
  T QA[NF], QB[NF];  // U^n rows pr+2 and (two rows in flight) pr+3
#pragma unroll
  for (int f = 0; f < NF; ++f) QB[f] = T(0);
  Win<T, NS> PW;
  {
    T qa[NF], qb[NF], q0[NF], q1[NF];
    load_row(plo - 2, qa);
    load_row(plo - 1, qb);
    load_row(plo, q0);
    load_row(plo + 1, q1);
    load_row(plo + 2, QA);
    if constexpr (fused_ahead<T, BCX, BCY, NS, CONS>() == 2) load_row(min(plo + 3, nlast), QB);
    put_n(plo, q0);
    put_n(plo + 1, q1);
    PW = prime_window<CONS, NS>(row_vars<CONS, NS>(qa, gm1), row_vars<CONS, NS>(qb, gm1),
                                row_vars<CONS, NS>(q0, gm1), row_vars<CONS, NS>(q1, gm1), beta, h, gam, gm1, igm1);
  }
  int pr = plo;  // next U* row to produce
  // U* of the last two rows produced (conservative, this lane's column):
  // S1 = row pr-1, S0 = row pr-2
  T S0[NF], S1[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) S0[f] = S1[f] = T(0);
  // U* row pr = U^n - dt R(U^n); it goes to S1 (S1 moves to S0) and to the
  // LDS row read across lanes (when there is one)
  auto produce = [&]() {
    const RowV<T, NS> rn = row_vars<CONS, NS>(QA, gm1);  // U^n row pr+2
    put_n(pr + 2, QA);
    // the next row, unconditional (past the last row it re-reads that row,
    // unused), so that the compiler can count the loads in flight and wait
    // only for the row it needs, not for the one loaded a row later
    if constexpr (fused_ahead<T, BCX, BCY, NS, CONS>() == 2) {
#pragma unroll
      for (int f = 0; f < NF; ++f) QA[f] = QB[f];
      load_row(min(pr + 4, nlast), QB);
    } else {
      load_row(min(pr + 3, nlast), QA);
    }
    T bal[NF];  // flux balances
    window_row<CONS, NS>(PW, rn, beta, h, gam, gm1, igm1, kxy, bal);
    const int sn = nslot(pr);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      S0[f] = S1[f];
      S1[f] = combine<kPredictor>(my_n[sn][f][lane], T(0), bal[f], dtx, idx);
      if constexpr (SROW) my_s[f][lane] = S1[f];
    }
    // U* of the strip's own rows, when asked for (halo rows belong to the
    // neighbouring strips)
    if (a.ustar && out_lane && pr >= y0 && pr < y1) {
      T* rp = a.ustar + (long long)pr * nx;
      const unsigned bo = lane_offset(rp, sboff);
#pragma unroll
      for (int f = 0; f < NF; ++f) st_lane(rp + f * P, bo, S1[f]);
    }
    ++pr;
  };
  // reconstruction variables of the newest U* row produced, at this lane's
  // column (ghost lanes: the edge column)
  auto star_row = [&]() {
    if constexpr (SROW) {
      T q[NF];
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int f = 0; f < NF; ++f) q[f] = my_s[f][src];
      return row_vars<CONS, NS>(q, gm1);
    } else {
      return row_vars<CONS, NS>(S1, gm1);  // src == lane
    }
  };

  // ---- corrector: window of row y0 from U* rows y0-2 .. y0+1 ----
  // Each needed row is read as soon as it is the newest one produced
  // (transmissive ghost rows reuse the edge row).
  RowV<T, NS> cw[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = rmap(y0 - 2 + k);
    while (pr <= r) produce();
    cw[k] = star_row();
  }
  Win<T, NS> CW = prime_window<CONS, NS>(cw[0], cw[1], cw[2], cw[3], beta, h, gam, gm1, igm1);
  // U* (conservative) of the rows the corrector combines next: row o in C0,
  // row o+1 in C1
  T C0[NF], C1[NF];
  {
    // rows y0 and y0+1 were the last ones produced, unless the strip ends
    // at a transmissive top (then row y0 is the newest: y0 == ny - 1)
    const bool two = pr - 1 >= y0 + 1;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      C0[f] = two ? S0[f] : S1[f];
      C1[f] = S1[f];
    }
  }

  T smax = T(0);
  bool bad = false;

  // One corrector row (and the predictor row two ahead of it).
  auto row = [&](int o) {
    const bool fresh = o + 2 <= phi;
    if (fresh) produce();
    const RowV<T, NS> rn = star_row();  // U* row rmap(o+2), the newest produced
    T bal[NF];
    window_row<CONS, NS>(CW, rn, beta, h, gam, gm1, igm1, kxy, bal);
    const int sn = nslot(o);
    T u[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) u[f] = combine<kCorrector>(C0[f], my_n[sn][f][lane], bal[f], dtx, idx);
    if (out_lane) {
      T* rp = a.out + (long long)o * nx;
      const unsigned bo = lane_offset(rp, sboff);
#pragma unroll
      for (int f = 0; f < NF; ++f) st_lane(rp + f * P, bo, u[f]);
    }
    // next row's U*: row o+1 (C1), and row o+2 (just produced, S1) behind it
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      C0[f] = C1[f];
      C1[f] = fresh ? S1[f] : C1[f];
    }
    if (a.reduce) {
      // CFL wave speed of the new state
      bool ok;
      const T sp = cfl_speed(u[0], u[1], u[2], u[3], gm1, gam, a.idx, a.idy, ok);
      if (out_lane) {
        if (ok) smax = speed_max(smax, sp);
        else bad = true;
      }
    }
  };
  // Three rows per trip: the window rows rotate w0 <- w1 <- new row, so
  // with three bodies per trip every loop-carried value is last read before
  // its successor is written, and the register rotation costs no moves
  // (about 6% of the loop's instructions).  The compiler does not unroll
  // this loop itself: it holds cross-lane operations.  FP64 with two or
  // more fractions keeps one row per trip: unrolled, it would need more
  // than 256 VGPRs.
  int o = y0;
  if constexpr (regs_to_spare<T, NS>()) {
#pragma unroll 1
    for (; o + 3 <= y1; o += 3) {
      row(o);
      row(o + 1);
      row(o + 2);
    }
  }
#pragma unroll 1
  for (; o < y1; ++o) row(o);

  if (a.reduce) {
    unsigned long long m = wave_max_u64((unsigned long long)__double_as_longlong(double(smax)));
    unsigned long long anybad = __ballot(bad);
    if (lane == 0) {
      if (m) atomicMax(&a.ctl->smax, m);
      if (anybad) atomicOr(&a.ctl->flag, 1u);
    }
  }
}

// Strip height of the fused kernel: 128 rows in FP64, 64 in FP32 (each
// strip recomputes 4 rows of U* for its halo; measured best on MI355X at
// 16384^2 in FP64; in FP32 128 rows are within 1% there and 5% slower at
// 8192^2).  FP64 halves it to 64 rows while the launch has fewer than
// 16384 waves (at 8192^2 64 rows are 2.5-3% faster than 128).  Then it is
// halved (down to 8) until the launch has 4096 waves in FP64 or 8192 in
// FP32, the best measured at 4096^2 (for FP64 at two and at three waves
// per SIMD).  LF_FUSED_ROWS (4..4096) overrides it.  The launch shape never
// changes the result.
static int fused_rows(int nx, int ny, int esize) {
  const long long tiles_x = (nx + kFTileW - 1) / kFTileW;
  auto waves = [&](int r) { return tiles_x * ((ny + r - 1) / r); };
  int r = esize == 8 ? 128 : 64;
  if (esize == 8)
    while (r > 64 && waves(r) < 16384) r /= 2;
  const long long min_waves = esize == 8 ? 4096 : 8192;
  while (r > 8 && waves(r) < min_waves) r /= 2;
  if (const char* env = getenv("LF_FUSED_ROWS")) {
    const int v = atoi(env);
    if (v >= 4 && v <= 4096) r = v;
  }
  return r > ny ? ny : r;
}

template <typename T, int BCX, int BCY, int NS, bool CONS>
static hipError_t launch_fused_t(const Grid& g, const void* in, void* out, void* ustar, double dt, Ctl* ctl,
                                 bool dt_dev, bool reduce, const GhostRows& gh, hipStream_t s) {
  constexpr int WPB = kFusedWaves;
  FusedArgs<T> a;
  a.in = static_cast<const T*>(in);
  a.out = static_cast<T*>(out);
  a.ustar = static_cast<T*>(ustar);
  a.ghost_lo = static_cast<const T*>(gh.lo);
  a.ghost_hi = static_cast<const T*>(gh.hi);
  a.ctl = ctl;
  a.nx = g.nx;
  a.ny = g.ny;
  a.rows = fused_rows(g.nx, g.ny, (int)sizeof(T));
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
  a.h = T(g.beta == 0.0 ? 0.0 : 0.5);
  a.idx = T(1.0 / g.dx);
  a.idy = T(1.0 / g.dy);
  a.kxy = T(g.dx / g.dy);
  a.rdx = 1.0 / g.dx;
  a.dt = dt;
  a.dt_dev = dt_dev ? 1 : 0;
  a.reduce = reduce ? 1 : 0;
  hipLaunchKernelGGL((fused_step_kernel<T, BCX, BCY, NS, CONS>), dim3(a.blocks_pad), dim3(kWave * WPB), 0, s, a);
  return hipGetLastError();
}

template <typename T, int BCX, int BCY>
static hipError_t launch_fused_ns(const Grid& g, const void* in, void* out, void* ustar, double dt, Ctl* ctl,
                                  bool dt_dev, bool reduce, const GhostRows& gh, hipStream_t s) {
  static_assert(kMaxSpecies == 4, "one instantiation per species count");
  if (g.recon) return launch_fused_t<T, BCX, BCY, 0, true>(g, in, out, ustar, dt, ctl, dt_dev, reduce, gh, s);
  switch (g.ns) {
    case 0: return launch_fused_t<T, BCX, BCY, 0, false>(g, in, out, ustar, dt, ctl, dt_dev, reduce, gh, s);
    case 1: return launch_fused_t<T, BCX, BCY, 1, false>(g, in, out, ustar, dt, ctl, dt_dev, reduce, gh, s);
    case 2: return launch_fused_t<T, BCX, BCY, 2, false>(g, in, out, ustar, dt, ctl, dt_dev, reduce, gh, s);
    case 3: return launch_fused_t<T, BCX, BCY, 3, false>(g, in, out, ustar, dt, ctl, dt_dev, reduce, gh, s);
    default: return launch_fused_t<T, BCX, BCY, 4, false>(g, in, out, ustar, dt, ctl, dt_dev, reduce, gh, s);
  }
}

template <typename T, int BCX>
static hipError_t launch_fused_by(const Grid& g, const void* in, void* out, void* ustar, double dt, Ctl* ctl,
                                  bool dt_dev, bool reduce, const GhostRows& gh, hipStream_t s) {
  if (gh.lo) return launch_fused_ns<T, BCX, kBcGhost>(g, in, out, ustar, dt, ctl, dt_dev, reduce, gh, s);
  if (g.bc_y == kBcPeriodic)
    return launch_fused_ns<T, BCX, kBcPeriodic>(g, in, out, ustar, dt, ctl, dt_dev, reduce, gh, s);
  return launch_fused_ns<T, BCX, kBcTransmissive>(g, in, out, ustar, dt, ctl, dt_dev, reduce, gh, s);
}

template <typename T>
static hipError_t launch_fused_bc(const Grid& g, const void* in, void* out, void* ustar, double dt, Ctl* ctl,
                                  bool dt_dev, bool reduce, const GhostRows& gh, hipStream_t s) {
  if (g.bc_x == kBcPeriodic)
    return launch_fused_by<T, kBcPeriodic>(g, in, out, ustar, dt, ctl, dt_dev, reduce, gh, s);
  return launch_fused_by<T, kBcTransmissive>(g, in, out, ustar, dt, ctl, dt_dev, reduce, gh, s);
}

hipError_t launch_fused_step(const Grid& g, const void* in, void* out, void* ustar, double dt, Ctl* ctl,
                             bool dt_dev, bool reduce, hipStream_t s, GhostRows gh) {
  if (g.dtype == 0) return launch_fused_bc<double>(g, in, out, ustar, dt, ctl, dt_dev, reduce, gh, s);
  return launch_fused_bc<float>(g, in, out, ustar, dt, ctl, dt_dev, reduce, gh, s);
}

}  // namespace lf
