// lf_forward.hip -- forward kernels of the gfx950 Lagrange-flux library.
//
// One fused stage kernel per Heun stage (Sec. 5, predictor items 2-6 and
// corrector items 7-11 of the paper's list), the CFL max-reduction
// (item 1), the device-side control of the time loop and the
// conservation totals.
//
// Stage kernel layout.  A wave of 64 lanes owns a strip of 64 consecutive
// columns (x, the fastest index of the structure-of-arrays state) and
// marches up kTileW-wide strips of `rows` rows.  Lanes 2..61 produce
// output; lanes 0, 1, 62, 63 are the stencil halo and only feed their
// neighbours.  x-neighbours are exchanged with DPP whole-wave shifts; the
// y-direction keeps a register window (two primitive rows, one row of
// y-slopes and differences, and the last y-face flux), so every face flux
// is evaluated exactly once per wave and never written to memory.
#include <stdlib.h>

#include "lf_internal.h"

namespace lf {

template <typename T>
struct StageArgs {
  const T* in;    // stencil input state
  const T* base;  // corrector: U^n (may alias out)
  T* out;
  Ctl* ctl;
  int nx, ny;
  int tiles_x, tiles_y, rows;
  int blocks_x, blocks, blocks_pad;
  long long plane;
  T gamma, gm1, inv_gm1, beta, idx, idy, kxy;  // kxy = dx / dy
  T h;  // weight of a slope in a face value: 1/2, or 0 for beta = 0
  double rdx;  // 1 / dx, for dt / dx
  double dt;
  int dt_dev;
  int reduce;
};

template <typename T, int MODE, int BCX, int BCY, int NS, bool CONS>
__global__ __launch_bounds__(kWave * waves_per_block<T>()) void stage_kernel(StageArgs<T> a) {
  static_assert(!CONS || NS == 0, "the conservative reconstruction is built without mass fractions");
  constexpr int WPB = waves_per_block<T>();
  constexpr int NF = 4 + NS;  // conservative fields: Euler, then rho*y_k
  if (a.dt_dev && a.ctl->done) return;
  const int lb = xcd_block(blockIdx.x, a.blocks_pad);
  if (lb >= a.blocks) return;  // whole block
  // block (bx, by): tiles bx*WPB .. bx*WPB+WPB-1 of row band by; a tile
  // past the right edge still runs (the block synchronises every row) but
  // stores nothing
  const int by = lb / a.blocks_x;
  const int bx = lb - by * a.blocks_x;
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & (kWave - 1);
  const int tx = bx * WPB + w;
  const int c = tx * kTileW - kHalo + lane;
  const int cm = map_index<BCX>(c, a.nx);
  const int y0 = by * a.rows;
  const int y1 = min(y0 + a.rows, a.ny);
  const bool out_lane = lane >= kHalo && lane < kWave - kHalo && c < a.nx;
  const double dt = a.dt_dev ? a.ctl->dt : a.dt;
  const double dtx = dt * a.rdx;
  const int nx = a.nx, ny = a.ny;
  const long long plane = a.plane;
  const T gm1 = a.gm1, gam = a.gamma, igm1 = a.inv_gm1, beta = a.beta, h = a.h;

  const T* __restrict__ I0 = a.in;
  const T* __restrict__ I1 = I0 + plane;
  const T* __restrict__ I2 = I1 + plane;
  const T* __restrict__ I3 = I2 + plane;
  const T* __restrict__ IS = I3 + plane;  // rho*y_k planes

  auto load_row = [&](int row, T (&q)[NF]) {
    const int off = map_index<BCY>(row, ny) * nx + cm;
    q[0] = I0[off];
    q[1] = I1[off];
    q[2] = I2[off];
    q[3] = I3[off];
#pragma unroll
    for (int s = 0; s < NS; ++s) q[4 + s] = IS[s * plane + off];
  };

  T* O0 = a.out;
  T* O1 = O0 + plane;
  T* O2 = O1 + plane;
  T* O3 = O2 + plane;
  T* OS = O3 + plane;
  // base is nullptr unless MODE == kCorrector; only the corrector reads it
  const T* B0 = a.base;
  const T* B1 = B0 + plane;
  const T* B2 = B1 + plane;
  const T* B3 = B2 + plane;
  const T* BS = B3 + plane;
  // U^n of the corrector is read through the caches: a wave's row of it
  // starts and ends inside 128-byte lines that the neighbouring waves
  // read too, and streaming (non-temporal) loads fetched each of those
  // lines once per wave (the corrector read 1.11x its bytes; now 1.08x).
  // The output, written in whole lines, goes as streaming stores.
  auto load_base = [&](int off, T (&b)[NF]) {
    b[0] = B0[off];
    b[1] = B1[off];
    b[2] = B2[off];
    b[3] = B3[off];
#pragma unroll
    for (int s = 0; s < NS; ++s) b[4 + s] = BS[s * plane + off];
  };

  // Row pipeline.  While row o is finished, the stencil rows o+3 and o+4
  // are in flight (prefetch distance two rows) and the corrector's U^n rows
  // o+1 and o+2 likewise.  The conservative values of rows o .. o+2, needed
  // only for the stage combination, wait in a per-wave LDS ring (each lane
  // reads back its own values, so no synchronisation is needed).  Slots
  // alternate between the even and odd rows of a strip; the loop is
  // unrolled by two so that they rotate by renaming.
  __shared__ T ring[WPB][3][NF][kWave];
  T(*my)[NF][kWave] = ring[w];
  // Output staging: the block's WPB * 60 new values of a row are gathered
  // in LDS (double buffered) and written back as whole 128-byte lines
  // starting at the block's first column, a multiple of 15 lines.
  constexpr int BW = WPB * kTileW;
  __shared__ T obuf[2][NF][BW];
  const int xb = bx * BW;   // first column of the block
  const int kst = w * kWave + lane;  // column (in the block) this lane stores
  int par = 0;
  auto ring_put = [&](int row, const T (&q)[NF]) {
    const int sl = row % 3;
#pragma unroll
    for (int f = 0; f < NF; ++f) my[sl][f][lane] = q[f];
  };
  // mass fractions y_k = (rho y_k) / rho of a loaded row
  auto fractions = [&](const T (&q)[NF]) {
    Frac<T, NS> y;
    if constexpr (NS > 0) {
      const T ir = rcp(q[0]);
#pragma unroll
      for (int s = 0; s < NS; ++s) y.v[s] = q[4 + s] * ir;
    }
    return y;
  };

  T QA[NF], QB[NF], BA[NF], BB[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) BA[f] = BB[f] = T(0);
  Prim<T> W0, W1, Sg0, Sg1;
  Flux<T> Gf0, Gf1;
  // the same window for the mass fractions: values, y-slopes and the flux
  // through the last y-face
  Frac<T, NS> Y0, Y1, Sy0, Sy1, Gy0, Gy1;
  {
    T qa[NF], qb[NF], q0[NF], q1[NF];
    load_row(y0 - 2, qa);
    load_row(y0 - 1, qb);
    load_row(y0, q0);
    load_row(y0 + 1, q1);
    load_row(y0 + 2, QA);
    load_row(y0 + 3, QB);
    if constexpr (MODE == kCorrector) {
      const int o0 = y0 * nx + cm;
      load_base(o0, BA);
      if (y0 + 1 < y1) load_base(o0 + nx, BB);
    }
    Prim<T> wa = rec_vars<CONS>(qa[0], qa[1], qa[2], qa[3], gm1);
    Prim<T> wb = rec_vars<CONS>(qb[0], qb[1], qb[2], qb[3], gm1);
    W0 = rec_vars<CONS>(q0[0], q0[1], q0[2], q0[3], gm1);
    W1 = rec_vars<CONS>(q1[0], q1[1], q1[2], q1[3], gm1);
    ring_put(y0, q0);
    ring_put(y0 + 1, q1);
    Prim<T> d_lo = sub(wb, wa);    // y0 - 3/2
    Prim<T> d_mid = sub(W0, wb);   // y0 - 1/2
    Prim<T> s_b = slope(d_lo, d_mid, beta);
    Sg0 = slope(d_mid, sub(W1, W0), beta);
    bool gl;
    Gf0 = face_flux(face_prim<CONS>(face_plus<T, true>(wb, s_b, h), gm1),
                    face_prim<CONS>(face_minus<T, true>(W0, Sg0, h), gm1), gam, igm1, gl);
    if constexpr (NS > 0) {
      const Frac<T, NS> ya = fractions(qa), yb = fractions(qb);
      Y0 = fractions(q0);
      Y1 = fractions(q1);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const T sb = sweby(Y0.v[s] - yb.v[s], yb.v[s] - ya.v[s], beta);
        Sy0.v[s] = sweby(Y1.v[s] - Y0.v[s], Y0.v[s] - yb.v[s], beta);
        Gy0.v[s] = Gf0.f0 * fma(gl ? h : -h, gl ? sb : Sy0.v[s], gl ? yb.v[s] : Y0.v[s]);
      }
    }
  }

  T smax = T(0);
  bool bad = false;

  // Row o: qc holds row o+2 (arrived) and then receives row o+4; bc holds
  // U^n of row o and then receives row o+2; wo/wo1 are the primitive rows
  // o and o+1 (wo is overwritten with row o+2); so/so1 the y-slopes of rows
  // o and o+1; Gp/G the fluxes through the y-faces o-1/2 and o+1/2.  The
  // mass fractions rotate the same way (yo, yo1, syo, syo1, gyp, gy).
  auto row = [&](int o, T (&qc)[NF], T (&bc)[NF], Prim<T>& wo, const Prim<T>& wo1, const Prim<T>& so,
                 Prim<T>& so1, const Flux<T>& Gp, Flux<T>& G, Frac<T, NS>& yo, const Frac<T, NS>& yo1,
                 const Frac<T, NS>& syo, Frac<T, NS>& syo1, const Frac<T, NS>& gyp, Frac<T, NS>& gy) {
    const int off = o * nx + cm;
    const Prim<T> wn = rec_vars<CONS>(qc[0], qc[1], qc[2], qc[3], gm1);
    const Frac<T, NS> yn = fractions(qc);
    ring_put(o + 2, qc);
    if (o + 3 <= y1) load_row(o + 4, qc);

    // y: slope of row o+1, flux through face o+1/2
    const Prim<T> dlo = sub(wo1, wo);
    so1 = slope(dlo, sub(wn, wo1), beta);
    bool gl;
    G = face_flux(face_prim<CONS>(face_plus<T, true>(wo, so, h), gm1),
                  face_prim<CONS>(face_minus<T, true>(wo1, so1, h), gm1), gam, igm1, gl);

    // x: slopes of row o from lane neighbours, flux through face c+1/2
    const Prim<T> wr1 = shl1(wo);       // w_{c+1}
    const Prim<T> dxp = sub(wr1, wo);   // w_{c+1} - w_c
    const Prim<T> dxm = shr1(dxp);      // w_c - w_{c-1}
    const Prim<T> sx = slope(dxm, dxp, beta);
    const Prim<T> sx1 = shl1(sx);       // sigma_{c+1}
    bool fl;
    const Flux<T> F = face_flux(face_prim<CONS>(face_plus<T, false>(wo, sx, h), gm1),
                                face_prim<CONS>(face_minus<T, false>(wr1, sx1, h), gm1), gam, igm1, fl);
    const Flux<T> Fm = shr1(F);         // flux through face c-1/2

    // R = (F_{c+1/2} - F_{c-1/2})/dx + (G_{o+1/2} - G_{o-1/2})/dy, eq. (11),
    // as the flux balance s = dF + dG (dx/dy) with R = s / dx (the stage
    // combination takes dt / dx): with square cells dx/dy = 1 and the
    // single rounding of dF + dG keeps the x/y mirror symmetry exact.
    const T b0 = fma(G.f0 - Gp.f0, a.kxy, F.f0 - Fm.f0);
    const T b1 = fma(G.f2 - Gp.f2, a.kxy, F.f1 - Fm.f1);
    const T b2 = fma(G.f1 - Gp.f1, a.kxy, F.f2 - Fm.f2);
    const T b3 = fma(G.f3 - Gp.f3, a.kxy, F.f3 - Fm.f3);

    // Mass fractions: reconstructed like the primitive variables and
    // carried by the face mass flux from its upwind side, (rho_A u*) y_A.
    // The upwind face value is one fma whose operands are selected
    // (y + h s from the left cell or y - h s from the right one): written
    // as a select of two fmas, the compiler may branch on the side and
    // move the lane shift of the right cell's slope into one arm, where
    // the lanes of the other arm are inactive and read as zero.
    T bs[NS > 0 ? NS : 1];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      syo1.v[s] = sweby(yn.v[s] - yo1.v[s], yo1.v[s] - yo.v[s], beta);
      gy.v[s] = G.f0 * fma(gl ? h : -h, gl ? syo.v[s] : syo1.v[s], gl ? yo.v[s] : yo1.v[s]);
      const T yr1 = shl1(yo.v[s]);
      const T dp = yr1 - yo.v[s];
      const T sxs = sweby(dp, shr1(dp), beta);
      const T sxs1 = shl1(sxs);
      const T fy = F.f0 * fma(fl ? h : -h, fl ? sxs : sxs1, fl ? yo.v[s] : yr1);
      bs[s] = fma(gy.v[s] - gyp.v[s], a.kxy, fy - shr1(fy));
    }

    const int sl = o % 3;
    const T u0 = combine<MODE>(my[sl][0][lane], bc[0], b0, dtx, a.idx);
    const T u1 = combine<MODE>(my[sl][1][lane], bc[1], b1, dtx, a.idx);
    const T u2 = combine<MODE>(my[sl][2][lane], bc[2], b2, dtx, a.idx);
    const T u3 = combine<MODE>(my[sl][3][lane], bc[3], b3, dtx, a.idx);
    T us_[NS > 0 ? NS : 1];
#pragma unroll
    for (int s = 0; s < NS; ++s) us_[s] = combine<MODE>(my[sl][4 + s][lane], bc[4 + s], bs[s], dtx, a.idx);
    if constexpr (MODE == kCorrector) {
      if (o + 2 < y1) load_base(off + 2 * nx, bc);
    }
    {
      if (out_lane) {
        const int k = w * kTileW + lane - kHalo;
        obuf[par][0][k] = u0;
        obuf[par][1][k] = u1;
        obuf[par][2][k] = u2;
        obuf[par][3][k] = u3;
#pragma unroll
        for (int s = 0; s < NS; ++s) obuf[par][4 + s][k] = us_[s];
      }
      __syncthreads();
      const int col = xb + kst;
      if (kst < BW && col < nx) {
        const int so = o * nx + col;
        __builtin_nontemporal_store(obuf[par][0][kst], &O0[so]);
        __builtin_nontemporal_store(obuf[par][1][kst], &O1[so]);
        __builtin_nontemporal_store(obuf[par][2][kst], &O2[so]);
        __builtin_nontemporal_store(obuf[par][3][kst], &O3[so]);
#pragma unroll
        for (int s = 0; s < NS; ++s) __builtin_nontemporal_store(obuf[par][4 + s][kst], &OS[s * plane + so]);
      }
      par ^= 1;
    }
    if constexpr (MODE == kCorrector) {
      if (a.reduce) {
        // CFL wave speed of the new state
        bool ok;
        const T sp = cfl_speed(u0, u1, u2, u3, gm1, gam, a.idx, a.idy, ok);
        if (out_lane) {
          if (ok) smax = speed_max(smax, sp);
          else bad = true;
        }
      }
    }
    wo = wn;  // slot of row o now holds row o+2
    yo = yn;
  };

  for (int o = y0; o < y1; o += 2) {
    row(o, QA, BA, W0, W1, Sg0, Sg1, Gf0, Gf1, Y0, Y1, Sy0, Sy1, Gy0, Gy1);
    if (o + 1 < y1) row(o + 1, QB, BB, W1, W0, Sg1, Sg0, Gf1, Gf0, Y1, Y0, Sy1, Sy0, Gy1, Gy0);
  }

  if constexpr (MODE == kCorrector) {
    if (a.reduce) {
      unsigned long long m = wave_max_u64((unsigned long long)__double_as_longlong(double(smax)));
      unsigned long long anybad = __ballot(bad);
      if (lane == 0) {
        if (m) atomicMax(&a.ctl->smax, m);
        if (anybad) atomicOr(&a.ctl->flag, 1u);
      }
    }
  }
}

// ---- standalone CFL reduction (lf_dt, start of lf_advance) ----------------

template <typename T>
__global__ __launch_bounds__(256) void wavespeed_kernel(const T* __restrict__ U, long long plane,
                                                        T gamma, T gm1, T idx, T idy, Ctl* ctl) {
  T smax = T(0);
  bool bad = false;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < plane; q += stride) {
    T q0 = U[q], q1 = U[plane + q], q2 = U[2 * plane + q], q3 = U[3 * plane + q];
    bool ok;
    const T s = cfl_speed(q0, q1, q2, q3, gm1, gamma, idx, idy, ok);
    if (ok) smax = speed_max(smax, s);
    else bad = true;
  }
  unsigned long long m = wave_max_u64((unsigned long long)__double_as_longlong(double(smax)));
  unsigned long long anybad = __ballot(bad);
  if ((threadIdx.x & (kWave - 1)) == 0) {
    if (m) atomicMax(&ctl->smax, m);
    if (anybad) atomicOr(&ctl->flag, 1u);
  }
}

// ---- time-loop control (single thread) -----------------------------------

__global__ void ctl_init_kernel(Ctl* c, double t0, double t_end, long long max_steps, double cfl) {
  c->smax = 0ull;
  c->flag = 0u;
  c->done = (t0 < t_end && max_steps > 0) ? 0u : 1u;
  c->dt = 0.0;
  c->t = t0;
  c->t_end = t_end;
  c->step = 0;
  c->max_steps = max_steps;
  c->cfl = cfl;
  c->clamped = 0u;
}

// dt of the next step from the reduced wave speed, clamped to t_end.
__device__ void ctl_next_dt(Ctl* c) {
  double s = __longlong_as_double((long long)c->smax);
  c->smax = 0ull;
  if (c->flag || !(s > 0.0)) {
    c->flag |= 1u;
    c->done = 1u;
    c->dt = 0.0;
    return;
  }
  double dt = c->cfl / s;
  double rem = c->t_end - c->t;
  c->clamped = 0u;
  if (dt >= rem) {
    dt = rem;
    c->clamped = 1u;
  }
  c->dt = dt;
}

// dt of the first step.  When the loop is empty (t0 >= t_end or no steps
// allowed) only the non-physical flag of the initial state is kept.
__global__ void ctl_first_kernel(Ctl* c) {
  if (c->done) return;
  ctl_next_dt(c);
}

__global__ void ctl_step_kernel(Ctl* c) {
  if (c->done) return;
  c->t = c->clamped ? c->t_end : c->t + c->dt;
  c->dt_hist[c->step % kDtHist] = c->dt;
  c->step += 1;
  if (c->flag) {
    c->done = 1u;
    return;
  }
  if (!(c->t < c->t_end) || c->step >= c->max_steps) {
    c->done = 1u;
    return;
  }
  ctl_next_dt(c);
}

// ---- deterministic compensated totals -----------------------------------------

struct Acc {
  double s, c;
};

__device__ __forceinline__ Acc acc_add(Acc a, double x) {
  double t = a.s + x;
  double e = (fabs(a.s) >= fabs(x)) ? ((a.s - t) + x) : ((x - t) + a.s);
  return {t, a.c + e};
}
__device__ __forceinline__ Acc acc_merge(Acc a, Acc b) {
  Acc r = acc_add(a, b.s);
  r.c += b.c;
  return r;
}

constexpr int kMaxFields = 4 + kMaxSpecies;

// The field count is a template parameter so that the accumulators stay in
// registers (a runtime-indexed array would live in scratch memory).
template <int NT, int NF>
__device__ void block_merge(Acc (&v)[NF], Acc (*sh)[NT]) {
#pragma unroll
  for (int f = 0; f < NF; ++f) sh[f][threadIdx.x] = v[f];
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int f = 0; f < NF; ++f) sh[f][threadIdx.x] = acc_merge(sh[f][threadIdx.x], sh[f][threadIdx.x + w]);
    __syncthreads();
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) v[f] = sh[f][0];
}

template <typename T, int NF>
__global__ __launch_bounds__(256) void totals_partial_kernel(const T* __restrict__ U, long long plane,
                                                             double* __restrict__ part) {
  __shared__ Acc sh[NF][256];
  Acc v[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) v[f] = Acc{0, 0};
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < plane; q += stride)
#pragma unroll
    for (int f = 0; f < NF; ++f) v[f] = acc_add(v[f], double(U[f * plane + q]));
  block_merge<256, NF>(v, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      part[(blockIdx.x * kMaxFields + f) * 2 + 0] = v[f].s;
      part[(blockIdx.x * kMaxFields + f) * 2 + 1] = v[f].c;
    }
}

template <int NF>
__global__ __launch_bounds__(256) void totals_final_kernel(const double* __restrict__ part, int nblk, double area,
                                                           Ctl* ctl) {
  __shared__ Acc sh[NF][256];
  Acc v[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) v[f] = Acc{0, 0};
  for (int b = threadIdx.x; b < nblk; b += blockDim.x)
#pragma unroll
    for (int f = 0; f < NF; ++f)
      v[f] = acc_merge(v[f], Acc{part[(b * kMaxFields + f) * 2], part[(b * kMaxFields + f) * 2 + 1]});
  block_merge<256, NF>(v, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int f = 0; f < NF; ++f) ctl->totals[f] = (v[f].s + v[f].c) * area;
}

// ---- host launchers -----------------------------------------------------------

template <typename T, int MODE, int BCX, int BCY, int NS, bool CONS>
static hipError_t launch_stage_t(const Grid& g, const void* in, const void* base, void* out, double dt,
                                 Ctl* ctl, bool dt_dev, bool reduce, hipStream_t s) {
  StageArgs<T> a;
  a.in = static_cast<const T*>(in);
  a.base = static_cast<const T*>(base);
  a.out = static_cast<T*>(out);
  a.ctl = ctl;
  a.nx = g.nx;
  a.ny = g.ny;
  a.tiles_x = g.tiles_x;
  a.tiles_y = g.tiles_y;
  a.rows = g.rows_per_wave;
  a.blocks_x = g.blocks_x;
  a.blocks = g.blocks;
  a.blocks_pad = g.blocks_pad;
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
  hipLaunchKernelGGL((stage_kernel<T, MODE, BCX, BCY, NS, CONS>), dim3(g.blocks_pad),
                     dim3(kWave * waves_per_block<T>()), 0, s, a);
  return hipGetLastError();
}

template <typename T, int MODE, int BCX, int BCY>
static hipError_t launch_stage_ns(const Grid& g, const void* in, const void* base, void* out, double dt,
                                  Ctl* ctl, bool dt_dev, bool reduce, hipStream_t s) {
  static_assert(kMaxSpecies == 4, "one instantiation per species count");
  if (g.recon) return launch_stage_t<T, MODE, BCX, BCY, 0, true>(g, in, base, out, dt, ctl, dt_dev, reduce, s);
  switch (g.ns) {
    case 0: return launch_stage_t<T, MODE, BCX, BCY, 0, false>(g, in, base, out, dt, ctl, dt_dev, reduce, s);
    case 1: return launch_stage_t<T, MODE, BCX, BCY, 1, false>(g, in, base, out, dt, ctl, dt_dev, reduce, s);
    case 2: return launch_stage_t<T, MODE, BCX, BCY, 2, false>(g, in, base, out, dt, ctl, dt_dev, reduce, s);
    case 3: return launch_stage_t<T, MODE, BCX, BCY, 3, false>(g, in, base, out, dt, ctl, dt_dev, reduce, s);
    default: return launch_stage_t<T, MODE, BCX, BCY, 4, false>(g, in, base, out, dt, ctl, dt_dev, reduce, s);
  }
}

template <typename T, int MODE>
static hipError_t launch_stage_bc(const Grid& g, const void* in, const void* base, void* out, double dt,
                                  Ctl* ctl, bool dt_dev, bool reduce, hipStream_t s) {
  if (g.bc_x == kBcPeriodic) {
    if (g.bc_y == kBcPeriodic)
      return launch_stage_ns<T, MODE, kBcPeriodic, kBcPeriodic>(g, in, base, out, dt, ctl, dt_dev, reduce, s);
    return launch_stage_ns<T, MODE, kBcPeriodic, kBcTransmissive>(g, in, base, out, dt, ctl, dt_dev, reduce, s);
  }
  if (g.bc_y == kBcPeriodic)
    return launch_stage_ns<T, MODE, kBcTransmissive, kBcPeriodic>(g, in, base, out, dt, ctl, dt_dev, reduce, s);
  return launch_stage_ns<T, MODE, kBcTransmissive, kBcTransmissive>(g, in, base, out, dt, ctl, dt_dev, reduce, s);
}

template <typename T>
static hipError_t launch_stage_mode(const Grid& g, int mode, const void* in, const void* base, void* out,
                                    double dt, Ctl* ctl, bool dt_dev, bool reduce, hipStream_t s) {
  switch (mode) {
    case kResidual: return launch_stage_bc<T, kResidual>(g, in, base, out, dt, ctl, dt_dev, reduce, s);
    case kPredictor: return launch_stage_bc<T, kPredictor>(g, in, base, out, dt, ctl, dt_dev, reduce, s);
    default: return launch_stage_bc<T, kCorrector>(g, in, base, out, dt, ctl, dt_dev, reduce, s);
  }
}

hipError_t launch_stage(const Grid& g, int mode, const void* in, const void* base, void* out, double dt,
                        Ctl* ctl, bool dt_dev, bool reduce, hipStream_t s) {
  if (g.dtype == 0) return launch_stage_mode<double>(g, mode, in, base, out, dt, ctl, dt_dev, reduce, s);
  return launch_stage_mode<float>(g, mode, in, base, out, dt, ctl, dt_dev, reduce, s);
}

static int reduction_blocks(long long plane) {
  long long b = (plane + 255) / 256;
  if (b > 2048) b = 2048;
  return (int)(b < 1 ? 1 : b);
}

hipError_t launch_wavespeed(const Grid& g, const void* U, Ctl* ctl, hipStream_t s) {
  const long long plane = (long long)g.nx * g.ny;
  const int nb = reduction_blocks(plane);
  if (g.dtype == 0)
    hipLaunchKernelGGL(wavespeed_kernel<double>, dim3(nb), dim3(256), 0, s, static_cast<const double*>(U),
                       plane, g.gamma, g.gamma - 1.0, 1.0 / g.dx, 1.0 / g.dy, ctl);
  else
    hipLaunchKernelGGL(wavespeed_kernel<float>, dim3(nb), dim3(256), 0, s, static_cast<const float*>(U),
                       plane, float(g.gamma), float(g.gamma - 1.0), float(1.0 / g.dx), float(1.0 / g.dy), ctl);
  return hipGetLastError();
}

hipError_t launch_ctl_init(Ctl* ctl, double t0, double t_end, long long max_steps, double cfl,
                           hipStream_t s) {
  hipLaunchKernelGGL(ctl_init_kernel, dim3(1), dim3(1), 0, s, ctl, t0, t_end, max_steps, cfl);
  return hipGetLastError();
}

hipError_t launch_ctl_first(Ctl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(ctl_first_kernel, dim3(1), dim3(1), 0, s, ctl);
  return hipGetLastError();
}

hipError_t launch_ctl_step(Ctl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(ctl_step_kernel, dim3(1), dim3(1), 0, s, ctl);
  return hipGetLastError();
}

template <int NF>
static void launch_totals_nf(const Grid& g, const void* U, long long plane, double* part, int nblk, Ctl* ctl,
                             hipStream_t s) {
  if (g.dtype == 0)
    hipLaunchKernelGGL((totals_partial_kernel<double, NF>), dim3(nblk), dim3(256), 0, s,
                       static_cast<const double*>(U), plane, part);
  else
    hipLaunchKernelGGL((totals_partial_kernel<float, NF>), dim3(nblk), dim3(256), 0, s,
                       static_cast<const float*>(U), plane, part);
  hipLaunchKernelGGL((totals_final_kernel<NF>), dim3(1), dim3(256), 0, s, part, nblk, g.dx * g.dy, ctl);
}

hipError_t launch_totals(const Grid& g, const Layout& L, const void* U, void* ws, hipStream_t s) {
  const long long plane = (long long)g.nx * g.ny;
  char* w = static_cast<char*>(ws);
  double* part = reinterpret_cast<double*>(w + L.partials);
  Ctl* ctl = reinterpret_cast<Ctl*>(w + L.ctl);
  static_assert(kMaxSpecies == 4, "one instantiation per field count");
  switch (4 + g.ns) {
    case 4: launch_totals_nf<4>(g, U, plane, part, L.totals_blocks, ctl, s); break;
    case 5: launch_totals_nf<5>(g, U, plane, part, L.totals_blocks, ctl, s); break;
    case 6: launch_totals_nf<6>(g, U, plane, part, L.totals_blocks, ctl, s); break;
    case 7: launch_totals_nf<7>(g, U, plane, part, L.totals_blocks, ctl, s); break;
    default: launch_totals_nf<8>(g, U, plane, part, L.totals_blocks, ctl, s); break;
  }
  return hipGetLastError();
}

// ---- grid / workspace planning ------------------------------------------------

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

Grid make_grid(int nx, int ny, double dx, double dy, double gamma, double cfl, double beta, int bc_x,
               int bc_y, int dtype, int ns, int recon) {
  Grid g;
  g.ns = ns;
  g.recon = recon;
  g.nx = nx;
  g.ny = ny;
  g.dx = dx;
  g.dy = dy;
  g.gamma = gamma;
  g.cfl = cfl;
  g.beta = beta;
  g.bc_x = bc_x;
  g.bc_y = bc_y;
  g.dtype = dtype;
  g.tiles_x = (nx + kTileW - 1) / kTileW;
  // Rows per wave (strip height).  Longer strips amortise the 4 halo rows
  // and the strip prologue; shorter strips keep the rows that the resident
  // waves stream through close together, which the memory system rewards.
  // Measured on MI355X: 32 rows is best in FP64 and 64 in FP32 at 16384^2,
  // 16 and 32 at 8192^2, 16 in both at 4096^2 (2-9% faster stages there
  // than 32 rows): halve it, down to 16, until at least 64k waves (FP64)
  // or 32k (FP32) exist.
  // LF_STRIP_ROWS (a power of two, 4..4096) overrides the choice; it
  // changes the launch shape only, never the result.
  int r = dtype == 0 ? 32 : 64;
  const long long min_waves = dtype == 0 ? 65536 : 32768;
  while (r > 16 && (long long)g.tiles_x * ((ny + r - 1) / r) < min_waves) r /= 2;
  if (const char* env = getenv("LF_STRIP_ROWS")) {
    const int v = atoi(env);
    if (v >= 4 && v <= 4096 && (v & (v - 1)) == 0) r = v;
  }
  if (r > ny) r = ny;
  g.rows_per_wave = r;
  g.tiles_y = (ny + r - 1) / r;
  g.wpb = dtype == 0 ? waves_per_block<double>() : waves_per_block<float>();
  g.blocks_x = (g.tiles_x + g.wpb - 1) / g.wpb;
  g.blocks = g.blocks_x * g.tiles_y;
  g.blocks_pad = (g.blocks + kXcds - 1) / kXcds * kXcds;
  return g;
}

Layout make_layout(const Grid& g) {
  Layout L;
  const size_t esz = g.dtype == 0 ? sizeof(double) : sizeof(float);
  const size_t plane = (size_t)g.nx * (size_t)g.ny * esz;
  L.totals_blocks = reduction_blocks((long long)g.nx * g.ny);
  L.ustar = 0;
  // U* carries every field; the adjoint intermediate only the Euler ones
  // (the adjoint is defined for states without mass fractions)
  L.mu = align256(L.ustar + (4 + g.ns) * plane);
  L.ctl = align256(L.mu + 4 * plane);
  L.partials = align256(L.ctl + sizeof(Ctl));
  L.total = align256(L.partials + (size_t)L.totals_blocks * kMaxFields * 2 * sizeof(double));
  return L;
}

}  // namespace lf
