// lf_adjoint.hip -- transpose of the residual's Jacobian, v = J_R(U)^T g,
// in gather form (no atomics), and the two adjoint stages of the Heun step.
//
// R_i = (F_{i+1/2} - F_{i-1/2})/dx + (G_{j+1/2} - G_{j-1/2})/dy, and the flux
// through x-face k (between cells k-1 and k) depends on the primitive
// states of cells k-2 .. k+1 (MUSCL slopes of k-1 and k).  The face's
// cotangent is (g_{k-1} - g_k)/dx; pulled back through eq. (12), eqs.
// (13)-(14) and the limited reconstruction (eq. (sweby)) it yields four
// "slot" contributions, to the primitive variables of cells k-2 .. k+1.
// A cell collects the slots of x-faces k = i-1 .. i+2 and of the same four
// y-faces, then its primitive cotangent goes through the perfect-gas law
// onto its conservative variables.
//
// Kernel layout (same idea as the forward stage kernel).  A wave owns 64
// consecutive columns and produces the middle 58 (the adjoint stencil
// reaches three cells to each side); it marches up a strip of rows.  Every
// face is evaluated once per wave: x-faces across the lanes, with the slot
// contributions moved to their cells by DPP shifts; y-faces one per row,
// with the slot contributions accumulated in a four-row register window.
// A row is finished when its last y-face (two rows above it) has been
// processed; its results are stored straight from the lanes.
//
// Boundaries.  Transmissive: ghost cells copy the edge cell, so the slots
// that point at ghost cells are folded onto the edge cell; faces beyond the
// boundary do not exist (their cotangent is zero: g is zero outside).
// Periodic: the stencil data wrap, faces are indexed in unwrapped
// coordinates and each (cell, face) pair is visited exactly once.
#include <stdlib.h>

#include "lf_internal.h"

namespace lf {

constexpr int kAdjHalo = 3;
// Waves per block, both precisions.  FP32 (~136 VGPRs) fits three waves
// per SIMD, twelve per CU: blocks of four fill that, blocks of eight leave
// room for one block only (eight waves; measured 12% slower at 4096^2).
constexpr int kAdjWaves = 4;
constexpr int kAdjTileW = kWave - 2 * kAdjHalo;  // 58 output columns per wave

template <typename T>
struct AdjArgs {
  const T* U;    // state at which J_R is taken
  const T* g;    // cotangent of R
  const T* lam;  // lambda^{n+1} (mode kAdjPred)
  T* out;
  int nx, ny;
  int rows;      // strip height
  int blocks_x, blocks, blocks_pad;
  long long plane;
  T gamma, gm1, inv_gm1, beta, hbeta, idx, idy;
  double dt;
};

template <typename T>
struct P4 {
  T r, u, v, p;
};

template <typename T>
__device__ __forceinline__ P4<T> p4_shl(const P4<T>& a) {
  return {shl1(a.r), shl1(a.u), shl1(a.v), shl1(a.p)};
}
template <typename T>
__device__ __forceinline__ P4<T> p4_shr(const P4<T>& a) {
  return {shr1(a.r), shr1(a.u), shr1(a.v), shr1(a.p)};
}
template <typename T>
__device__ __forceinline__ P4<T> p4_add(const P4<T>& a, const P4<T>& b) {
  return {a.r + b.r, a.u + b.u, a.v + b.v, a.p + b.p};
}
template <typename T>
__device__ __forceinline__ P4<T> p4_sel(bool c, const P4<T>& a) {
  return {c ? a.r : T(0), c ? a.u : T(0), c ? a.v : T(0), c ? a.p : T(0)};
}

// Slope of one cell and half its partial derivatives w.r.t. the backward
// and forward differences (hda, hdb), for the four primitive variables.
template <typename T>
struct SlopeD {
  P4<T> s, hda, hdb;
};

template <typename T>
__device__ __forceinline__ SlopeD<T> slope_d(const P4<T>& dm, const P4<T>& dp, T beta, T hbeta) {
  SlopeD<T> o;
  sweby_all(dm.r, dp.r, beta, hbeta, o.s.r, o.hda.r, o.hdb.r);
  sweby_all(dm.u, dp.u, beta, hbeta, o.s.u, o.hda.u, o.hdb.u);
  sweby_all(dm.v, dp.v, beta, hbeta, o.s.v, o.hda.v, o.hdb.v);
  sweby_all(dm.p, dp.p, beta, hbeta, o.s.p, o.hda.p, o.hdb.p);
  return o;
}

// One face: left cell state w1 with slope data S1 (cell k-1), right cell
// w2 with S2 (cell k); fb the flux cotangent in the face frame.  Returns
// the four slot contributions in (rho, u, v, p) order.  YF selects the
// y-face frame (normal velocity v).
template <typename T, bool YF>
__device__ __forceinline__ void face_slots(const P4<T>& w1, const SlopeD<T>& S1, const P4<T>& w2,
                                           const SlopeD<T>& S2, const Flux<T>& fb, T gamma, T inv_gm1,
                                           P4<T>& s0, P4<T>& s1, P4<T>& s2, P4<T>& s3) {
  const T h = T(0.5);
  const P4<T> L = {fma(h, S1.s.r, w1.r), fma(h, S1.s.u, w1.u), fma(h, S1.s.v, w1.v), fma(h, S1.s.p, w1.p)};
  const P4<T> R = {fma(-h, S2.s.r, w2.r), fma(-h, S2.s.u, w2.u), fma(-h, S2.s.v, w2.v), fma(-h, S2.s.p, w2.p)};
  FaceState<T> FL, FR, Lb, Rb;
  if constexpr (YF) {
    FL = {L.r, L.v, L.u, L.p};
    FR = {R.r, R.v, R.u, R.p};
  } else {
    FL = {L.r, L.u, L.v, L.p};
    FR = {R.r, R.u, R.v, R.p};
  }
  face_flux_vjp(FL, FR, gamma, inv_gm1, fb, Lb, Rb);
  P4<T> lb, rb;
  if constexpr (YF) {
    lb = {Lb.r, Lb.ut, Lb.un, Lb.p};
    rb = {Rb.r, Rb.ut, Rb.un, Rb.p};
  } else {
    lb = {Lb.r, Lb.un, Lb.ut, Lb.p};
    rb = {Rb.r, Rb.un, Rb.ut, Rb.p};
  }
  // w^L = w1 + phi(w1 - w0, w2 - w1)/2,  w^R = w2 - phi(w2 - w1, w3 - w2)/2;
  // a1, b1 (a2, b2): half partials of the left (right) cell's slope
  auto one = [&](T l, T r, T a1, T b1, T a2, T b2, T& o0, T& o1, T& o2, T& o3) {
    o0 = -a1 * l;
    o1 = fma(a1 - b1, l, fma(a2, r, l));
    o2 = fma(b1, l, fma(b2 - a2, r, r));
    o3 = -b2 * r;
  };
  one(lb.r, rb.r, S1.hda.r, S1.hdb.r, S2.hda.r, S2.hdb.r, s0.r, s1.r, s2.r, s3.r);
  one(lb.u, rb.u, S1.hda.u, S1.hdb.u, S2.hda.u, S2.hdb.u, s0.u, s1.u, s2.u, s3.u);
  one(lb.v, rb.v, S1.hda.v, S1.hdb.v, S2.hda.v, S2.hdb.v, s0.v, s1.v, s2.v, s3.v);
  one(lb.p, rb.p, S1.hda.p, S1.hdb.p, S2.hda.p, S2.hdb.p, s0.p, s1.p, s2.p, s3.p);
}

template <typename T>
__device__ __forceinline__ P4<T> prim4(T q0, T q1, T q2, T q3, T gm1) {
  Prim<T> w = to_prim(q0, q1, q2, q3, gm1);
  return {w.r, w.u, w.v, w.p};
}

// At least two waves per SIMD: without the bound the FP64 variants spill
// past 256 registers into AGPRs and drop to one wave.
template <typename T, int MODE, int BCX, int BCY>
__global__ __launch_bounds__(kWave * kAdjWaves, 8 / kAdjWaves)
void adjoint_kernel(AdjArgs<T> a) {
  constexpr int WPB = kAdjWaves;
  constexpr bool XT = BCX == kBcTransmissive;
  constexpr bool YT = BCY == kBcTransmissive;
  const int lb_ = xcd_block(blockIdx.x, a.blocks_pad);
  if (lb_ >= a.blocks) return;  // whole block
  const int by = lb_ / a.blocks_x;
  const int bx = lb_ - by * a.blocks_x;
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & (kWave - 1);
  const int nx = a.nx, ny = a.ny;
  const int c = (bx * WPB + w) * kAdjTileW - kAdjHalo + lane;  // unwrapped column of this lane
  const int cm = map_index<BCX>(c, nx);
  const bool c_in = c >= 0 && c < nx;
  const bool out_lane = lane >= kAdjHalo && lane < kWave - kAdjHalo && c < nx;
  // x-face computed by this lane: k = c + 1, between columns c and c + 1
  const bool xface = !XT || (c >= -1 && c <= nx - 1);
  const int y0 = by * a.rows;
  const int y1 = min(y0 + a.rows, ny);
  const long long P = a.plane;
  const T gm1 = a.gm1, gam = a.gamma, igm1 = a.inv_gm1, beta = a.beta, hbeta = a.hbeta;

  // rows are addressed as a uniform row pointer (scalar registers) plus
  // the lane's byte offset (see ld_lane)
  const unsigned boff = unsigned(cm) * sizeof(T);
  // raw conservative values of U at (row, this lane's column)
  auto load_q = [&](int row) -> P4<T> {
    const T* rp = a.U + (long long)map_index<BCY>(row, ny) * nx;
    const unsigned bo = lane_offset(rp, boff);
    return {ld_lane(rp, bo), ld_lane(rp + P, bo), ld_lane(rp + 2 * P, bo), ld_lane(rp + 3 * P, bo)};
  };
  auto prim_of = [&](const P4<T>& q) { return prim4(q.r, q.u, q.v, q.p, gm1); };
  // cotangent of R at (row, this lane's column): zero outside a
  // transmissive domain (those cells do not exist)
  auto load_g = [&](int row) -> P4<T> {
    const bool in = (!YT || (row >= 0 && row < ny)) && (!XT || c_in);
    const T* rp = a.g + (long long)map_index<BCY>(row, ny) * nx;
    const unsigned bo = lane_offset(rp, boff);
    P4<T> g = {ld_lane(rp, bo), ld_lane(rp + P, bo), ld_lane(rp + 2 * P, bo), ld_lane(rp + 3 * P, bo)};
    return p4_sel(in, g);
  };

  // window: prim rows k-2 .. k+1, y-accumulators rows k-2 .. k+1 (slots
  // rotate every row).  The rows of U and g an iteration uses were loaded
  // one iteration earlier, so that their memory latency overlaps a whole
  // row of arithmetic.  Per-wave LDS holds, for each lane, the slope data
  // of row k (value and half partials; row k-1's in the next iteration)
  // and the last three rows of g (rows k-2 .. k: the y-face and the x-faces
  // of row k-2 read them back).  Each lane reads back its own values, so
  // no barrier is needed; the slope data are stored as soon as they are
  // formed, so that they occupy no registers across the rest of the
  // iteration.
  __shared__ T scarry[WPB][12][kWave];
  __shared__ T gring[WPB][3][4][kWave];
  T(*my_c)[kWave] = scarry[w];
  auto put_slope = [&](const SlopeD<T>& S) {
    const T v[12] = {S.s.r, S.s.u, S.s.v, S.s.p, S.hda.r, S.hda.u, S.hda.v, S.hda.p,
                     S.hdb.r, S.hdb.u, S.hdb.v, S.hdb.p};
#pragma unroll
    for (int i = 0; i < 12; ++i) my_c[i][lane] = v[i];
  };
  // read through volatile LDS pointers: otherwise the compiler forwards
  // the stored values and keeps them in registers across the iteration
  using LdsV = __attribute__((address_space(3))) volatile T;
  LdsV* my_v = (LdsV*)&scarry[w][0][lane];
  auto get_slope = [&]() {
    SlopeD<T> S;
    S.s = {my_v[0 * kWave], my_v[1 * kWave], my_v[2 * kWave], my_v[3 * kWave]};
    S.hda = {my_v[4 * kWave], my_v[5 * kWave], my_v[6 * kWave], my_v[7 * kWave]};
    S.hdb = {my_v[8 * kWave], my_v[9 * kWave], my_v[10 * kWave], my_v[11 * kWave]};
    return S;
  };
  auto gslot = [](int row) { return (row % 3 + 3) % 3; };
  auto put_g = [&](int row, const P4<T>& g) {
    T(*sl)[kWave] = gring[w][gslot(row)];
    sl[0][lane] = g.r;
    sl[1][lane] = g.u;
    sl[2][lane] = g.v;
    sl[3][lane] = g.p;
  };
  auto get_g = [&](int row) -> P4<T> {
    LdsV* gv = (LdsV*)&gring[w][gslot(row)][0][lane];
    return {gv[0], gv[kWave], gv[2 * kWave], gv[3 * kWave]};
  };
  P4<T> Wm2 = prim_of(load_q(y0 - 3)), Wm1 = prim_of(load_q(y0 - 2)), W0 = prim_of(load_q(y0 - 1));
  // slope data of row y0-2 (rows y0-3 .. y0-1)
  put_slope(slope_d({Wm1.r - Wm2.r, Wm1.u - Wm2.u, Wm1.v - Wm2.v, Wm1.p - Wm2.p},
                    {W0.r - Wm1.r, W0.u - Wm1.u, W0.v - Wm1.v, W0.p - Wm1.p}, beta, hbeta));
  put_g(y0 - 2, load_g(y0 - 2));
  // in flight: U row k+1 and g row k of the first iteration
  P4<T> Qn = load_q(y0), Gn = load_g(y0 - 1);
  const P4<T> Z = {T(0), T(0), T(0), T(0)};
  P4<T> Am2 = Z, Am1 = Z, A0 = Z;  // accumulators for rows k-2, k-1, k
  P4<T> ghost_lo = Z;              // transmissive: slots aimed at rows < 0

#pragma unroll 1
  for (int k = y0 - 1; k <= y1 + 1; ++k) {
    // new data: prim row k+1, g row k (loaded last iteration); then the
    // loads for the next iteration (rows past the strip are mapped like
    // any other row and simply not used)
    const P4<T> W1 = prim_of(Qn);
    const P4<T> Gk = Gn;
    const P4<T> Gm1 = get_g(k - 1);
    put_g(k, Gk);
    Qn = load_q(k + 2);
    Gn = load_g(k + 1);
    // slopes of rows k-1 (rows k-2, k-1, k; carried) and k (rows k-1, k,
    // k+1)
    const SlopeD<T> Sk1 = get_slope();
    const SlopeD<T> Sk = slope_d({W0.r - Wm1.r, W0.u - Wm1.u, W0.v - Wm1.v, W0.p - Wm1.p},
                                 {W1.r - W0.r, W1.u - W0.u, W1.v - W0.v, W1.p - W0.p}, beta, hbeta);
    put_slope(Sk);
    P4<T> A1 = Z;  // accumulator of row k+1 starts here
    // ---- y-face k (between rows k-1 and k) ----
    if (!YT || (k >= 0 && k <= ny)) {
      const Flux<T> fb = {(Gm1.r - Gk.r) * a.idy, (Gm1.v - Gk.v) * a.idy, (Gm1.u - Gk.u) * a.idy,
                          (Gm1.p - Gk.p) * a.idy};
      P4<T> s0, s1, s2, s3;
      face_slots<T, true>(Wm1, Sk1, W0, Sk, fb, gam, igm1, s0, s1, s2, s3);
      Am2 = p4_add(Am2, s0);
      Am1 = p4_add(Am1, s1);
      A0 = p4_add(A0, s2);
      A1 = s3;
    }
    // ---- row r = k-2 is complete in y ----
    const int r = k - 2;
    if constexpr (YT) {
      if (r < 0) ghost_lo = p4_add(ghost_lo, Am2);
    }
    if (r >= y0) {
      P4<T> tot = Am2;
      if constexpr (YT) {
        if (r == 0) tot = p4_add(tot, ghost_lo);
        if (r == ny - 1) tot = p4_add(tot, p4_add(Am1, A0));  // rows ny, ny+1 are ghosts
      }
      // x-faces of row r across the lanes (Wm2 = prim row r)
      const P4<T> Gm2 = get_g(r);
      const P4<T> wr1 = p4_shl(Wm2);
      const P4<T> dxp = {wr1.r - Wm2.r, wr1.u - Wm2.u, wr1.v - Wm2.v, wr1.p - Wm2.p};
      const P4<T> dxm = p4_shr(dxp);
      const SlopeD<T> Sx = slope_d(dxm, dxp, beta, hbeta);
      SlopeD<T> Sx1;
      Sx1.s = p4_shl(Sx.s);
      Sx1.hda = p4_shl(Sx.hda);
      Sx1.hdb = p4_shl(Sx.hdb);
      const P4<T> g1 = p4_shl(Gm2);
      const Flux<T> fb = {(Gm2.r - g1.r) * a.idx, (Gm2.u - g1.u) * a.idx, (Gm2.v - g1.v) * a.idx,
                          (Gm2.p - g1.p) * a.idx};
      P4<T> s0, s1, s2, s3;
      face_slots<T, false>(Wm2, Sx, wr1, Sx1, fb, gam, igm1, s0, s1, s2, s3);
      // a face that does not exist contributes nothing (select, not
      // multiply: halo lanes may hold non-finite intermediates)
      s0 = p4_sel(xface, s0);
      s1 = p4_sel(xface, s1);
      s2 = p4_sel(xface, s2);
      s3 = p4_sel(xface, s3);
      // lane c collects slot 0 of the face at lane c+1, slot 1 of its own,
      // slot 2 of lane c-1 and slot 3 of lane c-2
      P4<T> tx = p4_add(p4_add(p4_shl(s0), s1), p4_shr(p4_add(s2, p4_shr(s3))));
      if constexpr (XT) {
        // ghost columns -1, -2 fold onto column 0; nx, nx+1 onto nx-1
        const P4<T> l1 = p4_shr(tx), l2 = p4_shr(l1);
        const P4<T> r1 = p4_shl(tx), r2 = p4_shl(r1);
        if (c == 0) tx = p4_add(tx, p4_add(l1, l2));
        if (c == nx - 1) tx = p4_add(tx, p4_add(r1, r2));
      }
      tot = p4_add(tot, tx);
      // primitive -> conservative: v = (dw/dU)^T wbar
      const T ir = rcp(Wm2.r);
      const T u = Wm2.u, v = Wm2.v;
      T vv[4];
      vv[0] = tot.r - (u * tot.u + v * tot.v) * ir + gm1 * T(0.5) * (u * u + v * v) * tot.p;
      vv[1] = tot.u * ir - gm1 * u * tot.p;
      vv[2] = tot.v * ir - gm1 * v * tot.p;
      vv[3] = gm1 * tot.p;
      const T gg[4] = {Gm2.r, Gm2.u, Gm2.v, Gm2.p};
      T res[4];
      // output lanes hold columns 0 .. nx-1, where cm = c
      const long long roff = (long long)r * nx;
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        if constexpr (MODE == kVjp) {
          res[f] = vv[f];
        } else if constexpr (MODE == kAdjCorr) {
          res[f] = T(0.5 * (double(gg[f]) - a.dt * double(vv[f])));  // mu = (lam - dt v)/2
        } else {
          const T* lp = a.lam + roff + f * P;
          const T lam = out_lane ? ld_lane(lp, lane_offset(lp, boff)) : T(0);  // lam/2 + mu - dt v
          res[f] = T(0.5 * double(lam) + double(gg[f]) - a.dt * double(vv[f]));
        }
      }
      // stored straight from the lanes: the kernel is bound by arithmetic,
      // and without staging no block barrier ties its waves together
      if (out_lane) {
        T* op = a.out + roff;
        const unsigned bo = lane_offset(op, boff);
#pragma unroll
        for (int f = 0; f < 4; ++f) st_lane(op + f * P, bo, res[f]);
      }
    }
    // slide the window
    Wm2 = Wm1;
    Wm1 = W0;
    W0 = W1;
    Am2 = Am1;
    Am1 = A0;
    A0 = A1;
  }
}

template <typename T, int MODE, int BCX, int BCY>
static hipError_t launch_adj_t(const Grid& g, const void* U, const void* gv, const void* lam, void* out,
                               double dt, hipStream_t s) {
  constexpr int WPB = kAdjWaves;
  AdjArgs<T> a;
  a.U = static_cast<const T*>(U);
  a.g = static_cast<const T*>(gv);
  a.lam = static_cast<const T*>(lam);
  a.out = static_cast<T*>(out);
  a.nx = g.nx;
  a.ny = g.ny;
  a.plane = (long long)g.nx * g.ny;
  a.gamma = T(g.gamma);
  a.gm1 = T(g.gamma - 1.0);
  a.inv_gm1 = T(1.0 / (g.gamma - 1.0));
  a.beta = T(g.beta);
  a.hbeta = T(0.5 * g.beta);
  a.idx = T(1.0 / g.dx);
  a.idy = T(1.0 / g.dy);
  a.dt = dt;
  // strip height: 32 rows, halved (to 8) until about 8k waves (FP64) or
  // 16k waves (FP32) exist: the best measured at 4096^2 (32 rows in FP64,
  // 2% faster than 16; 16 rows in FP32, 2% faster than 32) and at 8192^2
  // (32 rows); LF_ADJ_ROWS (4..4096) overrides it (launch shape only)
  const int tiles_x = (g.nx + kAdjTileW - 1) / kAdjTileW;
  const long long min_waves = sizeof(T) == 8 ? 8192 : 16384;
  int r = 32;
  while (r > 8 && (long long)tiles_x * ((g.ny + r - 1) / r) < min_waves) r /= 2;
  if (const char* env = getenv("LF_ADJ_ROWS")) {
    const int v = atoi(env);
    if (v >= 4 && v <= 4096) r = v;
  }
  if (r > g.ny) r = g.ny;
  a.rows = r;
  const int tiles_y = (g.ny + r - 1) / r;
  a.blocks_x = (tiles_x + WPB - 1) / WPB;
  a.blocks = a.blocks_x * tiles_y;
  a.blocks_pad = (a.blocks + kXcds - 1) / kXcds * kXcds;
  hipLaunchKernelGGL((adjoint_kernel<T, MODE, BCX, BCY>), dim3(a.blocks_pad), dim3(kWave * WPB), 0, s, a);
  return hipGetLastError();
}

template <typename T, int MODE>
static hipError_t launch_adj_bc(const Grid& g, const void* U, const void* gv, const void* lam, void* out,
                                double dt, hipStream_t s) {
  if (g.bc_x == kBcPeriodic) {
    if (g.bc_y == kBcPeriodic) return launch_adj_t<T, MODE, kBcPeriodic, kBcPeriodic>(g, U, gv, lam, out, dt, s);
    return launch_adj_t<T, MODE, kBcPeriodic, kBcTransmissive>(g, U, gv, lam, out, dt, s);
  }
  if (g.bc_y == kBcPeriodic) return launch_adj_t<T, MODE, kBcTransmissive, kBcPeriodic>(g, U, gv, lam, out, dt, s);
  return launch_adj_t<T, MODE, kBcTransmissive, kBcTransmissive>(g, U, gv, lam, out, dt, s);
}

template <typename T>
static hipError_t launch_adj_mode(const Grid& g, int mode, const void* U, const void* gv, const void* lam,
                                  void* out, double dt, hipStream_t s) {
  switch (mode) {
    case kVjp: return launch_adj_bc<T, kVjp>(g, U, gv, lam, out, dt, s);
    case kAdjCorr: return launch_adj_bc<T, kAdjCorr>(g, U, gv, lam, out, dt, s);
    default: return launch_adj_bc<T, kAdjPred>(g, U, gv, lam, out, dt, s);
  }
}

hipError_t launch_adjoint(const Grid& g, int mode, const void* U, const void* gvec, const void* lam,
                          void* out, double dt, hipStream_t s) {
  if (g.dtype == 0) return launch_adj_mode<double>(g, mode, U, gvec, lam, out, dt, s);
  return launch_adj_mode<float>(g, mode, U, gvec, lam, out, dt, s);
}

}  // namespace lf
