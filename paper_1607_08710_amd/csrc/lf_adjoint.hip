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

// ---- rows as buffer resources ---------------------------------------------
//
// One row of one field plane is a buffer resource: its base address and its
// length in bytes sit in scalar registers, and each lane adds its own byte
// offset, a loop-invariant vector register.  The hardware drops a store
// whose offset lies past the length (and a load there returns zero), so a
// lane that must not store gets an offset past the row instead of a branch
// around the store: the loop then has no path without stores, and the
// compiler can count the memory operations in flight exactly.
constexpr unsigned kOffNone = 0x80000000u;  // past any row: access dropped
// descriptor word 3 of a raw (untyped) gfx9 buffer: 32-bit data format
constexpr int kRawBufferWord3 = 0x00020000;

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const T* row, int n) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(row), 0, n * int(sizeof(T)), kRawBufferWord3);
}
typedef unsigned int U32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double buf_ld(double*, __amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ float buf_ld(float*, __amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U32x2, v), r, off, 0, 0);
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}
template <typename T>
__device__ __forceinline__ T ld_row(const T* row, int n, unsigned off) {
  return buf_ld((T*)nullptr, row_rsrc(row, n), off);
}
template <typename T>
__device__ __forceinline__ void st_row(T* row, int n, unsigned off, T v) {
  buf_st(row_rsrc(row, n), off, v);
}

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
// y-face frame (normal velocity v); then slot 0 comes back with acc0 (the
// running sum of its row) added.
template <typename T, bool YF>
__device__ __forceinline__ void face_slots(const P4<T>& w1, const SlopeD<T>& S1, const P4<T>& w2,
                                           const SlopeD<T>& S2, const Flux<T>& fb, T gamma, T inv_gm1,
                                           P4<T>& s0, P4<T>& s1, P4<T>& s2, P4<T>& s3,
                                           const P4<T>& acc0 = P4<T>{}) {
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
  // (y-faces: slot 0 is added straight into the accumulator acc0 of its
  // row, one fma instead of a product and an add)
  auto one = [&](T l, T r, T a1, T b1, T a2, T b2, T c0, T& o0, T& o1, T& o2, T& o3) {
    if constexpr (YF) o0 = fma(-a1, l, c0);
    else o0 = -a1 * l;
    o1 = fma(a1 - b1, l, fma(a2, r, l));
    o2 = fma(b1, l, fma(b2 - a2, r, r));
    o3 = -b2 * r;
  };
  one(lb.r, rb.r, S1.hda.r, S1.hdb.r, S2.hda.r, S2.hdb.r, acc0.r, s0.r, s1.r, s2.r, s3.r);
  one(lb.u, rb.u, S1.hda.u, S1.hdb.u, S2.hda.u, S2.hdb.u, acc0.u, s0.u, s1.u, s2.u, s3.u);
  one(lb.v, rb.v, S1.hda.v, S1.hdb.v, S2.hda.v, S2.hdb.v, acc0.v, s0.v, s1.v, s2.v, s3.v);
  one(lb.p, rb.p, S1.hda.p, S1.hdb.p, S2.hda.p, S2.hdb.p, acc0.p, s0.p, s1.p, s2.p, s3.p);
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
  // wave-uniform, and known to be (LDS bases derived from it can go to
  // scalar registers)
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
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

  // rows are buffer resources (see row_rsrc) addressed with the lane's byte
  // offset; output lanes hold columns 0 .. nx-1, where cm = c
  const unsigned boff = unsigned(cm) * sizeof(T);
  const unsigned soff = out_lane ? boff : kOffNone;
  // raw conservative values of U at (row, this lane's column)
  auto load_q = [&](int row) -> P4<T> {
    const T* rp = a.U + (long long)map_index<BCY>(row, ny) * nx;
    return {ld_row(rp, nx, boff), ld_row(rp + P, nx, boff), ld_row(rp + 2 * P, nx, boff),
            ld_row(rp + 3 * P, nx, boff)};
  };
  auto prim_of = [&](const P4<T>& q) { return prim4(q.r, q.u, q.v, q.p, gm1); };
  // cotangent of R at (row, this lane's column): zero outside a
  // transmissive domain (those cells do not exist)
  auto load_g = [&](int row) -> P4<T> {
    const bool in = (!YT || (row >= 0 && row < ny)) && (!XT || c_in);
    const T* rp = a.g + (long long)map_index<BCY>(row, ny) * nx;
    P4<T> g = {ld_row(rp, nx, boff), ld_row(rp + P, nx, boff), ld_row(rp + 2 * P, nx, boff),
               ld_row(rp + 3 * P, nx, boff)};
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
  // mode kAdjPred: lambda of the row an iteration outputs is copied from
  // memory straight into LDS at the top of the iteration (buffer loads with
  // the LDS flag: lane l's 32-bit word lands at M0 + 4 l), so that its
  // latency overlaps the iteration's arithmetic without holding registers.
  // All lanes copy their column (cm, in range); the halo lanes' values go
  // unused.  The compiler does not track these LDS writes: the reads wait
  // for them explicitly (lam_wait).
  constexpr int kDw = int(sizeof(T) / 4);  // 32-bit words per value
  __shared__ unsigned lam_lds[WPB][MODE == kAdjPred ? 4 : 1][kDw][kWave];
  auto fetch_lam = [&](int row) {
    if constexpr (MODE == kAdjPred) {
      const T* rp = a.lam + (long long)map_index<BCY>(row, ny) * nx;
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const __amdgpu_buffer_rsrc_t rs = row_rsrc(rp + f * P, nx);
#pragma unroll
        for (int h = 0; h < kDw; ++h)  // word h of the value: scalar offset 4 h
          __builtin_amdgcn_raw_ptr_buffer_load_lds(
              rs, (__attribute__((address_space(3))) void*)&lam_lds[w][f][h][0], 4, boff, 4 * h, 0, 0);
      }
    }
  };
  // every memory load of this wave complete: the copies above included
  auto lam_wait = [] { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); };
  auto lam_at = [&](int f) -> T {
    if constexpr (sizeof(T) == 8) {
      const unsigned long long lo = lam_lds[w][f][0][lane], hi = lam_lds[w][f][kDw - 1][lane];
      return __builtin_bit_cast(T, (hi << 32) | lo);
    } else {
      return __builtin_bit_cast(T, lam_lds[w][f][0][lane]);
    }
  };
  P4<T> Wm2 = prim_of(load_q(y0 - 3)), Wm1 = prim_of(load_q(y0 - 2)), W0 = prim_of(load_q(y0 - 1));
  // slope data of row y0-2 (rows y0-3 .. y0-1)
  put_slope(slope_d({Wm1.r - Wm2.r, Wm1.u - Wm2.u, Wm1.v - Wm2.v, Wm1.p - Wm2.p},
                    {W0.r - Wm1.r, W0.u - Wm1.u, W0.v - Wm1.v, W0.p - Wm1.p}, beta, hbeta));
  put_g(y0 - 2, load_g(y0 - 2));
  // In flight when the loop starts: U row k+1 and g row k of the first
  // iteration, then four stores that write nothing (an empty range).  The
  // loop is thus entered with the same memory operations in flight, in the
  // same order, as it goes round with (a U row, a g row, a row's four
  // stores).  The compiler counts the operations in flight over both ways
  // into the loop and keeps the smaller count, so any difference here would
  // make the loop's waits for its loads also wait for the stores of the
  // row before (a drain of every access in flight at the top of each row).
  P4<T> Qn = load_q(y0);
  __builtin_amdgcn_sched_barrier(0);
  P4<T> Gn = load_g(y0 - 1);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int f = 0; f < 4; ++f) st_row(a.out + f * P, 0, soff, T(0));  // four distinct stores
  const P4<T> Z = {T(0), T(0), T(0), T(0)};
  P4<T> Am2 = Z, Am1 = Z, A0 = Z;  // accumulators for rows k-2, k-1, k
  P4<T> ghost_lo = Z;              // transmissive: slots aimed at rows < 0

#pragma unroll 1
  for (int k = y0 - 1; k <= y1 + 1; ++k) {
    // new data: prim row k+1, g row k (loaded last iteration); then the
    // loads for the next iteration (rows past the strip are mapped like
    // any other row and simply not used).  Everything this iteration reads
    // from LDS is read here, at the top, so that the reads' latency
    // overlaps the arithmetic.
    const SlopeD<T> Sk1 = get_slope();
    const P4<T> W1 = prim_of(Qn);
    const P4<T> Gk = Gn;
    const P4<T> Gm1 = get_g(k - 1);
    const P4<T> Gm2 = get_g(k - 2);  // row r = k-2 (its x-faces, below)
    fetch_lam(k - 2);
    Qn = load_q(k + 2);
    put_g(k, Gk);
    Gn = load_g(k + 1);
    // slopes of rows k-1 (rows k-2, k-1, k; carried) and k (rows k-1, k,
    // k+1)
    const SlopeD<T> Sk = slope_d({W0.r - Wm1.r, W0.u - Wm1.u, W0.v - Wm1.v, W0.p - Wm1.p},
                                 {W1.r - W0.r, W1.u - W0.u, W1.v - W0.v, W1.p - W0.p}, beta, hbeta);
    put_slope(Sk);
    P4<T> A1 = Z;  // accumulator of row k+1 starts here
    // ---- y-face k (between rows k-1 and k) ----
    if (!YT || (k >= 0 && k <= ny)) {
      const Flux<T> fb = {(Gm1.r - Gk.r) * a.idy, (Gm1.v - Gk.v) * a.idy, (Gm1.u - Gk.u) * a.idy,
                          (Gm1.p - Gk.p) * a.idy};
      P4<T> s0, s1, s2, s3;
      face_slots<T, true>(Wm1, Sk1, W0, Sk, fb, gam, igm1, s0, s1, s2, s3, Am2);
      Am2 = s0;  // the accumulator of row k-2 with slot 0 added
      Am1 = p4_add(Am1, s1);
      A0 = p4_add(A0, s2);
      A1 = s3;
    }
    // ---- row r = k-2 is complete in y ----
    const int r = k - 2;
    if constexpr (YT) {
      if (r < 0) ghost_lo = p4_add(ghost_lo, Am2);
    }
    // results of row r; rows below the strip (the first three iterations)
    // have none, and their stores below are dropped
    T res[4] = {T(0), T(0), T(0), T(0)};
    if (r >= y0) {
      P4<T> tot = Am2;
      if constexpr (YT) {
        if (r == 0) tot = p4_add(tot, ghost_lo);
        if (r == ny - 1) tot = p4_add(tot, p4_add(Am1, A0));  // rows ny, ny+1 are ghosts
      }
      // x-faces of row r across the lanes (Wm2 = prim row r)
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
      // (products written as fmas, the build does not contract, except in
      // the sums over the two directions, which keep the x <-> y mirror
      // symmetry exact)
      const T ir = rcp(Wm2.r);
      const T u = Wm2.u, v = Wm2.v;
      const T gp = gm1 * tot.p;
      T vv[4];
      vv[0] = fma(T(0.5) * gp, u * u + v * v, fma(-(u * tot.u + v * tot.v), ir, tot.r));
      vv[1] = fma(-gp, u, tot.u * ir);
      vv[2] = fma(-gp, v, tot.v * ir);
      vv[3] = gp;
      const T gg[4] = {Gm2.r, Gm2.u, Gm2.v, Gm2.p};
      if constexpr (MODE == kAdjPred) lam_wait();
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        if constexpr (MODE == kVjp) {
          res[f] = vv[f];
        } else if constexpr (MODE == kAdjCorr) {
          res[f] = T(0.5 * fma(-a.dt, double(vv[f]), double(gg[f])));  // mu = (lam - dt v)/2
        } else {
          const T lam = lam_at(f);  // lam/2 + mu - dt v
          res[f] = T(fma(0.5, double(lam), fma(-a.dt, double(vv[f]), double(gg[f]))));
        }
      }
    }
    {
      // stored straight from the lanes (the kernel is bound by arithmetic,
      // and without staging no block barrier ties its waves together).  The
      // stores are issued in every iteration, outside the branch above, so
      // that no path through the loop lacks them and the compiler's count
      // of memory operations in flight never makes a load wait for them;
      // the halo lanes' stores are dropped (soff), and so are all of them
      // in the rows below the strip (an empty range)
      const bool mine = r >= y0;
      const long long roff = (long long)(mine ? r : y0) * nx;
      const int len = mine ? nx : 0;
#pragma unroll
      for (int f = 0; f < 4; ++f) st_row(a.out + roff + f * P, len, soff, res[f]);
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
  // strip height: 32 rows, halved (to 8) until about 8k waves exist: the
  // best measured at 4096^2 (32 rows: 2-5% faster than 16, 24 or 48 in
  // both precisions) and at 8192^2; LF_ADJ_ROWS (4..4096) overrides it
  // (launch shape only)
  const int tiles_x = (g.nx + kAdjTileW - 1) / kAdjTileW;
  const long long min_waves = 8192;
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
