// lf_device.h -- device-side building blocks of the gfx950 Lagrange-flux
// kernels (De Vuyst et al., arXiv:1607.08710).  Everything here is
// templated on the arithmetic type T (double or float) and is inlined into
// the stage and adjoint kernels.
//
// The x- and y-faces call the same face routine with the frame
// (rho, u_n, u_t, p), so the two directions execute identical arithmetic.
// No floating-point contraction is left to the compiler (built with
// -ffp-contract=off); every fused multiply-add below is explicit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lf {

constexpr int kWave = 64;        // wavefront width on CDNA
constexpr int kHalo = 2;         // stencil half-width along each axis
constexpr int kTileW = kWave - 2 * kHalo;  // output columns per wave (60)
// Waves per stage-kernel block: the block's tiles cover 60 * waves
// consecutive columns, i.e. exactly 15 cache lines of 128 bytes in either
// precision (240 doubles or 480 floats), so its stores can be line-aligned.
template <typename T>
constexpr int waves_per_block() { return sizeof(T) == 8 ? 4 : 8; }
constexpr int kXcds = 8;         // MI355X: 8 accelerator complex dies
constexpr int kDtHist = 4096;    // per-step dt records kept on the device
constexpr int kMaxSpecies = 4;   // passive mass fractions a state may carry

// y-boundaries; kBcGhost (single-pass step of a strip of a larger grid
// only): the kGhostRows rows beyond each end of the strip are read from
// caller-supplied ghost rows.
enum : int { kBcPeriodic = 0, kBcTransmissive = 1, kBcGhost = 2 };
constexpr int kGhostRows = 4;

// Stage kernel modes.
enum StageMode : int { kResidual = 0, kPredictor = 1, kCorrector = 2 };

// Device control block, stored at the start of the control area of the
// workspace.  dt and t of the time loop live here so that the loop never
// round-trips to the host between steps.
struct Ctl {
  unsigned long long smax;   // max wave speed of the last reduced state, as
                             // the bit pattern of a non-negative double
  unsigned int flag;         // non-zero once a non-physical state was seen
  unsigned int done;         // non-zero once the time loop has finished
  double dt;                 // time step of the step in flight
  double t;                  // time at the start of the step in flight
  double t_end;
  long long step;            // completed steps
  long long max_steps;
  double cfl;
  unsigned int clamped;      // the step in flight was clamped to t_end
  unsigned int pad;
  double totals[4 + kMaxSpecies];  // result of the conservation-totals reduction
  double dt_hist[kDtHist];   // dt of step k stored at k % kDtHist
};

// ---- boundary index mapping ------------------------------------------------

template <int BC>
__device__ __forceinline__ int map_index(int k, int n) {
  static_assert(BC == kBcPeriodic || BC == kBcTransmissive, "ghost rows are not an index mapping");
  if constexpr (BC == kBcPeriodic) {
    k %= n;
    return k < 0 ? k + n : k;
  } else {
    return k < 0 ? 0 : (k >= n ? n - 1 : k);
  }
}

// ---- cross-lane shifts (DPP whole-wave shifts, all 64 lanes active) -------

// Lane l receives the value of lane l-1 (lane 0 receives 0).
__device__ __forceinline__ int shr1_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true);
}
// Lane l receives the value of lane l+1 (lane 63 receives 0).
__device__ __forceinline__ int shl1_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true);
}

__device__ __forceinline__ double shr1(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(shr1_i(hi), shr1_i(lo));
}
__device__ __forceinline__ double shl1(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(shl1_i(hi), shl1_i(lo));
}
__device__ __forceinline__ float shr1(float v) {
  return __int_as_float(shr1_i(__float_as_int(v)));
}
__device__ __forceinline__ float shl1(float v) {
  return __int_as_float(shl1_i(__float_as_int(v)));
}

// ---- row access: uniform row address plus the lane's byte offset ----------
//
// A row's address is the same in every lane and is held in scalar
// registers; each lane adds a 32-bit byte offset, which the global load and
// store instructions take as a separate operand, so no per-lane 64-bit
// address is formed.  The empty asm statements emit no instruction; they
// keep the compiler from folding the lane's loop-invariant offset into a
// per-lane 64-bit base outside the row loop (it would then add every row's
// offset with vector instructions).  lane_offset() re-forms the offset for
// one row (one register move, shared by the row's fields); ld_lane() and
// st_lane() take the row address, which must be uniform, in scalar
// registers.

#define LF_GLOBAL __attribute__((address_space(1)))

template <typename T>
__device__ __forceinline__ unsigned lane_offset(const T* row, unsigned boff) {
  asm("" : "+v"(boff) : "s"(row));
  return boff;
}
template <typename T>
__device__ __forceinline__ T ld_lane(const T* row, unsigned boff) {
  const LF_GLOBAL char* g = (const LF_GLOBAL char*)row;
  asm("" : "+s"(g));
  return *(const LF_GLOBAL T*)(g + boff);
}
template <typename T>
__device__ __forceinline__ void st_lane(T* row, unsigned boff, T v) {
  LF_GLOBAL char* g = (LF_GLOBAL char*)row;
  asm("" : "+s"(g));
  *(LF_GLOBAL T*)(g + boff) = v;
}

// ---- reciprocal and reciprocal square root -------------------------------
//
// FP64: the hardware estimate (v_rcp_f64 / v_rsq_f64) refined by one
// third-order step -- far cheaper than the IEEE division and square-root
// sequences.  With e the residual of the estimate r (1 - x r, or 1 - x r^2
// for the square root), 1/x = r (1 + e + e^2 + ...) and 1/sqrt(x) =
// r (1 + e/2 + 3e^2/8 + ...); the dropped terms are of order e^3.  On
// gfx950 the estimates err by at most 2^-24 (relative; measured over 2^24
// inputs), so e^3 lies far below an ulp and the result is as close as two
// Newton steps bring it (within an ulp: the reciprocal correctly rounded in
// practice).  FP32: the hardware instruction alone (1 ulp).

__device__ __forceinline__ double rcp(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, fma(e, e, e), r);
}
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ double rsq(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * r, r, 1.0);  // 1 - x r^2
  return fma(r, fma(0.375, e, 0.5) * e, r);
}
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// ---- primitive variables (perfect gas, Sec. 3) -----------------------------

template <typename T>
struct Prim {
  T r, u, v, p;
};

template <typename T>
__device__ __forceinline__ Prim<T> to_prim(T q0, T q1, T q2, T q3, T gm1) {
  Prim<T> w;
  T ir = rcp(q0);
  w.r = q0;
  w.u = q1 * ir;
  w.v = q2 * ir;
  // p = (gamma-1) (rho E - (m_x u + m_y v)/2): the sum of the two rounded
  // products keeps the x <-> y mirror symmetry exact (an fma over one of
  // them would not); the halving is exact, so one fma takes it and the
  // difference with the same rounding as a product and a subtraction
  w.p = gm1 * fma(T(-0.5), q1 * w.u + q2 * w.v, q3);
  return w;
}

// Variables a cell is reconstructed in: the primitive (rho, u, v, p) of
// Sec. 5, or, for the conservative-variable ablation (CONS), the
// conservative (rho, rho u, rho v, rho E) themselves (kept in the same
// fields r, u, v, p).
template <bool CONS, typename T>
__device__ __forceinline__ Prim<T> rec_vars(T q0, T q1, T q2, T q3, T gm1) {
  if constexpr (CONS) return {q0, q1, q2, q3};
  else return to_prim(q0, q1, q2, q3, gm1);
}

// ---- Sweby limiter, eq. (sweby) ---------------------------------------------

// For beta >= 1 the max-min of eq. (sweby) equals min(beta min(|a|,|b|),
// max(|a|,|b|)) bit for bit (each minimum is taken against a value at least
// as large as the other argument), and for beta = 0 both give 0.  The
// library accepts beta = 0 or 1 <= beta <= 2.  With bs = b sign(a), a
// negative bs (ab < 0) makes the result negative before the max with 0,
// so one expression also covers the ab <= 0 branch.  The result carries
// the sign of a.
//
// FP32 has a median-of-three instruction, and there the limiter is
// med3(beta m, a, b) with m = med3(0, a, b) = minmod(a, b), three
// instructions.  For a, b > 0 and a <= b: m = a and beta a >= a, so the
// median is min(beta a, b); the max-min's other minimum, min(a, beta b),
// is a, so its value is min(beta a, b) as well; b < a is the same with a
// and b swapped.  Negative a, b mirror this (the rounded products are odd
// in their argument), and for ab <= 0, m = 0 and the median of (0, a, b)
// is 0.  So for beta >= 1 both forms give the same value, bit for bit;
// only the sign of a zero result can differ.  For beta = 0 the FP32 form
// returns minmod(a, b), not 0: the kernels then weight every slope by
// h = 0 in the face values (face_plus, face_minus), so no slope is used.
template <typename T>
__device__ __forceinline__ T sweby(T a, T b, T beta) {
  if constexpr (sizeof(T) == 4) {
    const float m = __builtin_amdgcn_fmed3f(0.0f, a, b);
    return __builtin_amdgcn_fmed3f(beta * m, a, b);
  } else {
    const T bs = copysign(T(1), a) * b;
    const T aa = fabs(a);
    const T lo = beta * fmin(aa, bs), hi = fmax(aa, bs);
    return copysign(fmax(fmin(lo, hi), T(0)), a);
  }
}

// Value of eq. (sweby) and half its partial derivatives in one pass (a
// face value is w + phi/2 or w - phi/2, so the adjoint needs the partials
// of phi/2), with the conventions: zero when ab <= 0; min(x, y) follows x
// when x <= y; max(m1, m2) follows m1 when m1 >= m2, where m1 = min(|a|,
// beta |b|) and m2 = min(beta |a|, |b|).  (a and b share their sign when
// ab > 0, so the sign factors cancel in the derivatives.)  For beta >= 1
// these select, with x = |a| and y = |b|:
//   x < y:  min(beta x, y), following beta x (partials beta, 0) when
//           beta x <= y, else y (0, 1);
//   x >= y: min(x, beta y), following x (1, 0) when x <= beta y, else
//           beta y (0, beta);
// i.e. phi = min(p, q) with (p, q) = (beta x, y) or (x, beta y), following
// a when p <= q, with the unit coefficient exactly when that choice differs
// from x < y.  For beta = 0 the value and both partials are 0, as the
// max-min form gives.  The value equals the max-min form, and sweby(), bit
// for bit (min and max return one of their exact arguments); hbeta =
// beta / 2.
template <typename T>
__device__ __forceinline__ void sweby_all(T a, T b, T beta, T hbeta, T& phi, T& hda, T& hdb) {
  const bool lt = fabs(a) < fabs(b);
  // the selects take the signed values and the magnitudes follow (|beta a|
  // = beta |a|): the absolute values then fold into the operand modifiers
  // of the compare and the minimum instead of being formed separately
  const T p = fabs(lt ? beta * a : a);
  const T q = fabs(lt ? b : beta * b);
  const bool act = a * b > T(0);
  const bool fa = p <= q;                       // follows a
  phi = act ? copysign(fmin(p, q), a) : T(0);
  const T hc = (fa != lt) ? T(0.5) : hbeta;     // coefficient 1 or beta, halved
  hda = (act && fa) ? hc : T(0);
  hdb = (act && !fa) ? hc : T(0);
}

// ---- face flux: Lagrangian HLL solve (eqs. (13)-(14)) + upwind + eq. (12) --

// State on one side of a face, in the face frame.
template <typename T>
struct FaceState {
  T r, un, ut, p;
};

// A reconstructed face state as primitive variables: unchanged for the
// primitive reconstruction; for the conservative one (rho, rho u_n,
// rho u_t, rho E) -> (rho, u_n, u_t, p) by the perfect-gas law (the same
// arithmetic as to_prim).
template <bool CONS, typename T>
__device__ __forceinline__ FaceState<T> face_prim(const FaceState<T>& f, T gm1) {
  if constexpr (!CONS) {
    return f;
  } else {
    const T ir = rcp(f.r);
    const T un = f.un * ir, ut = f.ut * ir;
    return {f.r, un, ut, gm1 * fma(T(-0.5), f.un * un + f.ut * ut, f.p)};
  }
}

template <typename T>
struct Flux {
  T f0, f1, f2, f3;  // mass, normal momentum, tangential momentum, energy
};

// left_out receives the upwind side (true: left, u* > 0), which the
// transport of the mass fractions shares.
template <typename T>
__device__ __forceinline__ Flux<T> face_flux(const FaceState<T>& L, const FaceState<T>& R,
                                             T gamma, T inv_gm1, bool& left_out) {
  // a = max(c_L, c_R), a^2 = gamma max(p_L/rho_L, p_R/rho_R), i.e.
  // a^2 rho_L rho_R = gamma max(p_L rho_R, p_R rho_L) =: g (densities > 0),
  // with no select.
  const T pr = L.p * R.r, rp = L.r * R.p;  // p_L rho_R, rho_L p_R
  const T rr = L.r * R.r;
  const T S = L.r + R.r;
  const T g = gamma * fmax(pr, rp);
  T a, iSa, iS;  // a, 1/(S a), 1/S
  if constexpr (sizeof(T) == 8) {
    // one reciprocal square root for everything (the refined FP64 one costs
    // six instructions, a reciprocal four): t = 1/sqrt(g rho_L rho_R S^2) =
    // 1/(a rho_L rho_R S) gives a = g t S, 1/(S a) = t rho_L rho_R and
    // 1/S = a/(S a)
    const T t = rsq(g * rr * (S * S));
    a = g * t * S;
    iSa = t * rr;
    iS = iSa * a;
  } else {
    // one instruction each; q = 1/(rho_L rho_R S) gives 1/S = rho_L rho_R q
    // and 1/(rho_L rho_R) = S q (no product of four state values: FP32
    // range)
    const T q = rcp(rr * S);
    iS = rr * q;
    const T a2 = g * (S * q);
    const T ia = rsq(a2);
    a = a2 * ia;
    iSa = iS * ia;
  }
  // eq. (13): p* = (rho_R p_L + rho_L p_R)/S - (rho_L rho_R / S) a (u_R - u_L)
  const T ps = fma(-(rr * iS) * a, R.un - L.un, (pr + rp) * iS);
  // eq. (14): u* = (rho_L u_L + rho_R u_R)/S - (p_R - p_L)/(S a)
  const T us = fma(-(R.p - L.p), iSa, fma(L.r, L.un, R.r * R.un) * iS);
  // upwind on the sign of u*: left when u* > 0
  const bool left = us > T(0);
  left_out = left;
  const T r = left ? L.r : R.r;
  const T un = left ? L.un : R.un;
  const T ut = left ? L.ut : R.ut;
  const T p = left ? L.p : R.p;
  const T E = fma(T(0.5) * r, fma(un, un, ut * ut), p * inv_gm1);  // rho E of the upwind state
  const T m = r * us;
  Flux<T> F;
  F.f0 = m;
  F.f1 = fma(m, un, ps);
  F.f2 = m * ut;
  F.f3 = (E + ps) * us;
  return F;
}

template <typename T>
__device__ __forceinline__ Flux<T> face_flux(const FaceState<T>& L, const FaceState<T>& R,
                                             T gamma, T inv_gm1) {
  bool left;
  return face_flux(L, R, gamma, inv_gm1, left);
}

// Vector-Jacobian product of face_flux: given the flux cotangent Fb,
// returns the cotangents of the two face states.  The forward values are
// recomputed as face_flux() forms them, except the sound speed: it is
// formed from the selected side's (p, rho), since its cotangent goes to
// that side (the same value up to rounding).  Conventions at the kinks:
// max(c_L, c_R) follows L on ties (p_L rho_R >= p_R rho_L); the upwind side
// is L iff u* > 0.  Every division goes through one reciprocal and one
// reciprocal square root: with q = 1/(rho_s S), 1/S = rho_s q,
// 1/rho_s = S q, and da/dp_s = a/(2 p_s) = gamma/(2 rho_s a).
template <typename T>
__device__ __forceinline__ void face_flux_vjp(const FaceState<T>& L, const FaceState<T>& R,
                                              T gamma, T inv_gm1, const Flux<T>& Fb,
                                              FaceState<T>& Lb, FaceState<T>& Rb) {
  const bool aleft = L.p * R.r >= R.p * L.r;
  const T ps_ = aleft ? L.p : R.p;
  const T rs_ = aleft ? L.r : R.r;
  const T S = L.r + R.r;
  const T q = rcp(rs_ * S);
  const T iS = rs_ * q;
  const T irs = S * q;
  const T a2 = gamma * ps_ * irs;
  const T ia = rsq(a2);
  const T a = a2 * ia;
  const T iS2 = iS * iS;
  const T B = L.r * R.r;
  const T Du = R.un - L.un;
  const T Dp = R.p - L.p;
  const T ps = fma(-(B * iS) * a, Du, fma(R.r, L.p, L.r * R.p) * iS);
  const T us = fma(-Dp, iS * ia, fma(L.r, L.un, R.r * R.un) * iS);
  const bool left = us > T(0);
  const T r = left ? L.r : R.r;
  const T un = left ? L.un : R.un;
  const T ut = left ? L.ut : R.ut;
  const T p = left ? L.p : R.p;
  const T q2 = fma(un, un, ut * ut);
  const T E = fma(T(0.5) * r, q2, p * inv_gm1);

  // through eq. (12) and the upwind state
  const T Eb = Fb.f3 * us;
  const T usb = fma(Fb.f3, E + ps, r * fma(Fb.f2, ut, fma(Fb.f1, un, Fb.f0)));
  const T psb = fma(Fb.f3, us, Fb.f1);
  const T rb = fma(Eb * T(0.5), q2, us * fma(Fb.f2, ut, fma(Fb.f1, un, Fb.f0)));
  const T unb = r * fma(Fb.f1, us, Eb * un);
  const T utb = r * fma(Fb.f2, us, Eb * ut);
  const T pb = Eb * inv_gm1;

  // through eqs. (13)-(14), with w = (p_R - p_L) / (S a):
  //   dp*/da = -(rho_L rho_R / S) (u_R - u_L),   du*/da = w / a,
  //   dp*/drho_L = rho_R (p_R - p_L - rho_R a (u_R - u_L)) / S^2,
  //   du*/drho_L = (w / S) - rho_R (u_R - u_L) / S^2, and the mirror images
  const T iSia = iS * ia;
  const T BiS = B * iS;
  const T BiSa = BiS * a;
  const T w = Dp * iSia;
  const T ab = fma(psb, -BiS * Du, usb * (w * ia));
  const T t1 = w * iS;
  const T psbiS2 = psb * iS2, aDu = a * Du, DuiS2 = Du * iS2;
  const T rlb = fma(psbiS2 * R.r, fma(-R.r, aDu, Dp), usb * fma(-R.r, DuiS2, t1));
  const T rrb = fma(-(psbiS2 * L.r), fma(L.r, aDu, Dp), usb * fma(L.r, DuiS2, t1));
  const T unlb = fma(psb, BiSa, usb * (L.r * iS));
  const T unrb = fma(-psb, BiSa, usb * (R.r * iS));
  const T plb = fma(psb, R.r * iS, usb * iSia);
  const T prb = fma(psb, L.r * iS, -usb * iSia);
  // a = sqrt(gamma p_s / rho_s): da/drho_s = -a / (2 rho_s), da/dp_s =
  // gamma / (2 rho_s a)
  const T habr = T(0.5) * ab * irs;
  const T dar = -habr * a;
  const T dap = habr * (gamma * ia);
  // the sound-speed and upwind terms each go to one side
  if constexpr (sizeof(T) == 8) {
    // 0/1 weights of the two sides (one select each, the low word being
    // zero, where a select of a double takes two), folded into fmas
    const T wa = aleft ? T(1) : T(0), wl = left ? T(1) : T(0);
    const T va = aleft ? T(0) : T(1), vl = left ? T(0) : T(1);
    Lb.r = fma(dar, wa, fma(rb, wl, rlb));
    Lb.un = fma(unb, wl, unlb);
    Lb.ut = utb * wl;
    Lb.p = fma(dap, wa, fma(pb, wl, plb));
    Rb.r = fma(dar, va, fma(rb, vl, rrb));
    Rb.un = fma(unb, vl, unrb);
    Rb.ut = utb * vl;
    Rb.p = fma(dap, va, fma(pb, vl, prb));
  } else {
    // the left side's share is selected and the right side takes the
    // rest, x - share, which is exactly x or 0
    const T darL = aleft ? dar : T(0), dapL = aleft ? dap : T(0);
    const T rbL = left ? rb : T(0), unbL = left ? unb : T(0);
    const T utbL = left ? utb : T(0), pbL = left ? pb : T(0);
    Lb.r = rlb + darL + rbL;
    Lb.un = unlb + unbL;
    Lb.ut = utbL;
    Lb.p = plb + dapL + pbL;
    Rb.r = rrb + (dar - darL) + (rb - rbL);
    Rb.un = unrb + (unb - unbL);
    Rb.ut = utb - utbL;
    Rb.p = prb + (dap - dapL) + (pb - pbL);
  }
}

// ---- pieces of a stage row shared by the stage kernels ----------------------

// Mass fractions of one row (NS of them; one unused slot when NS = 0).
template <typename T, int NS>
struct Frac {
  T v[NS > 0 ? NS : 1];
};

template <typename T>
__device__ __forceinline__ Prim<T> sub(const Prim<T>& a, const Prim<T>& b) {
  return {a.r - b.r, a.u - b.u, a.v - b.v, a.p - b.p};
}

// Limited slope from the backward and forward differences.  Eq. (sweby)
// is symmetric in its two arguments (for ab > 0 they share their sign;
// otherwise it is 0), and the forward difference goes first: it is always
// formed just before (a lane shift or a value carried from the previous
// row can hold anything as far as the compiler knows), so |dp| needs no
// IEEE quieting before the min and max.  Only the sign of a zero slope
// can differ from the other order.
template <typename T>
__device__ __forceinline__ Prim<T> slope(const Prim<T>& dm, const Prim<T>& dp, T beta) {
  return {sweby(dp.r, dm.r, beta), sweby(dp.u, dm.u, beta), sweby(dp.v, dm.v, beta),
          sweby(dp.p, dm.p, beta)};
}

// w + h s (face_plus) and w - h s (face_minus) in the x-face frame (u
// normal) or the y-face frame (v normal).  The weight h is 1/2, or 0 for
// beta = 0: then every face takes its cell's value (first order) whatever
// sweby() returned.
template <typename T, bool YFACE>
__device__ __forceinline__ FaceState<T> face_plus(const Prim<T>& w, const Prim<T>& s, T h) {
  T r = fma(h, s.r, w.r), u = fma(h, s.u, w.u), v = fma(h, s.v, w.v), p = fma(h, s.p, w.p);
  if constexpr (YFACE) return {r, v, u, p};
  else return {r, u, v, p};
}
template <typename T, bool YFACE>
__device__ __forceinline__ FaceState<T> face_minus(const Prim<T>& w, const Prim<T>& s, T h) {
  T r = fma(-h, s.r, w.r), u = fma(-h, s.u, w.u), v = fma(-h, s.v, w.v), p = fma(-h, s.p, w.p);
  if constexpr (YFACE) return {r, v, u, p};
  else return {r, u, v, p};
}

template <typename T>
__device__ __forceinline__ Prim<T> shl1(const Prim<T>& w) {
  return {shl1(w.r), shl1(w.u), shl1(w.v), shl1(w.p)};
}
template <typename T>
__device__ __forceinline__ Prim<T> shr1(const Prim<T>& w) {
  return {shr1(w.r), shr1(w.u), shr1(w.v), shr1(w.p)};
}
template <typename T>
__device__ __forceinline__ Flux<T> shr1(const Flux<T>& f) {
  return {shr1(f.f0), shr1(f.f1), shr1(f.f2), shr1(f.f3)};
}

// Combination of one stage, formed in FP64 from the cell's flux balance
// s = (F_{i+1/2} - F_{i-1/2}) + (dx/dy) (G_{j+1/2} - G_{j-1/2}), of which
// the residual of eq. (11) is R = s / dx: predictor U - dt R = U - dtx s;
// corrector (U^n + U* - dtx s(U*)) / 2, with dtx = dt / dx; the residual
// mode writes s / dx in T.
template <int MODE, typename T>
__device__ __forceinline__ T combine(T q, T b, T s, double dtx, T idx) {
  if constexpr (MODE == kResidual) {
    return s * idx;
  } else if constexpr (MODE == kPredictor) {
    return T(fma(-dtx, double(s), double(q)));
  } else {
    return T(0.5 * (double(b) + fma(-dtx, double(s), double(q))));
  }
}

// ---- CFL wave speed (item 1 of the Heun list) -------------------------------
//
// (|u| + c)/dx + (|v| + c)/dy of a cell from its conservative values, and
// whether the cell is physical (rho > 0, p > 0, finite speed).  One
// routine for every kernel that reduces it (lf_dt, the corrector epilogue,
// the single pass), so that they agree bit for bit; symmetric in x and y.
template <typename T>
__device__ __forceinline__ T cfl_speed(T q0, T q1, T q2, T q3, T gm1, T gam, T idx, T idy, bool& ok) {
  const T ir = rcp(q0);
  const T uu = q1 * ir, vv = q2 * ir;
  const T pp = gm1 * fma(T(-0.5), q1 * uu + q2 * vv, q3);  // as to_prim
  const T c2 = gam * pp * ir;
  const T cs = c2 * rsq(c2);
  const T sp = (fabs(uu) + cs) * idx + (fabs(vv) + cs) * idy;
  ok = (q0 > T(0)) && (pp > T(0)) && (sp <= T(3.0e38));
  return sp;
}
// running maximum of the speeds (non-negative, finite where used): a
// compare and a select, with none of the quieting an IEEE max needs for an
// operand carried from the previous row.  Kept in the state's precision (a
// maximum is exact in any precision) and widened once, for the reduction
// across lanes in FP64.
template <typename T>
__device__ __forceinline__ T speed_max(T m, T s) { return s > m ? s : m; }

// ---- wave-level reductions --------------------------------------------------

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long o = __shfl_xor(v, off, kWave);
    v = o > v ? o : v;
  }
  return v;
}

// Hardware assigns workgroup b to die b % 8.  Remap so each die works on a
// contiguous range of logical blocks (neighbouring tiles share halo rows
// and columns through that die's L2).  nblk_pad is a multiple of 8.
__device__ __forceinline__ int xcd_block(int b, int nblk_pad) {
  int per = nblk_pad / kXcds;
  return (b % kXcds) * per + b / kXcds;
}

}  // namespace lf
