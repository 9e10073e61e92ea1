// lf_adjoint.hip -- transpose of the residual's Jacobian, v = J_R(U)^T g,
// in gather form (no atomics), and the two adjoint stages of the Heun step.
//
// R_i = (F_{i+1/2} - F_{i-1/2})/dx + (G_{j+1/2} - G_{j-1/2})/dy, and the
// flux through x-face k (between cells k-1 and k) depends on the
// primitive states of cells k-2 .. k+1 (MUSCL slopes of k-1 and k).  Cell
// i therefore receives contributions from x-faces k = i-1 .. i+2 and the
// same four y-faces; each face's cotangent is (g_{k-1} - g_k)/dx.  A
// thread owns one cell, recomputes the forward state of each of its eight
// faces and pulls the face cotangent back through eq. (12), eqs. (13)-(14)
// and the limited reconstruction (eq. (sweby)) onto its own primitive
// variables, then through the perfect-gas law onto its conservative ones.
//
// With transmissive boundaries the ghost cells copy the edge cell, so an
// edge cell also collects the contributions of the stencil slots that
// point at its ghosts; with periodic boundaries each (face, slot) pair is
// visited exactly once through the extended face index.
#include "lf_internal.h"

namespace lf {

template <typename T>
struct AdjArgs {
  const T* U;
  const T* g;
  const T* lam;
  T* out;
  int nx, ny;
  long long plane;
  T gamma, gm1, inv_gm1, beta, idx, idy;
  double dt;
};

template <typename T>
struct Slots {
  FaceState<T> s[4];
};

// Forward face state of one stencil and the cotangents of its four cells.
template <typename T>
__device__ __forceinline__ void face_backprop(const FaceState<T> (&W)[4], const Flux<T>& fb, T gamma,
                                              T inv_gm1, T beta, Slots<T>& out) {
  T pa1[4], pb1[4], pa2[4], pb2[4];
  T wl[4], wr[4];
  const T* w0 = &W[0].r;
  const T* w1 = &W[1].r;
  const T* w2 = &W[2].r;
  const T* w3 = &W[3].r;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    T a1 = w1[v] - w0[v], b1 = w2[v] - w1[v];
    T a2 = w2[v] - w1[v], b2 = w3[v] - w2[v];
    T s1 = sweby(a1, b1, beta), s2 = sweby(a2, b2, beta);
    sweby_d(a1, b1, beta, pa1[v], pb1[v]);
    sweby_d(a2, b2, beta, pa2[v], pb2[v]);
    wl[v] = fma(T(0.5), s1, w1[v]);
    wr[v] = fma(T(-0.5), s2, w2[v]);
  }
  FaceState<T> L = {wl[0], wl[1], wl[2], wl[3]};
  FaceState<T> R = {wr[0], wr[1], wr[2], wr[3]};
  FaceState<T> Lb, Rb;
  face_flux_vjp(L, R, gamma, inv_gm1, fb, Lb, Rb);
  const T* lb = &Lb.r;
  const T* rb = &Rb.r;
  T* o0 = &out.s[0].r;
  T* o1 = &out.s[1].r;
  T* o2 = &out.s[2].r;
  T* o3 = &out.s[3].r;
  const T h = T(0.5);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    o0[v] = -h * pa1[v] * lb[v];
    o1[v] = (T(1) + h * (pa1[v] - pb1[v])) * lb[v] + h * pa2[v] * rb[v];
    o2[v] = h * pb1[v] * lb[v] + (T(1) - h * (pa2[v] - pb2[v])) * rb[v];
    o3[v] = -h * pb2[v] * rb[v];
  }
}

template <typename T>
__device__ __forceinline__ Prim<T> load_prim(const AdjArgs<T>& a, int off) {
  return to_prim(a.U[off], a.U[a.plane + off], a.U[2 * a.plane + off], a.U[3 * a.plane + off], a.gm1);
}

template <typename T, int MODE, int BCX, int BCY>
__global__ __launch_bounds__(256) void adjoint_kernel(AdjArgs<T> a) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.plane) return;
  const int nx = a.nx, ny = a.ny;
  const int j = (int)(q / nx);
  const int i = (int)(q - (long long)j * nx);
  const long long P = a.plane;
  T wr = 0, wu = 0, wv = 0, wp = 0;  // cotangent of (rho, u, v, p) of cell (i, j)

  // ---- x-faces k = i-1 .. i+2 (face k between cells k-1 and k) ----
#pragma unroll 1
  for (int kk = -1; kk <= 2; ++kk) {
    const int k = i + kk;
    if (BCX == kBcTransmissive && (k < 0 || k > nx)) continue;
    T gl[4] = {0, 0, 0, 0}, gr[4] = {0, 0, 0, 0};
    const bool has_l = (BCX == kBcPeriodic) || (k - 1 >= 0);
    const bool has_r = (BCX == kBcPeriodic) || (k < nx);
    if (has_l) {
      const int o = j * nx + map_index<BCX>(k - 1, nx);
      for (int f = 0; f < 4; ++f) gl[f] = a.g[f * P + o];
    }
    if (has_r) {
      const int o = j * nx + map_index<BCX>(k, nx);
      for (int f = 0; f < 4; ++f) gr[f] = a.g[f * P + o];
    }
    Flux<T> fb = {(gl[0] - gr[0]) * a.idx, (gl[1] - gr[1]) * a.idx, (gl[2] - gr[2]) * a.idx,
                  (gl[3] - gr[3]) * a.idx};
    FaceState<T> W[4];
    int cell[4];
    for (int s = 0; s < 4; ++s) {
      cell[s] = map_index<BCX>(k - 2 + s, nx);
      Prim<T> w = load_prim(a, j * nx + cell[s]);
      W[s] = {w.r, w.u, w.v, w.p};
    }
    Slots<T> sl;
    face_backprop(W, fb, a.gamma, a.inv_gm1, a.beta, sl);
    for (int s = 0; s < 4; ++s) {
      const bool mine = (BCX == kBcPeriodic) ? (s == 2 - kk) : (cell[s] == i);
      if (mine) {
        wr += sl.s[s].r;
        wu += sl.s[s].un;
        wv += sl.s[s].ut;
        wp += sl.s[s].p;
      }
    }
  }

  // ---- y-faces k = j-1 .. j+2 (frame: normal velocity v) ----
#pragma unroll 1
  for (int kk = -1; kk <= 2; ++kk) {
    const int k = j + kk;
    if (BCY == kBcTransmissive && (k < 0 || k > ny)) continue;
    T gl[4] = {0, 0, 0, 0}, gr[4] = {0, 0, 0, 0};
    const bool has_l = (BCY == kBcPeriodic) || (k - 1 >= 0);
    const bool has_r = (BCY == kBcPeriodic) || (k < ny);
    if (has_l) {
      const int o = map_index<BCY>(k - 1, ny) * nx + i;
      for (int f = 0; f < 4; ++f) gl[f] = a.g[f * P + o];
    }
    if (has_r) {
      const int o = map_index<BCY>(k, ny) * nx + i;
      for (int f = 0; f < 4; ++f) gr[f] = a.g[f * P + o];
    }
    // flux frame: (mass, y-momentum, x-momentum, energy)
    Flux<T> fb = {(gl[0] - gr[0]) * a.idy, (gl[2] - gr[2]) * a.idy, (gl[1] - gr[1]) * a.idy,
                  (gl[3] - gr[3]) * a.idy};
    FaceState<T> W[4];
    int cell[4];
    for (int s = 0; s < 4; ++s) {
      cell[s] = map_index<BCY>(k - 2 + s, ny);
      Prim<T> w = load_prim(a, cell[s] * nx + i);
      W[s] = {w.r, w.v, w.u, w.p};
    }
    Slots<T> sl;
    face_backprop(W, fb, a.gamma, a.inv_gm1, a.beta, sl);
    for (int s = 0; s < 4; ++s) {
      const bool mine = (BCY == kBcPeriodic) ? (s == 2 - kk) : (cell[s] == j);
      if (mine) {
        wr += sl.s[s].r;
        wv += sl.s[s].un;
        wu += sl.s[s].ut;
        wp += sl.s[s].p;
      }
    }
  }

  // ---- primitive -> conservative: v = (dw/dU)^T wbar ----
  const T q0 = a.U[q], q1 = a.U[P + q], q2 = a.U[2 * P + q];
  const T ir = T(1) / q0;
  const T u = q1 * ir, v = q2 * ir;
  const T gm1 = a.gm1;
  T v0 = wr - (u * wu + v * wv) * ir + gm1 * T(0.5) * (u * u + v * v) * wp;
  T v1 = wu * ir - gm1 * u * wp;
  T v2 = wv * ir - gm1 * v * wp;
  T v3 = gm1 * wp;
  T vv[4] = {v0, v1, v2, v3};
  for (int f = 0; f < 4; ++f) {
    T res;
    if constexpr (MODE == kVjp) {
      res = vv[f];
    } else if constexpr (MODE == kAdjCorr) {
      // mu = (lam - dt v) / 2 with g = lam
      res = T(0.5 * (double(a.g[f * P + q]) - a.dt * double(vv[f])));
    } else {
      // lam^n = lam / 2 + mu - dt v with g = mu
      res = T(0.5 * double(a.lam[f * P + q]) + double(a.g[f * P + q]) - a.dt * double(vv[f]));
    }
    a.out[f * P + q] = res;
  }
}

template <typename T, int MODE, int BCX, int BCY>
static hipError_t launch_adj_t(const Grid& g, const void* U, const void* gv, const void* lam, void* out,
                               double dt, hipStream_t s) {
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
  a.idx = T(1.0 / g.dx);
  a.idy = T(1.0 / g.dy);
  a.dt = dt;
  const long long nb = (a.plane + 255) / 256;
  hipLaunchKernelGGL((adjoint_kernel<T, MODE, BCX, BCY>), dim3((unsigned)nb), dim3(256), 0, s, a);
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
