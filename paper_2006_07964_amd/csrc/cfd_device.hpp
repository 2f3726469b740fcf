// cfd_device.hpp -- device-side building blocks of the curvilinear AFWENO right-hand side
// (Ye et al., arXiv 2006.07964, Sec. 2 and Sec. 4.5) for gfx950.
//
// All point-level arithmetic is templated on the compute type R (double for the FP64
// path, float for the mixed path).  State, metrics and Jacobian are always read as
// double; callers convert after the load.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cfd {

constexpr int kHalo = 3;   // state / metric halo
constexpr int kCHalo = 6;  // coordinate halo

// Geometry of one block's pitched SoA arrays (elements).
struct Geom {
  int ni, nj, nk;
  int64_t ld_i, ld_j;  // row and column pitch
  int64_t plane;       // ld_i * ld_j * (nk + 6)
};

__device__ __forceinline__ int64_t at(const Geom& g, int i, int j, int k) {
  return ((int64_t)(k + kHalo) * g.ld_j + (j + kHalo)) * g.ld_i + (i + kHalo);
}

// Physical constants of one block, converted to the compute type by the kernels.
struct Phys {
  double gamma;
  double visc_scale;  // Ma / Re
  double heat_scale;  // Ma / (Re Pr (gamma - 1))
  double suth;
  double eps;
  int linear;  // ideal WENO weights
};

// ---- sixth-order central difference (Sec. 2 after Eq 8), unit spacing ---------------
// g(m) returns the value at offset m in [-3, 3] (the centre is not used).
template <typename R, typename F>
__device__ __forceinline__ R d6(F g) {
  return R(0.75) * (g(1) - g(-1)) - R(0.15) * (g(2) - g(-2)) + R(1.0 / 60.0) * (g(3) - g(-3));
}

// ---- Sutherland viscosity, mu(T) = T^1.5 (1+S)/(T+S) ------------------------------------
template <typename R>
__device__ __forceinline__ R viscosity(R T, R suth) {
  return T * sqrt(T) * (R(1) + suth) / (T + suth);
}

// ---- primitive state ----------------------------------------------------------------
template <typename R>
struct Prim {
  R rho, rinv, u, v, w, p, c;
};

template <typename R>
__device__ __forceinline__ Prim<R> primitive(const R q[5], R gamma) {
  Prim<R> s;
  s.rho = q[0];
  s.rinv = R(1) / q[0];
  s.u = q[1] * s.rinv;
  s.v = q[2] * s.rinv;
  s.w = q[3] * s.rinv;
  s.p = (gamma - R(1)) * (q[4] - R(0.5) * s.rho * (s.u * s.u + s.v * s.v + s.w * s.w));
  s.c = sqrt(gamma * s.p * s.rinv);  // c^2 = gamma p / rho = T
  return s;
}

// ---- Eq 4: inviscid flux through the hatted metric vector (mx, my, mz) --------------
template <typename R>
__device__ __forceinline__ void phys_flux(const R q[5], R mx, R my, R mz, R gamma, R F[5]) {
  const R rinv = R(1) / q[0];
  const R u = q[1] * rinv, v = q[2] * rinv, w = q[3] * rinv;
  const R p = (gamma - R(1)) * (q[4] - R(0.5) * (q[1] * u + q[2] * v + q[3] * w));
  const R U = mx * u + my * v + mz * w;
  F[0] = q[0] * U;
  F[1] = q[1] * U + mx * p;
  F[2] = q[2] * U + my * p;
  F[3] = q[3] * U + mz * p;
  F[4] = (q[4] + p) * U;
}

// ---- Steger-Warming split flux of one sign (SIGN = +1 or -1) -------------------------
// lambda_{1,2,3} = |m| theta, lambda_{4,5} = |m| (theta +- c), lambda^{+-} = (lambda +- |lambda|)/2,
// F = rho/(2 gamma) [2 (gamma-1) l1 (1,u,v,w,|u|^2/2) + l4 (1, u + c k, H + c theta)
//                    + l5 (1, u - c k, H - c theta)].
template <int SIGN, typename R>
__device__ __forceinline__ void sw_flux(const R q[5], R mx, R my, R mz, R gamma, R F[5]) {
  const R rinv = R(1) / q[0];
  const R u = q[1] * rinv, v = q[2] * rinv, w = q[3] * rinv;
  const R ke = R(0.5) * (u * u + v * v + w * w);
  const R p = (gamma - R(1)) * (q[4] - q[0] * ke);
  const R c = sqrt(gamma * p * rinv);
  const R mag = sqrt(mx * mx + my * my + mz * mz);
  const R minv = R(1) / mag;
  const R kx = mx * minv, ky = my * minv, kz = mz * minv;
  const R theta = kx * u + ky * v + kz * w;
  const R H = (q[4] + p) * rinv;
  const R l1 = mag * theta, l4 = mag * (theta + c), l5 = mag * (theta - c);
  const R a1 = R(0.5) * (l1 + R(SIGN) * fabs(l1));
  const R a4 = R(0.5) * (l4 + R(SIGN) * fabs(l4));
  const R a5 = R(0.5) * (l5 + R(SIGN) * fabs(l5));
  const R f = q[0] / (R(2) * gamma);
  const R e1 = R(2) * (gamma - R(1)) * a1;
  const R s45 = a4 + a5, d45 = (a4 - a5) * c;
  F[0] = f * (e1 + s45);
  F[1] = f * (e1 * u + s45 * u + d45 * kx);
  F[2] = f * (e1 * v + s45 * v + d45 * ky);
  F[3] = f * (e1 * w + s45 * w + d45 * kz);
  F[4] = f * (e1 * ke + s45 * H + d45 * theta);
}

// ---- characteristic basis at a node (Pulliam-Chaussee right eigenvectors) ------------
// R = M R_W with M = dQ/d(rho,u,v,w,p) and, in primitive form, columns 1-3
// (k_m, k x e_m, 0) for eigenvalue theta and columns 4-5 rho/(sqrt2 c) (1, +-c k/rho, c^2)
// for theta +- c; L = R^-1 = R_W^-1 M^-1 in closed form.
template <typename R>
struct Basis {
  R kx, ky, kz;
  R rho, rinv, u, v, w, ke, gm1;
  R c2inv;   // 1 / c^2
  R rcinv;   // 1 / (rho c)
  R a;       // rho / (sqrt2 c)
  R b;       // rho c / sqrt2
  R gm1inv;  // 1 / (gamma - 1)
};

template <typename R>
__device__ __forceinline__ Basis<R> make_basis(const R q[5], R mx, R my, R mz, R gamma) {
  Basis<R> B;
  const R minv = R(1) / sqrt(mx * mx + my * my + mz * mz);
  B.kx = mx * minv;
  B.ky = my * minv;
  B.kz = mz * minv;
  B.rho = q[0];
  B.rinv = R(1) / q[0];
  B.u = q[1] * B.rinv;
  B.v = q[2] * B.rinv;
  B.w = q[3] * B.rinv;
  B.ke = R(0.5) * (B.u * B.u + B.v * B.v + B.w * B.w);
  B.gm1 = gamma - R(1);
  const R p = B.gm1 * (q[4] - B.rho * B.ke);
  const R c2 = gamma * p * B.rinv;
  const R c = sqrt(c2);
  B.c2inv = R(1) / c2;
  B.rcinv = R(1) / (B.rho * c);
  const R s2 = R(0.70710678118654752440);  // 1/sqrt2
  B.a = B.rho * s2 / c;
  B.b = B.rho * c * s2;
  B.gm1inv = R(1) / B.gm1;
  return B;
}

// V = L Q' for a conserved vector Q' (characteristic projection).
template <typename R>
__device__ __forceinline__ void project(const Basis<R>& B, const R qp[5], R V[5]) {
  const R yr = qp[0];
  const R yu = (qp[1] - B.u * qp[0]) * B.rinv;
  const R yv = (qp[2] - B.v * qp[0]) * B.rinv;
  const R yw = (qp[3] - B.w * qp[0]) * B.rinv;
  const R yp = B.gm1 * (B.ke * qp[0] - B.u * qp[1] - B.v * qp[2] - B.w * qp[3] + qp[4]);
  const R s = yr - yp * B.c2inv;
  V[0] = B.kx * s + (yv * B.kz - yw * B.ky);
  V[1] = B.ky * s + (yw * B.kx - yu * B.kz);
  V[2] = B.kz * s + (yu * B.ky - yv * B.kx);
  const R kd = B.kx * yu + B.ky * yv + B.kz * yw;
  const R pr = yp * B.rcinv;
  const R s2 = R(0.70710678118654752440);
  V[3] = (pr + kd) * s2;
  V[4] = (pr - kd) * s2;
}

// Q' = R v (back to conserved variables).
template <typename R>
__device__ __forceinline__ void unproject(const Basis<R>& B, const R V[5], R qp[5]) {
  const R s2 = R(0.70710678118654752440);
  const R kv = B.kx * V[0] + B.ky * V[1] + B.kz * V[2];
  const R sp = V[3] + V[4];
  const R sm = (V[3] - V[4]) * s2;
  const R yr = kv + B.a * sp;
  const R yu = (B.ky * V[2] - B.kz * V[1]) + B.kx * sm;
  const R yv = (B.kz * V[0] - B.kx * V[2]) + B.ky * sm;
  const R yw = (B.kx * V[1] - B.ky * V[0]) + B.kz * sm;
  const R yp = B.b * sp;
  qp[0] = yr;
  qp[1] = B.u * yr + B.rho * yu;
  qp[2] = B.v * yr + B.rho * yv;
  qp[3] = B.w * yr + B.rho * yw;
  qp[4] = B.ke * yr + B.rho * (B.u * yu + B.v * yv + B.w * yw) + yp * B.gm1inv;
}

// ---- WENO interpolation to both half points from one 5-point stencil ----------------
// Eqs 13-17 with the sub-stencil pairing of the fifth-order interpolant: ideal weight
// 1/16 and beta_1 on {i-2,i-1,i}, 5/8 on {i-1,i,i+1}, 5/16 on {i,i+1,i+2} for the
// left-biased value at i+1/2; the right-biased value at i-1/2 uses the mirror images with
// the same betas (modified AFWENO, Sec. 4.5.1).
template <typename R>
__device__ __forceinline__ void weno_pair(R a, R b, R c, R d, R e, R eps, bool linear, R& vl, R& vr) {
  const R p0 = R(0.375) * a - R(1.25) * b + R(1.875) * c;
  const R p1 = R(-0.125) * b + R(0.75) * c + R(0.375) * d;
  const R p2 = R(0.375) * c + R(0.75) * d - R(0.125) * e;
  const R m0 = R(-0.125) * a + R(0.75) * b + R(0.375) * c;
  const R m1 = R(0.375) * b + R(0.75) * c - R(0.125) * d;
  const R m2 = R(1.875) * c - R(1.25) * d + R(0.375) * e;
  if (linear) {
    vl = R(0.0625) * p0 + R(0.625) * p1 + R(0.3125) * p2;
    vr = R(0.3125) * m0 + R(0.625) * m1 + R(0.0625) * m2;
    return;
  }
  const R third = R(1.0 / 3.0);
  const R b0 = (R(4) * a * a - R(19) * a * b + R(25) * b * b + R(11) * a * c - R(31) * b * c + R(10) * c * c) * third;
  const R b1 = (R(4) * b * b - R(13) * b * c + R(13) * c * c + R(5) * b * d - R(13) * c * d + R(4) * d * d) * third;
  const R b2 = (R(10) * c * c - R(31) * c * d + R(25) * d * d + R(11) * c * e - R(19) * d * e + R(4) * e * e) * third;
  const R t0 = eps + b0, t1 = eps + b1, t2 = eps + b2;
  const R r0 = R(1) / (t0 * t0), r1 = R(1) / (t1 * t1), r2 = R(1) / (t2 * t2);
  const R wl0 = R(0.0625) * r0, wl1 = R(0.625) * r1, wl2 = R(0.3125) * r2;
  const R wr0 = R(0.3125) * r0, wr1 = R(0.625) * r1, wr2 = R(0.0625) * r2;
  vl = (wl0 * p0 + wl1 * p1 + wl2 * p2) / (wl0 + wl1 + wl2);
  vr = (wr0 * m0 + wr1 * m1 + wr2 * m2) / (wr0 + wr1 + wr2);
}

// ---- sixth-order half-point interpolation of node metrics ---------------------------
// m(i+1/2) = (3 m(i-2) - 25 m(i-1) + 150 m(i) + 150 m(i+1) - 25 m(i+2) + 3 m(i+3)) / 256;
// combined with Eq 19 it gives the sixth-order derivative of the metrics, so a uniform
// state stays uniform on curvilinear grids.  g(m) returns the node value at offset m.
template <typename F>
__device__ __forceinline__ double half_metric(F g) {
  return (3.0 * (g(-2) + g(3)) - 25.0 * (g(-1) + g(2)) + 150.0 * (g(0) + g(1))) * (1.0 / 256.0);
}

}  // namespace cfd
