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

// A pointer read from device memory (a per-block argument table) is generic to the
// compiler, which then emits flat memory instructions; flat loads count against both the
// vector-memory and the LDS counters and serialise waits in LDS-heavy kernels.  Kernels
// that take their pointers from such a table access memory through pointers typed in the
// global address space.
template <typename T>
using GP = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ GP<T> to_global(T* p) {
  return (GP<T>)p;
}

// Element e of the array at a wave-uniform base, with e < 2^32 / sizeof(T): the byte offset
// is formed in 32 bits so that the access takes the scalar-base + 32-bit vector-offset
// form, and accesses to several planes at one node share the offset register.
// The base of each plane is made opaque (a wave-uniform value read from lane 0) so that the
// compiler keeps it in scalar registers instead of re-associating it with the offsets.
template <typename T>
__device__ __forceinline__ GP<T> plane_ptr(GP<T> base, int64_t plane_off) {
  const uint64_t u = (uint64_t)(base + plane_off);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  return (GP<T>)(((uint64_t)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ T ldg(GP<const T> base, uint32_t e) {
  return *(GP<const T>)((GP<const char>)base + e * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void stg(GP<T> base, uint32_t e, T v) {
  *(GP<T>)((GP<char>)base + e * (uint32_t)sizeof(T)) = v;
}
// streaming forms (no reuse expected): the line is a first candidate for eviction, which
// keeps the cache for data that neighbouring workgroups read again
template <typename T>
__device__ __forceinline__ T ldg_nt(GP<const T> base, uint32_t e) {
  return __builtin_nontemporal_load((GP<const T>)((GP<const char>)base + e * (uint32_t)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ void stg_nt(GP<T> base, uint32_t e, T v) {
  __builtin_nontemporal_store(v, (GP<T>)((GP<char>)base + e * (uint32_t)sizeof(T)));
}

// Physical constants of one block (FP64 on the host side of the kernel arguments).
struct Phys {
  double gamma;
  double gm1;         // gamma - 1
  double gm1inv;      // 1 / (gamma - 1)
  double inv2g;       // 1 / (2 gamma)
  double visc_scale;  // Ma / Re
  double heat_scale;  // Ma / (Re Pr (gamma - 1))
  double suth;
  double eps;
  int linear;  // ideal WENO weights
  int scheme;  // 0: modified AFWENO (characteristic space at nodes), 1: original (half points)
};

// The same constants in the compute type.
template <typename R>
struct Gas {
  R gamma, gm1, gm1inv, inv2g;
  __device__ __forceinline__ explicit Gas(const Phys& p)
      : gamma(R(p.gamma)), gm1(R(p.gm1)), gm1inv(R(p.gm1inv)), inv2g(R(p.inv2g)) {}
};

// ---- reciprocal and reciprocal square root ------------------------------------------
// Hardware estimate refined once by the third-order (Householder) correction of its
// relative error e: with e = 1 - x r, 1/x = r (1 + e + e^2 + ...), and with
// e = 1 - x y^2, 1/sqrt(x) = y (1 + e/2 + 3 e^2/8 + ...).  Keeping the terms through e^2
// leaves an error of order e^3; the FP64 estimates are good to about 5e-8, so that is
// ~1e-22, below the rounding of the result, in fewer operations than two Newton steps.
// Float takes the hardware estimates as they are (within 1 ulp): a refinement step would
// cost the FP32 sweeps, whose VALU issue is their bound, about 5% of their instructions.
__device__ __forceinline__ double rcp(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, fma(e, e, e), r);
}
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rsq(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(y, e * fma(0.375, e, 0.5), y);
}
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// ---- sixth-order central difference (Sec. 2 after Eq 8), unit spacing ---------------
// g(m) returns the value at offset m in [-3, 3] (the centre is not used).
template <typename R, typename F>
__device__ __forceinline__ R d6(F g) {
  return R(0.75) * (g(1) - g(-1)) - R(0.15) * (g(2) - g(-2)) + R(1.0 / 60.0) * (g(3) - g(-3));
}

// ---- Sutherland viscosity, mu(T) = T^1.5 (1+S)/(T+S) ------------------------------------
template <typename R>
__device__ __forceinline__ R viscosity(R T, R suth) {
  return T * sqrt(T) * (R(1) + suth) * rcp(T + suth);
}

// ---- Eq 4: inviscid flux through the hatted metric vector (mx, my, mz) --------------
template <typename R>
__device__ __forceinline__ void phys_flux(const R q[5], R mx, R my, R mz, const Gas<R>& G, R F[5]) {
  const R rinv = rcp(q[0]);
  const R u = q[1] * rinv, v = q[2] * rinv, w = q[3] * rinv;
  const R p = G.gm1 * (q[4] - R(0.5) * (q[1] * u + q[2] * v + q[3] * w));
  const R U = mx * u + my * v + mz * w;
  F[0] = q[0] * U;
  F[1] = q[1] * U + mx * p;
  F[2] = q[2] * U + my * p;
  F[3] = q[3] * U + mz * p;
  F[4] = (q[4] + p) * U;
}

// ---- Steger-Warming split flux of one sign (SIGN = +1 or -1) -------------------------
// With |m| the metric magnitude, k = m/|m| and theta = k.u:
// lambda_{1,2,3} = |m| theta = m.u, lambda_{4,5} = |m| (theta +- c),
// lambda^{+-} = (lambda +- |lambda|)/2 and
// F = rho/(2 gamma) [2 (gamma-1) l1 (1,u,v,w,|u|^2/2) + l4 (1, u + c k, H + c theta)
//                    + l5 (1, u - c k, H - c theta)].
template <int SIGN, typename R>
__device__ __forceinline__ void sw_flux(const R q[5], R mx, R my, R mz, const Gas<R>& G, R F[5]) {
  const R rinv = rcp(q[0]);
  const R u = q[1] * rinv, v = q[2] * rinv, w = q[3] * rinv;
  const R ke = R(0.5) * (u * u + v * v + w * w);
  const R p = G.gm1 * (q[4] - q[0] * ke);
  const R c2 = G.gamma * p * rinv;
  const R c = c2 * rsq(c2);
  const R m2 = mx * mx + my * my + mz * mz;
  const R minv = rsq(m2);
  const R mag = m2 * minv;
  const R mu = mx * u + my * v + mz * w;  // |m| theta
  const R H = (q[4] + p) * rinv;
  const R l1 = mu, l4 = mu + mag * c, l5 = mu - mag * c;
  const R a1 = R(0.5) * (l1 + R(SIGN) * fabs(l1));
  const R a4 = R(0.5) * (l4 + R(SIGN) * fabs(l4));
  const R a5 = R(0.5) * (l5 + R(SIGN) * fabs(l5));
  const R f = q[0] * G.inv2g;
  const R e1 = R(2) * G.gm1 * a1;
  const R s45 = a4 + a5;
  const R d45 = (a4 - a5) * c * minv;  // multiplies m (= |m| k)
  F[0] = f * (e1 + s45);
  F[1] = f * ((e1 + s45) * u + d45 * mx);
  F[2] = f * ((e1 + s45) * v + d45 * my);
  F[3] = f * ((e1 + s45) * w + d45 * mz);
  F[4] = f * (e1 * ke + s45 * H + d45 * mu);
}

// ---- characteristic basis at a node (Pulliam-Chaussee right eigenvectors) ------------
// R = M R_W with M = dQ/d(rho,u,v,w,p) and, in primitive form, columns 1-3
// (k_m, k x e_m, 0) for eigenvalue theta and columns 4-5 rho/(sqrt2 c) (1, +-c k/rho, c^2)
// for theta +- c; L = R^-1 = R_W^-1 M^-1 in closed form.
template <typename R>
struct Basis {
  R kx, ky, kz;     // unit direction
  R rkx, rky, rkz;  // k / rho          (projection of velocity differences)
  R skx, sky, skz;  // k / (sqrt2 rho)  (acoustic projection)
  R u, v, w, ke;
  R gc2;            // (gamma-1) / c^2
  R gpr;            // (gamma-1) / (sqrt2 rho c)
  R rho, a, b;      // rho, rho / (sqrt2 c), rho c / sqrt2
  R kr1, kr2, kr3;  // rho k (back-projection)
};

template <typename R>
__device__ __forceinline__ Basis<R> make_basis(const R q[5], R mx, R my, R mz, const Gas<R>& G) {
  Basis<R> B;
  const R minv = rsq(mx * mx + my * my + mz * mz);
  B.kx = mx * minv;
  B.ky = my * minv;
  B.kz = mz * minv;
  B.rho = q[0];
  const R rinv = rcp(q[0]);
  B.u = q[1] * rinv;
  B.v = q[2] * rinv;
  B.w = q[3] * rinv;
  B.ke = R(0.5) * (B.u * B.u + B.v * B.v + B.w * B.w);
  const R p = G.gm1 * (q[4] - B.rho * B.ke);
  const R c2 = G.gamma * p * rinv;
  const R cinv = rsq(c2);
  const R c = c2 * cinv;
  const R s2 = R(0.70710678118654752440);  // 1/sqrt2
  B.rkx = B.kx * rinv;
  B.rky = B.ky * rinv;
  B.rkz = B.kz * rinv;
  B.skx = B.rkx * s2;
  B.sky = B.rky * s2;
  B.skz = B.rkz * s2;
  B.gc2 = G.gm1 * cinv * cinv;
  B.gpr = G.gm1 * rinv * cinv * s2;
  B.a = B.rho * s2 * cinv;
  B.b = B.rho * c * s2;
  B.kr1 = B.rho * B.kx;
  B.kr2 = B.rho * B.ky;
  B.kr3 = B.rho * B.kz;
  return B;
}

// V = L Q' for a conserved vector Q' (characteristic projection).  With
// y = (Q'_1 - u Q'_0, Q'_2 - v Q'_0, Q'_3 - w Q'_0) (rho times the velocity perturbation)
// and P = (gamma-1) times the pressure perturbation:
//   V_{0..2} = k (Q'_0 - P/c^2) + (y x k)/rho,  V_{3,4} = (P/(rho c) +- k.y/rho)/sqrt2.
template <typename R>
__device__ __forceinline__ void project(const Basis<R>& B, const Gas<R>& G, const R qp[5], R V[5]) {
  (void)G;
  const R yu = qp[1] - B.u * qp[0];
  const R yv = qp[2] - B.v * qp[0];
  const R yw = qp[3] - B.w * qp[0];
  const R pp = B.ke * qp[0] - B.u * qp[1] - B.v * qp[2] - B.w * qp[3] + qp[4];  // P / (gamma-1)
  const R s = qp[0] - pp * B.gc2;
  V[0] = B.kx * s + (yv * B.rkz - yw * B.rky);
  V[1] = B.ky * s + (yw * B.rkx - yu * B.rkz);
  V[2] = B.kz * s + (yu * B.rky - yv * B.rkx);
  const R kd = B.skx * yu + B.sky * yv + B.skz * yw;
  const R pr = pp * B.gpr;
  V[3] = pr + kd;
  V[4] = pr - kd;
}

// Q' = R v (back to conserved variables).
template <typename R>
__device__ __forceinline__ void unproject(const Basis<R>& B, const Gas<R>& G, const R V[5], R qp[5]) {
  const R s2 = R(0.70710678118654752440);
  const R kv = B.kx * V[0] + B.ky * V[1] + B.kz * V[2];
  const R sp = V[3] + V[4];
  const R sm = (V[3] - V[4]) * s2;
  const R yr = kv + B.a * sp;
  // rho times the velocity components of R v
  const R yu = B.rho * (B.ky * V[2] - B.kz * V[1]) + B.kr1 * sm;
  const R yv = B.rho * (B.kz * V[0] - B.kx * V[2]) + B.kr2 * sm;
  const R yw = B.rho * (B.kx * V[1] - B.ky * V[0]) + B.kr3 * sm;
  qp[0] = yr;
  qp[1] = B.u * yr + yu;
  qp[2] = B.v * yr + yv;
  qp[3] = B.w * yr + yw;
  qp[4] = B.ke * yr + (B.u * yu + B.v * yv + B.w * yw) + (B.b * sp) * G.gm1inv;
}

// ---- WENO interpolation to both half points from one 5-point stencil ----------------
// Eqs 13-17 with the sub-stencil pairing of the fifth-order interpolant: ideal weight
// 1/16 and beta_1 on {i-2,i-1,i}, 5/8 on {i-1,i,i+1}, 5/16 on {i,i+1,i+2} for the
// left-biased value at i+1/2; the right-biased value at i-1/2 uses the mirror images with
// the same betas (modified AFWENO, Sec. 4.5.1).
// CORR: the same weights and values in the correction form (each value c plus one eighth of
// a combination of the differences that also give the smoothness indicators), which takes
// fewer FP64 instructions and a few more VGPRs
template <typename R, bool CORR = false>
__device__ __forceinline__ void weno_pair(R a, R b, R c, R d, R e, R eps, bool linear, R& vl, R& vr) {
  if constexpr (CORR) {
    // second differences d_j and combinations e_j of first differences of the sub-stencils;
    // the smoothness indicators of Eq 17 are 13/12 d_j^2 + 1/4 e_j^2
    const R d0 = a - R(2) * b + c, e0 = a - R(4) * b + R(3) * c;
    const R d1 = b - R(2) * c + d, e1 = b - d;
    const R d2 = c - R(2) * d + e, e2 = R(3) * c - R(4) * d + e;
    // the quadratic interpolants of Eq 14 as c + (.)/8: at i+1/2 d0 + 2 e0, d1 - 2 e1,
    // d2 - 2 e2; at i-1/2 the mirror images d0 - 2 e0, d1 + 2 e1, d2 + 2 e2
    const R A0 = d0 + R(2) * e0, A1 = d1 - R(2) * e1, A2 = d2 - R(2) * e2;
    const R B0 = d0 - R(2) * e0, B1 = d1 + R(2) * e1, B2 = d2 + R(2) * e2;
    if (linear) {  // ideal weights (1, 10, 5)/16 at i+1/2 and (5, 10, 1)/16 at i-1/2
      vl = c + (A0 + R(10) * A1 + R(5) * A2) * R(1.0 / 128.0);
      vr = c + (R(5) * B0 + R(10) * B1 + B2) * R(1.0 / 128.0);
      return;
    }
    // t_j = 4 (eps + beta_j): the common factor 4 cancels in Eq 15
    const R eps4 = R(4) * eps;
    const R t0 = eps4 + (R(13.0 / 3.0) * d0 * d0 + e0 * e0);
    const R t1 = eps4 + (R(13.0 / 3.0) * d1 * d1 + e1 * e1);
    const R t2 = eps4 + (R(13.0 / 3.0) * d2 * d2 + e2 * e2);
    // Eq 15 over a common denominator, as below
    const R s0 = t0 * t0, s1 = t1 * t1, s2 = t2 * t2;
    const R q0 = s1 * s2, q1 = s0 * s2, q2 = s0 * s1;
    const R nl = q0 * A0 + R(10) * (q1 * A1) + R(5) * (q2 * A2);
    const R nr = R(5) * (q0 * B0) + R(10) * (q1 * B1) + q2 * B2;
    const R dl = q0 + R(10) * q1 + R(5) * q2;
    const R dr = R(5) * q0 + R(10) * q1 + q2;
    if constexpr (sizeof(R) == 8) {
      const R inv = R(0.125) * rcp(dl * dr);
      vl = c + nl * dr * inv;
      vr = c + nr * dl * inv;
    } else {
      vl = c + R(0.125) * nl * rcp(dl);
      vr = c + R(0.125) * nr * rcp(dr);
    }
  } else {
    // quadratic interpolants of Eq 14 at i+1/2 (p) and their mirror images at i-1/2 (m),
    // pre-multiplied by their ideal weights (1/16, 5/8, 5/16) and (5/16, 5/8, 1/16)
    const R p0 = R(3.0 / 128.0) * a - R(5.0 / 64.0) * b + R(15.0 / 128.0) * c;
    const R p1 = R(-5.0 / 64.0) * b + R(15.0 / 32.0) * c + R(15.0 / 64.0) * d;
    const R p2 = R(15.0 / 128.0) * c + R(15.0 / 64.0) * d - R(5.0 / 128.0) * e;
    const R m0 = R(-5.0 / 128.0) * a + R(15.0 / 64.0) * b + R(15.0 / 128.0) * c;
    const R m1 = R(15.0 / 64.0) * b + R(15.0 / 32.0) * c - R(5.0 / 64.0) * d;
    const R m2 = R(15.0 / 128.0) * c - R(5.0 / 64.0) * d + R(3.0 / 128.0) * e;
    if (linear) {
      vl = p0 + p1 + p2;
      vr = m0 + m1 + m2;
      return;
    }
    // smoothness indicators of Eq 17 written as sums of squares of the second and first
    // differences (13/12 (.)^2 + 1/4 (.)^2, algebraically identical); the differences cancel
    // before squaring, so beta carries a relative rounding error instead of one of |v|^2.
    const R d0 = a - R(2) * b + c, e0 = a - R(4) * b + R(3) * c;
    const R d1 = b - R(2) * c + d, e1 = b - d;
    const R d2 = c - R(2) * d + e, e2 = R(3) * c - R(4) * d + e;
    const R k13 = R(13.0 / 12.0), k14 = R(0.25);
    const R t0 = eps + (k13 * d0 * d0 + k14 * e0 * e0);
    const R t1 = eps + (k13 * d1 * d1 + k14 * e1 * e1);
    const R t2 = eps + (k13 * d2 * d2 + k14 * e2 * e2);
    // Eq 15 over a common denominator: w_j ~ gamma_j / s_j with s_j = t_j^2 equals
    // gamma_j * prod_{k != j} s_k up to a common factor, which the normalisation removes.
    const R s0 = t0 * t0, s1 = t1 * t1, s2 = t2 * t2;
    const R q0 = s1 * s2, q1 = s0 * s2, q2 = s0 * s1;
    const R nl = q0 * p0 + q1 * p1 + q2 * p2;
    const R nr = q0 * m0 + q1 * m1 + q2 * m2;
    const R dl = R(0.0625) * q0 + R(0.625) * q1 + R(0.3125) * q2;
    const R dr = R(0.3125) * q0 + R(0.625) * q1 + R(0.0625) * q2;
    if constexpr (sizeof(R) == 8) {
      // one reciprocal for both sides (the product stays far inside the double range)
      const R inv = rcp(dl * dr);
      vl = nl * dr * inv;
      vr = nr * dl * inv;
    } else {
      vl = nl * rcp(dl);
      vr = nr * rcp(dr);
    }
  }
}

// ---- one WENO value: the left-biased value at i+1/2 from the values at i-2..i+2 -------
// (the right-biased value at i-1/2 is this function of the mirrored stencil e..a).
// Same sub-stencils, ideal weights and indicators as weno_pair, one side only; the
// original AFWENO takes the two sides of a half point from two different stencils.
template <typename R>
__device__ __forceinline__ R weno_left(R a, R b, R c, R d, R e, R eps, bool linear) {
  const R p0 = R(3.0 / 128.0) * a - R(5.0 / 64.0) * b + R(15.0 / 128.0) * c;
  const R p1 = R(-5.0 / 64.0) * b + R(15.0 / 32.0) * c + R(15.0 / 64.0) * d;
  const R p2 = R(15.0 / 128.0) * c + R(15.0 / 64.0) * d - R(5.0 / 128.0) * e;
  if (linear) return p0 + p1 + p2;
  const R d0 = a - R(2) * b + c, e0 = a - R(4) * b + R(3) * c;
  const R d1 = b - R(2) * c + d, e1 = b - d;
  const R d2 = c - R(2) * d + e, e2 = R(3) * c - R(4) * d + e;
  const R k13 = R(13.0 / 12.0), k14 = R(0.25);
  const R t0 = eps + (k13 * d0 * d0 + k14 * e0 * e0);
  const R t1 = eps + (k13 * d1 * d1 + k14 * e1 * e1);
  const R t2 = eps + (k13 * d2 * d2 + k14 * e2 * e2);
  const R s0 = t0 * t0, s1 = t1 * t1, s2 = t2 * t2;
  const R q0 = s1 * s2, q1 = s0 * s2, q2 = s0 * s1;
  return (q0 * p0 + q1 * p1 + q2 * p2) * rcp(R(0.0625) * q0 + R(0.625) * q1 + R(0.3125) * q2);
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
