// cfd_kernels.hip -- gfx950 kernels of libcfd: metrics, viscous prepass, AFWENO direction
// sweeps with the fused RK3 update, halo copies, boundary fills and reductions.
//
// Method: Ye et al., arXiv 2006.07964, Sec. 2 (Eqs 1-21) and Sec. 4.5 (modified AFWENO).
#include <hip/hip_runtime.h>

#include "../../include/cfd.h"
#include "cfd_kernels.hpp"

namespace cfd {

// =====================================================================================
// Metrics (Sec. 2, Eqs 7-8), FP64, setup only.
// =====================================================================================
struct CBox {
  int sx, sy, sz;  // extents of the tight coordinate-box layout (n + 12)
};

__device__ __forceinline__ int64_t cat(const MetricArgs& a, int i, int j, int k) {
  return ((int64_t)(k + kCHalo) * a.cld_j + (j + kCHalo)) * a.cld_i + (i + kCHalo);
}
__device__ __forceinline__ int64_t tat(const CBox& b, int i, int j, int k) {
  return ((int64_t)(k + kCHalo) * b.sy + (j + kCHalo)) * b.sx + (i + kCHalo);
}

// Pass 1: inner derivatives dX_c/d(dir) for every coordinate-box point whose 7-point
// stencil along dir fits in the box.  Plane 3*c + dir of dcoord.
__global__ __launch_bounds__(256) void k_metric_inner(MetricArgs a) {
  const CBox b{a.g.ni + 12, a.g.nj + 12, a.g.nk + 12};
  const int i = blockIdx.x * 64 + (threadIdx.x & 63) - kCHalo;
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6) - kCHalo;
  const int k = blockIdx.z - kCHalo;
  if (i >= a.g.ni + kCHalo || j >= a.g.nj + kCHalo) return;
  const int64_t plane = (int64_t)b.sx * b.sy * b.sz;
  const int n[3] = {a.g.ni, a.g.nj, a.g.nk};
  const int idx[3] = {i, j, k};
  for (int dir = 0; dir < 3; ++dir) {
    if (idx[dir] < -3 || idx[dir] >= n[dir] + 3) continue;
    const int64_t st = dir == 0 ? 1 : dir == 1 ? a.cld_i : a.cld_i * a.cld_j;
    for (int c = 0; c < 3; ++c) {
      const double* X = a.xyz + c * a.cplane + cat(a, i, j, k);
      a.dcoord[(3 * c + dir) * plane + tat(b, i, j, k)] =
          d6<double>([&](int m) { return X[m * st]; });
    }
  }
}

// Pass 2: conservative metrics (Eq 7) and Jacobian (Eq 8) on the halo-3 box.
// hatted metric (d, c) = d/d(d2) (X_{c1,d1} X_{c2}) - d/d(d1) (X_{c1,d2} X_{c2}) with
// c1 = c+1, c2 = c+2, d1 = d+1, d2 = d+2 (mod 3).
__global__ __launch_bounds__(256) void k_metric_outer(MetricArgs a) {
  const CBox b{a.g.ni + 12, a.g.nj + 12, a.g.nk + 12};
  const int i = blockIdx.x * 64 + (threadIdx.x & 63) - kHalo;
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6) - kHalo;
  const int k = blockIdx.z - kHalo;
  if (i >= a.g.ni + kHalo || j >= a.g.nj + kHalo) return;
  const int64_t cplane = (int64_t)b.sx * b.sy * b.sz;
  const int64_t tp = tat(b, i, j, k);
  const int64_t cp = cat(a, i, j, k);
  const int64_t tst[3] = {1, b.sx, (int64_t)b.sx * b.sy};
  const int64_t cst[3] = {1, a.cld_i, a.cld_i * a.cld_j};
  const int64_t p = at(a.g, i, j, k);
  for (int d = 0; d < 3; ++d) {
    const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
    for (int c = 0; c < 3; ++c) {
      const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
      const double* Xb = a.xyz + c2 * a.cplane + cp;
      const double* Da = a.dcoord + (3 * c1 + d1) * cplane + tp;  // X_{c1} along d1
      const double* Db = a.dcoord + (3 * c1 + d2) * cplane + tp;  // X_{c1} along d2
      const double t1 = d6<double>([&](int m) { return Da[m * tst[d2]] * Xb[m * cst[d2]]; });
      const double t2 = d6<double>([&](int m) { return Db[m * tst[d1]] * Xb[m * cst[d1]]; });
      a.met[(3 * d + c) * a.g.plane + p] = t1 - t2;
    }
  }
  double D[3][3];  // D[c][dir] = dX_c/d(dir)
  for (int c = 0; c < 3; ++c)
    for (int dir = 0; dir < 3; ++dir) D[c][dir] = a.dcoord[(3 * c + dir) * cplane + tp];
  const double jinv = D[0][0] * D[1][1] * D[2][2] - D[0][0] * D[1][2] * D[2][1] + D[0][1] * D[1][2] * D[2][0] -
                      D[0][1] * D[1][0] * D[2][2] + D[0][2] * D[1][0] * D[2][1] - D[0][2] * D[1][1] * D[2][0];
  if (!(jinv > 0.0)) atomicOr(a.bad, 1);
  a.met[9 * a.g.plane + p] = 1.0 / jinv;
}

hipError_t launch_metrics(const MetricArgs& a, hipStream_t s) {
  dim3 blk(256);
  dim3 g1((a.g.ni + 12 + 63) / 64, (a.g.nj + 12 + 3) / 4, a.g.nk + 12);
  hipLaunchKernelGGL(k_metric_inner, g1, blk, 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 g2((a.g.ni + 6 + 63) / 64, (a.g.nj + 6 + 3) / 4, a.g.nk + 6);
  hipLaunchKernelGGL(k_metric_outer, g2, blk, 0, s, a);
  return hipGetLastError();
}

// =====================================================================================
// Viscous prepass (Eqs 5, 6, 21): nodal viscous fluxes of all three directions.
// Plane 4*d + (n-1) holds component n = 1..4 of the direction-d flux, divided by J.
// =====================================================================================
template <typename R>
__global__ __launch_bounds__(256) void k_visc(ViscArgs a) {
  const Geom& g = a.g;
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int k = blockIdx.z;
  if (i >= g.ni || j >= g.nj) return;
  const int64_t p = at(g, i, j, k);
  const R gamma = R(a.ph.gamma), gm1 = gamma - R(1);
  const int64_t st[3] = {1, g.ld_i, g.ld_i * g.ld_j};
  R gr[4][3];  // d(u, v, w, T)/d(xi, eta, zeta)
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int n = 0; n < 4; ++n) gr[n][d] = R(0);
#pragma unroll
    for (int m = -3; m <= 3; ++m) {
      if (m == 0) continue;
      const R wgt = (m == 1 || m == -1) ? R(0.75) : (m == 2 || m == -2) ? R(-0.15) : R(1.0 / 60.0);
      const R sgn = m > 0 ? R(1) : R(-1);
      const int64_t pp = p + m * st[d];
      R q[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) q[v] = R(a.q[v * g.plane + pp]);
      const R rinv = R(1) / q[0];
      const R u = q[1] * rinv, v = q[2] * rinv, w = q[3] * rinv;
      const R T = gamma * gm1 * (q[4] * rinv - R(0.5) * (u * u + v * v + w * w));
      const R f = sgn * wgt;
      gr[0][d] += f * u;
      gr[1][d] += f * v;
      gr[2][d] += f * w;
      gr[3][d] += f * T;
    }
  }
  R mh[3][3];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int c = 0; c < 3; ++c) mh[d][c] = R(a.met[(3 * d + c) * g.plane + p]);
  const R J = R(a.met[9 * g.plane + p]);
  R dx[4][3];  // d(u, v, w, T)/d(x, y, z), Eq 21
#pragma unroll
  for (int n = 0; n < 4; ++n)
#pragma unroll
    for (int c = 0; c < 3; ++c) dx[n][c] = J * (mh[0][c] * gr[n][0] + mh[1][c] * gr[n][1] + mh[2][c] * gr[n][2]);
  R q0[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) q0[v] = R(a.q[v * g.plane + p]);
  const R rinv = R(1) / q0[0];
  const R u = q0[1] * rinv, v = q0[2] * rinv, w = q0[3] * rinv;
  const R T = gamma * gm1 * (q0[4] * rinv - R(0.5) * (u * u + v * v + w * w));
  const R mu = viscosity(T, R(a.ph.suth));
  const R vs = R(a.ph.visc_scale) * mu;
  const R lam = R(-2.0 / 3.0) * vs;
  const R div = dx[0][0] + dx[1][1] + dx[2][2];
  R tau[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) tau[r][c] = vs * (dx[r][c] + dx[c][r]) + (r == c ? lam * div : R(0));
  const R hs = R(a.ph.heat_scale) * mu;
  R bet[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) bet[c] = u * tau[0][c] + v * tau[1][c] + w * tau[2][c] + hs * dx[3][c];
  R* out = static_cast<R*>(a.vis);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int n = 0; n < 3; ++n)
      out[(4 * d + n) * g.plane + p] = mh[d][0] * tau[n][0] + mh[d][1] * tau[n][1] + mh[d][2] * tau[n][2];
    out[(4 * d + 3) * g.plane + p] = mh[d][0] * bet[0] + mh[d][1] * bet[1] + mh[d][2] * bet[2];
  }
}

template <typename R>
hipError_t launch_visc(const ViscArgs& a, hipStream_t s) {
  dim3 grid((a.g.ni + 63) / 64, (a.g.nj + 3) / 4, a.g.nk);
  hipLaunchKernelGGL(k_visc<R>, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}
template hipError_t launch_visc<double>(const ViscArgs&, hipStream_t);
template hipError_t launch_visc<float>(const ViscArgs&, hipStream_t);

// =====================================================================================
// Direction sweep: modified AFWENO inviscid derivative (Sec. 4.5.1, Figs 10-11, Eq 19),
// the sixth-order derivative of the viscous flux, and the output (partial sum, R, or the
// RK3 stage of Eq 20).
//
// A workgroup owns a tile of TW grid lines (cross direction c1) by TS output nodes along
// the sweep direction.  Phase 1 evaluates, per node, the characteristic WENO pair and the
// two split fluxes (nodes d0-1 .. d0+TS) and the nodal fluxes (d0-3 .. d0+TS+2) into LDS;
// phase 2 assembles Eq 19 per output node.
// =====================================================================================
template <int DIR, int TW>
struct LdsIdx {
  // LDS order puts the lane-fastest tile axis innermost: along the line for DIR 0
  // (lanes walk i), across lines otherwise.
  static __device__ __forceinline__ int f(int v, int w, int s, int len) {
    return DIR == 0 ? (v * TW + w) * len + s : (v * len + s) * TW + w;
  }
};

template <int DIR, typename R, int TW, int TS>
__global__ __launch_bounds__(256) void k_sweep(SweepArgs a) {
  constexpr int NW = TS + 2;  // nodes with a WENO evaluation
  constexpr int NN = TS + 6;  // nodes with a nodal flux
  constexpr int NH = TS + 1;  // half points
  __shared__ R sFp[5 * TW * NH];
  __shared__ R sFm[5 * TW * NH];
  __shared__ R sFn[5 * TW * NN];
  using L = LdsIdx<DIR, TW>;

  const Geom& g = a.g;
  const int nd = DIR == 0 ? g.ni : DIR == 1 ? g.nj : g.nk;
  const int n1 = DIR == 0 ? g.nj : g.ni;
  const int64_t sd = DIR == 0 ? 1 : DIR == 1 ? g.ld_i : g.ld_i * g.ld_j;
  const int64_t s1 = DIR == 0 ? g.ld_i : 1;
  const int64_t s2 = DIR == 2 ? g.ld_i : g.ld_i * g.ld_j;
  const int tile1 = blockIdx.x % a.tiles_c1;
  const int tiled = blockIdx.x / a.tiles_c1;
  const int c1_0 = tile1 * TW;
  const int d0 = tiled * TS;
  const int64_t origin = at(g, 0, 0, 0) + (int64_t)blockIdx.y * s2;
  const double* Q = a.q;
  const double* met = a.met;
  const int64_t plane = g.plane;
  const R gamma = R(a.ph.gamma);
  const R eps = R(a.ph.eps);
  const bool linear = a.ph.linear != 0;
  const double* mx = met + (3 * DIR + 0) * plane;
  const double* my = met + (3 * DIR + 1) * plane;
  const double* mz = met + (3 * DIR + 2) * plane;

  if (a.do_inv) {
    // ---- nodal fluxes, Eq 4 -----------------------------------------------------------
    for (int e = threadIdx.x; e < TW * NN; e += 256) {
      const int s = DIR == 0 ? e % NN : e / TW;
      const int w = DIR == 0 ? e / NN : e % TW;
      const int n = d0 - 3 + s;
      const int c1 = c1_0 + w;
      if (c1 >= n1 || n > nd + 2) continue;
      const int64_t p = origin + c1 * s1 + n * sd;
      R q[5], F[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) q[v] = R(Q[v * plane + p]);
      phys_flux(q, R(mx[p]), R(my[p]), R(mz[p]), gamma, F);
#pragma unroll
      for (int v = 0; v < 5; ++v) sFn[L::f(v, w, s, NN)] = F[v];
    }
    // ---- characteristic WENO pair and split fluxes ------------------------------------
    for (int e = threadIdx.x; e < TW * NW; e += 256) {
      const int s = DIR == 0 ? e % NW : e / TW;
      const int w = DIR == 0 ? e / NW : e % TW;
      const int n = d0 - 1 + s;
      const int c1 = c1_0 + w;
      if (c1 >= n1 || n > nd) continue;
      const bool need_p = s <= TS && n <= nd - 1;  // F+ at n+1/2
      const bool need_m = s >= 1;                  // F- at n-1/2
      if (!need_p && !need_m) continue;
      const int64_t p = origin + c1 * s1 + n * sd;
      R q0[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) q0[v] = R(Q[v * plane + p]);
      const Basis<R> B = make_basis(q0, R(mx[p]), R(my[p]), R(mz[p]), gamma);
      R V[5][5];  // V[t][field] at node n + t - 2
#pragma unroll
      for (int t = 0; t < 5; ++t) {
        R qq[5];
        const int64_t pt = p + (t - 2) * sd;
#pragma unroll
        for (int v = 0; v < 5; ++v) qq[v] = R(Q[v * plane + pt]);
        project(B, qq, V[t]);
      }
      R vl[5], vr[5];
#pragma unroll
      for (int f = 0; f < 5; ++f) weno_pair(V[0][f], V[1][f], V[2][f], V[3][f], V[4][f], eps, linear, vl[f], vr[f]);
      if (need_p) {
        R ul[5], F[5];
        unproject(B, vl, ul);
        const R hx = R(half_metric([&](int m) { return mx[p + m * sd]; }));
        const R hy = R(half_metric([&](int m) { return my[p + m * sd]; }));
        const R hz = R(half_metric([&](int m) { return mz[p + m * sd]; }));
        sw_flux<+1>(ul, hx, hy, hz, gamma, F);
#pragma unroll
        for (int v = 0; v < 5; ++v) sFp[L::f(v, w, s, NH)] = F[v];
      }
      if (need_m) {
        R ur[5], F[5];
        unproject(B, vr, ur);
        const int64_t pm = p - sd;  // half point n-1/2 = (n-1)+1/2
        const R hx = R(half_metric([&](int m) { return mx[pm + m * sd]; }));
        const R hy = R(half_metric([&](int m) { return my[pm + m * sd]; }));
        const R hz = R(half_metric([&](int m) { return mz[pm + m * sd]; }));
        sw_flux<-1>(ur, hx, hy, hz, gamma, F);
#pragma unroll
        for (int v = 0; v < 5; ++v) sFm[L::f(v, w, s - 1, NH)] = F[v];
      }
    }
    __syncthreads();
  }

  // ---- assembly per output node ---------------------------------------------------------
  const R* vis = static_cast<const R*>(a.vis);
  const R* rin = static_cast<const R*>(a.rt_in);
  for (int e = threadIdx.x; e < TW * TS; e += 256) {
    const int s = DIR == 0 ? e % TS : e / TW;
    const int w = DIR == 0 ? e / TS : e % TW;
    const int n = d0 + s;
    const int c1 = c1_0 + w;
    if (c1 >= n1 || n >= nd) continue;
    const int64_t p = origin + c1 * s1 + n * sd;
    R r[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) r[v] = R(0);
    if (a.do_inv) {
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const R fp = sFp[L::f(v, w, s + 1, NH)] + sFm[L::f(v, w, s + 1, NH)];
        const R fm = sFp[L::f(v, w, s, NH)] + sFm[L::f(v, w, s, NH)];
        const R D = fp - fm + R(17.0 / 256.0) * (sFn[L::f(v, w, s + 4, NN)] - sFn[L::f(v, w, s + 2, NN)]) -
                    R(13.0 / 320.0) * (sFn[L::f(v, w, s + 5, NN)] - sFn[L::f(v, w, s + 1, NN)]) +
                    R(19.0 / 3840.0) * (sFn[L::f(v, w, s + 6, NN)] - sFn[L::f(v, w, s, NN)]);
        r[v] = -D;
      }
    }
    if (a.do_vis) {
#pragma unroll
      for (int v = 1; v < 5; ++v) {
        const R* vp = vis + (4 * DIR + v - 1) * plane + p;
        r[v] += d6<R>([&](int m) { return vp[m * sd]; });
      }
    }
    if (a.has_prev) {
#pragma unroll
      for (int v = 0; v < 5; ++v) r[v] += rin[v * plane + p];
    }
    if (a.out_kind == kOutPartial) {
      R* ro = static_cast<R*>(a.rt_out);
#pragma unroll
      for (int v = 0; v < 5; ++v) ro[v * plane + p] = r[v];
    } else {
      const double J = met[9 * plane + p];
      if (a.out_kind == kOutRhs) {
#pragma unroll
        for (int v = 0; v < 5; ++v) a.out[v * plane + p] = J * double(r[v]);
      } else {
        const double dt = a.dt_dev ? *a.dt_dev : a.dt;
        const double cdt = a.cc * dt * J;
#pragma unroll
        for (int v = 0; v < 5; ++v)
          a.out[v * plane + p] = a.ca * a.qn[v * plane + p] + a.cb * Q[v * plane + p] + cdt * double(r[v]);
      }
    }
  }
}

template <typename R>
hipError_t launch_sweep(int dir, SweepArgs a, hipStream_t s) {
  constexpr int TW = 16, TS = 14;
  const int nd = dir == 0 ? a.g.ni : dir == 1 ? a.g.nj : a.g.nk;
  const int n1 = dir == 0 ? a.g.nj : a.g.ni;
  const int n2 = dir == 2 ? a.g.nj : a.g.nk;
  a.tiles_c1 = (n1 + TW - 1) / TW;
  dim3 grid(a.tiles_c1 * ((nd + TS - 1) / TS), n2);
  if (dir == 0)
    hipLaunchKernelGGL((k_sweep<0, R, TW, TS>), grid, dim3(256), 0, s, a);
  else if (dir == 1)
    hipLaunchKernelGGL((k_sweep<1, R, TW, TS>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_sweep<2, R, TW, TS>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}
template hipError_t launch_sweep<double>(int, SweepArgs, hipStream_t);
template hipError_t launch_sweep<float>(int, SweepArgs, hipStream_t);

// =====================================================================================
// Halo copies across 1-to-1 faces (ghost layer m of the destination face <- interior
// layer m-1 inside the source face), boundary fills.
// =====================================================================================
template <typename T>
__global__ __launch_bounds__(256) void k_copy(const CopySeg* segs, PtrTable t) {
  const CopySeg S = segs[blockIdx.y];
  const int64_t per_plane = (int64_t)S.na * S.nb * kHalo;
  const int64_t total = per_plane * S.nplanes;
  T* dst = static_cast<T*>(t.p[S.dst]);
  const T* src = static_cast<const T*>(t.p[S.src]);
  const int64_t pd = t.plane[S.dst], ps = t.plane[S.src];
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int v = S.plane0 + (int)(e / per_plane);
    int64_t r = e % per_plane;
    const int a = (int)(r % S.na);
    r /= S.na;
    const int l = (int)(r % kHalo);
    const int b = (int)(r / kHalo);
    dst[v * pd + S.dst_off + a * S.dst_sa + b * S.dst_sb + l * S.dst_sl] =
        src[v * ps + S.src_off + a * S.src_sa + b * S.src_sb + l * S.src_sl];
  }
}

template <typename T>
hipError_t launch_copy(const CopySeg* segs_dev, int nseg, int max_elems, const PtrTable& t, hipStream_t s) {
  if (nseg == 0) return hipSuccess;
  int bx = (max_elems + 255) / 256;
  if (bx > 4096) bx = 4096;
  if (bx < 1) bx = 1;
  hipLaunchKernelGGL(k_copy<T>, dim3(bx, nseg), dim3(256), 0, s, segs_dev, t);
  return hipGetLastError();
}
template hipError_t launch_copy<double>(const CopySeg*, int, int, const PtrTable&, hipStream_t);
template hipError_t launch_copy<float>(const CopySeg*, int, int, const PtrTable&, hipStream_t);

__global__ __launch_bounds__(256) void k_wall_reset(const BcSeg* segs, BcArgs A) {
  const BcSeg S = segs[blockIdx.y];
  if (S.kind != CFD_BC_WALL) return;
  double* Q = static_cast<double*>(A.t.p[S.blk]);
  const int64_t pl = A.t.plane[S.blk];
  const int64_t total = (int64_t)S.na * S.nb;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int a = (int)(e % S.na), b = (int)(e / S.na);
    const int64_t p = S.wall_off + a * S.sa + b * S.sb;
    Q[1 * pl + p] = 0.0;
    Q[2 * pl + p] = 0.0;
    Q[3 * pl + p] = 0.0;
    Q[4 * pl + p] = Q[p] * A.t_wall / (A.gamma * (A.gamma - 1.0));
  }
}

__global__ __launch_bounds__(256) void k_ghost_fill(const BcSeg* segs, BcArgs A) {
  const BcSeg S = segs[blockIdx.y];
  double* Q = static_cast<double*>(A.t.p[S.blk]);
  const int64_t pl = A.t.plane[S.blk];
  const int64_t total = (int64_t)S.na * S.nb * kHalo;
  const double gm1 = A.gamma - 1.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int a = (int)(e % S.na);
    const int64_t r = e / S.na;
    const int m = 1 + (int)(r % kHalo);
    const int b = (int)(r / kHalo);
    const int64_t pw = S.wall_off + a * S.sa + b * S.sb;
    const int64_t pg = pw + m * S.sout, pm = pw - m * S.sout;
    if (S.kind == CFD_BC_FARFIELD) {
      for (int v = 0; v < 5; ++v) Q[v * pl + pg] = A.qinf[v];
    } else {
      const double rho = Q[pm], rinv = 1.0 / rho;
      const double u = Q[pl + pm] * rinv, v = Q[2 * pl + pm] * rinv, w = Q[3 * pl + pm] * rinv;
      const double ke = 0.5 * (u * u + v * v + w * w);
      const double p = gm1 * (Q[4 * pl + pm] - rho * ke);
      const double T = A.gamma * p * rinv;
      const double Tg = 2.0 * A.t_wall - T;
      const double rg = A.gamma * p / Tg;
      Q[pg] = rg;
      Q[pl + pg] = -rg * u;
      Q[2 * pl + pg] = -rg * v;
      Q[3 * pl + pg] = -rg * w;
      Q[4 * pl + pg] = p / gm1 + rg * ke;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_visc_ghost(const BcSeg* segs, PtrTable t) {
  const BcSeg S = segs[blockIdx.y];
  T* V = static_cast<T*>(t.p[S.blk]);
  const int64_t pl = t.plane[S.blk];
  const int64_t total = (int64_t)S.na * S.nb * kHalo * 4;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int a = (int)(e % S.na);
    int64_t r = e / S.na;
    const int m = 1 + (int)(r % kHalo);
    r /= kHalo;
    const int n = (int)(r % 4);
    const int b = (int)(r / 4);
    const int64_t pw = S.wall_off + a * S.sa + b * S.sb;
    T* P = V + (4 * S.axis + n) * pl;
    P[pw + m * S.sout] = T(2) * P[pw] - P[pw - m * S.sout];
  }
}

static dim3 bc_grid(int max_elems, int nseg) {
  int bx = (max_elems + 255) / 256;
  if (bx > 4096) bx = 4096;
  if (bx < 1) bx = 1;
  return dim3(bx, nseg);
}

hipError_t launch_wall_reset(const BcSeg* segs_dev, int nseg, int max_elems, const BcArgs& a, hipStream_t s) {
  if (nseg == 0) return hipSuccess;
  hipLaunchKernelGGL(k_wall_reset, bc_grid(max_elems, nseg), dim3(256), 0, s, segs_dev, a);
  return hipGetLastError();
}
hipError_t launch_ghost_fill(const BcSeg* segs_dev, int nseg, int max_elems, const BcArgs& a, hipStream_t s) {
  if (nseg == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ghost_fill, bc_grid(max_elems * kHalo, nseg), dim3(256), 0, s, segs_dev, a);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_visc_ghost(const BcSeg* segs_dev, int nseg, int max_elems, const PtrTable& t, hipStream_t s) {
  if (nseg == 0) return hipSuccess;
  hipLaunchKernelGGL(k_visc_ghost<T>, bc_grid(max_elems * kHalo * 4, nseg), dim3(256), 0, s, segs_dev, t);
  return hipGetLastError();
}
template hipError_t launch_visc_ghost<double>(const BcSeg*, int, int, const PtrTable&, hipStream_t);
template hipError_t launch_visc_ghost<float>(const BcSeg*, int, int, const PtrTable&, hipStream_t);

// =====================================================================================
// Reductions: CFL spectral-radius maximum and finiteness.
// =====================================================================================
__global__ __launch_bounds__(256) void k_dt_max(Geom g, const double* q, const double* met, double gamma,
                                                unsigned long long* acc) {
  __shared__ double red[256];
  double best = 0.0;
  const int64_t total = (int64_t)g.ni * g.nj * g.nk;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e % g.ni);
    const int64_t r = e / g.ni;
    const int j = (int)(r % g.nj), k = (int)(r / g.nj);
    const int64_t p = at(g, i, j, k);
    const double rho = q[p], rinv = 1.0 / rho;
    const double u = q[g.plane + p] * rinv, v = q[2 * g.plane + p] * rinv, w = q[3 * g.plane + p] * rinv;
    const double pr = (gamma - 1.0) * (q[4 * g.plane + p] - 0.5 * rho * (u * u + v * v + w * w));
    const double c = sqrt(gamma * pr * rinv);
    const double J = met[9 * g.plane + p];
    double sum = 0.0;
    for (int d = 0; d < 3; ++d) {
      const double ax = J * met[(3 * d) * g.plane + p], ay = J * met[(3 * d + 1) * g.plane + p],
                   az = J * met[(3 * d + 2) * g.plane + p];
      sum += fabs(ax * u + ay * v + az * w) + c * sqrt(ax * ax + ay * ay + az * az);
    }
    best = fmax(best, sum);
  }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  // non-negative doubles order like their bit patterns
  if (threadIdx.x == 0) atomicMax(acc, (unsigned long long)__double_as_longlong(red[0]));
}

hipError_t launch_dt_max(const Geom& g, const double* q, const double* met, double gamma, unsigned long long* acc,
                         hipStream_t s) {
  const int64_t total = (int64_t)g.ni * g.nj * g.nk;
  int bx = (int)((total + 255) / 256);
  if (bx > 8192) bx = 8192;
  hipLaunchKernelGGL(k_dt_max, dim3(bx), dim3(256), 0, s, g, q, met, gamma, acc);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_finite(Geom g, const double* q, int* flag) {
  const int64_t total = (int64_t)g.ni * g.nj * g.nk;
  int bad = 0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e % g.ni);
    const int64_t r = e / g.ni;
    const int j = (int)(r % g.nj), k = (int)(r / g.nj);
    const int64_t p = at(g, i, j, k);
    for (int v = 0; v < 5; ++v) bad |= !isfinite(q[v * g.plane + p]);
  }
  if (bad) atomicOr(flag, 1);
}

hipError_t launch_finite(const Geom& g, const double* q, int* flag, hipStream_t s) {
  const int64_t total = (int64_t)g.ni * g.nj * g.nk;
  int bx = (int)((total + 255) / 256);
  if (bx > 8192) bx = 8192;
  hipLaunchKernelGGL(k_finite, dim3(bx), dim3(256), 0, s, g, q, flag);
  return hipGetLastError();
}

}  // namespace cfd
