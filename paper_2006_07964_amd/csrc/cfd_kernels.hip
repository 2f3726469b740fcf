// cfd_kernels.hip -- gfx950 kernels of libcfd: metrics, viscous prepass, AFWENO direction
// sweeps with the fused RK3 update, halo copies, boundary fills and reductions.
//
// Method: Ye et al., arXiv 2006.07964, Sec. 2 (Eqs 1-21) and Sec. 4.5 (modified AFWENO).
#include <type_traits>
#include <hip/hip_runtime.h>

#include "../../include/cfd.h"
#include "cfd_kernels.hpp"

namespace cfd {

// Workgroups are handed to the eight XCDs round-robin (id mod 8).  Remap the id so that
// each XCD walks a contiguous range of logical tiles; with the sweep-direction tile index
// fastest, tiles that share halo rows run back to back on the same L2.
__device__ __forceinline__ int xcd_remap(int wg, int nwg) {
  const int x = wg & 7, local = wg >> 3;
  const int q = nwg >> 3, r = nwg & 7;
  return x * q + (x < r ? x : r) + local;
}

// Persistent schedule: the `total` work items are split into eight contiguous ranges, one
// per XCD; this workgroup is number *lane_wg of the *nwg_x workgroups on its XCD.
__device__ __forceinline__ void xcd_range(int total, int* start, int* count, int* lane_wg, int* nwg_x) {
  const int x = blockIdx.x & 7;
  const int q = total >> 3, r = total & 7;
  *start = x * q + (x < r ? x : r);
  *count = q + (x < r ? 1 : 0);
  *lane_wg = blockIdx.x >> 3;
  const int G = gridDim.x;
  *nwg_x = (G >> 3) + (x < (G & 7) ? 1 : 0);
}

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
//
// A workgroup owns a VI x VJ tile of (i, j) columns and marches along k through a chunk
// of kc planes.  Each thread keeps the primitives (u, v, w, T) of its own column at
// k-3..k+3 in registers for the zeta derivative; the primitives of plane k, with three
// halo columns / rows, go through LDS for the xi and eta derivatives.  Every primitive is
// formed about twice per chunk instead of at each of its eighteen stencil uses, and Q is
// read once per column.
// =====================================================================================
constexpr int VI = 64, VJ = 16, VNT = VI * VJ;
constexpr int kViscChunk = 128;    // most planes per workgroup (fewer when nk is smaller)
constexpr int kViscMinTiles = 256;  // workgroups a single-block launch aims for (one per CU)

template <typename R>
struct ViscShared {
  R p[4][VJ + 6][VI + 6];  // (u, v, w, T) of plane k at (j - j0 + 3, i - i0 + 3)
};

template <typename R>
__device__ __forceinline__ void primitives(GP<const double> Q, int64_t plane, uint32_t p, R gg, R out[4]) {
  R q[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) q[v] = R(ldg(plane_ptr(Q, v * plane), p));
  const R rinv = rcp(q[0]);
  out[0] = q[1] * rinv;
  out[1] = q[2] * rinv;
  out[2] = q[3] * rinv;
  out[3] = gg * (q[4] * rinv - R(0.5) * (out[0] * out[0] + out[1] * out[1] + out[2] * out[2]));
}

// One-sided closure of the viscous derivatives (Sec. 4.5.2 mentions one-sided differences
// near block boundaries without giving them): the derivative at node r = 0, 1, 2 of a face
// of the degree-6 polynomial through the seven nodes nearest it (node 0 on the face, node
// m at distance m inside) is sum_m kOS6[r][m] f(m) (Lagrange derivative weights, unit
// spacing); a node r away from the high face takes the mirror image with the opposite sign.
__constant__ double kOS6[3][7] = {
    {-49.0 / 20.0, 6.0, -15.0 / 2.0, 20.0 / 3.0, -15.0 / 4.0, 6.0 / 5.0, -1.0 / 6.0},
    {-1.0 / 6.0, -77.0 / 60.0, 5.0 / 2.0, -5.0 / 3.0, 5.0 / 6.0, -1.0 / 4.0, 1.0 / 30.0},
    {1.0 / 30.0, -2.0 / 5.0, -7.0 / 12.0, 4.0 / 3.0, -1.0 / 2.0, 2.0 / 15.0, -1.0 / 60.0}};

// Window of the one-sided closure for the node at index n of an axis of nd nodes, given
// the face mask bits of that axis (bit 0: low face one-sided, bit 1: high face): returns
// false for a central node, else the first window node, the weight row and the sign.
__device__ __forceinline__ bool one_sided_window(int bits, int n, int nd, int* first, int* row, int* sign) {
  if ((bits & 1) && n < 3) {
    *first = 0;
    *row = n;
    *sign = 1;
    return true;
  }
  if ((bits & 2) && n > nd - 4) {
    *first = nd - 7;
    *row = nd - 1 - n;
    *sign = -1;
    return true;
  }
  return false;
}
__device__ __forceinline__ double os6_weight(int row, int sign, int m) {
  return sign > 0 ? kOS6[row][m] : -kOS6[row][6 - m];
}

// d/dn of a field on a 7-point line, g(m) = value at offset m (sixth-order central)
template <typename R, typename F>
__device__ __forceinline__ R grad6(F g) {
  R s = R(0);
#pragma unroll
  for (int m = -3; m <= 3; ++m) {
    if (m == 0) continue;
    const R wgt = (m == 1 || m == -1) ? R(0.75) : (m == 2 || m == -2) ? R(-0.15) : R(1.0 / 60.0);
    s += (m > 0 ? wgt : -wgt) * g(m);
  }
  return s;
}

// OS: the block may have faces with the one-sided closure (a separate instantiation, so
// that blocks without them keep the register budget of the plain prepass)
template <typename R, bool OS>
__device__ __forceinline__ void visc_tile(const ViscArgs& a, int t, ViscShared<R>& sh) {
  const Geom& g = a.g;
  const int nti = (g.ni + VI - 1) / VI, ntj = (g.nj + VJ - 1) / VJ;
  const int i0 = (t % nti) * VI, j0 = ((t / nti) % ntj) * VJ;
  const int k0 = (t / (nti * ntj)) * a.kc;
  const int k1 = min(k0 + a.kc, g.nk);
  const int ti = threadIdx.x % VI, tj = threadIdx.x / VI;
  const int i = i0 + ti, j = j0 + tj;
  const bool own = i < g.ni + kHalo && j < g.nj + kHalo;  // column inside the stored array
  const bool act = i < g.ni && j < g.nj;                  // column with outputs
  const uint32_t sk = (uint32_t)(g.ld_i * g.ld_j);
  const uint32_t pc = (uint32_t)at(g, own ? i : 0, own ? j : 0, 0);  // (i, j, k = 0); plane < 2^29
  // halo node of this thread in plane k: eta rows below / above the tile, xi columns
  // left / right of it (the stencil is a cross, corners are not needed)
  int hi = 0, hj = 0;
  const int h = threadIdx.x;
  if (h < 2 * 3 * VI) {
    hi = i0 + h % VI;
    hj = h < 3 * VI ? j0 - 3 + h / VI : j0 + VJ + (h - 3 * VI) / VI;
  } else if (h < 2 * 3 * VI + 2 * 3 * VJ) {
    const int e = h - 2 * 3 * VI;
    hj = j0 + (e % (3 * VJ)) / 3;
    hi = e < 3 * VJ ? i0 - 3 + e % 3 : i0 + VI + e % 3;
  } else {
    hi = g.ni + kHalo;  // no halo node
  }
  const bool hval = hi < g.ni + kHalo && hj < g.nj + kHalo;
  const uint32_t ph = (uint32_t)at(g, hval ? hi : 0, hval ? hj : 0, 0);

  const R gg = R(a.ph.gamma) * (R(a.ph.gamma) - R(1));
  const GP<const double> Q = to_global(a.q);
  const GP<const R> met = to_global(static_cast<const R*>(a.met_r));
  const GP<R> out = to_global(static_cast<R*>(a.vis));
  const int64_t plane = g.plane;
  R P[7][4];  // own column, planes k-3 .. k+3
  if (own) {
#pragma unroll
    for (int m = 0; m < 6; ++m) primitives<R>(Q, plane, pc + (uint32_t)(k0 - 3 + m) * sk, gg, P[m]);
  }
  for (int k = k0; k < k1; ++k) {
    if (own) primitives<R>(Q, plane, pc + (uint32_t)(k + 3) * sk, gg, P[6]);
    if (own) {
#pragma unroll
      for (int n = 0; n < 4; ++n) sh.p[n][tj + 3][ti + 3] = P[3][n];
    }
    if (hval) {
      R ph4[4];
      primitives<R>(Q, plane, ph + (uint32_t)k * sk, gg, ph4);
#pragma unroll
      for (int n = 0; n < 4; ++n) sh.p[n][hj - j0 + 3][hi - i0 + 3] = ph4[n];
    }
    __syncthreads();
    if (act) {
      R gr[4][3];  // d(u, v, w, T)/d(xi, eta, zeta)
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        gr[n][0] = grad6<R>([&](int m) { return sh.p[n][tj + 3][ti + 3 + m]; });
        gr[n][1] = grad6<R>([&](int m) { return sh.p[n][tj + 3 + m][ti + 3]; });
        gr[n][2] = grad6<R>([&](int m) { return P[3 + m][n]; });
      }
      const uint32_t p = pc + (uint32_t)k * sk;
      if constexpr (OS) {
        // nodes next to a one-sided face of direction d: the seven-point one-sided
        // derivative over the nodes nearest the face replaces the central one (whose
        // ghost values it ignores); primitives of the window nodes from Q
        const int idx[3] = {i, j, k};
        const int nds[3] = {g.ni, g.nj, g.nk};
        const uint32_t st[3] = {1u, (uint32_t)g.ld_i, sk};
#pragma unroll 1
        for (int d = 0; d < 3; ++d) {
          int first, row, sign;
          if (!one_sided_window((a.one_sided >> (2 * d)) & 3, idx[d], nds[d], &first, &row, &sign)) continue;
          R acc[4] = {R(0), R(0), R(0), R(0)};
#pragma unroll 1
          for (int m = 0; m < 7; ++m) {
            R pr[4];
            primitives<R>(Q, plane, p + (uint32_t)(first + m - idx[d]) * st[d], gg, pr);
            const R wgt = R(os6_weight(row, sign, m));
#pragma unroll
            for (int n = 0; n < 4; ++n) acc[n] += wgt * pr[n];
          }
#pragma unroll
          for (int n = 0; n < 4; ++n) gr[n][d] = acc[n];
        }
      }
      // the metrics and the flux planes stream through (read or written once): streaming
      // accesses leave L2 to the Q rows and columns that the neighbouring tiles read as
      // their halo (measured on the 512 x 512 x 384 channel: 4% faster in FP64)
      R mh[3][3];
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int c = 0; c < 3; ++c) mh[d][c] = ldg_nt(plane_ptr(met, (3 * d + c) * plane), p);
      const R J = ldg_nt(plane_ptr(met, 9 * plane), p);
      R dx[4][3];  // d(u, v, w, T)/d(x, y, z), Eq 21
#pragma unroll
      for (int n = 0; n < 4; ++n)
#pragma unroll
        for (int c = 0; c < 3; ++c) dx[n][c] = J * (mh[0][c] * gr[n][0] + mh[1][c] * gr[n][1] + mh[2][c] * gr[n][2]);
      const R u = P[3][0], v = P[3][1], w = P[3][2];
      const R mu = viscosity(P[3][3], R(a.ph.suth));
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
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        R f[4];
#pragma unroll
        for (int n = 0; n < 3; ++n) f[n] = mh[d][0] * tau[n][0] + mh[d][1] * tau[n][1] + mh[d][2] * tau[n][2];
        f[3] = mh[d][0] * bet[0] + mh[d][1] * bet[1] + mh[d][2] * bet[2];
#pragma unroll
        for (int n = 0; n < 4; ++n) stg_nt(plane_ptr(out, (4 * d + n) * plane), p, f[n]);
        // a block periodic with itself along d: the node's image in the halo across the
        // d-faces (the direction-d flux is the one the d sweep differentiates)
        if (a.periodic & (1 << d)) {
          const int idx = d == 0 ? i : d == 1 ? j : k;
          const int nd = d == 0 ? g.ni : d == 1 ? g.nj : g.nk;
          const uint32_t sd = d == 0 ? 1u : d == 1 ? (uint32_t)g.ld_i : sk;
          if (idx < kHalo || idx >= nd - kHalo) {
            const uint32_t pi = idx < kHalo ? p + (uint32_t)nd * sd : p - (uint32_t)nd * sd;
#pragma unroll
            for (int n = 0; n < 4; ++n) stg_nt(plane_ptr(out, (4 * d + n) * plane), pi, f[n]);
          }
        }
      }
    }
#pragma unroll
    for (int m = 0; m < 6; ++m)
#pragma unroll
      for (int n = 0; n < 4; ++n) P[m][n] = P[m + 1][n];
    __syncthreads();  // plane k of the LDS tile is consumed
  }
}

template <typename R, bool OS>
__global__ __launch_bounds__(VNT) __attribute__((amdgpu_waves_per_eu(4))) void k_visc(ViscArgs a) {
  __shared__ ViscShared<R> sh;
  visc_tile<R, OS>(a, xcd_remap(blockIdx.x, gridDim.x), sh);
}

__global__ __launch_bounds__(256) void k_round(const double* __restrict__ src, float* __restrict__ dst, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) dst[e] = float(src[e]);
}

hipError_t launch_round(const double* src, float* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nwg = (n + 255) / 256;
  hipLaunchKernelGGL(k_round, dim3((unsigned)(nwg < 65536 ? nwg : 65536)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

// Half-point metrics of a mixed-precision block (one thread per stored node and direction).
__global__ __launch_bounds__(256) void k_half_metric(Geom g, const double* __restrict__ met, float* __restrict__ hm) {
  const int64_t pl = g.plane;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < 3 * pl; e += (int64_t)gridDim.x * 256) {
    const int d = (int)(e / pl);
    const int64_t p = e - d * pl;
    const int64_t ij = g.ld_i * g.ld_j;
    const int idx = d == 0 ? (int)(p % g.ld_i) - kHalo
                  : d == 1 ? (int)((p / g.ld_i) % g.ld_j) - kHalo
                           : (int)(p / ij) - kHalo;
    const int nd = d == 0 ? g.ni : d == 1 ? g.nj : g.nk;
    if (idx < -1 || idx > nd - 1) continue;  // the stencil idx-2 .. idx+3 stays in the halo
    const int64_t st = d == 0 ? 1 : d == 1 ? g.ld_i : ij;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double* m = met + (3 * d + c) * pl + p;
      hm[(3 * d + c) * pl + p] = float(half_metric([&](int o) { return m[o * st]; }));
    }
  }
}

hipError_t launch_half_metrics(const Geom& g, const double* met, float* hm, hipStream_t s) {
  const int64_t nwg = (3 * g.plane + 255) / 256;
  hipLaunchKernelGGL(k_half_metric, dim3((unsigned)(nwg < 65536 ? nwg : 65536)), dim3(256), 0, s, g, met, hm);
  return hipGetLastError();
}

// chunk length and tile count of one block (i-tile fastest, then j-tile, then k-chunk):
// at most kViscChunk planes per tile, that bound halved (down to 8) while the block would
// give fewer than min_tiles workgroups, and nk split into the fewest chunks of equal length
// under it; a longer chunk re-reads fewer priming planes, more tiles fill the chip
void visc_tiling(const Geom& g, int min_tiles, int* kc, int* tiles) {
  const int cols = ((g.ni + VI - 1) / VI) * ((g.nj + VJ - 1) / VJ);
  int c = kViscChunk;
  while (c > 8 && cols * ((g.nk + c - 1) / c) < min_tiles) c /= 2;
  const int nch = (g.nk + c - 1) / c;
  *kc = (g.nk + nch - 1) / nch;
  *tiles = cols * ((g.nk + *kc - 1) / *kc);
}

// one workgroup per tile of the concatenated list (ids remapped XCD-contiguously)
template <typename R, bool OS>
__global__ __launch_bounds__(VNT) __attribute__((amdgpu_waves_per_eu(4))) void k_visc_batch(const ViscArgs* __restrict__ args, TileList tl) {
  __shared__ ViscShared<R> sh;
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  int blk = 0;
  while (t >= tl.prefix[blk + 1]) ++blk;
  visc_tile<R, OS>(args[blk], t - tl.prefix[blk], sh);
}

template <typename R>
hipError_t launch_visc(ViscArgs a, hipStream_t s) {
  int tiles;
  visc_tiling(a.g, kViscMinTiles, &a.kc, &tiles);
  if (a.one_sided)
    hipLaunchKernelGGL((k_visc<R, true>), dim3(tiles), dim3(VNT), 0, s, a);
  else
    hipLaunchKernelGGL((k_visc<R, false>), dim3(tiles), dim3(VNT), 0, s, a);
  return hipGetLastError();
}
template hipError_t launch_visc<double>(ViscArgs, hipStream_t);
template hipError_t launch_visc<float>(ViscArgs, hipStream_t);

// args_dev[b].kc must be the chunk length visc_tiling gives for block b
template <typename R>
hipError_t launch_visc_batch(const ViscArgs* args_dev, const TileList& tl, bool one_sided, hipStream_t s) {
  if (one_sided)
    hipLaunchKernelGGL((k_visc_batch<R, true>), dim3(tl.prefix[tl.nblk]), dim3(VNT), 0, s, args_dev, tl);
  else
    hipLaunchKernelGGL((k_visc_batch<R, false>), dim3(tl.prefix[tl.nblk]), dim3(VNT), 0, s, args_dev, tl);
  return hipGetLastError();
}
template hipError_t launch_visc_batch<double>(const ViscArgs*, const TileList&, bool, hipStream_t);
template hipError_t launch_visc_batch<float>(const ViscArgs*, const TileList&, bool, hipStream_t);

// =====================================================================================
// Direction sweep: modified AFWENO inviscid derivative (Sec. 4.5.1, Figs 10-11, Eq 19),
// the sixth-order derivative of the viscous flux, and the output (partial sum, R, or the
// RK3 stage of Eq 20).
//
// A workgroup owns a tile of TW grid lines (cross direction c1) by TS output nodes along
// the sweep direction.  It stages Q, the direction's node metrics and the viscous
// fluxes of nodes d0-3 .. d0+TS+2 in LDS; evaluates per node the characteristic WENO pair
// and the two split fluxes (nodes d0-1 .. d0+TS, one per thread) into interface fluxes;
// replaces the staged Q by the nodal fluxes; and assembles Eq 19, the viscous derivative
// and the output per output node (one per thread).
// =====================================================================================
template <int DIR, int TW>
struct LdsIdx {
  // LDS order puts the lane-fastest tile axis innermost: along the line for DIR 0
  // (lanes walk i), across lines otherwise.
  static __device__ __forceinline__ int f(int v, int w, int s, int len) {
    return DIR == 0 ? (v * TW + w) * len + s : (v * len + s) * TW + w;
  }
};

template <int TW, int TS>
struct SweepLds {
  static constexpr int NH = TS + 1;  // half points
  static constexpr int NN = TS + 6;  // nodes with a nodal flux
  static constexpr int NW = TS + 2;  // nodes with a WENO evaluation
};

// Inviscid scheme of a sweep (Sec. 4.5.1): characteristic space at the nodes (modified
// AFWENO, Figs 10-11) or at the half points (original AFWENO, Fig 9).
constexpr int kModified = 0, kOriginal = 1;

// Metrics of a sweep in mixed precision: the node metrics are staged from their FP32
// copy (every use rounds them to FP32) and the half-point metrics from the planes that
// cfd_metrics interpolated once in FP64 and rounded (the values an FP64 interpolation in
// the sweep would give, without its FP64 arithmetic in the FP32 sweeps, whose VALU issue
// is their bound).  FP64 sweeps stage the FP64 node metrics and interpolate.
template <typename R>
constexpr bool kHalfPre = sizeof(R) == 4;
template <typename R>
using StageM = typename std::conditional<kHalfPre<R>, R, double>::type;

// LDS of one workgroup for the largest tile configuration in use.  The staged Q /
// nodal-flux tile is in the compute type: an FP64 tile gives the RK combination Q_cur from
// LDS; a mixed-precision RK sweep reads Q_cur again (from L2, moments after the staging
// read it) rather than convert an FP64 tile at every use (its FP32 tile runs that sweep 3%
// faster on the 512 x 512 x 384 channel).
template <typename R, int TW, int TS>
struct SweepShared {
  R F[5 * TW * SweepLds<TW, TS>::NH];   // interface fluxes f(n+1/2)
  R Fn[5 * TW * SweepLds<TW, TS>::NN];  // staged Q, then nodal fluxes
  StageM<R> M[3 * TW * SweepLds<TW, TS>::NN];  // node metrics of the sweep direction
  R V[4 * TW * SweepLds<TW, TS>::NN];  // viscous fluxes of the direction
  R H[kHalfPre<R> ? 3 * TW * SweepLds<TW, TS>::NH : 1];  // half-point metrics (mixed precision)
};

// One tile of a direction sweep: t is the logical tile index inside the block (sweep-
// direction tile fastest, then the cross tile c1, then the cross index c2).
// OS: some block of the launch has faces with the one-sided viscous closure (a separate
// instantiation keeps the register budget of the others)
template <int DIR, typename R, int TW, int TS, int NT, int SCHEME = kModified, bool OS = false>
__device__ __forceinline__ void sweep_tile(const SweepCommon& c, const SweepBlock& b, int t,
                                           SweepShared<R, TW, TS>& sh) {
  R* const sF = sh.F;
  R* const sFn = sh.Fn;
  StageM<R>* const sM = sh.M;
  R* const sV = sh.V;
  R* const sH = sh.H;
  constexpr int NH = SweepLds<TW, TS>::NH;
  constexpr int NN = SweepLds<TW, TS>::NN;
  constexpr int NW = SweepLds<TW, TS>::NW;
  using L = LdsIdx<DIR, TW>;

  const Geom& g = b.g;
  const int nd = DIR == 0 ? g.ni : DIR == 1 ? g.nj : g.nk;
  const int n1 = DIR == 0 ? g.nj : g.ni;
  // element offsets inside one plane fit in 32 bits (checked on the host); every array
  // is addressed as a uniform plane base plus a 32-bit per-lane offset
  const uint32_t sd = DIR == 0 ? 1u : DIR == 1 ? (uint32_t)g.ld_i : (uint32_t)(g.ld_i * g.ld_j);
  const uint32_t s1 = DIR == 0 ? (uint32_t)g.ld_i : 1u;
  const uint32_t s2 = DIR == 2 ? (uint32_t)g.ld_i : (uint32_t)(g.ld_i * g.ld_j);
  const int ts = b.tile_len;  // output nodes per tile along the sweep (<= TS)
  const int nw = ts + 2;      // WENO nodes
  const int nn = ts + 6;      // nodal-flux nodes
  const int tiled = t % b.tiles_d;
  const int rest = t / b.tiles_d;
  const int tile1 = rest % b.tiles_c1;
  const int c2 = rest / b.tiles_c1;
  const int c1_0 = tile1 * TW;
  const int d0 = tiled * ts;
  // offset of (c1 = 0, c2, n = 0)
  const uint32_t origin = (uint32_t)at(g, 0, 0, 0) + (uint32_t)c2 * s2;
  const int64_t plane = g.plane;
  const GP<const double> Q = to_global(b.q);
  const GP<const double> met = to_global(b.met);
  const Gas<R> G(c.ph);
  const R eps = R(c.ph.eps);
  const bool linear = c.ph.linear != 0;
  using MT = StageM<R>;
  // node metrics of the direction (FP64, or their FP32 copy), half-point metrics (mixed)
  const GP<const MT> mbase =
      kHalfPre<R> ? (GP<const MT>)to_global(b.met_r) : (GP<const MT>)to_global(b.met);
  const GP<const MT> mx = plane_ptr(mbase, (3 * DIR + 0) * plane);
  const GP<const MT> my = plane_ptr(mbase, (3 * DIR + 1) * plane);
  const GP<const MT> mz = plane_ptr(mbase, (3 * DIR + 2) * plane);
  const GP<const float> hbase = kHalfPre<R> ? to_global(b.met_r) + (10 + 3 * DIR) * plane : nullptr;

  // ---- the output node of this thread (at most one per thread) and its global operands,
  // requested before the last barrier so that their latency overlaps the nodal-flux phase
  static_assert(TW * TS <= NT, "one output node per thread");
  const GP<const R> vis = to_global(static_cast<const R*>(b.vis)) + (4 * DIR) * plane;
  const GP<const R> rin = to_global(static_cast<const R*>(b.rt_in));
  const int eo = threadIdx.x;
  const int so = DIR == 0 ? eo % TS : eo / TW;
  const int wo = DIR == 0 ? eo / TS : eo % TW;
  const bool out_here = eo < TW * TS && so < ts && c1_0 + wo < n1 && d0 + so < nd;
  const uint32_t po = origin + (uint32_t)(c1_0 + wo) * s1 + (uint32_t)(d0 + so) * sd;
  R vm[4][6];  // viscous fluxes of the direction at offsets -3, -2, -1, 1, 2, 3
  R rp[5];     // partial sums of the earlier directions
  double Jo = 0.0, qno[5], qco[5];
  auto fetch = [&]() {
    if (!out_here) return;
    if (c.do_vis && !c.do_inv) {  // else staged with the tile
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const GP<const R> vp = plane_ptr(vis, v * plane);
#pragma unroll
        for (int m = 0; m < 6; ++m) vm[v][m] = ldg(vp, po + (uint32_t)(m < 3 ? m - 3 : m - 2) * sd);
      }
    }
    if (c.has_prev) {
#pragma unroll
      for (int v = 0; v < 5; ++v) rp[v] = ldg(plane_ptr(rin, v * plane), po);
    }
    if (c.out_kind != kOutPartial) Jo = ldg(plane_ptr(met, 9 * plane), po);
    if (c.out_kind == kOutRK) {
      // Q at the output node (an inviscid FP64 sweep took it from its tile already)
      if (!(sizeof(R) == 8 && c.do_inv)) {
#pragma unroll
        for (int v = 0; v < 5; ++v) qco[v] = ldg(plane_ptr(Q, v * plane), po);
      }
      // stage 0 has Qn = Q
      if (b.qn == b.q) {
#pragma unroll
        for (int v = 0; v < 5; ++v) qno[v] = qco[v];
      } else {
        const GP<const double> qn = to_global(b.qn);
#pragma unroll
        for (int v = 0; v < 5; ++v) qno[v] = ldg(plane_ptr(qn, v * plane), po);
      }
    }
  };

  if (c.do_inv) {
    // ---- stage Q (compute type) and the sweep direction's node metrics (FP64) of nodes
    // d0-3 .. d0+ts+2 of the tile's lines in LDS; sFn holds Q until the nodal fluxes
    // replace it.  Items are laid out with the compile-time extents NN / NW / TS so that
    // the index split needs no runtime division; slots beyond the tile's length idle.
    // A thread's items (at most ITEMS) have all their loads issued before the first LDS
    // store, so the tile waits for one memory round trip rather than one per item.
    {
      constexpr int ITEMS = (TW * NN + NT - 1) / NT;
      double ld[ITEMS][12];  // Q, then (FP64) node metrics and viscous fluxes
      R lr[ITEMS][10];       // mixed precision: node metrics, viscous fluxes, half-point metrics
      bool ok[ITEMS], okh[ITEMS];
      int li[ITEMS], lhi[ITEMS];
#pragma unroll
      for (int it = 0; it < ITEMS; ++it) {
        const int e = threadIdx.x + it * NT;
        const int s = DIR == 0 ? e % NN : e / TW;
        const int w = DIR == 0 ? e / NN : e % TW;
        const int n = d0 - 3 + s;
        const int c1 = c1_0 + w;
        ok[it] = e < TW * NN && s < nn && c1 < n1 && n <= nd + 2;
        li[it] = L::f(0, w, s, NN);
        if (ok[it]) {
          const uint32_t p = origin + (uint32_t)c1 * s1 + (uint32_t)n * sd;
#pragma unroll
          for (int v = 0; v < 5; ++v) ld[it][v] = ldg(plane_ptr(Q, v * plane), p);
          if constexpr (kHalfPre<R>) {
            lr[it][0] = ldg(mx, p);
            lr[it][1] = ldg(my, p);
            lr[it][2] = ldg(mz, p);
            if (c.do_vis) {
#pragma unroll
              for (int v = 0; v < 4; ++v) lr[it][3 + v] = ldg(plane_ptr(vis, v * plane), p);
            }
            // the half point n+1/2 is interface slot s-2 (slots 0 .. ts, n <= nd-1)
            okh[it] = s >= 2 && s <= ts + 2 && n <= nd - 1;
            lhi[it] = L::f(0, w, s - 2, NH);
            if (okh[it]) {
#pragma unroll
              for (int v = 0; v < 3; ++v) lr[it][7 + v] = ldg(plane_ptr(hbase, v * plane), p);
            }
          } else {
            ld[it][5] = ldg(mx, p);
            ld[it][6] = ldg(my, p);
            ld[it][7] = ldg(mz, p);
            if (c.do_vis) {
#pragma unroll
              for (int v = 0; v < 4; ++v) ld[it][8 + v] = double(ldg(plane_ptr(vis, v * plane), p));
            }
          }
        }
      }
      // plane v of an LDS array starts TW*NN (TW*NH) entries after plane v-1 (both layouts)
#pragma unroll
      for (int it = 0; it < ITEMS; ++it) {
        if (!ok[it]) continue;
#pragma unroll
        for (int v = 0; v < 5; ++v) sFn[li[it] + v * TW * NN] = R(ld[it][v]);
        if constexpr (kHalfPre<R>) {
#pragma unroll
          for (int v = 0; v < 3; ++v) sM[li[it] + v * TW * NN] = lr[it][v];
          if (c.do_vis) {
#pragma unroll
            for (int v = 0; v < 4; ++v) sV[li[it] + v * TW * NN] = lr[it][3 + v];
          }
          if (okh[it]) {
#pragma unroll
            for (int v = 0; v < 3; ++v) sH[lhi[it] + v * TW * NH] = lr[it][7 + v];
          }
        } else {
#pragma unroll
          for (int v = 0; v < 3; ++v) sM[li[it] + v * TW * NN] = ld[it][5 + v];
          if (c.do_vis) {
#pragma unroll
            for (int v = 0; v < 4; ++v) sV[li[it] + v * TW * NN] = R(ld[it][8 + v]);
          }
        }
      }
    }
    __syncthreads();
    R Fkeep[5];
    bool need_m = false;
    int ww = 0, sw_ = 0;
    if constexpr (SCHEME == kModified) {
      // ---- characteristic WENO pair and split fluxes (one node per thread); node n = d0-1+s
      // sits at staged index s+2.  F+ at n+1/2 goes to LDS now; F- at n-1/2 is added to the
      // same interface after the barrier, so sF holds f(n+1/2) = F+(n) + F-(n+1). ----------
      static_assert(TW * NW <= NT, "one WENO node per thread");
      const int ew = threadIdx.x;
      sw_ = DIR == 0 ? ew % NW : ew / TW;
      ww = DIR == 0 ? ew / NW : ew % TW;
      const bool wvalid = ew < TW * NW && sw_ < nw && c1_0 + ww < n1 && d0 - 1 + sw_ <= nd;
      const bool need_p = wvalid && sw_ <= ts && d0 - 1 + sw_ <= nd - 1;  // F+ at n+1/2
      need_m = wvalid && sw_ >= 1;                                        // F- at n-1/2
      if (need_p || need_m) {
        const int s = sw_, w = ww;
        const int sc = s + 2;
        R q0[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) q0[v] = R(sFn[L::f(v, w, sc, NN)]);
        const Basis<R> B =
            make_basis(q0, R(sM[L::f(0, w, sc, NN)]), R(sM[L::f(1, w, sc, NN)]), R(sM[L::f(2, w, sc, NN)]), G);
        R V[5][5];  // V[t][field] at node n + t - 2
#pragma unroll
        for (int tt = 0; tt < 5; ++tt) {
          R qq[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) qq[v] = R(sFn[L::f(v, w, s + tt, NN)]);
          project(B, G, qq, V[tt]);
        }
        R vl[5], vr[5];
        // FP64: the correction form (2.4% and 1.5% faster zeta and eta sweeps), except in the
        // RK sweep, whose registers it would overflow (2 VGPRs spilled, 4% slower)
        constexpr bool kCorr = sizeof(R) == 8 && DIR != kSweepOrder[2];
#pragma unroll
        for (int f = 0; f < 5; ++f)
          weno_pair<R, kCorr>(V[0][f], V[1][f], V[2][f], V[3][f], V[4][f], eps, linear, vl[f], vr[f]);
        if constexpr (kHalfPre<R>) {
          // half-point metrics from LDS: slot s holds n+1/2, slot s-1 holds n-1/2
          if (need_p) {
            R ul[5], F[5];
            unproject(B, G, vl, ul);
            const R hx = sH[L::f(0, w, s, NH)], hy = sH[L::f(1, w, s, NH)], hz = sH[L::f(2, w, s, NH)];
            sw_flux<+1>(ul, hx, hy, hz, G, F);
#pragma unroll
            for (int v = 0; v < 5; ++v) sF[L::f(v, w, s, NH)] = F[v];
          }
          if (need_m) {
            R ur[5];
            unproject(B, G, vr, ur);
            const R hx = sH[L::f(0, w, s - 1, NH)], hy = sH[L::f(1, w, s - 1, NH)], hz = sH[L::f(2, w, s - 1, NH)];
            sw_flux<-1>(ur, hx, hy, hz, G, Fkeep);
          }
        } else {
          // half-point metrics interpolated from the staged node metrics
          if (need_p) {
            R ul[5], F[5];
            unproject(B, G, vl, ul);
            const R hx = R(half_metric([&](int m) { return sM[L::f(0, w, sc + m, NN)]; }));
            const R hy = R(half_metric([&](int m) { return sM[L::f(1, w, sc + m, NN)]; }));
            const R hz = R(half_metric([&](int m) { return sM[L::f(2, w, sc + m, NN)]; }));
            sw_flux<+1>(ul, hx, hy, hz, G, F);
#pragma unroll
            for (int v = 0; v < 5; ++v) sF[L::f(v, w, s, NH)] = F[v];
          }
          if (need_m) {
            R ur[5];
            unproject(B, G, vr, ur);
            // half point n-1/2 = (n-1)+1/2, centred on staged index sc-1
            const R hx = R(half_metric([&](int m) { return sM[L::f(0, w, sc - 1 + m, NN)]; }));
            const R hy = R(half_metric([&](int m) { return sM[L::f(1, w, sc - 1 + m, NN)]; }));
            const R hz = R(half_metric([&](int m) { return sM[L::f(2, w, sc - 1 + m, NN)]; }));
            sw_flux<-1>(ur, hx, hy, hz, G, Fkeep);
          }
        }
      }
    } else {
      // ---- original AFWENO: one half point per thread.  Slot s holds n+1/2 with
      // n = d0-1+s (staged index s+2), whose stencil is staged s .. s+5.  The
      // characteristic space sits at the half point: the mean state of n and n+1 and the
      // direction of the half-point metric; the value left of n+1/2 comes from nodes
      // n-2..n+2, the value right of it from n-1..n+3, and f(n+1/2) = F+ + F- directly.
      static_assert(TW * NH <= NT, "one half point per thread");
      const int eh = threadIdx.x;
      const int s = DIR == 0 ? eh % NH : eh / TW;
      const int w = DIR == 0 ? eh / NH : eh % TW;
      if (eh < TW * NH && s <= ts && c1_0 + w < n1 && d0 - 1 + s <= nd - 1) {
        const int sc = s + 2;
        // half-point metric: read from LDS in mixed precision; in FP64 formed again where it
        // is used rather than held in registers
        auto hm = [&](int c) {
          if constexpr (kHalfPre<R>) {
            return sH[L::f(c, w, s, NH)];
          } else {
            return R(half_metric([&](int m) { return sM[L::f(c, w, sc + m, NN)]; }));
          }
        };
        R qa[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) qa[v] = R(0.5) * (R(sFn[L::f(v, w, sc, NN)]) + R(sFn[L::f(v, w, sc + 1, NN)]));
        const Basis<R> B = make_basis(qa, hm(0), hm(1), hm(2), G);
        // V[t][field] at node n + t - 2; node n+3 replaces node n-2 once the left value is
        // formed, which keeps five stencil points live instead of six
        R V[5][5];
        auto proj = [&](int tt, R out[5]) {
          R qq[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) qq[v] = R(sFn[L::f(v, w, s + tt, NN)]);
          project(B, G, qq, out);
        };
#pragma unroll
        for (int tt = 0; tt < 5; ++tt) proj(tt, V[tt]);
        R vl[5], vr[5], uh[5], F[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) vl[f] = weno_left(V[0][f], V[1][f], V[2][f], V[3][f], V[4][f], eps, linear);
        proj(5, V[0]);
#pragma unroll
        for (int f = 0; f < 5; ++f) vr[f] = weno_left(V[0][f], V[4][f], V[3][f], V[2][f], V[1][f], eps, linear);
        // this thread alone writes slot s: F+ goes to LDS, F- is added to it
        unproject(B, G, vl, uh);
        sw_flux<+1>(uh, hm(0), hm(1), hm(2), G, F);
#pragma unroll
        for (int v = 0; v < 5; ++v) sF[L::f(v, w, s, NH)] = F[v];
        unproject(B, G, vr, uh);
        sw_flux<-1>(uh, hm(0), hm(1), hm(2), G, F);
#pragma unroll
        for (int v = 0; v < 5; ++v) sF[L::f(v, w, s, NH)] += F[v];
      }
    }
    // a staged Q in FP64 is exact: the output node's copy for the RK combination is read
    // here, before the barrier after which the nodal fluxes overwrite it
    if (sizeof(R) == 8 && c.out_kind == kOutRK && out_here) {
#pragma unroll
      for (int v = 0; v < 5; ++v) qco[v] = double(sFn[L::f(v, wo, so + 3, NN)]);
    }
    __syncthreads();
    if (need_m) {  // each interface receives exactly one F-
#pragma unroll
      for (int v = 0; v < 5; ++v) sF[L::f(v, ww, sw_ - 1, NH)] += Fkeep[v];
    }
    fetch();
    // ---- nodal fluxes, Eq 4, in place of the staged Q ------------------------------------
    for (int e = threadIdx.x; e < TW * NN; e += NT) {
      const int s = DIR == 0 ? e % NN : e / TW;
      const int w = DIR == 0 ? e / NN : e % TW;
      const int n = d0 - 3 + s;
      const int c1 = c1_0 + w;
      if (s >= nn || c1 >= n1 || n > nd + 2) continue;
      R q[5], F[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) q[v] = R(sFn[L::f(v, w, s, NN)]);
      phys_flux(q, R(sM[L::f(0, w, s, NN)]), R(sM[L::f(1, w, s, NN)]), R(sM[L::f(2, w, s, NN)]), G, F);
#pragma unroll
      for (int v = 0; v < 5; ++v) sFn[L::f(v, w, s, NN)] = F[v];
    }
    __syncthreads();
  }

  // ---- assembly at the output node ------------------------------------------------------
  if (!c.do_inv) fetch();
  if (!out_here) return;
  const int s = so, w = wo;
  R r[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) r[v] = R(0);
  if (c.do_inv) {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const R fp = sF[L::f(v, w, s + 1, NH)];
      const R fm = sF[L::f(v, w, s, NH)];
      auto fn = [&](int m) { return R(sFn[L::f(v, w, s + m, NN)]); };
      const R D = fp - fm + R(17.0 / 256.0) * (fn(4) - fn(2)) - R(13.0 / 320.0) * (fn(5) - fn(1)) +
                  R(19.0 / 3840.0) * (fn(6) - fn(0));
      r[v] = -D;
    }
  }
  if (c.do_vis) {
    int first = 0, row = 0, sign = 0;
    if (OS && one_sided_window((b.one_sided >> (2 * DIR)) & 3, d0 + s, nd, &first, &row, &sign)) {
      // a node next to a one-sided face: seven-point one-sided derivative over the nodes
      // nearest the face, read from memory (the tile need not hold them)
#pragma unroll 1
      for (int v = 1; v < 5; ++v) {
        const GP<const R> vp = plane_ptr(vis, (v - 1) * plane);
        R acc = R(0);
#pragma unroll 1
        for (int m = 0; m < 7; ++m) acc += R(os6_weight(row, sign, m)) * ldg(vp, po + (uint32_t)(first + m - d0 - s) * sd);
        r[v] += acc;
      }
    } else if (c.do_inv) {
#pragma unroll
      for (int v = 1; v < 5; ++v) r[v] += d6<R>([&](int m) { return sV[L::f(v - 1, w, s + 3 + m, NN)]; });
    } else {
#pragma unroll
      for (int v = 1; v < 5; ++v) r[v] += d6<R>([&](int m) { return vm[v - 1][m < 0 ? m + 3 : m + 2]; });
    }
  }
  if (c.has_prev) {
#pragma unroll
    for (int v = 0; v < 5; ++v) r[v] += rp[v];
  }
  if (c.out_kind == kOutPartial) {
    const GP<R> ro = to_global(static_cast<R*>(b.rt_out));
#pragma unroll
    for (int v = 0; v < 5; ++v) stg(plane_ptr(ro, v * plane), po, r[v]);
  } else {
    const GP<double> out = to_global(b.out);
    if (c.out_kind == kOutRhs) {
#pragma unroll
      for (int v = 0; v < 5; ++v) stg(plane_ptr(out, v * plane), po, Jo * double(r[v]));
    } else {
      // local time stepping reads the point's own step here rather than with the other
      // operands: the common scalar-step path keeps its register budget
      const double dt = b.dt_field ? ldg(to_global(b.dt_field), po) : c.dt_dev ? *c.dt_dev : c.dt;
      const double cdt = c.cc * dt * Jo;
#pragma unroll
      for (int v = 0; v < 5; ++v) stg(plane_ptr(out, v * plane), po, c.ca * qno[v] + c.cb * qco[v] + cdt * double(r[v]));
    }
  }
}

// Single block: one workgroup per tile, ids remapped XCD-contiguously.
template <int DIR, typename R, int TW, int TS, int NT, int SCHEME, bool OS>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_sweep(SweepArgs a) {
  __shared__ SweepShared<R, TW, TS> sh;
  sweep_tile<DIR, R, TW, TS, NT, SCHEME, OS>(a.c, a.b, xcd_remap(blockIdx.x, gridDim.x), sh);
}
// the original scheme in FP64 holds six stencil points and the half-point basis at once:
// three waves per SIMD give it the registers that four would make it spill
template <int DIR, typename R, int TW, int TS, int NT, bool OS>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void k_sweep_w3(SweepArgs a) {
  __shared__ SweepShared<R, TW, TS> sh;
  sweep_tile<DIR, R, TW, TS, NT, kOriginal, OS>(a.c, a.b, xcd_remap(blockIdx.x, gridDim.x), sh);
}

// Batched blocks: one launch walks a work list covering the tiles of every block
// (prefix[b] = first tile of block b).  The list is split into eight contiguous ranges, one
// per XCD.  PERSIST: a fixed grid of workgroups strides through its XCD's range; otherwise
// one workgroup per tile (ids remapped XCD-contiguously).  Blocks with one-sided faces (OS)
// run one workgroup per tile.
template <int DIR, typename R, int TW, int TS, int NT, bool PERSIST, bool OS>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(PERSIST && sizeof(R) == 8 ? 3 : 4))) void k_sweep_batch(
    const SweepBlock* __restrict__ blocks, SweepCommon c, TileList tl) {
  __shared__ SweepShared<R, TW, TS> sh;
  const int total = tl.prefix[tl.nblk];
  if (!PERSIST) {
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    int blk = 0;
    while (t >= tl.prefix[blk + 1]) ++blk;
    sweep_tile<DIR, R, TW, TS, NT, kModified, OS>(c, blocks[blk], t - tl.prefix[blk], sh);
    return;
  }
  static_assert(!(PERSIST && OS), "the persistent schedule is not built for one-sided closures");
  int start, count, lane_wg, nwg_x;
  xcd_range(total, &start, &count, &lane_wg, &nwg_x);
  int blk = 0;
  for (int u = lane_wg; u < count; u += nwg_x) {
    const int t = start + u;
    while (t >= tl.prefix[blk + 1]) ++blk;  // t only grows, so the scan resumes
    sweep_tile<DIR, R, TW, TS, NT>(c, blocks[blk], t - tl.prefix[blk], sh);
    __syncthreads();  // the next tile overwrites the LDS this one read
  }
}

// Batched original-scheme sweep (one workgroup per tile).  FP64 gets three waves per SIMD
// (see k_sweep_w3), FP32 the usual four.
template <int DIR, typename R, int TW, int TS, int NT, bool OS>
__device__ __forceinline__ void batch_orig_tile(const SweepBlock* __restrict__ blocks, const SweepCommon& c,
                                                const TileList& tl, SweepShared<R, TW, TS>& sh) {
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  int blk = 0;
  while (t >= tl.prefix[blk + 1]) ++blk;
  sweep_tile<DIR, R, TW, TS, NT, kOriginal, OS>(c, blocks[blk], t - tl.prefix[blk], sh);
}
template <int DIR, typename R, int TW, int TS, int NT, bool OS>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 8 ? 3 : 4))) void k_sweep_batch_orig(
    const SweepBlock* __restrict__ blocks, SweepCommon c, TileList tl) {
  __shared__ SweepShared<R, TW, TS> sh;
  batch_orig_tile<DIR, R, TW, TS, NT, OS>(blocks, c, tl, sh);
}

// tile configurations (lines across x nodes along the sweep x threads)
template <int CFG>
struct TileCfg;
template <>
struct TileCfg<0> {
  static constexpr int TW = 16, TS = 30, NT = 512;
};
template <>
struct TileCfg<1> {
  static constexpr int TW = 32, TS = 14, NT = 512;
};
template <>
struct TileCfg<2> {
  static constexpr int TW = 16, TS = 14, NT = 256;
};
template <>
struct TileCfg<3> {
  static constexpr int TW = 8, TS = 62, NT = 512;
};
template <>
struct TileCfg<4> {
  static constexpr int TW = 8, TS = 26, NT = 256;
};
template <>
struct TileCfg<5> {
  static constexpr int TW = 4, TS = 58, NT = 256;
};
// shapes whose WENO nodes (lines x (nodes + 2)) fill the 256 threads exactly
template <>
struct TileCfg<6> {
  static constexpr int TW = 8, TS = 30, NT = 256;
};
template <>
struct TileCfg<7> {
  static constexpr int TW = 4, TS = 62, NT = 256;
};

void sweep_tiling(int dir, int cfg, const Geom& g, int* tiles_c1, int* tiles_d, int* tile_len) {
  static const int tw[kTileCfgs] = {TileCfg<0>::TW, TileCfg<1>::TW, TileCfg<2>::TW,
                                    TileCfg<3>::TW, TileCfg<4>::TW, TileCfg<5>::TW,
                                    TileCfg<6>::TW, TileCfg<7>::TW};
  static const int tsz[kTileCfgs] = {TileCfg<0>::TS, TileCfg<1>::TS, TileCfg<2>::TS,
                                     TileCfg<3>::TS, TileCfg<4>::TS, TileCfg<5>::TS,
                                     TileCfg<6>::TS, TileCfg<7>::TS};
  const int nd = dir == 0 ? g.ni : dir == 1 ? g.nj : g.nk;
  const int n1 = dir == 0 ? g.nj : g.ni;
  *tiles_c1 = (n1 + tw[cfg] - 1) / tw[cfg];
  *tiles_d = (nd + tsz[cfg] - 1) / tsz[cfg];
  *tile_len = (nd + *tiles_d - 1) / *tiles_d;  // balanced tiles along the sweep
}

void tile_shape(int cfg, int* tw, int* ts, int* nt) {
  static const int w[kTileCfgs] = {TileCfg<0>::TW, TileCfg<1>::TW, TileCfg<2>::TW,
                                   TileCfg<3>::TW, TileCfg<4>::TW, TileCfg<5>::TW,
                                   TileCfg<6>::TW, TileCfg<7>::TW};
  static const int l[kTileCfgs] = {TileCfg<0>::TS, TileCfg<1>::TS, TileCfg<2>::TS,
                                   TileCfg<3>::TS, TileCfg<4>::TS, TileCfg<5>::TS,
                                   TileCfg<6>::TS, TileCfg<7>::TS};
  *tw = w[cfg];
  *ts = l[cfg];
  *nt = sweep_threads(cfg);
}

int sweep_threads(int cfg) {
  static const int nt[kTileCfgs] = {TileCfg<0>::NT, TileCfg<1>::NT, TileCfg<2>::NT,
                                    TileCfg<3>::NT, TileCfg<4>::NT, TileCfg<5>::NT,
                                    TileCfg<6>::NT, TileCfg<7>::NT};
  return nt[cfg];
}

template <typename R, int CFG, int SCHEME, bool OS>
hipError_t launch_sweep_scheme(int dir, const SweepArgs& a, int64_t nwg, hipStream_t s) {
  using C = TileCfg<CFG>;
  dim3 grid((unsigned)nwg);
  if constexpr (SCHEME == kOriginal && sizeof(R) == 8) {
    if (dir == 0)
      hipLaunchKernelGGL((k_sweep_w3<0, R, C::TW, C::TS, C::NT, OS>), grid, dim3(C::NT), 0, s, a);
    else if (dir == 1)
      hipLaunchKernelGGL((k_sweep_w3<1, R, C::TW, C::TS, C::NT, OS>), grid, dim3(C::NT), 0, s, a);
    else
      hipLaunchKernelGGL((k_sweep_w3<2, R, C::TW, C::TS, C::NT, OS>), grid, dim3(C::NT), 0, s, a);
    return hipGetLastError();
  } else {
    if (dir == 0)
      hipLaunchKernelGGL((k_sweep<0, R, C::TW, C::TS, C::NT, SCHEME, OS>), grid, dim3(C::NT), 0, s, a);
    else if (dir == 1)
      hipLaunchKernelGGL((k_sweep<1, R, C::TW, C::TS, C::NT, SCHEME, OS>), grid, dim3(C::NT), 0, s, a);
    else
      hipLaunchKernelGGL((k_sweep<2, R, C::TW, C::TS, C::NT, SCHEME, OS>), grid, dim3(C::NT), 0, s, a);
    return hipGetLastError();
  }
}

template <typename R, int CFG>
hipError_t launch_sweep_cfg(int dir, const SweepArgs& a, int64_t nwg, hipStream_t s) {
  const bool os = a.b.one_sided != 0;
  if (a.c.ph.scheme == kOriginal)
    return os ? launch_sweep_scheme<R, CFG, kOriginal, true>(dir, a, nwg, s)
              : launch_sweep_scheme<R, CFG, kOriginal, false>(dir, a, nwg, s);
  return os ? launch_sweep_scheme<R, CFG, kModified, true>(dir, a, nwg, s)
            : launch_sweep_scheme<R, CFG, kModified, false>(dir, a, nwg, s);
}

template <typename R>
hipError_t launch_sweep(int dir, SweepArgs a, hipStream_t s, int cfg) {
  const int n2 = dir == 2 ? a.b.g.nj : a.b.g.nk;
  sweep_tiling(dir, cfg, a.b.g, &a.b.tiles_c1, &a.b.tiles_d, &a.b.tile_len);
  const int64_t nwg = (int64_t)a.b.tiles_c1 * a.b.tiles_d * n2;
  if (nwg > 0x7fffffff) return hipErrorInvalidValue;
  switch (cfg) {
    case 0: return launch_sweep_cfg<R, 0>(dir, a, nwg, s);
    case 1: return launch_sweep_cfg<R, 1>(dir, a, nwg, s);
    case 2: return launch_sweep_cfg<R, 2>(dir, a, nwg, s);
    case 3: return launch_sweep_cfg<R, 3>(dir, a, nwg, s);
    case 4: return launch_sweep_cfg<R, 4>(dir, a, nwg, s);
    case 5: return launch_sweep_cfg<R, 5>(dir, a, nwg, s);
    case 6: return launch_sweep_cfg<R, 6>(dir, a, nwg, s);
    case 7: return launch_sweep_cfg<R, 7>(dir, a, nwg, s);
  }
  return hipErrorInvalidValue;
}
template hipError_t launch_sweep<double>(int, SweepArgs, hipStream_t, int);
template hipError_t launch_sweep<float>(int, SweepArgs, hipStream_t, int);

template <typename R, int CFG, bool P, bool OS>
hipError_t launch_sweep_batch_os(int dir, const SweepBlock* blocks, const SweepCommon& c, const TileList& tl, int nwg,
                                 hipStream_t s) {
  using C = TileCfg<CFG>;
  if (c.ph.scheme == kOriginal) {
    // the original scheme runs one workgroup per tile (the persistent schedule is not built
    // for it); in FP64 at three waves per SIMD like its single-block kernels
    if (P) return hipErrorInvalidValue;
    if (dir == 0)
      hipLaunchKernelGGL((k_sweep_batch_orig<0, R, C::TW, C::TS, C::NT, OS>), dim3(nwg), dim3(C::NT), 0, s, blocks, c, tl);
    else if (dir == 1)
      hipLaunchKernelGGL((k_sweep_batch_orig<1, R, C::TW, C::TS, C::NT, OS>), dim3(nwg), dim3(C::NT), 0, s, blocks, c, tl);
    else
      hipLaunchKernelGGL((k_sweep_batch_orig<2, R, C::TW, C::TS, C::NT, OS>), dim3(nwg), dim3(C::NT), 0, s, blocks, c, tl);
    return hipGetLastError();
  }
  if constexpr (P && OS) {
    return hipErrorInvalidValue;
  } else {
    if (dir == 0)
      hipLaunchKernelGGL((k_sweep_batch<0, R, C::TW, C::TS, C::NT, P, OS>), dim3(nwg), dim3(C::NT), 0, s, blocks, c, tl);
    else if (dir == 1)
      hipLaunchKernelGGL((k_sweep_batch<1, R, C::TW, C::TS, C::NT, P, OS>), dim3(nwg), dim3(C::NT), 0, s, blocks, c, tl);
    else
      hipLaunchKernelGGL((k_sweep_batch<2, R, C::TW, C::TS, C::NT, P, OS>), dim3(nwg), dim3(C::NT), 0, s, blocks, c, tl);
    return hipGetLastError();
  }
}
template <typename R, int CFG, bool P>
hipError_t launch_sweep_batch_cfg(int dir, const SweepBlock* blocks, const SweepCommon& c, const TileList& tl, int nwg,
                                  hipStream_t s) {
  return c.one_sided ? launch_sweep_batch_os<R, CFG, P, true>(dir, blocks, c, tl, nwg, s)
                     : launch_sweep_batch_os<R, CFG, P, false>(dir, blocks, c, tl, nwg, s);
}

// persist: nwg workgroups stride through the list; otherwise nwg must equal the tile count
template <typename R>
hipError_t launch_sweep_batch(int dir, int cfg, bool persist, const SweepBlock* blocks, const SweepCommon& c,
                              const TileList& tl, int nwg, hipStream_t s) {
  if (persist) {
    switch (cfg) {
      case 0: return launch_sweep_batch_cfg<R, 0, true>(dir, blocks, c, tl, nwg, s);
      case 1: return launch_sweep_batch_cfg<R, 1, true>(dir, blocks, c, tl, nwg, s);
      case 2: return launch_sweep_batch_cfg<R, 2, true>(dir, blocks, c, tl, nwg, s);
      case 3: return launch_sweep_batch_cfg<R, 3, true>(dir, blocks, c, tl, nwg, s);
      case 4: return launch_sweep_batch_cfg<R, 4, true>(dir, blocks, c, tl, nwg, s);
      case 5: return launch_sweep_batch_cfg<R, 5, true>(dir, blocks, c, tl, nwg, s);
      case 6: return launch_sweep_batch_cfg<R, 6, true>(dir, blocks, c, tl, nwg, s);
      case 7: return launch_sweep_batch_cfg<R, 7, true>(dir, blocks, c, tl, nwg, s);
    }
  } else {
    switch (cfg) {
      case 0: return launch_sweep_batch_cfg<R, 0, false>(dir, blocks, c, tl, nwg, s);
      case 1: return launch_sweep_batch_cfg<R, 1, false>(dir, blocks, c, tl, nwg, s);
      case 2: return launch_sweep_batch_cfg<R, 2, false>(dir, blocks, c, tl, nwg, s);
      case 3: return launch_sweep_batch_cfg<R, 3, false>(dir, blocks, c, tl, nwg, s);
      case 4: return launch_sweep_batch_cfg<R, 4, false>(dir, blocks, c, tl, nwg, s);
      case 5: return launch_sweep_batch_cfg<R, 5, false>(dir, blocks, c, tl, nwg, s);
      case 6: return launch_sweep_batch_cfg<R, 6, false>(dir, blocks, c, tl, nwg, s);
      case 7: return launch_sweep_batch_cfg<R, 7, false>(dir, blocks, c, tl, nwg, s);
    }
  }
  return hipErrorInvalidValue;
}
template hipError_t launch_sweep_batch<double>(int, int, bool, const SweepBlock*, const SweepCommon&, const TileList&, int,
                                               hipStream_t);
template hipError_t launch_sweep_batch<float>(int, int, bool, const SweepBlock*, const SweepCommon&, const TileList&, int,
                                              hipStream_t);

// =====================================================================================
// Halo copies across 1-to-1 faces (ghost layer m of the destination face <- interior
// layer m-1 inside the source face), boundary fills.
// =====================================================================================
template <typename T>
__global__ __launch_bounds__(256) void k_copy(const CopySeg* segs, PtrTable t) {
  const CopySeg S = segs[blockIdx.y];
  const int per_plane = S.na * S.nb * kHalo;
  const int total = per_plane * S.nplanes;
  T* dst = static_cast<T*>(t.p[S.dst]);
  const T* src = static_cast<const T*>(t.p[S.src]);
  const int64_t pd = t.plane[S.dst], ps = t.plane[S.src];
  for (int e = blockIdx.x * 256 + threadIdx.x; e < total; e += gridDim.x * 256) {
    const int vv = e / per_plane;
    int r = e % per_plane;
    int a, l;
    if (S.layer_fast) {
      l = r % kHalo;
      r /= kHalo;
      a = r % S.na;
      r /= S.na;
    } else {
      a = r % S.na;
      r /= S.na;
      l = r % kHalo;
      r /= kHalo;
    }
    const int b = r;
    const T x = src[(S.src_plane0 + vv) * ps + S.src_off + a * S.src_sa + b * S.src_sb + l * S.src_sl];
    dst[(S.plane0 + vv) * pd + S.dst_off + a * S.dst_sa + b * S.dst_sb + l * S.dst_sl] = S.negate ? -x : x;
  }
}

template <typename T>
hipError_t launch_copy(const CopySeg* segs_dev, int nseg, int max_elems, const PtrTable& t, hipStream_t s) {
  if (nseg == 0) return hipSuccess;
  int bx = (max_elems + 255) / 256;
  if (bx > 256) bx = 256;  // grid-stride: more workgroups mostly idle on short segments
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

// Characteristic far-field state for the boundary node's conserved state qb, the outward
// unit normal n and the far-field state qf: Riemann invariants u_n +- 2c/(gamma-1) along n,
// the outgoing one from qb and the incoming one from qf; entropy p/rho^gamma and the
// tangential velocity from qb on outflow, from qf on inflow; at supersonic normal speed
// the whole state of the upwind side.
__device__ void char_farfield(const double qb[5], const double n[3], const double qf[5], double gamma, double qg[5]) {
  const double gm1 = gamma - 1.0;
  const double rb = qb[0], ub = qb[1] / rb, vb = qb[2] / rb, wb = qb[3] / rb;
  const double pb = gm1 * (qb[4] - 0.5 * rb * (ub * ub + vb * vb + wb * wb));
  const double cb = sqrt(gamma * pb / rb);
  const double unb = ub * n[0] + vb * n[1] + wb * n[2];
  if (unb >= cb || unb <= -cb) {
    const double* src = unb >= cb ? qb : qf;
    for (int v = 0; v < 5; ++v) qg[v] = src[v];
    return;
  }
  const double rf = qf[0], uf = qf[1] / rf, vf = qf[2] / rf, wf = qf[3] / rf;
  const double pf = gm1 * (qf[4] - 0.5 * rf * (uf * uf + vf * vf + wf * wf));
  const double cf = sqrt(gamma * pf / rf);
  const double unf = uf * n[0] + vf * n[1] + wf * n[2];
  const double rplus = unb + 2.0 * cb / gm1, rminus = unf - 2.0 * cf / gm1;
  const double un = 0.5 * (rplus + rminus), c = 0.25 * gm1 * (rplus - rminus);
  const bool out = un > 0.0;
  const double s = out ? pb / pow(rb, gamma) : pf / pow(rf, gamma);
  const double un_s = out ? unb : unf;
  const double tx = (out ? ub : uf) - un_s * n[0], ty = (out ? vb : vf) - un_s * n[1], tz = (out ? wb : wf) - un_s * n[2];
  const double rho = pow(c * c / (gamma * s), 1.0 / gm1);
  const double p = rho * c * c / gamma;
  const double u = tx + un * n[0], v = ty + un * n[1], w = tz + un * n[2];
  qg[0] = rho;
  qg[1] = rho * u;
  qg[2] = rho * v;
  qg[3] = rho * w;
  qg[4] = p / gm1 + 0.5 * rho * (u * u + v * v + w * w);
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
    } else if (S.kind == CFD_BC_FARFIELD_CHAR) {
      // outward unit normal: the face-normal direction's hatted metric at the boundary node
      const double* M = static_cast<const double*>(A.mt.p[S.blk]);
      double nv[3] = {M[(3 * S.axis) * pl + pw], M[(3 * S.axis + 1) * pl + pw], M[(3 * S.axis + 2) * pl + pw]};
      const double scale = (S.sout > 0 ? 1.0 : -1.0) / sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
      for (int d = 0; d < 3; ++d) nv[d] *= scale;
      double qb[5], qg[5];
      for (int v = 0; v < 5; ++v) qb[v] = Q[v * pl + pw];
      char_farfield(qb, nv, A.qinf, A.gamma, qg);
      for (int v = 0; v < 5; ++v) Q[v * pl + pg] = qg[v];
    } else {
      const double rho = Q[pm], rinv = 1.0 / rho;
      const double u = Q[pl + pm] * rinv, v = Q[2 * pl + pm] * rinv, w = Q[3 * pl + pm] * rinv;
      const double ke = 0.5 * (u * u + v * v + w * w);
      const double p = gm1 * (Q[4 * pl + pm] - rho * ke);
      const double T = A.gamma * p * rinv;
      // reflection of T - T_w, floored at T_w / 2 (positive ghost density)
      const double Tg = fmax(2.0 * A.t_wall - T, 0.5 * A.t_wall);
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
  if (bx > 256) bx = 256;  // grid-stride: more workgroups mostly idle on short segments
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
  __shared__ uint64_t red[256];
  uint64_t best = 0;  // bit pattern of the largest spectral radius (+0.0 to start)
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
    // a non-finite point (NaN or infinite spectral radius) becomes the quiet-NaN pattern,
    // which orders above +inf as an unsigned integer, so the maximum keeps it
    const uint64_t bits = sum <= 1.7976931348623157e308 ? (uint64_t)__double_as_longlong(sum) : 0x7ff8000000000000ull;
    best = best > bits ? best : bits;
  }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = red[threadIdx.x] > red[threadIdx.x + h] ? red[threadIdx.x] : red[threadIdx.x + h];
    __syncthreads();
  }
  // non-negative doubles order like their bit patterns
  if (threadIdx.x == 0) atomicMax(acc, (unsigned long long)red[0]);
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

// ---- local time steps: the CFL step of every interior point ---------------------------
__global__ __launch_bounds__(256) void k_dt_local(Geom g, const double* q, const double* met, double gamma, double cfl,
                                                  double* dt_field) {
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
    dt_field[p] = cfl / sum;
  }
}

hipError_t launch_dt_local(const Geom& g, const double* q, const double* met, double gamma, double cfl,
                           double* dt_field, hipStream_t s) {
  const int64_t total = (int64_t)g.ni * g.nj * g.nk;
  int bx = (int)((total + 255) / 256);
  if (bx > 8192) bx = 8192;
  if (bx < 1) bx = 1;
  hipLaunchKernelGGL(k_dt_local, dim3(bx), dim3(256), 0, s, g, q, met, gamma, cfl, dt_field);
  return hipGetLastError();
}

// ---- CFL time step into device memory (no host round trip) -------------------------
__global__ void k_dt_reset(unsigned long long* acc) { *acc = 0ull; }

__global__ void k_dt_finish(const unsigned long long* acc, double cfl, double* dt) {
  const double smax = __longlong_as_double((long long)*acc);
  *dt = (smax > 0.0 && smax <= 1.7976931348623157e308) ? cfl / smax : __builtin_nan("");
}

hipError_t launch_dt_reset(unsigned long long* acc, hipStream_t s) {
  hipLaunchKernelGGL(k_dt_reset, dim3(1), dim3(1), 0, s, acc);
  return hipGetLastError();
}
hipError_t launch_dt_finish(const unsigned long long* acc, double cfl, double* dt, hipStream_t s) {
  hipLaunchKernelGGL(k_dt_finish, dim3(1), dim3(1), 0, s, acc, cfl, dt);
  return hipGetLastError();
}

// ---- residual norms: reduced-dimensional reductions (Sec. 4.5) ------------------------
// 3D -> lines: each wave walks grid lines (j, k) of the block, its lanes striding along i
// (coalesced), and keeps per lane the sums of squares and the maxima of the five fields of
// scale * (a - b) (b may be null); lines -> workgroup: a fixed-order tree in LDS; the
// kResGroups partial rows of every block are then reduced by one workgroup, again in a
// fixed order, so the result does not depend on timing.
__global__ __launch_bounds__(256) void k_res_partial(Geom g, const double* __restrict__ a, const double* __restrict__ b,
                                                     double scale, double* __restrict__ part) {
  __shared__ double red[10][256];
  double sq[5] = {0, 0, 0, 0, 0}, mx[5] = {0, 0, 0, 0, 0};
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lines = g.nj * g.nk;
  for (int l = blockIdx.x * 4 + wave; l < lines; l += gridDim.x * 4) {
    const int j = l % g.nj, k = l / g.nj;
    for (int i = lane; i < g.ni; i += 64) {
      const int64_t p = at(g, i, j, k);
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const double d = scale * (b ? a[v * g.plane + p] - b[v * g.plane + p] : a[v * g.plane + p]);
        sq[v] += d * d;
        mx[v] = fmax(mx[v], fabs(d));
      }
    }
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    red[v][threadIdx.x] = sq[v];
    red[5 + v][threadIdx.x] = mx[v];
  }
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        red[v][threadIdx.x] += red[v][threadIdx.x + h];
        red[5 + v][threadIdx.x] = fmax(red[5 + v][threadIdx.x], red[5 + v][threadIdx.x + h]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 10) part[(int64_t)blockIdx.x * 10 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_res_final(const double* __restrict__ part, int nparts, double inv_n,
                                                   double* __restrict__ out) {
  __shared__ double red[10][256];
  double sq[5] = {0, 0, 0, 0, 0}, mx[5] = {0, 0, 0, 0, 0};
  for (int r = threadIdx.x; r < nparts; r += 256) {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      sq[v] += part[(int64_t)r * 10 + v];
      mx[v] = fmax(mx[v], part[(int64_t)r * 10 + 5 + v]);
    }
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    red[v][threadIdx.x] = sq[v];
    red[5 + v][threadIdx.x] = mx[v];
  }
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        red[v][threadIdx.x] += red[v][threadIdx.x + h];
        red[5 + v][threadIdx.x] = fmax(red[5 + v][threadIdx.x], red[5 + v][threadIdx.x + h]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 5) out[threadIdx.x] = sqrt(red[threadIdx.x][0] * inv_n);
  else if (threadIdx.x < 10) out[threadIdx.x] = red[threadIdx.x][0];
}

hipError_t launch_res_partial(const Geom& g, const double* a, const double* b, double scale, double* part,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_res_partial, dim3(kResGroups), dim3(256), 0, s, g, a, b, scale, part);
  return hipGetLastError();
}
hipError_t launch_res_final(const double* part, int nparts, double inv_n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_res_final, dim3(1), dim3(256), 0, s, part, nparts, inv_n, out);
  return hipGetLastError();
}

}  // namespace cfd
