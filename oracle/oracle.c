/*
 * oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY; see oracle.h).
 *
 * It follows Sec. 2 of Ye et al. (arXiv 2006.07964) step by step, in the paper's order,
 * with plain loops over grid lines (OpenMP only across independent lines).  Nothing here
 * is blocked, fused or reordered for speed.  Readings of points the paper leaves open are
 * marked "Reading:".
 *
 * Nondimensionalisation (Eq 1): rho_inf = 1, c_inf = 1, T = gamma p / rho (so T_inf = 1,
 * p_inf = 1/gamma and the sound speed is c = sqrt(T)); the viscous terms carry Ma/Re.
 * Index spacing is one in xi, eta and zeta.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define HS 3  /* halo of state / metric arrays */
#define HX 6  /* halo of coordinate arrays     */

/* ------------------------------------------------------------------------------------ */
/* indexing                                                                              */
/* ------------------------------------------------------------------------------------ */
typedef struct { long sx, sy, sz, plane; } dims_t;

static dims_t state_dims(const oracle_cfg* c) {
  dims_t d;
  d.sx = c->ni + 2 * HS; d.sy = c->nj + 2 * HS; d.sz = c->nk + 2 * HS;
  d.plane = d.sx * d.sy * d.sz;
  return d;
}
static dims_t coord_dims(const oracle_cfg* c) {
  dims_t d;
  d.sx = c->ni + 2 * HX; d.sy = c->nj + 2 * HX; d.sz = c->nk + 2 * HX;
  d.plane = d.sx * d.sy * d.sz;
  return d;
}
/* (i,j,k) are interior-based indices (0 = first interior point) */
static long sidx(const dims_t* d, int i, int j, int k) {
  return ((long)(k + HS) * d->sy + (j + HS)) * d->sx + (i + HS);
}
static long xidx(const dims_t* d, int i, int j, int k) {
  return ((long)(k + HX) * d->sy + (j + HX)) * d->sx + (i + HX);
}
/* step of one index in direction dir (0: i, 1: j, 2: k) */
static void unit(int dir, int* di, int* dj, int* dk) {
  *di = dir == 0; *dj = dir == 1; *dk = dir == 2;
}
static int npts(const oracle_cfg* c, int dir) {
  return dir == 0 ? c->ni : dir == 1 ? c->nj : c->nk;
}

/* ------------------------------------------------------------------------------------ */
/* Sixth-order central first derivative (Sec. 2, after Eq 8), unit spacing:            */
/*   d6 g_i = 3/4 (g_{i+1}-g_{i-1}) - 3/20 (g_{i+2}-g_{i-2}) + 1/60 (g_{i+3}-g_{i-3})    */
/* g[0..6] holds g_{i-3} .. g_{i+3}.                                                     */
/* ------------------------------------------------------------------------------------ */
static double d6(const double* g) {
  return 3.0 / 4.0 * (g[4] - g[2]) - 3.0 / 20.0 * (g[5] - g[1]) + 1.0 / 60.0 * (g[6] - g[0]);
}

/* ------------------------------------------------------------------------------------ */
/* One-sided closures of the viscous derivatives (Sec. 4.5.2 mentions one-sided         */
/* differences near block boundaries but gives no coefficients).                        */
/* Reading: with visc_closure = ORACLE_VISC_ONE_SIDED, along direction d a node within  */
/* three nodes of a wall or far-field face of d takes the derivative of the degree-6    */
/* interpolating polynomial through the seven nodes nearest that face (the boundary     */
/* node and six inside), for the velocity and temperature gradients and for the         */
/* derivative of the direction-d viscous flux; the viscous terms then read no ghost     */
/* value across such a face.  Row r of OS6 gives the weights of nodes 0..6 for the      */
/* derivative at node r (unit spacing); these are the Lagrange derivative weights,      */
/* written as exact fractions.  A node r away from the high face uses the mirror image  */
/* with the opposite sign.                                                              */
/* ------------------------------------------------------------------------------------ */
static const double OS6[3][7] = {
    {-49.0 / 20.0, 6.0, -15.0 / 2.0, 20.0 / 3.0, -15.0 / 4.0, 6.0 / 5.0, -1.0 / 6.0},
    {-1.0 / 6.0, -77.0 / 60.0, 5.0 / 2.0, -5.0 / 3.0, 5.0 / 6.0, -1.0 / 4.0, 1.0 / 30.0},
    {1.0 / 30.0, -2.0 / 5.0, -7.0 / 12.0, 4.0 / 3.0, -1.0 / 2.0, 2.0 / 15.0, -1.0 / 60.0}};

static int physical_face(int kind) {
  return kind == ORACLE_BC_WALL || kind == ORACLE_BC_FARFIELD || kind == ORACLE_BC_FARFIELD_CHAR;
}

/* Viscous first derivative along dir at interior index node of a line: returns 0 for the
 * central d6 over nodes node-3..node+3, else 1 with w[0..6] the weights of the seven nodes
 * first..first+6 of a one-sided closure.                                                */
static int one_sided(const oracle_cfg* c, int dir, int node, int* first, double* w) {
  const int n = npts(c, dir);
  int m;
  if (c->visc_closure != ORACLE_VISC_ONE_SIDED) return 0;
  if (node < 3 && physical_face(c->bc[2 * dir])) {
    *first = 0;
    for (m = 0; m < 7; ++m) w[m] = OS6[node][m];
    return 1;
  }
  if (node > n - 4 && physical_face(c->bc[2 * dir + 1])) {
    const int r = n - 1 - node;
    *first = n - 7;
    for (m = 0; m < 7; ++m) w[m] = -OS6[r][6 - m];
    return 1;
  }
  return 0;
}

/* ------------------------------------------------------------------------------------ */
/* Eq 7 / Eq 8: conservative metrics and Jacobian                                       */
/* ------------------------------------------------------------------------------------ */
/* derivative along dir of coordinate array X at (i,j,k) */
static double dcoord(const dims_t* xd, const double* X, int dir, int i, int j, int k) {
  int di, dj, dk, s;
  double g[7];
  unit(dir, &di, &dj, &dk);
  for (s = -3; s <= 3; ++s) g[s + 3] = X[xidx(xd, i + s * di, j + s * dj, k + s * dk)];
  return d6(g);
}
/* outer derivative along dout of the product (d/din of coordinate a) * (coordinate b) */
static double dprod(const dims_t* xd, const double* A, const double* B, int din, int dout,
                    int i, int j, int k) {
  int di, dj, dk, s;
  double g[7];
  unit(dout, &di, &dj, &dk);
  for (s = -3; s <= 3; ++s) {
    int ii = i + s * di, jj = j + s * dj, kk = k + s * dk;
    g[s + 3] = dcoord(xd, A, din, ii, jj, kk) * B[xidx(xd, ii, jj, kk)];
  }
  return d6(g);
}

int oracle_metrics(const oracle_cfg* c, const double* xyz, double* met) {
  const dims_t xd = coord_dims(c), sd = state_dims(c);
  const double* x = xyz;
  const double* y = xyz + xd.plane;
  const double* z = xyz + 2 * xd.plane;
  enum { XI = 0, ETA = 1, ZETA = 2 };
  int bad = 0;
  int k;
#pragma omp parallel for reduction(| : bad) schedule(static)
  for (k = -HS; k < c->nk + HS; ++k) {
    int i, j;
    for (j = -HS; j < c->nj + HS; ++j)
      for (i = -HS; i < c->ni + HS; ++i) {
        long p = sidx(&sd, i, j, k);
        /* Eq 7, term by term as printed */
        met[0 * sd.plane + p] = dprod(&xd, y, z, ETA, ZETA, i, j, k) - dprod(&xd, y, z, ZETA, ETA, i, j, k);
        met[1 * sd.plane + p] = dprod(&xd, z, x, ETA, ZETA, i, j, k) - dprod(&xd, z, x, ZETA, ETA, i, j, k);
        met[2 * sd.plane + p] = dprod(&xd, x, y, ETA, ZETA, i, j, k) - dprod(&xd, x, y, ZETA, ETA, i, j, k);
        met[3 * sd.plane + p] = dprod(&xd, y, z, ZETA, XI, i, j, k) - dprod(&xd, y, z, XI, ZETA, i, j, k);
        met[4 * sd.plane + p] = dprod(&xd, z, x, ZETA, XI, i, j, k) - dprod(&xd, z, x, XI, ZETA, i, j, k);
        met[5 * sd.plane + p] = dprod(&xd, x, y, ZETA, XI, i, j, k) - dprod(&xd, x, y, XI, ZETA, i, j, k);
        met[6 * sd.plane + p] = dprod(&xd, y, z, XI, ETA, i, j, k) - dprod(&xd, y, z, ETA, XI, i, j, k);
        met[7 * sd.plane + p] = dprod(&xd, z, x, XI, ETA, i, j, k) - dprod(&xd, z, x, ETA, XI, i, j, k);
        met[8 * sd.plane + p] = dprod(&xd, x, y, XI, ETA, i, j, k) - dprod(&xd, x, y, ETA, XI, i, j, k);
        {
          /* Eq 8 */
          double xx = dcoord(&xd, x, XI, i, j, k), xe = dcoord(&xd, x, ETA, i, j, k), xz = dcoord(&xd, x, ZETA, i, j, k);
          double yx = dcoord(&xd, y, XI, i, j, k), ye = dcoord(&xd, y, ETA, i, j, k), yz = dcoord(&xd, y, ZETA, i, j, k);
          double zx = dcoord(&xd, z, XI, i, j, k), ze = dcoord(&xd, z, ETA, i, j, k), zz = dcoord(&xd, z, ZETA, i, j, k);
          double jinv = xx * ye * zz - xx * yz * ze + xe * yz * zx - xe * yx * zz + xz * yx * ze - xz * ye * zx;
          if (!(jinv > 0.0)) bad = 1;
          met[9 * sd.plane + p] = 1.0 / jinv;
        }
      }
  }
  return bad ? -5 : 0;
}

/* ------------------------------------------------------------------------------------ */
/* Gas model (Eq 1): primitives from Q = (rho, rho u, rho v, rho w, e)                   */
/* ------------------------------------------------------------------------------------ */
typedef struct { double rho, u, v, w, p, T, c, H; } prim_t;

static prim_t primitives(const double* q, double gamma) {
  prim_t s;
  s.rho = q[0];
  s.u = q[1] / q[0];
  s.v = q[2] / q[0];
  s.w = q[3] / q[0];
  s.p = (gamma - 1.0) * (q[4] - 0.5 * s.rho * (s.u * s.u + s.v * s.v + s.w * s.w));
  s.T = gamma * s.p / s.rho;
  s.c = sqrt(s.T);                 /* c^2 = gamma p / rho = T */
  s.H = (q[4] + s.p) / s.rho;      /* total enthalpy          */
  return s;
}

/* Reading: Sutherland's law for the nondimensional viscosity with T_inf = 1,
 * mu = T^{3/2} (1 + S) / (T + S); the paper stores mu without naming its law.            */
double oracle_viscosity(double T, double suth) {
  return T * sqrt(T) * (1.0 + suth) / (T + suth);
}

/* Eq 4: inviscid flux through the hatted metric vector m = (m_x, m_y, m_z)/J.           */
void oracle_phys_flux(const double* q, const double* m, double gamma, double* F) {
  prim_t s = primitives(q, gamma);
  double U = m[0] * s.u + m[1] * s.v + m[2] * s.w;  /* contravariant velocity / J */
  F[0] = s.rho * U;
  F[1] = s.rho * s.u * U + m[0] * s.p;
  F[2] = s.rho * s.v * U + m[1] * s.p;
  F[3] = s.rho * s.w * U + m[2] * s.p;
  F[4] = (q[4] + s.p) * U;
}

/* ------------------------------------------------------------------------------------ */
/* Eigenvectors of the flux Jacobian in the unit direction k (characteristic space).    */
/* Reading: the right eigenvectors of Pulliam & Chaussee (J. Comput. Phys. 39, 1981):   */
/* columns 1-3 (eigenvalue theta) k_m (1, u, v, w, q) + rho (0, k x e_m, u.(k x e_m)),   */
/* columns 4-5 (theta +- c) rho/(sqrt2 c) (1, u +- c k, H +- c theta).  L is the plain  */
/* numerical inverse of R.                                                              */
/* ------------------------------------------------------------------------------------ */
static int invert5(const double* A, double* Ainv) {
  double M[5][10];
  int r, col, i;
  for (r = 0; r < 5; ++r)
    for (col = 0; col < 10; ++col) M[r][col] = col < 5 ? A[r * 5 + col] : (double)(col - 5 == r);
  for (col = 0; col < 5; ++col) {
    int piv = col;
    for (r = col + 1; r < 5; ++r)
      if (fabs(M[r][col]) > fabs(M[piv][col])) piv = r;
    if (M[piv][col] == 0.0) return -1;
    if (piv != col)
      for (i = 0; i < 10; ++i) { double t = M[col][i]; M[col][i] = M[piv][i]; M[piv][i] = t; }
    {
      double s = M[col][col];
      for (i = 0; i < 10; ++i) M[col][i] /= s;
    }
    for (r = 0; r < 5; ++r)
      if (r != col) {
        double f = M[r][col];
        for (i = 0; i < 10; ++i) M[r][i] -= f * M[col][i];
      }
  }
  for (r = 0; r < 5; ++r)
    for (col = 0; col < 5; ++col) Ainv[r * 5 + col] = M[r][col + 5];
  return 0;
}

int oracle_eigvec(const double* q, const double* k, double gamma, double* L, double* R) {
  prim_t s = primitives(q, gamma);
  double kx = k[0], ky = k[1], kz = k[2];
  double qq = 0.5 * (s.u * s.u + s.v * s.v + s.w * s.w);
  double theta = kx * s.u + ky * s.v + kz * s.w;
  double a = s.rho / (sqrt(2.0) * s.c);
  /* R[row*5 + col] */
  double Rm[25] = {
      /* row rho   */ kx, ky, kz, a, a,
      /* row rho u */ kx * s.u, ky * s.u - kz * s.rho, kz * s.u + ky * s.rho, a * (s.u + kx * s.c), a * (s.u - kx * s.c),
      /* row rho v */ kx * s.v + kz * s.rho, ky * s.v, kz * s.v - kx * s.rho, a * (s.v + ky * s.c), a * (s.v - ky * s.c),
      /* row rho w */ kx * s.w - ky * s.rho, ky * s.w + kx * s.rho, kz * s.w, a * (s.w + kz * s.c), a * (s.w - kz * s.c),
      /* row e     */ kx * qq + s.rho * (kz * s.v - ky * s.w), ky * qq + s.rho * (kx * s.w - kz * s.u),
      kz * qq + s.rho * (ky * s.u - kx * s.v), a * (s.H + theta * s.c), a * (s.H - theta * s.c)};
  memcpy(R, Rm, sizeof Rm);
  return invert5(R, L);
}

/* ------------------------------------------------------------------------------------ */
/* Steger-Warming flux vector splitting (Sec. 2, the monotone flux h of Eq 12).          */
/* With |m| the metric magnitude, kt = m/|m| and theta = kt.u, the eigenvalues are       */
/* lambda_{1,2,3} = |m| theta, lambda_{4,5} = |m| (theta +- c); lambda^{+-} =            */
/* (lambda +- |lambda|)/2 and                                                           */
/* F^{+-} = rho/(2 gamma) [2(gamma-1) l1 (1,u,v,w,q) + l4 (1, u+c kt, H+c theta)         */
/*                        + l5 (1, u-c kt, H-c theta)].                                  */
/* ------------------------------------------------------------------------------------ */
static void sw_part(const double* q, const double* m, double gamma, int sign, double* F) {
  prim_t s = primitives(q, gamma);
  double mag = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
  double kx = m[0] / mag, ky = m[1] / mag, kz = m[2] / mag;
  double theta = kx * s.u + ky * s.v + kz * s.w;
  double lam[3] = {mag * theta, mag * (theta + s.c), mag * (theta - s.c)};
  double l[3];
  int n;
  double qq = 0.5 * (s.u * s.u + s.v * s.v + s.w * s.w);
  double f = s.rho / (2.0 * gamma);
  for (n = 0; n < 3; ++n) l[n] = 0.5 * (lam[n] + sign * fabs(lam[n]));
  F[0] = f * (2.0 * (gamma - 1.0) * l[0] + l[1] + l[2]);
  F[1] = f * (2.0 * (gamma - 1.0) * l[0] * s.u + l[1] * (s.u + s.c * kx) + l[2] * (s.u - s.c * kx));
  F[2] = f * (2.0 * (gamma - 1.0) * l[0] * s.v + l[1] * (s.v + s.c * ky) + l[2] * (s.v - s.c * ky));
  F[3] = f * (2.0 * (gamma - 1.0) * l[0] * s.w + l[1] * (s.w + s.c * kz) + l[2] * (s.w - s.c * kz));
  F[4] = f * (2.0 * (gamma - 1.0) * l[0] * qq + l[1] * (s.H + s.c * theta) + l[2] * (s.H - s.c * theta));
}

void oracle_split_flux(const double* q, const double* m, double gamma, double* Fp, double* Fm) {
  sw_part(q, m, gamma, +1, Fp);
  sw_part(q, m, gamma, -1, Fm);
}

/* ------------------------------------------------------------------------------------ */
/* WENO interpolation (Eqs 13-17).                                                       */
/* Reading: the sub-stencil that carries the ideal weight 1/16 and beta_1 is            */
/* {i-2,i-1,i} (value 3/8, -5/4, 15/8 at i+1/2); 5/8 goes with {i-1,i,i+1} and 5/16     */
/* with {i,i+1,i+2}.  Only this pairing makes the linear combination the fifth-order    */
/* interpolant (3,-20,90,60,-5)/128; Eq 14 lists the three stencils in reverse order.   */
/* The value at i-1/2 from the same five points is the mirror image (modified AFWENO,   */
/* Sec. 4.5.1, Figs 10-11): the betas are shared and the ideal weights are reversed.    */
/* ------------------------------------------------------------------------------------ */
void oracle_weno5(const double* v, double eps, int linear, double* out, double* beta_out) {
  const double a = v[0], b = v[1], cc = v[2], d = v[3], e = v[4];
  double beta[3], sub_p[3], sub_m[3], gam_p[3] = {1.0 / 16.0, 5.0 / 8.0, 5.0 / 16.0};
  double gam_m[3] = {5.0 / 16.0, 5.0 / 8.0, 1.0 / 16.0};
  double wp[3], wm[3], sp = 0.0, sm = 0.0;
  int j;
  /* Eq 17 */
  beta[0] = (4.0 * a * a - 19.0 * a * b + 25.0 * b * b + 11.0 * a * cc - 31.0 * b * cc + 10.0 * cc * cc) / 3.0;
  beta[1] = (4.0 * b * b - 13.0 * b * cc + 13.0 * cc * cc + 5.0 * b * d - 13.0 * cc * d + 4.0 * d * d) / 3.0;
  beta[2] = (10.0 * cc * cc - 31.0 * cc * d + 25.0 * d * d + 11.0 * cc * e - 19.0 * d * e + 4.0 * e * e) / 3.0;
  /* Eq 14: quadratic interpolants at i+1/2 ... */
  sub_p[0] = 3.0 / 8.0 * a - 5.0 / 4.0 * b + 15.0 / 8.0 * cc;
  sub_p[1] = -1.0 / 8.0 * b + 3.0 / 4.0 * cc + 3.0 / 8.0 * d;
  sub_p[2] = 3.0 / 8.0 * cc + 3.0 / 4.0 * d - 1.0 / 8.0 * e;
  /* ... and their mirror images at i-1/2 */
  sub_m[0] = -1.0 / 8.0 * a + 3.0 / 4.0 * b + 3.0 / 8.0 * cc;
  sub_m[1] = 3.0 / 8.0 * b + 3.0 / 4.0 * cc - 1.0 / 8.0 * d;
  sub_m[2] = 15.0 / 8.0 * cc - 5.0 / 4.0 * d + 3.0 / 8.0 * e;
  /* Eqs 15-16 */
  for (j = 0; j < 3; ++j) {
    if (linear) {
      wp[j] = gam_p[j];
      wm[j] = gam_m[j];
    } else {
      wp[j] = gam_p[j] / ((eps + beta[j]) * (eps + beta[j]));
      wm[j] = gam_m[j] / ((eps + beta[j]) * (eps + beta[j]));
    }
    sp += wp[j];
    sm += wm[j];
  }
  /* Eq 13 */
  out[0] = (wp[0] * sub_p[0] + wp[1] * sub_p[1] + wp[2] * sub_p[2]) / sp;
  out[1] = (wm[0] * sub_m[0] + wm[1] * sub_m[1] + wm[2] * sub_m[2]) / sm;
  if (beta_out) for (j = 0; j < 3; ++j) beta_out[j] = beta[j];
}

/* ------------------------------------------------------------------------------------ */
/* Viscous fluxes (Eqs 5, 6, 21).  Gradients of (u, v, w, T) by d6 along xi, eta, zeta  */
/* at interior points, the chain rule with unhatted metrics xi_x = J * (xi_x/J), then   */
/* tau and beta scaled by Ma/Re, and the nodal viscous flux of each direction through   */
/* its hatted metrics.  Output V[12]: plane 4*d + (n-1) holds component n = 1..4 of the  */
/* direction-d viscous flux (component 0, continuity, is zero).                          */
/* Reading: Stokes' hypothesis lambda = -2/3 mu (Eq 1), Ma/Re multiplies tau and q      */
/* (Eq 1; Eq 6 prints the flux without it), q = mu/(Pr (gamma-1)) grad T.              */
/* ------------------------------------------------------------------------------------ */
static void viscous_fluxes(const oracle_cfg* c, const double* met, const double* Q, double* V) {
  const dims_t sd = state_dims(c);
  const double scale = c->mach / c->reynolds;
  int k;
#pragma omp parallel for schedule(static)
  for (k = 0; k < c->nk; ++k) {
    int i, j;
    for (j = 0; j < c->nj; ++j)
      for (i = 0; i < c->ni; ++i) {
        long p = sidx(&sd, i, j, k);
        double g[4][3]; /* d(u,v,w,T)/d(xi,eta,zeta) */
        double dx[4][3]; /* d(u,v,w,T)/d(x,y,z)       */
        double mh[3][3], mu_, Jp, tau[3][3], bet[3], div, lam;
        prim_t s0;
        int dir, n, a, b;
        for (dir = 0; dir < 3; ++dir) {
          int di, dj, dk, st, first, os;
          double line[4][7], w[7];
          const int node = dir == 0 ? i : dir == 1 ? j : k;
          unit(dir, &di, &dj, &dk);
          /* the seven nodes of the stencil: node-3..node+3, or a one-sided window */
          os = one_sided(c, dir, node, &first, w);
          if (!os) first = node - 3;
          for (st = 0; st < 7; ++st) {
            double qv[5];
            prim_t s;
            const int off = first + st - node;
            long pp = sidx(&sd, i + off * di, j + off * dj, k + off * dk);
            for (n = 0; n < 5; ++n) qv[n] = Q[n * sd.plane + pp];
            s = primitives(qv, c->gamma);
            line[0][st] = s.u; line[1][st] = s.v; line[2][st] = s.w; line[3][st] = s.T;
          }
          for (n = 0; n < 4; ++n) {
            if (os) {
              g[n][dir] = 0.0;
              for (st = 0; st < 7; ++st) g[n][dir] += w[st] * line[n][st];
            } else {
              g[n][dir] = d6(line[n]);
            }
          }
        }
        Jp = met[9 * sd.plane + p];
        for (a = 0; a < 3; ++a)
          for (b = 0; b < 3; ++b) mh[a][b] = met[(3 * a + b) * sd.plane + p];
        /* Eq 21 */
        for (n = 0; n < 4; ++n)
          for (b = 0; b < 3; ++b)
            dx[n][b] = Jp * (mh[0][b] * g[n][0] + mh[1][b] * g[n][1] + mh[2][b] * g[n][2]);
        {
          double qv[5];
          for (n = 0; n < 5; ++n) qv[n] = Q[n * sd.plane + p];
          s0 = primitives(qv, c->gamma);
        }
        mu_ = oracle_viscosity(s0.T, c->suth);
        lam = -2.0 / 3.0 * mu_;
        div = dx[0][0] + dx[1][1] + dx[2][2];
        /* Eq 6 (x Ma/Re) */
        for (a = 0; a < 3; ++a)
          for (b = 0; b < 3; ++b)
            tau[a][b] = scale * (mu_ * (dx[a][b] + dx[b][a]) + (a == b ? lam * div : 0.0));
        for (a = 0; a < 3; ++a)
          bet[a] = s0.u * tau[0][a] + s0.v * tau[1][a] + s0.w * tau[2][a] +
                   scale * mu_ / (c->prandtl * (c->gamma - 1.0)) * dx[3][a];
        /* Eq 5 */
        for (dir = 0; dir < 3; ++dir) {
          for (n = 0; n < 3; ++n)
            V[(4 * dir + n) * sd.plane + p] = mh[dir][0] * tau[n][0] + mh[dir][1] * tau[n][1] + mh[dir][2] * tau[n][2];
          V[(4 * dir + 3) * sd.plane + p] = mh[dir][0] * bet[0] + mh[dir][1] * bet[1] + mh[dir][2] * bet[2];
        }
      }
  }
}

/* ------------------------------------------------------------------------------------ */
/* Halo handling                                                                         */
/* ------------------------------------------------------------------------------------ */
static int wrapi(int i, int n) { return ((i % n) + n) % n; }

void oracle_periodic_wrap(const oracle_cfg* c, double* A, int nvar) {
  const dims_t sd = state_dims(c);
  const int per[3] = {c->bc[0] == ORACLE_BC_PERIODIC, c->bc[2] == ORACLE_BC_PERIODIC,
                      c->bc[4] == ORACLE_BC_PERIODIC};
  int v;
  for (v = 0; v < nvar; ++v) {
    double* P = A + (long)v * sd.plane;
    int i, j, k;
    for (k = -HS; k < c->nk + HS; ++k)
      for (j = -HS; j < c->nj + HS; ++j)
        for (i = -HS; i < c->ni + HS; ++i) {
          int si = per[0] ? wrapi(i, c->ni) : i;
          int sj = per[1] ? wrapi(j, c->nj) : j;
          int sk = per[2] ? wrapi(k, c->nk) : k;
          if (si != i || sj != j || sk != k) P[sidx(&sd, i, j, k)] = P[sidx(&sd, si, sj, sk)];
        }
  }
}

/* interior index of the boundary node of face f and the outward step along its axis */
static void face_geom(const oracle_cfg* c, int f, int* axis, int* wall_idx, int* outward) {
  *axis = f / 2;
  *outward = (f % 2) ? +1 : -1;
  *wall_idx = (f % 2) ? npts(c, *axis) - 1 : 0;
}

/* Nodes of face f that a patched connection covers (the multi-block driver's map per
 * face, indexed p1 + n1 * p2 with p1, p2 the node's indices along the face's tangential
 * axes t1 < t2); cov == NULL or cov[f] == NULL: none.  Covered nodes take the values of
 * the connected block instead of the physical treatment.                               */
static int face_covered(const oracle_cfg* c, const unsigned char* const* cov, int f, const int* idx) {
  int t1, t2;
  if (!cov || !cov[f]) return 0;
  t1 = f / 2 == 0 ? 1 : 0;
  t2 = f / 2 == 2 ? 1 : 2;
  return cov[f][idx[t1] + (long)npts(c, t1) * idx[t2]] != 0;
}

/* Reading (physical boundaries, not specified by the paper): the boundary node itself
 * is part of the interior.  Isothermal no-slip wall: after every stage the wall node gets
 * zero velocity and T = T_w at its own density (oracle_wall_reset, before any halo copy);
 * ghost m mirrors interior node m with odd velocity, the same pressure and
 * T_g = max(2 T_w - T_m, T_w / 2).  Far field: ghosts hold qinf (oracle_bc_fill).
 * Pinned by closed forms of Eq 1 next to a wall: the right-hand side of a shear mode and
 * of a conduction mode between isothermal walls, and the decay rate of the shear mode.  */
static void wall_reset_cov(const oracle_cfg* c, double* Q, const unsigned char* const* cov) {
  const dims_t sd = state_dims(c);
  int f;
  for (f = 0; f < 6; ++f) {
    int axis, w, out, a, b, na, nb;
    if (c->bc[f] != ORACLE_BC_WALL) continue;
    face_geom(c, f, &axis, &w, &out);
    na = npts(c, (axis + 1) % 3);
    nb = npts(c, (axis + 2) % 3);
    for (b = 0; b < nb; ++b)
      for (a = 0; a < na; ++a) {
        int idx[3];
        long pw;
        idx[(axis + 1) % 3] = a;
        idx[(axis + 2) % 3] = b;
        idx[axis] = w;
        if (face_covered(c, cov, f, idx)) continue;
        pw = sidx(&sd, idx[0], idx[1], idx[2]);
        Q[1 * sd.plane + pw] = 0.0;
        Q[2 * sd.plane + pw] = 0.0;
        Q[3 * sd.plane + pw] = 0.0;
        Q[4 * sd.plane + pw] = Q[pw] * c->t_wall / (c->gamma * (c->gamma - 1.0));
      }
  }
}

void oracle_wall_reset(const oracle_cfg* c, double* Q) { wall_reset_cov(c, Q, NULL); }

/* Characteristic far field (reading; the paper names no far-field treatment): locally
 * one-dimensional Riemann invariants along the outward unit normal n.  From the boundary
 * node's state b and the far-field state f, with u_n = u.n:
 *   u_n,b >= c_b: every wave leaves, the ghost state is b;  u_n,b <= -c_b: every wave
 *   enters, the ghost state is f;  otherwise R+ = u_n,b + 2 c_b/(gamma-1) comes from b and
 *   R- = u_n,f - 2 c_f/(gamma-1) from f, u_n = (R+ + R-)/2, c = (gamma-1)(R+ - R-)/4, and
 *   the entropy p/rho^gamma and the tangential velocity come from b if u_n > 0 (outflow),
 *   else from f.                                                                      */
void oracle_char_farfield(const double* qb, const double* n, const double* qf, double gamma, double* qg) {
  prim_t b = primitives(qb, gamma), f = primitives(qf, gamma);
  double unb = b.u * n[0] + b.v * n[1] + b.w * n[2];
  double unf = f.u * n[0] + f.v * n[1] + f.w * n[2];
  double rp, rm, un, c, s, ut[3], rho, p, u[3];
  int a;
  if (unb >= b.c) {
    for (a = 0; a < 5; ++a) qg[a] = qb[a];
    return;
  }
  if (unb <= -b.c) {
    for (a = 0; a < 5; ++a) qg[a] = qf[a];
    return;
  }
  rp = unb + 2.0 * b.c / (gamma - 1.0);
  rm = unf - 2.0 * f.c / (gamma - 1.0);
  un = 0.5 * (rp + rm);
  c = 0.25 * (gamma - 1.0) * (rp - rm);
  if (un > 0.0) {
    s = b.p / pow(b.rho, gamma);
    ut[0] = b.u - unb * n[0]; ut[1] = b.v - unb * n[1]; ut[2] = b.w - unb * n[2];
  } else {
    s = f.p / pow(f.rho, gamma);
    ut[0] = f.u - unf * n[0]; ut[1] = f.v - unf * n[1]; ut[2] = f.w - unf * n[2];
  }
  rho = pow(c * c / (gamma * s), 1.0 / (gamma - 1.0));
  p = rho * c * c / gamma;
  for (a = 0; a < 3; ++a) u[a] = ut[a] + un * n[a];
  qg[0] = rho;
  qg[1] = rho * u[0];
  qg[2] = rho * u[1];
  qg[3] = rho * u[2];
  qg[4] = p / (gamma - 1.0) + 0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
}

static void bc_fill_cov(const oracle_cfg* c, const double* met, double* Q, const unsigned char* const* cov) {
  const dims_t sd = state_dims(c);
  int f;
  for (f = 0; f < 6; ++f) {
    int axis, w, out, a, b, m, n;
    int na, nb;
    if (c->bc[f] == ORACLE_BC_FARFIELD_CHAR) {
      /* ghost layers 1..3 hold the state of oracle_char_farfield at the boundary node, the
       * normal being the face-normal direction's hatted metric there, pointing outward */
      if (!met) continue;
      face_geom(c, f, &axis, &w, &out);
      na = npts(c, (axis + 1) % 3);
      nb = npts(c, (axis + 2) % 3);
      for (b = 0; b < nb; ++b)
        for (a = 0; a < na; ++a) {
          int idx[3];
          long pw;
          double qb[5], qg[5], nv[3], mag;
          idx[(axis + 1) % 3] = a;
          idx[(axis + 2) % 3] = b;
          idx[axis] = w;
          if (face_covered(c, cov, f, idx)) continue;
          pw = sidx(&sd, idx[0], idx[1], idx[2]);
          for (n = 0; n < 5; ++n) qb[n] = Q[n * sd.plane + pw];
          for (n = 0; n < 3; ++n) nv[n] = met[(3 * axis + n) * sd.plane + pw];
          mag = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
          for (n = 0; n < 3; ++n) nv[n] = out * nv[n] / mag;
          oracle_char_farfield(qb, nv, c->qinf, c->gamma, qg);
          for (m = 1; m <= HS; ++m) {
            idx[axis] = w + out * m;
            for (n = 0; n < 5; ++n) Q[n * sd.plane + sidx(&sd, idx[0], idx[1], idx[2])] = qg[n];
          }
        }
      continue;
    }
    if (c->bc[f] != ORACLE_BC_WALL && c->bc[f] != ORACLE_BC_FARFIELD) continue;
    face_geom(c, f, &axis, &w, &out);
    na = npts(c, (axis + 1) % 3);
    nb = npts(c, (axis + 2) % 3);
    for (b = 0; b < nb; ++b)
      for (a = 0; a < na; ++a) {
        int idx[3];
        idx[(axis + 1) % 3] = a;
        idx[(axis + 2) % 3] = b;
        idx[axis] = w;
        if (face_covered(c, cov, f, idx)) continue;
        for (m = 1; m <= HS; ++m) {
          long pg, pm;
          idx[axis] = w + out * m;
          pg = sidx(&sd, idx[0], idx[1], idx[2]);
          idx[axis] = w - out * m;
          pm = sidx(&sd, idx[0], idx[1], idx[2]);
          if (c->bc[f] == ORACLE_BC_FARFIELD) {
            for (n = 0; n < 5; ++n) Q[n * sd.plane + pg] = c->qinf[n];
          } else {
            double qm[5];
            prim_t s;
            double Tg, rg;
            for (n = 0; n < 5; ++n) qm[n] = Q[n * sd.plane + pm];
            s = primitives(qm, c->gamma);
            /* reflection of T - T_w; floored at T_w / 2 so that the ghost density stays
             * positive when the mirror node is 1.5 times hotter than the wall or more */
            Tg = 2.0 * c->t_wall - s.T;
            if (Tg < 0.5 * c->t_wall) Tg = 0.5 * c->t_wall;
            rg = c->gamma * s.p / Tg;
            Q[pg] = rg;
            Q[1 * sd.plane + pg] = -rg * s.u;
            Q[2 * sd.plane + pg] = -rg * s.v;
            Q[3 * sd.plane + pg] = -rg * s.w;
            Q[4 * sd.plane + pg] = s.p / (c->gamma - 1.0) + 0.5 * rg * (s.u * s.u + s.v * s.v + s.w * s.w);
          }
        }
      }
  }
}

void oracle_bc_fill(const oracle_cfg* c, double* Q) { bc_fill_cov(c, NULL, Q, NULL); }

void oracle_bc_fill_met(const oracle_cfg* c, const double* met, double* Q) { bc_fill_cov(c, met, Q, NULL); }

/* Reading: at a wall or far-field face the ghost values of the viscous flux are the
 * odd reflection about the boundary node, F(w+out*m) = 2 F(w) - F(w-out*m), which keeps
 * linear flux profiles exact (the default closure; with ORACLE_VISC_ONE_SIDED the
 * viscous terms use no ghost value there).                                            */
static void visc_bc_fill(const oracle_cfg* c, double* V) {
  const dims_t sd = state_dims(c);
  int f;
  for (f = 0; f < 6; ++f) {
    int axis, w, out, a, b, m, n;
    int na, nb;
    if (!physical_face(c->bc[f])) continue;
    /* one-sided closures read no viscous ghost value across the face */
    if (c->visc_closure == ORACLE_VISC_ONE_SIDED) continue;
    face_geom(c, f, &axis, &w, &out);
    na = npts(c, (axis + 1) % 3);
    nb = npts(c, (axis + 2) % 3);
    for (b = 0; b < nb; ++b)
      for (a = 0; a < na; ++a) {
        int idx[3];
        long pw;
        idx[(axis + 1) % 3] = a;
        idx[(axis + 2) % 3] = b;
        idx[axis] = w;
        pw = sidx(&sd, idx[0], idx[1], idx[2]);
        for (m = 1; m <= HS; ++m) {
          long pg, pm;
          idx[axis] = w + out * m;
          pg = sidx(&sd, idx[0], idx[1], idx[2]);
          idx[axis] = w - out * m;
          pm = sidx(&sd, idx[0], idx[1], idx[2]);
          for (n = 0; n < 12; ++n) V[n * sd.plane + pg] = 2.0 * V[n * sd.plane + pw] - V[n * sd.plane + pm];
        }
      }
  }
}

/* ------------------------------------------------------------------------------------ */
/* Inviscid derivative along one grid line (modified AFWENO, Sec. 4.5.1, Figs 10-11,    */
/* assembled by Eq 19).  Inputs along the line, index s = node + 3 for node in          */
/* [-3, n+2]: q[s][5] conserved state, m[s][3] hatted metrics of this direction.        */
/* Output D[node][5] for node in [0, n).                                                */
/* ------------------------------------------------------------------------------------ */
static void afweno_line(const oracle_cfg* c, int n, const double (*q)[5], const double (*m)[3],
                        double (*D)[5], double (*Fp)[5], double (*Fm)[5], double (*fnode)[5],
                        double (*fhalf)[5]) {
  int node, v, t;
  /* Reading: half-point metrics are the sixth-order central interpolation
   * (3, -25, 150, 150, -25, 3)/256 of the node metrics; with Eq 19 it reproduces the
   * sixth-order derivative of the metrics, which keeps a uniform flow exactly uniform.  */
#define MHALF(node, comp)                                                                     \
  ((3.0 * m[(node) - 2 + 3][comp] - 25.0 * m[(node) - 1 + 3][comp] + 150.0 * m[(node) + 3][comp] + \
    150.0 * m[(node) + 1 + 3][comp] - 25.0 * m[(node) + 2 + 3][comp] + 3.0 * m[(node) + 3 + 3][comp]) / 256.0)

  /* split fluxes: F+ at node+1/2 from nodes -1..n-1, F- at node-1/2 from nodes 0..n */
  for (node = -1; node <= n; ++node) {
    double L[25], R[25], kt[3], mag, V[5][5], vl[5], vr[5], ul[5], ur[5];
    int a;
    mag = sqrt(m[node + 3][0] * m[node + 3][0] + m[node + 3][1] * m[node + 3][1] + m[node + 3][2] * m[node + 3][2]);
    for (a = 0; a < 3; ++a) kt[a] = m[node + 3][a] / mag;
    /* left and right eigenvectors at node i */
    oracle_eigvec(q[node + 3], kt, c->gamma, L, R);
    /* characteristic variables of the five stencil points, V[t] = L_i Q_{i+t-2} */
    for (t = 0; t < 5; ++t)
      for (v = 0; v < 5; ++v) {
        double acc = 0.0;
        for (a = 0; a < 5; ++a) acc += L[v * 5 + a] * q[node - 2 + t + 3][a];
        V[t][v] = acc;
      }
    /* WENO interpolation per characteristic field */
    for (v = 0; v < 5; ++v) {
      double col[5], out[2];
      for (t = 0; t < 5; ++t) col[t] = V[t][v];
      oracle_weno5(col, c->eps, c->linear_weights, out, NULL);
      vl[v] = out[0];
      vr[v] = out[1];
    }
    /* back to conserved variables with R_i */
    for (v = 0; v < 5; ++v) {
      double al = 0.0, ar = 0.0;
      for (a = 0; a < 5; ++a) { al += R[v * 5 + a] * vl[a]; ar += R[v * 5 + a] * vr[a]; }
      ul[v] = al;
      ur[v] = ar;
    }
    /* Reading: the left-biased state at i+1/2 feeds F+ and the right-biased state at
     * i-1/2 feeds F-, so that each split flux is upwinded.                            */
    if (node <= n - 1) {
      double mh[3], Fpp[5], Fmm[5];
      for (a = 0; a < 3; ++a) mh[a] = MHALF(node, a);
      oracle_split_flux(ul, mh, c->gamma, Fpp, Fmm);
      for (v = 0; v < 5; ++v) Fp[node + 1][v] = Fpp[v];
    }
    if (node >= 0) {
      double mh[3], Fpp[5], Fmm[5];
      for (a = 0; a < 3; ++a) mh[a] = MHALF(node - 1, a);
      oracle_split_flux(ur, mh, c->gamma, Fpp, Fmm);
      for (v = 0; v < 5; ++v) Fm[node][v] = Fmm[v];
    }
  }
  /* numerical flux at the half points node+1/2, node = -1..n-1:  f = F+(node) + F-(node+1) */
  for (node = -1; node <= n - 1; ++node)
    for (v = 0; v < 5; ++v) fhalf[node + 1][v] = Fp[node + 1][v] + Fm[node + 1][v];
  /* nodal physical flux, Eq 4 */
  for (node = -3; node <= n + 2; ++node) oracle_phys_flux(q[node + 3], m[node + 3], c->gamma, fnode[node + 3]);
  /* Eq 19 */
  for (node = 0; node < n; ++node)
    for (v = 0; v < 5; ++v) {
      const double fp = fhalf[node + 1][v], fm = fhalf[node][v];
      D[node][v] = fp - fm + 17.0 / 256.0 * (fnode[node + 1 + 3][v] - fnode[node - 1 + 3][v]) -
                   13.0 / 320.0 * (fnode[node + 2 + 3][v] - fnode[node - 2 + 3][v]) +
                   19.0 / 3840.0 * (fnode[node + 3 + 3][v] - fnode[node - 3 + 3][v]);
    }
#undef MHALF
}

/* ------------------------------------------------------------------------------------ */
/* Inviscid derivative along one grid line with the original AFWENO (Sec. 4.5.1, Fig 9): */
/* the characteristic space of each half point i+1/2 is built there, and the two split  */
/* fluxes of that half point come from two complete WENO interpolations in it.  Same   */
/* line layout as afweno_line.                                                          */
/* Readings: the state at i+1/2 is the arithmetic mean of the conserved states at i and  */
/* i+1 (the paper names no average); the direction of the characteristic space is the   */
/* half-point metric of the split fluxes, normalised.                                   */
/* ------------------------------------------------------------------------------------ */
static void afweno_line_original(const oracle_cfg* c, int n, const double (*q)[5], const double (*m)[3],
                                 double (*D)[5], double (*fnode)[5], double (*fhalf)[5]) {
  int node, v, t, a;
  for (node = -1; node <= n - 1; ++node) {
    double mh[3], kt[3], mag, qa[5], L[25], R[25], Vl[5][5], Vr[5][5], vl[5], vr[5], ul[5], ur[5];
    double Fpp[5], Fmm[5], Fpm[5], Fmp[5];
    /* half-point metrics (same sixth-order interpolation as the modified scheme) */
    for (a = 0; a < 3; ++a)
      mh[a] = (3.0 * m[node - 2 + 3][a] - 25.0 * m[node - 1 + 3][a] + 150.0 * m[node + 3][a] +
               150.0 * m[node + 1 + 3][a] - 25.0 * m[node + 2 + 3][a] + 3.0 * m[node + 3 + 3][a]) / 256.0;
    mag = sqrt(mh[0] * mh[0] + mh[1] * mh[1] + mh[2] * mh[2]);
    for (a = 0; a < 3; ++a) kt[a] = mh[a] / mag;
    /* left and right eigenvectors at i+1/2 */
    for (v = 0; v < 5; ++v) qa[v] = 0.5 * (q[node + 3][v] + q[node + 1 + 3][v]);
    oracle_eigvec(qa, kt, c->gamma, L, R);
    /* characteristic variables of (i-2..i+2) for the value left of i+1/2 and of
     * (i-1..i+3) for the value right of it, both in the space of i+1/2 */
    for (t = 0; t < 5; ++t)
      for (v = 0; v < 5; ++v) {
        double al = 0.0, ar = 0.0;
        for (a = 0; a < 5; ++a) {
          al += L[v * 5 + a] * q[node - 2 + t + 3][a];
          ar += L[v * 5 + a] * q[node - 1 + t + 3][a];
        }
        Vl[t][v] = al;
        Vr[t][v] = ar;
      }
    /* two WENO interpolations per field: the left-biased value at i+1/2 of the stencil
     * centred on i, and the right-biased value at (i+1)-1/2 of the stencil centred on i+1 */
    for (v = 0; v < 5; ++v) {
      double col[5], out[2];
      for (t = 0; t < 5; ++t) col[t] = Vl[t][v];
      oracle_weno5(col, c->eps, c->linear_weights, out, NULL);
      vl[v] = out[0];
      for (t = 0; t < 5; ++t) col[t] = Vr[t][v];
      oracle_weno5(col, c->eps, c->linear_weights, out, NULL);
      vr[v] = out[1];
    }
    /* back to conserved variables with R at i+1/2 */
    for (v = 0; v < 5; ++v) {
      double al = 0.0, ar = 0.0;
      for (a = 0; a < 5; ++a) { al += R[v * 5 + a] * vl[a]; ar += R[v * 5 + a] * vr[a]; }
      ul[v] = al;
      ur[v] = ar;
    }
    /* f(i+1/2) = F+(left value) + F-(right value), both through the half-point metric */
    oracle_split_flux(ul, mh, c->gamma, Fpp, Fpm);
    oracle_split_flux(ur, mh, c->gamma, Fmp, Fmm);
    for (v = 0; v < 5; ++v) fhalf[node + 1][v] = Fpp[v] + Fmm[v];
  }
  /* nodal physical flux, Eq 4, and the assembly of Eq 19 as in the modified scheme */
  for (node = -3; node <= n + 2; ++node) oracle_phys_flux(q[node + 3], m[node + 3], c->gamma, fnode[node + 3]);
  for (node = 0; node < n; ++node)
    for (v = 0; v < 5; ++v) {
      const double fp = fhalf[node + 1][v], fm = fhalf[node][v];
      D[node][v] = fp - fm + 17.0 / 256.0 * (fnode[node + 1 + 3][v] - fnode[node - 1 + 3][v]) -
                   13.0 / 320.0 * (fnode[node + 2 + 3][v] - fnode[node - 2 + 3][v]) +
                   19.0 / 3840.0 * (fnode[node + 3 + 3][v] - fnode[node - 3 + 3][v]);
    }
}

/* Rtilde contributions of all requested terms, then R = J * Rtilde (Eq 2, A: Q is
 * stored without 1/J and the grid is stationary, so dQ/dt = J * Rtilde).             */
static void rhs_core(const oracle_cfg* c, const double* met, const double* Q, const double* V,
                     double* R, unsigned mask, int k0, int k1) {
  const dims_t sd = state_dims(c);
  int dir;
  double* Rt;
  long p;
  int i, j, k;
  Rt = (double*)calloc((size_t)5 * sd.plane, sizeof(double));
  for (dir = 0; dir < 3; ++dir) {
    const int n = npts(c, dir);
    int di, dj, dk, na, nb;
    int line;
    if (!(mask & (1u << dir))) continue;
    unit(dir, &di, &dj, &dk);
    na = npts(c, (dir + 1) % 3);
    nb = npts(c, (dir + 2) % 3);
#pragma omp parallel for schedule(dynamic, 4)
    for (line = 0; line < na * nb; ++line) {
      int a = line % na, b = line / na, s, v, node;
      int base[3];
      double(*q)[5] = malloc(sizeof(double[5]) * (n + 6));
      double(*m)[3] = malloc(sizeof(double[3]) * (n + 6));
      double(*D)[5] = malloc(sizeof(double[5]) * n);
      double(*Fp)[5] = malloc(sizeof(double[5]) * (n + 1));
      double(*Fm)[5] = malloc(sizeof(double[5]) * (n + 1));
      double(*fn)[5] = malloc(sizeof(double[5]) * (n + 6));
      double(*fh)[5] = malloc(sizeof(double[5]) * (n + 1));
      base[(dir + 1) % 3] = a;
      base[(dir + 2) % 3] = b;
      base[dir] = 0;
      /* the k-range restriction (used to time a slab of the domain) */
      if (dir != 2 && (base[2] < k0 || base[2] >= k1)) goto done;
      for (s = -3; s < n + 3; ++s) {
        long pp = sidx(&sd, base[0] + s * di, base[1] + s * dj, base[2] + s * dk);
        for (v = 0; v < 5; ++v) q[s + 3][v] = Q[v * sd.plane + pp];
        for (v = 0; v < 3; ++v) m[s + 3][v] = met[(3 * dir + v) * sd.plane + pp];
      }
      if ((mask & ORACLE_INV) && c->scheme == ORACLE_AFWENO_ORIGINAL) {
        afweno_line_original(c, n, (const double(*)[5])q, (const double(*)[3])m, D, fn, fh);
      } else if (mask & ORACLE_INV) {
        afweno_line(c, n, (const double(*)[5])q, (const double(*)[3])m, D, Fp, Fm, fn, fh);
      } else {
        for (node = 0; node < n; ++node)
          for (v = 0; v < 5; ++v) D[node][v] = 0.0;
      }
      for (node = 0; node < n; ++node) {
        long pp = sidx(&sd, base[0] + node * di, base[1] + node * dj, base[2] + node * dk);
        int kk = base[2] + node * dk;
        if (kk < k0 || kk >= k1) continue;
        /* inviscid part enters with a minus sign (Eq 2) */
        for (v = 0; v < 5; ++v) Rt[v * sd.plane + pp] -= D[node][v];
        /* viscous part: d6 along the line of the direction-dir viscous flux */
        if ((mask & ORACLE_VIS) && c->viscous) {
          double w[7];
          int first;
          const int os = one_sided(c, dir, node, &first, w);
          if (!os) first = node - 3;
          for (v = 1; v < 5; ++v) {
            double g[7], sum = 0.0;
            int st;
            for (st = 0; st < 7; ++st)
              g[st] = V[(4 * dir + v - 1) * sd.plane +
                        sidx(&sd, base[0] + (first + st) * di, base[1] + (first + st) * dj, base[2] + (first + st) * dk)];
            if (os) {
              for (st = 0; st < 7; ++st) sum += w[st] * g[st];
            } else {
              sum = d6(g);
            }
            Rt[v * sd.plane + pp] += sum;
          }
        }
      }
    done:
      free(q); free(m); free(D); free(Fp); free(Fm); free(fn); free(fh);
    }
  }
  for (k = k0; k < k1; ++k)
    for (j = 0; j < c->nj; ++j)
      for (i = 0; i < c->ni; ++i) {
        int v;
        p = sidx(&sd, i, j, k);
        for (v = 0; v < 5; ++v) R[v * sd.plane + p] = met[9 * sd.plane + p] * Rt[v * sd.plane + p];
      }
  free(Rt);
}

static int check_cfg(const oracle_cfg* c) {
  if (c->ni < 7 || c->nj < 7 || c->nk < 7) return -1;
  if (c->scheme != ORACLE_AFWENO_MODIFIED && c->scheme != ORACLE_AFWENO_ORIGINAL) return -1;
  if (c->visc_closure != ORACLE_VISC_REFLECT && c->visc_closure != ORACLE_VISC_ONE_SIDED) return -1;
  return 0;
}

/* Viscous flux planes with halos filled for a single block (periodic wrap + physical
 * faces).  Interface faces are left for the multi-block driver.                        */
static double* visc_planes(const oracle_cfg* c, const double* met, const double* Q) {
  const dims_t sd = state_dims(c);
  double* V = (double*)calloc((size_t)12 * sd.plane, sizeof(double));
  viscous_fluxes(c, met, Q, V);
  oracle_periodic_wrap(c, V, 12);
  visc_bc_fill(c, V);
  return V;
}

int oracle_rhs(const oracle_cfg* c, const double* met, const double* Q, double* R, unsigned mask,
               int k0, int k1) {
  double* V = NULL;
  if (check_cfg(c)) return -1;
  if (k0 < 0) k0 = 0;
  if (k1 > c->nk) k1 = c->nk;
  if ((mask & ORACLE_VIS) && c->viscous) V = visc_planes(c, met, Q);
  rhs_core(c, met, Q, V, R, mask, k0, k1);
  free(V);
  return 0;
}

/* Eq 20 coefficients (a, b, c) of Qout = a Qn + b Qcur + c dt R(Qcur) */
static const double RK3[3][3] = {{1.0, 0.0, 1.0}, {3.0 / 4.0, 1.0 / 4.0, 1.0 / 4.0}, {1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0}};

/* dtf: a time step per point (one plane in the state layout) in place of dt, or NULL */
static void rk_combine_dt(const oracle_cfg* c, int stage, double dt, const double* dtf, const double* Qn,
                          const double* Qcur, const double* R, double* Qout) {
  const dims_t sd = state_dims(c);
  int i, j, k, v;
  for (v = 0; v < 5; ++v)
    for (k = 0; k < c->nk; ++k)
      for (j = 0; j < c->nj; ++j)
        for (i = 0; i < c->ni; ++i) {
          long pp = sidx(&sd, i, j, k), p = v * sd.plane + pp;
          double h = dtf ? dtf[pp] : dt;
          Qout[p] = RK3[stage][0] * Qn[p] + RK3[stage][1] * Qcur[p] + RK3[stage][2] * h * R[p];
        }
}

static void rk_combine(const oracle_cfg* c, int stage, double dt, const double* Qn, const double* Qcur,
                       const double* R, double* Qout) {
  rk_combine_dt(c, stage, dt, NULL, Qn, Qcur, R, Qout);
}

static int rk_stage_dt(const oracle_cfg* c, const double* met, int stage, double dt, const double* dtf,
                       const double* Qn, const double* Qcur, double* Qout) {
  const dims_t sd = state_dims(c);
  double* R;
  int rc;
  if (stage < 0 || stage > 2) return -1;
  R = (double*)calloc((size_t)5 * sd.plane, sizeof(double));
  rc = oracle_rhs(c, met, Qcur, R, ORACLE_ALL, 0, c->nk);
  if (rc == 0) {
    rk_combine_dt(c, stage, dt, dtf, Qn, Qcur, R, Qout);
    oracle_wall_reset(c, Qout);
    oracle_periodic_wrap(c, Qout, 5);
    oracle_bc_fill_met(c, met, Qout);
  }
  free(R);
  return rc;
}

int oracle_rk_stage(const oracle_cfg* c, const double* met, int stage, double dt, const double* Qn,
                    const double* Qcur, double* Qout) {
  return rk_stage_dt(c, met, stage, dt, NULL, Qn, Qcur, Qout);
}

static int rk_step_dt(const oracle_cfg* c, const double* met, double dt, const double* dtf, double* Q) {
  const dims_t sd = state_dims(c);
  size_t bytes = (size_t)5 * sd.plane * sizeof(double);
  double* A = (double*)malloc(bytes);
  double* B = (double*)malloc(bytes);
  int rc;
  memcpy(A, Q, bytes);
  memcpy(B, Q, bytes);
  rc = rk_stage_dt(c, met, 0, dt, dtf, Q, Q, A);
  if (!rc) rc = rk_stage_dt(c, met, 1, dt, dtf, Q, A, B);
  if (!rc) rc = rk_stage_dt(c, met, 2, dt, dtf, Q, B, A);
  if (!rc) memcpy(Q, A, bytes);
  free(A);
  free(B);
  return rc;
}

int oracle_rk_step(const oracle_cfg* c, const double* met, double dt, double* Q) {
  return rk_step_dt(c, met, dt, NULL, Q);
}

int oracle_rk_step_local(const oracle_cfg* c, const double* met, const double* dt_field, double* Q) {
  if (!dt_field) return -1;
  return rk_step_dt(c, met, 0.0, dt_field, Q);
}

/* Reading: dt = CFL / max over interior points of sum_d (|U_d| + c |grad d|) with the
 * unhatted metrics grad d = J * (hatted metrics of d); the inviscid limit only.         */
double oracle_dt_cfl(const oracle_cfg* c, const double* met, const double* Q, double cfl) {
  const dims_t sd = state_dims(c);
  double smax = 0.0;
  int bad = 0;
  int k;
#pragma omp parallel for reduction(max : smax) reduction(| : bad) schedule(static)
  for (k = 0; k < c->nk; ++k) {
    int i, j, d, n;
    for (j = 0; j < c->nj; ++j)
      for (i = 0; i < c->ni; ++i) {
        long p = sidx(&sd, i, j, k);
        double q[5], sum = 0.0, Jp = met[9 * sd.plane + p];
        prim_t s;
        for (n = 0; n < 5; ++n) q[n] = Q[n * sd.plane + p];
        s = primitives(q, c->gamma);
        for (d = 0; d < 3; ++d) {
          double mx = Jp * met[(3 * d + 0) * sd.plane + p];
          double my = Jp * met[(3 * d + 1) * sd.plane + p];
          double mz = Jp * met[(3 * d + 2) * sd.plane + p];
          sum += fabs(mx * s.u + my * s.v + mz * s.w) + s.c * sqrt(mx * mx + my * my + mz * mz);
        }
        if (!(sum <= 1.7976931348623157e308)) bad = 1;  /* NaN or infinite */
        if (sum > smax) smax = sum;
      }
  }
  return bad ? NAN : cfl / smax;
}

/* Local time steps (steady runs): the same spectral radius, point by point.  Reading: the
 * stored step of each point is cfl / sum_d (|U_d| + c |grad d|) (inviscid limit only, as
 * for the global step); halo entries are left untouched.                                */
void oracle_dt_local(const oracle_cfg* c, const double* met, const double* Q, double cfl, double* dt_field) {
  const dims_t sd = state_dims(c);
  int k;
#pragma omp parallel for schedule(static)
  for (k = 0; k < c->nk; ++k) {
    int i, j, d, n;
    for (j = 0; j < c->nj; ++j)
      for (i = 0; i < c->ni; ++i) {
        long p = sidx(&sd, i, j, k);
        double q[5], sum = 0.0, Jp = met[9 * sd.plane + p];
        prim_t s;
        for (n = 0; n < 5; ++n) q[n] = Q[n * sd.plane + p];
        s = primitives(q, c->gamma);
        for (d = 0; d < 3; ++d) {
          double mx = Jp * met[(3 * d + 0) * sd.plane + p];
          double my = Jp * met[(3 * d + 1) * sd.plane + p];
          double mz = Jp * met[(3 * d + 2) * sd.plane + p];
          sum += fabs(mx * s.u + my * s.v + mz * s.w) + s.c * sqrt(mx * mx + my * my + mz * mz);
        }
        dt_field[p] = cfl / sum;
      }
  }
}

/* ------------------------------------------------------------------------------------ */
/* Multi-block: 1-to-1 aligned faces.  Face f of block a abuts face g of block b; the    */
/* halo of a across f holds b's interior layers adjacent to g, with the tangential      */
/* indices identical (identity orientation).                                            */
/* ------------------------------------------------------------------------------------ */
/* The axes of block B that the index directions of block A run along across the face
 * pair (fa, fb) with tangential map `orient` (see oracle_iface), and their senses:
 * dir[d] is B's axis for A's axis d, sgn[d] = +1 if both indices increase together.     */
static void face_dirs(int fa, int fb, int orient, int* dir, int* sgn) {
  int axa = fa / 2, axb = fb / 2, outa = (fa % 2) ? +1 : -1, outb = (fb % 2) ? +1 : -1;
  int ta[2], tb[2], q;
  ta[0] = axa == 0 ? 1 : 0; ta[1] = axa == 2 ? 1 : 2;
  tb[0] = axb == 0 ? 1 : 0; tb[1] = axb == 2 ? 1 : 2;
  /* across the face, A's normal index grows outward while B's grows inward from fb */
  dir[axa] = axb;
  sgn[axa] = -outa * outb;
  for (q = 0; q < 2; ++q) {
    dir[ta[q]] = (orient & 1) ? tb[1 - q] : tb[q];
    sgn[ta[q]] = ((orient >> (1 + q)) & 1) ? -1 : +1;
  }
}

/* Ghost layers beyond the rectangle of face fa of block A that starts at alo and spans n
 * nodes along A's tangential axes t1 < t2, from the interior layers inside the partner
 * rectangle of face fb of block B, which starts at blo along B's t1 < t2 (see
 * oracle_patch).  visc = 0: nvar planes copied as they are.  visc = 1: the 12
 * viscous-flux planes, 4 per index direction (Eqs 5-6 through that direction's hatted
 * metric): A's direction d is B's direction dir[d], so A's planes of d take B's planes of
 * dir[d], with the sign of sgn[d] (a reversed index reverses the hatted metric and the
 * flux).                                                                               */
static void copy_patch(const oracle_cfg* ca, double* A, int fa, const int* alo, const int* n,
                       const oracle_cfg* cb, const double* B, int fb, const int* blo, int orient, int nvar,
                       int visc) {
  const dims_t da = state_dims(ca), db = state_dims(cb);
  int axa = fa / 2, axb = fb / 2, outa = (fa % 2) ? +1 : -1, outb = (fb % 2) ? +1 : -1;
  int wa = (fa % 2) ? npts(ca, axa) - 1 : 0;
  int wb = (fb % 2) ? npts(cb, axb) - 1 : 0;
  int ta0 = axa == 0 ? 1 : 0, ta1 = axa == 2 ? 1 : 2;
  int tb0 = axb == 0 ? 1 : 0;
  int dir[3], sgn[3];
  int lo0, lo1;  /* B's rectangle corner along the axes that A's t1 and t2 run along */
  int a, b, m, v, d;
  face_dirs(fa, fb, orient, dir, sgn);
  lo0 = dir[ta0] == tb0 ? blo[0] : blo[1];
  lo1 = dir[ta1] == tb0 ? blo[0] : blo[1];
  for (b = 0; b < n[1]; ++b)
    for (a = 0; a < n[0]; ++a)
      for (m = 1; m <= HS; ++m) {
        int ia[3], ib[3];
        long pa, pb;
        ia[ta0] = alo[0] + a; ia[ta1] = alo[1] + b; ia[axa] = wa + outa * m;
        /* ghost m beyond face fa is interior layer m-1 inside face fb */
        ib[axb] = wb - outb * (m - 1);
        ib[dir[ta0]] = sgn[ta0] > 0 ? lo0 + a : lo0 + n[0] - 1 - a;
        ib[dir[ta1]] = sgn[ta1] > 0 ? lo1 + b : lo1 + n[1] - 1 - b;
        pa = sidx(&da, ia[0], ia[1], ia[2]);
        pb = sidx(&db, ib[0], ib[1], ib[2]);
        if (!visc) {
          for (v = 0; v < nvar; ++v) A[v * da.plane + pa] = B[v * db.plane + pb];
        } else {
          for (d = 0; d < 3; ++d)
            for (v = 0; v < 4; ++v) A[(4 * d + v) * da.plane + pa] = sgn[d] * B[(4 * dir[d] + v) * db.plane + pb];
        }
      }
}

/* The whole face fa of A from the whole face fb of B. */
static void copy_face(const oracle_cfg* ca, double* A, int fa, const oracle_cfg* cb, const double* B,
                      int fb, int orient, int nvar, int visc) {
  const int axa = fa / 2, zero[2] = {0, 0};
  const int n[2] = {npts(ca, axa == 0 ? 1 : 0), npts(ca, axa == 2 ? 1 : 2)};
  copy_patch(ca, A, fa, zero, n, cb, B, fb, zero, orient, nvar, visc);
}

static int exchange(const oracle_cfg* cfgs, int nb, double* const* arrays, int nvar, int visc,
                    const oracle_iface* ifc, int nifc) {
  int n, d;
  for (n = 0; n < nifc; ++n) {
    const oracle_iface* f = &ifc[n];
    int dir[3], sgn[3];
    if (f->block_a < 0 || f->block_a >= nb || f->block_b < 0 || f->block_b >= nb) return -1;
    if (f->face_a < 0 || f->face_a > 5 || f->face_b < 0 || f->face_b > 5 || f->orient < 0 || f->orient > 7) return -1;
    face_dirs(f->face_a, f->face_b, f->orient, dir, sgn);
    for (d = 0; d < 3; ++d)
      if (d != f->face_a / 2 && npts(&cfgs[f->block_a], d) != npts(&cfgs[f->block_b], dir[d])) return -1;
  }
  for (n = 0; n < nifc; ++n) {
    const oracle_iface* f = &ifc[n];
    /* the same interface seen from b: swap stays, the reversals follow their axes */
    int r1 = (f->orient >> 1) & 1, r2 = (f->orient >> 2) & 1;
    int inv = (f->orient & 1) ? (1 | (r2 << 1) | (r1 << 2)) : f->orient;
    copy_face(&cfgs[f->block_a], arrays[f->block_a], f->face_a, &cfgs[f->block_b], arrays[f->block_b], f->face_b,
              f->orient, nvar, visc);
    copy_face(&cfgs[f->block_b], arrays[f->block_b], f->face_b, &cfgs[f->block_a], arrays[f->block_a], f->face_a,
              inv, nvar, visc);
  }
  return 0;
}

int oracle_exchange(const oracle_cfg* cfgs, int nb, double* const* arrays, int nvar,
                    const oracle_iface* ifc, int nifc) {
  return exchange(cfgs, nb, arrays, nvar, 0, ifc, nifc);
}

int oracle_rhs_multi(const oracle_cfg* cfgs, int nb, const double* const* met, const double* const* Q,
                     double* const* R, unsigned mask, const oracle_iface* ifc, int nifc) {
  double** V = (double**)calloc((size_t)nb, sizeof(double*));
  int b, rc = 0;
  for (b = 0; b < nb; ++b)
    if (check_cfg(&cfgs[b])) rc = -1;
  if (!rc && (mask & ORACLE_VIS)) {
    for (b = 0; b < nb; ++b)
      if (cfgs[b].viscous) V[b] = visc_planes(&cfgs[b], met[b], Q[b]);
      else V[b] = (double*)calloc((size_t)12 * state_dims(&cfgs[b]).plane, sizeof(double));
    /* viscous flux layers across interfaces (interior scheme at block interfaces) */
    rc = exchange(cfgs, nb, V, 12, 1, ifc, nifc);
  }
  if (!rc)
    for (b = 0; b < nb; ++b) rhs_core(&cfgs[b], met[b], Q[b], V[b], R[b], mask, 0, cfgs[b].nk);
  for (b = 0; b < nb; ++b) free(V[b]);
  free(V);
  return rc;
}

int oracle_rk_step_multi(const oracle_cfg* cfgs, int nb, const double* const* met, double dt,
                         double* const* Q, const oracle_iface* ifc, int nifc) {
  double **Qn = malloc(sizeof(double*) * nb), **A = malloc(sizeof(double*) * nb),
         **Bq = malloc(sizeof(double*) * nb), **R = malloc(sizeof(double*) * nb);
  int b, stage, rc = 0;
  for (b = 0; b < nb; ++b) {
    size_t bytes = (size_t)5 * state_dims(&cfgs[b]).plane * sizeof(double);
    Qn[b] = Q[b];
    A[b] = malloc(bytes);
    Bq[b] = malloc(bytes);
    R[b] = calloc(1, bytes);
    memcpy(A[b], Q[b], bytes);
    memcpy(Bq[b], Q[b], bytes);
  }
  for (stage = 0; stage < 3 && !rc; ++stage) {
    double** cur = stage == 0 ? Qn : stage == 1 ? A : Bq;
    double** out = stage == 0 ? A : stage == 1 ? Bq : A;
    rc = oracle_rhs_multi(cfgs, nb, (const double* const*)met, (const double* const*)cur, R, ORACLE_ALL, ifc, nifc);
    if (rc) break;
    for (b = 0; b < nb; ++b) rk_combine(&cfgs[b], stage, dt, Qn[b], cur[b], R[b], out[b]);
    for (b = 0; b < nb; ++b) oracle_wall_reset(&cfgs[b], out[b]);
    for (b = 0; b < nb; ++b) oracle_periodic_wrap(&cfgs[b], out[b], 5);
    rc = oracle_exchange(cfgs, nb, out, 5, ifc, nifc);
    for (b = 0; b < nb; ++b) oracle_bc_fill_met(&cfgs[b], met[b], out[b]);
  }
  for (b = 0; b < nb && !rc; ++b) memcpy(Q[b], A[b], (size_t)5 * state_dims(&cfgs[b]).plane * sizeof(double));
  for (b = 0; b < nb; ++b) { free(A[b]); free(Bq[b]); free(R[b]); }
  free(Qn); free(A); free(Bq); free(R);
  return rc;
}

/* ------------------------------------------------------------------------------------ */
/* Multi-block with patched connections (Sec. 3: arbitrary splits, connecting and        */
/* physical faces defined anywhere on a block's faces).                                  */
/* ------------------------------------------------------------------------------------ */
/* The same patch seen from block_b: the corners trade places, the extents follow b's
 * axes, and the orientation is inverted (the swap stays, the reversals follow their axes). */
static oracle_patch patch_from_b(const oracle_patch* p) {
  oracle_patch q;
  const int r1 = (p->orient >> 1) & 1, r2 = (p->orient >> 2) & 1;
  q.block_a = p->block_b;
  q.face_a = p->face_b;
  q.block_b = p->block_a;
  q.face_b = p->face_a;
  q.a_lo[0] = p->b_lo[0];
  q.a_lo[1] = p->b_lo[1];
  q.b_lo[0] = p->a_lo[0];
  q.b_lo[1] = p->a_lo[1];
  if (p->orient & 1) {
    q.n[0] = p->n[1];
    q.n[1] = p->n[0];
    q.orient = 1 | (r2 << 1) | (r1 << 2);
  } else {
    q.n[0] = p->n[0];
    q.n[1] = p->n[1];
    q.orient = p->orient;
  }
  return q;
}

typedef struct {
  unsigned char* cov[6];  /* per face: 1 at the nodes a patch covers (see face_covered) */
} block_cover;

static void free_cover(block_cover* cv, int nb) {
  int b, f;
  for (b = 0; b < nb; ++b)
    for (f = 0; f < 6; ++f) free(cv[b].cov[f]);
  free(cv);
}

/* Check the patches against the rules of oracle_patch and mark the nodes they cover on
 * both sides.  Returns NULL on a violation.                                            */
static block_cover* cover_patches(const oracle_cfg* cfgs, int nb, const oracle_patch* p, int np) {
  block_cover* cv = (block_cover*)calloc((size_t)nb, sizeof(block_cover));
  int k, side, b, f;
  for (k = 0; k < np; ++k)
    for (side = 0; side < 2; ++side) {
      const oracle_patch q = side ? patch_from_b(&p[k]) : p[k];
      const oracle_cfg *ca, *cb;
      int t1a, t2a, t1b, t2b, e0, e1, x, y, n1;
      if (q.block_a < 0 || q.block_a >= nb || q.block_b < 0 || q.block_b >= nb || q.face_a < 0 || q.face_a > 5 ||
          q.face_b < 0 || q.face_b > 5 || q.orient < 0 || q.orient > 7 ||
          (q.block_a == q.block_b && q.face_a == q.face_b))
        goto bad;
      ca = &cfgs[q.block_a];
      cb = &cfgs[q.block_b];
      t1a = q.face_a / 2 == 0 ? 1 : 0;
      t2a = q.face_a / 2 == 2 ? 1 : 2;
      t1b = q.face_b / 2 == 0 ? 1 : 0;
      t2b = q.face_b / 2 == 2 ? 1 : 2;
      e0 = (q.orient & 1) ? q.n[1] : q.n[0]; /* extents along b's t1, t2 */
      e1 = (q.orient & 1) ? q.n[0] : q.n[1];
      if (q.n[0] < 1 || q.n[1] < 1 || q.a_lo[0] < 0 || q.a_lo[1] < 0 || q.a_lo[0] + q.n[0] > npts(ca, t1a) ||
          q.a_lo[1] + q.n[1] > npts(ca, t2a) || q.b_lo[0] < 0 || q.b_lo[1] < 0 || q.b_lo[0] + e0 > npts(cb, t1b) ||
          q.b_lo[1] + e1 > npts(cb, t2b))
        goto bad;
      if (ca->bc[q.face_a] == ORACLE_BC_PERIODIC) goto bad;
      if (physical_face(ca->bc[q.face_a]) && ca->visc_closure == ORACLE_VISC_ONE_SIDED) goto bad;
      n1 = npts(ca, t1a);
      if (!cv[q.block_a].cov[q.face_a]) cv[q.block_a].cov[q.face_a] = (unsigned char*)calloc((size_t)n1 * npts(ca, t2a), 1);
      for (y = 0; y < q.n[1]; ++y)
        for (x = 0; x < q.n[0]; ++x) {
          unsigned char* c = &cv[q.block_a].cov[q.face_a][(q.a_lo[0] + x) + (long)n1 * (q.a_lo[1] + y)];
          if (*c) goto bad; /* a node covered twice */
          *c = 1;
        }
    }
  for (b = 0; b < nb; ++b)
    for (f = 0; f < 6; ++f)
      if (cfgs[b].bc[f] == ORACLE_BC_INTERFACE) {
        const int t1 = f / 2 == 0 ? 1 : 0, t2 = f / 2 == 2 ? 1 : 2;
        long e, ne = (long)npts(&cfgs[b], t1) * npts(&cfgs[b], t2);
        if (!cv[b].cov[f]) goto bad;
        for (e = 0; e < ne; ++e)
          if (!cv[b].cov[f][e]) goto bad; /* an interface face with a node left open */
      }
  return cv;
bad:
  free_cover(cv, nb);
  return NULL;
}

static void exchange_patched(const oracle_cfg* cfgs, double* const* arrays, int nvar, int visc, const oracle_patch* p,
                             int np) {
  int k, side;
  for (k = 0; k < np; ++k)
    for (side = 0; side < 2; ++side) {
      const oracle_patch q = side ? patch_from_b(&p[k]) : p[k];
      copy_patch(&cfgs[q.block_a], arrays[q.block_a], q.face_a, q.a_lo, q.n, &cfgs[q.block_b], arrays[q.block_b],
                 q.face_b, q.b_lo, q.orient, nvar, visc);
    }
}

static void halo_cov(const oracle_cfg* cfgs, int nb, const double* const* met, double* const* Q, const oracle_patch* p,
                     int np, const block_cover* cv) {
  int b;
  for (b = 0; b < nb; ++b) wall_reset_cov(&cfgs[b], Q[b], (const unsigned char* const*)cv[b].cov);
  for (b = 0; b < nb; ++b) oracle_periodic_wrap(&cfgs[b], Q[b], 5);
  exchange_patched(cfgs, Q, 5, 0, p, np);
  for (b = 0; b < nb; ++b) bc_fill_cov(&cfgs[b], met ? met[b] : NULL, Q[b], (const unsigned char* const*)cv[b].cov);
}

int oracle_halo_patched(const oracle_cfg* cfgs, int nb, const double* const* met, double* const* Q,
                        const oracle_patch* p, int np) {
  block_cover* cv = cover_patches(cfgs, nb, p, np);
  if (!cv) return -1;
  halo_cov(cfgs, nb, met, Q, p, np, cv);
  free_cover(cv, nb);
  return 0;
}

static int rhs_patched(const oracle_cfg* cfgs, int nb, const double* const* met, const double* const* Q,
                       double* const* R, unsigned mask, const oracle_patch* p, int np) {
  double** V = (double**)calloc((size_t)nb, sizeof(double*));
  int b, rc = 0;
  for (b = 0; b < nb; ++b)
    if (check_cfg(&cfgs[b])) rc = -1;
  if (!rc && (mask & ORACLE_VIS)) {
    for (b = 0; b < nb; ++b)
      if (cfgs[b].viscous) V[b] = visc_planes(&cfgs[b], met[b], Q[b]);
      else V[b] = (double*)calloc((size_t)12 * state_dims(&cfgs[b]).plane, sizeof(double));
    /* the covered nodes of partly physical faces get the connected block's fluxes over
     * the reflected ghosts visc_planes put there */
    exchange_patched(cfgs, V, 12, 1, p, np);
  }
  if (!rc)
    for (b = 0; b < nb; ++b) rhs_core(&cfgs[b], met[b], Q[b], V[b], R[b], mask, 0, cfgs[b].nk);
  for (b = 0; b < nb; ++b) free(V[b]);
  free(V);
  return rc;
}

int oracle_rhs_patched(const oracle_cfg* cfgs, int nb, const double* const* met, const double* const* Q,
                       double* const* R, unsigned mask, const oracle_patch* p, int np) {
  block_cover* cv = cover_patches(cfgs, nb, p, np);
  int rc;
  if (!cv) return -1;
  rc = rhs_patched(cfgs, nb, met, Q, R, mask, p, np);
  free_cover(cv, nb);
  return rc;
}

int oracle_rk_step_patched(const oracle_cfg* cfgs, int nb, const double* const* met, double dt,
                           double* const* Q, const oracle_patch* p, int np) {
  block_cover* cv = cover_patches(cfgs, nb, p, np);
  double **Qn, **A, **Bq, **R;
  int b, stage, rc = 0;
  if (!cv) return -1;
  Qn = malloc(sizeof(double*) * nb);
  A = malloc(sizeof(double*) * nb);
  Bq = malloc(sizeof(double*) * nb);
  R = malloc(sizeof(double*) * nb);
  for (b = 0; b < nb; ++b) {
    size_t bytes = (size_t)5 * state_dims(&cfgs[b]).plane * sizeof(double);
    Qn[b] = Q[b];
    A[b] = malloc(bytes);
    Bq[b] = malloc(bytes);
    R[b] = calloc(1, bytes);
    memcpy(A[b], Q[b], bytes);
    memcpy(Bq[b], Q[b], bytes);
  }
  for (stage = 0; stage < 3 && !rc; ++stage) {
    double** cur = stage == 0 ? Qn : stage == 1 ? A : Bq;
    double** out = stage == 0 ? A : stage == 1 ? Bq : A;
    rc = rhs_patched(cfgs, nb, met, (const double* const*)cur, R, ORACLE_ALL, p, np);
    if (rc) break;
    for (b = 0; b < nb; ++b) rk_combine(&cfgs[b], stage, dt, Qn[b], cur[b], R[b], out[b]);
    halo_cov(cfgs, nb, met, out, p, np, cv);
  }
  for (b = 0; b < nb && !rc; ++b) memcpy(Q[b], A[b], (size_t)5 * state_dims(&cfgs[b]).plane * sizeof(double));
  for (b = 0; b < nb; ++b) {
    free(A[b]);
    free(Bq[b]);
    free(R[b]);
  }
  free(Qn);
  free(A);
  free(Bq);
  free(R);
  free_cover(cv, nb);
  return rc;
}

int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int oracle_set_threads(int n) {
  int before = oracle_threads();
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
  return before;
}
