// cfd_api.hip -- host side of libcfd: the C ABI declared in include/cfd.h.
//
// Block objects own the metric planes and the RHS scratch; exchange plans own device
// tables of face-copy segments; batches own work lists and captured HIP graphs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cfd.h"
#include "cfd_kernels.hpp"

using namespace cfd;

// =====================================================================================
// errors
// =====================================================================================
namespace {
thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
int hip_fail(hipError_t e, const char* what) {
  return fail(CFD_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}
#define HIP_TRY(expr, what)                   \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

bool is_real_size(int n) { return n >= 7 && n <= (1 << 20); }

// ---- profiling ----------------------------------------------------------------------
struct ProfPending {
  const char* name;
  hipEvent_t a, b;
};
struct Profiler {
  bool on = false;
  std::vector<ProfPending> pending;
  std::vector<hipEvent_t> pool;
  std::map<std::string, std::pair<int64_t, double>> acc;
  std::vector<std::string> order;

  hipEvent_t ev() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void drain() {
    for (auto& p : pending) {
      float ms = 0.f;
      if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        auto it = acc.find(p.name);
        if (it == acc.end()) {
          order.push_back(p.name);
          acc[p.name] = {1, (double)ms};
        } else {
          it->second.first += 1;
          it->second.second += ms;
        }
      }
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
  }
  ~Profiler() {
    for (auto& p : pending) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// RAII bracket: records the start event on construction and the stop event on done().
struct ProfScope {
  Profiler* P;
  const char* name;
  hipStream_t s;
  hipEvent_t a = nullptr;
  ProfScope(Profiler* p, const char* n, hipStream_t st) : P(p), name(n), s(st) {
    if (P && P->on) {
      a = P->ev();
      if (a) (void)hipEventRecord(a, s);
    }
  }
  void done() {
    if (P && P->on && a) {
      hipEvent_t b = P->ev();
      if (b) {
        (void)hipEventRecord(b, s);
        P->pending.push_back({name, a, b});
        if (P->pending.size() > 4096) P->drain();
      }
      a = nullptr;
    }
  }
};
}  // namespace

// =====================================================================================
// block
// =====================================================================================
// tile shapes of a block's own sweeps until cfd_block_set_tiles, [FP64 / mixed][direction]
// (measured on the 512 x 512 x 384 channel): 4 lines x 58 nodes along xi; 8 x 30 along eta
// and zeta in FP64; 16 x 14 along eta and 16 x 30 (512 threads) along zeta in mixed
// precision
constexpr int kDefaultTiles[2][3] = {{5, 6, 6}, {5, 2, 0}};

struct cfd_block {
  cfd_block_desc d;
  Geom g;
  hipStream_t stream = nullptr;
  int device = 0;
  double* met = nullptr;  // 10 planes FP64
  void* vis = nullptr;    // 12 planes (compute type)
  void* rt = nullptr;     // 5 planes (compute type)
  // metrics in the compute type: met itself (FP64), or (mixed) a rounded copy followed by
  // the 9 half-point metric planes of the sweeps
  void* met_r = nullptr;
  void* met_raw = nullptr;  // allocations behind met, met_r, vis, rt (see aligned_planes)
  void* met_r_raw = nullptr;
  void* vis_raw = nullptr;
  void* rt_raw = nullptr;
  size_t esize = 8;       // bytes of the compute type
  bool have_metrics = false;
  int64_t bytes = 0;
  // block-local viscous halo work: self-periodic copies and physical-face ghosts
  CopySeg* local_copy_dev = nullptr;
  int n_local_copy = 0, max_local_copy = 0;
  BcSeg* local_bc_dev = nullptr;
  int n_local_bc = 0, max_local_bc = 0;
  bool has_interface = false;
  int patched = 0;  // exchanges that connect part of one of its physical faces to a block
  int cfg[3] = {0, 0, 0};  // sweep tile shape per direction (set at creation)
  // small device scratch for reductions
  unsigned long long* red_dev = nullptr;
  int* flag_dev = nullptr;
  double* res_dev = nullptr;  // residual partial rows of up to kMaxBlocks blocks (allocated on first use)
  const double* dt_field = nullptr;  // caller's per-point time steps (local time stepping) or null
  hipEvent_t ev = nullptr;    // orders this block's stream before another block's
  Profiler prof;
};

namespace {

// faces that get ghost fills (and reflected viscous-flux ghosts)
bool is_physical(int kind) { return kind == CFD_BC_WALL || kind == CFD_BC_FARFIELD || kind == CFD_BC_FARFIELD_CHAR; }

Phys make_phys(const cfd_params& p) {
  Phys ph;
  ph.gamma = p.gamma;
  ph.gm1 = p.gamma - 1.0;
  ph.gm1inv = 1.0 / (p.gamma - 1.0);
  ph.inv2g = 1.0 / (2.0 * p.gamma);
  ph.visc_scale = p.mach / p.reynolds;
  ph.heat_scale = p.mach / (p.reynolds * p.prandtl * (p.gamma - 1.0));
  ph.suth = p.suth;
  ph.eps = p.weno_eps;
  ph.linear = p.weights == CFD_WENO_LINEAR;
  ph.scheme = p.scheme;
  return ph;
}

bool same_params(const cfd_params& a, const cfd_params& b) {
  bool same = a.gamma == b.gamma && a.mach == b.mach && a.reynolds == b.reynolds && a.prandtl == b.prandtl &&
              a.suth == b.suth && a.weno_eps == b.weno_eps && a.viscous == b.viscous && a.weights == b.weights &&
              a.scheme == b.scheme &&
              a.t_wall == b.t_wall;
  for (int v = 0; v < 5; ++v) same = same && a.qinf[v] == b.qinf[v];
  return same;
}

int npts(const Geom& g, int axis) { return axis == 0 ? g.ni : axis == 1 ? g.nj : g.nk; }
int64_t stride(const Geom& g, int axis) { return axis == 0 ? 1 : axis == 1 ? g.ld_i : g.ld_i * g.ld_j; }
int64_t at_h(const Geom& g, int i, int j, int k) {
  return ((int64_t)(k + kHalo) * g.ld_j + (j + kHalo)) * g.ld_i + (i + kHalo);
}

// boundary node index of face f along its axis, and the outward sign
void face_geom(const Geom& g, int f, int* axis, int* w, int* out) {
  *axis = f / 2;
  *out = (f % 2) ? +1 : -1;
  *w = (f % 2) ? npts(g, *axis) - 1 : 0;
}

// halo copy of face fa of block A (index ia) from face fb of block B (index ib):
// ghost layer m (1..3) beyond fa <- interior layer m-1 inside fb.
// tangential axes of a face on `axis`; the contiguous i axis comes first whenever it is
// tangential, so that neighbouring threads of the halo kernels touch neighbouring elements
void tangential(int axis, int* ta, int* tb) {
  *ta = axis == 0 ? 1 : 0;
  *tb = axis == 2 ? 1 : 2;
}

// Tangential index map of an interface (orient bits: 0 swap, 1 reverse a's t1, 2 reverse
// a's t2): a's tangential axis q (0: t1, 1: t2) runs along b's axis map_axis[q], reversed
// when map_rev[q].
struct FaceMap {
  int axis_a, axis_b;      // face-normal axes
  int ta[2], tb[2];        // tangential axes of both faces (increasing)
  int map_axis[2];         // b's axis that a's ta[q] runs along
  bool map_rev[2];
  int normal_sign;         // +1: a's normal index and b's run the same way through the face
};

FaceMap face_map(int fa, int fb, int orient) {
  FaceMap m;
  m.axis_a = fa / 2;
  m.axis_b = fb / 2;
  tangential(m.axis_a, &m.ta[0], &m.ta[1]);
  tangential(m.axis_b, &m.tb[0], &m.tb[1]);
  const bool swap = orient & 1;
  m.map_axis[0] = swap ? m.tb[1] : m.tb[0];
  m.map_axis[1] = swap ? m.tb[0] : m.tb[1];
  m.map_rev[0] = (orient >> 1) & 1;
  m.map_rev[1] = (orient >> 2) & 1;
  const int outa = (fa % 2) ? +1 : -1, outb = (fb % 2) ? +1 : -1;
  m.normal_sign = -outa * outb;  // ghost m of a = interior m-1 of b: a steps outward as b steps inward
  return m;
}

// determinant of the signed axis permutation taking a's index directions to b's
int face_map_det(const FaceMap& m) {
  int M[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // M[b axis][a axis]
  M[m.axis_b][m.axis_a] = m.normal_sign;
  for (int q = 0; q < 2; ++q) M[m.map_axis[q]][m.ta[q]] = m.map_rev[q] ? -1 : 1;
  return M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
         M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
}

// orient of the same interface seen from b
int inverse_orient(int orient) {
  const int r1 = (orient >> 1) & 1, r2 = (orient >> 2) & 1;
  return (orient & 1) ? (1 | (r2 << 1) | (r1 << 2)) : orient;
}

// A rectangle of a face: corner and extents along the face's tangential axes t1 < t2
struct FaceRect {
  int lo[2], n[2];
};
FaceRect whole_face(const Geom& g, int f) {
  int ta, tb;
  tangential(f / 2, &ta, &tb);
  return FaceRect{{0, 0}, {npts(g, ta), npts(g, tb)}};
}

// halo copy of the rectangle ra of face fa of block A (index ia) from face fb of block B
// (index ib) under the tangential map orient: ghost layer m (1..3) beyond fa <- interior
// layer m-1 inside fb, B's rectangle starting at blo (along B's t1, t2).  Planes plane0..
// of A receive planes src_plane0.. of B, negated if negate.
CopySeg make_copy_rect(const Geom& A, int ia, int fa, const FaceRect& ra, const Geom& B, int ib, int fb,
                       const int* blo, int plane0, int nplanes, int orient, int src_plane0, int negate) {
  int axis, wa, outa, wb, outb;
  face_geom(A, fa, &axis, &wa, &outa);
  int axis_b;
  face_geom(B, fb, &axis_b, &wb, &outb);
  const FaceMap m = face_map(fa, fb, orient);
  CopySeg s;
  std::memset(&s, 0, sizeof s);
  s.layer_fast = axis == 0;  // on i faces the three halo layers are the contiguous run
  s.dst = ia;
  s.src = ib;
  s.na = ra.n[0];
  s.nb = ra.n[1];
  s.plane0 = plane0;
  s.src_plane0 = src_plane0;
  s.negate = negate;
  s.nplanes = nplanes;
  int ida[3] = {0, 0, 0}, idb[3] = {0, 0, 0};
  ida[axis] = wa + outa;  // ghost layer 1
  idb[axis_b] = wb;       // interior layer 0
  for (int q = 0; q < 2; ++q) {
    ida[m.ta[q]] = ra.lo[q];
    const int lo = m.map_axis[q] == m.tb[0] ? blo[0] : blo[1];  // B's corner along that axis
    idb[m.map_axis[q]] = m.map_rev[q] ? lo + ra.n[q] - 1 : lo;
  }
  s.dst_off = at_h(A, ida[0], ida[1], ida[2]);
  s.src_off = at_h(B, idb[0], idb[1], idb[2]);
  s.dst_sa = stride(A, m.ta[0]);
  s.dst_sb = stride(A, m.ta[1]);
  s.dst_sl = outa * stride(A, axis);
  s.src_sa = (m.map_rev[0] ? -1 : 1) * stride(B, m.map_axis[0]);
  s.src_sb = (m.map_rev[1] ? -1 : 1) * stride(B, m.map_axis[1]);
  s.src_sl = -outb * stride(B, axis_b);
  return s;
}

// the whole face fa of A from the whole face fb of B
CopySeg make_copy(const Geom& A, int ia, int fa, const Geom& B, int ib, int fb, int plane0, int nplanes,
                  int orient = 0, int src_plane0 = -1, int negate = 0) {
  const int zero[2] = {0, 0};
  return make_copy_rect(A, ia, fa, whole_face(A, fa), B, ib, fb, zero, plane0, nplanes, orient,
                        src_plane0 < 0 ? plane0 : src_plane0, negate);
}

// wall / far-field treatment of the rectangle r of face f
BcSeg make_bc_rect(const Geom& G, int blk, int f, int kind, const FaceRect& r) {
  int axis, w, out;
  face_geom(G, f, &axis, &w, &out);
  int ta, tb;
  tangential(axis, &ta, &tb);
  BcSeg s;
  s.blk = blk;
  s.kind = kind;
  s.na = r.n[0];
  s.nb = r.n[1];
  int id[3] = {0, 0, 0};
  id[ta] = r.lo[0];
  id[tb] = r.lo[1];
  id[axis] = w;
  s.wall_off = at_h(G, id[0], id[1], id[2]);
  s.sa = stride(G, ta);
  s.sb = stride(G, tb);
  s.sout = out * stride(G, axis);
  s.axis = axis;
  return s;
}
BcSeg make_bc(const Geom& G, int blk, int f, int kind) { return make_bc_rect(G, blk, f, kind, whole_face(G, f)); }

// Allocate nplanes planes of esize-byte elements.  The base is shifted so that the first
// interior point of every row, element ((k+3)*ld_j + j+3)*ld_i + 3, starts a 128-byte cache
// line whenever ld_i*esize is a multiple of 128 (the layout callers are advised to use).
int aligned_planes(size_t plane, int nplanes, size_t esize, void** raw, void** base) {
  const size_t pad = (128 - 3 * esize) / esize;
  if (hipMalloc(raw, (nplanes * plane + pad + 64) * esize) != hipSuccess) return CFD_ERR_ALLOC;
  *base = static_cast<char*>(*raw) + pad * esize;
  if (hipMemset(*raw, 0, (nplanes * plane + pad + 64) * esize) != hipSuccess) return CFD_ERR_HIP;
  return CFD_OK;
}

template <typename T>
int upload(const std::vector<T>& v, T** dev) {
  *dev = nullptr;
  if (v.empty()) return CFD_OK;
  HIP_TRY(hipMalloc((void**)dev, v.size() * sizeof(T)), "hipMalloc(table)");
  HIP_TRY(hipMemcpy(*dev, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy(table)");
  return CFD_OK;
}

int validate_desc(const cfd_block_desc* d) {
  if (!d) return fail(CFD_ERR_ARG, "null descriptor");
  if (!is_real_size(d->ni) || !is_real_size(d->nj) || !is_real_size(d->nk))
    return fail(CFD_ERR_ARG, "ni, nj and nk must each be at least 7");
  if (d->ld_i < d->ni + 6 || d->ld_j < d->nj + 6) return fail(CFD_ERR_ARG, "pitches must satisfy ld_i >= ni+6, ld_j >= nj+6");
  // kernels address one plane with 32-bit byte offsets
  if (d->ld_i * d->ld_j * (int64_t)(d->nk + 6) >= ((int64_t)1 << 29))
    return fail(CFD_ERR_UNSUPPORTED, "a block plane must hold fewer than 2^29 points (split larger grids into blocks)");
  if (d->precision != CFD_FP64 && d->precision != CFD_MIXED) return fail(CFD_ERR_ARG, "unknown precision");
  const cfd_params& p = d->params;
  if (!(p.gamma > 1.0) || !(p.reynolds > 0.0) || !(p.prandtl > 0.0) || !(p.weno_eps > 0.0) || !(p.suth > 0.0))
    return fail(CFD_ERR_ARG, "gamma > 1, Re, Pr, Sutherland constant and WENO epsilon > 0 required");
  if (p.weights != CFD_WENO_JS && p.weights != CFD_WENO_LINEAR) return fail(CFD_ERR_ARG, "unknown WENO weights");
  if (p.scheme != CFD_AFWENO_MODIFIED && p.scheme != CFD_AFWENO_ORIGINAL) return fail(CFD_ERR_ARG, "unknown AFWENO scheme");
  if (p.visc_closure != CFD_VISC_REFLECT && p.visc_closure != CFD_VISC_ONE_SIDED)
    return fail(CFD_ERR_ARG, "unknown viscous closure");
  // Eq 15 is evaluated over a common denominator whose terms scale as weno_eps^4 (FP32)
  // and weno_eps^8 (FP64 product of the two sides' denominators) where the smoothness
  // indicators vanish; these floors keep them inside the normal range of the type
  if (p.weights == CFD_WENO_JS && d->precision == CFD_MIXED && p.weno_eps < 1e-8)
    return fail(CFD_ERR_ARG, "WENO epsilon below 1e-8 underflows the FP32 weights (mixed precision)");
  if (p.weights == CFD_WENO_JS && p.weno_eps < 1e-30)
    return fail(CFD_ERR_ARG, "WENO epsilon below 1e-30 underflows the FP64 weights");
  for (int f = 0; f < 6; ++f)
    if (d->bc[f] < CFD_BC_PERIODIC || d->bc[f] > CFD_BC_FARFIELD_CHAR) return fail(CFD_ERR_ARG, "unknown face kind");
  for (int ax = 0; ax < 3; ++ax)
    if ((d->bc[2 * ax] == CFD_BC_PERIODIC) != (d->bc[2 * ax + 1] == CFD_BC_PERIODIC))
      return fail(CFD_ERR_ARG, "periodic faces come in pairs on one axis");
  if (d->bc[2] == CFD_BC_WALL || d->bc[3] == CFD_BC_WALL || d->bc[0] == CFD_BC_WALL || d->bc[1] == CFD_BC_WALL ||
      d->bc[4] == CFD_BC_WALL || d->bc[5] == CFD_BC_WALL) {
    if (!(p.t_wall > 0.0)) return fail(CFD_ERR_ARG, "wall faces need t_wall > 0");
  }
  for (int f = 0; f < 6; ++f)
    if (d->bc[f] == CFD_BC_FARFIELD_CHAR) {
      const double* q = p.qinf;
      const double pinf = (p.gamma - 1.0) * (q[4] - 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0]);
      if (!(q[0] > 0.0) || !(pinf > 0.0)) return fail(CFD_ERR_ARG, "a characteristic far field needs qinf with positive density and pressure");
    }
  return CFD_OK;
}

template <typename T>
PtrTable single_table(void* p, int64_t plane) {
  PtrTable t;
  std::memset(&t, 0, sizeof t);
  t.p[0] = p;
  t.plane[0] = plane;
  return t;
}

// faces whose viscous derivatives take the one-sided closure (bit 2*axis + side)
int one_sided_mask(const cfd_block_desc& d) {
  if (d.params.visc_closure != CFD_VISC_ONE_SIDED) return 0;
  int m = 0;
  for (int f = 0; f < 6; ++f)
    if (is_physical(d.bc[f])) m |= 1 << f;
  return m;
}

// viscous fluxes of one block with block-local halos (periodic wraps, physical ghosts)
int run_visc(cfd_block* b, const double* Q) {
  ViscArgs va;
  std::memset(&va, 0, sizeof va);
  va.g = b->g;
  va.q = Q;
  va.met = b->met;
  va.met_r = b->met_r;
  va.vis = b->vis;
  va.ph = make_phys(b->d.params);
  va.one_sided = one_sided_mask(b->d);
  // the prepass writes the periodic images itself (they were the only local copies)
  for (int ax = 0; ax < 3; ++ax)
    if (b->d.bc[2 * ax] == CFD_BC_PERIODIC) va.periodic |= 1 << ax;
  ProfScope ps(&b->prof, "visc_prepass", b->stream);
  hipError_t e = b->d.precision == CFD_FP64 ? launch_visc<double>(va, b->stream) : launch_visc<float>(va, b->stream);
  ps.done();
  if (e != hipSuccess) return hip_fail(e, "visc_prepass launch");
  if (b->n_local_copy && !va.periodic) {
    PtrTable t = single_table<double>(b->vis, b->g.plane);
    ProfScope pc(&b->prof, "visc_halo", b->stream);
    e = b->d.precision == CFD_FP64 ? launch_copy<double>(b->local_copy_dev, b->n_local_copy, b->max_local_copy, t, b->stream)
                                   : launch_copy<float>(b->local_copy_dev, b->n_local_copy, b->max_local_copy, t, b->stream);
    pc.done();
    if (e != hipSuccess) return hip_fail(e, "visc halo copy");
  }
  if (b->n_local_bc) {
    PtrTable t = single_table<double>(b->vis, b->g.plane);
    e = b->d.precision == CFD_FP64 ? launch_visc_ghost<double>(b->local_bc_dev, b->n_local_bc, b->max_local_bc, t, b->stream)
                                   : launch_visc_ghost<float>(b->local_bc_dev, b->n_local_bc, b->max_local_bc, t, b->stream);
    if (e != hipSuccess) return hip_fail(e, "visc ghost fill");
  }
  return CFD_OK;
}

const char* kSweepNames[3] = {"sweep_xi", "sweep_eta", "sweep_zeta"};
const char* kSweepRkNames[3] = {"sweep_xi_rk", "sweep_eta_rk", "sweep_zeta_rk"};
const char* kProfNames[] = {"sweep_xi",    "sweep_eta",    "sweep_zeta",   "sweep_xi_rk", "sweep_eta_rk",
                            "sweep_zeta_rk", "visc_prepass", "visc_halo", "halo_q",      "halo_visc"};

// run the direction sweeps selected by mask; the last one writes R or the RK stage
int run_sweeps(cfd_block* b, const double* Q, unsigned mask, int out_kind, double* out, const double* qn,
               const double* dt_dev, double dt, double ca, double cb, double cc) {
  const bool inv = (mask & CFD_TERM_INV) != 0;
  const bool vis = (mask & CFD_TERM_VIS) != 0 && b->d.params.viscous;
  int dirs[3], nd = 0;
  for (int n = 0; n < 3; ++n)
    if (mask & (1u << kSweepOrder[n])) dirs[nd++] = kSweepOrder[n];
  SweepArgs a;
  std::memset(&a, 0, sizeof a);
  a.b.g = b->g;
  a.b.q = Q;
  a.b.met = b->met;
  a.b.met_r = b->esize == sizeof(double) ? nullptr : static_cast<const float*>(b->met_r);
  a.b.vis = b->vis;
  a.b.qn = qn;
  a.b.dt_field = b->dt_field;
  a.b.one_sided = one_sided_mask(b->d);
  a.c.ph = make_phys(b->d.params);
  a.c.do_inv = inv;
  a.c.do_vis = vis;
  a.c.dt_dev = dt_dev;
  a.c.dt = dt;
  a.c.ca = ca;
  a.c.cb = cb;
  a.c.cc = cc;
  if (nd == 0 || (!inv && !vis)) {
    // nothing to evaluate: R = 0 or Qout = ca Qn + cb Q, via a zero-term sweep along xi
    a.c.do_inv = 0;
    a.c.do_vis = 0;
    a.c.has_prev = 0;
    a.c.out_kind = out_kind;
    a.b.out = out;
    ProfScope ps(&b->prof, kSweepNames[0], b->stream);
    hipError_t e = b->d.precision == CFD_FP64 ? launch_sweep<double>(0, a, b->stream, b->cfg[0])
                                              : launch_sweep<float>(0, a, b->stream, b->cfg[0]);
    ps.done();
    return e == hipSuccess ? CFD_OK : hip_fail(e, "sweep launch");
  }
  for (int n = 0; n < nd; ++n) {
    const bool last = n == nd - 1;
    a.c.has_prev = n > 0;
    a.b.rt_in = b->rt;
    a.b.rt_out = b->rt;
    a.c.out_kind = last ? out_kind : kOutPartial;
    a.b.out = last ? out : nullptr;
    const char* name = (last && out_kind == kOutRK) ? kSweepRkNames[dirs[n]] : kSweepNames[dirs[n]];
    ProfScope ps(&b->prof, name, b->stream);
    hipError_t e = b->d.precision == CFD_FP64 ? launch_sweep<double>(dirs[n], a, b->stream, b->cfg[dirs[n]])
                                              : launch_sweep<float>(dirs[n], a, b->stream, b->cfg[dirs[n]]);
    ps.done();
    if (e != hipSuccess) return hip_fail(e, "sweep launch");
  }
  return CFD_OK;
}

const double kRK[3][3] = {{1.0, 0.0, 1.0}, {0.75, 0.25, 0.25}, {1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0}};

int check_rk_args(cfd_block* b, int stage, const double* Qn, const double* Qcur, double* Qout) {
  if (!b) return fail(CFD_ERR_ARG, "null block");
  if (stage < 0 || stage > 2) return fail(CFD_ERR_ARG, "stage must be 0, 1 or 2");
  if (!Qn || !Qcur || !Qout) return fail(CFD_ERR_ARG, "null state pointer");
  if (Qout == Qcur) return fail(CFD_ERR_ARG, "Qout must not alias Qcur");
  if (Qout == Qn && stage != 2) return fail(CFD_ERR_ARG, "Qout may alias Qn only at stage 2");
  if (stage == 0 && Qcur != Qn) return fail(CFD_ERR_ARG, "at stage 0 Qcur must be Qn");
  if (!b->have_metrics) return fail(CFD_ERR_STATE, "cfd_metrics has not been run on this block");
  return CFD_OK;
}

// Residual scratch of cfd_residual_noalloc: kResGroups partial rows of up to kMaxBlocks
// blocks and the 10 results, in a file-scope device array (1.31 MB per device, held until
// the process ends).  Host code never uses the array's name as an address: the device
// address of each GPU's copy comes from hipGetSymbolAddress, taken once per device with
// that device current.
constexpr size_t kResScratch = (size_t)kMaxBlocks * kResGroups * 10 + 10;
static __device__ __align__(256) double scratch[kResScratch];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

int residual_scratch(int device, double** ptr) {
  if (device < 0 || device >= kMaxDevices) return fail(CFD_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur), "hipGetDevice");
    if (cur != device) HIP_TRY(hipSetDevice(device), "hipSetDevice");
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(residual scratch)");
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  *ptr = g_scratch_ptr[device];
  return CFD_OK;
}

}  // namespace

extern "C" {

const char* cfd_last_error(void) { return g_err.c_str(); }

int cfd_block_create(const cfd_block_desc* d, void* hip_stream, cfd_block** out) {
  if (!out) return fail(CFD_ERR_ARG, "null output handle");
  *out = nullptr;
  int rc = validate_desc(d);
  if (rc) return rc;
  cfd_block* b = new cfd_block();
  b->d = *d;
  b->g.ni = d->ni;
  b->g.nj = d->nj;
  b->g.nk = d->nk;
  b->g.ld_i = d->ld_i;
  b->g.ld_j = d->ld_j;
  b->g.plane = d->ld_i * d->ld_j * (int64_t)(d->nk + 6);
  b->stream = (hipStream_t)hip_stream;
  b->esize = d->precision == CFD_FP64 ? 8 : 4;
  for (int dir = 0; dir < 3; ++dir) b->cfg[dir] = kDefaultTiles[d->precision == CFD_FP64 ? 0 : 1][dir];
  (void)hipGetDevice(&b->device);
  const size_t plane = (size_t)b->g.plane;
  auto cleanup = [&](int code, const std::string& msg) {
    cfd_block_destroy(b);
    return fail(code, msg);
  };
  void* mbase = nullptr;
  if (aligned_planes(plane, 10, sizeof(double), &b->met_raw, &mbase)) return cleanup(CFD_ERR_ALLOC, "metrics allocation");
  b->met = static_cast<double*>(mbase);
  b->met_r = b->met;
  // mixed precision: the metric planes rounded to FP32 and the 9 half-point metric planes
  if (b->esize != sizeof(double) && aligned_planes(plane, 10 + 9, b->esize, &b->met_r_raw, &b->met_r))
    return cleanup(CFD_ERR_ALLOC, "metrics allocation");
  if (aligned_planes(plane, 12, b->esize, &b->vis_raw, &b->vis)) return cleanup(CFD_ERR_ALLOC, "viscous scratch allocation");
  if (aligned_planes(plane, 5, b->esize, &b->rt_raw, &b->rt)) return cleanup(CFD_ERR_ALLOC, "partial-sum allocation");
  if (hipMalloc((void**)&b->red_dev, sizeof(unsigned long long)) != hipSuccess ||
      hipMalloc((void**)&b->flag_dev, sizeof(int)) != hipSuccess)
    return cleanup(CFD_ERR_ALLOC, "reduction scratch");
  if (hipEventCreateWithFlags(&b->ev, hipEventDisableTiming) != hipSuccess) return cleanup(CFD_ERR_HIP, "block event");
  b->bytes = (int64_t)plane * (10 * 8 + (b->esize == sizeof(double) ? 17 : 36) * (int64_t)b->esize);
  // block-local viscous halo work
  std::vector<CopySeg> cs;
  std::vector<BcSeg> bs;
  for (int ax = 0; ax < 3; ++ax) {
    if (d->bc[2 * ax] == CFD_BC_PERIODIC) {
      cs.push_back(make_copy(b->g, 0, 2 * ax, b->g, 0, 2 * ax + 1, 4 * ax, 4));
      cs.push_back(make_copy(b->g, 0, 2 * ax + 1, b->g, 0, 2 * ax, 4 * ax, 4));
    }
  }
  for (int f = 0; f < 6; ++f) {
    if (is_physical(d->bc[f])) bs.push_back(make_bc(b->g, 0, f, d->bc[f]));
    if (d->bc[f] == CFD_BC_INTERFACE) b->has_interface = true;
  }
  for (auto& s : cs) b->max_local_copy = std::max(b->max_local_copy, s.na * s.nb * kHalo * s.nplanes);
  for (auto& s : bs) b->max_local_bc = std::max(b->max_local_bc, s.na * s.nb);
  if (upload(cs, &b->local_copy_dev) || upload(bs, &b->local_bc_dev)) return cleanup(CFD_ERR_HIP, "halo tables");
  b->n_local_copy = (int)cs.size();
  b->n_local_bc = (int)bs.size();
  *out = b;
  return CFD_OK;
}

int cfd_block_destroy(cfd_block* b) {
  if (!b) return CFD_OK;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  else (void)hipDeviceSynchronize();
  b->prof.drain();
  (void)hipFree(b->met_raw);
  (void)hipFree(b->met_r_raw);
  (void)hipFree(b->vis_raw);
  (void)hipFree(b->rt_raw);
  (void)hipFree(b->red_dev);
  (void)hipFree(b->flag_dev);
  (void)hipFree(b->res_dev);
  if (b->ev) (void)hipEventDestroy(b->ev);
  (void)hipFree(b->local_copy_dev);
  (void)hipFree(b->local_bc_dev);
  delete b;
  return CFD_OK;
}

int cfd_block_set_stream(cfd_block* b, void* hip_stream) {
  if (!b) return fail(CFD_ERR_ARG, "null block");
  b->stream = (hipStream_t)hip_stream;
  return CFD_OK;
}

int cfd_block_bytes(const cfd_block* b, int64_t* bytes) {
  if (!b || !bytes) return fail(CFD_ERR_ARG, "null argument");
  *bytes = b->bytes;
  return CFD_OK;
}

int cfd_metrics(cfd_block* b, const double* xyz, int64_t cld_i, int64_t cld_j) {
  if (!b || !xyz) return fail(CFD_ERR_ARG, "null argument");
  if (cld_i < b->g.ni + 12 || cld_j < b->g.nj + 12) return fail(CFD_ERR_ARG, "coordinate pitches too small (halo 6)");
  MetricArgs a;
  a.g = b->g;
  a.xyz = xyz;
  a.cld_i = cld_i;
  a.cld_j = cld_j;
  a.cplane = cld_i * cld_j * (int64_t)(b->g.nk + 12);
  const size_t tplane = (size_t)(b->g.ni + 12) * (b->g.nj + 12) * (b->g.nk + 12);
  a.met = b->met;
  a.bad = b->flag_dev;
  HIP_TRY(hipMalloc((void**)&a.dcoord, 9 * tplane * sizeof(double)), "hipMalloc(metric scratch)");
  int rc = CFD_OK;
  hipError_t e = hipMemsetAsync(b->flag_dev, 0, sizeof(int), b->stream);
  if (e == hipSuccess) e = launch_metrics(a, b->stream);
  // the FP32 consumers of a mixed block read the metrics rounded once here, and its sweeps
  // the half-point metrics interpolated once in FP64 and rounded
  if (e == hipSuccess && b->met_r != b->met)
    e = launch_round(b->met, static_cast<float*>(b->met_r), (int64_t)10 * b->g.plane, b->stream);
  if (e == hipSuccess && b->met_r != b->met)
    e = launch_half_metrics(b->g, b->met, static_cast<float*>(b->met_r) + 10 * b->g.plane, b->stream);
  int bad = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, b->flag_dev, sizeof(int), hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  (void)hipFree(a.dcoord);
  if (e != hipSuccess) return hip_fail(e, "cfd_metrics");
  if (bad) rc = fail(CFD_ERR_JACOBIAN, "non-positive 1/J: folded or left-handed grid");
  b->have_metrics = rc == CFD_OK;
  return rc;
}

int cfd_metrics_ptr(const cfd_block* b, const double** met) {
  if (!b || !met) return fail(CFD_ERR_ARG, "null argument");
  *met = b->met;
  return CFD_OK;
}

int cfd_viscous_fluxes(cfd_block* b, const double* Q) {
  if (!b || !Q) return fail(CFD_ERR_ARG, "null argument");
  if (!b->have_metrics) return fail(CFD_ERR_STATE, "cfd_metrics has not been run on this block");
  if (!b->d.params.viscous) return CFD_OK;
  return run_visc(b, Q);
}

int cfd_rhs_sweeps(cfd_block* b, const double* Q, double* R, unsigned mask) {
  if (!b || !Q || !R) return fail(CFD_ERR_ARG, "null argument");
  if (Q == R) return fail(CFD_ERR_ARG, "R must not alias Q");
  if (!b->have_metrics) return fail(CFD_ERR_STATE, "cfd_metrics has not been run on this block");
  return run_sweeps(b, Q, mask, kOutRhs, R, nullptr, nullptr, 0.0, 0.0, 0.0, 0.0);
}

int cfd_rhs(cfd_block* b, const double* Q, double* R, unsigned mask) {
  if (!b || !Q || !R) return fail(CFD_ERR_ARG, "null argument");
  if (b->has_interface || b->patched)
    return fail(CFD_ERR_STATE, "block has interface faces: use cfd_viscous_fluxes, cfd_halo_exchange(VISC), cfd_rhs_sweeps");
  if ((mask & CFD_TERM_VIS) && b->d.params.viscous) {
    int rc = cfd_viscous_fluxes(b, Q);
    if (rc) return rc;
  }
  return cfd_rhs_sweeps(b, Q, R, mask);
}

static int rk_sweeps(cfd_block* b, int stage, const double* dt_dev, double dt, const double* Qn, const double* Qcur,
                     double* Qout) {
  int rc = check_rk_args(b, stage, Qn, Qcur, Qout);
  if (rc) return rc;
  return run_sweeps(b, Qcur, CFD_ALL, kOutRK, Qout, Qn, dt_dev, dt, kRK[stage][0], kRK[stage][1], kRK[stage][2]);
}

int cfd_rk_sweeps(cfd_block* b, int stage, double dt, const double* Qn, const double* Qcur, double* Qout) {
  if (!std::isfinite(dt)) return fail(CFD_ERR_ARG, "dt must be finite");
  return rk_sweeps(b, stage, nullptr, dt, Qn, Qcur, Qout);
}

int cfd_rk_stage(cfd_block* b, int stage, double dt, const double* Qn, const double* Qcur, double* Qout) {
  int rc = check_rk_args(b, stage, Qn, Qcur, Qout);
  if (rc) return rc;
  if (!std::isfinite(dt)) return fail(CFD_ERR_ARG, "dt must be finite");
  if (b->has_interface || b->patched)
    return fail(CFD_ERR_STATE, "block has interface faces: use cfd_viscous_fluxes, cfd_halo_exchange(VISC), cfd_rk_sweeps");
  if (b->d.params.viscous) {
    rc = run_visc(b, Qcur);
    if (rc) return rc;
  }
  return rk_sweeps(b, stage, nullptr, dt, Qn, Qcur, Qout);
}

int cfd_rk_stage_dev(cfd_block* b, int stage, const double* dt_dev, const double* Qn, const double* Qcur,
                     double* Qout) {
  int rc = check_rk_args(b, stage, Qn, Qcur, Qout);
  if (rc) return rc;
  if (!dt_dev) return fail(CFD_ERR_ARG, "null dt_dev");
  if (b->has_interface || b->patched)
    return fail(CFD_ERR_STATE, "block has interface faces: use cfd_viscous_fluxes, cfd_halo_exchange(VISC), cfd_rk_sweeps");
  if (b->d.params.viscous) {
    rc = run_visc(b, Qcur);
    if (rc) return rc;
  }
  return rk_sweeps(b, stage, dt_dev, 0.0, Qn, Qcur, Qout);
}

int cfd_sync(cfd_block* b) {
  if (!b) return fail(CFD_ERR_ARG, "null block");
  HIP_TRY(hipStreamSynchronize(b->stream), "stream synchronize");
  HIP_TRY(hipGetLastError(), "pending device error");
  return CFD_OK;
}

int cfd_check_finite(cfd_block* b, const double* Q, int* ok) {
  if (!b || !Q || !ok) return fail(CFD_ERR_ARG, "null argument");
  int flag = 0;
  HIP_TRY(hipMemsetAsync(b->flag_dev, 0, sizeof(int), b->stream), "memset");
  HIP_TRY(launch_finite(b->g, Q, b->flag_dev, b->stream), "finite check launch");
  HIP_TRY(hipMemcpyAsync(&flag, b->flag_dev, sizeof(int), hipMemcpyDeviceToHost, b->stream), "copy flag");
  HIP_TRY(hipStreamSynchronize(b->stream), "stream synchronize");
  *ok = flag ? 0 : 1;
  return flag ? fail(CFD_ERR_NONFINITE, "non-finite value in state") : CFD_OK;
}

int cfd_dt_cfl(cfd_block* const* blocks, int nb, const double* const* Q, double cfl, double* dt_out) {
  if (!blocks || nb <= 0 || !Q || !dt_out) return fail(CFD_ERR_ARG, "null argument");
  if (!(cfl > 0.0)) return fail(CFD_ERR_ARG, "cfl must be positive");
  cfd_block* b0 = blocks[0];
  if (!b0) return fail(CFD_ERR_ARG, "null block");
  for (int n = 0; n < nb; ++n) {
    if (!blocks[n] || !Q[n]) return fail(CFD_ERR_ARG, "null block or state");
    if (!blocks[n]->have_metrics) return fail(CFD_ERR_STATE, "cfd_metrics has not been run on a block");
  }
  // the reduction runs on the first block's stream: finish earlier work of the others
  for (int n = 1; n < nb; ++n)
    if (blocks[n]->stream != b0->stream) HIP_TRY(hipStreamSynchronize(blocks[n]->stream), "stream synchronize");
  HIP_TRY(hipMemsetAsync(b0->red_dev, 0, sizeof(unsigned long long), b0->stream), "memset");
  for (int n = 0; n < nb; ++n) {
    cfd_block* b = blocks[n];
    HIP_TRY(launch_dt_max(b->g, Q[n], b->met, b->d.params.gamma, b0->red_dev, b0->stream), "dt launch");
  }
  unsigned long long bits = 0;
  HIP_TRY(hipMemcpyAsync(&bits, b0->red_dev, sizeof bits, hipMemcpyDeviceToHost, b0->stream), "copy dt");
  HIP_TRY(hipStreamSynchronize(b0->stream), "stream synchronize");
  double smax;
  std::memcpy(&smax, &bits, sizeof smax);
  if (!(smax > 0.0) || !std::isfinite(smax)) return fail(CFD_ERR_NONFINITE, "spectral radius is not positive and finite");
  *dt_out = cfl / smax;
  return CFD_OK;
}

// Work of every block up to now, ordered before later work on blocks[0]'s stream.
static int order_on_first(cfd_block* const* blocks, int nb) {
  cfd_block* b0 = blocks[0];
  for (int n = 1; n < nb; ++n) {
    if (blocks[n]->stream == b0->stream) continue;
    HIP_TRY(hipEventRecord(blocks[n]->ev, blocks[n]->stream), "event record");
    HIP_TRY(hipStreamWaitEvent(b0->stream, blocks[n]->ev, 0), "stream wait");
  }
  return CFD_OK;
}

int cfd_dt_cfl_dev(cfd_block* const* blocks, int nb, const double* const* Q, double cfl, double* dt_dev) {
  if (!blocks || nb <= 0 || !Q || !dt_dev) return fail(CFD_ERR_ARG, "null argument");
  if (!(cfl > 0.0)) return fail(CFD_ERR_ARG, "cfl must be positive");
  for (int n = 0; n < nb; ++n) {
    if (!blocks[n] || !Q[n]) return fail(CFD_ERR_ARG, "null block or state");
    if (!blocks[n]->have_metrics) return fail(CFD_ERR_STATE, "cfd_metrics has not been run on a block");
  }
  cfd_block* b0 = blocks[0];
  int rc = order_on_first(blocks, nb);
  if (rc != CFD_OK) return rc;
  HIP_TRY(launch_dt_reset(b0->red_dev, b0->stream), "dt reset launch");
  for (int n = 0; n < nb; ++n) {
    cfd_block* b = blocks[n];
    HIP_TRY(launch_dt_max(b->g, Q[n], b->met, b->d.params.gamma, b0->red_dev, b0->stream), "dt launch");
  }
  HIP_TRY(launch_dt_finish(b0->red_dev, cfl, dt_dev, b0->stream), "dt finish launch");
  return CFD_OK;
}

int cfd_dt_local(cfd_block* const* blocks, int nb, const double* const* Q, double cfl, double* const* dt_field) {
  if (!blocks || nb <= 0 || !Q || !dt_field) return fail(CFD_ERR_ARG, "null argument");
  if (!(cfl > 0.0)) return fail(CFD_ERR_ARG, "cfl must be positive");
  for (int n = 0; n < nb; ++n) {
    if (!blocks[n] || !Q[n] || !dt_field[n]) return fail(CFD_ERR_ARG, "null block, state or step field");
    if (!blocks[n]->have_metrics) return fail(CFD_ERR_STATE, "cfd_metrics has not been run on a block");
  }
  for (int n = 0; n < nb; ++n) {
    cfd_block* b = blocks[n];
    HIP_TRY(launch_dt_local(b->g, Q[n], b->met, b->d.params.gamma, cfl, dt_field[n], b->stream), "local dt launch");
  }
  return CFD_OK;
}

int cfd_block_set_local_dt(cfd_block* b, const double* dt_field) {
  if (!b) return fail(CFD_ERR_ARG, "null block");
  b->dt_field = dt_field;
  return CFD_OK;
}

int cfd_residual(cfd_block* const* blocks, int nb, const double* const* A, const double* const* Bm, double scale,
                 double* out) {
  if (!blocks || nb <= 0 || nb > kMaxBlocks || !A || !out) return fail(CFD_ERR_ARG, "need 1..64 blocks, A and out");
  int64_t npts = 0;
  for (int n = 0; n < nb; ++n) {
    if (!blocks[n] || !A[n]) return fail(CFD_ERR_ARG, "null block or array");
    npts += (int64_t)blocks[n]->g.ni * blocks[n]->g.nj * blocks[n]->g.nk;
  }
  if (!std::isfinite(scale)) return fail(CFD_ERR_ARG, "scale must be finite");
  cfd_block* b0 = blocks[0];
  if (!b0->res_dev) {
    HIP_TRY(hipStreamSynchronize(b0->stream), "stream synchronize");
    if (hipMalloc((void**)&b0->res_dev, ((size_t)kMaxBlocks * kResGroups * 10 + 10) * sizeof(double)) != hipSuccess) {
      b0->res_dev = nullptr;
      return fail(CFD_ERR_ALLOC, "residual scratch");
    }
  }
  int rc = order_on_first(blocks, nb);
  if (rc != CFD_OK) return rc;
  for (int n = 0; n < nb; ++n)
    HIP_TRY(launch_res_partial(blocks[n]->g, A[n], Bm ? Bm[n] : nullptr, scale, b0->res_dev + (int64_t)n * kResGroups * 10,
                               b0->stream),
            "residual launch");
  double* res_out = b0->res_dev + (int64_t)kMaxBlocks * kResGroups * 10;
  HIP_TRY(launch_res_final(b0->res_dev, nb * kResGroups, 1.0 / (double)npts, res_out, b0->stream), "residual launch");
  HIP_TRY(hipMemcpyAsync(out, res_out, 10 * sizeof(double), hipMemcpyDeviceToHost, b0->stream), "copy residual");
  HIP_TRY(hipStreamSynchronize(b0->stream), "stream synchronize");
  for (int v = 0; v < 10; ++v)
    if (!std::isfinite(out[v])) return fail(CFD_ERR_NONFINITE, "non-finite residual");
  return CFD_OK;
}

int cfd_residual_noalloc(cfd_block* const* blocks, int nb, const double* const* A, const double* const* Bm,
                         double scale, double* out) {
  if (!blocks || nb <= 0 || nb > kMaxBlocks || !A || !out) return fail(CFD_ERR_ARG, "need 1..64 blocks, A and out");
  int64_t npts = 0;
  for (int n = 0; n < nb; ++n) {
    if (!blocks[n] || !A[n]) return fail(CFD_ERR_ARG, "null block or array");
    npts += (int64_t)blocks[n]->g.ni * blocks[n]->g.nj * blocks[n]->g.nk;
  }
  if (!std::isfinite(scale)) return fail(CFD_ERR_ARG, "scale must be finite");
  cfd_block* b0 = blocks[0];
  double* part = nullptr;
  int rc = residual_scratch(b0->device, &part);
  if (rc != CFD_OK) return rc;
  rc = order_on_first(blocks, nb);
  if (rc != CFD_OK) return rc;
  // every partial row of the nb blocks is written before the final reduction reads it, so
  // the scratch needs no clearing
  for (int n = 0; n < nb; ++n)
    HIP_TRY(launch_res_partial(blocks[n]->g, A[n], Bm ? Bm[n] : nullptr, scale, part + (int64_t)n * kResGroups * 10,
                               b0->stream),
            "residual launch");
  double* res_out = part + (int64_t)kMaxBlocks * kResGroups * 10;
  HIP_TRY(launch_res_final(part, nb * kResGroups, 1.0 / (double)npts, res_out, b0->stream), "residual launch");
  HIP_TRY(hipMemcpyAsync(out, res_out, 10 * sizeof(double), hipMemcpyDeviceToHost, b0->stream), "copy residual");
  HIP_TRY(hipStreamSynchronize(b0->stream), "stream synchronize");
  for (int v = 0; v < 10; ++v)
    if (!std::isfinite(out[v])) return fail(CFD_ERR_NONFINITE, "non-finite residual");
  return CFD_OK;
}

int cfd_profile_enable(cfd_block* b, int enable) {
  if (!b) return fail(CFD_ERR_ARG, "null block");
  b->prof.on = enable != 0;
  return CFD_OK;
}

int cfd_profile_read(cfd_block* b, const char** names, int64_t* launches, double* ms, int cap, int* n) {
  if (!b || !n) return fail(CFD_ERR_ARG, "null argument");
  b->prof.drain();
  int k = 0;
  for (const auto& name : b->prof.order) {
    if (k < cap) {
      auto& v = b->prof.acc[name];
      // names are static strings owned by the library
      const char* stat = "other";
      for (const char* known : kProfNames)
        if (name == known) stat = known;
      if (names) names[k] = stat;
      if (launches) launches[k] = v.first;
      if (ms) ms[k] = v.second;
    }
    ++k;
  }
  *n = k;
  return CFD_OK;
}

int cfd_profile_reset(cfd_block* b) {
  if (!b) return fail(CFD_ERR_ARG, "null block");
  b->prof.drain();
  b->prof.acc.clear();
  b->prof.order.clear();
  return CFD_OK;
}

}  // extern "C"

// =====================================================================================
// exchange plans
// =====================================================================================
struct cfd_exchange {
  std::vector<cfd_block*> blocks;
  CopySeg* q_dev = nullptr;    // Q copies (interfaces + periodic wraps)
  int nq = 0, maxq = 0;
  CopySeg* v_dev = nullptr;    // viscous copies (interfaces only)
  int nv = 0, maxv = 0;
  BcSeg* bc_dev = nullptr;     // wall / far-field faces
  int nbc = 0, maxbc = 0;
  int precision = CFD_FP64;
  std::vector<CopySeg> qs_host, vs_host;  // host copies of the segment tables
  std::vector<BcSeg> bc_host;
  std::vector<cfd_block*> patched;  // blocks with a partly connected physical face
};


// =====================================================================================
// batched multi-block form
// =====================================================================================
struct cfd_batch {
  std::vector<cfd_block*> blocks;
  cfd_exchange* x = nullptr;
  hipStream_t user = nullptr;    // caller's stream (may be the legacy default stream)
  hipStream_t stream = nullptr;  // the batch's own stream: graphs are captured and replayed here
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  int precision = CFD_FP64;
  bool viscous = true;
  bool one_sided = false;  // some block has faces with the one-sided viscous closure
  // work lists
  TileList visc_tl{};
  TileList sweep_tl[3]{};
  int cfg[3] = {0, 0, 0};       // tile configuration per direction
  int persist[3] = {0, 0, 0};   // persistent schedule per direction
  bool tuned = false;
  float tune_ms[3][kTileCfgs][2];  // autotuner timings (ms per launch, -1: not measured)
  int persist_wgs = 2048;       // workgroups of a persistent launch
  // combined viscous halo work of all blocks: self-periodic + interface copies, ghosts
  CopySeg* vcopy_dev = nullptr;
  int nvcopy = 0, maxvcopy = 0;
  BcSeg* vbc_dev = nullptr;
  int nvbc = 0, maxvbc = 0;
  // argument tables of the captured pointer set: 3 stages x (visc + 3 sweeps)
  ViscArgs* visc_args_dev = nullptr;      // [3][nb]
  SweepBlock* sweep_args_dev = nullptr;   // [3][3][nb]
  SweepCommon sweep_common[3][3]{};       // [stage][direction], passed by value
  std::vector<const void*> key;         // pointers the graph was captured for
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

int batch_destroy(cfd_batch* bt) {
  if (!bt) return CFD_OK;
  if (bt->stream) (void)hipStreamSynchronize(bt->stream);
  if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
  if (bt->ev_in) (void)hipEventDestroy(bt->ev_in);
  if (bt->ev_out) (void)hipEventDestroy(bt->ev_out);
  if (bt->stream) (void)hipStreamDestroy(bt->stream);
  if (bt->graph) (void)hipGraphDestroy(bt->graph);
  (void)hipFree(bt->vcopy_dev);
  (void)hipFree(bt->vbc_dev);
  (void)hipFree(bt->visc_args_dev);
  (void)hipFree(bt->sweep_args_dev);
  delete bt;
  return CFD_OK;
}

void fill_tiles(cfd_batch* bt) {
  const int nb = (int)bt->blocks.size();
  bt->visc_tl.nblk = nb;
  bt->visc_tl.prefix[0] = 0;
  for (int b = 0; b < nb; ++b) {
    int kc, t;
    visc_tiling(bt->blocks[b]->g, kViscMinTilesBatch, &kc, &t);
    bt->visc_tl.prefix[b + 1] = bt->visc_tl.prefix[b] + t;
  }
  for (int d = 0; d < 3; ++d) {
    TileList& tl = bt->sweep_tl[d];
    tl.nblk = nb;
    tl.prefix[0] = 0;
    for (int b = 0; b < nb; ++b) {
      const Geom& g = bt->blocks[b]->g;
      int tc1, td, tlen;
      sweep_tiling(d, bt->cfg[d], g, &tc1, &td, &tlen);
      const int n2 = d == 2 ? g.nj : g.nk;
      tl.prefix[b + 1] = tl.prefix[b] + tc1 * td * n2;
    }
  }
}

int batch_create(cfd_block* const* blocks, int nb, cfd_exchange* x, void* hip_stream, cfd_batch** out) {
  if (!out) return fail(CFD_ERR_ARG, "null output handle");
  *out = nullptr;
  if (!blocks || nb <= 0 || nb > kMaxBlocks || !x) return fail(CFD_ERR_ARG, "need 1..64 blocks and an exchange plan");
  if ((int)x->blocks.size() != nb) return fail(CFD_ERR_ARG, "exchange plan was made for a different block list");
  for (int b = 0; b < nb; ++b) {
    if (!blocks[b] || blocks[b] != x->blocks[b]) return fail(CFD_ERR_ARG, "exchange plan was made for a different block list");
    if (!blocks[b]->have_metrics) return fail(CFD_ERR_STATE, "cfd_metrics has not been run on every block");
    if (blocks[b]->d.precision != blocks[0]->d.precision) return fail(CFD_ERR_ARG, "blocks of a batch share one precision");
    if (!same_params(blocks[b]->d.params, blocks[0]->d.params))
      return fail(CFD_ERR_ARG, "blocks of a batch share one set of physical parameters");
  }
  cfd_batch* bt = new cfd_batch();
  bt->blocks.assign(blocks, blocks + nb);
  bt->x = x;
  bt->user = (hipStream_t)hip_stream;
  // the legacy default stream cannot be captured: work on an own stream (default
  // priority) ordered after / before the caller's stream with events
  if (hipStreamCreateWithFlags(&bt->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&bt->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&bt->ev_out, hipEventDisableTiming) != hipSuccess) {
    batch_destroy(bt);
    return fail(CFD_ERR_HIP, "batch stream and events");
  }
  bt->precision = blocks[0]->d.precision;
  bt->viscous = blocks[0]->d.params.viscous != 0;
  for (int b = 0; b < nb; ++b) bt->one_sided = bt->one_sided || one_sided_mask(blocks[b]->d) != 0;
  for (int d = 0; d < 3; ++d) {
    bt->cfg[d] = kDefaultTiles[bt->precision == CFD_FP64 ? 0 : 1][d];
    for (int c = 0; c < kTileCfgs; ++c) bt->tune_ms[d][c][0] = bt->tune_ms[d][c][1] = -1.f;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, blocks[0]->device) == hipSuccess) bt->persist_wgs = prop.multiProcessorCount * 8;
  // viscous halo work of the whole batch
  std::vector<CopySeg> vc = x->vs_host;
  std::vector<BcSeg> vb;
  for (int b = 0; b < nb; ++b) {
    const cfd_block* B = blocks[b];
    for (int ax = 0; ax < 3; ++ax)
      if (B->d.bc[2 * ax] == CFD_BC_PERIODIC) {
        vc.push_back(make_copy(B->g, b, 2 * ax, B->g, b, 2 * ax + 1, 4 * ax, 4));
        vc.push_back(make_copy(B->g, b, 2 * ax + 1, B->g, b, 2 * ax, 4 * ax, 4));
      }
  }
  // wall / far-field rectangles of the exchange (the parts of physical faces no patch
  // covers): the viscous ghosts run after the copies and must not overwrite them
  vb = x->bc_host;
  for (auto& c : vc) bt->maxvcopy = std::max(bt->maxvcopy, c.na * c.nb * kHalo * c.nplanes);
  for (auto& c : vb) bt->maxvbc = std::max(bt->maxvbc, c.na * c.nb);
  if (upload(vc, &bt->vcopy_dev) || upload(vb, &bt->vbc_dev)) {
    batch_destroy(bt);
    return fail(CFD_ERR_HIP, "batch halo tables");
  }
  bt->nvcopy = (int)vc.size();
  bt->nvbc = (int)vb.size();
  if (hipMalloc((void**)&bt->visc_args_dev, 3 * nb * sizeof(ViscArgs)) != hipSuccess ||
      hipMalloc((void**)&bt->sweep_args_dev, 9 * nb * sizeof(SweepBlock)) != hipSuccess) {
    batch_destroy(bt);
    return fail(CFD_ERR_ALLOC, "batch argument tables");
  }
  fill_tiles(bt);
  *out = bt;
  return CFD_OK;
}

// argument tables for stage s reading Qcur[b] and writing Qout[b]: per-block parts in
// va / sa, the parts shared by every block in bt->sweep_common
void build_args(cfd_batch* bt, double* const* Qn, double* const* QA, double* const* QB, const double* dt_dev,
                std::vector<ViscArgs>& va, std::vector<SweepBlock>& sa) {
  const int nb = (int)bt->blocks.size();
  va.assign(3 * nb, ViscArgs{});
  sa.assign(9 * nb, SweepBlock{});
  const Phys ph = make_phys(bt->blocks[0]->d.params);
  for (int st = 0; st < 3; ++st) {
    double* const* cur = st == 0 ? Qn : st == 1 ? QA : QB;
    double* const* outp = st == 0 ? QA : st == 1 ? QB : Qn;
    for (int n = 0; n < 3; ++n) {
      SweepCommon& c = bt->sweep_common[st][kSweepOrder[n]];
      std::memset(&c, 0, sizeof c);
      c.ph = ph;
      c.do_inv = 1;
      c.do_vis = bt->viscous;
      c.has_prev = n > 0;
      c.out_kind = n == 2 ? kOutRK : kOutPartial;
      c.dt_dev = dt_dev;
      c.one_sided = bt->one_sided;
      c.ca = kRK[st][0];
      c.cb = kRK[st][1];
      c.cc = kRK[st][2];
    }
    for (int b = 0; b < nb; ++b) {
      cfd_block* B = bt->blocks[b];
      ViscArgs& v = va[st * nb + b];
      v.g = B->g;
      v.q = cur[b];
      v.met = B->met;
      v.met_r = B->met_r;
      v.vis = B->vis;
      v.ph = ph;
      v.one_sided = one_sided_mask(B->d);
      int tiles;
      visc_tiling(B->g, kViscMinTilesBatch, &v.kc, &tiles);
      for (int d = 0; d < 3; ++d) {
        SweepBlock& a = sa[(st * 3 + d) * nb + b];
        std::memset(&a, 0, sizeof a);
        a.g = B->g;
        a.q = cur[b];
        a.met = B->met;
        a.met_r = B->esize == sizeof(double) ? nullptr : static_cast<const float*>(B->met_r);
        a.vis = B->vis;
        a.rt_in = B->rt;
        a.rt_out = B->rt;
        a.out = d == kSweepOrder[2] ? outp[b] : nullptr;
        a.qn = Qn[b];
        a.dt_field = B->dt_field;
        a.one_sided = one_sided_mask(B->d);
        sweep_tiling(d, bt->cfg[d], B->g, &a.tiles_c1, &a.tiles_d, &a.tile_len);
      }
    }
  }
}

hipError_t launch_batch_sweep(cfd_batch* bt, int st, int d) {
  const int nb = (int)bt->blocks.size();
  const TileList& tl = bt->sweep_tl[d];
  const int ntiles = tl.prefix[nb];
  const int nwg = bt->persist[d] ? std::min(ntiles, bt->persist_wgs) : ntiles;
  const SweepBlock* a = bt->sweep_args_dev + (st * 3 + d) * nb;
  const SweepCommon& c = bt->sweep_common[st][d];
  return bt->precision == CFD_FP64
             ? launch_sweep_batch<double>(d, bt->cfg[d], bt->persist[d] != 0, a, c, tl, nwg, bt->stream)
             : launch_sweep_batch<float>(d, bt->cfg[d], bt->persist[d] != 0, a, c, tl, nwg, bt->stream);
}

// one RK stage of every block (all launches on bt->stream)
hipError_t enqueue_stage(cfd_batch* bt, int st, double* const* outp) {
  const int nb = (int)bt->blocks.size();
  hipError_t e = hipSuccess;
  if (bt->viscous) {
    const ViscArgs* va = bt->visc_args_dev + st * nb;
    e = bt->precision == CFD_FP64 ? launch_visc_batch<double>(va, bt->visc_tl, bt->one_sided, bt->stream)
                                  : launch_visc_batch<float>(va, bt->visc_tl, bt->one_sided, bt->stream);
    if (e != hipSuccess) return e;
    PtrTable t;
    std::memset(&t, 0, sizeof t);
    for (int b = 0; b < nb; ++b) {
      t.p[b] = bt->blocks[b]->vis;
      t.plane[b] = bt->blocks[b]->g.plane;
    }
    e = bt->precision == CFD_FP64 ? launch_copy<double>(bt->vcopy_dev, bt->nvcopy, bt->maxvcopy, t, bt->stream)
                                  : launch_copy<float>(bt->vcopy_dev, bt->nvcopy, bt->maxvcopy, t, bt->stream);
    if (e != hipSuccess) return e;
    e = bt->precision == CFD_FP64 ? launch_visc_ghost<double>(bt->vbc_dev, bt->nvbc, bt->maxvbc, t, bt->stream)
                                  : launch_visc_ghost<float>(bt->vbc_dev, bt->nvbc, bt->maxvbc, t, bt->stream);
    if (e != hipSuccess) return e;
  }
  for (int n = 0; n < 3 && e == hipSuccess; ++n) e = launch_batch_sweep(bt, st, kSweepOrder[n]);
  if (e != hipSuccess) return e;
  // Q halos of every block: wall reset, interface / periodic copies, ghost fills
  BcArgs ba;
  std::memset(&ba, 0, sizeof ba);
  for (int b = 0; b < nb; ++b) {
    ba.t.p[b] = outp[b];
    ba.t.plane[b] = bt->blocks[b]->g.plane;
    ba.mt.p[b] = bt->blocks[b]->met;
    ba.mt.plane[b] = bt->blocks[b]->g.plane;
  }
  const cfd_params& P = bt->blocks[0]->d.params;
  ba.gamma = P.gamma;
  ba.t_wall = P.t_wall;
  for (int v = 0; v < 5; ++v) ba.qinf[v] = P.qinf[v];
  cfd_exchange* x = bt->x;
  e = launch_wall_reset(x->bc_dev, x->nbc, x->maxbc, ba, bt->stream);
  if (e == hipSuccess) e = launch_copy<double>(x->q_dev, x->nq, x->maxq, ba.t, bt->stream);
  if (e == hipSuccess) e = launch_ghost_fill(x->bc_dev, x->nbc, x->maxbc, ba, bt->stream);
  return e;
}

int upload_args(cfd_batch* bt, double* const* Qn, double* const* QA, double* const* QB, const double* dt_dev) {
  std::vector<ViscArgs> va;
  std::vector<SweepBlock> sa;
  build_args(bt, Qn, QA, QB, dt_dev, va, sa);
  HIP_TRY(hipMemcpy(bt->visc_args_dev, va.data(), va.size() * sizeof(ViscArgs), hipMemcpyHostToDevice), "upload args");
  HIP_TRY(hipMemcpy(bt->sweep_args_dev, sa.data(), sa.size() * sizeof(SweepBlock), hipMemcpyHostToDevice), "upload args");
  return CFD_OK;
}

// Autotuner: time every (tile configuration, schedule) candidate of each direction's
// batched sweep on the current state (stage 0 arguments; the RK sweep writes QA, which is
// scratch at this point) and keep the fastest.
int autotune(cfd_batch* bt, double* const* Qn, double* const* QA, double* const* QB, const double* dt_dev) {
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0), "event");
  HIP_TRY(hipEventCreate(&e1), "event");
  int rc = CFD_OK;
  if (bt->viscous) {  // the sweeps read the viscous-flux planes of the state being tuned on
    rc = upload_args(bt, Qn, QA, QB, dt_dev);
    if (rc == CFD_OK) {
      hipError_t e = bt->precision == CFD_FP64
                         ? launch_visc_batch<double>(bt->visc_args_dev, bt->visc_tl, bt->one_sided, bt->stream)
                         : launch_visc_batch<float>(bt->visc_args_dev, bt->visc_tl, bt->one_sided, bt->stream);
      if (e != hipSuccess) rc = hip_fail(e, "tuning prepass");
    }
  }
  for (int d = 0; d < 3 && rc == CFD_OK; ++d) {
    float best = 1e30f;
    int best_cfg = 0, best_p = 0;
    for (int c = 0; c < kTileCfgs && rc == CFD_OK; ++c)
      for (int p = 0; p < 2 && rc == CFD_OK; ++p) {
        // not built: the persistent schedule of the original scheme or of one-sided closures
        if (p == 1 && (bt->blocks[0]->d.params.scheme == CFD_AFWENO_ORIGINAL || bt->one_sided)) continue;
        bt->cfg[d] = c;
        bt->persist[d] = p;
        fill_tiles(bt);
        if ((rc = upload_args(bt, Qn, QA, QB, dt_dev)) != CFD_OK) break;
        float ms = 0.f, total = 0.f;
        for (int rep = 0; rep < 3 && rc == CFD_OK; ++rep) {
          hipError_t e = hipEventRecord(e0, bt->stream);
          if (e == hipSuccess) e = launch_batch_sweep(bt, 0, d);
          if (e == hipSuccess) e = hipEventRecord(e1, bt->stream);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
          if (e != hipSuccess) rc = hip_fail(e, "tuning launch");
          if (rep > 0) total += ms;  // first launch warms caches and code
        }
        if (rc == CFD_OK) bt->tune_ms[d][c][p] = total / 2;
        if (rc == CFD_OK && total < best) {
          best = total;
          best_cfg = c;
          best_p = p;
        }
      }
    bt->cfg[d] = best_cfg;
    bt->persist[d] = best_p;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  fill_tiles(bt);
  bt->tuned = rc == CFD_OK;
  return rc;
}

int batch_step(cfd_batch* bt, const double* dt_dev, double* const* Qn, double* const* QA, double* const* QB) {
  if (!bt || !dt_dev || !Qn || !QA || !QB) return fail(CFD_ERR_ARG, "null argument");
  const int nb = (int)bt->blocks.size();
  std::vector<const void*> key;
  key.push_back(dt_dev);
  for (int b = 0; b < nb; ++b) {
    if (!Qn[b] || !QA[b] || !QB[b]) return fail(CFD_ERR_ARG, "null state pointer");
    if (Qn[b] == QA[b] || Qn[b] == QB[b] || QA[b] == QB[b]) return fail(CFD_ERR_ARG, "Qn, QA and QB must be distinct");
    key.push_back(Qn[b]);
    key.push_back(QA[b]);
    key.push_back(QB[b]);
    key.push_back(bt->blocks[b]->dt_field);
  }
  // order the batch stream after the caller's work
  HIP_TRY(hipEventRecord(bt->ev_in, bt->user), "event record");
  HIP_TRY(hipStreamWaitEvent(bt->stream, bt->ev_in, 0), "stream wait");
  if (key != bt->key || !bt->exec) {
    // the argument tables are rewritten below: earlier replays must have finished reading them
    HIP_TRY(hipStreamSynchronize(bt->stream), "stream synchronize");
    if (!bt->tuned) {
      int rc = autotune(bt, Qn, QA, QB, dt_dev);
      if (rc) return rc;
    }
    int rc = upload_args(bt, Qn, QA, QB, dt_dev);
    if (rc) return rc;
    if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
    if (bt->graph) (void)hipGraphDestroy(bt->graph);
    bt->exec = nullptr;
    bt->graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(bt->stream, hipStreamCaptureModeThreadLocal), "begin capture");
    hipError_t e = hipSuccess;
    for (int st = 0; st < 3 && e == hipSuccess; ++st) e = enqueue_stage(bt, st, st == 0 ? QA : st == 1 ? QB : Qn);
    hipGraph_t g = nullptr;
    hipError_t ec = hipStreamEndCapture(bt->stream, &g);
    if (e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return hip_fail(e, "capture of the RK step");
    }
    if (ec != hipSuccess) return hip_fail(ec, "end capture");
    bt->graph = g;
    HIP_TRY(hipGraphInstantiate(&bt->exec, bt->graph, nullptr, nullptr, 0), "graph instantiate");
    bt->key = key;
  }
  HIP_TRY(hipGraphLaunch(bt->exec, bt->stream), "graph launch");
  // and the caller's later work after the step
  HIP_TRY(hipEventRecord(bt->ev_out, bt->stream), "event record");
  HIP_TRY(hipStreamWaitEvent(bt->user, bt->ev_out, 0), "stream wait");
  return CFD_OK;
}

int batch_tuning(const cfd_batch* bt, int* cfg, int* persist) {
  if (!bt || !cfg || !persist) return fail(CFD_ERR_ARG, "null argument");
  for (int d = 0; d < 3; ++d) {
    cfg[d] = bt->cfg[d];
    persist[d] = bt->persist[d];
  }
  return CFD_OK;
}

int batch_tuning_times(const cfd_batch* bt, float* ms, int cap) {
  if (!bt || !ms) return fail(CFD_ERR_ARG, "null argument");
  if (cap < 6 * kTileCfgs) return fail(CFD_ERR_ARG, "timing array too short");
  for (int d = 0; d < 3; ++d)
    for (int c = 0; c < kTileCfgs; ++c)
      for (int p = 0; p < 2; ++p) ms[(d * kTileCfgs + c) * 2 + p] = bt->tune_ms[d][c][p];
  return CFD_OK;
}

int batch_set_tuning(cfd_batch* bt, const int* cfg, const int* persist) {
  if (!bt || !cfg || !persist) return fail(CFD_ERR_ARG, "null argument");
  for (int d = 0; d < 3; ++d)
    if (cfg[d] < 0 || cfg[d] >= kTileCfgs) return fail(CFD_ERR_ARG, "tile configuration out of range");
  if (bt->blocks[0]->d.params.scheme == CFD_AFWENO_ORIGINAL || bt->one_sided)
    for (int d = 0; d < 3; ++d)
      if (persist[d])
        return fail(CFD_ERR_UNSUPPORTED, "the original scheme and one-sided viscous closures have no persistent schedule");
  for (int d = 0; d < 3; ++d) {
    bt->cfg[d] = cfg[d];
    bt->persist[d] = persist[d] != 0;
  }
  fill_tiles(bt);
  bt->tuned = true;
  bt->key.clear();  // recapture with the new tiling
  return CFD_OK;
}

// the same patch seen from block_b: corners trade places, the extents follow b's axes and
// the orientation is inverted
cfd_patch patch_seen_from_b(const cfd_patch& p) {
  cfd_patch q;
  q.block_a = p.block_b;
  q.face_a = p.face_b;
  q.block_b = p.block_a;
  q.face_b = p.face_a;
  q.a_lo[0] = p.b_lo[0];
  q.a_lo[1] = p.b_lo[1];
  q.b_lo[0] = p.a_lo[0];
  q.b_lo[1] = p.a_lo[1];
  const bool swap = p.orient & 1;
  q.n[0] = swap ? p.n[1] : p.n[0];
  q.n[1] = swap ? p.n[0] : p.n[1];
  q.orient = inverse_orient(p.orient);
  return q;
}

// Uncovered parts of a face as rectangles: the face is cut at every patch edge along each
// tangential axis, and every cell of that grid is uniformly covered or not.
std::vector<FaceRect> uncovered_rects(const std::vector<uint8_t>& cov, int n0, int n1,
                                      const std::vector<FaceRect>& patches) {
  std::vector<int> c0{0, n0}, c1{0, n1};
  for (const FaceRect& r : patches) {
    c0.push_back(r.lo[0]);
    c0.push_back(r.lo[0] + r.n[0]);
    c1.push_back(r.lo[1]);
    c1.push_back(r.lo[1] + r.n[1]);
  }
  std::sort(c0.begin(), c0.end());
  c0.erase(std::unique(c0.begin(), c0.end()), c0.end());
  std::sort(c1.begin(), c1.end());
  c1.erase(std::unique(c1.begin(), c1.end()), c1.end());
  std::vector<FaceRect> out;
  const size_t nc0 = c0.size() - 1, nc1 = c1.size() - 1;  // cells along t1, t2
  for (size_t y = 0; y < nc1; ++y)
    for (size_t x = 0; x < nc0; ++x) {
      if (cov[(size_t)c1[y] * n0 + c0[x]]) continue;
      size_t e = x + 1;  // run of uncovered cells along t1: cells x .. e-1
      while (e < nc0 && !cov[(size_t)c1[y] * n0 + c0[e]]) ++e;
      out.push_back(FaceRect{{c0[x], c1[y]}, {c0[e] - c0[x], c1[y + 1] - c1[y]}});
      x = e;  // cell e is covered (or past the end)
    }
  return out;
}

int build_exchange(cfd_block* const* blocks, int nb, const std::vector<cfd_patch>& patches, cfd_exchange** out) {
  if (!out) return fail(CFD_ERR_ARG, "null output handle");
  *out = nullptr;
  if (!blocks || nb <= 0 || nb > kMaxBlocks) return fail(CFD_ERR_ARG, "need 1..64 blocks");
  for (int n = 0; n < nb; ++n)
    if (!blocks[n]) return fail(CFD_ERR_ARG, "null block");
  const int prec = blocks[0]->d.precision;
  for (int n = 0; n < nb; ++n)
    if (blocks[n]->d.precision != prec) return fail(CFD_ERR_ARG, "all blocks of an exchange share one precision");
  std::vector<std::vector<uint8_t>> cov(6 * nb);          // covered nodes per face (t1 fastest)
  std::vector<std::vector<FaceRect>> rects(6 * nb);        // patch rectangles per face
  std::vector<CopySeg> qs, vs;
  std::vector<BcSeg> bs;
  for (const cfd_patch& p : patches) {
    if (p.block_a < 0 || p.block_a >= nb || p.block_b < 0 || p.block_b >= nb || p.face_a < 0 || p.face_a > 5 ||
        p.face_b < 0 || p.face_b > 5)
      return fail(CFD_ERR_ARG, "patch index out of range");
    if (p.block_a == p.block_b && p.face_a == p.face_b) return fail(CFD_ERR_ARG, "a patch joins two faces");
    if (p.orient < 0 || p.orient > 7) return fail(CFD_ERR_ARG, "patch orient must be 0..7");
    if (face_map_det(face_map(p.face_a, p.face_b, p.orient)) != 1)
      return fail(CFD_ERR_ARG, "patch orientation reverses handedness");
    for (int side = 0; side < 2; ++side) {
      const cfd_patch q = side ? patch_seen_from_b(p) : p;
      const cfd_block* A = blocks[q.block_a];
      const cfd_block* B = blocks[q.block_b];
      int ta, tb, ua, ub;
      tangential(q.face_a / 2, &ta, &tb);
      tangential(q.face_b / 2, &ua, &ub);
      const bool swap = q.orient & 1;
      const int eb0 = swap ? q.n[1] : q.n[0], eb1 = swap ? q.n[0] : q.n[1];  // extents along b's t1, t2
      if (q.n[0] < 1 || q.n[1] < 1 || q.a_lo[0] < 0 || q.a_lo[1] < 0 || q.a_lo[0] + q.n[0] > npts(A->g, ta) ||
          q.a_lo[1] + q.n[1] > npts(A->g, tb) || q.b_lo[0] < 0 || q.b_lo[1] < 0 || q.b_lo[0] + eb0 > npts(B->g, ua) ||
          q.b_lo[1] + eb1 > npts(B->g, ub))
        return fail(CFD_ERR_ARG, "patch rectangle outside its face");
      const int kind = A->d.bc[q.face_a];
      if (kind == CFD_BC_PERIODIC) return fail(CFD_ERR_ARG, "a periodic face takes no patch");
      if (is_physical(kind) && A->d.params.visc_closure == CFD_VISC_ONE_SIDED)
        return fail(CFD_ERR_UNSUPPORTED, "a patch on a physical face of a block with the one-sided viscous closure");
      const int fi = 6 * q.block_a + q.face_a;
      const int n0 = npts(A->g, ta);
      if (cov[fi].empty()) cov[fi].assign((size_t)n0 * npts(A->g, tb), 0);
      for (int y = 0; y < q.n[1]; ++y)
        for (int x = 0; x < q.n[0]; ++x) {
          uint8_t& c = cov[fi][(size_t)(q.a_lo[1] + y) * n0 + q.a_lo[0] + x];
          if (c) return fail(CFD_ERR_ARG, "a face node is covered by two patches");
          c = 1;
        }
      const FaceRect ra{{q.a_lo[0], q.a_lo[1]}, {q.n[0], q.n[1]}};
      rects[fi].push_back(ra);
      const FaceMap m = face_map(q.face_a, q.face_b, q.orient);
      qs.push_back(make_copy_rect(A->g, q.block_a, q.face_a, ra, B->g, q.block_b, q.face_b, q.b_lo, 0, 5, q.orient, 0, 0));
      // the face-normal direction's viscous flux: a's direction axis_a is b's axis_b
      vs.push_back(make_copy_rect(A->g, q.block_a, q.face_a, ra, B->g, q.block_b, q.face_b, q.b_lo, 4 * m.axis_a, 4,
                                  q.orient, 4 * m.axis_b, m.normal_sign < 0));
    }
  }
  for (int n = 0; n < nb; ++n) {
    const cfd_block* B = blocks[n];
    for (int f = 0; f < 6; ++f) {
      const int k = B->d.bc[f];
      const int fi = 6 * n + f;
      if (k == CFD_BC_INTERFACE) {
        if (cov[fi].empty() || std::find(cov[fi].begin(), cov[fi].end(), 0) != cov[fi].end())
          return fail(CFD_ERR_ARG, "an interface face is not covered completely");
      }
      if (k == CFD_BC_PERIODIC && (f % 2) == 0) {
        qs.push_back(make_copy(B->g, n, f, B->g, n, f + 1, 0, 5));
        qs.push_back(make_copy(B->g, n, f + 1, B->g, n, f, 0, 5));
      }
      if (is_physical(k)) {
        if (cov[fi].empty()) {
          bs.push_back(make_bc(B->g, n, f, k));
        } else {
          int ta, tb;
          tangential(f / 2, &ta, &tb);
          for (const FaceRect& r : uncovered_rects(cov[fi], npts(B->g, ta), npts(B->g, tb), rects[fi]))
            bs.push_back(make_bc_rect(B->g, n, f, k, r));
        }
      }
    }
  }
  cfd_exchange* x = new cfd_exchange();
  x->blocks.assign(blocks, blocks + nb);
  x->precision = prec;
  for (auto& s : qs) x->maxq = std::max(x->maxq, s.na * s.nb * kHalo * s.nplanes);
  for (auto& s : vs) x->maxv = std::max(x->maxv, s.na * s.nb * kHalo * s.nplanes);
  for (auto& s : bs) x->maxbc = std::max(x->maxbc, s.na * s.nb);
  if (upload(qs, &x->q_dev) || upload(vs, &x->v_dev) || upload(bs, &x->bc_dev)) {
    cfd_exchange_destroy(x);
    return fail(CFD_ERR_HIP, "exchange tables");
  }
  x->nq = (int)qs.size();
  x->nv = (int)vs.size();
  x->nbc = (int)bs.size();
  x->qs_host = qs;
  x->vs_host = vs;
  x->bc_host = bs;
  // blocks whose physical faces are partly connected need the split form from now on
  for (int n = 0; n < nb; ++n)
    for (int f = 0; f < 6; ++f)
      if (is_physical(blocks[n]->d.bc[f]) && !cov[6 * n + f].empty()) {
        x->patched.push_back(blocks[n]);
        ++blocks[n]->patched;
        break;
      }
  *out = x;
  return CFD_OK;
}

}  // namespace

extern "C" {

int cfd_exchange_create(cfd_block* const* blocks, int nb, const cfd_interface* ifc, int nifc, cfd_exchange** out) {
  if (!out) return fail(CFD_ERR_ARG, "null output handle");
  *out = nullptr;
  if (!blocks || nb <= 0 || nb > kMaxBlocks) return fail(CFD_ERR_ARG, "need 1..64 blocks");
  if (nifc < 0 || (nifc > 0 && !ifc)) return fail(CFD_ERR_ARG, "bad interface list");
  for (int n = 0; n < nb; ++n)
    if (!blocks[n]) return fail(CFD_ERR_ARG, "null block");
  std::vector<cfd_patch> ps;
  for (int n = 0; n < nifc; ++n) {
    const cfd_interface& f = ifc[n];
    if (f.block_a < 0 || f.block_a >= nb || f.block_b < 0 || f.block_b >= nb || f.face_a < 0 || f.face_a > 5 ||
        f.face_b < 0 || f.face_b > 5)
      return fail(CFD_ERR_ARG, "interface index out of range");
    if (f.orient < 0 || f.orient > 7) return fail(CFD_ERR_ARG, "interface orient must be 0..7");
    const cfd_block* A = blocks[f.block_a];
    const cfd_block* B = blocks[f.block_b];
    if (A->d.bc[f.face_a] != CFD_BC_INTERFACE || B->d.bc[f.face_b] != CFD_BC_INTERFACE)
      return fail(CFD_ERR_ARG, "interface faces must have kind CFD_BC_INTERFACE");
    const FaceMap m = face_map(f.face_a, f.face_b, f.orient);
    for (int q = 0; q < 2; ++q)
      if (npts(A->g, m.ta[q]) != npts(B->g, m.map_axis[q])) return fail(CFD_ERR_ARG, "interface face sizes differ");
    const FaceRect r = whole_face(A->g, f.face_a);
    cfd_patch p;
    p.block_a = f.block_a;
    p.face_a = f.face_a;
    p.a_lo[0] = p.a_lo[1] = 0;
    p.n[0] = r.n[0];
    p.n[1] = r.n[1];
    p.block_b = f.block_b;
    p.face_b = f.face_b;
    p.b_lo[0] = p.b_lo[1] = 0;
    p.orient = f.orient;
    ps.push_back(p);
  }
  return build_exchange(blocks, nb, ps, out);
}

int cfd_exchange_create_patched(cfd_block* const* blocks, int nb, const cfd_patch* p, int np, cfd_exchange** out) {
  if (!out) return fail(CFD_ERR_ARG, "null output handle");
  *out = nullptr;
  if (np < 0 || (np > 0 && !p)) return fail(CFD_ERR_ARG, "bad patch list");
  return build_exchange(blocks, nb, std::vector<cfd_patch>(p, p + np), out);
}

int cfd_exchange_destroy(cfd_exchange* x) {
  if (!x) return CFD_OK;
  for (cfd_block* b : x->patched) --b->patched;
  (void)hipFree(x->q_dev);
  (void)hipFree(x->v_dev);
  (void)hipFree(x->bc_dev);
  delete x;
  return CFD_OK;
}

int cfd_halo_exchange(cfd_exchange* x, int field_set, void* const* block_bufs, void* hip_stream) {
  if (!x) return fail(CFD_ERR_ARG, "null exchange");
  hipStream_t s = hip_stream ? (hipStream_t)hip_stream : x->blocks[0]->stream;
  const int nb = (int)x->blocks.size();
  PtrTable t;
  std::memset(&t, 0, sizeof t);
  if (field_set == CFD_FIELDS_Q) {
    if (!block_bufs) return fail(CFD_ERR_ARG, "CFD_FIELDS_Q needs the block buffers");
    for (int n = 0; n < nb; ++n) {
      if (!block_bufs[n]) return fail(CFD_ERR_ARG, "null block buffer");
      t.p[n] = block_bufs[n];
      t.plane[n] = x->blocks[n]->g.plane;
    }
    BcArgs ba;
    std::memset(&ba, 0, sizeof ba);
    ba.t = t;
    for (int b = 0; b < nb; ++b) {
      ba.mt.p[b] = x->blocks[b]->met;
      ba.mt.plane[b] = x->blocks[b]->g.plane;
    }
    const cfd_params& P = x->blocks[0]->d.params;
    ba.gamma = P.gamma;
    ba.t_wall = P.t_wall;
    for (int v = 0; v < 5; ++v) ba.qinf[v] = P.qinf[v];
    Profiler* prof = &x->blocks[0]->prof;
    ProfScope ps(prof, "halo_q", s);
    hipError_t e = launch_wall_reset(x->bc_dev, x->nbc, x->maxbc, ba, s);
    if (e == hipSuccess) e = launch_copy<double>(x->q_dev, x->nq, x->maxq, t, s);
    if (e == hipSuccess) e = launch_ghost_fill(x->bc_dev, x->nbc, x->maxbc, ba, s);
    ps.done();
    return e == hipSuccess ? CFD_OK : hip_fail(e, "halo exchange (Q)");
  }
  if (field_set == CFD_FIELDS_VISC) {
    if (block_bufs) return fail(CFD_ERR_ARG, "CFD_FIELDS_VISC uses library buffers: pass NULL");
    for (int n = 0; n < nb; ++n) {
      t.p[n] = x->blocks[n]->vis;
      t.plane[n] = x->blocks[n]->g.plane;
    }
    hipError_t e = x->precision == CFD_FP64 ? launch_copy<double>(x->v_dev, x->nv, x->maxv, t, s)
                                            : launch_copy<float>(x->v_dev, x->nv, x->maxv, t, s);
    return e == hipSuccess ? CFD_OK : hip_fail(e, "halo exchange (viscous)");
  }
  return fail(CFD_ERR_ARG, "unknown field set");
}

int cfd_batch_create(cfd_block* const* blocks, int nb, cfd_exchange* x, void* hip_stream, cfd_batch** out) {
  return batch_create(blocks, nb, x, hip_stream, out);
}
int cfd_batch_destroy(cfd_batch* bt) { return batch_destroy(bt); }
int cfd_batch_step(cfd_batch* bt, const double* dt_dev, double* const* Qn, double* const* QA, double* const* QB) {
  return batch_step(bt, dt_dev, Qn, QA, QB);
}
int cfd_batch_tuning(const cfd_batch* bt, int* cfg, int* persist) { return batch_tuning(bt, cfg, persist); }
int cfd_batch_set_tuning(cfd_batch* bt, const int* cfg, const int* persist) { return batch_set_tuning(bt, cfg, persist); }
int cfd_batch_tuning_times(const cfd_batch* bt, float* ms, int cap) { return batch_tuning_times(bt, ms, cap); }

int cfd_sweep_order(int* dirs) {
  if (!dirs) return fail(CFD_ERR_ARG, "null argument");
  for (int n = 0; n < 3; ++n) dirs[n] = kSweepOrder[n];
  return CFD_OK;
}

int cfd_tile_config_count(void) { return kTileCfgs; }

int cfd_tile_config(int cfg, int* lines, int* nodes, int* threads) {
  if (cfg < 0 || cfg >= kTileCfgs) return fail(CFD_ERR_ARG, "tile configuration out of range");
  if (!lines || !nodes || !threads) return fail(CFD_ERR_ARG, "null argument");
  tile_shape(cfg, lines, nodes, threads);
  return CFD_OK;
}

int cfd_block_set_tiles(cfd_block* b, const int* cfg) {
  if (!b || !cfg) return fail(CFD_ERR_ARG, "null argument");
  for (int d = 0; d < 3; ++d)
    if (cfg[d] < 0 || cfg[d] >= kTileCfgs) return fail(CFD_ERR_ARG, "tile configuration out of range");
  for (int d = 0; d < 3; ++d) b->cfg[d] = cfg[d];
  return CFD_OK;
}

int cfd_block_tiles(const cfd_block* b, int* cfg) {
  if (!b || !cfg) return fail(CFD_ERR_ARG, "null argument");
  for (int d = 0; d < 3; ++d) cfg[d] = b->cfg[d];
  return CFD_OK;
}

}  // extern "C"
