// cfd_kernels.hpp -- kernel argument structures and host-side launchers of libcfd.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cfd_device.hpp"

namespace cfd {

constexpr int kMaxBlocks = 64;

// work list of a batched launch: block b owns logical tiles [prefix[b], prefix[b+1])
struct TileList {
  int nblk;
  int prefix[kMaxBlocks + 1];
};

// ---- metrics ------------------------------------------------------------------------
struct MetricArgs {
  Geom g;
  const double* xyz;  // caller coordinates, halo 6
  int64_t cld_i, cld_j, cplane;
  double* dcoord;     // 9 planes of inner derivatives, coordinate-box layout (tight)
  double* met;        // 10 planes, state layout
  int* bad;           // set to 1 if some 1/J <= 0
};
hipError_t launch_metrics(const MetricArgs& a, hipStream_t s);

// ---- viscous prepass ----------------------------------------------------------------
struct ViscArgs {
  Geom g;
  const double* q;
  const double* met;
  const void* met_r;  // the 10 metric planes in the compute type
  void* vis;  // 12 planes of the compute type
  Phys ph;
  int kc;     // planes per tile (set by visc_tiling)
  int periodic;  // bit d: the block is periodic with itself along d, the kernel fills
                 // the direction-d flux halos across the d-faces
  int one_sided;  // bit 2*axis + side (side 1: high face): a physical face whose viscous
                  // derivatives use the one-sided closure (the gradients at the three
                  // nodes next to it)
};
template <typename R>
hipError_t launch_visc(ViscArgs a, hipStream_t s);
// dst[e] = float(src[e]) for e < n
hipError_t launch_round(const double* src, float* dst, int64_t n, hipStream_t s);
// Half-point metrics of a mixed-precision block: plane 3 d + c of hm holds, at node n along
// direction d, component c of the direction-d metric at n+1/2 (sixth-order interpolation in
// FP64, rounded once), for n = -1 .. nd-1 along d at every stored position across.
hipError_t launch_half_metrics(const Geom& g, const double* met, float* hm, hipStream_t s);
// batched viscous prepass over the tiles (64 x 16 columns, a chunk of k planes) of every
// block; one_sided: some block has faces with the one-sided closure
template <typename R>
hipError_t launch_visc_batch(const ViscArgs* args_dev, const TileList& tl, bool one_sided, hipStream_t s);
void visc_tiling(const Geom& g, int min_tiles, int* kc, int* tiles);
// the tiles each block of a batched prepass aims for: a block too small to give them with
// long chunks (the 24-block O-grid: 21 columns of 72-96 planes) is cut into chunks of 16
// planes, which balances the launch over the CUs better than whole columns (1% faster step
// in mixed precision, 1.5% in FP64, measured) despite 6 priming planes per chunk; large
// blocks keep chunks of up to 128 planes
constexpr int kViscMinTilesBatch = 84;

// ---- direction sweep ----------------------------------------------------------------
enum OutKind { kOutPartial = 0, kOutRhs = 1, kOutRK = 2 };
// per-block part of a sweep launch
struct SweepBlock {
  Geom g;
  const double* q;    // state whose RHS is evaluated (Qcur)
  const double* met;  // 10 metric planes
  const void* vis;    // 12 viscous-flux planes (compute type)
  const void* rt_in;  // partial sums of earlier directions (compute type) or null
  void* rt_out;       // partial sums out (kOutPartial)
  double* out;        // R (kOutRhs) or Qout (kOutRK)
  const double* qn;   // RK base state (kOutRK)
  const double* dt_field;  // a time step per point (one plane) in place of the scalar one, or null
  int tiles_c1, tiles_d, tile_len;  // filled by the launcher
  int one_sided;  // faces with the one-sided viscous closure (bit 2*axis + side): the
                  // viscous derivative at the three nodes next to them
  // mixed precision: the 10 metric planes rounded to FP32, then the 9 half-point metric
  // planes of launch_half_metrics (null in FP64)
  const float* met_r;
};
// part shared by every block of a launch
struct SweepCommon {
  const double* dt_dev;  // device time step or null (then dt)
  double dt;
  double ca, cb, cc;     // Qout = ca Qn + cb Q + cc dt J Rtilde
  Phys ph;
  int do_inv, do_vis, has_prev, out_kind;
  int one_sided;  // some block of the launch has faces with the one-sided viscous closure
                  // (selects the kernels that evaluate it; batched launches only)
};
struct SweepArgs {
  SweepCommon c;
  SweepBlock b;
};
// Order of the direction sweeps within an RHS evaluation: zeta first, xi last.  The last
// sweep carries the output (R or the RK combination); its extra loads are cheapest along
// xi, whose stencils stay within rows.
constexpr int kSweepOrder[3] = {2, 1, 0};
constexpr int kTileCfgs = 8;
// shape of tile configuration cfg (lines across, nodes along the sweep, threads)
void tile_shape(int cfg, int* tw, int* ts, int* nt);  // sweep tile configurations (see TileCfg in cfd_kernels.hip)
// tiles of one block for direction dir under configuration cfg
void sweep_tiling(int dir, int cfg, const Geom& g, int* tiles_c1, int* tiles_d, int* tile_len);
int sweep_threads(int cfg);
template <typename R>
hipError_t launch_sweep(int dir, SweepArgs a, hipStream_t s, int cfg = 0);

template <typename R>
hipError_t launch_sweep_batch(int dir, int cfg, bool persist, const SweepBlock* blocks_dev, const SweepCommon& c,
                              const TileList& tl, int nwg, hipStream_t s);

// ---- halo copies and boundary fills -------------------------------------------------
struct CopySeg {
  int32_t dst, src;          // block indices
  int32_t na, nb;            // tangential extents
  int32_t plane0, nplanes;   // planes copied
  int32_t layer_fast, pad;   // 1: halo layer is the fastest thread index, else a
  int32_t src_plane0;        // first source plane (dst planes start at plane0)
  int32_t negate;            // 1: copy the negated values
  int64_t dst_off, src_off;  // element offsets of (a=0, b=0, layer 0)
  int64_t dst_sa, dst_sb, dst_sl;
  int64_t src_sa, src_sb, src_sl;
};
struct PtrTable {
  void* p[kMaxBlocks];
  int64_t plane[kMaxBlocks];
};
template <typename T>
hipError_t launch_copy(const CopySeg* segs_dev, int nseg, int max_elems, const PtrTable& t, hipStream_t s);

struct BcSeg {
  int32_t blk, kind;  // kind: CFD_BC_WALL, CFD_BC_FARFIELD or CFD_BC_FARFIELD_CHAR
  int32_t na, nb;
  int64_t wall_off;   // element offset of the boundary node (a=0, b=0)
  int64_t sa, sb;     // tangential strides
  int64_t sout;       // outward step along the face normal
  int32_t axis;
};
struct BcArgs {
  PtrTable t;
  PtrTable mt;  // metric planes of the blocks (characteristic far field)
  double gamma, t_wall;
  double qinf[5];
};
hipError_t launch_wall_reset(const BcSeg* segs_dev, int nseg, int max_elems, const BcArgs& a, hipStream_t s);
hipError_t launch_ghost_fill(const BcSeg* segs_dev, int nseg, int max_elems, const BcArgs& a, hipStream_t s);
template <typename T>
hipError_t launch_visc_ghost(const BcSeg* segs_dev, int nseg, int max_elems, const PtrTable& t, hipStream_t s);

// ---- reductions ---------------------------------------------------------------------
hipError_t launch_dt_max(const Geom& g, const double* q, const double* met, double gamma,
                         unsigned long long* acc, hipStream_t s);
hipError_t launch_finite(const Geom& g, const double* q, int* flag, hipStream_t s);
hipError_t launch_dt_reset(unsigned long long* acc, hipStream_t s);
hipError_t launch_dt_local(const Geom& g, const double* q, const double* met, double gamma, double cfl,
                           double* dt_field, hipStream_t s);
hipError_t launch_dt_finish(const unsigned long long* acc, double cfl, double* dt, hipStream_t s);
// residual norms: kResGroups partial rows (10 doubles: 5 sums of squares, 5 maxima) per
// block, then one reduction of nparts rows to (5 RMS values, 5 maxima)
constexpr int kResGroups = 256;
hipError_t launch_res_partial(const Geom& g, const double* a, const double* b, double scale, double* part,
                              hipStream_t s);
hipError_t launch_res_final(const double* part, int nparts, double inv_n, double* out, hipStream_t s);

}  // namespace cfd
