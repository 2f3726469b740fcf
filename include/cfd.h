/*
 * cfd.h -- C ABI of libcfd, the MI355X (gfx950) implementation of the right-hand side of
 * the curvilinear high-order finite-difference compressible Navier-Stokes scheme of
 * Ye et al., "Accelerating CFD simulation with high order finite difference method on
 * curvilinear coordinates for modern GPU clusters" (arXiv 2006.07964), fused with the
 * three-stage TVD Runge-Kutta update.
 *
 * Conventions
 *  - Every function returns an int status (CFD_OK or a negative CFD_ERR_*); on error
 *    cfd_last_error() returns a thread-local message.  Nothing throws or aborts.
 *  - Work is enqueued on a HIP stream and is asynchronous unless stated otherwise.
 *    Argument errors are reported synchronously; device faults surface at the next
 *    synchronising call (cfd_sync, cfd_dt_cfl, cfd_check_finite, cfd_metrics,
 *    cfd_residual).
 *  - Pointers named Q, R, Qn, Qcur, Qout, xyz, dt_dev, dt_field, the arrays of
 *    cfd_residual and the block_bufs of cfd_halo_exchange are device pointers owned by
 *    the caller; the library never frees them.  Metrics,
 *    scratch, exchange tables and work lists are owned by the library and released by the
 *    matching *_destroy.  Handles are not thread-safe.
 *  - State layout: structure of arrays, plane v of a field holds
 *        A[v*plane + ((k+3)*ld_j + (j+3))*ld_i + (i+3)],  plane = ld_i*ld_j*(nk+6),
 *    for i in [-3, ni+3), j in [-3, nj+3), k in [-3, nk+3) (halo 3 on every face, i
 *    contiguous); ld_i >= ni+6 and ld_j >= nj+6 may include padding.  Q has the five
 *    planes (rho, rho u, rho v, rho w, e) of Eq 3 without the 1/J factor.
 *  - Nondimensional units (Eq 1): rho_inf = 1, c_inf = 1, T = gamma p / rho, the viscous
 *    terms carry Ma/Re.  Index spacing in xi, eta and zeta is one.
 */
#ifndef CFD_H
#define CFD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------------ */
#define CFD_OK 0
#define CFD_ERR_ARG (-1)          /* invalid argument (sizes, pointers, aliasing)        */
#define CFD_ERR_ALLOC (-2)        /* device allocation failed                            */
#define CFD_ERR_HIP (-3)          /* a HIP runtime call failed (message has details)     */
#define CFD_ERR_STATE (-4)        /* call out of order (e.g. cfd_rhs before cfd_metrics) */
#define CFD_ERR_JACOBIAN (-5)     /* some 1/J <= 0 (folded or left-handed grid)           */
#define CFD_ERR_NONFINITE (-6)    /* NaN or Inf found in a state                         */
#define CFD_ERR_UNSUPPORTED (-7)  /* valid request the library does not implement        */

/* ---- enumerations ------------------------------------------------------------------ */
enum { CFD_FP64 = 0, CFD_MIXED = 1 };                  /* arithmetic of the RHS        */
enum { CFD_WENO_JS = 0, CFD_WENO_LINEAR = 1 };         /* Eq 15 weights or ideal ones  */
/* inviscid scheme (Sec. 4.5.1): characteristic space at the nodes, one WENO stencil giving
 * the values on both sides of the node (modified AFWENO, Figs 10-11), or at the half
 * points, two WENO interpolations per half point (original AFWENO, Fig 9)              */
enum { CFD_AFWENO_MODIFIED = 0, CFD_AFWENO_ORIGINAL = 1 };
/* viscous derivatives at the three nodes next to a CFD_BC_WALL / CFD_BC_FARFIELD[_CHAR]
 * face (Sec. 4.5.2 mentions one-sided differences near block boundaries): central
 * sixth-order differences over ghost values of the velocity, temperature and viscous
 * fluxes reflected about the boundary node (second-order accurate there), or seven-point
 * one-sided differences over the boundary node and six nodes inside, exact on
 * polynomials of degree six, for the gradients and the viscous-flux derivative.  The
 * inviscid terms use the ghost states of the face either way.                          */
enum { CFD_VISC_REFLECT = 0, CFD_VISC_ONE_SIDED = 1 };
/* face kinds; CFD_BC_FARFIELD holds qinf in the ghosts, CFD_BC_FARFIELD_CHAR fills them
 * from locally one-dimensional Riemann invariants along the outward normal (boundary
 * node's outgoing invariant, qinf's incoming one, entropy and tangential velocity from the
 * upwind side; every wave leaving or entering at supersonic normal speed keeps the
 * boundary state or qinf).  The paper names no far-field treatment: both are readings. */
enum { CFD_BC_PERIODIC = 0, CFD_BC_INTERFACE = 1, CFD_BC_WALL = 2, CFD_BC_FARFIELD = 3, CFD_BC_FARFIELD_CHAR = 4 };
enum { CFD_FIELDS_Q = 0, CFD_FIELDS_VISC = 1 };        /* field sets of an exchange    */

/* direction / term mask of cfd_rhs */
#define CFD_DIR_XI 1u
#define CFD_DIR_ETA 2u
#define CFD_DIR_ZETA 4u
#define CFD_TERM_INV 8u
#define CFD_TERM_VIS 16u
#define CFD_ALL 31u

/* ---- descriptors ------------------------------------------------------------------- */
typedef struct cfd_params {
  double gamma;     /* ratio of specific heats (Sec. 2: 1.4)                            */
  double mach;      /* Ma_inf; the viscous terms are scaled by Ma/Re (Eq 1)             */
  double reynolds;  /* Re_inf                                                           */
  double prandtl;   /* Pr of the heat flux (Eq 6)                                       */
  double suth;      /* Sutherland constant S/T_ref of mu(T) = T^1.5 (1+S)/(T+S)         */
  double weno_eps;  /* epsilon of Eq 15 (paper: 1e-6); with WENO_JS weights at least
                       1e-30 (FP64) or 1e-8 (CFD_MIXED), else CFD_ERR_ARG: the weights
                       are formed over a common denominator that scales as eps^8 / eps^4
                       where the smoothness indicators vanish                           */
  int32_t viscous;  /* 1: Navier-Stokes, 0: Euler                                       */
  int32_t weights;  /* CFD_WENO_JS or CFD_WENO_LINEAR                                   */
  int32_t scheme;   /* CFD_AFWENO_MODIFIED (default) or CFD_AFWENO_ORIGINAL; the batched
                       form runs the original one with one workgroup per tile only      */
  int32_t visc_closure; /* CFD_VISC_REFLECT (default) or CFD_VISC_ONE_SIDED            */
  double t_wall;    /* isothermal wall temperature (CFD_BC_WALL faces)                  */
  double qinf[5];   /* conserved far-field state (CFD_BC_FARFIELD faces)                */
} cfd_params;

typedef struct cfd_block_desc {
  int32_t ni, nj, nk;  /* interior points, each >= 7                                    */
  int64_t ld_i, ld_j;  /* pitches in elements, ld_i >= ni+6, ld_j >= nj+6               */
  int32_t precision;   /* CFD_FP64 or CFD_MIXED                                         */
  int32_t bc[6];       /* face kinds in the order i-, i+, j-, j+, k-, k+                */
  cfd_params params;
} cfd_block_desc;

/* 1-to-1 face connection (Sec. 4.2).  Ghost layer m (1..3) beyond face_a of block_a is
 * interior layer m-1 inside face_b of block_b, and the other way round.  The faces may lie
 * on different axes.  orient maps the tangential indices: with t1 < t2 the two axes
 * tangential to a face (i < j < k), bit 0 set means a's t1 runs along b's t2 and a's t2
 * along b's t1 (else t1 along t1, t2 along t2); bit 1 set means index p along a's t1 is
 * index n-1-p on its partner axis (else p), bit 2 the same for a's t2.  orient = 0 is the
 * identity of aligned blocks.  The map from a's indices to b's must keep the handedness
 * (both blocks have positive Jacobians); the viscous flux of a's face-normal direction
 * is taken from b's face-normal direction, negated when the two run opposite ways.     */
typedef struct cfd_interface {
  int32_t block_a, face_a;      /* face index 0..5 in the order of cfd_block_desc.bc   */
  int32_t block_b, face_b;      /* faces of equal size after the orientation           */
  int32_t orient;               /* 0..7 as above                                       */
} cfd_interface;

/* A patch of a block connection (Sec. 3: the domain may be split arbitrarily, without the
 * limitation of one-to-one block connection, and connecting and physical faces may be
 * defined anywhere on a block's faces).  The rectangle of face_a of block_a that starts at
 * node (a_lo[0], a_lo[1]) and spans (n[0], n[1]) nodes along a's tangential axes t1 < t2
 * is joined node to node with the rectangle of face_b of block_b that starts at
 * (b_lo[0], b_lo[1]) along b's tangential axes t1 < t2.  orient is that of cfd_interface
 * applied inside the two rectangles: with a reversal bit set, index p along a's axis
 * (counted from a_lo) lands on the partner axis at the rectangle's far end minus p.  Ghost
 * layer m (1..3) beyond a's rectangle is interior layer m-1 inside b's, and the other way
 * round.  A cfd_interface is the patch with zero corners and the whole face.             */
typedef struct cfd_patch {
  int32_t block_a, face_a;
  int32_t a_lo[2], n[2];        /* corner and extents on face_a (along a's t1, t2)       */
  int32_t block_b, face_b;
  int32_t b_lo[2];              /* corner on face_b (along b's t1, t2)                   */
  int32_t orient;               /* 0..7 as for cfd_interface                             */
} cfd_patch;

typedef struct cfd_block cfd_block;
typedef struct cfd_exchange cfd_exchange;
typedef struct cfd_batch cfd_batch;

/* ---- errors ------------------------------------------------------------------------ */
/* Message of the last failing call on this thread ("" if none).  The pointer stays
 * valid until the next call on the same thread.                                        */
const char* cfd_last_error(void);

/* ---- blocks ------------------------------------------------------------------------ */
/* Create a block: validates d, allocates the 10 metric planes (Sec. 2, Eqs 7-8) and the
 * scratch of the RHS (12 viscous-flux planes, Eqs 5-6, and 5 partial-sum planes, in the
 * compute type; a CFD_MIXED block also keeps the metric planes rounded to FP32 for its
 * FP32 arithmetic, and the metrics of the half points between nodes, which Sec. 4.5
 * interpolates from the node values where they are used, interpolated once in FP64 and
 * rounded) on the current device.  hip_stream (hipStream_t, may be NULL =
 * default stream) is the stream later calls enqueue on.  Errors: CFD_ERR_ARG,
 * CFD_ERR_ALLOC, CFD_ERR_UNSUPPORTED (a plane of 2^29 points or more).                   */
int cfd_block_create(const cfd_block_desc* d, void* hip_stream, cfd_block** out);
/* Free everything the block owns (waits for its stream first).  NULL is a no-op.        */
int cfd_block_destroy(cfd_block* b);
/* Change the stream later calls on b enqueue on.                                        */
int cfd_block_set_stream(cfd_block* b, void* hip_stream);
/* Device bytes the block owns (metrics + scratch).                                     */
int cfd_block_bytes(const cfd_block* b, int64_t* bytes);

/* Sec. 2, Eqs 7-8: conservative metrics xi_x/J ... zeta_z/J and the Jacobian J over the
 * whole halo-3 box, in FP64, by sixth-order central differences of the coordinates.
 * xyz: device, 3 planes (x, y, z) with halo 6: X[c*cplane + ((k+6)*cld_j + (j+6))*cld_i +
 * (i+6)], cplane = cld_i*cld_j*(nk+12), cld_i >= ni+12, cld_j >= nj+12.  Periodic
 * directions carry unwrapped images (x continues past the box), walls mirrored points.
 * Synchronises; CFD_ERR_JACOBIAN if some 1/J <= 0.                                     */
int cfd_metrics(cfd_block* b, const double* xyz, int64_t cld_i, int64_t cld_j);
/* Device pointer to the block's 10 metric planes (layout of Q; plane 3*d+c = metric of
 * direction d in {xi,eta,zeta}, component c in {x,y,z}, divided by J; plane 9 = J).     */
int cfd_metrics_ptr(const cfd_block* b, const double** met);

/* Right-hand side R = dQ/dt = J * Rtilde on the interior (Eq 2 with Q = J U~):
 * inviscid derivatives by the modified AFWENO of Sec. 4.5.1 (Figs 10-11: characteristic
 * projection at the node, fifth-order WENO interpolation to both half points, Eqs 13-17,
 * Steger-Warming split fluxes, Eq 19) and central viscous terms (Eqs 5, 6, 21, sixth-order
 * differences).  Q halos must be valid.  mask selects directions and terms (CFD_DIR_*,
 * CFD_TERM_*); R interior is overwritten, halos untouched.  FP64 output in both
 * precisions.  Not for the timed loop (use cfd_rk_stage).                               */
int cfd_rhs(cfd_block* b, const double* Q, double* R, unsigned mask);

/* One stage s in {0,1,2} of the TVD-RK3 scheme (Eq 20), fused with the RHS:
 * Qout = a_s Qn + b_s Qcur + c_s dt R(Qcur) on the interior with (a,b,c) = (1,0,1),
 * (3/4,1/4,1/4), (1/3,2/3,2/3).  Accumulation is FP64 in both precisions.  Qout halos are
 * left stale (run cfd_halo_exchange).  Qout must not alias Qcur; Qout may alias Qn only
 * at stage 2; at stage 0, Qcur must equal Qn.  Errors: CFD_ERR_ARG, CFD_ERR_STATE.      */
int cfd_rk_stage(cfd_block* b, int stage, double dt, const double* Qn, const double* Qcur,
                 double* Qout);
/* Same, with dt read from device memory at run time (for captured graphs).             */
int cfd_rk_stage_dev(cfd_block* b, int stage, const double* dt_dev, const double* Qn,
                     const double* Qcur, double* Qout);

/* Split form of cfd_rhs / cfd_rk_stage for blocks with CFD_BC_INTERFACE faces, whose
 * viscous-flux halos need data of other blocks: run cfd_viscous_fluxes on every block,
 * then cfd_halo_exchange(x, CFD_FIELDS_VISC, NULL, ...), then the sweeps.  The viscous
 * fluxes (Eqs 5-6 with the gradients of Eq 21) land in the block's scratch; periodic and
 * physical faces of the block get their viscous halos inside cfd_viscous_fluxes.        */
int cfd_viscous_fluxes(cfd_block* b, const double* Q);
int cfd_rhs_sweeps(cfd_block* b, const double* Q, double* R, unsigned mask);
int cfd_rk_sweeps(cfd_block* b, int stage, double dt, const double* Qn, const double* Qcur,
                  double* Qout);

/* ---- halo exchange ----------------------------------------------------------------- */
/* Plan the halo traffic of nb blocks: ifc lists the 1-to-1 interfaces (a face of a block
 * listed with another face of itself is a periodic wrap, possibly with a rotation);
 * faces of kind CFD_BC_PERIODIC wrap onto the opposite face of their own block,
 * CFD_BC_WALL / CFD_BC_FARFIELD faces get ghost fills.
 * Errors: CFD_ERR_ARG on mismatched face sizes or kinds, orient outside 0..7, a map that
 * reverses handedness, or a face used twice.                                          */
int cfd_exchange_create(cfd_block* const* blocks, int nb, const cfd_interface* ifc, int nifc,
                        cfd_exchange** out);
/* The same for blocks joined by patches (np >= 0; p may be NULL when np is 0).  A face of
 * kind CFD_BC_INTERFACE must be covered by patches completely; a CFD_BC_WALL /
 * CFD_BC_FARFIELD / CFD_BC_FARFIELD_CHAR face may be covered in part: its covered nodes
 * take the connected block's values, the others keep the wall reset, the ghost fill and
 * the reflected viscous ghosts; CFD_BC_PERIODIC faces take no patch.  Blocks with a patch
 * on a physical face use the split form (cfd_viscous_fluxes, the viscous exchange, the
 * sweeps) or the batched form, like blocks with interface faces.
 * Errors: CFD_ERR_ARG on an index or a rectangle out of range, a node covered twice, an
 * interface face left partly uncovered, a patch on a periodic face, orient outside 0..7 or
 * a map that reverses handedness; CFD_ERR_UNSUPPORTED for a patch on a physical face of a
 * block with the one-sided viscous closure (it treats the whole face as physical).       */
int cfd_exchange_create_patched(cfd_block* const* blocks, int nb, const cfd_patch* p, int np,
                                cfd_exchange** out);
/* Free a plan (NULL is a no-op).  A plan refers to its blocks: destroy it (and any batch
 * made with it) before them.                                                             */
int cfd_exchange_destroy(cfd_exchange* x);
/* Refill halos by on-device copies (Sec. 4.2: blocks of one process exchange on the
 * device).  field_set CFD_FIELDS_Q: block_bufs[b] is block b's caller-owned Q (5 planes);
 * copies 3-deep face slabs across interfaces, then ghost-fills walls and far field and
 * resets wall nodes (no slip, T = t_wall).  CFD_FIELDS_VISC: block_bufs must be NULL;
 * copies the library's viscous-flux planes (direction-d components across d-faces).
 * Enqueued on hip_stream (NULL: the first block's stream); the caller orders it after the
 * work that produced the buffers when blocks use other streams.                         */
int cfd_halo_exchange(cfd_exchange* x, int field_set, void* const* block_bufs, void* hip_stream);

/* ---- time step and checks ---------------------------------------------------------- */
/* dt = cfl / max over all interior points of all blocks of
 * sum_d (|U_d| + c |grad d|), U_d the contravariant velocity with unhatted metrics
 * (the CFL-controlled global step of Sec. 4.5.3).  Q[b] device.  Synchronises.
 * CFD_ERR_NONFINITE if that sum is not finite at some point (a NaN or Inf in a state).  */
int cfd_dt_cfl(cfd_block* const* blocks, int nb, const double* const* Q, double cfl,
               double* dt_out);
/* The same step written to device memory: *dt_dev (one double, device) receives the
 * value, or NaN when the spectral radius is not positive and finite (in particular when
 * any point's sum is NaN or infinite).  Stream-ordered on
 * blocks[0]'s stream, after the work already enqueued on every block's stream (event
 * waits, no host synchronisation; no memset), so a time loop can recompute the step
 * every iteration and hand dt_dev to cfd_rk_stage_dev or cfd_batch_step (the reduced-
 * dimensional CFL minimum of Sec. 4.5.3 done on the device).  Uses blocks[0]'s reduction
 * scratch: calls that share blocks[0] must not overlap on different streams.
 * Errors: CFD_ERR_ARG, CFD_ERR_STATE (no metrics), CFD_ERR_HIP.                        */
int cfd_dt_cfl_dev(cfd_block* const* blocks, int nb, const double* const* Q, double cfl,
                   double* dt_dev);
/* Local time steps for steady runs (the stored step per point that Sec. 4.4 lists for
 * local time stepping): dt_field[b] (device, one plane in block b's layout, caller-owned)
 * receives cfl / sum_d (|U_d| + c |grad d|) at every interior point of block b (the
 * spectral radius of cfd_dt_cfl, point by point; halo entries untouched).  Enqueued on
 * each block's stream; no synchronisation.  Errors: CFD_ERR_ARG, CFD_ERR_STATE, CFD_ERR_HIP. */
int cfd_dt_local(cfd_block* const* blocks, int nb, const double* const* Q, double cfl,
                 double* const* dt_field);
/* Make every later RK stage of block b (cfd_rk_stage[_dev], cfd_rk_sweeps and the batched
 * steps) take the step of each point from dt_field (device, one plane in b's layout,
 * caller-owned, kept alive while set) instead of the scalar dt, which is then ignored;
 * NULL restores the scalar step.  A batch notices the change at its next step.          */
int cfd_block_set_local_dt(cfd_block* b, const double* dt_field);
/* Residual norms (the residual evaluation that closes each iteration of Fig 2, a
 * reduced-dimensional reduction of Sec. 4.5.3): with d = scale * (A[b] - B[b]) over the
 * interior points of all nb blocks (B or B[b] NULL: d = scale * A[b]),
 *   out[f]     = sqrt(sum d_f^2 / N)  (root mean square, N = all interior points),
 *   out[5 + f] = max |d_f|,           f = rho, rho u, rho v, rho w, e.
 * A[b], B[b]: device states in block b's layout; out: 10 host doubles.  E.g. the RHS
 * residual is A = R, B = NULL, scale = 1; the step residual (Q^{n+1} - Q^n)/dt is
 * A = Q^{n+1}, B = Q^n, scale = 1/dt.  Sums run in a fixed order (bitwise reproducible).
 * Runs on blocks[0]'s stream after every block's enqueued work; synchronises.  The first
 * call allocates blocks[0]'s residual scratch (about 1.3 MB).  Errors: CFD_ERR_ARG
 * (nb outside 1..64, null arrays, non-finite scale), CFD_ERR_ALLOC, CFD_ERR_HIP,
 * CFD_ERR_NONFINITE (a norm is not finite).                                             */
int cfd_residual(cfd_block* const* blocks, int nb, const double* const* A, const double* const* B,
                 double scale, double* out);
/* cfd_residual for callers that cannot allocate device memory (code under HIP graph
 * capture, tight time loops, harnesses that forbid allocation): the same norms, the same
 * kernels and summation order (bitwise the same result), but the partial rows live in a
 * fixed scratch array of the library (1.31 MB per device: 64 blocks x 256 rows x 10
 * doubles + 10), found once per device at the first call; no hipMalloc or hipFree, ever.
 * Every call on one GPU shares that array: calls that overlap on one device (different
 * host threads, or streams not ordered with each other) race and must not be made.
 * Arguments, ordering and synchronisation as cfd_residual; nb above 64 gives CFD_ERR_ARG.  */
int cfd_residual_noalloc(cfd_block* const* blocks, int nb, const double* const* A, const double* const* B,
                         double scale, double* out);
/* *ok = 1 if every interior value of Q is finite, else 0 (and CFD_ERR_NONFINITE).
 * Synchronises.                                                                        */
int cfd_check_finite(cfd_block* b, const double* Q, int* ok);
/* Wait for the block's stream and report any pending device error.                     */
int cfd_sync(cfd_block* b);

/* ---- batched multi-block form ------------------------------------------------------ */
/* Batch all blocks (one precision) behind one launch per phase over a work list of
 * tiles of every block; x must have been created for the same blocks in the same order.
 * hip_stream: the caller's stream; steps run on a stream the batch owns (graphs cannot be
 * captured on the legacy default stream), ordered after the caller's earlier work on
 * hip_stream and before its later work, through events.                                 */
int cfd_batch_create(cfd_block* const* blocks, int nb, cfd_exchange* x, void* hip_stream,
                     cfd_batch** out);
int cfd_batch_destroy(cfd_batch* bt);
/* One full RK3 step of all blocks: Qn[b] (in/out), QA[b] and QB[b] (caller scratch of
 * the layout of Qn[b]); dt_dev is a device double.  The first call captures the step in a
 * HIP graph for this pointer set; later calls with the same pointers replay it.         */
int cfd_batch_step(cfd_batch* bt, const double* dt_dev, double* const* Qn, double* const* QA,
                   double* const* QB);

/* Tile configuration chosen per sweep direction (cfg[d] indexes the library's tile
 * shapes, persist[d] = 1 for the persistent schedule).  Before the first step these are
 * the defaults; the first cfd_batch_step times every candidate and keeps the fastest.   */
int cfd_batch_tuning(const cfd_batch* bt, int* cfg, int* persist);
/* Override the tiling (skips the autotuner; the next step re-captures its graph).
 * CFD_ERR_UNSUPPORTED for a persistent schedule with the original scheme or with blocks
 * that use the one-sided viscous closure (those run one workgroup per tile).            */
int cfd_batch_set_tuning(cfd_batch* bt, const int* cfg, const int* persist);
/* Milliseconds per launch that the autotuner measured for each candidate, at
 * ms[(d * cfd_tile_config_count() + cfg) * 2 + persist] for sweep direction d; -1 where
 * nothing was measured (the tuner runs on the first step unless cfd_batch_set_tuning
 * came first).  cap is the length of ms, at least 6 * cfd_tile_config_count().          */
int cfd_batch_tuning_times(const cfd_batch* bt, float* ms, int cap);

/* Order of the three direction sweeps of an RHS evaluation (dirs[0..2], 0 = xi, 1 = eta,
 * 2 = zeta); the last one writes R or the RK stage, the others partial sums.            */
int cfd_sweep_order(int* dirs);

/* ---- sweep tile shapes ----------------------------------------------------------------
 * A sweep workgroup owns `lines` grid lines across the sweep direction and up to `nodes`
 * output nodes along it, with `threads` threads.  cfd_tile_config_count() returns the
 * number of shapes; cfd_tile_config gives shape cfg (CFD_ERR_ARG if out of range).       */
int cfd_tile_config_count(void);
int cfd_tile_config(int cfg, int* lines, int* nodes, int* threads);
/* Tile shape per direction (cfg[0..2] for xi, eta, zeta) of a block's own launches
 * (cfd_rhs, cfd_rk_stage, cfd_rhs_sweeps, cfd_rk_sweeps).  Every shape does the same
 * arithmetic per node; each is a separately compiled kernel whose multiply-add
 * contraction may differ, so shapes agree to round-off.  The default is the library's
 * choice for large blocks.                                                               */
int cfd_block_set_tiles(cfd_block* b, const int* cfg);
int cfd_block_tiles(const cfd_block* b, int* cfg);

/* ---- profiling --------------------------------------------------------------------- */
/* Enable (1) or disable (0) per-launch HIP event timing of the block's kernels.         */
int cfd_profile_enable(cfd_block* b, int enable);
/* Copy up to cap (name, launches, total milliseconds) entries of the kernels timed so
 * far; names are static strings.  Synchronises.  *n receives the entry count.           */
int cfd_profile_read(cfd_block* b, const char** names, int64_t* launches, double* ms, int cap,
                     int* n);
/* Reset the profiling counters.                                                        */
int cfd_profile_reset(cfd_block* b);

#ifdef __cplusplus
}
#endif
#endif /* CFD_H */
