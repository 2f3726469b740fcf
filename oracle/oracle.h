/*
 * oracle.h -- plain FP64 CPU oracle of the curvilinear high-order finite-difference
 * Navier-Stokes right-hand side and TVD-RK3 stage of Ye et al., "Accelerating CFD
 * simulation with high order finite difference method on curvilinear coordinates for
 * modern GPU clusters" (arXiv 2006.07964).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no source with the GPU
 * library; the two meet only through the seeded input arrays.
 *
 * Array layout (all host memory, C order, FP64):
 *   state / metric arrays  A[var][k+3][j+3][i+3], dims (nk+6, nj+6, ni+6), halo 3
 *   coordinates            X[c][k+6][j+6][i+6],  dims (nk+12, nj+12, ni+12), halo 6
 *   metrics                met[10][...]: 3*d+c holds the hatted metric (d in xi,eta,zeta;
 *                          c in x,y,z), i.e. xi_x/J etc. (Sec. 2, Eq 7); met[9] holds J.
 * Return values: 0 on success, negative on error (see each function).
 *
 * Pins: every function is checked by the CPU tests against closed forms, invariants,
 * exact solutions or brute force, except where the paper fixes nothing to check against
 * ("parity unpinned"): the Sutherland constant of oracle_viscosity (only mu(1) = 1 is
 * pinned), the choice of eigenvector basis in oracle_eigvec beyond L R = I and
 * L A R = diag(lambda), and, for the original AFWENO scheme, the arithmetic mean as the
 * state of the half-point characteristic space beyond its mirror symmetry (any symmetric
 * average of the two nodes passes the pins).  The isothermal no-slip wall (ghost
 * velocity, ghost temperature, viscous-flux reflection) and the one-sided viscous
 * closures are pinned by closed forms of Eq 1 next to a wall (shear and conduction modes,
 * the shear mode's decay rate, exactness on degree-6 profiles); the far-field ghost
 * states by their Riemann invariants.
 */
#ifndef CFD_ORACLE_H
#define CFD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* inviscid scheme: characteristic space at the nodes (modified AFWENO, Sec. 4.5.1,
 * Figs 10-11) or at the half points (original AFWENO, Fig 9) */
enum { ORACLE_AFWENO_MODIFIED = 0, ORACLE_AFWENO_ORIGINAL = 1 };

/* face boundary kinds, one per face in the order (i-,i+,j-,j+,k-,k+) */
enum { ORACLE_BC_PERIODIC = 0, ORACLE_BC_INTERFACE = 1, ORACLE_BC_WALL = 2, ORACLE_BC_FARFIELD = 3,
       ORACLE_BC_FARFIELD_CHAR = 4 };

typedef struct oracle_cfg {
  int ni, nj, nk;          /* interior points per direction (>= 7)               */
  double gamma;            /* ratio of specific heats (Sec. 2)                    */
  double mach, reynolds;   /* Ma_inf, Re_inf: viscous factor Ma/Re (Eq 1)         */
  double prandtl;          /* Pr for the heat flux (Eq 6)                         */
  double suth;             /* Sutherland constant S/T_ref (viscosity law)         */
  double eps;              /* WENO epsilon (Eq 15)                                */
  int viscous;             /* 1: add the viscous terms, 0: Euler                  */
  int linear_weights;      /* 1: ideal weights gamma_j instead of Eq 15           */
  int scheme;              /* ORACLE_AFWENO_MODIFIED (Fig 11) or _ORIGINAL (Fig 9) */
  int bc[6];               /* face kinds (ORACLE_BC_*)                            */
  double t_wall;           /* isothermal wall temperature                         */
  double qinf[5];          /* far-field conserved state                           */
  int visc_closure;        /* viscous terms next to wall / far-field faces:       */
                           /* ORACLE_VISC_REFLECT or ORACLE_VISC_ONE_SIDED         */
} oracle_cfg;

/* Viscous derivatives at the three nodes next to a wall or far-field face (Sec. 4.5.2
 * names one-sided differences near block boundaries without giving them): central
 * differences over reflected ghosts (the default), or one-sided seven-point differences
 * over the boundary node and six nodes inside, exact on polynomials of degree six.      */
enum { ORACLE_VISC_REFLECT = 0, ORACLE_VISC_ONE_SIDED = 1 };

/* direction / term mask for oracle_rhs */
#define ORACLE_XI   1u
#define ORACLE_ETA  2u
#define ORACLE_ZETA 4u
#define ORACLE_INV  8u   /* inviscid terms   */
#define ORACLE_VIS 16u   /* viscous terms    */
#define ORACLE_ALL 31u

/* Eq 7 and Eq 8: conservative metrics and Jacobian over the halo-3 box from
 * coordinates with halo 6.  Returns -5 if some J^-1 <= 0.                             */
int oracle_metrics(const oracle_cfg* c, const double* xyz, double* met);

/* R_Q = J * Rtilde on interior points with k in [k0,k1) (pass 0,nk for all); other
 * points of R are left untouched.  Q halos must be valid.  Viscous-flux halos are
 * produced internally with the same face treatment as Q (periodic wrap, or a one-sided
 * copy of the mirrored ghost state at walls/far field, see oracle.c).                    */
int oracle_rhs(const oracle_cfg* c, const double* met, const double* Q, double* R,
               unsigned mask, int k0, int k1);

/* Eq 20 stage s in {0,1,2}: Qout = a*Qn + b*Qcur + cdt*R(Qcur) on the interior, then the
 * halos of Qout are refilled (periodic wrap and physical ghost fill).                    */
int oracle_rk_stage(const oracle_cfg* c, const double* met, int stage, double dt,
                    const double* Qn, const double* Qcur, double* Qout);

/* One full RK3 step in place on Q (three stages), using two scratch state arrays.       */
int oracle_rk_step(const oracle_cfg* c, const double* met, double dt, double* Q);

/* Fill the halo of nvar planes of a single periodic block by periodic wrap.             */
void oracle_periodic_wrap(const oracle_cfg* c, double* A, int nvar);

/* Wall nodes of one block: zero velocity, T = t_wall at their own density (a reading:
 * the paper does not specify its boundary conditions; pinned by the wall-mode tests).  */
void oracle_wall_reset(const oracle_cfg* c, double* Q);
/* Ghost fill of wall / far-field faces of one block (after the halo copies; a reading,
 * pinned as above).                                                                     */
void oracle_bc_fill(const oracle_cfg* c, double* Q);
/* The same with the metrics at hand, which the characteristic far field needs for its
 * normal (faces of kind ORACLE_BC_FARFIELD_CHAR; oracle_bc_fill skips them).            */
void oracle_bc_fill_met(const oracle_cfg* c, const double* met, double* Q);
/* Characteristic far-field ghost state qg from the boundary node's state qb, the outward
 * unit normal n and the far-field state qf (locally one-dimensional Riemann invariants;
 * parity unpinned by the paper, which names no far-field treatment).                    */
void oracle_char_farfield(const double* qb, const double* n, const double* qf, double gamma, double* qg);

/* CFL time step: cfl / max over interior of sum_d (|U_d| + c |grad d|); NaN when the
 * spectral radius of some point is not finite (a non-finite state).                     */
double oracle_dt_cfl(const oracle_cfg* c, const double* met, const double* Q, double cfl);
/* Local time steps for steady runs: dt_field (one plane, state layout) receives
 * cfl / sum_d (|U_d| + c |grad d|) at every interior point; halo entries untouched.       */
void oracle_dt_local(const oracle_cfg* c, const double* met, const double* Q, double cfl, double* dt_field);
/* One RK3 step in place on Q with a time step per point (dt_field) in Eq 20.              */
int oracle_rk_step_local(const oracle_cfg* c, const double* met, const double* dt_field, double* Q);

/* ---- point-level pieces, exposed so that tests can pin them individually ---------- */
/* Eqs 13-17 (with the sub-stencil pairing of the 5th-order interpolant): from the five
 * values v[0..4] at nodes i-2..i+2 return out[0] = left-biased value at i+1/2 and
 * out[1] = right-biased value at i-1/2; beta[0..2] receives the smoothness indicators. */
void oracle_weno5(const double* v, double eps, int linear, double* out, double* beta);
/* Right eigenvectors R (columns, row-major 5x5) and L = R^-1 of the flux Jacobian in
 * the unit direction k at the conserved state q (L R = I and L A R = diag are pinned;
 * the basis of the triple eigenvalue is a reading, parity unpinned beyond that).       */
int oracle_eigvec(const double* q, const double* k, double gamma, double* L, double* R);
/* Steger-Warming split fluxes F+ and F- of state q for the hatted metric vector m.     */
void oracle_split_flux(const double* q, const double* m, double gamma, double* Fp, double* Fm);
/* Physical (inviscid) flux of Eq 4 for the hatted metric vector m.                     */
void oracle_phys_flux(const double* q, const double* m, double gamma, double* F);
/* Sutherland viscosity law used for mu(T) (parity unpinned: the paper names no law;
 * mu(1) = 1 is pinned).                                                                 */
double oracle_viscosity(double T, double suth);

/* ---- multi-block (blocks on one host, 1-to-1 aligned face interfaces) ------------- */
/* A 1-to-1 face connection: ghost layer m (1..3) beyond face_a of block_a is interior
 * layer m-1 inside face_b of block_b (faces may lie on different axes).  orient maps the
 * tangential indices, t1 < t2 being the two axes tangential to a face: bit 0 set pairs a's
 * t1 with b's t2 and a's t2 with b's t1 (else t1-t1, t2-t2); bit 1 set sends index p of
 * a's t1 to n-1-p on its partner axis; bit 2 the same for a's t2.                       */
typedef struct oracle_iface {
  int block_a, face_a, block_b, face_b;  /* face = 0..5 in (i-,i+,j-,j+,k-,k+) */
  int orient;                            /* 0..7, 0 = aligned blocks            */
} oracle_iface;

/* Copy the 3-wide halos of nvar planes (values that do not depend on the index
 * directions, e.g. the state) across every interface, both directions.  Returns -1 on an
 * index out of range, orient outside 0..7 or faces of different sizes.                 */
int oracle_exchange(const oracle_cfg* cfgs, int nb, double* const* arrays, int nvar,
                    const oracle_iface* ifc, int nifc);

/* R_Q for all blocks with interface exchange of the viscous flux planes.               */
int oracle_rhs_multi(const oracle_cfg* cfgs, int nb, const double* const* met,
                     const double* const* Q, double* const* R, unsigned mask,
                     const oracle_iface* ifc, int nifc);

/* One RK3 step of all blocks in place (exchanges and ghost fills after every stage).   */
int oracle_rk_step_multi(const oracle_cfg* cfgs, int nb, const double* const* met,
                         double dt, double* const* Q, const oracle_iface* ifc, int nifc);

/* ---- multi-block with patched connections (Sec. 3: the domain may be split arbitrarily,
 * without the limitation of one-to-one block connection, and connecting and physical
 * faces may be defined anywhere on a block's faces) ----------------------------------- */
/* A patch joins a rectangle of face_a of block_a to an equal rectangle of face_b of
 * block_b, node to node.  The rectangle on face_a starts at (a_lo[0], a_lo[1]) and spans
 * (n[0], n[1]) nodes along a's two tangential axes t1 < t2; the one on face_b starts at
 * (b_lo[0], b_lo[1]) along b's t1 < t2.  orient is that of oracle_iface inside the two
 * rectangles: the swap bit pairs a's t1 with b's t2, a reversal bit sends index p (counted
 * from a's low corner) to the far end minus p of the partner rectangle's axis.  Ghost layer
 * m (1..3) beyond face_a takes interior layer m-1 inside face_b, and the other way round.
 * Rules (violations give -1): no node of a face is covered twice; a face of kind
 * ORACLE_BC_INTERFACE is covered completely; a face of kind ORACLE_BC_PERIODIC takes no
 * patch; a wall or far-field face may be covered in part, its uncovered nodes keeping the
 * physical treatment (wall reset, ghost fill, reflected viscous ghosts), but not with
 * ORACLE_VISC_ONE_SIDED.  A whole-face oracle_iface is the patch with zero corners and
 * the face's extents.                                                                   */
typedef struct oracle_patch {
  int block_a, face_a;
  int a_lo[2], n[2];
  int block_b, face_b;
  int b_lo[2];
  int orient;
} oracle_patch;

/* Halos of all blocks as the solver refills them after a stage: wall reset on the
 * uncovered wall nodes, periodic wraps, copies across the patches (both sides), ghost
 * fill of the uncovered wall and far-field nodes.  Returns -1 on a rule violation.        */
int oracle_halo_patched(const oracle_cfg* cfgs, int nb, const double* const* met, double* const* Q,
                        const oracle_patch* p, int np);
/* R_Q for all blocks, the viscous flux planes exchanged across the patches.             */
int oracle_rhs_patched(const oracle_cfg* cfgs, int nb, const double* const* met, const double* const* Q,
                       double* const* R, unsigned mask, const oracle_patch* p, int np);
/* One RK3 step of all blocks in place (oracle_halo_patched after every stage).          */
int oracle_rk_step_patched(const oracle_cfg* cfgs, int nb, const double* const* met, double dt,
                           double* const* Q, const oracle_patch* p, int np);

/* Number of OpenMP threads the oracle's parallel loops use.                             */
int oracle_threads(void);
/* Use n threads from now on (n > 0); returns the previous count.  Results do not depend
 * on it: every parallel loop writes disjoint outputs in a fixed order per output.        */
int oracle_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
