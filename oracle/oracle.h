/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 implementation of the geometry queries of the paper
 * (Sec. III.C: is a particle inside or outside a solid, what is its minimal
 * distance to the border, and what is the maximal step along its direction)
 * and of step selection along a placed-volume tree (Sec. III.A: the particle is
 * transported to the border when the proposed physics step is longer; Sec. III.B:
 * elementary solids with coordinate transforms, arranged hierarchically).
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may call
 * this code.  It shares no source, header, table or helper with the HIP library;
 * the two meet only in the geometry blob format and the seeded inputs.
 *
 * Rules of the oracle:
 *   - FP64, IEEE round-to-nearest, built with -ffp-contract=off (no FMA).
 *   - Distances are computed by the event-list definition: every root of every
 *     full bounding surface splits the ray into intervals; each interval is
 *     classified by probing the Inside code at 1/4, 1/2 and 3/4 of it (or at
 *     +1, +2, +4 mm for the last, infinite one); DistanceToIn is the start of
 *     the first inside interval, DistanceToOut the start of the first outside
 *     interval.  No per-face analytic logic.
 *   - One track at a time (Geant4's serial per-particle model, Sec. III.B); the
 *     batch wrappers only spread independent tracks over threads.
 *
 * Parity pins live in tests/test_oracle_*.py.  Functions whose result is a
 * chosen formula rather than a unique quantity are marked "parity unpinned"
 * below where no independent check reaches them.
 */
#ifndef GV_ORACLE_H
#define GV_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#define OR_KTOL 1e-9   /* kTolerance, mm */
#define OR_KHALF 5e-10 /* half-width of the surface band, mm */
#define OR_MAX_NZ 64   /* polycone planes */
#define OR_MAX_ROOTS (2 * (4 * OR_MAX_NZ + 16)) /* a composite holds two solids */

enum { OR_BOX = 0, OR_TUBS = 1, OR_CONS = 2, OR_SPHERE = 3, OR_TRD = 4, OR_PCON = 5, OR_BOOL = 6 };
/* composite operations: A u C, A \ C, A n C */
enum { OR_UNION = 0, OR_SUBTRACTION = 1, OR_INTERSECTION = 2 };
enum { OR_OUTSIDE = 0, OR_SURFACE = 1, OR_INSIDE = 2 };
enum { OR_SAFETY_AUTO = 0, OR_SAFETY_IN = 1, OR_SAFETY_OUT = 2 };

/* Per-track flags that are part of the transport contract. */
#define OR_F_OVERFLOW 1u
#define OR_F_STUCK 2u
#define OR_F_LOCATE_FAIL 4u
/* Oracle-only diagnostics: ill-conditioned decisions that two correct FP64
 * codes may take differently; such tracks are listed, not counted. */
#define OR_D_NEAR_TIE 16u
#define OR_D_GRAZE 32u
#define OR_D_ZERO_STEP 64u
#define OR_D_BAND_EDGE 128u
#define OR_D_NO_EXIT 256u
/* A solid-level distance whose hit no FP64 code can fix to the 1e-12 relative
 * bar: its conditioning bound 16 eps L / |cos theta| exceeds
 * 1e-12 max(|t|, 1 mm), theta the angle between the ray and the normal of the
 * surface hit (or_hit_cond). */
#define OR_D_COND 512u

typedef struct or_solid {
  int type;
  int nz; /* polycone planes */
  double p[8];
  /* phi segment (tubs, cons) */
  int full_phi, convex_wedge;
  double ns[2], ne[2], us[2], ue[2];
  /* cons */
  double ao, bo, co, ai, bi, ci;
  int has_inner;
  /* trd */
  double x0, tx, cx, y0, ty, cy;
  /* pcon */
  double z[OR_MAX_NZ], rmin[OR_MAX_NZ], rmax[OR_MAX_NZ];
  double pc_bo[OR_MAX_NZ], pc_co[OR_MAX_NZ], pc_bi[OR_MAX_NZ], pc_ci[OR_MAX_NZ];
  int pc_inner[OR_MAX_NZ];
  /* composite: comp[0] = A at the composite's origin, comp[1] = C placed by
   * x = R x_C + t (R row major); heap-owned, see or_solid_release */
  int op;
  double bR[9], bt[3];
  struct or_solid* comp;
} or_solid;

/* returns 0 on success, negative on invalid parameters; a composite's
 * components are allocated and must be released with or_solid_release */
int or_solid_init(or_solid* s, int type, const double* params, int nparams);
void or_solid_release(or_solid* s);

/* composites (or_bool.c) */
int or_bool_init(or_solid* s, const double* q, int nq);
void or_bool_to_c(const or_solid* s, const double p[3], const double d[3], double pc[3], double dc[3]);
double or_bool_signed(const or_solid* s, const double p[3]);
double or_bool_safety_in(const or_solid* s, const double p[3]);
double or_bool_safety_out(const or_solid* s, const double p[3]);
int or_bool_roots(const or_solid* s, const double p[3], const double d[3], double* roots);

double or_signed(const or_solid* s, const double p[3]);
int or_code(double s);
int or_inside(const or_solid* s, const double p[3]);
double or_safety_in(const or_solid* s, const double p[3]);  /* SafetyToIn, point outside */
double or_safety_out(const or_solid* s, const double p[3]); /* SafetyToOut, point inside */
double or_safety(const or_solid* s, int mode, const double p[3]);
double or_dist_in(const or_solid* s, const double p[3], const double d[3], unsigned* diag);
double or_dist_out(const or_solid* s, const double p[3], const double d[3], unsigned* diag);
/* as above; *t_suspect receives the start of the first ill-conditioned interval */
double or_dist_in_ex(const or_solid* s, const double p[3], const double d[3], unsigned* diag,
                     double* t_suspect);
double or_dist_out_ex(const or_solid* s, const double p[3], const double d[3], unsigned* diag,
                      double* t_suspect);
int or_roots(const or_solid* s, const double p[3], const double d[3], double* roots);
/* Conditioning of a finite hit at t > 0 along p + t d: returns 1 when
 * 16 eps L / |cos theta| > 1e-12 max(t, 1 mm), with eps = 2^-52,
 * L = (|p|^2 + |q|^2) / max(1 mm, |q|) (the scale of the coordinates and of the
 * quadric's constant term |p|^2 - R^2), q = p + t d, and cos theta = n.d / |n|
 * with n the central-difference gradient of the signed term at q
 * (h = 1e-6 max(1 mm, |q|inf)). */
int or_hit_cond(const or_solid* s, const double p[3], const double d[3], double t);

/* ---------------------------------------------------------------- geometry */
typedef struct {
  int n_lv, n_pv, n_place, world_lv, max_depth;
  or_solid* lv_solid;
  int* pv_lv;
  int* pv_parent;
  int* pv_depth;
  double* pv_xf;   /* 12 per PV: R (row major) and t, relative to the parent */
  int* pv_child_off; /* CSR over PVs, children in ascending id order */
  int* pv_child;
} or_geom;

int or_geom_load(const void* blob, size_t nbytes, or_geom** out);
void or_geom_free(or_geom* g);

void or_to_local(const or_geom* g, int pv, const double p[3], const double d[3], double pl[3],
                 double dl[3]);
int or_locate(const or_geom* g, const double p[3]);
double or_compute_step(const or_geom* g, const double p[3], const double d[3], int pv,
                       double pstep, int* next, unsigned* flags, unsigned* diag);
double or_nav_safety(const or_geom* g, const double p[3], int pv);
int or_nav_inside(const or_geom* g, const double p[3], int pv);
int or_transport(const or_geom* g, const double p0[3], const double d[3], int start_pv,
                 int max_steps, int32_t* out_pv, double* out_step, unsigned* flags,
                 unsigned* diag);

/* ------------------------------------------------------ physics-limited steps */
typedef struct {
  int n_mat, n_proc;
  const double* density; /* [n_mat] number density n of each material */
  const double* sigma;   /* [n_mat][n_proc] cross section of each process */
  const int* lv_mat;     /* [n_lv] material of each logical volume */
} or_phys;

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double or_uniform(uint64_t seed, uint32_t track, uint32_t step, uint32_t proc);
double or_phys_length(const or_phys* ph, int mat, uint64_t seed, uint32_t track, uint32_t step, int* proc);
int or_transport_phys(const or_geom* g, const or_phys* ph, const double p0[3], const double d[3],
                      int start_pv, int max_steps, uint64_t seed, uint32_t track, int32_t* out_pv,
                      double* out_step, int8_t* out_proc, unsigned* flags, unsigned* diag);

#endif
