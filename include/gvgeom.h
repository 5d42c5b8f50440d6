/*
 * gvgeom -- batched geometry queries and basket navigation on MI355X (gfx950).
 *
 * The paper (Sec. III.C) states the geometry work of particle transport as three
 * questions asked for every particle: is it inside or outside a solid, what is
 * its minimal distance to the solid's border, and how far may it travel along
 * its direction.  Particles located in the same kind of volume are collected into
 * baskets and processed together (Sec. II.A, item 1 "Scheduler"; Sec. III.C).
 * A particle is moved by the proposed physics length unless the border of its
 * volume is nearer, in which case it is transported to the border and continues
 * in the next volume (Sec. III.A); the detector is a hierarchy of elementary
 * solids placed with rotations and translations (Sec. III.B).
 *
 * This header is the whole boundary.  Every entry point:
 *   - takes plain pointers and sizes; basket arrays are DEVICE pointers (HBM),
 *     structure-of-arrays, one element per track, owned by the caller, 8-byte
 *     aligned for double and 4-byte aligned for int32, disjoint between inputs
 *     and outputs;
 *   - only enqueues work on `stream` (a hipStream_t, NULL = the default stream)
 *     and returns; outputs are valid after the caller synchronises the stream;
 *   - returns GV_OK (0) or a negative GV_E* code, and on error sets a
 *     thread-local message readable with gv_last_error(); nothing is enqueued
 *     when an argument check fails; n == 0 is a no-op returning GV_OK;
 *   - never aborts and never throws across the boundary.
 *
 * Units are mm.  kTolerance = 1e-9 mm; a point is on a surface when its signed
 * distance-like term s lies in [-kTolerance/2, +kTolerance/2].
 */
#ifndef GVGEOM_H
#define GVGEOM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gv_geom gv_geom; /* opaque, device resident, owned by the library */

enum { GV_OK = 0, GV_EINVAL = -1, GV_ENOMEM = -2, GV_EHIP = -3, GV_EFORMAT = -4, GV_ESTATE = -5 };

/* Inside codes (int8) */
enum { GV_OUTSIDE = 0, GV_SURFACE = 1, GV_INSIDE = 2 };
/* basket_distance direction */
enum { GV_TO_IN = 0, GV_TO_OUT = 1 };
/* basket_safety side */
enum { GV_SAFETY_AUTO = 0, GV_SAFETY_IN = 1, GV_SAFETY_OUT = 2 };
/* arithmetic of the navigation entry points */
enum { GV_FP64 = 0, GV_FP32_REFINE = 1 };
/* per-track transport flags */
#define GV_FLAG_OVERFLOW 1u    /* max_steps reached before leaving the world */
#define GV_FLAG_STUCK 2u       /* 8 consecutive steps shorter than kTolerance */
#define GV_FLAG_LOCATE_FAIL 4u /* point found outside its volume or inside a daughter */

/* Solid types of the geometry blob: 0 box, 1 tube segment, 2 cone segment,
 * 3 sphere shell, 4 trapezoid (Trd), 5 polycone (Sec. III.B elementary solids). */

/* ------------------------------------------------------------------ geometry */

/* Parse a geometry blob (host memory, `nbytes` long, format version 1: logical
 * volumes with solid parameters and ordered daughter placements x_mother =
 * R x_child + t) and upload it to the current device.  Placed volumes are the
 * DFS pre-order expansion from the world LV; PV 0 is the world (Sec. III.B
 * hierarchy).  The blob is only read during the call.  On success *out owns
 * device memory until geom_free.  Errors: GV_EFORMAT for a malformed blob or an
 * invalid solid, GV_ENOMEM, GV_EHIP. */
int geom_load(const void* blob, size_t nbytes, gv_geom** out);

/* Release a geometry and its workspaces.  Synchronises the device first.
 * NULL is accepted (no-op). */
int geom_free(gv_geom* g);

/* counts[0..3] = number of LVs, number of PVs, maximum depth, world LV
 * (host pointer to 4 int32). */
int geom_info(const gv_geom* g, int32_t* counts);

/* ------------------------------------------------------- solid-level queries */
/* Points/directions are in the local frame of logical volume `lv`'s solid. */

/* Inside code of each point (Sec. III.C question 1): out[i] = GV_INSIDE,
 * GV_SURFACE or GV_OUTSIDE (int8). */
int basket_inside(gv_geom* g, int32_t lv, int64_t n, const double* x, const double* y,
                  const double* z, int8_t* out, void* stream);

/* Minimal distance to the solid's border (Sec. III.C question 2) as each solid's
 * fixed lower-bound formula (exact for box/Trd/sphere/polycone from inside and
 * for sphere/polycone from outside).  side GV_SAFETY_AUTO: 0 on the surface,
 * SafetyToOut inside, SafetyToIn outside; GV_SAFETY_IN (point expected outside)
 * and GV_SAFETY_OUT (expected inside) return -1 on the wrong side and 0 on the
 * surface.  out_inside (nullable) receives the Inside code computed on the way.
 * precision must be GV_FP64. */
int basket_safety(gv_geom* g, int32_t lv, int32_t side, int64_t n, const double* x,
                  const double* y, const double* z, double* out_safety, int8_t* out_inside,
                  int32_t precision, void* stream);

/* Distance along the unit direction (Sec. III.C question 3): dir GV_TO_IN gives
 * DistanceToIn (-1 for inside points, +inf on a miss), GV_TO_OUT gives
 * DistanceToOut (-1 for outside points).  A point on the surface leaving
 * (entering) the solid gets DistanceToOut (DistanceToIn) 0.  Stretches of the
 * ray inside or outside the solid shorter than kTolerance are ignored.
 * Directions must be unit vectors (not renormalised).  precision GV_FP64. */
int basket_distance(gv_geom* g, int32_t lv, int32_t dir, int64_t n, const double* x,
                    const double* y, const double* z, const double* dx, const double* dy,
                    const double* dz, double* out, int32_t precision, void* stream);

/* All four answers in one pass over the basket (input read once): any output
 * pointer may be NULL to skip it.  Same definitions as above. */
int basket_solid_all(gv_geom* g, int32_t lv, int64_t n, const double* x, const double* y,
                     const double* z, const double* dx, const double* dy, const double* dz,
                     int8_t* out_inside, double* out_safety, double* out_dist_in,
                     double* out_dist_out, void* stream);

/* ------------------------------------------------------ navigation queries */
/* Points/directions are global; pv[i] is the track's placed volume (its full
 * navigation state). */

/* Deepest placed volume holding each point: descends from the world into the
 * first daughter (lowest index) whose Inside code is not GV_OUTSIDE.  -1 when
 * the point is outside the world. */
int basket_locate(gv_geom* g, int64_t n, const double* x, const double* y, const double* z,
                  int32_t* out_pv, void* stream);

/* ComputeStep (Sec. III.A step selection): step = min(pstep, DistanceToOut of
 * the current volume, DistanceToIn of every daughter).  out_next_pv = pv when
 * the physics length wins, the daughter entered (ties: lowest daughter index;
 * a daughter wins a tie with the exit), else the parent, or -1 when leaving the
 * world.  pstep NULL means +inf.  precision GV_FP64 or GV_FP32_REFINE.
 * Errors: GV_EINVAL for a pv outside [0, n_pv) is NOT checked per track on the
 * device; such tracks get out_next_pv = -1, step 0, flags LOCATE_FAIL via
 * out_flags (nullable). */
int basket_step(gv_geom* g, int64_t n, const double* x, const double* y, const double* z,
                const double* dx, const double* dy, const double* dz, const int32_t* pv,
                const double* pstep, double* out_step, int32_t* out_next_pv,
                uint32_t* out_flags, int32_t precision, void* stream);

/* Isotropic safety of each point in its volume: max(0, min(SafetyToOut of the
 * volume, SafetyToIn of every daughter)); 0 when the point is not strictly
 * inside its volume or not strictly outside every daughter. */
int basket_nav_safety(gv_geom* g, int64_t n, const double* x, const double* y, const double* z,
                      const int32_t* pv, double* out, int32_t precision, void* stream);

/* Inside code of each point against the solid of its own placed volume. */
int basket_nav_inside(gv_geom* g, int64_t n, const double* x, const double* y, const double* z,
                      const int32_t* pv, int8_t* out, void* stream);

/* Transport every track along its straight line until it leaves the world
 * (Sec. III.A: tracking ends when the particle leaves the geometry), with no
 * physics limit.  start_pv NULL: locate first.  Outputs (device, row per track):
 *   out_pv    [n][max_steps+1] int32: entry 0 = start PV, entry k = volume after
 *             step k (-1 = left the world); entries past out_nsteps untouched;
 *   out_step  [n][max_steps] double: step lengths;
 *   out_nsteps[n] int32, out_flags[n] uint32 (GV_FLAG_*).
 * 1 <= max_steps <= 4096.  The library keeps a device workspace inside `g`,
 * grown on demand (hipMalloc) and freed by geom_free; concurrent calls on the
 * same `g` from several streams are not allowed (GV_ESTATE is not detected). */
int nav_transport(gv_geom* g, int64_t n, const double* x, const double* y, const double* z,
                  const double* dx, const double* dy, const double* dz, const int32_t* start_pv,
                  int32_t max_steps, int32_t* out_pv, double* out_step, int32_t* out_nsteps,
                  uint32_t* out_flags, int32_t precision, void* stream);

/* ------------------------------------------------------------ measurement */

/* Kernel timing for measurement.  While enabled, nav_transport records a pair
 * of HIP events on the caller's stream around every launch of its per-step
 * kernel.  gv_profile_read waits for those events and returns the summed
 * kernel milliseconds and the number of launches since the last read (then
 * forgets them), and, if `work` is not NULL, the operation counts of the last
 * basket transport (host array of 20 uint64: [0] steps taken, [1] daughter
 * bounding-box tests, [2+t] daughter lower-bound checks, [8+t] daughter
 * DistanceToIn evaluations in culled loops, [14+t] DistanceToIn evaluations in
 * plain loops, t = daughter solid type 0..5).  Reading synchronises the device. */
int gv_profile(gv_geom* g, int enable);
int gv_profile_read(gv_geom* g, double* step_ms, int64_t* step_launches, uint64_t* work);

/* Thread-local text of the last error on this thread ("" if none). */
const char* gv_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
