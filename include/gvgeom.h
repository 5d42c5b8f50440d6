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

enum { GV_OK = 0, GV_EINVAL = -1, GV_ENOMEM = -2, GV_EHIP = -3, GV_EFORMAT = -4, GV_ESTATE = -5, GV_EAGAIN = -6 };

/* Inside codes (int8) */
enum { GV_OUTSIDE = 0, GV_SURFACE = 1, GV_INSIDE = 2 };
/* basket_distance direction */
enum { GV_TO_IN = 0, GV_TO_OUT = 1 };
/* basket_safety side */
enum { GV_SAFETY_AUTO = 0, GV_SAFETY_IN = 1, GV_SAFETY_OUT = 2 };
/* Arithmetic of the navigation entry points.  GV_FP32_REFINE screens the
 * daughters of box- and tube-daughter volumes in FP32 (bounding-box slab test
 * and a SafetyToIn lower bound, on FP32 copies of the tables, with rounding
 * margins that keep both conservative) and computes every surviving distance
 * in FP64, so its outputs equal those of GV_FP64 bit for bit; a wavefront whose
 * points lie outside the range the FP32 margins cover falls back to the FP64
 * screens.  (The paper, Sec. III.C, describes vectorised solid and navigation
 * code; it names no precision.  The mixed form is this library's own.) */
enum { GV_FP64 = 0, GV_FP32_REFINE = 1 };
/* per-track transport flags */
#define GV_FLAG_OVERFLOW 1u    /* max_steps reached before leaving the world */
#define GV_FLAG_STUCK 2u       /* 8 consecutive steps shorter than kTolerance */
#define GV_FLAG_LOCATE_FAIL 4u /* point found outside its volume or inside a daughter */

/* Solid types of the geometry blob: 0 box, 1 tube segment, 2 cone segment,
 * 3 sphere shell, 4 trapezoid (Trd), 5 polycone (Sec. III.B elementary solids),
 * 6 composite: union, A minus C or intersection of two solids of types 0-5, A
 * at the composite's origin and C placed by a rotation and translation
 * (Sec. III.B: complex elements built with Boolean operations).  A composite's
 * Inside code composes its parts' signed terms (union the smaller, intersection
 * the larger, A minus C the larger of s_A and -s_C); its distances follow the
 * Boolean combination of the parts' pieces along the ray under the elementary
 * solids' kTolerance rules; its safeties are bounds composed from the parts'. */

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
 * inside its volume or not strictly outside every daughter.  precision GV_FP64
 * or GV_FP32_REFINE (same values). */
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
 * precision GV_FP64 or GV_FP32_REFINE (same outputs).
 * 1 <= max_steps <= 4096.  The library keeps a device workspace inside `g`,
 * grown on demand (hipMalloc) and freed by geom_free; concurrent calls on the
 * same `g` from several streams are not allowed (GV_ESTATE is not detected).
 * The call only enqueues: for 8,192 or more tracks it enqueues every step up
 * to max_steps (steps past the longest track find an empty list and cost one
 * dispatch each), so it never waits for the device and may be captured into
 * a HIP graph.  Under stream capture nothing is allocated: GV_ESTATE unless
 * an earlier call outside the capture has sized the workspace for at least n
 * tracks (and GV_ESTATE while profiling events are on). */
int nav_transport(gv_geom* g, int64_t n, const double* x, const double* y, const double* z,
                  const double* dx, const double* dy, const double* dz, const int32_t* start_pv,
                  int32_t max_steps, int32_t* out_pv, double* out_step, int32_t* out_nsteps,
                  uint32_t* out_flags, int32_t precision, void* stream);

/* Allocation-free nav_transport, for callers that cannot allocate device
 * memory: code under HIP graph capture, serving loops, harnesses that forbid
 * allocation.  Same arguments, definitions and outputs as nav_transport (its
 * lane form, whatever the tuned transport field says), but the keys, order and
 * counters live in a static device array of the library, 16.06 MiB per device
 * and held until the process ends, so the call allocates nothing and needs no
 * earlier call.  1 <= n <= 2,097,152 (GV_EINVAL beyond; n == 0 is a no-op).
 * Every call on one device shares that device's array, which keeps the last
 * call's contents; each call clears what must start at zero.  Calls that
 * overlap on one device (several streams or threads) race on the array and
 * must be serialised by the caller.  No profiling events or work counters
 * (gv_profile) are recorded. */
int nav_transport_noalloc(gv_geom* g, int64_t n, const double* x, const double* y, const double* z,
                          const double* dx, const double* dy, const double* dz, const int32_t* start_pv,
                          int32_t max_steps, int32_t* out_pv, double* out_step, int32_t* out_nsteps,
                          uint32_t* out_flags, int32_t precision, void* stream);

/* ------------------------------------------------- physics-limited transport */
/* Materials for physics-limited steps: n_mat materials with number density
 * density[m] and, for each of n_proc (1..16) processes, a cross section
 * sigma[m][p] (host arrays, row-major), and the material of every logical
 * volume, lv_material[n_lv].  The mean free path of process p in material m is
 * 1 / (density[m] sigma[m][p]) (Sec. III, Eq. (1)); units such that it comes out
 * in mm.  Copied to the device; replaces earlier tables.  Errors: GV_EINVAL for
 * negative or non-finite values or a material index out of range. */
int geom_set_materials(gv_geom* g, int32_t n_mat, int32_t n_proc, const double* density, const double* sigma,
                       const int32_t* lv_material);

#define GV_PHYS_SAFETY_SHORTCUT 1 /* nav_transport_phys option */

/* Transport with physics-limited steps (Sec. III.A with Eqs. (1)-(3): the process with the shortest
 * sampled interaction length acts unless the border is nearer; the lengths are
 * drawn again in every volume).  At step k of track i every process p draws
 * s_p = -ln(u) / (density sigma_p) of the current volume's material, u in
 * (0, 1) from Philox4x32-10 (Salmon et al., SC'11) with counter (i, k, p, 0) and
 * key (seed & 0xffffffff, seed >> 32), u = ((w0 << 32 | w1) >> 11 + 0.5) 2^-53
 * of the first two output words; the shortest is the proposed step of
 * basket_step.  The direction does not change (no physics action).  Outputs as
 * nav_transport, plus out_proc [n][max_steps] int8 (nullable): the process of
 * a physics-limited step, -1 for a step that ends on a boundary.  Option
 * GV_PHYS_SAFETY_SHORTCUT takes a physics step without any geometry when it is
 * shorter (by kTolerance) than the distance still to go along the unchanged
 * direction to the boundary found by the last full step; the outputs do not
 * change.  GV_ESTATE without materials. */
int nav_transport_phys(gv_geom* g, int64_t n, const double* x, const double* y, const double* z,
                       const double* dx, const double* dy, const double* dz, const int32_t* start_pv,
                       int32_t max_steps, uint64_t seed, int32_t* out_pv, double* out_step, int8_t* out_proc,
                       int32_t* out_nsteps, uint32_t* out_flags, int32_t options, int32_t precision, void* stream);

/* ------------------------------------------------------------ measurement */

/* Measurement.  flags GV_PROF_EVENTS: nav_transport records a pair of HIP
 * events on the caller's stream around every launch of its transport kernel
 * (the persistent lane kernel, or each step kernel of the basket form: the
 * production kernels, so the times are those of unprofiled calls).
 * GV_PROF_WORK: transports of 8,192 tracks or more run the basket form with
 * the per-step kernel instance that keeps operation counters (a ballot and an
 * LDS atomic per counted event, so slower; geometries without composites
 * only; every track takes the same steps with the same work in both forms),
 * and basket_distance / basket_solid_all on a polycone are followed by a
 * kernel that counts their walks' work (outputs untouched).  0 turns both off.
 * gv_profile_read waits for the events and returns the summed
 * kernel milliseconds and the number of launches since the last read (then
 * forgets them), and, if `work` is not NULL, a host array of 33 uint64: the
 * operation counts of the last basket transport run with GV_PROF_WORK, then
 * those of the polycone queries since the last read ([28] sections whose cone
 * intersections DistanceToIn walks computed, [29] the same for DistanceToOut,
 * [30] DistanceToIn rays rejected by the bounding cylinder, [31] DistanceToIn
 * walks, [32] DistanceToOut walks; then cleared).  Transport counters: [0] steps taken, [1] daughter
 * bounding-box tests, [2+t] daughter lower-bound checks, [8+t] daughter
 * DistanceToIn evaluations in culled loops (and radial walks), [14+t]
 * DistanceToIn evaluations in plain loops, t = daughter solid type 0..5
 * (composites are not counted there), [20] track-steps of culled loops
 * screened in FP32, [21] those screened in FP64, [22] physics-limited steps,
 * [23] of which taken by the safety short-cut, [24] steps in an LV whose
 * daughters are walked in radial order, [25] crossing-parameter bounds of
 * those walks, [26] steps whose daughters came from phi sectors, [27] sector
 * masks read).  Reading synchronises the device. */
#define GV_PROF_EVENTS 1
#define GV_PROF_WORK 2
int gv_profile(gv_geom* g, int flags);
int gv_profile_read(gv_geom* g, double* step_ms, int64_t* step_launches, uint64_t* work);

/* Roof probes (measurement only; device pointers, enqueued on `stream`).
 * gv_probe_stream: c[i] = a[i] + s b[i] for i < n (n even, arrays 16-byte
 * aligned), 24 n bytes of HBM traffic; with b NULL the copy c[i] = a[i],
 * 16 n bytes.  gv_probe_fma64: n_lanes lanes (a positive multiple of 256)
 * each run eight independent chains of `iters` FP64 fused multiply-adds
 * (8 iters n_lanes FMAs = 16 iters n_lanes flops) and store one double to
 * out[lane]. */
int gv_probe_stream(const double* a, const double* b, double* c, double s, int64_t n, void* stream);
int gv_probe_fma64(double* out, int64_t n_lanes, int32_t iters, void* stream);

/* ---------------------------------------------------------- launch shapes */
/* How the library's kernels are launched on this geometry.  These choose the
 * form of the transport, workgroup counts and sizes, the coarse direction
 * cells of the orderings and the register budget of the per-step kernel; none
 * of them changes any result (every track's arithmetic is the same), only
 * speed.  An autotuner measures them per device architecture (the Python
 * package's tune module) and the binding applies the stored choice at load.
 *
 * The transports have two forms.  The lane form (default) orders the tracks
 * once by a direction key (counting sort into 2^sort_bits x 2^sort_bits
 * direction cells), then one
 * persistent kernel carries each track in one lane from its start to its end,
 * wavefronts taking 64 places of the order at a time from an atomic counter.
 * The basket form (Sec. II.A baskets of tracks in the same volume) regroups
 * the live tracks by (logical volume, direction cell) before every step.
 * Fields (0 = the default; cell_bits and sort_bits -1 = the default):
 *   step_grid     workgroups of the per-step basket kernel, 1..1024
 *                 (default one per four tiles of 64 tracks, at most 1024);
 *   scatter_grid  workgroups of the regrouping kernels, 1..1024
 *                 (default one per 4,096 tracks, at most 256);
 *   cell_bits     0, 2 or 4: 1, 2 x 2 or 4 x 4 direction cells per logical
 *                 volume in the regrouping key (default 2; ignored when
 *                 volumes x cells would exceed 4,096);
 *   solid_block   threads per workgroup of the one-lane-per-track kernels
 *                 (solid-level queries, basket_step/_locate/_nav_*, small
 *                 transports), a multiple of 64 in 64..1024 (default 256);
 *   solid_grid    at most this many workgroups for those kernels (each lane
 *                 then loops over several tracks), >= 1 (default: one lane
 *                 per track);
 *   step_waves    3 or 4: waves per SIMD the navigation step kernel is built
 *                 for (default 4);
 *   transport     1 basket form, 2 lane form (default: lane, or basket for
 *                 geometries holding composites; the basket form needs
 *                 n >= 8,192, smaller batches take the lane form);
 *   sort_bits     0..7: the lane form's direction cells are 2^sort_bits x
 *                 2^sort_bits (0: no ordering, tracks in index order;
 *                 default 7);
 *   sort_key      1 octahedral cells in Morton order, 2 z-axis cells (cos
 *                 theta bands x azimuth sectors, bands outermost) (default 1);
 *   lane_waves    3 or 4: waves per SIMD the lane kernel is built for
 *                 (default 4; 3 for physics-limited transport);
 *   lane_stage    1 off, 2 on: the lane kernel stages 8 steps of outputs in
 *                 LDS before writing a track's rows (default on);
 *   lane_grid     workgroups (256 threads) of the persistent lane kernel,
 *                 >= 0 (default: as many as the device holds at once);
 *   lane_sched    1: every live lane of a wavefront takes a step in every
 *                 iteration; 2: only the lanes whose volume is in the step
 *                 class (solid type and daughter access) most of the
 *                 wavefront's live lanes are in take a step, the others wait,
 *                 so lanes that fell behind catch up (default 2; geometries
 *                 with composites always 1).
 * A change of cell_bits re-sizes the transport workspace at the next
 * transport.  GV_EINVAL for a field out of range (nothing changed). */
typedef struct {
  int32_t step_grid, scatter_grid, cell_bits, solid_block, solid_grid, step_waves;
  int32_t transport, sort_bits, sort_key, lane_waves, lane_stage, lane_grid, lane_sched;
} gv_tuning;
int gv_set_tuning(gv_geom* g, const gv_tuning* t);
int gv_get_tuning(const gv_geom* g, gv_tuning* t);

/* --------------------------------------------------------------- serving */
/* A serving engine answers baskets of navigation queries that arrive over
 * time.  The paper's scheduler gathers tracks into baskets and hands each full
 * basket to the vectorised geometry code (Sec. II.A item 1, Sec. III.C); here
 * clients hand in baskets, and every basket waiting when a stream falls idle
 * is answered by one round: one copy of the round's inputs per contiguous run,
 * ONE fused kernel over all of its queries, one copy back per run.
 *
 * Host byte layout of one basket of n tracks (packed, in this order):
 *   GV_Q_STEP    in : x y z dx dy dz pstep (n double each), pv (n int32)   60 n bytes
 *                out: step (n double), next_pv (n int32), flags (n uint32) 16 n bytes
 *   GV_Q_SAFETY  in : x y z (n double each), pv (n int32)                  28 n bytes
 *                out: safety (n double)                                     8 n bytes
 *   GV_Q_INSIDE  in : as GV_Q_SAFETY;  out: Inside code (n int8)              n bytes
 * The answers are those of basket_step (pstep = +inf: no physics limit),
 * basket_nav_safety and basket_nav_inside, in the basket's precision.
 *
 * The engine runs on the calling thread only, inside submit, poll and drain
 * (no background thread); one server is used from one thread at a time.  A
 * server must be destroyed before its geometry.  After a GV_EHIP return the
 * server should only be destroyed. */
typedef struct gv_server gv_server;
enum { GV_Q_STEP = 0, GV_Q_SAFETY = 1, GV_Q_INSIDE = 2 };

/* Creates a server on the geometry's device: at most `slots` (1..1024)
 * baskets admitted and not yet returned, an HBM arena of `hbm_budget` bytes
 * (64 KiB .. 1 TiB; 4/5 for inputs, 1/5 for outputs, one hipMalloc here and
 * none later) with a pinned host mirror of the same size, and `nstreams`
 * (1..8) streams, so up to nstreams rounds are in flight.  options
 * GV_SERVE_GRAPH: every round is one launch of a HIP graph instantiated here
 * per stream (two input-copy runs, the descriptor copy, the fused kernel, two
 * output-copy runs), its node parameters set for the round; without it a
 * round is enqueued as plain copies and a launch.  The answers are the same. */
#define GV_SERVE_GRAPH 1
int gv_server_create(gv_geom* g, int32_t slots, int64_t hbm_budget, int32_t nstreams, int32_t options,
                     gv_server** out);

/* Admits one basket (n >= 1 tracks; kind GV_Q_*; precision GV_FP64 or
 * GV_FP32_REFINE).  `in` (host, layout above) is copied into pinned staging
 * before the call returns; `out` (host, layout above) must stay valid until
 * gv_server_poll returns this basket's *ticket, and is written then.
 * GV_EAGAIN: all slots taken or no contiguous room in an arena (nothing
 * admitted); slots and room come back only through gv_server_poll or
 * gv_server_drain, so poll and retry.  GV_EINVAL: the basket can never fit the
 * budget.  The basket is launched at once if a stream is idle (as last seen by
 * a poll), else with the next round. */
int gv_server_submit(gv_server* s, int32_t kind, int32_t precision, int64_t n, const void* in, void* out,
                     uint64_t* ticket);

/* Non-blocking.  Completes every finished round (outputs written to the
 * callers' buffers, slots and arena space released), launches waiting baskets,
 * and returns up to `max` completed tickets in completion order, with
 * t_done[i] (nullable) the device completion time of the ticket's round on the
 * gv_now() clock (mapped from HIP events). */
int gv_server_poll(gv_server* s, int32_t max, uint64_t* tickets, double* t_done, int32_t* count);

/* Blocks until every admitted basket has completed (tickets still come from
 * gv_server_poll). */
int gv_server_drain(gv_server* s);

/* out[0..7] = admitted, waiting (not yet launched), rounds launched, baskets
 * launched, tracks launched, largest round (baskets), input-arena bytes held,
 * output-arena bytes held. */
int gv_server_stats(const gv_server* s, int64_t* out);

/* Drains, then frees the server's memory, streams and events.  NULL is a no-op. */
int gv_server_destroy(gv_server* s);

/* Seconds on the monotonic clock that gv_server_poll's times use. */
double gv_now(void);

/* Thread-local text of the last error on this thread ("" if none). */
const char* gv_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
