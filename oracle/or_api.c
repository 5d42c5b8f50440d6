/*
 * CPU ORACLE (test infrastructure only) -- batch entry points for ctypes.
 * Each call evaluates independent tracks one at a time; `nthreads` only
 * spreads them over host cores in static chunks of 4096 tracks.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>

#include "oracle.h"

#define CHUNK 4096

static int nthr(int nthreads) { return nthreads > 0 ? nthreads : 1; }

int orc_solid_check(int type, const double* params, int np) {
  or_solid s;
  const int rc = or_solid_init(&s, type, params, np);
  if (rc == 0) or_solid_release(&s);
  return rc;
}

int orc_solid_signed(int type, const double* params, int np, int64_t n, const double* x,
                     const double* y, const double* z, double* out, int nthreads) {
  or_solid s;
  if (or_solid_init(&s, type, params, np)) return -1;
#pragma omp parallel for schedule(static, CHUNK) num_threads(nthr(nthreads))
  for (int64_t i = 0; i < n; ++i) {
    double p[3] = {x[i], y[i], z[i]};
    out[i] = or_signed(&s, p);
  }
  or_solid_release(&s);
  return 0;
}

int orc_solid_inside(int type, const double* params, int np, int64_t n, const double* x,
                     const double* y, const double* z, int8_t* out, int nthreads) {
  or_solid s;
  if (or_solid_init(&s, type, params, np)) return -1;
#pragma omp parallel for schedule(static, CHUNK) num_threads(nthr(nthreads))
  for (int64_t i = 0; i < n; ++i) {
    double p[3] = {x[i], y[i], z[i]};
    out[i] = (int8_t)or_inside(&s, p);
  }
  or_solid_release(&s);
  return 0;
}

int orc_solid_safety(int type, const double* params, int np, int mode, int64_t n,
                     const double* x, const double* y, const double* z, double* out,
                     int nthreads) {
  or_solid s;
  if (mode < 0 || mode > 2) return -1;
  if (or_solid_init(&s, type, params, np)) return -1;
#pragma omp parallel for schedule(static, CHUNK) num_threads(nthr(nthreads))
  for (int64_t i = 0; i < n; ++i) {
    double p[3] = {x[i], y[i], z[i]};
    out[i] = or_safety(&s, mode, p);
  }
  or_solid_release(&s);
  return 0;
}

int orc_solid_distance(int type, const double* params, int np, int dir, int64_t n,
                       const double* x, const double* y, const double* z, const double* dx,
                       const double* dy, const double* dz, double* out, uint32_t* diag,
                       int nthreads) {
  or_solid s;
  if (dir != 0 && dir != 1) return -1;
  if (or_solid_init(&s, type, params, np)) return -1;
#pragma omp parallel for schedule(static, CHUNK) num_threads(nthr(nthreads))
  for (int64_t i = 0; i < n; ++i) {
    double p[3] = {x[i], y[i], z[i]}, d[3] = {dx[i], dy[i], dz[i]};
    unsigned dg = 0;
    out[i] = dir == 0 ? or_dist_in(&s, p, d, &dg) : or_dist_out(&s, p, d, &dg);
    if (or_hit_cond(&s, p, d, out[i])) dg |= OR_D_COND;
    if (diag) diag[i] = dg;
  }
  or_solid_release(&s);
  return 0;
}

int orc_solid_roots(int type, const double* params, int np, const double* p, const double* d,
                    double* roots, int cap) {
  or_solid s;
  if (or_solid_init(&s, type, params, np)) return -1;
  double R[OR_MAX_ROOTS];
  int n = or_roots(&s, p, d, R);
  for (int i = 0; i < n && i < cap; ++i) roots[i] = R[i];
  or_solid_release(&s);
  return n;
}

void* orc_geom_load(const void* blob, int64_t nbytes, int* status) {
  or_geom* g = NULL;
  *status = or_geom_load(blob, (size_t)nbytes, &g);
  return g;
}

void orc_geom_free(void* h) { or_geom_free((or_geom*)h); }

int orc_geom_info(void* h, int32_t* out) {
  or_geom* g = (or_geom*)h;
  out[0] = g->n_lv;
  out[1] = g->n_pv;
  out[2] = g->max_depth;
  out[3] = g->world_lv;
  return 0;
}

int orc_geom_pv_table(void* h, int32_t* lv, int32_t* parent, int32_t* depth) {
  or_geom* g = (or_geom*)h;
  for (int i = 0; i < g->n_pv; ++i) {
    lv[i] = g->pv_lv[i];
    parent[i] = g->pv_parent[i];
    depth[i] = g->pv_depth[i];
  }
  return 0;
}

int orc_to_local(void* h, int64_t n, const double* x, const double* y, const double* z,
                 const int32_t* pv, double* out /* 3n */) {
  or_geom* g = (or_geom*)h;
  for (int64_t i = 0; i < n; ++i) {
    double p[3] = {x[i], y[i], z[i]}, pl[3];
    if (pv[i] < 0 || pv[i] >= g->n_pv) return -1;
    or_to_local(g, pv[i], p, NULL, pl, NULL);
    out[3 * i] = pl[0];
    out[3 * i + 1] = pl[1];
    out[3 * i + 2] = pl[2];
  }
  return 0;
}

int orc_locate(void* h, int64_t n, const double* x, const double* y, const double* z,
               int32_t* out, int nthreads) {
  or_geom* g = (or_geom*)h;
#pragma omp parallel for schedule(static, CHUNK) num_threads(nthr(nthreads))
  for (int64_t i = 0; i < n; ++i) {
    double p[3] = {x[i], y[i], z[i]};
    out[i] = or_locate(g, p);
  }
  return 0;
}

int orc_step(void* h, int64_t n, const double* x, const double* y, const double* z,
             const double* dx, const double* dy, const double* dz, const int32_t* pv,
             const double* pstep, double* out_step, int32_t* out_next, uint32_t* out_flags,
             uint32_t* out_diag, int nthreads) {
  or_geom* g = (or_geom*)h;
  for (int64_t i = 0; i < n; ++i)
    if (pv[i] < 0 || pv[i] >= g->n_pv) return -1;
#pragma omp parallel for schedule(static, CHUNK) num_threads(nthr(nthreads))
  for (int64_t i = 0; i < n; ++i) {
    double p[3] = {x[i], y[i], z[i]}, d[3] = {dx[i], dy[i], dz[i]};
    unsigned fl = 0, dg = 0;
    int next = -1;
    out_step[i] = or_compute_step(g, p, d, pv[i], pstep ? pstep[i] : INFINITY, &next, &fl, &dg);
    out_next[i] = next;
    if (out_flags) out_flags[i] = fl;
    if (out_diag) out_diag[i] = dg;
  }
  return 0;
}

int orc_nav_safety(void* h, int64_t n, const double* x, const double* y, const double* z,
                   const int32_t* pv, double* out, int nthreads) {
  or_geom* g = (or_geom*)h;
  for (int64_t i = 0; i < n; ++i)
    if (pv[i] < 0 || pv[i] >= g->n_pv) return -1;
#pragma omp parallel for schedule(static, CHUNK) num_threads(nthr(nthreads))
  for (int64_t i = 0; i < n; ++i) {
    double p[3] = {x[i], y[i], z[i]};
    out[i] = or_nav_safety(g, p, pv[i]);
  }
  return 0;
}

int orc_nav_inside(void* h, int64_t n, const double* x, const double* y, const double* z,
                   const int32_t* pv, int8_t* out, int nthreads) {
  or_geom* g = (or_geom*)h;
  for (int64_t i = 0; i < n; ++i)
    if (pv[i] < 0 || pv[i] >= g->n_pv) return -1;
#pragma omp parallel for schedule(static, CHUNK) num_threads(nthr(nthreads))
  for (int64_t i = 0; i < n; ++i) {
    double p[3] = {x[i], y[i], z[i]};
    out[i] = (int8_t)or_nav_inside(g, p, pv[i]);
  }
  return 0;
}

/* out_pv: n x (max_steps + 1), out_step: n x max_steps, row per track */
int orc_transport(void* h, int64_t n, const double* x, const double* y, const double* z,
                  const double* dx, const double* dy, const double* dz, const int32_t* start_pv,
                  int max_steps, int32_t* out_pv, double* out_step, int32_t* out_nsteps,
                  uint32_t* out_flags, uint32_t* out_diag, int nthreads) {
  or_geom* g = (or_geom*)h;
  if (max_steps < 1) return -1;
  if (start_pv)
    for (int64_t i = 0; i < n; ++i)
      if (start_pv[i] < -1 || start_pv[i] >= g->n_pv) return -1;
#pragma omp parallel for schedule(static, 256) num_threads(nthr(nthreads))
  for (int64_t i = 0; i < n; ++i) {
    double p[3] = {x[i], y[i], z[i]}, d[3] = {dx[i], dy[i], dz[i]};
    unsigned fl = 0, dg = 0;
    int pv0 = start_pv ? start_pv[i] : or_locate(g, p);
    int32_t* rp = out_pv + (size_t)i * (max_steps + 1);
    double* rs = out_step + (size_t)i * max_steps;
    int k = or_transport(g, p, d, pv0, max_steps, rp, rs, &fl, &dg);
    out_nsteps[i] = k;
    if (out_flags) out_flags[i] = fl;
    if (out_diag) out_diag[i] = dg;
  }
  return 0;
}

/* Philox4x32-10 block (for its known-answer checks) and the uniform draw */
void orc_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out) { or_philox4x32_10(ctr, key, out); }
double orc_uniform(uint64_t seed, uint32_t track, uint32_t step, uint32_t proc) {
  return or_uniform(seed, track, step, proc);
}

/* Shortest sampled interaction length for each (material, track, step) triple */
int orc_phys_length(int n_mat, int n_proc, const double* density, const double* sigma, int64_t n,
                    const int32_t* mat, uint64_t seed, const uint32_t* track, const uint32_t* step, double* out,
                    int32_t* out_proc) {
  or_phys ph = {n_mat, n_proc, density, sigma, NULL};
  for (int64_t i = 0; i < n; ++i) {
    if (mat[i] < 0 || mat[i] >= n_mat) return -1;
    int pr = -1;
    out[i] = or_phys_length(&ph, mat[i], seed, track[i], step[i], &pr);
    out_proc[i] = pr;
  }
  return 0;
}

/* Physics-limited transport; track i draws with counter track = track_id[i]
 * (track_id NULL: i), so a sample of a batch draws what it drew in the batch.
 * out_proc: n x max_steps int8 (nullable): process of a physics-limited step,
 * -1 for a step that ends on a boundary. */
int orc_transport_phys(void* h, int n_mat, int n_proc, const double* density, const double* sigma,
                       const int32_t* lv_mat, int64_t n, const double* x, const double* y, const double* z,
                       const double* dx, const double* dy, const double* dz, const int32_t* start_pv, int max_steps,
                       uint64_t seed, const uint32_t* track_id, int32_t* out_pv, double* out_step, int8_t* out_proc, int32_t* out_nsteps,
                       uint32_t* out_flags, uint32_t* out_diag, int nthreads) {
  or_geom* g = (or_geom*)h;
  if (max_steps < 1 || n_mat < 1 || n_proc < 1) return -1;
  for (int i = 0; i < g->n_lv; ++i)
    if (lv_mat[i] < 0 || lv_mat[i] >= n_mat) return -1;
  if (start_pv)
    for (int64_t i = 0; i < n; ++i)
      if (start_pv[i] < -1 || start_pv[i] >= g->n_pv) return -1;
  or_phys ph = {n_mat, n_proc, density, sigma, lv_mat};
#pragma omp parallel for schedule(static, 256) num_threads(nthr(nthreads))
  for (int64_t i = 0; i < n; ++i) {
    double p[3] = {x[i], y[i], z[i]}, d[3] = {dx[i], dy[i], dz[i]};
    unsigned fl = 0, dg = 0;
    int pv0 = start_pv ? start_pv[i] : or_locate(g, p);
    int32_t* rp = out_pv + (size_t)i * (max_steps + 1);
    double* rs = out_step + (size_t)i * max_steps;
    int8_t* rq = out_proc ? out_proc + (size_t)i * max_steps : NULL;
    const uint32_t tid = track_id ? track_id[i] : (uint32_t)i;
    int k = or_transport_phys(g, &ph, p, d, pv0, max_steps, seed, tid, rp, rs, rq, &fl, &dg);
    out_nsteps[i] = k;
    if (out_flags) out_flags[i] = fl;
    if (out_diag) out_diag[i] = dg;
  }
  return 0;
}

int orc_max_threads(void) { return omp_get_max_threads(); }
