/*
 * CPU ORACLE (test infrastructure only) -- geometry hierarchy and navigation.
 *
 * Hierarchy (paper Sec. III.B): logical volumes hold one solid and an ordered
 * list of daughter placements; the placed-volume tree is their DFS pre-order
 * expansion from the world, so a PV id is a complete navigation state.
 *
 * Step selection (paper Sec. III.A): the particle moves by the proposed
 * physics length unless the geometric border is nearer, in which case it is
 * transported to the border and continues in the next volume.  The geometric
 * border is the nearest of the mother's DistanceToOut and every daughter's
 * DistanceToIn.  Tracking of a particle ends when it leaves the geometry.
 *
 * Readings fixed here (the paper does not state them):
 *   - ties between daughters go to the lowest daughter index, and a daughter
 *     beats the mother's exit on equality;
 *   - after leaving a daughter the track continues in the mother with no
 *     relocation search (a touching neighbour is entered by a 0-length step);
 *   - the local point is recomputed from the global point every step by
 *     applying the placements root to leaf;
 *   - a track stops after max_steps steps (OVERFLOW) or after 8 consecutive
 *     steps shorter than kTolerance (STUCK).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* ------------------------------------------------------------ blob parse */
static int rd_i32(const unsigned char* b, size_t off) {
  int32_t v;
  memcpy(&v, b + off, 4);
  return v;
}
static double rd_f64(const unsigned char* b, size_t off) {
  double v;
  memcpy(&v, b + off, 8);
  return v;
}

#define OR_MAX_DEPTH 32
#define OR_MAX_PV (1 << 24)

typedef struct {
  int n_lv;
  const int* place_off;
  const int* place_cnt;
  const int* place_child;
} lvtab;

static long count_pvs(const lvtab* t, int lv, int depth, int* maxdepth) {
  if (depth > OR_MAX_DEPTH) return -1;
  if (depth > *maxdepth) *maxdepth = depth;
  long n = 1;
  for (int k = 0; k < t->place_cnt[lv]; ++k) {
    long c = count_pvs(t, t->place_child[t->place_off[lv] + k], depth + 1, maxdepth);
    if (c < 0) return -1;
    n += c;
    if (n > OR_MAX_PV) return -1;
  }
  return n;
}

typedef struct {
  or_geom* g;
  const lvtab* t;
  const double* place_xf;
  int next;
  int child_fill;
} expander;

static void expand(expander* e, int lv, int parent, const double* xf, int depth) {
  or_geom* g = e->g;
  int me = e->next++;
  g->pv_lv[me] = lv;
  g->pv_parent[me] = parent;
  g->pv_depth[me] = depth;
  memcpy(&g->pv_xf[12 * me], xf, 12 * sizeof(double));
  int nch = e->t->place_cnt[lv];
  int off = e->child_fill;
  g->pv_child_off[me] = off;
  e->child_fill += nch;
  for (int k = 0; k < nch; ++k) {
    int pl = e->t->place_off[lv] + k;
    g->pv_child[off + k] = e->next;
    expand(e, e->t->place_child[pl], me, &e->place_xf[12 * pl], depth + 1);
  }
}

int or_geom_load(const void* blob, size_t nbytes, or_geom** out) {
  const unsigned char* b = (const unsigned char*)blob;
  static const unsigned char magic[8] = {'G', 'V', 'G', 'E', 'O', 'M', 0, 1};
  *out = NULL;
  if (nbytes < 32 || memcmp(b, magic, 8) != 0) return -4;
  int version = rd_i32(b, 8), n_lv = rd_i32(b, 12), n_place = rd_i32(b, 16);
  int n_param = rd_i32(b, 20), world = rd_i32(b, 24);
  if (version != 1 || n_lv <= 0 || n_place < 0 || n_param < 0 || world < 0 || world >= n_lv)
    return -4;
  size_t need = 32 + (size_t)n_lv * 32 + (size_t)n_place * 104 + (size_t)n_param * 8;
  if (need != nbytes) return -4;
  size_t lv_off = 32, pl_off = lv_off + (size_t)n_lv * 32, pa_off = pl_off + (size_t)n_place * 104;

  int* place_off = calloc(n_lv, sizeof(int));
  int* place_cnt = calloc(n_lv, sizeof(int));
  int* place_child = calloc(n_place ? n_place : 1, sizeof(int));
  double* place_xf = calloc(n_place ? (size_t)n_place * 12 : 1, sizeof(double));
  double* params = calloc(n_param ? n_param : 1, sizeof(double));
  or_geom* g = calloc(1, sizeof(or_geom));
  int rc = -4;
  if (!place_off || !place_cnt || !place_child || !place_xf || !params || !g) {
    rc = -2;
    goto fail;
  }
  for (int i = 0; i < n_param; ++i) params[i] = rd_f64(b, pa_off + 8 * (size_t)i);
  g->lv_solid = calloc(n_lv, sizeof(or_solid));
  if (!g->lv_solid) {
    rc = -2;
    goto fail;
  }
  g->n_lv = n_lv; /* lets or_geom_free release composites on failure */
  for (int i = 0; i < n_lv; ++i) {
    size_t o = lv_off + 32 * (size_t)i;
    int type = rd_i32(b, o), poff = rd_i32(b, o + 4), pcnt = rd_i32(b, o + 8);
    place_off[i] = rd_i32(b, o + 12);
    place_cnt[i] = rd_i32(b, o + 16);
    if (poff < 0 || pcnt < 0 || (long)poff + pcnt > n_param) goto fail;
    if (place_off[i] < 0 || place_cnt[i] < 0 || (long)place_off[i] + place_cnt[i] > n_place)
      goto fail;
    if (or_solid_init(&g->lv_solid[i], type, params + poff, pcnt) != 0) goto fail;
  }
  for (int k = 0; k < n_place; ++k) {
    size_t o = pl_off + 104 * (size_t)k;
    place_child[k] = rd_i32(b, o);
    if (place_child[k] < 0 || place_child[k] >= n_lv) goto fail;
    for (int j = 0; j < 12; ++j) place_xf[12 * k + j] = rd_f64(b, o + 8 + 8 * (size_t)j);
  }
  lvtab t = {n_lv, place_off, place_cnt, place_child};
  int maxdepth = 0;
  long npv = count_pvs(&t, world, 0, &maxdepth);
  if (npv < 0) goto fail;
  g->n_lv = n_lv;
  g->n_pv = (int)npv;
  g->n_place = n_place;
  g->world_lv = world;
  g->max_depth = maxdepth;
  g->pv_lv = calloc(npv, sizeof(int));
  g->pv_parent = calloc(npv, sizeof(int));
  g->pv_depth = calloc(npv, sizeof(int));
  g->pv_xf = calloc((size_t)npv * 12, sizeof(double));
  g->pv_child_off = calloc(npv + 1, sizeof(int));
  g->pv_child = calloc(npv, sizeof(int));
  if (!g->pv_lv || !g->pv_parent || !g->pv_depth || !g->pv_xf || !g->pv_child_off ||
      !g->pv_child) {
    rc = -2;
    goto fail;
  }
  double ident[12] = {1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0};
  expander e = {g, &t, place_xf, 0, 0};
  expand(&e, world, -1, ident, 0);
  g->pv_child_off[npv] = e.child_fill;
  free(place_off);
  free(place_cnt);
  free(place_child);
  free(place_xf);
  free(params);
  *out = g;
  return 0;
fail:
  free(place_off);
  free(place_cnt);
  free(place_child);
  free(place_xf);
  free(params);
  or_geom_free(g);
  return rc;
}

void or_geom_free(or_geom* g) {
  if (!g) return;
  if (g->lv_solid)
    for (int i = 0; i < g->n_lv; ++i) or_solid_release(&g->lv_solid[i]);
  free(g->lv_solid);
  free(g->pv_lv);
  free(g->pv_parent);
  free(g->pv_depth);
  free(g->pv_xf);
  free(g->pv_child_off);
  free(g->pv_child);
  free(g);
}

/* ------------------------------------------------------------ transforms */
/* x_child = R^T (x_parent - t) for points, R^T x for directions */
static void to_child(const double* xf, const double p[3], const double d[3], double pc[3],
                     double dc[3]) {
  const double* R = xf;
  double q0 = p[0] - xf[9], q1 = p[1] - xf[10], q2 = p[2] - xf[11];
  for (int i = 0; i < 3; ++i) {
    pc[i] = R[0 + i] * q0 + R[3 + i] * q1 + R[6 + i] * q2;
    if (d) dc[i] = R[0 + i] * d[0] + R[3 + i] * d[1] + R[6 + i] * d[2];
  }
}

void or_to_local(const or_geom* g, int pv, const double p[3], const double d[3], double pl[3],
                 double dl[3]) {
  int path[OR_MAX_DEPTH + 2];
  int n = 0;
  for (int v = pv; v >= 0; v = g->pv_parent[v]) path[n++] = v;
  double cp[3] = {p[0], p[1], p[2]}, cd[3] = {0, 0, 0};
  if (d) {
    cd[0] = d[0];
    cd[1] = d[1];
    cd[2] = d[2];
  }
  /* path[n-1] is the world, whose frame is the global frame */
  for (int k = n - 2; k >= 0; --k) {
    double np[3], nd[3];
    to_child(&g->pv_xf[12 * path[k]], cp, d ? cd : NULL, np, nd);
    cp[0] = np[0];
    cp[1] = np[1];
    cp[2] = np[2];
    if (d) {
      cd[0] = nd[0];
      cd[1] = nd[1];
      cd[2] = nd[2];
    }
  }
  pl[0] = cp[0];
  pl[1] = cp[1];
  pl[2] = cp[2];
  if (d) {
    dl[0] = cd[0];
    dl[1] = cd[1];
    dl[2] = cd[2];
  }
}

static const or_solid* pv_solid(const or_geom* g, int pv) { return &g->lv_solid[g->pv_lv[pv]]; }

/* --------------------------------------------------------------- queries */
int or_locate(const or_geom* g, const double p[3]) {
  if (or_inside(pv_solid(g, 0), p) == OR_OUTSIDE) return -1;
  int pv = 0;
  double pl[3] = {p[0], p[1], p[2]};
  for (;;) {
    int found = -1;
    double pc[3];
    for (int k = g->pv_child_off[pv]; k < g->pv_child_off[pv + 1]; ++k) {
      int c = g->pv_child[k];
      to_child(&g->pv_xf[12 * c], pl, NULL, pc, NULL);
      if (or_inside(pv_solid(g, c), pc) != OR_OUTSIDE) {
        found = c;
        break;
      }
    }
    if (found < 0) return pv;
    pv = found;
    pl[0] = pc[0];
    pl[1] = pc[1];
    pl[2] = pc[2];
  }
}

double or_compute_step(const or_geom* g, const double p[3], const double d[3], int pv,
                       double pstep, int* next, unsigned* flags, unsigned* diag) {
  double pl[3], dl[3];
  or_to_local(g, pv, p, d, pl, dl);
  unsigned dg = 0;
  double sus_out = INFINITY;
  double dout = or_dist_out_ex(pv_solid(g, pv), pl, dl, &dg, &sus_out);
  if (dout < 0.0) {
    dout = 0.0;
    *flags |= OR_F_LOCATE_FAIL;
  }
  unsigned dg_out = dg;
  /* two smallest finite candidate lengths, for the near-tie diagnostic */
  double c1 = INFINITY, c2 = INFINITY;
#define PUSH_CAND(v)            \
  do {                          \
    double v_ = (v);            \
    if (v_ < c1) {              \
      c2 = c1;                  \
      c1 = v_;                  \
    } else if (v_ < c2) {       \
      c2 = v_;                  \
    }                           \
  } while (0)
  PUSH_CAND(dout);
  if (isfinite(pstep)) PUSH_CAND(pstep);
  double best = INFINITY;
  int bestc = -1;
  double sus_min = sus_out;
  unsigned dg_all = 0;
  int edge_any = 0;
  for (int k = g->pv_child_off[pv]; k < g->pv_child_off[pv + 1]; ++k) {
    int c = g->pv_child[k];
    double pc[3], dc[3];
    to_child(&g->pv_xf[12 * c], pl, dl, pc, dc);
    unsigned dk = 0;
    double sus = INFINITY;
    double t = or_dist_in_ex(pv_solid(g, c), pc, dc, &dk, &sus);
    if (t < 0.0) {
      t = 0.0;
      *flags |= OR_F_LOCATE_FAIL;
    }
    if (dk & OR_D_BAND_EDGE) edge_any = 1;
    if (sus < sus_min) sus_min = sus;
    dg_all |= dk;
    PUSH_CAND(t);
    if (t < best) {
      best = t;
      bestc = c;
    }
  }
#undef PUSH_CAND
  double step;
  if (pstep < best && pstep < dout) {
    step = pstep;
    *next = pv;
  } else if (best <= dout) {
    step = best;
    *next = bestc;
  } else {
    step = dout;
    *next = g->pv_parent[pv];
  }
  if (isfinite(c2) && c2 - c1 < OR_KTOL) *diag |= OR_D_NEAR_TIE;
  if (step < OR_KTOL) *diag |= OR_D_ZERO_STEP;
  /* an ill-conditioned interval matters only if it starts before the border */
  if (sus_min <= step + OR_KTOL) *diag |= OR_D_GRAZE;
  if (edge_any || (dg_out & OR_D_BAND_EDGE)) *diag |= OR_D_BAND_EDGE;
  if ((dg_out | dg_all) & OR_D_NO_EXIT) *diag |= OR_D_NO_EXIT;
  return step;
}

double or_nav_safety(const or_geom* g, const double p[3], int pv) {
  double pl[3];
  or_to_local(g, pv, p, NULL, pl, NULL);
  const or_solid* ms = pv_solid(g, pv);
  if (or_inside(ms, pl) != OR_INSIDE) return 0.0;
  double s = or_safety_out(ms, pl);
  for (int k = g->pv_child_off[pv]; k < g->pv_child_off[pv + 1]; ++k) {
    int c = g->pv_child[k];
    double pc[3];
    to_child(&g->pv_xf[12 * c], pl, NULL, pc, NULL);
    const or_solid* cs = pv_solid(g, c);
    if (or_inside(cs, pc) != OR_OUTSIDE) return 0.0;
    double v = or_safety_in(cs, pc);
    if (v < s) s = v;
  }
  return s > 0.0 ? s : 0.0;
}

int or_nav_inside(const or_geom* g, const double p[3], int pv) {
  double pl[3];
  or_to_local(g, pv, p, NULL, pl, NULL);
  return or_inside(pv_solid(g, pv), pl);
}

int or_transport(const or_geom* g, const double p0[3], const double d[3], int start_pv,
                 int max_steps, int32_t* out_pv, double* out_step, unsigned* flags,
                 unsigned* diag) {
  double p[3] = {p0[0], p0[1], p0[2]};
  int pv = start_pv;
  out_pv[0] = pv;
  if (pv < 0) return 0;
  int zero_run = 0, k = 0;
  for (k = 0; k < max_steps; ++k) {
    int next = -1;
    double step = or_compute_step(g, p, d, pv, INFINITY, &next, flags, diag);
    p[0] = p[0] + step * d[0];
    p[1] = p[1] + step * d[1];
    p[2] = p[2] + step * d[2];
    out_step[k] = step;
    out_pv[k + 1] = next;
    if (next < 0) return k + 1;
    zero_run = (step < OR_KTOL) ? zero_run + 1 : 0;
    if (zero_run >= 8) {
      *flags |= OR_F_STUCK;
      return k + 1;
    }
    pv = next;
  }
  *flags |= OR_F_OVERFLOW;
  return max_steps;
}
