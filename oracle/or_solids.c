/*
 * CPU ORACLE (test infrastructure only) -- elementary solids.
 *
 * The three per-particle questions of the paper (Sec. III.C) for one solid:
 * Inside (three-way code), Safety (distance to the border, as a lower bound
 * formula fixed per solid), and DistanceToIn / DistanceToOut along a direction.
 * The solids are the paper's "rectangular solids and tubes" (Sec. III.B) plus
 * the rest of the basic set: cone segment, sphere shell, trapezoid (Trd) and
 * polycone.
 *
 * Conventions (readings where the paper is silent):
 *   kTolerance = 1e-9 mm; a point is on the surface when |s| <= kTolerance/2,
 *   where s is the solid's signed term (max over its bounding surfaces of the
 *   signed distance-like term, > 0 outside).  DistanceToIn of an inside point
 *   and DistanceToOut of an outside point are -1; a miss is +inf.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static double dmax(double a, double b) { return a > b ? a : b; }
static double dmin(double a, double b) { return a < b ? a : b; }

int or_code(double s) {
  if (s < -OR_KHALF) return OR_INSIDE;
  if (s > OR_KHALF) return OR_OUTSIDE;
  return OR_SURFACE;
}

/* ------------------------------------------------------------------ setup */
static void phi_init(or_solid* s, double sphi, double dphi) {
  const double two_pi = 2.0 * M_PI;
  if (dphi >= two_pi) {
    s->full_phi = 1;
    return;
  }
  double pe = sphi + dphi;
  s->full_phi = 0;
  s->convex_wedge = dphi <= M_PI;
  /* outward normals of the two bounding half-planes and their in-plane
   * directions away from the z axis */
  s->ns[0] = sin(sphi);
  s->ns[1] = -cos(sphi);
  s->ne[0] = -sin(pe);
  s->ne[1] = cos(pe);
  s->us[0] = cos(sphi);
  s->us[1] = sin(sphi);
  s->ue[0] = cos(pe);
  s->ue[1] = sin(pe);
}

int or_solid_init(or_solid* s, int type, const double* q, int nq) {
  memset(s, 0, sizeof *s);
  s->type = type;
  for (int i = 0; i < nq && i < 8; ++i) s->p[i] = q[i];
  switch (type) {
    case OR_BOX:
      if (nq != 3 || !(q[0] > 0 && q[1] > 0 && q[2] > 0)) return -1;
      return 0;
    case OR_TUBS:
      if (nq != 5 || !(q[0] >= 0 && q[1] > q[0] && q[2] > 0 && q[4] > 0)) return -1;
      phi_init(s, q[3], q[4]);
      return 0;
    case OR_CONS: {
      if (nq != 7) return -1;
      double rmin1 = q[0], rmax1 = q[1], rmin2 = q[2], rmax2 = q[3], dz = q[4];
      if (!(rmin1 >= 0 && rmax1 >= rmin1 && rmin2 >= 0 && rmax2 >= rmin2 && rmax1 + rmax2 > 0 &&
            dz > 0 && q[6] > 0))
        return -1;
      s->ao = 0.5 * (rmax1 + rmax2);
      s->bo = (rmax2 - rmax1) / (2.0 * dz);
      s->co = 1.0 / sqrt(1.0 + s->bo * s->bo);
      s->ai = 0.5 * (rmin1 + rmin2);
      s->bi = (rmin2 - rmin1) / (2.0 * dz);
      s->ci = 1.0 / sqrt(1.0 + s->bi * s->bi);
      s->has_inner = rmin1 > 0 || rmin2 > 0;
      phi_init(s, q[5], q[6]);
      return 0;
    }
    case OR_SPHERE:
      if (nq != 2 || !(q[0] >= 0 && q[1] > q[0])) return -1;
      return 0;
    case OR_TRD: {
      if (nq != 5 || !(q[0] > 0 && q[1] > 0 && q[2] > 0 && q[3] > 0 && q[4] > 0)) return -1;
      double dz = q[4];
      s->x0 = 0.5 * (q[0] + q[1]);
      s->tx = (q[1] - q[0]) / (2.0 * dz);
      s->cx = 1.0 / sqrt(1.0 + s->tx * s->tx);
      s->y0 = 0.5 * (q[2] + q[3]);
      s->ty = (q[3] - q[2]) / (2.0 * dz);
      s->cy = 1.0 / sqrt(1.0 + s->ty * s->ty);
      return 0;
    }
    case OR_PCON: {
      if (nq < 1) return -1;
      int nz = (int)q[0];
      if (nz < 2 || nz > OR_MAX_NZ || nq != 1 + 3 * nz || (double)nz != q[0]) return -1;
      s->nz = nz;
      for (int j = 0; j < nz; ++j) {
        s->z[j] = q[1 + j];
        s->rmin[j] = q[1 + nz + j];
        s->rmax[j] = q[1 + 2 * nz + j];
        if (!(s->rmin[j] >= 0 && s->rmax[j] >= s->rmin[j])) return -1;
        if (j > 0 && !(s->z[j] > s->z[j - 1])) return -1;
      }
      for (int j = 0; j + 1 < nz; ++j) {
        double h = s->z[j + 1] - s->z[j];
        if (!(s->rmax[j] + s->rmax[j + 1] > 0)) return -1;
        s->pc_bo[j] = (s->rmax[j + 1] - s->rmax[j]) / h;
        s->pc_co[j] = 1.0 / sqrt(1.0 + s->pc_bo[j] * s->pc_bo[j]);
        s->pc_bi[j] = (s->rmin[j + 1] - s->rmin[j]) / h;
        s->pc_ci[j] = 1.0 / sqrt(1.0 + s->pc_bi[j] * s->pc_bi[j]);
        s->pc_inner[j] = s->rmin[j] > 0 || s->rmin[j + 1] > 0;
      }
      return 0;
    }
    case OR_BOOL:
      return or_bool_init(s, q, nq);
  }
  return -1;
}

void or_solid_release(or_solid* s) {
  if (s->type == OR_BOOL && s->comp) {
    or_solid_release(&s->comp[0]);
    or_solid_release(&s->comp[1]);
    free(s->comp);
    s->comp = NULL;
  }
}

/* ------------------------------------------------------------ signed term */
static double phi_term(const or_solid* s, double x, double y) {
  double a = x * s->ns[0] + y * s->ns[1];
  double b = x * s->ne[0] + y * s->ne[1];
  /* wedge <= pi is the intersection of the two half-spaces, wider wedges the union */
  return s->convex_wedge ? dmax(a, b) : dmin(a, b);
}

static int pcon_section(const or_solid* s, double z) {
  int j = 0;
  for (int k = 0; k + 1 < s->nz; ++k)
    if (s->z[k] <= z) j = k;
  return j;
}

double or_signed(const or_solid* s, const double p[3]) {
  double x = p[0], y = p[1], z = p[2];
  switch (s->type) {
    case OR_BOX:
      return dmax(dmax(fabs(x) - s->p[0], fabs(y) - s->p[1]), fabs(z) - s->p[2]);
    case OR_TUBS: {
      double r = sqrt(x * x + y * y);
      double t = r - s->p[1];
      if (s->p[0] > 0) t = dmax(t, s->p[0] - r);
      t = dmax(t, fabs(z) - s->p[2]);
      if (!s->full_phi) t = dmax(t, phi_term(s, x, y));
      return t;
    }
    case OR_CONS: {
      double r = sqrt(x * x + y * y);
      double t = (r - (s->ao + s->bo * z)) * s->co;
      if (s->has_inner) t = dmax(t, ((s->ai + s->bi * z) - r) * s->ci);
      t = dmax(t, fabs(z) - s->p[4]);
      if (!s->full_phi) t = dmax(t, phi_term(s, x, y));
      return t;
    }
    case OR_SPHERE: {
      double rho = sqrt(x * x + y * y + z * z);
      double t = rho - s->p[1];
      if (s->p[0] > 0) t = dmax(t, s->p[0] - rho);
      return t;
    }
    case OR_TRD: {
      double t = (fabs(x) - (s->x0 + s->tx * z)) * s->cx;
      t = dmax(t, (fabs(y) - (s->y0 + s->ty * z)) * s->cy);
      return dmax(t, fabs(z) - s->p[4]);
    }
    case OR_PCON: {
      int j = pcon_section(s, z);
      double r = sqrt(x * x + y * y);
      double zl = z - s->z[j];
      double t = (r - (s->rmax[j] + s->pc_bo[j] * zl)) * s->pc_co[j];
      if (s->pc_inner[j]) t = dmax(t, ((s->rmin[j] + s->pc_bi[j] * zl) - r) * s->pc_ci[j]);
      t = dmax(t, s->z[0] - z);
      return dmax(t, z - s->z[s->nz - 1]);
    }
    case OR_BOOL:
      return or_bool_signed(s, p);
  }
  return NAN;
}

int or_inside(const or_solid* s, const double p[3]) { return or_code(or_signed(s, p)); }

/* ---------------------------------------------------------------- safety */
static double half_plane_dist(const double n[2], const double u[2], double x, double y, double r) {
  /* distance from (x,y,z) to the half-plane {q : q.n = 0, q.u >= 0} */
  if (x * u[0] + y * u[1] >= 0.0) return fabs(x * n[0] + y * n[1]);
  return r;
}

static double seg_dist(double r, double z, double r1, double z1, double r2, double z2) {
  double er = r2 - r1, ez = z2 - z1;
  double wr = r - r1, wz = z - z1;
  double ll = er * er + ez * ez;
  double u = 0.0;
  if (ll > 0.0) {
    u = (wr * er + wz * ez) / ll;
    if (u < 0.0) u = 0.0;
    if (u > 1.0) u = 1.0;
  }
  double qr = r1 + u * er - r, qz = z1 + u * ez - z;
  return sqrt(qr * qr + qz * qz);
}

/* Exact distance in the meridian half-plane to the polycone's boundary
 * polygon (lateral segments, inner segments off the axis, two end caps). */
static double pcon_boundary_dist(const or_solid* s, const double p[3]) {
  double r = sqrt(p[0] * p[0] + p[1] * p[1]), z = p[2];
  int nz = s->nz;
  double best = INFINITY;
  for (int j = 0; j + 1 < nz; ++j) {
    best = dmin(best, seg_dist(r, z, s->rmax[j], s->z[j], s->rmax[j + 1], s->z[j + 1]));
    if (s->rmin[j] > 0 || s->rmin[j + 1] > 0)
      best = dmin(best, seg_dist(r, z, s->rmin[j], s->z[j], s->rmin[j + 1], s->z[j + 1]));
  }
  best = dmin(best, seg_dist(r, z, s->rmin[0], s->z[0], s->rmax[0], s->z[0]));
  best = dmin(best, seg_dist(r, z, s->rmin[nz - 1], s->z[nz - 1], s->rmax[nz - 1], s->z[nz - 1]));
  return best;
}

double or_safety_out(const or_solid* s, const double p[3]) {
  double x = p[0], y = p[1], z = p[2];
  switch (s->type) {
    case OR_BOX:
      return dmin(dmin(s->p[0] - fabs(x), s->p[1] - fabs(y)), s->p[2] - fabs(z));
    case OR_TUBS: {
      double r = sqrt(x * x + y * y);
      double m = s->p[1] - r;
      if (s->p[0] > 0) m = dmin(m, r - s->p[0]);
      m = dmin(m, s->p[2] - fabs(z));
      if (!s->full_phi) {
        m = dmin(m, half_plane_dist(s->ns, s->us, x, y, r));
        m = dmin(m, half_plane_dist(s->ne, s->ue, x, y, r));
      }
      return m;
    }
    case OR_CONS: {
      double r = sqrt(x * x + y * y);
      double m = ((s->ao + s->bo * z) - r) * s->co;
      if (s->has_inner) m = dmin(m, (r - (s->ai + s->bi * z)) * s->ci);
      m = dmin(m, s->p[4] - fabs(z));
      if (!s->full_phi) {
        m = dmin(m, half_plane_dist(s->ns, s->us, x, y, r));
        m = dmin(m, half_plane_dist(s->ne, s->ue, x, y, r));
      }
      return m;
    }
    case OR_SPHERE: {
      double rho = sqrt(x * x + y * y + z * z);
      double m = s->p[1] - rho;
      if (s->p[0] > 0) m = dmin(m, rho - s->p[0]);
      return m;
    }
    case OR_TRD: {
      double m = ((s->x0 + s->tx * z) - fabs(x)) * s->cx;
      m = dmin(m, ((s->y0 + s->ty * z) - fabs(y)) * s->cy);
      return dmin(m, s->p[4] - fabs(z));
    }
    case OR_PCON:
      return pcon_boundary_dist(s, p);
    case OR_BOOL:
      return or_bool_safety_out(s, p);
  }
  return NAN;
}

double or_safety_in(const or_solid* s, const double p[3]) {
  double x = p[0], y = p[1], z = p[2];
  switch (s->type) {
    case OR_BOX:
      return dmax(dmax(fabs(x) - s->p[0], fabs(y) - s->p[1]), fabs(z) - s->p[2]);
    case OR_TUBS:
    case OR_CONS: {
      double r = sqrt(x * x + y * y);
      double m;
      if (s->type == OR_TUBS) {
        m = r - s->p[1];
        if (s->p[0] > 0) m = dmax(m, s->p[0] - r);
        m = dmax(m, fabs(z) - s->p[2]);
      } else {
        m = (r - (s->ao + s->bo * z)) * s->co;
        if (s->has_inner) m = dmax(m, ((s->ai + s->bi * z) - r) * s->ci);
        m = dmax(m, fabs(z) - s->p[4]);
      }
      if (!s->full_phi && phi_term(s, x, y) > 0.0) {
        double w = dmin(half_plane_dist(s->ns, s->us, x, y, r), half_plane_dist(s->ne, s->ue, x, y, r));
        m = dmax(m, w);
      }
      return m;
    }
    case OR_SPHERE: {
      double rho = sqrt(x * x + y * y + z * z);
      double m = rho - s->p[1];
      if (s->p[0] > 0) m = dmax(m, s->p[0] - rho);
      return m;
    }
    case OR_TRD: {
      double m = (fabs(x) - (s->x0 + s->tx * z)) * s->cx;
      m = dmax(m, (fabs(y) - (s->y0 + s->ty * z)) * s->cy);
      return dmax(m, fabs(z) - s->p[4]);
    }
    case OR_PCON:
      return pcon_boundary_dist(s, p);
    case OR_BOOL:
      return or_bool_safety_in(s, p);
  }
  return NAN;
}

double or_safety(const or_solid* s, int mode, const double p[3]) {
  int c = or_inside(s, p);
  if (mode == OR_SAFETY_IN) {
    if (c == OR_INSIDE) return -1.0;
    if (c == OR_SURFACE) return 0.0;
    return dmax(0.0, or_safety_in(s, p));
  }
  if (mode == OR_SAFETY_OUT) {
    if (c == OR_OUTSIDE) return -1.0;
    if (c == OR_SURFACE) return 0.0;
    return dmax(0.0, or_safety_out(s, p));
  }
  if (c == OR_SURFACE) return 0.0;
  if (c == OR_INSIDE) return dmax(0.0, or_safety_out(s, p));
  return dmax(0.0, or_safety_in(s, p));
}

/* ----------------------------------------------------------------- roots */
static int add_root(double* R, int n, double t) {
  if (t > 0.0 && isfinite(t)) R[n++] = t;
  return n;
}

/* A t^2 + 2 B t + C = 0, cancellation-free pair t1 = q/A, t2 = C/q */
static int quad_roots(double* R, int n, double A, double B, double C) {
  if (A == 0.0) {
    if (B != 0.0) n = add_root(R, n, -C / (2.0 * B));
    return n;
  }
  double D = B * B - A * C;
  if (D < 0.0) return n;
  double sq = sqrt(D);
  double q = (B >= 0.0) ? -(B + sq) : -(B - sq);
  if (q == 0.0) return n; /* double root at t = 0 */
  n = add_root(R, n, q / A);
  n = add_root(R, n, C / q);
  return n;
}

static int plane_root(double* R, int n, double nx, double ny, double nz, double c, const double p[3],
                      const double d[3]) {
  double den = nx * d[0] + ny * d[1] + nz * d[2];
  if (den == 0.0) return n;
  double num = c - (nx * p[0] + ny * p[1] + nz * p[2]);
  return add_root(R, n, num / den);
}

static int cyl_roots(double* R, int n, double rad, const double p[3], const double d[3]) {
  double A = d[0] * d[0] + d[1] * d[1];
  double B = p[0] * d[0] + p[1] * d[1];
  double C = p[0] * p[0] + p[1] * p[1] - rad * rad;
  return quad_roots(R, n, A, B, C);
}

/* full double cone x^2 + y^2 = (a + b (z - z0))^2 */
static int cone_roots(double* R, int n, double a, double b, double z0, const double p[3],
                      const double d[3]) {
  double rz = a + b * (p[2] - z0);
  double A = d[0] * d[0] + d[1] * d[1] - b * b * d[2] * d[2];
  double B = p[0] * d[0] + p[1] * d[1] - b * rz * d[2];
  double C = p[0] * p[0] + p[1] * p[1] - rz * rz;
  return quad_roots(R, n, A, B, C);
}

static int sph_roots(double* R, int n, double rad, const double p[3], const double d[3]) {
  double A = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  double B = p[0] * d[0] + p[1] * d[1] + p[2] * d[2];
  double C = p[0] * p[0] + p[1] * p[1] + p[2] * p[2] - rad * rad;
  return quad_roots(R, n, A, B, C);
}

static int phi_roots(const or_solid* s, double* R, int n, const double p[3], const double d[3]) {
  if (s->full_phi) return n;
  n = plane_root(R, n, s->ns[0], s->ns[1], 0.0, 0.0, p, d);
  n = plane_root(R, n, s->ne[0], s->ne[1], 0.0, 0.0, p, d);
  return n;
}

int or_roots(const or_solid* s, const double p[3], const double d[3], double* R) {
  int n = 0;
  switch (s->type) {
    case OR_BOX:
      for (int a = 0; a < 3; ++a) {
        double nv[3] = {0, 0, 0};
        nv[a] = 1.0;
        n = plane_root(R, n, nv[0], nv[1], nv[2], s->p[a], p, d);
        n = plane_root(R, n, nv[0], nv[1], nv[2], -s->p[a], p, d);
      }
      return n;
    case OR_TUBS:
      n = cyl_roots(R, n, s->p[1], p, d);
      if (s->p[0] > 0) n = cyl_roots(R, n, s->p[0], p, d);
      n = plane_root(R, n, 0, 0, 1, s->p[2], p, d);
      n = plane_root(R, n, 0, 0, 1, -s->p[2], p, d);
      return phi_roots(s, R, n, p, d);
    case OR_CONS:
      n = cone_roots(R, n, s->ao, s->bo, 0.0, p, d);
      if (s->has_inner) n = cone_roots(R, n, s->ai, s->bi, 0.0, p, d);
      n = plane_root(R, n, 0, 0, 1, s->p[4], p, d);
      n = plane_root(R, n, 0, 0, 1, -s->p[4], p, d);
      return phi_roots(s, R, n, p, d);
    case OR_SPHERE:
      n = sph_roots(R, n, s->p[1], p, d);
      if (s->p[0] > 0) n = sph_roots(R, n, s->p[0], p, d);
      return n;
    case OR_TRD:
      /* x = +-(x0 + tx z), y = +-(y0 + ty z), z = +-dz */
      n = plane_root(R, n, 1.0, 0.0, -s->tx, s->x0, p, d);
      n = plane_root(R, n, -1.0, 0.0, -s->tx, s->x0, p, d);
      n = plane_root(R, n, 0.0, 1.0, -s->ty, s->y0, p, d);
      n = plane_root(R, n, 0.0, -1.0, -s->ty, s->y0, p, d);
      n = plane_root(R, n, 0, 0, 1, s->p[4], p, d);
      n = plane_root(R, n, 0, 0, 1, -s->p[4], p, d);
      return n;
    case OR_PCON:
      for (int j = 0; j + 1 < s->nz; ++j) {
        n = cone_roots(R, n, s->rmax[j], s->pc_bo[j], s->z[j], p, d);
        if (s->pc_inner[j]) n = cone_roots(R, n, s->rmin[j], s->pc_bi[j], s->z[j], p, d);
      }
      n = plane_root(R, n, 0, 0, 1, s->z[0], p, d);
      n = plane_root(R, n, 0, 0, 1, s->z[s->nz - 1], p, d);
      return n;
    case OR_BOOL:
      return or_bool_roots(s, p, d, R);
  }
  return 0;
}

/* ------------------------------------------------------- event-list rule */
static void sort_small(double* a, int n) {
  for (int i = 1; i < n; ++i) {
    double v = a[i];
    int j = i - 1;
    while (j >= 0 && a[j] > v) {
      a[j + 1] = a[j];
      --j;
    }
    a[j + 1] = v;
  }
}

static double infnorm(const double p[3]) { return dmax(dmax(fabs(p[0]), fabs(p[1])), fabs(p[2])); }

/* The Inside code of a point whose |s| lies this close to the band edge can
 * flip between two correct FP64 codes: rounding of s is a few ulp of the
 * coordinates and navigated points drift by ~1e-12 mm between codes. */
static void band_edge(double sv, const double p[3], unsigned* diag) {
  if (fabs(fabs(sv) - OR_KHALF) < 1e-11 + 1e-14 * infnorm(p)) *diag |= OR_D_BAND_EDGE;
}

/* Classify the open interval (a, b) of the ray by the Inside code at three
 * probes.  *marginal is set when a probe lies within kTolerance of a surface. */
static int classify(const or_solid* s, const double p[3], const double d[3], double a, double b,
                    int* marginal) {
  double tp[3];
  if (isinf(b)) {
    tp[0] = a + 1.0;
    tp[1] = a + 2.0;
    tp[2] = a + 4.0;
  } else {
    double h = b - a;
    tp[0] = a + 0.25 * h;
    tp[1] = a + 0.5 * h;
    tp[2] = a + 0.75 * h;
  }
  int nin = 0, nout = 0;
  *marginal = 0;
  for (int k = 0; k < 3; ++k) {
    double q[3] = {p[0] + tp[k] * d[0], p[1] + tp[k] * d[1], p[2] + tp[k] * d[2]};
    double sv = or_signed(s, q);
    int c = or_code(sv);
    if (fabs(sv) <= OR_KTOL) *marginal = 1;
    if (c == OR_INSIDE) ++nin;
    if (c == OR_OUTSIDE) ++nout;
  }
  if (nin && nout) *marginal = 1;
  if (nin) return OR_INSIDE;
  if (nout == 3) return OR_OUTSIDE;
  return OR_SURFACE;
}

/* first interval of class `want`; *t_suspect = start of the first interval
 * whose classification is ill-conditioned (or +inf) */
static double first_interval(const or_solid* s, const double p[3], const double d[3], int want,
                             unsigned* diag, double* t_suspect) {
  double R[OR_MAX_ROOTS];
  int n = or_roots(s, p, d, R);
  sort_small(R, n);
  double short_a = -1.0; /* start of the band-only short interval just passed */
  double a = 0.0;
  for (int i = 0; i <= n; ++i) {
    double b = (i < n) ? R[i] : INFINITY;
    if (!(b > a)) continue;
    int marg;
    int c = classify(s, p, d, a, b, &marg);
    if (c == want) {
      if (marg) {
        *diag |= OR_D_GRAZE;
        if (a < *t_suspect) *t_suspect = a;
      }
      /* the answer follows a band-only interval no longer than kTolerance
       * (two surfaces met within kTolerance of each other along the ray, a
       * plane's line crossed just beyond a surface, or a start point in the
       * band with a crossing within kTolerance ahead): either end of that
       * interval is a correct answer */
      if (short_a >= 0.0) {
        *diag |= OR_D_NEAR_TIE;
        if (short_a < *t_suspect) *t_suspect = short_a;
      }
      return a;
    }
    if (c == OR_SURFACE && b - a > OR_KTOL) {
      *diag |= OR_D_GRAZE;
      if (a < *t_suspect) *t_suspect = a;
    }
    short_a = (c == OR_SURFACE && !(b - a > OR_KTOL)) ? a : -1.0;
    a = b;
  }
  return INFINITY;
}

double or_dist_in_ex(const or_solid* s, const double p[3], const double d[3], unsigned* diag,
                     double* t_suspect) {
  double sv = or_signed(s, p);
  band_edge(sv, p, diag);
  if (or_code(sv) == OR_INSIDE) return -1.0;
  return first_interval(s, p, d, OR_INSIDE, diag, t_suspect);
}

double or_dist_out_ex(const or_solid* s, const double p[3], const double d[3], unsigned* diag,
                      double* t_suspect) {
  double sv = or_signed(s, p);
  band_edge(sv, p, diag);
  if (or_code(sv) == OR_OUTSIDE) return -1.0;
  double t = first_interval(s, p, d, OR_OUTSIDE, diag, t_suspect);
  if (isinf(t)) *diag |= OR_D_NO_EXIT;
  return t;
}

double or_dist_in(const or_solid* s, const double p[3], const double d[3], unsigned* diag) {
  double ts = INFINITY;
  return or_dist_in_ex(s, p, d, diag, &ts);
}

double or_dist_out(const or_solid* s, const double p[3], const double d[3], unsigned* diag) {
  double ts = INFINITY;
  return or_dist_out_ex(s, p, d, diag, &ts);
}

/* The size of a correct FP64 hit distance's rounding, against the bar it is
 * held to.  The inputs and the quadric coefficients carry a few units of
 * roundoff eps of the coordinate scale L; a hit at angle theta to the surface
 * normal moves by that over |cos theta|.  16 covers the few ulp of each
 * coefficient; the hit is flagged when this bound exceeds the bar. */
int or_hit_cond(const or_solid* s, const double p[3], const double d[3], double t) {
  if (!(t > 0.0) || !isfinite(t)) return 0;
  const double eps = 0x1p-52;
  double q[3] = {p[0] + t * d[0], p[1] + t * d[1], p[2] + t * d[2]};
  const double h = 1e-6 * dmax(1.0, infnorm(q));
  double g[3];
  for (int k = 0; k < 3; ++k) {
    double a[3] = {q[0], q[1], q[2]}, b[3] = {q[0], q[1], q[2]};
    a[k] += h;
    b[k] -= h;
    g[k] = (or_signed(s, a) - or_signed(s, b)) / (2.0 * h);
  }
  const double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  const double c = gn > 0.0 ? fabs(g[0] * d[0] + g[1] * d[1] + g[2] * d[2]) / gn : 0.0;
  const double pn2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
  const double qn2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
  const double L = (pn2 + qn2) / dmax(1.0, sqrt(qn2));
  const double bar = 1e-12 * dmax(t, 1.0);
  return 16.0 * eps * L > bar * c;  /* 16 eps L / |cos theta| > bar, without dividing by 0 */
}
