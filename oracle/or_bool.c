/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Composite solids built from two elementary solids by a Boolean operation
 * (Sec. III.B, detector geometry: complex elements are composed of the basic
 * bodies with Boolean operations).  The paper names the construction and not
 * its arithmetic, so the rules below are this project's reading of it:
 *
 *   - A sits at the composite's origin; C is placed by x = R x_C + t.
 *   - Point classification composes the components' signed terms: the union
 *     takes the smaller, the intersection the larger, and A minus C the larger
 *     of s_A and -s_C.  The three-way code then follows from the composite
 *     term with the same surface band as an elementary solid; a point on a face
 *     shared by the two parts of a union is a surface point.
 *   - Distances need no rule of their own: the roots of both components' full
 *     surfaces form the event list, and the event-list definition (intervals
 *     classified by probing the composite's code) gives DistanceToIn and
 *     DistanceToOut exactly as for an elementary solid.
 *   - Safeties are lower bounds composed from the components' safeties (each
 *     component's own formula, in its own frame):
 *       union, outside:        min(SafetyToIn A, SafetyToIn C)
 *       union, inside:         max of SafetyToOut over the components that
 *                              hold the point
 *       intersection, inside:  min(SafetyToOut A, SafetyToOut C)
 *       intersection, outside: max of SafetyToIn over the components the point
 *                              is outside of
 *       A minus C, inside:     min(SafetyToOut A, SafetyToIn C)
 *       A minus C, outside:    max of SafetyToIn A (point outside A) and
 *                              SafetyToOut C (point inside C)
 *     A ball of that radius around the point stays on its side of every
 *     component surface that decides it, hence on its side of the composite.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static double dmax(double a, double b) { return a > b ? a : b; }
static double dmin(double a, double b) { return a < b ? a : b; }

/* parameters: op, type_A, n_A, A[n_A], type_C, n_C, C[n_C], R[9], t[3] */
int or_bool_init(or_solid* s, const double* q, int nq) {
  if (nq < 3) return -1;
  const int op = (int)q[0];
  if ((double)op != q[0] || op < OR_UNION || op > OR_INTERSECTION) return -1;
  int at = 1;
  int type[2], np[2], off[2];
  for (int c = 0; c < 2; ++c) {
    if (at + 2 > nq) return -1;
    type[c] = (int)q[at];
    np[c] = (int)q[at + 1];
    if ((double)type[c] != q[at] || (double)np[c] != q[at + 1]) return -1;
    if (type[c] < OR_BOX || type[c] > OR_PCON || np[c] < 1) return -1; /* elementary parts only */
    off[c] = at + 2;
    at = off[c] + np[c];
    if (at > nq) return -1;
  }
  if (at + 12 != nq) return -1;
  s->op = op;
  for (int i = 0; i < 9; ++i) s->bR[i] = q[at + i];
  for (int i = 0; i < 3; ++i) s->bt[i] = q[at + 9 + i];
  /* R must be a rotation: R R^T = I within 1e-9 */
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double v = 0.0;
      for (int k = 0; k < 3; ++k) v += s->bR[3 * i + k] * s->bR[3 * j + k];
      if (fabs(v - (i == j ? 1.0 : 0.0)) > 1e-9) return -1;
    }
  s->comp = calloc(2, sizeof(or_solid));
  if (!s->comp) return -1;
  for (int c = 0; c < 2; ++c)
    if (or_solid_init(&s->comp[c], type[c], q + off[c], np[c]) != 0) {
      free(s->comp);
      s->comp = NULL;
      return -1;
    }
  return 0;
}

/* point and direction in C's frame: x_C = R^T (x - t), d_C = R^T d */
void or_bool_to_c(const or_solid* s, const double p[3], const double d[3], double pc[3], double dc[3]) {
  const double* R = s->bR;
  const double q[3] = {p[0] - s->bt[0], p[1] - s->bt[1], p[2] - s->bt[2]};
  for (int i = 0; i < 3; ++i) {
    pc[i] = R[i] * q[0] + R[3 + i] * q[1] + R[6 + i] * q[2];
    if (d) dc[i] = R[i] * d[0] + R[3 + i] * d[1] + R[6 + i] * d[2];
  }
}

double or_bool_signed(const or_solid* s, const double p[3]) {
  double pc[3];
  or_bool_to_c(s, p, NULL, pc, NULL);
  const double a = or_signed(&s->comp[0], p), c = or_signed(&s->comp[1], pc);
  switch (s->op) {
    case OR_UNION: return dmin(a, c);
    case OR_SUBTRACTION: return dmax(a, -c);
    default: return dmax(a, c);
  }
}

double or_bool_safety_in(const or_solid* s, const double p[3]) {
  double pc[3];
  or_bool_to_c(s, p, NULL, pc, NULL);
  const or_solid *A = &s->comp[0], *C = &s->comp[1];
  const int ca = or_inside(A, p), cc = or_inside(C, pc);
  double m = -INFINITY;
  switch (s->op) {
    case OR_UNION: return dmin(or_safety_in(A, p), or_safety_in(C, pc));
    case OR_SUBTRACTION:
      if (ca == OR_OUTSIDE) m = dmax(m, or_safety_in(A, p));
      if (cc == OR_INSIDE) m = dmax(m, or_safety_out(C, pc));
      break;
    default:
      if (ca == OR_OUTSIDE) m = dmax(m, or_safety_in(A, p));
      if (cc == OR_OUTSIDE) m = dmax(m, or_safety_in(C, pc));
  }
  return isinf(m) ? 0.0 : m;
}

double or_bool_safety_out(const or_solid* s, const double p[3]) {
  double pc[3];
  or_bool_to_c(s, p, NULL, pc, NULL);
  const or_solid *A = &s->comp[0], *C = &s->comp[1];
  double m = -INFINITY;
  switch (s->op) {
    case OR_UNION:
      if (or_inside(A, p) == OR_INSIDE) m = dmax(m, or_safety_out(A, p));
      if (or_inside(C, pc) == OR_INSIDE) m = dmax(m, or_safety_out(C, pc));
      return isinf(m) ? 0.0 : m;
    case OR_SUBTRACTION: return dmin(or_safety_out(A, p), or_safety_in(C, pc));
    default: return dmin(or_safety_out(A, p), or_safety_out(C, pc));
  }
}

/* the roots of both components' full surfaces along the same parameter t
 * (the placement is rigid, so t measures the same length in both frames) */
int or_bool_roots(const or_solid* s, const double p[3], const double d[3], double* R) {
  double pc[3], dc[3];
  or_bool_to_c(s, p, d, pc, dc);
  int n = or_roots(&s->comp[0], p, d, R);
  return n + or_roots(&s->comp[1], pc, dc, R + n);
}
