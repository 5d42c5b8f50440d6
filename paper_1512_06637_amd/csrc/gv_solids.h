// Device-side elementary solids: Inside code, Safety and DistanceToIn/Out
// (the three per-particle questions of Sec. III.C) for box, tube segment, cone
// segment, sphere shell, Trd and polycone (Sec. III.B elementary solids).
//
// Every distance is computed analytically along the ray r(t) = p + t d:
//   * an intersection solid (box, tubs, cons, sphere, Trd) is the intersection
//     of convex "allowed" components (cylinder/cone/sphere interiors, slabs,
//     half-spaces, a convex phi wedge) minus convex "excluded" components
//     (inner cylinder/cone/sphere, the complement of a phi wedge wider than pi);
//   * a polycone is the union over its z sections of such solids; pieces of
//     adjacent sections that touch at a junction plane are merged.
// On the ray every component is one interval, so the solid is a short list of
// pieces.  Pieces shorter than kTolerance after clipping to t >= 0 are not
// entries, and excluded gaps shorter than kTolerance ahead of the point are
// not exits.  DistanceToIn is the start of the first remaining piece;
// DistanceToOut is the end of the piece that starts within kTolerance of t = 0.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gv {

constexpr double kTol = 1e-9;
constexpr double kHalf = 5e-10;
#define GV_INF __builtin_huge_val()

enum SolidType { kBox = 0, kTubs = 1, kCons = 2, kSphere = 3, kTrd = 4, kPcon = 5, kBool = 6 };
enum BoolOp { kUnion = 0, kSubtraction = 1, kIntersection = 2 };
enum { kOutside = 0, kSurface = 1, kInside = 2 };

// ---- derived parameter layouts (filled on the host by geom_load) ----------
// box   : dx dy dz
// tubs  : rmin rmax dz phimode ns[2] ne[2] us[2] ue[2] rmin^2 rmax^2
// cons  : rmin1 rmax1 rmin2 rmax2 dz phimode ns[2] ne[2] us[2] ue[2] ao bo co ai bi ci inner
// sphere: rmin rmax rmin^2 rmax^2
// trd   : dx1 dx2 dy1 dy2 dz x0 tx cx y0 ty cy
// pcon  : nz z[nz] rmin[nz] rmax[nz] bo[nz-1] co[nz-1] bi[nz-1] ci[nz-1] inner[nz-1]
//         ilo[nz-1] ili[nz-1] icap[2] rbound  (ilo/ili/icap: 1/|e|^2 of the outer
//         and inner side segments and of the caps of the meridian polygon, 0 for
//         a degenerate one; rbound: the largest rmax)
// bool  : op typeA offA typeC offC R[9] t[3], then the parts' own tables at
//         offA / offC from the start of this one (R row major, x = R x_C + t)
// phimode: 0 full circle, 1 wedge <= pi (intersection of two half-spaces),
//          2 wedge > pi (union of two half-spaces).
namespace L {
enum { TB_RMIN = 0, TB_RMAX, TB_DZ, TB_PHI, TB_NS, TB_NE = 6, TB_US = 8, TB_UE = 10, TB_RMIN2 = 12, TB_RMAX2, TB_N };
enum { CN_RMIN1 = 0, CN_RMAX1, CN_RMIN2, CN_RMAX2, CN_DZ, CN_PHI, CN_NS, CN_NE = 8, CN_US = 10, CN_UE = 12,
       CN_AO = 14, CN_BO, CN_CO, CN_AI, CN_BI, CN_CI, CN_INNER, CN_N };
enum { SP_RMIN = 0, SP_RMAX, SP_RMIN2, SP_RMAX2, SP_N };
enum { TD_DX1 = 0, TD_DX2, TD_DY1, TD_DY2, TD_DZ, TD_X0, TD_TX, TD_CX, TD_Y0, TD_TY, TD_CY, TD_N };
enum { BO_OP = 0, BO_TA, BO_OA, BO_TC, BO_OC, BO_R, BO_T = 14, BO_N = 17 };
}  // namespace L

struct V3 {
  double x, y, z;
};

// Geometry tables never change while a kernel runs, so they are read through
// the constant address space: a wavefront-uniform address (the LV of a basket,
// its daughter table) then becomes a scalar load into SGPRs, and a per-lane
// address an ordinary vector load.
typedef const __attribute__((address_space(4))) double* CQ;
typedef const __attribute__((address_space(4))) int* CQI;
typedef const __attribute__((address_space(4))) float* CQF;
typedef const __attribute__((address_space(4))) unsigned long long* CQL;

// Pseudo-angle of (x, y) around the z axis: a monotone map of the polar angle
// [0, 2 pi) onto [0, 4), one unit per quadrant, with a half turn adding
// exactly 2 (modulo 4).  One division instead of an arctangent.
__host__ __device__ inline double pseudo_angle(double x, double y) {
  const double s = fabs(x) + fabs(y);
  if (y >= 0.0) return x >= 0.0 ? y / s : 1.0 - x / s;
  return x < 0.0 ? 2.0 - y / s : 3.0 + x / s;
}

// 1/d from the hardware reciprocal plus one Newton step: within a few ulp
// (11 ulp worst over 2^22 random operands), i.e. 3e-15 relative, three orders
// inside the 1e-12 parity bar.  Zero, denormal and infinite d keep the
// hardware value (+-inf or 0), where the Newton step would give NaN.
__device__ __forceinline__ double rcp_fast(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double r1 = fma(r, fma(-d, r, 1.0), r);
  return r1 == r1 ? r1 : r;
}
__device__ __forceinline__ double div_fast(double a, double b) { return a * rcp_fast(b); }

// pseudo_angle with the reciprocal of rcp_fast: a few ulp from it, for the
// sector lookups of navigation, whose sector masks are widened by 1e-4.
__device__ __forceinline__ double pseudo_angle_fast(double x, double y) {
  const double r = rcp_fast(fabs(x) + fabs(y));
  if (y >= 0.0) return x >= 0.0 ? y * r : 1.0 - x * r;
  return x < 0.0 ? 2.0 - y * r : 3.0 + x * r;
}

__device__ __forceinline__ int code_of(double s) {
  return s < -kHalf ? kInside : (s > kHalf ? kOutside : kSurface);
}

// ------------------------------------------------------------ ray intervals
struct Iv {
  double lo, hi;  // empty when !(lo <= hi)
};
__device__ __forceinline__ Iv iv_all() { return Iv{-GV_INF, GV_INF}; }
__device__ __forceinline__ Iv iv_none() { return Iv{GV_INF, -GV_INF}; }
__device__ __forceinline__ Iv iv_and(Iv a, Iv b) { return Iv{fmax(a.lo, b.lo), fmin(a.hi, b.hi)}; }
__device__ __forceinline__ bool iv_empty(Iv a) { return !(a.lo <= a.hi); }

// {t : a + b t <= 0}, or with `open` {t : a + b t < 0}: the two differ only
// for a ray parallel to the plane (b == 0) that lies in it (a == 0)
__device__ __forceinline__ Iv halfspace(double a, double b, bool open = false) {
  if (b > 0.0) return Iv{-GV_INF, -div_fast(a, b)};
  if (b < 0.0) return Iv{-div_fast(a, b), GV_INF};
  return (open ? a < 0.0 : a <= 0.0) ? iv_all() : iv_none();
}

// {t : |z + t dz| <= h}
__device__ __forceinline__ Iv slab(double z, double dz, double h) {
  if (dz != 0.0) {
    double iz = rcp_fast(dz);
    double t1 = (-h - z) * iz, t2 = (h - z) * iz;
    return Iv{fmin(t1, t2), fmax(t1, t2)};
  }
  return fabs(z) <= h ? iv_all() : iv_none();
}

// {t : z_lo <= z + t dz <= z_hi}
__device__ __forceinline__ Iv zrange(double z, double dz, double zlo, double zhi) {
  if (dz != 0.0) {
    double iz = rcp_fast(dz);
    double t1 = (zlo - z) * iz, t2 = (zhi - z) * iz;
    return Iv{fmin(t1, t2), fmax(t1, t2)};
  }
  return (z >= zlo && z <= zhi) ? iv_all() : iv_none();
}

// Roots of A t^2 + 2 B t + C (cancellation-free pair q/A, C/q); returns false
// when there is no real root.  The coefficients are formed without FMA
// contraction so near-surface cancellation rounds the same way on every FP64
// implementation of the formula.
__device__ __forceinline__ bool quad(double A, double B, double C, double& t1, double& t2) {
  double D = B * B - A * C;
  if (D < 0.0) return false;
  double sq = sqrt(D);
  double q = -(B + copysign(sq, B));
  if (q == 0.0) {
    t1 = t2 = 0.0;
    return true;
  }
  double r1 = div_fast(q, A), r2 = div_fast(C, q);
  t1 = fmin(r1, r2);
  t2 = fmax(r1, r2);
  return true;
}

// interior of the infinite cylinder x^2 + y^2 <= R^2
__device__ __forceinline__ Iv cyl_interior(double R2, V3 p, V3 d) {
#pragma clang fp contract(off)
  double A = d.x * d.x + d.y * d.y;
  double B = p.x * d.x + p.y * d.y;
  double C = p.x * p.x + p.y * p.y - R2;
  if (A == 0.0) return C < 0.0 ? iv_all() : iv_none();
  double t1, t2;
  if (!quad(A, B, C, t1, t2)) return iv_none();
  return Iv{t1, t2};
}

// cyl_interior for an excluded cylinder (a tube's rmin): with C >= 0 (the
// point on or outside it) and B >= 0 (moving away from the axis) both roots
// are <= 0 -- q = -(B + sqrt D) <= 0, so q / A <= 0 and C / q <= 0, signs
// exact -- and pieces_of treats such an interval exactly as no interval, so
// it is returned as none without the square root and the divisions
__device__ __forceinline__ Iv cyl_interior_ahead(double R2, V3 p, V3 d) {
#pragma clang fp contract(off)
  double B = p.x * d.x + p.y * d.y;
  double C = p.x * p.x + p.y * p.y - R2;
  if (C >= 0.0 && B >= 0.0) return iv_none();
  return cyl_interior(R2, p, d);
}

// interior of the sphere |x|^2 <= R^2
__device__ __forceinline__ Iv sph_interior(double R2, V3 p, V3 d) {
#pragma clang fp contract(off)
  double A = d.x * d.x + d.y * d.y + d.z * d.z;
  double B = p.x * d.x + p.y * d.y + p.z * d.z;
  double C = p.x * p.x + p.y * p.y + p.z * p.z - R2;
  double t1, t2;
  if (!quad(A, B, C, t1, t2)) return iv_none();
  return Iv{t1, t2};
}

// interior of the truncated cone r <= a + b (z - z0) restricted to the slab
// interval S (where z lies in the section).  Over S the radius line is >= 0, so
// the set is convex and one interval; A <= 0 can split {f <= 0} in two, of
// which the piece on the right nappe is kept.
__device__ __forceinline__ Iv cone_interior(double a, double b, double z0, Iv S, V3 p, V3 d) {
#pragma clang fp contract(off)
  if (iv_empty(S)) return S;
  double rz = a + b * (p.z - z0);
  double A = d.x * d.x + d.y * d.y - b * b * d.z * d.z;
  double B = p.x * d.x + p.y * d.y - b * rz * d.z;
  double C = p.x * p.x + p.y * p.y - rz * rz;
  if (A > 0.0) {
    double t1, t2;
    if (!quad(A, B, C, t1, t2)) return iv_none();
    return iv_and(S, Iv{t1, t2});
  }
  Iv P1, P2;
  if (A == 0.0) {
    if (B > 0.0) {
      P1 = Iv{-GV_INF, -div_fast(C, 2.0 * B)};
    } else if (B < 0.0) {
      P1 = Iv{-div_fast(C, 2.0 * B), GV_INF};
    } else {
      P1 = C <= 0.0 ? iv_all() : iv_none();
    }
    P2 = iv_none();
  } else {
    double t1, t2;
    if (!quad(A, B, C, t1, t2)) {
      P1 = iv_all();
      P2 = iv_none();
    } else {
      P1 = Iv{-GV_INF, t1};
      P2 = Iv{t2, GV_INF};
    }
  }
  P1 = iv_and(S, P1);
  P2 = iv_and(S, P2);
  // keep the piece on the nappe a + b (z - z0) >= 0
  bool ok1 = !iv_empty(P1) && (a + b * ((p.z + 0.5 * (P1.lo + P1.hi) * d.z) - z0)) >= 0.0;
  bool ok2 = !iv_empty(P2) && (a + b * ((p.z + 0.5 * (P2.lo + P2.hi) * d.z) - z0)) >= 0.0;
  if (ok1 && ok2) return (P1.hi - P1.lo >= P2.hi - P2.lo) ? P1 : P2;
  if (ok1) return P1;
  if (ok2) return P2;
  return iv_none();
}

// ------------------------------------------------- pieces of one ray and solid
// allowed interval A minus up to two excluded intervals, after clipping to
// t >= 0.  Pieces are returned in increasing t.
struct Pieces {
  Iv p0, p1, p2;  // increasing t; empty slots have lo > hi
};

__device__ __forceinline__ Iv clip0(Iv a) { return Iv{fmax(a.lo, 0.0), a.hi}; }

__device__ __forceinline__ void pieces_of(Iv A, Iv X1, Iv X2, Pieces& P) {
  P.p0 = P.p1 = P.p2 = iv_none();
  A = clip0(A);
  if (!(A.hi >= A.lo)) return;
  // an excluded gap shorter than kTolerance is ignored (the ray only grazes
  // it) unless it holds the start point: a point in the surface band on the
  // excluded side enters the solid where the gap ends
  bool u1 = X1.lo <= 0.0 ? X1.hi > 0.0 : X1.hi - X1.lo >= kTol;
  bool u2 = X2.lo <= 0.0 ? X2.hi > 0.0 : X2.hi - X2.lo >= kTol;
  X1 = clip0(X1);
  X2 = clip0(X2);
  if (!u1) {
    X1 = X2;
    u1 = u2;
    u2 = false;
  }
  if (u1 && u2 && X2.lo < X1.lo) {
    Iv t = X1;
    X1 = X2;
    X2 = t;
  }
  double cur = A.lo;
  if (u1) {
    if (X1.lo > cur) P.p0 = Iv{cur, fmin(X1.lo, A.hi)};
    cur = fmax(cur, X1.hi);
  }
  if (u2 && cur < A.hi) {
    if (X2.lo > cur) P.p1 = Iv{cur, fmin(X2.lo, A.hi)};
    cur = fmax(cur, X2.hi);
  }
  if (cur <= A.hi) P.p2 = Iv{cur, A.hi};
}

__device__ __forceinline__ double first_entry(const Pieces& P) {
  if (P.p0.hi - P.p0.lo >= kTol) return P.p0.lo;
  if (P.p1.hi - P.p1.lo >= kTol) return P.p1.lo;
  if (P.p2.hi - P.p2.lo >= kTol) return P.p2.lo;
  return GV_INF;
}

__device__ __forceinline__ double exit_of(const Pieces& P) {
  Iv f = !iv_empty(P.p0) ? P.p0 : (!iv_empty(P.p1) ? P.p1 : P.p2);
  if (!iv_empty(f) && f.lo <= kTol) return fmax(f.hi, 0.0);
  return 0.0;
}

// ------------------------------------------------------------- phi wedges
__device__ __forceinline__ double phi_term(CQ q, int ns, int ne, int mode, double x, double y) {
  double a = x * q[ns] + y * q[ns + 1];
  double b = x * q[ne] + y * q[ne + 1];
  return mode == 1 ? fmax(a, b) : fmin(a, b);
}

// allowed interval of a wedge <= pi, or the excluded interval (complement
// wedge) of a wedge > pi
__device__ __forceinline__ void phi_intervals(CQ q, int ns, int ne, int mode, V3 p, V3 d, Iv& allow,
                                              Iv& excl) {
  allow = iv_all();
  excl = iv_none();
  if (mode == 0) return;
  double as = p.x * q[ns] + p.y * q[ns + 1], bs = d.x * q[ns] + d.y * q[ns + 1];
  double ae = p.x * q[ne] + p.y * q[ne + 1], be = d.x * q[ne] + d.y * q[ne + 1];
  if (mode == 1) {
    allow = iv_and(halfspace(as, bs), halfspace(ae, be));
  } else {
    // the excluded wedge is open: its planes belong to the solid, as a
    // wedge <= pi holds its own planes
    excl = iv_and(halfspace(-as, -bs, true), halfspace(-ae, -be, true));
  }
}

__device__ __forceinline__ double half_plane_dist(CQ q, int n, int u, double x, double y, double r) {
  if (x * q[u] + y * q[u + 1] >= 0.0) return fabs(x * q[n] + y * q[n + 1]);
  return r;
}

// ======================================================================= BOX
struct Box {
  static constexpr int kType = kBox;
  __device__ static __forceinline__ double sgn(CQ q, V3 p) {
    return fmax(fmax(fabs(p.x) - q[0], fabs(p.y) - q[1]), fabs(p.z) - q[2]);
  }
  __device__ static __forceinline__ double safety_out(CQ q, V3 p) {
    return fmin(fmin(q[0] - fabs(p.x), q[1] - fabs(p.y)), q[2] - fabs(p.z));
  }
  __device__ static __forceinline__ double safety_in(CQ q, V3 p) { return sgn(q, p); }
  __device__ static __forceinline__ double dist_out(CQ q, V3 p, V3 d) {
    if (sgn(q, p) > kHalf) return -1.0;
    double t = GV_INF;
    if (d.x != 0.0) t = fmin(t, div_fast(copysign(q[0], d.x) - p.x, d.x));
    if (d.y != 0.0) t = fmin(t, div_fast(copysign(q[1], d.y) - p.y, d.y));
    if (d.z != 0.0) t = fmin(t, div_fast(copysign(q[2], d.z) - p.z, d.z));
    return fmax(t, 0.0);
  }
  // Slab method with one reciprocal per axis.  A zero direction component
  // gives an infinite reciprocal: the slab then imposes nothing when |p| < h
  // and empties the interval otherwise (0 * inf = NaN is dropped by min/max,
  // and leaves the other bound at -inf or +inf, which also empties it).
  __device__ static __forceinline__ double dist_in_hd(double hx, double hy, double hz, V3 p, V3 d) {
    double s = fmax(fmax(fabs(p.x) - hx, fabs(p.y) - hy), fabs(p.z) - hz);
    double ix = rcp_fast(d.x), iy = rcp_fast(d.y), iz = rcp_fast(d.z);
    double ax = (-hx - p.x) * ix, bx = (hx - p.x) * ix;
    double ay = (-hy - p.y) * iy, by = (hy - p.y) * iy;
    double az = (-hz - p.z) * iz, bz = (hz - p.z) * iz;
    double lo = fmax(fmax(fmin(ax, bx), fmin(ay, by)), fmax(fmin(az, bz), 0.0));
    double hi = fmin(fmin(fmax(ax, bx), fmax(ay, by)), fmax(az, bz));
    double t = (hi - lo >= kTol) ? lo : GV_INF;
    return s < -kHalf ? -1.0 : t;
  }
  __device__ static __forceinline__ double dist_in(CQ q, V3 p, V3 d) {
    return dist_in_hd(q[0], q[1], q[2], p, d);
  }
};

// ============================================================= TUBE SEGMENT
struct Tubs {
  static constexpr int kType = kTubs;
  __device__ static __forceinline__ double sgn(CQ q, V3 p) {
    double r = sqrt(p.x * p.x + p.y * p.y);
    double t = r - q[L::TB_RMAX];
    if (q[L::TB_RMIN] > 0.0) t = fmax(t, q[L::TB_RMIN] - r);
    t = fmax(t, fabs(p.z) - q[L::TB_DZ]);
    int mode = (int)q[L::TB_PHI];
    if (mode) t = fmax(t, phi_term(q, L::TB_NS, L::TB_NE, mode, p.x, p.y));
    return t;
  }
  __device__ static __forceinline__ double safety_out(CQ q, V3 p) {
    double r = sqrt(p.x * p.x + p.y * p.y);
    double m = q[L::TB_RMAX] - r;
    if (q[L::TB_RMIN] > 0.0) m = fmin(m, r - q[L::TB_RMIN]);
    m = fmin(m, q[L::TB_DZ] - fabs(p.z));
    if ((int)q[L::TB_PHI]) {
      m = fmin(m, half_plane_dist(q, L::TB_NS, L::TB_US, p.x, p.y, r));
      m = fmin(m, half_plane_dist(q, L::TB_NE, L::TB_UE, p.x, p.y, r));
    }
    return m;
  }
  __device__ static __forceinline__ double safety_in(CQ q, V3 p) {
    double r = sqrt(p.x * p.x + p.y * p.y);
    double m = r - q[L::TB_RMAX];
    if (q[L::TB_RMIN] > 0.0) m = fmax(m, q[L::TB_RMIN] - r);
    m = fmax(m, fabs(p.z) - q[L::TB_DZ]);
    int mode = (int)q[L::TB_PHI];
    if (mode && phi_term(q, L::TB_NS, L::TB_NE, mode, p.x, p.y) > 0.0)
      m = fmax(m, fmin(half_plane_dist(q, L::TB_NS, L::TB_US, p.x, p.y, r),
                       half_plane_dist(q, L::TB_NE, L::TB_UE, p.x, p.y, r)));
    return m;
  }
  __device__ static __forceinline__ void pieces(CQ q, V3 p, V3 d, Pieces& P) {
    Iv A = iv_and(cyl_interior(q[L::TB_RMAX2], p, d), slab(p.z, d.z, q[L::TB_DZ]));
    Iv X1 = q[L::TB_RMIN] > 0.0 ? cyl_interior_ahead(q[L::TB_RMIN2], p, d) : iv_none();
    Iv allow, excl;
    phi_intervals(q, L::TB_NS, L::TB_NE, (int)q[L::TB_PHI], p, d, allow, excl);
    pieces_of(iv_and(A, allow), X1, excl, P);
  }
  __device__ static __forceinline__ double dist_in(CQ q, V3 p, V3 d) {
    if (sgn(q, p) < -kHalf) return -1.0;
    Pieces P;
    pieces(q, p, d, P);
    return first_entry(P);
  }
  __device__ static __forceinline__ double dist_out(CQ q, V3 p, V3 d) {
    if (sgn(q, p) > kHalf) return -1.0;
    Pieces P;
    pieces(q, p, d, P);
    return exit_of(P);
  }
};

// ============================================================ CONE SEGMENT
struct Cons {
  static constexpr int kType = kCons;
  __device__ static __forceinline__ double sgn(CQ q, V3 p) {
    double r = sqrt(p.x * p.x + p.y * p.y);
    double t = (r - (q[L::CN_AO] + q[L::CN_BO] * p.z)) * q[L::CN_CO];
    if (q[L::CN_INNER] != 0.0) t = fmax(t, ((q[L::CN_AI] + q[L::CN_BI] * p.z) - r) * q[L::CN_CI]);
    t = fmax(t, fabs(p.z) - q[L::CN_DZ]);
    int mode = (int)q[L::CN_PHI];
    if (mode) t = fmax(t, phi_term(q, L::CN_NS, L::CN_NE, mode, p.x, p.y));
    return t;
  }
  __device__ static __forceinline__ double safety_out(CQ q, V3 p) {
    double r = sqrt(p.x * p.x + p.y * p.y);
    double m = ((q[L::CN_AO] + q[L::CN_BO] * p.z) - r) * q[L::CN_CO];
    if (q[L::CN_INNER] != 0.0) m = fmin(m, (r - (q[L::CN_AI] + q[L::CN_BI] * p.z)) * q[L::CN_CI]);
    m = fmin(m, q[L::CN_DZ] - fabs(p.z));
    if ((int)q[L::CN_PHI]) {
      m = fmin(m, half_plane_dist(q, L::CN_NS, L::CN_US, p.x, p.y, r));
      m = fmin(m, half_plane_dist(q, L::CN_NE, L::CN_UE, p.x, p.y, r));
    }
    return m;
  }
  __device__ static __forceinline__ double safety_in(CQ q, V3 p) {
    double r = sqrt(p.x * p.x + p.y * p.y);
    double m = (r - (q[L::CN_AO] + q[L::CN_BO] * p.z)) * q[L::CN_CO];
    if (q[L::CN_INNER] != 0.0) m = fmax(m, ((q[L::CN_AI] + q[L::CN_BI] * p.z) - r) * q[L::CN_CI]);
    m = fmax(m, fabs(p.z) - q[L::CN_DZ]);
    int mode = (int)q[L::CN_PHI];
    if (mode && phi_term(q, L::CN_NS, L::CN_NE, mode, p.x, p.y) > 0.0)
      m = fmax(m, fmin(half_plane_dist(q, L::CN_NS, L::CN_US, p.x, p.y, r),
                       half_plane_dist(q, L::CN_NE, L::CN_UE, p.x, p.y, r)));
    return m;
  }
  __device__ static __forceinline__ void pieces(CQ q, V3 p, V3 d, Pieces& P) {
    Iv S = slab(p.z, d.z, q[L::CN_DZ]);
    Iv A = cone_interior(q[L::CN_AO], q[L::CN_BO], 0.0, S, p, d);
    Iv X1 = q[L::CN_INNER] != 0.0 ? cone_interior(q[L::CN_AI], q[L::CN_BI], 0.0, S, p, d) : iv_none();
    Iv allow, excl;
    phi_intervals(q, L::CN_NS, L::CN_NE, (int)q[L::CN_PHI], p, d, allow, excl);
    pieces_of(iv_and(A, allow), X1, excl, P);
  }
  __device__ static __forceinline__ double dist_in(CQ q, V3 p, V3 d) {
    if (sgn(q, p) < -kHalf) return -1.0;
    Pieces P;
    pieces(q, p, d, P);
    return first_entry(P);
  }
  __device__ static __forceinline__ double dist_out(CQ q, V3 p, V3 d) {
    if (sgn(q, p) > kHalf) return -1.0;
    Pieces P;
    pieces(q, p, d, P);
    return exit_of(P);
  }
};

// ============================================================ SPHERE SHELL
struct Sphere {
  static constexpr int kType = kSphere;
  __device__ static __forceinline__ double sgn(CQ q, V3 p) {
    double rho = sqrt(p.x * p.x + p.y * p.y + p.z * p.z);
    double t = rho - q[L::SP_RMAX];
    if (q[L::SP_RMIN] > 0.0) t = fmax(t, q[L::SP_RMIN] - rho);
    return t;
  }
  __device__ static __forceinline__ double safety_out(CQ q, V3 p) {
    double rho = sqrt(p.x * p.x + p.y * p.y + p.z * p.z);
    double m = q[L::SP_RMAX] - rho;
    if (q[L::SP_RMIN] > 0.0) m = fmin(m, rho - q[L::SP_RMIN]);
    return m;
  }
  __device__ static __forceinline__ double safety_in(CQ q, V3 p) { return sgn(q, p); }
  __device__ static __forceinline__ void pieces(CQ q, V3 p, V3 d, Pieces& P) {
    Iv A = sph_interior(q[L::SP_RMAX2], p, d);
    Iv X1 = q[L::SP_RMIN] > 0.0 ? sph_interior(q[L::SP_RMIN2], p, d) : iv_none();
    pieces_of(A, X1, iv_none(), P);
  }
  __device__ static __forceinline__ double dist_in(CQ q, V3 p, V3 d) {
    if (sgn(q, p) < -kHalf) return -1.0;
    Pieces P;
    pieces(q, p, d, P);
    return first_entry(P);
  }
  __device__ static __forceinline__ double dist_out(CQ q, V3 p, V3 d) {
    if (sgn(q, p) > kHalf) return -1.0;
    Pieces P;
    pieces(q, p, d, P);
    return exit_of(P);
  }
};

// ====================================================================== TRD
struct Trd {
  static constexpr int kType = kTrd;
  __device__ static __forceinline__ double sgn(CQ q, V3 p) {
    double t = (fabs(p.x) - (q[L::TD_X0] + q[L::TD_TX] * p.z)) * q[L::TD_CX];
    t = fmax(t, (fabs(p.y) - (q[L::TD_Y0] + q[L::TD_TY] * p.z)) * q[L::TD_CY]);
    return fmax(t, fabs(p.z) - q[L::TD_DZ]);
  }
  __device__ static __forceinline__ double safety_out(CQ q, V3 p) {
    double m = ((q[L::TD_X0] + q[L::TD_TX] * p.z) - fabs(p.x)) * q[L::TD_CX];
    m = fmin(m, ((q[L::TD_Y0] + q[L::TD_TY] * p.z) - fabs(p.y)) * q[L::TD_CY]);
    return fmin(m, q[L::TD_DZ] - fabs(p.z));
  }
  __device__ static __forceinline__ double safety_in(CQ q, V3 p) { return sgn(q, p); }
  // the four slanted faces as half-spaces (+-x - t z - x0 <= 0); false when a
  // face is parallel to the ray and the ray is not inside it beyond the band
  __device__ static __forceinline__ bool face(double a, double b, double c, double& lo, double& hi) {
    if (b > 0.0) {
      hi = fmin(hi, -div_fast(a, b));
    } else if (b < 0.0) {
      lo = fmax(lo, -div_fast(a, b));
    } else {
      return a * c < -kHalf;
    }
    return true;
  }
  __device__ static __forceinline__ bool interval(CQ q, V3 p, V3 d, double& lo, double& hi) {
    double tx = q[L::TD_TX], ty = q[L::TD_TY];
    double nxp = p.x - tx * p.z, nxd = d.x - tx * d.z;
    double mxp = -p.x - tx * p.z, mxd = -d.x - tx * d.z;
    double nyp = p.y - ty * p.z, nyd = d.y - ty * d.z;
    double myp = -p.y - ty * p.z, myd = -d.y - ty * d.z;
    lo = -GV_INF;
    hi = GV_INF;
    if (!face(nxp - q[L::TD_X0], nxd, q[L::TD_CX], lo, hi)) return false;
    if (!face(mxp - q[L::TD_X0], mxd, q[L::TD_CX], lo, hi)) return false;
    if (!face(nyp - q[L::TD_Y0], nyd, q[L::TD_CY], lo, hi)) return false;
    if (!face(myp - q[L::TD_Y0], myd, q[L::TD_CY], lo, hi)) return false;
    if (d.z != 0.0) {
      double iz = rcp_fast(d.z);
      double t1 = (-q[L::TD_DZ] - p.z) * iz, t2 = (q[L::TD_DZ] - p.z) * iz;
      lo = fmax(lo, fmin(t1, t2));
      hi = fmin(hi, fmax(t1, t2));
    } else if (!(fabs(p.z) < q[L::TD_DZ] - kHalf)) {
      return false;
    }
    return true;
  }
  __device__ static __forceinline__ double dist_in(CQ q, V3 p, V3 d) {
    if (sgn(q, p) < -kHalf) return -1.0;
    double lo, hi;
    if (!interval(q, p, d, lo, hi)) return GV_INF;
    lo = fmax(lo, 0.0);
    return (hi - lo >= kTol) ? lo : GV_INF;
  }
  __device__ static __forceinline__ double dist_out(CQ q, V3 p, V3 d) {
    if (sgn(q, p) > kHalf) return -1.0;
    double lo, hi;
    if (!interval(q, p, d, lo, hi)) return 0.0;
    return (lo <= kTol) ? fmax(hi, 0.0) : 0.0;
  }
};

// ================================================================= POLYCONE
struct Pcon {
  static constexpr int kType = kPcon;
  struct View {
    int nz;
    CQ z, rmin, rmax, bo, co, bi, ci, inner, ilo, ili, icap;
    double rbound;
  };
  __device__ static __forceinline__ View view(CQ q) {
    View v;
    v.nz = (int)q[0];
    v.z = q + 1;
    v.rmin = v.z + v.nz;
    v.rmax = v.rmin + v.nz;
    v.bo = v.rmax + v.nz;
    v.co = v.bo + (v.nz - 1);
    v.bi = v.co + (v.nz - 1);
    v.ci = v.bi + (v.nz - 1);
    v.inner = v.ci + (v.nz - 1);
    v.ilo = v.inner + (v.nz - 1);
    v.ili = v.ilo + (v.nz - 1);
    v.icap = v.ili + (v.nz - 1);
    v.rbound = v.icap[2];
    return v;
  }
  // largest j with z_j <= z, clamped to [0, nz-2]
  __device__ static __forceinline__ int section(const View& v, double z) {
    int j = 0;
    for (int k = 1; k + 1 < v.nz; ++k)
      if (v.z[k] <= z) j = k;
    return j;
  }
  __device__ static __forceinline__ double sgn(CQ q, V3 p) {
    View v = view(q);
    int j = section(v, p.z);
    double r = sqrt(p.x * p.x + p.y * p.y);
    double zl = p.z - v.z[j];
    double t = (r - (v.rmax[j] + v.bo[j] * zl)) * v.co[j];
    if (v.inner[j] != 0.0) t = fmax(t, ((v.rmin[j] + v.bi[j] * zl) - r) * v.ci[j]);
    t = fmax(t, v.z[0] - p.z);
    return fmax(t, p.z - v.z[v.nz - 1]);
  }
  // squared distance from (r, z) to the segment (r1, z1)-(r2, z2), il =
  // 1/|e|^2 (0 for a degenerate segment: its first point)
  __device__ static __forceinline__ double seg2(double r, double z, double r1, double z1, double r2, double z2,
                                                double il) {
    double er = r2 - r1, ez = z2 - z1, wr = r - r1, wz = z - z1;
    double u = fmin(fmax((wr * er + wz * ez) * il, 0.0), 1.0);
    double qr = r1 + u * er - r, qz = z1 + u * ez - z;
    return qr * qr + qz * qz;
  }
  // exact distance in the meridian plane to the boundary polygon: the
  // smallest squared distance over its segments, one square root at the end
  // (the square root is monotone, so this equals the smallest root)
  __device__ static double boundary(CQ q, V3 p) {
    View v = view(q);
    double r = sqrt(p.x * p.x + p.y * p.y), z = p.z;
    double best = GV_INF;
    for (int j = 0; j + 1 < v.nz; ++j) {
      best = fmin(best, seg2(r, z, v.rmax[j], v.z[j], v.rmax[j + 1], v.z[j + 1], v.ilo[j]));
      if (v.rmin[j] > 0.0 || v.rmin[j + 1] > 0.0)
        best = fmin(best, seg2(r, z, v.rmin[j], v.z[j], v.rmin[j + 1], v.z[j + 1], v.ili[j]));
    }
    int e = v.nz - 1;
    best = fmin(best, seg2(r, z, v.rmin[0], v.z[0], v.rmax[0], v.z[0], v.icap[0]));
    best = fmin(best, seg2(r, z, v.rmin[e], v.z[e], v.rmax[e], v.z[e], v.icap[1]));
    return sqrt(best);
  }
  __device__ static __forceinline__ double safety_out(CQ q, V3 p) { return boundary(q, p); }
  __device__ static __forceinline__ double safety_in(CQ q, V3 p) { return boundary(q, p); }

  // Walks the sections in the order the ray meets them and merges touching
  // pieces.  want_in: start of the first merged piece of length >= kTol;
  // otherwise: end of the merged piece starting within kTol of t = 0.  The
  // slabs of later sections start later along the ray, so once a section's
  // slab starts beyond the current piece no later piece can join it: the
  // piece is complete there, and the walk stops as soon as it has its answer.
  // [t0, t1]: the part of the ray that can hold pieces (DistanceToIn: the
  // bounding cylinder's interval), the walk starting at the section that holds
  // the ray at t0 (one section earlier in the walk's direction when t0 > 0, so
  // that the rounding of that point's z at a plane cannot skip a section) and
  // stopping at the first section that starts beyond t1.  CNT: *nsec counts
  // the sections whose cone intersections are computed (the work measurement
  // of the profiling kernel; never in production).
  template <bool CNT = false>
  __device__ static double walk(CQ q, V3 p, V3 d, bool want_in, int* nsec = nullptr, double t0 = 0.0,
                                double t1 = GV_INF) {
    View v = view(q);
    int j0 = section(v, t0 > 0.0 ? p.z + t0 * d.z : p.z), j1, step;
    if (d.z > 0.0) {
      j1 = v.nz - 2;
      step = 1;
      if (t0 > 0.0 && j0 > 0) --j0;
    } else if (d.z < 0.0) {
      j1 = 0;
      step = -1;
      if (t0 > 0.0 && j0 < v.nz - 2) ++j0;
    } else {
      // a horizontal ray only meets the section(s) whose slab holds z
      j1 = j0;
      step = 1;
      if (j0 > 0 && p.z == v.z[j0]) j0 = j0 - 1;
    }
    double cl = GV_INF, ch = -GV_INF;  // current merged piece
    bool have = false;
    for (int j = j0;; j += step) {
      Iv S = zrange(p.z, d.z, v.z[j], v.z[j + 1]);
      if (S.lo > t1) break;  // beyond the part of the ray that can hold pieces
      if (have && S.lo > ch) {  // no piece of this or a later section joins the current one
        if (!want_in) return cl <= kTol ? fmax(ch, 0.0) : 0.0;
        if (ch - cl >= kTol) return cl;
      }
      if (CNT) ++*nsec;
      Iv A = cone_interior(v.rmax[j], v.bo[j], v.z[j], S, p, d);
      Iv X = v.inner[j] != 0.0 ? cone_interior(v.rmin[j], v.bi[j], v.z[j], S, p, d) : iv_none();
      Pieces P;
      pieces_of(A, X, iv_none(), P);
      Iv pk[3] = {P.p0, P.p1, P.p2};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (iv_empty(pk[k])) continue;
        if (have && pk[k].lo <= ch) {
          ch = fmax(ch, pk[k].hi);
          continue;
        }
        if (have) {  // the current piece is complete
          if (want_in) {
            if (ch - cl >= kTol) return cl;
          } else {
            return cl <= kTol ? fmax(ch, 0.0) : 0.0;
          }
        }
        cl = pk[k].lo;
        ch = pk[k].hi;
        have = true;
      }
      if (j == j1) break;
    }
    if (!have) return want_in ? GV_INF : 0.0;
    if (want_in) return (ch - cl >= kTol) ? cl : GV_INF;
    return cl <= kTol ? fmax(ch, 0.0) : 0.0;
  }
  // The ray's interval inside the bounding cylinder (padded by 1e-6 mm, far
  // above the rounding of either test) within the z range: every piece of the
  // solid along the ray lies in it.
  __device__ static __forceinline__ Iv bound_iv(const View& v, V3 p, V3 d) {
    const double rb = v.rbound + 1e-6;
    return iv_and(cyl_interior(rb * rb, p, d), zrange(p.z, d.z, v.z[0] - 1e-6, v.z[v.nz - 1] + 1e-6));
  }
  __device__ static __forceinline__ bool misses(Iv B) { return !(B.hi >= fmax(B.lo, 0.0)); }
  __device__ static double dist_in(CQ q, V3 p, V3 d) {
    if (sgn(q, p) < -kHalf) return -1.0;
    const Iv B = bound_iv(view(q), p, d);
    if (misses(B)) return GV_INF;
    return walk(q, p, d, true, nullptr, fmax(B.lo, 0.0), B.hi);
  }
  __device__ static double dist_out(CQ q, V3 p, V3 d) {
    if (sgn(q, p) > kHalf) return -1.0;
    return walk(q, p, d, false);
  }
};

// ------------------------------------------------------- runtime dispatch
// elementary solids
__device__ __forceinline__ double prim_sgn(int type, CQ q, V3 p) {
  switch (type) {
    case kBox: return Box::sgn(q, p);
    case kTubs: return Tubs::sgn(q, p);
    case kCons: return Cons::sgn(q, p);
    case kSphere: return Sphere::sgn(q, p);
    case kTrd: return Trd::sgn(q, p);
    default: return Pcon::sgn(q, p);
  }
}
__device__ __forceinline__ double prim_dist_in(int type, CQ q, V3 p, V3 d) {
  switch (type) {
    case kBox: return Box::dist_in(q, p, d);
    case kTubs: return Tubs::dist_in(q, p, d);
    case kCons: return Cons::dist_in(q, p, d);
    case kSphere: return Sphere::dist_in(q, p, d);
    case kTrd: return Trd::dist_in(q, p, d);
    default: return Pcon::dist_in(q, p, d);
  }
}
__device__ __forceinline__ double prim_dist_out(int type, CQ q, V3 p, V3 d) {
  switch (type) {
    case kBox: return Box::dist_out(q, p, d);
    case kTubs: return Tubs::dist_out(q, p, d);
    case kCons: return Cons::dist_out(q, p, d);
    case kSphere: return Sphere::dist_out(q, p, d);
    case kTrd: return Trd::dist_out(q, p, d);
    default: return Pcon::dist_out(q, p, d);
  }
}
__device__ __forceinline__ double prim_safety_in(int type, CQ q, V3 p) {
  switch (type) {
    case kBox: return Box::safety_in(q, p);
    case kTubs: return Tubs::safety_in(q, p);
    case kCons: return Cons::safety_in(q, p);
    case kSphere: return Sphere::safety_in(q, p);
    case kTrd: return Trd::safety_in(q, p);
    default: return Pcon::safety_in(q, p);
  }
}
__device__ __forceinline__ double prim_safety_out(int type, CQ q, V3 p) {
  switch (type) {
    case kBox: return Box::safety_out(q, p);
    case kTubs: return Tubs::safety_out(q, p);
    case kCons: return Cons::safety_out(q, p);
    case kSphere: return Sphere::safety_out(q, p);
    case kTrd: return Trd::safety_out(q, p);
    default: return Pcon::safety_out(q, p);
  }
}

// ================================================================ COMPOSITE
// op(A, C) of two elementary solids (Sec. III.B: complex elements composed
// with Boolean operations); A at the composite's origin, C placed by
// x = R x_C + t.  The Inside term composes the parts' terms (union: the
// smaller; intersection: the larger; A minus C: the larger of s_A and -s_C).
// Along a ray the composite is the Boolean combination of the parts' pieces,
// walked with the parts' own DistanceToIn/Out from the point reached so far:
// an entry needs a run of at least kTolerance inside the composite, and a gap
// of less than kTolerance before a part resumes is no exit (the elementary
// solids' rules).  Safeties are bounds composed from the parts' safeties.
// The navigation kernels reach these functions through BoolCall, out of line.
struct Bool {
  static constexpr int kType = kBool;
  static constexpr int kMaxIter = 64;  // > the pieces two elementary solids can have on a ray
  __device__ static __forceinline__ int op(CQ q) { return (int)q[L::BO_OP]; }
  __device__ static __forceinline__ int ta(CQ q) { return (int)q[L::BO_TA]; }
  __device__ static __forceinline__ int tc(CQ q) { return (int)q[L::BO_TC]; }
  __device__ static __forceinline__ CQ qa(CQ q) { return q + (int)q[L::BO_OA]; }
  __device__ static __forceinline__ CQ qc(CQ q) { return q + (int)q[L::BO_OC]; }
  __device__ static __forceinline__ V3 rt(CQ q, V3 v) {  // R^T v
    CQ R = q + L::BO_R;
    return V3{R[0] * v.x + R[3] * v.y + R[6] * v.z, R[1] * v.x + R[4] * v.y + R[7] * v.z,
              R[2] * v.x + R[5] * v.y + R[8] * v.z};
  }
  __device__ static __forceinline__ V3 to_c(CQ q, V3 p) {
    CQ T = q + L::BO_T;
    return rt(q, V3{p.x - T[0], p.y - T[1], p.z - T[2]});
  }
  __device__ static __forceinline__ V3 at(V3 p, V3 d, double t) {
    return V3{p.x + t * d.x, p.y + t * d.y, p.z + t * d.z};
  }
  // entry of a part: 0 when the point is inside it or enters it at once
  __device__ static __forceinline__ double entry(int type, CQ q, V3 p, V3 d) {
    return fmax(prim_dist_in(type, q, p, d), 0.0);
  }
  // t + s for t >= 0, s > 0, but at least the next double above t: a part's
  // distance below the resolution of t (a point within rounding of a
  // surface) must still move the walk forward
  __device__ static __forceinline__ double ahead(double t, double s) {
    const double u = t + s;
    return u > t ? u : __longlong_as_double(__double_as_longlong(t) + 1);
  }

  __device__ __forceinline__ static double sgn(CQ q, V3 p) {
    const double a = prim_sgn(ta(q), qa(q), p), c = prim_sgn(tc(q), qc(q), to_c(q, p));
    const int o = op(q);
    return o == kUnion ? fmin(a, c) : (o == kSubtraction ? fmax(a, -c) : fmax(a, c));
  }

  // point outside: union min(SafetyToIn A, C); intersection the larger
  // SafetyToIn of the parts the point is outside of; A minus C the larger of
  // SafetyToIn A (outside A) and SafetyToOut C (inside C)
  __device__ __forceinline__ static double safety_in(CQ q, V3 p) {
    const int A = ta(q), C = tc(q), o = op(q);
    CQ a = qa(q), c = qc(q);
    const V3 pc = to_c(q, p);
    if (o == kUnion) return fmin(prim_safety_in(A, a, p), prim_safety_in(C, c, pc));
    double m = -GV_INF;
    if (code_of(prim_sgn(A, a, p)) == kOutside) m = fmax(m, prim_safety_in(A, a, p));
    const int cc = code_of(prim_sgn(C, c, pc));
    if (o == kSubtraction) {
      if (cc == kInside) m = fmax(m, prim_safety_out(C, c, pc));
    } else if (cc == kOutside) {
      m = fmax(m, prim_safety_in(C, c, pc));
    }
    return m == -GV_INF ? 0.0 : m;
  }

  // point inside: union the larger SafetyToOut of the parts holding it;
  // intersection min(SafetyToOut A, C); A minus C min(SafetyToOut A, SafetyToIn C)
  __device__ __forceinline__ static double safety_out(CQ q, V3 p) {
    const int A = ta(q), C = tc(q), o = op(q);
    CQ a = qa(q), c = qc(q);
    const V3 pc = to_c(q, p);
    if (o == kSubtraction) return fmin(prim_safety_out(A, a, p), prim_safety_in(C, c, pc));
    if (o == kIntersection) return fmin(prim_safety_out(A, a, p), prim_safety_out(C, c, pc));
    double m = -GV_INF;
    if (code_of(prim_sgn(A, a, p)) == kInside) m = fmax(m, prim_safety_out(A, a, p));
    if (code_of(prim_sgn(C, c, pc)) == kInside) m = fmax(m, prim_safety_out(C, c, pc));
    return m == -GV_INF ? 0.0 : m;
  }

  __device__ __forceinline__ static double dist_in(CQ q, V3 p, V3 d) {
    if (sgn(q, p) < -kHalf) return -1.0;
    const int A = ta(q), C = tc(q), o = op(q);
    CQ a = qa(q), c = qc(q);
    const V3 pc = to_c(q, p), dc = rt(q, d);
    if (o == kUnion) return fmin(entry(A, a, p, d), entry(C, c, pc, dc));
    double t = 0.0;
    for (int it = 0; it < kMaxIter; ++it) {
      const V3 x = at(p, d, t), xc = at(pc, dc, t);
      const double ea = entry(A, a, x, d);
      if (!(ea < GV_INF)) return GV_INF;
      double run;
      if (o == kIntersection) {
        const double ec = entry(C, c, xc, dc);
        if (!(ec < GV_INF)) return GV_INF;
        if (ea > 0.0 || ec > 0.0) {  // nothing before the later of the two entries
          t = ahead(t, fmax(ea, ec));
          continue;
        }
        run = fmin(prim_dist_out(A, a, x, d), prim_dist_out(C, c, xc, dc));
      } else {
        if (ea > 0.0) {
          t = ahead(t, ea);
          continue;
        }
        const double xcv = prim_dist_out(C, c, xc, dc);
        if (xcv > 0.0) {  // inside C: skip to its exit
          t = ahead(t, xcv);
          continue;
        }
        run = fmin(prim_dist_out(A, a, x, d), entry(C, c, xc, dc));
      }
      if (run >= kTol) return t;
      t = ahead(t, run);
    }
    return t;
  }

  __device__ __forceinline__ static double dist_out(CQ q, V3 p, V3 d) {
    if (sgn(q, p) > kHalf) return -1.0;
    const int A = ta(q), C = tc(q), o = op(q);
    CQ a = qa(q), c = qc(q);
    const V3 pc = to_c(q, p), dc = rt(q, d);
    if (o == kIntersection) return fmax(fmin(prim_dist_out(A, a, p, d), prim_dist_out(C, c, pc, dc)), 0.0);
    if (o == kSubtraction) return fmax(fmin(prim_dist_out(A, a, p, d), entry(C, c, pc, dc)), 0.0);
    double t = 0.0;
    for (int it = 0; it < kMaxIter; ++it) {
      const V3 x = at(p, d, t), xc = at(pc, dc, t);
      const double m = fmax(prim_dist_out(A, a, x, d), prim_dist_out(C, c, xc, dc));
      if (m > 0.0) {  // still inside a part: go to the farther exit
        t = ahead(t, m);
        continue;
      }
      const double e = fmin(entry(A, a, x, d), entry(C, c, xc, dc));
      if (e > 0.0 && e < kTol) {  // a part resumes within kTolerance
        t = ahead(t, e);
        continue;
      }
      return t;
    }
    return t;
  }
};

// Out-of-line entry points of the composite code for the navigation kernels
// (inlined there it would set their register budget for every geometry); the
// solid-level kernels, instantiated per solid type, inline Bool directly.
struct BoolCall {
  __device__ __noinline__ static double sgn(CQ q, V3 p) { return Bool::sgn(q, p); }
  __device__ __noinline__ static double safety_in(CQ q, V3 p) { return Bool::safety_in(q, p); }
  __device__ __noinline__ static double safety_out(CQ q, V3 p) { return Bool::safety_out(q, p); }
  __device__ __noinline__ static double dist_in(CQ q, V3 p, V3 d) { return Bool::dist_in(q, p, d); }
  __device__ __noinline__ static double dist_out(CQ q, V3 p, V3 d) { return Bool::dist_out(q, p, d); }
};

// Any solid.  B: the geometry may hold composites.  Kernels instantiated with
// B false (geometries of elementary solids only) contain no composite code.
template <bool B>
__device__ __forceinline__ double solid_sgn(int type, CQ q, V3 p) {
  if constexpr (B)
    if (type == kBool) return BoolCall::sgn(q, p);
  return prim_sgn(type, q, p);
}
template <bool B>
__device__ __forceinline__ double solid_dist_in(int type, CQ q, V3 p, V3 d) {
  if constexpr (B)
    if (type == kBool) return BoolCall::dist_in(q, p, d);
  return prim_dist_in(type, q, p, d);
}
template <bool B>
__device__ __forceinline__ double solid_dist_out(int type, CQ q, V3 p, V3 d) {
  if constexpr (B)
    if (type == kBool) return BoolCall::dist_out(q, p, d);
  return prim_dist_out(type, q, p, d);
}
template <bool B>
__device__ __forceinline__ double solid_safety_in(int type, CQ q, V3 p) {
  if constexpr (B)
    if (type == kBool) return BoolCall::safety_in(q, p);
  return prim_safety_in(type, q, p);
}
template <bool B>
__device__ __forceinline__ double solid_safety_out(int type, CQ q, V3 p) {
  if constexpr (B)
    if (type == kBool) return BoolCall::safety_out(q, p);
  return prim_safety_out(type, q, p);
}

}  // namespace gv
