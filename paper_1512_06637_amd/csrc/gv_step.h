// ComputeStep with culled daughter loops (Sec. III.A step selection).  The
// plain step takes the minimum of DistanceToIn over every daughter; the forms
// here reach the same daughter, the same length and the same flags with fewer
// full evaluations, by discarding daughters that provably cannot win.  Two
// screens do the discarding: a padded bounding-box slab test and the child's
// SafetyToIn, each a lower bound of the child's DistanceToIn.  Every distance
// that decides the step is computed in FP64.
//
// Precision FP32 + FP64 refinement runs both screens in FP32 on FP32 copies
// of the tables, with error margins that keep them conservative, and refines
// the surviving daughters in FP64: its outputs equal the FP64 form's bit for
// bit.  A wavefront whose rays fall outside the range the FP32 margins were
// sized for runs the FP64 screens for that step instead.
#pragma once
#include <type_traits>

#include "gv_kernels.h"
#include "gv_phys.h"

namespace gv {

// Work counters: steps, daughter bounding-box tests, then per daughter solid
// type the lower-bound checks, the full DistanceToIn evaluations of culled
// loops and those of plain loops (6 types each), then the track-steps of culled
// loops whose screens ran in FP32 and those that fell back to FP64 screens,
// then the physics-limited steps and those of them taken by the safety
// short-cut.
enum {
  kWorkSteps = 0,
  kWorkBox = 1,
  kWorkBound = 2,
  kWorkFull = 8,
  kWorkPlain = 14,
  kWorkScr32 = 20,
  kWorkScr64 = 21,
  kWorkPhys = 22,   // physics-limited steps
  kWorkShort = 23,  // of which taken without geometry (safety short-cut)
  kWorkRadial = 24,    // radial-order lookups (steps in an LV with a radial list)
  kWorkRadBound = 25,  // crossing-parameter bounds computed by the radial walk
  kWorkPhi = 26,       // phi-sector lookups
  kWorkPhiSec = 27,    // sectors whose masks were read
  kWorkN = 28
};

// Exact counting inside divergent code: the first active lane adds the number
// of active lanes (times `mult`, which must be wavefront-uniform) to an LDS
// counter of the workgroup.
__device__ __forceinline__ void count_active(unsigned long long* ctr, unsigned mult = 1) {
  uint64_t m = __ballot(1);
  if ((int)__lane_id() == __ffsll((unsigned long long)m) - 1) atomicAdd(ctr, (unsigned long long)__popcll(m) * mult);
}
struct LdsWork {
  unsigned long long* c;  // [kWorkN] in LDS
  __device__ __forceinline__ void add(int i, unsigned mult = 1) { count_active(&c[i], mult); }
};
struct NoWork {
  __device__ __forceinline__ NoWork(unsigned long long* = nullptr) {}
  __device__ __forceinline__ void add(int, unsigned = 1) {}
};

// ----------------------------------------------------------- plain loop
struct Placement {
  double R[12];
  int par;
};

__device__ __forceinline__ Placement load_placement(const DevGeom& G, int k) {
  Placement P;
  CQ Y = G.dau_xf + 12 * (size_t)k;
#pragma unroll
  for (int j = 0; j < 12; ++j) P.R[j] = Y[j];
  P.par = G.dau_par[k];
  return P;
}

template <class S>
__device__ __forceinline__ void daughters_of_type(const DevGeom& G, int off, int cnt, V3 pl, V3 dl, double& best,
                                                  int& bestk, bool& neg) {
  // the next placement is fetched while the current one is evaluated
  Placement cur = load_placement(G, off);
  for (int k = 0; k < cnt; ++k) {
    Placement nxt = load_placement(G, off + (k + 1 < cnt ? k + 1 : k));
    const double* R = cur.R;
    V3 pc, dc;
    {
      double q0 = pl.x - R[9], q1 = pl.y - R[10], q2 = pl.z - R[11];
      pc = V3{R[0] * q0 + R[3] * q1 + R[6] * q2, R[1] * q0 + R[4] * q1 + R[7] * q2, R[2] * q0 + R[5] * q1 + R[8] * q2};
      dc = V3{R[0] * dl.x + R[3] * dl.y + R[6] * dl.z, R[1] * dl.x + R[4] * dl.y + R[7] * dl.z,
              R[2] * dl.x + R[5] * dl.y + R[8] * dl.z};
    }
    double t = S::dist_in(G.par + cur.par, pc, dc);
    neg = neg || t < 0.0;
    t = fmax(t, 0.0);
    if (t < best) {
      best = t;
      bestk = k;
    }
    cur = nxt;
  }
}

// ------------------------------------------------------------- screens
constexpr float kU32 = 5.9604645e-08f;  // 2^-24, unit roundoff of FP32

struct F3 {
  float x, y, z;
};
__device__ __forceinline__ float max3f(float a, float b, float c) { return fmaxf(fmaxf(a, b), c); }

// Reciprocal direction components for the slab screens below, which form
// (B - p) / d as B * inv + (-p * inv).  A zero (or denormal) component would
// give an infinite reciprocal and then inf - inf = NaN or an infinity of the
// wrong sign; a huge finite value of the component's sign keeps the product
// difference finite with the sign of B - p (|B|, |p| < 2^20 mm).
__device__ __forceinline__ double inv_dir64(double d) {
  const double r = rcp_fast(d);
  return fabs(r) < 0x1p900 ? r : copysign(0x1p900, d);
}
__device__ __forceinline__ float inv_dir32(float d) {
  const float r = __builtin_amdgcn_rcpf(d);
  return fabsf(r) < 0x1p100f ? r : copysignf(0x1p100f, d);
}

// Whether a lane's ray may enter a padded box at a parameter in [0, bound]:
// false only when the ray provably misses the box or meets it beyond the
// bound.  Undecidable (NaN) comparisons keep the box.
__device__ __forceinline__ bool box_hit64(CQ B, V3 inv, V3 pin, double bound) {
  const double ax = fma(B[0], inv.x, pin.x), bx = fma(B[3], inv.x, pin.x);
  const double ay = fma(B[1], inv.y, pin.y), by = fma(B[4], inv.y, pin.y);
  const double az = fma(B[2], inv.z, pin.z), bz = fma(B[5], inv.z, pin.z);
  const double nr = fmax(fmax(fmin(ax, bx), fmin(ay, by)), fmin(az, bz));
  const double fr = fmin(fmin(fmax(ax, bx), fmax(ay, by)), fmax(az, bz));
  return !(nr > fr || fr < 0.0 || nr > bound);
}

// The same test in FP32.  The FP32 boxes are the FP64 ones widened by
// delta = 128 u (S + |box|inf), S of the mother, u = 2^-24, which covers the
// rounding of the point, of the direction over a parameter up to 4 S and of
// the slab arithmetic's absolute part, for every point with |p|inf <= S.  The
// parameters' remaining relative error (a few u) is covered by moving the
// entry down and the exit up by 8 u of their size before comparing.
__device__ __forceinline__ bool box_hit32(CQF B, F3 inv, F3 pin, float bound) {
  const float r = 8.0f * kU32;
  const float ax = fmaf(B[0], inv.x, pin.x), bx = fmaf(B[3], inv.x, pin.x);
  const float ay = fmaf(B[1], inv.y, pin.y), by = fmaf(B[4], inv.y, pin.y);
  const float az = fmaf(B[2], inv.z, pin.z), bz = fmaf(B[5], inv.z, pin.z);
  float nr = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fminf(az, bz));
  float fr = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fmaxf(az, bz));
  nr = fmaf(-r, fabsf(nr), nr);
  fr = fmaf(r, fabsf(fr), fr);
  return !(nr > fr || fr < 0.0f || nr > bound);
}

// Group size of the two-level box screen and the daughter count from which an
// LV gets group boxes (placement order is assumed to carry spatial locality;
// a group box is the union of its members' boxes, so the screen stays exact).
constexpr int kGroup = 8, kGroupMin = 16;

// Pass 1 over daughters c0 .. c0+m-1 (m <= 64) of an LV: per lane, the bit mask
// of daughters whose box the ray may enter within the bound.  With groups, a
// group whose box no lane of the wavefront enters skips its members' tests.
template <class Hit, class HitG, class W>
__device__ __forceinline__ uint64_t box_screen(int c0, int m, int grp, Hit hit, HitG hitg, W& w) {
  uint64_t cand = 0;
  if (grp < 0) {
    for (int k = 0; k < m; ++k) {
      const bool h = hit(c0 + k);
      cand |= h ? (1ull << k) : 0ull;
    }
    w.add(kWorkBox, (unsigned)m);
    return cand;
  }
  for (int g0 = 0; g0 < m; g0 += kGroup) {
    const bool gh = hitg(grp + (c0 + g0) / kGroup);
    w.add(kWorkBox);
    if (__ballot(gh) == 0) continue;
    const int mm = min(kGroup, m - g0);
    for (int k = 0; k < mm; ++k) {
      const bool h = gh && hit(c0 + g0 + k);
      cand |= h ? (1ull << (g0 + k)) : 0ull;
    }
    w.add(kWorkBox, (unsigned)mm);
  }
  return cand;
}

// FP32 lower bound of a box or tube child's SafetyToIn minus its error bound:
// max(|x|-dx, |y|-dy, |z|-dz) for a box, max(r-rmax, rmin-r, |z|-dz) for a tube
// (a subset of the terms of the FP64 formula, so never above it).  The point
// goes through R and t in FP32; the error of the result stays below
// 64 u (|p|inf + e), e = |t|inf + child extent + 1 mm.
template <class S>
__device__ __forceinline__ float lower_bound32(CQF Y, F3 p, float pmax) {
  const float q0 = p.x - Y[9], q1 = p.y - Y[10], q2 = p.z - Y[11];
  const float x = Y[0] * q0 + Y[3] * q1 + Y[6] * q2;
  const float y = Y[1] * q0 + Y[4] * q1 + Y[7] * q2;
  const float z = Y[2] * q0 + Y[5] * q1 + Y[8] * q2;
  float lb;
  if (S::kType == kBox) {
    lb = max3f(fabsf(x) - Y[12], fabsf(y) - Y[13], fabsf(z) - Y[14]);
  } else {
    const float rr = sqrtf(x * x + y * y);
    lb = max3f(rr - Y[13], Y[12] - rr, fabsf(z) - Y[14]);
  }
  return lb - 64.0f * kU32 * (pmax + Y[15]);
}

// ---------------------------------------------------------- culled loop
// A daughter can only win if its DistanceToIn is at most the mother's
// DistanceToOut (+ kTolerance, the daughter wins ties) and below the best
// daughter found so far, and its DistanceToIn is never below its padded
// bounding box's entry distance nor below its SafetyToIn.  Pass 1 tests every
// daughter's box against each lane's ray (table reads are uniform when the LV
// is) and collects per-lane candidate masks; pass 2 takes each lane's
// candidates in index order, checks the SafetyToIn bound, and evaluates
// DistanceToIn only where it can still win.  Index order with a strict < keeps
// the lowest index among equal minima, as the plain loop does.  left: a box
// daughter the ray has left (-1: none), not a candidate (as in daughters_phi).
template <class S, bool F32, class W>
__device__ __forceinline__ void daughters_culled(const DevGeom& G, int lv, int off, int cnt, V3 pl, V3 dl,
                                                 double dout, double& best, int& bestk, bool& neg, W& w,
                                                 int left) {
  const double bound = dout + kTol;
  bool use32 = false;
  F3 p32{}, inv32{}, pin32{};
  float pmax = 0.0f, bound32 = 0.0f;
  if (F32) {
    p32 = F3{(float)pl.x, (float)pl.y, (float)pl.z};
    pmax = max3f(fabsf(p32.x), fabsf(p32.y), fabsf(p32.z));
    const float sl = G.lv_scr[lv];
    const bool safe = pmax <= sl && bound <= 4.0 * (double)sl;
    use32 = __ballot(!safe) == 0;  // over the active lanes: all must be in range
    w.add(use32 ? kWorkScr32 : kWorkScr64, 1);
    if (use32) {
      inv32 = F3{inv_dir32((float)dl.x), inv_dir32((float)dl.y), inv_dir32((float)dl.z)};
      pin32 = F3{-p32.x * inv32.x, -p32.y * inv32.y, -p32.z * inv32.z};
      bound32 = (float)bound;
      bound32 = fmaf(4.0f * kU32, bound32, bound32);
    }
  }
  V3 inv{}, pin{};
  if (!use32) {
    inv = V3{inv_dir64(dl.x), inv_dir64(dl.y), inv_dir64(dl.z)};
    pin = V3{-pl.x * inv.x, -pl.y * inv.y, -pl.z * inv.z};
  }
  const int grp = G.lv_grp[lv];
  for (int c0 = 0; c0 < cnt; c0 += 64) {
    const int m = min(64, cnt - c0);
    uint64_t cand;
    if (use32) {
      cand = box_screen(
          c0, m, grp, [&](int k) { return box_hit32(G.dau_box32 + 8 * (size_t)(off + k), inv32, pin32, bound32); },
          [&](int gi) { return box_hit32(G.grp_box32 + 8 * (size_t)gi, inv32, pin32, bound32); }, w);
    } else {
      cand = box_screen(
          c0, m, grp, [&](int k) { return box_hit64(G.dau_box + 6 * (size_t)(off + k), inv, pin, bound); },
          [&](int gi) { return box_hit64(G.grp_box + 6 * (size_t)gi, inv, pin, bound); }, w);
    }
    if (S::kType == kBox && left >= c0 && left < c0 + m) cand &= ~(1ull << (left - c0));
    while (cand) {
      const int k = __builtin_ctzll(cand);
      cand &= cand - 1;
      const int pk = off + c0 + k;
      CQ Y = G.dau_xf + 12 * (size_t)pk;
      CQ q = G.par + G.dau_par[pk];
      const bool ident = G.dau_ident[pk] != 0;  // then the child frame is the mother's
      const double thr = fmin(best, dout) + kTol;
      w.add(kWorkBound + S::kType);
      V3 pc = pl;
      if (use32) {
        const float lb = lower_bound32<S>(G.dau_scr32 + 16 * (size_t)pk, p32, pmax);
        const float t32 = (float)thr;
        if (lb > fmaf(4.0f * kU32, t32, t32)) continue;
        if (!ident) pc = to_child_p(Y, pl);
      } else {
        if (!ident) pc = to_child_p(Y, pl);
        if (S::safety_in(q, pc) > thr) continue;
      }
      w.add(kWorkFull + S::kType);
      V3 dc = dl;
      if (!ident) dc = to_child_d(Y, dl);
      double t = S::dist_in(q, pc, dc);
      neg = neg || t < 0.0;
      t = fmax(t, 0.0);
      if (t < best) {
        best = t;
        bestk = c0 + k;
      }
    }
  }
}

constexpr int kCullMin = 8;  // LVs with fewer daughters run the plain loop

// Ordered radial walk over an LV's concentric tube daughters (identity
// placements, full tubes, disjoint radial ranges, listed by radius).  Along a
// ray r^2(t) = A t^2 + 2 B t + rho^2 is convex: a tube lying outside the
// start radius can only be entered at or after the parameter where the ray
// reaches its rmin moving outward, one lying inside only at or after the ray
// reaches its rmax moving inward, and both parameters grow with the tube's
// distance from the start radius.  So the tubes are visited outward and then
// inward from the start; each walk stops at the first tube whose parameter
// exceeds the best distance so far (or the mother's exit) by more than
// kTolerance + 1e-6 mm (a margin well above the parameters' rounding), and a
// tube radially holding the point is evaluated directly -- unless the ray
// leaves it within kTolerance / 8 while moving outward: a point that has just
// left a tube through its rmax holds it radially to rounding, and since r^2
// grows by at least 2 B t (B >= 0), rmax^2 - rho^2 < B kTolerance / 4 keeps
// the ray inside rmax for less than kTolerance / 8 (no entry) and the point
// within kTolerance / 2 of rmax (not inside), so the tube's DistanceToIn would
// return +inf.  Equal distances keep the lowest placement index, as the plain
// loop does.
template <class W>
__device__ __forceinline__ void daughters_radial(const DevGeom& G, int r0, int off, int cnt, V3 pl, V3 dl,
                                                 double dout, double& best, int& bestk, bool& neg, W& w) {
  CQ R2 = G.rad_r2 + 2 * (size_t)r0;
  CQI K = G.rad_k + r0;
  const double rho2 = pl.x * pl.x + pl.y * pl.y;
  const double A = dl.x * dl.x + dl.y * dl.y, B = pl.x * dl.x + pl.y * dl.y;
  w.add(kWorkRadial);
  int j = 0;  // entries with rmin^2 <= rho^2
  for (int m = 0; m < cnt; ++m) j += R2[2 * m] <= rho2 ? 1 : 0;
  auto eval = [&](int m) {
    const int k = K[m];
    w.add(kWorkFull + kTubs);
    double t = Tubs::dist_in(G.par + G.dau_par[off + k], pl, dl);
    neg = neg || t < 0.0;
    t = fmax(t, 0.0);
    if (t < best || (t == best && k < bestk)) {
      best = t;
      bestk = k;
    }
  };
  auto beyond = [&](double t) { return t - 1e-6 - 1e-12 * t > fmin(best, dout) + kTol; };
  const bool holds = j > 0 && rho2 <= R2[2 * (j - 1) + 1];
  if (holds && !(B >= 0.0 && R2[2 * (j - 1) + 1] - rho2 < 0.25 * kTol * B)) eval(j - 1);
  if (!(A > 0.0)) return;  // parallel to the axis: the radius never changes
  for (int m = j; m < cnt; ++m) {  // outward: larger root of A t^2 + 2 B t + (rho^2 - rmin^2), C < 0
    const double C = rho2 - R2[2 * m];
    const double sq = sqrt(B * B - A * C);
    const double t = B <= 0.0 ? div_fast(sq - B, A) : -div_fast(C, B + sq);
    w.add(kWorkRadBound);
    if (beyond(t)) break;
    eval(m);
  }
  if (!(B < 0.0)) return;  // moving outward: the radius only grows
  for (int m = holds ? j - 2 : j - 1; m >= 0; --m) {  // inward: smaller root with rmax^2, C > 0
    const double C = rho2 - R2[2 * m + 1];
    const double disc = B * B - A * C;
    if (disc < -1e-12 * (B * B + A * C)) break;  // misses rmax_m, hence every inner tube
    const double t = div_fast(C, sqrt(fmax(disc, 0.0)) - B);
    w.add(kWorkRadBound);
    if (beyond(t)) break;
    eval(m);
  }
}

// Daughters by phi sector: the ray's segment [0, exit + kTolerance] seen from
// the z axis sweeps an angle of less than a half turn (it does not pass within
// 1e-3 (|p|inf + 1) mm of the axis, else the culled loop runs instead); the
// union of the masks of the sectors it sweeps holds every daughter whose
// extent it can meet, and those candidates go through the SafetyToIn bound
// and DistanceToIn in index order, as in the culled loop's second pass.
// left: the index of a box daughter the ray has left (-1: none); a straight
// ray leaves a convex solid once, so it is not a candidate.
template <class S, bool F32, class W>
__device__ __forceinline__ void daughters_phi(const DevGeom& G, int lv, int m0, int off, int cnt, V3 pl, V3 dl,
                                              double dout, double& best, int& bestk, bool& neg, W& w, int left) {
  const double T = dout + kTol;
  const double A = dl.x * dl.x + dl.y * dl.y;
  const double tc = A > 0.0 ? fmin(fmax(-div_fast(pl.x * dl.x + pl.y * dl.y, A), 0.0), T) : 0.0;
  const double cx = pl.x + tc * dl.x, cy = pl.y + tc * dl.y;
  const double guard = 1e-3 * (fmax(fmax(fabs(pl.x), fabs(pl.y)), fabs(pl.z)) + 1.0);
  if (!(cx * cx + cy * cy > guard * guard) || !(T < GV_INF)) {
    daughters_culled<S, F32>(G, lv, off, cnt, pl, dl, dout, best, bestk, neg, w, left);
    return;
  }
  w.add(kWorkPhi);
  const double a0 = pseudo_angle_fast(pl.x, pl.y), a1 = pseudo_angle_fast(pl.x + T * dl.x, pl.y + T * dl.y);
  const bool ccw = pl.x * dl.y - pl.y * dl.x >= 0.0;
  auto sec = [](double a) { return min(kPhiSectors - 1, max(0, (int)(a * (kPhiSectors / 4.0)))); };
  const int s1 = sec(ccw ? a1 : a0);
  CQL M = G.phi_mask + (size_t)m0;
  uint64_t cand = 0;
  for (int s = sec(ccw ? a0 : a1);; s = (s + 1) & (kPhiSectors - 1)) {
    cand |= M[s];
    w.add(kWorkPhiSec);
    if (s == s1) break;
  }
  if (S::kType == kBox && left >= 0) cand &= ~(1ull << left);
  // FP32 screen of the bound (as in the culled loop): only when every active
  // lane's point and exit lie in the range the FP32 margins cover
  bool use32 = false;
  F3 p32{};
  float pmax = 0.0f;
  if (F32) {
    p32 = F3{(float)pl.x, (float)pl.y, (float)pl.z};
    pmax = max3f(fabsf(p32.x), fabsf(p32.y), fabsf(p32.z));
    const float sl = G.lv_scr[lv];
    use32 = __ballot(!(pmax <= sl && dout + kTol <= 4.0 * (double)sl)) == 0;
    w.add(use32 ? kWorkScr32 : kWorkScr64, 1);
  }
  while (cand) {
    const int k = __builtin_ctzll(cand);
    cand &= cand - 1;
    const int pk = off + k;
    CQ Y = G.dau_xf + 12 * (size_t)pk;
    CQ q = G.par + G.dau_par[pk];
    const bool ident = G.dau_ident[pk] != 0;
    const double thr = fmin(best, dout) + kTol;
    w.add(kWorkBound + S::kType);
    V3 pc = pl;
    if (use32) {
      const float lb = lower_bound32<S>(G.dau_scr32 + 16 * (size_t)pk, p32, pmax);
      const float t32 = (float)thr;
      if (lb > fmaf(4.0f * kU32, t32, t32)) continue;
      if (!ident) pc = to_child_p(Y, pl);
    } else {
      if (!ident) pc = to_child_p(Y, pl);
      if (S::safety_in(q, pc) > thr) continue;
    }
    w.add(kWorkFull + S::kType);
    const V3 dc = ident ? dl : to_child_d(Y, dl);
    double t = S::dist_in(q, pc, dc);
    neg = neg || t < 0.0;
    t = fmax(t, 0.0);
    if (t < best) {
      best = t;
      bestk = k;
    }
  }
}

// One ComputeStep of a track in placed volume pv (logical volume lv) with no
// physics limit.  Valid for any lv; fastest when lv is wavefront-uniform.
// left: placement index of a box daughter of lv the track has left along its
// present line (-1: none), which the ray cannot meet again; *exited (if given)
// says whether the step ends at the mother's exit.
template <bool F32, bool B, class W>
__device__ __forceinline__ double step_culled(const DevGeom& G, int lv, int pv, V3 p, V3 d, int* next,
                                              uint32_t* flags, W& w, int left = -1, bool* exited = nullptr) {
  CQ X = G.pv_gxf + 12 * (size_t)pv;
  V3 pl = to_child_p(X, p), dl = to_child_d(X, d);
  double dout = solid_dist_out<B>(G.lv_type[lv], G.par + G.lv_par[lv], pl, dl);
  uint32_t fl = *flags;
  if (dout < 0.0) {
    dout = 0.0;
    fl |= kFlagLocateFail;
  }
  double best = GV_INF;
  int bestk = -1;
  const int off = G.lv_dau_off[lv], cnt = G.lv_dau_cnt[lv], dtype = G.lv_dau_type[lv];
  bool neg = false;
  const int rad = G.lv_rad[lv], phs = G.lv_phi[lv];
  if (rad >= 0) {
    daughters_radial(G, rad, off, cnt, pl, dl, dout, best, bestk, neg, w);
  } else if (phs >= 0 && dtype == kBox) {
    daughters_phi<Box, F32>(G, lv, phs, off, cnt, pl, dl, dout, best, bestk, neg, w, left);
  } else if (phs >= 0 && dtype == kTubs) {
    daughters_phi<Tubs, F32>(G, lv, phs, off, cnt, pl, dl, dout, best, bestk, neg, w, -1);
  } else if (dtype == kBox && cnt >= kCullMin) {
    daughters_culled<Box, F32>(G, lv, off, cnt, pl, dl, dout, best, bestk, neg, w, left);
  } else if (dtype == kTubs && cnt >= kCullMin) {
    daughters_culled<Tubs, F32>(G, lv, off, cnt, pl, dl, dout, best, bestk, neg, w, -1);
  } else if (dtype == kBox) {
    daughters_of_type<Box>(G, off, cnt, pl, dl, best, bestk, neg);
    w.add(kWorkPlain + kBox, (unsigned)cnt);
  } else if (dtype == kTubs) {
    daughters_of_type<Tubs>(G, off, cnt, pl, dl, best, bestk, neg);
    w.add(kWorkPlain + kTubs, (unsigned)cnt);
  } else {
    for (int k = 0; k < cnt; ++k) {
      CQ Y = G.dau_xf + 12 * (size_t)(off + k);
      const int clv = G.dau_lv[off + k];
      V3 pc = to_child_p(Y, pl), dc = to_child_d(Y, dl);
      const int ct = G.lv_type[clv];
      double t = solid_dist_in<B>(ct, G.par + G.lv_par[clv], pc, dc);
      if (ct <= kPcon) w.add(kWorkPlain + ct);  // composites have no counter
      neg = neg || t < 0.0;
      t = fmax(t, 0.0);
      if (t < best) {
        best = t;
        bestk = k;
      }
    }
  }
  if (neg) fl |= kFlagLocateFail;
  *flags = fl;
  if (bestk >= 0 && best <= dout) {
    *next = G.pv_child[G.pv_child_off[pv] + bestk];
    if (exited) *exited = false;
    return best;
  }
  *next = G.pv_parent[pv];
  if (exited) *exited = true;
  return dout;
}

// ComputeStep with a physics limit: as step_culled, then the physics length
// wins when it is below both the daughter minimum and the exit.
template <bool F32, bool B, class W>
__device__ __forceinline__ double step_culled_limited(const DevGeom& G, int pv, V3 p, V3 d, double pstep, int* next,
                                                      uint32_t* flags, W& w) {
  int nx;
  const double s = step_culled<F32, B>(G, G.pv_lv[pv], pv, p, d, &nx, flags, w);
  // s is the daughter minimum when a daughter was chosen, else the exit
  if (pstep < s) {
    *next = pv;
    return pstep;
  }
  *next = nx;
  return s;
}

// Physics-limited ComputeStep (physics-limited transport).  `safe` is kept per
// track: the distance still to go along the ray to the boundary found by the
// last full ComputeStep.  The direction does not change at a physics step, so
// that boundary stays the first one on the ray; when the proposed physics length
// is below the distance still to go (by kTolerance, so that the rounding of the
// difference cannot matter) the step is physics-limited for sure and is taken
// without any geometry (the short-cut), and the distance shrinks by the step.
// Otherwise the full ComputeStep runs and, if physics wins, the distance is its
// geometric step minus the physics step; after a boundary step it is 0.  The
// short-cut never changes a result.
struct PhysArgs {
  uint64_t seed;
  int shortcut;
};

template <bool F32, bool B, class W>
__device__ __forceinline__ double step_physics(const DevGeom& G, int lv, int pv, V3& p, V3 d, uint32_t track, int k,
                                               const PhysArgs& P, double& safe, int* next, int* proc,
                                               uint32_t* flags, W& w, int left = -1, bool* exited = nullptr) {
  int pr = -1;
  const double ps = physics_length(G.mat_rate, G.n_proc, G.lv_mat[lv], P.seed, track, (uint32_t)k, &pr);
  if (P.shortcut && ps + kTol < safe) {
    w.add(kWorkPhys);
    w.add(kWorkShort);
    safe -= ps;
    *next = pv;
    *proc = pr;
    p = advance(p, ps, d);
    if (exited) *exited = false;
    return ps;
  }
  int nx;
  const double sg = step_culled<F32, B>(G, lv, pv, p, d, &nx, flags, w, left, exited);  // min(best daughter, exit)
  double st;
  if (ps < sg) {
    w.add(kWorkPhys);
    st = ps;
    *next = pv;
    *proc = pr;
    p = advance(p, st, d);
    safe = P.shortcut ? sg - ps : 0.0;
    if (exited) *exited = false;
  } else {
    st = sg;
    *next = nx;
    *proc = -1;
    p = advance(p, st, d);
    safe = 0.0;
  }
  return st;
}

// NavSafety with the FP32 SafetyToIn screen: a box or tube daughter is skipped
// when its FP32 lower bound (minus its error) exceeds both the running minimum
// and the surface half-band by kTolerance, i.e. when the point is provably
// outside it and it cannot lower the minimum.  Equal to nav_safety bit for bit.
template <bool B>
__device__ __forceinline__ double nav_safety_screened(const DevGeom& G, int pv, V3 p) {
  const int lv = G.pv_lv[pv];
  const V3 pl = to_child_p(G.pv_gxf + 12 * (size_t)pv, p);
  const int t = G.lv_type[lv];
  CQ q = G.par + G.lv_par[lv];
  if (code_of(solid_sgn<B>(t, q, pl)) != kInside) return 0.0;
  double s = solid_safety_out<B>(t, q, pl);
  const int off = G.lv_dau_off[lv], cnt = G.lv_dau_cnt[lv], dtype = G.lv_dau_type[lv];
  const F3 p32{(float)pl.x, (float)pl.y, (float)pl.z};
  const float pmax = max3f(fabsf(p32.x), fabsf(p32.y), fabsf(p32.z));
  const bool scr = dtype == kBox || dtype == kTubs;
  for (int k = 0; k < cnt; ++k) {
    if (scr) {
      CQF Y = G.dau_scr32 + 16 * (size_t)(off + k);
      const float lb = dtype == kBox ? lower_bound32<Box>(Y, p32, pmax) : lower_bound32<Tubs>(Y, p32, pmax);
      // kTolerance above the FP64 values keeps their own rounding from mattering
      const float t32 = (float)(fmax(s, kHalf) + kTol);
      if (lb > fmaf(4.0f * kU32, t32, t32)) continue;
    }
    const int clv = G.dau_lv[off + k];
    const V3 pc = to_child_p(G.dau_xf + 12 * (size_t)(off + k), pl);
    CQ qc = G.par + G.lv_par[clv];
    const int tc = G.lv_type[clv];
    if (code_of(solid_sgn<B>(tc, qc, pc)) != kOutside) return 0.0;
    s = fmin(s, solid_safety_in<B>(tc, qc, pc));
  }
  return fmax(s, 0.0);
}

// --------------------------------------------------------- per-lane kernels
// ComputeStep for every track of a basket, each lane in its own volume.
template <bool F32, bool B>
__global__ void k_step_nav(DevGeom G, int64_t n, const double* __restrict__ x, const double* __restrict__ y,
                           const double* __restrict__ z, const double* __restrict__ dx, const double* __restrict__ dy,
                           const double* __restrict__ dz, const int32_t* __restrict__ pv,
                           const double* __restrict__ pstep, double* __restrict__ out_step,
                           int32_t* __restrict__ out_next, uint32_t* __restrict__ out_flags) {
  NoWork w;
  for (int64_t i = gtid(); i < n; i += gstride()) {
    int v = pv[i];
    uint32_t fl = 0;
    int nx = -1;
    double st = 0.0;
    if (v >= 0 && v < G.n_pv) {
      st = step_culled_limited<F32, B>(G, v, ld3(x, y, z, i), ld3(dx, dy, dz, i), pstep ? pstep[i] : GV_INF, &nx, &fl,
                                    w);
    } else {
      fl = kFlagLocateFail;
    }
    out_step[i] = st;
    out_next[i] = nx;
    if (out_flags) out_flags[i] = fl;
  }
}

template <bool B>
__global__ void k_nav_safety_scr(DevGeom G, int64_t n, const double* __restrict__ x, const double* __restrict__ y,
                                 const double* __restrict__ z, const int32_t* __restrict__ pv,
                                 double* __restrict__ out) {
  for (int64_t i = gtid(); i < n; i += gstride()) {
    int v = pv[i];
    out[i] = (v >= 0 && v < G.n_pv) ? nav_safety_screened<B>(G, v, ld3(x, y, z, i)) : 0.0;
  }
}

}  // namespace gv
