// Kernels of the basket geometry library.  One lane handles one track; every
// launch is grid-stride over the basket, reading structure-of-arrays inputs
// with coalesced loads.  Solid-level kernels are instantiated per solid type so
// a wavefront never diverges on the type.
#pragma once
#include "gv_geom.h"

namespace gv {

__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }

// ------------------------------------------------------------ solid level
template <class S>
__global__ void k_inside(CQ q, int64_t n, const double* __restrict__ x,
                         const double* __restrict__ y, const double* __restrict__ z, int8_t* __restrict__ out) {
  for (int64_t i = gtid(); i < n; i += gstride()) out[i] = (int8_t)code_of(S::sgn(q, ld3(x, y, z, i)));
}

template <class S>
__device__ __forceinline__ double safety_value(CQ q, V3 p, int side, int c) {
  if (side == 1) {  // SafetyToIn
    if (c == kInside) return -1.0;
    if (c == kSurface) return 0.0;
    return fmax(S::safety_in(q, p), 0.0);
  }
  if (side == 2) {  // SafetyToOut
    if (c == kOutside) return -1.0;
    if (c == kSurface) return 0.0;
    return fmax(S::safety_out(q, p), 0.0);
  }
  if (c == kSurface) return 0.0;
  return c == kInside ? fmax(S::safety_out(q, p), 0.0) : fmax(S::safety_in(q, p), 0.0);
}

template <class S>
__global__ void k_safety(CQ q, int side, int64_t n, const double* __restrict__ x,
                         const double* __restrict__ y, const double* __restrict__ z, double* __restrict__ out,
                         int8_t* __restrict__ out_code) {
  for (int64_t i = gtid(); i < n; i += gstride()) {
    V3 p = ld3(x, y, z, i);
    int c = code_of(S::sgn(q, p));
    double v = safety_value<S>(q, p, side, c);
    if (out) out[i] = v;
    if (out_code) out_code[i] = (int8_t)c;
  }
}

template <class S, int DIR>
__global__ void k_distance(CQ q, int64_t n, const double* __restrict__ x,
                           const double* __restrict__ y, const double* __restrict__ z, const double* __restrict__ dx,
                           const double* __restrict__ dy, const double* __restrict__ dz, double* __restrict__ out) {
  for (int64_t i = gtid(); i < n; i += gstride()) {
    V3 p = ld3(x, y, z, i), d = ld3(dx, dy, dz, i);
    out[i] = DIR == 0 ? S::dist_in(q, p, d) : S::dist_out(q, p, d);
  }
}

// All four answers with one read of the basket.  Only the distance that is
// defined on the point's side is computed; the other is the -1 sentinel.
template <class S>
__global__ void k_solid_all(CQ q, int64_t n, const double* __restrict__ x,
                            const double* __restrict__ y, const double* __restrict__ z, const double* __restrict__ dx,
                            const double* __restrict__ dy, const double* __restrict__ dz, int8_t* __restrict__ o_in,
                            double* __restrict__ o_saf, double* __restrict__ o_din, double* __restrict__ o_dout) {
  for (int64_t i = gtid(); i < n; i += gstride()) {
    V3 p = ld3(x, y, z, i), d = ld3(dx, dy, dz, i);
    int c = code_of(S::sgn(q, p));
    if (o_in) o_in[i] = (int8_t)c;
    if (o_saf) o_saf[i] = safety_value<S>(q, p, 0, c);
    if (o_din) o_din[i] = c == kInside ? -1.0 : S::dist_in(q, p, d);
    if (o_dout) o_dout[i] = c == kOutside ? -1.0 : S::dist_out(q, p, d);
  }
}

// Polycone distances with the walking rays compacted per wavefront.  A
// wavefront takes 64 tracks at a time, answers those that need no walk (wrong
// side, and DistanceToIn rays that miss the bounding cylinder) and appends the
// others to its own LDS queue (ballot ranks); whenever the queue holds 64
// rays it walks them with all 64 lanes, and at the end the rest.  A quarter
// to a half of the rays walk and a wavefront's time is that of its longest
// walk, so walking them where they fall would pay that time in every
// wavefront with few lanes busy (18 % of lanes active per VALU instruction).
// No barrier couples the wavefronts of a workgroup.  Every ray takes the same
// steps as in Pcon::dist_in / dist_out (inside test, bounding-cylinder
// interval, walk), so the values are those of the one-lane-per-track kernels.
// KIND 0: DistanceToIn into o_din; 2: all four answers (k_solid_all's
// outputs, any of them NULL); 1: DistanceToOut into o_dout (not launched: half
// of the rays walk there, and compacting them measured no faster than the
// one-lane-per-track kernel).  Each wavefront takes 64 tracks at a time,
// grid-stride.
struct PconQueue {
  int64_t* idx;   // [128] queued tracks
  double* t0;     // [128] DistanceToIn walks: the bounding-cylinder interval
  double* t1;
  int n;          // wavefront-uniform count
};

// Appends lane's track i (if take) to the wavefront's queue Q.
__device__ __forceinline__ void pcon_push(PconQueue& Q, bool take, int64_t i, double a, double b) {
  const uint64_t m = __ballot(take);
  if (take) {
    const int k = Q.n + __popcll(m & ((1ull << __lane_id()) - 1));
    Q.idx[k] = i;
    if (Q.t0) {
      Q.t0[k] = a;
      Q.t1[k] = b;
    }
  }
  Q.n += __popcll(m);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Walks the first min(n, 64) queued rays (all of them when all), one per lane,
// and drops them from the queue.
template <bool IN>
__device__ __forceinline__ void pcon_walk(CQ q, PconQueue& Q, bool all, const double* __restrict__ x,
                                          const double* __restrict__ y, const double* __restrict__ z,
                                          const double* __restrict__ dx, const double* __restrict__ dy,
                                          const double* __restrict__ dz, double* __restrict__ out) {
  while (Q.n >= 64 || (all && Q.n > 0)) {
    const int lane = __lane_id();
    if (lane < Q.n) {
      const int64_t j = Q.idx[lane];
      const V3 p = ld3(x, y, z, j), d = ld3(dx, dy, dz, j);
      out[j] = IN ? Pcon::walk(q, p, d, true, nullptr, Q.t0[lane], Q.t1[lane]) : Pcon::walk(q, p, d, false);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane + 64 < Q.n) {  // move the rest to the front
      Q.idx[lane] = Q.idx[lane + 64];
      if (Q.t0) {
        Q.t0[lane] = Q.t0[lane + 64];
        Q.t1[lane] = Q.t1[lane + 64];
      }
    }
    Q.n = Q.n > 64 ? Q.n - 64 : 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

template <int KIND>
__global__ void __launch_bounds__(256) k_pcon_compact(CQ q, int64_t n, const double* __restrict__ x,
                                                      const double* __restrict__ y, const double* __restrict__ z,
                                                      const double* __restrict__ dx, const double* __restrict__ dy,
                                                      const double* __restrict__ dz, int8_t* __restrict__ o_in,
                                                      double* __restrict__ o_saf, double* __restrict__ o_din,
                                                      double* __restrict__ o_dout) {
  __shared__ int64_t s_in[4][128], s_out[4][128];
  __shared__ double s_t0[4][128], s_t1[4][128];
  const int w = threadIdx.x / 64, lane = __lane_id();
  const bool want_in = KIND == 0 || (KIND == 2 && o_din);
  const bool want_out = KIND == 1 || (KIND == 2 && o_dout);
  PconQueue Qi{s_in[w], s_t0[w], s_t1[w], 0}, Qo{s_out[w], nullptr, nullptr, 0};
  const int64_t nw = (int64_t)gridDim.x * 4;
  for (int64_t base = ((int64_t)blockIdx.x * 4 + w) * 64; base < n; base += nw * 64) {
    const int64_t i = base + lane;
    bool walk_in = false, walk_out = false;
    double t0 = 0.0, t1 = 0.0;
    if (i < n) {
      const V3 p = ld3(x, y, z, i), d = ld3(dx, dy, dz, i);
      const double sg = Pcon::sgn(q, p);
      const int c = code_of(sg);
      if (KIND == 2 && o_in) o_in[i] = (int8_t)c;
      if (KIND == 2 && o_saf) o_saf[i] = safety_value<Pcon>(q, p, 0, c);
      if (want_in) {
        if ((KIND == 2 && c == kInside) || sg < -kHalf) {
          o_din[i] = -1.0;
        } else {
          const Iv B = Pcon::bound_iv(Pcon::view(q), p, d);
          if (Pcon::misses(B)) {
            o_din[i] = GV_INF;
          } else {
            walk_in = true;
            t0 = fmax(B.lo, 0.0);
            t1 = B.hi;
          }
        }
      }
      if (want_out) {
        if ((KIND == 2 && c == kOutside) || sg > kHalf)
          o_dout[i] = -1.0;
        else
          walk_out = true;
      }
    }
    if (want_in) {
      pcon_push(Qi, walk_in, i, t0, t1);
      pcon_walk<true>(q, Qi, false, x, y, z, dx, dy, dz, o_din);
    }
    if (want_out) {
      pcon_push(Qo, walk_out, i, 0.0, 0.0);
      pcon_walk<false>(q, Qo, false, x, y, z, dx, dy, dz, o_dout);
    }
  }
  if (want_in) pcon_walk<true>(q, Qi, true, x, y, z, dx, dy, dz, o_din);
  if (want_out) pcon_walk<false>(q, Qo, true, x, y, z, dx, dy, dz, o_dout);
}

// Work of the polycone distance queries (profiling only, no outputs): per
// track as one query (dir 0 in, 1 out) or the fused one (dir 2: DistanceToIn
// of points not inside, DistanceToOut of points not outside) would run it,
// adds to out[0] / out[1]
// the sections whose cone intersections the DistanceToIn / DistanceToOut
// walks compute, to out[2] the DistanceToIn rays rejected by the bounding
// cylinder, and to out[3] / out[4] the walks (one atomic per wavefront and
// counter).
__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__global__ void k_pcon_work(CQ q, int dir, int64_t n, const double* __restrict__ x, const double* __restrict__ y,
                            const double* __restrict__ z, const double* __restrict__ dx,
                            const double* __restrict__ dy, const double* __restrict__ dz,
                            unsigned long long* __restrict__ out) {
  unsigned long long c[5] = {0, 0, 0, 0, 0};
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const V3 p = ld3(x, y, z, i), d = ld3(dx, dy, dz, i);
    const int code = code_of(Pcon::sgn(q, p));
    if (dir != 1 && code != kInside) {
      const Iv B = Pcon::bound_iv(Pcon::view(q), p, d);
      if (Pcon::misses(B)) {
        ++c[2];
      } else {
        int ns = 0;
        (void)Pcon::walk<true>(q, p, d, true, &ns, fmax(B.lo, 0.0), B.hi);
        c[0] += ns;
        ++c[3];
      }
    }
    if (dir != 0 && code != kOutside) {
      int ns = 0;
      (void)Pcon::walk<true>(q, p, d, false, &ns);
      c[1] += ns;
      ++c[4];
    }
  }
  for (int k = 0; k < 5; ++k) {
    const unsigned long long t = wave_sum(c[k]);
    if (__lane_id() == 0 && t) atomicAdd(&out[k], t);
  }
}

// ------------------------------------------------------------- navigation
template <bool B>
__global__ void k_locate(DevGeom G, int64_t n, const double* __restrict__ x, const double* __restrict__ y,
                         const double* __restrict__ z, int32_t* __restrict__ out) {
  for (int64_t i = gtid(); i < n; i += gstride()) out[i] = locate<B>(G, ld3(x, y, z, i));
}

template <bool B>
__global__ void k_nav_safety(DevGeom G, int64_t n, const double* __restrict__ x, const double* __restrict__ y,
                             const double* __restrict__ z, const int32_t* __restrict__ pv, double* __restrict__ out) {
  for (int64_t i = gtid(); i < n; i += gstride()) {
    int v = pv[i];
    out[i] = (v >= 0 && v < G.n_pv) ? nav_safety<B>(G, v, ld3(x, y, z, i)) : 0.0;
  }
}

template <bool B>
__global__ void k_nav_inside(DevGeom G, int64_t n, const double* __restrict__ x, const double* __restrict__ y,
                             const double* __restrict__ z, const int32_t* __restrict__ pv, int8_t* __restrict__ out) {
  for (int64_t i = gtid(); i < n; i += gstride()) {
    int v = pv[i];
    if (v < 0 || v >= G.n_pv) {
      out[i] = (int8_t)kOutside;
      continue;
    }
    int lv = G.pv_lv[v];
    V3 pl = to_child_p(G.pv_gxf + 12 * (size_t)v, ld3(x, y, z, i));
    out[i] = (int8_t)code_of(solid_sgn<B>(G.lv_type[lv], G.par + G.lv_par[lv], pl));
  }
}

// p + s d without FMA: the global point advances exactly as a plain FP64 code
// would, so the position does not drift through contraction.
__device__ __forceinline__ V3 advance(V3 p, double s, V3 d) {
#pragma clang fp contract(off)
  return V3{p.x + s * d.x, p.y + s * d.y, p.z + s * d.z};
}

}  // namespace gv
