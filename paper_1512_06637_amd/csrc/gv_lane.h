// Whole-track transport with one lane per track, persistent over the batch
// (Sec. III.A: a particle is stepped, volume after volume, until it leaves the
// geometry).
//
// The basket regrouping of gv_baskets.h keeps a wavefront's tracks in one
// logical volume by moving 16 bytes of indices per track and step and a
// 64-byte record through HBM.  With the daughter indexes of gv_step.h a step
// evaluates one or two daughter distances in any volume, so the divergence
// the regrouping avoids has become cheaper than the traffic it costs.  The
// form here keeps each track's state in registers for its whole life:
//
//  * coherent order -- the tracks are counting-sorted once by a direction
//    key (the octahedral map of the direction cut into 2^h x 2^h cells,
//    numbered along a Morton curve).  Straight tracks leaving a common region
//    in neighbouring directions cross the same volumes in the same order, so
//    the 64 lanes of a wavefront mostly run the same branch of the step and
//    read the same table entries.  The order changes no result: every track's
//    arithmetic is its own.
//  * persistent workers -- as many workgroups as the device holds at once;
//    each wavefront takes 64 consecutive places of the order from an atomic
//    counter and steps its tracks to the end, then takes the next 64.  The
//    64 tracks of a wavefront start together, so every step is taken by all
//    of its live lanes at once.  (Giving a lane whose track has ended a new
//    track at once was measured 2x slower: the lanes then run different
//    volume classes at every step.)
//
// Every output row is written by the lane that owns the track, so the results
// (sequences, lengths, counts, flags) are independent of the order and the
// grid.
#pragma once
#include "gv_step.h"

namespace gv {

constexpr int kSortMaxBits = 7;  // at most 2^7 x 2^7 direction cells
constexpr int kSortMaxCells = 1 << (2 * kSortMaxBits);

// Interleaves the low 7 bits of x with zeros (bit b to bit 2b).
__device__ __forceinline__ uint32_t spread_bits7(uint32_t x) {
  x &= 0x7Fu;
  x = (x | (x << 4)) & 0x0F0Fu;
  x = (x | (x << 2)) & 0x3333u;
  x = (x | (x << 1)) & 0x5555u;
  return x;
}

// Direction key: the octahedral map of the direction onto [-1, 1]^2 (the
// lower hemisphere folded over the diagonals), cut into 2^h x 2^h cells and
// numbered in Morton order, so that consecutive keys are neighbouring cones.
// Only the order of the work depends on it.
__device__ __forceinline__ uint32_t direction_key(double dx, double dy, double dz, int h) {
  const double a = fabs(dx) + fabs(dy) + fabs(dz);
  double u = dx / a, v = dy / a;
  if (dz < 0.0) {
    const double uu = (1.0 - fabs(v)) * (u < 0.0 ? -1.0 : 1.0), vv = (1.0 - fabs(u)) * (v < 0.0 ? -1.0 : 1.0);
    u = uu;
    v = vv;
  }
  const int side = 1 << h, m = side - 1;
  // a NaN converts to some integer, clamped into the grid: order only
  const uint32_t iu = (uint32_t)min(m, max(0, (int)((u + 1.0) * (0.5 * side))));
  const uint32_t iv = (uint32_t)min(m, max(0, (int)((v + 1.0) * (0.5 * side))));
  return spread_bits7(iu) | (spread_bits7(iv) << 1);
}

// Direction key aligned with the z axis: cos(theta) = dz cut into 2^h
// equal-area bands, the azimuth (pseudo-angle of (dx, dy)) into 2^h sectors,
// bands outermost, so that consecutive keys share a band and neighbouring
// azimuths -- the symmetry of detectors built around the z axis (layers in r,
// modules in phi).  Only the order of the work depends on it.
__device__ __forceinline__ uint32_t direction_key_zaxis(double dx, double dy, double dz, int h) {
  const int side = 1 << h, m = side - 1;
  const uint32_t it = (uint32_t)min(m, max(0, (int)((dz + 1.0) * (0.5 * side))));
  const uint32_t ip = (uint32_t)min(m, max(0, (int)(pseudo_angle(dx, dy) * (0.25 * side))));
  return it << h | ip;
}

// Lane-transport control words (device workspace): cnt[cells] key counts,
// then the running place of each cell during the scatter, and the work
// counter the persistent workers take places from.
struct LaneCtl {
  uint32_t* key;    // [n] direction key of each track
  int32_t* perm;    // [n] track of each place in the coherent order
  uint32_t* cnt;    // [cells] tracks per key
  uint32_t* queue;  // [1] next place to hand out
};

// Zeroes the key counts and the work counter before a transport.
__global__ void k_ls_clear(LaneCtl L, int cells) {
  for (int64_t i = gtid(); i < cells; i += gstride()) L.cnt[i] = 0u;
  if (gtid() == 0) *L.queue = 0u;
}

// Key of every track (z-axis or octahedral) and the per-key counts
// (workgroup histogram in LDS, 4 cells bytes of dynamic LDS, one global
// atomic per workgroup and key).
__global__ void k_ls_count(int64_t n, const double* __restrict__ dx, const double* __restrict__ dy,
                           const double* __restrict__ dz, int h, int zaxis, LaneCtl L) {
  extern __shared__ uint32_t key_hist[];
  const int cells = 1 << (2 * h);
  for (int c = threadIdx.x; c < cells; c += blockDim.x) key_hist[c] = 0u;
  __syncthreads();
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const uint32_t k = zaxis ? direction_key_zaxis(dx[i], dy[i], dz[i], h) : direction_key(dx[i], dy[i], dz[i], h);
    L.key[i] = k;
    atomicAdd(&key_hist[k], 1u);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < cells; c += blockDim.x)
    if (key_hist[c]) atomicAdd(&L.cnt[c], key_hist[c]);
}

// Exclusive scan of the key counts in place (one workgroup of 1024 threads):
// cnt[c] becomes the first place of key c.
__global__ void __launch_bounds__(1024) k_ls_scan(LaneCtl L, int cells) {
  __shared__ uint32_t part[1024];
  const int t = threadIdx.x;
  const int per = (cells + 1023) / 1024;
  const int c0 = t * per, c1 = min(cells, c0 + per);
  uint32_t s = 0;
  for (int c = c0; c < c1; ++c) s += L.cnt[c];
  part[t] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan over the 1024 partial sums
  for (int o = 1; o < 1024; o <<= 1) {
    const uint32_t v = t >= o ? part[t - o] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t run = t > 0 ? part[t - 1] : 0u;
  for (int c = c0; c < c1; ++c) {
    const uint32_t v = L.cnt[c];
    L.cnt[c] = run;
    run += v;
  }
}

// Places: each workgroup takes `chunk` consecutive tracks, counts their keys
// in LDS, reserves each key's run of places with one global atomic, and gives
// each of its tracks the next place of its key's run (4 cells bytes of
// dynamic LDS).  The order inside a key depends on the atomics' order, which
// changes no result.
__global__ void __launch_bounds__(1024) k_ls_scatter(int64_t n, int64_t chunk, int cells, LaneCtl L) {
  extern __shared__ uint32_t key_run[];
  const int64_t a = (int64_t)blockIdx.x * chunk, b = min(n, a + chunk);
  for (int c = threadIdx.x; c < cells; c += blockDim.x) key_run[c] = 0u;
  __syncthreads();
  for (int64_t i = a + threadIdx.x; i < b; i += blockDim.x) atomicAdd(&key_run[L.key[i]], 1u);
  __syncthreads();
  for (int c = threadIdx.x; c < cells; c += blockDim.x)
    if (key_run[c]) key_run[c] = atomicAdd(&L.cnt[c], key_run[c]);
  __syncthreads();
  for (int64_t i = a + threadIdx.x; i < b; i += blockDim.x) L.perm[atomicAdd(&key_run[L.key[i]], 1u)] = (int32_t)i;
}

// One track's state while a lane carries it.
struct LaneTrack {
  V3 p, d;
  double safe;  // physics: distance still to go to the last boundary found
  int64_t i;    // track index
  int pv, k, zero_run;
  int left;     // placement index of the box daughter of pv the track left last (-1: none)
  uint32_t fl;
  uint64_t procs;  // physics, staged outputs: the process codes of the run, byte k % 8 for step k
};

// Starts track i: its volume (given or located) and entry 0 of its sequence.
// Returns false (and writes the track's zero count and flags) when it starts
// outside the world.
template <bool B>
__device__ __forceinline__ bool lane_begin(const DevGeom& G, LaneTrack& T, int64_t i, const double* __restrict__ x,
                                           const double* __restrict__ y, const double* __restrict__ z,
                                           const double* __restrict__ dx, const double* __restrict__ dy,
                                           const double* __restrict__ dz, const int32_t* __restrict__ start_pv,
                                           int max_steps, int32_t* __restrict__ out_pv,
                                           int32_t* __restrict__ out_nsteps, uint32_t* __restrict__ out_flags) {
  T.i = i;
  T.p = ld3(x, y, z, i);
  T.d = ld3(dx, dy, dz, i);
  T.fl = 0u;
  T.k = 0;
  T.zero_run = 0;
  T.left = -1;
  T.safe = 0.0;
  T.procs = 0;
  int pv = start_pv ? start_pv[i] : locate<B>(G, T.p);
  if (pv < -1 || pv >= G.n_pv) {
    pv = -1;
    T.fl = kFlagLocateFail;
  }
  T.pv = pv;
  out_pv[(size_t)i * (max_steps + 1)] = pv;
  if (pv < 0) {
    out_nsteps[i] = 0;
    out_flags[i] = T.fl;
    return false;
  }
  return true;
}

// A lane's column of its wavefront's output staging in LDS: entry j of the
// column holds the j-th step since the last flush, 64 entries apart (the 64
// lanes write one row of the buffer per step, without bank conflicts).
struct LaneStage {
  double* st;
  int32_t* pv;
};

// One step of a carried track; returns true when the track has ended (left
// the world, stuck, or out of steps), after writing its count and flags.
// With ST > 0 the step length and next volume go to the lane's LDS column
// (and a physics step's process code to a byte of T.procs) and are written
// to the track's rows ST steps at a time (and at its end), so the row stores
// of a lane come in runs of consecutive addresses; all lanes of a wavefront
// that started together write their runs in the same iteration, and a full
// run goes out in 16-byte stores (its process codes in one 8-byte store).
template <bool F32, bool PHYS, bool B, int ST>
__device__ __forceinline__ bool lane_step(const DevGeom& G, LaneTrack& T, int lv, int pv, int max_steps,
                                          int32_t* __restrict__ out_pv, double* __restrict__ out_step,
                                          int32_t* __restrict__ out_nsteps, uint32_t* __restrict__ out_flags,
                                          const PhysArgs& P, int8_t* __restrict__ out_proc, LaneStage S) {
  static_assert(ST == 0 || ST == 8, "a staged run is 8 steps (the process codes of a run fill 64 bits)");
  NoWork w;
  int nx;
  double st;
  bool exited = false;
  if (PHYS) {
    int proc;
    st = step_physics<F32, B>(G, lv, pv, T.p, T.d, (uint32_t)T.i, T.k, P, T.safe, &nx, &proc, &T.fl, w, T.left,
                              &exited);
    if (ST == 0) {
      if (out_proc) out_proc[(size_t)T.i * max_steps + T.k] = (int8_t)proc;
    } else {
      T.procs |= (uint64_t)(uint8_t)proc << (8 * (T.k % 8));
    }
  } else {
    st = step_culled<F32, B>(G, lv, pv, T.p, T.d, &nx, &T.fl, w, T.left, &exited);
    T.p = advance(T.p, st, T.d);
  }
  // a track that leaves pv into its mother carries pv's placement index there
  // (the line does not change, so pv is behind it); entering a daughter clears it
  if (nx != pv) T.left = exited ? G.pv_k[pv] : -1;
  if (ST == 0) {
    out_step[(size_t)T.i * max_steps + T.k] = st;
    out_pv[(size_t)T.i * (max_steps + 1) + T.k + 1] = nx;
  } else {
    S.st[64 * (T.k % ST)] = st;
    S.pv[64 * (T.k % ST)] = nx;
  }
  ++T.k;
  bool end = nx < 0;
  if (!end) {
    T.zero_run = st < kTol ? T.zero_run + 1 : 0;
    if (T.zero_run >= 8) {
      T.fl |= kFlagStuck;
      end = true;
    } else if (T.k == max_steps) {
      T.fl |= kFlagOverflow;
      end = true;
    }
  }
  T.pv = nx;
  if (ST > 0 && (end || T.k % ST == 0)) {
    const int m = (T.k - 1) % ST + 1, k0 = T.k - m;
    double* rs = out_step + (size_t)T.i * max_steps + k0;
    int32_t* rp = out_pv + (size_t)T.i * (max_steps + 1) + k0 + 1;
    if (m == ST) {
      double vs[ST > 0 ? ST : 1];
      int32_t vp[ST > 0 ? ST : 1];
      for (int j = 0; j < ST; ++j) {
        vs[j] = S.st[64 * j];
        vp[j] = S.pv[64 * j];
      }
      __builtin_memcpy(rs, vs, sizeof vs);
      __builtin_memcpy(rp, vp, sizeof vp);
    } else {
      for (int j = 0; j < m; ++j) {
        rs[j] = S.st[64 * j];
        rp[j] = S.pv[64 * j];
      }
    }
    if (PHYS) {
      if (out_proc) {
        int8_t* rq = out_proc + (size_t)T.i * max_steps + k0;
        if (m == ST) {
          __builtin_memcpy(rq, &T.procs, 8);
        } else {
          for (int j = 0; j < m; ++j) rq[j] = (int8_t)(T.procs >> (8 * j));
        }
      }
      T.procs = 0;
    }
  }
  if (end) {
    out_nsteps[T.i] = T.k;
    out_flags[T.i] = T.fl;
  }
  return end;
}

// Persistent whole-track transport.  Places 0..n-1 of the order (perm, or the
// identity when perm is NULL) are handed out from *queue, which must be 0 at
// launch: a wavefront takes 64 places at a time and carries their tracks to
// their ends.  WV: waves per SIMD the kernel is built for (its register
// budget); ST: steps staged in LDS per lane before its rows are written (0:
// every step writes its rows at once).  CLS: per-class scheduling -- in each
// iteration only the lanes whose volume is in the step class (the branch of
// the step code: mother solid type and daughter access) that most live lanes
// are in take their step, and the others wait; lanes that fell behind (a
// track that crossed a module is two steps behind one that passed between
// modules) thus catch up before the wavefront moves on, instead of every
// iteration running the branches of every class with partial masks.
// (Taking each step one logical volume at a time with every lane stepping in
// every iteration, was measured 2.3x slower: lanes in different layers then
// run the same branch separately.  Giving a lane whose track has ended the
// next track at once, which let its new track wait for its class like any
// other, was measured slower as well: 2.66 against 2.56 ms.)
template <bool F32, bool PHYS, bool B, int WV, int ST, bool CLS = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WV))) k_lane_transport(
    DevGeom G, int64_t n, const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const double* __restrict__ dx, const double* __restrict__ dy, const double* __restrict__ dz,
    const int32_t* __restrict__ start_pv, const int32_t* __restrict__ perm, uint32_t* __restrict__ queue,
    int max_steps, int32_t* __restrict__ out_pv, double* __restrict__ out_step, int32_t* __restrict__ out_nsteps,
    uint32_t* __restrict__ out_flags, PhysArgs P, int8_t* __restrict__ out_proc) {
  constexpr int kStage = ST > 0 ? 4 * ST * 64 : 1;  // 4 wavefronts per workgroup
  __shared__ double stage_st[kStage];
  __shared__ int32_t stage_pv[kStage];
  const int lane = __lane_id();
  const int wbase = ST > 0 ? (int)(threadIdx.x / 64) * ST * 64 + lane : 0;
  const LaneStage S{stage_st + wbase, stage_pv + wbase};
  LaneTrack T;
  for (;;) {
    uint32_t b = 0;
    if (lane == 0) b = atomicAdd(queue, 64u);
    const int64_t base = (int64_t)__shfl(b, 0);
    if (base >= n) break;
    const int64_t j = base + lane;
    bool live = false;
    if (j < n) {
      const int64_t i = perm ? perm[j] : j;
      live = lane_begin<B>(G, T, i, x, y, z, dx, dy, dz, start_pv, max_steps, out_pv, out_nsteps, out_flags);
    }
    if (!CLS) {
      if (live)
        while (!lane_step<F32, PHYS, B, ST>(G, T, G.pv_lv[T.pv], T.pv, max_steps, out_pv, out_step, out_nsteps,
                                            out_flags, P, out_proc, S)) {
        }
      continue;
    }
    for (uint64_t lm = __ballot(live); lm; lm = __ballot(live)) {
      int lv = -1, cl = -1;
      if (live) {  // volume and class in one load
        const unsigned long long lc = reinterpret_cast<CQL>(G.pv_lc)[T.pv];
        lv = (int)(uint32_t)lc;
        cl = (int)(uint32_t)(lc >> 32);
      }
      // the class most live lanes are in (few classes are present at once;
      // on equal counts the first found)
      int best = -1, nbest = 0;
      for (uint64_t rest = lm; rest;) {
        const int c = __builtin_amdgcn_readlane(cl, __ffsll((unsigned long long)rest) - 1);
        const uint64_t m = __ballot(cl == c);
        const int nm = __popcll(m);
        if (nm > nbest) {
          nbest = nm;
          best = c;
        }
        rest &= ~m;
      }
      // When every stepping lane is in one logical volume (always in the
      // world, whose volume is unique; in a layer or a module when the
      // wavefront's tracks are all in one), the step runs with that volume
      // (and, for navigation, the placed volume too when shared) as
      // wavefront-uniform values: the volume's tables then come through
      // scalar loads instead of per-lane gathers.
      const bool mine = live && cl == best;
      const int lead = __ffsll((unsigned long long)__ballot(mine)) - 1;
      const int lv0 = __builtin_amdgcn_readlane(lv, lead);
      const bool uni_lv = __ballot(mine && lv != lv0) == 0;
      if (!PHYS && uni_lv) {
        const int pv0 = __builtin_amdgcn_readlane(T.pv, lead);
        if (__ballot(mine && T.pv != pv0) == 0) {
          if (mine)
            live = !lane_step<F32, PHYS, B, ST>(G, T, lv0, pv0, max_steps, out_pv, out_step, out_nsteps, out_flags,
                                                P, out_proc, S);
        } else if (mine) {
          live = !lane_step<F32, PHYS, B, ST>(G, T, lv0, T.pv, max_steps, out_pv, out_step, out_nsteps, out_flags, P,
                                              out_proc, S);
        }
      } else if (uni_lv) {
        if (mine)
          live = !lane_step<F32, PHYS, B, ST>(G, T, lv0, T.pv, max_steps, out_pv, out_step, out_nsteps, out_flags, P,
                                              out_proc, S);
      } else if (mine) {
        live = !lane_step<F32, PHYS, B, ST>(G, T, lv, T.pv, max_steps, out_pv, out_step, out_nsteps, out_flags, P,
                                            out_proc, S);
      }
    }
  }
}

}  // namespace gv
