// Basket transport: tracks are regrouped by the logical volume they are in
// before every step (the paper's baskets: particles located in the same kind of
// volume are collected and processed together, Sec. II.A item 1 and Sec. III.C).
//
// Track states stay in place (one 64-byte record per track, slot = track id);
// what is regrouped is a list of slot indices with one contiguous bucket per LV.
// A wavefront takes a tile of 64 consecutive list entries of one bucket, so its
// LV -- the mother solid and the whole daughter table -- is wavefront-uniform:
// the daughter loop reads transforms and solid parameters with scalar loads into
// SGPRs and the lanes never diverge on the solid type.  After the step each
// wavefront adds its tracks to the per-LV counts of the next step; a
// one-workgroup kernel turns the counts into the next bucket layout, and an
// index-scatter kernel writes each live slot index into its new bucket
// (workgroup-aggregated atomics keep one workgroup's writes to a bucket
// contiguous).  Per track and step that moves 12 bytes of indices instead of
// the 64-byte state.
#pragma once
#include "gv_step.h"

namespace gv {

constexpr int kWave = 64;

// one 64-byte record per track
struct alignas(64) TRec {
  double x, y, z, dx, dy, dz;
  int pv, zr, fl, pad;
};

__device__ __forceinline__ uint64_t lanemask_lt() { return __lanemask_lt(); }

// Per-step control arrays.  Counts and cursors are triple-buffered: step k
// reads counts k and accumulates counts k+1; the index kernel after it reads
// counts k+1 through cursors k+1 and clears counts and cursors k+2, which no
// kernel of steps k..k+1 reads.
struct TCtl {
  int* cnt[3];    // [nlv] tracks per LV in list k % 3
  int* cur[3];    // [nlv] index-scatter cursors of list k % 3
  unsigned long long* work;  // [kWorkN] operation counts of the current call
};

// wavefront-aggregated histogram update: one atomic per distinct LV in the wave
__device__ __forceinline__ void wave_count(int v, bool on, int* cnt) {
  uint64_t mask = __ballot(on);
  while (mask) {
    int leader = __ffsll((unsigned long long)mask) - 1;
    int lv = __shfl(v, leader);
    uint64_t m = __ballot(on && v == lv) & mask;
    if ((int)__lane_id() == leader) atomicAdd(&cnt[lv], __popcll(m));
    mask &= ~m;
  }
}

// Bucket layout of a list from its per-LV counts, computed by the first
// wavefront of the workgroup into LDS: start[b] (exclusive prefix, start[nlv] =
// total) and tile[b] (exclusive prefix of ceil(count/64), tile[nlv] = number
// of tiles).  Chunks of 64 LVs, a shuffle scan per chunk.  All threads of the
// workgroup must call it (it ends with a barrier); any block size works.
__device__ void block_layout(const int* __restrict__ cnt, int nlv, int* start, int* tile) {
  if (threadIdx.x < kWave) {
    const int lane = threadIdx.x;
    int carry = 0, tcarry = 0;
    for (int b0 = 0; b0 < nlv; b0 += kWave) {
      const int b = b0 + lane;
      const int c = b < nlv ? cnt[b] : 0;
      const int tc = (c + kWave - 1) / kWave;
      int s = c, ts = tc;  // inclusive scans
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        int u = __shfl_up(s, o), tu = __shfl_up(ts, o);
        if (lane >= o) {
          s += u;
          ts += tu;
        }
      }
      if (b < nlv) {
        start[b] = carry + s - c;
        tile[b] = tcarry + ts - tc;
      }
      carry += __shfl(s, kWave - 1);
      tcarry += __shfl(ts, kWave - 1);
    }
    if (lane == 0) {
      start[nlv] = carry;
      tile[nlv] = tcarry;
    }
  }
  __syncthreads();
}

// Clears the control arrays at the start of a transport.
__global__ void k_bt_clear(TCtl C, int nlv) {
  for (int64_t i = gtid(); i < nlv; i += gstride()) {
    for (int s = 0; s < 3; ++s) {
      C.cnt[s][i] = 0;
      C.cur[s][i] = 0;
    }
  }
  if (gtid() < kWorkN) C.work[gtid()] = 0ull;
}

// ---------------------------------------------------------------- init
// Start volume of every track (given or located), entry 0 of its sequence, its
// record, and the counts of the first layout.  Tracks that start outside the
// world finish here with zero steps.  List position = track id.
__global__ void k_bt_init(DevGeom G, int64_t n, const double* __restrict__ x, const double* __restrict__ y,
                          const double* __restrict__ z, const double* __restrict__ dx, const double* __restrict__ dy,
                          const double* __restrict__ dz, const int32_t* __restrict__ start_pv, int max_steps,
                          int32_t* __restrict__ out_pv, int32_t* __restrict__ out_nsteps,
                          uint32_t* __restrict__ out_flags, TRec* __restrict__ rec, int* __restrict__ nxt_lv, TCtl C) {
  int64_t stride = gstride();
  int64_t nround = ((n + stride - 1) / stride) * stride;
  for (int64_t i = gtid(); i < nround; i += stride) {
    bool act = i < n;
    int v = -1, lv = -1;
    if (act) {
      uint32_t fl = 0;
      V3 p = ld3(x, y, z, i);
      v = start_pv ? start_pv[i] : locate(G, p);
      if (v < -1 || v >= G.n_pv) {
        v = -1;
        fl = kFlagLocateFail;
      }
      out_pv[(size_t)i * (max_steps + 1)] = v;
      if (v < 0) {
        out_nsteps[i] = 0;
        out_flags[i] = fl;
      } else {
        lv = G.pv_lv[v];
        TRec r;
        r.x = p.x;
        r.y = p.y;
        r.z = p.z;
        r.dx = dx[i];
        r.dy = dy[i];
        r.dz = dz[i];
        r.pv = v;
        r.zr = 0;
        r.fl = 0;
        r.pad = 0;
        rec[i] = r;
      }
      nxt_lv[i] = lv;
    }
    wave_count(lv >= 0 ? lv : 0, lv >= 0, C.cnt[0]);
  }
}

// wavefront-aggregated reservation in an LDS counter array: returns, for lanes
// with on, old count + rank among the wave's lanes with the same value
__device__ __forceinline__ int wave_lds_reserve(int v, bool on, int* cnt) {
  uint64_t mask = __ballot(on);
  int pos = 0;
  while (mask) {
    int leader = __ffsll((unsigned long long)mask) - 1;
    int lv = __shfl(v, leader);
    uint64_t m = __ballot(on && v == lv) & mask;
    int base = 0;
    if ((int)__lane_id() == leader) base = atomicAdd(&cnt[lv], __popcll(m));
    base = __shfl(base, leader);
    if (on && v == lv) pos = base + __popcll(m & lanemask_lt());
    mask &= ~m;
  }
  return pos;
}

// Writes the slot index of every live entry of list k (positions [0, total of
// counts k), or [0, n) with identity slots for the first list) into its bucket
// of list k+1.  Each workgroup owns one contiguous range of entries: it counts
// them per destination LV in LDS, reserves one contiguous range per LV with a
// single global atomic, then writes them in a second pass.  Workgroup 0 also
// publishes the live count and clears counts and cursors of list k+2.  Needs
// 16 * nlv + 8 bytes of dynamic LDS.  `live` (nullable; device memory or
// mapped pinned host memory) receives the number of entries of list k+1.
__global__ void __launch_bounds__(1024) k_bt_reindex(const int* __restrict__ src_idx, const int* __restrict__ cnt_src,
                                                      int64_t nsrc_fixed, const int* __restrict__ nxt_lv,
                                                      int* __restrict__ dst_idx, const int* __restrict__ cnt_dst,
                                                      int* __restrict__ cur_dst, int* __restrict__ cnt_clear,
                                                      int* __restrict__ cur_clear, int* __restrict__ live, int nlv) {
  extern __shared__ int lds[];
  int* cnt = lds;
  int* base = lds + nlv;
  int* start = lds + 2 * nlv;     // nlv + 1 entries
  int* tile = lds + 3 * nlv + 1;  // nlv + 1 entries (unused here)
  block_layout(cnt_dst, nlv, start, tile);
  int64_t nsrc = nsrc_fixed;
  if (cnt_src) {
    __shared__ int total;
    if (threadIdx.x == 0) total = 0;
    __syncthreads();
    int acc = 0;
    for (int b = threadIdx.x; b < nlv; b += blockDim.x) acc += cnt_src[b];
    atomicAdd(&total, acc);
    __syncthreads();
    nsrc = total;
  }
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0 && live) __hip_atomic_store(live, start[nlv], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    for (int b = threadIdx.x; b < nlv; b += blockDim.x) {
      cnt_clear[b] = 0;
      cur_clear[b] = 0;
    }
  }
  const int64_t per = ((nsrc + gridDim.x - 1) / gridDim.x + blockDim.x - 1) / blockDim.x * blockDim.x;
  const int64_t j0 = (int64_t)blockIdx.x * per, j1 = min(nsrc, j0 + per);
  if (j0 >= j1) return;  // the whole workgroup leaves together
  for (int b = threadIdx.x; b < nlv; b += blockDim.x) cnt[b] = 0;
  __syncthreads();
  // every thread runs the same number of rounds (the round's first entry is < j1)
  for (int64_t j = j0 + threadIdx.x; j - threadIdx.x < j1; j += blockDim.x) {
    const int v = j < j1 ? nxt_lv[j] : -1;
    (void)wave_lds_reserve(v >= 0 ? v : 0, v >= 0, cnt);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nlv; b += blockDim.x) {
    int c = cnt[b];
    base[b] = c ? start[b] + atomicAdd(&cur_dst[b], c) : 0;
    cnt[b] = 0;
  }
  __syncthreads();
  for (int64_t j = j0 + threadIdx.x; j - threadIdx.x < j1; j += blockDim.x) {
    const int v = j < j1 ? nxt_lv[j] : -1;
    const int r = wave_lds_reserve(v >= 0 ? v : 0, v >= 0, cnt);
    if (v >= 0) dst_idx[base[v] + r] = src_idx ? src_idx[j] : (int)j;
  }
}

// ---------------------------------------------------------------- step
template <bool F32>
__global__ void __launch_bounds__(256) k_bt_step(DevGeom G, int k, int max_steps, const int* __restrict__ idx,
                                                  TRec* __restrict__ rec, const int* __restrict__ cnt_cur,
                                                  int* __restrict__ nxt_lv, int* __restrict__ cnt_next, TCtl C,
                                                  int32_t* __restrict__ out_pv, double* __restrict__ out_step,
                                                  int32_t* __restrict__ out_nsteps, uint32_t* __restrict__ out_flags) {
  // dynamic LDS: next-LV histogram [nlv], this list's layout start/tile [nlv+1] each
  extern __shared__ int lds[];
  __shared__ unsigned long long wsum[kWorkN];
  const int nlv = G.n_lv;
  int* hist = lds;
  int* start = lds + nlv;
  int* tilep = lds + 2 * nlv + 1;
  for (int v = threadIdx.x; v < nlv; v += blockDim.x) hist[v] = 0;
  for (int i = threadIdx.x; i < kWorkN; i += blockDim.x) wsum[i] = 0;
  block_layout(cnt_cur, nlv, start, tilep);
  LdsWork w{wsum};
  const int tiles = tilep[nlv];
  const int lane = __lane_id();
  const int wave = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave);
  const int nwaves = (int)(gridDim.x * (int64_t)blockDim.x / kWave);
  for (int t = wave; t < tiles; t += nwaves) {
    // bucket of tile t: largest b with tile[b] <= t (wavefront-uniform search)
    int lo = 0, hi = nlv - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (tilep[mid] <= t) lo = mid;
      else hi = mid - 1;
    }
    const int b = __builtin_amdgcn_readfirstlane(lo);
    const int j = t - tilep[b];
    const int within = j * kWave + lane;
    const bool act = within < start[b + 1] - start[b];
    const int e = start[b] + within;
    int nlv_out = -1;
    if (act) {
      const int id = idx[e];
      TRec r = rec[id];
      V3 p{r.x, r.y, r.z}, d{r.dx, r.dy, r.dz};
      uint32_t fl = (uint32_t)r.fl;
      int nx;
      double st = step_culled<F32>(G, b, r.pv, p, d, &nx, &fl, w);
      p = advance(p, st, d);
      out_step[(size_t)id * max_steps + k] = st;
      out_pv[(size_t)id * (max_steps + 1) + k + 1] = nx;
      int zr = st < kTol ? r.zr + 1 : 0;
      bool done = nx < 0;
      if (!done && zr >= 8) {
        fl |= kFlagStuck;
        done = true;
      }
      if (!done && k + 1 == max_steps) {
        fl |= kFlagOverflow;
        done = true;
      }
      if (done) {
        out_nsteps[id] = k + 1;
        out_flags[id] = fl;
      } else {
        rec[id].x = p.x;
        rec[id].y = p.y;
        rec[id].z = p.z;
        rec[id].pv = nx;
        rec[id].zr = zr;
        rec[id].fl = (int)fl;
        nlv_out = G.pv_lv[nx];
      }
      nxt_lv[e] = nlv_out;
    }
    if (act) count_active(&wsum[kWorkSteps]);
    wave_count(nlv_out >= 0 ? nlv_out : 0, nlv_out >= 0, hist);
  }
  __syncthreads();
  for (int v = threadIdx.x; v < nlv; v += blockDim.x)
    if (hist[v]) atomicAdd(&cnt_next[v], hist[v]);
  for (int i = threadIdx.x; i < kWorkN; i += blockDim.x)
    if (wsum[i]) atomicAdd(&C.work[i], wsum[i]);
}


}  // namespace gv
