// Basket transport: tracks are regrouped by the logical volume they are in
// before every step (the paper's baskets: particles located in the same kind of
// volume are collected and processed together, Sec. II.A item 1 and Sec. III.C).
//
// Track states stay in place (one 64-byte record per track, slot = track id);
// what is regrouped is a list of slot indices with one contiguous bucket per
// (LV, coarse direction cell), the cells of one LV next to each other.  A
// wavefront takes a tile of 64 consecutive list entries of one LV's range, so
// its LV -- the mother solid and the whole daughter table -- is
// wavefront-uniform: the daughter loop reads transforms and solid
// parameters with scalar loads into SGPRs and the lanes never diverge on the
// solid type.  The direction cell keeps a tile's rays within one cone of
// directions, so they tend to meet the same daughters (the group screen of the
// culled loop then skips most daughters for the whole wavefront).  After the
// step each workgroup reserves, per next bucket, one share with a single
// atomic on the bucket's count and gives each of its tracks a rank in its
// share (LDS atomics); a scatter kernel then writes each live slot index at
// bucket start + share offset + rank.  Per track and step that moves 16 bytes
// of indices instead of the 64-byte state.
#pragma once
#include "gv_phys.h"
#include "gv_step.h"

namespace gv {

constexpr int kWave = 64;

// One 64-byte record per track (one cache line), read and rewritten whole
// every step.
struct alignas(64) TRec {
  double x, y, z, dx, dy, dz;
  double safe;  // physics-limited transport: lower bound of the distance to the volume's boundaries
  int pv;
  // zero-length steps in a row (bits 0-3) | flags (4-7) | 1 + placement index
  // of the box daughter of pv the track left last (8-15; 0: none, or an index
  // beyond 254, which only forgoes skipping it) | coarse direction cell (16-31)
  int zfc;
};
static_assert(sizeof(TRec) == 64, "record layout");
static_assert((kFlagOverflow | kFlagStuck | kFlagLocateFail) <= 0xfu, "flags fit in 4 bits");
__device__ __forceinline__ int zfc_pack(int zr, uint32_t fl, int left, int cc) {
  return zr | (int)(fl << 4) | ((left >= 0 && left < 255 ? left + 1 : 0) << 8) | (cc << 16);
}
__device__ __forceinline__ int zfc_zr(int v) { return v & 0xf; }
__device__ __forceinline__ uint32_t zfc_fl(int v) { return (uint32_t)(v >> 4) & 0xfu; }
__device__ __forceinline__ int zfc_left(int v) { return ((v >> 8) & 0xff) - 1; }
__device__ __forceinline__ int zfc_cc(int v) { return (v >> 16) & 0xffff; }

__device__ __forceinline__ uint64_t lanemask_lt() { return __lanemask_lt(); }

// Per-step control arrays.  Counts are triple-buffered: step k reads counts k
// and accumulates counts k+1; the scatter kernel after it reads counts k+1 and
// clears counts k+2, which no kernel of steps k..k+1 reads.
struct TCtl {
  int* cnt[3];    // [nlv] tracks per bucket in list k % 3
  int* cur[3];    // [nlv] cursors of the first list's index kernel
  unsigned long long* work;  // [kWorkN] operation counts of the current call
  int* nlive;                // live tracks at the start (slots in use)
  int* seg;                  // [kMaxStepGrid][nb] offset of a step workgroup's share of each next bucket
  int* len;                  // [2] list lengths: list k in len[k & 1] (list 0 in nlive)
};

// Step-kernel workgroups at most, and the packing of an entry's place in the
// next list: workgroup (high 10 bits) | rank within that workgroup's share of
// its bucket (low 22 bits).
constexpr int kMaxStepGrid = 1024;
constexpr int kRankBits = 22;

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

// Bucket layout of a list from its per-bucket counts `cnt` (in LDS), computed
// by the first wavefront of the workgroup: start[b] (exclusive prefix,
// start[nlv] = total) and tile[b] (exclusive prefix of ceil(count/64),
// tile[nlv] = number of tiles; tile may be NULL).  Chunks of 64 buckets, a
// shuffle scan per chunk.  All threads of the workgroup must call it (it ends
// with a barrier); any block size works.
__device__ void block_layout(const int* cnt, int nlv, int* start, int* tile) {
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
        if (tile) tile[b] = tcarry + ts - tc;
      }
      carry += __shfl(s, kWave - 1);
      tcarry += __shfl(ts, kWave - 1);
    }
    if (lane == 0) {
      start[nlv] = carry;
      if (tile) tile[nlv] = tcarry;
    }
  }
  __syncthreads();
}

// Copies n counts from global memory into LDS with every thread of the
// workgroup (one round trip), then a barrier.
__device__ __forceinline__ void stage_counts(const int* __restrict__ src, int n, int* dst) {
  for (int b = threadIdx.x; b < n; b += blockDim.x) dst[b] = src[b];
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
// Coarse direction cell of a unit direction: the octahedral map onto
// [-1, 1]^2 cut into 2^(cb/2) x 2^(cb/2) cells (cb even, <= 4).  Tracks of one
// bucket then share a cone of directions.
__device__ __forceinline__ int dir_cell(double dx, double dy, double dz, int cb) {
  const double a = fabs(dx) + fabs(dy) + fabs(dz);
  double u = dx / a, v = dy / a;
  if (dz < 0.0) {
    const double uu = (1.0 - fabs(v)) * (u < 0.0 ? -1.0 : 1.0), vv = (1.0 - fabs(u)) * (v < 0.0 ? -1.0 : 1.0);
    u = uu;
    v = vv;
  }
  const int side = 1 << (cb / 2), m = side - 1;
  const int iu = min(m, max(0, (int)((u + 1.0) * (0.5 * side))));
  const int iv = min(m, max(0, (int)((v + 1.0) * (0.5 * side))));
  return iv * side + iu;
}

// Start volume of every track (given or located), entry 0 of its sequence,
// and its start bucket (LV, coarse direction cell) into key, with the bucket
// counts of the first list (per-workgroup LDS histogram, 4 nb bytes of dynamic
// LDS).  Tracks that start outside the world finish here with zero steps and
// get bucket -1.
template <bool B>
__global__ void k_bt_init(DevGeom G, int64_t n, const double* __restrict__ x, const double* __restrict__ y,
                          const double* __restrict__ z, const double* __restrict__ dx, const double* __restrict__ dy,
                          const double* __restrict__ dz, const int32_t* __restrict__ start_pv, int max_steps,
                          int32_t* __restrict__ out_pv, int32_t* __restrict__ out_nsteps,
                          uint32_t* __restrict__ out_flags, int* __restrict__ key, int cb, TCtl C) {
  extern __shared__ int hist[];
  const int nb = G.n_lv << cb;
  for (int v = threadIdx.x; v < nb; v += blockDim.x) hist[v] = 0;
  __syncthreads();
  int64_t stride = gstride();
  int64_t nround = ((n + stride - 1) / stride) * stride;
  for (int64_t i = gtid(); i < nround; i += stride) {
    bool act = i < n;
    int bk = -1;
    if (act) {
      uint32_t fl = 0;
      V3 p = ld3(x, y, z, i);
      int v = start_pv ? start_pv[i] : locate<B>(G, p);
      if (v < -1 || v >= G.n_pv) {
        v = -1;
        fl = kFlagLocateFail;
      }
      out_pv[(size_t)i * (max_steps + 1)] = v;
      if (v < 0) {
        out_nsteps[i] = 0;
        out_flags[i] = fl;
      } else {
        bk = G.pv_lv[v] << cb | dir_cell(dx[i], dy[i], dz[i], cb);
      }
      key[i] = bk;
    }
    wave_count(bk >= 0 ? bk : 0, bk >= 0, hist);
  }
  __syncthreads();
  for (int v = threadIdx.x; v < nb; v += blockDim.x)
    if (hist[v]) atomicAdd(&C.cnt[0][v], hist[v]);
}

// Slots: the live tracks renumbered in the order of the first list (ordered by
// bucket), so the tracks of a tile are mostly consecutive slots and their
// records and staged outputs are read and written in contiguous runs.  Slot s
// takes track perm[s]: its record, slot_id[s] = track id, and entry s of the
// first list.  Also stores the number of live tracks.
__global__ void k_bt_place(const int* __restrict__ perm, const double* __restrict__ x, const double* __restrict__ y,
                           const double* __restrict__ z, const double* __restrict__ dx,
                           const double* __restrict__ dy, const double* __restrict__ dz,
                           const int32_t* __restrict__ out_pv, int max_steps, int cb, int nb, TRec* __restrict__ rec,
                           int* __restrict__ slot_id, int* __restrict__ list0, TCtl C) {
  __shared__ int total;
  if (threadIdx.x == 0) total = 0;
  __syncthreads();
  int acc = 0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += C.cnt[0][b];
  atomicAdd(&total, acc);
  __syncthreads();
  const int64_t nl = total;
  if (blockIdx.x == 0 && threadIdx.x == 0) *C.nlive = (int)nl;
  for (int64_t sl = gtid(); sl < nl; sl += gstride()) {
    const int id = perm[sl];
    TRec r;
    r.x = x[id];
    r.y = y[id];
    r.z = z[id];
    r.dx = dx[id];
    r.dy = dy[id];
    r.dz = dz[id];
    r.safe = 0.0;
    r.pv = out_pv[(size_t)id * (max_steps + 1)];
    r.zfc = zfc_pack(0, 0u, -1, dir_cell(r.dx, r.dy, r.dz, cb));
    rec[sl] = r;
    slot_id[sl] = id;
    list0[sl] = (int)sl;
  }
}

// Outputs staged step-major by slot (entry k * cap + s) go to the caller's
// row-per-track arrays: a workgroup takes 64 slots and moves them through LDS
// 64 steps at a time, so both the staged reads (64 slots of one step) and the
// row writes (64 steps of one track) are contiguous.  Only the kmax steps that
// were run are read; entries past a track's step count are not written.  The
// process indices of physics-limited transport move along when staged.
template <bool PROC>
__global__ void __launch_bounds__(512) k_bt_emit(const double* __restrict__ ob_step, const int* __restrict__ ob_pv,
                                                 const int8_t* __restrict__ ob_proc, int64_t cap,
                                                 const int* __restrict__ slot_id, TCtl C, int max_steps, int kmax,
                                                 const int32_t* __restrict__ out_nsteps, double* __restrict__ out_step,
                                                 int32_t* __restrict__ out_pv, int8_t* __restrict__ out_proc) {
  __shared__ double ts[64][65];
  __shared__ int tp[64][65];
  __shared__ int8_t tq[PROC ? 64 : 1][65];
  __shared__ int sid[64], sns[64], kwg;
  const int64_t s0 = (int64_t)blockIdx.x * 64;
  const int64_t nl = *C.nlive;
  if (s0 >= nl) return;  // the whole workgroup leaves together
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (threadIdx.x < 64) {
    const int64_t sl = s0 + threadIdx.x;
    int id = 0, ns = 0;
    if (sl < nl) {
      id = slot_id[sl];
      ns = min(out_nsteps[id], kmax);
    }
    sid[threadIdx.x] = id;
    sns[threadIdx.x] = ns;
    int m = ns;  // the workgroup's longest track bounds its step loop
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o));
    if (threadIdx.x == 0) kwg = m;
  }
  __syncthreads();
  const int kend = kwg;
  for (int k0 = 0; k0 < kend; k0 += 64) {
    __syncthreads();
    for (int r = wv; r < 64; r += 8) {  // row r = step k0 + r, lanes = slots
      const int k = k0 + r;
      const int64_t sl = s0 + lane;
      if (k < sns[lane]) {  // steps a slot did not take hold stale values
        ts[lane][r] = ob_step[(size_t)k * cap + sl];
        tp[lane][r] = ob_pv[(size_t)k * cap + sl];
        if (PROC) tq[lane][r] = ob_proc[(size_t)k * cap + sl];
      }
    }
    __syncthreads();
    for (int r = wv; r < 64; r += 8) {  // row r = slot s0 + r, lanes = steps
      const int k = k0 + lane;
      if (k < sns[r]) {
        const int id = sid[r];
        out_step[(size_t)id * max_steps + k] = ts[r][lane];
        out_pv[(size_t)id * (max_steps + 1) + k + 1] = tp[r][lane];
        if (PROC) out_proc[(size_t)id * max_steps + k] = tq[r][lane];
      }
    }
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

// Writes the slot index of every live entry of a list into its bucket of the
// next list.  The source is list k (positions [0, sum of cnt_src[0..nsrc_bins)),
// slots src_idx) or, with cnt_src NULL, positions [0, nsrc_fixed) with slots
// src_idx (identity if NULL).  The destination bucket of position j is key[j],
// or key[slot] with `gather`; negative keys are dropped.  Each workgroup owns
// one contiguous range of positions: it counts them per bucket in LDS, reserves
// one contiguous range per bucket with a single global atomic, then writes them
// in a second pass, so a workgroup's entries keep their order in each bucket.
// Workgroup 0 clears cnt_clear/cur_clear (nullable).  Needs 12 * nb + 4 bytes
// of dynamic LDS.
__global__ void __launch_bounds__(1024) k_bt_reindex(const int* __restrict__ src_idx, const int* __restrict__ cnt_src,
                                                      int nsrc_bins, int64_t nsrc_fixed, const int* __restrict__ key,
                                                      int gather, int* __restrict__ dst_idx,
                                                      const int* __restrict__ cnt_dst, int* __restrict__ cur_dst,
                                                      int* __restrict__ cnt_clear, int* __restrict__ cur_clear,
                                                      int nb) {
  extern __shared__ int lds[];
  int* cnt = lds;
  int* base = lds + nb;
  int* start = lds + 2 * nb;  // nb + 1 entries
  stage_counts(cnt_dst, nb, base);  // base is free until the layout is done
  block_layout(base, nb, start, nullptr);
  int64_t nsrc = nsrc_fixed;
  if (cnt_src) {
    __shared__ int total;
    if (threadIdx.x == 0) total = 0;
    __syncthreads();
    int acc = 0;
    for (int b = threadIdx.x; b < nsrc_bins; b += blockDim.x) acc += cnt_src[b];
    atomicAdd(&total, acc);
    __syncthreads();
    nsrc = total;
  }
  if (blockIdx.x == 0) {
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
      if (cnt_clear) cnt_clear[b] = 0;
      if (cur_clear) cur_clear[b] = 0;
    }
  }
  const int64_t per = ((nsrc + gridDim.x - 1) / gridDim.x + blockDim.x - 1) / blockDim.x * blockDim.x;
  const int64_t j0 = (int64_t)blockIdx.x * per, j1 = min(nsrc, j0 + per);
  if (j0 >= j1) return;  // the whole workgroup leaves together
  for (int b = threadIdx.x; b < nb; b += blockDim.x) cnt[b] = 0;
  __syncthreads();
  // every thread runs the same number of rounds (the round's first entry is < j1)
  for (int64_t j = j0 + threadIdx.x; j - threadIdx.x < j1; j += blockDim.x) {
    int v = -1;
    if (j < j1) v = key[gather ? src_idx[j] : j];
    (void)wave_lds_reserve(v >= 0 ? v : 0, v >= 0, cnt);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    int c = cnt[b];
    base[b] = c ? start[b] + atomicAdd(&cur_dst[b], c) : 0;
    cnt[b] = 0;
  }
  __syncthreads();
  for (int64_t j = j0 + threadIdx.x; j - threadIdx.x < j1; j += blockDim.x) {
    int v = -1, slot = 0;
    if (j < j1) {
      slot = src_idx ? src_idx[j] : (int)j;
      v = key[gather ? slot : j];
    }
    const int r = wave_lds_reserve(v >= 0 ? v : 0, v >= 0, cnt);
    if (v >= 0) dst_idx[base[v] + r] = slot;
  }
}

// Writes list k+1 from the places the step kernel reserved: entry j of list k
// (slot src_idx[j], next bucket nxt_lv[j] >= 0) goes to start[b] (the bucket's
// start, from the new counts cnt_dst) + seg[w][b] (its workgroup's share) +
// its rank in that share.  One pass, no atomics.  A thread's first kScatterUnroll
// entries are loaded before the bucket layout is computed, so their latency
// overlaps it.  len_src holds list k's length; workgroup 0 stores list k+1's
// into len_dst and clears the counts two lists ahead.  An empty list k leaves
// at once with list k+1's length 0 (the counts are then untouched and nothing
// reads them before the next transport clears them).  Needs 8 * nb + 4 bytes
// of dynamic LDS.
constexpr int kScatterUnroll = 4;
__global__ void __launch_bounds__(1024) k_bt_scatter(const int* __restrict__ src_idx, const int* __restrict__ len_src,
                                                      const int* __restrict__ nxt_lv,
                                                      const uint32_t* __restrict__ nxt_pos,
                                                      const int* __restrict__ seg, const int* __restrict__ cnt_dst,
                                                      int* __restrict__ dst_idx, int* __restrict__ len_dst,
                                                      int* __restrict__ cnt_clear, int nb) {
  extern __shared__ int lds[];
  int* base = lds;
  int* start = lds + nb;  // nb + 1 entries
  const int64_t nsrc = *len_src;
  if (nsrc == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *len_dst = 0;
    return;
  }
  const int64_t chunk = (int64_t)blockDim.x * kScatterUnroll;
  int64_t j0 = (int64_t)blockIdx.x * chunk + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * chunk;
  int b[kScatterUnroll], sl[kScatterUnroll];
  uint32_t u[kScatterUnroll];
  auto load = [&](int64_t j0_, int64_t bound) {
#pragma unroll
    for (int q = 0; q < kScatterUnroll; ++q) {
      const int64_t j = j0_ + (int64_t)q * blockDim.x;
      const bool in = j < bound;
      b[q] = in ? nxt_lv[j] : -1;
      u[q] = in ? nxt_pos[j] : 0u;
      sl[q] = in ? src_idx[j] : 0;
    }
  };
  load(j0, nsrc);
  stage_counts(cnt_dst, nb, base);
  block_layout(base, nb, start, nullptr);
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) *len_dst = start[nb];
    for (int v = threadIdx.x; v < nb; v += blockDim.x) cnt_clear[v] = 0;
  }
  for (; j0 < nsrc; j0 += stride) {
    int o[kScatterUnroll];
#pragma unroll
    for (int q = 0; q < kScatterUnroll; ++q)
      o[q] = b[q] >= 0 ? seg[(size_t)(u[q] >> kRankBits) * nb + b[q]] : 0;
#pragma unroll
    for (int q = 0; q < kScatterUnroll; ++q)
      if (b[q] >= 0) dst_idx[start[b[q]] + o[q] + (int)(u[q] & ((1u << kRankBits) - 1))] = sl[q];
    if (j0 + stride < nsrc) load(j0 + stride, nsrc);
  }
}

// ---------------------------------------------------------------- step
// Register budget per variant (WV waves per SIMD): the navigation step fits
// 128 VGPRs (4 waves per SIMD) without spilling; the physics-limited step
// (process lengths, generator state, distance still to go) spills 80 bytes per
// lane at 128 and runs faster with 168 VGPRs at 3 waves.  The launch shape
// chooses among the instances that are built.
// WK selects the instance that keeps the work counters (measurement only: a
// ballot and an LDS atomic per counted event); the production instance counts
// nothing.  The kernel leaves at once when its list is empty (len_cur), so the
// host may enqueue every step up to the bound without looking at the device.
template <bool F32, bool PHYS, bool B, bool WK, int WV>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WV))) k_bt_step(DevGeom G, int k, int max_steps, int cb, const int* __restrict__ idx,
                                                  const int* __restrict__ len_cur,
                                                  TRec* __restrict__ rec, const int* __restrict__ cnt_cur,
                                                  int* __restrict__ nxt_lv, uint32_t* __restrict__ nxt_pos,
                                                  int* __restrict__ cnt_next, TCtl C,
                                                  int32_t* __restrict__ out_pv, double* __restrict__ out_step,
                                                  int32_t* __restrict__ out_nsteps, uint32_t* __restrict__ out_flags,
                                                  const int* __restrict__ slot_id, double* __restrict__ ob_step,
                                                  int* __restrict__ ob_pv, int64_t cap, PhysArgs P,
                                                  int8_t* __restrict__ ob_proc, int8_t* __restrict__ out_proc) {
  // Dynamic LDS: next-bucket histogram [nb], this list's per-LV counts [nlv]
  // and per-LV layout start/tile [nlv+1] each.  The list is ordered by
  // bucket = (LV, coarse direction cell), so each LV's entries are contiguous
  // and ordered by direction cell; tiles cover whole LV ranges (a tile may
  // span two neighbouring cells) so that cells add no partial tiles.
  extern __shared__ int lds[];
  __shared__ unsigned long long wsum[WK ? kWorkN : 1];
  if (*len_cur == 0) return;  // nothing left to transport: the whole grid leaves
  const int nlv = G.n_lv, nb = nlv << cb;
  int* hist = lds;
  int* lvc = lds + nb;
  int* start = lvc + nlv;
  int* tilep = start + nlv + 1;
  if (WK)
    for (int i = threadIdx.x; i < kWorkN; i += blockDim.x) wsum[i] = 0;
  stage_counts(cnt_cur, nb, hist);  // hist is free until the layout is done
  for (int v = threadIdx.x; v < nlv; v += blockDim.x) {
    int c = 0;
    for (int q = 0; q < (1 << cb); ++q) c += hist[v << cb | q];
    lvc[v] = c;
  }
  __syncthreads();
  block_layout(lvc, nlv, start, tilep);
  for (int v = threadIdx.x; v < nb; v += blockDim.x) hist[v] = 0;
  __syncthreads();
  std::conditional_t<WK, LdsWork, NoWork> w{wsum};
  const int tiles = tilep[nlv];
  const int lane = __lane_id();
  const int wave = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave);
  const int nwaves = (int)(gridDim.x * (int64_t)blockDim.x / kWave);
  for (int t = wave; t < tiles; t += nwaves) {
    // LV of tile t: largest b with tile[b] <= t (wavefront-uniform search)
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
      const int sl = idx[e];
      // the track id is a dependent gather: read it only where it is needed
      const int id = (PHYS || !ob_step) ? slot_id[sl] : -1;
      TRec r = rec[sl];
      V3 p{r.x, r.y, r.z}, d{r.dx, r.dy, r.dz};
      uint32_t fl = zfc_fl(r.zfc);
      int nx, proc = -1;
      double st;
      bool exited = false;
      if (PHYS) {
        st = step_physics<F32, B>(G, b, r.pv, p, d, (uint32_t)id, k, P, r.safe, &nx, &proc, &fl, w,
                                  zfc_left(r.zfc), &exited);
      } else {
        st = step_culled<F32, B>(G, b, r.pv, p, d, &nx, &fl, w, zfc_left(r.zfc), &exited);
        p = advance(p, st, d);
      }
      // leaving pv into its mother: pv's placement index goes along (see the lane form)
      const int left = nx != r.pv ? (exited ? G.pv_k[r.pv] : -1) : zfc_left(r.zfc);
      if (ob_step) {  // staged by slot, moved to the rows at the end
        ob_step[(size_t)k * cap + sl] = st;
        ob_pv[(size_t)k * cap + sl] = nx;
        if (PHYS && ob_proc) ob_proc[(size_t)k * cap + sl] = (int8_t)proc;
      } else {
        out_step[(size_t)id * max_steps + k] = st;
        out_pv[(size_t)id * (max_steps + 1) + k + 1] = nx;
        if (PHYS && out_proc) out_proc[(size_t)id * max_steps + k] = (int8_t)proc;
      }
      int zr = st < kTol ? zfc_zr(r.zfc) + 1 : 0;
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
        const int tid = id >= 0 ? id : slot_id[sl];
        out_nsteps[tid] = k + 1;
        out_flags[tid] = fl;
      } else {
        // the whole 64-byte record in one go: full-line writes need no
        // read-modify-write of the line
        r.x = p.x;
        r.y = p.y;
        r.z = p.z;
        r.pv = nx;
        r.zfc = zfc_pack(zr, fl, left, zfc_cc(r.zfc));
        rec[sl] = r;
        nlv_out = G.pv_lv[nx] << cb | zfc_cc(r.zfc);
      }
      nxt_lv[e] = nlv_out;
    }
    if (act) w.add(kWorkSteps);
    // place in this workgroup's share of the next bucket
    const int rank = wave_lds_reserve(nlv_out >= 0 ? nlv_out : 0, nlv_out >= 0, hist);
    if (nlv_out >= 0) nxt_pos[e] = ((uint32_t)blockIdx.x << kRankBits) | (uint32_t)rank;
  }
  __syncthreads();
  // the workgroup's share of each next bucket starts where the count stood
  for (int v = threadIdx.x; v < nb; v += blockDim.x)
    if (hist[v]) C.seg[(size_t)blockIdx.x * nb + v] = atomicAdd(&cnt_next[v], hist[v]);
  if (WK)
    for (int i = threadIdx.x; i < kWorkN; i += blockDim.x)
      if (wsum[i]) atomicAdd(&C.work[i], wsum[i]);
}


}  // namespace gv
