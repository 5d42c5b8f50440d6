// Basket transport: tracks are regrouped by the logical volume they are in
// before every step (the paper's baskets: particles located in the same kind of
// volume are collected and processed together, Sec. II.A item 1 and Sec. III.C).
//
// Per step the state buffer holds one contiguous bucket per LV.  A wavefront
// takes a tile of 64 consecutive tracks of one bucket, so its LV -- the mother
// solid and the whole daughter table -- is wavefront-uniform: the daughter loop
// reads transforms and solid parameters with scalar loads into SGPRs and the
// lanes never diverge on the solid type.  After the step each wavefront adds
// its tracks to the per-LV counts of the next step; a one-workgroup kernel turns
// the counts into the next bucket layout, and a scatter kernel moves every live
// track into its new bucket (workgroup-aggregated atomics keep the writes of one
// workgroup to one bucket contiguous).
#pragma once
#include "gv_kernels.h"

namespace gv {

constexpr int kWave = 64;

struct TState {
  double *x, *y, *z, *dx, *dy, *dz;
  int *pv, *tid, *zr, *fl;
};

// bucket layout: start[b] (exclusive prefix of count, start[nlv] = total),
// count[b], tile[b] (exclusive prefix of ceil(count/64), tile[nlv] = tiles)
struct TLayout {
  int *start, *count, *tile;
};

struct TCtl {
  int* cnt_next;  // [nlv] tracks entering each LV at the next step
  int* cursor;    // [nlv] scatter cursors
  int* live;      // live tracks after the latest step (device copy)
};

__device__ __forceinline__ uint64_t lanemask_lt() { return __lanemask_lt(); }

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

__device__ __forceinline__ int ld_acq(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Next layout from the counts, then reset counts and cursors (one workgroup).
__device__ void finish_layout(int nlv, TCtl C, TLayout out) {
  __shared__ int part[256];
  __shared__ int tpart[256];
  int tid = threadIdx.x, nt = blockDim.x;
  int per = (nlv + nt - 1) / nt;
  int b0 = tid * per, b1 = min(nlv, b0 + per);
  int s = 0, ts = 0;
  for (int b = b0; b < b1; ++b) {
    int c = ld_acq(&C.cnt_next[b]);
    s += c;
    ts += (c + kWave - 1) / kWave;
  }
  part[tid] = s;
  tpart[tid] = ts;
  __syncthreads();
  if (tid == 0) {
    int a = 0, ta = 0;
    for (int k = 0; k < nt; ++k) {
      int v = part[k], tv = tpart[k];
      part[k] = a;
      tpart[k] = ta;
      a += v;
      ta += tv;
    }
    out.start[nlv] = a;
    out.tile[nlv] = ta;
    out.count[nlv] = 0;
    *C.live = a;
  }
  __syncthreads();
  s = part[tid];
  ts = tpart[tid];
  for (int b = b0; b < b1; ++b) {
    int c = ld_acq(&C.cnt_next[b]);
    out.start[b] = s;
    out.count[b] = c;
    out.tile[b] = ts;
    s += c;
    ts += (c + kWave - 1) / kWave;
    C.cnt_next[b] = 0;
    C.cursor[b] = 0;
  }
}

// ---------------------------------------------------------------- init
// Start volume of every track (given or located), entry 0 of its sequence, and
// the counts of the first layout.  Tracks that start outside the world finish
// here with zero steps.
__global__ void k_bt_init(DevGeom G, int64_t n, const double* __restrict__ x, const double* __restrict__ y,
                          const double* __restrict__ z, const int32_t* __restrict__ start_pv, int max_steps,
                          int32_t* __restrict__ out_pv, int32_t* __restrict__ out_nsteps,
                          uint32_t* __restrict__ out_flags, int* __restrict__ newlv, int* __restrict__ pv_tmp, TCtl C) {
  int64_t stride = gstride();
  int64_t nround = ((n + stride - 1) / stride) * stride;
  for (int64_t i = gtid(); i < nround; i += stride) {
    bool act = i < n;
    int v = -1;
    uint32_t fl = 0;
    if (act) {
      v = start_pv ? start_pv[i] : locate(G, ld3(x, y, z, i));
      if (v < -1 || v >= G.n_pv) {
        v = -1;
        fl = kFlagLocateFail;
      }
      out_pv[(size_t)i * (max_steps + 1)] = v;
      pv_tmp[i] = v;
      int lv = v >= 0 ? G.pv_lv[v] : -1;
      newlv[i] = lv;
      if (v < 0) {
        out_nsteps[i] = 0;
        out_flags[i] = fl;
      }
    }
    int lv = act && v >= 0 ? G.pv_lv[v] : 0;
    wave_count(lv, act && v >= 0, C.cnt_next);
  }
}

// Moves every live track of `src` (slots [0, nsrc)) into its bucket of `dst`.
// Each workgroup handles 256 consecutive slots at a time: LDS atomics rank the
// tracks per destination LV, then one global atomic per (workgroup, LV)
// reserves a contiguous range of the bucket.  A NULL src.tid means identity
// ids; NULL zr / fl mean zero.  Needs 8 * nlv bytes of dynamic LDS.
__global__ void __launch_bounds__(256) k_bt_scatter(TState src, const int* __restrict__ nsrc_ptr, int64_t nsrc_fixed,
                                                     const int* __restrict__ newlv, TState dst, TLayout Lnext, TCtl C,
                                                     int nlv) {
  extern __shared__ int lds[];
  int* cnt = lds;
  int* base = lds + nlv;
  const int64_t nsrc = nsrc_ptr ? *nsrc_ptr : nsrc_fixed;
  for (int64_t c0 = (int64_t)blockIdx.x * blockDim.x; c0 < nsrc; c0 += (int64_t)gridDim.x * blockDim.x) {
    for (int b = threadIdx.x; b < nlv; b += blockDim.x) cnt[b] = 0;
    __syncthreads();
    const int64_t i = c0 + threadIdx.x;
    const int v = i < nsrc ? newlv[i] : -1;
    int rank = 0;
    if (v >= 0) rank = atomicAdd(&cnt[v], 1);
    __syncthreads();
    for (int b = threadIdx.x; b < nlv; b += blockDim.x) {
      int c = cnt[b];
      base[b] = c ? Lnext.start[b] + atomicAdd(&C.cursor[b], c) : 0;
    }
    __syncthreads();
    if (v >= 0) {
      const int slot = base[v] + rank;
      dst.x[slot] = src.x[i];
      dst.y[slot] = src.y[i];
      dst.z[slot] = src.z[i];
      dst.dx[slot] = src.dx[i];
      dst.dy[slot] = src.dy[i];
      dst.dz[slot] = src.dz[i];
      dst.pv[slot] = src.pv[i];
      dst.tid[slot] = src.tid ? src.tid[i] : (int)i;
      dst.zr[slot] = src.zr ? src.zr[i] : 0;
      dst.fl[slot] = src.fl ? src.fl[i] : 0;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- step
// Daughter loop of one ComputeStep with the LV wavefront-uniform: transforms
// and solid parameters come from scalar loads.  An LV whose daughters share one
// solid type runs that solid's code only.
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

__device__ __forceinline__ double step_uniform_lv(const DevGeom& G, int lv, int pv, V3 p, V3 d, int* next,
                                                  uint32_t* flags) {
  CQ X = G.pv_gxf + 12 * (size_t)pv;
  V3 pl = to_child_p(X, p), dl = to_child_d(X, d);
  double dout = solid_dist_out(G.lv_type[lv], G.par + G.lv_par[lv], pl, dl);
  uint32_t fl = *flags;
  if (dout < 0.0) {
    dout = 0.0;
    fl |= kFlagLocateFail;
  }
  double best = GV_INF;
  int bestk = -1;
  const int off = G.lv_dau_off[lv], cnt = G.lv_dau_cnt[lv], dtype = G.lv_dau_type[lv];
  bool neg = false;
  if (dtype == kBox) {
    daughters_of_type<Box>(G, off, cnt, pl, dl, best, bestk, neg);
  } else if (dtype == kTubs) {
    daughters_of_type<Tubs>(G, off, cnt, pl, dl, best, bestk, neg);
  } else {
    for (int k = 0; k < cnt; ++k) {
      CQ Y = G.dau_xf + 12 * (size_t)(off + k);
      const int clv = G.dau_lv[off + k];
      V3 pc = to_child_p(Y, pl), dc = to_child_d(Y, dl);
      double t = solid_dist_in(G.lv_type[clv], G.par + G.lv_par[clv], pc, dc);
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
    return best;
  }
  *next = G.pv_parent[pv];
  return dout;
}

__global__ void __launch_bounds__(256) k_bt_step(DevGeom G, int k, int max_steps, TState S, TLayout L,
                                                  int* __restrict__ newlv, TCtl C,
                                                  int32_t* __restrict__ out_pv, double* __restrict__ out_step,
                                                  int32_t* __restrict__ out_nsteps, uint32_t* __restrict__ out_flags) {
  const int nlv = G.n_lv;
  const int tiles = L.tile[nlv];
  const int lane = __lane_id();
  const int wave = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave);
  const int nwaves = (int)(gridDim.x * (int64_t)blockDim.x / kWave);
  for (int t = wave; t < tiles; t += nwaves) {
    // bucket of tile t: largest b with tile[b] <= t (wavefront-uniform search)
    int lo = 0, hi = nlv - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (L.tile[mid] <= t) lo = mid;
      else hi = mid - 1;
    }
    const int b = __builtin_amdgcn_readfirstlane(lo);
    const int j = t - L.tile[b];
    const int within = j * kWave + lane;
    const bool act = within < L.count[b];
    const int i = L.start[b] + within;
    int nlv_out = -1;
    if (act) {
      V3 p = ld3(S.x, S.y, S.z, i), d = ld3(S.dx, S.dy, S.dz, i);
      int pv = S.pv[i];
      uint32_t fl = (uint32_t)S.fl[i];
      int nx;
      double st = step_uniform_lv(G, b, pv, p, d, &nx, &fl);
      p = advance(p, st, d);
      int id = S.tid[i];
      out_step[(size_t)id * max_steps + k] = st;
      out_pv[(size_t)id * (max_steps + 1) + k + 1] = nx;
      int zr = st < kTol ? S.zr[i] + 1 : 0;
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
        S.x[i] = p.x;
        S.y[i] = p.y;
        S.z[i] = p.z;
        S.pv[i] = nx;
        S.zr[i] = zr;
        S.fl[i] = (int)fl;
        nlv_out = G.pv_lv[nx];
      }
      newlv[i] = nlv_out;
    }
    wave_count(nlv_out >= 0 ? nlv_out : 0, nlv_out >= 0, C.cnt_next);
  }
}

// Next bucket layout from the counts (one workgroup).
__global__ void __launch_bounds__(256) k_bt_scan(int nlv, TCtl C, TLayout Lnext) { finish_layout(nlv, C, Lnext); }

}  // namespace gv
