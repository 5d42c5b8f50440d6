// Serving engine: baskets of navigation queries arriving over time are
// admitted under a slot count and an HBM budget, staged in pinned host memory,
// and answered in rounds -- every basket waiting when a stream falls idle goes
// into one round, whose inputs reach HBM with one copy per contiguous run, are
// answered by ONE fused kernel over all of the round's queries, and whose
// outputs come back the same way.  The paper's scheduler collects tracks into
// baskets and hands full baskets to the vectorised code (Sec. II.A, item 1);
// here the baskets come from clients and a launch serves many of them.
//
// Included once, at the end of gv_abi.hip (uses its error and launch helpers).
#pragma once
#include <chrono>
#include <deque>
#include <utility>

#include "gv_arena.h"

namespace gv {

enum { kQStep = 0, kQSafety = 1, kQInside = 2 };

// One basket of a round; the fused kernel reads the round's table.
struct SDesc {
  int32_t kind, prec;
  int64_t n;
  int64_t tile0;    // first 64-track tile of the basket within the round
  int64_t in_off;   // byte offset of its inputs in the input arena
  int64_t out_off;  // byte offset of its outputs in the output arena
  int64_t pad;
};
static_assert(sizeof(SDesc) == 48, "SDesc layout");

constexpr int kServeMaxSlots = 1024;

// Bytes of one basket in host layout (gvgeom.h, serving section).
__host__ __device__ inline int64_t serve_in_bytes(int kind, int64_t n) { return (kind == kQStep ? 60 : 28) * n; }
__host__ __device__ inline int64_t serve_out_bytes(int kind, int64_t n) {
  return (kind == kQStep ? 16 : kind == kQSafety ? 8 : 1) * n;
}

// Fused mixed-query kernel: one wavefront answers one tile of 64 tracks of one
// basket, so the query kind and precision are wavefront-uniform; a basket's
// tracks may sit in different volumes (per-lane navigation state).
template <bool B>
__global__ void __launch_bounds__(256) k_serve(DevGeom G, const SDesc* __restrict__ desc, int nb, int64_t ntiles,
                                               const char* __restrict__ din, char* __restrict__ dout) {
  __shared__ int64_t t0[kServeMaxSlots + 1];
  for (int b = threadIdx.x; b < nb; b += blockDim.x) t0[b] = desc[b].tile0;
  if (threadIdx.x == 0) t0[nb] = ntiles;
  __syncthreads();
  const int lane = __lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
  const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / 64;
  NoWork w;
  for (int64_t t = wave; t < ntiles; t += nwaves) {
    int lo = 0, hi = nb - 1;  // largest b with t0[b] <= t
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (t0[mid] <= t) lo = mid;
      else hi = mid - 1;
    }
    const int b = __builtin_amdgcn_readfirstlane(lo);
    const int kind = desc[b].kind, prec = desc[b].prec;
    const int64_t n = desc[b].n;
    const int64_t i = (t - t0[b]) * 64 + lane;
    if (i >= n) continue;
    const double* X = (const double*)(din + desc[b].in_off);
    char* O = dout + desc[b].out_off;
    const V3 p{X[i], X[n + i], X[2 * n + i]};
    if (kind == kQStep) {
      const V3 d{X[3 * n + i], X[4 * n + i], X[5 * n + i]};
      const double ps = X[6 * n + i];
      const int v = ((const int32_t*)(X + 7 * n))[i];
      uint32_t fl = 0;
      int nx = -1;
      double st = 0.0;
      if (v >= 0 && v < G.n_pv) {
        st = prec == 0 ? step_culled_limited<false, B>(G, v, p, d, ps, &nx, &fl, w)
                       : step_culled_limited<true, B>(G, v, p, d, ps, &nx, &fl, w);
      } else {
        fl = kFlagLocateFail;
      }
      double* os = (double*)O;
      int32_t* on = (int32_t*)(os + n);
      uint32_t* of = (uint32_t*)(on + n);
      os[i] = st;
      on[i] = nx;
      of[i] = fl;
    } else {
      const int v = ((const int32_t*)(X + 3 * n))[i];
      const bool ok = v >= 0 && v < G.n_pv;
      if (kind == kQSafety) {
        ((double*)O)[i] = !ok ? 0.0 : prec == 0 ? nav_safety<B>(G, v, p) : nav_safety_screened<B>(G, v, p);
      } else {
        int8_t c = (int8_t)kOutside;
        if (ok) {
          const int lv = G.pv_lv[v];
          const V3 pl = to_child_p(G.pv_gxf + 12 * (size_t)v, p);
          c = (int8_t)code_of(solid_sgn<B>(G.lv_type[lv], G.par + G.lv_par[lv], pl));
        }
        ((int8_t*)O)[i] = c;
      }
    }
  }
}

}  // namespace gv

// ----------------------------------------------------------- host engine
struct gv_server {
  gv_geom* g = nullptr;
  int device = 0, slots = 0, nstreams = 0;
  gv::RingAlloc rin, rout;
  char* d_mem = nullptr;  // device: input arena | output arena | descriptor tables
  char *d_in = nullptr, *d_out = nullptr;
  gv::SDesc* d_desc = nullptr;  // [nstreams][slots]
  char* h_mem = nullptr;        // pinned host mirror of d_mem
  char *h_in = nullptr, *h_out = nullptr;
  gv::SDesc* h_desc = nullptr;
  std::vector<hipStream_t> st;
  std::vector<hipEvent_t> ev;
  // rounds launched as a graph per stream (GV_SERVE_GRAPH): fixed topology
  // (two input-copy runs and the descriptor copy, the fused kernel, two
  // output-copy runs) whose node parameters are set for every round; copies a
  // round does not need move 8 bytes between per-stream spare words
  bool graphs = false;
  struct RoundGraph {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    hipGraphNode_t in[2] = {nullptr, nullptr}, desc = nullptr, kern = nullptr, out[2] = {nullptr, nullptr};
  };
  std::vector<RoundGraph> rg;
  char *d_spare = nullptr, *h_spare = nullptr;  // [nstreams][64] bytes
  hipEvent_t ev_ref = nullptr;
  double t_ref = 0.0;
  struct Bk {
    uint64_t ticket;
    int kind, prec;
    int64_t n;
    size_t in_off, in_len, out_off, out_len;
    void* user_out;
  };
  std::deque<Bk> waiting;
  struct Round {
    std::vector<Bk> bs;
    bool busy = false;
    uint64_t seq = 0;
  };
  std::vector<Round> rd;
  std::deque<std::pair<uint64_t, double>> done;
  int admitted = 0;  // waiting or in a round
  uint64_t next_ticket = 1, seq = 0;
  int64_t n_rounds = 0, n_baskets = 0, n_tracks = 0, max_round = 0;
};

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void server_release(gv_server* s) {
  if (!s) return;
  for (auto& r : s->rg) {
    if (r.x) (void)hipGraphExecDestroy(r.x);
    if (r.g) (void)hipGraphDestroy(r.g);
  }
  for (auto& e : s->ev)
    if (e) (void)hipEventDestroy(e);
  if (s->ev_ref) (void)hipEventDestroy(s->ev_ref);
  for (auto& q : s->st)
    if (q) (void)hipStreamDestroy(q);
  if (s->d_mem) (void)hipFree(s->d_mem);
  if (s->h_mem) (void)hipHostFree(s->h_mem);
  delete s;
}

// Contiguous runs of a round's blocks (ascending, allocation order) as
// (offset, bytes) pairs.
template <class Get>
std::vector<std::pair<size_t, size_t>> runs(const std::vector<gv_server::Bk>& bs, Get get) {
  std::vector<std::pair<size_t, size_t>> r;
  for (const auto& b : bs) {
    size_t off = get(b).first, len = gv::RingAlloc::round_up(get(b).second);
    if (!r.empty() && r.back().first + r.back().second == off) r.back().second += len;
    else r.emplace_back(off, len);
  }
  return r;
}

int server_launch(gv_server* s, int k) {
  const char* fn = "gv_server";
  gv_server::Round& R = s->rd[k];
  R.bs.assign(s->waiting.begin(), s->waiting.end());
  s->waiting.clear();
  hipStream_t q = s->st[k];
  gv::SDesc* hd = s->h_desc + (size_t)k * s->slots;
  int64_t tiles = 0;
  for (size_t j = 0; j < R.bs.size(); ++j) {
    const auto& b = R.bs[j];
    hd[j] = gv::SDesc{b.kind, b.prec, b.n, tiles, (int64_t)b.in_off, (int64_t)b.out_off, 0};
    tiles += (b.n + 63) / 64;
  }
  hipError_t e = hipSuccess;
  const auto rin = runs(R.bs, [](const gv_server::Bk& b) { return std::make_pair(b.in_off, b.in_len); });
  const auto rout = runs(R.bs, [](const gv_server::Bk& b) { return std::make_pair(b.out_off, b.out_len); });
  gv::SDesc* dd = s->d_desc + (size_t)k * s->slots;
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((tiles + 3) / 4, 2048));
  auto kernel = s->g->has_bool ? gv::k_serve<true> : gv::k_serve<false>;
  if (s->graphs && rin.size() <= 2 && rout.size() <= 2) {
    // one graph launch: the round's copies and kernel as the node parameters
    gv_server::RoundGraph& G = s->rg[k];
    char* ds = s->d_spare + 64 * (size_t)k;
    char* hs = s->h_spare + 64 * (size_t)k;
    for (int i = 0; i < 2 && e == hipSuccess; ++i)
      e = i < (int)rin.size()
              ? hipGraphExecMemcpyNodeSetParams1D(G.x, G.in[i], s->d_in + rin[i].first, s->h_in + rin[i].first,
                                                  rin[i].second, hipMemcpyHostToDevice)
              : hipGraphExecMemcpyNodeSetParams1D(G.x, G.in[i], ds + 8 * i, hs + 8 * i, 8, hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipGraphExecMemcpyNodeSetParams1D(G.x, G.desc, dd, hd, R.bs.size() * sizeof(gv::SDesc),
                                            hipMemcpyHostToDevice);
    gv::DevGeom dg = s->g->dg;
    const gv::SDesc* cdd = dd;
    int nb = (int)R.bs.size();
    const char* din = s->d_in;
    char* dout = s->d_out;
    void* args[] = {&dg, &cdd, &nb, &tiles, &din, &dout};
    hipKernelNodeParams kp{};
    kp.func = reinterpret_cast<void*>(kernel);
    kp.gridDim = dim3(grid);
    kp.blockDim = dim3(kBlock);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    if (e == hipSuccess) e = hipGraphExecKernelNodeSetParams(G.x, G.kern, &kp);
    for (int i = 0; i < 2 && e == hipSuccess; ++i)
      e = i < (int)rout.size()
              ? hipGraphExecMemcpyNodeSetParams1D(G.x, G.out[i], s->h_out + rout[i].first, s->d_out + rout[i].first,
                                                  rout[i].second, hipMemcpyDeviceToHost)
              : hipGraphExecMemcpyNodeSetParams1D(G.x, G.out[i], hs + 32 + 8 * i, ds + 32 + 8 * i, 8,
                                                  hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipGraphLaunch(G.x, q);
    if (e == hipSuccess) e = hipEventRecord(s->ev[k], q);
    if (e != hipSuccess) return hip_fail(e, "gv_server: round graph");
  } else {
    for (auto& r : rin)
      if (e == hipSuccess) e = hipMemcpyAsync(s->d_in + r.first, s->h_in + r.first, r.second, hipMemcpyHostToDevice, q);
    if (e == hipSuccess) e = hipMemcpyAsync(dd, hd, R.bs.size() * sizeof(gv::SDesc), hipMemcpyHostToDevice, q);
    if (e != hipSuccess) return hip_fail(e, "gv_server: input copy");
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), 0, q, s->g->dg, (const gv::SDesc*)dd, (int)R.bs.size(), tiles,
                       (const char*)s->d_in, s->d_out);
    GV_TRY(launched(fn));
    for (auto& r : rout)
      if (e == hipSuccess) e = hipMemcpyAsync(s->h_out + r.first, s->d_out + r.first, r.second, hipMemcpyDeviceToHost, q);
    if (e == hipSuccess) e = hipEventRecord(s->ev[k], q);
    if (e != hipSuccess) return hip_fail(e, "gv_server: output copy");
  }
  R.busy = true;
  R.seq = ++s->seq;
  s->n_rounds++;
  s->n_baskets += (int64_t)R.bs.size();
  for (const auto& b : R.bs) s->n_tracks += b.n;
  s->max_round = std::max<int64_t>(s->max_round, (int64_t)R.bs.size());
  return GV_OK;
}

int server_try_launch(gv_server* s) {
  while (!s->waiting.empty()) {
    int k = -1;
    for (int i = 0; i < s->nstreams; ++i)
      if (!s->rd[i].busy) {
        k = i;
        break;
      }
    if (k < 0) return GV_OK;
    GV_TRY(server_launch(s, k));
  }
  return GV_OK;
}

// Completes round k (its event has fired): outputs to the callers, space and
// slots back, tickets to the done queue.
int server_complete(gv_server* s, int k) {
  gv_server::Round& R = s->rd[k];
  float ms = 0.0f;
  hipError_t e = hipEventElapsedTime(&ms, s->ev_ref, s->ev[k]);
  if (e != hipSuccess) return hip_fail(e, "gv_server: hipEventElapsedTime");
  const double t = s->t_ref + 1e-3 * (double)ms;
  for (const auto& b : R.bs) {
    std::memcpy(b.user_out, s->h_out + b.out_off, b.out_len);
    s->rin.release(b.in_off);
    s->rout.release(b.out_off);
    s->admitted--;
    s->done.emplace_back(b.ticket, t);
  }
  R.bs.clear();
  R.busy = false;
  return GV_OK;
}

// Completes every round whose event has fired, oldest first; with `wait`,
// waits for the oldest busy round first.
int server_progress(gv_server* s, bool wait) {
  for (;;) {
    int k = -1;
    for (int i = 0; i < s->nstreams; ++i)
      if (s->rd[i].busy && (k < 0 || s->rd[i].seq < s->rd[k].seq)) k = i;
    if (k < 0) break;
    hipError_t e = wait ? hipEventSynchronize(s->ev[k]) : hipEventQuery(s->ev[k]);
    if (e == hipErrorNotReady) break;
    if (e != hipSuccess) return hip_fail(e, "gv_server: round completion");
    GV_TRY(server_complete(s, k));
    wait = false;
  }
  return server_try_launch(s);
}

}  // namespace

extern "C" double gv_now(void) { return now_s(); }

// The round graph of stream k: nodes with placeholder parameters (8-byte
// copies between the stream's spare words, a one-workgroup launch with no
// baskets), instantiated once; every round sets them.
int server_round_graph(gv_server* s, int k) {
  gv_server::RoundGraph& G = s->rg[k];
  char* ds = s->d_spare + 64 * (size_t)k;
  char* hs = s->h_spare + 64 * (size_t)k;
  hipError_t e = hipGraphCreate(&G.g, 0);
  for (int i = 0; i < 2 && e == hipSuccess; ++i)
    e = hipGraphAddMemcpyNode1D(&G.in[i], G.g, nullptr, 0, ds + 8 * i, hs + 8 * i, 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipGraphAddMemcpyNode1D(&G.desc, G.g, nullptr, 0, ds + 16, hs + 16, 8, hipMemcpyHostToDevice);
  gv::DevGeom dg = s->g->dg;
  const gv::SDesc* cdd = s->d_desc + (size_t)k * s->slots;
  int nb = 0;
  int64_t tiles = 0;
  const char* din = s->d_in;
  char* dout = s->d_out;
  void* args[] = {&dg, &cdd, &nb, &tiles, &din, &dout};
  hipKernelNodeParams kp{};
  kp.func = reinterpret_cast<void*>(s->g->has_bool ? gv::k_serve<true> : gv::k_serve<false>);
  kp.gridDim = dim3(1);
  kp.blockDim = dim3(kBlock);
  kp.sharedMemBytes = 0;
  kp.kernelParams = args;
  kp.extra = nullptr;
  hipGraphNode_t deps[3] = {G.in[0], G.in[1], G.desc};
  if (e == hipSuccess) e = hipGraphAddKernelNode(&G.kern, G.g, deps, 3, &kp);
  for (int i = 0; i < 2 && e == hipSuccess; ++i)
    e = hipGraphAddMemcpyNode1D(&G.out[i], G.g, &G.kern, 1, hs + 32 + 8 * i, ds + 32 + 8 * i, 8,
                                hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipGraphInstantiate(&G.x, G.g, nullptr, nullptr, 0);
  if (e != hipSuccess) return hip_fail(e, "gv_server_create: round graph");
  return GV_OK;
}

extern "C" int gv_server_create(gv_geom* g, int32_t slots, int64_t hbm_budget, int32_t nstreams, int32_t options,
                                gv_server** out) {
  const char* fn = "gv_server_create";
  if (!out) return fail(GV_EINVAL, "%s: out is NULL", fn);
  *out = nullptr;
  if (!g) return fail(GV_EINVAL, "%s: geometry handle is NULL", fn);
  if (options & ~GV_SERVE_GRAPH) return fail(GV_EINVAL, "%s: options %d", fn, options);
  if (slots < 1 || slots > kServeMaxSlots) return fail(GV_EINVAL, "%s: slots %d not in [1, %d]", fn, slots, kServeMaxSlots);
  if (hbm_budget < (64 << 10) || hbm_budget > ((int64_t)1 << 40))
    return fail(GV_EINVAL, "%s: hbm_budget %lld not in [64 KiB, 1 TiB]", fn, (long long)hbm_budget);
  if (nstreams < 1 || nstreams > 8) return fail(GV_EINVAL, "%s: nstreams %d not in [1, 8]", fn, nstreams);
  DeviceGuard dgd(g->device);
  gv_server* s = new (std::nothrow) gv_server();
  if (!s) return fail(GV_ENOMEM, "%s: host allocation", fn);
  s->g = g;
  s->device = g->device;
  s->slots = slots;
  s->nstreams = nstreams;
  const size_t a = gv::RingAlloc::kAlign;
  const size_t cin = (size_t)hbm_budget / 5 * 4 / a * a, cout = ((size_t)hbm_budget - cin) / a * a;
  s->rin = gv::RingAlloc(cin);
  s->rout = gv::RingAlloc(cout);
  const size_t desc_bytes = (size_t)nstreams * slots * sizeof(gv::SDesc);
  const size_t total = cin + cout + gv::RingAlloc::round_up(desc_bytes) + gv::RingAlloc::round_up(64 * (size_t)nstreams);
  hipError_t e = hipMalloc(&s->d_mem, total);
  if (e != hipSuccess) {
    server_release(s);
    return fail(GV_ENOMEM, "%s: hipMalloc(%zu): %s", fn, total, hipGetErrorString(e));
  }
  e = hipHostMalloc((void**)&s->h_mem, total, hipHostMallocDefault);
  if (e != hipSuccess) {
    server_release(s);
    return fail(GV_ENOMEM, "%s: hipHostMalloc(%zu): %s", fn, total, hipGetErrorString(e));
  }
  s->d_in = s->d_mem;
  s->d_out = s->d_mem + cin;
  s->d_desc = (gv::SDesc*)(s->d_mem + cin + cout);
  s->h_in = s->h_mem;
  s->h_out = s->h_mem + cin;
  s->h_desc = (gv::SDesc*)(s->h_mem + cin + cout);
  s->d_spare = s->d_mem + cin + cout + gv::RingAlloc::round_up(desc_bytes);
  s->h_spare = s->h_mem + cin + cout + gv::RingAlloc::round_up(desc_bytes);
  s->st.assign(nstreams, nullptr);
  s->ev.assign(nstreams, nullptr);
  s->rd.resize(nstreams);
  for (int i = 0; i < nstreams && e == hipSuccess; ++i) {
    e = hipStreamCreateWithFlags(&s->st[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&s->ev[i]);
  }
  if (e == hipSuccess) e = hipEventCreate(&s->ev_ref);
  if (e != hipSuccess) {
    server_release(s);
    return hip_fail(e, "gv_server_create: streams and events");
  }
  if (options & GV_SERVE_GRAPH) {
    s->graphs = true;
    s->rg.resize(nstreams);
    for (int i = 0; i < nstreams; ++i) {
      const int rc = server_round_graph(s, i);
      if (rc != GV_OK) {
        server_release(s);
        return rc;
      }
    }
  }
  // the device clock's reference: an event and the host time right after it
  // completes (nothing else may come between the two)
  e = hipEventRecord(s->ev_ref, s->st[0]);
  if (e == hipSuccess) e = hipEventSynchronize(s->ev_ref);
  if (e != hipSuccess) {
    server_release(s);
    return hip_fail(e, "gv_server_create: reference event");
  }
  s->t_ref = now_s();
  *out = s;
  t_err.clear();
  return GV_OK;
}

extern "C" int gv_server_submit(gv_server* s, int32_t kind, int32_t precision, int64_t n, const void* in, void* out,
                                uint64_t* ticket) {
  const char* fn = "gv_server_submit";
  if (!s) return fail(GV_EINVAL, "%s: server handle is NULL", fn);
  if (kind < GV_Q_STEP || kind > GV_Q_INSIDE) return fail(GV_EINVAL, "%s: kind %d", fn, kind);
  GV_TRY(check_nav_precision(fn, precision));
  if (n < 1) return fail(GV_EINVAL, "%s: n = %lld < 1", fn, (long long)n);
  if (!in || !out || !ticket) return fail(GV_EINVAL, "%s: NULL argument", fn);
  const size_t li = (size_t)gv::serve_in_bytes(kind, n), lo = (size_t)gv::serve_out_bytes(kind, n);
  if (gv::RingAlloc::round_up(li) > s->rin.capacity() || gv::RingAlloc::round_up(lo) > s->rout.capacity())
    return fail(GV_EINVAL, "%s: a basket of %lld tracks never fits the HBM budget", fn, (long long)n);
  DeviceGuard dgd(s->device);
  // no completion here: slots and arena space come back only in poll/drain
  if (s->admitted >= s->slots) return fail(GV_EAGAIN, "%s: all %d slots busy", fn, s->slots);
  const size_t oi = s->rin.alloc(li);
  if (oi == gv::RingAlloc::npos) return fail(GV_EAGAIN, "%s: input arena full", fn);
  const size_t oo = s->rout.alloc(lo);
  if (oo == gv::RingAlloc::npos) {
    s->rin.release(oi);
    return fail(GV_EAGAIN, "%s: output arena full", fn);
  }
  std::memcpy(s->h_in + oi, in, li);
  const uint64_t tk = s->next_ticket++;
  s->waiting.push_back(gv_server::Bk{tk, kind, precision, n, oi, li, oo, lo, out});
  s->admitted++;
  *ticket = tk;
  GV_TRY(server_try_launch(s));
  t_err.clear();
  return GV_OK;
}

extern "C" int gv_server_poll(gv_server* s, int32_t max, uint64_t* tickets, double* t_done, int32_t* count) {
  const char* fn = "gv_server_poll";
  if (!s || !count) return fail(GV_EINVAL, "%s: NULL argument", fn);
  if (max < 0 || (max > 0 && !tickets)) return fail(GV_EINVAL, "%s: bad max/tickets", fn);
  DeviceGuard dgd(s->device);
  *count = 0;
  GV_TRY(server_progress(s, false));
  int c = 0;
  while (c < max && !s->done.empty()) {
    tickets[c] = s->done.front().first;
    if (t_done) t_done[c] = s->done.front().second;
    s->done.pop_front();
    ++c;
  }
  *count = c;
  return GV_OK;
}

extern "C" int gv_server_drain(gv_server* s) {
  if (!s) return fail(GV_EINVAL, "gv_server_drain: server handle is NULL");
  DeviceGuard dgd(s->device);
  while (s->admitted > 0) GV_TRY(server_progress(s, true));
  return GV_OK;
}

extern "C" int gv_server_stats(const gv_server* s, int64_t* out) {
  if (!s || !out) return fail(GV_EINVAL, "gv_server_stats: NULL argument");
  out[0] = s->admitted;
  out[1] = (int64_t)s->waiting.size();
  out[2] = s->n_rounds;
  out[3] = s->n_baskets;
  out[4] = s->n_tracks;
  out[5] = s->max_round;
  out[6] = (int64_t)s->rin.in_use();
  out[7] = (int64_t)s->rout.in_use();
  return GV_OK;
}

extern "C" int gv_server_destroy(gv_server* s) {
  if (!s) return GV_OK;
  DeviceGuard dgd(s->device);
  int rc = gv_server_drain(s);
  for (auto& q : s->st)
    if (q) (void)hipStreamSynchronize(q);
  server_release(s);
  return rc;
}
