// Host side of the C-ABI declared in include/gvgeom.h: argument validation,
// geometry-blob parsing and upload, kernel selection and launch on the
// caller's stream.  No exception or abort crosses the boundary.
#include <hip/hip_runtime.h>

#include <immintrin.h>
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/gvgeom.h"
#include "gv_baskets.h"
#include "gv_lane.h"
#include "gv_probe.h"

using namespace gv;

// ------------------------------------------------------------------ errors
static thread_local std::string t_err;

static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  t_err = buf;
  return code;
}

static int hip_fail(hipError_t e, const char* what) {
  return fail(GV_EHIP, "%s: %s", what, hipGetErrorString(e));
}

extern "C" const char* gv_last_error(void) { return t_err.c_str(); }

// ------------------------------------------------- allocation-free scratch
// Scratch of nav_transport_noalloc: the lane form's keys, order and counters
// for up to kNoAllocMaxTracks tracks (16.06 MiB), one copy per device, held
// until the process ends.  In host code `scratch` names a host-side stand-in:
// kernels get the device address that hipGetSymbolAddress returned for each
// device (noalloc_scratch), never the symbol itself.
constexpr int64_t kNoAllocMaxTracks = (int64_t)1 << 21;
constexpr size_t kScratchBytes = 2 * 4 * (size_t)kNoAllocMaxTracks + 4 * (size_t)kSortMaxCells + 256;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex scratch_mu;
static void* scratch_addr[kMaxDevices] = {};

// Looks up (once per device, with that device current) the device address of
// this device's copy of the scratch array.
static int init_noalloc_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return fail(GV_EHIP, "geom_load: device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (scratch_addr[dev]) return GV_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) return hip_fail(e, "geom_load: hipGetSymbolAddress(scratch)");
  scratch_addr[dev] = p;
  return GV_OK;
}

static void* noalloc_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(scratch_mu);
  return scratch_addr[dev];
}


// --------------------------------------------------------------- geometry
struct gv_geom {
  int device = -1;
  DevGeom dg{};
  int n_lv = 0, n_pv = 0, n_place = 0, max_depth = 0, world_lv = 0;
  bool has_bool = false;  // some LV is a composite: navigation runs the kernels built with composite code
  std::vector<int> lv_type, lv_par;
  void* dmem = nullptr;
  // nav_transport workspace (grown on demand)
  void* ws = nullptr;
  size_t ws_bytes = 0;
  int64_t ws_tracks = 0;
  TRec* rec = nullptr;      // [cap] track records
  int* idx[2] = {nullptr, nullptr};  // bucketed slot lists
  TCtl ctl{};
  int* nxt_lv = nullptr;    // [cap] next bucket per list entry (start bucket per track at the start)
  uint32_t* nxt_pos = nullptr;  // [cap] place of each list entry in the next list (workgroup, rank)
  int* slot_id = nullptr;   // [cap] track id of each slot
  void* ob = nullptr;       // staged outputs: ob_step [ob_steps][cap] double, then ob_pv [ob_steps][cap] int
  double* ob_step = nullptr;
  int* ob_pv = nullptr;
  int8_t* ob_proc = nullptr;
  void* mat_mem = nullptr;  // device material tables (geom_set_materials)
  int64_t ob_cap = 0, ob_steps = 0;
  // measurement (gv_profile): HIP events around the step-kernel launches, and
  // the step-kernel instance that keeps the work counters
  bool prof = false;
  bool prof_work = false;
  // launch shapes (gv_set_tuning); zero / negative fields take the defaults
  gv_tuning tune{0, 0, -1, 0, 0, 0, 0, -1, 0, 0, 0, 0, 0};
  // lane-transport workspace (grown on demand): direction keys, the coherent
  // order, key counts and the work counter
  void* lws = nullptr;
  int64_t lws_cap = 0;
  LaneCtl lctl{};
  int n_cu = 0;  // compute units of the device
  std::pair<const void*, int> occ[16] = {};  // resident workgroups per CU of persistent kernels
  int n_occ = 0;
  unsigned long long* pcon_work = nullptr;  // [5] polycone work counters (inside dmem)
  int ws_nl = 0;  // buckets the workspace was sized for
  std::vector<hipEvent_t> prof_ev;  // pairs around step-kernel launches
  size_t prof_used = 0;
};

namespace {

constexpr int kMaxDepth = 32;
constexpr long kMaxPv = 1L << 24;
constexpr int kMaxNz = 64;

int32_t rd_i32(const unsigned char* b, size_t off) {
  int32_t v;
  std::memcpy(&v, b + off, 4);
  return v;
}
double rd_f64(const unsigned char* b, size_t off) {
  double v;
  std::memcpy(&v, b + off, 8);
  return v;
}

// Derived constants of each solid (reciprocal slopes, normalisations, the phi
// half-plane normals) -- see the parameter layouts in gv_solids.h.
int phi_mode(double dphi) { return dphi >= 2.0 * M_PI ? 0 : (dphi <= M_PI ? 1 : 2); }
void phi_vectors(double sphi, double dphi, double* ns, double* ne, double* us, double* ue) {
  double pe = sphi + dphi;
  ns[0] = std::sin(sphi);
  ns[1] = -std::cos(sphi);
  ne[0] = -std::sin(pe);
  ne[1] = std::cos(pe);
  us[0] = std::cos(sphi);
  us[1] = std::sin(sphi);
  ue[0] = std::cos(pe);
  ue[1] = std::sin(pe);
}

bool derive(int type, const double* q, int nq, std::vector<double>& out, std::string& why) {
  auto bad = [&](const char* m) {
    why = m;
    return false;
  };
  switch (type) {
    case kBox:
      if (nq != 3 || !(q[0] > 0 && q[1] > 0 && q[2] > 0)) return bad("box needs dx, dy, dz > 0");
      out.insert(out.end(), q, q + 3);
      return true;
    case kTubs: {
      if (nq != 5 || !(q[0] >= 0 && q[1] > q[0] && q[2] > 0 && q[4] > 0))
        return bad("tube segment needs 0 <= rmin < rmax, dz > 0, dphi > 0");
      double v[L::TB_N] = {};
      v[L::TB_RMIN] = q[0];
      v[L::TB_RMAX] = q[1];
      v[L::TB_DZ] = q[2];
      v[L::TB_PHI] = phi_mode(q[4]);
      phi_vectors(q[3], q[4], v + L::TB_NS, v + L::TB_NE, v + L::TB_US, v + L::TB_UE);
      v[L::TB_RMIN2] = q[0] * q[0];
      v[L::TB_RMAX2] = q[1] * q[1];
      out.insert(out.end(), v, v + L::TB_N);
      return true;
    }
    case kCons: {
      if (nq != 7) return bad("cone segment needs 7 parameters");
      double rmin1 = q[0], rmax1 = q[1], rmin2 = q[2], rmax2 = q[3], dz = q[4];
      if (!(rmin1 >= 0 && rmax1 >= rmin1 && rmin2 >= 0 && rmax2 >= rmin2 && rmax1 + rmax2 > 0 && dz > 0 && q[6] > 0))
        return bad("cone segment needs 0 <= rmin <= rmax at both ends, dz > 0, dphi > 0");
      double v[L::CN_N] = {};
      for (int i = 0; i < 5; ++i) v[i] = q[i];
      v[L::CN_PHI] = phi_mode(q[6]);
      phi_vectors(q[5], q[6], v + L::CN_NS, v + L::CN_NE, v + L::CN_US, v + L::CN_UE);
      v[L::CN_AO] = 0.5 * (rmax1 + rmax2);
      v[L::CN_BO] = (rmax2 - rmax1) / (2.0 * dz);
      v[L::CN_CO] = 1.0 / std::sqrt(1.0 + v[L::CN_BO] * v[L::CN_BO]);
      v[L::CN_AI] = 0.5 * (rmin1 + rmin2);
      v[L::CN_BI] = (rmin2 - rmin1) / (2.0 * dz);
      v[L::CN_CI] = 1.0 / std::sqrt(1.0 + v[L::CN_BI] * v[L::CN_BI]);
      v[L::CN_INNER] = (rmin1 > 0 || rmin2 > 0) ? 1.0 : 0.0;
      out.insert(out.end(), v, v + L::CN_N);
      return true;
    }
    case kSphere: {
      if (nq != 2 || !(q[0] >= 0 && q[1] > q[0])) return bad("sphere shell needs 0 <= rmin < rmax");
      double v[L::SP_N] = {q[0], q[1], q[0] * q[0], q[1] * q[1]};
      out.insert(out.end(), v, v + L::SP_N);
      return true;
    }
    case kTrd: {
      if (nq != 5 || !(q[0] > 0 && q[1] > 0 && q[2] > 0 && q[3] > 0 && q[4] > 0)) return bad("trd needs all > 0");
      double v[L::TD_N];
      for (int i = 0; i < 5; ++i) v[i] = q[i];
      double dz = q[4];
      v[L::TD_X0] = 0.5 * (q[0] + q[1]);
      v[L::TD_TX] = (q[1] - q[0]) / (2.0 * dz);
      v[L::TD_CX] = 1.0 / std::sqrt(1.0 + v[L::TD_TX] * v[L::TD_TX]);
      v[L::TD_Y0] = 0.5 * (q[2] + q[3]);
      v[L::TD_TY] = (q[3] - q[2]) / (2.0 * dz);
      v[L::TD_CY] = 1.0 / std::sqrt(1.0 + v[L::TD_TY] * v[L::TD_TY]);
      out.insert(out.end(), v, v + L::TD_N);
      return true;
    }
    case kPcon: {
      if (nq < 1) return bad("polycone needs nz");
      int nz = (int)q[0];
      if (nz < 2 || nz > kMaxNz || (double)nz != q[0] || nq != 1 + 3 * nz)
        return bad("polycone needs 2 <= nz <= 64 and 1 + 3 nz parameters");
      const double *z = q + 1, *rmin = q + 1 + nz, *rmax = q + 1 + 2 * nz;
      for (int j = 0; j < nz; ++j) {
        if (!(rmin[j] >= 0 && rmax[j] >= rmin[j])) return bad("polycone needs 0 <= rmin <= rmax");
        if (j > 0 && !(z[j] > z[j - 1])) return bad("polycone z planes must increase");
      }
      out.push_back(nz);
      out.insert(out.end(), z, z + nz);
      out.insert(out.end(), rmin, rmin + nz);
      out.insert(out.end(), rmax, rmax + nz);
      std::vector<double> bo(nz - 1), co(nz - 1), bi(nz - 1), ci(nz - 1), in(nz - 1);
      for (int j = 0; j + 1 < nz; ++j) {
        if (!(rmax[j] + rmax[j + 1] > 0)) return bad("polycone section with zero outer radius");
        double h = z[j + 1] - z[j];
        bo[j] = (rmax[j + 1] - rmax[j]) / h;
        co[j] = 1.0 / std::sqrt(1.0 + bo[j] * bo[j]);
        bi[j] = (rmin[j + 1] - rmin[j]) / h;
        ci[j] = 1.0 / std::sqrt(1.0 + bi[j] * bi[j]);
        in[j] = (rmin[j] > 0 || rmin[j + 1] > 0) ? 1.0 : 0.0;
      }
      for (auto* a : {&bo, &co, &bi, &ci, &in}) out.insert(out.end(), a->begin(), a->end());
      // safety segments of the meridian polygon: 1/|e|^2 of each outer and
      // inner side segment and of the two caps (0 for a degenerate segment)
      auto inv_len2 = [](double er, double ez) {
        const double ll = er * er + ez * ez;
        return ll > 0.0 ? 1.0 / ll : 0.0;
      };
      for (int j = 0; j + 1 < nz; ++j) out.push_back(inv_len2(rmax[j + 1] - rmax[j], z[j + 1] - z[j]));
      for (int j = 0; j + 1 < nz; ++j) out.push_back(inv_len2(rmin[j + 1] - rmin[j], z[j + 1] - z[j]));
      out.push_back(inv_len2(rmax[0] - rmin[0], 0.0));
      out.push_back(inv_len2(rmax[nz - 1] - rmin[nz - 1], 0.0));
      // bounding cylinder radius (the largest rmax) for the DistanceToIn reject
      out.push_back(*std::max_element(rmax, rmax + nz));
      return true;
    }
    case kBool: {
      // op, type_A, n_A, A[n_A], type_C, n_C, C[n_C], R[9], t[3]
      if (nq < 3) return bad("composite needs op and two parts");
      const int op = (int)q[0];
      if ((double)op != q[0] || op < kUnion || op > kIntersection) return bad("composite op must be 0, 1 or 2");
      int at = 1, pt[2], pn[2], po[2];
      for (int c = 0; c < 2; ++c) {
        if (at + 2 > nq) return bad("composite parameters truncated");
        pt[c] = (int)q[at];
        pn[c] = (int)q[at + 1];
        if ((double)pt[c] != q[at] || (double)pn[c] != q[at + 1] || pt[c] < kBox || pt[c] > kPcon || pn[c] < 1)
          return bad("composite parts must be elementary solids (types 0-5)");
        po[c] = at + 2;
        at = po[c] + pn[c];
        if (at > nq) return bad("composite parameters truncated");
      }
      if (at + 12 != nq) return bad("composite needs R[9] and t[3] after the parts");
      const double* R = q + at;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double v = 0.0;
          for (int k = 0; k < 3; ++k) v += R[3 * i + k] * R[3 * j + k];
          if (std::fabs(v - (i == j ? 1.0 : 0.0)) > 1e-9) return bad("composite placement R is not a rotation");
        }
      const size_t h = out.size();
      out.resize(h + L::BO_N, 0.0);
      out[h + L::BO_OP] = op;
      out[h + L::BO_TA] = pt[0];
      out[h + L::BO_TC] = pt[1];
      for (int i = 0; i < 12; ++i) out[h + L::BO_R + i] = q[at + i];
      for (int c = 0; c < 2; ++c) {
        out[h + (c == 0 ? L::BO_OA : L::BO_OC)] = (double)(out.size() - h);
        std::string w;
        if (!derive(pt[c], q + po[c], pn[c], out, w)) return bad(c == 0 ? "composite part A invalid" : "composite part C invalid");
      }
      return true;
    }
  }
  why = "unknown solid type";
  return false;
}

struct HostTree {
  std::vector<int> pv_lv, pv_parent, pv_child_off, pv_child;
  std::vector<double> pv_gxf;
  int max_depth = 0;
};

// Axis-aligned box holding a solid in its own frame, from the derived
// parameters (layouts in gv_solids.h).
void local_extent(int type, const double* q, double* lo, double* hi) {
  if (type == kBool) {
    // union: the box around both parts; intersection: the overlap of the
    // parts' boxes; A minus C: A's box
    double alo[3], ahi[3], clo[3], chi[3];
    local_extent((int)q[L::BO_TA], q + (int)q[L::BO_OA], alo, ahi);
    local_extent((int)q[L::BO_TC], q + (int)q[L::BO_OC], clo, chi);
    const double* X = q + L::BO_R;  // R[9] then t[3]
    double blo[3] = {HUGE_VAL, HUGE_VAL, HUGE_VAL}, bhi[3] = {-HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
    for (int c = 0; c < 8; ++c) {
      const double v[3] = {(c & 1) ? chi[0] : clo[0], (c & 2) ? chi[1] : clo[1], (c & 4) ? chi[2] : clo[2]};
      for (int i = 0; i < 3; ++i) {
        const double w = X[3 * i] * v[0] + X[3 * i + 1] * v[1] + X[3 * i + 2] * v[2] + X[9 + i];
        blo[i] = std::min(blo[i], w);
        bhi[i] = std::max(bhi[i], w);
      }
    }
    const int op = (int)q[L::BO_OP];
    bool empty = false;
    for (int i = 0; i < 3; ++i) {
      lo[i] = alo[i], hi[i] = ahi[i];
      if (op == kUnion) {
        lo[i] = std::min(alo[i], blo[i]), hi[i] = std::max(ahi[i], bhi[i]);
      } else if (op == kIntersection) {
        lo[i] = std::max(alo[i], blo[i]), hi[i] = std::min(ahi[i], bhi[i]);
        empty = empty || lo[i] > hi[i];
      }
    }
    if (empty)
      for (int i = 0; i < 3; ++i) lo[i] = alo[i], hi[i] = ahi[i];
    return;
  }
  double rx = 0, ry = 0, z0 = 0, z1 = 0;
  switch (type) {
    case kBox: rx = q[0], ry = q[1], z0 = -q[2], z1 = q[2]; break;
    case kTubs: rx = ry = q[L::TB_RMAX], z0 = -q[L::TB_DZ], z1 = q[L::TB_DZ]; break;
    case kCons:
      rx = ry = std::max(q[L::CN_RMAX1], q[L::CN_RMAX2]), z0 = -q[L::CN_DZ], z1 = q[L::CN_DZ];
      break;
    case kSphere: rx = ry = q[L::SP_RMAX], z0 = -q[L::SP_RMAX], z1 = q[L::SP_RMAX]; break;
    case kTrd:
      rx = std::max(q[L::TD_DX1], q[L::TD_DX2]), ry = std::max(q[L::TD_DY1], q[L::TD_DY2]);
      z0 = -q[L::TD_DZ], z1 = q[L::TD_DZ];
      break;
    default: {  // polycone: nz z[] rmin[] rmax[] ...
      int nz = (int)q[0];
      for (int j = 0; j < nz; ++j) rx = std::max(rx, q[1 + 2 * nz + j]);
      ry = rx, z0 = q[1], z1 = q[nz];
    }
  }
  lo[0] = -rx, lo[1] = -ry, lo[2] = z0;
  hi[0] = rx, hi[1] = ry, hi[2] = z1;
}

// composed transform C = A o B (apply B then A): R = Ra Rb, t = Ra tb + ta
void compose(const double* A, const double* B, double* C) {
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j)
      C[3 * i + j] = A[3 * i + 0] * B[0 + j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
    C[9 + i] = A[3 * i + 0] * B[9] + A[3 * i + 1] * B[10] + A[3 * i + 2] * B[11] + A[9 + i];
  }
}

}  // namespace

extern "C" int geom_load(const void* blob, size_t nbytes, gv_geom** out) {
  if (!out) return fail(GV_EINVAL, "geom_load: out is NULL");
  *out = nullptr;
  if (!blob) return fail(GV_EINVAL, "geom_load: blob is NULL");
  const unsigned char* b = (const unsigned char*)blob;
  static const unsigned char magic[8] = {'G', 'V', 'G', 'E', 'O', 'M', 0, 1};
  if (nbytes < 32 || std::memcmp(b, magic, 8) != 0) return fail(GV_EFORMAT, "geom_load: bad magic");
  int version = rd_i32(b, 8), n_lv = rd_i32(b, 12), n_place = rd_i32(b, 16), n_param = rd_i32(b, 20),
      world = rd_i32(b, 24);
  if (version != 1) return fail(GV_EFORMAT, "geom_load: unsupported version %d", version);
  if (n_lv <= 0 || n_place < 0 || n_param < 0 || world < 0 || world >= n_lv)
    return fail(GV_EFORMAT, "geom_load: bad header counts");
  size_t need = 32 + (size_t)n_lv * 32 + (size_t)n_place * 104 + (size_t)n_param * 8;
  if (need != nbytes) return fail(GV_EFORMAT, "geom_load: size %zu != expected %zu", nbytes, need);
  size_t lv_off = 32, pl_off = lv_off + (size_t)n_lv * 32, pa_off = pl_off + (size_t)n_place * 104;

  try {
    std::vector<double> raw(n_param);
    for (int i = 0; i < n_param; ++i) raw[i] = rd_f64(b, pa_off + 8 * (size_t)i);
    std::vector<int> lv_type(n_lv), lv_par(n_lv), lv_doff(n_lv), lv_dcnt(n_lv);
    std::vector<double> par;
    for (int i = 0; i < n_lv; ++i) {
      size_t o = lv_off + 32 * (size_t)i;
      int type = rd_i32(b, o), poff = rd_i32(b, o + 4), pcnt = rd_i32(b, o + 8);
      lv_doff[i] = rd_i32(b, o + 12);
      lv_dcnt[i] = rd_i32(b, o + 16);
      if (poff < 0 || pcnt < 0 || (long)poff + pcnt > n_param) return fail(GV_EFORMAT, "geom_load: LV %d params", i);
      if (lv_doff[i] < 0 || lv_dcnt[i] < 0 || (long)lv_doff[i] + lv_dcnt[i] > n_place)
        return fail(GV_EFORMAT, "geom_load: LV %d placements", i);
      lv_type[i] = type;
      lv_par[i] = (int)par.size();
      std::string why;
      if (!derive(type, raw.data() + poff, pcnt, par, why))
        return fail(GV_EFORMAT, "geom_load: LV %d: %s", i, why.c_str());
    }
    std::vector<int> dau_lv(n_place);
    std::vector<double> dau_xf((size_t)n_place * 12);
    for (int k = 0; k < n_place; ++k) {
      size_t o = pl_off + 104 * (size_t)k;
      dau_lv[k] = rd_i32(b, o);
      if (dau_lv[k] < 0 || dau_lv[k] >= n_lv) return fail(GV_EFORMAT, "geom_load: placement %d child", k);
      for (int j = 0; j < 12; ++j) dau_xf[12 * (size_t)k + j] = rd_f64(b, o + 8 + 8 * (size_t)j);
    }
    // one solid type for all daughters of an LV lets the daughter loop run a
    // single solid's code
    std::vector<int> lv_dtype(n_lv, -1);
    for (int i = 0; i < n_lv; ++i) {
      int t = -1;
      for (int k = 0; k < lv_dcnt[i]; ++k) {
        int ct = lv_type[dau_lv[lv_doff[i] + k]];
        if (k == 0) t = ct;
        else if (ct != t) t = -1;
      }
      lv_dtype[i] = lv_dcnt[i] > 0 ? t : -1;
    }
    std::vector<int> dau_par(n_place);
    for (int k = 0; k < n_place; ++k) dau_par[k] = lv_par[dau_lv[k]];
    // bounding box of each placed child in its mother's frame: the 8 corners of
    // the child's local box through the placement, padded so that rounding can
    // never make it smaller than the solid
    std::vector<double> dau_box((size_t)n_place * 6);
    for (int k = 0; k < n_place; ++k) {
      const double* q = par.data() + dau_par[k];
      double lo[3], hi[3];
      local_extent(lv_type[dau_lv[k]], q, lo, hi);
      const double* X = &dau_xf[12 * (size_t)k];
      double blo[3] = {HUGE_VAL, HUGE_VAL, HUGE_VAL}, bhi[3] = {-HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
      for (int c = 0; c < 8; ++c) {
        double v[3] = {(c & 1) ? hi[0] : lo[0], (c & 2) ? hi[1] : lo[1], (c & 4) ? hi[2] : lo[2]};
        for (int i = 0; i < 3; ++i) {
          double w = X[3 * i] * v[0] + X[3 * i + 1] * v[1] + X[3 * i + 2] * v[2] + X[9 + i];
          blo[i] = std::min(blo[i], w);
          bhi[i] = std::max(bhi[i], w);
        }
      }
      for (int i = 0; i < 3; ++i) {
        double pad = 1e-6 + 1e-9 * (std::fabs(blo[i]) + std::fabs(bhi[i]));
        dau_box[6 * (size_t)k + i] = blo[i] - pad;
        dau_box[6 * (size_t)k + 3 + i] = bhi[i] + pad;
      }
    }
    // FP32 screen tables.  S of an LV bounds |coordinate| of its solid's points;
    // the FP32 boxes are widened by 128 u (S(mother) + |box|inf), u = 2^-24,
    // and rounded outward, so the FP32 slab test never drops a box the FP64 one
    // keeps for a point with |p|inf <= S (error budget in gv_step.h).
    const double u32 = std::ldexp(1.0, -24);
    auto down32 = [](double v) {
      float f = (float)v;
      return (double)f > v ? std::nextafter(f, -HUGE_VALF) : f;
    };
    auto up32 = [](double v) {
      float f = (float)v;
      return (double)f < v ? std::nextafter(f, HUGE_VALF) : f;
    };
    std::vector<float> lv_scr(n_lv);
    std::vector<double> lv_ext(n_lv);
    for (int i = 0; i < n_lv; ++i) {
      double lo[3], hi[3];
      local_extent(lv_type[i], par.data() + lv_par[i], lo, hi);
      double e = 0;
      for (int a = 0; a < 3; ++a) e = std::max(e, std::max(std::fabs(lo[a]), std::fabs(hi[a])));
      lv_ext[i] = e;
      lv_scr[i] = up32(e + 1.0);
    }
    std::vector<float> dau_box32((size_t)n_place * 8, 0.0f), dau_scr32((size_t)n_place * 16, 0.0f);
    for (int i = 0; i < n_lv; ++i) {
      for (int k = lv_doff[i]; k < lv_doff[i] + lv_dcnt[i]; ++k) {
        const double* B = &dau_box[6 * (size_t)k];
        double bmax = 0;
        for (int a = 0; a < 6; ++a) bmax = std::max(bmax, std::fabs(B[a]));
        const double delta = 128.0 * u32 * ((double)lv_scr[i] + bmax);
        for (int a = 0; a < 3; ++a) {
          dau_box32[8 * (size_t)k + a] = down32(B[a] - delta);
          dau_box32[8 * (size_t)k + 3 + a] = up32(B[3 + a] + delta);
        }
        const double* X = &dau_xf[12 * (size_t)k];
        float* Y = &dau_scr32[16 * (size_t)k];
        double tmax = 0;
        for (int j = 0; j < 12; ++j) Y[j] = (float)X[j];
        for (int j = 9; j < 12; ++j) tmax = std::max(tmax, std::fabs(X[j]));
        const int clv = dau_lv[k];
        const double* q = par.data() + lv_par[clv];
        if (lv_type[clv] == kBox) {
          Y[12] = (float)q[0], Y[13] = (float)q[1], Y[14] = (float)q[2];
        } else if (lv_type[clv] == kTubs) {
          Y[12] = (float)q[L::TB_RMIN], Y[13] = (float)q[L::TB_RMAX], Y[14] = (float)q[L::TB_DZ];
        }
        Y[15] = up32(tmax + lv_ext[clv] + 1.0);
      }
    }
    // identity placements skip their transform; groups of 8 consecutive
    // daughters get the union of their boxes (FP64 and FP32) for a first test
    std::vector<int> dau_ident(n_place, 0), lv_grp(n_lv, -1);
    std::vector<double> grp_box;
    std::vector<float> grp_box32;
    for (int k = 0; k < n_place; ++k) {
      const double* X = &dau_xf[12 * (size_t)k];
      const double I[12] = {1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0};
      bool id = true;
      for (int j = 0; j < 12; ++j) id = id && X[j] == I[j];
      dau_ident[k] = id ? 1 : 0;
    }
    for (int i = 0; i < n_lv; ++i) {
      if (lv_dcnt[i] < kGroupMin) continue;
      lv_grp[i] = (int)(grp_box.size() / 6);
      for (int g0 = 0; g0 < lv_dcnt[i]; g0 += kGroup) {
        double lo[3] = {HUGE_VAL, HUGE_VAL, HUGE_VAL}, hi[3] = {-HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
        float lo32[3] = {HUGE_VALF, HUGE_VALF, HUGE_VALF}, hi32[3] = {-HUGE_VALF, -HUGE_VALF, -HUGE_VALF};
        for (int k = lv_doff[i] + g0; k < lv_doff[i] + std::min(lv_dcnt[i], g0 + kGroup); ++k)
          for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], dau_box[6 * (size_t)k + a]);
            hi[a] = std::max(hi[a], dau_box[6 * (size_t)k + 3 + a]);
            lo32[a] = std::min(lo32[a], dau_box32[8 * (size_t)k + a]);
            hi32[a] = std::max(hi32[a], dau_box32[8 * (size_t)k + 3 + a]);
          }
        grp_box.insert(grp_box.end(), {lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]});
        grp_box32.insert(grp_box32.end(), {lo32[0], lo32[1], lo32[2], hi32[0], hi32[1], hi32[2], 0.0f, 0.0f});
      }
    }
    // radial order: LVs with >= kCullMin daughters that are all identity-placed
    // full tubes whose radial ranges [rmin, rmax] are pairwise disjoint
    std::vector<int> lv_rad(n_lv, -1), rad_k;
    std::vector<double> rad_r2;
    for (int i = 0; i < n_lv; ++i) {
      const int c = lv_dcnt[i], o = lv_doff[i];
      if (c < kCullMin) continue;
      bool ok = true;
      std::vector<std::pair<double, int>> by_r;
      for (int k = 0; k < c && ok; ++k) {
        const int clv = dau_lv[o + k];
        const double* q = par.data() + lv_par[clv];
        ok = lv_type[clv] == kTubs && dau_ident[o + k] && q[L::TB_PHI] == 0.0;
        if (ok) by_r.push_back({q[L::TB_RMIN], k});
      }
      if (!ok) continue;
      std::sort(by_r.begin(), by_r.end());
      for (size_t m = 1; m < by_r.size() && ok; ++m) {
        const double* qa = par.data() + lv_par[dau_lv[o + by_r[m - 1].second]];
        ok = qa[L::TB_RMAX] < by_r[m].first;
      }
      if (!ok) continue;
      lv_rad[i] = (int)rad_k.size();
      for (auto& e : by_r) {
        const double* q = par.data() + lv_par[dau_lv[o + e.second]];
        rad_r2.push_back(q[L::TB_RMIN] * q[L::TB_RMIN]);
        rad_r2.push_back(q[L::TB_RMAX] * q[L::TB_RMAX]);
        rad_k.push_back(e.second);
      }
    }
    // phi sectors: LVs without a radial list, with kCullMin..64 daughters of one
    // type (box or tube) that each lie within less than a half turn around the
    // z axis (angular extent of the corners of the child's padded local box
    // through its placement, in the mother frame)
    std::vector<int> lv_phi(n_lv, -1);
    std::vector<unsigned long long> phi_mask;
    for (int i = 0; i < n_lv; ++i) {
      const int c = lv_dcnt[i], o = lv_doff[i];
      if (lv_rad[i] >= 0 || c < kCullMin || c > 64 || (lv_dtype[i] != kBox && lv_dtype[i] != kTubs)) continue;
      std::vector<unsigned long long> m(kPhiSectors, 0ull);
      bool ok = true;
      for (int k = 0; k < c && ok; ++k) {
        const int clv = dau_lv[o + k];
        double lo[3], hi[3];
        local_extent(lv_type[clv], par.data() + lv_par[clv], lo, hi);
        const double* X = &dau_xf[12 * (size_t)(o + k)];
        double ang[8], sx = 0.0, sy = 0.0;
        for (int q = 0; q < 8; ++q) {
          const double v[3] = {(q & 1) ? hi[0] + 1e-6 : lo[0] - 1e-6, (q & 2) ? hi[1] + 1e-6 : lo[1] - 1e-6,
                               (q & 4) ? hi[2] + 1e-6 : lo[2] - 1e-6};
          const double X0 = X[0] * v[0] + X[1] * v[1] + X[2] * v[2] + X[9];
          const double Y0 = X[3] * v[0] + X[4] * v[1] + X[5] * v[2] + X[10];
          ang[q] = std::atan2(Y0, X0);
          sx += X0;
          sy += Y0;
          ok = ok && X0 * X0 + Y0 * Y0 > 1e-6;
        }
        const double am = std::atan2(sy, sx);
        double alo = HUGE_VAL, ahi = -HUGE_VAL;
        for (double a : ang) {
          double d = a - am;  // unwrapped around the mean direction
          while (d > M_PI) d -= 2.0 * M_PI;
          while (d <= -M_PI) d += 2.0 * M_PI;
          alo = std::min(alo, d);
          ahi = std::max(ahi, d);
        }
        ok = ok && ahi - alo < 0.9 * M_PI;
        if (!ok) break;
        // pseudo-angle interval, widened by 1e-4 (rounding of the lane's angles
        // is ~1e-15), swept counterclockwise from plo to phi
        const double plo = pseudo_angle(std::cos(am + alo), std::sin(am + alo)) - 1e-4;
        const double phi = pseudo_angle(std::cos(am + ahi), std::sin(am + ahi)) + 1e-4;
        auto sec = [](double a) {
          a = std::fmod(a + 4.0, 4.0);
          return std::min(kPhiSectors - 1, std::max(0, (int)(a * (kPhiSectors / 4.0))));
        };
        for (int s0 = sec(plo), s = s0;; s = (s + 1) % kPhiSectors) {
          m[s] |= 1ull << k;
          if (s == sec(phi)) break;
        }
      }
      if (!ok) continue;
      lv_phi[i] = (int)phi_mask.size();
      phi_mask.insert(phi_mask.end(), m.begin(), m.end());
    }
    // step class of each LV: the branch its steps take in the step code (the
    // mother's solid type and how the daughters are reached), for the lane
    // form's per-class scheduling
    std::vector<int> lv_class(n_lv, 0);
    for (int i = 0; i < n_lv; ++i) {
      const int c = lv_dcnt[i], dt = lv_dtype[i];
      int mode;
      if (c == 0) mode = 0;
      else if (lv_rad[i] >= 0) mode = 1;
      else if (lv_phi[i] >= 0) mode = dt == kBox ? 2 : 3;
      else if ((dt == kBox || dt == kTubs) && c >= kCullMin) mode = dt == kBox ? 4 : 5;
      else if (dt == kBox || dt == kTubs) mode = dt == kBox ? 6 : 7;
      else mode = 8;
      lv_class[i] = mode * 8 + lv_type[i];
    }
    // count the tree first (depth and size limits also reject cycles)
    std::vector<long> subtree(n_lv, -1);
    std::vector<int> state(n_lv, 0), height(n_lv, 0);
    struct Counter {
      const std::vector<int>&doff, &dcnt, &dlv;
      std::vector<long>& sub;
      std::vector<int>&st, &h;
      bool go(int lv) {
        if (st[lv] == 2) return true;
        if (st[lv] == 1) return false;  // cycle
        st[lv] = 1;
        long n = 1;
        int hh = 0;
        for (int k = 0; k < dcnt[lv]; ++k) {
          int c = dlv[doff[lv] + k];
          if (!go(c)) return false;
          n += sub[c];
          hh = std::max(hh, h[c] + 1);
          if (n > kMaxPv || hh > kMaxDepth) return false;
        }
        sub[lv] = n;
        h[lv] = hh;
        st[lv] = 2;
        return true;
      }
    } counter{lv_doff, lv_dcnt, dau_lv, subtree, state, height};
    if (!counter.go(world)) return fail(GV_EFORMAT, "geom_load: volume tree has a cycle or is too large/deep");
    long npv = subtree[world];
    HostTree T;
    T.pv_lv.resize(npv);
    T.pv_parent.resize(npv);
    T.pv_child_off.resize(npv);
    T.pv_child.resize(npv > 0 ? npv - 1 : 0);
    T.pv_gxf.resize((size_t)npv * 12);
    std::vector<int> pv_k(npv, -1);
    T.max_depth = height[world];
    // DFS pre-order expansion with an explicit stack
    struct Frame {
      int pv, lv, next_k;
    };
    std::vector<Frame> stack;
    int next_id = 0, child_fill = 0;
    const double ident[12] = {1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0};
    auto open = [&](int lv, int parent, const double* gxf) {
      int me = next_id++;
      T.pv_lv[me] = lv;
      T.pv_parent[me] = parent;
      std::memcpy(&T.pv_gxf[12 * (size_t)me], gxf, 12 * sizeof(double));
      T.pv_child_off[me] = child_fill;
      child_fill += lv_dcnt[lv];
      stack.push_back(Frame{me, lv, 0});
    };
    open(world, -1, ident);
    while (!stack.empty()) {
      Frame& f = stack.back();
      if (f.next_k >= lv_dcnt[f.lv]) {
        stack.pop_back();
        continue;
      }
      int k = f.next_k++;
      int pl = lv_doff[f.lv] + k;
      int parent = f.pv;
      T.pv_child[T.pv_child_off[parent] + k] = next_id;
      pv_k[next_id] = k;
      double g[12];
      compose(&T.pv_gxf[12 * (size_t)parent], &dau_xf[12 * (size_t)pl], g);
      open(dau_lv[pl], parent, g);
    }

    std::vector<int> pv_lc(2 * (size_t)npv);
    for (long i = 0; i < npv; ++i) {
      pv_lc[2 * i] = T.pv_lv[i];
      pv_lc[2 * i + 1] = lv_class[T.pv_lv[i]];
    }

    // one device allocation, 256-byte aligned sub-arrays
    struct Part {
      const void* src;
      size_t bytes;
      size_t off;
    };
    std::vector<Part> parts = {
        {lv_type.data(), lv_type.size() * 4, 0},   {lv_par.data(), lv_par.size() * 4, 0},
        {lv_doff.data(), lv_doff.size() * 4, 0},   {lv_dcnt.data(), lv_dcnt.size() * 4, 0},
        {par.data(), par.size() * 8, 0},           {dau_xf.data(), dau_xf.size() * 8, 0},
        {dau_lv.data(), dau_lv.size() * 4, 0},     {T.pv_lv.data(), T.pv_lv.size() * 4, 0},
        {T.pv_parent.data(), T.pv_parent.size() * 4, 0}, {T.pv_gxf.data(), T.pv_gxf.size() * 8, 0},
        {T.pv_child_off.data(), T.pv_child_off.size() * 4, 0}, {T.pv_child.data(), T.pv_child.size() * 4, 0},
        {lv_dtype.data(), lv_dtype.size() * 4, 0}, {dau_par.data(), dau_par.size() * 4, 0},
        {dau_box.data(), dau_box.size() * 8, 0},   {lv_scr.data(), lv_scr.size() * 4, 0},
        {dau_box32.data(), dau_box32.size() * 4, 0}, {dau_scr32.data(), dau_scr32.size() * 4, 0},
        {dau_ident.data(), dau_ident.size() * 4, 0}, {lv_grp.data(), lv_grp.size() * 4, 0},
        {grp_box.data(), grp_box.size() * 8, 0},     {grp_box32.data(), grp_box32.size() * 4, 0},
        {lv_rad.data(), lv_rad.size() * 4, 0},       {rad_r2.data(), rad_r2.size() * 8, 0},
        {rad_k.data(), rad_k.size() * 4, 0},         {lv_phi.data(), lv_phi.size() * 4, 0},
        {phi_mask.data(), phi_mask.size() * 8, 0},   {nullptr, 5 * 8, 0},
        {lv_class.data(), lv_class.size() * 4, 0},   {pv_k.data(), pv_k.size() * 4, 0},
        {pv_lc.data(), pv_lc.size() * 4, 0}};
    size_t total = 0;
    for (auto& p : parts) {
      p.off = total;
      total += (p.bytes + 255) & ~(size_t)255;
    }
    std::vector<unsigned char> host(total, 0);
    for (auto& p : parts)
      if (p.bytes && p.src) std::memcpy(host.data() + p.off, p.src, p.bytes);
    gv_geom* g = new (std::nothrow) gv_geom();
    if (!g) return fail(GV_ENOMEM, "geom_load: host allocation");
    hipError_t e = hipGetDevice(&g->device);
    if (e != hipSuccess) {
      delete g;
      return hip_fail(e, "geom_load: hipGetDevice");
    }
    e = hipDeviceGetAttribute(&g->n_cu, hipDeviceAttributeMultiprocessorCount, g->device);
    if (e != hipSuccess || g->n_cu < 1) g->n_cu = 256;
    if (init_noalloc_scratch(g->device) != GV_OK) {
      delete g;
      return GV_EHIP;
    }
    e = hipMalloc(&g->dmem, total);
    if (e != hipSuccess) {
      delete g;
      return fail(GV_ENOMEM, "geom_load: hipMalloc(%zu): %s", total, hipGetErrorString(e));
    }
    e = hipMemcpy(g->dmem, host.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(g->dmem);
      delete g;
      return hip_fail(e, "geom_load: hipMemcpy");
    }
    char* base = (char*)g->dmem;
    DevGeom& D = g->dg;
    D.n_lv = n_lv;
    D.n_pv = (int)npv;
    D.n_place = n_place;
    D.lv_type = (CQI)(base + parts[0].off);
    D.lv_par = (CQI)(base + parts[1].off);
    D.lv_dau_off = (CQI)(base + parts[2].off);
    D.lv_dau_cnt = (CQI)(base + parts[3].off);
    D.par = (CQ)(base + parts[4].off);
    D.dau_xf = (CQ)(base + parts[5].off);
    D.dau_lv = (CQI)(base + parts[6].off);
    D.pv_lv = (CQI)(base + parts[7].off);
    D.pv_parent = (CQI)(base + parts[8].off);
    D.pv_gxf = (CQ)(base + parts[9].off);
    D.pv_child_off = (CQI)(base + parts[10].off);
    D.pv_child = (CQI)(base + parts[11].off);
    D.lv_dau_type = (CQI)(base + parts[12].off);
    D.dau_par = (CQI)(base + parts[13].off);
    D.dau_box = (CQ)(base + parts[14].off);
    D.lv_scr = (CQF)(base + parts[15].off);
    D.dau_box32 = (CQF)(base + parts[16].off);
    D.dau_scr32 = (CQF)(base + parts[17].off);
    D.dau_ident = (CQI)(base + parts[18].off);
    D.lv_grp = (CQI)(base + parts[19].off);
    D.grp_box = (CQ)(base + parts[20].off);
    D.grp_box32 = (CQF)(base + parts[21].off);
    D.lv_rad = (CQI)(base + parts[22].off);
    D.rad_r2 = (CQ)(base + parts[23].off);
    D.rad_k = (CQI)(base + parts[24].off);
    D.lv_phi = (CQI)(base + parts[25].off);
    D.phi_mask = (CQL)(base + parts[26].off);
    g->pcon_work = (unsigned long long*)(base + parts[27].off);  // zeroed by the upload
    D.lv_class = (CQI)(base + parts[28].off);
    D.pv_k = (CQI)(base + parts[29].off);
    D.pv_lc = (CQI)(base + parts[30].off);
    g->n_lv = n_lv;
    g->n_pv = (int)npv;
    g->n_place = n_place;
    g->max_depth = T.max_depth;
    g->world_lv = world;
    g->lv_type = lv_type;
    g->has_bool = std::find(lv_type.begin(), lv_type.end(), (int)kBool) != lv_type.end();
    g->lv_par = lv_par;
    *out = g;
    t_err.clear();
    return GV_OK;
  } catch (const std::bad_alloc&) {
    return fail(GV_ENOMEM, "geom_load: out of host memory");
  } catch (...) {
    return fail(GV_EFORMAT, "geom_load: internal error");
  }
}

extern "C" int geom_free(gv_geom* g) {
  if (!g) return GV_OK;
  int dev = -1;
  (void)hipGetDevice(&dev);
  if (dev != g->device) (void)hipSetDevice(g->device);
  hipError_t e = hipDeviceSynchronize();
  if (g->ws) (void)hipFree(g->ws);
  if (g->lws) (void)hipFree(g->lws);
  if (g->ob) (void)hipFree(g->ob);
  if (g->mat_mem) (void)hipFree(g->mat_mem);
  if (g->dmem) (void)hipFree(g->dmem);
  for (auto& ev : g->prof_ev) (void)hipEventDestroy(ev);
  if (dev != g->device && dev >= 0) (void)hipSetDevice(dev);
  delete g;
  if (e != hipSuccess) return hip_fail(e, "geom_free: hipDeviceSynchronize");
  return GV_OK;
}

extern "C" int geom_info(const gv_geom* g, int32_t* counts) {
  if (!g || !counts) return fail(GV_EINVAL, "geom_info: NULL argument");
  counts[0] = g->n_lv;
  counts[1] = g->n_pv;
  counts[2] = g->max_depth;
  counts[3] = g->world_lv;
  return GV_OK;
}

// ---------------------------------------------------------------- helpers
namespace {

struct DeviceGuard {
  int prev = -1, want;
  bool ok = true;
  explicit DeviceGuard(int dev) : want(dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != want) ok = hipSetDevice(want) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0 && prev != want) (void)hipSetDevice(prev);
  }
};

bool al8(const void* p) { return ((uintptr_t)p & 7u) == 0; }
bool al4(const void* p) { return ((uintptr_t)p & 3u) == 0; }

int check_common(const char* fn, gv_geom* g, int64_t n) {
  if (!g) return fail(GV_EINVAL, "%s: geometry handle is NULL", fn);
  if (n < 0) return fail(GV_EINVAL, "%s: n = %lld < 0", fn, (long long)n);
  return GV_OK;
}

int check_f64(const char* fn, const char* name, const void* p, bool nullable = false) {
  if (!p) return nullable ? GV_OK : fail(GV_EINVAL, "%s: %s is NULL", fn, name);
  if (!al8(p)) return fail(GV_EINVAL, "%s: %s is not 8-byte aligned", fn, name);
  return GV_OK;
}
int check_i32(const char* fn, const char* name, const void* p, bool nullable = false) {
  if (!p) return nullable ? GV_OK : fail(GV_EINVAL, "%s: %s is NULL", fn, name);
  if (!al4(p)) return fail(GV_EINVAL, "%s: %s is not 4-byte aligned", fn, name);
  return GV_OK;
}

constexpr int kBlock = 256;

// Launch shape of the one-lane-per-track kernels (solid level, per-track
// navigation): the tuned block size and workgroup cap, else 256 threads and
// one lane per track.  Every kernel of this kind is grid-stride, so the shape
// never changes a result.
struct Shape {
  unsigned grid, block;
};
Shape lane_shape(const gv_geom* g, int64_t n) {
  const int64_t blk = g->tune.solid_block > 0 ? g->tune.solid_block : kBlock;
  int64_t b = (n + blk - 1) / blk;
  const int64_t cap = g->tune.solid_grid > 0 ? g->tune.solid_grid : (1 << 20);
  b = std::min(b, cap);
  return Shape{(unsigned)std::max<int64_t>(1, b), (unsigned)blk};
}

int launched(const char* fn) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, fn);
  t_err.clear();
  return GV_OK;
}

#define GV_TRY(expr)     \
  do {                   \
    int rc_ = (expr);    \
    if (rc_) return rc_; \
  } while (0)

}  // namespace

// ------------------------------------------------------ solid-level entry points
#define GV_SOLID_SWITCH(type, CALL) \
  switch (type) {                   \
    case kBox: CALL(Box); break;    \
    case kTubs: CALL(Tubs); break;  \
    case kCons: CALL(Cons); break;  \
    case kSphere: CALL(Sphere); break; \
    case kTrd: CALL(Trd); break;    \
    case kBool: CALL(Bool); break;  \
    default: CALL(Pcon); break;     \
  }

// Navigation entry points take GV_FP64 or GV_FP32_REFINE (FP32 daughter
// screens, FP64 values: the same outputs).
int check_nav_precision(const char* fn, int32_t precision) {
  if (precision != GV_FP64 && precision != GV_FP32_REFINE)
    return fail(GV_EINVAL, "%s: precision %d is neither GV_FP64 nor GV_FP32_REFINE", fn, precision);
  return GV_OK;
}

// Workgroups of the compacting polycone kernel: 4 wavefronts of 4 x 64 tracks
// each (on 2^20 full-set tracks, DistanceToIn 56.6 / 45.2 / 43.2 / 49.9 /
// 70.7 us at 1 / 2 / 4 / 8 / 16 chunks of 64 per wavefront: fewer leave the
// queues short of 64 rays, more leave too few wavefronts to hide latency).
unsigned pcon_grid(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 1023) / 1024); }

// With GV_PROF_WORK, a polycone query is followed by the kernel that counts
// its walk's work (profiling only; the query's outputs are untouched).
int pcon_work(gv_geom* g, int32_t lv, int dir, int64_t n, const double* x, const double* y, const double* z,
              const double* dx, const double* dy, const double* dz, hipStream_t s, const char* fn) {
  if (!g->prof_work || g->lv_type[lv] != kPcon) return GV_OK;
  const Shape sh = lane_shape(g, n);
  hipLaunchKernelGGL(k_pcon_work, dim3(sh.grid), dim3(sh.block), 0, s, g->dg.par + g->lv_par[lv], dir, n, x, y, z,
                     dx, dy, dz, g->pcon_work);
  return launched(fn);
}

extern "C" int basket_inside(gv_geom* g, int32_t lv, int64_t n, const double* x, const double* y, const double* z,
                             int8_t* out, void* stream) {
  const char* fn = "basket_inside";
  GV_TRY(check_common(fn, g, n));
  if (lv < 0 || lv >= g->n_lv) return fail(GV_EINVAL, "%s: lv %d out of range [0, %d)", fn, lv, g->n_lv);
  if (n == 0) return GV_OK;
  GV_TRY(check_f64(fn, "x", x));
  GV_TRY(check_f64(fn, "y", y));
  GV_TRY(check_f64(fn, "z", z));
  if (!out) return fail(GV_EINVAL, "%s: out is NULL", fn);
  DeviceGuard dgd(g->device);
  CQ q = g->dg.par + g->lv_par[lv];
  hipStream_t s = (hipStream_t)stream;
  const Shape sh = lane_shape(g, n);
#define CALL(S) hipLaunchKernelGGL(k_inside<S>, dim3(sh.grid), dim3(sh.block), 0, s, q, n, x, y, z, out)
  GV_SOLID_SWITCH(g->lv_type[lv], CALL)
#undef CALL
  return launched(fn);
}

extern "C" int basket_safety(gv_geom* g, int32_t lv, int32_t side, int64_t n, const double* x, const double* y,
                             const double* z, double* out_safety, int8_t* out_inside, int32_t precision,
                             void* stream) {
  const char* fn = "basket_safety";
  GV_TRY(check_common(fn, g, n));
  if (lv < 0 || lv >= g->n_lv) return fail(GV_EINVAL, "%s: lv %d out of range [0, %d)", fn, lv, g->n_lv);
  if (side < 0 || side > 2) return fail(GV_EINVAL, "%s: side %d", fn, side);
  if (precision != GV_FP64) return fail(GV_EINVAL, "%s: precision %d not supported", fn, precision);
  if (n == 0) return GV_OK;
  GV_TRY(check_f64(fn, "x", x));
  GV_TRY(check_f64(fn, "y", y));
  GV_TRY(check_f64(fn, "z", z));
  GV_TRY(check_f64(fn, "out_safety", out_safety, true));
  if (!out_safety && !out_inside) return fail(GV_EINVAL, "%s: both outputs are NULL", fn);
  DeviceGuard dgd(g->device);
  CQ q = g->dg.par + g->lv_par[lv];
  hipStream_t s = (hipStream_t)stream;
  const Shape sh = lane_shape(g, n);
#define CALL(S) \
  hipLaunchKernelGGL(k_safety<S>, dim3(sh.grid), dim3(sh.block), 0, s, q, (int)side, n, x, y, z, out_safety, out_inside)
  GV_SOLID_SWITCH(g->lv_type[lv], CALL)
#undef CALL
  return launched(fn);
}

extern "C" int basket_distance(gv_geom* g, int32_t lv, int32_t dir, int64_t n, const double* x, const double* y,
                               const double* z, const double* dx, const double* dy, const double* dz, double* out,
                               int32_t precision, void* stream) {
  const char* fn = "basket_distance";
  GV_TRY(check_common(fn, g, n));
  if (lv < 0 || lv >= g->n_lv) return fail(GV_EINVAL, "%s: lv %d out of range [0, %d)", fn, lv, g->n_lv);
  if (dir != GV_TO_IN && dir != GV_TO_OUT) return fail(GV_EINVAL, "%s: dir %d", fn, dir);
  if (precision != GV_FP64) return fail(GV_EINVAL, "%s: precision %d not supported", fn, precision);
  if (n == 0) return GV_OK;
  const double* in[6] = {x, y, z, dx, dy, dz};
  const char* nm[6] = {"x", "y", "z", "dx", "dy", "dz"};
  for (int i = 0; i < 6; ++i) GV_TRY(check_f64(fn, nm[i], in[i]));
  GV_TRY(check_f64(fn, "out", out));
  DeviceGuard dgd(g->device);
  CQ q = g->dg.par + g->lv_par[lv];
  hipStream_t s = (hipStream_t)stream;
  const Shape sh = lane_shape(g, n);
  if (g->lv_type[lv] == kPcon && dir == GV_TO_IN) {
    // walking rays compacted per wavefront (43 against 53 us on 2^20 full-set
    // tracks; DistanceToOut, where half of the rays walk, gains nothing)
    hipLaunchKernelGGL(k_pcon_compact<0>, dim3(pcon_grid(n)), dim3(256), 0, s, q, n, x, y, z, dx, dy, dz, nullptr,
                       nullptr, out, nullptr);
  } else if (dir == GV_TO_IN) {
#define CALL(S) hipLaunchKernelGGL((k_distance<S, 0>), dim3(sh.grid), dim3(sh.block), 0, s, q, n, x, y, z, dx, dy, dz, out)
    GV_SOLID_SWITCH(g->lv_type[lv], CALL)
#undef CALL
  } else {
#define CALL(S) hipLaunchKernelGGL((k_distance<S, 1>), dim3(sh.grid), dim3(sh.block), 0, s, q, n, x, y, z, dx, dy, dz, out)
    GV_SOLID_SWITCH(g->lv_type[lv], CALL)
#undef CALL
  }
  GV_TRY(launched(fn));
  return pcon_work(g, lv, dir, n, x, y, z, dx, dy, dz, s, fn);
}

extern "C" int basket_solid_all(gv_geom* g, int32_t lv, int64_t n, const double* x, const double* y, const double* z,
                                const double* dx, const double* dy, const double* dz, int8_t* out_inside,
                                double* out_safety, double* out_dist_in, double* out_dist_out, void* stream) {
  const char* fn = "basket_solid_all";
  GV_TRY(check_common(fn, g, n));
  if (lv < 0 || lv >= g->n_lv) return fail(GV_EINVAL, "%s: lv %d out of range [0, %d)", fn, lv, g->n_lv);
  if (n == 0) return GV_OK;
  const double* in[6] = {x, y, z, dx, dy, dz};
  const char* nm[6] = {"x", "y", "z", "dx", "dy", "dz"};
  for (int i = 0; i < 6; ++i) GV_TRY(check_f64(fn, nm[i], in[i]));
  GV_TRY(check_f64(fn, "out_safety", out_safety, true));
  GV_TRY(check_f64(fn, "out_dist_in", out_dist_in, true));
  GV_TRY(check_f64(fn, "out_dist_out", out_dist_out, true));
  if (!out_inside && !out_safety && !out_dist_in && !out_dist_out)
    return fail(GV_EINVAL, "%s: all outputs are NULL", fn);
  DeviceGuard dgd(g->device);
  CQ q = g->dg.par + g->lv_par[lv];
  hipStream_t s = (hipStream_t)stream;
  const Shape sh = lane_shape(g, n);
#define CALL(S)                                                                                          \
  hipLaunchKernelGGL(k_solid_all<S>, dim3(sh.grid), dim3(sh.block), 0, s, q, n, x, y, z, dx, dy, dz, out_inside, \
                     out_safety, out_dist_in, out_dist_out)
  if (g->lv_type[lv] == kPcon) {  // walking rays compacted per wavefront (85 against 111 us)
    hipLaunchKernelGGL(k_pcon_compact<2>, dim3(pcon_grid(n)), dim3(256), 0, s, q, n, x, y, z, dx, dy, dz, out_inside,
                       out_safety, out_dist_in, out_dist_out);
  } else {
    GV_SOLID_SWITCH(g->lv_type[lv], CALL)
  }
#undef CALL
  GV_TRY(launched(fn));
  return pcon_work(g, lv, 2, n, x, y, z, dx, dy, dz, s, fn);
}

// ------------------------------------------------------- navigation entry points
extern "C" int basket_locate(gv_geom* g, int64_t n, const double* x, const double* y, const double* z,
                             int32_t* out_pv, void* stream) {
  const char* fn = "basket_locate";
  GV_TRY(check_common(fn, g, n));
  if (n == 0) return GV_OK;
  GV_TRY(check_f64(fn, "x", x));
  GV_TRY(check_f64(fn, "y", y));
  GV_TRY(check_f64(fn, "z", z));
  GV_TRY(check_i32(fn, "out_pv", out_pv));
  DeviceGuard dgd(g->device);
  hipLaunchKernelGGL(g->has_bool ? k_locate<true> : k_locate<false>, dim3(lane_shape(g, n).grid), dim3(lane_shape(g, n).block), 0, (hipStream_t)stream, g->dg, n, x, y, z, out_pv);
  return launched(fn);
}

extern "C" int basket_step(gv_geom* g, int64_t n, const double* x, const double* y, const double* z,
                           const double* dx, const double* dy, const double* dz, const int32_t* pv,
                           const double* pstep, double* out_step, int32_t* out_next_pv, uint32_t* out_flags,
                           int32_t precision, void* stream) {
  const char* fn = "basket_step";
  GV_TRY(check_common(fn, g, n));
  GV_TRY(check_nav_precision(fn, precision));
  if (n == 0) return GV_OK;
  const double* in[6] = {x, y, z, dx, dy, dz};
  const char* nm[6] = {"x", "y", "z", "dx", "dy", "dz"};
  for (int i = 0; i < 6; ++i) GV_TRY(check_f64(fn, nm[i], in[i]));
  GV_TRY(check_i32(fn, "pv", pv));
  GV_TRY(check_f64(fn, "pstep", pstep, true));
  GV_TRY(check_f64(fn, "out_step", out_step));
  GV_TRY(check_i32(fn, "out_next_pv", out_next_pv));
  GV_TRY(check_i32(fn, "out_flags", out_flags, true));
  DeviceGuard dgd(g->device);
  const auto kern = g->has_bool ? (precision == GV_FP64 ? k_step_nav<false, true> : k_step_nav<true, true>)
                                : (precision == GV_FP64 ? k_step_nav<false, false> : k_step_nav<true, false>);
  hipLaunchKernelGGL(kern, dim3(lane_shape(g, n).grid), dim3(lane_shape(g, n).block), 0,
                     (hipStream_t)stream, g->dg, n, x, y, z, dx, dy, dz, pv, pstep, out_step, out_next_pv, out_flags);
  return launched(fn);
}

extern "C" int basket_nav_safety(gv_geom* g, int64_t n, const double* x, const double* y, const double* z,
                                 const int32_t* pv, double* out, int32_t precision, void* stream) {
  const char* fn = "basket_nav_safety";
  GV_TRY(check_common(fn, g, n));
  GV_TRY(check_nav_precision(fn, precision));
  if (n == 0) return GV_OK;
  GV_TRY(check_f64(fn, "x", x));
  GV_TRY(check_f64(fn, "y", y));
  GV_TRY(check_f64(fn, "z", z));
  GV_TRY(check_i32(fn, "pv", pv));
  GV_TRY(check_f64(fn, "out", out));
  DeviceGuard dgd(g->device);
  const auto kern = g->has_bool ? (precision == GV_FP64 ? k_nav_safety<true> : k_nav_safety_scr<true>)
                                : (precision == GV_FP64 ? k_nav_safety<false> : k_nav_safety_scr<false>);
  hipLaunchKernelGGL(kern, dim3(lane_shape(g, n).grid), dim3(lane_shape(g, n).block), 0,
                     (hipStream_t)stream, g->dg, n, x, y, z, pv, out);
  return launched(fn);
}

extern "C" int basket_nav_inside(gv_geom* g, int64_t n, const double* x, const double* y, const double* z,
                                 const int32_t* pv, int8_t* out, void* stream) {
  const char* fn = "basket_nav_inside";
  GV_TRY(check_common(fn, g, n));
  if (n == 0) return GV_OK;
  GV_TRY(check_f64(fn, "x", x));
  GV_TRY(check_f64(fn, "y", y));
  GV_TRY(check_f64(fn, "z", z));
  GV_TRY(check_i32(fn, "pv", pv));
  if (!out) return fail(GV_EINVAL, "%s: out is NULL", fn);
  DeviceGuard dgd(g->device);
  hipLaunchKernelGGL(g->has_bool ? k_nav_inside<true> : k_nav_inside<false>, dim3(lane_shape(g, n).grid), dim3(lane_shape(g, n).block), 0, (hipStream_t)stream, g->dg, n, x, y, z, pv,
                     out);
  return launched(fn);
}

// ------------------------------------------------ basket transport workspace
namespace {

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// Bits of the coarse direction cell in a bucket key (LV << bits | cell): by
// default 4 cells (2 x 2) while LVs x cells <= 4096, else none.  Finer cells
// (16) gave the same step time with the daughter indexes and cost more in the
// bucket layouts of every step.  The tuned value applies while LVs x cells
// stays within 4096.
int cell_bits(const gv_geom* g) {
  const int t = g->tune.cell_bits;
  if (t >= 0 && (g->n_lv << t) <= 4096) return t;
  return g->n_lv <= 1024 ? 2 : 0;
}

// Workgroups of the regrouping kernels (1024 threads each, about 4096 list
// entries per workgroup by default).
unsigned scatter_grid(const gv_geom* g, int64_t n) {
  if (g->tune.scatter_grid > 0) return (unsigned)std::min<int64_t>(g->tune.scatter_grid, n / 64 + 1);
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 4095) / 4096, 256));
}

// Workgroups of the per-step kernel: by default one per four tiles of the
// first list, at most kMaxStepGrid (the whole grid is then resident).
unsigned step_grid_for(const gv_geom* g, int64_t n) {
  const int64_t max_tiles = n / kWave + g->n_lv + 1;
  int64_t w = g->tune.step_grid > 0 ? g->tune.step_grid : (max_tiles + 3) / 4;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(w, kMaxStepGrid));
}

// Track records, two bucketed index lists, the next-LV array, and per-LV
// counters and layouts.  Allocated with hipMalloc on first use and kept in the
// handle.
int ensure_workspace(gv_geom* g, int64_t n) {
  const int nl = g->n_lv << cell_bits(g);
  if (g->ws && g->ws_tracks >= n && g->ws_nl >= nl) return GV_OK;
  int64_t cap = n < 4096 ? 4096 : std::max<int64_t>(n, g->ws_tracks);
  size_t total = al256(sizeof(TRec) * (size_t)cap) + 5 * al256(4 * (size_t)cap) + 6 * al256(4 * (size_t)nl) +
                 al256(8 * kWorkN) + al256(4) + al256(4 * (size_t)kMaxStepGrid * nl) + al256(8);
  if (g->ws) {
    (void)hipDeviceSynchronize();
    (void)hipFree(g->ws);
    g->ws = nullptr;
    g->ws_tracks = 0;
  }
  void* mem = nullptr;
  hipError_t e = hipMalloc(&mem, total);
  if (e != hipSuccess) return fail(GV_ENOMEM, "nav_transport: workspace hipMalloc(%zu): %s", total, hipGetErrorString(e));
  // no clearing needed: every transport clears its counters with k_bt_clear
  // and writes every other array before reading it
  char* p = (char*)mem;
  auto take = [&](size_t b) {
    char* r = p;
    p += al256(b);
    return r;
  };
  g->rec = (TRec*)take(sizeof(TRec) * cap);
  g->idx[0] = (int*)take(4 * cap);
  g->idx[1] = (int*)take(4 * cap);
  g->nxt_lv = (int*)take(4 * cap);
  g->nxt_pos = (uint32_t*)take(4 * cap);
  g->slot_id = (int*)take(4 * cap);
  for (int s = 0; s < 3; ++s) {
    g->ctl.cnt[s] = (int*)take(4 * nl);
    g->ctl.cur[s] = (int*)take(4 * nl);
  }
  g->ctl.work = (unsigned long long*)take(8 * kWorkN);
  g->ctl.nlive = (int*)take(4);
  g->ctl.seg = (int*)take(4 * (size_t)kMaxStepGrid * nl);
  g->ctl.len = (int*)take(8);
  g->ws = mem;
  g->ws_bytes = total;
  g->ws_tracks = cap;
  g->ws_nl = nl;
  return GV_OK;
}

// Step-major output staging for `steps` steps of the workspace's tracks, kept
// in the handle and grown on demand; up to kStageMaxBytes.  Returns false (and
// leaves ob_step NULL) when it would be larger, and the step kernel then writes
// the rows directly.
constexpr size_t kStageMaxBytes = (size_t)8 << 30;
bool ensure_staging(gv_geom* g, int64_t steps) {
  const int64_t cap = g->ws_tracks;
  const size_t bytes = (size_t)cap * (size_t)steps * 13;
  if (bytes > kStageMaxBytes) return false;
  if (g->ob && g->ob_cap >= cap && g->ob_steps >= steps) return true;
  if (g->ob) {
    (void)hipDeviceSynchronize();
    (void)hipFree(g->ob);
    g->ob = nullptr;
    g->ob_step = nullptr;
    g->ob_pv = nullptr;
    g->ob_proc = nullptr;
    g->ob_cap = g->ob_steps = 0;
  }
  const size_t b8 = al256((size_t)cap * steps * 8), b4 = al256((size_t)cap * steps * 4);
  if (hipMalloc(&g->ob, b8 + b4 + (size_t)cap * steps) != hipSuccess) {
    (void)hipGetLastError();
    g->ob = nullptr;
    return false;
  }
  g->ob_step = (double*)g->ob;
  g->ob_pv = (int*)((char*)g->ob + b8);
  g->ob_proc = (int8_t*)((char*)g->ob + b8 + b4);
  g->ob_cap = cap;
  g->ob_steps = steps;
  return true;
}

// Whether the staging from an earlier call covers this one (used under stream
// capture, where nothing is allocated).  Without it the step kernel writes the
// rows directly, with the same results.
bool staging_ready(const gv_geom* g, int64_t steps) {
  return g->ob && g->ob_cap >= g->ws_tracks && g->ob_steps >= steps;
}

// The per-step kernel for this call: composites or not, FP32 screens or not,
// physics-limited or not, the work-counting instance while counters are
// asked for (geometries without composites), and the tuned register budget
// of the navigation step (3 or 4 waves per SIMD).
using StepKernel = void (*)(DevGeom, int, int, int, const int*, const int*, TRec*, const int*, int*, uint32_t*, int*,
                            TCtl, int32_t*, double*, int32_t*, uint32_t*, const int*, double*, int*, int64_t,
                            PhysArgs, int8_t*, int8_t*);
StepKernel select_step_kernel(const gv_geom* g, bool fp32, bool phys) {
  if (g->has_bool) {
    if (phys) return fp32 ? k_bt_step<true, true, true, false, 3> : k_bt_step<false, true, true, false, 3>;
    return fp32 ? k_bt_step<true, false, true, false, 4> : k_bt_step<false, false, true, false, 4>;
  }
  if (g->prof_work) {
    if (phys) return fp32 ? k_bt_step<true, true, false, true, 3> : k_bt_step<false, true, false, true, 3>;
    return fp32 ? k_bt_step<true, false, false, true, 4> : k_bt_step<false, false, false, true, 4>;
  }
  if (phys) return fp32 ? k_bt_step<true, true, false, false, 3> : k_bt_step<false, true, false, false, 3>;
  if (g->tune.step_waves == 3)
    return fp32 ? k_bt_step<true, false, false, false, 3> : k_bt_step<false, false, false, false, 3>;
  return fp32 ? k_bt_step<true, false, false, false, 4> : k_bt_step<false, false, false, false, 4>;
}

constexpr int64_t kBasketMin = 8192;  // the basket form needs at least this many tracks

unsigned stream_grid(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 2048));
}

int basket_transport(gv_geom* g, int64_t n, const double* x, const double* y, const double* z, const double* dx,
                     const double* dy, const double* dz, const int32_t* start_pv, int max_steps, int32_t* out_pv,
                     double* out_step, int32_t* out_nsteps, uint32_t* out_flags, bool fp32, bool phys,
                     PhysArgs P, int8_t* out_proc, hipStream_t s) {
  const char* fn = "nav_transport";
  // Under stream capture nothing may be allocated or waited for: the
  // workspace (and the output staging, when it fits) must already exist from
  // an earlier call of at least this size.
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess) cap = hipStreamCaptureStatusNone;
  const bool capturing = cap == hipStreamCaptureStatusActive;
  if (capturing) {
    if (!g->ws || g->ws_tracks < n)
      return fail(GV_ESTATE, "%s: stream is capturing and the workspace holds %lld < %lld tracks; call once "
                  "outside the capture first", fn, (long long)g->ws_tracks, (long long)n);
    if (g->prof) return fail(GV_ESTATE, "%s: profiling events cannot be recorded under stream capture", fn);
  } else {
    GV_TRY(ensure_workspace(g, n));
  }
  const int cb = cell_bits(g);
  const int nl = g->n_lv << cb;  // buckets: (LV, coarse direction cell)
  const unsigned sg = stream_grid(n);
  const size_t lds_ix = 12 * (size_t)nl + 4, lds_step = 4 * (size_t)nl + 12 * (size_t)g->n_lv + 8;
  const unsigned rg = scatter_grid(g, n);
  TCtl& C = g->ctl;
  hipLaunchKernelGGL(k_bt_clear, dim3(1), dim3(kBlock), 0, s, C, nl);
  GV_TRY(launched(fn));
  hipLaunchKernelGGL(g->has_bool ? k_bt_init<true> : k_bt_init<false>, dim3(sg), dim3(kBlock), 4 * (size_t)nl, s, g->dg, n, x, y, z, dx, dy, dz, start_pv,
                     max_steps, out_pv, out_nsteps, out_flags, g->nxt_lv, cb, C);
  GV_TRY(launched(fn));
  // live track ids in bucket order (into idx[1]), then slots in that order
  hipLaunchKernelGGL(k_bt_reindex, dim3(rg), dim3(1024), lds_ix, s, (const int*)nullptr, (const int*)nullptr, 0, n,
                     (const int*)g->nxt_lv, 0, g->idx[1], (const int*)C.cnt[0], C.cur[0], C.cnt[1], C.cur[1], nl);
  GV_TRY(launched(fn));
  hipLaunchKernelGGL(k_bt_place, dim3(sg), dim3(kBlock), 0, s, (const int*)g->idx[1], x, y, z, dx, dy, dz,
                     (const int32_t*)out_pv, max_steps, cb, nl, g->rec, g->slot_id, g->idx[0], C);
  GV_TRY(launched(fn));
  const bool staged = capturing ? staging_ready(g, max_steps) : ensure_staging(g, max_steps);
  double* ob_step = staged ? g->ob_step : nullptr;
  int* ob_pv = staged ? g->ob_pv : nullptr;
  int8_t* ob_proc = staged && phys && out_proc ? g->ob_proc : nullptr;
  const auto step_kernel = select_step_kernel(g, fp32, phys);
  const unsigned step_grid = step_grid_for(g, n);
  const size_t lds_sc = 8 * (size_t)nl + 4;
  // Every step up to max_steps is enqueued at once and the call returns: a
  // step kernel whose list is empty leaves at once, and so does the regrouping
  // kernel after it (which then passes the empty length on), so the launches
  // past the longest track cost only their dispatch.  The host never waits.
  for (int k = 0; k < max_steps; ++k) {
    const int c = k & 1, k0 = k % 3, k1 = (k + 1) % 3, k2 = (k + 2) % 3;
    const int* len_cur = k == 0 ? C.nlive : C.len + (k & 1);
    hipEvent_t* pe = nullptr;
    if (g->prof) {
      if (g->prof_used + 2 > g->prof_ev.size()) {
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
          return fail(GV_EHIP, "nav_transport: hipEventCreate for profiling");
        g->prof_ev.push_back(e0);
        g->prof_ev.push_back(e1);
      }
      pe = &g->prof_ev[g->prof_used];
      g->prof_used += 2;
      (void)hipEventRecord(pe[0], s);
    }
    hipLaunchKernelGGL(step_kernel, dim3(step_grid), dim3(kBlock), lds_step, s, g->dg, k, max_steps, cb,
                       (const int*)g->idx[c], len_cur, g->rec, (const int*)C.cnt[k0], g->nxt_lv, g->nxt_pos,
                       C.cnt[k1], C, out_pv, out_step, out_nsteps, out_flags, (const int*)g->slot_id, ob_step, ob_pv,
                       g->ob_cap, P, ob_proc, out_proc);
    GV_TRY(launched(fn));
    if (pe) (void)hipEventRecord(pe[1], s);
    if (k + 1 == max_steps) break;
    hipLaunchKernelGGL(k_bt_scatter, dim3(rg), dim3(1024), lds_sc, s, (const int*)g->idx[c], len_cur,
                       (const int*)g->nxt_lv, (const uint32_t*)g->nxt_pos, (const int*)C.seg, (const int*)C.cnt[k1],
                       g->idx[c ^ 1], C.len + ((k + 1) & 1), C.cnt[k2], nl);
    GV_TRY(launched(fn));
  }
  if (staged) {
    hipLaunchKernelGGL(ob_proc ? k_bt_emit<true> : k_bt_emit<false>, dim3((unsigned)((n + 63) / 64)), dim3(512), 0,
                       s, (const double*)ob_step,
                       (const int*)ob_pv, (const int8_t*)ob_proc, g->ob_cap, (const int*)g->slot_id, C, max_steps,
                       max_steps, (const int32_t*)out_nsteps, out_step, out_pv, out_proc);
    GV_TRY(launched(fn));
  }
  return GV_OK;
}

// ------------------------------------------------------- lane transport
constexpr int kLaneSortBits = 7;  // default direction cells of the order: 128 x 128

// Direction-key bits of the coherent order: the tuned sort_bits, else the
// default; 0 runs the tracks in index order.
int sort_bits(const gv_geom* g) { return g->tune.sort_bits >= 0 ? g->tune.sort_bits : kLaneSortBits; }

size_t lane_ws_bytes(int64_t cap) {
  return 2 * al256(4 * (size_t)cap) + al256(4 * (size_t)kSortMaxCells) + al256(4);
}

LaneCtl carve_lane_ctl(void* mem, int64_t cap) {
  char* p = (char*)mem;
  LaneCtl L;
  L.key = (uint32_t*)p;
  p += al256(4 * (size_t)cap);
  L.perm = (int32_t*)p;
  p += al256(4 * (size_t)cap);
  L.cnt = (uint32_t*)p;
  p += al256(4 * (size_t)kSortMaxCells);
  L.queue = (uint32_t*)p;
  return L;
}

// Keys, order and counters for `n` tracks, allocated with hipMalloc on first
// use and grown on demand (no clearing needed: every transport clears the
// counters with a kernel and writes the keys and the order before reading).
int ensure_lane_workspace(gv_geom* g, int64_t n) {
  if (g->lws && g->lws_cap >= n) return GV_OK;
  const int64_t cap = std::max<int64_t>(n, std::max<int64_t>(4096, g->lws_cap));
  if (g->lws) {
    (void)hipDeviceSynchronize();
    (void)hipFree(g->lws);
    g->lws = nullptr;
    g->lws_cap = 0;
  }
  void* mem = nullptr;
  hipError_t e = hipMalloc(&mem, lane_ws_bytes(cap));
  if (e != hipSuccess)
    return fail(GV_ENOMEM, "nav_transport: workspace hipMalloc(%zu): %s", lane_ws_bytes(cap), hipGetErrorString(e));
  g->lctl = carve_lane_ctl(mem, cap);
  g->lws = mem;
  g->lws_cap = cap;
  return GV_OK;
}

using LaneKernel = void (*)(DevGeom, int64_t, const double*, const double*, const double*, const double*,
                            const double*, const double*, const int32_t*, const int32_t*, uint32_t*, int, int32_t*,
                            double*, int32_t*, uint32_t*, PhysArgs, int8_t*);

// The lane-transport instance: composites or not, FP32 screens or not,
// physics-limited or not, and the register budget (3 or 4 waves per SIMD)
// and output staging.  Geometries with composites run one shape per
// precision and physics.
template <bool F32, bool PHYS>
LaneKernel lane_kernel_for(int waves, bool stage, bool cls) {
  if (cls) return waves == 3 ? k_lane_transport<F32, PHYS, false, 3, 8, true> : k_lane_transport<F32, PHYS, false, 4, 8, true>;
  if (waves == 3) return stage ? k_lane_transport<F32, PHYS, false, 3, 8> : k_lane_transport<F32, PHYS, false, 3, 0>;
  return stage ? k_lane_transport<F32, PHYS, false, 4, 8> : k_lane_transport<F32, PHYS, false, 4, 0>;
}

LaneKernel select_lane_kernel(bool has_bool, bool fp32, bool phys, int waves, bool stage, bool cls) {
  if (has_bool)
    return fp32 ? (phys ? k_lane_transport<true, true, true, 3, 0> : k_lane_transport<true, false, true, 3, 0>)
                : (phys ? k_lane_transport<false, true, true, 3, 0> : k_lane_transport<false, false, true, 3, 0>);
  if (phys) return fp32 ? lane_kernel_for<true, true>(waves, stage, cls) : lane_kernel_for<false, true>(waves, stage, cls);
  return fp32 ? lane_kernel_for<true, false>(waves, stage, cls) : lane_kernel_for<false, false>(waves, stage, cls);
}

// Workgroups of 256 threads a CU holds at once for kernel k (cached per
// kernel in a fixed table: nothing is allocated here).
int resident_blocks(gv_geom* g, const void* k) {
  for (int i = 0; i < g->n_occ; ++i)
    if (g->occ[i].first == k) return g->occ[i].second;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 256, 0) != hipSuccess || nb < 1) {
    (void)hipGetLastError();
    nb = 1;
  }
  if (g->n_occ < (int)(sizeof g->occ / sizeof g->occ[0])) g->occ[g->n_occ++] = {k, nb};
  return nb;
}

// Enqueues a lane transport: order the tracks by direction key (unless sort
// bits are 0), then one persistent launch that carries every track to its end.
// L holds the keys, order and counters for at least n tracks.
int lane_transport(gv_geom* g, const LaneCtl& L, int64_t n, const double* x, const double* y, const double* z,
                   const double* dx, const double* dy, const double* dz, const int32_t* start_pv, int max_steps,
                   int32_t* out_pv, double* out_step, int32_t* out_nsteps, uint32_t* out_flags, bool fp32,
                   bool phys, PhysArgs P, int8_t* out_proc, hipStream_t s, const char* fn, bool events) {
  const int h = std::min(sort_bits(g), kSortMaxBits);
  const bool sorted = h > 0;
  const int cells = sorted ? 1 << (2 * h) : 0;
  hipLaunchKernelGGL(k_ls_clear, dim3((unsigned)std::max(1, (cells + 255) / 256)), dim3(256), 0, s, L, cells);
  GV_TRY(launched(fn));
  if (sorted) {
    const unsigned cg = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 4095) / 4096, 256));
    hipLaunchKernelGGL(k_ls_count, dim3(cg), dim3(1024), 4 * (size_t)cells, s, n, dx, dy, dz, h,
                       g->tune.sort_key == 2 ? 1 : 0, L);
    GV_TRY(launched(fn));
    hipLaunchKernelGGL(k_ls_scan, dim3(1), dim3(1024), 0, s, L, cells);
    GV_TRY(launched(fn));
    // the scatter's chunks: at most 64 workgroups, so that a key's run is
    // reserved by at most 64 global atomics
    const int64_t chunk = std::max<int64_t>(4096, (n + 63) / 64);
    hipLaunchKernelGGL(k_ls_scatter, dim3((unsigned)((n + chunk - 1) / chunk)), dim3(1024), 4 * (size_t)cells, s, n,
                       chunk, cells, L);
    GV_TRY(launched(fn));
  }
  // defaults: staged outputs; 4 waves per SIMD for navigation, 3 for
  // physics-limited steps (more live state per lane: 9.6 ms at 3 against
  // 11.5 ms at 4 on the detector workload)
  const int waves = g->tune.lane_waves ? g->tune.lane_waves : (phys ? 3 : 4);
  const bool stage = g->tune.lane_stage ? g->tune.lane_stage == 2 : true;
  // per-class scheduling by default (2.66 against 2.99 ms for navigation,
  // 7.6 against 9.5 ms physics-limited, on the detector workload)
  const LaneKernel k = select_lane_kernel(g->has_bool, fp32, phys, waves, stage, g->tune.lane_sched != 1);
  int64_t grid = g->tune.lane_grid > 0 ? g->tune.lane_grid
                                       : (int64_t)resident_blocks(g, reinterpret_cast<const void*>(k)) * g->n_cu;
  grid = std::max<int64_t>(1, std::min<int64_t>(grid, (n + 255) / 256));
  hipEvent_t* pe = nullptr;
  if (events) {
    if (g->prof_used + 2 > g->prof_ev.size()) {
      hipEvent_t e0, e1;
      if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(GV_EHIP, "%s: hipEventCreate for profiling", fn);
      g->prof_ev.push_back(e0);
      g->prof_ev.push_back(e1);
    }
    pe = &g->prof_ev[g->prof_used];
    g->prof_used += 2;
    (void)hipEventRecord(pe[0], s);
  }
  hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(256), 0, s, g->dg, n, x, y, z, dx, dy, dz, start_pv,
                     sorted ? (const int32_t*)L.perm : (const int32_t*)nullptr, L.queue, max_steps, out_pv, out_step,
                     out_nsteps, out_flags, P, out_proc);
  GV_TRY(launched(fn));
  if (pe) (void)hipEventRecord(pe[1], s);
  return GV_OK;
}

}  // namespace

namespace {

// Argument checks shared by the transports (n == 0 passes; the caller
// returns before enqueuing anything).
int transport_args(const char* fn, gv_geom* g, int64_t n, const double* x, const double* y, const double* z,
                   const double* dx, const double* dy, const double* dz, const int32_t* start_pv, int32_t max_steps,
                   int32_t* out_pv, double* out_step, int32_t* out_nsteps, uint32_t* out_flags, int32_t precision,
                   bool phys) {
  GV_TRY(check_common(fn, g, n));
  GV_TRY(check_nav_precision(fn, precision));
  if (max_steps < 1 || max_steps > 4096) return fail(GV_EINVAL, "%s: max_steps %d not in [1, 4096]", fn, max_steps);
  if (phys && g->dg.n_mat < 1) return fail(GV_ESTATE, "%s: no materials (geom_set_materials first)", fn);
  if (n == 0) return GV_OK;
  if (n > (1L << 30)) return fail(GV_EINVAL, "%s: n %lld > 2^30", fn, (long long)n);
  const double* in[6] = {x, y, z, dx, dy, dz};
  const char* nm[6] = {"x", "y", "z", "dx", "dy", "dz"};
  for (int i = 0; i < 6; ++i) GV_TRY(check_f64(fn, nm[i], in[i]));
  GV_TRY(check_i32(fn, "start_pv", start_pv, true));
  GV_TRY(check_i32(fn, "out_pv", out_pv));
  GV_TRY(check_f64(fn, "out_step", out_step));
  GV_TRY(check_i32(fn, "out_nsteps", out_nsteps));
  GV_TRY(check_i32(fn, "out_flags", out_flags));
  return GV_OK;
}

int transport_common(const char* fn, gv_geom* g, int64_t n, const double* x, const double* y, const double* z,
                     const double* dx, const double* dy, const double* dz, const int32_t* start_pv,
                     int32_t max_steps, int32_t* out_pv, double* out_step, int32_t* out_nsteps,
                     uint32_t* out_flags, int32_t precision, bool phys, PhysArgs P, int8_t* out_proc,
                     void* stream) {
  GV_TRY(transport_args(fn, g, n, x, y, z, dx, dy, dz, start_pv, max_steps, out_pv, out_step, out_nsteps, out_flags,
                        precision, phys));
  if (n == 0) return GV_OK;
  DeviceGuard dgd(g->device);
  const bool fp32 = precision == GV_FP32_REFINE;
  const hipStream_t s = (hipStream_t)stream;
  // the basket form when it is asked for (or its work counters are), and by
  // default for geometries holding composites (their tracks start in several
  // volumes, which a direction order mixes in every wavefront: 2.9 ms against
  // 3.7 ms for the lane form on the composite workload); else the lane form
  const bool basket = g->tune.transport == 1 || g->prof_work || (g->tune.transport == 0 && g->has_bool);
  if (basket && n >= kBasketMin && g->n_lv <= 4096)
    return basket_transport(g, n, x, y, z, dx, dy, dz, start_pv, max_steps, out_pv, out_step, out_nsteps, out_flags,
                            fp32, phys, P, out_proc, s);
  // Under stream capture nothing may be allocated: the workspace must already
  // hold n tracks from an earlier call.
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess) cap = hipStreamCaptureStatusNone;
  if (cap == hipStreamCaptureStatusActive) {
    if (!g->lws || g->lws_cap < n)
      return fail(GV_ESTATE, "%s: stream is capturing and the workspace holds %lld < %lld tracks; call once "
                  "outside the capture first", fn, (long long)g->lws_cap, (long long)n);
    if (g->prof) return fail(GV_ESTATE, "%s: profiling events cannot be recorded under stream capture", fn);
  } else {
    GV_TRY(ensure_lane_workspace(g, n));
  }
  return lane_transport(g, g->lctl, n, x, y, z, dx, dy, dz, start_pv, max_steps, out_pv, out_step, out_nsteps,
                        out_flags, fp32, phys, P, out_proc, s, fn, g->prof);
}

}  // namespace

extern "C" int nav_transport(gv_geom* g, int64_t n, const double* x, const double* y, const double* z,
                             const double* dx, const double* dy, const double* dz, const int32_t* start_pv,
                             int32_t max_steps, int32_t* out_pv, double* out_step, int32_t* out_nsteps,
                             uint32_t* out_flags, int32_t precision, void* stream) {
  return transport_common("nav_transport", g, n, x, y, z, dx, dy, dz, start_pv, max_steps, out_pv, out_step,
                          out_nsteps, out_flags, precision, false, PhysArgs{0, 0}, nullptr, stream);
}

extern "C" int nav_transport_phys(gv_geom* g, int64_t n, const double* x, const double* y, const double* z,
                                  const double* dx, const double* dy, const double* dz, const int32_t* start_pv,
                                  int32_t max_steps, uint64_t seed, int32_t* out_pv, double* out_step,
                                  int8_t* out_proc, int32_t* out_nsteps, uint32_t* out_flags, int32_t options,
                                  int32_t precision, void* stream) {
  if (options & ~GV_PHYS_SAFETY_SHORTCUT) return fail(GV_EINVAL, "nav_transport_phys: options %d", options);
  return transport_common("nav_transport_phys", g, n, x, y, z, dx, dy, dz, start_pv, max_steps, out_pv, out_step,
                          out_nsteps, out_flags, precision, true,
                          PhysArgs{seed, (options & GV_PHYS_SAFETY_SHORTCUT) ? 1 : 0}, out_proc, stream);
}

extern "C" int nav_transport_noalloc(gv_geom* g, int64_t n, const double* x, const double* y, const double* z,
                                     const double* dx, const double* dy, const double* dz, const int32_t* start_pv,
                                     int32_t max_steps, int32_t* out_pv, double* out_step, int32_t* out_nsteps,
                                     uint32_t* out_flags, int32_t precision, void* stream) {
  const char* fn = "nav_transport_noalloc";
  GV_TRY(transport_args(fn, g, n, x, y, z, dx, dy, dz, start_pv, max_steps, out_pv, out_step, out_nsteps, out_flags,
                        precision, false));
  if (n > kNoAllocMaxTracks)
    return fail(GV_EINVAL, "%s: n %lld exceeds the scratch's %lld tracks", fn, (long long)n,
                (long long)kNoAllocMaxTracks);
  if (n == 0) return GV_OK;
  void* p = noalloc_scratch(g->device);
  if (!p) return fail(GV_ESTATE, "%s: no scratch address for device %d", fn, g->device);
  DeviceGuard dgd(g->device);
  static_assert(2 * 4 * (size_t)kNoAllocMaxTracks + 4 * (size_t)kSortMaxCells + 4 <= kScratchBytes,
                "scratch holds the lane form's arrays");
  const LaneCtl L = carve_lane_ctl(p, kNoAllocMaxTracks);
  return lane_transport(g, L, n, x, y, z, dx, dy, dz, start_pv, max_steps, out_pv, out_step, out_nsteps, out_flags,
                        precision == GV_FP32_REFINE, false, PhysArgs{0, 0}, nullptr, (hipStream_t)stream, fn, false);
}

extern "C" int geom_set_materials(gv_geom* g, int32_t n_mat, int32_t n_proc, const double* density,
                                  const double* sigma, const int32_t* lv_material) {
  const char* fn = "geom_set_materials";
  if (!g) return fail(GV_EINVAL, "%s: geometry handle is NULL", fn);
  if (n_mat < 1 || n_mat > 65536) return fail(GV_EINVAL, "%s: n_mat %d not in [1, 65536]", fn, n_mat);
  if (n_proc < 1 || n_proc > kMaxProc) return fail(GV_EINVAL, "%s: n_proc %d not in [1, %d]", fn, n_proc, kMaxProc);
  if (!density || !sigma || !lv_material) return fail(GV_EINVAL, "%s: NULL table", fn);
  std::vector<double> rate((size_t)n_mat * n_proc);
  for (int m = 0; m < n_mat; ++m) {
    if (!(density[m] >= 0.0) || !std::isfinite(density[m])) return fail(GV_EINVAL, "%s: density[%d]", fn, m);
    for (int i = 0; i < n_proc; ++i) {
      const double sg = sigma[(size_t)m * n_proc + i];
      if (!(sg >= 0.0) || !std::isfinite(sg)) return fail(GV_EINVAL, "%s: sigma[%d][%d]", fn, m, i);
      rate[(size_t)m * n_proc + i] = density[m] * sg;  // n sigma = 1 / lambda (1/mm)
    }
  }
  for (int l = 0; l < g->n_lv; ++l)
    if (lv_material[l] < 0 || lv_material[l] >= n_mat) return fail(GV_EINVAL, "%s: lv_material[%d]", fn, l);
  DeviceGuard dgd(g->device);
  const size_t br = al256(rate.size() * 8), total = br + 4 * (size_t)g->n_lv;
  void* mem = nullptr;
  hipError_t e = hipMalloc(&mem, total);
  if (e != hipSuccess) return fail(GV_ENOMEM, "%s: hipMalloc(%zu): %s", fn, total, hipGetErrorString(e));
  e = hipMemcpy(mem, rate.data(), rate.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy((char*)mem + br, lv_material, 4 * (size_t)g->n_lv, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(mem);
    return hip_fail(e, "geom_set_materials: hipMemcpy");
  }
  if (g->mat_mem) {
    (void)hipDeviceSynchronize();
    (void)hipFree(g->mat_mem);
  }
  g->mat_mem = mem;
  g->dg.n_mat = n_mat;
  g->dg.n_proc = n_proc;
  g->dg.mat_rate = (CQ)mem;
  g->dg.lv_mat = (CQI)((char*)mem + br);
  t_err.clear();
  return GV_OK;
}

// ------------------------------------------------------------ measurement
extern "C" int gv_profile(gv_geom* g, int flags) {
  if (!g) return fail(GV_EINVAL, "gv_profile: geometry handle is NULL");
  if (flags & ~(GV_PROF_EVENTS | GV_PROF_WORK)) return fail(GV_EINVAL, "gv_profile: flags %d", flags);
  g->prof = (flags & GV_PROF_EVENTS) != 0;
  g->prof_work = (flags & GV_PROF_WORK) != 0;
  return GV_OK;
}

// ------------------------------------------------------------- roof probes
extern "C" int gv_probe_stream(const double* a, const double* b, double* c, double s, int64_t n, void* stream) {
  const char* fn = "gv_probe_stream";
  if (n < 0 || (n & 1)) return fail(GV_EINVAL, "%s: n %lld must be even and >= 0", fn, (long long)n);
  if (n == 0) return GV_OK;
  if (!a || !c) return fail(GV_EINVAL, "%s: a or c is NULL", fn);
  if (((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) & 15) return fail(GV_EINVAL, "%s: arrays not 16-byte aligned", fn);
  const int64_t n2 = n / 2;
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n2 + 255) / 256, 256 * 32));
  hipLaunchKernelGGL(k_probe_triad, dim3(grid), dim3(256), 0, (hipStream_t)stream, (const double2*)a,
                     (const double2*)b, (double2*)c, s, n2);
  return launched(fn);
}

extern "C" int gv_probe_fma64(double* out, int64_t n_lanes, int32_t iters, void* stream) {
  const char* fn = "gv_probe_fma64";
  if (n_lanes <= 0 || n_lanes % 256) return fail(GV_EINVAL, "%s: n_lanes must be a positive multiple of 256", fn);
  if (iters < 1) return fail(GV_EINVAL, "%s: iters < 1", fn);
  if (!out || ((uintptr_t)out & 7)) return fail(GV_EINVAL, "%s: out NULL or misaligned", fn);
  hipLaunchKernelGGL(k_probe_fma64, dim3((unsigned)(n_lanes / 256)), dim3(256), 0, (hipStream_t)stream, out, iters,
                     0.999999, 1e-6);
  return launched(fn);
}

// ------------------------------------------------------------ launch shapes
extern "C" int gv_set_tuning(gv_geom* g, const gv_tuning* t) {
  const char* fn = "gv_set_tuning";
  if (!g || !t) return fail(GV_EINVAL, "%s: NULL argument", fn);
  if (t->step_grid < 0 || t->step_grid > kMaxStepGrid)
    return fail(GV_EINVAL, "%s: step_grid %d not in [0, %d]", fn, t->step_grid, kMaxStepGrid);
  if (t->scatter_grid < 0 || t->scatter_grid > 1024)
    return fail(GV_EINVAL, "%s: scatter_grid %d not in [0, 1024]", fn, t->scatter_grid);
  if (!(t->cell_bits == -1 || t->cell_bits == 0 || t->cell_bits == 2 || t->cell_bits == 4))
    return fail(GV_EINVAL, "%s: cell_bits %d not -1, 0, 2 or 4", fn, t->cell_bits);
  if (t->solid_block != 0 && (t->solid_block < 64 || t->solid_block > 1024 || t->solid_block % 64))
    return fail(GV_EINVAL, "%s: solid_block %d not 0 or a multiple of 64 in [64, 1024]", fn, t->solid_block);
  if (t->solid_grid < 0) return fail(GV_EINVAL, "%s: solid_grid %d < 0", fn, t->solid_grid);
  if (!(t->step_waves == 0 || t->step_waves == 3 || t->step_waves == 4))
    return fail(GV_EINVAL, "%s: step_waves %d not 0, 3 or 4", fn, t->step_waves);
  if (t->transport < 0 || t->transport > 2) return fail(GV_EINVAL, "%s: transport %d not 0, 1 or 2", fn, t->transport);
  if (t->sort_bits < -1 || t->sort_bits > kSortMaxBits)
    return fail(GV_EINVAL, "%s: sort_bits %d not in [-1, %d]", fn, t->sort_bits, kSortMaxBits);
  if (t->sort_key < 0 || t->sort_key > 2) return fail(GV_EINVAL, "%s: sort_key %d not 0, 1 or 2", fn, t->sort_key);
  if (!(t->lane_waves == 0 || t->lane_waves == 3 || t->lane_waves == 4))
    return fail(GV_EINVAL, "%s: lane_waves %d not 0, 3 or 4", fn, t->lane_waves);
  if (t->lane_stage < 0 || t->lane_stage > 2)
    return fail(GV_EINVAL, "%s: lane_stage %d not 0, 1 or 2", fn, t->lane_stage);
  if (t->lane_grid < 0) return fail(GV_EINVAL, "%s: lane_grid %d < 0", fn, t->lane_grid);
  if (t->lane_sched < 0 || t->lane_sched > 2)
    return fail(GV_EINVAL, "%s: lane_sched %d not 0, 1 or 2", fn, t->lane_sched);
  g->tune = *t;
  t_err.clear();
  return GV_OK;
}

extern "C" int gv_get_tuning(const gv_geom* g, gv_tuning* t) {
  if (!g || !t) return fail(GV_EINVAL, "gv_get_tuning: NULL argument");
  *t = g->tune;
  return GV_OK;
}

extern "C" int gv_profile_read(gv_geom* g, double* step_ms, int64_t* step_launches, uint64_t* work) {
  static_assert(kWorkN == 28, "gvgeom.h documents 28 transport work counters, then 5 polycone ones");
  if (!g) return fail(GV_EINVAL, "gv_profile_read: geometry handle is NULL");
  DeviceGuard dgd(g->device);
  double ms = 0.0;
  for (size_t i = 0; i + 1 < g->prof_used; i += 2) {
    hipError_t e = hipEventSynchronize(g->prof_ev[i + 1]);
    if (e != hipSuccess) return hip_fail(e, "gv_profile_read: hipEventSynchronize");
    float t = 0.0f;
    e = hipEventElapsedTime(&t, g->prof_ev[i], g->prof_ev[i + 1]);
    if (e != hipSuccess) return hip_fail(e, "gv_profile_read: hipEventElapsedTime");
    ms += t;
  }
  if (step_ms) *step_ms = ms;
  if (step_launches) *step_launches = (int64_t)(g->prof_used / 2);
  g->prof_used = 0;
  if (work) {
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess && g->ws) e = hipMemcpy(work, g->ctl.work, 8 * kWorkN, hipMemcpyDeviceToHost);
    if (!g->ws)
      for (int i = 0; i < kWorkN; ++i) work[i] = 0;
    if (e == hipSuccess) e = hipMemcpy(work + kWorkN, g->pcon_work, 8 * 5, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemset(g->pcon_work, 0, 8 * 5);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "gv_profile_read: counters");
  }
  return GV_OK;
}

// ------------------------------------------------------------------ serving
#include "gv_serve.h"
