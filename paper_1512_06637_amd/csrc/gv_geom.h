// Device-resident geometry tables and per-track navigation (Sec. III.A step
// selection over the Sec. III.B volume hierarchy).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gv_solids.h"

namespace gv {

// All arrays live in HBM; geom_load fills them once.  Transforms are 12
// doubles: R row-major then t, with x_mother = R x_child + t.
constexpr int kPhiSectors = 256;

struct DevGeom {
  int n_lv, n_pv, n_place;
  CQI lv_type;       // [n_lv]
  CQI lv_par;        // [n_lv] offset into par
  CQI lv_dau_off;    // [n_lv] first daughter placement
  CQI lv_dau_cnt;    // [n_lv]
  CQI lv_dau_type;   // [n_lv] solid type shared by all daughters, -1 if mixed or none
  CQ par;            // derived solid parameters
  CQ dau_xf;         // [n_place][12] placement transform, LV frame
  CQI dau_lv;        // [n_place]
  CQI dau_par;       // [n_place] offset of the child solid's parameters in par
  CQ dau_box;        // [n_place][6] child's bounding box in the mother frame (lo xyz, hi xyz), padded
  CQI pv_lv;         // [n_pv]
  CQI pv_parent;     // [n_pv]
  CQ pv_gxf;         // [n_pv][12] composed world <- PV transform
  CQI pv_child_off;  // [n_pv] children of a PV follow their LV's placement order
  CQI pv_child;      // [n_pv]
  // FP32 screen tables (daughter culling in FP32 with FP64 refinement)
  CQF lv_scr;        // [n_lv] S: max |coordinate| of a point of the LV's solid + 1 mm
  CQF dau_box32;     // [n_place][8] dau_box widened by 128 u (S(mother) + |box|inf), rounded outward; 2 unused
  CQF dau_scr32;     // [n_place][16] R (9), t (3), child a b c (box: dx dy dz; tube: rmin rmax dz), e
  // daughter groups: 8 consecutive daughters of an LV with >= 16 daughters
  CQI dau_ident;     // [n_place] 1 when the placement is the identity (R = I, t = 0)
  CQI lv_grp;        // [n_lv] index of the LV's first group box, -1 without groups
  CQ grp_box;        // [n_grp][6] union of the group's padded daughter boxes (lo xyz, hi xyz)
  CQF grp_box32;     // [n_grp][8] union of the group's FP32 boxes; 2 unused
  // radial order: an LV whose daughters are identity-placed full tubes with
  // disjoint radial ranges lists them by radius
  CQI lv_rad;        // [n_lv] first entry of the LV's radial list, -1 without one
  CQ rad_r2;         // [n_rad][2] rmin^2, rmax^2 in radial order
  CQI rad_k;         // [n_rad] daughter index (placement order) of each entry
  // phi sectors: an LV whose (<= 64) daughters lie around the z axis, each
  // within less than a half turn, has kPhiSectors masks of the daughters
  // whose angular extent (widened) meets each sector of pseudo-angle
  CQI lv_phi;        // [n_lv] first mask of the LV, -1 without sectors
  CQL phi_mask;      // [n_phi_lv][kPhiSectors]
  // materials for physics-limited steps (geom_set_materials); n_mat 0 if unset
  int n_mat, n_proc;
  CQ mat_rate;       // [n_mat][n_proc] n sigma = 1 / mean free path, 1/mm
  CQI lv_mat;        // [n_lv] material of each LV
  CQI lv_class;      // [n_lv] step class: branch of the step code (daughter access mode x 8 + solid type)
  CQI pv_k;          // [n_pv] placement index of each PV among its parent's daughters (-1: the world)
  CQI pv_lc;         // [2 n_pv] logical volume and step class of each PV (one 8-byte load)
};

__device__ __forceinline__ V3 ld3(const double* x, const double* y, const double* z, int64_t i) {
  return V3{x[i], y[i], z[i]};
}

// x_child = R^T (x_mother - t)
__device__ __forceinline__ V3 to_child_p(CQ X, V3 p) {
  double q0 = p.x - X[9], q1 = p.y - X[10], q2 = p.z - X[11];
  return V3{X[0] * q0 + X[3] * q1 + X[6] * q2, X[1] * q0 + X[4] * q1 + X[7] * q2,
            X[2] * q0 + X[5] * q1 + X[8] * q2};
}
__device__ __forceinline__ V3 to_child_d(CQ X, V3 d) {
  return V3{X[0] * d.x + X[3] * d.y + X[6] * d.z, X[1] * d.x + X[4] * d.y + X[7] * d.z,
            X[2] * d.x + X[5] * d.y + X[8] * d.z};
}

constexpr uint32_t kFlagOverflow = 1u, kFlagStuck = 2u, kFlagLocateFail = 4u;

template <bool B>
__device__ __forceinline__ int locate(const DevGeom& G, V3 p) {
  int lv0 = G.pv_lv[0];
  if (code_of(solid_sgn<B>(G.lv_type[lv0], G.par + G.lv_par[lv0], p)) == kOutside) return -1;
  int pv = 0;
  V3 pl = p;
  for (;;) {
    int lv = G.pv_lv[pv];
    int off = G.lv_dau_off[lv], cnt = G.lv_dau_cnt[lv];
    int found = -1;
    V3 pc;
    for (int k = 0; k < cnt; ++k) {
      int clv = G.dau_lv[off + k];
      pc = to_child_p(G.dau_xf + 12 * (size_t)(off + k), pl);
      if (code_of(solid_sgn<B>(G.lv_type[clv], G.par + G.lv_par[clv], pc)) != kOutside) {
        found = k;
        break;
      }
    }
    if (found < 0) return pv;
    pv = G.pv_child[G.pv_child_off[pv] + found];
    pl = pc;
  }
}

template <bool B>
__device__ __forceinline__ double nav_safety(const DevGeom& G, int pv, V3 p) {
  int lv = G.pv_lv[pv];
  V3 pl = to_child_p(G.pv_gxf + 12 * (size_t)pv, p);
  int t = G.lv_type[lv];
  CQ q = G.par + G.lv_par[lv];
  if (code_of(solid_sgn<B>(t, q, pl)) != kInside) return 0.0;
  double s = solid_safety_out<B>(t, q, pl);
  int off = G.lv_dau_off[lv], cnt = G.lv_dau_cnt[lv];
  for (int k = 0; k < cnt; ++k) {
    int clv = G.dau_lv[off + k];
    V3 pc = to_child_p(G.dau_xf + 12 * (size_t)(off + k), pl);
    CQ qc = G.par + G.lv_par[clv];
    int tc = G.lv_type[clv];
    if (code_of(solid_sgn<B>(tc, qc, pc)) != kOutside) return 0.0;
    s = fmin(s, solid_safety_in<B>(tc, qc, pc));
  }
  return fmax(s, 0.0);
}

}  // namespace gv
