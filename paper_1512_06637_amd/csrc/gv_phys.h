// Physics-limited steps.  Each process i of the current volume's material has
// the mean free path lambda_i = 1 / (n sigma_i) (Sec. III, Eq. (1)); every step,
// each process draws an interaction length by Monte Carlo and the shortest is
// proposed as the physics step (the rates add up, Eqs. (2)-(3)); the navigator
// then takes the border instead when it is nearer (Sec. III.A).
//
// A length is s_i = -ln(u) / (n sigma_i), u in (0, 1) from the counter-based
// generator Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with counter
// (track, step, process, 0) and key (seed low, seed high): any track's draws
// are reproducible whatever the order in which tracks are processed.
#pragma once
#include "gv_geom.h"

namespace gv {

constexpr int kMaxProc = 16;  // processes per material

// Philox4x32 with 10 rounds.  A round multiplies words 0 and 2 by the two
// Philox multipliers, and the new words are the high product halves mixed with
// the other words and the round key, and the low product halves; the key
// advances by the two Weyl constants before each round after the first.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u, kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint32_t lo0 = kM0 * c[0], hi0 = __umulhi(kM0, c[0]);
    const uint32_t lo1 = kM1 * c[2], hi1 = __umulhi(kM1, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// u in (0, 1): the first two output words as a 64-bit integer, its top 53
// bits, centred in their 2^-53 interval.
__device__ __forceinline__ double draw_uniform(uint64_t seed, uint32_t track, uint32_t step, uint32_t proc) {
  uint32_t c[4] = {track, step, proc, 0u};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t v = ((uint64_t)c[0] << 32) | c[1];
  return ((double)(v >> 11) + 0.5) * 0x1p-53;
}

// Shortest sampled interaction length of the processes of material `mat`
// (rate[mat][i] = n sigma_i precomputed), *proc its process (lowest index on
// equal lengths); +inf and -1 when no process acts.
__device__ __forceinline__ double physics_length(CQ rate, int n_proc, int mat, uint64_t seed, uint32_t track,
                                                 uint32_t step, int* proc) {
  double best = GV_INF;
  int bp = -1;
  for (int i = 0; i < n_proc; ++i) {
    const double r = rate[mat * n_proc + i];
    if (!(r > 0.0)) continue;
    const double s = -log(draw_uniform(seed, track, step, (uint32_t)i)) / r;
    if (s < best) {
      best = s;
      bp = i;
    }
  }
  *proc = bp;
  return best;
}

}  // namespace gv
