/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Physics-limited transport.  The step of a particle is set by the mean free
 * path of each process, lambda_i = 1 / (n sigma_i) with n the number density of
 * the medium and sigma_i the process's cross section (Sec. III, Eq. (1)); the
 * total rate is the sum of the process rates (Eqs. (2), (3)).  Following the
 * Physics subsection, every process draws an interaction length by Monte Carlo,
 * the shortest one is proposed, and when it is longer than the distance to the
 * border the particle is moved to the border instead (and the lengths are drawn
 * again with the material of the next volume).
 *
 * A length is drawn as s_i = -ln(u_i) / (n sigma_i) (the exponential law with
 * mean lambda_i), u_i in (0, 1) from the counter-based generator Philox4x32-10
 * (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 * SC'11), written here from its published definition: counter (track, step,
 * process, 0), key (seed low 32 bits, seed high 32 bits).
 */
#include <math.h>
#include <stdint.h>

#include "oracle.h"

/* one Philox4x32 round: two 32x32->64 products, the halves exchanged and
 * mixed with the other words and the round key */
static void philox_round(uint32_t c[4], const uint32_t k[2]) {
  const uint64_t a = (uint64_t)0xD2511F53u * c[0];
  const uint64_t b = (uint64_t)0xCD9E8D57u * c[2];
  const uint32_t r0 = (uint32_t)(b >> 32) ^ c[1] ^ k[0];
  const uint32_t r1 = (uint32_t)b;
  const uint32_t r2 = (uint32_t)(a >> 32) ^ c[3] ^ k[1];
  const uint32_t r3 = (uint32_t)a;
  c[0] = r0;
  c[1] = r1;
  c[2] = r2;
  c[3] = r3;
}

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { /* the key advances by the Weyl constants before each later round */
      k[0] += 0x9E3779B9u;
      k[1] += 0xBB67AE85u;
    }
    philox_round(c, k);
  }
  for (int i = 0; i < 4; ++i) out[i] = c[i];
}

/* u in (0, 1): the top 53 bits of the first two output words, centred in
 * their 2^-53 interval */
double or_uniform(uint64_t seed, uint32_t track, uint32_t step, uint32_t proc) {
  const uint32_t ctr[4] = {track, step, proc, 0u};
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t o[4];
  or_philox4x32_10(ctr, key, o);
  const uint64_t v = ((uint64_t)o[0] << 32) | o[1];
  return ((double)(v >> 11) + 0.5) * 0x1p-53;
}

/* Shortest of the processes' sampled interaction lengths in material `mat`;
 * *proc receives its process (lowest index on equal lengths), -1 if no process
 * acts (all cross sections zero: +inf). */
double or_phys_length(const or_phys* ph, int mat, uint64_t seed, uint32_t track, uint32_t step, int* proc) {
  double best = INFINITY;
  int bp = -1;
  for (int i = 0; i < ph->n_proc; ++i) {
    const double rate = ph->density[mat] * ph->sigma[mat * ph->n_proc + i]; /* n sigma_i = 1 / lambda_i */
    if (!(rate > 0.0)) continue;
    const double s = -log(or_uniform(seed, track, step, (uint32_t)i)) / rate;
    if (s < best) {
      best = s;
      bp = i;
    }
  }
  *proc = bp;
  return best;
}

int or_transport_phys(const or_geom* g, const or_phys* ph, const double p0[3], const double d[3],
                      int start_pv, int max_steps, uint64_t seed, uint32_t track, int32_t* out_pv,
                      double* out_step, int8_t* out_proc, unsigned* flags, unsigned* diag) {
  double p[3] = {p0[0], p0[1], p0[2]};
  int pv = start_pv;
  out_pv[0] = pv;
  if (pv < 0) return 0;
  int zero_run = 0, k = 0;
  for (k = 0; k < max_steps; ++k) {
    int proc = -1, next = -1;
    const int mat = ph->lv_mat[g->pv_lv[pv]];
    const double pstep = or_phys_length(ph, mat, seed, track, (uint32_t)k, &proc);
    double step = or_compute_step(g, p, d, pv, pstep, &next, flags, diag);
    p[0] = p[0] + step * d[0];
    p[1] = p[1] + step * d[1];
    p[2] = p[2] + step * d[2];
    out_step[k] = step;
    out_pv[k + 1] = next;
    if (out_proc) out_proc[k] = (int8_t)(next == pv ? proc : -1);
    if (next < 0) return k + 1;
    zero_run = (step < OR_KTOL) ? zero_run + 1 : 0;
    if (zero_run >= 8) {
      *flags |= OR_F_STUCK;
      return k + 1;
    }
    pv = next;
  }
  *flags |= OR_F_OVERFLOW;
  return max_steps;
}
