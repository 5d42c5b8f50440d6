/*
 * Sanitizer run of the CPU oracle (test infrastructure): built together with
 * the oracle's sources under AddressSanitizer and UndefinedBehaviorSanitizer,
 * it drives every oracle entry point over seeded inputs and checks a few of
 * the pins on the way (surface landing of finite distances, path length equal
 * to the world's DistanceToOut).  Inputs come from files the test writes:
 *   argv[1]  solids: lines "type nparams p0 p1 ..."
 *   argv[2]  geometry blob (layered detector)
 * Prints "OK" and exits 0 when every check holds.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/oracle.h"

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static double urand(void) { /* splitmix64 -> [0, 1) */
  uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (double)(z >> 11) * 0x1p-53;
}
static void iso(double d[3]) {
  const double c = 2.0 * urand() - 1.0, ph = 2.0 * M_PI * urand(), s = sqrt(1.0 - c * c);
  d[0] = s * cos(ph);
  d[1] = s * sin(ph);
  d[2] = c;
}

static int check_solids(const char* path) {
  FILE* f = fopen(path, "r");
  if (!f) return 1;
  int bad = 0, nsol = 0, type, np;
  while (fscanf(f, "%d %d", &type, &np) == 2) {
    double* q = (double*)calloc((size_t)np, sizeof(double));
    for (int i = 0; i < np; ++i)
      if (fscanf(f, "%lf", &q[i]) != 1) return 1;
    or_solid s;
    if (or_solid_init(&s, type, q, np)) {
      fprintf(stderr, "solid %d rejected\n", type);
      return 1;
    }
    ++nsol;
    for (int i = 0; i < 4000; ++i) {
      double p[3], d[3];
      for (int k = 0; k < 3; ++k) p[k] = 240.0 * urand() - 120.0;
      iso(d);
      (void)or_safety(&s, OR_SAFETY_AUTO, p);
      double R[OR_MAX_ROOTS];
      (void)or_roots(&s, p, d, R);
      for (int dir = 0; dir < 2; ++dir) {
        unsigned dg = 0;
        const double t = dir == 0 ? or_dist_in(&s, p, d, &dg) : or_dist_out(&s, p, d, &dg);
        (void)or_hit_cond(&s, p, d, t);
        if (t > 0.0 && isfinite(t) && !(dg & (OR_D_GRAZE | OR_D_NEAR_TIE | OR_D_BAND_EDGE))) {
          const double q2[3] = {p[0] + t * d[0], p[1] + t * d[1], p[2] + t * d[2]};
          /* surface landing, within the rounding of the landing point */
          if (fabs(or_signed(&s, q2)) > OR_KHALF + 1e-9) ++bad;
        }
      }
    }
    or_solid_release(&s);
    free(q);
  }
  fclose(f);
  if (nsol < 6) return 1;
  return bad;
}

static int check_nav(const char* path) {
  FILE* f = fopen(path, "rb");
  if (!f) return 1;
  fseek(f, 0, SEEK_END);
  const long nb = ftell(f);
  fseek(f, 0, SEEK_SET);
  char* blob = (char*)malloc((size_t)nb);
  if (fread(blob, 1, (size_t)nb, f) != (size_t)nb) return 1;
  fclose(f);
  or_geom* g = NULL;
  if (or_geom_load(blob, (size_t)nb, &g)) return 1;
  free(blob);
  const int ms = 128;
  int32_t* pv = (int32_t*)malloc(sizeof(int32_t) * (ms + 1));
  double* st = (double*)malloc(sizeof(double) * ms);
  int8_t* pr = (int8_t*)malloc((size_t)ms);
  int bad = 0;
  const double dens[3] = {1.0, 1.0, 8.0};
  const double sig[9] = {5e-6, 2e-6, 1e-6, 2e-4, 5e-5, 1e-5, 1.0 / 480.0, 1.0 / 1200.0, 1.0 / 3200.0};
  int* lvm = (int*)malloc(sizeof(int) * (size_t)g->n_lv);
  for (int l = 0; l < g->n_lv; ++l) lvm[l] = l == 0 ? 0 : (l % 2 ? 1 : 2);
  or_phys ph = {3, 3, dens, sig, lvm};
  for (int i = 0; i < 300; ++i) {
    double p[3], d[3];
    for (int k = 0; k < 3; ++k) p[k] = 2.0 * urand() - 1.0;
    iso(d);
    unsigned fl = 0, dg = 0;
    const int pv0 = or_locate(g, p);
    if (pv0 < 0) return 1;
    const int n = or_transport(g, p, d, pv0, ms, pv, st, &fl, &dg);
    double sum = 0.0;
    for (int k = 0; k < n; ++k) sum += st[k];
    unsigned d2 = 0;
    const double w = or_dist_out(&g->lv_solid[g->world_lv], p, d, &d2);
    if (!fl && !dg && fabs(sum - w) > 1e-9 * fmax(1.0, w)) ++bad;
    (void)or_nav_safety(g, p, pv0);
    (void)or_nav_inside(g, p, pv0);
    fl = dg = 0;
    (void)or_transport_phys(g, &ph, p, d, pv0, ms, 1234567ull, (uint32_t)i, pv, st, pr, &fl, &dg);
  }
  free(lvm);
  free(pv);
  free(st);
  free(pr);
  or_geom_free(g);
  return bad;
}

int main(int argc, char** argv) {
  if (argc < 3) return 2;
  const int a = check_solids(argv[1]);
  const int b = check_nav(argv[2]);
  if (a || b) {
    printf("FAIL solids %d nav %d\n", a, b);
    return 1;
  }
  printf("OK\n");
  return 0;
}
