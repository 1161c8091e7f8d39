/* The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a
 * few coupled steps of small beds with every face type, the contact searches,
 * the float hard-sphere stage, and the 3-D lattice steps.  Exits 0 when every
 * call succeeds; a memory or undefined-behaviour error aborts the run. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/lbdps_oracle.c"

static double unif(uint64_t *s) { /* splitmix64 (Steele, Lea & Flood 2014) */
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * 0x1.0p-53;
}

static int bed(int bcx, int bcy0, int bcy1, int loop, int nsub, double cs) {
  orc_params p;
  memset(&p, 0, sizeof p);
  p.nx = 13;
  p.ny = 17;
  p.bc[0] = p.bc[1] = bcx;
  p.bc[2] = bcy0;
  p.bc[3] = bcy1;
  p.tau = 0.6;
  p.rho_g = 1.0;
  p.rho_s = 788.5;
  p.d = 0.5;
  p.e_pp = 0.9;
  p.e_pw = 0.8;
  p.g[1] = -1e-5;
  p.G[1] = 1e-6;
  p.pressure_sign = -1;
  p.omega_dense = 1.0;
  p.cs_smag = cs;
  p.n_sub = nsub;
  p.particles_periodic_y = loop;
  const int64_t C = (int64_t)p.nx * p.ny, n = 300;
  double *f = malloc(sizeof(double) * 9 * C), *pos = malloc(sizeof(double) * 2 * n),
         *vel = malloc(sizeof(double) * 2 * n), *inlet = malloc(sizeof(double) * p.nx);
  uint64_t s = 42;
  for (int64_t c = 0; c < C; ++c)
    for (int i = 0; i < 9; ++i) f[i * C + c] = orc_feq(i, 1.0, 0.0, 0.0);
  for (int i = 0; i < p.nx; ++i) inlet[i] = 0.01;
  for (int64_t k = 0; k < n; ++k) {
    pos[2 * k] = 0.3 + (p.nx - 0.6) * unif(&s);
    pos[2 * k + 1] = 0.3 + (p.ny - 0.6) * unif(&s);
    vel[2 * k] = 0.02 * (unif(&s) - 0.5);
    vel[2 * k + 1] = 0.2 * (unif(&s) - 0.5);
  }
  orc_out o;
  memset(&o, 0, sizeof o);
  int32_t *pairs = malloc(sizeof(int32_t) * 2 * 32 * n);
  o.pairs = pairs;
  o.pair_cap = 32 * n;
  int rc = 0;
  for (int step = 0; step < 8 && rc == 0; ++step) rc = orc_step(&p, inlet, f, n, pos, vel, &o);
  int64_t m1 = 0, m2 = 0;
  if (rc == 0) rc = orc_contacts_brute(&p, n, pos, pairs, 32 * n, &m1);
  if (rc == 0) rc = orc_contacts_cells(&p, n, pos, pairs, 32 * n, &m2);
  if (rc == 0 && m1 != m2) rc = 99;
  int32_t *cell = malloc(sizeof(int32_t) * 2 * n);
  float *off = malloc(sizeof(float) * 2 * n), *v32 = malloc(sizeof(float) * 2 * n);
  for (int64_t k = 0; k < 2 * n; ++k) {
    cell[k] = (int32_t)floor(pos[k]);
    off[k] = (float)(pos[k] - cell[k]);
    if (off[k] >= 1.0f) off[k] = 0.99999994f;
    v32[k] = (float)vel[k];
  }
  int64_t np2 = 0, nc = 0, nw = 0;
  if (rc == 0)
    rc = orc_collide_f32(p.nx, p.ny, bcx == 0, bcy0 == 0 || loop, p.d, p.rho_s, p.e_pp, p.e_pw, n, cell, off, v32,
                         pairs, 32 * n, &np2, &nc, &nw);
  double cons[5];
  orc_conservation(&p, f, n, vel, cons);
  free(f);
  free(pos);
  free(vel);
  free(inlet);
  free(pairs);
  free(cell);
  free(off);
  free(v32);
  return rc;
}

int main(void) {
  int rc = 0;
  rc |= bed(ORC_PERIODIC, ORC_INLET, ORC_OUTLET, 0, 1, 0.0);
  rc |= bed(ORC_WALL, ORC_WALL, ORC_WALL, 0, 3, 0.0);
  rc |= bed(ORC_WALL, ORC_PERIODIC, ORC_PERIODIC, 0, 1, 1.0);
  rc |= bed(ORC_WALL, ORC_INLET, ORC_OUTLET, 1, 2, 0.3);
  /* the 3-D lattice, with and without solids */
  const int nx = 5, ny = 4, nz = 3, C = nx * ny * nz;
  double *f = malloc(sizeof(double) * 19 * C), *vs = calloc(3 * (size_t)C, sizeof(double)),
         *force = malloc(sizeof(double) * 3 * C);
  int32_t *n = calloc((size_t)C, sizeof(int32_t));
  for (int c = 0; c < C; ++c) {
    for (int i = 0; i < 19; ++i) f[i * C + c] = orc3_feq(i, 1.0, 0.01, 0.0, -0.02);
    n[c] = c % 4;
    vs[c] = 0.003;
  }
  orc3_bgk_step(nx, ny, nz, 0.7, f);
  orc3_psm_step(nx, ny, nz, 0.7, 0.5, n, vs, f, force);
  free(f);
  free(vs);
  free(force);
  free(n);
  printf("oracle driver: rc %d\n", rc);
  return rc;
}
