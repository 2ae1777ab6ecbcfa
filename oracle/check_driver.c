/*
 * check_driver.c -- TEST INFRASTRUCTURE ONLY: a small program that runs the
 * oracle's entry points on a ragged grid, so that the tests can build it
 * with the address and undefined-behaviour sanitizers.  Usage:
 *   check_driver <params file: one orc_params struct, native layout>
 * Prints "ok" and exits 0 when every call returned normally.
 */
#include <stdio.h>
#include <stdlib.h>

#include "pf_oracle.h"

int main(int argc, char** argv) {
  if (argc != 2) return 2;
  orc_params p;
  FILE* f = fopen(argv[1], "rb");
  if (!f || fread(&p, sizeof(p), 1, f) != 1) return 3;
  fclose(f);
  const orc_grid g = {11, 9, 14, 1.0};
  const size_t n = (size_t)g.nx * g.ny * g.nz;
  double* phi = malloc(sizeof(double) * 4 * n);
  double* mu = malloc(sizeof(double) * 2 * n);
  if (!phi || !mu) return 4;
  const double mu0[2] = {0.0, 0.0}, fill[2] = {0.01, -0.02};
  orc_init_voronoi(&g, 7, 5, 6, mu0, phi, mu);
  if (orc_run(&g, &p, 0, 3, phi, mu, 2) != 0) return 5;
  int64_t shifts = 0;
  if (orc_run_window(&g, &p, 3, 3, 4, fill, &shifts, phi, mu, 2) != 0) return 6;
  orc_params q = p;
  q.top_dirichlet = 1;
  q.mu_top[0] = fill[0];
  q.mu_top[1] = fill[1];
  if (orc_run(&g, &q, 6, 2, phi, mu, 1) != 0) return 7;
  orc_diag dg;
  orc_diagnostics(&g, &p, 8 * p.dt, phi, mu, &dg);
  int64_t total = 0;
  for (int a = 0; a < 4; ++a) {
    const int64_t m = orc_mesh_phase(&g, phi, a, 0.5, NULL, 0);
    float* tri = malloc(sizeof(float) * 9 * (size_t)(m > 0 ? m : 1));
    if (!tri) return 8;
    if (orc_mesh_phase(&g, phi, a, 0.5, tri, m) != m) return 9;
    total += m;
    free(tri);
  }
  printf("ok %lld %lld %g\n", (long long)shifts, (long long)total, dg.sum_phi[3]);
  free(phi);
  free(mu);
  return 0;
}
