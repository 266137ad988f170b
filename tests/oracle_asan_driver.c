/* Drives the CPU oracle (oracle/chem_oracle.c) under AddressSanitizer and
 * UndefinedBehaviorSanitizer. TEST INFRASTRUCTURE ONLY.
 *
 * Usage: oracle_asan_driver <mech>   (load only: prints "ok" or "error <message>")
 *        oracle_asan_driver <mech> <states.bin> <n_cells> <dt> <scheme> <jacobian> <state> <out.bin>
 * states.bin holds n_cells rows of Ns + 2 doubles (T, p, Y). The driver
 * integrates them on two threads with evaluation counts, writes phi_out,
 * h, n_acc, n_rej, n_jac, n_fev and status to out.bin, and also runs the
 * single-state entry points (f, J, FD J, LU and solve, one step, element
 * counts) on the first cell. A sanitizer report stops it with a non-zero
 * exit status. */
#include <stdio.h>
#include <stdlib.h>

#include "../oracle/chem_oracle.h"

int main(int argc, char** argv) {
  orc_mech* m = NULL;
  if (argc == 2) {
    if (orc_mech_load(argv[1], &m) != 0) {
      printf("error %s\n", orc_last_error());
    } else {
      printf("ok\n");
      orc_mech_free(m);
    }
    return 0;
  }
  if (argc != 9) return 2;
  if (orc_mech_load(argv[1], &m) != 0) {
    fprintf(stderr, "%s\n", orc_last_error());
    return 3;
  }
  int ns, nr;
  orc_mech_dims(m, &ns, &nr);
  const long nc = atol(argv[3]);
  const double dt = atof(argv[4]);
  const int w = ns + 2, n = ns + 1;
  double* phi = malloc(sizeof(double) * nc * w);
  FILE* f = fopen(argv[2], "rb");
  if (!f || fread(phi, sizeof(double), (size_t)(nc * w), f) != (size_t)(nc * w)) return 4;
  fclose(f);
  double* out = malloc(sizeof(double) * nc * w);
  double* h = calloc(nc, sizeof(double));
  int *na = malloc(sizeof(int) * nc), *nrj = malloc(sizeof(int) * nc);
  int *nj = malloc(sizeof(int) * nc), *nf = malloc(sizeof(int) * nc);
  signed char* st = malloc(nc);
  orc_opts o = {1e-6, 1e-10, 100000, atoi(argv[5]), atoi(argv[6]), atoi(argv[7])};
  if (orc_integrate_counts(m, nc, dt, &o, phi, out, h, na, nrj, nj, nf, st, 2) != 0) return 5;
  FILE* g = fopen(argv[8], "wb");
  fwrite(out, sizeof(double), (size_t)(nc * w), g);
  fwrite(h, sizeof(double), (size_t)nc, g);
  fwrite(na, sizeof(int), (size_t)nc, g);
  fwrite(nrj, sizeof(int), (size_t)nc, g);
  fwrite(nj, sizeof(int), (size_t)nc, g);
  fwrite(nf, sizeof(int), (size_t)nc, g);
  fwrite(st, 1, (size_t)nc, g);
  fclose(g);
  /* single-state entry points on the first cell */
  double* y = malloc(sizeof(double) * n);
  y[0] = phi[0];
  for (int i = 0; i < ns; ++i) y[1 + i] = phi[2 + i];
  const double p = phi[1];
  double *fv = malloc(sizeof(double) * n), *J = malloc(sizeof(double) * n * n), *J2 = malloc(sizeof(double) * n * n);
  double *yn = malloc(sizeof(double) * n), *ev = malloc(sizeof(double) * n);
  int* piv = malloc(sizeof(int) * n);
  orc_rhs(m, p, y, fv);
  orc_jac(m, p, y, J);
  orc_jac_fd(m, p, y, fv, J2);
  orc_state_rhs(m, ORC_STATE_NO_BATH, p, y, fv);
  orc_state_jac(m, ORC_STATE_NO_BATH, p, y, J2);
  for (int i = 0; i < n; ++i) J[(size_t)i * n + i] -= 1e7;
  if (orc_lu(n, J, piv) != 0) return 6;
  orc_lu_solve(n, J, piv, fv);
  orc_step(m, ORC_ROS4, p, y, 1e-8, yn, ev);
  int ne = 0;
  orc_mech_elements(m, &ne, NULL);
  int* counts = malloc(sizeof(int) * ns * ne);
  orc_mech_elements(m, &ne, counts);
  free(counts); free(piv); free(ev); free(yn); free(J2); free(J); free(fv); free(y);
  free(st); free(nf); free(nj); free(nrj); free(na); free(h); free(out); free(phi);
  orc_mech_free(m);
  return 0;
}
