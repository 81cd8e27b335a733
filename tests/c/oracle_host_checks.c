/* The oracle's entry points on a tiny lattice (test code, built with the
 * address and undefined-behaviour sanitizers): blocks, transforms, the four
 * modes of the four-point functions, two-point functions, counts. */
#include <complex.h>
#include <stdio.h>
#include <stdlib.h>

#include "nbs_oracle.h"

int main(void) {
  const int L[3] = {2, 3, 2};
  const int V = 12;
  double* S[3];
  unsigned x = 12345u;
  for (int f = 0; f < 3; ++f) {
    S[f] = (double*)malloc(sizeof(double) * 2 * 144 * V);
    for (int i = 0; i < 2 * 144 * V; ++i) {
      x = x * 1664525u + 1013904223u;
      S[f][i] = (double)(x >> 8) / 16777216.0 - 0.5;
    }
  }
  const double* cs[3] = {S[0], S[1], S[2]};
  int fails = 0;
  double cg[16];
  ora_cg5(cg);
  int fl[9];
  double w[3];
  for (int op = 0; op < 11; ++op) fails += ora_expand_op(op, fl, w) < 1;
  double* nb = (double*)malloc(sizeof(double) * 2 * V * 3456);
  fails += ora_normal_blocks(L, cs, 0, 1, 2, nb) != 0;
  fails += ora_dft3(nb, 3456, L, -1) != 0;
  const int chans[] = {0, 0, 0, 0, 0, 2, 0, 8, 2, 2, 3, 5, 6, 7, 6, 7};
  double* F = (double*)malloc(sizeof(double) * 2 * 4 * 16 * V);
  fails += ora_correlators(0, L, cs, 4, chans, F) != 0;
  fails += ora_correlators(1, L, cs, 4, chans, F) != 0;
  const int q[3] = {1, 2, 1};
  double Fq[2 * 4 * 16];
  fails += ora_correlators_at_q(L, cs, 4, chans, q, Fq) != 0;
  const int pairs[] = {0, 0, 2, 4, 6, 6};
  double C[2 * 3 * 4];
  fails += ora_two_point(L, cs, 3, pairs, C) != 0;
  int nt = 0, np = 0;
  fails += ora_count_perms(chans + 4, &nt, &np) != 0 || nt != 3 || np != 36;
  free(nb);
  free(F);
  for (int f = 0; f < 3; ++f) free(S[f]);
  printf(fails ? "oracle_host_checks: %d failures\n" : "oracle_host_checks: ok\n", fails);
  return fails ? 1 : 0;
}
