/*
 * nbs_oracle.h -- CPU oracle for the two-baryon four-point function.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this code; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It is a plain FP64 evaluation of
 * the definition (Nemura, LATTICE 2015, Sec. 2, Eqs. (1)-(5)) written to be
 * checked by eye, not to be fast.
 *
 * Conventions (each one a reading of the paper, listed in the design notes):
 *   - propagator S_f(x) for flavour f in {u=0,d=1,s=2} is a 12x12 complex
 *     matrix per site, row = 3*spin + colour at the sink, column =
 *     3*spin + colour at the (wall) source; sites are x + Lx*(y + Ly*z).
 *   - normal block N[alpha][j1][j2][j3], alpha in {0,1} (upper Dirac
 *     components), j = 3*spin + colour, Eq. (5) / Sec. 4(i).
 *   - F[s][r] with s = 8*a1 + 4*a2 + 2*a3 + a4, r = x_{B1} - x_{B2} mod L.
 */
#ifndef NBS_ORACLE_H
#define NBS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Operator codes, in the order the paper lists them in Eqs. (2)-(3). */
enum {
  ORA_P = 0, ORA_N, ORA_LAMBDA, ORA_SIGMA_P, ORA_SIGMA_0, ORA_SIGMA_M,
  ORA_XI_0, ORA_XI_M, ORA_X_U, ORA_X_D, ORA_X_S, ORA_NUM_OPS
};

/* C*gamma_5 in the Dirac representation, row-major 4x4 (real). */
void ora_cg5(double out[16]);

/* Weighted flavour triplets of an operator (Eqs. (2)-(3)).  Returns the
 * number of terms (<= 3); fl[3*k + i] is the flavour of quark i of term k. */
int ora_expand_op(int op, int fl[9], double w[3]);

/* Normal blocks N_{f1 f2 f3}(x) for every site: out is [V][2][12][12][12]
 * complex (interleaved re,im).  S[f] points at [V][12][12] complex. */
int ora_normal_blocks(const int L[3], const double* const S[3],
                      int f1, int f2, int f3, double* out);

/* In-place 3-D DFT of nfield fields stored site-major ([V][nfield]):
 * out(q) = sum_x in(x) exp(sign * 2 pi i q.x / L), no normalisation. */
int ora_dft3(double* data, int nfield, const int L[3], int sign);

/* Four-point functions of n_ch channels on one time slice.
 * chans[4*c + k] = (B1, B2, B3, B4) operator codes.
 * mode 0: direct O(V^2) sum over X (Eq. (4));
 * mode 1: DFT correlation (Eq. (6)).
 * F is [n_ch][16][V] complex. */
int ora_correlators(int mode, const int L[3], const double* const S[3],
                    int n_ch, const int* chans, double* F);

/* Momentum-space F~_c(q) at one momentum q (integer components, taken mod
 * L) for n_ch channels: out is [n_ch][16] complex.  F(r) is (1/V) times the
 * inverse DFT of F~. */
int ora_correlators_at_q(const int L[3], const double* const S[3],
                         int n_ch, const int* chans, const int q[3],
                         double* out);

/* Single-baryon two-point functions at zero momentum on one time slice:
 *   C[a][a'] = sum_x sum over the operators' weighted flavour terms and the
 *   flavour-respecting permutations P of the three source quarks, sgn(P)
 *   times the one-baryon source tensor eps_{c1c2c3} (C g5)_{s1 s2}
 *   delta_{s3 a'} times N_sink(x)[a][j_{P(0)}][j_{P(1)}][j_{P(2)}]
 * (Eq. (1) with one baryon at sink and source, Eqs. (2)-(5)).
 * pairs[2*k] = sink operator, pairs[2*k+1] = source operator; out is
 * [n_pairs][2][2] complex (a = sink spin, a' = source spin). */
int ora_two_point(const int L[3], const double* const S[3], int n_pairs,
                  const int* pairs, double* out);

/* Number of flavour-consistent Wick permutations summed for a channel,
 * over all weighted operator terms, and the number of such terms. */
int ora_count_perms(const int chan[4], int* n_terms, int* n_perms);

#ifdef __cplusplus
}
#endif
#endif
