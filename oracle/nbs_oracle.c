/*
 * nbs_oracle.c -- plain FP64 CPU oracle for the two-baryon four-point
 * function F^{<B1 B2 B3bar B4bar>}_{a1 a2, a3 a4}(r) of Nemura (LATTICE 2015).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline leg of the benchmark, never by the product library.
 *
 * What it computes, step by step, in the paper's order:
 *   1. normal baryon blocks by the explicit 24-term colour/spin sum
 *      (Sec. 2, Eq. (5); Sec. 4(i), Eq. (8));
 *   2. every Wick contraction of the six sink quarks with the six source
 *      quarks that respects flavour, with the sign of the permutation
 *      (Sec. 2, Eq. (4));
 *   3. the source tensor eps eps (C g5)(C g5) delta delta of Eq. (4);
 *   4. the sum over X, either directly (the O(L^6) evaluation mentioned in
 *      Sec. 2 below Eq. (4)) or through the DFT correlation of Eq. (6).
 * No effective blocks, no factorisation: the permutation sum is done term
 * by term so that each line can be checked against Eqs. (4)-(6).
 */
#include "nbs_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

enum { FL_U = 0, FL_D = 1, FL_S = 2 };

/* ---- constants of the operators (Sec. 2, Eqs. (2)-(3)) ---------------- */

/* Levi-Civita symbol on {0,1,2}. */
static int eps3(int a, int b, int c) { return (a - b) * (b - c) * (c - a) / 2; }

/* C gamma_5 = diag(i sigma_2, i sigma_2) in the Dirac representation. */
static const int CG5[4][4] = {
    {0, 1, 0, 0}, {-1, 0, 0, 0}, {0, 0, 0, 1}, {0, 0, -1, 0}};

void ora_cg5(double out[16]) {
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) out[4 * i + j] = CG5[i][j];
}

static void set3(int* f, int a, int b, int c) { f[0] = a; f[1] = b; f[2] = c; }

int ora_expand_op(int op, int fl[9], double w[3]) {
  const double r6 = 1.0 / sqrt(6.0), r2 = 1.0 / sqrt(2.0);
  switch (op) {
    case ORA_P:       set3(fl, FL_U, FL_D, FL_U); w[0] = +1; return 1; /* eps (u Cg5 d) u   */
    case ORA_N:       set3(fl, FL_U, FL_D, FL_D); w[0] = -1; return 1; /* -eps (u Cg5 d) d  */
    case ORA_SIGMA_P: set3(fl, FL_U, FL_S, FL_U); w[0] = -1; return 1; /* -eps (u Cg5 s) u  */
    case ORA_SIGMA_M: set3(fl, FL_D, FL_S, FL_D); w[0] = -1; return 1; /* -eps (d Cg5 s) d  */
    case ORA_XI_0:    set3(fl, FL_U, FL_S, FL_S); w[0] = +1; return 1; /* eps (u Cg5 s) s   */
    case ORA_XI_M:    set3(fl, FL_D, FL_S, FL_S); w[0] = -1; return 1; /* -eps (d Cg5 s) s  */
    case ORA_X_U:     set3(fl, FL_D, FL_S, FL_U); w[0] = +1; return 1; /* eps (d Cg5 s) u   */
    case ORA_X_D:     set3(fl, FL_S, FL_U, FL_D); w[0] = +1; return 1; /* eps (s Cg5 u) d   */
    case ORA_X_S:     set3(fl, FL_U, FL_D, FL_S); w[0] = +1; return 1; /* eps (u Cg5 d) s   */
    case ORA_LAMBDA: /* (X_u + X_d - 2 X_s) / sqrt 6 */
      set3(fl + 0, FL_D, FL_S, FL_U); w[0] = r6;
      set3(fl + 3, FL_S, FL_U, FL_D); w[1] = r6;
      set3(fl + 6, FL_U, FL_D, FL_S); w[2] = -2.0 * r6;
      return 3;
    case ORA_SIGMA_0: /* (X_u - X_d) / sqrt 2 */
      set3(fl + 0, FL_D, FL_S, FL_U); w[0] = r2;
      set3(fl + 3, FL_S, FL_U, FL_D); w[1] = -r2;
      return 2;
    default: return 0;
  }
}

/* ---- the 24 non-zero (colour, spin) terms of eps_abc (C g5)_{beta gamma} */

typedef struct { int a, b, c, be, ga; double sgn; } diq_term;

static int diquark_terms(diq_term* t) {
  int n = 0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c) {
        int e = eps3(a, b, c);
        if (!e) continue;
        for (int be = 0; be < 4; ++be)
          for (int ga = 0; ga < 4; ++ga) {
            if (!CG5[be][ga]) continue;
            t[n].a = a; t[n].b = b; t[n].c = c; t[n].be = be; t[n].ga = ga;
            t[n].sgn = (double)(e * CG5[be][ga]);
            ++n;
          }
      }
  return n;
}

/* ---- normal baryon blocks (Eq. (5)) ------------------------------------ */

/* N[al][j1][j2][j3] = sum_{abc} sum_{be ga} eps_abc Cg5_{be ga}
 *     S1[(be,a)][j1] S2[(ga,b)][j2] S3[(al,c)][j3],  al in {0,1}. */
static void normal_block_site(const cplx* S1, const cplx* S2, const cplx* S3,
                              const diq_term* dt, int ndt, cplx* out) {
  for (int al = 0; al < 2; ++al)
    for (int j1 = 0; j1 < 12; ++j1)
      for (int j2 = 0; j2 < 12; ++j2)
        for (int j3 = 0; j3 < 12; ++j3) {
          cplx acc = 0;
          for (int k = 0; k < ndt; ++k) {
            const diq_term* t = &dt[k];
            acc += t->sgn * S1[(3 * t->be + t->a) * 12 + j1] *
                   S2[(3 * t->ga + t->b) * 12 + j2] *
                   S3[(3 * al + t->c) * 12 + j3];
          }
          out[((al * 12 + j1) * 12 + j2) * 12 + j3] = acc;
        }
}

int ora_normal_blocks(const int L[3], const double* const S[3], int f1, int f2,
                      int f3, double* out) {
  if (f1 < 0 || f1 > 2 || f2 < 0 || f2 > 2 || f3 < 0 || f3 > 2) return -1;
  const long V = (long)L[0] * L[1] * L[2];
  diq_term dt[64];
  const int ndt = diquark_terms(dt);
  const cplx* s1 = (const cplx*)S[f1];
  const cplx* s2 = (const cplx*)S[f2];
  const cplx* s3 = (const cplx*)S[f3];
  cplx* o = (cplx*)out;
#pragma omp parallel for schedule(static)
  for (long x = 0; x < V; ++x)
    normal_block_site(s1 + 144 * x, s2 + 144 * x, s3 + 144 * x, dt, ndt,
                      o + 3456 * x);
  return 0;
}

/* ---- discrete Fourier transform by its definition, axis by axis ------- */

int ora_dft3(double* data, int nfield, const int L[3], int sign) {
  cplx* d = (cplx*)data;
  const long V = (long)L[0] * L[1] * L[2];
  const long stride[3] = {1, L[0], (long)L[0] * L[1]};
  for (int ax = 0; ax < 3; ++ax) {
    const int n = L[ax];
    const long st = stride[ax];
    const long nlines = V / n;
#pragma omp parallel
    {
      cplx* tmp = (cplx*)malloc(sizeof(cplx) * n * nfield);
      cplx* w = (cplx*)malloc(sizeof(cplx) * n);
      for (int m = 0; m < n; ++m) {
        double ph = sign * 2.0 * M_PI * (double)m / (double)n;
        w[m] = cos(ph) + I * sin(ph);
      }
#pragma omp for schedule(static)
      for (long li = 0; li < nlines; ++li) {
        /* site of element 0 of this line */
        long rest = li, base = 0, mul = 1;
        for (int a = 0; a < 3; ++a) {
          if (a == ax) { mul *= L[a]; continue; }
          base += (rest % L[a]) * mul;
          rest /= L[a];
          mul *= L[a];
        }
        for (int k = 0; k < n; ++k)
          for (int f = 0; f < nfield; ++f) {
            cplx acc = 0;
            for (int m = 0; m < n; ++m)
              acc += d[(base + m * st) * nfield + f] * w[(k * m) % n];
            tmp[k * nfield + f] = acc;
          }
        for (int k = 0; k < n; ++k)
          for (int f = 0; f < nfield; ++f)
            d[(base + k * st) * nfield + f] = tmp[k * nfield + f];
      }
      free(tmp);
      free(w);
    }
  }
  return 0;
}

/* ---- Wick permutations ------------------------------------------------- */

typedef struct { int p[6]; int sgn; } perm6;

/* All permutations P of the six source quarks with
 * flavour(sink quark i) == flavour(source quark P[i]); sign = sgn(P). */
static int wick_perms(const int sinkfl[6], const int srcfl[6], perm6* out) {
  int n = 0, p[6];
  for (int i0 = 0; i0 < 6; ++i0)
  for (int i1 = 0; i1 < 6; ++i1)
  for (int i2 = 0; i2 < 6; ++i2)
  for (int i3 = 0; i3 < 6; ++i3)
  for (int i4 = 0; i4 < 6; ++i4)
  for (int i5 = 0; i5 < 6; ++i5) {
    p[0] = i0; p[1] = i1; p[2] = i2; p[3] = i3; p[4] = i4; p[5] = i5;
    int used = 0, ok = 1;
    for (int k = 0; k < 6; ++k) {
      if (used & (1 << p[k])) { ok = 0; break; }
      used |= 1 << p[k];
      if (sinkfl[k] != srcfl[p[k]]) { ok = 0; break; }
    }
    if (!ok) continue;
    int inv = 0;
    for (int a = 0; a < 6; ++a)
      for (int b = a + 1; b < 6; ++b) inv += p[a] > p[b];
    memcpy(out[n].p, p, sizeof p);
    out[n].sgn = (inv & 1) ? -1 : 1;
    ++n;
  }
  return n;
}

/* ---- source tensor (Eq. (4)) --------------------------------------------
 * eps_{c1c2c3} (Cg5)_{s1 s2} delta_{s3 a3} for one source baryon: 24
 * non-zero (colour, spin) assignments of its three quarks for a given a3. */
typedef struct { int j[3]; double sgn; } src_term;

static int source_terms(int alpha, src_term* t) {
  int n = 0;
  for (int c1 = 0; c1 < 3; ++c1)
    for (int c2 = 0; c2 < 3; ++c2)
      for (int c3 = 0; c3 < 3; ++c3) {
        int e = eps3(c1, c2, c3);
        if (!e) continue;
        for (int s1 = 0; s1 < 4; ++s1)
          for (int s2 = 0; s2 < 4; ++s2) {
            if (!CG5[s1][s2]) continue;
            t[n].j[0] = 3 * s1 + c1;
            t[n].j[1] = 3 * s2 + c2;
            t[n].j[2] = 3 * alpha + c3;
            t[n].sgn = (double)(e * CG5[s1][s2]);
            ++n;
          }
      }
  return n;
}

/* ---- one channel = list of (weight, sink types, permutation) ----------- */

typedef struct {
  int f1[3], f2[3]; /* flavour triplets of the sink terms */
  double coef;      /* w1 w2 w3 w4 sgn(P) */
  int p[6];
} wick_term;

/* Expand the four operators and enumerate permutations; returns the count
 * (and fills out if non-NULL). */
static int channel_terms(const int chan[4], wick_term* out, int* n_terms) {
  int fl[4][9];
  double w[4][3];
  int nt[4];
  for (int k = 0; k < 4; ++k) {
    nt[k] = ora_expand_op(chan[k], fl[k], w[k]);
    if (nt[k] <= 0) return -1;
  }
  int n = 0, terms = 0;
  perm6 perms[720];
  for (int t1 = 0; t1 < nt[0]; ++t1)
  for (int t2 = 0; t2 < nt[1]; ++t2)
  for (int t3 = 0; t3 < nt[2]; ++t3)
  for (int t4 = 0; t4 < nt[3]; ++t4) {
    int sinkfl[6], srcfl[6];
    for (int i = 0; i < 3; ++i) {
      sinkfl[i] = fl[0][3 * t1 + i];
      sinkfl[3 + i] = fl[1][3 * t2 + i];
      srcfl[i] = fl[2][3 * t3 + i];
      srcfl[3 + i] = fl[3][3 * t4 + i];
    }
    const double wt = w[0][t1] * w[1][t2] * w[2][t3] * w[3][t4];
    const int np = wick_perms(sinkfl, srcfl, perms);
    ++terms;
    for (int k = 0; k < np; ++k) {
      if (out) {
        memcpy(out[n].f1, sinkfl, sizeof(int) * 3);
        memcpy(out[n].f2, sinkfl + 3, sizeof(int) * 3);
        out[n].coef = wt * perms[k].sgn;
        memcpy(out[n].p, perms[k].p, sizeof(int) * 6);
      }
      ++n;
    }
  }
  if (n_terms) *n_terms = terms;
  return n;
}

int ora_count_perms(const int chan[4], int* n_terms, int* n_perms) {
  int n = channel_terms(chan, NULL, n_terms);
  if (n < 0) return -1;
  *n_perms = n;
  return 0;
}

/* Contribution of one Wick term to the 16 spin components:
 * acc[s] += coef * sum_{source tensor} N1[a1][j_{P1} j_{P2} j_{P3}]
 *                                       N2[a2][j_{P4} j_{P5} j_{P6}] J(j). */
static void contract_term(const cplx* N1, const cplx* N2, const wick_term* wt,
                          const src_term st[2][24], cplx acc[16]) {
  for (int a3 = 0; a3 < 2; ++a3)
    for (int a4 = 0; a4 < 2; ++a4) {
      cplx part[2][2] = {{0, 0}, {0, 0}};
      for (int ka = 0; ka < 24; ++ka)
        for (int kb = 0; kb < 24; ++kb) {
          int j[6];
          j[0] = st[a3][ka].j[0]; j[1] = st[a3][ka].j[1]; j[2] = st[a3][ka].j[2];
          j[3] = st[a4][kb].j[0]; j[4] = st[a4][kb].j[1]; j[5] = st[a4][kb].j[2];
          const double jv = st[a3][ka].sgn * st[a4][kb].sgn;
          const int i1 = (j[wt->p[0]] * 12 + j[wt->p[1]]) * 12 + j[wt->p[2]];
          const int i2 = (j[wt->p[3]] * 12 + j[wt->p[4]]) * 12 + j[wt->p[5]];
          for (int a1 = 0; a1 < 2; ++a1)
            for (int a2 = 0; a2 < 2; ++a2)
              part[a1][a2] += jv * N1[a1 * 1728 + i1] * N2[a2 * 1728 + i2];
        }
      for (int a1 = 0; a1 < 2; ++a1)
        for (int a2 = 0; a2 < 2; ++a2)
          acc[8 * a1 + 4 * a2 + 2 * a3 + a4] += wt->coef * part[a1][a2];
    }
}

static int type_index(const int f[3]) { return (f[0] * 3 + f[1]) * 3 + f[2]; }

static long wrap(long v, long n) { v %= n; return v < 0 ? v + n : v; }

/* Normal blocks of every flavour triplet a set of channels needs:
 * blocks[type_index] = [V][3456] or NULL. */
static int build_needed_blocks(const int L[3], const double* const S[3],
                               int n_ch, const int* chans, cplx* blocks[27],
                               wick_term** terms, int* nterms) {
  const long V = (long)L[0] * L[1] * L[2];
  for (int t = 0; t < 27; ++t) blocks[t] = NULL;
  for (int c = 0; c < n_ch; ++c) {
    int nt;
    int n = channel_terms(chans + 4 * c, NULL, &nt);
    if (n < 0) return -1;
    terms[c] = (wick_term*)malloc(sizeof(wick_term) * (n > 0 ? n : 1));
    nterms[c] = channel_terms(chans + 4 * c, terms[c], &nt);
    for (int k = 0; k < nterms[c]; ++k) {
      const int* fs[2] = {terms[c][k].f1, terms[c][k].f2};
      for (int s = 0; s < 2; ++s) {
        int ti = type_index(fs[s]);
        if (blocks[ti]) continue;
        blocks[ti] = (cplx*)malloc(sizeof(cplx) * 3456 * V);
        if (!blocks[ti]) return -2;
        ora_normal_blocks(L, S, fs[s][0], fs[s][1], fs[s][2], (double*)blocks[ti]);
      }
    }
  }
  return 0;
}

static void free_blocks(cplx* blocks[27], wick_term** terms, int n_ch) {
  for (int t = 0; t < 27; ++t) free(blocks[t]);
  for (int c = 0; c < n_ch; ++c) free(terms[c]);
}

int ora_correlators(int mode, const int L[3], const double* const S[3],
                    int n_ch, const int* chans, double* Fout) {
  if (mode != 0 && mode != 1) return -1;
  const long V = (long)L[0] * L[1] * L[2];
  cplx* blocks[27];
  wick_term** terms = (wick_term**)calloc(n_ch, sizeof(wick_term*));
  int* nterms = (int*)calloc(n_ch, sizeof(int));
  int rc = build_needed_blocks(L, S, n_ch, chans, blocks, terms, nterms);
  if (rc) { free_blocks(blocks, terms, n_ch); free(terms); free(nterms); return rc; }
  src_term st[2][24];
  source_terms(0, st[0]);
  source_terms(1, st[1]);
  cplx* F = (cplx*)Fout;

  if (mode == 1) /* Eq. (6): forward DFT of every block field */
    for (int t = 0; t < 27; ++t)
      if (blocks[t]) ora_dft3((double*)blocks[t], 3456, L, -1);

  for (int c = 0; c < n_ch; ++c) {
    cplx* Fc = F + (long)c * 16 * V;
#pragma omp parallel for schedule(dynamic, 1)
    for (long r = 0; r < V; ++r) {
      const long rx = r % L[0], ry = (r / L[0]) % L[1], rz = r / ((long)L[0] * L[1]);
      cplx acc[16];
      for (int s = 0; s < 16; ++s) acc[s] = 0;
      if (mode == 0) {
        /* F(r) = sum_X sum_P B1(X + r) B2(X) J  (Eq. (4)) */
        for (long X = 0; X < V; ++X) {
          const long xx = X % L[0], xy = (X / L[0]) % L[1], xz = X / ((long)L[0] * L[1]);
          const long x1 = wrap(xx + rx, L[0]) +
                          L[0] * (wrap(xy + ry, L[1]) + L[1] * wrap(xz + rz, L[2]));
          for (int k = 0; k < nterms[c]; ++k) {
            const wick_term* wt = &terms[c][k];
            contract_term(blocks[type_index(wt->f1)] + 3456 * x1,
                          blocks[type_index(wt->f2)] + 3456 * X, wt, st, acc);
          }
        }
      } else {
        /* here r plays the role of q: F~(q) = sum_P B~1(q) B~2(-q) J */
        const long mq = wrap(-rx, L[0]) +
                        L[0] * (wrap(-ry, L[1]) + L[1] * wrap(-rz, L[2]));
        for (int k = 0; k < nterms[c]; ++k) {
          const wick_term* wt = &terms[c][k];
          contract_term(blocks[type_index(wt->f1)] + 3456 * r,
                        blocks[type_index(wt->f2)] + 3456 * mq, wt, st, acc);
        }
      }
      for (int s = 0; s < 16; ++s) Fc[s * V + r] = acc[s];
    }
    if (mode == 1) {
      /* F(r) = (1/V) sum_q F~(q) exp(+i q.r): 16 fields stored [16][V];
       * transpose to site-major for ora_dft3 and back. */
      cplx* tmp = (cplx*)malloc(sizeof(cplx) * 16 * V);
      for (long x = 0; x < V; ++x)
        for (int s = 0; s < 16; ++s) tmp[x * 16 + s] = Fc[s * V + x];
      ora_dft3((double*)tmp, 16, L, +1);
      for (long x = 0; x < V; ++x)
        for (int s = 0; s < 16; ++s) Fc[s * V + x] = tmp[x * 16 + s] / (double)V;
      free(tmp);
    }
  }
  free_blocks(blocks, terms, n_ch);
  free(terms);
  free(nterms);
  return 0;
}

int ora_correlators_at_q(const int L[3], const double* const S[3], int n_ch,
                         const int* chans, const int q[3], double* out) {
  const long V = (long)L[0] * L[1] * L[2];
  wick_term** terms = (wick_term**)calloc(n_ch, sizeof(wick_term*));
  int* nterms = (int*)calloc(n_ch, sizeof(int));
  int needed[27] = {0};
  for (int c = 0; c < n_ch; ++c) {
    int nt;
    int n = channel_terms(chans + 4 * c, NULL, &nt);
    if (n < 0) { for (int k = 0; k < c; ++k) free(terms[k]); free(terms); free(nterms); return -1; }
    terms[c] = (wick_term*)malloc(sizeof(wick_term) * (n > 0 ? n : 1));
    nterms[c] = channel_terms(chans + 4 * c, terms[c], &nt);
    for (int k = 0; k < nterms[c]; ++k) {
      needed[type_index(terms[c][k].f1)] = 1;
      needed[type_index(terms[c][k].f2)] = 1;
    }
  }
  diq_term dt[64];
  const int ndt = diquark_terms(dt);
  /* B~(+q) and B~(-q) of every needed block, by the DFT definition */
  cplx* bq[27][2];
  for (int t = 0; t < 27; ++t) {
    bq[t][0] = bq[t][1] = NULL;
    if (!needed[t]) continue;
    const int f1 = t / 9, f2 = (t / 3) % 3, f3 = t % 3;
    bq[t][0] = (cplx*)calloc(3456, sizeof(cplx));
    bq[t][1] = (cplx*)calloc(3456, sizeof(cplx));
    const cplx* s1 = (const cplx*)S[f1];
    const cplx* s2 = (const cplx*)S[f2];
    const cplx* s3 = (const cplx*)S[f3];
#pragma omp parallel
    {
      cplx* nb = (cplx*)malloc(sizeof(cplx) * 3456);
      cplx* a0 = (cplx*)calloc(3456, sizeof(cplx));
      cplx* a1 = (cplx*)calloc(3456, sizeof(cplx));
#pragma omp for schedule(static)
      for (long x = 0; x < V; ++x) {
        const long xs[3] = {x % L[0], (x / L[0]) % L[1], x / ((long)L[0] * L[1])};
        double ph = 0;
        for (int a = 0; a < 3; ++a)
          ph += (double)((wrap(q[a], L[a]) * xs[a]) % L[a]) / (double)L[a];
        const cplx e = cos(2 * M_PI * ph) - I * sin(2 * M_PI * ph); /* exp(-i q.x) */
        normal_block_site(s1 + 144 * x, s2 + 144 * x, s3 + 144 * x, dt, ndt, nb);
        for (int k = 0; k < 3456; ++k) {
          a0[k] += nb[k] * e;
          a1[k] += nb[k] * conj(e);
        }
      }
#pragma omp critical
      for (int k = 0; k < 3456; ++k) { bq[t][0][k] += a0[k]; bq[t][1][k] += a1[k]; }
      free(nb); free(a0); free(a1);
    }
  }
  src_term st[2][24];
  source_terms(0, st[0]);
  source_terms(1, st[1]);
  cplx* o = (cplx*)out;
  for (int c = 0; c < n_ch; ++c) {
    cplx acc[16];
    for (int s = 0; s < 16; ++s) acc[s] = 0;
    for (int k = 0; k < nterms[c]; ++k) {
      const wick_term* wt = &terms[c][k];
      contract_term(bq[type_index(wt->f1)][0], bq[type_index(wt->f2)][1], wt, st, acc);
    }
    for (int s = 0; s < 16; ++s) o[16 * c + s] = acc[s];
  }
  for (int t = 0; t < 27; ++t) { free(bq[t][0]); free(bq[t][1]); }
  for (int c = 0; c < n_ch; ++c) free(terms[c]);
  free(terms);
  free(nterms);
  return 0;
}

/* ---- single-baryon two-point functions (zero momentum) ----------------- */

int ora_two_point(const int L[3], const double* const S[3], int n_pairs,
                  const int* pairs, double* out) {
  const long V = (long)L[0] * L[1] * L[2];
  src_term st[2][24];
  for (int a = 0; a < 2; ++a)
    if (source_terms(a, st[a]) != 24) return -2;
  cplx* C = (cplx*)out;
  cplx* blk = (cplx*)malloc(sizeof(cplx) * 3456 * (size_t)V);
  if (!blk) return -3;
  int rc = 0;
  for (int k = 0; k < n_pairs && !rc; ++k) {
    int fs[9], fc[9];
    double ws[3], wc[3];
    const int ns = ora_expand_op(pairs[2 * k], fs, ws);
    const int nc = ora_expand_op(pairs[2 * k + 1], fc, wc);
    if (ns <= 0 || nc <= 0) { rc = -1; break; }
    cplx acc[2][2] = {{0, 0}, {0, 0}};
    for (int ts = 0; ts < ns; ++ts) {
      /* the sink term's normal block, summed over the sites of the slice */
      if (ora_normal_blocks(L, S, fs[3 * ts], fs[3 * ts + 1], fs[3 * ts + 2], (double*)blk)) { rc = -1; break; }
      cplx Nsum[3456];
      for (int i = 0; i < 3456; ++i) Nsum[i] = 0;
      for (long x = 0; x < V; ++x)
        for (int i = 0; i < 3456; ++i) Nsum[i] += blk[3456 * x + i];
      for (int tc = 0; tc < nc; ++tc) {
        /* permutations P of the three source quarks with
         * flavour(sink quark i) == flavour(source quark P[i]) */
        for (int p0 = 0; p0 < 3; ++p0)
          for (int p1 = 0; p1 < 3; ++p1)
            for (int p2 = 0; p2 < 3; ++p2) {
              const int p[3] = {p0, p1, p2};
              if (p0 == p1 || p0 == p2 || p1 == p2) continue;
              int ok = 1;
              for (int i = 0; i < 3; ++i)
                if (fs[3 * ts + i] != fc[3 * tc + p[i]]) ok = 0;
              if (!ok) continue;
              const int inv = (p0 > p1) + (p0 > p2) + (p1 > p2);
              const double coef = ws[ts] * wc[tc] * ((inv & 1) ? -1.0 : 1.0);
              for (int ap = 0; ap < 2; ++ap)
                for (int m = 0; m < 24; ++m) {
                  const int* j = st[ap][m].j;
                  const int idx = (j[p[0]] * 12 + j[p[1]]) * 12 + j[p[2]];
                  for (int a = 0; a < 2; ++a)
                    acc[a][ap] += coef * st[ap][m].sgn * Nsum[a * 1728 + idx];
                }
            }
      }
    }
    for (int a = 0; a < 2; ++a)
      for (int ap = 0; ap < 2; ++ap) C[4 * k + 2 * a + ap] = acc[a][ap];
  }
  free(blk);
  return rc;
}
