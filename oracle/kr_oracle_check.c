/*
 * kr_oracle_check.c -- stand-alone driver of the FP64 oracle for sanitizer
 * builds (TEST INFRASTRUCTURE ONLY).
 *
 * Built together with kr_oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer by the tests, it runs every exported oracle
 * routine on one network and batch read from a file and writes the results,
 * so that out-of-bounds accesses, uses of uninitialised stack slots turned
 * into undefined behaviour, signed overflow and the like stop the run.
 *
 * Input file (native endianness):
 *   int32  S, n_rows, n_elem, R, n_cells, has_arr_r
 *   int32  comp[n_rows * S], reservoir[n_rows], reac[3R], prod[3R]
 *   double cv[S], h_form[S], s_form[S], arr_f[3R], arr_r[3R] (if has_arr_r),
 *          p_ref, T_min, T_max
 *   double n[S * n_cells] ([S][n_cells]), T[n_cells], dt[n_cells]
 * Output file:
 *   double n[S * n_cells], T[n_cells], h_hint[n_cells], resid[n_cells]
 *   int32  status[n_cells], stats[4 * n_cells], h_log_n[n_cells],
 *          post[n_cells]
 *   double J[N * N], M[N * N], x_lu[N], x_full[N], tau, kf[R], kr[R]
 *          (cell 0; N = S + 1)
 * Exit status: 0 ok, 1 bad input, 2 the oracle rejected the input, 3 the
 * replay of the recorded substeps did not reproduce the adaptive result.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "kr_oracle.h"

static int rd(FILE *f, void *p, size_t sz, size_t n) { return fread(p, sz, n, f) == n; }

int main(int argc, char **argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s input output\n", argv[0]);
    return 1;
  }
  FILE *f = fopen(argv[1], "rb");
  if (!f) return 1;
  int32_t hd[6];
  if (!rd(f, hd, sizeof(int32_t), 6)) return 1;
  const int S = hd[0], nr = hd[1], ne = hd[2], R = hd[3], nc = hd[4], has_r = hd[5];
  if (S < 1 || S > 63 || nr < 0 || R < 0 || nc < 1) return 1;
  const int N = S + 1;
  int32_t *comp = malloc(sizeof(int32_t) * (size_t)(nr * S + 1));
  int32_t *res = malloc(sizeof(int32_t) * (size_t)(nr + 1));
  int32_t *reac = malloc(sizeof(int32_t) * (size_t)(3 * R + 1));
  int32_t *prod = malloc(sizeof(int32_t) * (size_t)(3 * R + 1));
  double *cv = malloc(sizeof(double) * S), *hf = malloc(sizeof(double) * S);
  double *sf = malloc(sizeof(double) * S);
  double *af = malloc(sizeof(double) * (size_t)(3 * R + 1));
  double *ar = has_r ? malloc(sizeof(double) * (size_t)(3 * R + 1)) : NULL;
  double lim[3];
  double *n = malloc(sizeof(double) * (size_t)S * nc), *T = malloc(sizeof(double) * nc);
  double *dt = malloc(sizeof(double) * nc);
  int ok = rd(f, comp, sizeof(int32_t), (size_t)(nr * S)) && rd(f, res, sizeof(int32_t), (size_t)nr) &&
           rd(f, reac, sizeof(int32_t), (size_t)(3 * R)) && rd(f, prod, sizeof(int32_t), (size_t)(3 * R)) &&
           rd(f, cv, sizeof(double), (size_t)S) && rd(f, hf, sizeof(double), (size_t)S) &&
           rd(f, sf, sizeof(double), (size_t)S) && rd(f, af, sizeof(double), (size_t)(3 * R)) &&
           (!has_r || rd(f, ar, sizeof(double), (size_t)(3 * R))) && rd(f, lim, sizeof(double), 3) &&
           rd(f, n, sizeof(double), (size_t)S * nc) && rd(f, T, sizeof(double), (size_t)nc) &&
           rd(f, dt, sizeof(double), (size_t)nc);
  fclose(f);
  if (!ok) return 1;
  int err = 0;
  kro_net *net = kro_net_create(S, nr, ne, comp, res, cv, hf, sf, R, reac, prod, af, ar, lim[0],
                                lim[1], lim[2], &err);
  if (!net) return 2;

  /* adaptive run with every extra, then its replay */
  const int cap = 20000;
  double *n1 = malloc(sizeof(double) * (size_t)S * nc), *T1 = malloc(sizeof(double) * nc);
  memcpy(n1, n, sizeof(double) * (size_t)S * nc);
  memcpy(T1, T, sizeof(double) * nc);
  double *hint = calloc((size_t)nc, sizeof(double));
  double *hlog = calloc((size_t)cap * nc, sizeof(double));
  int32_t *hlog_n = calloc((size_t)nc, sizeof(int32_t)), *post = calloc((size_t)nc, sizeof(int32_t));
  int32_t *status = calloc((size_t)nc, sizeof(int32_t)), *stats = calloc((size_t)4 * nc, sizeof(int32_t));
  kro_opts o;
  kro_default_opts(&o);
  kro_extras ex = {hint, hlog, nc, cap, hlog_n, post};
  if (kro_integrate_ex(net, nc, n1, nc, T1, NULL, dt, 0.0, &o, status, stats, &ex, 1) != 0) return 2;
  double *n2 = malloc(sizeof(double) * (size_t)S * nc), *T2 = malloc(sizeof(double) * nc);
  memcpy(n2, n, sizeof(double) * (size_t)S * nc);
  memcpy(T2, T, sizeof(double) * nc);
  int32_t *st2 = calloc((size_t)nc, sizeof(int32_t));
  kro_opts orp = o;
  orp.mode = KRO_REPLAY;
  kro_extras exr = {NULL, hlog, nc, cap, hlog_n, NULL};
  if (kro_integrate_ex(net, nc, n2, nc, T2, NULL, dt, 0.0, &orp, st2, NULL, &exr, 1) != 0) return 2;
  for (int c = 0; c < nc; ++c) {
    if (status[c] == 2 || hlog_n[c] > cap) continue;
    for (int s = 0; s < S; ++s)
      if (n2[(size_t)s * nc + c] != n1[(size_t)s * nc + c]) return 3;
    if (T2[c] != T1[c]) return 3;
  }
  double *resid = malloc(sizeof(double) * nc);
  kro_element_residual(net, nc, n, n1, nc, resid);

  /* the pieces, on cell 0 */
  double y[64], J[64 * 64], M[64 * 64], LU[64 * 64], b[64], xl[64], xf[64];
  int32_t p[64];
  for (int s = 0; s < S; ++s) y[s] = n[(size_t)s * nc];
  y[S] = T[0];
  kro_jacobian(net, y, J);
  kro_newton_matrix(net, y, dt[0], M);
  memcpy(LU, M, sizeof(double) * (size_t)N * N);
  for (int i = 0; i < N; ++i) b[i] = 1.0 + i;
  memcpy(xl, b, sizeof(double) * N);
  if (kro_lu_decompose(N, LU, p) == 0) kro_lu_solve(N, LU, p, xl);
  if (kro_gauss_full_pivot(N, M, b, xf) != 0) memset(xf, 0, sizeof(double) * N);
  double tau = kro_fastest_timescale(net, y);
  double *kf = malloc(sizeof(double) * (size_t)(R + 1)), *kr = malloc(sizeof(double) * (size_t)(R + 1));
  kro_rate_coeffs(net, T[0], kf, kr);
  double *par = malloc(sizeof(double) * (size_t)(6 * R + 1));
  kro_arrhenius(net, par);
  double E0[8] = {0}, post_n[64];
  for (int s = 0; s < S; ++s) post_n[s] = y[s] * (s % 2 ? 1.0 + 1e-9 : 1.0 - 1e-9);
  (void)kro_postprocess_flags(net, E0, post_n);

  FILE *g = fopen(argv[2], "wb");
  if (!g) return 1;
  fwrite(n1, sizeof(double), (size_t)S * nc, g);
  fwrite(T1, sizeof(double), (size_t)nc, g);
  fwrite(hint, sizeof(double), (size_t)nc, g);
  fwrite(resid, sizeof(double), (size_t)nc, g);
  fwrite(status, sizeof(int32_t), (size_t)nc, g);
  fwrite(stats, sizeof(int32_t), (size_t)4 * nc, g);
  fwrite(hlog_n, sizeof(int32_t), (size_t)nc, g);
  fwrite(post, sizeof(int32_t), (size_t)nc, g);
  fwrite(J, sizeof(double), (size_t)N * N, g);
  fwrite(M, sizeof(double), (size_t)N * N, g);
  fwrite(xl, sizeof(double), (size_t)N, g);
  fwrite(xf, sizeof(double), (size_t)N, g);
  fwrite(&tau, sizeof(double), 1, g);
  fwrite(kf, sizeof(double), (size_t)R, g);
  fwrite(kr, sizeof(double), (size_t)R, g);
  fclose(g);

  kro_net_destroy(net);
  free(comp); free(res); free(reac); free(prod); free(cv); free(hf); free(sf); free(af); free(ar);
  free(n); free(T); free(dt); free(n1); free(T1); free(hint); free(hlog); free(hlog_n); free(post);
  free(status); free(stats); free(n2); free(T2); free(st2); free(resid); free(kf); free(kr); free(par);
  return 0;
}
