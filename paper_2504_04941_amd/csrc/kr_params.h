/*
 * kr_params.h -- launch parameters shared by the host runtime and the
 * device code of the per-cell integrator (the device source is compiled at
 * network creation, so this struct is the one contract between the two).
 */
#ifndef KR_PARAMS_H
#define KR_PARAMS_H

struct KrParams {
  long long n_cells;
  double *states;        /* [S][ld] in/out */
  long long ld;
  double *T;             /* [n_cells] in/out */
  const double *rho;     /* [n_cells] or null */
  const double *dt;      /* [n_cells] or null */
  double dt_scalar;
  double rtol;
  double floor;          /* atol = floor * nuclei density */
  double newton_tol;
  double rho_floor;
  int max_newton;
  int max_substeps;
  int mode;              /* 0 adaptive, 1 fixed */
  int n_fixed;
  int *status;           /* [n_cells] or null */
  int *cell_stats;       /* [n_cells][4] or null */
  unsigned long long *counter; /* next unclaimed cell */
  const double *guess;   /* [S+1][guess_ld] first-substep Newton guess, or null */
  long long guess_ld;
  unsigned long long *counters; /* [8] statistics (see kr_options), or null */
  const unsigned *order;  /* [n_cells] cell handed out at each claim, or null
                             for the input order */
  double *h_hint;        /* [n_cells] in: first substep of the first attempt
                            (used when positive and finite); out: the
                            controller's proposed next length; or null */
  double *h_log;         /* [h_log_cap][h_log_ld] accepted substep lengths of
                            the attempt that produced the result, or null */
  long long h_log_ld;
  int h_log_cap;
  int *h_log_n;          /* [n_cells] number of accepted substeps logged, or null */
  unsigned long long *totals; /* [8] per-call totals (see KR_TOT_*), or null */
  const double *photo_flux;   /* [n_cells] optically thin photon flux, or null */
  const double *photo_length; /* [n_cells] path length, or null */
};

/* Per-call totals accumulated by the integrators (each wave flushes its own
 * sums once, when the queue is empty). */
enum { KR_TOT_CELLS = 0, KR_TOT_SUBSTEPS = 1, KR_TOT_ITERS = 2, KR_TOT_REJECTED = 3,
       KR_TOT_NFAIL = 4, KR_TOT_RETRIED = 5, KR_TOT_REVERTED = 6, KR_TOT_MAXRESID = 7 };

#endif
