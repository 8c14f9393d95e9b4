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
};

#endif
