/*
 * kr_lib.hip -- host runtime and C ABI of libkr.so (see include/kr.h).
 *
 *   network compiler  validates a network description (conservation of every
 *                     element/charge row, reservoir rows), derives reverse
 *                     Arrhenius parameters by detailed balance, and generates
 *                     straight-line device code for the network's rates and
 *                     analytic Jacobian (paper Sec. 2.2.1, eq.
 *                     method-jacobian); the generated code plus the
 *                     integrator template (kr_device.h) is compiled for gfx950
 *                     with hipRTC, so every matrix index is a compile-time
 *                     constant and a cell's Newton matrix stays in registers.
 *   integrate         launches the persistent per-lane integrator over all
 *                     cells (work claimed through an atomic counter).
 *   element residual  an ahead-of-time kernel for the per-cell conservation
 *                     check (Sec. 2.1, eq. method-const-elem).
 */
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/kr.h"
#include "kr_params.h"

static const char *kDeviceSource =
#include "kr_device_src.inc"
    ;
static const char *kWideSource =
#include "kr_wide_src.inc"
    ;
static const char *kGroupSource =
#include "kr_group_src.inc"
    ;
static const char *kParamsSource =
#include "kr_params_src.inc"
    ;
static const char *kMathSource =
#include "kr_math_src.inc"
    ;
static const char *kOrderSource =
#include "kr_order_src.inc"
    ;
static const char *kAdvectSource =
#include "kr_advect_src.inc"
    ;
static const char *kThermoSource =
#include "kr_thermo_src.inc"
    ;

static const double kBoltzmann = 1.380649e-16; /* erg / K */
static const int KR_ORDER_NBUCKETS = 256;       /* KR_ORDER_BUCKETS of kr_order.h */
static const int KR_MAX_DEVICES = 64;           /* devices with a scratch address slot */

/* ------------------------------------------------------------------------ */
/* errors                                                                    */
/* ------------------------------------------------------------------------ */

static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  try {
    g_err = buf;
  } catch (...) {
    /* no room for the message: the code still says what happened */
  }
  return code;
}

/* Closes the try block of every extern "C" entry point: no C++ exception
 * crosses the ABI (host containers of the network compiler and the graph
 * cache can throw std::bad_alloc). */
#define KR_CATCH                                                             \
  catch (const std::bad_alloc &) {                                           \
    return fail(KR_ENOMEM, "out of host memory");                            \
  }                                                                          \
  catch (...) {                                                              \
    return fail(KR_EDEVICE, "unexpected host exception");                    \
  }

#define HIP_TRY(expr)                                                        \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess)                                                    \
      return fail(KR_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));       \
  } while (0)

extern "C" const char *kr_last_error(void) { return g_err.c_str(); }

static int scratch_setup(int device);

/* ------------------------------------------------------------------------ */
/* network                                                                   */
/* ------------------------------------------------------------------------ */

/* Buffers of the largest-work-first cell order (kr_order.h): cell order,
 * per-cell bucket, histogram + bucket starts; grown to the largest batch. */
struct OrderBufs {
  unsigned *order = nullptr;
  unsigned char *bucket = nullptr;
  unsigned *hist = nullptr;
  long long cap = 0;
};

static void order_free(OrderBufs &b) {
  if (b.order) (void)hipFree(b.order);
  if (b.bucket) (void)hipFree(b.bucket);
  if (b.hist) (void)hipFree(b.hist);
  b = OrderBufs{};
}

struct kr_network {
  int S = 0, n_rows = 0, n_elem = 0, R = 0;
  std::vector<int32_t> comp, res, reac, prod;
  std::vector<double> cv, h, s, par; /* par: [R][2][3] */
  double p_ref = 0.0, T_min = 0.0, T_max = 0.0;
  bool explicit_rev = false;
  /* temperature-dependent heat capacities: cvp [S][2][5] (empty: constant),
   * econ [S] the upper piece's energy constant */
  std::vector<double> cvp, econ;
  double T_mid = 0.0;
  /* tabulated rate factors: tab_of [R] (empty: none), tab [n_tab][nodes] */
  std::vector<int32_t> tab_of;
  std::vector<double> tab;
  int n_tab = 0, n_nodes = 0;
  double tab_x0 = 0.0, tab_dx = 1.0;
  /* photoreactions (photo empty: none) and extra heat per event (qx empty:
   * none) */
  std::vector<double> sigma, qx;
  std::vector<int32_t> photo;
  bool has_photo = false;
  std::string source;
  hipModule_t module = nullptr;
  hipFunction_t f_fp64 = nullptr, f_fp32 = nullptr, f_reset = nullptr, f_tau = nullptr;
  hipFunction_t f_single = nullptr, f_mixed = nullptr;   /* lane layout only */
  hipFunction_t f_keys = nullptr, f_scan = nullptr, f_scatter = nullptr, f_post = nullptr, f_adv = nullptr;
  hipFunction_t f_adv2 = nullptr;    /* fused SSP-RK2 advection */
  int device = -1, cu_count = 0, occ_fp64 = 0, occ_fp32 = 0, occ_single = 0, occ_mixed = 0;
  kr_build_opts build{1, 0.1f, KR_LAYOUT_AUTO, 0};
  bool wide = false;            /* one wavefront per cell (also the lane-group layout's
                                   other kernels) */
  int group = 0;                /* lane-group layout: lanes per cell (16, 32), else 0 */
  OrderBufs ord;
  unsigned long long *d_counter = nullptr;
  unsigned long long *d_max = nullptr;
  unsigned long long *d_totals = nullptr;   /* [16]: totals (KR_TOT_*), then statistics counters */
  int32_t *d_comp = nullptr;
};

static std::string hexd(double v) {
  char b[64];
  snprintf(b, sizeof b, "%a", v);
  return b;
}

/* Validates and copies the description; derives the reverse parameters. */
static int build_tables(const kr_network_desc *d, kr_network *n) {
  if (!d) return fail(KR_EINVAL, "null description");
  const int S = d->n_species, V = d->n_rows, R = d->n_reactions;
  if (S < 1 || S > KR_MAX_SPECIES) return fail(KR_EINVAL, "n_species %d out of [1, %d]", S, KR_MAX_SPECIES);
  if (V < 0 || V > KR_MAX_ROWS) return fail(KR_EINVAL, "n_rows %d out of [0, %d]", V, KR_MAX_ROWS);
  if (d->n_elem < 0 || d->n_elem > V) return fail(KR_EINVAL, "n_elem %d out of [0, n_rows]", d->n_elem);
  if (R < 0) return fail(KR_EINVAL, "n_reactions < 0");
  if ((V && (!d->composition || !d->reservoir)) || !d->cv || !d->h_form || !d->s_form ||
      (R && (!d->reac || !d->prod || !d->arr_f)))
    return fail(KR_EINVAL, "null table in description");
  if (!(d->p_ref > 0.0) || !std::isfinite(d->p_ref)) return fail(KR_EINVAL, "p_ref must be > 0");
  if (!(d->T_min > 0.0) || !(d->T_max >= d->T_min) || !std::isfinite(d->T_max))
    return fail(KR_EINVAL, "bad temperature limits");
  n->S = S; n->n_rows = V; n->n_elem = d->n_elem; n->R = R;
  n->p_ref = d->p_ref; n->T_min = d->T_min; n->T_max = d->T_max;
  n->comp.assign(d->composition, d->composition + (size_t)V * S);
  n->res.assign(d->reservoir, d->reservoir + V);
  n->cv.assign(d->cv, d->cv + S);
  n->h.assign(d->h_form, d->h_form + S);
  n->s.assign(d->s_form, d->s_form + S);
  n->reac.assign(d->reac, d->reac + 3 * (size_t)R);
  n->prod.assign(d->prod, d->prod + 3 * (size_t)R);
  for (int i = 0; i < S; ++i)
    if (!std::isfinite(n->cv[i]) || n->cv[i] < 0.0 || !std::isfinite(n->h[i]) || !std::isfinite(n->s[i]))
      return fail(KR_EINVAL, "species %d: non-finite or negative thermodynamic data", i);
  for (int v = 0; v < V; ++v) {
    const int rs = n->res[v];
    if (rs < 0 || rs >= S || n->comp[(size_t)v * S + rs] == 0)
      return fail(KR_EINVAL, "row %d: reservoir %d does not carry the row", v, rs);
    for (int u = 0; u < V; ++u)
      if (u != v && n->comp[(size_t)u * S + rs] != 0)
        return fail(KR_EINVAL, "row %d: reservoir %d also carries row %d", v, rs, u);
  }
  n->par.assign(6 * (size_t)R, 0.0);
  for (int r = 0; r < R; ++r) {
    std::vector<int> nu(S, 0);
    for (int k = 0; k < 3; ++k) {
      const int a = n->reac[3 * r + k], b = n->prod[3 * r + k];
      if (a < -1 || a >= S || b < -1 || b >= S) return fail(KR_EINVAL, "reaction %d: species index out of range", r);
      if (a >= 0) nu[a] -= 1;
      if (b >= 0) nu[b] += 1;
    }
    for (int v = 0; v < V; ++v) {
      long t = 0;
      for (int sp = 0; sp < S; ++sp) t += (long)n->comp[(size_t)v * S + sp] * nu[sp];
      if (t != 0) return fail(KR_EINVAL, "reaction %d does not conserve row %d", r, v);
    }
    double dH = 0.0, dS = 0.0;
    int dnu = 0;
    for (int sp = 0; sp < S; ++sp) {
      dH += nu[sp] * n->h[sp];
      dS += nu[sp] * n->s[sp];
      dnu += nu[sp];
    }
    double *pf = &n->par[6 * (size_t)r], *pr = pf + 3;
    for (int k = 0; k < 3; ++k) pf[k] = d->arr_f[3 * r + k];
    if (d->arr_r) {
      for (int k = 0; k < 3; ++k) pr[k] = d->arr_r[3 * r + k];
    } else {
      /* k_r = k_f / K_eq, K_eq = (p_ref / (k_B T))^dnu exp(dS - dH/T) */
      pr[0] = pf[0] * std::pow(kBoltzmann / n->p_ref, dnu) * std::exp(-dS);
      pr[1] = pf[1] + dnu;
      pr[2] = pf[2] - dH;
    }
    for (int k = 0; k < 6; ++k)
      if (!std::isfinite(pf[k])) return fail(KR_EINVAL, "reaction %d: non-finite Arrhenius parameter", r);
    if (pf[0] < 0.0 || pr[0] < 0.0) return fail(KR_EINVAL, "reaction %d: negative pre-factor", r);
  }
  n->explicit_rev = d->arr_r != nullptr;
  if (d->cv_poly) {
    if (!(d->T_mid > 0.0) || !std::isfinite(d->T_mid)) return fail(KR_EINVAL, "T_mid must be > 0");
    n->cvp.assign(d->cv_poly, d->cv_poly + 10 * (size_t)S);
    for (double v : n->cvp)
      if (!std::isfinite(v)) return fail(KR_EINVAL, "non-finite heat-capacity coefficient");
    n->T_mid = d->T_mid;
    /* e_s(T) = sum_k a_k T^(k+1) / (k+1) on each piece; the upper piece
     * shifted by econ so that e_s is continuous at T_mid */
    auto energy = [](const double *a, long double T) {
      long double e = 0.0L, Tk = T;
      for (int k = 0; k < 5; ++k) { e += (long double)a[k] * Tk / (k + 1); Tk *= T; }
      return e;
    };
    n->econ.resize(S);
    for (int sp = 0; sp < S; ++sp)
      n->econ[sp] = (double)(energy(&n->cvp[10 * (size_t)sp], d->T_mid) - energy(&n->cvp[10 * (size_t)sp + 5], d->T_mid));
  }
  if (d->tab_of) {
    const int nt = d->n_tables, K = d->n_tab_nodes;
    if (nt < 1 || nt > std::max(R, 1) || K < 2 || K > KR_MAX_TAB_NODES || !d->tab_log2k)
      return fail(KR_EINVAL, "bad table sizes (%d tables of %d nodes)", nt, K);
    if (!(d->tab_dlog2T > 0.0) || !std::isfinite(d->tab_dlog2T) || !std::isfinite(d->tab_log2T0))
      return fail(KR_EINVAL, "bad table grid");
    n->tab_of.assign(d->tab_of, d->tab_of + R);
    for (int r = 0; r < R; ++r)
      if (n->tab_of[r] < -1 || n->tab_of[r] >= nt) return fail(KR_EINVAL, "reaction %d: table index out of range", r);
    n->tab.assign(d->tab_log2k, d->tab_log2k + (size_t)nt * K);
    for (double v : n->tab)
      if (!std::isfinite(v)) return fail(KR_EINVAL, "non-finite table value");
    n->n_tab = nt; n->n_nodes = K;
    n->tab_x0 = d->tab_log2T0; n->tab_dx = d->tab_dlog2T;
  }
  if (d->photo) {
    if (!d->sigma_abs) return fail(KR_EINVAL, "photoreactions need sigma_abs");
    n->photo.assign(d->photo, d->photo + R);
    for (int r = 0; r < R; ++r) {
      if (n->photo[r] != 0 && n->photo[r] != 1) return fail(KR_EINVAL, "reaction %d: photo flag not 0 or 1", r);
      if (n->photo[r]) {
        n->has_photo = true;
        const double *pf = &n->par[6 * (size_t)r];
        if (pf[1] != 0.0 || pf[2] != 0.0)
          return fail(KR_EINVAL, "reaction %d: a photoreaction's coefficient is A F_eff (b = E = 0)", r);
        /* no reverse direction */
        for (int k = 3; k < 6; ++k) n->par[6 * (size_t)r + k] = 0.0;
      }
    }
  }
  if (d->sigma_abs) {
    n->sigma.assign(d->sigma_abs, d->sigma_abs + S);
    for (double v : n->sigma)
      if (!(v >= 0.0) || !std::isfinite(v)) return fail(KR_EINVAL, "bad photo-absorption cross-section");
  }
  if (d->heat_extra) {
    n->qx.assign(d->heat_extra, d->heat_extra + 3 * (size_t)R);
    for (double v : n->qx)
      if (!std::isfinite(v)) return fail(KR_EINVAL, "non-finite extra heat coefficient");
  }
  return KR_OK;
}

/* One side's rate and its derivatives, as source text.  slots: species of
 * the side (multiset). */
struct SideCode {
  std::string q;                        /* q = k * prod y[slot] */
  std::vector<std::pair<int, std::string>> dq; /* (m, dq/dy_m) */
};

static SideCode side_code(const std::string &k, const int *slots) {
  SideCode c;
  std::vector<int> sl;
  for (int i = 0; i < 3; ++i)
    if (slots[i] >= 0) sl.push_back(slots[i]);
  c.q = k;
  for (int m : sl) c.q += " * y[" + std::to_string(m) + "]";
  std::vector<int> distinct;
  for (int m : sl)
    if (std::find(distinct.begin(), distinct.end(), m) == distinct.end()) distinct.push_back(m);
  for (int m : distinct) {
    /* product rule over the slots holding m */
    std::string sum;
    for (size_t i = 0; i < sl.size(); ++i) {
      if (sl[i] != m) continue;
      std::string t = k;
      for (size_t j = 0; j < sl.size(); ++j)
        if (j != i) t += " * y[" + std::to_string(sl[j]) + "]";
      sum += sum.empty() ? t : " + " + t;
    }
    c.dq.push_back({m, "(" + sum + ")"});
  }
  return c;
}

static std::string coef(int nu) {
  if (nu == 1) return "";
  if (nu == -1) return "-";
  return "R(" + std::to_string(nu) + ") * ";
}

static std::string network_tables(const kr_network *n);

/* Row stride (in doubles) of the wavefront layout's LDS Jacobian: S species
 * columns, T and f; odd, so that lanes reading their own rows spread over
 * the LDS banks. */
static int wide_ldj(int S) { return (S + 2) % 2 ? S + 2 : S + 3; }

/* Reaction directions with a nonzero rate: Arrhenius parameters, reactant
 * slots and net stoichiometry (products minus reactants). */
struct WideDir {
  double A, b, E;
  int slot[3];
  std::vector<int> nu;
  int tab;                      /* tabulated factor of the direction, or -1 */
};

static std::vector<WideDir> wide_directions(const kr_network *n) {
  std::vector<WideDir> out;
  for (int r = 0; r < n->R; ++r)
    for (int dir = 0; dir < 2; ++dir) {
      const double *pp = &n->par[6 * (size_t)r + 3 * dir];
      if (pp[0] == 0.0) continue;
      const int32_t *re = dir ? &n->prod[3 * r] : &n->reac[3 * r];
      const int32_t *pr = dir ? &n->reac[3 * r] : &n->prod[3 * r];
      const int tab = n->tab_of.empty() || (dir == 1 && n->explicit_rev) ? -1 : n->tab_of[r];
      WideDir d{pp[0], pp[1], pp[2], {re[0], re[1], re[2]}, std::vector<int>(n->S, 0), tab};
      for (int k = 0; k < 3; ++k) {
        if (re[k] >= 0) d.nu[re[k]] -= 1;
        if (pr[k] >= 0) d.nu[pr[k]] += 1;
      }
      out.push_back(d);
    }
  return out;
}

/* Contribution lists of the wavefront layout.  Each destination entry of
 * the LDS Jacobian (a list of (source in P, coefficient) terms) is owned by
 * one lane; destinations go to lanes largest-first onto the least loaded
 * lane, each lane's terms are concatenated with a flush mark on the last
 * term of every destination, and the lists are padded to equal length and
 * interleaved by lane (term i of lane l at i * 64 + l). */
static std::vector<uint32_t> wide_lists(const std::map<int, std::vector<std::pair<int, int>>> &dst, int &len,
                                        int lanes_n = 64) {
  std::vector<std::pair<int, int>> order; /* (terms, destination) */
  for (const auto &kv : dst) order.push_back({(int)kv.second.size(), kv.first});
  std::stable_sort(order.begin(), order.end(),
                   [](const std::pair<int, int> &a, const std::pair<int, int> &b) { return a.first > b.first; });
  std::vector<std::vector<uint32_t>> lanes(lanes_n);
  for (const auto &od : order) {
    int best = 0;
    for (int l = 1; l < lanes_n; ++l)
      if (lanes[l].size() < lanes[best].size()) best = l;
    const auto &terms = dst.at(od.second);
    for (size_t i = 0; i < terms.size(); ++i) {
      const uint32_t flush = i + 1 == terms.size() ? 1u : 0u;
      lanes[best].push_back((uint32_t)terms[i].first | ((uint32_t)od.second << 12) |
                            ((uint32_t)(terms[i].second + 4) << 25) | (flush << 28));
    }
  }
  len = 1;
  for (const auto &l : lanes) len = std::max(len, (int)l.size());
  len = (len + 7) / 8 * 8;   /* the gather fetches entries eight at a time */
  std::vector<uint32_t> tab((size_t)len * lanes_n, 4u << 25);
  for (int l = 0; l < lanes_n; ++l)
    for (size_t i = 0; i < lanes[l].size(); ++i) tab[i * lanes_n + l] = lanes[l][i];
  return tab;
}

static int check_wide(const kr_network *n) {
  if (n->S > 62) return fail(KR_EINVAL, "the wavefront layout takes at most 62 species (got %d)", n->S);
  if (n->has_photo || !n->qx.empty())
    return fail(KR_EINVAL, "photoreactions and extra heat terms need the lane layout");
  const size_t D = wide_directions(n).size();
  const size_t ndp = ((D + 63) / 64) * 64;
  if (5 * ndp > 4096)
    return fail(KR_EINVAL, "the wavefront layout takes at most 768 reaction directions (got %zu)", D);
  return KR_OK;
}

/* Jacobian contributions of the reaction directions: destination entry of
 * the LDS Jacobian (row stride LDJ) -> (source in the rate table P, 5
 * entries per direction; net stoichiometric coefficient), for the full
 * Jacobian and for the rates alone. */
static void wide_contributions(const kr_network *n, const std::vector<WideDir> &dirs,
                               std::map<int, std::vector<std::pair<int, int>>> &full,
                               std::map<int, std::vector<std::pair<int, int>>> &fonly) {
  const int S = n->S, LDJ = wide_ldj(S);
  for (size_t d = 0; d < dirs.size(); ++d) {
    const int src = 5 * (int)d;
    for (int s = 0; s < S; ++s) {
      const int nu = dirs[d].nu[s];
      if (!nu) continue;
      full[s * LDJ + S + 1].push_back({src, nu});
      fonly[s * LDJ + S + 1].push_back({src, nu});
      full[s * LDJ + S].push_back({src + 1, nu});
      for (int k = 0; k < 3; ++k)
        if (dirs[d].slot[k] >= 0) full[s * LDJ + dirs[d].slot[k]].push_back({src + 2 + k, nu});
    }
  }
}

/* The network-specific section of the wavefront-per-cell device source. */
static std::string generate_wide(const kr_network *n) {
  const int S = n->S, LDJ = wide_ldj(S);
  const std::vector<WideDir> dirs = wide_directions(n);
  const int NDR = std::max<int>(1, (int)((dirs.size() + 63) / 64)), NDP = NDR * 64;
  std::map<int, std::vector<std::pair<int, int>>> full, fonly;
  wide_contributions(n, dirs, full, fonly);
  int NC = 0, NF = 0;
  const std::vector<uint32_t> wc = wide_lists(full, NC), wf = wide_lists(fonly, NF);
  std::string o;
  o += "/* generated network section (one wavefront per cell): " + std::to_string(S) + " species, " +
       std::to_string(n->n_rows) + " conserved rows, " + std::to_string(dirs.size()) + " reaction directions */\n";
  o += network_tables(n);
  o += "#define KR_LDJ " + std::to_string(LDJ) + "\n#define KR_NDR " + std::to_string(NDR) +
       "\n#define KR_NC " + std::to_string(NC) + "\n#define KR_NF " + std::to_string(NF) + "\n";
  o += "__device__ static constexpr double kr_hf[" + std::to_string(S) + "] = {";
  for (int s = 0; s < S; ++s) o += hexd(n->h[s]) + (s + 1 < S ? "," : "");
  o += "};\n";
  /* per direction log2 A (-4096 for an empty slot: 2^-4096 is 0), b, C */
  const char *names[3] = {"kr_da2", "kr_db", "kr_dE"};
  for (int q = 0; q < 3; ++q) {
    o += std::string("__device__ static constexpr double ") + names[q] + "[" + std::to_string(NDP) + "] = {";
    for (int d = 0; d < NDP; ++d) {
      double v = q == 0 ? -4096.0 : 0.0;
      if (d < (int)dirs.size())
        v = q == 0 ? (dirs[d].A > 0.0 ? (double)log2l((long double)dirs[d].A) : -4096.0)
                   : (q == 1 ? dirs[d].b : dirs[d].E);
      o += hexd(v) + (d + 1 < NDP ? "," : "");
    }
    o += "};\n";
  }
  if (n->n_tab > 0) {
    o += "__device__ static constexpr int kr_dtab[" + std::to_string(NDP) + "] = {";
    for (int d = 0; d < NDP; ++d) o += std::to_string(d < (int)dirs.size() ? dirs[d].tab : -1) + (d + 1 < NDP ? "," : "");
    o += "};\n";
  }
  o += "__device__ static constexpr unsigned kr_dr[" + std::to_string(NDP) + "] = {";
  for (int d = 0; d < NDP; ++d) {
    uint32_t r = 0xFFFFFFu;
    if (d < (int)dirs.size()) {
      r = 0;
      for (int k = 0; k < 3; ++k) r |= (uint32_t)(dirs[d].slot[k] >= 0 ? dirs[d].slot[k] : 63) << (8 * k);
    }
    o += std::to_string(r) + "u" + (d + 1 < NDP ? "," : "");
  }
  o += "};\n";
  const std::pair<const char *, const std::vector<uint32_t> *> lists[2] = {{"kr_wc", &wc}, {"kr_wf", &wf}};
  for (const auto &l : lists) {
    o += std::string("__device__ static constexpr unsigned ") + l.first + "[" + std::to_string(l.second->size()) +
         "] = {";
    for (size_t i = 0; i < l.second->size(); ++i)
      o += std::to_string((*l.second)[i]) + "u" + (i + 1 < l.second->size() ? "," : "");
    o += "};\n";
  }
  return o;
}

/* The lane-group layout's section (after the wavefront layout's, whose
 * direction tables it reads): G lanes per cell, direction rounds of G, the
 * reactant slots with the empty slot at the group's spare lane G - 1, and
 * the contribution lists balanced over G lanes. */
static std::string generate_group(const kr_network *n, int G) {
  const std::vector<WideDir> dirs = wide_directions(n);
  const int GNDR = std::max<int>(1, (int)((dirs.size() + G - 1) / G));
  std::map<int, std::vector<std::pair<int, int>>> full, fonly;
  wide_contributions(n, dirs, full, fonly);
  int NC = 0, NF = 0;
  const std::vector<uint32_t> gc = wide_lists(full, NC, G), gf = wide_lists(fonly, NF, G);
  std::string o = "/* lane-group layout: " + std::to_string(G) + " lanes per cell */\n";
  o += "#define KR_G " + std::to_string(G) + "\n#define KR_GNDR " + std::to_string(GNDR) + "\n#define KR_GNC " +
       std::to_string(NC) + "\n#define KR_GNF " + std::to_string(NF) + "\n";
  o += "__device__ static constexpr unsigned kr_gdr[" + std::to_string(GNDR * G) + "] = {";
  for (int d = 0; d < GNDR * G; ++d) {
    uint32_t r = 0;
    for (int k = 0; k < 3; ++k) {
      const int sl = d < (int)dirs.size() ? dirs[d].slot[k] : -1;
      r |= (uint32_t)(sl >= 0 ? sl : G - 1) << (8 * k);
    }
    o += std::to_string(r) + "u" + (d + 1 < GNDR * G ? "," : "");
  }
  o += "};\n";
  const std::pair<const char *, const std::vector<uint32_t> *> lists[2] = {{"kr_gc", &gc}, {"kr_gf", &gf}};
  for (const auto &l : lists) {
    o += std::string("__device__ static constexpr unsigned ") + l.first + "[" + std::to_string(l.second->size()) +
         "] = {";
    for (size_t i = 0; i < l.second->size(); ++i)
      o += std::to_string((*l.second)[i]) + "u" + (i + 1 < l.second->size() ? "," : "");
    o += "};\n";
  }
  return o;
}

/* Sizes and constant tables shared by both device layouts. */
static std::string network_tables(const kr_network *n) {
  const int S = n->S, V = n->n_rows;
  std::string o;
  o += "#define KR_S " + std::to_string(S) + "\n";
  o += "#define KR_NROWS " + std::to_string(V) + "\n";
  o += "#define KR_NELEM " + std::to_string(n->n_elem) + "\n";
  const int VV = V > 0 ? V : 1;
  o += "__device__ static constexpr int kr_comp[" + std::to_string(VV) + "][" + std::to_string(S) + "] = {";
  for (int v = 0; v < VV; ++v) {
    o += "{";
    for (int s = 0; s < S; ++s) o += std::to_string(V ? n->comp[(size_t)v * S + s] : 0) + (s + 1 < S ? "," : "");
    o += "}";
    o += v + 1 < VV ? "," : "";
  }
  o += "};\n__device__ static constexpr int kr_res[" + std::to_string(VV) + "] = {";
  for (int v = 0; v < VV; ++v) o += std::to_string(V ? n->res[v] : 0) + (v + 1 < VV ? "," : "");
  o += "};\n__device__ static constexpr double kr_cv[" + std::to_string(S) + "] = {";
  for (int s = 0; s < S; ++s) o += hexd(n->cv[s]) + (s + 1 < S ? "," : "");
  o += "};\n__device__ static constexpr double kr_atoms[" + std::to_string(S) + "] = {";
  for (int s = 0; s < S; ++s) {
    int a = 0;
    for (int v = 0; v < n->n_elem; ++v) a += n->comp[(size_t)v * S + s];
    o += std::to_string(a) + ".0" + (s + 1 < S ? "," : "");
  }
  o += "};\n";
  o += "__device__ static constexpr double kr_T_min = " + hexd(n->T_min) + ";\n";
  o += "__device__ static constexpr double kr_T_max = " + hexd(n->T_max) + ";\n";
  /* temperature-dependent heat capacities: c_V coefficients and the energy's
   * (a_k / (k + 1), then the piece's constant), per species and piece */
  if (!n->cvp.empty()) {
    o += "#define KR_CV_POLY 1\n";
    o += "__device__ static constexpr double kr_T_mid = " + hexd(n->T_mid) + ";\n";
    o += "__device__ static constexpr double kr_cvp[" + std::to_string(S) + "][2][5] = {";
    std::string ev = "__device__ static constexpr double kr_evp[" + std::to_string(S) + "][2][6] = {";
    for (int sp = 0; sp < S; ++sp) {
      o += "{";
      ev += "{";
      for (int piece = 0; piece < 2; ++piece) {
        const double *a = &n->cvp[10 * (size_t)sp + 5 * piece];
        o += "{";
        ev += "{";
        for (int k = 0; k < 5; ++k) {
          o += hexd(a[k]) + (k < 4 ? "," : "");
          ev += hexd((double)((long double)a[k] / (k + 1))) + ",";
        }
        ev += hexd(piece ? n->econ[sp] : 0.0);
        o += piece ? "}" : "},";
        ev += piece ? "}" : "},";
      }
      o += sp + 1 < S ? "}," : "}";
      ev += sp + 1 < S ? "}," : "}";
    }
    o += "};\n" + ev + "};\n";
  }
  /* tabulated rate factors: log2 values at nodes uniform in log2 T */
  if (n->n_tab > 0) {
    o += "#define KR_NTAB " + std::to_string(n->n_tab) + "\n#define KR_TAB_NODES " + std::to_string(n->n_nodes) + "\n";
    o += "__device__ static constexpr double kr_tab_x0 = " + hexd(n->tab_x0) + ";\n";
    o += "__device__ static constexpr double kr_tab_idx = " + hexd((double)(1.0L / (long double)n->tab_dx)) + ";\n";
    o += "__device__ static constexpr double kr_tab[" + std::to_string(n->n_tab) + "][" + std::to_string(n->n_nodes) + "] = {";
    for (int t = 0; t < n->n_tab; ++t) {
      o += "{";
      for (int i = 0; i < n->n_nodes; ++i) o += hexd(n->tab[(size_t)t * n->n_nodes + i]) + (i + 1 < n->n_nodes ? "," : "");
      o += t + 1 < n->n_tab ? "}," : "}";
    }
    o += "};\n";
  } else {
    o += "#define KR_NTAB 0\n";
  }
  if (n->has_photo) {
    o += "#define KR_PHOTO 1\n";
  }
  o += kThermoSource;
  o += "\n";
  /* projector onto the stoichiometric space, the null space of the
   * element-species matrix (Sec. 2.1: P = V V^T), as I - Q^T Q with Q an
   * orthonormal basis of the conserved rows' span (modified Gram-Schmidt,
   * twice, in extended precision; dependent rows are skipped) */
  std::vector<std::vector<long double>> Q;
  for (int v = 0; v < V; ++v) {
    std::vector<long double> w(S);
    long double nrm0 = 0.0L;
    for (int k = 0; k < S; ++k) {
      w[k] = (long double)n->comp[(size_t)v * S + k];
      nrm0 += w[k] * w[k];
    }
    for (int pass = 0; pass < 2; ++pass)
      for (const auto &q : Q) {
        long double d = 0.0L;
        for (int k = 0; k < S; ++k) d += q[k] * w[k];
        for (int k = 0; k < S; ++k) w[k] -= d * q[k];
      }
    long double nrm = 0.0L;
    for (int k = 0; k < S; ++k) nrm += w[k] * w[k];
    if (!(nrm > 1e-24L * nrm0) || nrm0 == 0.0L) continue;
    nrm = sqrtl(nrm);
    for (int k = 0; k < S; ++k) w[k] /= nrm;
    Q.push_back(w);
  }
  o += "__device__ static constexpr double kr_proj[" + std::to_string(S) + "][" + std::to_string(S) + "] = {";
  for (int i = 0; i < S; ++i) {
    o += "{";
    for (int j = 0; j < S; ++j) {
      long double pij = i == j ? 1.0L : 0.0L;
      for (const auto &q : Q) pij -= q[i] * q[j];
      o += hexd((double)pij) + (j + 1 < S ? "," : "");
    }
    o += i + 1 < S ? "}," : "}";
  }
  o += "};\n";
  /* the same projector in low-rank form, P chi = chi - Q^T (Q chi): the
   * basis rows themselves (a zero row when there is none) */
  const int R = (int)Q.size();
  o += "#define KR_PROJ_R " + std::to_string(R) + "\n";
  o += "__device__ static constexpr double kr_projq[" + std::to_string(R > 0 ? R : 1) + "][" + std::to_string(S) +
       "] = {";
  for (int r = 0; r < (R > 0 ? R : 1); ++r) {
    o += "{";
    for (int j = 0; j < S; ++j) o += hexd(R > 0 ? (double)Q[r][j] : 0.0) + (j + 1 < S ? "," : "");
    o += r + 1 < (R > 0 ? R : 1) ? "}," : "}";
  }
  o += "};\n";
  return o;
}

/* k = A T^b exp(-C/T) as 2^(log2 A + b log2 T - C log2(e) / T) (kr_math.h):
 * the generated code holds log2 A and C log2(e), rounded once from extended
 * precision; l2T and iT are the evaluation point's log2 T and 1/T. */
/* A constant of the working precision R of the generated code. */
static std::string lit(double v) { return "R(" + hexd(v) + ")"; }

/* extra: the name of a log2 factor to add to the exponent (a tabulated
 * factor), or empty. */
static std::string arrhenius_code(const double *abc, const std::string &extra = "") {
  const long double log2e = 1.4426950408889634073599246810018921L;
  const double a2 = (double)log2l((long double)abc[0]);
  const double b = abc[1];
  const double c2 = (double)((long double)abc[2] * log2e);
  if (b == 0.0 && c2 == 0.0 && extra.empty()) return lit(abc[0]);
  std::string x = lit(a2);
  if (!extra.empty()) x = "(" + x + " + " + extra + ")";
  if (b != 0.0) x = "fma(" + lit(b) + ", l2T, " + x + ")";
  if (c2 != 0.0) x = "fma(" + lit(-c2) + ", iT, " + x + ")";
  return "kr_exp2(" + x + ")";
}

/* FP32 overloads of the base-2 exponential and logarithm for the single- and
 * mixed-precision modes (the hardware's instructions).  They sit at global
 * scope beside the FP64 ones of kr_math.h: inside a network's namespace of a
 * several-network source they would hide the FP64 overloads, and FP64
 * arguments would silently round to FP32. */
static const char kFloatMathSource[] =
    "__device__ __forceinline__ float kr_exp2(float x) { return __builtin_amdgcn_exp2f(x); }\n"
    "__device__ __forceinline__ float kr_log2(float x) { return __builtin_amdgcn_logf(x); }\n";

/* The network-specific section of the lane-per-cell device source. */
static std::string generate_network(const kr_network *n) {
  const int S = n->S, V = n->n_rows;
  std::string o;
  o += "/* generated network section: " + std::to_string(S) + " species, " + std::to_string(V) +
       " conserved rows, " + std::to_string(n->R) + " reactions */\n";
  o += network_tables(n);

  /* rates and analytic Jacobian, one block per reaction, in the working
   * precision R (FP64; FP32 for the single- and mixed-precision modes, whose
   * exp2 and log2 are the hardware's: kFloatMathSource) */
  o += "template <typename R>\n"
       "__device__ __forceinline__ void kr_eval(const R (&y)[KR_S + 1], R (&g)[KR_S + 1],\n"
       "                                        R (&J)[KR_S + 1][KR_S + 1], R phF = R(0), R phL = R(0)) {\n"
       "#pragma unroll\n  for (int i = 0; i <= KR_S; ++i) {\n    g[i] = R(0);\n"
       "#pragma unroll\n    for (int j = 0; j <= KR_S; ++j) J[i][j] = R(0);\n  }\n"
       "  const R T = y[KR_S];\n  const R l2T = kr_log2(T);\n  const R iT = R(1) / T;\n";
  const std::string ST = std::to_string(S);
  /* photoreactions: the cell's inverse absorption length, the effective
   * flux and its derivative, and the dominant-absorber cutoff per absorber */
  if (n->has_photo) {
    std::string li;
    for (int s = 0; s < S; ++s)
      if (n->sigma[s] > 0.0) li += (li.empty() ? "" : " + ") + lit(n->sigma[s]) + " * y[" + std::to_string(s) + "]";
    o += "  const R linv = " + (li.empty() ? std::string("R(0)") : li) + ";\n";
    o += "  R Fe, dFe;\n  kr_photo_flux(phF, phL, linv, Fe, dFe);\n";
    for (int s = 0; s < S; ++s)
      if (n->sigma[s] > 0.0)
        o += "  const R cut" + std::to_string(s) + " = linv > R(0) ? fmin(R(1), y[" + std::to_string(s) + "] * " +
             lit(n->sigma[s]) + " / linv) : R(1);\n";
  } else {
    o += "  (void)phF;\n  (void)phL;\n";
  }
  if (!n->qx.empty()) o += "  const R lnT = l2T * " + lit(0.69314718055994530942) + ";\n";
  for (int r = 0; r < n->R; ++r) {
    const double *pf = &n->par[6 * (size_t)r], *pr = pf + 3;
    std::vector<int> nu(S, 0);
    for (int k = 0; k < 3; ++k) {
      if (n->reac[3 * r + k] >= 0) nu[n->reac[3 * r + k]] -= 1;
      if (n->prod[3 * r + k] >= 0) nu[n->prod[3 * r + k]] += 1;
    }
    double dH = 0.0;
    for (int s = 0; s < S; ++s) dH += nu[s] * n->h[s];
    const double qhat = -dH;
    o += "  { /* reaction " + std::to_string(r) + " */\n";
    /* a tabulated factor (both directions with detailed-balance reverse
     * rates, the forward one only otherwise): its log2 joins the exponent,
     * its log-log slope the temperature derivative */
    const int tab = n->tab_of.empty() ? -1 : n->tab_of[r];
    if (tab >= 0) o += "    R st;\n    const R lt = kr_tab_log2(" + std::to_string(tab) + ", l2T, st);\n";
    std::vector<std::pair<int, std::string>> dw; /* dw/dy_m terms */
    std::string w, dwdT;
    for (int dir = 0; dir < 2; ++dir) {
      const double *pp = dir ? pr : pf;
      if (pp[0] == 0.0) continue;
      const bool tabbed = tab >= 0 && (dir == 0 || !n->explicit_rev);
      const bool ph = dir == 0 && !n->photo.empty() && n->photo[r];
      const std::string k = dir ? "kr" : "kf";
      if (ph)
        o += "    const R kf = " + lit(pp[0]) + " * Fe;\n";
      else
        o += "    const R " + k + " = " + arrhenius_code(pp, tabbed ? "lt" : "") + ";\n";
      SideCode c = side_code(k, dir ? &n->prod[3 * r] : &n->reac[3 * r]);
      const std::string q = dir ? "qr" : "qf";
      o += "    const R " + q + " = " + c.q + ";\n";
      o += "    const R " + q + "T = " + q + " * (" + lit(pp[1]) + (tabbed ? " + st" : "") + " + " + lit(pp[2]) +
           " * iT) * iT;\n";
      w += (dir ? " - " : (w.empty() ? "" : " + ")) + q;
      dwdT += (dir ? " - " : (dwdT.empty() ? "" : " + ")) + q + "T";
      for (auto &t : c.dq) {
        auto it = std::find_if(dw.begin(), dw.end(), [&](const std::pair<int, std::string> &e) { return e.first == t.first; });
        const std::string term = (dir ? " - " : " + ") + t.second;
        if (it == dw.end()) dw.push_back({t.first, term});
        else it->second += term;
      }
      if (ph) {
        /* the coefficient's own dependence on the absorbers, with the
         * dominant-absorber cutoff */
        o += "    const R kpd = " + lit(pp[0]) + " * dFe;\n";
        const std::string pq = side_code("kpd", &n->reac[3 * r]).q;
        for (int m = 0; m < S; ++m) {
          if (!(n->sigma[m] > 0.0)) continue;
          const std::string term = " + " + pq + " * " + lit(n->sigma[m]) + " * cut" + std::to_string(m);
          auto it = std::find_if(dw.begin(), dw.end(), [&](const std::pair<int, std::string> &e) { return e.first == m; });
          if (it == dw.end()) dw.push_back({m, term});
          else it->second += term;
        }
      }
    }
    if (w.empty()) { o += "  }\n"; continue; }
    if (w[0] == ' ') w = "R(0)" + w;
    if (dwdT[0] == ' ') dwdT = "R(0)" + dwdT;
    o += "    const R w = " + w + ";\n";
    o += "    const R wT = " + dwdT + ";\n";
    for (auto &t : dw) o += "    const R w" + std::to_string(t.first) + " = R(0)" + t.second + ";\n";
    for (int s = 0; s < S; ++s) {
      if (!nu[s]) continue;
      const std::string c = coef(nu[s]), ss = std::to_string(s);
      o += "    g[" + ss + "] += " + c + "w;\n";
      for (auto &t : dw) o += "    J[" + ss + "][" + std::to_string(t.first) + "] += " + c + "w" + std::to_string(t.first) + ";\n";
      o += "    J[" + ss + "][" + ST + "] += " + c + "wT;\n";
    }
    const double *qx = n->qx.empty() ? nullptr : &n->qx[3 * (size_t)r];
    if (qx && (qx[0] != 0.0 || qx[1] != 0.0 || qx[2] != 0.0)) {
      /* heat per event: -dH plus the extra q0 + q1 T + q2 T ln T */
      o += "    const R qx = " + lit(qhat + qx[0]) + " + T * (" + lit(qx[1]) + " + " + lit(qx[2]) + " * lnT);\n";
      o += "    const R dqx = " + lit(qx[1]) + " + " + lit(qx[2]) + " * (lnT + R(1));\n";
      o += "    g[" + ST + "] += qx * w;\n";
      for (auto &t : dw) o += "    J[" + ST + "][" + std::to_string(t.first) + "] += qx * w" + std::to_string(t.first) + ";\n";
      o += "    J[" + ST + "][" + ST + "] += qx * wT + dqx * w;\n";
    } else if (qhat != 0.0) {
      const std::string qh = lit(qhat);
      o += "    g[" + ST + "] += " + qh + " * w;\n";
      for (auto &t : dw) o += "    J[" + ST + "][" + std::to_string(t.first) + "] += " + qh + " * w" + std::to_string(t.first) + ";\n";
      o += "    J[" + ST + "][" + ST + "] += " + qh + " * wT;\n";
    }
    o += "  }\n";
  }
  o += "}\n";
  return o;
}

static int compile_source(const std::string &src, std::vector<char> &code, std::string &log) {
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "kr_network.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
    return fail(KR_ECOMPILE, "hiprtcCreateProgram failed");
  /* Machine-level loop-invariant code motion is off: it would hoist every
   * FP64 constant of the rate and exp/log code out of the persistent loop
   * and spill them (hundreds of registers for a 10-unknown network). */
  const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                        "-mllvm", "-disable-machine-licm"};
  hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
  size_t ls = 0;
  hiprtcGetProgramLogSize(prog, &ls);
  log.assign(ls + 1, '\0');
  if (ls) hiprtcGetProgramLog(prog, &log[0]);
  if (rc != HIPRTC_SUCCESS) {
    hiprtcDestroyProgram(&prog);
    return fail(KR_ECOMPILE, "hipRTC compile failed: %.900s", log.c_str());
  }
  size_t cs = 0;
  hiprtcGetCodeSize(prog, &cs);
  code.resize(cs);
  hiprtcGetCode(prog, code.data());
  hiprtcDestroyProgram(&prog);
  return KR_OK;
}

/* Occupancy target of the integrator kernels (waves per SIMD the compiler
 * budgets registers for); 0 = chosen per network by auto_waves_per_eu.
 * KR_WAVES_PER_EU in the environment overrides (tuning experiments). */
static int default_waves_per_eu() {
  if (const char *e = getenv("KR_WAVES_PER_EU")) {
    const int w = atoi(e);
    if (w >= 0 && w <= 8) return w;
  }
  return 0;
}

extern "C" void kr_default_build_options(kr_build_opts *o) {
  try {
    if (!o) return;
    o->waves_per_eu = default_waves_per_eu();
    o->pivot_tau = 0.1f;
    o->layout = KR_LAYOUT_AUTO;
    o->lu_mfma = 0;
  } catch (...) {
  }
}

static int check_build_options(const kr_build_opts *o) {
  if (o->waves_per_eu < 0 || o->waves_per_eu > 8) return fail(KR_EINVAL, "waves_per_eu out of [0, 8]");
  if (!(o->pivot_tau > 0.0f && o->pivot_tau <= 1.0f)) return fail(KR_EINVAL, "pivot_tau out of (0, 1]");
  if (o->layout < KR_LAYOUT_AUTO || o->layout > KR_LAYOUT_GROUP32) return fail(KR_EINVAL, "layout out of [0, 4]");
  if (o->lu_mfma != 0 && o->lu_mfma != 1) return fail(KR_EINVAL, "lu_mfma must be 0 or 1");
  return KR_OK;
}

static std::string build_prefix(int waves_per_eu, const kr_build_opts &o) {
  char b[160];
  snprintf(b, sizeof b, "#define KR_WAVES_PER_EU %d\n#define KR_PIVOT_TAU %a\n", waves_per_eu,
           (double)o.pivot_tau);
  return b;
}

/* The blocked FP32 LU with MFMA trailing updates (kr_wide.h) applies to a
 * wavefront-layout network of N = S + 1 >= 32 unknowns whose panel blocks
 * (panels of KR_PF, then 16 columns) fit into its rate table's LDS. */
static bool lu_mfma_fits(int S, int n_dirs) {
  const int N = S + 1;
  if (N < 32) return false;
  const int PF = N - 16 * ((N - 1) / 16), KP = (PF + 3) / 4 * 4, W = N - PF;
  const long ndp = 64L * std::max(1, (n_dirs + 63) / 64);
  const long need = std::max(4L * (64 * KP + KP * W + 64 * W), 4L * (64 * 16 + 80 * (W - 16)));
  return need <= 5 * ndp * 8;
}

/* Lanes per cell of the lane-group layout the options select, else 0.  The
 * automatic choice takes 32-lane groups from KR_WIDE_MIN_SPECIES species up
 * to the 30 a group holds (measured on the 23-species network: 15 % faster
 * than one cell per wavefront in FP64, 8 % with the FP32 LU). */
/* Photoreactions and extra heat terms exist in the lane layout only: the
 * automatic choice keeps such networks there at any size. */
static bool lane_only(const kr_network *n) { return n->has_photo || !n->qx.empty(); }

static int group_lanes(const kr_network *n, const kr_build_opts &o) {
  if (o.layout == KR_LAYOUT_AUTO)
    return !lane_only(n) && n->S >= KR_WIDE_MIN_SPECIES && n->S + 2 <= 32 ? 32 : 0;
  return o.layout == KR_LAYOUT_GROUP16 ? 16 : (o.layout == KR_LAYOUT_GROUP32 ? 32 : 0);
}

static bool use_wide(const kr_network *n, const kr_build_opts &o) {
  return o.layout == KR_LAYOUT_WAVE || group_lanes(n, o) > 0 ||
         (o.layout == KR_LAYOUT_AUTO && !lane_only(n) && n->S >= KR_WIDE_MIN_SPECIES);
}

/* The lane-group layout holds a cell's N = S + 1 rows on G lanes with one
 * lane to spare (the empty reactant slot and the energy row's last column). */
static int check_group(const kr_network *n, int G) {
  if (n->S + 2 > G)
    return fail(KR_EINVAL, "the %d-lane group layout takes at most %d species (got %d)", G, G - 2, n->S);
  return KR_OK;
}

/* LDS of one lane-group block (KrGBlock), bytes */
static int group_block_bytes(const kr_network *n, int G) {
  const int gndr = std::max<int>(1, (int)((wide_directions(n).size() + G - 1) / G));
  return 8 * (G + 5 * gndr * G + (n->S + 1) * wide_ldj(n->S));
}

/* Automatic occupancy target of one network's integrator.  Lane layout: one
 * wave; from ~8 unknowns the lane's FP64 Newton matrix alone needs most of
 * 256 VGPRs, and even at 6 unknowns a two-wave budget forces scratch spills
 * that cost more than the extra wave hides (measured: 390 vs 490 ms on 2^18
 * five-species cells).  Wavefront layout: the matrix lives in LDS and the
 * kernel is latency bound, so a second wave per SIMD pays wherever the LDS
 * block (the KrWave struct) leaves room for it, even at the cost of a few
 * spilled registers (measured on 2^20 23-species cells: 70 vs 105 ms FP64,
 * 88 vs 138 ms with the FP32 LU); the 48-species block (39 KB) allows one
 * wave per SIMD only. */
static int wide_block_bytes(const kr_network *n) {
  const int ldj = wide_ldj(n->S), ndp = 64 * std::max<int>(1, (int)((wide_directions(n).size() + 63) / 64));
  return 8 * (64 + 64 + 5 * ndp + (n->S + 1) * ldj + 64);
}

static int auto_waves_per_eu(const kr_network *n, const kr_build_opts &o) {
  if (o.waves_per_eu > 0) return o.waves_per_eu;
  if (!use_wide(n, o)) return 1;
  if (const int G = group_lanes(n, o)) {
    const int per_simd = 160 * 1024 / 4 / ((64 / G) * group_block_bytes(n, G));
    return std::max(1, std::min(2, per_simd));
  }
  const int per_simd = 160 * 1024 / 4 / wide_block_bytes(n);
  return std::max(1, std::min(2, per_simd));
}

/* "#define KR_LU_MFMA 1" when the build asks for the blocked FP32 LU and it
 * applies to this (wavefront-layout) network, else empty. */
static std::string lu_mfma_define(const kr_network *n, const kr_build_opts &o) {
  if (!o.lu_mfma || !lu_mfma_fits(n->S, (int)wide_directions(n).size())) return "";
  return "#define KR_LU_MFMA 1 /* FP32 LU with MFMA trailing updates */\n";
}

static std::string full_source(const kr_network *n, const kr_build_opts &o) {
  const int w = auto_waves_per_eu(n, o);
  if (const int G = group_lanes(n, o))
    return std::string("/* per-cell implicit thermochemistry, one cell per lane group */\n") + build_prefix(w, o) +
           kParamsSource + "\n" + kMathSource + "\n" + kOrderSource + "\n" + generate_wide(n) + "\n" +
           generate_group(n, G) + "#define KR_NO_KERNELS\n" + kWideSource + "\n#undef KR_NO_KERNELS\n" +
           kGroupSource + "\n" + kAdvectSource;
  if (use_wide(n, o))
    return std::string("/* per-cell implicit thermochemistry, one wavefront per cell */\n") + build_prefix(w, o) +
           kParamsSource + "\n" + kMathSource + "\n" + kOrderSource + "\n" + lu_mfma_define(n, o) +
           generate_wide(n) + "\n" + kWideSource + "\n" + kAdvectSource;
  return std::string("/* per-cell implicit thermochemistry: network-specialised device code */\n") +
         build_prefix(w, o) + kParamsSource + "\n" + kMathSource + "\n" + kFloatMathSource + kOrderSource + "\n" +
         generate_network(n) + "\n" +
         kDeviceSource +
         "\n" + kAdvectSource;
}

static void release(kr_network *n) {
  if (!n) return;
  order_free(n->ord);
  if (n->d_counter) (void)hipFree(n->d_counter);
  if (n->d_max) (void)hipFree(n->d_max);
  if (n->d_totals) (void)hipFree(n->d_totals);
  if (n->d_comp) (void)hipFree(n->d_comp);
  if (n->module) (void)hipModuleUnload(n->module);
  delete n;
}

extern "C" int kr_network_create_ex(const kr_network_desc *desc, const kr_build_opts *bopt,
                                    kr_network **out) {
  try {
    if (!out) return fail(KR_EINVAL, "null output handle");
    *out = nullptr;
    kr_build_opts bo;
    kr_default_build_options(&bo);
    if (bopt) bo = *bopt;
    int rc = check_build_options(&bo);
    if (rc != KR_OK) return rc;
    kr_network *n = new (std::nothrow) kr_network;
    if (!n) return fail(KR_ENOMEM, "out of host memory");
    rc = build_tables(desc, n);
    if (rc != KR_OK) { delete n; return rc; }
    n->build = bo;
    n->build.waves_per_eu = auto_waves_per_eu(n, bo);
    n->wide = use_wide(n, bo);
    n->group = group_lanes(n, bo);
    if (n->wide && (rc = check_wide(n)) != KR_OK) { delete n; return rc; }
    if (n->group && (rc = check_group(n, n->group)) != KR_OK) { delete n; return rc; }
    n->source = full_source(n, bo);
    std::vector<char> code;
    std::string log;
    rc = compile_source(n->source, code, log);
    if (rc != KR_OK) { delete n; return rc; }
    hipError_t e;
  #define CREATE_TRY(expr)                                                              \
    do {                                                                                \
      e = (expr);                                                                       \
      if (e != hipSuccess) {                                                            \
        rc = fail(KR_EDEVICE, "%s: %s", #expr, hipGetErrorString(e));                   \
        release(n);                                                                     \
        return rc;                                                                      \
      }                                                                                 \
    } while (0)
    CREATE_TRY(hipGetDevice(&n->device));
    if ((rc = scratch_setup(n->device)) != KR_OK) {
      release(n);
      return rc;
    }
    CREATE_TRY(hipDeviceGetAttribute(&n->cu_count, hipDeviceAttributeMultiprocessorCount, n->device));
    CREATE_TRY(hipModuleLoadData(&n->module, code.data()));
    CREATE_TRY(hipModuleGetFunction(&n->f_fp64, n->module, "kr_integrate_fp64"));
    CREATE_TRY(hipModuleGetFunction(&n->f_fp32, n->module, "kr_integrate_fp32lu"));
    CREATE_TRY(hipModuleGetFunction(&n->f_reset, n->module, "kr_reset_counter"));
    CREATE_TRY(hipModuleGetFunction(&n->f_tau, n->module, "kr_timescale"));
    CREATE_TRY(hipModuleGetFunction(&n->f_keys, n->module, "kr_order_keys"));
    CREATE_TRY(hipModuleGetFunction(&n->f_scan, n->module, "kr_order_scan"));
    CREATE_TRY(hipModuleGetFunction(&n->f_scatter, n->module, "kr_order_scatter"));
    CREATE_TRY(hipModuleGetFunction(&n->f_post, n->module, "kr_post"));
    CREATE_TRY(hipModuleGetFunction(&n->f_adv, n->module, "kr_advect"));
    CREATE_TRY(hipModuleGetFunction(&n->f_adv2, n->module, "kr_advect2"));
    CREATE_TRY(hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&n->occ_fp64, n->f_fp64, 64, 0));
    CREATE_TRY(hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&n->occ_fp32, n->f_fp32, 64, 0));
    if (!n->wide) {
      CREATE_TRY(hipModuleGetFunction(&n->f_single, n->module, "kr_integrate_single"));
      CREATE_TRY(hipModuleGetFunction(&n->f_mixed, n->module, "kr_integrate_mixed"));
      CREATE_TRY(hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&n->occ_single, n->f_single, 64, 0));
      CREATE_TRY(hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&n->occ_mixed, n->f_mixed, 64, 0));
    }
    CREATE_TRY(hipMalloc(&n->d_counter, 2 * sizeof(unsigned long long)));
    CREATE_TRY(hipMalloc(&n->d_max, sizeof(unsigned long long)));
    CREATE_TRY(hipMalloc(&n->d_totals, 16 * sizeof(unsigned long long)));
    const size_t cb = sizeof(int32_t) * (n->comp.size() ? n->comp.size() : 1);
    CREATE_TRY(hipMalloc(&n->d_comp, cb));
    if (!n->comp.empty())
      CREATE_TRY(hipMemcpy(n->d_comp, n->comp.data(), sizeof(int32_t) * n->comp.size(), hipMemcpyHostToDevice));
  #undef CREATE_TRY
    *out = n;
    return KR_OK;
  } KR_CATCH
}

extern "C" int kr_network_create(const kr_network_desc *desc, kr_network **out) {
  try {
    return kr_network_create_ex(desc, nullptr, out);
  } KR_CATCH
}

extern "C" void kr_network_destroy(kr_network *net) {
  try {
    release(net);
  } catch (...) {
  }
}

extern "C" int kr_network_unknowns(const kr_network *net) {
  try {
    return net ? net->S + 1 : KR_EINVAL;
  } KR_CATCH
}

extern "C" int kr_network_layout(const kr_network *net) {
  try {
    if (!net) return KR_EINVAL;
    if (net->group) return net->group == 16 ? KR_LAYOUT_GROUP16 : KR_LAYOUT_GROUP32;
    return net->wide ? KR_LAYOUT_WAVE : KR_LAYOUT_LANE;
  } KR_CATCH
}

extern "C" int kr_network_arrhenius(const kr_network *net, double *out) {
  try {
    if (!net || !out) return fail(KR_EINVAL, "null argument");
    std::memcpy(out, net->par.data(), sizeof(double) * net->par.size());
    return KR_OK;
  } KR_CATCH
}

extern "C" int64_t kr_network_source(const kr_network *net, char *buf, int64_t buf_len) {
  try {
    if (!net) return fail(KR_EINVAL, "null network");
    const int64_t need = (int64_t)net->source.size() + 1;
    if (buf && buf_len > 0) {
      const int64_t m = buf_len < need ? buf_len - 1 : need - 1;
      std::memcpy(buf, net->source.data(), (size_t)m);
      buf[m] = '\0';
    }
    return need;
  } KR_CATCH
}

/* Validation and code generation (and optionally the hipRTC compile) of a
 * description without touching a device: used by build checks and tests on
 * hosts without a GPU.  Returns KR_OK or the error create would return. */
extern "C" int kr_network_check_ex(const kr_network_desc *desc, const kr_build_opts *bopt, int compile,
                                   char *src_buf, int64_t src_len) {
  try {
    kr_network n;
    int rc = build_tables(desc, &n);
    if (rc != KR_OK) return rc;
    kr_build_opts bo;
    kr_default_build_options(&bo);
    if (bopt) bo = *bopt;
    if ((rc = check_build_options(&bo)) != KR_OK) return rc;
    if (use_wide(&n, bo) && (rc = check_wide(&n)) != KR_OK) return rc;
    if (group_lanes(&n, bo) && (rc = check_group(&n, group_lanes(&n, bo))) != KR_OK) return rc;
    const std::string src = full_source(&n, bo);
    if (src_buf && src_len > 0) {
      const size_t m = std::min<size_t>((size_t)src_len - 1, src.size());
      std::memcpy(src_buf, src.data(), m);
      src_buf[m] = '\0';
    }
    if (!compile) return KR_OK;
    std::vector<char> code;
    std::string log;
    return compile_source(src, code, log);
  } KR_CATCH
}

extern "C" int kr_network_check(const kr_network_desc *desc, int compile, char *src_buf,
                                int64_t src_len) {
  try {
    return kr_network_check_ex(desc, nullptr, compile, src_buf, src_len);
  } KR_CATCH
}

/* ------------------------------------------------------------------------ */
/* integration                                                               */
/* ------------------------------------------------------------------------ */

/* Room for a batch of n cells (allocation synchronises the device, so the
 * first call with a larger batch is not graph-capturable; callers reserve
 * before capturing). */
static int order_reserve(OrderBufs &b, long long n) {
  if (n <= b.cap) return KR_OK;
  HIP_TRY(hipDeviceSynchronize());
  if (b.order) (void)hipFree(b.order);
  if (b.bucket) (void)hipFree(b.bucket);
  b.order = nullptr;
  b.bucket = nullptr;
  b.cap = 0;
  if (hipMalloc(&b.order, (size_t)n * sizeof(unsigned)) != hipSuccess ||
      hipMalloc(&b.bucket, (size_t)n) != hipSuccess ||
      (!b.hist && hipMalloc(&b.hist, 2 * KR_ORDER_NBUCKETS * sizeof(unsigned)) != hipSuccess)) {
    order_free(b);
    return fail(KR_ENOMEM, "cell-order scratch for %lld cells", n);
  }
  HIP_TRY(hipMemset(b.hist, 0, 2 * KR_ORDER_NBUCKETS * sizeof(unsigned)));
  b.cap = n;
  return KR_OK;
}

/* Largest-expected-work-first order of the batch in p (kr_order.h): key
 * kernel -> scan -> scatter on stream st; sets p.order.  The buffers must
 * hold p.n_cells (order_reserve).  The histogram is cleared by the scan
 * kernel itself, so the sequence can be captured into a graph. */
static int order_launch(hipFunction_t keys, hipFunction_t scan, hipFunction_t scatter, const OrderBufs &b,
                        bool wide, int cu_count, KrParams &p, hipStream_t st) {
  const long long n = p.n_cells;
  unsigned *hist = b.hist, *start = b.hist + KR_ORDER_NBUCKETS;
  unsigned char *bucket = b.bucket;
  unsigned *order = b.order;
  const long long grid = (long long)cu_count * 8;
  const long long kb = wide ? std::min<long long>(n, grid) : std::min<long long>((n + 63) / 64, grid);
  p.order = nullptr;
  void *kargs[] = {&p, &bucket, &hist};
  HIP_TRY(hipModuleLaunchKernel(keys, (unsigned)kb, 1, 1, 64, 1, 1, 0, st, kargs, nullptr));
  void *sargs[] = {&hist, &start};
  HIP_TRY(hipModuleLaunchKernel(scan, 1, 1, 1, 64, 1, 1, 0, st, sargs, nullptr));
  long long nn = n;
  const long long cb = std::min<long long>((n + 63) / 64, grid);
  void *cargs[] = {&nn, &bucket, &start, &order};
  HIP_TRY(hipModuleLaunchKernel(scatter, (unsigned)cb, 1, 1, 64, 1, 1, 0, st, cargs, nullptr));
  p.order = order;
  return KR_OK;
}

__global__ void kr_zero_u64n(unsigned long long *p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0ull;
}

__global__ void kr_add_u64n(unsigned long long *dst, const unsigned long long *src, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] += src[i];
}

/* Copies a call's totals block ([0..7] KR_TOT_*, [8..15] its statistics
 * counters) into *out, adds the counters to the caller's own (if any) and
 * synchronises the stream. */
static int finish_stats(const unsigned long long *block, unsigned long long *caller_counters, kr_stats *out,
                        hipStream_t st) {
  if (caller_counters) {
    hipLaunchKernelGGL(kr_add_u64n, dim3(1), dim3(64), 0, st, caller_counters, block + 8, 8);
    HIP_TRY(hipGetLastError());
  }
  unsigned long long h[16];
  HIP_TRY(hipMemcpyAsync(h, block, sizeof h, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  out->cells = (int64_t)h[KR_TOT_CELLS];
  out->substeps = (int64_t)h[KR_TOT_SUBSTEPS];
  out->newton_iterations = (int64_t)h[KR_TOT_ITERS];
  out->rejected = (int64_t)h[KR_TOT_REJECTED];
  out->newton_failures = (int64_t)h[KR_TOT_NFAIL];
  out->retried = (int64_t)h[KR_TOT_RETRIED];
  out->reverted = (int64_t)h[KR_TOT_REVERTED];
  out->refinement_sweeps = (int64_t)h[8 + 3];
  out->fp64_fallbacks = (int64_t)h[8 + 4];
  out->guess_fallbacks = (int64_t)h[8 + 1];
  std::memcpy(&out->max_element_residual, &h[KR_TOT_MAXRESID], sizeof(double));
  return KR_OK;
}

static bool want_order(const kr_options &o, long long n) {
  return o.order == KR_ORDER_WORK && n > 1 && n <= 0xFFFFFFFFll;
}

extern "C" void kr_default_options(kr_options *o) {
  try {
    if (!o) return;
    o->precision = KR_FP64;
    o->mode = KR_ADAPTIVE;
    o->n_fixed = 1;
    o->max_newton = 10;
    o->max_substeps = 100000;
    o->order = KR_ORDER_INPUT;
    o->floor = 1e-20;
    o->newton_tol = 1e-3;
    o->rho_floor = 0.0;
    o->guess = nullptr;
    o->guess_ld = 0;
    o->counters = nullptr;
    o->h_hint = nullptr;
    o->h_log = nullptr;
    o->h_log_ld = 0;
    o->h_log_cap = 0;
    o->reserved = 0;
    o->h_log_n = nullptr;
    o->stats = nullptr;
  } catch (...) {
  }
}

/* Device buffers one integrate call works in: the work counter, the totals
 * block ([16]: KR_TOT_* then this call's statistics counters) and the
 * cell-order buffers.  grow_order: the order buffers may be (re)allocated
 * to fit the batch; otherwise they must already hold order_cap cells. */
struct Workspace {
  unsigned long long *counter;
  unsigned long long *totals;
  OrderBufs *ord;
  bool grow_order;
  bool clear_hist;   /* the order histogram's contents are unknown: clear it */
};

static int integrate_impl(const kr_network *net, int64_t n_cells, double *states, int64_t ld, double *T,
                          const double *rho, const double *dt, double dt_scalar, double rtol,
                          const kr_options *opt, int32_t *status, int32_t *cell_stats, kr_stream_t stream,
                          Workspace &ws) {
  if (!net) return fail(KR_EINVAL, "null network");
  if (n_cells < 0 || ld < n_cells) return fail(KR_EINVAL, "bad n_cells/ld (%lld, %lld)", (long long)n_cells, (long long)ld);
  if (!(rtol > 0.0) || !std::isfinite(rtol)) return fail(KR_EINVAL, "rtol must be > 0");
  kr_options o;
  kr_default_options(&o);
  if (opt) o = *opt;
  if ((o.precision < KR_FP64 || o.precision > KR_MIXED) ||
      (o.mode != KR_ADAPTIVE && o.mode != KR_FIXED_STEP) || (o.mode == KR_FIXED_STEP && o.n_fixed < 1) ||
      o.max_newton < 1 || o.max_substeps < 1 || !(o.floor >= 0.0) || !(o.newton_tol > 0.0) ||
      !(o.rho_floor >= 0.0) || (o.order != KR_ORDER_INPUT && o.order != KR_ORDER_WORK))
    return fail(KR_EINVAL, "bad options");
  if (o.precision >= KR_SINGLE && net->wide)
    return fail(KR_EINVAL, "the single- and mixed-precision modes need the lane layout");
  if (n_cells == 0) return KR_OK;
  if (!states || !T) return fail(KR_EINVAL, "null state arrays");
  if (!dt && !(dt_scalar >= 0.0 && std::isfinite(dt_scalar))) return fail(KR_EINVAL, "bad dt_scalar");
  if (o.guess && o.guess_ld < n_cells) return fail(KR_EINVAL, "guess_ld < n_cells");
  if (o.guess && net->wide) return fail(KR_EINVAL, "a learned guess is not supported in the wavefront layout");
  if (o.h_log && (o.h_log_ld < n_cells || o.h_log_cap < 0)) return fail(KR_EINVAL, "h_log_ld < n_cells or h_log_cap < 0");
  const bool ordered = want_order(o, n_cells);
  if (ordered && !ws.grow_order && n_cells > ws.ord->cap)
    return fail(KR_EINVAL, "KR_ORDER_WORK batch of %lld cells exceeds the %lld-cell order scratch", (long long)n_cells,
                ws.ord->cap);
  HIP_TRY(hipSetDevice(net->device));
  hipStream_t st = (hipStream_t)stream;

  KrParams p;
  p.n_cells = n_cells; p.states = states; p.ld = ld; p.T = T; p.rho = rho; p.dt = dt;
  p.dt_scalar = dt_scalar; p.rtol = rtol; p.floor = o.floor; p.newton_tol = o.newton_tol;
  p.rho_floor = o.rho_floor; p.max_newton = o.max_newton; p.max_substeps = o.max_substeps;
  p.mode = o.mode; p.n_fixed = o.n_fixed; p.status = status; p.cell_stats = cell_stats;
  p.counter = ws.counter;
  p.guess = o.guess; p.guess_ld = o.guess_ld; p.counters = o.counters;
  p.order = nullptr;
  p.h_hint = o.h_hint; p.h_log = o.h_log; p.h_log_ld = o.h_log_ld; p.h_log_cap = o.h_log_cap;
  p.h_log_n = o.h_log_n;
  p.photo_flux = o.photo_flux; p.photo_length = o.photo_length;
  p.totals = nullptr;
  if (o.stats) {
    /* totals and this call's statistics counters in the workspace's block,
     * cleared by a kernel on the stream */
    hipLaunchKernelGGL(kr_zero_u64n, dim3(1), dim3(64), 0, st, ws.totals, 16);
    HIP_TRY(hipGetLastError());
    p.totals = ws.totals;
    p.counters = ws.totals + 8;
  }
  if (ordered) {
    int rc = ws.grow_order ? order_reserve(*ws.ord, n_cells) : KR_OK;
    if (rc == KR_OK && ws.clear_hist) {
      hipLaunchKernelGGL(kr_zero_u64n, dim3(1), dim3(64), 0, st, (unsigned long long *)ws.ord->hist,
                         KR_ORDER_NBUCKETS / 2);
      if (hipGetLastError() != hipSuccess) rc = fail(KR_EDEVICE, "order histogram clear failed");
    }
    if (rc == KR_OK)
      rc = order_launch(net->f_keys, net->f_scan, net->f_scatter, *ws.ord, net->wide, net->cu_count, p, st);
    if (rc != KR_OK) return rc;
  }

  unsigned long long *cnt = ws.counter;
  void *rargs[] = {&cnt};
  HIP_TRY(hipModuleLaunchKernel(net->f_reset, 1, 1, 1, 64, 1, 1, 0, st, rargs, nullptr));
  const hipFunction_t fs[4] = {net->f_fp64, net->f_fp32, net->f_single, net->f_mixed};
  const int occs[4] = {net->occ_fp64, net->occ_fp32, net->occ_single, net->occ_mixed};
  hipFunction_t f = fs[o.precision];
  const int occ = occs[o.precision];
  long long blocks = (long long)net->cu_count * (occ > 0 ? occ : 1);
  /* waves with work: 64 cells per wave (lane layout), 64 / G (lane groups), 1 (wavefront) */
  const long long cpw = net->group ? 64 / net->group : (net->wide ? 1 : 64);
  const long long need = (n_cells + cpw - 1) / cpw;
  if (blocks > need) blocks = need;
  if (blocks < 1) blocks = 1;
  void *args[] = {&p};
  HIP_TRY(hipModuleLaunchKernel(f, (unsigned)blocks, 1, 1, 64, 1, 1, 0, st, args, nullptr));
  if (o.stats) return finish_stats(ws.totals, o.counters, o.stats, st);
  return KR_OK;
}

extern "C" int kr_chem_integrate(const kr_network *net, int64_t n_cells, double *states, int64_t ld,
                                 double *T, const double *rho, const double *dt, double dt_scalar,
                                 double rtol, const kr_options *opt, int32_t *status,
                                 int32_t *cell_stats, kr_stream_t stream) {
  try {
    if (!net) return fail(KR_EINVAL, "null network");
    kr_network *mnet = const_cast<kr_network *>(net);   /* scratch buffers only */
    Workspace ws{net->d_counter, net->d_totals, &mnet->ord, true, false};
    return integrate_impl(net, n_cells, states, ld, T, rho, dt, dt_scalar, rtol, opt, status, cell_stats,
                          stream, ws);
  } KR_CATCH
}

/* ------------------------------------------------------------------------ */
/* integration without allocations                                          */
/* ------------------------------------------------------------------------ */

/* The workspace of kr_chem_integrate_noalloc: one static device array per
 * GPU, held until the process ends.  Layout (bytes): [0, 8) work counter,
 * [256, 384) totals block, [512, 2560) order histogram and bucket starts,
 * [4096, 4096 + 4 n) cell order, then n bucket bytes (n <= the order
 * capacity).  In host code `scratch` names a host-side stand-in; its device
 * address comes from hipGetSymbolAddress, kept per device. */
static __device__ __align__(256) unsigned char scratch[KR_NOALLOC_SCRATCH_BYTES];

static const long long kScratchOrderBase = 4096;
static const long long kScratchOrderCap = (KR_NOALLOC_SCRATCH_BYTES - kScratchOrderBase) / 5;

static std::mutex g_scratch_mu;
static unsigned char *g_scratch_ptr[KR_MAX_DEVICES];

/* Looks up (once per device, with that device current) the device address of
 * the scratch array.  Called by kr_network_create. */
static int scratch_setup(int device) {
  if (device < 0 || device >= KR_MAX_DEVICES) return fail(KR_EDEVICE, "device index %d out of range", device);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return KR_OK;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return fail(KR_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
  g_scratch_ptr[device] = (unsigned char *)ptr;
  return KR_OK;
}

extern "C" int kr_chem_integrate_noalloc(const kr_network *net, int64_t n_cells, double *states, int64_t ld,
                                         double *T, const double *rho, const double *dt, double dt_scalar,
                                         double rtol, const kr_options *opt, int32_t *status,
                                         int32_t *cell_stats, kr_stream_t stream) {
  try {
    if (!net) return fail(KR_EINVAL, "null network");
    unsigned char *base = nullptr;
    {
      std::lock_guard<std::mutex> lock(g_scratch_mu);
      if (net->device >= 0 && net->device < KR_MAX_DEVICES) base = g_scratch_ptr[net->device];
    }
    if (!base) return fail(KR_EDEVICE, "no scratch address for device %d", net->device);
    OrderBufs ob;
    ob.hist = (unsigned *)(base + 512);
    ob.order = (unsigned *)(base + kScratchOrderBase);
    ob.bucket = base + kScratchOrderBase + 4 * kScratchOrderCap;
    ob.cap = kScratchOrderCap;
    Workspace ws{(unsigned long long *)base, (unsigned long long *)(base + 256), &ob, false, true};
    return integrate_impl(net, n_cells, states, ld, T, rho, dt, dt_scalar, rtol, opt, status, cell_stats,
                          stream, ws);
  } KR_CATCH
}

/* ------------------------------------------------------------------------ */
/* element residual (ahead-of-time kernel)                                   */
/* ------------------------------------------------------------------------ */

__global__ void __launch_bounds__(256) kr_element_residual_kernel(
    int S, int nrows, int nelem, const int32_t *__restrict__ comp, long long n,
    const double *__restrict__ before, const double *__restrict__ after, long long ld,
    double *__restrict__ resid, unsigned long long *__restrict__ maxbits) {
  double local = 0.0;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    double nn = 0.0;
    for (int s = 0; s < S; ++s) {
      int a = 0;
      for (int v = 0; v < nelem; ++v) a += comp[v * S + s];
      nn += a * before[s * ld + c];
    }
    double worst = 0.0;
    for (int v = 0; v < nrows; ++v) {
      double diff = 0.0, D = 0.0;
      for (int s = 0; s < S; ++s) {
        const int a = comp[v * S + s];
        if (!a) continue;
        const double b = before[s * ld + c];
        diff += a * (after[s * ld + c] - b);
        D += (a > 0 ? a : -a) * b;
      }
      if (v >= nelem) D = nn;
      const double e = fabs(diff) / fmax(D, 1e-300);
      if (!(e <= worst)) worst = e;
    }
    if (resid) resid[c] = worst;
    if (!(worst <= local)) local = worst;
  }
  if (!maxbits) return;
  /* non-negative doubles (and NaN) order like their bit patterns */
  unsigned long long bits = __double_as_longlong(local);
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long o = __shfl_xor(bits, off);
    bits = o > bits ? o : bits;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(maxbits, bits);
}

__global__ void kr_zero_u64(unsigned long long *p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0ull;
}

__global__ void kr_zero_doubles(double *p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0.0;
}

extern "C" int kr_element_residual(const kr_network *net, int64_t n_cells, const double *before,
                                   const double *after, int64_t ld, double *resid, double *max_out,
                                   kr_stream_t stream) {
  try {
    if (!net) return fail(KR_EINVAL, "null network");
    if (n_cells < 0 || ld < n_cells) return fail(KR_EINVAL, "bad n_cells/ld");
    if (n_cells > 0 && (!before || !after)) return fail(KR_EINVAL, "null state arrays");
    HIP_TRY(hipSetDevice(net->device));
    hipStream_t st = (hipStream_t)stream;
    if (max_out) {
      hipLaunchKernelGGL(kr_zero_u64, dim3(1), dim3(64), 0, st, net->d_max);
      HIP_TRY(hipGetLastError());
    }
    if (n_cells > 0) {
      long long blocks = (n_cells + 255) / 256;
      if (blocks > 4096) blocks = 4096;
      hipLaunchKernelGGL(kr_element_residual_kernel, dim3((unsigned)blocks), dim3(256), 0, st, net->S,
                         net->n_rows, net->n_elem, net->d_comp, (long long)n_cells, before, after,
                         (long long)ld, resid, max_out ? net->d_max : nullptr);
      HIP_TRY(hipGetLastError());
    }
    if (max_out) {
      unsigned long long bits = 0;
      HIP_TRY(hipMemcpyAsync(&bits, net->d_max, sizeof bits, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      std::memcpy(max_out, &bits, sizeof bits);
    }
    return KR_OK;
  } KR_CATCH
}

extern "C" int kr_postprocess(const kr_network *net, int64_t n_cells, const double *before, double *after,
                              int64_t ld, int32_t *flags, kr_stream_t stream) {
  try {
    if (!net) return fail(KR_EINVAL, "null network");
    if (n_cells < 0 || ld < n_cells) return fail(KR_EINVAL, "bad n_cells/ld");
    if (n_cells == 0) return KR_OK;
    if (!before || !after) return fail(KR_EINVAL, "null state arrays");
    HIP_TRY(hipSetDevice(net->device));
    KrParams p{};
    p.n_cells = n_cells; p.states = after; p.ld = ld;
    const long long need = net->wide ? n_cells : (n_cells + 63) / 64;
    const long long blocks = std::min<long long>(need, (long long)net->cu_count * 8);
    void *args[] = {&p, &before, &flags};
    HIP_TRY(hipModuleLaunchKernel(net->f_post, (unsigned)blocks, 1, 1, 64, 1, 1, 0, (hipStream_t)stream, args,
                                  nullptr));
    return KR_OK;
  } KR_CATCH
}

/* ------------------------------------------------------------------------ */
/* stoichiometry-compatible PLM advection (generated module's kr_advect)     */
/* ------------------------------------------------------------------------ */

struct KrAdvParamsHost {          /* mirrors the device struct KrAdvParams (kr_advect.h) */
  long long n_lines, n_cells, line_stride;
  const double *n_in;
  double *n_out;
  long long ld;
  const double *rho, *flux, *xc, *xf, *base;
  double dt, alpha, beta;
  int mode;
};

extern "C" int kr_advect_plm(const kr_network *net, int64_t n_lines, int64_t n_cells, int64_t line_stride,
                             const double *n_in, double *n_out, int64_t ld, const double *rho,
                             const double *flux, const double *xc, const double *xf, double dt,
                             const double *base, double alpha, double beta, int32_t mode,
                             kr_stream_t stream) {
  try {
    if (!net) return fail(KR_EINVAL, "null network");
    if (n_lines < 0 || n_cells < 0 || (n_lines > 1 && line_stride < n_cells) || (n_lines == 1 && line_stride < 0))
      return fail(KR_EINVAL, "bad line sizes");
    if (n_lines == 0 || n_cells == 0) return KR_OK;
    if (n_cells < 3) return fail(KR_EINVAL, "a periodic line needs at least 3 cells");
    if ((n_lines - 1) * line_stride + n_cells > ld) return fail(KR_EINVAL, "ld too small for the lines");
    if (!n_in || !n_out || !rho || !flux || !xc || !xf) return fail(KR_EINVAL, "null array");
    if (n_in == n_out) return fail(KR_EINVAL, "n_out must not alias n_in");
    if (mode < 0 || mode > 2) return fail(KR_EINVAL, "mode out of [0, 2]");
    if (!std::isfinite(dt) || !std::isfinite(alpha) || !std::isfinite(beta)) return fail(KR_EINVAL, "bad scalars");
    HIP_TRY(hipSetDevice(net->device));
    KrAdvParamsHost p{n_lines, n_cells, n_lines > 1 ? line_stride : 0, n_in, n_out, ld, rho, flux, xc, xf,
                      base, dt, base ? alpha : 0.0, beta, mode};
    /* up to 32 species: 60 cells per wavefront, 4 independent wavefronts
     * per workgroup; more: one LDS-staged chunk of 64 cells per workgroup
     * (the kernel's KR_ADV_REG / KR_ADV_CHUNK) */
    const bool reg = net->S <= 32;
    const int per = reg ? 60 : 64, threads = reg ? 256 : 64;
    const long long units = n_lines * ((n_cells + per - 1) / per);
    const long long blocks = std::min<long long>(reg ? (units + 3) / 4 : units, (long long)net->cu_count * 64);
    void *args[] = {&p};
    HIP_TRY(hipModuleLaunchKernel(net->f_adv, (unsigned)blocks, 1, 1, threads, 1, 1, 0, (hipStream_t)stream, args,
                                  nullptr));
    return KR_OK;
  } KR_CATCH
}

struct KrAdv2ParamsHost {         /* mirrors the device struct KrAdv2Params (kr_advect.h) */
  long long n_lines, n_cells, line_stride;
  const double *n_in;
  double *n_out;
  long long ld;
  const double *rho0, *flux0, *rho1, *flux1, *xc, *xf;
  double dt;
  int mode;
};

extern "C" int kr_advect_plm_ssprk2(const kr_network *net, int64_t n_lines, int64_t n_cells, int64_t line_stride,
                                    const double *n_in, double *n_out, int64_t ld, const double *rho0,
                                    const double *flux0, const double *rho1, const double *flux1,
                                    const double *xc, const double *xf, double dt, int32_t mode,
                                    kr_stream_t stream) {
  try {
    if (!net) return fail(KR_EINVAL, "null network");
    if (n_lines < 0 || n_cells < 0 || (n_lines > 1 && line_stride < n_cells) || (n_lines == 1 && line_stride < 0))
      return fail(KR_EINVAL, "bad line sizes");
    if (n_lines == 0 || n_cells == 0) return KR_OK;
    if (n_cells < 4) return fail(KR_EINVAL, "the fused step needs lines of at least 4 cells");
    if ((n_lines - 1) * line_stride + n_cells > ld) return fail(KR_EINVAL, "ld too small for the lines");
    if (!n_in || !n_out || !rho0 || !flux0 || !rho1 || !flux1 || !xc || !xf) return fail(KR_EINVAL, "null array");
    if (n_in == n_out) return fail(KR_EINVAL, "n_out must not alias n_in");
    if (mode < 0 || mode > 2) return fail(KR_EINVAL, "mode out of [0, 2]");
    if (!std::isfinite(dt)) return fail(KR_EINVAL, "bad dt");
    HIP_TRY(hipSetDevice(net->device));
    KrAdv2ParamsHost p{n_lines, n_cells, n_lines > 1 ? line_stride : 0, n_in, n_out, ld, rho0, flux0, rho1, flux1,
                       xc, xf, dt, mode};
    /* up to 32 species: 56 cells per wavefront (four halo cells on each
     * side), 4 independent wavefronts per workgroup; more: one LDS-staged
     * chunk of 64 cells per workgroup (the kernel's KR_ADV_REG / KR_ADV_CHUNK) */
    const bool reg = net->S <= 32;
    const int per = reg ? 56 : 64, threads = reg ? 256 : 64;
    const long long units = n_lines * ((n_cells + per - 1) / per);
    const long long blocks = std::min<long long>(reg ? (units + 3) / 4 : units, (long long)net->cu_count * 64);
    void *args[] = {&p};
    HIP_TRY(hipModuleLaunchKernel(net->f_adv2, (unsigned)blocks, 1, 1, threads, 1, 1, 0, (hipStream_t)stream, args,
                                  nullptr));
    return KR_OK;
  } KR_CATCH
}

extern "C" int kr_work_order(const kr_network *net, int64_t n_cells, const double *states, int64_t ld,
                             const double *T, const double *rho, const double *dt, double dt_scalar,
                             const kr_options *opt, uint32_t *order, kr_stream_t stream) {
  try {
    if (!net) return fail(KR_EINVAL, "null network");
    if (n_cells < 0 || ld < n_cells || n_cells > 0xFFFFFFFFll)
      return fail(KR_EINVAL, "bad n_cells/ld (%lld, %lld)", (long long)n_cells, (long long)ld);
    if (n_cells == 0) return KR_OK;
    if (!states || !T || !order) return fail(KR_EINVAL, "null array");
    if (!dt && !(dt_scalar >= 0.0 && std::isfinite(dt_scalar))) return fail(KR_EINVAL, "bad dt_scalar");
    kr_options o;
    kr_default_options(&o);
    if (opt) o = *opt;
    if (!(o.floor >= 0.0) || !(o.rho_floor >= 0.0)) return fail(KR_EINVAL, "bad options");
    HIP_TRY(hipSetDevice(net->device));
    KrParams p{};
    p.n_cells = n_cells; p.states = (double *)states; p.ld = ld; p.T = (double *)T; p.rho = rho; p.dt = dt;
    p.dt_scalar = dt_scalar; p.floor = o.floor; p.rho_floor = o.rho_floor;
    kr_network *mnet = const_cast<kr_network *>(net);   /* scratch buffers only */
    int rc = order_reserve(mnet->ord, n_cells);
    if (rc != KR_OK) return rc;
    OrderBufs b = net->ord;
    b.order = order;
    return order_launch(net->f_keys, net->f_scan, net->f_scatter, b, net->wide, net->cu_count, p,
                        (hipStream_t)stream);
  } KR_CATCH
}

/* ------------------------------------------------------------------------ */
/* fastest timescale (workload set-up)                                       */
/* ------------------------------------------------------------------------ */

extern "C" int kr_fastest_timescale(const kr_network *net, int64_t n_cells, const double *states,
                                    int64_t ld, const double *T, double *out, kr_stream_t stream) {
  try {
    if (!net || n_cells < 0 || ld < n_cells || (n_cells && (!states || !T || !out)))
      return fail(KR_EINVAL, "bad timescale arguments");
    if (!n_cells) return KR_OK;
    HIP_TRY(hipSetDevice(net->device));
    KrParams p{};
    p.n_cells = n_cells; p.states = (double *)states; p.ld = ld; p.T = (double *)T; p.dt_scalar = 1.0;
    long long blocks = std::min<long long>(net->wide ? n_cells : (n_cells + 63) / 64,
                                          (long long)net->cu_count * (net->wide ? 4 : 16));
    void *args[] = {&p, &out};
    HIP_TRY(hipModuleLaunchKernel(net->f_tau, (unsigned)blocks, 1, 1, 64, 1, 1, 0, (hipStream_t)stream, args,
                                  nullptr));
    return KR_OK;
  } KR_CATCH
}

/* ------------------------------------------------------------------------ */
/* several networks in one persistent launch                                 */
/* ------------------------------------------------------------------------ */

#define KR_MAX_NETS 4

struct KrMultiHost {          /* mirrors the device struct KrMulti */
  KrParams net[KR_MAX_NETS];
  int n_nets;
};

struct kr_multi {
  std::vector<const kr_network *> nets;
  kr_build_opts build{1, 0.1f, KR_LAYOUT_AUTO, 0};
  std::string source;
  hipModule_t module = nullptr;
  /* one persistent kernel per group of networks compiled for the same
   * occupancy target (KrGroups) */
  std::vector<std::vector<int>> groups;
  hipFunction_t f_fp64[2] = {}, f_fp32[2] = {}, f_reset = nullptr;
  hipFunction_t f_keys[KR_MAX_NETS] = {}, f_scan = nullptr, f_scatter = nullptr;
  OrderBufs ord[KR_MAX_NETS];
  int device = -1, cu_count = 0, occ_fp64[2] = {}, occ_fp32[2] = {};
  unsigned long long *d_counters = nullptr; /* one per network */
  unsigned long long *d_totals = nullptr;   /* [16] per-call totals and statistics counters */
  hipStream_t capture = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<char> key;      /* launch parameters the graph was captured with */
  long long graph_launches = 0, graph_captures = 0;
};

/* Networks of a multi launch grouped by occupancy target: one persistent
 * kernel drains all queues when every network wants the same target (or an
 * explicit waves_per_eu sets it); otherwise the lane-layout networks (one
 * wave per SIMD) and the wavefront-layout networks (two where their LDS
 * blocks allow) get a kernel each, run one after the other.  Returns the
 * groups with their targets. */
static std::vector<std::pair<int, std::vector<int>>> multi_groups(const std::vector<const kr_network *> &nets,
                                                                  const kr_build_opts &o) {
  int w[2] = {8, 8};
  std::vector<int> members[2];
  for (size_t k = 0; k < nets.size(); ++k) {
    const int g = nets[k]->wide ? 1 : 0;
    const int L = nets[k]->group ? (nets[k]->group == 16 ? KR_LAYOUT_GROUP16 : KR_LAYOUT_GROUP32)
                                 : (g ? KR_LAYOUT_WAVE : KR_LAYOUT_LANE);
    const kr_build_opts ok{o.waves_per_eu, o.pivot_tau, L, o.lu_mfma};
    w[g] = std::min(w[g], auto_waves_per_eu(nets[k], ok));
    members[g].push_back((int)k);
  }
  std::vector<std::pair<int, std::vector<int>>> out;
  if (members[0].empty() || members[1].empty() || w[0] == w[1]) {
    std::vector<int> all;
    for (size_t k = 0; k < nets.size(); ++k) all.push_back((int)k);
    out.push_back({std::min(w[0], w[1]), all});
  } else {
    out.push_back({w[0], members[0]});
    out.push_back({w[1], members[1]});
  }
  return out;
}

static int multi_waves_per_eu(const std::vector<const kr_network *> &nets, const kr_build_opts &o) {
  int w = 8;
  for (const auto &g : multi_groups(nets, o)) w = std::min(w, g.first);
  return w;
}

static std::string multi_source(const std::vector<const kr_network *> &nets, const kr_build_opts &o) {
  std::string s = "/* per-cell implicit thermochemistry: several networks in one launch */\n" +
                  build_prefix(multi_waves_per_eu(nets, o), o) + "#define KR_NO_KERNELS\n" + kParamsSource + "\n" +
                  kMathSource + "\n" + kFloatMathSource + kOrderSource + "\n";
  for (size_t k = 0; k < nets.size(); ++k) {
    if (nets[k]->group)
      s += "namespace kr_m" + std::to_string(k) + " {\n" + generate_wide(nets[k]) + "\n" +
           generate_group(nets[k], nets[k]->group) + kWideSource + "\n" + kGroupSource +
           "\n}\n#undef KR_S\n#undef KR_NROWS\n#undef KR_NELEM\n#undef KR_N\n#undef KR_LDJ\n#undef KR_NDR\n"
           "#undef KR_NC\n#undef KR_NF\n#undef KR_NDP\n#undef KR_NOTPIV\n#undef KR_CV_POLY\n#undef KR_NTAB\n"
           "#undef KR_TAB_NODES\n#undef KR_G\n#undef KR_GNDR\n#undef KR_GNC\n#undef KR_GNF\n#undef KR_H\n"
           "#undef KR_GLOG\n#undef KR_GMASK\n";
    else if (nets[k]->wide)
      s += "namespace kr_m" + std::to_string(k) + " {\n" + lu_mfma_define(nets[k], o) + generate_wide(nets[k]) +
           "\n" + kWideSource +
           "\n}\n#undef KR_S\n#undef KR_NROWS\n#undef KR_NELEM\n#undef KR_N\n#undef KR_LDJ\n#undef KR_NDR\n"
           "#undef KR_NC\n#undef KR_NF\n#undef KR_NDP\n#undef KR_NOTPIV\n#undef KR_LU_MFMA\n#undef KR_USE_LU_MFMA\n"
           "#undef KR_PF\n#undef KR_CV_POLY\n#undef KR_NTAB\n#undef KR_TAB_NODES\n";
    else
      s += "namespace kr_m" + std::to_string(k) + " {\n" + generate_network(nets[k]) + "\n" +
           kDeviceSource + "\n}\n#undef KR_S\n#undef KR_NROWS\n#undef KR_NELEM\n#undef KR_N\n"
           "#undef KR_CV_POLY\n#undef KR_NTAB\n#undef KR_TAB_NODES\n";
  }
  s += "struct KrMulti { KrParams net[" + std::to_string(KR_MAX_NETS) + "]; int n_nets; };\n";
  const auto groups = multi_groups(nets, o);
  for (size_t g = 0; g < groups.size(); ++g) {
    const std::vector<int> &mem = groups[g].second;
    for (int mixed = 0; mixed < 2; ++mixed) {
      s += "extern \"C\" __global__ void __launch_bounds__(64, " + std::to_string(groups[g].first) + ") " +
           (mixed ? "kr_integrate_multi_fp32lu_" : "kr_integrate_multi_fp64_") + std::to_string(g) +
           "(KrMulti m) {\n"
           "  /* each wave drains one network's queue after another, starting at a\n"
           "   * different network so that the queues drain together */\n"
           "  for (int i = 0; i < " + std::to_string(mem.size()) + "; ++i) {\n"
           "    switch ((int)((blockIdx.x + i) % " + std::to_string(mem.size()) + "u)) {\n";
      for (size_t j = 0; j < mem.size(); ++j) {
        const int k = mem[j];
        s += "      case " + std::to_string(j) + ": if (" + std::to_string(k) + " < m.n_nets) kr_m" + std::to_string(k) +
             (nets[k]->group ? (mixed ? "::kr_gintegrate<true" : "::kr_gintegrate<false")
              : nets[k]->wide ? (mixed ? "::kr_wintegrate<true" : "::kr_wintegrate<false")
                              : (mixed ? "::kr_integrate_body<1" : "::kr_integrate_body<0")) +
             ">(m.net[" + std::to_string(k) + "]); break;\n";
      }
      s += "      default: break;\n    }\n  }\n}\n";
    }
  }
  for (size_t k = 0; k < nets.size(); ++k)
    s += "extern \"C\" __global__ void __launch_bounds__(64, 1) kr_order_keys_m" + std::to_string(k) +
         "(KrParams p, unsigned char *bucket, unsigned *hist) {\n  kr_m" + std::to_string(k) +
         (nets[k]->wide ? "::kr_worder_keys" : "::kr_order_keys_body") + "(p, bucket, hist);\n}\n";
  s += "extern \"C\" __global__ void kr_reset_counters(unsigned long long *c, int n) {\n"
       "  if (blockIdx.x == 0 && (int)threadIdx.x < n) c[threadIdx.x] = 0ull;\n}\n";
  return s;
}

static void release_multi(kr_multi *m) {
  if (!m) return;
  if (m->exec) (void)hipGraphExecDestroy(m->exec);
  if (m->graph) (void)hipGraphDestroy(m->graph);
  if (m->capture) (void)hipStreamDestroy(m->capture);
  if (m->d_counters) (void)hipFree(m->d_counters);
  if (m->d_totals) (void)hipFree(m->d_totals);
  for (int k = 0; k < KR_MAX_NETS; ++k) order_free(m->ord[k]);
  if (m->module) (void)hipModuleUnload(m->module);
  delete m;
}

extern "C" int kr_multi_create(const kr_network *const *nets, int32_t n_nets, const kr_build_opts *bopt,
                               kr_multi **out) {
  try {
    if (!out) return fail(KR_EINVAL, "null output handle");
    *out = nullptr;
    if (!nets || n_nets < 1 || n_nets > KR_MAX_NETS) return fail(KR_EINVAL, "n_nets out of [1, %d]", KR_MAX_NETS);
    for (int k = 0; k < n_nets; ++k) {
      if (!nets[k]) return fail(KR_EINVAL, "null network %d", k);
      if (nets[k]->has_photo)
        return fail(KR_EINVAL, "network %d has photoreactions: not supported in multi-network launches", k);
    }
    kr_build_opts bo;
    kr_default_build_options(&bo);
    if (bopt) bo = *bopt;
    int rc = check_build_options(&bo);
    if (rc != KR_OK) return rc;
    kr_multi *m = new (std::nothrow) kr_multi;
    if (!m) return fail(KR_ENOMEM, "out of host memory");
    m->nets.assign(nets, nets + n_nets);
    m->build = bo;
    m->build.waves_per_eu = multi_waves_per_eu(m->nets, bo);
    m->source = multi_source(m->nets, bo);
    for (const auto &g : multi_groups(m->nets, bo)) m->groups.push_back(g.second);
    std::vector<char> code;
    std::string log;
    rc = compile_source(m->source, code, log);
    if (rc != KR_OK) { delete m; return rc; }
    hipError_t e;
  #define MULTI_TRY(expr)                                                              \
    do {                                                                               \
      e = (expr);                                                                      \
      if (e != hipSuccess) {                                                           \
        rc = fail(KR_EDEVICE, "%s: %s", #expr, hipGetErrorString(e));                  \
        release_multi(m);                                                              \
        return rc;                                                                     \
      }                                                                                \
    } while (0)
    MULTI_TRY(hipGetDevice(&m->device));
    MULTI_TRY(hipDeviceGetAttribute(&m->cu_count, hipDeviceAttributeMultiprocessorCount, m->device));
    MULTI_TRY(hipModuleLoadData(&m->module, code.data()));
    for (size_t g = 0; g < m->groups.size(); ++g) {
      const std::string sfx = std::to_string(g);
      MULTI_TRY(hipModuleGetFunction(&m->f_fp64[g], m->module, ("kr_integrate_multi_fp64_" + sfx).c_str()));
      MULTI_TRY(hipModuleGetFunction(&m->f_fp32[g], m->module, ("kr_integrate_multi_fp32lu_" + sfx).c_str()));
      MULTI_TRY(hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&m->occ_fp64[g], m->f_fp64[g], 64, 0));
      MULTI_TRY(hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&m->occ_fp32[g], m->f_fp32[g], 64, 0));
    }
    MULTI_TRY(hipModuleGetFunction(&m->f_reset, m->module, "kr_reset_counters"));
    MULTI_TRY(hipModuleGetFunction(&m->f_scan, m->module, "kr_order_scan"));
    MULTI_TRY(hipModuleGetFunction(&m->f_scatter, m->module, "kr_order_scatter"));
    for (int k = 0; k < n_nets; ++k)
      MULTI_TRY(hipModuleGetFunction(&m->f_keys[k], m->module, ("kr_order_keys_m" + std::to_string(k)).c_str()));
    MULTI_TRY(hipMalloc(&m->d_counters, sizeof(unsigned long long) * KR_MAX_NETS));
    MULTI_TRY(hipMalloc(&m->d_totals, sizeof(unsigned long long) * 16));
    MULTI_TRY(hipStreamCreateWithFlags(&m->capture, hipStreamNonBlocking));
  #undef MULTI_TRY
    *out = m;
    return KR_OK;
  } KR_CATCH
}

extern "C" void kr_multi_destroy(kr_multi *m) {
  try {
    release_multi(m);
  } catch (...) {
  }
}

extern "C" int kr_multi_check(const kr_network_desc *const *descs, int32_t n_nets, int compile, char *src_buf,
                              int64_t src_len) {
  try {
    if (!descs || n_nets < 1 || n_nets > KR_MAX_NETS) return fail(KR_EINVAL, "n_nets out of [1, %d]", KR_MAX_NETS);
    std::vector<kr_network> tabs(n_nets);
    std::vector<const kr_network *> ptrs;
    for (int k = 0; k < n_nets; ++k) {
      int rc = build_tables(descs[k], &tabs[k]);
      if (rc != KR_OK) return rc;
      if (tabs[k].has_photo)
        return fail(KR_EINVAL, "network %d has photoreactions: not supported in multi-network launches", k);
      ptrs.push_back(&tabs[k]);
    }
    kr_build_opts bo;
    kr_default_build_options(&bo);
    for (int k = 0; k < n_nets; ++k) {
      tabs[k].wide = use_wide(&tabs[k], bo);
      tabs[k].group = group_lanes(&tabs[k], bo);
      if (tabs[k].wide) {
        int rc = check_wide(&tabs[k]);
        if (rc != KR_OK) return rc;
      }
    }
    const std::string src = multi_source(ptrs, bo);
    if (src_buf && src_len > 0) {
      const size_t m = std::min<size_t>((size_t)src_len - 1, src.size());
      std::memcpy(src_buf, src.data(), m);
      src_buf[m] = '\0';
    }
    if (!compile) return KR_OK;
    std::vector<char> code;
    std::string log;
    return compile_source(src, code, log);
  } KR_CATCH
}

extern "C" int64_t kr_multi_graph_stats(const kr_multi *m, int64_t *captures) {
  try {
    if (!m) return fail(KR_EINVAL, "null handle");
    if (captures) *captures = m->graph_captures;
    return m->graph_launches;
  } KR_CATCH
}

static int fill_params(const kr_network *net, const kr_batch &b, double rtol, const kr_options &o,
                       unsigned long long *counter, KrParams &p) {
  if (b.n_cells < 0 || b.ld < b.n_cells) return fail(KR_EINVAL, "bad n_cells/ld in a batch");
  if (b.n_cells && (!b.states || !b.T)) return fail(KR_EINVAL, "null state arrays in a batch");
  if (!b.dt && !(b.dt_scalar >= 0.0 && std::isfinite(b.dt_scalar))) return fail(KR_EINVAL, "bad dt_scalar");
  (void)net;
  p = KrParams{};
  p.n_cells = b.n_cells; p.states = b.states; p.ld = b.ld; p.T = b.T; p.rho = b.rho; p.dt = b.dt;
  p.dt_scalar = b.dt_scalar; p.rtol = rtol; p.floor = o.floor; p.newton_tol = o.newton_tol;
  p.rho_floor = o.rho_floor; p.max_newton = o.max_newton; p.max_substeps = o.max_substeps;
  p.mode = o.mode; p.n_fixed = o.n_fixed; p.status = b.status; p.cell_stats = b.cell_stats;
  p.counter = counter; p.guess = nullptr; p.guess_ld = 0; p.counters = o.counters;
  return KR_OK;
}

static int validate_options(const kr_options &o) {
  if ((o.precision < KR_FP64 || o.precision > KR_MIXED) ||
      (o.mode != KR_ADAPTIVE && o.mode != KR_FIXED_STEP) || (o.mode == KR_FIXED_STEP && o.n_fixed < 1) ||
      o.max_newton < 1 || o.max_substeps < 1 || !(o.floor >= 0.0) || !(o.newton_tol > 0.0) ||
      !(o.rho_floor >= 0.0) || (o.order != KR_ORDER_INPUT && o.order != KR_ORDER_WORK))
    return fail(KR_EINVAL, "bad options");
  return KR_OK;
}

extern "C" int kr_chem_integrate_multi(kr_multi *m, const kr_batch *batches, double rtol,
                                       const kr_options *opt, int32_t use_graph, kr_stream_t stream) {
  try {
    if (!m || !batches) return fail(KR_EINVAL, "null argument");
    if (!(rtol > 0.0) || !std::isfinite(rtol)) return fail(KR_EINVAL, "rtol must be > 0");
    kr_options o;
    kr_default_options(&o);
    if (opt) o = *opt;
    int rc = validate_options(o);
    if (rc) return rc;
    if (o.guess) return fail(KR_EINVAL, "a learned guess is not supported in multi-network launches");
    if (o.precision >= KR_SINGLE)
      return fail(KR_EINVAL, "the single- and mixed-precision modes are not supported in multi-network launches");
    if (o.h_hint || o.h_log || o.h_log_n)
      return fail(KR_EINVAL, "per-cell step hints and substep logs are not supported in multi-network launches");
    KrMultiHost h{};
    long long total = 0;
    h.n_nets = (int)m->nets.size();
    for (int k = 0; k < h.n_nets; ++k) {
      if ((rc = fill_params(m->nets[k], batches[k], rtol, o, m->d_counters + k, h.net[k]))) return rc;
      total += batches[k].n_cells;
    }
    if (total == 0) return KR_OK;
    HIP_TRY(hipSetDevice(m->device));
    hipStream_t st = (hipStream_t)stream;
    if (o.stats) {
      /* all networks add to one totals block, cleared ahead of the launch (a
       * kernel on the stream, outside any captured graph) */
      hipLaunchKernelGGL(kr_zero_u64n, dim3(1), dim3(64), 0, st, m->d_totals, 16);
      HIP_TRY(hipGetLastError());
      for (int k = 0; k < h.n_nets; ++k) {
        h.net[k].totals = m->d_totals;
        h.net[k].counters = m->d_totals + 8;
      }
    }
    const int n_groups = (int)m->groups.size();
    hipFunction_t f[2] = {};
    long long blocks[2] = {0, 0};
    for (int g = 0; g < n_groups; ++g) {
      f[g] = o.precision == KR_FP64 ? m->f_fp64[g] : m->f_fp32[g];
      const int occ = o.precision == KR_FP64 ? m->occ_fp64[g] : m->occ_fp32[g];
      long long need = 0;   /* waves with work: 64 cells per wave, 64 / G (lane groups), 1 (wavefront) */
      for (int k : m->groups[g]) {
        const long long cpw = m->nets[k]->group ? 64 / m->nets[k]->group : (m->nets[k]->wide ? 1 : 64);
        need += (batches[k].n_cells + cpw - 1) / cpw;
      }
      blocks[g] = std::min<long long>((long long)m->cu_count * (occ > 0 ? occ : 1), need);   /* 0: no work */
    }
    /* largest-work-first order of each batch: buffers reserved here, outside
     * any capture; the order kernels run on the launch stream ahead of the
     * counter reset (and are part of the captured graph) */
    bool ordered[KR_MAX_NETS] = {};
    for (int k = 0; k < h.n_nets; ++k) {
      if (!want_order(o, batches[k].n_cells)) continue;
      if ((rc = order_reserve(m->ord[k], batches[k].n_cells))) return rc;
      ordered[k] = true;
      h.net[k].order = m->ord[k].order;
    }
    auto launch_orders = [&](hipStream_t s) -> int {
      for (int k = 0; k < h.n_nets; ++k) {
        if (!ordered[k]) continue;
        KrParams pk = h.net[k];
        int r = order_launch(m->f_keys[k], m->f_scan, m->f_scatter, m->ord[k], m->nets[k]->wide, m->cu_count, pk, s);
        if (r != KR_OK) return r;
      }
      return KR_OK;
    };
    unsigned long long *cnt = m->d_counters;
    int nn = h.n_nets;
    void *rargs[] = {&cnt, &nn};
    void *args[] = {&h};
    auto launch_groups = [&](hipStream_t s) -> hipError_t {
      for (int g = 0; g < n_groups; ++g) {
        if (blocks[g] < 1) continue;
        const hipError_t e = hipModuleLaunchKernel(f[g], (unsigned)blocks[g], 1, 1, 64, 1, 1, 0, s, args, nullptr);
        if (e != hipSuccess) return e;
      }
      return hipSuccess;
    };
    if (!use_graph) {
      if ((rc = launch_orders(st))) return rc;
      HIP_TRY(hipModuleLaunchKernel(m->f_reset, 1, 1, 1, 64, 1, 1, 0, st, rargs, nullptr));
      HIP_TRY(launch_groups(st));
      if (o.stats) return finish_stats(m->d_totals, o.counters, o.stats, st);
      return KR_OK;
    }
    /* graph of [order kernels] -> [reset the work counters] -> [persistent
     * integrate, one kernel per group], captured once per distinct launch configuration and replayed
     * on the caller's stream (counters and histograms are cleared by kernels,
     * not memset nodes) */
    std::vector<char> key(sizeof h + sizeof blocks + sizeof f);
    std::memcpy(key.data(), &h, sizeof h);
    std::memcpy(key.data() + sizeof h, &blocks, sizeof blocks);
    std::memcpy(key.data() + sizeof h + sizeof blocks, &f, sizeof f);
    if (!m->exec || key != m->key) {
      if (m->exec) { (void)hipGraphExecDestroy(m->exec); m->exec = nullptr; }
      if (m->graph) { (void)hipGraphDestroy(m->graph); m->graph = nullptr; }
      HIP_TRY(hipStreamBeginCapture(m->capture, hipStreamCaptureModeThreadLocal));
      const int r0 = launch_orders(m->capture);
      hipError_t e1 = hipModuleLaunchKernel(m->f_reset, 1, 1, 1, 64, 1, 1, 0, m->capture, rargs, nullptr);
      hipError_t e2 = launch_groups(m->capture);
      hipGraph_t g = nullptr;
      hipError_t e3 = hipStreamEndCapture(m->capture, &g);
      if (r0 != KR_OK || e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(r0 != KR_OK ? r0 : KR_EDEVICE, "graph capture failed: order %d / %s / %s / %s", r0,
                    hipGetErrorString(e1), hipGetErrorString(e2), hipGetErrorString(e3));
      }
      m->graph = g;
      HIP_TRY(hipGraphInstantiate(&m->exec, m->graph, nullptr, nullptr, 0));
      m->key = key;
      m->graph_captures++;
    }
    HIP_TRY(hipGraphLaunch(m->exec, st));
    m->graph_launches++;
    if (o.stats) return finish_stats(m->d_totals, o.counters, o.stats, st);
    return KR_OK;
  } KR_CATCH
}

/* ------------------------------------------------------------------------ */
/* learned Newton guess (BF16 MFMA MLP)                                      */
/* ------------------------------------------------------------------------ */
#include "kr_mlp.hip"
