/*
 * kr_thermo.h -- per-species thermal energy and heat capacity, and the
 * tabulated rate factors (gfx950; both device layouts), over the tables the
 * network compiler generates.
 *
 * Heat capacities (paper Sec. 2.2: T follows from eps through c_V(T, n);
 * Sec. 4.2: c_V as piecewise polynomials in T, NASA style): with KR_CV_POLY
 * the network gives per species c_V,s(T)/k_B = sum_k a_k T^k on T < T_mid
 * and on T >= T_mid (kr_cvp) and e_s(T) = T sum_k a_k T^k / (k + 1) + const
 * (kr_evp, the constant making e_s continuous at T_mid); the energy
 * equation is written in eps = sum_s n_s e_s(T).  Without it c_V,s is the
 * constant kr_cv[s] and e_s = c_s T.
 *
 * Photoreactions (Sec. 2.2.1, second rate type; with KR_PHOTO): the
 * effective flux of the cell and its derivative (kr_photo_flux).
 *
 * Tabulated factors (Sec. 2.2.1, third rate type, with analytic dk/dT): a
 * table t holds log2 tau_t at nodes log2 T = kr_tab_x0 + i / kr_tab_idx;
 * between nodes log2 tau is linear in log2 T (the end segments extended),
 * so d ln tau / d ln T is the segment's slope.
 */

#if KR_CV_POLY
/* c_V,s and e_s of species s at T (s a compile-time index in the lane
 * layout: the coefficients fold into selects of constants) */
template <typename R>
__device__ __forceinline__ void kr_species_thermo(int s, R T, R &e, R &c) {
  const bool up = T >= R(kr_T_mid);
  R cc = up ? R(kr_cvp[s][1][4]) : R(kr_cvp[s][0][4]);
  R ee = up ? R(kr_evp[s][1][4]) : R(kr_evp[s][0][4]);
#pragma unroll
  for (int k = 3; k >= 0; --k) {
    cc = fma(cc, T, up ? R(kr_cvp[s][1][k]) : R(kr_cvp[s][0][k]));
    ee = fma(ee, T, up ? R(kr_evp[s][1][k]) : R(kr_evp[s][0][k]));
  }
  c = cc;
  e = fma(ee, T, up ? R(kr_evp[s][1][5]) : R(0));
}
#endif

#if KR_PHOTO
/* Effective photon flux of the cell (Sec. 2.2.1 and eq.
 * method-rad-equiv-flux: the optically thin flux F averaged over the path L
 * through the cell's own absorbers, inverse absorption length linv):
 * Fe = F (1 - e^-tau) / tau, tau = L linv, and dFe = dFe / dlinv; below
 * tau = 1e-4 the two-term series of both. */
template <typename R>
__device__ __forceinline__ void kr_photo_flux(R F, R L, R linv, R &Fe, R &dFe) {
  const R tau = L * linv;
  R g, dg;
  if (tau < R(1e-4)) {
    g = R(1) - tau * R(0.5) + tau * tau * R(1.0 / 6.0);
    dg = R(-0.5) + tau * R(1.0 / 3.0) - tau * tau * R(0.125);
  } else {
    const R em = expm1(-tau);
    g = -em / tau;
    dg = (tau * exp(-tau) + em) / (tau * tau);
  }
  Fe = F * g;
  dFe = F * L * dg;
}
#endif

#if KR_NTAB > 0
/* log2 tau_t at log2 T = l2T; slope = d log2 tau / d log2 T */
template <typename R>
__device__ __forceinline__ R kr_tab_log2(int t, R l2T, R &slope) {
  const R u = (l2T - R(kr_tab_x0)) * R(kr_tab_idx);
  int i = (int)floor(u);
  i = i < 0 ? 0 : (i > KR_TAB_NODES - 2 ? KR_TAB_NODES - 2 : i);
  const R f = u - R(i);
  const R L0 = R(kr_tab[t][i]), L1 = R(kr_tab[t][i + 1]);
  slope = (L1 - L0) * R(kr_tab_idx);
  return fma(f, L1 - L0, L0);
}
#endif
