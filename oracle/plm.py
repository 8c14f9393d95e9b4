"""Plain FP64 reference of the stoichiometry-compatible PLM advection of
chemical species (TEST INFRASTRUCTURE ONLY: tests, smoke and the benchmark's
CPU-baseline leg use it; the product library never does).

What it computes (paper Sec. 2.1, eqs. method-flux-sp, method-recon-general,
method-plm-general, method-sto-plm-def, method-sto-plm-proj,
method-sto-plm-recon), for a 1-D line of cells with periodic boundaries:

* cell values of the species per mass, x_s = n_s / rho;
* per cell, forward and backward slopes over the cell-centre spacing and the
  geometric coefficients c_f = (xc_{i+1} - xc_i) / (xf_{i+1/2} - xc_i),
  c_b = (xc_i - xc_{i-1}) / (xc_i - xf_{i-1/2}) (eq. method-sto-plm-def; the
  forward coefficient's denominator is read as the distance from the cell
  centre to its own right face, the printed index being garbled);
* the limited slope of the modified van Leer limiter for non-uniform grids
  the paper cites (Mignone 2014): zero where the two slopes differ in sign,
  else df db (c_f db + c_b df) / (df^2 + (c_f + c_b - 2) df db + db^2),
  the harmonic mean 2 df db / (df + db) on a uniform grid;
* the correction chi = slope * (face - centre) of the face's two adjacent
  cells (eq. method-plm-general), projected onto the stoichiometric space,
  x_face = x_cell + P chi (eq. method-sto-plm-proj), P = V V^T from the SVD
  of the element-species matrix with V the right singular vectors of zero
  singular value (the null space of N); without projection x_face = x_cell
  + chi (the uncorrected PLM the paper compares against);
* the upwind face state by the sign of the mass flux (eq.
  method-sto-plm-recon), the species flux F_s = x_s F_rho (eq.
  method-flux-sp), and the conservative update n_s -= dt / dx (F_s(i+1/2) -
  F_s(i-1/2)), with rho updated alike by the mass fluxes;
* two such stages as the second-order strong-stability-preserving
  Runge-Kutta step (Heun's form) for the advection test of Sec. 4.1.

Every function takes arrays [S, cells] (species rows) like the library.
"""
from __future__ import annotations

import numpy as np


def projector_svd(comp):
    """P = V V^T, V the right singular vectors of N (rows: conserved rows,
    columns: species) belonging to zero singular values."""
    N = np.asarray(comp, np.float64)
    S = N.shape[1]
    if N.shape[0] == 0:
        return np.eye(S)
    u, sv, vt = np.linalg.svd(N, full_matrices=True)
    rank = int(np.sum(sv > sv.max() * S * np.finfo(float).eps)) if sv.size else 0
    V = vt[rank:].T
    return V @ V.T


def limited_slope(df, db, cf, cb):
    """Modified van Leer slope for non-uniform grids (elementwise)."""
    df = np.asarray(df, np.float64)
    db = np.asarray(db, np.float64)
    prod = df * db
    den = df * df + (cf + cb - 2.0) * prod + db * db
    with np.errstate(invalid="ignore", divide="ignore"):
        s = prod * (cf * db + cb * df) / den
    return np.where(prod > 0.0, s, 0.0)


def face_states(x, xc, xf, P=None, limit=True):
    """Left and right states of every face i-1/2 (i = 0..n-1, periodic) of a
    line: x [S, n] cell values, xc [n] centres, xf [n+1] faces (xf[i] the left
    face of cell i, xf[n] - xf[0] the period).  Returns (xl, xr), each
    [S, n]: xl[:, i] from cell i-1 at face i-1/2, xr[:, i] from cell i.
    limit=False gives zero corrections (donor cell)."""
    x = np.asarray(x, np.float64)
    S, n = x.shape
    L = xf[n] - xf[0]
    # centres and faces of the periodic neighbours
    idx = np.arange(n)
    xcm = np.where(idx == 0, xc[n - 1] - L, xc[(idx - 1) % n])
    xcp = np.where(idx == n - 1, xc[0] + L, xc[(idx + 1) % n])
    df = (x[:, (idx + 1) % n] - x) / (xcp - xc)[None, :]
    db = (x - x[:, (idx - 1) % n]) / (xc - xcm)[None, :]
    cf = (xcp - xc) / (xf[idx + 1] - xc)
    cb = (xc - xcm) / (xc - xf[idx])
    slope = limited_slope(df, db, cf[None, :], cb[None, :]) if limit else np.zeros_like(x)
    chi_right_face = slope * (xf[idx + 1] - xc)[None, :]     # cell i at face i+1/2
    chi_left_face = slope * (xf[idx] - xc)[None, :]          # cell i at face i-1/2
    if P is not None:
        chi_right_face = P @ chi_right_face
        chi_left_face = P @ chi_left_face
    xr = x + chi_left_face                                     # right state of face i-1/2
    xl_at_right = x + chi_right_face                           # left state of face i+1/2
    xl = xl_at_right[:, (idx - 1) % n]                         # left state of face i-1/2
    return xl, xr


def stage(n, rho, F_rho, xc, xf, dt, P=None, limit=True):
    """One forward-Euler stage: (n', rho') after dt with the face mass fluxes
    F_rho [n] (face i-1/2 of cell i)."""
    n = np.asarray(n, np.float64)
    x = n / rho[None, :]
    xl, xr = face_states(x, xc, xf, P, limit)
    xface = np.where(F_rho[None, :] > 0.0, xl, xr)
    Fs = xface * F_rho[None, :]
    idx = np.arange(n.shape[1])
    dx = xf[idx + 1] - xf[idx]
    nn = n - dt / dx[None, :] * (Fs[:, (idx + 1) % n.shape[1]] - Fs)
    rr = rho - dt / dx * (F_rho[(idx + 1) % n.shape[1]] - F_rho)
    return nn, rr


def ssp_rk2(n, rho, v, xc, xf, dt, P=None, limit=True):
    """One SSP-RK2 step for a constant velocity v: the face mass flux is the
    upwind density times v."""
    def flux(r):
        idx = np.arange(r.size)
        return (r[(idx - 1) % r.size] if v > 0 else r) * v
    n1, r1 = stage(n, rho, flux(rho), xc, xf, dt, P, limit)
    n2, r2 = stage(n1, r1, flux(r1), xc, xf, dt, P, limit)
    return 0.5 * (n + n2), 0.5 * (rho + r2)


# --------------------------------------------------------------------------
# the advection test of Sec. 4.1 (its inputs: synthetic.e1_initial)
# --------------------------------------------------------------------------

E1_COMP = np.array([[1, 2, 1, 0],      # element A
                    [0, 0, 1, 1]])     # element B
