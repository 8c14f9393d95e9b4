"""Plain FP64 reference of the learned-guess MLP (TEST INFRASTRUCTURE ONLY).

Same model and rounding points as the library's BF16 MFMA kernels, written
with numpy matrix products: a0 = bf16(standardised x); z_l = a_{l-1}
bf16(W_l)^T + b_l; a_l = bf16(gelu(z_l)); out = a_L bf16(W_out)^T + b_out;
loss = mean((out - t)^2) with t the standardised target; d_out = 2 (out -
t) / (B n_out); dW_l = bf16(dz_l)^T a_{l-1}; db_l = sum_b dz_l; da_{l-1} =
bf16(dz_l) bf16(W_l); dz_{l-1} = da_{l-1} * gelu'(z_{l-1}).  With
``rounding=False`` every bf16() is the identity, which turns this into the
exact FP64 gradient of the same function (pinned by finite differences).

Parameter layout: for each linear layer, W [fan_out][fan_in] row-major then
b [fan_out], flattened in layer order.  Normalisation block: mu_in[16],
sd_in[16], mu_out[16], sd_out[16].

The map between a cell and the network (the learned Newton start of one
backward-Euler substep; the paper names a learned solver as the route to
acceleration, Sec. 5): inputs are log10 max(n_s / n_nuc, 1e-20) for every
species, log10 T and log10 h (n_nuc the nuclei density, sum over species of
atoms times abundance); outputs are the change of those species logarithms
and of log10 T over the substep; the starting point maps back as
n_nuc 10^(x_s + dx_s) and T 10^(dlog10 T).  All in FP64 here.
"""
from __future__ import annotations

import numpy as np

SQRT_2_OVER_PI = np.sqrt(2.0 / np.pi)


def bf16_round(x) -> np.ndarray:
    """Round to float32, then to bfloat16 (nearest, ties to even); returned
    as float64 values."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(SQRT_2_OVER_PI * (z + 0.044715 * z ** 3)))


def gelu_grad(z):
    t = np.tanh(SQRT_2_OVER_PI * (z + 0.044715 * z ** 3))
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * SQRT_2_OVER_PI * (1.0 + 3 * 0.044715 * z * z)


def layer_shapes(n_in, n_out, hidden, layers):
    return [(hidden if l < layers else n_out, n_in if l == 0 else hidden) for l in range(layers + 1)]


def unflatten(w, n_in, n_out, hidden, layers):
    out, off = [], 0
    for fo, fi in layer_shapes(n_in, n_out, hidden, layers):
        W = np.asarray(w[off:off + fo * fi], np.float64).reshape(fo, fi)
        off += fo * fi
        b = np.asarray(w[off:off + fo], np.float64)
        off += fo
        out.append((W, b))
    return out


def flatten(parts):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in parts])


class MLP:
    def __init__(self, n_in, n_out, hidden, layers, rounding=True):
        self.n_in, self.n_out, self.hidden, self.layers = n_in, n_out, hidden, layers
        self.rnd = bf16_round if rounding else (lambda a: np.asarray(a, np.float64))

    def forward(self, w, norm, X):
        """Returns (out, cache) for raw features X [B, n_in]."""
        P = unflatten(w, self.n_in, self.n_out, self.hidden, self.layers)
        mu, sd = norm[:self.n_in], norm[16:16 + self.n_in]
        a = self.rnd((np.asarray(X, np.float64) - mu) / sd)
        acts, zs = [a], []
        for l in range(self.layers):
            W, b = P[l]
            z = a @ self.rnd(W).T + b
            a = self.rnd(gelu(z))
            zs.append(z)
            acts.append(a)
        W, b = P[-1]
        out = a @ self.rnd(W).T + b
        return out, (P, acts, zs)

    def targets(self, norm, Y):
        return (np.asarray(Y, np.float64) - norm[32:32 + self.n_out]) / norm[48:48 + self.n_out]

    def loss(self, w, norm, X, Y):
        out, _ = self.forward(w, norm, X)
        return float(np.mean((out - self.targets(norm, Y)) ** 2))

    def gradient_scales(self, w, norm, X, Y):
        """Per-entry scale of the gradient's rounding error: the gradient's
        sums taken over absolute values (|bf16(dz)|^T |a| for weights,
        sum |dz| for biases), same layout as the gradient.  An entry's
        accumulation error is a small multiple of its scale whatever the
        cancellation between the summed terms."""
        out, (P, acts, zs) = self.forward(w, norm, X)
        t = self.targets(norm, Y)
        B = out.shape[0]
        d = 2.0 * (out - t) / (B * self.n_out)
        scales = [None] * (self.layers + 1)
        dz = d
        for l in range(self.layers, -1, -1):
            W, _ = P[l]
            dzr = self.rnd(dz)
            scales[l] = (np.abs(dzr).T @ np.abs(acts[l]), np.abs(dz).sum(axis=0))
            if l > 0:
                dz = (dzr @ self.rnd(W)) * gelu_grad(zs[l - 1])
        return flatten(scales)

    def gradients(self, w, norm, X, Y):
        """(loss, flat gradient) of the mean squared error."""
        out, (P, acts, zs) = self.forward(w, norm, X)
        t = self.targets(norm, Y)
        B = out.shape[0]
        loss = float(np.mean((out - t) ** 2))
        d = 2.0 * (out - t) / (B * self.n_out)
        grads = [None] * (self.layers + 1)
        dz = d
        for l in range(self.layers, -1, -1):
            W, _ = P[l]
            dzr = self.rnd(dz)
            grads[l] = (dzr.T @ acts[l], dz.sum(axis=0))
            if l > 0:
                dz = (dzr @ self.rnd(W)) * gelu_grad(zs[l - 1])
        return loss, flatten(grads)


def adam_step(w, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), returns (w, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


# --------------------------------------------------------------------------
# the cell <-> network map (features, targets, starting point)
# --------------------------------------------------------------------------

FRACTION_FLOOR = 1e-20


def nuclei(atoms, n):
    """n_nuc per cell: sum_s atoms_s n_s for n [S, cells]."""
    return np.asarray(atoms, np.float64) @ np.asarray(n, np.float64)


def log_fractions(atoms, n):
    """log10 max(n_s / n_nuc, 1e-20), [S, cells]."""
    n = np.asarray(n, np.float64)
    return np.log10(np.maximum(n / nuclei(atoms, n)[None, :], FRACTION_FLOOR))


def features(atoms, n, T, h):
    """Raw inputs [cells, S + 2] (FP64) of cells n [S, cells], T [cells] and
    substep lengths h [cells] (or a scalar)."""
    lf = log_fractions(atoms, n)
    T = np.asarray(T, np.float64)
    h = np.broadcast_to(np.asarray(h, np.float64), T.shape)
    return np.concatenate([lf.T, np.log10(T)[:, None], np.log10(h)[:, None]], axis=1)


def targets(atoms, n_before, T_before, n_after, T_after):
    """Raw targets [cells, S + 1]: change of the species logarithms and of
    log10 T from before to after."""
    d = log_fractions(atoms, n_after) - log_fractions(atoms, n_before)
    dT = np.log10(np.asarray(T_after, np.float64)) - np.log10(np.asarray(T_before, np.float64))
    return np.concatenate([d.T, dT[:, None]], axis=1)


def starting_point(atoms, n, T, out, norm):
    """The Newton starting point [S + 1, cells] from the network's
    standardised outputs out [cells, S + 1]: the predicted change
    dx = out * sd_out + mu_out applied to the log fractions and to log10 T."""
    n = np.asarray(n, np.float64)
    S = n.shape[0]
    out = np.asarray(out, np.float64)
    norm = np.asarray(norm, np.float64)
    dx = out * norm[48:48 + S + 1][None, :] + norm[32:32 + S + 1][None, :]
    nn = nuclei(atoms, n)
    y = np.empty((S + 1, n.shape[1]))
    y[:S] = nn[None, :] * 10.0 ** (log_fractions(atoms, n) + dx[:, :S].T)
    y[S] = np.asarray(T, np.float64) * 10.0 ** dx[:, S]
    return y
