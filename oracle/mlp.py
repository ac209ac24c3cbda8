"""Learned importance proposal over cut terms: fp64 MLP with hand-derived
backprop, the proposal q, term sampling and the importance-sampling
estimator of the recombination sum (test infrastructure).

The recombination sum (Sec. V-C) is R[b] = sum_P w_P(b) with
w_P(b) = 2^-k prod_f T_f[b_f; P|f] over the 4^k cut terms (Sec. III-B: the
cost grows as 4^k).  A proposal q over terms gives the unbiased estimator
    R_hat[b] = (1/N) sum_j w_{P_j}(b) / q(P_j),   P_j ~ q.
Readings (the paper has no learned part):
* the network regresses y(P) = log(||w_P||_2 + 2^-60) with mean squared
  error; q = (1 - eps) softmax(y_hat) + eps / 4^k (defensive mixture,
  eps = 0.05);
* the network is F -> H -> H -> H -> 1 with ReLU activations;
* term sampling: integer weights W_P = floor(q_P 2^40), inclusive prefix
  sums C_P; draw j takes u = (o1 2^32 + o0) mod C_last from
  philox(ctr = (j, 0, lo32(cid), hi32(cid)), key = (lo32(seed) ^ 0x7E570001,
  hi32(seed))) and picks the smallest P with C_P > u (the modulo bias is at
  most C_last / 2^64).
* term features (F = 6k, padded to a multiple of 64): per cut c, a one-hot
  of P_c, then phi(s_up) and phi(s_dn), where s_side(c, p) is the share of
  the squared column-norm mass of the fragment on that side of cut c (up =
  the fragment where c is a quantum output, dn = where it is a quantum
  input) carried by columns whose digit for c equals p, and
  phi(s) = max(ln s, -40) / 40.
"""
from __future__ import annotations

import numpy as np

from .philox import philox4x32_10

EPS = 0.05
LABEL_FLOOR = 2.0 ** -60


def init_params(F: int, H: int, seed: int):
    """He-style uniform initialisation; returns a list of (W, b) with W of
    shape (out, in)."""
    rng = np.random.default_rng([seed, 31])
    dims = [F, H, H, H, 1]
    params = []
    for i in range(4):
        fan_in = dims[i]
        lim = np.sqrt(6.0 / fan_in) if i < 3 else np.sqrt(3.0 / fan_in)
        W = rng.uniform(-lim, lim, size=(dims[i + 1], fan_in))
        b = np.zeros(dims[i + 1])
        params.append((W, b))
    return params


def forward(params, X):
    """Returns the prediction y_hat (shape (B,)) and the activations."""
    acts = [X]
    h = X
    for i, (W, b) in enumerate(params):
        z = h @ W.T + b
        h = np.maximum(z, 0.0) if i < 3 else z
        acts.append(h)
    return h[:, 0], acts


def loss_and_grads(params, X, y):
    """Mean squared error and its gradients, by hand:
    L = mean (y_hat - y)^2;  dL/dy_hat = 2 (y_hat - y) / B;
    for a layer z = h W^T + b:  dW = dz^T h,  db = sum dz,  dh = dz W;
    through a ReLU, dz = dh * [z > 0] (and [h > 0] is the same test)."""
    y_hat, acts = forward(params, X)
    B = X.shape[0]
    r = y_hat - y
    L = float(np.mean(r * r))
    dz = (2.0 / B) * r[:, None]
    grads = [None] * 4
    for i in range(3, -1, -1):
        W, b = params[i]
        h_in = acts[i]
        grads[i] = (dz.T @ h_in, dz.sum(axis=0))
        if i > 0:
            dh = dz @ W
            dz = dh * (acts[i] > 0.0)
    return L, grads


def adam_step(params, grads, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Adam (Kingma & Ba) on every tensor; state holds (m, v, t)."""
    m, v, t = state
    t += 1
    new = []
    for i, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        out = []
        for j, (p, g) in enumerate(((W, gW), (b, gb))):
            m[i][j] = b1 * m[i][j] + (1 - b1) * g
            v[i][j] = b2 * v[i][j] + (1 - b2) * g * g
            mh = m[i][j] / (1 - b1 ** t)
            vh = v[i][j] / (1 - b2 ** t)
            out.append(p - lr * mh / (np.sqrt(vh) + eps))
        new.append(tuple(out))
    return new, (m, v, t)


def adam_state(params):
    m = [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]
    v = [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]
    return (m, v, 0)


# ------------------------------------------------------------ proposal

def proposal(logits, eps=EPS):
    """q = (1 - eps) softmax(logits) + eps / K."""
    z = logits - logits.max()
    e = np.exp(z)
    return (1.0 - eps) * e / e.sum() + eps / logits.size


def integer_cdf(q):
    W = np.floor(q * 2.0 ** 40).astype(np.uint64)
    return np.cumsum(W, dtype=np.uint64)


def sample_terms(cdf, n, seed, cid):
    """n term indices drawn by inverse CDF from the Philox stream above."""
    total = int(cdf[-1])
    key = ((seed & 0xFFFFFFFF) ^ 0x7E570001, (seed >> 32) & 0xFFFFFFFF)
    out = np.empty(n, dtype=np.int64)
    for j in range(n):
        o = philox4x32_10((j, 0, cid & 0xFFFFFFFF, (cid >> 32) & 0xFFFFFFFF), key)
        u = ((o[1] << 32) | o[0]) % total
        out[j] = int(np.searchsorted(cdf, np.uint64(u), side="right"))
    return out


def is_estimate(term_weight, terms, q):
    """R_hat[b] = (1/N) sum_j w_{P_j}(b) / q(P_j); term_weight(P) returns
    the vector w_P(b) over all b."""
    acc = None
    for P in terms:
        v = term_weight(int(P)) / q[P]
        acc = v if acc is None else acc + v
    return acc / len(terms)


def is_stderr_l1(term_weight, terms, q):
    """Summed plug-in standard error of R_hat: with Y_j = w_{P_j} / q(P_j),
    se[b] = sqrt(max(0, (1/N^2) sum_j Y_j[b]^2 - R_hat[b]^2 / N)), the
    square root of the population variance of the Y_j[b] over N; returns
    sum_b se[b]."""
    N = len(terms)
    s1 = s2 = None
    for P in terms:
        v = term_weight(int(P)) / q[P]
        s1 = v if s1 is None else s1 + v
        s2 = v * v if s2 is None else s2 + v * v
    est = s1 / N
    return float(np.sum(np.sqrt(np.maximum(0.0, s2 / (N * N) - est * est / N))))


# ------------------------------------------------------ term model inputs

FEATURE_FLOOR = -40.0
# the network regresses y / LABEL_SCALE; its logits are LABEL_SCALE times
# its output
LABEL_SCALE = 40.0


def column_norms(T):
    """n_f[p] = ||T_f[.; p]||_2 for a fragment tensor T_f[b][p]."""
    return np.sqrt(np.sum(np.asarray(T, dtype=np.float64) ** 2, axis=0))


def cut_shares(frags, tensors, k):
    """(up, dn): arrays [k][4]; side[c][p] = sum over columns p_f of the
    fragment on that side of cut c with digit p on c of n_f[p_f]^2, divided
    by the sum over all columns."""
    up = np.zeros((k, 4))
    dn = np.zeros((k, 4))
    for f, T in zip(frags, tensors):
        n2 = column_norms(T) ** 2
        tot = n2.sum()
        idx = np.arange(n2.size)
        for j, ax in enumerate(f.axes):
            digit = (idx >> (2 * j)) & 3
            share = np.array([n2[digit == p].sum() for p in range(4)]) / tot
            (up if ax.side == 0 else dn)[ax.cut] = share
    return up, dn


def phi(s):
    with np.errstate(divide="ignore"):
        return np.maximum(np.log(np.asarray(s, dtype=np.float64)), FEATURE_FLOOR) / -FEATURE_FLOOR


def features(P, k, up, dn, F=None):
    """Feature row of term P (length F, default 6k rounded up to 64)."""
    if F is None:
        F = -(-6 * k // 64) * 64
    x = np.zeros(F)
    for c in range(k):
        p = (P >> (2 * c)) & 3
        x[6 * c + p] = 1.0
        x[6 * c + 4] = phi(up[c][p])
        x[6 * c + 5] = phi(dn[c][p])
    return x


def log_weight(P, frags, tensors, k):
    """y(P) = ln(2^-k prod_f n_f[P|f] + 2^-60): the outer-product structure
    of w_P makes its 2-norm the product of the fragments' column norms."""
    v = 2.0 ** (-k)
    for f, T in zip(frags, tensors):
        v *= column_norms(T)[f.p_index(P)]
    return float(np.log(v + LABEL_FLOOR))


def term_vector(frags, reqs, tensors, k, P, nq):
    """w_P(b) = 2^-k prod_f T_f[b_f; P|f] over all 2^nq outputs b."""
    b = np.arange(1 << nq, dtype=np.int64)
    out = np.full(1 << nq, 2.0 ** (-k))
    for f, r, T in zip(frags, reqs, tensors):
        bi = np.zeros_like(b)
        for i, u in enumerate(r.req_user):
            bi |= ((b >> u) & 1) << i
        out = out * T[bi, f.p_index(P)]
    return out
