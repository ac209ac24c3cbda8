"""Maximum-likelihood fragment correction, plainly (Sec. V-C, distribution
builder): before the contraction the fragment models are made
self-consistent, which mitigates the sampling error of the variant data.

Test infrastructure: only the tests, the smoke check and the benchmark's
CPU baseline use this module; the GPU path never does.

The paper names the step and defers its details to its reference on
maximum-likelihood fragment tomography.  The reading taken here, whose
parity is pinned by the mathematics of each step:

* the model of a fragment under one preparation combination s of its
  quantum inputs is the set of conditional states {rho_x}: rho_x is the
  unnormalised state of the fragment's quantum outputs jointly with the
  outcome x of its requested circuit outputs, so that
      p(o, x | s, b) = Tr(Pi_{b,o} rho_x)
  for the measurement basis combination b on the quantum outputs and their
  outcome o (Pi_{b,o} the product of the one-qubit eigenprojectors);
* a model is physical (self-consistent) when every rho_x is positive
  semidefinite and sum_x Tr rho_x = 1;
* the raw model is the least-squares linear inversion of the variant data:
  the Pauli coefficient Tr(sigma_P rho_x) is the mean, over every basis
  combination that measures P (the basis letter equals P's letter on every
  qubit where P is not the identity), of that basis's parity estimate
  sum_o (-1)^(o on P's support) p(o, x | s, b).  For Pauli products
  measured with equal shots this mean is the least-squares solution;
* the corrected model is the physical model nearest the raw one in the
  Frobenius norm, the maximum-likelihood model under Gaussian noise
  (Smolin, Gambetta and Smith 2012): the blocks rho_x are diagonalised and
  their joint spectrum is projected onto the probability simplex
  {lambda >= 0, sum lambda = 1}, eigenvectors kept;
* the corrected model goes on as corrected variant data,
  p'(o, x | s, b) = Tr(Pi_{b,o} rho'_x), so the Pauli-basis transform and
  the contraction stay as they are.  A fragment without quantum outputs is
  left unchanged: its histograms already are a physical model.
"""
from __future__ import annotations

import itertools

import numpy as np

from .cutting import BASIS_X, BASIS_Y, BASIS_Z, I_, X_, Y_, Z_

SIGMA = {
    I_: np.eye(2, dtype=np.complex128),
    X_: np.array([[0, 1], [1, 0]], dtype=np.complex128),
    Y_: np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    Z_: np.array([[1, 0], [0, -1]], dtype=np.complex128),
}
BASIS_PAULI = {BASIS_X: X_, BASIS_Y: Y_, BASIS_Z: Z_}


def kron_all(mats):
    """The tensor product, first factor most significant (qubit 0 first)."""
    out = np.eye(1, dtype=np.complex128)
    for m in mats:
        out = np.kron(out, m)
    return out


def simplex_projection(mu) -> np.ndarray:
    """Euclidean projection of mu onto {lambda >= 0, sum lambda = 1}:
    lambda = max(mu - tau, 0) with the shift tau that makes the sum 1.
    With the entries sorted in descending order u_1 >= u_2 >= ..., r is the
    largest i with u_i > (u_1 + ... + u_i - 1) / i and tau is that ratio
    for i = r (for a spectrum of trace 1 this is the eigenvalue step of
    Smolin, Gambetta and Smith)."""
    mu = np.asarray(mu, dtype=np.float64)
    u = np.sort(mu)[::-1]
    css = np.cumsum(u)
    i = np.arange(1, len(u) + 1)
    r = int(i[u - (css - 1.0) / i > 0][-1])
    tau = (css[r - 1] - 1.0) / r
    return np.maximum(mu - tau, 0.0)


def raw_states(p: np.ndarray) -> np.ndarray:
    """The least-squares conditional states of one preparation combination.
    p[b][o][x]: p(o, x | b) for basis combination b (base 3 over the n
    quantum outputs, output 0 least significant, digits X, Y, Z) and outcome
    o (bit i = output i).  Returns rho[x] (d x d, d = 2^n), with output i the
    i-th tensor factor."""
    nb, d, nx = p.shape
    n = d.bit_length() - 1
    assert nb == 3 ** n and d == 1 << n
    bases = [tuple((bi // 3 ** i) % 3 for i in range(n)) for bi in range(nb)]
    rho = np.zeros((nx, d, d), dtype=np.complex128)
    for P in itertools.product((I_, X_, Y_, Z_), repeat=n):
        sign = np.array([(-1.0) ** sum((o >> i) & 1 for i in range(n) if P[i] != I_) for o in range(d)])
        ests = [sign @ p[bi] for bi, b in enumerate(bases)
                if all(P[i] == I_ or BASIS_PAULI[b[i]] == P[i] for i in range(n))]
        c = np.mean(ests, axis=0)                       # Tr(sigma_P rho_x) for every x
        rho += c[:, None, None] * kron_all([SIGMA[q] for q in P])[None] / d
    return rho


def project_states(rho: np.ndarray) -> np.ndarray:
    """The physical model nearest {rho_x} in the Frobenius norm: the joint
    spectrum projected onto the simplex, each block's eigenvectors kept."""
    nx, d, _ = rho.shape
    w, V = np.linalg.eigh(rho)
    lam = simplex_projection(w.reshape(-1)).reshape(nx, d)
    return np.einsum("xik,xk,xjk->xij", V, lam, V.conj())


def model_probabilities(rho: np.ndarray) -> np.ndarray:
    """p[b][o][x] = Tr(Pi_{b,o} rho_x), layout of raw_states' input."""
    nx, d, _ = rho.shape
    n = d.bit_length() - 1
    nb = 3 ** n
    out = np.zeros((nb, d, nx))
    for bi in range(nb):
        b = [(bi // 3 ** i) % 3 for i in range(n)]
        for o in range(d):
            Pi = kron_all([(SIGMA[I_] + (-1.0) ** ((o >> i) & 1) * SIGMA[BASIS_PAULI[b[i]]]) / 2
                           for i in range(n)])
            out[bi, o] = np.real(np.einsum("ij,xji->x", Pi, rho))
    return out


def correct_block(p: np.ndarray) -> np.ndarray:
    """One preparation combination: raw data p[b][o][x] in, the corrected
    model's probabilities in the same layout out."""
    return model_probabilities(project_states(raw_states(p)))


def correct_tables(frag, req, dists: np.ndarray) -> np.ndarray:
    """Corrected variant tables ``[n_variants][2^len(meas)]`` of a fragment
    (layout of ``cutting.variant_distributions``)."""
    outs = [j for j, ax in enumerate(frag.axes) if ax.side == 0]
    if not outs:
        return dists.copy()
    ins = [j for j, ax in enumerate(frag.axes) if ax.side == 1]
    n, d = len(outs), 1 << len(outs)
    opos = [req.out_pos[j] for j in outs]
    xpos = list(req.req_pos)
    nx = 1 << len(xpos)

    def col(o, x):
        idx = 0
        for i, q in enumerate(opos):
            idx |= ((o >> i) & 1) << q
        for i, q in enumerate(xpos):
            idx |= ((x >> i) & 1) << q
        return idx

    out = dists.copy()
    for s in itertools.product(range(4), repeat=len(ins)):
        rows = []
        for bi in range(3 ** n):
            digits = [0] * len(frag.axes)
            for j, dg in zip(ins, s):
                digits[j] = dg
            for i, j in enumerate(outs):
                digits[j] = (bi // 3 ** i) % 3
            rows.append(frag.variant_index(digits))
        p = np.array([[[dists[rows[bi], col(o, x)] for x in range(nx)] for o in range(d)]
                      for bi in range(3 ** n)])
        q = correct_block(p)
        for bi in range(3 ** n):
            for o in range(d):
                for x in range(nx):
                    out[rows[bi], col(o, x)] = q[bi, o, x]
    return out
