"""Pins for the learned-proposal oracle: hand-derived gradients against
finite differences, Adam against its definition on a quadratic, the
proposal's normalisation, term sampling against the empirical distribution,
and unbiasedness of the importance-sampling estimator."""
import numpy as np
import pytest

from oracle import mlp


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    F, H, B = 7, 9, 13
    params = mlp.init_params(F, H, 1)
    params = [(W + 0.05 * rng.normal(size=W.shape), b + 0.1 * rng.normal(size=b.shape)) for W, b in params]
    X = rng.normal(size=(B, F))
    y = rng.normal(size=B)
    L, grads = mlp.loss_and_grads(params, X, y)
    h = 1e-6
    for i in range(4):
        for j in range(2):
            p = params[i][j]
            g = grads[i][j]
            idx = [tuple(rng.integers(0, s) for s in p.shape) for _ in range(6)]
            for ix in idx:
                plus = [list(t) for t in params]
                minus = [list(t) for t in params]
                pp = p.copy(); pp[ix] += h
                pm = p.copy(); pm[ix] -= h
                plus[i][j] = pp
                minus[i][j] = pm
                Lp, _ = mlp.loss_and_grads([tuple(t) for t in plus], X, y)
                Lm, _ = mlp.loss_and_grads([tuple(t) for t in minus], X, y)
                fd = (Lp - Lm) / (2 * h)
                assert abs(fd - g[ix]) <= 1e-6 * max(1.0, abs(fd)), (i, j, ix)


def test_training_reduces_loss():
    rng = np.random.default_rng(2)
    X = rng.normal(size=(256, 6))
    y = np.sin(X[:, 0]) + 0.5 * X[:, 1] ** 2
    params = mlp.init_params(6, 32, 3)
    st = mlp.adam_state(params)
    L0, _ = mlp.loss_and_grads(params, X, y)
    for _ in range(300):
        L, g = mlp.loss_and_grads(params, X, y)
        params, st = mlp.adam_step(params, g, st, 1e-2)
    assert L < 0.1 * L0


def test_adam_matches_definition_on_quadratic():
    params = [(np.array([[3.0]]), np.array([0.0]))] * 4
    grads = [(np.array([[6.0]]), np.array([0.0]))] * 4
    st = mlp.adam_state(params)
    new, _ = mlp.adam_step(params, grads, st, 0.1)
    # first Adam step moves each coordinate by lr * sign(g) (bias-corrected m/sqrt(v) = g/|g|)
    assert np.isclose(new[0][0][0, 0], 3.0 - 0.1, atol=1e-7)


def test_adam_constant_gradient_moves_lr_every_step():
    """Bias correction at every step: with a constant gradient g the
    corrected moments are exactly g and g^2 at every t, so every step (not
    only the first) moves each coordinate by lr g / (|g| + eps).  A missing or
    wrong bias correction, or a moment update without its (1 - beta)
    factor, moves by a different amount from t = 2 on."""
    p0 = [(np.array([[3.0, -1.0]]), np.array([0.5]))]
    g = [(np.array([[6.0, -0.25]]), np.array([1e-3]))]
    st = mlp.adam_state(p0)
    params = p0
    lr = 0.01
    for t in range(1, 6):
        prev = params
        params, st = mlp.adam_step(params, g, st, lr)
        assert st[2] == t
        for (W1, b1), (W0, b0), (gW, gb) in zip(params, prev, g):
            assert np.allclose(W1 - W0, -lr * gW / (np.abs(gW) + 1e-8), rtol=1e-12, atol=0)
            assert np.allclose(b1 - b0, -lr * gb / (np.abs(gb) + 1e-8), rtol=1e-12, atol=0)


def test_adam_alternating_gradient_closed_form():
    """Gradients g then -g: after two steps the first moment is
    (1 - b1)(b1 g - g) = -g (1 - b1)^2, corrected -g (1 - b1) / (1 + b1); the
    second moment (1 - b2)(b2 + 1) g^2, corrected g^2; so the second step moves
    by +lr (1 - b1) / (1 + b1) sign(g) (= lr / 19 for b1 = 0.9).  At t = 3
    with g again: m_hat = g (b1^2 - b1 + 1)(1 - b1) / (1 - b1^3), v_hat = g^2."""
    g = 4.0
    lr = 0.1
    p = [(np.array([[1.0]]), np.array([0.0]))]
    st = mlp.adam_state(p)
    p1, st = mlp.adam_step(p, [(np.array([[g]]), np.array([0.0]))], st, lr)
    p2, st = mlp.adam_step(p1, [(np.array([[-g]]), np.array([0.0]))], st, lr)
    step2 = p2[0][0][0, 0] - p1[0][0][0, 0]
    assert np.isclose(step2, lr / 19.0 * g / (g + 1e-8), rtol=1e-12)
    p3, st = mlp.adam_step(p2, [(np.array([[g]]), np.array([0.0]))], st, lr)
    step3 = p3[0][0][0, 0] - p2[0][0][0, 0]
    mhat = g * (0.81 - 0.9 + 1.0) * 0.1 / (1 - 0.729)
    assert np.isclose(step3, -lr * mhat / (g + 1e-8), rtol=1e-12)


def test_proposal_and_cdf():
    rng = np.random.default_rng(5)
    logits = rng.normal(size=1000) * 3
    q = mlp.proposal(logits)
    assert np.isclose(q.sum(), 1.0)
    assert q.min() >= mlp.EPS / 1000 * 0.999
    cdf = mlp.integer_cdf(q)
    assert np.all(np.diff(cdf.astype(np.float64)) >= 0)
    assert abs(float(cdf[-1]) / 2 ** 40 - 1.0) < 1e-6


def test_term_sampling_distribution():
    q = np.array([0.5, 0.25, 0.125, 0.125])
    cdf = mlp.integer_cdf(q)
    terms = mlp.sample_terms(cdf, 4000, seed=9, cid=1)
    freq = np.bincount(terms, minlength=4) / 4000
    assert np.all(np.abs(freq - q) < 4 * np.sqrt(q * (1 - q) / 4000))


def test_is_estimator_unbiased():
    rng = np.random.default_rng(11)
    K, nb = 64, 8
    w = rng.normal(size=(K, nb)) * (rng.random(K) < 0.3)[:, None]
    exact = w.sum(axis=0)
    q = mlp.proposal(rng.normal(size=K))
    cdf = mlp.integer_cdf(q)
    ests = np.array([mlp.is_estimate(lambda P: w[P], mlp.sample_terms(cdf, 200, seed=s, cid=0), q)
                     for s in range(60)])
    se = ests.std(axis=0, ddof=1) / np.sqrt(len(ests))
    assert np.all(np.abs(ests.mean(axis=0) - exact) <= 4 * se + 1e-12)


def test_exact_proposal_gives_zero_variance_estimator():
    # q proportional to |w| with a single output: every sample gives the exact sum
    w = np.array([0.0, 2.0, 0.0, 1.0, 1.0])
    q = np.abs(w) / np.abs(w).sum()
    est = mlp.is_estimate(lambda P: np.array([w[P]]), [1, 3, 4, 1], q)
    assert np.isclose(est[0], w.sum())


def test_is_stderr_matches_population_std():
    # the summed standard error is sum_b std_pop(Y[:, b]) / sqrt(N) with
    # Y_j = w_{P_j} / q(P_j): numpy's standard deviation of the same draws
    rng = np.random.default_rng(12)
    K, nb = 64, 8
    w = rng.normal(size=(K, nb)) * (rng.random(K) < 0.5)[:, None]
    q = mlp.proposal(rng.normal(size=K))
    terms = mlp.sample_terms(mlp.integer_cdf(q), 500, seed=4, cid=2)
    Y = np.array([w[P] / q[P] for P in terms])
    ref = np.sum(Y.std(axis=0) / np.sqrt(len(terms)))
    assert np.isclose(mlp.is_stderr_l1(lambda P: w[P], terms, q), ref, rtol=1e-10)


def test_is_stderr_predicts_spread_and_vanishes_for_exact_proposal():
    rng = np.random.default_rng(13)
    K, nb = 64, 4
    w = rng.normal(size=(K, nb))
    q = mlp.proposal(rng.normal(size=K))
    cdf = mlp.integer_cdf(q)
    ests, ses = [], []
    for s in range(80):
        t = mlp.sample_terms(cdf, 300, seed=s, cid=0)
        ests.append(mlp.is_estimate(lambda P: w[P], t, q))
        ses.append(mlp.is_stderr_l1(lambda P: w[P], t, q))
    spread = np.sum(np.std(ests, axis=0, ddof=1))
    assert 0.7 < np.mean(ses) / spread < 1.3
    # zero-variance proposal (q proportional to |w|, one output, one sign)
    w1 = np.array([0.0, 2.0, 0.0, 1.0, 1.0])
    q1 = w1 / w1.sum()
    assert mlp.is_stderr_l1(lambda P: np.array([w1[P]]), [1, 3, 4, 1], q1) < 1e-12


# ---------------------------------------------------------- term model inputs

def _small_cut_parts(seed=3):
    import workloads as W
    from oracle import cutting as C
    ops = W.random_circuit(9, 40, seed)
    cuts = W.random_cuts(9, ops, 3, seed)
    qubits = [0, 2, 3, 5, 7, 8]
    R, parts = C.marginal(9, ops, cuts, qubits, return_parts=True)
    return ops, cuts, qubits, R, parts


def test_term_vectors_sum_to_uncut_marginal():
    from oracle import statevector as SV
    ops, cuts, qubits, R, parts = _small_cut_parts()
    k = len(cuts)
    tot = sum(mlp.term_vector(parts["frags"], parts["reqs"], parts["tensors"], k, P, len(qubits))
              for P in range(4 ** k))
    ref = SV.uncut_marginal(9, ops, qubits)
    assert np.abs(tot - ref).max() <= 1e-12


def test_log_weight_is_norm_of_term_vector():
    ops, cuts, qubits, R, parts = _small_cut_parts()
    k = len(cuts)
    for P in range(4 ** k):
        v = mlp.term_vector(parts["frags"], parts["reqs"], parts["tensors"], k, P, len(qubits))
        y = mlp.log_weight(P, parts["frags"], parts["tensors"], k)
        assert abs(y - np.log(np.linalg.norm(v) + mlp.LABEL_FLOOR)) <= 1e-9, P


def test_cut_shares_closed_form_on_product_tensor():
    from types import SimpleNamespace as NS
    rng = np.random.default_rng(4)
    a = [rng.normal(size=4) for _ in range(3)]
    # one fragment, three axes (cuts 2, 0, 1; outputs on the first two), one row
    cols = np.array([a[0][p & 3] * a[1][(p >> 2) & 3] * a[2][(p >> 4) & 3] for p in range(64)])
    frag = NS(axes=[NS(cut=2, side=0), NS(cut=0, side=0), NS(cut=1, side=1)])
    up, dn = mlp.cut_shares([frag], [cols[None, :]], 3)
    assert np.allclose(up[2], a[0] ** 2 / (a[0] ** 2).sum())
    assert np.allclose(up[0], a[1] ** 2 / (a[1] ** 2).sum())
    assert np.allclose(dn[1], a[2] ** 2 / (a[2] ** 2).sum())
    assert np.allclose(up[1], 0) and np.allclose(dn[0], 0) and np.allclose(dn[2], 0)


def test_cut_shares_sum_to_one_on_real_fragments():
    ops, cuts, qubits, R, parts = _small_cut_parts()
    up, dn = mlp.cut_shares(parts["frags"], parts["tensors"], len(cuts))
    assert np.allclose(up.sum(axis=1), 1.0) and np.allclose(dn.sum(axis=1), 1.0)


def test_feature_layout():
    up = np.array([[1.0, np.exp(-20.0), 0.0, 0.5]])
    dn = np.array([[0.25, 0.25, 0.25, 0.25]])
    x = mlp.features(1, 1, up, dn)
    assert x.shape == (64,)
    assert list(x[:4]) == [0, 1, 0, 0]
    assert np.isclose(x[4], -0.5) and np.isclose(x[5], np.log(0.25) / 40)
    assert np.all(x[6:] == 0)
    x2 = mlp.features(2, 1, up, dn)
    assert x2[4] == -1.0 and x2[2] == 1.0
