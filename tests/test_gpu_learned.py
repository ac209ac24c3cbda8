"""Learned term proposal on the GPU against the oracle.

* The network: forward and mean-squared-error gradients of the BF16-MFMA
  kernels against the fp64 oracle at the same bf16-rounded weights and
  inputs (forward rel err <= 2e-2, per-tensor gradient cosine >= 0.999 and
  rel err <= 5e-2); the first Adam step; training lowers the loss.
* The term model: features, labels, product-of-shares log-weights and the
  support against the oracle's definitions on the fragment tensors.
* Sampling: the proposal against the oracle's, terms bit-exact for the same
  q, the importance-sampling estimate against the oracle's estimator.
* The gain: on the 10-cut workload a network trained on other circuits
  gives an estimate much closer to the exhaustive one than uniform term
  sampling with the same number of terms.
"""
import numpy as np
import pytest

import paper_2303_10788_amd as cc
import workloads as W
from oracle import cutting as C, mlp as O

pytestmark = pytest.mark.gpu


def _log(m):
    print(m, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return cc.Context()


def _bf16(a):
    import torch
    return torch.tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float32).numpy()


def _random_net(F, H, seed):
    rng = np.random.default_rng([seed, 7])
    params = O.init_params(F, H, seed)
    params = [(W, b + 0.05 * rng.normal(size=b.shape)) for W, b in params]
    return [(_bf16(W).astype(np.float64), _bf16(b).astype(np.float64)) for W, b in params]


def _inputs(B, F, seed):
    rng = np.random.default_rng([seed, 8])
    X = _bf16(rng.normal(size=(B, F))).astype(np.float64)
    y = rng.normal(size=B).astype(np.float32).astype(np.float64)
    return X, y


def _dev(a, dtype):
    import torch
    return torch.tensor(np.asarray(a), dtype=torch.float32).to(dtype).cuda().contiguous()


@pytest.mark.parametrize("F,H,B", [(64, 64, 128), (64, 256, 512), (128, 192, 256)])
def test_mlp_forward_and_gradients_vs_oracle(ctx, F, H, B):
    import torch
    _log(f"mlp forward/gradients F={F} H={H} B={B}")
    params = _random_net(F, H, F + H)
    X, y = _inputs(B, F, H)
    net = cc.Mlp(ctx, F, H)
    net.set_params(cc.mlp_pack(params))
    xd = _dev(X, torch.bfloat16)
    yd = _dev(y, torch.float32)
    got = net.forward(xd).cpu().numpy().astype(np.float64)
    ref, _ = O.forward(params, X)
    fwd = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    g, loss = net.gradients(xd, yd)
    Lref, gref = O.loss_and_grads(params, X, y)
    flat_ref = cc.mlp_pack(gref).astype(np.float64)
    assert g.size == flat_ref.size
    got_t = cc.mlp_unpack(g.astype(np.float64), F, H)
    stats = []
    for li, ((gw, gb), (rw, rb)) in enumerate(zip(got_t, gref)):
        for name, a, r in (("W", gw, rw), ("b", gb, rb)):
            a, r = np.ravel(a), np.ravel(r)
            nr = np.linalg.norm(r)
            cos = float(a @ r) / max(np.linalg.norm(a) * nr, 1e-300)
            stats.append((f"{name}{li + 1}", cos, np.linalg.norm(a - r) / max(nr, 1e-300)))
    _log(f"forward rel err {fwd:.3e}, loss {loss:.6f} vs {Lref:.6f}; "
         + ", ".join(f"{n}: cos {c:.5f} rel {e:.3e}" for n, c, e in stats))
    assert fwd <= 2e-2
    assert abs(loss - Lref) <= 2e-2 * abs(Lref)
    # The stored activations are bf16: at the production width (F 64, H 256)
    # the gradients stay within cosine 0.999 / rel 5e-2 of the fp64 oracle;
    # narrower nets over fewer rows amplify the activation rounding more (a
    # CPU emulation of the same rounding points gives W1 rel 6.7e-2 at
    # H 64, B 128), so they are held to cosine 0.995 / rel 1e-1.
    cmin, rmax = (0.999, 5e-2) if (F, H) == (64, 256) else (0.995, 1e-1)
    for n, cos, rel in stats:
        assert cos >= cmin and rel <= rmax, (n, cos, rel)


def test_mlp_first_adam_step(ctx):
    import torch
    F, H, B = 64, 128, 256
    params = _random_net(F, H, 3)
    X, y = _inputs(B, F, 4)
    net = cc.Mlp(ctx, F, H)
    flat0 = cc.mlp_pack(params)
    net.set_params(flat0)
    lr = 1e-3
    net.train(_dev(X, torch.bfloat16), _dev(y, torch.float32), batch=B, steps=1, lr=lr)
    delta = net.get_params().astype(np.float64) - flat0
    _, gref = O.loss_and_grads(params, X, y)
    g = cc.mlp_pack(gref).astype(np.float64)
    big = np.abs(g) > 1e-2 * np.abs(g).max()
    # the first Adam step moves every coordinate by lr * g / (|g| + eps)
    assert np.all(np.sign(delta[big]) == -np.sign(g[big]))
    assert np.allclose(np.abs(delta[big]), lr, rtol=2e-2)


def test_mlp_adam_steps_two_and_three(ctx):
    """Adam at t = 1, 2, 3 on the GPU against the oracle's Adam applied to
    the same gradients (the network's own, read back before each step):
    the moment updates and the bias corrections of later steps."""
    import torch
    F, H, B = 64, 128, 256
    params = _random_net(F, H, 13)
    X, y = _inputs(B, F, 14)
    net = cc.Mlp(ctx, F, H)
    net.set_params(cc.mlp_pack(params))
    Xd, yd = _dev(X, torch.bfloat16), _dev(y, torch.float32)
    lr = 1e-3
    state = O.adam_state(cc.mlp_unpack(cc.mlp_pack(params).astype(np.float64), F, H))
    for t in range(1, 4):
        before = net.get_params().astype(np.float64)
        g, _ = net.gradients(Xd, yd)
        net.train(Xd, yd, batch=B, steps=1, lr=lr)
        got = net.get_params().astype(np.float64)
        exp_struct, state = O.adam_step(cc.mlp_unpack(before, F, H), cc.mlp_unpack(g.astype(np.float64), F, H),
                                        state, lr)
        exp = np.concatenate([np.ravel(a) for W_, b_ in exp_struct for a in (W_, b_)])
        err = np.abs(got - exp)
        assert np.all(err <= 1e-3 * lr + 2e-7 * np.abs(exp)), (t, float(err.max()))


def test_mlp_training_reduces_loss(ctx):
    import torch
    F, H, n = 64, 256, 4096
    rng = np.random.default_rng(12)
    X = _bf16(rng.normal(size=(n, F)))
    y = (np.sin(X[:, 0]) + 0.5 * X[:, 1] ** 2 - X[:, 2] * X[:, 3]).astype(np.float32)
    net = cc.Mlp(ctx, F, H)
    losses = net.train(_dev(X, torch.bfloat16), _dev(y, torch.float32), batch=512, steps=300, lr=2e-3, seed=5)
    _log(f"training loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert np.all(np.isfinite(losses))
    assert losses[-20:].mean() < 0.2 * losses[:5].mean()


# ------------------------------------------------------------ term model

def _small(case):
    """10-qubit, 3-cut circuits: a 5-qubit non-Clifford block feeding an
    8-qubit Clifford fragment (mirrored: the Clifford fragment upstream), or
    an unstructured random circuit."""
    kind, seed = case
    n = 10
    if kind == "random":
        ops = W.random_circuit(n, 45, seed)
        cuts = W.random_cuts(n, ops, 3, seed)
    else:
        ops, cuts = W.block_circuit(n, 12, [W.Block([0, 1, 2, 3, 4], [2, 3, 4])], t_c=5, p_cx=0.3, seed=seed,
                                    n_t=3, mirrored=(kind == "mirrored"))
    qubits = [0, 1, 5, 6, 7, 8, 9]
    return ops, cuts, qubits


CASES = [("block", 1), ("mirrored", 2), ("random", 7)]


@pytest.mark.parametrize("case", CASES)
def test_term_model_vs_oracle(ctx, case):
    import torch
    ops, cuts, qubits = _small(case)
    k = len(cuts)
    seed = case[1]
    _log(f"term model {case} k={k}")
    R, parts = C.marginal(10, ops, cuts, qubits, return_parts=True)
    frags, tensors = parts["frags"], parts["tensors"]
    up, dn = O.cut_shares(frags, tensors, k)
    plan = cc.Plan(ctx, 10, ops, cuts)
    L = cc.Learned(plan, qubits)
    assert (L.k, L.K, L.width) == (k, 4 ** k, 64)
    K = 4 ** k
    feats = L.features().float().cpu().numpy()
    ref = np.stack([O.features(P, k, up, dn) for P in range(K)])
    assert np.abs(feats - ref).max() <= 4e-3
    assert np.array_equal(feats[:, :6 * k].reshape(K, k, 6)[:, :, :4], ref[:, :6 * k].reshape(K, k, 6)[:, :, :4])
    terms = torch.tensor(np.random.default_rng(seed).permutation(K)[:37], dtype=torch.int64).cuda()
    f2 = L.features(terms).float().cpu().numpy()
    assert np.array_equal(f2, feats[terms.cpu().numpy()])
    y = L.log_weights().cpu().numpy().astype(np.float64)
    yref = np.array([O.log_weight(P, frags, tensors, k) for P in range(K)])
    # weights that are zero in exact arithmetic come out as exact zeros or
    # as rounding residue (~1e-18) depending on the summation: compare the
    # labels above 1e-12 and require both sides below it elsewhere
    live = yref > np.log(1e-12)
    assert np.abs(y - yref)[live].max() <= 1e-4
    assert np.all(y[~live] <= np.log(1e-12) + 1e-3)
    y2 = L.log_weights(kind=2).cpu().numpy().astype(np.float64)
    assert np.abs(y2 - yref / O.LABEL_SCALE)[live].max() <= 1e-5
    ys = L.log_weights(kind=1).cpu().numpy().astype(np.float64)
    ysref = np.array([40.0 * sum(O.phi(up[c][(P >> 2 * c) & 3]) + O.phi(dn[c][(P >> 2 * c) & 3])
                                 for c in range(k)) for P in range(K)])
    assert np.abs(ys - ysref).max() <= 1e-3
    sup, cnt = L.support(cap=K)
    sup = set(sup.cpu().numpy().tolist())
    assert cnt == len(sup)
    big = {P for P in range(K) if yref[P] > np.log(1e-12)}
    assert big <= sup
    assert all(yref[P] <= np.log(1e-12) for P in sup - big)
    ex = L.exhaustive()
    assert np.abs(ex - R).max() <= 1e-10


@pytest.mark.parametrize("case", CASES)
def test_fused_logits_equal_layered_forward(ctx, case):
    """The one-launch forward pass over every term (features built in the
    kernel, activations on chip) equals the layer-by-layer forward of the
    same network on the same feature rows bit for bit, times the label
    scale, and the fp64 oracle network within the bf16 forward bound."""
    import torch
    ops, cuts, qubits = _small(case)
    k = len(cuts)
    _log(f"fused logits {case} k={k}")
    plan = cc.Plan(ctx, 10, ops, cuts)
    L = cc.Learned(plan, qubits)
    net = cc.Mlp(ctx, 64, 256)
    params = _random_net(64, 256, 11 + case[1])
    net.set_params(cc.mlp_pack(params))
    fused = L.logits(net).cpu().numpy()
    X = L.features()
    layered = net.forward(X).cpu().numpy() * np.float32(O.LABEL_SCALE)
    assert np.array_equal(fused, layered.astype(np.float32))
    ref, _ = O.forward(params, X.float().cpu().numpy().astype(np.float64))
    rel = np.abs(fused / O.LABEL_SCALE - ref).max() / max(np.abs(ref).max(), 1e-30)
    assert rel <= 2e-2


def test_proposal_vs_oracle(ctx):
    import torch
    rng = np.random.default_rng(21)
    logits = (rng.normal(size=4 ** 6) * 4).astype(np.float32)
    q = cc.proposal(ctx, torch.tensor(logits).cuda()).cpu().numpy()
    qref = O.proposal(logits.astype(np.float64))
    assert np.allclose(q, qref, rtol=1e-12, atol=0)
    qu = cc.proposal(ctx, None, K=4 ** 6).cpu().numpy()
    assert np.all(qu == 1.0 / 4 ** 6)


@pytest.mark.parametrize("K,n", [(4, 1000), (4 ** 6, 5000), (4 ** 10, 3000)])
def test_sample_terms_bit_exact(ctx, K, n):
    import torch
    rng = np.random.default_rng(K)
    q = O.proposal(rng.normal(size=K) * 3)
    got = cc.sample_terms(ctx, torch.tensor(q).cuda(), n, seed=0x1234_5678_9ABC, cid=(3 << 40) | 17).cpu().numpy()
    ref = O.sample_terms(O.integer_cdf(q), n, seed=0x1234_5678_9ABC, cid=(3 << 40) | 17)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("case", CASES)
def test_is_estimate_vs_oracle(ctx, case):
    import torch
    ops, cuts, qubits = _small(case)
    seed = case[1]
    k = len(cuts)
    R, parts = C.marginal(10, ops, cuts, qubits, return_parts=True)
    rng = np.random.default_rng(seed + 100)
    q = O.proposal(rng.normal(size=4 ** k))
    n, s = 3000, 77
    plan = cc.Plan(ctx, 10, ops, cuts)
    L = cc.Learned(plan, qubits, circuit=5)
    terms = torch.empty(n, dtype=torch.int64, device="cuda")
    est = L.estimate(torch.tensor(q).cuda(), n, s, terms_out=terms)
    tref = O.sample_terms(O.integer_cdf(q), n, seed=s, cid=5)
    assert np.array_equal(terms.cpu().numpy(), tref)
    ref = O.is_estimate(lambda P: O.term_vector(parts["frags"], parts["reqs"], parts["tensors"], k, P, len(qubits)),
                        tref, q)
    assert np.abs(est - ref).max() <= 1e-10
    assert abs(est.sum() - 1.0) < 0.5  # an unbiased estimate of a distribution


@pytest.mark.parametrize("case", CASES[:2])
def test_learned_marginal_vs_oracle(ctx, case):
    """One call through the whole learned path: network logits, q, the
    draw and the contraction.  The oracle takes the same q (from the
    kernel's logits; the network itself is checked against the oracle
    elsewhere), draws the same terms and forms the estimate and its
    standard error in fp64."""
    import torch
    ops, cuts, qubits = _small(case)
    k = len(cuts)
    _log(f"learned marginal {case} k={k}")
    R, parts = C.marginal(10, ops, cuts, qubits, return_parts=True)
    plan = cc.Plan(ctx, 10, ops, cuts)
    net = cc.Mlp(ctx, 64, 256)
    # a damped head keeps the logits' spread a few units (an untrained
    # network at full scale puts nearly all mass on one term, and a draw can
    # then miss the whole support)
    params = _random_net(64, 256, 5 + case[1])
    params[-1] = (params[-1][0] * 0.02, params[-1][1] * 0.0)
    net.set_params(cc.mlp_pack(params))
    n, s = 2000, 31
    est, se = plan.learned_marginal(net, qubits, n, seed=s, circuit=9)
    L = cc.Learned(plan, qubits, seed=s, circuit=9)
    logits = L.logits(net).cpu().numpy().astype(np.float64)
    q = O.proposal(logits)
    tref = O.sample_terms(O.integer_cdf(q), n, seed=s, cid=9)
    tw = lambda P: O.term_vector(parts["frags"], parts["reqs"], parts["tensors"], k, P, len(qubits))
    ref = O.is_estimate(tw, tref, q)
    ref_se = O.is_stderr_l1(tw, tref, q)
    assert np.abs(est - ref).max() <= 1e-10
    assert abs(se - ref_se) <= 1e-9 * max(ref_se, 1.0)
    # device output: the same values
    out = torch.empty(1 << len(qubits), dtype=torch.float64, device="cuda")
    _, se2 = plan.learned_marginal(net, qubits, n, seed=s, circuit=9, out=out)
    assert np.array_equal(out.cpu().numpy(), est) and se2 == se
    # the estimate is within a few standard errors of the exact marginal
    assert se > 0 and np.abs(est - R).sum() <= 6 * se


def test_train_step_equals_one_train_step(ctx):
    import torch
    F, H, n = 64, 128, 256
    rng = np.random.default_rng(8)
    x = torch.tensor(rng.integers(0, 2, size=(n, F)).astype(np.float32)).cuda()
    t = torch.tensor(rng.normal(size=n).astype(np.float32)).cuda()
    p0 = cc.mlp_pack(_random_net(F, H, 4))
    a, b = cc.Mlp(ctx, F, H), cc.Mlp(ctx, F, H)
    a.set_params(p0)
    b.set_params(p0)
    for step in range(3):
        la = a.train_step(x, t, lr=1e-3)
        lb = b.train(x.to(torch.bfloat16), t, batch=n, steps=1, lr=1e-3)[0]
        assert la == lb, step
        assert np.array_equal(a.get_params(), b.get_params()), step
    with pytest.raises(cc.CcutError):
        a.train_step(x[:100], t[:100])


# ------------------------------------------------------------ the gain

def _dataset(ctx, seeds, n_support=1024, n_shares=2048, n_uniform=1024):
    """Feature rows and scaled labels of each training circuit's support
    terms, of terms drawn from its product-of-shares proposal and of
    uniformly drawn terms."""
    import torch
    xs, ys = [], []
    for s in seeds:
        w = W.learned_circuit(s)
        plan = cc.Plan(ctx, w.n, w.ops, w.cuts)
        L = cc.Learned(plan, w.qubits)
        sup, cnt = L.support(cap=n_support)
        q_sh = cc.proposal(ctx, L.log_weights(kind=1))
        drawn = cc.sample_terms(ctx, q_sh, n_shares, seed=s, cid=1)
        uni = cc.sample_terms(ctx, cc.proposal(ctx, None, K=L.K), n_uniform, seed=s, cid=2)
        terms = torch.cat([sup, drawn, uni]).contiguous()
        xs.append(L.features(terms))
        ys.append(L.log_weights(terms, kind=2))
    return torch.cat(xs).contiguous(), torch.cat(ys).contiguous()


def _tvd(a, b):
    return 0.5 * float(np.abs(a - b).sum())


def test_learned_proposal_beats_uniform_on_ten_cuts(ctx):
    _log("learned proposal: building training set")
    X, y = _dataset(ctx, [100000 + i for i in range(16)])
    rows = (X.shape[0] // 64) * 64
    X, y = X[:rows].contiguous(), y[:rows].contiguous()
    net = cc.Mlp(ctx, 64, 256)
    losses = net.train(X, y, batch=1024, steps=2000, lr=1e-3, seed=1)
    _log(f"training rows {rows}, loss {losses[:5].mean():.4f} -> {losses[-50:].mean():.5f}")
    assert losses[-50:].mean() < 0.2 * losses[:5].mean()
    w = W.learned_circuit(200000)
    plan = cc.Plan(ctx, w.n, w.ops, w.cuts)
    L = cc.Learned(plan, w.qubits)
    exact = L.exhaustive()
    assert abs(exact.sum() - 1.0) < 1e-9
    n = 16384
    props = {"learned": cc.proposal(ctx, L.logits(net)),
             "uniform": cc.proposal(ctx, None, K=L.K),
             "shares": cc.proposal(ctx, L.log_weights(kind=1)),
             "exact_norm": cc.proposal(ctx, L.log_weights(kind=0))}
    tv = {name: _tvd(L.estimate(q, n, 9), exact) for name, q in props.items()}
    _log(f"TVD vs exhaustive at N={n}: {tv}")
    assert tv["learned"] < 0.2 * tv["uniform"]


def test_network_free_proposals_on_held_out_circuits(ctx):
    """The comparison the learned proposal is measured against, on the
    held-out circuit and on one that measures its exit wires one Clifford
    layer after the cuts: the Clifford fragment's exact Pauli tensor leaves
    only a handful of the 4^10 terms nonzero (Sec. IX), the sparse
    exhaustive contraction equals the dense one, and the network-free
    proposal from the product of the fragments' column norms (the network's
    own training labels, exact) reaches TVD <= 1e-2 at 16384 samples."""
    for w in (W.learned_circuit(200000), W.learned_circuit(200001, tail=1, near_exits=True)):
        _log(f"network-free proposals on {w.name}")
        plan = cc.Plan(ctx, w.n, w.ops, w.cuts)
        L = cc.Learned(plan, w.qubits)
        exact = L.exhaustive()
        _, n_support = L.support(cap=0)
        assert 1 <= n_support <= 64
        sparse = plan.marginal(w.qubits, flags=cc.CCUT_FLAG_SPARSE)
        assert np.max(np.abs(sparse - exact)) <= 1e-12
        q = cc.proposal(ctx, L.log_weights(kind=0))
        assert _tvd(L.estimate(q, 16384, 9), exact) <= 1e-2
        L.close()
        plan.close()
