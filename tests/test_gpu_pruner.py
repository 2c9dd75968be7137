"""GPU tests of the learned pruning (a policy on top of Algorithm 1):
network kernels against the FP64 reference network, and what the trained
network gains over pruning by the rigorous per-term bound."""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import mlp as omlp
from oracle import network
from paper_2211_17028_amd import pruner, tn
from tests import parity_checks as pc

GOLD = os.path.join(os.path.dirname(__file__), "golden")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def test_mlp_kernels_match_the_fp64_reference(torch):
    print("mlp gradient check", flush=True)
    rng = np.random.default_rng(5)
    n_in, width, depth, n = 36, 128, 3, 777
    net = tn.MLP(n_in=n_in, width=width, depth=depth, seed=11, max_batch=1024)
    x = rng.standard_normal((n, n_in)).astype(np.float32) * 3 + 1
    t = rng.standard_normal(n).astype(np.float32)
    w = rng.uniform(0.5, 2.0, n).astype(np.float32)
    xd, td, wd = (torch.from_numpy(a).cuda() for a in (x, t, w))
    net.fit_normalizer(xd)
    net.gradients(xd, td, wd)
    torch.cuda.synchronize()
    st = net.state.cpu().numpy().astype(np.float64)
    # normalizer = column mean and 1/std
    assert np.allclose(st[:n_in], x.mean(0), rtol=1e-5, atol=1e-5)
    assert np.allclose(st[n_in:2 * n_in], 1 / x.std(0), rtol=1e-4)
    P = net.n_params
    y_ref, _ = omlp.forward(st, x, n_in, width, depth)
    y_gpu = net.forward(xd).cpu().numpy()
    assert np.allclose(y_gpu, y_ref, rtol=1e-4, atol=1e-4)
    g_ref = omlp.gradients(st, x, t, w, n_in, width, depth)
    g_gpu = st[2 * n_in + P:2 * n_in + 2 * P]
    rel = np.linalg.norm(g_gpu - g_ref) / np.linalg.norm(g_ref)
    assert rel <= 1e-4, rel
    loss_ref = omlp.loss(st, x, t, w, n_in, width, depth)
    assert abs(net.loss.item() - loss_ref) <= 1e-4 * loss_ref
    # one Adam step
    params = st[2 * n_in:2 * n_in + P]
    net.adam(1e-3)
    torch.cuda.synchronize()
    p_ref, _, _ = omlp.adam(params, g_gpu, np.zeros(P), np.zeros(P), 1e-3, 1)
    p_gpu = net.state.cpu().numpy().astype(np.float64)[2 * n_in:2 * n_in + P]
    assert np.allclose(p_gpu, p_ref, rtol=1e-5, atol=1e-6)


def test_learned_pruning_beats_the_bound_policy(torch):
    """Train on the term values of configs 2-4 (config 4: 16 of its circuits),
    then prune the level-2/3 candidates of config 5 (15x15 grid, level 3,
    held out).  Thresholds of both policies come from the same training
    budget.  The pruned run drops exactly the rejected candidates (their
    values are 0, every other term matches the oracle's stored value), so the
    pruned estimate is the oracle's full sum minus the dropped values; its
    error stays within the training budget (1e-7 of the estimate), which is
    below the candidates' whole mass; at the network's kept count, ranking by
    the rigorous per-term bound drops more mass, and the bound ranking needs
    more terms to reach the network's error."""
    print("pruner training", flush=True)
    data = [pruner.training_data(W.config(2)), pruner.training_data(W.config(3))]
    for c in W.config(4)[:16]:
        data.append(pruner.training_data(c))
    net, hist, (f_dev, xs) = pruner.train(data, epochs=30)
    assert hist[-1] < 0.5 * hist[0]
    feats = f_dev.cpu().numpy()
    total = sum(d[2]["A"][-1] for d in data)
    budget = 1e-7 * total
    tau_mlp = pruner.threshold(pruner.score_candidates(net, feats, "mlp"), xs, budget)
    tau_bnd = pruner.threshold(pruner.score_candidates(net, feats, "bound"), xs, budget)
    c5 = W.config(5)
    plan, terms, full, x = pruner.full_run(c5)
    a_full = full["A"][-1]
    rm = pruner.pruned_estimate(c5, net, tau_mlp, "mlp")
    rb = pruner.pruned_estimate(c5, net, tau_bnd, "bound")
    err_m = a_full - rm["result"]["A"][-1]
    err_b = a_full - rb["result"]["A"][-1]
    print(f"full {a_full:.12f}; mlp kept {rm['kept']}/{rm['candidates']} err {err_m:.3e}; "
          f"bound kept {rb['kept']}/{rb['candidates']} err {err_b:.3e}", flush=True)
    assert err_m >= -1e-12 and err_b >= -1e-12
    # what the pruned run computed: dropped candidates exactly 0, every other
    # term within its FP32 bound of the oracle's stored value, level sums equal
    # to math.fsum of its own values
    gold_a = np.loadtxt(os.path.join(GOLD, "config5_oracle.txt"))
    gold_x = np.load(os.path.join(GOLD, "config5_terms.npy"))
    cand, live = pruner.candidate_mask(terms)
    ci = np.flatnonzero(cand)
    dropped = ci[rm["keep"] == 0]
    kept = np.setdiff1d(np.flatnonzero(live), dropped)
    xp = rm["x"]
    assert np.all(xp[dropped] == 0.0)
    pat, _ = terms.get()
    tol = pc.term_tols(network.slot_split(c5), pat, gold_x)
    assert np.all(np.abs(xp[kept] - gold_x[kept]) <= tol[kept])
    lv = (pat != 0).sum(axis=1)
    for u in range(c5.level + 1):
        fs = math.fsum(float(v) for v in xp[lv == u])
        assert abs(rm["result"]["T"][u] - fs) <= 1e-12 * fs + 1e-300, (u, rm["result"]["T"][u], fs)
    # full - pruned = the dropped terms' values: the pruned estimate equals the
    # oracle's full sum minus its dropped terms, plus the measured FP32
    # differences of the kept terms, to 1e-12
    d_mass = math.fsum(float(v) for v in gold_x[dropped])
    diff_kept = math.fsum(float(v) for v in (xp[kept] - gold_x[kept]))
    a_pruned = rm["result"]["A"][-1]
    assert abs(a_pruned - (gold_a[-1] - d_mass) - diff_kept) <= 1e-12 * gold_a[-1], \
        (a_pruned, gold_a[-1], d_mass, diff_kept)
    # the pruning error stays within the training budget (1e-7 of the
    # estimate), far below the candidates' whole mass (pruning them all fails)
    c_mass = math.fsum(float(v) for v in gold_x[ci])
    err_gold = gold_a[-1] - a_pruned
    print(f"dropped mass {d_mass:.3e} of the candidates' {c_mass:.3e}; error {err_gold:.3e}", flush=True)
    assert err_gold <= 1e-7 * gold_a[-1] < c_mass
    assert err_gold <= 0.5 * c_mass
    # matched kept count: the bound policy keeps the same number of top-ranked terms
    n1 = 1 + 3 * c5.n_noises
    x1 = x[:n1]
    f5 = tn.tn_terms_features(plan, terms, x1)[cand]
    xc = x[cand]
    s_m = pruner.score_candidates(net, f5, "mlp")
    s_b = pruner.score_candidates(net, f5, "bound")
    k = rm["kept"]
    drop_m = xc[np.argsort(-s_m)[k:]].sum()
    drop_b = xc[np.argsort(-s_b)[k:]].sum()
    # kept count the bound ranking needs for the network's dropped mass
    xb_sorted = xc[np.argsort(-s_b)]
    tail = np.cumsum(xb_sorted[::-1])[::-1]          # tail[j] = mass dropped when keeping j terms
    need = int(np.argmax(np.append(tail, 0.0) <= drop_m))
    print(f"matched count {k}: dropped mass mlp {drop_m:.3e} bound {drop_b:.3e}; "
          f"bound ranking needs {need} terms for the network's error", flush=True)
    assert drop_m < drop_b
    assert need > k


def test_pruner_save_load_round_trip(torch):
    print("pruner save / load", flush=True)
    rng = np.random.default_rng(6)
    net = tn.MLP(n_in=36, width=64, depth=2, seed=3, max_batch=1024)
    x = torch.from_numpy(rng.standard_normal((500, 36)).astype(np.float32)).cuda()
    t = torch.from_numpy(rng.standard_normal(500).astype(np.float32)).cuda()
    net.fit_normalizer(x)
    for _ in range(3):
        net.train_step(x, t, lr=1e-3)
    blob = net.save()
    assert blob[:8] == b"TNPRUNE1" and len(blob) == 32 + 4 * (2 * 36 + net.n_params)
    other = tn.MLP(n_in=36, width=64, depth=2, seed=99, max_batch=1024)
    other.load(blob)
    assert torch.equal(net.forward(x), other.forward(x))
    with pytest.raises(tn.TNError):
        tn.MLP(n_in=36, width=32, depth=2, seed=1, max_batch=1024).load(blob)
