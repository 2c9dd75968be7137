"""Learned pruning of level-2/3 terms, on top of Algorithm 1.

Flow (all arithmetic in the library: estimates, features, network training
and inference, targets, threshold):
  1. training data: full estimates of training circuits give every term's
     value X_t; the candidates are the live terms of level >= 2, their
     features come from tn_terms_features (with the same run's level-1 values)
     and their targets are log X_t;
  2. the network is trained on the GPU (tn_mlp_* kernels, Adam, mini-batches);
  3. tau is the largest threshold on predicted log X whose pruned training mass
     stays within a budget relative to the training circuits' estimates;
  4. on a new circuit: a level-1 estimate (cheap) gives the level-1 values, the
     network scores every level >= 2 candidate, candidates below tau are
     dropped, and the pruned level-l estimate runs.  The full expansion is the
     reference for the pruning error.
The policy without the network ranks candidates by their rigorous bound
w * prod ||K_hat||^2 (feature 35) with a threshold chosen the same way.
"""
from __future__ import annotations

import time

import numpy as np

from . import tn

BOUND_FEATURE = 35


def full_run(circ, level=None, graph=False):
    level = circ.level if level is None else level
    plan = tn.tn_plan_build(circ, level)
    terms = tn.tn_terms_enumerate(plan, level)
    ex = tn.tn_exec_prepare([plan], [terms], tn.exec_opts(use_graph=graph))
    res = ex.run()[0]
    x, _ = ex.values()
    return plan, terms, res, x


def candidate_mask(terms):
    pat, w = terms.get()
    lv = (pat != 0).sum(axis=1)
    return lv >= 2, w > 0


def training_data(circ):
    """(features, X, estimate) of the live level >= 2 terms of a full run."""
    plan, terms, res, x = full_run(circ)
    n1 = 1 + 3 * circ.n_noises
    feats = tn.tn_terms_features(plan, terms, x[:n1])
    cand, live = candidate_mask(terms)
    sel = cand & live
    return feats[sel], x[sel], res


def train(datasets, width=128, depth=3, epochs=40, batch=4096, lr=2e-3, seed=2211170280, log=None):
    import torch
    feats = np.concatenate([d[0] for d in datasets]).astype(np.float32)
    xs = np.concatenate([d[1] for d in datasets]).astype(np.float64)
    f_dev = torch.from_numpy(feats).cuda()
    t_dev = tn.tn_mlp_log_targets(torch.from_numpy(xs).cuda())
    mlp = tn.MLP(n_in=feats.shape[1], width=width, depth=depth, seed=seed, max_batch=max(batch, 1 << 12))
    mlp.fit_normalizer(f_dev)
    rng = np.random.default_rng(seed)
    n = feats.shape[0]
    hist = []
    for ep in range(epochs):
        order = torch.from_numpy(rng.permutation(n)).cuda()
        tot = 0.0
        for s in range(0, n, batch):
            idx = order[s:s + batch]
            xb = f_dev.index_select(0, idx).contiguous()
            tb = t_dev.index_select(0, idx).contiguous()
            mlp.train_step(xb, tb, lr=lr)
            tot += float(mlp.loss.item()) * idx.shape[0]
        hist.append(tot / n)
        if log:
            log(f"epoch {ep} mse {hist[-1]:.4f}")
    return mlp, hist, (f_dev, xs)


def threshold(scores, xs, budget_abs):
    return tn.tn_prune_threshold(np.asarray(scores, np.float32), np.asarray(xs, np.float64), budget_abs)


def score_candidates(mlp, feats, policy):
    import torch
    if policy == "bound":
        return feats[:, BOUND_FEATURE].astype(np.float32)
    return mlp.forward(torch.from_numpy(np.ascontiguousarray(feats, dtype=np.float32)).cuda()).cpu().numpy()


def pruned_estimate(circ, mlp, tau, policy="mlp", level=None, plan=None):
    """Level-1 pre-pass, scoring, pruned estimate.  Returns dict with the
    result, the kept count, the keep flags of the candidates (enumeration
    order), the pruned run's per-term values and the wall time of the whole
    procedure (from the plan when `plan` is given: the plan is what the full
    estimate needs too)."""
    import torch
    level = circ.level if level is None else level
    t0 = time.perf_counter()
    if plan is None:
        plan = tn.tn_plan_build(circ, level)
    t1 = tn.tn_terms_enumerate(plan, 1)
    ex1 = tn.tn_exec_prepare([plan], [t1], tn.exec_opts(use_graph=False))
    ex1.run()
    x1, _ = ex1.values()
    terms = tn.tn_terms_enumerate(plan, level)
    feats = tn.tn_terms_features(plan, terms, x1)
    cand, _ = candidate_mask(terms)
    scores = score_candidates(mlp, feats[cand], policy)
    keep = (scores >= tau).astype(np.uint8)
    tp = tn.tn_terms_enumerate(plan, level, keep=keep, min_level=2)
    ex = tn.tn_exec_prepare([plan], [tp], tn.exec_opts(use_graph=False))
    res = ex.run()[0]
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    x, _ = ex.values()
    return {"result": res, "kept": int(keep.sum()), "candidates": int(cand.sum()), "keep": keep,
            "x": x, "seconds": seconds}
