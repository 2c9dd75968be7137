"""GPU tests of the C ABI's one-call entry points (Section III, Problem 1;
Section IV, Algorithm 1's Require / Ensure): tn_estimate (one schedule, kept
between calls; term ranges below the one-schedule workspace) and
tn_contract_batch (term ranges, stitched), against the FP64 oracle."""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import estimate, network
from paper_2211_17028_amd import tn
from tests import parity_checks as pc

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a HIP device"
    tn.lib()
    return t


def _level_tols(split, pat, x_ref):
    """Per level: 2e-5 T_u plus the level's summed FP32 term bounds."""
    tol = pc.term_tols(split, pat, x_ref)
    lv = (np.asarray(pat) != 0).sum(axis=1)
    return [2e-5 * x_ref[lv == u].sum() + tol[lv == u].sum() for u in range(lv.max() + 1)]


def _check_result(r, gold_a, gold_t, tols):
    for u in range(len(gold_t)):
        assert abs(r["T"][u] - gold_t[u]) <= tols[u], (u, r["T"][u], gold_t[u], tols[u])
        assert abs(r["A"][u] - gold_a[u]) <= 1e-6 * gold_a[u], (u, r["A"][u], gold_a[u])


def test_tn_estimate_against_oracle(torch):
    """tn_estimate on config 1 (8 qubits, level 2) against the oracle's
    estimate, and on config 5 (225 qubits, level 3, 32551 terms) against the
    stored oracle sums; a second call reuses the kept schedule and gives the
    same bits, and so does a call with a fresh workspace."""
    print("tn_estimate config1 / config5", flush=True)
    c1 = W.config(1, level=2)
    p1 = tn.tn_plan_build(c1, 2)
    t1 = tn.tn_terms_enumerate(p1, 2)
    ref = estimate.estimate(c1, 2, "network")
    pat1, _ = t1.get()
    r1 = tn.tn_estimate([p1], [t1])[0]
    _check_result(r1, ref["A"], ref["T"], _level_tols(network.slot_split(c1), pat1, ref["X"]))
    assert abs(r1["T"][0] - ref["T"][0]) <= 1e-12 * ref["T"][0]     # FP64 dominant term
    c5 = W.config(5)
    p5 = tn.tn_plan_build(c5, 3)
    t5 = tn.tn_terms_enumerate(p5, 3)
    pat5, _ = t5.get()
    gold_a = np.loadtxt(os.path.join(GOLD, "config5_oracle.txt"))
    gold_t = np.loadtxt(os.path.join(GOLD, "config5_levels.txt"))
    gold_x = np.load(os.path.join(GOLD, "config5_terms.npy"))
    tols = _level_tols(network.slot_split(c5), pat5, gold_x)
    _, full = tn.tn_plan_workspace([p5], [t5])
    ws = torch.empty(full, dtype=torch.uint8, device="cuda")
    r5 = tn.tn_estimate([p5], [t5], ws=ws)[0]
    assert r5["n_terms"] == 32551
    _check_result(r5, gold_a, gold_t, tols)
    assert abs(r5["T"][0] - gold_t[0]) <= 1e-12 * gold_t[0]
    ws.fill_(0xAB)                               # the caller used the workspace in between
    again = tn.tn_estimate([p5], [t5], ws=ws)[0]
    assert again["A"] == r5["A"] and again["T"] == r5["T"]
    fresh = tn.tn_estimate([p5], [t5])[0]
    assert fresh["A"] == r5["A"]
    tn.tn_release_cached()


def test_tn_contract_batch_ranges_against_oracle_terms(torch):
    """Config 5's 32551 terms contracted as four ranges (one of a single
    term); the stitched amplitudes give X_t = w_t 2^-N |a_t|^2 within the FP32
    term bound of the oracle's stored values; a repeated range (kept
    schedule, constants uploaded again) gives the same bits."""
    print("tn_contract_batch config5", flush=True)
    c5 = W.config(5)
    plan = tn.tn_plan_build(c5, 3)
    terms = tn.tn_terms_enumerate(plan, 3)
    pat, w = terms.get()
    gold_x = np.load(os.path.join(GOLD, "config5_terms.npy"))
    _, full = tn.tn_plan_workspace([plan], [terms])
    ws = torch.empty(full, dtype=torch.uint8, device="cuda")
    bounds = [0, 7, 8, 20000, terms.n]
    amps = []
    for lo, hi in zip(bounds[:-1], bounds[1:]):
        a = tn.tn_contract_batch([plan], [terms], lo, hi - lo, ws=ws)
        torch.cuda.synchronize()
        amps.append(a[0].cpu().numpy())
    amp = np.concatenate(amps)
    assert amp.shape == (terms.n,)
    x = w * 2.0 ** -c5.n_noises * np.abs(amp.astype(np.complex128)) ** 2
    tol = pc.term_tols(network.slot_split(c5), pat, gold_x, fp64_first=False)   # all FP32 here
    bad = np.flatnonzero(np.abs(x - gold_x) > tol)
    assert bad.size == 0, (bad[:5], x[bad[:5]], gold_x[bad[:5]])
    assert np.all(amp[w == 0] == 0)              # zero-weight terms are never contracted
    again = tn.tn_contract_batch([plan], [terms], 8, 19992, ws=ws)
    torch.cuda.synchronize()
    assert np.array_equal(again[0].cpu().numpy().view(np.float32), amps[2].view(np.float32))
    tn.tn_release_cached()


def test_tn_contract_batch_packed_plans(torch):
    """Two packed circuits (configs 1 and 2, 8 and 25 qubits): terms
    [4, 49) of each contracted in one call, against the oracle (config 2's
    depolarizing corrections are degenerate: the range holds whole
    noise-position groups, whose sums are compared)."""
    print("tn_contract_batch packed", flush=True)
    c1 = W.config(1, level=2)
    p1 = tn.tn_plan_build(c1, 2)
    t1 = tn.tn_terms_enumerate(p1, 2)
    c2 = W.config(2)
    p2 = tn.tn_plan_build(c2, 2)
    t2 = tn.tn_terms_enumerate(p2, 2)
    lo, hi = 4, 49
    a = tn.tn_contract_batch([p1, p2], [t1, t2], lo, hi - lo)
    torch.cuda.synchronize()
    pat1, w1 = t1.get()
    ref = estimate.estimate(c1, 2, "network")
    x1 = w1[lo:hi] * 2.0 ** -c1.n_noises * np.abs(a[0].cpu().numpy().astype(np.complex128)) ** 2
    pc.check_terms(x1, ref["X"][lo:hi], pat1[lo:hi], network.slot_split(c1), degenerate=False,
                   fp64_first=False)
    pat2, w2 = t2.get()
    gold_x = np.load(os.path.join(GOLD, "config2_terms.npy"))
    x2 = w2[lo:hi] * 2.0 ** -c2.n_noises * np.abs(a[1].cpu().numpy().astype(np.complex128)) ** 2
    pc.check_terms(x2, gold_x[lo:hi], pat2[lo:hi], network.slot_split(c2), degenerate=True,
                   fp64_first=False)
    tn.tn_release_cached()


@pytest.mark.parametrize("cfg,frac", [(1, 0.0), (5, 0.3)])
def test_ranged_estimate_matches_one_schedule(torch, cfg, frac):
    """A workspace between tn_plan_workspace's minimum and full size runs the
    estimate as consecutive term ranges (config 1 at the minimum: ranges of a
    term or two): level sums within the FP32 term bounds of the one-schedule
    estimate and of the oracle, the dominant term in FP64."""
    print(f"ranged estimate config{cfg} frac {frac}", flush=True)
    c = W.config(cfg) if cfg != 1 else W.config(1, level=2)
    plan = tn.tn_plan_build(c, c.level)
    terms = tn.tn_terms_enumerate(plan, c.level)
    mn, full = tn.tn_plan_workspace([plan], [terms])
    assert 0 < mn < full
    ws = torch.empty(mn + int(frac * (full - mn)), dtype=torch.uint8, device="cuda")
    r = tn.tn_estimate([plan], [terms], ws=ws)[0]
    one = tn.tn_estimate([plan], [terms])[0]
    pat, _ = terms.get()
    if cfg == 1:
        ref = estimate.estimate(c, c.level, "network")
        gold_a, gold_t, gold_x = ref["A"], ref["T"], ref["X"]
    else:
        gold_a = np.loadtxt(os.path.join(GOLD, "config5_oracle.txt"))
        gold_t = np.loadtxt(os.path.join(GOLD, "config5_levels.txt"))
        gold_x = np.load(os.path.join(GOLD, "config5_terms.npy"))
    tols = _level_tols(network.slot_split(c), pat, gold_x)
    _check_result(r, gold_a, gold_t, tols)
    _check_result(one, gold_a, gold_t, tols)
    for u in range(c.level + 1):
        assert abs(r["T"][u] - one["T"][u]) <= 2 * tols[u]
    assert abs(r["T"][0] - gold_t[0]) <= 1e-12 * gold_t[0]
    assert r["n_terms"] == one["n_terms"] and r["n_contracted"] == one["n_contracted"]
    tn.tn_release_cached()
