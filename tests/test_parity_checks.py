"""CPU tests of the full-size parity checks (tests/parity_checks.py) on the
host replay of the real schedules of configs 2, 3 and 5: the replay passes
them, and plausible mistakes planted in its results fail them (a level's
terms dropped, one term off, level sums not those of the per-term values).
The stored oracle values they compare with are pinned to the oracle here:
sampled terms recomputed now, and the stored sums recomputed from the stored
terms."""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import estimate, network, terms as oterms
from paper_2211_17028_amd import tn
from tests import parity_checks as pc
from tests.schedule_sim import Sim

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden(cfg):
    return (np.loadtxt(os.path.join(GOLD, f"config{cfg}_oracle.txt")),
            np.loadtxt(os.path.join(GOLD, f"config{cfg}_levels.txt")),
            np.load(os.path.join(GOLD, f"config{cfg}_terms.npy")))


def _replay(cfg):
    c = W.config(cfg)
    plan = tn.tn_plan_build(c, c.level)
    t = tn.tn_terms_enumerate(plan, c.level)
    desc, cb = tn.tn_exec_describe_only([plan], [t], tn.exec_opts(use_graph=False))
    pat, w = t.get()
    sim = Sim(desc, cb)
    sim.run([[i for i in range(t.n) if w[i] != 0.0]])
    x, _ = sim.outputs()
    return c, pat, x


def _sums(x, pat, level):
    lv = (pat != 0).sum(axis=1)
    return [math.fsum(float(v) for v in x[lv == u]) for u in range(level + 1)]


@pytest.mark.parametrize("cfg", [2, 3, 5])
def test_stored_oracle_values_are_the_oracles(cfg):
    c = W.config(cfg)
    gold_a, gold_t, gold_x = _golden(cfg)
    tl = oterms.enumerate_terms(c.n_noises, c.level)
    assert gold_x.shape == (len(tl),)
    # the stored sums are the stored terms' Neumaier sums, level by level
    lv = np.array([oterms.term_level(t) for t in tl])
    for u in range(c.level + 1):
        s = estimate.Neumaier()
        for v in gold_x[lv == u]:
            s.add(float(v))
        assert s.value == gold_t[u]
    acc = estimate.Neumaier()
    for u in range(c.level + 1):
        acc.add(gold_t[u])
        assert acc.value == gold_a[u]
    # sampled terms of every level recomputed by the oracle now
    net = network.KetNetwork(c, diagonal=True)
    sp = network.slot_split(c)
    rng = np.random.default_rng(cfg)
    for u in range(c.level + 1):
        for j in rng.choice(np.flatnonzero(lv == u), size=min(3, int((lv == u).sum())), replace=False):
            x, _ = network.term_value(net, sp, tl[j])
            # BLAS threading changes the oracle's rounding: for a small term a
            # multiple of eps64 times its bound, not of the term
            tol = 1e-12 * abs(x) + 2.0 ** -40 * math.sqrt(abs(x) * pc.term_bound(sp, tl[j]))
            assert abs(x - gold_x[j]) <= tol, (j, x, gold_x[j], tol)


@pytest.mark.parametrize("cfg", [2, 3, 5])
def test_replay_passes_and_planted_mistakes_fail(cfg):
    c, pat, x = _replay(cfg)
    gold_a, gold_t, gold_x = _golden(cfg)
    sp = network.slot_split(c)
    deg = cfg == 2
    pc.check_against_golden(_sums(x, pat, c.level), x, pat, gold_t, gold_x, sp, deg)
    lv = (pat != 0).sum(axis=1)
    # the top level's terms dropped (the full-size check of A(l) at 1e-6 alone
    # would not see this on config 5: T_2 + T_3 is below 1e-6 A(3))
    bad = x.copy()
    bad[lv == c.level] = 0.0
    with pytest.raises(AssertionError):
        pc.check_against_golden(_sums(bad, pat, c.level), bad, pat, gold_t, gold_x, sp, deg)
    # one term of level 2 off by 1 % (its position group on config 2)
    j = int(np.flatnonzero(lv == 2)[np.argmax(gold_x[lv == 2])])
    bad = x.copy()
    bad[j] *= 1.01
    with pytest.raises(AssertionError):
        pc.check_against_golden(_sums(bad, pat, c.level), bad, pat, gold_t, gold_x, sp, deg)
    # level sums not the per-term values' (a summation slip of 1e-9 relative)
    t = _sums(x, pat, c.level)
    t[1] *= 1 + 1e-9
    with pytest.raises(AssertionError):
        pc.check_against_golden(t, x, pat, gold_t, gold_x, sp, deg)
    # the all-dominant term in FP32 instead of FP64 (relative error ~1e-7)
    bad = x.copy()
    bad[0] *= 1 + 3e-8
    with pytest.raises(AssertionError):
        pc.check_against_golden(_sums(bad, pat, c.level), bad, pat, gold_t, gold_x, sp, deg)
