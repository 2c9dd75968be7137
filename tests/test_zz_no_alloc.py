"""GPU test of tn_estimate_noalloc (the estimate in the library's fixed device
workspace, for callers that cannot allocate) against tn_estimate on the same
plans: two calls in a row, the second with a smaller input, each to the
parity bar of the level sums (2e-5 T_u plus the level's summed FP32 term
bounds; the FP64 dominant term at 1e-12).  An estimate larger than the fixed
workspace is refused with TN_ENOMEM before any device call."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import network
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


def _tols(c, terms, x_ref):
    pat, _ = terms.get()
    tol = pc.term_tols(network.slot_split(c), pat, x_ref)
    lv = (pat != 0).sum(axis=1)
    return [2e-5 * x_ref[lv == u].sum() + tol[lv == u].sum() for u in range(c.level + 1)]


def test_noalloc_estimate_matches_tn_estimate(torch):
    from oracle import estimate
    cases = []
    c5 = W.config(5)
    p5 = tn.tn_plan_build(c5, 3)
    t5 = tn.tn_terms_enumerate(p5, 3)
    cases.append((c5, p5, t5, np.load(os.path.join(GOLD, "config5_terms.npy"))))
    c1 = W.config(1, level=2)                     # the second, smaller input
    p1 = tn.tn_plan_build(c1, 2)
    t1 = tn.tn_terms_enumerate(p1, 2)
    cases.append((c1, p1, t1, estimate.estimate(c1, 2, "network")["X"]))
    for c, p, t, x_ref in cases:
        print(f"noalloc {c.name}", flush=True)
        got = tn.tn_estimate_noalloc([p], [t])[0]
        torch.cuda.synchronize()
        want = tn.tn_estimate([p], [t])[0]
        tols = _tols(c, t, x_ref)
        assert got["n_terms"] == want["n_terms"] and got["n_contracted"] == want["n_contracted"]
        for u in range(c.level + 1):
            assert abs(got["T"][u] - want["T"][u]) <= tols[u], (c.name, u, got["T"][u], want["T"][u])
            assert abs(got["A"][u] - want["A"][u]) <= 1e-6 * want["A"][u]
        assert abs(got["T"][0] - want["T"][0]) <= 1e-12 * want["T"][0]
        print(f"  bitwise equal level sums: {got['T'] == want['T']}", flush=True)
    tn.tn_release_cached()


def test_noalloc_refuses_an_estimate_above_its_workspace(torch):
    c3 = W.config(3)                              # 36-qubit QAOA: about 0.7 GB of workspace
    p3 = tn.tn_plan_build(c3, 2)
    t3 = tn.tn_terms_enumerate(p3, 2)
    with pytest.raises(tn.TNError) as e:
        tn.tn_estimate_noalloc([p3], [t3])
    assert e.value.code == tn.TN_ENOMEM and "fixed" in str(e.value)
    # and the array still serves a small estimate afterwards
    c1 = W.config(1, level=1)
    p1 = tn.tn_plan_build(c1, 1)
    t1 = tn.tn_terms_enumerate(p1, 1)
    r = tn.tn_estimate_noalloc([p1], [t1])[0]
    assert r["n_terms"] == 13 and r["A"][1] > r["A"][0] > 0
