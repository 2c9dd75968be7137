"""CPU tests of the HIP library's host side: exported symbols, plan building,
noise split, term enumeration, error codes, and a host replay of the device
schedule against the oracle (no GPU needed)."""
import ctypes
import itertools
import math
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import channels, dense, doubled, estimate, network, offdiag, terms as oterms
from paper_2211_17028_amd import tn
from tests.schedule_sim import Sim

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "tn.h")).read()
    declared = set(re.findall(r"^\s*(?:int|void|const char\*)\s+(tn_[a-z0-9_]+)\s*\(", hdr, re.M))
    assert "tn_plan_build" in declared and "tn_estimate" in declared
    L = tn.lib()
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert declared <= set(tn.EXPORTS) | declared


def test_noise_split_matches_lapack_eigendecomposition():
    rng = np.random.default_rng(3)
    cases = [W.kraus_depolarizing(1e-3), W.kraus_ad_pd(2e-3, 5e-3), W.kraus_ad_pd(0.3, 0.2)]
    cases += [W.random_isometry_kraus(rng, k) for k in (1, 2, 3, 4, 4)]
    for kr in cases:
        c = W.Circuit(1, [W.Op("noise", (0,), kraus=kr)], W.circuits.zero_product(1), "product",
                      W.circuits.zero_product(1), 1)
        try:
            plan = tn.tn_plan_build(c, 1)
        except tn.TNError as e:
            assert e.code == tn.TN_EDEGENERATE
            continue
        d, K, rate = plan.noise(0)
        m = channels.superoperator(kr)
        mt = channels.permute(m)
        ev = np.sort(np.linalg.eigvalsh(mt))[::-1]
        assert np.allclose(d, np.abs(ev), atol=1e-14)
        # reconstruction M = sum d_i K_i (x) conj(K_i)
        rec = sum(d[i] * np.kron(K[i], K[i].conj()) for i in range(4))
        assert np.allclose(rec, m, atol=1e-13)
        assert math.isclose(rate, channels.noise_rate(m), rel_tol=1e-9, abs_tol=1e-15)


@pytest.mark.parametrize("n,l", [(4, 1), (4, 2), (4, 4), (6, 3), (10, 2)])
def test_enumeration_order_and_weights_match_the_oracle(n, l):
    rng = np.random.default_rng(n * 10 + l)
    c = W.tiny_random_circuit(rng, 3, 6 + n, n, noise="adpd", level=l)
    plan = tn.tn_plan_build(c, l)
    t = tn.tn_terms_enumerate(plan, l)
    pat, w = t.get()
    want = oterms.enumerate_terms(n, l)
    assert t.n == len(want) == oterms.count_terms(n, l)
    assert [tuple(int(x) for x in row) for row in pat] == want
    sp = network.slot_split(c)
    for row, wt in zip(pat, w):
        ref = np.prod([sp[s][0][row[s]] for s in range(n)])
        zero = any(sp[s][0][row[s]] <= 4 * np.finfo(float).eps * sp[s][0][0] for s in range(n))
        assert (wt == 0.0) if zero else math.isclose(wt, ref, rel_tol=1e-12)


def _circuit_with(op):
    z = W.circuits.zero_product(2)
    return W.Circuit(2, [op], z, "product", z, 1)


def test_error_codes_are_forced_from_the_host():
    bad_tp = _circuit_with(W.Op("noise", (0,), kraus=[1.01 * np.eye(2, dtype=complex)]))
    with pytest.raises(tn.TNError) as e:
        tn.tn_plan_build(bad_tp, 1)
    assert e.value.code == tn.TN_ENOTCPTP
    nonunitary = _circuit_with(W.Op("gate", (0,), mat=np.array([[1, 1], [0, 1]], dtype=complex)))
    with pytest.raises(tn.TNError) as e:
        tn.tn_plan_build(nonunitary, 1)
    assert e.value.code == tn.TN_EINVAL
    two_qubit_noise = _circuit_with(W.Op("noise", (0, 1), kraus=[np.eye(4, dtype=complex)]))
    with pytest.raises(tn.TNError) as e:
        tn.tn_plan_build(two_qubit_noise, 1)
    assert e.value.code == tn.TN_EUNSUPPORTED
    # identity channel: all four singular values degenerate except d0 -> fine;
    # a channel with two equal largest singular values -> degenerate
    half = [np.sqrt(0.5) * np.eye(2, dtype=complex), np.sqrt(0.5) * W.gate_z()]
    with pytest.raises(tn.TNError) as e:
        tn.tn_plan_build(_circuit_with(W.Op("noise", (0,), kraus=half)), 1)
    assert e.value.code == tn.TN_EDEGENERATE
    bad_q = _circuit_with(W.Op("gate", (5,), mat=np.eye(2, dtype=complex)))
    with pytest.raises(tn.TNError) as e:
        tn.tn_plan_build(bad_q, 1)
    assert e.value.code == tn.TN_EINVAL
    assert "out of range" in tn.lib().tn_last_error().decode()


def test_workspace_sizes_and_boundary_errors_without_a_device():
    """tn_plan_workspace's minimum (terms in ranges of one) lies below the
    one-schedule size; tn_estimate refuses a workspace below the minimum with
    TN_ENOMEM and tn_contract_batch one below its range's schedule, both before
    any device call (the pointers here are not device memory: none is
    touched); malformed arguments give TN_EINVAL."""
    c = W.config(1, level=2)
    plan = tn.tn_plan_build(c, 2)
    terms = tn.tn_terms_enumerate(plan, 2)
    mn, full = tn.tn_plan_workspace([plan], [terms])
    assert 0 < mn < full
    L = tn.lib()
    P, T = tn._handles([plan]), tn._handles([terms])
    fake = ctypes.c_void_p(4096)
    res = (tn.tn_result * 1)()

    assert L.tn_estimate(1, P, T, fake, mn - 1, None, res) == tn.TN_ENOMEM
    assert "minimum" in L.tn_last_error().decode()
    assert L.tn_estimate(1, P, T, None, full, None, res) == tn.TN_EINVAL
    assert L.tn_estimate(1, P, T, fake, 0, None, res) == tn.TN_EINVAL
    assert L.tn_estimate(1, P, T, fake, full, None, None) == tn.TN_EINVAL
    amp = ctypes.c_void_p(8192)
    assert L.tn_contract_batch(1, P, T, 0, 10, amp, fake, 1024, None) == tn.TN_ENOMEM
    assert L.tn_contract_batch(1, P, T, 0, 10, None, fake, full, None) == tn.TN_EINVAL
    assert L.tn_contract_batch(1, P, T, 0, 10, amp, fake, 0, None) == tn.TN_EINVAL
    assert L.tn_contract_batch(1, P, T, 0, 10, amp, None, full, None) == tn.TN_EINVAL
    assert L.tn_contract_batch(1, P, T, 60, 10, amp, fake, full, None) == tn.TN_EINVAL
    assert L.tn_contract_batch(1, P, T, -1, 10, amp, fake, full, None) == tn.TN_EINVAL
    assert L.tn_contract_batch(1, P, T, 5, 0, amp, fake, full, None) == tn.TN_OK
    assert L.tn_plan_workspace(1, P, T, None, None) == tn.TN_EINVAL
    # full_bytes is the size of the one schedule tn_exec_prepare builds
    desc, _ = tn.tn_exec_describe_only([plan], [terms])
    assert desc["const_bytes"] + desc["work_bytes"] == full


def test_level_above_noise_count_is_clamped():
    c = W.tiny_random_circuit(np.random.default_rng(5), 3, 8, 2, noise="adpd", level=5)
    plan = tn.tn_plan_build(c, 5)
    info = plan.info()
    assert info["level"] == 2 and info["clamped"] == 1
    t = tn.tn_terms_enumerate(plan, 5)
    assert t.n == 16


def test_plan_legs_are_closed_and_paths_are_trees():
    for cfg in (1, 2, 5):
        c = W.config(cfg)
        plan = tn.tn_plan_build(c)
        d = plan.describe()
        cnt = {}
        for lf in d["leaves"]:
            for e in lf["legs"]:
                cnt[e] = cnt.get(e, 0) + 1
        # every leg is held by at least two tensors (more for the wire index
        # of diagonal gates, which stays shared)
        assert min(cnt.values()) >= 2
        for cl in d["clusters"]:
            L = len(cl["leaves"])
            used = set()
            for j, (a, b) in enumerate(cl["path"]):
                assert a not in used and b not in used and a < L + j and b < L + j
                used |= {a, b}
            assert len(used) == 2 * L - 2
        slots = sorted(s for cl in d["clusters"] for s in cl["slots"])
        assert slots == list(range(c.n_noises))


def grouped_by_positions(pat, x):
    """Sum of X over the corrections of each position set.  Inside a
    degenerate correction block (depolarizing) single terms depend on the
    chosen singular basis; these sums do not."""
    out = {}
    for row, v in zip(pat, x):
        key = tuple(i for i, c in enumerate(row) if c)
        out[key] = out.get(key, 0.0) + v
    return out


def _replay(circ, level, mode=tn.TN_MODE_BATCHED, fp64=True, gather=True, group=True, max_ksplit=0,
            one_shape=True, all_tiles=False):
    plan = tn.tn_plan_build(circ, level)
    t = tn.tn_terms_enumerate(plan, level)
    desc, cb = tn.tn_exec_describe_only([plan], [t], tn.exec_opts(mode=mode, use_graph=False,
                                                                  fp64_level0=fp64, gather=gather,
                                                                  group=group, max_ksplit=max_ksplit,
                                                                  one_shape_per_level=one_shape,
                                                                  all_tiles=all_tiles))
    pat, w = t.get()
    live = [i for i in range(t.n) if w[i] != 0.0]
    sim = Sim(desc, cb)
    sim.run([live])
    x, amp = sim.outputs()
    return x, pat, desc


@pytest.mark.parametrize("seed,kind,target", [(1, "random", "circuit_output"), (2, "adpd", "product"),
                                               (3, "depol", "dense"), (4, "random", "circuit_output")])
def test_schedule_replay_matches_oracle_terms(seed, kind, target):
    c = W.tiny_random_circuit(np.random.default_rng(seed), 4, 18, 4, noise=kind, level=4, target=target)
    x, pat, _ = _replay(c, 4)
    r = estimate.estimate(c, 4, "network")
    assert [tuple(p) for p in pat] == r["terms"]
    if kind == "depol":
        g1, g2 = grouped_by_positions(pat, x), grouped_by_positions(pat, r["X"])
        assert g1.keys() == g2.keys()
        for k in g1:
            assert abs(g1[k] - g2[k]) <= 2e-5 * abs(g2[k]) + 1e-9
    else:
        assert np.allclose(x, r["X"], rtol=2e-5, atol=1e-9)


def test_schedule_replay_plain_mode_matches_batched():
    c = W.tiny_random_circuit(np.random.default_rng(7), 4, 16, 3, noise="adpd", level=2)
    xb, _, _ = _replay(c, 2)
    xp, _, _ = _replay(c, 2, mode=tn.TN_MODE_PLAIN, fp64=False)
    assert np.allclose(xb, xp, rtol=2e-5, atol=1e-9)


@pytest.mark.parametrize("n,gates,noises,target,seed,merge,split", [(16, 160, 4, "circuit_output", 1, 2, 16),
                                                                     (16, 160, 4, "circuit_output", 4, 1, 2)])
def test_schedule_replay_gathered_operands(n, gates, noises, target, seed, merge, split):
    """Circuits wide enough for matrix-core steps.  Batched mode groups each
    tree level (small steps in one launch, matrix-core steps in one launch per
    tile shape, operands read in stored order); without grouping the MFMA
    steps that need a transpose read their operands in stored order instead;
    PLAIN runs step by step.  Every schedule's replay matches the oracle."""
    c = W.tiny_random_circuit(np.random.default_rng(seed), n, gates, noises, noise="adpd", level=2,
                              target=target)
    r = estimate.estimate(c, 2, "network", reduce=True)
    x_s, _, desc_s = _replay(c, 2)            # levels under 32 MFLOP: all steps in one small-step launch
    x, pat, desc = _replay(c, 2, all_tiles=True)

    def tile_levels(d):
        return {L["level"] for L in d["launches"] if L["kind"] == 6 and not L["fp64"] and L["phase"] == "batch"}
    assert tile_levels(desc_s) <= tile_levels(desc), (tile_levels(desc_s), tile_levels(desc))
    assert any(L["kind"] == 6 and not L["fp64"] for L in desc["launches"]), "no grouped matrix-core launch"
    assert any(L["kind"] == 6 and L["fp64"] for L in desc["launches"]), "no grouped FP64 tile launch"
    merges = {j["merge"] for L in desc["launches"] if L["kind"] == 6 for j in L["jobs"]}
    assert merge in merges, merges          # the two circuits cover both merge modes
    splits = {j["ksplit"] for L in desc["launches"] if L["kind"] == 6 for j in L["jobs"]}
    assert max(splits) == split, splits      # inner sums split over 16 (2^9 terms) or 2 (2^6) tiles
    kinds = [L["kind"] for L in desc["launches"]]
    assert 7 in kinds and all(kinds[q - 1] == 6 for q, kd in enumerate(kinds) if kd == 7)
    x_2, _, desc_2 = _replay(c, 2, max_ksplit=2, all_tiles=True)
    assert {j["ksplit"] for L in desc_2["launches"] if L["kind"] == 6 for j in L["jobs"]} == {1, 2}
    x_1, _, desc_1 = _replay(c, 2, max_ksplit=1, all_tiles=True)
    assert {j["ksplit"] for L in desc_1["launches"] if L["kind"] == 6 for j in L["jobs"]} == {1}
    x_m, _, desc_m = _replay(c, 2, one_shape=False, all_tiles=True)   # every job its own tile shape

    def shapes_per_level(d):
        lv = {}
        for L in d["launches"]:
            if L["kind"] == 6 and not L["fp64"]:
                lv.setdefault(L["level"], set()).add((L["bm"], L["bn"]))
        return lv
    assert sum(map(len, shapes_per_level(desc).values())) <= sum(map(len, shapes_per_level(desc_m).values()))
    x_g, _, desc_g = _replay(c, 2, group=False)
    assert any(L["kind"] == 1 and L.get("gather") for L in desc_g["launches"]), "no gathered step"
    x_t, _, desc_t = _replay(c, 2, gather=False, group=False)
    assert not any(L.get("gather") for L in desc_t["launches"] if L["kind"] == 1)
    x_p, _, desc_p = _replay(c, 2, mode=tn.TN_MODE_PLAIN, fp64=False)
    for v in (x, x_s, x_2, x_1, x_m, x_g, x_t, x_p):
        assert np.allclose(v, r["X"], rtol=2e-5, atol=1e-10)


def test_small_levels_run_in_one_launch_and_depth_is_reduced():
    """The 225-qubit workload's per-estimate work is small at every level: its
    matrix-core-shaped steps join their level's small-step launch (one launch
    per level; all_tiles keeps the tile launches), the dominant-term pass
    shares those launches, slot-free subtrees run once per binding, and the
    tree's per-estimate depth is 6 (the cheapest path's is 9)."""
    c = W.config(5)
    plan = tn.tn_plan_build(c, 3)
    t = tn.tn_terms_enumerate(plan, 3)
    d, _ = tn.tn_exec_describe_only([plan], [t])
    batch = [L for L in d["launches"] if L["phase"] in ("batch", "batch64")]
    assert all(L["kind"] == 5 for L in batch) and len(batch) == 6, [(L["kind"], L["level"]) for L in batch]
    assert sorted(L["level"] for L in batch) == [1, 2, 3, 4, 5, 6]
    assert any(j["fp64"] for L in batch for j in L["jobs"]) and any(not j["fp64"] for L in batch for j in L["jobs"])
    assert any(L["phase"] == "const" for L in d["launches"])
    assert d["tail_blocks"] == (t.n + 255) // 256
    d_all, _ = tn.tn_exec_describe_only([plan], [t], tn.exec_opts(all_tiles=True))
    assert any(L["kind"] == 6 and not L["fp64"] for L in d_all["launches"] if L["phase"] == "batch")


@pytest.mark.parametrize("cfg", [2, 3])
def test_merged_slices_are_grouped_and_b_groups_ordered_by_their_a(cfg):
    """Slice order of the merged matrix-core jobs in the real schedules: a job
    whose tiles stack slices sharing B holds each B's slices in one run, the
    runs ordered by their smallest A (neighbouring tiles then share A panels);
    a job whose tiles put slices sharing A side by side keeps A ascending."""
    c = W.config(cfg)
    plan = tn.tn_plan_build(c, c.level)
    t = tn.tn_terms_enumerate(plan, c.level)
    d, cb = tn.tn_exec_describe_only([plan], [t], tn.exec_opts(use_graph=False))
    sim = Sim(d, cb)
    seen = {1: 0, 2: 0}
    for L in d["launches"]:
        if L["kind"] != 6:
            continue
        for jb in L["jobs"]:
            if jb["merge"] == 0:
                continue
            ns = jb["ns"]
            oa = sim.view(jb["oa"], np.int64, ns)
            ob = sim.view(jb["ob"], np.int64, ns)
            seen[jb["merge"]] += 1
            if jb["merge"] == 1:
                assert np.all(np.diff(oa) >= 0)
                continue
            starts = np.flatnonzero(np.r_[True, ob[1:] != ob[:-1]])
            assert len(starts) == len(np.unique(ob)), "a B's slices split into several runs"
            mins = [oa[a:b].min() for a, b in zip(starts, np.r_[starts[1:], ns])]
            assert all(x <= y for x, y in zip(mins, mins[1:]))
    assert seen[1] > 0 and (cfg != 3 or seen[2] > 0), seen


def test_schedule_replay_config1_against_oracle():
    c = W.config(1, level=2)
    x, pat, desc = _replay(c, 2)
    r = estimate.estimate(c, 2, "network")
    assert np.allclose(x, r["X"], rtol=2e-5, atol=1e-10)
    assert abs(x.sum() - r["A"][2]) < 1e-6 * r["A"][2]


def test_bound_feature_bounds_every_term_and_features_are_finite():
    # |a| <= prod of the slot spectral norms for unit states and unitary gates,
    # so X_t <= w_t prod ||K_hat||^2 = exp(feature 35) for every term
    for seed, kind in ((41, "adpd"), (42, "random"), (43, "depol")):
        c = W.tiny_random_circuit(np.random.default_rng(seed), 4, 20, 5, noise=kind, level=3)
        plan = tn.tn_plan_build(c, 3)
        t = tn.tn_terms_enumerate(plan, 3)
        r = estimate.estimate(c, 3, "network")
        f = tn.tn_terms_features(plan, t, r["X"][:16])
        assert f.shape == (t.n, tn.TN_N_FEATURES) and np.all(np.isfinite(f))
        pat, w = t.get()
        # terms whose weight the library takes as exactly zero (a singular
        # value at rounding level) are excluded; the oracle gives them ~1e-18
        live = (r["X"] > 0) & (w > 0)
        assert np.all(r["X"][live] <= np.exp(f[live, 35].astype(np.float64)) * (1 + 1e-5))
        assert np.all(r["X"][w == 0] < 1e-15)
        assert np.array_equal(f[:, 34], (pat != 0).sum(1))


def test_prune_threshold_respects_the_budget():
    rng = np.random.default_rng(9)
    x = rng.exponential(1.0, 1000)
    pred = np.log(x) + rng.normal(0, 0.5, 1000)
    for budget in (0.0, 1.0, 10.0, 100.0, 1e9):
        tau = tn.tn_prune_threshold(pred, x, budget)
        dropped = x[pred.astype(np.float32) < np.float32(tau)].sum()
        assert dropped <= budget + 1e-9
        # dropping one more candidate (the next by score) would exceed the budget
        rest = np.sort(pred.astype(np.float32)[pred.astype(np.float32) >= np.float32(tau)])
        if rest.size and budget < 1e9:
            nxt = pred.astype(np.float32) == rest[0]
            assert dropped + x[nxt].sum() > budget


# ---------------------------------------------------------------------------
# exact value: the doubled network (every noise as its whole superoperator)
# ---------------------------------------------------------------------------
def _replay_doubled(circ, mode=tn.TN_MODE_BATCHED, fp64=True, **plan_kw):
    plan = tn.tn_plan_build_doubled(circ, **plan_kw)
    t = tn.tn_terms_enumerate(plan, 0)
    desc, cb = tn.tn_exec_describe_only([plan], [t], tn.exec_opts(mode=mode, use_graph=False,
                                                                  fp64_level0=fp64))
    sim = Sim(desc, cb)
    sim.run([[0]])
    x, _ = sim.outputs()
    return x, plan, t, desc


def test_doubled_plan_has_one_term_and_no_slots():
    c = W.tiny_random_circuit(np.random.default_rng(51), 4, 16, 5, noise="random", level=3)
    plan = tn.tn_plan_build_doubled(c)
    info = plan.info()
    assert info["doubled"] == 1 and info["n_channels"] == 5 and info["n_noise"] == 0 and info["level"] == 0
    assert all(leaf.get("slot", -1) < 0 for leaf in plan.describe().get("leaves", []))
    for level in (0, 3):
        t = tn.tn_terms_enumerate(plan, level)
        pat, w = t.get()
        assert t.n == 1 and list(w) == [1.0]
    # the estimate's plan of the same circuit is unchanged by the doubled one
    assert tn.tn_plan_build(c, 3).info()["doubled"] == 0


def test_doubled_accepts_a_degenerate_channel_the_split_rejects():
    c = W.tiny_random_circuit(np.random.default_rng(52), 3, 10, 0, noise="random", level=1)
    ops = list(c.ops) + [W.Op("noise", (1,), kraus=W.kraus_depolarizing(0.75))]
    c = W.Circuit(c.n_qubits, ops, c.psi, c.target, c.v, 1)
    with pytest.raises(tn.TNError) as e:
        tn.tn_plan_build(c, 1)
    assert e.value.code == tn.TN_EDEGENERATE
    x, _, _, _ = _replay_doubled(c)
    assert abs(x[0] - dense.exact_value(c)) <= 1e-12


@pytest.mark.parametrize("seed,kind,target", [(53, "random", "circuit_output"), (54, "adpd", "product"),
                                               (55, "depol", "dense"), (56, "random", "product")])
def test_doubled_replay_matches_the_exact_value(seed, kind, target):
    """The doubled schedule replayed on the CPU (FP64 pass for its one term)
    gives the density-matrix value and the oracle's doubled contraction."""
    c = W.tiny_random_circuit(np.random.default_rng(seed), 4, 18, 5, noise=kind, level=2, target=target)
    x, _, _, _ = _replay_doubled(c)
    f = dense.exact_value(c)
    assert abs(x[0] - f) <= 1e-12 * max(1.0, abs(f))
    assert abs(x[0] - doubled.doubled_value(c).real) <= 1e-12 * max(1.0, abs(f))
    # without the FP64 pass the one term runs in FP32
    x32, _, _, _ = _replay_doubled(c, fp64=False)
    assert abs(x32[0] - f) <= 1e-5 * max(1.0, abs(f))


def test_doubled_replay_wide_circuit_with_matrix_core_steps():
    """16 qubits: the doubled network's tensors reach the matrix-core and FP64
    tile paths; no density matrix, so the oracle's doubled contraction and the
    full expansion at level N pin the value."""
    c = W.tiny_random_circuit(np.random.default_rng(57), 16, 160, 4, noise="adpd", level=4,
                              target="circuit_output")
    x, plan, _, desc = _replay_doubled(c)
    steps = [L for L in desc["launches"] if L["kind"] in (5, 6)]
    assert steps and all(L["fp64"] for L in steps)      # the FP64 pass alone: no FP32 chain
    _, _, _, desc32 = _replay_doubled(c, fp64=False)
    assert any(L["kind"] == 6 and not L["fp64"] for L in desc32["launches"])
    want = doubled.doubled_value(c, diagonal=True).real
    assert abs(x[0] - want) <= 1e-12 * max(1.0, abs(want))
    r = estimate.estimate(c, 4, "network", reduce=True)
    assert abs(x[0] - r["A"][-1]) <= 1e-12 * max(1.0, abs(want))


# ---------------------------------------------------------------------------
# off-diagonal elements: bond-2 targets of the polarization identity
# ---------------------------------------------------------------------------
def _rand_product(rng, n):
    z = rng.standard_normal((n, 2)) + 1j * rng.standard_normal((n, 2))
    return z / np.linalg.norm(z, axis=1, keepdims=True)


def test_polarization_combine_matches_the_identity():
    rng = np.random.default_rng(81)
    res = (tn.tn_result * 4)()
    a = rng.standard_normal((4, 3))
    for k in range(4):
        res[k].level = 2
        for u in range(3):
            res[k].A[u] = a[k, u]
    re = (ctypes.c_double * 3)()
    im = (ctypes.c_double * 3)()
    assert tn.lib().tn_polarization_combine(res, re, im) == tn.TN_OK
    want = sum((1j ** k) / 4 * a[k] for k in range(4))
    assert np.allclose([complex(re[u], im[u]) for u in range(3)], want, rtol=0, atol=1e-15)
    res[3].level = 1
    assert tn.lib().tn_polarization_combine(res, re, im) == tn.TN_EINVAL


def _levels_from_replay(x, pat, level):
    t = np.zeros(level + 1)
    for row, v in zip(pat, x):
        t[int(np.count_nonzero(row))] += v
    return np.cumsum(t)


@pytest.mark.parametrize("seed,kind,output", [(82, "random", True), (83, "adpd", False), (84, "random", False)])
def test_bond2_targets_replay_matches_the_cross_form(seed, kind, output):
    """Each of the four polarization targets is a bond-2 network end (one
    shared 2-valued index); the replayed estimates combined with i^k / 4 give
    the oracle's cross-form element level by level."""
    rng = np.random.default_rng(seed)
    c = W.tiny_random_circuit(rng, 4, 18, 4, noise=kind, level=3,
                              target="circuit_output" if output else "product")
    x, y = _rand_product(rng, 4), _rand_product(rng, 4)
    got = np.zeros(4, dtype=np.complex128)
    for k, ck in enumerate(tn.polarization_circuits(c, x, y, output)):
        xs, pat, _ = _replay(ck, 3)
        got += (1j ** k) / 4 * _levels_from_replay(xs, pat, 3)
    want = offdiag.element_cross(c, 3, x, y, output)["A"]
    assert np.allclose(got, want, rtol=0, atol=2e-6), (got, want)
    # the all-dominant terms come from the FP64 pass: level 0 agrees to rounding
    assert abs(got[0] - want[0]) <= 1e-12


def test_bond2_doubled_networks_give_the_exact_element():
    rng = np.random.default_rng(85)
    c = W.tiny_random_circuit(rng, 4, 16, 5, noise="random", level=2, target="circuit_output")
    x, y = _rand_product(rng, 4), _rand_product(rng, 4)
    got = 0j
    for k, ck in enumerate(tn.polarization_circuits(c, x, y, True)):
        xs, _, _, _ = _replay_doubled(ck)
        got += (1j ** k) / 4 * xs[0]
    assert abs(got - offdiag.element_exact(c, x, y, True)) <= 1e-12


# ---------------------------------------------------------------------------
# exact cross-term reuse: factored term sets over independent clusters
# ---------------------------------------------------------------------------
def _two_blocks(seed, kind="random"):
    from tests.test_oracle_factored import two_blocks
    return two_blocks(seed, kind=kind)


def test_factored_terms_cover_single_cluster_patterns():
    c = W.config(5)
    plan = tn.tn_plan_build(c, 3)
    t = tn.tn_terms_enumerate_factored(plan, 3)
    starts, lv, cl = t.groups
    pat, w = t.get()
    assert starts[0] == 0 and starts[-1] == t.n and lv[0] == 0 and cl[0] == -1
    assert np.all(np.diff(lv) >= 0)                       # levels ascending
    clusters = [set(x["slots"]) for x in plan.describe()["clusters"]]
    for g in range(1, len(lv)):
        rows = pat[starts[g]:starts[g + 1]]
        assert np.all((rows != 0).sum(1) == lv[g])
        assert all(set(np.flatnonzero(r)) <= clusters[cl[g]] for r in rows)
    # every single-cluster pattern up to level 3, once
    import math
    want = 1 + sum(math.comb(len(s), u) * 3 ** u for s in clusters for u in range(1, 4))
    assert t.n == want < 32551
    with pytest.raises(tn.TNError):
        tn.tn_terms_enumerate_factored(tn.tn_plan_build_doubled(c), 1)


@pytest.mark.parametrize("seed,kind", [(111, "random"), (112, "adpd")])
def test_factored_replay_matches_the_global_oracle(seed, kind):
    c = _two_blocks(seed, kind)
    plan = tn.tn_plan_build(c, 4)
    assert plan.info()["n_clusters"] >= 2
    t = tn.tn_terms_enumerate_factored(plan, 4)
    desc, cb = tn.tn_exec_describe_only([plan], [t], tn.exec_opts(use_graph=False))
    sim = Sim(desc, cb)
    _, w = t.get()
    sim.run([[i for i in range(t.n) if w[i] != 0.0]])
    x, _ = sim.outputs()
    starts = t.groups[0]
    h = np.array([x[starts[g]:starts[g + 1]].sum() for g in range(len(starts) - 1)])
    A = np.zeros(5)
    assert tn.lib().tn_factored_levels(t.handle, h.ctypes.data, A.ctypes.data) == tn.TN_OK
    ref = estimate.estimate(c, 4, "network")["A"]
    assert np.allclose(A, ref, rtol=2e-6, atol=0), (A, ref)
    assert abs(A[0] - ref[0]) <= 1e-12 * ref[0]


# ---------------------------------------------------------------------------
# quantum trajectories on the same engine
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed,kind,target", [(141, "random", "circuit_output"), (142, "adpd", "product"),
                                               (143, "depol", "dense")])
def test_trajectories_replay_matches_the_oracle_sample_by_sample(seed, kind, target):
    from oracle import trajectories
    c = W.tiny_random_circuit(np.random.default_rng(seed), 4, 18, 4, noise=kind, level=1, target=target,
                              scale=5.0)
    u = W.trajectory_uniforms(300, c.n_noises, seed)
    plan = tn.tn_plan_build_trajectories(c)
    t = tn.tn_terms_trajectories(plan, u)
    pat, w = t.get()
    ref = trajectories.estimate(c, u)
    assert np.array_equal(pat, ref["idx"])                  # the same draws from the same uniforms
    assert np.allclose(w, 1.0 / 300)
    desc, cb = tn.tn_exec_describe_only([plan], [t], tn.exec_opts(use_graph=False))
    sim = Sim(desc, cb)
    sim.run([list(range(t.n))])
    x, _ = sim.outputs()
    assert np.allclose(x * 300, ref["X"], rtol=2e-5, atol=1e-9)
    assert abs(x.sum() - ref["mean"]) <= 2e-6 * ref["mean"]


def test_trajectories_plan_rejects_enumeration_and_bad_input():
    c = W.tiny_random_circuit(np.random.default_rng(144), 3, 10, 3, noise="random", level=1)
    plan = tn.tn_plan_build_trajectories(c)
    for call in (lambda: tn.tn_terms_enumerate(plan, 1), lambda: tn.tn_terms_enumerate_factored(plan, 1),
                 lambda: tn.tn_terms_trajectories(plan, np.full((2, 3), 1.0)),
                 lambda: tn.tn_terms_trajectories(tn.tn_plan_build(c, 1), np.zeros((2, 3)))):
        with pytest.raises(tn.TNError) as e:
            call()
        assert e.value.code == tn.TN_EINVAL
    ops = list(c.ops) + [W.Op("noise", (0,), kraus=[np.eye(2) * np.sqrt(0.2)] * 5)]
    with pytest.raises(tn.TNError) as e:
        tn.tn_plan_build_trajectories(W.Circuit(3, ops, c.psi, c.target, c.v, 1))
    assert e.value.code == tn.TN_EUNSUPPORTED


def test_pruner_save_size_query_and_header_check():
    shape = tn.tn_mlp_shape(36, 64, 2)
    L = tn._mlp_lib()
    need = ctypes.c_size_t()
    assert L.tn_pruner_save(ctypes.byref(shape), None, None, 0, ctypes.byref(need), None) == tn.TN_OK
    npar = ctypes.c_int64()
    assert L.tn_mlp_sizes(ctypes.byref(shape), 1, ctypes.byref(npar), None, None) == tn.TN_OK
    assert need.value == 32 + 4 * (2 * 36 + npar.value)
    bad = (ctypes.c_uint8 * need.value)()
    dummy = ctypes.c_void_p(1)      # rejected before any device access
    assert L.tn_pruner_load(ctypes.byref(shape), dummy, bad, need.value, None) == tn.TN_EINVAL


# ---------------------------------------------------------------------------
# edge cases of the exact value, factored sums, trajectories, off-diagonals
# ---------------------------------------------------------------------------
def test_doubled_without_noise_is_the_squared_overlap():
    c = W.tiny_random_circuit(np.random.default_rng(161), 4, 16, 0, noise="random", level=1, target="product")
    x, plan, _, _ = _replay_doubled(c)
    st = dense.ideal_state(c, dense.product_state(c.psi))
    want = abs(np.vdot(dense.target_vector(c), st)) ** 2
    assert plan.info()["n_channels"] == 0 and abs(x[0] - want) <= 1e-12


def test_factored_level0_and_single_cluster_equal_the_global_sums():
    rng = np.random.default_rng(162)
    c = W.tiny_random_circuit(rng, 4, 18, 4, noise="adpd", level=2)
    plan = tn.tn_plan_build(c, 2)
    for level in (0, 2):
        t = tn.tn_terms_enumerate_factored(plan, level)
        desc, cb = tn.tn_exec_describe_only([plan], [t], tn.exec_opts(use_graph=False))
        sim = Sim(desc, cb)
        _, w = t.get()
        sim.run([[i for i in range(t.n) if w[i] != 0.0]])
        x, _ = sim.outputs()
        st = t.groups[0]
        h = np.array([x[st[g]:st[g + 1]].sum() for g in range(len(st) - 1)])
        A = np.zeros(level + 1)
        assert tn.lib().tn_factored_levels(t.handle, h.ctypes.data, A.ctypes.data) == tn.TN_OK
        ref = estimate.estimate(c, level, "network")["A"]
        assert np.allclose(A, ref, rtol=2e-6, atol=0)
        if plan.info()["n_clusters"] == 1:
            assert t.n == len(oterms.enumerate_terms(c.n_noises, level))   # one cluster: every term


def test_trajectories_never_draw_a_zero_kraus_operator():
    from oracle import trajectories
    c = W.tiny_random_circuit(np.random.default_rng(163), 3, 12, 2, noise="random", level=1)
    kr = W.kraus_ad_pd(0.3, 0.2)                   # three Kraus operators
    assert len(kr) == 3
    kr = [kr[0], np.zeros((2, 2), dtype=np.complex128), kr[1], kr[2]]   # an empty slot in between
    ops = list(c.ops) + [W.Op("noise", (1,), kraus=kr)]
    c = W.Circuit(c.n_qubits, ops, c.psi, c.target, c.v, 1)
    u = W.trajectory_uniforms(500, c.n_noises, 163)
    plan = tn.tn_plan_build_trajectories(c)
    t = tn.tn_terms_trajectories(plan, u)
    pat, _ = t.get()
    assert not np.any(pat[:, -1] == 1)
    assert np.array_equal(pat, trajectories.sample_indices(c, u))


def test_offdiagonal_with_equal_targets_is_the_diagonal_estimate():
    rng = np.random.default_rng(164)
    c = W.tiny_random_circuit(rng, 4, 16, 3, noise="adpd", level=2, target="circuit_output")
    got = np.zeros(3, dtype=np.complex128)
    for k, ck in enumerate(tn.polarization_circuits(c, c.v, c.v, True)):
        xs, pat, _ = _replay(ck, 2)
        got += (1j ** k) / 4 * _levels_from_replay(xs, pat, 2)
    ref = estimate.estimate(c, 2, "network")["A"]
    assert np.allclose(got.real, ref, rtol=2e-6, atol=0) and np.all(np.abs(got.imag) <= 1e-9)
