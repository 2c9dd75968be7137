"""GPU parity tests: the HIP kernels against numpy references, and the full
estimate through the C ABI against the FP64 oracle.

Tolerances.  Term networks are contracted in complex64 with FP32 MFMA
accumulation: an inner product of length k carries a relative rounding error
of order sqrt(k) * 6e-8 per step, so per-term values are compared at 2e-5
relative (plus an absolute floor below the smallest term that matters).  The
all-dominant term is recomputed in FP64 and compared at 1e-12.  Level sums
A(l) must match the oracle within 1e-6 relative (the FP32 error of the
correction terms is scaled by their small share of the total).
"""
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


def crandn(rng, shape, dtype):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(dtype)


GEMM_CASES = [
    # m_log, n_log, k_log, transA, transB, n_inst, gathered
    (7, 6, 3, 0, 0, 1, False), (5, 4, 0, 0, 0, 3, False), (8, 7, 5, 1, 0, 2, True),
    (6, 5, 10, 0, 1, 2, True), (10, 6, 2, 1, 1, 4, True), (7, 10, 13, 0, 0, 3, True),
    (5, 5, 7, 0, 0, 5, True), (3, 2, 2, 0, 0, 7, True), (10, 1, 2, 1, 0, 2, False),
    (0, 3, 4, 0, 1, 3, True), (0, 0, 12, 0, 0, 4, True), (1, 1, 10, 1, 1, 2, False),
    (4, 9, 6, 0, 0, 2, False), (6, 6, 6, 1, 1, 9, True),
]


@pytest.mark.parametrize("case", GEMM_CASES)
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_gemm_kernels_against_numpy(torch, case, dtype):
    m_log, n_log, k_log, ta, tb, ni, gathered = case
    print(f"gemm case {case} {dtype}", flush=True)
    rng = np.random.default_rng(hash(case) % 2 ** 31)
    m, n, k = 1 << m_log, 1 << n_log, 1 << k_log
    npdt = np.complex64 if dtype == "c64" else np.complex128
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    na, nb = (3, 2) if gathered else (ni, ni)
    A = crandn(rng, (na, m * k), npdt)
    B = crandn(rng, (nb, k * n), npdt)
    ia = rng.integers(0, na, ni).astype(np.int32) if gathered else np.arange(ni, dtype=np.int32)
    ib = rng.integers(0, nb, ni).astype(np.int32) if gathered else np.arange(ni, dtype=np.int32)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dC = torch.zeros((ni, m * n), dtype=tdt, device="cuda")
    dia = torch.from_numpy(ia).cuda() if gathered else None
    dib = torch.from_numpy(ib).cuda() if gathered else None
    kc = tn.kernel_gemm(dA, dB, dC, m_log, n_log, k_log, ta, tb, dia, dib)
    torch.cuda.synchronize()
    Am = A.reshape(na, k, m).transpose(0, 2, 1) if ta else A.reshape(na, m, k)
    Bm = B.reshape(nb, n, k).transpose(0, 2, 1) if tb else B.reshape(nb, k, n)
    ref = np.matmul(Am[ia].astype(np.complex128), Bm[ib].astype(np.complex128)).reshape(ni, m * n)
    got = dC.cpu().numpy()
    tol = (2e-6 if dtype == "c64" else 1e-13) * math.sqrt(k) * 4
    err = np.max(np.abs(got - ref)) / max(1.0, math.sqrt(k))
    assert err < tol, (kc, err)


@pytest.mark.parametrize("r", [0, 1, 3, 5, 6, 9, 12])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_permute_kernel_is_exact(torch, r, dtype):
    print(f"permute r={r} {dtype}", flush=True)
    rng = np.random.default_rng(100 + r)
    npdt = np.complex64 if dtype == "c64" else np.complex128
    ni = 3
    x = crandn(rng, (ni, 1 << r), npdt)
    for trial in range(3):
        perm = rng.permutation(r).astype(np.int32)
        src = torch.from_numpy(x).cuda()
        dst = torch.zeros_like(src)
        tn.kernel_permute(src, dst, r, perm)
        torch.cuda.synchronize()
        t = x.reshape((ni,) + (2,) * r)
        axes = [0] + [1 + (r - 1 - perm[r - 1 - a]) for a in range(r)]
        ref = np.transpose(t, axes).reshape(ni, -1)
        assert np.array_equal(dst.cpu().numpy(), ref)


def run_gpu(circ, level, mode=tn.TN_MODE_BATCHED, graph=False, fp64=True):
    plan = tn.tn_plan_build(circ, level)
    terms = tn.tn_terms_enumerate(plan, level)
    ex = tn.tn_exec_prepare([plan], [terms], tn.exec_opts(mode=mode, use_graph=graph, fp64_level0=fp64))
    res = ex.run()[0]
    x, _ = ex.values()
    pat, w = terms.get()
    return res, x, pat, ex


def grouped_by_positions(pat, x):
    out = {}
    for row, v in zip(pat, x):
        key = tuple(i for i, c in enumerate(row) if c)
        out[key] = out.get(key, 0.0) + v
    return out


def assert_terms_close(x_gpu, x_ref, pat, degenerate, rtol=2e-5, atol=1e-12):
    if degenerate:
        g1, g2 = grouped_by_positions(pat, x_gpu), grouped_by_positions(pat, x_ref)
        for k in g2:
            assert abs(g1[k] - g2[k]) <= rtol * abs(g2[k]) + atol, (k, g1[k], g2[k])
    else:
        err = np.abs(x_gpu - x_ref)
        bad = err > rtol * np.abs(x_ref) + atol
        assert not bad.any(), (np.flatnonzero(bad)[:5], x_gpu[bad][:5], x_ref[bad][:5])


@pytest.mark.parametrize("level", [1, 2, 4])
def test_config1_against_oracle(torch, level):
    print(f"config1 level {level}", flush=True)
    c = W.config(1, level=level)
    res, x, pat, _ = run_gpu(c, level)
    ref = estimate.estimate(c, level, "network")
    assert [tuple(p) for p in pat] == ref["terms"]
    assert abs(x[0] - ref["X"][0]) <= 1e-12 * ref["X"][0]          # FP64 dominant term
    assert_terms_close(x, ref["X"], pat, degenerate=False)
    for u in range(level + 1):
        assert abs(res["A"][u] - ref["A"][u]) <= 1e-6 * ref["A"][u], (u, res["A"][u], ref["A"][u])
        assert abs(res["T"][u] - ref["T"][u]) <= 2e-5 * abs(ref["T"][u]) + 1e-12
    pc.check_against_golden(res["T"], x, pat, ref["T"], ref["X"], network.slot_split(c), degenerate=False)
    if level == 4:
        from oracle import dense
        f = dense.exact_value(c)
        assert abs(res["A"][4] - f) <= 1e-6 * f


@pytest.mark.parametrize("seed,kind,target,n,gates,noise", [
    (1, "random", "circuit_output", 5, 30, 4), (2, "adpd", "product", 4, 24, 5),
    (3, "depol", "dense", 5, 30, 4), (4, "random", "product", 6, 40, 3),
    (5, "adpd", "circuit_output", 7, 50, 6)])
def test_tiny_circuits_against_oracle(torch, seed, kind, target, n, gates, noise):
    print(f"tiny {seed} {kind} {target}", flush=True)
    c = W.tiny_random_circuit(np.random.default_rng(seed), n, gates, noise, noise=kind, level=3,
                              target=target)
    res, x, pat, _ = run_gpu(c, 3)
    ref = estimate.estimate(c, 3, "network")
    assert_terms_close(x, ref["X"], pat, degenerate=(kind == "depol"), atol=1e-10)
    for u in range(4):
        assert abs(res["A"][u] - ref["A"][u]) <= 1e-6 * abs(ref["A"][u]) + 1e-12


def test_plain_mode_equals_batched(torch):
    c = W.config(1, level=2)
    rb, xb, pat, _ = run_gpu(c, 2)
    rp, xp, _, _ = run_gpu(c, 2, mode=tn.TN_MODE_PLAIN, fp64=False)
    assert np.allclose(xb[1:], xp[1:], rtol=1e-5, atol=1e-12)
    assert abs(rb["A"][2] - rp["A"][2]) <= 1e-6 * rb["A"][2]


def test_graph_replays_match_eager_and_are_deterministic(torch):
    c = W.config(1, level=2)
    plan = tn.tn_plan_build(c, 2)
    terms = tn.tn_terms_enumerate(plan, 2)
    eager = tn.tn_exec_prepare([plan], [terms], tn.exec_opts(use_graph=False)).run()[0]
    ex = tn.tn_exec_prepare([plan], [terms], tn.exec_opts(use_graph=True))
    for rep in range(4):
        r = ex.run()[0]
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()      # eager work between replays
        assert r["A"] == eager["A"], (rep, r["A"], eager["A"])
        assert r["T"] == eager["T"]


def _golden(cfg):
    return (np.loadtxt(os.path.join(GOLD, f"config{cfg}_oracle.txt")),
            np.loadtxt(os.path.join(GOLD, f"config{cfg}_levels.txt")),
            np.load(os.path.join(GOLD, f"config{cfg}_terms.npy")))


def test_config2_every_term_against_oracle(torch):
    """5x5 grid, 12 layers, 10 depolarizing noises, level 2 (436 terms): every
    term on the GPU against the oracle's stored per-term values (depolarizing
    corrections are degenerate, so the sums over each of the 56 noise-position
    sets are compared, each within the summed FP32 bounds of its terms), every
    T_u against the stored level sums, and every T_u against math.fsum of the
    same GPU X_t at 1e-12."""
    print("config2 full size", flush=True)
    c = W.config(2)
    res, x, pat, _ = run_gpu(c, 2)
    assert res["n_terms"] == 436
    assert np.all(x >= 0)
    assert res["A"][0] <= res["A"][1] <= res["A"][2] <= 1.0 + 1e-6
    gold_a, gold_t, gold_x = _golden(2)
    pc.check_against_golden(res["T"], x, pat, gold_t, gold_x, network.slot_split(c), degenerate=True)
    for u in range(3):
        assert abs(res["A"][u] - gold_a[u]) <= 1e-6 * gold_a[u], (u, res["A"][u], gold_a[u])
    # the all-dominant term from the FP32 batch (diagnostic, written by the finalize)
    # agrees with its FP64 value to FP32 accuracy
    assert abs(res["x0_fp32"] - x[0]) <= 2e-5 * x[0], (res["x0_fp32"], x[0])


def fp32_term_tol(split, term, ref):
    return pc.fp32_term_tol(split, term, ref)


def _sample_terms(pat, w, rng, per_level):
    """A few live terms of every level (always the all-dominant one)."""
    lv = (pat != 0).sum(axis=1)
    out = [0]
    for u in range(1, lv.max() + 1):
        idx = np.flatnonzero((lv == u) & (w > 0))
        if idx.size:
            out += list(rng.choice(idx, size=min(per_level, idx.size), replace=False))
    return out


@pytest.mark.parametrize("cfg", [3, 5])
def test_full_size_config_against_oracle(torch, cfg):
    """Config 3 (QAOA p=2, 36 qubits, 20 AD+PD, level 2, 1771 terms) and
    config 5 (15x15 grid, 6 layers, 20 AD+PD, level 3, 32551 terms): every
    term on the GPU against the oracle's stored per-term values (FP32 terms
    within fp32_term_tol, the FP64 dominant term within 1e-12), every T_u
    against the stored level sums within 2e-5 T_u plus the level's summed
    term bounds, every T_u against math.fsum of the same GPU X_t at 1e-12,
    and A(l) against the stored sums at 1e-6."""
    print(f"config{cfg} full size", flush=True)
    c = W.config(cfg)
    res, x, pat, _ = run_gpu(c, c.level)
    assert res["n_terms"] == {3: 1771, 5: 32551}[cfg]
    assert np.all(x >= 0)
    assert all(res["A"][u] <= res["A"][u + 1] + 1e-12 for u in range(c.level))
    gold_a, gold_t, gold_x = _golden(cfg)
    pc.check_against_golden(res["T"], x, pat, gold_t, gold_x, network.slot_split(c), degenerate=False)
    for u in range(c.level + 1):
        assert abs(res["A"][u] - gold_a[u]) <= 1e-6 * gold_a[u], (u, res["A"][u], gold_a[u])
    # a few terms of every level recomputed by the oracle now (the stored file
    # is the oracle's; BLAS threading changes its rounding, which for a small
    # term is a multiple of eps64 times its bound, not of the term)
    net = network.KetNetwork(c, diagonal=True)
    sp = network.slot_split(c)
    w = terms_weights(c)
    for j in _sample_terms(pat, w, np.random.default_rng(cfg), 2):
        term = tuple(int(v) for v in pat[j])
        ref, _ = network.term_value(net, sp, term)
        tol = 1e-12 * ref + 2.0 ** -40 * math.sqrt(ref * pc.term_bound(sp, term))
        assert abs(ref - gold_x[j]) <= tol, (j, ref, gold_x[j], tol)


def terms_weights(c):
    sp = network.slot_split(c)
    from oracle import terms as oterms
    tl = oterms.enumerate_terms(c.n_noises, c.level)
    return np.array([np.prod([sp[s][0][t[s]] for s in range(len(t))]) for t in tl])


def test_packed_uneven_batch_against_oracle(torch):
    """Config 4: 64 chain / grid circuits of 16..100 qubits packed into one
    prepared schedule; per circuit: terms non-negative, levels monotone,
    sampled terms against the oracle one by one; full A(l) against the oracle
    for the circuits with at most 300 terms."""
    print("config4 packed", flush=True)
    cs = W.config(4)
    plans = [tn.tn_plan_build(c, c.level) for c in cs]
    terms = [tn.tn_terms_enumerate(p, c.level) for p, c in zip(plans, cs)]
    ex = tn.tn_exec_prepare(plans, terms, tn.exec_opts(use_graph=False))
    results = ex.run()
    with pytest.raises(tn.TNError):    # packed outputs are per plan: no single device array
        ex.outputs()
    rng = np.random.default_rng(4)
    n_full = 0
    for i, (c, r) in enumerate(zip(cs, results)):
        x, _ = ex.values(i)
        pat, w = terms[i].get()
        assert r["n_terms"] == terms[i].n
        assert np.all(x >= 0)
        lv = (pat != 0).sum(axis=1)
        for u in range(r["level"] + 1):     # FP64 level sums of the same X_t
            fs = math.fsum(float(v) for v in x[lv == u])
            assert abs(r["T"][u] - fs) <= 1e-12 * fs + 1e-300, (c.name, u, r["T"][u], fs)
        assert all(r["A"][u] <= r["A"][u + 1] + 1e-12 for u in range(r["level"]))
        net = network.KetNetwork(c, diagonal=True)
        sp = network.slot_split(c)
        if terms[i].n <= 300 and n_full < 6:
            n_full += 1
            ref = estimate.estimate(c, c.level, "network")
            for u in range(r["level"] + 1):
                assert abs(r["A"][u] - ref["A"][u]) <= 1e-6 * ref["A"][u], (c.name, u)
        else:
            # depolarizing corrections are degenerate: compare the sum over
            # the corrections of each sampled term's position set
            keys = [tuple(np.flatnonzero(row)) for row in pat]
            for j in _sample_terms(pat, w, rng, 1):
                group = [t for t in range(len(pat)) if keys[t] == keys[j]]
                ref = sum(network.term_value(net, sp, tuple(int(v) for v in pat[t]))[0] for t in group)
                got = float(sum(x[t] for t in group))
                tol = 1e-12 if j == 0 else 2e-5
                assert abs(got - ref) <= tol * ref + 1e-15, (c.name, keys[j], got, ref)
    assert n_full >= 3


def test_autotuned_grouped_schedule_gives_the_same_estimate(torch):
    """Grouped launches with tile shapes chosen by timing (every FP32 level
    with tile launches: whole estimates with the model's choice at the level
    against estimates with each of the 8 shapes imposed on all its jobs):
    every term within its FP32 bound of the oracle's stored values, the level
    sums within the parity bar; a level keeps the model's choice unless a
    shape was more than 5 % faster, and a kept shape is what the level's tile
    launches use."""
    print("autotuned grouped config2", flush=True)
    c = W.config(2)
    plan = tn.tn_plan_build(c, 2)
    terms = tn.tn_terms_enumerate(plan, 2)
    ext = tn.tn_exec_prepare([plan], [terms], tn.exec_opts(use_graph=False, tune=True))
    r1 = ext.run()[0]
    x, _ = ext.values()
    pat, _ = terms.get()
    gold_a, gold_t, gold_x = _golden(2)
    pc.check_against_golden(r1["T"], x, pat, gold_t, gold_x, network.slot_split(c), degenerate=True)
    for u in range(3):
        assert abs(r1["A"][u] - gold_a[u]) <= 1e-6 * gold_a[u]
    d = ext.describe()
    tuned = d["tuning"]
    levels = {L["level"] for L in d["launches"] if L["kind"] == 6 and not L["fp64"] and L["phase"] == "batch"}
    assert tuned and {t["level"] for t in tuned} == levels, (tuned, levels)
    for t in tuned:
        if t["us"]:            # timed here (not a cached choice)
            timed = [v for v in t["us"] if v >= 0]
            kept = t["model_us"] if t["tile"] < 0 else t["us"][t["tile"]]
            # a shape replaces the model's only when more than 5 % faster
            # (the autotuner's margin), so nothing timed beats the kept one by more
            assert kept > 0 and all(v >= 0.95 * kept * (1 - 1e-12) for v in timed), t
            if t["tile"] >= 0:
                assert kept < 0.95 * t["model_us"], t
        if t["tile"] >= 0:
            shapes = {(L["bm"], L["bn"]) for L in d["launches"]
                      if L["kind"] == 6 and not L["fp64"] and L["level"] == t["level"]}
            assert shapes == {(t["bm"], t["bn"])}, (t, shapes)


def test_autotuned_schedule_gives_the_same_estimate(torch):
    """Tiles chosen by timing on the per-step schedule (no grouping) change
    rounding only: the estimate stays within the parity bar of the oracle's
    stored sums and of the untuned run."""
    c = W.config(2)
    plan = tn.tn_plan_build(c, 2)
    terms = tn.tn_terms_enumerate(plan, 2)
    r0 = tn.tn_exec_prepare([plan], [terms], tn.exec_opts(use_graph=False, group=False)).run()[0]
    ext = tn.tn_exec_prepare([plan], [terms], tn.exec_opts(use_graph=True, tune=True, group=False))
    r1 = ext.run()[0]
    gold = np.loadtxt(os.path.join(GOLD, "config2_oracle.txt"))
    for u in range(3):
        assert abs(r1["A"][u] - gold[u]) <= 1e-6 * gold[u]
        assert abs(r1["A"][u] - r0["A"][u]) <= 1e-9 * gold[u]
    kernels = {L.get("kernel") for L in ext.describe()["launches"] if L["kind"] == 1}
    assert any(k and k.startswith("k_gemm_mfma") for k in kernels)


@pytest.mark.parametrize("cfg", [2, 3])
def test_schedule_variants_agree(torch, cfg):
    """Level-grouped launches, per-step launches with operands gathered in
    stored order, and per-step launches with transposes compute the same
    terms (FP32 rounding apart) and the same level sums."""
    print(f"schedule variants config{cfg}", flush=True)
    c = W.config(cfg)
    plan = tn.tn_plan_build(c, c.level)
    terms = tn.tn_terms_enumerate(plan, c.level)
    out = []
    for kw in (dict(), dict(group=False), dict(group=False, gather=False)):
        ex = tn.tn_exec_prepare([plan], [terms], tn.exec_opts(use_graph=False, **kw))
        r = ex.run()[0]
        x, _ = ex.values()
        out.append((r, x))
    gold = np.loadtxt(os.path.join(GOLD, f"config{cfg}_oracle.txt"))
    r0, x0 = out[0]
    for r, x in out:
        for u in range(c.level + 1):
            assert abs(r["A"][u] - gold[u]) <= 1e-6 * gold[u]
        # every term: same value within FP32 rounding of the larger terms
        scale = np.maximum(x, x0)
        assert np.all(np.abs(x - x0) <= 1e-4 * scale + 1e-6 * x0.max() * 1e-6)


def _deposit_np(count, pos):
    x = np.arange(count, dtype=np.int64)
    o = np.zeros(count, dtype=np.int64)
    for j, p in enumerate(pos):
        o |= ((x >> j) & 1) << p
    return o


def _random_mfma_job(torch, rng, m_log, n_log, k_log, n_slices, share, merge, tile, ksplit):
    """A job whose operands sit in random stored bit orders; slices share the
    merged operand in groups of `share`; tiles cut as the planner does."""
    m, n, k = 1 << m_log, 1 << n_log, 1 << k_log
    pa = list(rng.permutation(m_log + k_log))
    pb = list(rng.permutation(k_log + n_log))
    a_row, a_k = [int(v) for v in pa[:m_log]], [int(v) for v in pa[m_log:]]
    b_k, b_col = [int(v) for v in pb[:k_log]], [int(v) for v in pb[k_log:]]
    sa, sb = m * k, k * n
    if merge == 1:
        ka = np.arange(n_slices) // share
        kb = np.arange(n_slices)
    elif merge == 2:
        ka = np.arange(n_slices)
        kb = np.arange(n_slices) // share
    else:
        ka = kb = np.arange(n_slices)
    na, nb = int(ka.max()) + 1, int(kb.max()) + 1
    A = (rng.standard_normal(na * sa) + 1j * rng.standard_normal(na * sa)).astype(np.complex64)
    B = (rng.standard_normal(nb * sb) + 1j * rng.standard_normal(nb * sb)).astype(np.complex64)
    oa, ob = ka * sa, kb * sb
    oc = np.arange(n_slices) * m * n
    ref = np.empty((n_slices, m, n), np.complex128)
    ar, ak, bk, bc = (_deposit_np(m, a_row), _deposit_np(k, a_k), _deposit_np(k, b_k), _deposit_np(n, b_col))
    for s in range(n_slices):
        As = A[oa[s] + ar[:, None] + ak[None, :]].astype(np.complex128)
        Bs = B[ob[s] + bk[:, None] + bc[None, :]].astype(np.complex128)
        ref[s] = As @ Bs
    bm, bn = tn.MFMA_TILE_SHAPES[tile]
    tiles = []
    if merge == 0:
        for s in range(n_slices):
            for r in range(max(1, m // bm)):
                for c in range(max(1, n // bn)):
                    tiles.append((0, 1, s, r * bm, c * bn, 0, 0))
    else:
        segs = (bn // n) if merge == 1 else (bm // m)
        for g0 in range(0, n_slices, share):
            g1 = min(n_slices, g0 + share)
            for p0 in range(g0, g1, segs):
                cnt = min(segs, g1 - p0)
                if merge == 1:
                    for r in range(max(1, m // bm)):
                        tiles.append((0, cnt, p0, r * bm, 0, 0, 0))
                else:
                    for c in range(max(1, n // bn)):
                        tiles.append((0, cnt, p0, 0, c * bn, 0, 0))
    job = dict(A=torch.from_numpy(A).cuda(), B=torch.from_numpy(B).cuda(),
               C=torch.zeros(n_slices * m * n, dtype=torch.complex64, device="cuda"),
               oa=torch.from_numpy(oa.astype(np.int64)).cuda(), ob=torch.from_numpy(ob.astype(np.int64)).cuda(),
               oc=torch.from_numpy(oc.astype(np.int64)).cuda(), m_log=m_log, n_log=n_log, k_log=k_log,
               merge=merge, a_rowfast=int(a_row[0] == 0) if m_log else 0,
               b_colfast=int(b_col[0] == 0) if n_log else 0, a_row=a_row, a_k=a_k, b_k=b_k, b_col=b_col)
    if ksplit > 1:
        # S tiles in a row per output tile, one per part of the inner chunks
        assert k_log >= 3 and ((1 << k_log) // 8) % ksplit == 0
        parts = []
        for q, t in enumerate(tiles):
            parts += [t[:5] + (h, q) for h in range(ksplit)]
        job.update(ksplit=ksplit,
                   partial=torch.empty(len(parts) * bm * bn * 2, dtype=torch.float32, device="cuda"))
        tiles = parts
    return job, np.array(tiles, dtype=tn.MFMA_TILE), ref


@pytest.mark.parametrize("m_log,n_log,k_log,n_slices,share,merge,tile,ksplit", [
    (8, 6, 5, 3, 1, 0, 0, 1),       # plain slices, 128 x 64 tiles
    (7, 4, 6, 9, 3, 1, 0, 1),       # columns hold 4 slices sharing A (ragged groups of 3)
    (3, 5, 4, 10, 4, 2, 2, 1),      # rows hold 16 slices sharing B, 128 x 32 tiles
    (6, 3, 2, 5, 5, 1, 6, 1),       # k < 8 (padded inner chunk), n < 16
    (8, 4, 8, 12, 3, 1, 0, 2),      # split inner sum over tile pairs
    (5, 5, 7, 4, 1, 0, 4, 2),       # split, 32 x 32 tiles
    (8, 4, 8, 12, 3, 1, 0, 8),      # split over 8 tiles (4 chunks each)
    (5, 5, 9, 2, 1, 0, 4, 16),      # split over 16 tiles, 32 x 32
    (5, 5, 10, 2, 1, 0, 4, 128),    # more parts than tile rows: element ranges, FP64 tree
    (3, 5, 7, 10, 4, 2, 2, 4),      # merged rows, split over 4 tiles
])
def test_grouped_mfma_kernel_against_numpy(torch, m_log, n_log, k_log, n_slices, share, merge, tile, ksplit):
    """tn_kernel_mfma_group on operands in random stored bit orders, against a
    complex128 numpy product of the gathered slices; FP32 accumulation over k
    products of O(1) numbers bounds the error by ~k u32 of the row norms."""
    print(f"mfma group {m_log} {n_log} {k_log} x{n_slices} merge {merge} tile {tile} split {ksplit}", flush=True)
    rng = np.random.default_rng(1000 + m_log * 100 + k_log * 10 + merge)
    job, tiles, ref = _random_mfma_job(torch, rng, m_log, n_log, k_log, n_slices, share, merge, tile, ksplit)
    d = tn.mfma_group_descriptors([job], tiles)
    first = None
    for rep in range(2):     # the second launch reuses the partial buffer
        job["C"].zero_()
        tn.kernel_mfma_group(tile, d)
        if ksplit > 1:
            tn.kernel_mfma_split_reduce(tile, d)
        torch.cuda.synchronize()
        got = job["C"].cpu().numpy().reshape(ref.shape)
        err = np.abs(got - ref).max()
        scale = np.sqrt(2.0 * (1 << k_log)) * 2.0
        assert err <= 4e-6 * scale * max(1.0, np.sqrt(1 << k_log) / 4), (rep, err)
        if first is None:
            first = got.copy()
        else:           # parts are added in a fixed order: the same bits every launch
            assert np.array_equal(first.view(np.float32), got.view(np.float32))


def test_degenerate_cases_against_oracle(torch):
    """Edge cases of the method: no noise (one term, the noiseless value),
    level 0 (only the all-dominant term), every level-2 candidate pruned
    (levels 0-1 contracted, the level-2 sum equals the level-1 sum), and a
    level above the noise count (clamped, every term, the exact value)."""
    from oracle import dense
    print("degenerate cases", flush=True)
    # no noise
    c0 = W.tiny_random_circuit(np.random.default_rng(3), 5, 20, 0, noise="adpd", level=0)
    res, x, pat, _ = run_gpu(c0, 0)
    assert res["n_terms"] == 1
    assert abs(res["A"][0] - dense.exact_value(c0)) <= 1e-12
    # level 0 of C1
    c1 = W.config(1, level=2)
    res, x, pat, _ = run_gpu(c1, 0)
    r = estimate.estimate(c1, 0, "network")
    assert res["n_terms"] == 1 and abs(res["A"][0] - r["A"][0]) <= 1e-12 * r["A"][0]
    # all level-2 candidates pruned
    plan = tn.tn_plan_build(c1, 2)
    full = tn.tn_terms_enumerate(plan, 2)
    pat, w = full.get()
    ncand = int(((pat != 0).sum(axis=1) >= 2).sum())
    tp = tn.tn_terms_enumerate(plan, 2, keep=np.zeros(ncand, np.uint8), min_level=2)
    ex = tn.tn_exec_prepare([plan], [tp], tn.exec_opts(use_graph=True))
    rp = ex.run()[0]
    r2 = estimate.estimate(c1, 2, "network")
    assert abs(rp["A"][1] - r2["A"][1]) <= 1e-6 * r2["A"][1]
    assert rp["A"][2] == rp["A"][1]
    # level above the noise count: clamped to the full expansion = exact value
    c3 = W.tiny_random_circuit(np.random.default_rng(8), 4, 14, 2, noise="random", level=5)
    res, x, pat, _ = run_gpu(c3, 5)
    assert res["clamped"] and res["level"] == 2
    assert abs(res["A"][2] - dense.exact_value(c3)) <= 1e-6 * abs(dense.exact_value(c3)) + 1e-12


# ---------------------------------------------------------------------------
# exact value: the doubled network (every noise as its whole superoperator),
# one term computed in FP64 (the dominant-term pass) or in FP32
# ---------------------------------------------------------------------------
def run_doubled(circ, fp64=True, **plan_kw):
    plan = tn.tn_plan_build_doubled(circ, **plan_kw)
    terms = tn.tn_terms_enumerate(plan, 0)
    ex = tn.tn_exec_prepare([plan], [terms], tn.exec_opts(use_graph=False, fp64_level0=fp64))
    res = ex.run()[0]
    return res, plan


@pytest.mark.parametrize("seed,kind,target,n,gates,noise", [
    (61, "random", "circuit_output", 5, 30, 6), (62, "adpd", "product", 4, 24, 5),
    (63, "depol", "dense", 5, 30, 4), (64, "random", "product", 6, 40, 7)])
def test_doubled_tiny_circuits_against_density_matrix(torch, seed, kind, target, n, gates, noise):
    from oracle import dense
    print(f"doubled tiny {seed} {kind} {target}", flush=True)
    c = W.tiny_random_circuit(np.random.default_rng(seed), n, gates, noise, noise=kind, level=2,
                              target=target)
    f = dense.exact_value(c)
    res, _ = run_doubled(c)
    assert res["n_terms"] == 1 and res["bound"] == 0.0
    assert abs(res["A"][0] - f) <= 1e-12 * max(1.0, abs(f)), (res["A"][0], f)
    # FP32 chain only: about 1e-7 relative per step, a few dozen steps
    res32, _ = run_doubled(c, fp64=False)
    assert abs(res32["A"][0] - f) <= 1e-5 * max(1.0, abs(f)), (res32["A"][0], f)


def test_doubled_wide_circuit_against_oracle(torch):
    """16 qubits, 160 gates: the doubled network's steps reach the grouped
    matrix-core and FP64 tile launches; the oracle's own doubled contraction
    and its full expansion at level N pin the value."""
    from oracle import doubled
    print("doubled wide", flush=True)
    c = W.tiny_random_circuit(np.random.default_rng(65), 16, 160, 4, noise="adpd", level=4,
                              target="circuit_output")
    want = doubled.doubled_value(c, diagonal=True).real
    res, plan = run_doubled(c)
    assert plan.info()["max_log_size"] >= 14
    assert abs(res["A"][0] - want) <= 1e-12 * want, (res["A"][0], want)
    ref = estimate.estimate(c, 4, "network")
    assert abs(res["A"][0] - ref["A"][-1]) <= 1e-12 * want


@pytest.mark.parametrize("cfg", [1, 5])
def test_doubled_configs_against_oracle(torch, cfg):
    """Config 1 (8 qubits) and config 5 (15x15 grid, 20 AD+PD): the exact value
    against the oracle's doubled contraction, and the level-l estimate's
    remainder F - A(l) within Theorem 1's bound."""
    from oracle import bounds, doubled
    print(f"doubled config{cfg}", flush=True)
    c = W.config(cfg)
    want = doubled.doubled_value(c, diagonal=True).real
    res, _ = run_doubled(c)
    f = res["A"][0]
    assert abs(f - want) <= 1e-12 * want, (f, want)
    est, _, _, _ = run_gpu(c, c.level)
    b = bounds.rigorous_bound([bounds.split_norms(op.kraus) for op in c.noise_ops()], c.level)
    assert est["A"][c.level] - 1e-9 <= f <= est["A"][c.level] + b + 1e-12, (f, est["A"], b)


def test_doubled_config2_brackets_the_estimate(torch):
    """Config 2 (5x5 grid, 12 layers, 25 qubits: no density matrix): the exact
    value lies between the oracle's full level-2 sum and that sum plus Theorem
    1's bound; a second contraction order (another path seed) agrees."""
    from oracle import bounds
    print("doubled config2", flush=True)
    c = W.config(2)
    gold = np.loadtxt(os.path.join(GOLD, "config2_oracle.txt"))
    b = bounds.rigorous_bound([bounds.split_norms(op.kraus) for op in c.noise_ops()], c.level)
    res, plan = run_doubled(c, path_trials=16384)
    f = res["A"][0]
    print(f"F {f:.17g} A(2) {gold[-1]:.17g} F-A(2) {f - gold[-1]:.3e} bound {b:.3e} "
          f"max_log {plan.info()['max_log_size']}", flush=True)
    assert gold[-1] - 1e-12 <= f <= gold[-1] + b + 1e-12
    res2, plan2 = run_doubled(c, path_trials=16384, seed=7)
    assert abs(res2["A"][0] - f) <= 1e-12 * f, (res2["A"][0], f)


# ---------------------------------------------------------------------------
# off-diagonal elements <x| E |y>: four bond-2 targets packed in one schedule,
# combined by the polarization identity
# ---------------------------------------------------------------------------
def _rand_product(rng, n):
    z = rng.standard_normal((n, 2)) + 1j * rng.standard_normal((n, 2))
    return z / np.linalg.norm(z, axis=1, keepdims=True)


def _basis(n, bits):
    out = np.zeros((n, 2), dtype=np.complex128)
    for q in range(n):
        out[q, bits[q]] = 1.0
    return out


def _offdiag_tol(parts, u):
    # each of the four values is its FP64 all-dominant term (1e-12) plus FP32
    # corrections (about 1e-6 of their own size; 1e-5 allowed); the element
    # itself can be far smaller than the four values
    corr = max(abs(p["A"][u] - p["A"][0]) for p in parts)
    return 1e-5 * corr + 1e-12 * max(abs(p["A"][0]) for p in parts) + 1e-15


@pytest.mark.parametrize("seed,kind,output,n", [(91, "random", True, 5), (92, "adpd", False, 4),
                                                (93, "depol", True, 6)])
def test_offdiagonal_tiny_circuits_against_oracle(torch, seed, kind, output, n):
    from oracle import offdiag
    print(f"offdiag tiny {seed} {kind} {output}", flush=True)
    rng = np.random.default_rng(seed)
    c = W.tiny_random_circuit(rng, n, 8 * n, 4, noise=kind, level=3,
                              target="circuit_output" if output else "product")
    x, y = _rand_product(rng, n), _rand_product(rng, n)
    got, parts, _ = tn.offdiagonal(c, x, y, 3, output)
    ref = offdiag.element_cross(c, 3, x, y, output)["A"]
    for u in range(4):
        assert abs(got[u] - ref[u]) <= _offdiag_tol(parts, u), (u, got[u], ref[u])
    assert abs(got[0] - ref[0]) <= 1e-12 * max(abs(p["A"][0]) for p in parts)   # FP64 dominant terms
    ex, _, _ = tn.offdiagonal(c, x, y, output=output, exact=True)
    assert abs(ex[0] - offdiag.element_exact(c, x, y, output)) <= 1e-12


def test_offdiagonal_config1_against_density_matrix(torch):
    from oracle import offdiag
    print("offdiag config1", flush=True)
    c = W.config(1, level=4)
    n = c.n_qubits
    x, y = _basis(n, [0] * n), _basis(n, [0] * (n - 1) + [1])
    got, parts, _ = tn.offdiagonal(c, x, y, 4, True)
    ref = offdiag.element_cross(c, 4, x, y, True)["A"]
    for u in range(5):
        assert abs(got[u] - ref[u]) <= _offdiag_tol(parts, u), (u, got[u], ref[u])
    f = offdiag.element_exact(c, x, y, True)
    assert abs(got[4] - f) <= _offdiag_tol(parts, 4)
    ex, _, _ = tn.offdiagonal(c, x, y, output=True, exact=True)
    assert abs(ex[0] - f) <= 1e-12


def test_offdiagonal_config2_against_oracle(torch):
    """25 qubits (no density matrix): <0..0|E|0..01> on the circuit's outputs
    at level 2 against the oracle's cross form (every term, two networks
    each), and <y|E|x> = conj(<x|E|y>) from four other targets."""
    from oracle import offdiag
    print("offdiag config2", flush=True)
    c = W.config(2)
    n = c.n_qubits
    x, y = _basis(n, [0] * n), _basis(n, [0] * (n - 1) + [1])
    got, parts, _ = tn.offdiagonal(c, x, y, c.level, True)
    ref = offdiag.element_cross(c, c.level, x, y, True, diagonal=True)["A"]
    for u in range(c.level + 1):
        assert abs(got[u] - ref[u]) <= _offdiag_tol(parts, u), (u, got[u], ref[u])
    back, parts2, _ = tn.offdiagonal(c, y, x, c.level, True)
    for u in range(c.level + 1):
        assert abs(back[u] - np.conj(got[u])) <= _offdiag_tol(parts, u) + _offdiag_tol(parts2, u)


# ---------------------------------------------------------------------------
# exact cross-term reuse: factored term sets over independent clusters
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed,kind", [(121, "random"), (122, "adpd"), (123, "depol")])
def test_factored_two_block_circuits_against_oracle(torch, seed, kind):
    from tests.test_oracle_factored import two_blocks
    print(f"factored two blocks {seed} {kind}", flush=True)
    c = two_blocks(seed, kind=kind)
    A, _ = tn.FactoredEstimate(c, 4).run()
    r = estimate.estimate(c, 4, "network")
    ref = r["A"]
    assert abs(A[0] - ref[0]) <= 1e-12 * ref[0]
    # each level's sum T_u = A(u) - A(u-1) within 2e-5 T_u plus the summed FP32
    # bounds of its terms (and the FP64 rounding of the differences)
    pat = np.array(r["terms"])
    tol = pc.term_tols(network.slot_split(c), pat, r["X"])
    lv = (pat != 0).sum(axis=1)
    for u in range(1, 5):
        got, want = A[u] - A[u - 1], ref[u] - ref[u - 1]
        bound = 2e-5 * abs(r["T"][u]) + tol[lv == u].sum() + 4e-16 * ref[u]
        assert abs(got - want) <= bound, (u, got, want, bound)
    for u in range(5):   # and the 1e-6 bar of the level sums
        assert abs(A[u] - ref[u]) <= 1e-6 * ref[u], (u, A[u], ref[u])


def test_factored_config5_against_oracle(torch):
    """225 qubits, 20 noises in 9 independent clusters: level 3 from 2815
    factored terms against the stored sums of all 32551; level 5 (4.19M terms
    in the full expansion, 43720 factored) against the oracle's per-part polynomials; the
    levels rise toward the exact value (doubled network)."""
    from oracle import factored
    print("factored config5", flush=True)
    c = W.config(5)
    fe3 = tn.FactoredEstimate(c, 3)
    assert fe3.terms.n == 2815
    A3, _ = fe3.run()
    gold = np.loadtxt(os.path.join(GOLD, "config5_oracle.txt"))
    for u in range(4):
        assert abs(A3[u] - gold[u]) <= 1e-8 * gold[u], (u, A3[u], gold[u])
    A5, _ = tn.FactoredEstimate(c, 5).run()
    ref = factored.factored_levels(c, 5)["A"]
    for u in range(6):
        assert abs(A5[u] - ref[u]) <= 1e-8 * ref[u], (u, A5[u], ref[u])
    f, _ = run_doubled(c)
    assert all(A5[u] <= A5[u + 1] + 1e-15 for u in range(5)) and A5[5] <= f["A"][0] + 1e-12


# ---------------------------------------------------------------------------
# quantum trajectories on the same engine
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed,kind,target", [(151, "random", "circuit_output"), (152, "adpd", "product"),
                                               (153, "depol", "dense")])
def test_trajectories_tiny_circuits_against_oracle(torch, seed, kind, target):
    from oracle import dense, trajectories
    print(f"trajectories tiny {seed} {kind}", flush=True)
    c = W.tiny_random_circuit(np.random.default_rng(seed), 5, 30, 5, noise=kind, level=1, target=target,
                              scale=5.0)
    u = W.trajectory_uniforms(2000, c.n_noises, seed)
    mean, x, _ = tn.trajectories_estimate(c, u)
    ref = trajectories.estimate(c, u)
    assert np.allclose(x, ref["X"], rtol=2e-5, atol=1e-9)
    assert abs(mean - ref["mean"]) <= 2e-6 * ref["mean"]
    assert abs(mean - dense.exact_value(c)) <= 5 * ref["stderr"]


def test_trajectories_config2_against_oracle(torch):
    """25 qubits: 4096 draws of the 10 depolarizing noises; 64 sampled scores
    against the oracle one by one; the mean within five standard errors of
    the exact value (the oracle's full level-2 sum, 2.6e-11 below it)."""
    from oracle import trajectories
    print("trajectories config2", flush=True)
    c = W.config(2)
    u = W.trajectory_uniforms(4096, c.n_noises, 2211)
    mean, x, _ = tn.trajectories_estimate(c, u)
    net = network.KetNetwork(c, diagonal=True)
    idx = trajectories.sample_indices(c, u)
    for i in np.random.default_rng(5).choice(4096, 64, replace=False):
        ref = trajectories.sample_value(net, c, idx[i])
        assert abs(x[i] - ref) <= 2e-5 * ref + 1e-9, (i, x[i], ref)
    gold = np.loadtxt(os.path.join(GOLD, "config2_oracle.txt"))
    se = x.std(ddof=1) / np.sqrt(len(x))
    print(f"mean {mean:.9f} exact {gold[-1]:.9f} stderr {se:.2e}", flush=True)
    assert abs(mean - gold[-1]) <= 5 * se + 1e-10


def test_pipelined_estimates_equal_sequential_runs(torch):
    """Two estimates in flight (submit / collect) give the same bits as
    tn_exec_run, every time; a third submit, an out-of-order collect and a
    run with estimates outstanding are refused."""
    print("pipelined estimates", flush=True)
    c = W.config(2)
    plan = tn.tn_plan_build(c, c.level)
    terms = tn.tn_terms_enumerate(plan, c.level)
    for graph in (False, True):
        ex = tn.tn_exec_prepare([plan], [terms], tn.exec_opts(use_graph=graph))
        ref = ex.run()[0]
        prev = ex.submit()
        for _ in range(6):
            t = ex.submit()
            assert ex.collect(prev)[0]["A"] == ref["A"]
            prev = t
        t2 = ex.submit()
        other = torch.cuda.Stream()
        with pytest.raises(tn.TNError):
            ex.submit(other)                  # outstanding estimates on another stream
        with pytest.raises(tn.TNError):
            ex.submit()                       # a third outstanding estimate
        with pytest.raises(tn.TNError):
            ex.collect(t2)                    # out of order
        with pytest.raises(tn.TNError):
            ex.run()                          # estimates outstanding
        assert ex.collect(prev)[0]["A"] == ref["A"]
        assert ex.collect(t2)[0]["A"] == ref["A"]
        assert ex.run()[0]["A"] == ref["A"]


def test_run_many_equals_sequential_runs(torch):
    """tn_exec_run_many (several estimates in one call, two in flight) gives
    the same bits as tn_exec_run for every estimate, on the caller's stream and
    on another; zero estimates is a no-op; it is refused while a submitted
    estimate is outstanding, and with per-launch timing; tn_exec_timing's
    per-kind breakdown is recorded with per-launch timing and -1 without."""
    print("run_many", flush=True)
    for cfg in (5, 2):
        c = W.config(cfg)
        plan = tn.tn_plan_build(c, c.level)
        terms = tn.tn_terms_enumerate(plan, c.level)
        for graph in (False, True):
            ex = tn.tn_exec_prepare([plan], [terms], tn.exec_opts(use_graph=graph))
            ref = ex.run()[0]
            for count in (1, 2, 7):
                rs = ex.run_many(count)
                assert len(rs) == count and all(r[0]["A"] == ref["A"] and r[0]["T"] == ref["T"] for r in rs)
            other = torch.cuda.Stream()
            assert all(r[0]["A"] == ref["A"] for r in ex.run_many(5, other))
            assert ex.run_many(0) == []
            t = ex.submit()
            with pytest.raises(tn.TNError):
                ex.run_many(2)                    # a submitted estimate is outstanding
            assert ex.collect(t)[0]["A"] == ref["A"]
            assert ex.run()[0]["A"] == ref["A"]
    tk = tn.tn_exec_prepare([plan], [terms], tn.exec_opts(time_kernels=True))
    with pytest.raises(tn.TNError):
        tk.run_many(2)
    # timing breakdown: per-launch sums with per-launch timing, -1 without
    a_tk = tk.run()[0]["A"]
    assert all(abs(x - y) <= 1e-12 * abs(y) for x, y in zip(a_tk, ref["A"]))
    total, contraction, permute, other = tk.timing()
    assert total > 0 and contraction > 0 and permute >= 0 and other >= 0
    assert contraction + permute + other <= 2 * total    # two streams at most overlap
    ex.run()
    total, contraction, permute, other = ex.timing()
    assert total > 0 and contraction == permute == other == -1
