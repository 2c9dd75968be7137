"""End-to-end pins of the oracle's Algorithm 1.

What fixes the answer independently of the oracle's own arithmetic:
* no noise: the value is |<v|U|psi>|^2 (Problem 1; = 1 when v = U psi);
* the full expansion (l = N) equals the exact density-matrix value (Section
  IV: A(N) is exact), and a sum over all 4^N patterns equals it too;
* the enumerated level sums equal an enumeration-free graded recursion;
* the literal two-network evaluation equals the one-network form;
* trace preservation: summing the value over all computational-basis targets
  gives 1;
* every term is >= 0, so A(l) increases with l and stays <= F;
* Theorem 1's remainder bound, in the form its proof establishes;
* the level-l error scales as p^(l+1) when the noise parameters shrink;
* light-cone reduction does not change a term.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import bounds, channels, dense, estimate, literal, network, terms


def tiny(seed, n=3, gates=10, noise=3, kind="random", target="circuit_output", level=1, scale=1.0):
    rng = np.random.default_rng(seed)
    return W.tiny_random_circuit(rng, n, gates, noise, noise=kind, level=level, target=target,
                                 scale=scale)


def noiseless_value(circ):
    st = dense.ideal_state(circ, dense.product_state(circ.psi))
    v = dense.target_vector(circ)
    return abs(np.vdot(v, st)) ** 2


@pytest.mark.parametrize("target", ["circuit_output", "product", "dense"])
def test_no_noise_gives_squared_overlap(target):
    c = tiny(10, n=4, gates=14, noise=0, target=target)
    want = noiseless_value(c)
    assert math.isclose(dense.exact_value(c), want, rel_tol=1e-12)
    for method in ("literal", "network"):
        r = estimate.estimate(c, 0, method)
        assert math.isclose(r["A"][0], want, rel_tol=1e-12)


def test_no_noise_circuit_output_target_is_one():
    c = W.config(1)
    c = W.Circuit(c.n_qubits, [o for o in c.ops if o.kind == "gate"], c.psi, c.target, c.v, 0)
    assert math.isclose(dense.exact_value(c), 1.0, rel_tol=1e-12)
    r = estimate.estimate(c, 0, "network")
    assert math.isclose(r["A"][0], 1.0, rel_tol=1e-12)


@pytest.mark.parametrize("seed,kind,target", [(11, "random", "circuit_output"), (12, "adpd", "product"),
                                               (13, "depol", "dense"), (14, "random", "product"),
                                               (15, "random", "dense")])
def test_full_expansion_equals_exact_value(seed, kind, target):
    c = tiny(seed, n=3, gates=12, noise=4, kind=kind, target=target)
    f = dense.exact_value(c)
    for method in ("literal", "network"):
        r = estimate.estimate(c, 4, method)
        assert abs(r["A"][-1] - f) <= 1e-12 * max(1.0, abs(f))


def test_all_patterns_sum_to_exact_value():
    c = tiny(16, n=3, gates=9, noise=3, kind="random")
    sp = literal.splits(c)
    import itertools
    tot = 0.0
    for p in itertools.product(range(4), repeat=3):
        tot += literal.term_value(c, p, sp)[0]
    assert abs(tot - dense.exact_value(c)) < 1e-12


@pytest.mark.parametrize("seed,kind", [(20, "random"), (21, "adpd"), (22, "depol")])
def test_graded_recursion_equals_enumerated_level_sums(seed, kind):
    c = tiny(seed, n=4, gates=14, noise=5, kind=kind)
    g = dense.graded_levels(c, 3)
    r = estimate.estimate(c, 3, "network")
    for u in range(4):
        assert abs(g[u].imag) < 1e-14
        assert abs(g[u].real - r["T"][u]) < 1e-13


def test_literal_equals_single_network_per_term():
    for seed, kind in ((30, "random"), (31, "adpd"), (32, "depol")):
        c = tiny(seed, n=4, gates=14, noise=4, kind=kind)
        sp = literal.splits(c)
        net = network.KetNetwork(c)
        ns = network.slot_split(c)
        for t in terms.enumerate_terms(4, 4):
            x_lit, a, b = literal.term_value(c, t, sp)
            x_net, _ = network.term_value(net, ns, t)
            assert abs(x_lit.imag) <= 1e-12 * max(abs(x_lit), 1e-300) + 1e-17
            assert x_lit.real >= -1e-15
            assert abs(x_lit.real - x_net) <= 1e-13 * max(1.0, abs(x_net))


def test_trace_preservation_over_basis_targets():
    c = tiny(40, n=3, gates=10, noise=3, kind="random", target="dense")
    tot = 0.0
    for x in range(8):
        v = np.zeros(8, dtype=np.complex128)
        v[x] = 1
        cx = W.Circuit(c.n_qubits, c.ops, c.psi, "dense", v, 3)
        tot += dense.exact_value(cx)
    assert abs(tot - 1.0) < 1e-13


def test_terms_nonnegative_and_levels_monotone_below_exact():
    for seed, kind in ((50, "random"), (51, "adpd"), (52, "depol")):
        c = tiny(seed, n=4, gates=16, noise=5, kind=kind)
        f = dense.exact_value(c)
        r = estimate.estimate(c, 5, "network")
        assert np.all(r["X"] >= 0.0)
        a = r["A"]
        assert all(a[i + 1] >= a[i] - 1e-15 for i in range(len(a) - 1))
        assert all(x <= f + 1e-13 for x in a)


def test_config1_levels_against_exact_density_matrix():
    c = W.config(1, level=4)
    f = dense.exact_value(c)
    g = dense.graded_levels(c, 4)
    r = estimate.estimate(c, 4, "network")
    assert len(r["terms"]) == 256
    assert abs(r["A"][4] - f) < 1e-14
    for u in range(5):
        assert abs(g[u].real - r["T"][u]) < 1e-14
    # levels 1 and 2 on the way
    assert r["A"][1] < r["A"][2] < f


def test_theorem1_rigorous_bound_holds():
    for seed, kind, sc in ((60, "random", 1.0), (61, "adpd", 1.0), (62, "depol", 1.0), (63, "depol", 0.1)):
        c = tiny(seed, n=3, gates=12, noise=5, kind=kind, scale=sc)
        f = dense.exact_value(c)
        r = estimate.estimate(c, 5, "network")
        norms = [bounds.split_norms(o.kraus) for o in c.noise_ops()]
        for l in range(5):
            assert abs(f - r["A"][l]) <= bounds.rigorous_bound(norms, l) * (1 + 1e-12) + 1e-15


def test_theorem1_printed_bound_in_small_noise_regime():
    # With every noise rate below p, the printed bound of Theorem 1 should hold
    # for small depolarizing noise (checked, not relied upon).
    c = tiny(70, n=3, gates=12, noise=5, kind="depol", scale=0.2)
    f = dense.exact_value(c)
    r = estimate.estimate(c, 5, "network")
    p = max(channels.noise_rate(channels.superoperator(o.kraus)) for o in c.noise_ops())
    for l in range(3):
        assert abs(f - r["A"][l]) <= bounds.paper_bound(5, l, p)


def test_error_scales_as_p_to_level_plus_one():
    errs = {}
    for sc in (1.0, 0.1):
        c = tiny(80, n=3, gates=12, noise=4, kind="depol", scale=sc)
        f = dense.exact_value(c)
        r = estimate.estimate(c, 2, "network")
        errs[sc] = [abs(f - r["A"][l]) for l in range(3)]
    for l in range(3):
        ratio = errs[1.0][l] / errs[0.1][l]
        want = 10.0 ** (l + 1)
        assert want / 3 < ratio < want * 3, (l, ratio)


def test_light_cone_reduction_does_not_change_terms():
    c = tiny(90, n=5, gates=30, noise=3, kind="random")
    full = network.KetNetwork(c, reduce=False)
    red = network.KetNetwork(c, reduce=True)
    assert len(red.tensors) < len(full.tensors)
    sp = network.slot_split(c)
    for t in terms.enumerate_terms(3, 3):
        x1, _ = network.term_value(full, sp, t)
        x2, _ = network.term_value(red, sp, t)
        assert abs(x1 - x2) <= 1e-13 * max(1.0, x1)


def test_table4_structure_matches_nonnegative_terms():
    # Table IV's levels 0..2 rise and agree on one exact value (result + error)
    # to the printed precision; level 3 is printed above that value, which
    # nonnegative terms rule out, so only levels 0..2 are used.
    import os
    rows = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "table4_levels.txt"))
    res, err = rows[:3, 2], rows[:3, 3]
    assert np.all(np.diff(res) > 0)
    implied = res + err
    # printed precision: 7 decimals on results, 3 significant digits on errors
    assert abs(implied[0] - implied[2]) < 1e-5       # 4.59e-3 is known to +-5e-6
    assert abs(implied[1] - implied[2]) < 2e-7
    assert rows[3, 2] > implied[2] + 1e-6


def test_diagonal_gates_as_shared_indices_give_the_same_terms():
    # QAOA-like circuit (H, RZZ, RX) and a grid circuit with CZ: the
    # shared-index form of diagonal gates must reproduce every term
    rng = np.random.default_rng(91)
    gates = [W.Op("gate", (q,), W.gate_h()) for q in range(5)]
    for (a, b) in [(0, 1), (1, 2), (2, 3), (3, 4), (0, 4), (1, 3)]:
        gates.append(W.Op("gate", (a, b), W.gate_rzz(0.7)))
    gates += [W.Op("gate", (q,), W.gate_rx(0.3)) for q in range(5)]
    gates += [W.Op("gate", (q,), W.gate_rz(0.4 * q)) for q in range(5)]
    kr = [W.kraus_ad_pd(0.01, 0.02), W.kraus_depolarizing(0.01), W.random_isometry_kraus(rng, 3)]
    ops = W.circuits.place_noises(gates, kr, rng)
    z = W.circuits.zero_product(5)
    circs = [W.Circuit(5, ops, z, "circuit_output", z, 3),
             W.tiny_random_circuit(np.random.default_rng(92), 5, 30, 3, noise="adpd", level=3,
                                   target="product")]
    for c in circs:
        a = network.KetNetwork(c)
        b = network.KetNetwork(c, diagonal=True)
        sp = network.slot_split(c)
        for t in terms.enumerate_terms(3, 3):
            x1, _ = network.term_value(a, sp, t)
            x2, _ = network.term_value(b, sp, t)
            assert abs(x1 - x2) <= 1e-13 * max(1.0, x1)
