"""Circuit and noise generators for the synthetic workloads.

Conventions (shared by every consumer):

* A circuit acts on ``n`` qubits.  A pure n-qubit state is a length-2^n
  vector whose index has qubit 0 as the MOST significant bit.
* A 1-qubit gate is a 2x2 matrix; a 2-qubit gate on qubits (q0, q1) is a 4x4
  matrix in the basis |b_q0 b_q1> with b_q0 the more significant bit.
* A noise is a single-qubit channel given by its Kraus matrices (2x2 each).
  It acts right after the op that precedes it in ``Circuit.ops``.
* ``psi`` is a product input state given as an (n, 2) array of per-qubit
  amplitudes.  The target is one of
    - ``"circuit_output"``: |v> = U_ideal |psi_v> with ``v`` an (n, 2)
      product state (U_ideal = the circuit with every noise removed);
    - ``"product"``: |v> given as an (n, 2) product state;
    - ``"dense"``: |v> given as a length-2^n vector.

Gate definitions follow the paper's Table I (H, X, Y, Z, T, Rx, Ry, Rz) and
its CZ.  RZZ(g) = exp(-i g Z(x)Z / 2), in the same sign convention as Rz.
Depolarizing uses the paper's Kraus set {sqrt(1-p) I, sqrt(p/3) X, Y, Z}
(Section II).  Amplitude damping and phase damping use the textbook Kraus
sets; their composition stands in for the paper's realistic decoherence model,
whose parameters the paper does not print.

Random draws: NumPy PCG64.  Config c uses seed 2211170280 + c.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

CONFIG_SEED_BASE = 2211170280


@dataclasses.dataclass
class Op:
    kind: str                      # "gate" or "noise"
    qubits: tuple                  # (q,) or (q0, q1)
    mat: Optional[np.ndarray] = None          # gate matrix, complex128
    kraus: Optional[List[np.ndarray]] = None  # noise Kraus matrices, 2x2 complex128
    label: str = ""


@dataclasses.dataclass
class Circuit:
    n_qubits: int
    ops: List[Op]
    psi: np.ndarray                # (n, 2) product input state
    target: str                    # "circuit_output" | "product" | "dense"
    v: np.ndarray                  # (n, 2) or (2^n,)
    level: int = 1
    name: str = ""

    @property
    def n_noises(self) -> int:
        return sum(1 for o in self.ops if o.kind == "noise")

    def noise_ops(self) -> List[Op]:
        return [o for o in self.ops if o.kind == "noise"]

    def gate_ops(self) -> List[Op]:
        return [o for o in self.ops if o.kind == "gate"]

    def with_level(self, level: int) -> "Circuit":
        return dataclasses.replace(self, level=level)


# ----------------------------------------------------------------------------
# gates (Table I of the paper, plus CZ and RZZ)
# ----------------------------------------------------------------------------
def gate_h():
    return np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2.0)


def gate_x():
    return np.array([[0, 1], [1, 0]], dtype=np.complex128)


def gate_y():
    return np.array([[0, -1j], [1j, 0]], dtype=np.complex128)


def gate_z():
    return np.array([[1, 0], [0, -1]], dtype=np.complex128)


def gate_t():
    return np.array([[1, 0], [0, np.exp(1j * math.pi / 4)]], dtype=np.complex128)


def gate_rx(theta):
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


def gate_ry(theta):
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def gate_rz(theta):
    return np.array([[np.exp(-1j * theta / 2), 0], [0, np.exp(1j * theta / 2)]],
                    dtype=np.complex128)


def gate_cz():
    return np.diag([1, 1, 1, -1]).astype(np.complex128)


def gate_rzz(gamma):
    a = np.exp(-1j * gamma / 2)
    b = np.exp(1j * gamma / 2)
    return np.diag([a, b, b, a]).astype(np.complex128)


def haar_su2(rng: np.random.Generator) -> np.ndarray:
    """[[z0, -z1*], [z1, z0*]] with (z0, z1) a normalised complex Gaussian pair."""
    z = rng.standard_normal(4)
    z0 = complex(z[0], z[1])
    z1 = complex(z[2], z[3])
    nrm = math.sqrt(abs(z0) ** 2 + abs(z1) ** 2)
    z0 /= nrm
    z1 /= nrm
    return np.array([[z0, -z1.conjugate()], [z1, z0.conjugate()]], dtype=np.complex128)


# ----------------------------------------------------------------------------
# noise channels (Kraus sets)
# ----------------------------------------------------------------------------
def kraus_depolarizing(p: float) -> List[np.ndarray]:
    s0 = math.sqrt(1.0 - p)
    s1 = math.sqrt(p / 3.0)
    return [s0 * np.eye(2, dtype=np.complex128), s1 * gate_x(), s1 * gate_y(), s1 * gate_z()]


def kraus_ad_pd(gamma: float, lam: float) -> List[np.ndarray]:
    """Amplitude damping (gamma) followed by phase damping (lam).

    AD = {diag(1, sqrt(1-g)), [[0, sqrt(g)], [0, 0]]},
    PD = {diag(1, sqrt(1-l)), diag(0, sqrt(l))}.
    The Kraus set of the composition is {P_j A_i}; the product that vanishes
    identically (PD_1 * AD_1) is dropped.
    """
    a0 = np.array([[1, 0], [0, math.sqrt(1 - gamma)]], dtype=np.complex128)
    a1 = np.array([[0, math.sqrt(gamma)], [0, 0]], dtype=np.complex128)
    p0 = np.array([[1, 0], [0, math.sqrt(1 - lam)]], dtype=np.complex128)
    p1 = np.array([[0, 0], [0, math.sqrt(lam)]], dtype=np.complex128)
    out = []
    for p in (p0, p1):
        for a in (a0, a1):
            k = p @ a
            if np.any(k != 0):
                out.append(k)
    return out


def random_isometry_kraus(rng: np.random.Generator, n_kraus: int) -> List[np.ndarray]:
    """A random CPTP channel: the Kraus matrices are the 2x2 blocks of a random
    (2 n_kraus) x 2 isometry (QR of a complex Gaussian matrix)."""
    g = rng.standard_normal((2 * n_kraus, 2)) + 1j * rng.standard_normal((2 * n_kraus, 2))
    q, _ = np.linalg.qr(g)
    return [q[2 * k:2 * k + 2, :].astype(np.complex128) for k in range(n_kraus)]


# ----------------------------------------------------------------------------
# circuit skeletons
# ----------------------------------------------------------------------------
def chain_layers(n: int, layers: int, rng: np.random.Generator) -> List[Op]:
    """Layer l: Haar SU(2) on every qubit, then CZ on (0,1),(2,3),... if l is
    even, else on (1,2),(3,4),..."""
    ops: List[Op] = []
    for layer in range(layers):
        for q in range(n):
            ops.append(Op("gate", (q,), haar_su2(rng), label="su2"))
        start = 0 if layer % 2 == 0 else 1
        for q in range(start, n - 1, 2):
            ops.append(Op("gate", (q, q + 1), gate_cz(), label="cz"))
    return ops


def grid_edges(rows: int, cols: int, colour: str):
    """Edges of one colour of the 4-colour grid schedule; qubit q = r*cols + c.
    A: horizontal, c even; B: horizontal, c odd; C: vertical, r even;
    D: vertical, r odd."""
    e = []
    for r in range(rows):
        for c in range(cols):
            q = r * cols + c
            if colour == "A" and c % 2 == 0 and c + 1 < cols:
                e.append((q, q + 1))
            elif colour == "B" and c % 2 == 1 and c + 1 < cols:
                e.append((q, q + 1))
            elif colour == "C" and r % 2 == 0 and r + 1 < rows:
                e.append((q, q + cols))
            elif colour == "D" and r % 2 == 1 and r + 1 < rows:
                e.append((q, q + cols))
    return e


def grid_layers(rows: int, cols: int, layers: int, colours: str,
                rng: np.random.Generator) -> List[Op]:
    ops: List[Op] = []
    n = rows * cols
    for layer in range(layers):
        for q in range(n):
            ops.append(Op("gate", (q,), haar_su2(rng), label="su2"))
        for (a, b) in grid_edges(rows, cols, colours[layer % len(colours)]):
            ops.append(Op("gate", (a, b), gate_cz(), label="cz"))
    return ops


def random_3regular_edges(n: int, seed: int):
    import networkx as nx
    g = nx.random_regular_graph(3, n, seed=seed)
    return sorted(tuple(sorted(e)) for e in g.edges())


def qaoa_3regular(n: int, p: int, graph_seed: int, rng: np.random.Generator) -> List[Op]:
    """H on every qubit, then p rounds of [RZZ(gamma_r) on every edge in sorted
    edge order; RX(beta_r) on every qubit], gamma_r, beta_r ~ U[0, pi]."""
    edges = random_3regular_edges(n, graph_seed)
    ops = [Op("gate", (q,), gate_h(), label="h") for q in range(n)]
    for _ in range(p):
        gamma = rng.uniform(0.0, math.pi)
        beta = rng.uniform(0.0, math.pi)
        for (a, b) in edges:
            ops.append(Op("gate", (a, b), gate_rzz(gamma), label="rzz"))
        for q in range(n):
            ops.append(Op("gate", (q,), gate_rx(beta), label="rx"))
    return ops


def place_noises(gates: Sequence[Op], kraus_sets: Sequence[List[np.ndarray]],
                 rng: np.random.Generator) -> List[Op]:
    """Append each noise right after a distinct gate drawn uniformly without
    replacement; on a 2-qubit gate the noisy qubit is one of its two qubits,
    drawn uniformly.  ``kraus_sets[k]`` goes to the k-th chosen gate in circuit
    order."""
    n_noise = len(kraus_sets)
    if n_noise > len(gates):
        raise ValueError("more noises than gates")
    chosen = np.sort(rng.choice(len(gates), size=n_noise, replace=False))
    which = [int(rng.integers(len(gates[int(g)].qubits))) for g in chosen]
    slot_of = {int(g): (k, w) for k, (g, w) in enumerate(zip(chosen, which))}
    out: List[Op] = []
    for i, g in enumerate(gates):
        out.append(g)
        if i in slot_of:
            k, w = slot_of[i]
            out.append(Op("noise", (g.qubits[w],), kraus=list(kraus_sets[k]), label="noise"))
    return out


def zero_product(n: int) -> np.ndarray:
    s = np.zeros((n, 2), dtype=np.complex128)
    s[:, 0] = 1.0
    return s


# ----------------------------------------------------------------------------
# the five configurations
# ----------------------------------------------------------------------------
CONFIG_NAMES = {
    1: "chain8_10L_4adpd",
    2: "grid5x5_12L_10depol",
    3: "qaoa36_p2_20adpd",
    4: "mixed64",
    5: "grid15x15_6L_20adpd",
}


def _adpd_sets(rng, n_noise, lo, hi):
    sets = []
    for _ in range(n_noise):
        g = rng.uniform(lo, hi)
        lam = rng.uniform(lo, hi)
        sets.append(kraus_ad_pd(g, lam))
    return sets


def _depol_sets(rng, n_noise, lo, hi):
    return [kraus_depolarizing(rng.uniform(lo, hi)) for _ in range(n_noise)]


def config(c: int, level: Optional[int] = None, sub: Optional[int] = None):
    """Build config ``c`` (1..5).  Config 4 returns a list of 64 circuits
    (``sub`` selects one).  ``level`` overrides the config's default level."""
    rng = np.random.Generator(np.random.PCG64(CONFIG_SEED_BASE + c))
    if c == 1:
        n = 8
        gates = chain_layers(n, 10, rng)
        kr = _adpd_sets(rng, 4, 1e-3, 1e-2)
        ops = place_noises(gates, kr, rng)
        circ = Circuit(n, ops, zero_product(n), "circuit_output", zero_product(n),
                       level=2 if level is None else level, name=CONFIG_NAMES[1])
        return circ
    if c == 2:
        gates = grid_layers(5, 5, 12, "ABCD", rng)
        kr = _depol_sets(rng, 10, 1e-4, 5e-3)
        ops = place_noises(gates, kr, rng)
        return Circuit(25, ops, zero_product(25), "circuit_output", zero_product(25),
                       level=2 if level is None else level, name=CONFIG_NAMES[2])
    if c == 3:
        gates = qaoa_3regular(36, 2, CONFIG_SEED_BASE + 3, rng)
        kr = _adpd_sets(rng, 20, 1e-4, 1e-3)
        ops = place_noises(gates, kr, rng)
        return Circuit(36, ops, zero_product(36), "circuit_output", zero_product(36),
                       level=2 if level is None else level, name=CONFIG_NAMES[3])
    if c == 4:
        return mixed_batch(level=level, sub=sub)
    if c == 5:
        gates = grid_layers(15, 15, 6, "ABCDAB", rng)
        kr = _adpd_sets(rng, 20, 1e-4, 1e-3)
        ops = place_noises(gates, kr, rng)
        return Circuit(225, ops, zero_product(225), "circuit_output", zero_product(225),
                       level=3 if level is None else level, name=CONFIG_NAMES[5])
    raise ValueError(f"unknown config {c}")


def mixed_batch(count: int = 64, level: Optional[int] = None, sub: Optional[int] = None,
                max_qubits: int = 100, grid_budget: int = 200):
    """Uneven batch: chains and near-square grids of 16..max_qubits qubits,
    6..16 layers, 5..20 noises each (depolarizing U[1e-4, 5e-3] or AD+PD
    U[1e-4, 1e-3], chosen per noise), level 2 or 3 per circuit.  Circuit k is
    drawn from SeedSequence(2211170284).spawn(count)[k].

    Resampling rule: a grid whose qubits x layers exceeds `grid_budget` has no
    contraction path of bounded width (random 2D circuits of that depth), so
    its shape (qubits, layers) is redrawn from the same stream until it fits;
    chains are never redrawn."""
    seqs = np.random.SeedSequence(CONFIG_SEED_BASE + 4).spawn(count)
    out = []
    for k, ss in enumerate(seqs):
        if sub is not None and k != sub:
            continue
        rng = np.random.Generator(np.random.PCG64(ss))
        while True:
            n = int(rng.integers(16, max_qubits + 1))
            layers = int(rng.integers(6, 17))
            grid = rng.uniform() >= 0.5
            if grid:
                rows = int(math.floor(math.sqrt(n)))
                cols = int(math.ceil(n / rows))
                n = rows * cols
                if n * layers > grid_budget:
                    continue
            break
        n_noise = int(rng.integers(5, 21))
        lev = int(rng.integers(2, 4)) if level is None else level
        if not grid:
            gates = chain_layers(n, layers, rng)
            shape = f"chain{n}"
        else:
            gates = grid_layers(rows, cols, layers, "ABCD", rng)
            shape = f"grid{rows}x{cols}"
        kr = []
        for _ in range(n_noise):
            if rng.uniform() < 0.5:
                kr.append(kraus_depolarizing(rng.uniform(1e-4, 5e-3)))
            else:
                kr.append(kraus_ad_pd(rng.uniform(1e-4, 1e-3), rng.uniform(1e-4, 1e-3)))
        ops = place_noises(gates, kr, rng)
        out.append(Circuit(n, ops, zero_product(n), "circuit_output", zero_product(n),
                           level=lev, name=f"mixed{k}_{shape}_{layers}L_{n_noise}n"))
    if sub is not None:
        return out[0]
    return out


def tiny_random_circuit(rng: np.random.Generator, n: int, n_gates: int, n_noise: int,
                        noise: str = "random", level: int = 1, target: str = "circuit_output",
                        scale: float = 1.0) -> Circuit:
    """Small random circuit for property tests: random 1-qubit Haar gates and
    CZ / random-2-qubit-unitary gates on random pairs; noises placed by
    ``place_noises``.  ``noise`` is "random" (random CPTP channel with 1..4 Kraus
    matrices), "depol" or "adpd".  ``scale`` scales the noise parameters of
    depol / adpd."""
    gates: List[Op] = []
    for _ in range(n_gates):
        if n >= 2 and rng.uniform() < 0.4:
            a, b = rng.choice(n, size=2, replace=False)
            if rng.uniform() < 0.5:
                m = gate_cz()
            else:
                g = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
                m, _ = np.linalg.qr(g)
            gates.append(Op("gate", (int(a), int(b)), m.astype(np.complex128), label="u2"))
        else:
            q = int(rng.integers(n))
            gates.append(Op("gate", (q,), haar_su2(rng), label="su2"))
    kr = []
    for _ in range(n_noise):
        if noise == "depol":
            kr.append(kraus_depolarizing(scale * rng.uniform(1e-3, 5e-2)))
        elif noise == "adpd":
            kr.append(kraus_ad_pd(scale * rng.uniform(1e-3, 5e-2), scale * rng.uniform(1e-3, 5e-2)))
        else:
            kr.append(random_isometry_kraus(rng, int(rng.integers(1, 5))))
    ops = place_noises(gates, kr, rng)
    psi = np.zeros((n, 2), dtype=np.complex128)
    for q in range(n):
        z = rng.standard_normal(2) + 1j * rng.standard_normal(2)
        psi[q] = z / np.linalg.norm(z)
    if target == "circuit_output":
        v = np.zeros((n, 2), dtype=np.complex128)
        for q in range(n):
            z = rng.standard_normal(2) + 1j * rng.standard_normal(2)
            v[q] = z / np.linalg.norm(z)
    elif target == "product":
        v = np.zeros((n, 2), dtype=np.complex128)
        for q in range(n):
            z = rng.standard_normal(2) + 1j * rng.standard_normal(2)
            v[q] = z / np.linalg.norm(z)
    elif target == "dense":
        z = rng.standard_normal(2 ** n) + 1j * rng.standard_normal(2 ** n)
        v = z / np.linalg.norm(z)
    else:
        raise ValueError(target)
    return Circuit(n, ops, psi, target, v, level=level, name=f"tiny{n}")


def trajectory_uniforms(n_samples: int, n_noise: int, seed: int) -> np.ndarray:
    """Seeded uniforms in [0, 1), one per (sample, noise): the random input of
    a trajectories run (the draws are made from them by each implementation)."""
    return np.random.default_rng(seed).random((n_samples, n_noise))
