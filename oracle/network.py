"""Algorithm 1 with one tensor network per term (any n).

Why one network suffices: the split of Section IV gives
Mt = S D T^dagger with Mt = sum_k vec(E_k) vec(E_k)^dagger Hermitian positive
semidefinite, so on every non-zero singular value S|i> = T|i>.  Hence
U_i = d_i K_i and V_i = conj(K_i) with K_i = unvec(S|i>), the bra network of a
term is the complex conjugate of its ket network with slots K_i, and the term
is X = (prod_s d_{c_s}) |a|^2 with a = <v| U~_c |psi> (slots K_{c_s}).  This
identity is checked against the literal two-network evaluation in
tests/test_oracle_estimate.py.

Contraction: the ket network is built as a list of tensors whose legs all have
dimension 2, reduced by the light cone of the noise slots when the target is
the circuit's own ideal output (gates with no slot in their causal future
cancel against their inverses in <psi_v| U^dagger U~ |psi>), and contracted
pairwise with numpy.tensordot in a greedy order (smallest growth first, fixed
tie-break).  The order changes rounding only.

With ``diagonal=True`` a gate whose matrix is diagonal keeps the basis index
of its wires: it becomes a tensor of its diagonal on the wires' current
indices, which are then shared by more than two tensors.  Pairs are then
contracted with numpy.einsum, summing an index only when no other remaining
tensor carries it.  Same value, far smaller intermediates for CZ / RZZ
circuits.
"""
from __future__ import annotations

import heapq
from typing import List, Tuple

import numpy as np

from . import channels


class KetNetwork:
    """Topology + fixed tensors of the ket network of a circuit; slot tensors
    are filled in per term."""

    def __init__(self, circ, reduce: bool = True, diagonal: bool = False):
        self.circ = circ
        self.diagonal = diagonal
        n = circ.n_qubits
        tensors: List[Tuple[object, list]] = []   # (array or ("slot", s), legs)
        scalar = 1.0 + 0.0j
        ops = list(circ.ops)
        noise_index = {}
        s = 0
        for k, op in enumerate(ops):
            if op.kind == "noise":
                noise_index[k] = s
                s += 1
        self.n_noise = s
        if circ.target == "circuit_output":
            keep = [True] * len(ops)
            if reduce:
                live = set()
                for k in range(len(ops) - 1, -1, -1):
                    op = ops[k]
                    if op.kind == "noise":
                        live.add(op.qubits[0])
                    elif live & set(op.qubits):
                        live |= set(op.qubits)
                    else:
                        keep[k] = False
            fwd = [k for k in range(len(ops)) if keep[k]]
            touched = set()
            for k in fwd:
                touched |= set(ops[k].qubits)
            # qubits with nothing left: <psi_v,q | psi_q>
            for q in range(n):
                if q not in touched:
                    scalar *= np.vdot(circ.v[q], circ.psi[q])
            bwd = [k for k in reversed(fwd) if ops[k].kind == "gate"]
            seq = [(k, False) for k in fwd] + [(k, True) for k in bwd]
            end = "product_v"
        elif circ.target in ("product", "dense"):
            touched = set(range(n))
            seq = [(k, False) for k in range(len(ops))]
            end = circ.target
        else:
            raise ValueError(circ.target)
        edge = 0
        cur = {}
        for q in sorted(touched):
            cur[q] = edge
            tensors.append((np.asarray(circ.psi[q], dtype=np.complex128), [edge]))
            edge += 1
        for k, inverse in seq:
            op = ops[k]
            qs = list(op.qubits)
            if diagonal and op.kind == "gate" and np.count_nonzero(op.mat - np.diag(np.diag(op.mat))) == 0:
                dg = np.diag(op.mat)
                dg = dg.conj() if inverse else dg
                tensors.append((np.asarray(dg, dtype=np.complex128).reshape((2,) * len(qs)),
                                [cur[q] for q in qs]))
                continue
            ins = [cur[q] for q in qs]
            outs = list(range(edge, edge + len(qs)))
            edge += len(qs)
            for q, e in zip(qs, outs):
                cur[q] = e
            if op.kind == "gate":
                m = op.mat.conj().T if inverse else op.mat
                arr = np.asarray(m, dtype=np.complex128).reshape((2,) * (2 * len(qs)))
                tensors.append((arr, outs + ins))
            else:
                tensors.append((("slot", noise_index[k]), outs + ins))
        if end == "product_v":
            for q in sorted(touched):
                tensors.append((np.asarray(circ.v[q], dtype=np.complex128).conj(), [cur[q]]))
        elif end == "product":
            for q in range(n):
                tensors.append((np.asarray(circ.v[q], dtype=np.complex128).conj(), [cur[q]]))
        else:
            vv = np.asarray(circ.v, dtype=np.complex128).reshape((2,) * n).conj()
            tensors.append((vv, [cur[q] for q in range(n)]))
        self.tensors = tensors
        self.scalar = scalar
        if diagonal:
            self.path = hyper_greedy_path([legs for _, legs in tensors])
        else:
            self.path = greedy_path([legs for _, legs in tensors])

    def value(self, slot_mats) -> complex:
        """Contract with slot s set to the 2x2 matrix slot_mats[s]."""
        arrs = []
        legs = []
        for t, lg in self.tensors:
            if isinstance(t, tuple):
                arrs.append(np.asarray(slot_mats[t[1]], dtype=np.complex128))
            else:
                arrs.append(t)
            legs.append(list(lg))
        if self.diagonal:
            return self.scalar * contract_hyper(arrs, legs, self.path)
        return self.scalar * contract_path(arrs, legs, self.path)


def greedy_path(legs_list: List[List[int]]):
    """Pairwise order: repeatedly merge the pair of tensors sharing a leg whose
    result grows the total size least (2^|C| - 2^|A| - 2^|B|), ties broken by
    the smaller tensor ids; disconnected leftovers are multiplied at the end.
    Returns a list of (id_a, id_b, id_new)."""
    legs = {i: frozenset(l) for i, l in enumerate(legs_list)}
    owners = {}
    for i, l in legs.items():
        for e in l:
            owners.setdefault(e, set()).add(i)
    heap = []

    def push(a, b):
        if a == b:
            return
        if a > b:
            a, b = b, a
        lc = legs[a] ^ legs[b]
        score = 2.0 ** len(lc) - 2.0 ** len(legs[a]) - 2.0 ** len(legs[b])
        heapq.heappush(heap, (score, a, b))

    for e, os in owners.items():
        os = sorted(os)
        if len(os) == 2:
            push(os[0], os[1])
    nxt = len(legs_list)
    path = []
    alive = set(legs)
    while heap:
        score, a, b = heapq.heappop(heap)
        if a not in alive or b not in alive:
            continue
        la, lb = legs[a], legs[b]
        lc = la ^ lb
        alive.discard(a)
        alive.discard(b)
        legs[nxt] = lc
        alive.add(nxt)
        for e in la | lb:
            owners[e].discard(a)
            owners[e].discard(b)
        for e in la & lb:
            del owners[e]
        for e in lc:
            owners[e].add(nxt)
        path.append((a, b, nxt))
        for e in lc:
            for o in owners[e]:
                if o != nxt:
                    push(o, nxt)
        nxt += 1
    rest = sorted(alive)
    while len(rest) > 1:
        a, b = rest[0], rest[1]
        legs[nxt] = legs[a] ^ legs[b]
        path.append((a, b, nxt))
        rest = [nxt] + rest[2:]
        nxt += 1
    return path


def _hyper_greedy_once(legs_list, rng, temp):
    legs = {i: frozenset(l) for i, l in enumerate(legs_list)}
    owners = {}
    for i, l in legs.items():
        for e in l:
            owners.setdefault(e, set()).add(i)

    def result(a, b):
        return frozenset(e for e in legs[a] | legs[b] if owners[e] - {a, b})

    heap = []

    def push(a, b):
        if a > b:
            a, b = b, a
        lc = result(a, b)
        score = 2.0 ** len(lc) - 2.0 ** len(legs[a]) - 2.0 ** len(legs[b])
        if temp > 0:
            score = np.sign(score) * np.log2(1 + abs(score)) - temp * rng.gumbel()
        heapq.heappush(heap, (score, a, b))

    for e, os in owners.items():
        os = sorted(os)
        for i in range(len(os)):
            for j in range(i + 1, len(os)):
                push(os[i], os[j])
    alive = set(legs)
    nxt = len(legs_list)
    path = []
    cost = 0.0
    while heap:
        _, a, b = heapq.heappop(heap)
        if a not in alive or b not in alive:
            continue
        lc = result(a, b)
        cost += 2.0 ** len(legs[a] | legs[b])
        for e in legs[a] | legs[b]:
            owners[e] -= {a, b}
        legs[nxt] = lc
        for e in lc:
            owners[e].add(nxt)
        alive -= {a, b}
        alive.add(nxt)
        path.append((a, b, nxt, lc))
        for e in lc:
            for o in owners[e]:
                if o != nxt:
                    push(o, nxt)
        nxt += 1
    rest = sorted(alive)
    while len(rest) > 1:
        a, b = rest[0], rest[1]
        lc = frozenset(e for e in legs[a] | legs[b] if owners.get(e, set()) - {a, b})
        for e in legs[a] | legs[b]:
            owners[e] = owners.get(e, set()) - {a, b}
        legs[nxt] = lc
        path.append((a, b, nxt, lc))
        rest = [nxt] + rest[2:]
        nxt += 1
    return cost, path


def hyper_greedy_path(legs_list: List[List[int]], trials: int = 16):
    """Greedy order for networks whose indices may be shared by more than two
    tensors: repeatedly merge a pair (sharing an index) whose result grows the
    total size least; an index survives a merge while any other tensor still
    carries it.  The first trial is deterministic, the others add seeded
    Gumbel noise to the scores; the cheapest (sum of 2^|legs of both|) wins.
    Returns [(id_a, id_b, id_new, result_legs)]."""
    rng = np.random.default_rng(12345)
    best = None
    for t in range(trials):
        cost, path = _hyper_greedy_once(legs_list, rng, 0.0 if t == 0 else 1.0)
        if best is None or cost < best[0]:
            best = (cost, path)
    return best[1]


def contract_hyper(arrs, legs, path) -> complex:
    """Apply a hyper_greedy_path: each pair is transposed to
    [kept shared | own | summed] x [kept shared | summed | own] and multiplied
    with numpy.matmul (complex128), batched over the kept shared indices."""
    store = {i: (a, list(l)) for i, (a, l) in enumerate(zip(arrs, legs))}
    if not store:
        return 1.0 + 0.0j
    for a, b, c, lc in path:
        ta, la = store.pop(a)
        tb, lb = store.pop(b)
        shared = [e for e in la if e in lb]
        batch = [e for e in shared if e in lc]
        summed = [e for e in shared if e not in lc]
        fa = [e for e in la if e not in lb]
        fb = [e for e in lb if e not in la]
        pa = np.transpose(ta, [la.index(e) for e in batch + fa + summed])
        pb = np.transpose(tb, [lb.index(e) for e in batch + summed + fb])
        nb, na, nk, nf = 2 ** len(batch), 2 ** len(fa), 2 ** len(summed), 2 ** len(fb)
        tc = np.matmul(pa.reshape(nb, na, nk), pb.reshape(nb, nk, nf))
        out = batch + fa + fb
        store[c] = (tc.reshape((2,) * len(out)), out)
    assert len(store) == 1
    (t, l), = store.values()
    assert len(l) == 0
    return complex(np.asarray(t).reshape(()))


def contract_path(arrs, legs, path) -> complex:
    store = {i: (a, l) for i, (a, l) in enumerate(zip(arrs, legs))}
    if not store:
        return 1.0 + 0.0j          # everything cancelled: empty network
    for a, b, c in path:
        ta, la = store.pop(a)
        tb, lb = store.pop(b)
        shared = [e for e in la if e in lb]
        ia = [la.index(e) for e in shared]
        ib = [lb.index(e) for e in shared]
        tc = np.tensordot(ta, tb, axes=(ia, ib))
        lc = [e for e in la if e not in shared] + [e for e in lb if e not in shared]
        store[c] = (tc, lc)
    assert len(store) == 1
    (t, l), = store.values()
    assert len(l) == 0
    return complex(t)


def slot_split(circ):
    """For every noise: (d[4], K[4,2,2]) with K_i = U_i / d_i (zero when
    d_i = 0), and the assertion that V_i = conj(K_i) holds."""
    out = []
    for op in circ.noise_ops():
        d, u, v = channels.svd_split(channels.superoperator(op.kraus))
        k = np.zeros((4, 2, 2), dtype=np.complex128)
        for i in range(4):
            if d[i] > 0:
                k[i] = u[i] / d[i]
        out.append((d, k, v))
    return out


def term_value(net: KetNetwork, split, term):
    """(X, a): X = prod_s d_{c_s} |a|^2, a the ket network value with slots K."""
    w = 1.0
    mats = []
    for s, c in enumerate(term):
        d, k, _ = split[s]
        w *= d[c]
        mats.append(k[c])
    if w == 0.0:
        return 0.0, 0.0j
    a = net.value(mats)
    return w * (a.real * a.real + a.imag * a.imag), a
