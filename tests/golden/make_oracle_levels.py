"""Write the stored oracle values of workload config <c>, computed by the FP64
oracle alone (one network per term, every term, diagonal gates as shared
indices; Algorithm 1's level sums with Neumaier summation in term order):

  config<c>_oracle.txt   A(0..l), one value per line
  config<c>_levels.txt   T_u (u = 0..l), the per-level sums, one per line
  config<c>_terms.npy    X_t of every term in enumeration order (float64)

Usage: python tests/golden/make_oracle_levels.py <config> [procs]"""
import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import estimate, network, terms  # noqa: E402

_state = {}


def _init(cfg):
    c = W.config(cfg)
    _state["net"] = network.KetNetwork(c, diagonal=True)
    _state["split"] = network.slot_split(c)


def _value(t):
    return network.term_value(_state["net"], _state["split"], t)[0]


def main():
    cfg = int(sys.argv[1])
    procs = int(sys.argv[2]) if len(sys.argv) > 2 else 4
    c = W.config(cfg)
    tl = terms.enumerate_terms(c.n_noises, c.level)
    with Pool(procs, initializer=_init, initargs=(cfg,)) as pool:
        xs = pool.map(_value, tl, chunksize=16)
    sums = [estimate.Neumaier() for _ in range(c.level + 1)]
    for t, x in zip(tl, xs):
        sums[terms.term_level(t)].add(float(x))
    acc = estimate.Neumaier()
    out = []
    for s in sums:
        acc.add(s.value)
        out.append(acc.value)
    head = f"of workload {c.name} ({len(tl)} terms)\n# written by tests/golden/make_oracle_levels.py (FP64 oracle, every term)\n"
    with open(os.path.join(HERE, f"config{cfg}_oracle.txt"), "w") as f:
        f.write(f"# A(0..{c.level}) " + head)
        for v in out:
            f.write(f"{v:.17g}\n")
    with open(os.path.join(HERE, f"config{cfg}_levels.txt"), "w") as f:
        f.write(f"# T_0..T_{c.level} " + head)
        for s in sums:
            f.write(f"{s.value:.17g}\n")
    np.save(os.path.join(HERE, f"config{cfg}_terms.npy"), np.asarray(xs, dtype=np.float64))
    print(cfg, out, [s.value for s in sums], flush=True)


if __name__ == "__main__":
    main()
