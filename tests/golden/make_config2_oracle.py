"""Write tests/golden/config2_oracle.txt: A(0), A(1), A(2) of the 5x5-grid,
12-layer, 10-depolarizing-noise workload, computed by the FP64 oracle alone
(one network per term, every term).  Usage: python tests/golden/make_config2_oracle.py [procs]"""
import os
import sys
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import estimate, network, terms  # noqa: E402

_state = {}


def _init():
    c = W.config(2)
    _state["net"] = network.KetNetwork(c)
    _state["split"] = network.slot_split(c)


def _value(t):
    return network.term_value(_state["net"], _state["split"], t)[0]


def main():
    procs = int(sys.argv[1]) if len(sys.argv) > 1 else 4
    c = W.config(2)
    tl = terms.enumerate_terms(c.n_noises, 2)
    with Pool(procs, initializer=_init) as pool:
        xs = pool.map(_value, tl, chunksize=4)
    r = estimate.estimate(c, 2, "network", term_list=[])  # empty: reuse the summation only
    sums = [estimate.Neumaier() for _ in range(3)]
    for t, x in zip(tl, xs):
        sums[terms.term_level(t)].add(float(x))
    acc = estimate.Neumaier()
    out = []
    for s in sums:
        acc.add(s.value)
        out.append(acc.value)
    with open(os.path.join(HERE, "config2_oracle.txt"), "w") as f:
        f.write("# A(0) A(1) A(2) of the 5x5 grid / 12 layers / 10 depolarizing noises workload\n")
        f.write("# written by tests/golden/make_config2_oracle.py (FP64 oracle, every term)\n")
        for v in out:
            f.write(f"{v:.17g}\n")
    print(out)


if __name__ == "__main__":
    main()
