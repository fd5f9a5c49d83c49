"""Writes tests/golden/schedule_keys.json: the oracle's GrowLocal schedule
keys (Algorithm 3.1 plus the order of Sec. 5; see tests/paper_schedule_keys.py
for the key) of

* the 60 systems of the paper's synthetic sets at n = 1e5 (Sec. 6.2.4/6.2.5,
  Tables A.4/A.5), at the paper's parameters and at the GPU's;
* the single-system benchmark matrix: Erdos-Renyi, n = 1e7, 10 off-diagonals
  per row on average (q = 2e-6), seed 2503054280, at the GPU's parameters.

Only the oracle and the input generator are called.  Usage (from the
repository root):  python tests/golden/make_schedule_keys.py
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))                    # tests/
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))   # repository root

import paper_schedule_keys as K  # noqa: E402

BENCH_N = 10_000_000


def bench_matrix():
    from paper_2503_05408_amd import gen
    m = gen.er_n1e7()
    assert m.n == BENCH_N
    return m


def main():
    import oracle
    t0 = time.time()
    sets = K.all_instance_keys(with_library=False)
    print(f"paper sets: {time.time() - t0:.0f} s", flush=True)
    t0 = time.time()
    m = bench_matrix()
    prm = K.PARAMS["device"]
    pi, sigma, S = oracle.growlocal(m, prm["k"], L=prm["L"], alpha0=prm["alpha0"])
    perm, _ = oracle.reorder(m, pi, sigma)
    _, nl = oracle.levels(m)
    bench = {"name": m.name, "n": m.n, "nnz": m.nnz, "wavefronts": nl, "params": prm,
             "S": int(S), "key": K.key_of(pi, sigma, perm)}
    print(f"bench matrix: {time.time() - t0:.0f} s, S={S}", flush=True)
    out = {"about": "oracle GrowLocal (Algorithm 3.1) + Sec. 5 order; key = sha256 of int32 pi, sigma, perm",
           "params": K.PARAMS, "paper_sets": sets, "bench_er_n1e7": bench}
    with open(os.path.join(HERE, "schedule_keys.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
