"""Schedule keys of the paper's synthetic sets (helper of the paper-size
schedule tests and of tests/golden/make_schedule_keys.py; not a test module).

A key is the SHA-256 of the per-row core (pi), superstep (sigma) and the
Sec. 5 order (perm) as little-endian int32 arrays, with S and the number of
wavefronts beside it.  ``instance_keys`` computes, for one instance of the
ER or NB set of Sec. 6.2.4/6.2.5 at n = 1e5, the oracle's keys under
Algorithm 3.1 (and, when asked, the library's) at two parameter sets: the
paper's (k = 22, L = 500, alpha0 = 20, growth 1.5, acceptance 0.97) and the
GPU's (k = 65,536 lane-cores, L = 50, alpha0 = 1)."""
from __future__ import annotations

import hashlib
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PARAMS = {"paper": dict(k=22, L=500.0, alpha0=20.0), "device": dict(k=1 << 16, L=50.0, alpha0=1.0)}


def key_of(pi, sigma, perm) -> str:
    h = hashlib.sha256()
    for a in (pi, sigma, perm):
        h.update(np.ascontiguousarray(a, dtype="<i4").tobytes())
    return h.hexdigest()


def instances():
    """(family, p, B, seed index) of the 60 systems: three ER probabilities
    and three NB (p, B) pairs, ten instances each (letters A..J)."""
    from paper_2503_05408_amd import gen
    out = [("ER", p, None, i) for p in gen.ER_PROBS for i in range(10)]
    out += [("NB", p, Bw, i) for p, Bw in gen.NB_PAIRS for i in range(10)]
    return out


def make(fam, p, Bw, i):
    from paper_2503_05408_amd import gen
    if fam == "ER":
        return gen.erdos_renyi_paper(100_000, p, gen.SEED_BASE + i)
    return gen.narrow_band(100_000, p, Bw, gen.SEED_BASE + 10 + i)


def oracle_keys(m) -> dict:
    import oracle
    _, nl = oracle.levels(m)
    out = {"wavefronts": nl}
    for name, prm in PARAMS.items():
        pi, sigma, S = oracle.growlocal(m, prm["k"], L=prm["L"], alpha0=prm["alpha0"])
        perm, _ = oracle.reorder(m, pi, sigma)
        out[name] = {"S": int(S), "key": key_of(pi, sigma, perm)}
    return out


def library_keys(m) -> dict:
    from paper_2503_05408_amd import binding as B
    out = {}
    for name, prm in PARAMS.items():
        core, sup, S = B.schedule(m, B.default_opts(**prm))
        perm = B.reorder(core, sup)
        out[name] = {"S": int(S), "key": key_of(core, sup, perm)}
    return out


def instance_keys(args) -> dict:
    """Worker entry: args = (family, p, B, i, with_library)."""
    fam, p, Bw, i, with_library = args
    m = make(fam, p, Bw, i)
    out = {"family": fam, "p": p, "B": Bw, "instance": i, "n": m.n, "nnz": m.nnz, "oracle": oracle_keys(m)}
    if with_library:
        out["library"] = library_keys(m)
    return out


def all_instance_keys(with_library: bool, workers: int | None = None) -> list:
    """Every instance, computed in worker processes (spawned: each has its own
    oracle and library), in the order of ``instances()``."""
    import concurrent.futures as cf
    import multiprocessing as mp
    jobs = [(*t, with_library) for t in instances()]
    # the largest ER instances first, so the pool's tail is short
    order = sorted(range(len(jobs)), key=lambda j: (jobs[j][0] != "ER", -(jobs[j][1] or 0)))
    workers = workers or max(1, min(6, (os.cpu_count() or 2) - 1))
    res = [None] * len(jobs)
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        futs = {ex.submit(instance_keys, jobs[j]): j for j in order}
        for f in cf.as_completed(futs):
            res[futs[f]] = f.result()
    return res
