"""MDAS with the linear lambda path (Eq. 2) against the soft-core path of
Eq. 4: work statistics and acceptance of the same alchemical transitions.

For each system the program runs n_cycles MDAS cycles (P pairs, K
increments, M MD steps per increment, n_md plain MD steps between cycles)
from the same relaxed start, once per path, and reports the acceptance,
the mean and spread of the work, and the acceptance estimated from the
works.  The paper applies the soft-core form to its atomistic runs only.

    python -m paper_2005_08348_amd.paths [--cycles 400] [--systems mix c1 toy]

prints one JSON line.  ``toy`` is the topology-changing exchange fluid
(``systems.topo_exchange_toy``: the two kinds differ in their bonded terms).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import systems as S
from .mixing import acceptance_from_work


def run(sysm, path, n_cycles, P=1, K=50, M=1, n_md=50, delta=0.05, precision="mixed"):
    from . import membx as Mx
    g = Mx.System(sysm, precision=precision)
    g.minimize(100)
    g.md_step(2000)
    g.set_mdas_path(path, delta)
    works, acc = [], 0
    t0 = time.perf_counter()
    for _ in range(n_cycles):
        g.md_step(n_md)
        r = g.mdas_cycle(P, K, M)
        works.append(r["work"])
        acc += int(r["accept"])
    wall = time.perf_counter() - t0
    g.close()
    w = np.asarray(works)
    kT = S.KB * sysm.temperature
    return {"path": "soft-core" if path == 1 else "linear", "cycles": n_cycles, "accepted": acc,
            "acceptance": acc / n_cycles, "work_mean": float(w.mean()), "work_sd": float(w.std()),
            "acceptance_from_work": acceptance_from_work(w, kT), "wall_s": wall}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--cycles", type=int, default=400)
    ap.add_argument("--systems", nargs="+", default=["mix", "c1"])
    args = ap.parse_args(argv)
    out = {"mdas": "1 pair, K = 50, M = 1, 50 MD steps between cycles", "delta_nm2": 0.05,
           "runs": {}}
    for name in args.systems:
        if name == "toy":
            sysm = S.topo_exchange_toy()
        else:
            sysm = S.make(name, demix=False) if name == "mix" else S.make(name)
        for path in (0, 1):
            print(f"[paths] {name} path {path}", file=sys.stderr, flush=True)
            out["runs"].setdefault(name, []).append(run(sysm, path, args.cycles))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
