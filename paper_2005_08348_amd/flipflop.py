"""Interleaflet exchange on an asymmetric bilayer (the application the
paper's Discussion proposes for exchange moves between the two layers).

The ``mix`` bilayer is made fully asymmetric: every lipid of the upper
leaflet is of kind A and every lipid of the lower leaflet of kind D (the
anionic twin of A).  Lipids do not flip between leaflets on MD time
scales, so plain MD keeps the asymmetry; exchanges across leaflets
(``System.set_exchange_regions(2, leaflet)``) relax it.  The observable is
the fraction of kind D in the upper leaflet against force evaluations
(FE), for MC-MD and MDAS with interleaflet partners, and for MC-MD with
partners within a leaflet as the control that must keep the asymmetry.

    python -m paper_2005_08348_amd.flipflop [--fe 100000] [--every 500]

prints one JSON line.  FE are counted as in ``mixing``.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import systems as S


def asymmetric_mix(seed=None):
    """The mix bilayer with kind A in the upper and kind D in the lower leaflet."""
    s = S.make("mix", seed=seed)
    lf = s.meta["leaflet"]
    mk = s.mol_kind.copy()
    mk[lf == 0] = S.KIND_A
    mk[lf == 1] = S.KIND_D
    s.mol_kind = mk
    return s


def fe_to_fraction(x, y, target):
    """First force evaluation count at which the trace reaches `target`
    (None if it never does)."""
    y = np.asarray(y, dtype=np.float64)
    hit = np.nonzero(y >= target)[0]
    return float(x[hit[0]]) if len(hit) else None


def run(method, sysm, fe_total, every, mode, precision="mixed", equil=2000,
        mc_trials=8, mc_steps=2, mdas_pairs=1, mdas_k=50, mdas_m=1, mdas_md=50):
    from . import membx as M
    lf = sysm.meta["leaflet"]
    upper = lf == 0
    n_up = int(np.count_nonzero(upper))
    g = M.System(sysm, precision=precision)
    g.set_exchange_regions(mode, np.maximum(lf, 0))
    g.minimize(100)
    g.md_step(equil)

    def frac():
        return float(np.count_nonzero(g.state()["mol_kind"][upper] == S.KIND_D)) / n_up

    fe, trace, acc, tried = 0, [(0, frac())], 0, 0
    next_pt = every
    t0 = time.perf_counter()
    while fe < fe_total:
        if method == "mcmd":
            r = g.swap_trials(mc_trials)
            g.md_step(mc_steps)
            tried += len(r["accept"])
            acc += int(np.count_nonzero(r["accept"]))
            fe += len(r["accept"]) + mc_steps
        elif method == "mdas":
            g.md_step(mdas_md)
            r = g.mdas_cycle(mdas_pairs, mdas_k, mdas_m)
            tried += 1
            acc += int(r["accept"])
            fe += mdas_md + mdas_k * mdas_m
        else:
            raise ValueError(method)
        if fe >= next_pt:
            trace.append((fe, frac()))
            next_pt += every
    wall = time.perf_counter() - t0
    g.close()
    return dict(trace=trace, accepted=acc, tried=tried, wall_s=wall)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--fe", type=int, default=100000)
    ap.add_argument("--every", type=int, default=500)
    ap.add_argument("--seed", type=int, default=None)
    args = ap.parse_args(argv)
    s = asymmetric_mix(args.seed)
    out = {"system": "mix bilayer, upper leaflet all A, lower leaflet all D (200 lipids each) + 4000 W",
           "observable": "fraction of kind D in the upper leaflet",
           "fe_counting": "1 per MD step, per exchange trial and per MDAS step", "runs": {}}
    for name, method, mode in (("mcmd_interleaflet", "mcmd", 2), ("mdas_interleaflet", "mdas", 2),
                               ("mcmd_within_leaflet", "mcmd", 1)):
        print(f"[flipflop] {name}", file=sys.stderr, flush=True)
        r = run(method, s, args.fe, args.every, mode)
        x = np.array([p[0] for p in r["trace"]], dtype=np.float64)
        y = np.array([p[1] for p in r["trace"]], dtype=np.float64)
        tail = y[len(y) * 3 // 4:]
        out["runs"][name] = {"fe": x.tolist(), "fraction_d_upper": y.tolist(),
                             "accepted": r["accepted"], "tried": r["tried"], "wall_s": r["wall_s"],
                             "fe_to_quarter": fe_to_fraction(x, y, 0.25),
                             "final_mean": float(tail.mean()), "final_sd": float(tail.std())}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
