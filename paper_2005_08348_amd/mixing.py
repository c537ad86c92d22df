"""Mixing analysis and the sampler comparison of the paper's Results.

The paper follows the mixing of a two-lipid bilayer through the pair
correlation g(r) of the PO4 beads of one lipid type: its highest peak,
max[g(r)], decays towards the value of a uniformly mixed membrane, and an
exponential fitted to that decay against the number of force evaluations
gives each sampler's relaxation rate; the ratio of rates is the speed-up per
force evaluation of MC-MD or MDAS over straightforward MD.  It also
estimates an acceptance probability from the recorded work values.

Here g(r) is the lateral (in-plane) correlation within each leaflet, from
the GPU pair histogram (``System.pair_histogram``), normalised by the ideal
two-dimensional expectation of each leaflet.

    python -m paper_2005_08348_amd.mixing [--fe 200000] [--every 4000]
                                          [--thermostat vrescale] [--repeats 4]

runs MD, MC-MD and MDAS from the same far-from-mixed start (the ``mix``
bilayer: 400 lipids in stripes) and prints one JSON line with the traces,
the fits and the speed-ups.  Force evaluations are counted as the paper
does: one per MD step, per exchange trial and per MDAS step (a frozen MDAS
cycle, M = 0, counts one).  With ``--thermostat vrescale`` every sampler
integrates with the paper's thermostat (velocity rescaling, tau_t = 1 ps,
membrane and solvent coupled separately) instead of Langevin dynamics, and
``--thermostat npt`` adds the overdamped semi-isotropic barostat at 1 bar
(tau_p 12 ps), and ``--thermostat paper`` is the paper's ensemble: 335 K,
velocity rescaling and the semi-isotropic Parrinello-Rahman barostat (1 bar,
tau_p 12 ps), switched on after the uncounted equilibration, which runs
under the overdamped barostat;
``--repeats`` runs independent seeds and summarises the halfway speed-ups
(mean and standard deviation over the runs); ``--combine`` summarises the
repeats of several earlier outputs together.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import systems as S


# ---------------------------------------------------------------- analysis
def g_of_r(counts, n_per_leaflet, area, bin_width):
    """g(r) at the bin centres from lateral pair counts within leaflets:
    counts over the number of pairs an ideal 2-D gas of the same densities
    would put in each annulus, sum over leaflets of n (n - 1) / 2 times the
    annulus area over the leaflet area."""
    counts = np.asarray(counts, dtype=np.float64)
    k = np.arange(len(counts), dtype=np.float64)
    annulus = math.pi * ((k + 1.0) ** 2 - k ** 2) * bin_width ** 2
    pairs = sum(0.5 * n * (n - 1) for n in n_per_leaflet)
    expected = pairs * annulus / area
    g = np.divide(counts, expected, out=np.zeros_like(counts), where=expected > 0)
    r = (k + 0.5) * bin_width
    return r, g


def max_g(counts, n_per_leaflet, area, bin_width, r_min=0.0):
    """the highest peak of g(r) at r >= r_min (the sparse bins below the
    contact distance only carry noise)"""
    r, g = g_of_r(counts, n_per_leaflet, area, bin_width)
    return float(g[r >= r_min].max())


def fe_to_half(x, y, y_mixed, smooth=3, min_gap=0.0):
    """Force evaluations until the running mean (over `smooth` samples) of
    the trace first falls halfway from its start to the mixed level; None if
    it never does within the run, or if the start lies less than `min_gap`
    above the mixed level (no signal to follow)."""
    y = np.asarray(y, dtype=np.float64)
    if len(y) < smooth or y[0] - y_mixed < min_gap:
        return None
    ys = np.convolve(y, np.ones(smooth) / smooth, mode="valid")
    half = 0.5 * (y[0] + y_mixed)
    hit = np.nonzero(ys <= half)[0]
    return float(x[hit[0] + smooth - 1]) if len(hit) else None


def fit_exponential(x, y):
    """Least-squares fit y = c + a exp(-x / tau); returns (c, a, tau) or
    None when the fit does not converge."""
    from scipy.optimize import curve_fit
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    span = max(float(x.max() - x.min()), 1.0)
    p0 = (float(y[-1]), float(y[0] - y[-1]), span / 3.0)

    def f(t, c, a, tau):
        return c + a * np.exp(-t / tau)
    try:
        p, _ = curve_fit(f, x, y, p0=p0, bounds=([-np.inf, -np.inf, 1e-9], [np.inf, np.inf, np.inf]),
                         maxfev=20000)
    except (RuntimeError, ValueError):
        return None
    return float(p[0]), float(p[1]), float(p[2])


def acceptance_from_work(w, kT):
    """Acceptance estimated from work values: the mean of min(1, exp(-w/kT))."""
    w = np.asarray(w, dtype=np.float64)
    return float(np.mean(np.minimum(1.0, np.exp(-w / kT)))) if len(w) else float("nan")


# -------------------------------------------------------------- experiment
R_MIN = 0.5      # nm, the peak search starts here
BIN = 0.1        # nm
N_BINS = 45      # up to 4.5 nm
# MD steps before counting starts (400 ps at 20 fs): the lattice order of the
# synthetic start melts within them, while lateral diffusion (~0.1 nm in that
# time) leaves the stripes in place, so the traces follow demixing only
EQUIL = 20000
PAPER_T = 335.0  # K, the temperature of the paper's runs (Methods)
# the halfway metric needs the start clearly above the mixed level: max[g] of
# 100 lipids per leaflet scatters by about 0.1 between samples
MIN_GAP = 0.2


def _trace_point(g, sysm, kind, leaflet, n_bins, bin_width):
    mk = g.state()["mol_kind"]
    n_leaf = [int(np.count_nonzero((mk == kind) & (leaflet == lf))) for lf in (0, 1)]
    h = g.pair_histogram(kind, S.PO4, leaflet, n_bins, bin_width)
    box = g.box()                       # changes under pressure coupling
    return max_g(h, n_leaf, box[0] * box[1], bin_width, R_MIN)


def run(method, sysm, fe_total, every, kind=S.KIND_D, n_bins=N_BINS, bin_width=BIN,
        mc_trials=8, mc_steps=2, mdas_pairs=1, mdas_k=50, mdas_m=1, mdas_md=50, precision="mixed",
        thermostat="langevin", equil=EQUIL):
    """One sampler from the start structure after `equil` MD steps that are
    not counted: (force evaluations, max[g]) pairs every `every` force
    evaluations, plus acceptance counts and works."""
    from . import membx as M
    leaflet = sysm.meta["leaflet"]
    g = M.System(sysm, precision=precision)
    if thermostat in ("vrescale", "npt", "paper"):
        g.set_ensemble(1, tau_t=1.0, kind_group=[1 if k.name == "W" else 0 for k in sysm.kinds])
    if thermostat == "npt":   # and the semi-isotropic barostat at 1 bar
        g.set_barostat(10, p_ref_bar=1.0, compressibility=3e-4, tau_p=12.0)
    if thermostat == "paper":   # overdamped towards 1 bar while equilibrating
        g.set_barostat(10, p_ref_bar=1.0, compressibility=3e-4, tau_p=1.0)
    g.minimize(100)
    g.md_step(max(equil, 200))           # thermalise (not counted)
    if thermostat == "paper":   # then the paper's Parrinello-Rahman coupling
        g.set_barostat_pr(10, p_ref_bar=1.0, compressibility=3e-4, tau_p=12.0)
    fe, trace, works, acc, tried = 0, [], [], 0, 0
    trace.append((0, _trace_point(g, sysm, kind, leaflet, n_bins, bin_width)))
    next_pt = every
    t0 = time.perf_counter()
    stopped = None

    def advance():
        """one unit of the sampler; returns (force evaluations, trials, accepted)"""
        if method == "md":
            g.md_step(every)
            return every, 0, 0
        if method == "mcmd":
            r = g.swap_trials(mc_trials)
            g.md_step(mc_steps)
            n = len(r["accept"])
            return n + mc_steps, n, int(np.count_nonzero(r["accept"]))
        if method == "mdas":
            g.md_step(mdas_md)
            r = g.mdas_cycle(mdas_pairs, mdas_k, mdas_m)
            works.append(r["work"])
            return mdas_md + (mdas_k * mdas_m if mdas_m > 0 else 1), 1, int(r["accept"])
        raise ValueError(method)

    while fe < fe_total:
        try:
            dfe, dt, da = advance()
            fe += dfe
            tried += dt
            acc += da
            if fe >= next_pt:
                trace.append((fe, _trace_point(g, sysm, kind, leaflet, n_bins, bin_width)))
                next_pt += every
        except M.MembxError as ex:   # e.g. a box the barostat shrank below three list radii
            stopped = f"stopped at {fe} FE: {ex}"
            break
    wall = time.perf_counter() - t0
    g.close()
    return dict(method=method, trace=trace, accepted=acc, tried=tried, works=works, wall_s=wall,
                stopped=stopped)


def experiment(seed, fe_total, every, thermostat="langevin", equil=EQUIL):
    """MD, MC-MD and MDAS from the striped start of one seed, with the mixed
    level from the randomly mixed start of the same seed."""
    sysm = S.make("mix", seed=seed)
    if thermostat == "paper":
        sysm.temperature = PAPER_T
    kT = S.KB * sysm.temperature
    out = {"seed": int(sysm.seed), "runs": {}}
    # the level of a uniformly mixed membrane: the same lipids randomly mixed
    mixed = S.make("mix", seed=seed, demix=False)
    mixed.temperature = sysm.temperature
    ref = run("md", mixed, max(fe_total // 10, 4 * every), every, thermostat=thermostat, equil=equil)
    y_mixed = float(np.mean([p[1] for p in ref["trace"]]))
    out["mixed_level"] = y_mixed
    for method in ("md", "mcmd", "mdas"):
        print(f"[mixing] seed {out['seed']} {method}", file=sys.stderr, flush=True)
        r = run(method, sysm, fe_total, every, thermostat=thermostat, equil=equil)
        x = np.array([p[0] for p in r["trace"]], dtype=np.float64)
        y = np.array([p[1] for p in r["trace"]], dtype=np.float64)
        entry = {"fe": x.tolist(), "max_g": y.tolist(), "stopped": r["stopped"],
                 "accepted": r["accepted"], "tried": r["tried"], "wall_s": r["wall_s"]}
        if method == "mdas":
            entry["acceptance_from_work"] = acceptance_from_work(r["works"], kT)
        out["runs"][method] = entry
    return halfway_metrics(out, fe_total)


def halfway_metrics(out, fe_total):
    """Fits, force evaluations to halfway and the speed-ups per force
    evaluation of one repeat, from its traces and mixed level: the ratio of
    fitted decay constants (when both fits decay within the run), and the
    ratio of force evaluations to reach halfway to the mixed level (a lower
    bound when MD never does)."""
    for e in out["runs"].values():
        x = np.asarray(e["fe"], dtype=np.float64)
        y = np.asarray(e["max_g"], dtype=np.float64)
        e["fit_c_a_tau"] = fit_exponential(x, y)
        e["fe_to_half"] = fe_to_half(x, y, out["mixed_level"], min_gap=MIN_GAP)
    md = out["runs"]["md"]
    f_md = md["fit_c_a_tau"]
    tau_md = f_md[2] if (f_md and f_md[2] < 3 * fe_total) else None
    for method in ("mcmd", "mdas"):
        e = out["runs"][method]
        f = e["fit_c_a_tau"]
        e["speedup_fit"] = tau_md / f[2] if (tau_md and f and 0 < f[2] < 3 * fe_total) else None
        h = e["fe_to_half"]
        e["speedup_half"] = (md["fe_to_half"] / h) if (h and md["fe_to_half"]) else None
        e["speedup_half_lower_bound"] = fe_total / h if (h and not md["fe_to_half"]) else None
    return out


def summarize(reps):
    """Per sampler over the repeats: force evaluations to halfway (median,
    range, how many runs got there), acceptance, and the halfway speed-ups
    (mean and sample standard deviation; lower bounds where MD did not get
    halfway).  Repeats whose start lies less than MIN_GAP above their mixed
    level carry no signal and are counted apart."""
    def signal(r):
        y = r["runs"]["md"].get("max_g")
        return y is None or y[0] - r["mixed_level"] >= MIN_GAP
    good = [r for r in reps if signal(r)]
    summ = {"repeats": len(reps), "without_signal": len(reps) - len(good)}
    for method in ("md", "mcmd", "mdas"):
        h = [r["runs"][method]["fe_to_half"] for r in good]
        hh = [v for v in h if v]
        e = {"fe_to_half_median": float(np.median(hh)) if hh else None,
             "fe_to_half_range": [min(hh), max(hh)] if hh else None,
             "reached_half": f"{len(hh)}/{len(h)}",
             "acceptance": float(np.mean([r["runs"][method]["accepted"] / r["runs"][method]["tried"]
                                          for r in reps])) if method != "md" else None}
        if method != "md":
            sp = [r["runs"][method]["speedup_half"] for r in good if r["runs"][method]["speedup_half"]]
            lb = [r["runs"][method]["speedup_half_lower_bound"] for r in good
                  if r["runs"][method].get("speedup_half_lower_bound")]
            e["speedup_half_mean"] = float(np.mean(sp)) if sp else None
            e["speedup_half_sd"] = float(np.std(sp, ddof=1)) if len(sp) > 1 else None
            e["speedup_half_n"] = len(sp)
            e["speedup_half_lower_bounds"] = lb
        summ[method] = e
    return summ


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--fe", type=int, default=200000, help="force evaluations per sampler")
    ap.add_argument("--every", type=int, default=4000, help="force evaluations between g(r) samples")
    ap.add_argument("--seed", type=int, default=None, help="first seed (default: the mix workload's)")
    ap.add_argument("--repeats", type=int, default=1, help="independent runs, seeds seed, seed + 1, ...")
    ap.add_argument("--thermostat", choices=["langevin", "vrescale", "npt", "paper"], default="langevin",
                    help="vrescale: velocity rescaling; npt: plus the overdamped barostat; paper: 335 K, velocity rescaling and Parrinello-Rahman (the paper's ensemble)")
    ap.add_argument("--equil", type=int, default=EQUIL, help="uncounted MD steps before each run")
    ap.add_argument("--combine", nargs="+", metavar="JSON",
                    help="no runs: summarise the repeats of earlier outputs of this program")
    args = ap.parse_args(argv)
    if args.combine:
        reps, fe = [], None
        for path in args.combine:
            with open(path) as fh:
                d = json.loads(fh.read().strip().splitlines()[-1])
            if fe is not None and d["fe"] != fe:
                raise SystemExit("outputs with different --fe cannot be combined")
            fe = d["fe"]
            reps += [halfway_metrics(r, fe) for r in d["repeats"]]
        print(json.dumps({"combined": args.combine, "seeds": [r["seed"] for r in reps],
                          "summary": summarize(reps)}))
        return
    seed0 = S.SEEDS["mix"] if args.seed is None else args.seed
    reps = [experiment(seed0 + r, args.fe, args.every, args.thermostat, args.equil)
            for r in range(args.repeats)]
    out = {"system": "mix: 400 lipids (A:D 1:1) in stripes + 4000 W, 11.31 x 11.31 x 9 nm",
           "observable": f"max g(r) at r >= {R_MIN} nm, lateral PO4-PO4 of kind D within leaflets, "
                         f"bins {BIN} nm",
           "samplers": "MD; MC-MD: 8 exchange trials per batch + 2 MD steps; MDAS: 1 pair, "
                       "K = 50, M = 1, after 50 MD steps",
           "fe_counting": "1 per MD step, per exchange trial and per MDAS step",
           "thermostat": args.thermostat, "fe": args.fe, "every": args.every,
           "equil_md_steps": args.equil,
           "summary": summarize(reps), "repeats": reps}
    # the single-run layout of earlier versions: the first repeat at the top level
    out["mixed_level"] = reps[0]["mixed_level"]
    out["runs"] = reps[0]["runs"]
    print(json.dumps(out))


if __name__ == "__main__":
    main()
