"""Benchmark of the MC-MD / MDAS force and energy hot path on one MI355X.

Workload (one "step" = one MD step of the whole path: Verlet-list rebuild
every R steps, ghost refresh, nonbonded + bonded forces, BAOAB update):
the 4,096-lipid bilayer with 50,000 water beads (95,876 beads,
36.2 x 36.2 x 10 nm), float32 forces with float64 energies.  Side legs in
the same run: the float64 GPU form on the same system, batches of 256
exchange trials every 2 MD steps on it, and MDAS cycles (32 pairs, 50
lambda increments, 1 step each) on the 1.14M-bead bilayer.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32 = 157.3e12      # MI355X FP32 vector FLOP/s
PEAK_HBM = 8.0e12         # MI355X HBM3E B/s
FLOP_PAIR_F = 31          # algorithmic flops per in-cutoff pair, forces only
CALIB_BYTES = 512 << 20   # plain copy used to scale the HBM byte counters
NB_LAUNCHES = 200         # graph-replayed launches for the kernel duration
# the force pass and the list layout it walks (cell order, lane interleave)
KERNEL_SOURCES = ("paper_2005_08348_amd/csrc/k_force.hip", "paper_2005_08348_amd/csrc/membx_dev.h",
                  "paper_2005_08348_amd/csrc/k_list.hip")


WORKLOAD = {
    "c1": "bilayer 4096 lipids (A:B:C 1639:1638:819) + 50000 W, 95876 beads, box 36.2x36.2x10 nm, "
          "LJ+RF r_c 1.1 nm, Langevin BAOAB dt 20 fs",
    "c3": "bilayer 49152 lipids (A:B:C:D 30:30:20:20) + 590000 W, 1140504 beads, "
          "box 125.4x125.4x11 nm, LJ+RF r_c 1.1 nm, Langevin BAOAB dt 20 fs",
}


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(lpb, list_kind, skin, skin_inner):
    """HBM bytes per launch of the force pass from the counter summary
    profiles/k_nb_float_c1_traffic.md (FETCH_SIZE and WRITE_SIZE runs scaled
    by a plain copy of known size), one row per tuning; None when no row
    matches or the rows were taken on other kernel source."""
    path = os.path.join(ROOT, "profiles", "k_nb_float_c1_traffic.md")
    if not os.path.exists(path):
        return None
    sha, rows = None, []
    with open(path) as fh:
        for line in fh:
            if line.startswith("- kernel_source_sha256:"):
                sha = line.split(":", 1)[1].strip().strip("`")
            elif line.startswith("| ") and not line.startswith("| lanes") and not line.startswith("|---"):
                cells = [c.strip() for c in line.strip().strip("|").split("|")]
                try:
                    rows.append((int(cells[0]), int(cells[1]), float(cells[2]), float(cells[3]),
                                 float(cells[6])))
                except (ValueError, IndexError):
                    pass
    if sha != kernel_source_sha():
        return None
    for r in rows:
        if (r[0] == lpb and r[1] == list_kind and abs(r[2] - skin) < 1e-9
                and abs(r[3] - skin_inner) < 1e-9):
            return r[4]
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_system(sysm, precision, **tun):
    from paper_2005_08348_amd import membx as M
    return M.System(sysm, precision=precision, **tun)


def timed(fn, sync):
    sync()
    t0 = time.perf_counter()
    fn()
    sync()
    return time.perf_counter() - t0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sysm, target_s=10.0):
    """The float64 oracle (oracle/) on a bounded sample of the same system,
    on the host cores this process may use (OMP_NUM_THREADS when set; the
    oracle's nonbonded slabs run under OpenMP) and on one thread."""
    from oracle import oracle as O
    O.build()
    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        ncpu = min(ncpu, int(os.environ["OMP_NUM_THREADS"]))

    def rate(threads):
        O.threads(threads)
        o = O.Oracle(sysm)
        t0 = time.perf_counter()
        o.md_step(1)
        t1 = time.perf_counter() - t0
        n = max(1, min(400, int(target_s / max(t1, 1e-6))))
        t0 = time.perf_counter()
        o.md_step(n)
        dt = time.perf_counter() - t0
        return n / dt, n + 1, dt + t1
    r_all, n_all, t_all = rate(ncpu)
    used = O.threads(0)
    r_one, n_one, t_one = rate(1)
    O.threads(ncpu)
    return dict(value=r_all, unit="MD steps/s", cores=used, kind="oracle",
                sample=f"{n_all} float64 MD steps of the same 95,876-bead system on {used} "
                       f"threads ({t_all:.1f} s) and {n_one} on one thread ({t_one:.1f} s)",
                one_thread=r_one, host_cpus=os.cpu_count(), cpu_model=cpu_model())


def _serve(jobs, req, budget, arrivals=None, one_at_a_time=False):
    """Run jobs through one server.  arrivals: submit times (s from the
    start; None: all at once); one_at_a_time: each job is submitted when the
    previous one finished (sequential reference)."""
    import numpy as np
    import torch
    from paper_2005_08348_amd import membx as M
    srv = M.Server(budget)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, max_wait, max_res, nxt = [], 0, 0, 0
    last = t0
    while len(done) < len(jobs):
        now = time.perf_counter() - t0
        if one_at_a_time:
            if nxt == len(done) and nxt < len(jobs):
                srv.submit(jobs[nxt], **req)
                nxt += 1
        else:
            while nxt < len(jobs) and (arrivals is None or arrivals[nxt] <= now):
                srv.submit(jobs[nxt], **req)
                nxt += 1
        res, nres, nwait = srv.poll()
        done += res
        max_wait, max_res = max(max_wait, nwait), max(max_res, nres)
        if time.perf_counter() - last > 20:
            last = time.perf_counter()
            log(f"[bench] serving: {len(done)}/{len(jobs)} jobs done")
    wall = time.perf_counter() - t0
    cyc = srv.cycle_times()
    cpairs = srv.cycle_pairs()
    srv.close()
    bad = [r for r in done if r["status"] != 0]
    steps = sum(r["md_steps"] for r in done)
    pair_int = sum(r["pair_interactions"] for r in done)
    turn = np.array([r["finish_s"] - r["submit_s"] for r in done])
    wait = np.array([r["admit_s"] - r["submit_s"] for r in done])
    return {"jobs": len(done), "failed": len(bad), "budget_bytes": budget,
            "max_resident": max_res, "max_waiting": max_wait,
            "wall_s": wall, "jobs_per_s": len(done) / wall,
            "md_steps_per_s": steps / wall,
            # measured: each cycle's in-cutoff pair count (energy pass at the
            # cycle's end) times its MD steps, summed over all cycles
            "pair_interactions_per_s": pair_int / wall,
            "pair_interactions_cycle_sum_check": bool(abs(float(cpairs.sum()) - pair_int) < 0.5),
            "device_s_sum": float(cyc.sum()) / 1e3,
            "cycle_ms_p50": float(np.percentile(cyc, 50)), "cycle_ms_p99": float(np.percentile(cyc, 99)),
            "turnaround_s_p50": float(np.percentile(turn, 50)),
            "turnaround_s_p99": float(np.percentile(turn, 99)),
            "admission_wait_s_p50": float(np.percentile(wait, 50)),
            "admission_wait_s_p99": float(np.percentile(wait, 99)),
            "mdas_accepted": int(sum(r["mdas_accepted"] for r in done))}


def serving_leg(n_jobs, budget=2 << 30):
    """Serving: n_jobs bilayers with N log-uniform in [1.4k, 250k] beads, each
    relaxed (100 steepest-descent steps) at admission, then 4 cycles of 50 MD
    steps and 20 MDAS cycles (8 pairs, K 50, M 1), every cycle closed by a
    pair count.  Three runs of the same jobs through a server whose arena
    budget makes admission wait for finished jobs: one job at a time (the
    sequential capacity), Poisson arrivals at 0.8 x that capacity (seeded),
    and all jobs at once (the burst)."""
    import numpy as np
    from paper_2005_08348_amd import systems as S
    log(f"[bench] serving leg: building {n_jobs} jobs")
    jobs = S.serving_jobs(48)[:n_jobs]
    req = dict(minimize_iters=100, md_cycles=4, md_steps=50, mdas_cycles=20, mdas_pairs=8,
               mdas_k=50, mdas_m=1, count_pairs=True)
    _serve(jobs[:2], req, budget)                     # first admissions: code objects, graphs
    log("[bench] serving: sequential")
    seq = _serve(jobs, req, budget, one_at_a_time=True)
    rate = 0.8 * seq["jobs_per_s"]
    arrivals = np.cumsum(np.random.default_rng(200508348).exponential(1.0 / rate, size=len(jobs)))
    log(f"[bench] serving: Poisson arrivals at {rate:.2f} jobs/s")
    poi = _serve(jobs, req, budget, arrivals=arrivals)
    poi["arrival_rate_jobs_per_s"] = rate
    poi["last_arrival_s"] = float(arrivals[-1])
    log("[bench] serving: burst")
    burst = _serve(jobs, req, budget)
    return {"jobs": len(jobs), "beads_total": int(sum(s.n_beads for s in jobs)),
            "request": req, "sequential": seq, "poisson_0.8x": poi, "burst": burst,
            # share of the sequential run's wall time outside the cycles'
            # device time (admission with upload and minimiser, host polls,
            # launch gaps, closing queries): the most a persistent kernel
            # that keeps the cycles' arithmetic could recover there
            "sequential_outside_cycles_share": 1.0 - seq["device_s_sum"] / seq["wall_s"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-legs", action="store_true", help="main timed region only")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serving-jobs", type=int, default=48,
                    help="jobs of the serving leg (0: skip it)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use --skin/--rebuild/--lpb instead of the autotuner")
    ap.add_argument("--lpb", type=int, default=8, help="lanes per bead of the pair kernel")
    ap.add_argument("--rebuild", type=int, default=9, help="steps between list rebuilds")
    ap.add_argument("--skin", type=float, default=0.5)
    ap.add_argument("--skin-inner", type=float, default=0.15)
    ap.add_argument("--prune", type=int, default=3, help="force passes per inner-list prune")
    ap.add_argument("--mdas-cycles", type=int, default=0,
                    help="also time this many MDAS cycles (32 pairs, K = 50, M = 1) on the main "
                         "system after its timed region (for kernel profiles of the cycle)")
    ap.add_argument("--system", choices=["c1", "c3"], default="c1",
                    help="system of the main timed region (c3, the 1,140,504-bead MDAS bilayer, "
                         "for kernel profiles; use with --no-legs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2005_08348_amd import systems as S

    dev = torch.device("cuda:0")
    sync = torch.cuda.synchronize
    K, W = args.steps, args.warmup

    log(f"[bench] building {args.system}")
    c1 = S.make(args.system)
    tun = dict(skin=args.skin, rebuild_interval=args.rebuild, lanes_per_bead=args.lpb,
               skin_inner=args.skin_inner, prune_interval=args.prune)
    g = gpu_system(c1, "mixed", **tun)
    log("[bench] relaxing start structure on the GPU")
    g.minimize(100)
    relaxed = g.state()
    c1r = c1.copy()
    c1r.pos = relaxed["pos"]
    g.md_step(W)
    if not args.no_autotune:
        log("[bench] autotuning skin / rebuild interval / lanes per bead")
        tun = g.autotune(200)
        log(f"[bench] tuned: {tun}")
    # replay every step-sequence graph the timed region uses once, untimed:
    # the sequences are keyed by chunk length, steps since the last rebuild
    # and the coordinate buffer in use, which repeat within 2 R calls of K
    # steps (one call covers them when K spans many chunks)
    R = tun["rebuild_interval"]
    for _ in range(2 * R if K < 64 * R else 2):
        g.md_step(K)
    sync()
    # ---- main timed region (graph replay)
    log(f"[bench] timed region: {K} MD steps, mixed precision")
    t_main = timed(lambda: g.md_step(K), sync)
    e = g.energies(check=False)
    steps_s = K / t_main
    pairs = e["n_pairs_in_cutoff"]
    # ---- a plain copy of known size (3 launches of CALIB_BYTES): under a
    # counter profiler its FETCH_SIZE / WRITE_SIZE give the scale of those
    # counters in bytes
    src = torch.empty(CALIB_BYTES, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        g.calib_copy(dst, src, CALIB_BYTES)
    sync()
    del src, dst
    # ---- nonbonded kernel duration at the end state of the timed region:
    # NB_LAUNCHES launches replayed back to back from one HIP graph, HIP
    # events on the library stream around the replay
    nb_ms = g.kernel_bench(NB_LAUNCHES)
    e2 = g.energies(check=False)
    pairs2 = e2["n_pairs_in_cutoff"]
    slots = e2["n_list_entries"]   # Verlet-list entries (both directions)
    nb_flops = pairs2 * FLOP_PAIR_F
    achieved = nb_flops / (nb_ms * 1e-3)
    list_kind = 1 if tun["prune_interval"] > 1 else 0
    traffic = measured_traffic(tun["lanes_per_bead"], list_kind, tun["skin"],
                               tun["skin_inner"] if list_kind else 0.0) if args.system == "c1" else None
    result = {
        "metric": "MD steps/s & pair-interactions/s (FP32-mixed vs FP64); swap trials/s",
        "value": steps_s,
        "unit": "MD steps/s",
        "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": 1e3 * t_main / K,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (f64 energies)", "data": "synthetic",
        "config": {"workload": WORKLOAD[args.system],
                   "n_beads": c1.n_beads, "precision": "mixed",
                   "skin_nm": tun["skin"], "rebuild_interval": tun["rebuild_interval"],
                   "lanes_per_bead": tun["lanes_per_bead"],
                   "inner_skin_nm": tun["skin_inner"], "prune_interval": tun["prune_interval"]},
        "pair_interactions_per_s": pairs * steps_s,
        "pairs_in_cutoff": pairs,
        "skin_violations": e2["n_skin_violations"],
        "max_displacement_nm": e2["max_displacement"],
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32, "traffic": traffic,
                     "kernel": f"k_nb<float,{tun['lanes_per_bead']},false,1,{list_kind}> "
                               "(nonbonded + bonded forces + next step's B-A-O-A)",
                     "launches_timed": NB_LAUNCHES, "mean_launch_ms": nb_ms,
                     "flop_per_launch": nb_flops,
                     # computed pair slots of the Verlet list (each unordered
                     # pair twice, masked slots included) and the share of
                     # them within the cutoff; the same 31 flop per slot
                     # gives the throughput of all computed slots
                     "pair_slots_verlet": slots,
                     "slot_efficiency": (2 * pairs2 / slots) if slots else None,
                     "slot_tflops": slots * FLOP_PAIR_F / (nb_ms * 1e-3) / 1e12},
    }
    if args.mdas_cycles > 0:
        log(f"[bench] {args.mdas_cycles} MDAS cycles (32 pairs, K = 50, M = 1) on the main system")
        g.mdas_cycle(32, 50, 1, results=False)
        tcy = timed(lambda: [g.mdas_cycle(32, 50, 1, results=False)
                             for _ in range(args.mdas_cycles)], sync)
        result["mdas_main"] = {"pairs": 32, "k_increments": 50, "m_steps": 1,
                               "cycles": args.mdas_cycles, "cycles_per_s": args.mdas_cycles / tcy}
    g.close()
    del g
    torch.cuda.empty_cache()

    if not args.no_legs:
        # ---- float64 GPU form on the same relaxed system
        log("[bench] float64 leg")
        g64 = gpu_system(c1r, "fp64", **tun)
        g64.md_step(50)
        tun64 = tun if args.no_autotune else g64.autotune(200)
        k64 = max(100, K // 4)
        t64 = timed(lambda: g64.md_step(k64), sync)
        e64 = g64.energies(check=False)
        result["fp64"] = {"md_steps_per_s": k64 / t64, "tuning": tun64,
                          "skin_violations": e64["n_skin_violations"],
                          "pair_interactions_per_s": e64["n_pairs_in_cutoff"] * k64 / t64,
                          "mixed_speedup": steps_s / (k64 / t64)}
        # exchange batches of the float64 form (256 trials every 2 steps)
        g64.md_step(20)
        g64.swap_trials(256, results=False)
        nb64 = 20

        def run_swaps64():
            for _ in range(nb64):
                g64.md_step(2)
                g64.swap_trials(256, results=False)
        tsw64 = timed(run_swaps64, sync)
        r64 = g64.swap_trials(256)
        result["fp64"]["swap"] = {"batches": nb64, "batch_plus_2_steps_ms": 1e3 * tsw64 / nb64,
                                  "admitted_last_batch": len(r64["du"]),
                                  "trials_per_s": nb64 * len(r64["du"]) / tsw64}
        # energy error of the mixed form on the identical state
        gm = gpu_system(c1r, "mixed", **tun)
        em, ef = gm.energies(check=False), None
        g64.set_state(pos=c1r.pos, vel=c1r.vel)
        ef = g64.energies(check=False)
        result["fp64"]["mixed_energy_rel_err"] = abs(em["potential"] - ef["potential"]) / abs(ef["potential"])
        g64.close(); del g64
        # ---- exchange batches on the same system (256 trials every 2 steps)
        log("[bench] exchange-trial leg")
        gm.md_step(20)
        gm.swap_trials(256, results=False)
        nb = 50
        adm = acc = 0

        def run_swaps():
            for _ in range(nb):
                gm.md_step(2)
                gm.swap_trials(256, results=False)
        tsw = timed(run_swaps, sync)
        r = gm.swap_trials(256)
        gm.md_step(2)
        result["swap"] = {"batches": nb, "trials_per_batch_requested": 256,
                          "admitted_last_batch": len(r["du"]),
                          "accepted_last_batch": int(r["n_accepted"]),
                          "batch_plus_2_steps_ms": 1e3 * tsw / nb,
                          "trials_per_s": nb * len(r["du"]) / tsw}
        if "swap" in result["fp64"]:
            result["swap"]["mixed_speedup_vs_fp64"] = (result["swap"]["trials_per_s"] /
                                                       result["fp64"]["swap"]["trials_per_s"])
        # ---- the paper's thermostat: velocity rescaling, tau_t 1 ps,
        # membrane and solvent in two coupling groups (two launches per
        # step instead of one: the update, which draws and applies the
        # previous step's factors, and the force pass with the closing
        # half-kick and the kinetic-energy sums)
        log("[bench] velocity-rescaling leg")
        groups = [1 if k.name == "W" else 0 for k in c1.kinds]
        t_lang = 2.0 * gm.energies(check=False)["kinetic"] / (3 * c1.n_beads * S.KB)
        gm.set_ensemble(1, tau_t=1.0, kind_group=groups)
        gm.md_step(20)
        kvr = max(100, K // 4)
        tvr = timed(lambda: gm.md_step(kvr), sync)
        evr = gm.energies(check=False)
        result["vrescale"] = {"md_steps_per_s": kvr / tvr, "tau_t_ps": 1.0,
                              "groups": "membrane, solvent",
                              "temperature_K": 2.0 * evr["kinetic"] / (3 * c1.n_beads * S.KB),
                              "temperature_K_langevin_before": t_lang,
                              "skin_violations": evr["n_skin_violations"],
                              "vs_langevin": (kvr / tvr) / steps_s}
        # the paper's full ensemble: plus the semi-isotropic barostat at 1 bar
        # (tau_p 12 ps, compressibility 3e-4 / bar), coupling every 10 steps
        gm.set_barostat(10, p_ref_bar=1.0, compressibility=3e-4, tau_p=12.0)
        gm.md_step(20)
        tnpt = timed(lambda: gm.md_step(kvr), sync)
        enpt = gm.energies(check=False)
        result["vrescale"]["npt"] = {"md_steps_per_s": kvr / tnpt, "coupling_interval": 10,
                                     "box_nm": [float(x) for x in gm.box()],
                                     "pressure_bar": [float(x) for x in enpt["pressure"]],
                                     "skin_violations": enpt["n_skin_violations"]}
        gm.set_barostat(0)
        gm.set_ensemble(0)
        gm.close(); del gm
        torch.cuda.empty_cache()
        # ---- MDAS on the 1.14M-bead bilayer
        log("[bench] building c3 (1,140,504 beads)")
        c3 = S.make("c3")
        g3 = gpu_system(c3, "mixed", **tun)
        g3.minimize(60)
        g3.md_step(20)
        tun3 = tun if args.no_autotune else g3.autotune(100)
        g3.mdas_cycle(32, 50, 1, results=False)
        ncyc = 4
        t3 = timed(lambda: [g3.mdas_cycle(32, 50, 1, results=False) for _ in range(ncyc)], sync)
        r3 = g3.mdas_cycle(32, 50, 1)
        k3 = 200
        t3md = timed(lambda: g3.md_step(k3), sync)
        e3 = g3.energies(check=False)
        result["mdas"] = {"n_beads": c3.n_beads, "pairs": 32, "k_increments": 50, "m_steps": 1,
                          "tuning": tun3, "skin_violations": e3["n_skin_violations"],
                          "cycles_per_s": ncyc / t3, "last_work_kJmol": r3["work"],
                          "last_accepted": r3["accept"],
                          "md_steps_per_s": k3 / t3md,
                          "pair_interactions_per_s": e3["n_pairs_in_cutoff"] * k3 / t3md}
        # the soft-core lambda path (Eq. 4): the same cycles with the changed
        # beads' LJ switched through soft-core terms (two extra small kernels
        # per step and per increment)
        g3.set_mdas_path(1, 0.05)
        g3.mdas_cycle(32, 50, 1, results=False)
        tsc = timed(lambda: [g3.mdas_cycle(32, 50, 1, results=False) for _ in range(ncyc)], sync)
        rsc = g3.mdas_cycle(32, 50, 1)
        result["mdas"]["soft_core"] = {"cycles_per_s": ncyc / tsc, "delta_nm2": 0.05,
                                       "last_work_kJmol": rsc["work"], "last_accepted": rsc["accept"]}
        g3.set_mdas_path(0)
        g3.close(); del g3
        torch.cuda.empty_cache()

    if not args.no_legs and args.serving_jobs > 0:
        result["serving"] = serving_leg(args.serving_jobs)

    if not args.no_cpu:
        log("[bench] cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(c1r)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
