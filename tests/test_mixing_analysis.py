"""Host tests of the mixing analysis (g(r) normalisation, max[g], the
exponential fit, the acceptance estimate from work values); the pair counts
come from the oracle's histogram."""
import math

import numpy as np

from paper_2005_08348_amd import mixing, systems as S


def _random_leaflets(n, L, seed):
    """n two-bead molecules [head, PO4] uniformly in each of two leaflets"""
    rng = np.random.default_rng(seed)
    kh = S.Kind("H", [S.TYPE_N, S.TYPE_Q], [0.0, 0.0], [(0, 1, 0.47, 1250.0)], [], 0)
    pos, leaf = [], []
    for lf, z in ((0, 6.0), (1, 2.0)):
        xy = rng.uniform(0.0, L, size=(n, 2))
        for x, y in xy:
            pos += [[x, y, z + 0.47], [x, y, z]]
            leaf.append(lf)
    s = S.custom("gas", [kh], [0] * (2 * n), pos, [L, L, 9.0],
                 np.full((S.N_TYPES, S.N_TYPES), 2.0))
    return s, np.asarray(leaf, dtype=np.int32)


def test_ideal_gas_g_is_one(oracle_mod):
    n, L, w, nb = 900, 20.0, 0.25, 32
    s, leaf = _random_leaflets(n, L, 7)
    o = oracle_mod.Oracle(s)
    h = o.pair_histogram(0, 1, leaf, nb, w)
    r, g = mixing.g_of_r(h, [n, n], L * L, w)
    sel = r > 1.0                       # enough pairs per annulus
    assert abs(g[sel].mean() - 1.0) < 0.02
    assert np.abs(g[sel] - 1.0).max() < 0.15
    assert math.isclose(r[0], 0.5 * w)


def test_square_lattice_first_shell(oracle_mod):
    """8 x 8 lattice of spacing 1 in one leaflet: the first shell holds
    4 N / 2 pairs, so g there is that over the ideal count of its annulus."""
    kh = S.Kind("H", [S.TYPE_N, S.TYPE_Q], [0.0, 0.0], [(0, 1, 0.47, 1250.0)], [], 0)
    n, a, w = 8, 1.0, 0.07
    pos = []
    for i in range(n):
        for j in range(n):
            pos += [[i * a, j * a, 6.47], [i * a, j * a, 6.0]]
    s = S.custom("lat", [kh], [0] * (n * n), pos, [n * a, n * a, 9.0],
                 np.full((S.N_TYPES, S.N_TYPES), 2.0))
    leaf = np.zeros(n * n, dtype=np.int32)
    h = oracle_mod.Oracle(s).pair_histogram(0, 1, leaf, 40, w)
    _, g = mixing.g_of_r(h, [n * n], (n * a) ** 2, w)
    k = int(a / w)
    ideal = 0.5 * n * n * (n * n - 1) * math.pi * ((k + 1) ** 2 - k ** 2) * w * w / (n * a) ** 2
    assert math.isclose(g[k], (n * n * 4 / 2) / ideal, rel_tol=1e-12)
    assert mixing.max_g(h, [n * n], (n * a) ** 2, w) == g.max()


def test_fit_exponential_recovers_parameters():
    x = np.linspace(0, 40000, 41)
    rng = np.random.default_rng(3)
    y = 1.2 + 3.0 * np.exp(-x / 9000.0) + rng.normal(0, 0.01, size=x.shape)
    c, a, tau = mixing.fit_exponential(x, y)
    assert abs(c - 1.2) < 0.03 and abs(a - 3.0) < 0.05 and abs(tau / 9000.0 - 1) < 0.03


def test_acceptance_from_work():
    kT = 2.5
    w = np.array([0.0, kT * math.log(2.0), -5.0, kT * math.log(4.0)])
    assert math.isclose(mixing.acceptance_from_work(w, kT), (1 + 0.5 + 1 + 0.25) / 4, rel_tol=1e-12)


def test_fe_to_half():
    x = np.arange(10) * 1000.0
    y = np.array([2.2, 2.1, 1.9, 1.7, 1.5, 1.4, 1.3, 1.3, 1.2, 1.2])
    # half-way level 1.7; running means of 3: 2.067, 1.9, 1.7 -> ends at sample 4
    assert mixing.fe_to_half(x, y, 1.2) == 4000.0
    assert mixing.fe_to_half(x, np.full(10, 2.2), 1.2) is None


def test_summary_over_repeats():
    """Halfway medians, ranges and speed-up statistics over repeats, with a
    run that never reaches halfway left out of the statistics."""
    from paper_2005_08348_amd import mixing as X

    def rep(md_h, mc_h, da_h, y0=2.0):
        runs = {"md": {"fe_to_half": md_h, "accepted": 0, "tried": 0, "max_g": [y0, 1.5]},
                "mcmd": {"fe_to_half": mc_h, "accepted": 1, "tried": 100,
                         "speedup_half": (md_h / mc_h) if (md_h and mc_h) else None},
                "mdas": {"fe_to_half": da_h, "accepted": 3, "tried": 100,
                         "speedup_half": (md_h / da_h) if (md_h and da_h) else None}}
        return {"runs": runs, "mixed_level": 1.3}
    reps = [rep(100000.0, 2000.0, 10000.0), rep(120000.0, 3000.0, 20000.0), rep(None, 1000.0, 5000.0),
            rep(1000.0, 1000.0, 1000.0, y0=1.4)]   # start within MIN_GAP of the mixed level
    s = X.summarize(reps)
    assert s["repeats"] == 4 and s["without_signal"] == 1
    assert s["md"]["fe_to_half_median"] == 110000.0 and s["md"]["reached_half"] == "2/3"
    assert s["mcmd"]["fe_to_half_range"] == [1000.0, 3000.0]
    assert s["mcmd"]["speedup_half_n"] == 2
    assert abs(s["mcmd"]["speedup_half_mean"] - 45.0) < 1e-12
    assert abs(s["mcmd"]["speedup_half_sd"] - np.std([50.0, 40.0], ddof=1)) < 1e-12
    assert abs(s["mdas"]["speedup_half_mean"] - 8.0) < 1e-12
    assert abs(s["mdas"]["acceptance"] - 0.03) < 1e-12


def test_halfway_needs_a_gap():
    from paper_2005_08348_amd import mixing as X
    x = np.arange(10) * 100.0
    y = np.array([2.0, 1.9, 1.6, 1.5, 1.5, 1.4, 1.4, 1.4, 1.4, 1.4])
    assert X.fe_to_half(x, y, 1.3) == 400.0   # mean of samples 2..4 is the first <= 1.65
    assert X.fe_to_half(x, y, 1.9, min_gap=0.2) is None


def test_flipflop_inputs_and_crossing():
    from paper_2005_08348_amd import flipflop as F
    s = F.asymmetric_mix()
    lf = s.meta["leaflet"]
    assert np.all(s.mol_kind[lf == 0] == S.KIND_A) and np.all(s.mol_kind[lf == 1] == S.KIND_D)
    assert np.count_nonzero(lf == 0) == np.count_nonzero(lf == 1) == 200
    x = np.arange(6) * 10.0
    assert F.fe_to_fraction(x, [0, 0.1, 0.2, 0.3, 0.2, 0.4], 0.25) == 30.0
    assert F.fe_to_fraction(x, [0, 0.1, 0.1, 0.1, 0.1, 0.1], 0.25) is None
