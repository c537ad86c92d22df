"""Pins of the float64 CPU oracle against facts that do not come from the
oracle itself: closed forms of the potential, invariants of the mechanics,
brute force, an independent library implementation of the random number
generator, the paper's special cases and exact statistics of small toys.

Each test names the passage of the paper (or the definition) it pins."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2005_08348_amd import systems as S

KB = 0.00831446261815324
RC = 1.1


@pytest.fixture(scope="module")
def c0(oracle_mod):
    s = S.make("c0")
    return s


@pytest.fixture(scope="module")
def c0_relaxed(oracle_mod, c0):
    o = oracle_mod.Oracle(c0)
    o.minimize(60)
    st = o.state()
    s = c0.copy()
    s.pos = st["pos"].astype(np.float32).astype(np.float64) % s.box
    return s


# ------------------------------------------------------------ Philox4x32-10
ROCRAND_SRC = os.path.join(os.path.dirname(__file__), "rocrand_philox_ref.cpp")


def _rocrand_blocks(ctrs_keys, tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path / "rr_ref")
    subprocess.check_call([hipcc, "-O1", "-o", exe, ROCRAND_SRC], cwd=str(tmp_path))
    inp = "\n".join(" ".join(str(int(v)) for v in row) for row in ctrs_keys) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    return np.array([[int(t) for t in line.split()] for line in out.strip().splitlines()],
                    dtype=np.uint64)


def test_philox_matches_rocrand(oracle_mod, tmp_path):
    """Philox4x32-10 (Salmon et al., SC'11) against rocRAND's implementation,
    called as a black box, on random counters and keys."""
    rng = np.random.default_rng(7)
    rows = []
    for _ in range(200):
        c = rng.integers(0, 2**32, size=4, dtype=np.uint64)
        c[1] = c[1] % (2**30)   # rocRAND takes the low counter words as 4*offset
        k = rng.integers(0, 2**32, size=2, dtype=np.uint64)
        rows.append(list(c) + list(k))
    rows.append([0, 0, 0, 0, 0, 0])
    ref = _rocrand_blocks(rows, tmp_path)
    for row, r in zip(rows, ref):
        got = oracle_mod.philox(row[:4], row[4:])
        assert list(map(int, got)) == list(map(int, r)), row


def test_box_muller_special_values(oracle_mod):
    """u1 = 1 gives radius 0; u2 = 1/4 puts the pair on the sine axis."""
    g = oracle_mod.gauss3([0xFFFFFFFF, 123, 0xFFFFFFFF, 5])
    assert np.all(np.abs(g) < 1e-12)
    # u1 = e^{-1/2}: radius 1; u2 = 2^30/2^32 = 1/4: (cos, sin) = (0, 1)
    w0 = int(round(math.exp(-0.5) * 2**32)) - 1
    g = oracle_mod.gauss3([w0, 2**30, w0, 0])
    r = math.sqrt(-2 * math.log((w0 + 1) / 2**32))
    assert abs(g[0]) < 1e-9 and abs(g[1] - r) < 1e-12 and abs(g[2] - r) < 1e-12


def test_gaussian_moments(oracle_mod):
    """Box-Muller output of Philox blocks is standard normal (statistical)."""
    gs = []
    for i in range(20000):
        w = oracle_mod.philox([i, 3, 0, 0], [11, 12])
        gs.append(oracle_mod.gauss3(w))
    g = np.array(gs).ravel()
    n = g.size
    assert abs(g.mean()) < 5 / math.sqrt(n)
    assert abs(g.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    assert abs(np.mean(g**4) - 3.0) < 0.1


# ------------------------------------------------------- pair potential (P1, P2)
def _eps_sigma_system(oracle_mod, eps_val):
    eps = np.full((S.N_TYPES, S.N_TYPES), eps_val)
    k = S.Kind("P", [0], [0.0], [], [], -1)
    s = S.custom("pair", [k, k], [0, 1], [[1, 1, 1], [2, 1, 1]], [6, 6, 6], eps)
    return oracle_mod.Oracle(s)


@pytest.mark.parametrize("eps_val", [5.6, 2.0])
def test_lj_closed_forms(oracle_mod, eps_val):
    """Potential-shifted LJ 12-6 with 1.1 nm cutoff (Section 3): minimum at
    r = 2^(1/6) sigma with depth -eps minus the shift, zero at the cutoff,
    force at the cutoff equal to the plain LJ force there."""
    o = _eps_sigma_system(oracle_mod, eps_val)
    sig = S.SIGMA
    rmin = 2 ** (1 / 6) * sig
    shift = 4 * eps_val * ((sig / RC) ** 12 - (sig / RC) ** 6)
    vlj, vrf, fs = o.pair_term(0, 0, 0.0, 0.0, rmin * rmin)
    assert abs(vlj - (-eps_val - shift)) < 1e-12
    assert abs(fs) < 1e-10 and vrf == 0.0
    vlj, _, fs = o.pair_term(0, 0, 0.0, 0.0, RC * RC * (1 - 1e-15))
    assert abs(vlj) < 1e-12
    f_cut = 24 * eps_val / RC * (2 * (sig / RC) ** 12 - (sig / RC) ** 6)
    assert abs(fs * RC - f_cut) < 1e-10
    if eps_val == 5.6:
        assert abs(f_cut - (-0.734)) < 2e-3          # the worked number at eps 5.6
        assert abs(shift - (-0.135465)) < 1e-6


def test_lj_force_is_minus_derivative(oracle_mod):
    o = _eps_sigma_system(oracle_mod, 4.0)
    for r in [0.45, 0.55, 0.8, 1.05]:
        h = 1e-6
        vp = o.pair_term(0, 0, 0, 0, (r + h) ** 2)[0]
        vm = o.pair_term(0, 0, 0, 0, (r - h) ** 2)[0]
        fs = o.pair_term(0, 0, 0, 0, r * r)[2]
        assert abs(-(vp - vm) / (2 * h) - fs * r) < 1e-6 * max(1, abs(fs * r))


def test_reaction_field_closed_forms(oracle_mod):
    """Reaction field with eps_r = 15 and eps_rf = infinity (Section 3):
    energy and force vanish at the cutoff; +1/-1 at 0.47 nm gives
    -7.8453 kJ/mol."""
    o = _eps_sigma_system(oracle_mod, 0.0)
    v = o.pair_term(0, 0, 1.0, -1.0, 0.47 ** 2)
    assert abs(v[1] - (-7.8453)) < 1e-4
    vc = o.pair_term(0, 0, 1.0, -1.0, RC * RC * (1 - 1e-15))
    assert abs(vc[1]) < 1e-12 and abs(vc[2]) < 1e-10
    # Coulomb part alone at short range dominates: r -> small, V ~ f q q / (eps_r r)
    r = 1e-3
    v = o.pair_term(0, 0, 1.0, 1.0, r * r)
    assert abs(v[1] * r * 15 / 138.935458 - 1.0) < 2e-3


# ------------------------------------------------------------- bonded (P3)
def _bonded_toy(oracle_mod, pos, angle=False):
    eps = np.zeros((S.N_TYPES, S.N_TYPES))
    kb = 0.0 if angle else 1250.0       # angle toys: bonds carry no force
    bonds = [(0, 1, 0.47, kb)] + ([(1, 2, 0.47, kb)] if angle else [])
    angles = [(0, 1, 2, 180.0, 25.0)] if angle else []
    n = 3 if angle else 2
    k = S.Kind("T", [0] * n, [0.0] * n, bonds, angles, -1)
    s = S.custom("b", [k], [0], pos, [8, 8, 8], eps)
    return oracle_mod.Oracle(s)


def test_bond_closed_form(oracle_mod):
    for dlt in [0.03, -0.05]:
        r = 0.47 + dlt
        o = _bonded_toy(oracle_mod, [[1, 1, 1], [1 + r, 1, 1]])
        dlt = float(np.float32(1 + r)) - 1.0 - 0.47   # inputs are float32 values
        e = o.energy_forces(cells=False)
        assert abs(e["bond"] - 0.5 * 1250 * dlt * dlt) < 1e-9
        # the pair of beads feels -k (r - b0) along the bond
        assert abs(e["force"][1, 0] - (-1250 * dlt)) < 1e-6
        assert abs(e["force"][0, 0] - (1250 * dlt)) < 1e-6


def test_angle_closed_forms(oracle_mod):
    """cos^2 angle with theta0 = 180 deg: zero energy and force when straight;
    1/2 k at 90 degrees (cos = 0)."""
    o = _bonded_toy(oracle_mod, [[1, 1, 1], [1.47, 1, 1], [1.94, 1, 1]], angle=True)
    e = o.energy_forces(cells=False)
    assert abs(e["angle"]) < 1e-12 and np.abs(e["force"]).max() < 1e-8
    o = _bonded_toy(oracle_mod, [[1, 1, 1], [1.47, 1, 1], [1.47, 1.47, 1]], angle=True)
    e = o.energy_forces(cells=False)
    assert abs(e["angle"] - 0.5 * 25.0) < 1e-9
    # at 90 degrees d(cos)/dx_i = x_k-direction unit / |u| -> |F_i| = k / |u|
    u = float(np.float32(1.47)) - 1.0          # inputs are float32 values
    assert abs(np.linalg.norm(e["force"][0]) - 25.0 / u) < 1e-9


# ----------------------------------------------------- invariants (P5-P8)
def test_cells_equal_all_pairs(oracle_mod, c0):
    o = oracle_mod.Oracle(c0)
    a = o.energy_forces(cells=False)
    b = o.energy_forces(cells=True)
    assert a["n_pairs"] == b["n_pairs"]
    for k in ["lj", "rf", "bond", "angle"]:
        assert abs(a[k] - b[k]) <= 1e-11 * max(1.0, abs(a[k]))
    assert np.abs(a["force"] - b["force"]).max() < 1e-9
    pa = o.pairset(1.3, cells=False)
    pb = o.pairset(1.3, cells=True)
    sa = set(map(tuple, np.sort(pa, axis=1)))
    sb = set(map(tuple, np.sort(pb, axis=1)))
    assert sa == sb and len(sa) == len(pa)


def test_net_force_zero(oracle_mod, c0):
    o = oracle_mod.Oracle(c0)
    f = o.energy_forces()["force"]
    assert np.abs(f.sum(axis=0)).max() <= 1e-12 * np.abs(f).sum()


def test_forces_are_minus_gradient(oracle_mod, c0_relaxed):
    o = oracle_mod.Oracle(c0_relaxed)
    f = o.energy_forces()["force"]
    x0 = c0_relaxed.pos.copy()
    rng = np.random.default_rng(3)
    beads = rng.choice(c0_relaxed.n_beads, 24, replace=False)
    h = 1e-5
    bad = 0
    for b in beads:
        for a in range(3):
            xp = x0.copy(); xp[b, a] += h
            xm = x0.copy(); xm[b, a] -= h
            o.set_state(pos=xp); ep = o.energy_forces(forces=False)
            o.set_state(pos=xm); em = o.energy_forces(forces=False)
            if ep["n_pairs"] != em["n_pairs"]:
                continue  # a pair crosses the cutoff inside the stencil
            fd = -(ep["potential"] - em["potential"]) / (2 * h)
            if abs(fd - f[b, a]) > 1e-6 * max(abs(f[b, a]), 10.0):
                bad += 1
    assert bad == 0


def test_translation_and_permutation_invariance(oracle_mod, c0):
    o = oracle_mod.Oracle(c0)
    e0 = o.energy_forces()
    s2 = c0.copy()
    s2.pos = (c0.pos + np.array([1.3, -2.1, 0.7])) % c0.box
    e1 = oracle_mod.Oracle(s2).energy_forces()
    assert abs(e1["potential"] - e0["potential"]) < 1e-8 * abs(e0["potential"])
    # reverse the molecule order (beads move with their molecules)
    first, sizes = c0.mol_first()
    order = np.arange(c0.n_mols)[::-1]
    s3 = c0.copy()
    s3.mol_kind = c0.mol_kind[order]
    s3.pos = np.concatenate([c0.pos[first[m]:first[m] + sizes[m]] for m in order])
    s3.vel = np.concatenate([c0.vel[first[m]:first[m] + sizes[m]] for m in order])
    e3 = oracle_mod.Oracle(s3).energy_forces()
    assert abs(e3["potential"] - e0["potential"]) < 1e-9 * abs(e0["potential"])
    assert e3["n_pairs"] == e0["n_pairs"]


# ------------------------------------------------------------ dynamics (P9)
def test_nve_reversibility_and_drift(oracle_mod, c0_relaxed):
    """gamma = 0 reduces BAOAB to velocity Verlet: time-reversible and
    energy-conserving to O(dt^2)."""
    s = c0_relaxed.copy(); s.gamma = 0.0; s.dt = 0.01
    o = oracle_mod.Oracle(s)
    e0 = o.energy_forces()["total"]
    o.md_step(100)
    st = o.state()
    e1 = o.energy_forces()["total"]
    o.set_state(pos=st["pos"], vel=-st["vel"])
    o.md_step(100)
    back = o.state()["pos"]
    d = back - c0_relaxed.pos
    d -= s.box * np.rint(d / s.box)
    assert np.abs(d).max() < 1e-8
    assert abs(e1 - e0) < 0.05 * s.n_beads * KB * 323   # per-bead fraction of kT
    # halving dt cuts the energy error about four-fold
    errs = []
    for dt in (0.01, 0.005):
        s2 = c0_relaxed.copy(); s2.gamma = 0.0; s2.dt = dt
        o2 = oracle_mod.Oracle(s2)
        ea = o2.energy_forces()["total"]
        o2.md_step(int(round(0.4 / dt)))
        errs.append(abs(o2.energy_forces()["total"] - ea))
    assert errs[1] < errs[0] / 2.0


def test_langevin_equipartition(oracle_mod):
    """Free particles under the O step keep the Maxwell-Boltzmann
    distribution: <KE> = 3/2 N kT."""
    n = 300
    eps = np.zeros((S.N_TYPES, S.N_TYPES))
    k = S.Kind("W", [4], [0.0], [], [], -1)
    rng = np.random.default_rng(5)
    pos = rng.uniform(0, 9, size=(n, 3))
    s = S.custom("gas", [k], [0] * n, pos, [9, 9, 9], eps, seed=99)
    s.gamma = 5.0
    o = oracle_mod.Oracle(s)
    kes = []
    for _ in range(40):
        o.md_step(10)
        kes.append(o.energy_forces(forces=False)["kinetic"])
    ke = np.mean(kes[5:])
    expect = 1.5 * n * KB * 323.0
    assert abs(ke / expect - 1.0) < 0.05


# ----------------------------------------------------- exchange moves (P10-P12)
def test_delta_u_incremental_equals_full(oracle_mod, c0):
    """Eq. 1's energy difference (after minus before) from the pair terms of
    the changed beads equals two full recomputations."""
    o = oracle_mod.Oracle(c0)
    mk = c0.mol_kind
    A = np.where(mk == S.KIND_A)[0]
    B = np.where(mk == S.KIND_B)[0]
    for X, Y in [(A[0], B[0]), (A[3], B[7]), (A[10], B[2])]:
        assert abs(o.delta_u_pair(X, Y) - o.delta_u_full(X, Y)) < 1e-8


def _toy_du(r, eps_a, eps_b):
    sig = S.SIGMA
    def v(e):
        return 4 * e * ((sig / r) ** 12 - (sig / r) ** 6) - 4 * e * ((sig / RC) ** 12 - (sig / RC) ** 6)
    return v(eps_b) - v(eps_a)


@pytest.mark.parametrize("r", [0.5, 0.62, 0.9])
def test_two_lipid_toy_delta_u(oracle_mod, r):
    s = S.two_lipid_toy(r)
    o = oracle_mod.Oracle(s)
    du = o.delta_u_pair(0, 1)
    r = float(np.linalg.norm(s.pos[4] - s.pos[1]))   # float32-rounded geometry
    assert abs(du - _toy_du(r, 5.6, 3.1)) < 1e-9
    assert abs(o.delta_u_full(0, 1) - du) < 1e-9


def test_two_lipid_toy_metropolis_chain(oracle_mod):
    """Frozen two-state chain under Eq. 1: the uphill move is accepted with
    p = exp(-dU/kT), the downhill one always, so the chain spends a fraction
    1/(1+p) of its trials in the low-energy state."""
    s = S.two_lipid_toy(0.6)
    o = oracle_mod.Oracle(s)
    r = float(np.linalg.norm(s.pos[4] - s.pos[1]))
    du = _toy_du(r, 5.6, 3.1)   # > 0: the start state is the low one
    assert du > 0
    p = math.exp(-du / (KB * 323.0))
    n = 6000
    low, accepted = 0, 0
    for _ in range(n):
        st = o.state()["mol_kind"]
        if st[0] == 0:
            low += 1
        res = o.swap_batch(1)
        assert len(res["du"]) == 1
        accepted += int(res["accept"][0])
    frac = low / n
    expect = 1 / (1 + p)
    assert abs(frac - expect) < 5 * math.sqrt(expect * (1 - expect) / n) + 0.01
    rate = accepted / n
    expect_rate = 2 * p / (1 + p)
    assert abs(rate - expect_rate) < 5 * math.sqrt(expect_rate * (1 - expect_rate) / n) + 0.01


def test_batch_trials_are_independent(oracle_mod, c0):
    """Admitted trials of a batch have changed beads at least r_c apart, so
    each trial's energy difference equals the one computed alone."""
    o = oracle_mod.Oracle(c0)
    st0 = o.state()
    res = o.swap_batch(4)
    o2 = oracle_mod.Oracle(c0)
    for X, Y, du in zip(res["X"], res["Y"], res["du"]):
        assert abs(o2.delta_u_full(X, Y) - du) < 1e-8
    assert len(set(res["X"]) | set(res["Y"])) == 2 * len(res["X"])


def test_mdas_single_step_equals_mc(oracle_mod, c0):
    """Section 2: MDAS with dlambda = 1 and M = 0 is the single-step MC
    exchange, so its work equals dU of the exchanged pairs; with M = 0 and
    any K the work is U_B - U_A (coordinates frozen)."""
    for K in (1, 7):
        o = oracle_mod.Oracle(c0)
        before = o.state()
        res = o.mdas_cycle(3, K, 0)
        o2 = oracle_mod.Oracle(c0)
        du = o2.pairs_delta_u(res["pairs"])
        assert abs(res["work"] - du) < 1e-8 * max(1, abs(du))
        if not res["accept"]:
            after = o.state()
            assert np.array_equal(after["mol_kind"], before["mol_kind"])
            assert np.array_equal(after["pos"], before["pos"])


def test_mdas_continuation_rules(oracle_mod, c0_relaxed):
    """Section 2 continuation: an accepted trajectory keeps the lambda=1
    state with the pair's kinds exchanged; a rejected one restores the
    coordinates, velocities and kinds from before the trajectory."""
    seen = set()
    for cyc in range(12):
        o = oracle_mod.Oracle(c0_relaxed)
        o.set_state(counters=[0, 0, cyc])
        before = o.state()
        res = o.mdas_cycle(1, 3, 2)
        after = o.state()
        X, Y = res["pairs"][0]
        if res["accept"]:
            assert after["mol_kind"][X] == before["mol_kind"][Y]
            assert after["mol_kind"][Y] == before["mol_kind"][X]
        else:
            assert np.array_equal(after["pos"], before["pos"])
            assert np.array_equal(after["vel"], before["vel"])
            assert np.array_equal(after["mol_kind"], before["mol_kind"])
        assert after["step"] == before["step"] + 6     # noise is never reused
        seen.add(bool(res["accept"]))
    assert seen == {True, False}


# ------------------------------------------------------------ mixing observable
def _lattice_po4_system(n, a, second_leaflet_kind):
    """n x n periodic square lattice (spacing a) of two-bead molecules
    [head, PO4] in the upper leaflet, plus the same lattice shifted by a/2 in
    the lower leaflet with molecules of another kind."""
    kh = S.Kind("H", [S.TYPE_N, S.TYPE_Q], [0.0, 0.0], [(0, 1, 0.47, 1250.0)], [], 0)
    kh2 = S.Kind("H2", [S.TYPE_N, S.TYPE_Q], [0.0, 0.0], [(0, 1, 0.47, 1250.0)], [], 0)
    L = n * a
    pos, mk, leaf = [], [], []
    for lf, kind, off, z in ((0, 0, 0.0, 6.0), (1, second_leaflet_kind, 0.5 * a, 2.0)):
        for i in range(n):
            for j in range(n):
                x, y = i * a + off, j * a + off
                pos += [[x, y, z + 0.47], [x, y, z]]
                mk.append(kind)
                leaf.append(lf)
    s = S.custom("lattice", [kh, kh2], mk, pos, [L, L, 9.0], np.full((S.N_TYPES, S.N_TYPES), 2.0))
    return s, np.asarray(leaf, dtype=np.int32)


@pytest.mark.parametrize("second_kind", [0, 1])
def test_pair_histogram_square_lattice(oracle_mod, second_kind):
    """Exact shell counts on a periodic square lattice: every point has 4
    neighbours at a, 4 at a sqrt 2, 4 at 2a and 8 at a sqrt 5; pairs across
    leaflets never count, whatever the kinds."""
    n, a, w = 8, 1.0, 0.07
    s, leaf = _lattice_po4_system(n, a, second_kind)
    o = oracle_mod.Oracle(s)
    h = o.pair_histogram(0, 1, leaf, 80, w)
    N = n * n
    m = 2 if second_kind == 0 else 1   # leaflets holding kind 0
    assert h[int(a / w)] == m * N * 4 // 2                    # bin 14
    assert h[int(a * math.sqrt(2) / w)] == m * N * 4 // 2     # bin 20
    assert h[int(2 * a / w)] == m * N * 4 // 2                # bin 28
    assert h[int(a * math.sqrt(5) / w)] == m * N * 8 // 2     # bin 31
    # cross-leaflet pairs (lateral a / sqrt 2, bin 10) never count: nothing
    # below the first shell; all same-leaflet pairs in range, nothing else
    assert h[:14].sum() == 0
    assert h.sum() == m * np.count_nonzero(_lattice_d2(n, a) < (80 * w) ** 2)


def _lattice_d2(n, a):
    ij = np.array([(i, j) for i in range(n) for j in range(n)], dtype=np.float64) * a
    L = n * a
    d = ij[:, None, :] - ij[None, :, :]
    d -= L * np.rint(d / L)
    d2 = (d ** 2).sum(-1)
    iu = np.triu_indices(len(ij), 1)
    return d2[iu]


def test_pair_histogram_equals_explicit_images(oracle_mod, c0):
    """Random bilayer (C0): the oracle's minimum-image histogram equals one
    built from the nine explicit periodic images of every pair (smallest
    distance) and numpy's histogram, per leaflet and kind."""
    o = oracle_mod.Oracle(c0)
    leaf = c0.meta["leaflet"]
    first, _ = c0.mol_first()
    w, nb = 0.05, 50
    for kind in (S.KIND_A, S.KIND_B):
        h = o.pair_histogram(kind, S.PO4, leaf, nb, w)
        ref = np.zeros(nb, dtype=np.int64)
        for lf in (0, 1):
            sel = np.where((c0.mol_kind == kind) & (leaf == lf))[0]
            p = c0.pos[first[sel] + S.PO4][:, :2]
            best = np.full((len(p), len(p)), np.inf)
            for sx in (-1, 0, 1):
                for sy in (-1, 0, 1):
                    sh = np.array([sx * c0.box[0], sy * c0.box[1]])
                    d = p[:, None, :] - (p[None, :, :] + sh)
                    best = np.minimum(best, np.sqrt((d ** 2).sum(-1)))
            iu = np.triu_indices(len(p), 1)
            ref += np.histogram(best[iu], bins=np.arange(nb + 1) * w)[0]
        assert np.array_equal(h, ref), (kind, h, ref)
        assert h.sum() > 0


# ------------------------------------------- stochastic velocity rescaling
# The paper's ensemble (Methods) uses the velocity rescaling thermostat of
# Bussi, Donadio and Parrinello; these pins hold its oracle against
# statistics fixed by the method's definition and by an independent
# construction, never against its own formulas.

@pytest.mark.parametrize("a", [1.0, 1.5, 7.0, 300.0, 1e5])
def test_gamma_sampler_distribution(oracle_mod, c0, a):
    """The thermostat's gamma draws follow Gamma(a, 1) (Kolmogorov-Smirnov
    against scipy's distribution)."""
    from scipy import stats
    o = oracle_mod.Oracle(c0)
    g = o.gamma_mt(1, a, 1000, 20000)
    assert stats.kstest(g, stats.gamma(a).cdf).pvalue > 1e-4
    assert abs(g.mean() / a - 1.0) < 6.0 / math.sqrt(a * len(g))


def _o_step_alphas(K, nf, c, kT, n, seed):
    """Velocity factors from an independent construction: nf unit-mass
    velocity components with kinetic energy K, one Ornstein-Uhlenbeck step
    v' = sqrt(c) v + sqrt((1 - c) kT) xi, and alpha = sign(v'.v) |v'| / |v|.
    The kinetic energy dynamics of the rescaling thermostat is exactly this
    step's, so both give the same distribution of alpha."""
    rng = np.random.default_rng(seed)
    v = np.zeros(nf); v[0] = math.sqrt(2.0 * K)
    xi = rng.standard_normal((n, nf))
    vp = math.sqrt(c) * v + math.sqrt((1.0 - c) * kT) * xi
    return np.sign(vp[:, 0]) * np.linalg.norm(vp, axis=1) / np.linalg.norm(v)


@pytest.mark.parametrize("nf,k_over_kt,c", [(3, 0.1, 0.5), (3, 2.0, 0.95), (30, 1.5, 0.9),
                                            (300, 0.8, 0.3)])
def test_vrescale_alpha_equals_ou_step(oracle_mod, c0, nf, k_over_kt, c):
    from scipy import stats
    s = c0.copy()
    kT = KB * s.temperature
    o = oracle_mod.Oracle(s)
    o.set_ensemble(1, tau_t=-s.dt / math.log(c))
    K = k_over_kt * 0.5 * nf * kT
    a_or = o.vr_alpha(0, K, float(nf), 0, 20000)
    a_ou = _o_step_alphas(K, nf, c, kT, 20000, seed=nf)
    assert stats.ks_2samp(a_or, a_ou).pvalue > 1e-4
    # the sign: reversals happen as often as the velocity turns round
    p_neg = np.mean(a_ou < 0)
    assert abs(np.mean(a_or < 0) - p_neg) < 6.0 * math.sqrt(max(p_neg, 1e-4) / 20000)


def test_vrescale_limits(oracle_mod, c0):
    """tau_t -> infinity leaves the velocities alone; tau_t -> 0 draws a
    fresh kinetic energy from the canonical Gamma(nf / 2, kT) whatever K was."""
    from scipy import stats
    s = c0.copy()
    kT = KB * s.temperature
    o = oracle_mod.Oracle(s)
    o.set_ensemble(1, tau_t=math.inf)
    assert np.all(o.vr_alpha(1, 3.7, 12.0, 5, 100) == 1.0)
    o.set_ensemble(1, tau_t=1e-9)
    nf = 24.0
    K = 10.0 * 0.5 * nf * kT
    kp = o.vr_alpha(0, K, nf, 0, 20000) ** 2 * K
    assert stats.kstest(kp, stats.gamma(0.5 * nf, scale=kT).cdf).pvalue > 1e-4


def test_vrescale_tau_inf_is_velocity_verlet(oracle_mod, c0_relaxed):
    """With tau_t = infinity the thermostatted integrator is plain velocity
    Verlet whatever the Langevin friction of the system (the O step is off)."""
    s0 = c0_relaxed.copy(); s0.gamma = 0.0
    s1 = c0_relaxed.copy(); s1.gamma = 3.0
    a = oracle_mod.Oracle(s0)
    b = oracle_mod.Oracle(s1)
    b.set_ensemble(1, tau_t=math.inf, kind_group=[0, 0, 0, 0, 1])
    a.md_step(10)
    b.md_step(10)
    sa, sb = a.state(), b.state()
    assert np.array_equal(sa["pos"], sb["pos"]) and np.array_equal(sa["vel"], sb["vel"])
    assert sa["step"] == sb["step"] == 10


def test_vrescale_two_groups_canonical(oracle_mod):
    """A free gas of two kinds in two coupling groups, started one hot and
    one cold: each group relaxes to <K> = 3/2 N kT with the canonical
    fluctuation var K = 3/2 N (kT)^2 (a rescaling to the mean alone would
    give none)."""
    n = 100
    eps = np.zeros((S.N_TYPES, S.N_TYPES))
    ka = S.Kind("P", [4], [0.0], [], [], -1, masses=[72.0])
    kb = S.Kind("Q", [4], [0.0], [], [], -1, masses=[36.0])
    rng = np.random.default_rng(11)
    pos = rng.uniform(0, 9, size=(2 * n, 3))
    mk = [0] * n + [1] * n
    kT = KB * 323.0
    vel = np.concatenate([rng.standard_normal((n, 3)) * math.sqrt(4.0 * kT / 72.0),
                          rng.standard_normal((n, 3)) * math.sqrt(0.25 * kT / 36.0)])
    s = S.custom("gas2", [ka, kb], mk, pos, [9, 9, 9], eps, vel=vel, seed=7)
    o = oracle_mod.Oracle(s)
    o.set_ensemble(1, tau_t=0.1, kind_group=[0, 1])
    o.md_step(100)
    ks = [[], []]
    for _ in range(400):
        o.md_step(5)
        v = o.state()["vel"]
        ks[0].append(0.5 * 72.0 * (v[:n] ** 2).sum())
        ks[1].append(0.5 * 36.0 * (v[n:] ** 2).sum())
    for g in (0, 1):
        k = np.asarray(ks[g])
        assert abs(k.mean() / (1.5 * n * kT) - 1.0) < 0.05, (g, k.mean() / (1.5 * n * kT))
        r = k.var() / (1.5 * n * kT * kT)
        assert 0.6 < r < 1.6, (g, r)


# ------------------------------------------------- exchange regions (leaflets)
def _hypergeom_moments(m, t):
    """number of the t Q molecules found in one region of m out of 2m places,
    all arrangements equally likely"""
    p = t / (2.0 * m)
    return m * p, m * p * (1 - p) * (2 * m - t) / (2 * m - 1)


def _region_chain(oracle_mod, mode, n_batches, m=8, t=8):
    s = S.twin_exchange_toy(m, t)
    o = oracle_mod.Oracle(s)
    o.set_exchange_regions(mode, s.meta["leaflet"])
    lf = s.meta["leaflet"]
    ns, pairs = [], []
    for _ in range(n_batches):
        r = o.swap_batch(1)
        pairs += list(zip(r["X"], r["Y"]))
        mk = o.state()["mol_kind"]
        ns.append(int(np.count_nonzero((mk == 1) & (lf == 0))))
    return np.asarray(ns), pairs, lf


@pytest.mark.parametrize("mode", [0, 2])
def test_exchange_chain_samples_uniform_arrangements(oracle_mod, mode):
    """Kinds with identical parameters (dU = 0, every trial accepted): the
    number of Q molecules in region 0 must follow the hypergeometric law of
    uniformly random arrangements, whatever partner rule the proposal uses,
    if the proposal is symmetric.  (Drawing the interleaflet partner among
    molecules of the other kind only would give the binomial law, twice the
    variance.)"""
    ns, pairs, lf = _region_chain(oracle_mod, mode, 20000)
    mean, var = _hypergeom_moments(8, 8)
    x = ns[1000:]
    assert abs(x.mean() - mean) < 0.15, x.mean()
    assert abs(x.var() / var - 1.0) < 0.12, (x.var(), var)
    if mode == 2:
        assert all(lf[a] != lf[b] for a, b in pairs)


def test_exchange_within_regions_keeps_compositions(oracle_mod):
    ns, pairs, lf = _region_chain(oracle_mod, 1, 2000, m=8, t=5)
    assert np.all(ns == 5)
    assert len(pairs) == 2000 and all(lf[a] == lf[b] for a, b in pairs)


# ------------------------------------------------------- virial, pressure
def _stretched_potential(oracle_mod, sysm, axis, eps):
    s = sysm.copy()
    s.pos = sysm.pos.copy()
    s.box = np.asarray(sysm.box, dtype=np.float64).copy()
    s.pos[:, axis] *= 1.0 + eps
    s.box[axis] *= 1.0 + eps
    return oracle_mod.Oracle(s).energy_forces(forces=False)["potential"]


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_virial_is_minus_strain_derivative(oracle_mod, c0_relaxed, axis):
    """W_aa = -dU/d eps for the affine stretch of all beads and the box
    along axis a, on the C0 bilayer: LJ, reaction field, bonds and angles
    together.  The shifted LJ force jumps at the cutoff, so a pair crossing
    it inside the difference interval adds a kink; the median of central
    differences over five small intervals sets such rare crossings aside."""
    fds = []
    for h in (1e-7, 2e-7, 3e-7, 5e-7, 7e-7):
        up = _stretched_potential(oracle_mod, c0_relaxed, axis, h)
        dn = _stretched_potential(oracle_mod, c0_relaxed, axis, -h)
        fds.append(-(up - dn) / (2 * h))
    w = oracle_mod.Oracle(c0_relaxed).virial()["w"][axis]
    fd = float(np.median(fds))
    assert abs(w - fd) < 5e-6 * max(abs(w), 1e3), (w, fds)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_virial_of_an_angle(oracle_mod, axis):
    """An angle alone (bonds carry no force): the same identity on a bent
    three-bead molecule across a periodic boundary."""
    pos = [[7.8, 1.0, 1.2], [0.2, 1.3, 1.0], [0.5, 0.9, 1.4]]
    eps = np.zeros((S.N_TYPES, S.N_TYPES))
    k = S.Kind("T", [0] * 3, [0.0] * 3, [(0, 1, 0.47, 0.0), (1, 2, 0.47, 0.0)],
               [(0, 1, 2, 180.0, 25.0)], -1)
    s = S.custom("b", [k], [0], pos, [8, 8, 8], eps)
    h = 1e-6
    up = _stretched_potential(oracle_mod, s, axis, h)
    dn = _stretched_potential(oracle_mod, s, axis, -h)
    w = oracle_mod.Oracle(s).virial(cells=False)["w"][axis]
    assert abs(w + (up - dn) / (2 * h)) < 1e-6 * max(1.0, abs(w))
    assert abs(w) > 1e-3


def test_pressure_of_an_ideal_gas(oracle_mod):
    """No interactions: P_aa V = sum m v_a^2, which averages N kT under the
    Langevin thermostat."""
    n = 400
    eps = np.zeros((S.N_TYPES, S.N_TYPES))
    k = S.Kind("W", [4], [0.0], [], [], -1)
    rng = np.random.default_rng(3)
    s = S.custom("gas", [k], [0] * n, rng.uniform(0, 9, size=(n, 3)), [9, 9, 9], eps, seed=5)
    s.gamma = 5.0
    o = oracle_mod.Oracle(s)
    ps = []
    for _ in range(60):
        o.md_step(10)
        v = o.virial(cells=False)
        assert np.all(v["w"] == 0.0)
        ps.append(v["pressure"])
    p = np.mean(ps[10:], axis=0)
    ideal = n * KB * 323.0 / 729.0 * oracle_mod.BAR
    assert np.all(np.abs(p / ideal - 1.0) < 0.06), (p, ideal)


# --------------------------------------------------- pressure coupling
def test_barostat_ideal_gas_volume_law(oracle_mod):
    """Ideal gas of N = 30 beads under the semi-isotropic cell rescaling at
    P0: the volume must follow Gamma(N + 1, kT / P0), mean (N + 1) kT / P0
    and variance (N + 1) (kT / P0)^2 (a drift that added kT / V, as for
    velocity-scaled kinetic pressures, would give shape N + 2, 3% more
    volume); x and y stay equal.  Coupling every
    step with dt / tau_p = 0.05: the Euler-Maruyama step widens the law of
    ln V by the factor 1 / (1 - dt / tau_p) at this compressibility, which
    the variance bound allows for."""
    n = 30
    eps = np.zeros((S.N_TYPES, S.N_TYPES))
    k = S.Kind("W", [4], [0.0], [], [], -1)
    rng = np.random.default_rng(17)
    L0 = 3.0
    s = S.custom("gas", [k], [0] * n, rng.uniform(0, L0, size=(n, 3)), [L0, L0, L0], eps, seed=21)
    s.gamma = 2.0
    kT = KB * 323.0
    p0 = (n + 1) * kT / 27.0                          # law mean 27 nm^3 (box ~3 nm)
    p0_bar = p0 * oracle_mod.BAR
    o = oracle_mod.Oracle(s)
    # the ideal gas's own compressibility 1 / P0, tau_p = 0.4 ps
    o.set_barostat(1, p_ref_bar=p0_bar, compressibility=1.0 / p0_bar, tau_p=0.4)
    vols = []
    for _ in range(4000):
        o.md_step(25)
        b = o.box()
        assert abs(b[0] - b[1]) < 1e-12 * b[0]
        vols.append(b[0] * b[1] * b[2])
    v = np.asarray(vols[200:])
    mean, var = (n + 1) * kT / p0, (n + 1) * (kT / p0) ** 2
    print("V mean %.3f (law %.3f), var %.3f (law %.3f)" % (v.mean(), mean, v.var(), var))
    assert abs(v.mean() / mean - 1.0) < 0.01
    assert abs(v.var() / (var / (1 - 0.05)) - 1.0) < 0.12


# ------------------------------------------- soft-core lambda path (Eq. 4)
def _c6c12(eps, sig):
    return 4 * eps * sig ** 6, 4 * eps * sig ** 12


def test_soft_core_reduces_to_lj(oracle_mod):
    """mu = 1: the shifted 12-6 form of the pair term; mu = 0: nothing."""
    eps, sig = 3.5, 0.47
    c6, c12 = _c6c12(eps, sig)
    s = S.make("c0")
    o = oracle_mod.Oracle(s)
    ti = tj = int(np.argmin(np.abs(s.eps.diagonal() - eps)))
    eps = s.eps[ti, tj]; sig = s.sigma[ti, tj]
    c6, c12 = _c6c12(eps, sig)
    for r in (0.45, 0.6, 0.95):
        v, f = oracle_mod.sc_lj(c6, c12, r * r, 1.0, 0.05, s.rc)
        vlj, vrf, fs = o.pair_term(ti, tj, 0.0, 0.0, r * r)
        assert abs(v - vlj) < 1e-12 * max(1.0, abs(vlj)) and abs(f - fs) < 1e-10 * max(1.0, abs(fs))
        assert oracle_mod.sc_lj(c6, c12, r * r, 0.0, 0.05, s.rc) == (0.0, 0.0)


@pytest.mark.parametrize("mu", [0.2, 0.7])
def test_soft_core_force_and_origin(oracle_mod, mu):
    """fscal = -dV/dr / r (central difference), V(r_c) = 0, and at r = 0 the
    finite value mu (c12 / (delta (1 - mu))^6 - c6 / (delta (1 - mu))^3)
    minus the shift: no end-point singularity for mu < 1."""
    c6, c12 = _c6c12(5.6, 0.47)
    delta, rc = 0.05, 1.1
    for r in (0.1, 0.4, 0.8):
        h = 1e-6
        vp, _ = oracle_mod.sc_lj(c6, c12, (r + h) ** 2, mu, delta, rc)
        vm, _ = oracle_mod.sc_lj(c6, c12, (r - h) ** 2, mu, delta, rc)
        _, f = oracle_mod.sc_lj(c6, c12, r * r, mu, delta, rc)
        assert abs(f * r + (vp - vm) / (2 * h)) < 1e-6 * max(1.0, abs(f * r))
    assert abs(oracle_mod.sc_lj(c6, c12, rc * rc, mu, delta, rc)[0]) < 1e-15
    s0 = delta * (1 - mu)
    sc = rc * rc + s0
    v0 = mu * (c12 / s0 ** 6 - c6 / s0 ** 3) - mu * (c12 / sc ** 6 - c6 / sc ** 3)
    assert abs(oracle_mod.sc_lj(c6, c12, 0.0, mu, delta, rc)[0] - v0) < 1e-9 * abs(v0)


@pytest.mark.parametrize("name", ["c0", "mix"])
def test_soft_core_path_end_states(oracle_mod, name):
    """With two exchanged pairs (C0: A <-> B changes bead types; mix: A <-> D
    changes a head charge): U_0 = U_A and U_1 = U_B of the full system; a
    frozen MDAS cycle on the soft-core path gives the same work U_B - U_A as
    the linear path, for any K."""
    c0 = S.make(name)
    o = oracle_mod.Oracle(c0)
    r = o.mdas_cycle(2, 1, 0)            # selects two pairs; frozen, so the state is kept or swapped
    pairs = r["pairs"]
    o = oracle_mod.Oracle(c0)
    ua = o.energy_forces(forces=False)["potential"]
    mk = c0.mol_kind.copy()
    for x, y in pairs:
        mk[x], mk[y] = mk[y], mk[x]
    ob = oracle_mod.Oracle(c0)
    ob.set_state(mol_kind=mk)
    ub = ob.energy_forces(forces=False)["potential"]
    assert abs(o.sc_energy(pairs, 0.0) - ua) < 1e-9 * abs(ua)
    assert abs(o.sc_energy(pairs, 1.0) - ub) < 1e-9 * abs(ub)
    mid = o.sc_energy(pairs, 0.5)
    assert np.isfinite(mid)
    for K in (1, 5):
        lin = oracle_mod.Oracle(c0).mdas_cycle(2, K, 0)
        osc = oracle_mod.Oracle(c0)
        osc.set_mdas_path(1, 0.05)
        sc = osc.mdas_cycle(2, K, 0)
        assert np.array_equal(lin["pairs"], sc["pairs"])
        assert abs(sc["work"] - (ub - ua)) < 1e-8 * max(1.0, abs(ua))
        assert abs(sc["work"] - lin["work"]) < 1e-8 * max(1.0, abs(ua))


# ---------------------------------------------------------------- minimizer
def _pair_system(r, eps_nn=5.0, bonded=False):
    """Two beads of type N at distance r along x in a 6 nm box: two one-bead
    molecules (LJ between them), or one two-bead molecule whose beads are
    bonded with b0 = 0.47 nm, k = 1250 kJ/mol/nm^2 (LJ excluded)."""
    eps = np.zeros((S.N_TYPES, S.N_TYPES))
    eps[S.TYPE_N, S.TYPE_N] = eps_nn
    pos = [[2.0, 3.0, 3.0], [2.0 + r, 3.0, 3.0]]
    if bonded:
        k = S.Kind("B", [S.TYPE_N, S.TYPE_N], [0.0, 0.0], [(0, 1, 0.47, 1250.0)], [], -1)
        return S.custom("pair", [k], [0], pos, [6.0, 6.0, 6.0], eps)
    k = S.Kind("P", [S.TYPE_N], [0.0], [], [], -1)
    return S.custom("pair", [k], [0, 0], pos, [6.0, 6.0, 6.0], eps)


def _sep(o):
    p = o.state()["pos"]
    return float(np.linalg.norm(p[1] - p[0]))


@pytest.mark.parametrize("r0", [0.45, 0.6, 0.9])
def test_minimize_lj_pair_reaches_lj_minimum(oracle_mod, r0):
    """Capped steepest descent on two LJ beads stops where the 12-6 force
    vanishes, r = 2^(1/6) sigma (the potential shift at the cutoff is a
    constant and moves no minimum), from either side."""
    o = oracle_mod.Oracle(_pair_system(r0))
    o.minimize(400, alpha=1e-4, cap=0.01)
    assert abs(_sep(o) - 2.0 ** (1.0 / 6.0) * S.SIGMA) < 1e-9
    e = o.energy_forces()
    assert np.abs(e["force"]).max() < 1e-6
    vc = 4.0 * 5.0 * ((S.SIGMA / RC) ** 12 - (S.SIGMA / RC) ** 6)
    assert abs(e["lj"] - (-5.0 - vc)) < 1e-9   # the well depth, shifted at r_c


def test_minimize_bond_reaches_rest_length(oracle_mod):
    """A harmonic bond alone (its pair is excluded from LJ) relaxes to b0."""
    o = oracle_mod.Oracle(_pair_system(0.55, bonded=True))
    o.minimize(400, alpha=1e-4, cap=0.01)
    assert abs(_sep(o) - 0.47) < 1e-9


def test_minimize_step_cap(oracle_mod):
    """From a deep overlap every bead moves by exactly the cap, along the
    force: one iteration separates the pair by 2 cap."""
    s = _pair_system(0.3)
    r0 = float(np.linalg.norm(s.pos[1] - s.pos[0]))
    o = oracle_mod.Oracle(s)
    o.minimize(1, alpha=1e-4, cap=0.01)
    p = o.state()["pos"]
    assert abs(_sep(o) - (r0 + 0.02)) < 1e-12
    assert abs(p[0][1] - 3.0) < 1e-12 and abs(p[1][2] - 3.0) < 1e-12
