"""Pins of the oracle's sampled forces, of the forces an alchemical
trajectory runs on, and of the MDAS work statistics, against facts that do
not come from the oracle itself:

- the direct O(N) force sum on chosen beads equals the force of the full
  potential (the definition of F_i, the Methods' potential);
- the hybrid force F(lambda) of the linear coupling of Eq. 2 (and of the
  soft-core path of Eq. 4) is minus the gradient of U(lambda), by central
  differences;
- for an exchange of two molecules of the same topology the free-energy
  change is zero by symmetry, so Jarzynski's equality gives
  <exp(-w/kT)> = 1 for the work of Eq. 2 along trajectories that start in
  equilibrium, and the second law <w> > 0;
- the lateral pair histogram of the mixing observable does not depend on
  which periodic image the coordinates are stored in."""
import math

import numpy as np
import pytest

from paper_2005_08348_amd import systems as S

KB = 0.00831446261815324


@pytest.fixture(scope="module")
def c0_relaxed(oracle_mod):
    s = S.make("c0")
    o = oracle_mod.Oracle(s)
    o.minimize(60)
    st = o.state()
    s = s.copy()
    s.pos = st["pos"].astype(np.float32).astype(np.float64) % s.box
    return s


def _face_crossing_bonds(s):
    """bonds whose two beads sit on opposite sides of a periodic face"""
    first, _ = s.mol_first()
    n = 0
    for m, k in enumerate(s.mol_kind):
        for (i, j, _b0, _k) in s.kinds[k].bonds:
            d = s.pos[first[m] + i] - s.pos[first[m] + j]
            n += int(np.any(np.abs(d) > 0.5 * s.box))
    return n


@pytest.mark.parametrize("shift", [0.0, 0.5])
def test_forces_on_equals_full_forces(oracle_mod, c0_relaxed, shift):
    """o_forces_on (the reference of every sampled-force comparison) sums
    the pair terms of one bead over all others plus the bonded terms of its
    molecule; it must equal the force of the full potential on every bead,
    also for molecules that straddle a periodic face."""
    s = c0_relaxed.copy()
    s.pos = (s.pos + shift * s.box) % s.box
    assert _face_crossing_bonds(s) > 0
    o = oracle_mod.Oracle(s)
    ref = o.energy_forces(cells=False)["force"]
    got, near = o.forces_on(np.arange(s.n_beads))
    scale = max(np.abs(ref).max(), 1.0)
    assert np.abs(got - ref).max() <= 1e-12 * scale
    assert np.all(near >= 0.0)


def _exchange_pairs(s, n):
    mk = s.mol_kind
    A = np.where(mk == S.KIND_A)[0]
    B = np.where(mk == S.KIND_B)[0]
    return [(int(A[q]), int(B[q])) for q in range(n)]


@pytest.mark.parametrize("path", [0, 1])
@pytest.mark.parametrize("lam", [0.25, 0.6])
def test_hybrid_force_is_minus_gradient(oracle_mod, c0_relaxed, lam, path):
    """The dynamics of an alchemical trajectory at coupling lambda (Eq. 2:
    U(lambda) = (1 - lambda) U_A + lambda U_B; Eq. 4 on the soft-core path)
    run on F(lambda) = -grad U(lambda): central differences of U(lambda)
    over the changed molecules' beads and their neighbours."""
    o = oracle_mod.Oracle(c0_relaxed)
    if path == 1:
        o.set_mdas_path(1, 0.05)
    pairs = _exchange_pairs(c0_relaxed, 2)
    u0, f = o.hybrid_energy_forces(pairs, lam)
    first, sizes = c0_relaxed.mol_first()
    beads = [int(first[m] + q) for X, Y in pairs for m in (X, Y) for q in (0, 1, 6, 10)]
    rng = np.random.default_rng(17)
    beads += list(map(int, rng.choice(c0_relaxed.n_beads, 8, replace=False)))
    x0 = c0_relaxed.pos.copy()
    h = 1e-5
    checked = 0
    for b in beads:
        for a in range(3):
            xp = x0.copy(); xp[b, a] += h
            xm = x0.copy(); xm[b, a] -= h
            o.set_state(pos=xp); up, _ = o.hybrid_energy_forces(pairs, lam)
            np_p = o.energy_forces(forces=False)["n_pairs"]
            o.set_state(pos=xm); um, _ = o.hybrid_energy_forces(pairs, lam)
            np_m = o.energy_forces(forces=False)["n_pairs"]
            if np_p != np_m:
                continue   # a pair crosses the cutoff inside the stencil
            fd = -(up - um) / (2 * h)
            assert abs(fd - f[b, a]) <= 1e-6 * max(abs(f[b, a]), 10.0), (b, a, fd, f[b, a])
            checked += 1
    assert checked >= 3 * len(beads) - 6
    o.set_state(pos=x0)
    # the end states are the plain potentials of the two kind assignments
    ua, _ = o.hybrid_energy_forces(pairs, 0.0)
    ub, _ = o.hybrid_energy_forces(pairs, 1.0)
    assert abs((ub - ua) - o.pairs_delta_u(pairs)) < 1e-8


def _jarzynski_toy(nmol=64, box=3.6, seed=11):
    """A fluid of two-bead molecules [h, s] of two kinds X (s of type C) and
    Y (s of type U) with the same topology, in one swap family."""
    kx = S.Kind("X", [S.TYPE_N, S.TYPE_C], [0.0, 0.0], [(0, 1, 0.47, 1250.0)], [], 0)
    ky = S.Kind("Y", [S.TYPE_N, S.TYPE_U], [0.0, 0.0], [(0, 1, 0.47, 1250.0)], [], 0)
    eps = np.full((S.N_TYPES, S.N_TYPES), 3.5)
    eps[S.TYPE_C, S.TYPE_C] = 4.5
    eps[S.TYPE_C, S.TYPE_U] = eps[S.TYPE_U, S.TYPE_C] = 4.0
    eps[S.TYPE_N, S.TYPE_C] = eps[S.TYPE_C, S.TYPE_N] = 3.1
    eps[S.TYPE_N, S.TYPE_U] = eps[S.TYPE_U, S.TYPE_N] = 4.0
    rng = np.random.default_rng(seed)
    n = int(math.ceil(nmol ** (1 / 3)))
    a = box / n
    pts = [(i, j, k) for i in range(n) for j in range(n) for k in range(n)][:nmol]
    pos = []
    for p in pts:
        hd = (np.array(p) + 0.25) * a
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        pos += [hd, hd + 0.47 * u]
    pos = np.mod(np.array(pos), box)
    mk = np.array([i % 2 for i in range(nmol)], dtype=np.int32)
    return S.custom("jarzynski", [kx, ky], mk, pos, [box] * 3, eps, seed=seed)


def test_jarzynski_symmetric_exchange(oracle_mod):
    """Theory, Eqs. 2-3 (SURVEY pin P14): exchanging the kinds of two
    molecules of the same topology leaves the free energy unchanged
    (swapping their coordinates maps one ensemble onto the other), so the
    work of alchemical trajectories with M > 0 MD steps per increment obeys
    <exp(-w/kT)> = 1 and <w> > 0.  Trajectories start from the sampled
    chain with 10 MD steps in between."""
    s = _jarzynski_toy()
    o = oracle_mod.Oracle(s)
    o.minimize(200)
    st = o.state()
    s.pos = st["pos"].astype(np.float32).astype(np.float64) % s.box
    o = oracle_mod.Oracle(s)
    o.md_step(2000)
    w = []
    for _ in range(400):
        o.md_step(10)
        w.append(o.mdas_cycle(1, 8, 2)["work"])
    w = np.array(w) / (KB * s.temperature)
    z = np.exp(-w)
    se = z.std() / math.sqrt(len(z))
    assert w.std() > 0.3                       # the work is not trivially zero
    assert abs(z.mean() - 1.0) < 4.0 * se, (z.mean(), se)
    assert w.mean() > 4.0 * w.std() / math.sqrt(len(w))   # dissipation


def test_pair_histogram_is_image_invariant(oracle_mod, c0_relaxed):
    """The lateral separations of the mixing observable are minimum-image
    ones, so moving beads by whole box lengths (as an unwrapped trajectory
    does) leaves the histogram unchanged."""
    s = c0_relaxed
    o = oracle_mod.Oracle(s)
    leaflet = np.where(np.arange(s.n_mols) < 32, 0, 1).astype(np.int32)
    leaflet[s.mol_kind == S.KIND_W] = -1
    ref = o.pair_histogram(S.KIND_A, S.PO4, leaflet, 60, 0.05)
    rng = np.random.default_rng(5)
    k = rng.integers(-3, 4, size=(s.n_beads, 3)).astype(np.float64)
    o.set_state(pos=s.pos + k * s.box)
    got = o.pair_histogram(S.KIND_A, S.PO4, leaflet, 60, 0.05)
    assert np.array_equal(got, ref) and ref.sum() > 0
