"""Pins of topology-changing exchanges in the oracle (soft-core path, Eq. 4,
for beads that appear and vanish): the ``topo`` bilayer puts lipid A and
S12, the sterol padded to the lipid's 12 bead slots with four dummy beads,
in one swap family, so an exchange changes bead classes (dummies become
lipid beads and back) and the bonded terms of both molecules.

* Nonbonded exclusions are the union of the pairs bonded in either kind, so
  a molecule's nonbonded pair set does not depend on its current kind.
* The incremental exchange energy (pair terms of the changed beads plus the
  two molecules' bonded energies in their new and old kinds) equals the
  difference of two full evaluations.
* On both MDAS paths the trajectory's forces are F(lambda) = -grad
  U(lambda) (central differences), with bonded terms mixed linearly, and the
  end states give U_B - U_A.
"""
import numpy as np
import pytest

from paper_2005_08348_amd import systems as S


@pytest.fixture(scope="module")
def topo_relaxed(oracle_mod):
    s = S.make("topo")
    o = oracle_mod.Oracle(s)
    o.minimize(100)
    r = s.copy()
    r.pos = o.state()["pos"].astype(np.float32).astype(np.float64) % s.box
    r.pos = np.where(r.pos >= s.box, 0.0, r.pos)
    return r


def _topo_pairs(s, n, seed=5):
    rng = np.random.default_rng(seed)
    a = rng.permutation(np.where(s.mol_kind == S.KIND_A)[0])[:n]
    b = rng.permutation(np.where(s.mol_kind == S.KIND_B)[0])[:n]
    return [(int(x), int(y)) for x, y in zip(a, b)]


def test_topo_exclusions_are_the_union(oracle_mod, topo_relaxed):
    s = topo_relaxed
    o = oracle_mod.Oracle(s)
    ps = o.pairset(1.3)
    listed = set(map(tuple, np.sort(ps, axis=1)))
    first, sizes = s.mol_first()
    bonded_pairs = {(i, j) for k in (S.KIND_A, S.KIND_B) for i, j, _, _ in s.kinds[k].bonds}
    assert any((i, j) not in {(a, b) for a, b, _, _ in s.kinds[S.KIND_A].bonds}
               for i, j in bonded_pairs)          # S12 brings bonds A lacks
    for m in np.where((s.mol_kind == S.KIND_A) | (s.mol_kind == S.KIND_B))[0]:
        f0 = int(first[m])
        for i, j in bonded_pairs:
            assert (min(f0 + i, f0 + j), max(f0 + i, f0 + j)) not in listed
    n0 = o.energy_forces(forces=False)["n_pairs"]
    mk = s.mol_kind.copy()
    for x, y in _topo_pairs(s, 6):
        mk[x], mk[y] = mk[y], mk[x]
    o.set_state(mol_kind=mk)
    assert o.energy_forces(forces=False)["n_pairs"] == n0


def test_topo_delta_u_incremental_equals_full(oracle_mod, topo_relaxed):
    o = oracle_mod.Oracle(topo_relaxed)
    for x, y in _topo_pairs(topo_relaxed, 4):
        inc, full = o.delta_u_pair(x, y), o.delta_u_full(x, y)
        assert abs(inc - full) <= 1e-9 * max(1.0, abs(full)), (x, y, inc, full)
        # the bonded terms changed: the exchange energy is not the pair
        # terms alone (their part is bounded by the changed beads' pairs)
        assert abs(full) > 1e3


@pytest.mark.parametrize("path", [0, 1])
def test_topo_hybrid_force_is_minus_gradient(oracle_mod, topo_relaxed, path):
    s = topo_relaxed
    o = oracle_mod.Oracle(s)
    if path == 1:
        o.set_mdas_path(1, 0.05)
    pairs = _topo_pairs(s, 2)
    lam = 0.3
    u0, f = o.hybrid_energy_forces(pairs, lam)
    first, _ = s.mol_first()
    # a surviving bead, a vanishing one and appearing ones of each molecule
    beads = [int(first[m] + q) for x, y in pairs for m in (x, y) for q in (0, 3, 5, 9)]
    x0 = s.pos.copy()
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
    ua, _ = o.hybrid_energy_forces(pairs, 0.0)
    ub, _ = o.hybrid_energy_forces(pairs, 1.0)
    dfull = o.pairs_delta_u(pairs)
    assert abs((ub - ua) - dfull) <= 1e-9 * max(1.0, abs(dfull))
