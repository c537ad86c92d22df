"""Edge and degenerate cases of the GPU path against the oracle: a 5-bead
system (one partial wave, one cell per axis), the single-trial exchange
chain of the two-molecule toy (trial by trial), the smallest batch and MDAS
cycle, and a system with nothing to exchange."""
import math

import numpy as np
import pytest

from paper_2005_08348_amd import systems as S

pytestmark = pytest.mark.gpu

KB = 0.00831446261815324


def _membx():
    from paper_2005_08348_amd import membx
    return membx


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_toy_forces_energies(oracle_mod, prec, pairs_in_cutoff_ok):
    m = _membx()
    s = S.two_lipid_toy(0.6)
    g = m.System(s, precision=prec)
    o = oracle_mod.Oracle(s)
    ref = o.energy_forces(cells=False)
    f = g.forces()
    tol = 1e-9 if prec == "fp64" else 1e-5
    scale = max(np.abs(ref["force"]).max(), 1.0)
    assert np.abs(f - ref["force"]).max() < tol * scale
    e = g.energies()
    for k in ["lj", "rf", "bond", "angle"]:
        assert abs(e[k] - ref[k]) < tol * max(abs(ref[k]), 1.0), k
    assert pairs_in_cutoff_ok(o, s.rc, e["n_pairs_in_cutoff"], ref["n_pairs"], prec)
    g.close()


def test_toy_exchange_chain_trial_by_trial(oracle_mod):
    """Single-trial batches on the two-molecule toy: every decision, dU and
    uniform equal the oracle's, and the chain's state follows it."""
    m = _membx()
    s = S.two_lipid_toy(0.6)
    g = m.System(s, precision="fp64")
    o = oracle_mod.Oracle(s)
    for _ in range(200):
        rg = g.swap_trials(1)
        ro = o.swap_batch(1)
        assert list(rg["X"]) == list(ro["X"]) and list(rg["Y"]) == list(ro["Y"])
        assert np.array_equal(rg["u"], ro["u"])
        assert np.abs(rg["du"] - ro["du"]).max() < 1e-9
        assert list(rg["accept"]) == list(ro["accept"])
    assert np.array_equal(g.state()["mol_kind"], o.state()["mol_kind"])
    g.close()


def test_smallest_mdas_cycle_equals_exchange(oracle_mod):
    """One pair, K = 1, M = 0: the work is the exchange energy dU (the
    paper's special case of MDAS)."""
    m = _membx()
    s = S.make("c0")
    g = m.System(s, precision="fp64")
    o = oracle_mod.Oracle(s)
    rg = g.mdas_cycle(1, 1, 0)
    ro = o.mdas_cycle(1, 1, 0)
    assert np.array_equal(rg["pairs"], ro["pairs"])
    assert abs(rg["work"] - ro["work"]) < 1e-8
    assert rg["accept"] == ro["accept"]
    g.close()


def test_nothing_to_exchange():
    """Water only: a batch admits no trial, an MDAS cycle is refused."""
    m = _membx()
    kinds = [S.water_kind()]
    rng = np.random.default_rng(5)
    box = 6.0
    n = 600
    pos = rng.uniform(0, box, size=(n, 3))
    eps = np.full((S.N_TYPES, S.N_TYPES), 2.0)
    s = S.custom("water", kinds, [0] * n, pos, [box, box, box], eps)
    g = m.System(s, precision="mixed")
    r = g.swap_trials(4)
    assert len(r["du"]) == 0
    with pytest.raises(m.MembxError):
        g.mdas_cycle(2, 2, 1)
    g.close()
