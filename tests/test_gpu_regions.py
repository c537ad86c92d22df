"""Exchange regions (leaflets) on the GPU against the float64 oracle: the
partner rules within a leaflet and across leaflets (the interleaflet move
of the paper's Discussion) select the identical trials and decide them as
the oracle does; on a toy of identical twin kinds the GPU chain samples
the hypergeometric law of uniform arrangements.

Tolerances as in test_gpu_parity: dU within 1e-8 (float64) / 5e-4 kJ/mol
(mixed), decisions identical outside the near-tie band, trials and u
identical.
"""
import math

import numpy as np
import pytest

from paper_2005_08348_amd import systems as S

pytestmark = pytest.mark.gpu

KB = 0.00831446261815324


def _membx():
    from paper_2005_08348_amd import membx
    return membx


@pytest.fixture(scope="module")
def c0_relaxed(oracle_mod):
    c0 = S.make("c0")
    o = oracle_mod.Oracle(c0)
    o.minimize(60)
    s = c0.copy()
    s.pos = o.state()["pos"].astype(np.float32).astype(np.float64) % s.box
    s.pos = np.where(s.pos >= s.box, 0.0, s.pos)
    return s


def _regions(sysm):
    return np.maximum(sysm.meta["leaflet"], 0).astype(np.int32)


def _same_batch(rg, ro, tol, kT):
    assert list(rg["draw"]) == list(ro["draw"])
    assert list(rg["X"]) == list(ro["X"]) and list(rg["Y"]) == list(ro["Y"])
    assert np.abs(rg["du"] - ro["du"]).max() < tol
    assert np.array_equal(rg["u"], ro["u"])
    for a, b, u, du in zip(rg["accept"], ro["accept"], ro["u"], ro["du"]):
        if a != b:
            assert abs(math.log(u) + du / kT) < tol / kT


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("mode", [1, 2])
def test_region_swap_batches_c0(oracle_mod, c0_relaxed, mode, prec):
    m = _membx()
    g = m.System(c0_relaxed, precision=prec)
    o = oracle_mod.Oracle(c0_relaxed)
    rg_ = _regions(c0_relaxed)
    g.set_exchange_regions(mode, rg_)
    o.set_exchange_regions(mode, rg_)
    kT = KB * c0_relaxed.temperature
    tol = 1e-8 if prec == "fp64" else 5e-4
    for _ in range(4):
        rg = g.swap_trials(4)
        ro = o.swap_batch(4)
        assert len(ro["X"]) > 0
        _same_batch(rg, ro, tol, kT)
        same = rg_[ro["X"]] == rg_[ro["Y"]]
        assert np.all(same) if mode == 1 else not np.any(same)
        g.set_state(mol_kind=o.state()["mol_kind"])
        g.md_step(2)
        o.set_state(pos=g.state()["pos"], vel=g.state()["vel"])
    # per-leaflet compositions: unchanged within leaflets
    if mode == 1:
        mk0, mk1 = c0_relaxed.mol_kind, o.state()["mol_kind"]
        for lf in (0, 1):
            sel = rg_ == lf
            assert np.array_equal(np.bincount(mk0[sel], minlength=5), np.bincount(mk1[sel], minlength=5))
    g.close()


def test_region_mdas_cycle_c0(oracle_mod, c0_relaxed):
    """An interleaflet MDAS cycle: same pairs, work, decision and end state."""
    m = _membx()
    g = m.System(c0_relaxed, precision="fp64", rebuild_interval=4)
    o = oracle_mod.Oracle(c0_relaxed)
    rg_ = _regions(c0_relaxed)
    g.set_exchange_regions(2, rg_)
    o.set_exchange_regions(2, rg_)
    for _ in range(2):
        r1 = g.mdas_cycle(2, 5, 2)
        r2 = o.mdas_cycle(2, 5, 2)
        assert np.array_equal(r1["pairs"], r2["pairs"])
        assert np.all(rg_[r2["pairs"][:, 0]] != rg_[r2["pairs"][:, 1]])
        assert abs(r1["work"] - r2["work"]) < 1e-6
        assert r1["accept"] == r2["accept"]
    sg, so = g.state(), o.state()
    assert np.array_equal(sg["mol_kind"], so["mol_kind"])
    d = sg["pos"] - so["pos"]
    d -= c0_relaxed.box * np.rint(d / c0_relaxed.box)
    assert np.abs(d).max() < 1e-7
    g.close()


def test_twin_chain_gpu(oracle_mod):
    """Identical twin kinds (dU = 0): the first 300 single-trial batches pick
    the oracle's pairs, and the long chain samples the hypergeometric law."""
    m = _membx()
    s = S.twin_exchange_toy(8, 8)
    lf = s.meta["leaflet"]
    g = m.System(s, precision="fp64")
    o = oracle_mod.Oracle(s)
    g.set_exchange_regions(2, lf)
    o.set_exchange_regions(2, lf)
    ns = []
    for b in range(12000):
        rg = g.swap_trials(1)
        if b < 300:
            ro = o.swap_batch(1)
            assert list(rg["X"]) == list(ro["X"]) and list(rg["Y"]) == list(ro["Y"])
            assert np.all(rg["du"] == 0.0) and np.all(rg["accept"])
        mk = g.state()["mol_kind"]
        ns.append(int(np.count_nonzero((mk == 1) & (lf == 0))))
    x = np.asarray(ns[1000:])
    p = 0.5
    mean, var = 8 * p, 8 * p * (1 - p) * 8 / 15
    assert abs(x.mean() - mean) < 0.2, x.mean()
    assert abs(x.var() / var - 1.0) < 0.15, (x.var(), var)
    g.close()


def test_region_batch_256_c1(oracle_mod):
    """Within-leaflet exchange batch at the benchmark size (256 trials on the
    95,876-bead bilayer)."""
    m = _membx()
    s = S.make("c1")
    g = m.System(s, precision="mixed")
    o = oracle_mod.Oracle(s)
    rg_ = _regions(s)
    g.set_exchange_regions(1, rg_)
    o.set_exchange_regions(1, rg_)
    rg = g.swap_trials(256)
    ro = o.swap_batch(256)
    assert len(ro["draw"]) > 100
    _same_batch(rg, ro, 5e-4, KB * s.temperature)
    assert np.all(rg_[ro["X"]] == rg_[ro["Y"]])
    g.close()


def test_region_refused_arguments(c0_relaxed):
    m = _membx()
    g = m.System(c0_relaxed, precision="mixed")
    bad = _regions(c0_relaxed).copy()
    bad[np.nonzero(c0_relaxed.meta["leaflet"] >= 0)[0][0]] = 2
    for mode, rg in [(3, None), (-1, None), (1, bad)]:
        with pytest.raises(m.MembxError):
            g.set_exchange_regions(mode, rg)
    with pytest.raises(ValueError):
        g.set_exchange_regions(1, np.zeros(5, dtype=np.int32))
    # water may carry any label: it is never exchanged
    ok = _regions(c0_relaxed).copy()
    ok[c0_relaxed.meta["leaflet"] < 0] = 7
    g.set_exchange_regions(2, ok)
    r = g.swap_trials(4)
    assert len(r["X"]) > 0
    g.close()
