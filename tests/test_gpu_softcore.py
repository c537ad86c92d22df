"""Soft-core MDAS lambda path (Eq. 4) on the GPU against the float64
oracle.  Tolerances as for the linear path: work within 1e-6 kJ/mol
(float64) / 2e-2 (mixed), identical pairs and decisions, positions within
1e-7 / 1e-3 nm."""
import numpy as np
import pytest

from paper_2005_08348_amd import systems as S

pytestmark = pytest.mark.gpu


def _membx():
    from paper_2005_08348_amd import membx
    return membx


def _relaxed(oracle_mod, name):
    s0 = S.make(name)
    o = oracle_mod.Oracle(s0)
    o.minimize(60)
    s = s0.copy()
    s.pos = o.state()["pos"].astype(np.float32).astype(np.float64) % s.box
    s.pos = np.where(s.pos >= s.box, 0.0, s.pos)
    return s


@pytest.fixture(scope="module")
def c0_relaxed(oracle_mod):
    return _relaxed(oracle_mod, "c0")


def _cycles(oracle_mod, sysm, prec, n, P, K, M, **kw):
    m = _membx()
    g = m.System(sysm, precision=prec, rebuild_interval=4, **kw)
    o = oracle_mod.Oracle(sysm)
    g.set_mdas_path(1, 0.05)
    o.set_mdas_path(1, 0.05)
    tol = 1e-6 if prec == "fp64" else 2e-2
    for _ in range(n):
        rg = g.mdas_cycle(P, K, M)
        ro = o.mdas_cycle(P, K, M)
        print(prec, "soft-core work gpu %.8f oracle %.8f" % (rg["work"], ro["work"]))
        assert np.array_equal(rg["pairs"], ro["pairs"])
        assert abs(rg["work"] - ro["work"]) < tol
        assert rg["accept"] == ro["accept"]
    sg, so = g.state(), o.state()
    assert np.array_equal(sg["mol_kind"], so["mol_kind"])
    d = sg["pos"] - so["pos"]
    d -= sysm.box * np.rint(d / sysm.box)
    assert np.abs(d).max() < (1e-7 if prec == "fp64" else 1e-3)
    g.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_softcore_cycles_c0(oracle_mod, c0_relaxed, prec):
    _cycles(oracle_mod, c0_relaxed, prec, 2, 2, 5, 2)


def test_softcore_cycles_charged_exchange(oracle_mod):
    """A <-> D on the mix bilayer: the exchange changes a head charge, so the
    interpolated reaction field is exercised."""
    s = _relaxed(oracle_mod, "mix")
    _cycles(oracle_mod, s, "fp64", 2, 3, 5, 2)


def test_softcore_frozen_equals_linear(oracle_mod, c0_relaxed):
    """M = 0: the soft-core work telescopes to U_B - U_A, the linear path's."""
    m = _membx()
    for K in (1, 7):
        a = m.System(c0_relaxed, precision="fp64")
        b = m.System(c0_relaxed, precision="fp64")
        b.set_mdas_path(1, 0.05)
        ra, rb = a.mdas_cycle(3, K, 0), b.mdas_cycle(3, K, 0)
        assert np.array_equal(ra["pairs"], rb["pairs"])
        assert abs(ra["work"] - rb["work"]) < 1e-8
        a.close(); b.close()


def test_softcore_cycle_c1_mixed(oracle_mod):
    """The 95,876-bead bilayer at the benchmark tuning: 4 pairs, K = 10, M = 1."""
    m = _membx()
    s = S.make("c1")
    g = m.System(s, precision="mixed", skin=0.4, rebuild_interval=7, lanes_per_bead=4)
    g.minimize(50)
    st = g.state()
    o = oracle_mod.Oracle(s)
    o.set_state(pos=st["pos"], vel=st["vel"], mol_kind=st["mol_kind"])
    g.set_mdas_path(1, 0.05)
    o.set_mdas_path(1, 0.05)
    rg = g.mdas_cycle(4, 10, 1)
    ro = o.mdas_cycle(4, 10, 1)
    assert np.array_equal(rg["pairs"], ro["pairs"])
    assert abs(rg["work"] - ro["work"]) < 2e-2
    assert rg["accept"] == ro["accept"]
    d = g.state()["pos"] - o.state()["pos"]
    d -= s.box * np.rint(d / s.box)
    assert np.abs(d).max() < 1e-3
    g.close()


def test_softcore_refused_arguments(c0_relaxed):
    m = _membx()
    g = m.System(c0_relaxed, precision="mixed")
    for path, delta in [(2, 0.05), (1, 0.0), (1, float("nan")), (-1, 0.05)]:
        with pytest.raises(m.MembxError):
            g.set_mdas_path(path, delta)
    g.set_mdas_path(0, 0.0)      # linear: the shift is not used
    g.close()
