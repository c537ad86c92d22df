"""Semi-isotropic pressure coupling (stochastic cell rescaling) on the GPU
against the float64 oracle: same virial, same Philox draw, same scale
factors, so the box and the trajectory follow the oracle's.

Tolerances: float64 box lengths within 1e-11 relative and positions within
1e-7 nm after 20 steps with 4 couplings; mixed box within 1e-6 relative
(the virial carries float32 pair forces) and positions within 1e-4 nm.
"""
import math

import numpy as np
import pytest

from paper_2005_08348_amd import systems as S

pytestmark = pytest.mark.gpu

BARO = dict(p_ref_bar=1.0, compressibility=3e-4, tau_p=1.0)


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


def _pos_err(a, b, box):
    d = a - b
    d -= box * np.rint(d / box)
    return np.abs(d).max()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_barostat_c0(oracle_mod, c0_relaxed, prec):
    m = _membx()
    g = m.System(c0_relaxed, precision=prec, rebuild_interval=5)
    o = oracle_mod.Oracle(c0_relaxed)
    g.set_barostat(5, **BARO)
    o.set_barostat(5, **BARO)
    boxes = []
    for _ in range(4):
        g.md_step(5)
        o.md_step(5)
        bg, bo = g.box(), o.box()
        boxes.append(bo)
        tol = 1e-11 if prec == "fp64" else 1e-6
        assert np.all(np.abs(bg / bo - 1.0) < tol), (bg, bo)
        assert bg[0] == bg[1]
    # the box moved (the start is far from 1 bar)
    assert abs(boxes[-1][2] / c0_relaxed.box[2] - 1.0) > 1e-4
    err = _pos_err(g.state()["pos"], o.state()["pos"], o.box())
    print(prec, "box", g.box(), "pos err %.2e" % err)
    assert err < (1e-7 if prec == "fp64" else 1e-4)
    e = g.energies()
    assert e["n_skin_violations"] == 0
    g.close()


def test_barostat_c1_fp64(oracle_mod):
    """The 95,876-bead bilayer: one coupling after 10 steps, then 10 more."""
    m = _membx()
    s = S.make("c1")
    g = m.System(s, precision="fp64", skin=0.4, rebuild_interval=7, lanes_per_bead=4)
    g.minimize(50)
    st = g.state()
    o = oracle_mod.Oracle(s)
    o.set_state(pos=st["pos"], vel=st["vel"], mol_kind=st["mol_kind"])
    g.set_barostat(10, p_ref_bar=1.0, compressibility=3e-4, tau_p=12.0)
    o.set_barostat(10, p_ref_bar=1.0, compressibility=3e-4, tau_p=12.0)
    g.md_step(20)
    o.md_step(20)
    assert np.all(np.abs(g.box() / o.box() - 1.0) < 1e-11), (g.box(), o.box())
    assert _pos_err(g.state()["pos"], o.state()["pos"], o.box()) < 1e-7
    g.close()


def test_barostat_c1_mixed_run():
    """Mixed precision at the benchmark size, 600 steps with coupling every
    10 (tau_p 12 ps): no list or skin failures, x and y equal, the box
    moves smoothly (per coupling by far less than the skin)."""
    m = _membx()
    s = S.make("c1")
    g = m.System(s, precision="mixed", skin=0.3, rebuild_interval=5, lanes_per_bead=4)
    g.minimize(100)
    g.set_barostat(10, p_ref_bar=1.0, compressibility=3e-4, tau_p=12.0)
    b0 = g.box()
    prev = b0
    for _ in range(60):
        g.md_step(10)
        b = g.box()
        assert b[0] == b[1]
        assert np.all(np.abs(b / prev - 1.0) < 5e-3)
        prev = b
    e = g.energies()
    assert e["n_skin_violations"] == 0
    print("box", b0, "->", g.box(), "P", e["pressure"])
    assert np.any(np.abs(g.box() / b0 - 1.0) > 1e-5)
    g.close()


def test_barostat_refused_arguments(c0_relaxed):
    m = _membx()
    g = m.System(c0_relaxed, precision="mixed")
    for bad in [dict(compressibility=0.0), dict(tau_p=0.0), dict(p_ref_bar=math.nan),
                dict(compressibility=-1.0)]:
        args = dict(BARO)
        args.update(bad)
        with pytest.raises(m.MembxError):
            g.set_barostat(5, **args)
    g.set_barostat(0, **BARO)          # off: always accepted
    b = g.box()
    g.md_step(10)
    assert np.array_equal(g.box(), b)
    g.close()


def test_barostat_c1_pressure_converges():
    """1 ns of the 95,876-bead bilayer under the paper's thermostat and the
    barostat (1 bar, tau_p 12 ps, coupling every 10 steps): over the second
    half the lateral and normal pressures average to the reference within
    30 bar (one sample scatters by about 60 bar; 250 samples, correlated
    over tau_p) and the box settles (its last-quarter drift below 0.2%)."""
    m = _membx()
    s = S.make("c1")
    g = m.System(s, precision="mixed", skin=0.3, rebuild_interval=5, lanes_per_bead=4)
    g.minimize(100)
    g.set_ensemble(1, tau_t=1.0, kind_group=[0, 0, 0, 0, 1])
    g.set_barostat(10, p_ref_bar=1.0, compressibility=3e-4, tau_p=12.0)
    ps, boxes = [], []
    for _ in range(500):
        g.md_step(100)
        e = g.energies(check=False)
        ps.append(e["pressure"])
        boxes.append(g.box())
    assert g.energies()["n_skin_violations"] == 0
    p = np.asarray(ps[250:])
    pa, pz = 0.5 * (p[:, 0] + p[:, 1]), p[:, 2]
    b = np.asarray(boxes)
    print("P_A %.1f +- %.1f, P_z %.1f +- %.1f bar; box %s -> %s"
          % (pa.mean(), pa.std(), pz.mean(), pz.std(), b[0], b[-1]))
    assert abs(pa.mean() - 1.0) < 30.0 and abs(pz.mean() - 1.0) < 30.0
    vol = b[:, 0] * b[:, 1] * b[:, 2]
    assert abs(vol[375:].mean() / vol[-125:].mean() - 1.0) < 2e-3
    g.close()


def test_barostat_shrunk_box_limits_the_skin(c0_relaxed):
    """A box compressed by a high reference pressure: skins that would leave
    fewer than three cells of edge r_cut + skin are refused by set_tuning,
    and the autotuner only tries the ones that fit."""
    m = _membx()
    g = m.System(c0_relaxed, precision="mixed", skin=0.2, rebuild_interval=4)
    g.set_barostat(2, p_ref_bar=3000.0, compressibility=3e-4, tau_p=2.0)
    while g.box()[0] / 3.0 - 1.1 > 0.35:
        g.md_step(2)
    lim = g.box().min() / 3.0 - 1.1
    assert lim < 0.4
    with pytest.raises(m.MembxError):
        g.set_tuning(0.4, 4, 4)
    g.set_barostat(0)
    t = g.autotune(40)
    assert t["skin"] <= lim + 1e-9
    g.md_step(20)
    assert g.energies()["n_skin_violations"] == 0
    g.close()
