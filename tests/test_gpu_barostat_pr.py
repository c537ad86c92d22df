"""The paper's barostat, semi-isotropic Parrinello-Rahman, on the GPU against
the float64 oracle: same pressure tensor, same box impulse, same scaling of
coordinates and velocities, so box, box velocity and trajectory follow the
oracle's.

Tolerances as for the cell-rescaling barostat: float64 box lengths within
1e-11 relative, box velocities within 1e-9 of their scale, positions within
1e-7 nm after 20 steps with 4 couplings; mixed box within 1e-6 relative
(the virial carries float32 pair forces), box velocities within 1e-3 of
their scale (the impulse is the small difference P - P0 of pressures
whose float32 terms are much larger), positions within 1e-4 nm.
"""
import math

import numpy as np
import pytest

from paper_2005_08348_amd import systems as S

pytestmark = pytest.mark.gpu

PR = dict(p_ref_bar=1.0, compressibility=3e-4, tau_p=1.0)
GROUPS = [0, 0, 0, 0, 1]          # membrane kinds, water


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
def test_pr_c0(oracle_mod, c0_relaxed, prec):
    m = _membx()
    g = m.System(c0_relaxed, precision=prec, rebuild_interval=5)
    o = oracle_mod.Oracle(c0_relaxed)
    g.set_barostat_pr(5, **PR)
    o.set_barostat_pr(5, **PR)
    tol = 1e-11 if prec == "fp64" else 1e-6
    for _ in range(4):
        g.md_step(5)
        o.md_step(5)
        bg, bo = g.box(), o.box()
        assert np.all(np.abs(bg / bo - 1.0) < tol), (bg, bo)
        assert bg[0] == bg[1]
        (vg, hg), (vo, ho) = g.barostat_state(), o.barostat_state()
        scale = np.abs(vo).max()
        assert np.all(np.abs(vg - vo) <= (1e-9 if prec == "fp64" else 1e-3) * scale), (vg, vo)
        assert abs(hg - ho) <= (1e-9 if prec == "fp64" else 1e-3) * abs(ho)
    assert abs(g.box()[2] / c0_relaxed.box[2] - 1.0) > 1e-4      # the box moved
    err = _pos_err(g.state()["pos"], o.state()["pos"], o.box())
    verr = np.abs(g.state()["vel"] - o.state()["vel"]).max()
    print(prec, "box", g.box(), "pos err %.2e, vel err %.2e" % (err, verr))
    assert err < (1e-7 if prec == "fp64" else 1e-4)
    if prec == "fp64":
        assert verr < 1e-6
    assert g.energies()["n_skin_violations"] == 0
    g.close()


def test_pr_paper_ensemble_fp64_c0(oracle_mod, c0_relaxed):
    """Velocity rescaling of two groups with Parrinello-Rahman, the paper's
    ensemble, through MD, an exchange batch, an MDAS cycle and a restart of
    the box velocity."""
    m = _membx()
    g = m.System(c0_relaxed, precision="fp64", rebuild_interval=4)
    o = oracle_mod.Oracle(c0_relaxed)
    for obj in (g, o):
        obj.set_ensemble(1, tau_t=0.5, kind_group=GROUPS)
        obj.set_barostat_pr(5, p_ref_bar=1.0, compressibility=3e-4, tau_p=2.0)
    for _ in range(2):
        g.md_step(10)
        o.md_step(10)
        assert np.all(np.abs(g.box() / o.box() - 1.0) < 1e-11), (g.box(), o.box())
        rg, ro = g.swap_trials(4), o.swap_batch(4)
        assert list(rg["X"]) == list(ro["X"]) and list(rg["accept"]) == list(ro["accept"])
        mg, mo = g.mdas_cycle(2, 5, 2), o.mdas_cycle(2, 5, 2)
        assert np.array_equal(mg["pairs"], mo["pairs"])
        assert abs(mg["work"] - mo["work"]) < 1e-6
    # a changed box velocity takes effect at the next coupling on both sides
    vo, _ = o.barostat_state()
    nv = vo * 0.5 + np.array([1e-3, 1e-3, -2e-3])
    g.barostat_state(set_box_vel=nv)
    o.set_box_velocity(nv)
    g.md_step(10)
    o.md_step(10)
    assert np.all(np.abs(g.box() / o.box() - 1.0) < 1e-11), (g.box(), o.box())
    assert _pos_err(g.state()["pos"], o.state()["pos"], o.box()) < 1e-7
    g.close()


def test_pr_c1_fp64(oracle_mod):
    """The 95,876-bead bilayer: couplings every 10 steps over 30 steps at the
    paper's settings (1 bar, tau_p 12 ps)."""
    m = _membx()
    s = S.make("c1")
    g = m.System(s, precision="fp64", skin=0.4, rebuild_interval=7, lanes_per_bead=4)
    g.minimize(50)
    st = g.state()
    o = oracle_mod.Oracle(s)
    o.set_state(pos=st["pos"], vel=st["vel"], mol_kind=st["mol_kind"])
    g.set_barostat_pr(10, p_ref_bar=1.0, compressibility=3e-4, tau_p=12.0)
    o.set_barostat_pr(10, p_ref_bar=1.0, compressibility=3e-4, tau_p=12.0)
    g.md_step(30)
    o.md_step(30)
    assert np.all(np.abs(g.box() / o.box() - 1.0) < 1e-11), (g.box(), o.box())
    assert _pos_err(g.state()["pos"], o.state()["pos"], o.box()) < 1e-7
    g.close()


def test_pr_c1_paper_ensemble_run():
    """0.5 ns of the 95,876-bead bilayer in the paper's ensemble (velocity
    rescaling of two groups, tau_t 1 ps; Parrinello-Rahman, 1 bar, tau_p 12
    ps, coupling every 10 steps), mixed precision, after 200 ps under the
    overdamped cell rescaling (the synthetic start is hundreds of bar from
    1 bar, and the undamped Parrinello-Rahman box would swing by about
    beta dP = 10% from there): no list or skin failures, x and y equal, the
    box moves by less than 3% per 100 steps, and over the second half the
    lateral and normal pressures average to the reference within 40 bar
    (the box swings with period tau_p about its equilibrium; 125
    samples)."""
    m = _membx()
    s = S.make("c1")
    g = m.System(s, precision="mixed", skin=0.3, rebuild_interval=5, lanes_per_bead=4)
    g.minimize(100)
    g.set_ensemble(1, tau_t=1.0, kind_group=GROUPS)
    g.set_barostat(10, p_ref_bar=1.0, compressibility=3e-4, tau_p=1.0)
    g.md_step(10000)
    g.set_barostat_pr(10, p_ref_bar=1.0, compressibility=3e-4, tau_p=12.0)
    ps, boxes = [], []
    prev = g.box()
    for _ in range(250):
        g.md_step(100)
        e = g.energies(check=False)
        ps.append(e["pressure"])
        b = g.box()
        assert b[0] == b[1]
        assert np.all(np.abs(b / prev - 1.0) < 3e-2)
        prev = b
        boxes.append(b)
    assert g.energies()["n_skin_violations"] == 0
    p = np.asarray(ps[125:])
    pa, pz = 0.5 * (p[:, 0] + p[:, 1]), p[:, 2]
    b = np.asarray(boxes)
    print("P_A %.1f +- %.1f, P_z %.1f +- %.1f bar; box %s -> %s"
          % (pa.mean(), pa.std(), pz.mean(), pz.std(), b[0], b[-1]))
    assert abs(pa.mean() - 1.0) < 40.0 and abs(pz.mean() - 1.0) < 40.0
    g.close()


def test_pr_refused_arguments(c0_relaxed):
    m = _membx()
    g = m.System(c0_relaxed, precision="mixed")
    for bad in [dict(compressibility=0.0), dict(tau_p=0.0), dict(p_ref_bar=math.nan)]:
        args = dict(PR)
        args.update(bad)
        with pytest.raises(m.MembxError):
            g.set_barostat_pr(5, **args)
    with pytest.raises(m.MembxError):
        g.barostat_state(set_box_vel=[0.0, math.inf, 0.0])
    g.close()
