"""Every option at once against the oracle (float64 C0): the paper's
thermostat, the semi-isotropic barostat, interleaflet exchange partners and
the soft-core MDAS path, through a sequence of MD segments, exchange
batches and MDAS cycles.  Tolerances as in the single-feature tests."""
import numpy as np
import pytest

from paper_2005_08348_amd import systems as S

pytestmark = pytest.mark.gpu

GROUPS = [0, 0, 0, 0, 1]


@pytest.fixture(scope="module")
def c0_relaxed(oracle_mod):
    c0 = S.make("c0")
    o = oracle_mod.Oracle(c0)
    o.minimize(60)
    s = c0.copy()
    s.pos = o.state()["pos"].astype(np.float32).astype(np.float64) % s.box
    s.pos = np.where(s.pos >= s.box, 0.0, s.pos)
    return s


def test_all_options_fp64_c0(oracle_mod, c0_relaxed):
    from paper_2005_08348_amd import membx
    g = membx.System(c0_relaxed, precision="fp64", rebuild_interval=4)
    o = oracle_mod.Oracle(c0_relaxed)
    lf = np.maximum(c0_relaxed.meta["leaflet"], 0)
    for obj in (g, o):
        obj.set_ensemble(1, tau_t=0.5, kind_group=GROUPS)
        obj.set_barostat(5, p_ref_bar=1.0, compressibility=3e-4, tau_p=2.0)
        obj.set_exchange_regions(2, lf)
        obj.set_mdas_path(1, 0.05)
    for rnd in range(2):
        g.md_step(10)
        o.md_step(10)
        assert np.all(np.abs(g.box() / o.box() - 1.0) < 1e-11), (rnd, g.box(), o.box())
        rg, ro = g.swap_trials(4), o.swap_batch(4)
        assert list(rg["X"]) == list(ro["X"]) and list(rg["Y"]) == list(ro["Y"])
        assert np.abs(rg["du"] - ro["du"]).max() < 1e-8
        assert list(rg["accept"]) == list(ro["accept"])
        mg, mo = g.mdas_cycle(2, 5, 2), o.mdas_cycle(2, 5, 2)
        assert np.array_equal(mg["pairs"], mo["pairs"])
        assert abs(mg["work"] - mo["work"]) < 1e-6
        assert mg["accept"] == mo["accept"]
    sg, so = g.state(), o.state()
    assert np.array_equal(sg["mol_kind"], so["mol_kind"])
    box = o.box()
    d = sg["pos"] - so["pos"]
    d -= box * np.rint(d / box)
    assert np.abs(d).max() < 1e-7
    assert np.abs(sg["vel"] - so["vel"]).max() < 1e-6
    e, eo = g.energies(), o.virial()
    assert np.all(np.abs(e["virial"] - eo["w"]) < 1e-9 * eo["w_abs"])
    g.close()
