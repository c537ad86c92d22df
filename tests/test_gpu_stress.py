"""The paper's protocol at the benchmark size, all options on, as a long
run: velocity rescaling and the semi-isotropic barostat, exchange batches
between short MD segments, MDAS cycles in between.  Checks what must hold
at any length: finite energies, no list or skin failures, conserved
composition of each swap family, x = y, the force-evaluation count."""
import numpy as np
import pytest

from paper_2005_08348_amd import systems as S

pytestmark = pytest.mark.gpu


def test_paper_protocol_c1_long_run():
    from paper_2005_08348_amd import membx
    s = S.make("c1")
    g = membx.System(s, precision="mixed", skin=0.3, rebuild_interval=5, lanes_per_bead=4)
    g.minimize(100)
    g.set_ensemble(1, tau_t=1.0, kind_group=[1 if k.name == "W" else 0 for k in s.kinds])
    g.set_barostat(10, p_ref_bar=1.0, compressibility=3e-4, tau_p=12.0)
    mk0 = g.state()["mol_kind"].copy()
    fe0 = g.energies()["fe_count"]
    n_md = n_tr = n_cyc = 0
    for block in range(20):
        for _ in range(100):
            g.md_step(10)
            n_md += 10
            r = g.swap_trials(64)
            n_tr += 1
        c = g.mdas_cycle(8, 25, 2)
        n_cyc += 1
        e = g.energies()
        assert np.isfinite(e["total"]) and e["n_skin_violations"] == 0
        b = g.box()
        assert b[0] == b[1] and np.all(b > 4.5)
    mk = g.state()["mol_kind"]
    for k in range(len(s.kinds)):
        assert np.count_nonzero(mk == k) == np.count_nonzero(mk0 == k)
    assert np.any(mk != mk0)                     # exchanges happened
    e = g.energies()
    # one FE per MD step, per exchange batch, per MDAS step (K M per cycle)
    assert e["fe_count"] - fe0 == n_md + n_tr + n_cyc * 25 * 2
    print("box", g.box(), "P", e["pressure"], "T", 2 * e["kinetic"] / (3 * s.n_beads * S.KB))
    g.close()
