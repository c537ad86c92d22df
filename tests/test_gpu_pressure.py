"""Virial and pressure tensor diagonal on the GPU (energy pass) against the
float64 oracle.

Tolerances: float64 1e-10 of the sum of |terms| of W_aa; mixed 1e-6 of it
(pair and bonded forces in float32, relative error ~6e-8 per term, summed
in float64; a pair that float32 rounding moves across the cutoff changes W
by about F(r_c) r_c ~ 1e-2 kJ/mol, far below).  sum m v_a^2 relative
1e-12 / 1e-6 (velocities stored in float32 in the mixed form).
"""
import numpy as np
import pytest

from paper_2005_08348_amd import systems as S

pytestmark = pytest.mark.gpu


def _membx():
    from paper_2005_08348_amd import membx
    return membx


def oracle_bar():
    from oracle import oracle as O
    return O.BAR


def _compare(g, o, prec):
    e = g.energies()
    st = g.state()
    o.set_state(pos=st["pos"], vel=st["vel"], mol_kind=st["mol_kind"])
    ref = o.virial()
    tw = 1e-10 if prec == "fp64" else 1e-6
    tk = 1e-12 if prec == "fp64" else 1e-6
    vol = float(np.prod(o.system.box))
    for a in range(3):
        err_w = tw * ref["w_abs"][a]
        assert abs(e["virial"][a] - ref["w"][a]) < err_w, (a, e["virial"], ref["w"], ref["w_abs"])
        assert abs(e["mv2"][a] - ref["mv2"][a]) < tk * ref["mv2"][a] + 1e-9
        err_p = (err_w + tk * ref["mv2"][a] + 1e-9) / vol * oracle_bar()
        assert abs(e["pressure"][a] - ref["pressure"][a]) < err_p
    return e, ref


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_virial_c0(oracle_mod, prec):
    m = _membx()
    c0 = S.make("c0")
    g = m.System(c0, precision=prec)
    g.minimize(40)
    g.md_step(30)
    o = oracle_mod.Oracle(c0)
    e, ref = _compare(g, o, prec)
    print(prec, "P_aa (bar)", e["pressure"], "oracle", ref["pressure"])
    g.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_virial_c1(oracle_mod, prec):
    """The 95,876-bead bilayer after minimisation and 30 steps (list several
    steps old, bonds across the periodic boundaries)."""
    m = _membx()
    c1 = S.make("c1")
    g = m.System(c1, precision=prec, skin=0.4, rebuild_interval=7, lanes_per_bead=4)
    g.minimize(50)
    g.md_step(30)
    o = oracle_mod.Oracle(c1)
    _compare(g, o, prec)
    g.close()
