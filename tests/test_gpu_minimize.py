"""The GPU steepest-descent hook (membx_minimize, used at every serving
admission and at the start of the bench) against the oracle's o_minimize on
the unrelaxed C0 structure, whose overlaps make most steps hit the step cap:
20 iterations of x += alpha F, shortened to at most the cap, each from the
forces of the current coordinates.

Tolerances: float64 form 1e-9 nm per coordinate (a capped step is a
normalised force direction, so force errors of 1e-10 relative move beads by
far less); mixed form 1e-4 nm (float32 coordinates and forces)."""
import numpy as np
import pytest

from paper_2005_08348_amd import systems as S

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("mixed", 1e-4)])
def test_minimizer_matches_oracle(oracle_mod, prec, tol):
    from paper_2005_08348_amd import membx as M
    s = S.make("c0")
    o = oracle_mod.Oracle(s)
    g = M.System(s, precision=prec)
    o.minimize(20, 1e-4, 0.01)
    g.minimize(20, 1e-4, 0.01)
    d = g.state()["pos"] - o.state()["pos"]
    d -= s.box * np.rint(d / s.box)
    moved = s.pos - o.state()["pos"]
    moved -= s.box * np.rint(moved / s.box)
    print(f"{prec}: max |dx| {np.abs(d).max():.2e} nm, largest move {np.abs(moved).max():.3f} nm")
    assert np.abs(moved).max() > 0.05          # the structure did relax
    assert np.abs(d).max() < tol
    eg, eo = g.energies(), o.energy_forces()
    assert abs(eg["potential"] - eo["potential"]) < (1e-9 if prec == "fp64" else 1e-4) * abs(eo["potential"])
    g.close()
