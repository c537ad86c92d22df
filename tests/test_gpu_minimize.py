"""The GPU steepest-descent hook (membx_minimize, used at every serving
admission and at the start of the bench) against the oracle's o_minimize on
the unrelaxed C0 structure, whose overlaps make most steps hit the step cap:
20 iterations of x += alpha F, shortened to at most the cap, each from the
forces of the current coordinates.

Tolerances: float64 form 1e-9 nm per coordinate after 20 iterations (a
capped step is a normalised force direction, so force errors of 1e-10
relative move beads by far less).  Mixed form: one iteration within 2e-5 nm
(float32 rounding of coordinates and of the step); over 20 iterations the
difference is not bounded by rounding, since an uncapped step alpha F on a
bead in a stiff contact (alpha dF/dx ~ 100) amplifies the float32 position
rounding (measured: 99th percentile 1.1e-4 nm, max 6.4e-4 nm), so the
mixed form is held to relaxing as far: potential energy within 1e-3 of the
oracle's after 20 iterations."""
import numpy as np
import pytest

from paper_2005_08348_amd import systems as S

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_minimizer_matches_oracle(oracle_mod, prec):
    from paper_2005_08348_amd import membx as M
    s = S.make("c0")
    o = oracle_mod.Oracle(s)
    g = M.System(s, precision=prec)
    n1 = 20 if prec == "fp64" else 1
    o.minimize(n1, 1e-4, 0.01)
    g.minimize(n1, 1e-4, 0.01)
    d = g.state()["pos"] - o.state()["pos"]
    d -= s.box * np.rint(d / s.box)
    moved = s.pos - o.state()["pos"]
    moved -= s.box * np.rint(moved / s.box)
    print(f"{prec}: {n1} iterations, max |dx| {np.abs(d).max():.2e} nm, "
          f"largest move {np.abs(moved).max():.3f} nm")
    assert np.abs(moved).max() >= 0.0099        # steps were taken (capped at 0.01 nm)
    assert np.abs(d).max() < (1e-9 if prec == "fp64" else 2e-5)
    if prec == "mixed":
        o.minimize(19, 1e-4, 0.01)
        g.minimize(19, 1e-4, 0.01)
    eg, eo = g.energies(), o.energy_forces()
    print(f"{prec}: potential {eg['potential']:.6f} vs {eo['potential']:.6f}")
    assert abs(eg["potential"] - eo["potential"]) < (1e-9 if prec == "fp64" else 1e-3) * abs(eo["potential"])
    g.close()
