"""Failure handling and checkpoint/restart through the C-ABI, every failure
forced from the host so that each kernel runs to its normal end:

* a list capacity below what the system needs: the list build clamps its
  writes at the capacity and raises a sticky flag; every later query returns
  E_LIST_OVERFLOW with the capacity a bead needed, and a system recreated
  with that capacity runs;
* a non-finite coordinate or velocity handed to membx_set_state: rejected
  on the host with E_NONFINITE before anything reaches the device, state
  unchanged;
* a state taken with membx_get_state right after a list rebuild and restored
  into a fresh system continues bit for bit as the run it was taken from
  (same coordinates, velocities, kinds and counters give the same list, the
  same forces and the same Philox noise).
"""
import re

import numpy as np
import pytest

from paper_2005_08348_amd import systems as S

pytestmark = pytest.mark.gpu


def _membx():
    from paper_2005_08348_amd import membx
    return membx


def test_list_capacity_too_small_is_a_clean_error():
    m = _membx()
    c0 = S.make("c0")
    # about 107 neighbours per bead within r_cut + 0.4 nm at this density
    g = m.System(c0, precision="fp64", skin=0.4, list_capacity=96)
    with pytest.raises(m.MembxError) as ei:
        g.md_step(3)
        g.energies()
    assert ei.value.code == 4
    msg = str(ei.value)
    print(msg)
    need = int(re.search(r"needed (\d+) entries", msg).group(1))
    assert need > 96
    with pytest.raises(m.MembxError) as ei2:     # sticky
        g.energies()
    assert ei2.value.code == 4
    g.close()
    cap = (need + 7) // 8 * 8 + 16
    g2 = m.System(c0, precision="fp64", skin=0.4, list_capacity=cap)
    g2.minimize(20)
    g2.md_step(3)
    assert g2.energies()["n_list_entries"] > 0
    g2.close()


@pytest.mark.parametrize("what", ["pos", "vel"])
def test_nonfinite_state_is_rejected(what):
    m = _membx()
    c0 = S.make("c0")
    g = m.System(c0, precision="mixed")
    g.minimize(20)
    before = g.state()
    bad = before[what].copy()
    bad[17, 1] = np.nan if what == "pos" else np.inf
    with pytest.raises(m.MembxError) as ei:
        g.set_state(**{what: bad})
    assert ei.value.code == 5
    after = g.state()
    for k in ("pos", "vel", "mol_kind"):
        assert np.array_equal(before[k], after[k])
    g.md_step(2)
    g.energies()
    g.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_checkpoint_restart_is_bit_identical(prec):
    """C1 at the bench's tuning (list rebuilt every 7 steps, graphs, fused
    force pass): checkpoint after 14 steps and a batch of exchange trials,
    then 10 more steps in the original system and in a fresh one restored
    from the checkpoint."""
    m = _membx()
    c1 = S.make("c1")
    tun = dict(skin=0.4, rebuild_interval=7, lanes_per_bead=4)
    a = m.System(c1, precision=prec, **tun)
    a.minimize(50)
    a.md_step(7)
    a.swap_trials(64, results=False)
    a.md_step(7)           # the list is rebuilt at this step
    ck = a.state()
    a.md_step(10)
    ra = a.state()
    ea = a.energies()
    a.close()
    b = m.System(c1, precision=prec, **tun)
    b.set_state(pos=ck["pos"], vel=ck["vel"], mol_kind=ck["mol_kind"],
                counters=[ck["step"], ck["batch"], ck["cycle"]])
    b.md_step(10)
    rb = b.state()
    eb = b.energies()
    b.close()
    assert ck["step"] == 14 and ck["batch"] == 1
    assert rb["step"] == ra["step"] == 24
    for k in ("pos", "vel", "mol_kind"):
        assert np.array_equal(ra[k], rb[k]), k
    assert ea["potential"] == eb["potential"]
