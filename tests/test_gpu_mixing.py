"""The mixing observable on the GPU against the oracle: lateral PO4-PO4
pair histograms (one lipid kind, pairs within a leaflet) must be identical,
count for count (integer counts, bins decided on the float64 squared
distance of identical coordinates)."""
import numpy as np
import pytest

from paper_2005_08348_amd import systems as S

pytestmark = pytest.mark.gpu


def _membx():
    from paper_2005_08348_amd import membx
    return membx


def _same_state(o, g):
    st = g.state()
    o.set_state(pos=st["pos"], vel=st["vel"], mol_kind=st["mol_kind"])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_histogram_c0(oracle_mod, prec):
    m = _membx()
    s = S.make("c0")
    g = m.System(s, precision=prec)
    o = oracle_mod.Oracle(s)
    g.md_step(10)
    _same_state(o, g)
    leaf = s.meta["leaflet"]
    for kind in (S.KIND_A, S.KIND_B):
        hg = g.pair_histogram(kind, S.PO4, leaf, 90, 0.05)
        ho = o.pair_histogram(kind, S.PO4, leaf, 90, 0.05)
        assert np.array_equal(hg, ho), kind
        assert hg.sum() > 0
    g.close()


def test_histogram_c1_after_moves(oracle_mod):
    """95,876-bead bilayer after MD steps and an exchange batch (current
    kinds), both swap kinds, 400 bins of 0.05 nm (several pair tiles)."""
    m = _membx()
    s = S.make("c1")
    g = m.System(s, precision="mixed")
    g.md_step(20)
    g.swap_trials(64)
    o = oracle_mod.Oracle(s)
    _same_state(o, g)
    leaf = s.meta["leaflet"]
    for kind in (S.KIND_A, S.KIND_B):
        hg = g.pair_histogram(kind, S.PO4, leaf, 400, 0.05)
        ho = o.pair_histogram(kind, S.PO4, leaf, 400, 0.05)
        assert np.array_equal(hg, ho), kind
    g.close()


def test_histogram_edges(oracle_mod):
    """One bin; a kind with no molecule (all zero); a leaflet mask that
    drops every molecule; bad arguments are refused."""
    m = _membx()
    s = S.make("mix")
    g = m.System(s, precision="fp64")
    o = oracle_mod.Oracle(s)
    leaf = s.meta["leaflet"]
    h1 = g.pair_histogram(S.KIND_A, S.PO4, leaf, 1, 2.0)
    assert np.array_equal(h1, o.pair_histogram(S.KIND_A, S.PO4, leaf, 1, 2.0)) and h1[0] > 0
    assert not g.pair_histogram(S.KIND_B, S.PO4, leaf, 16, 0.1).any()      # no B in "mix"
    assert not g.pair_histogram(S.KIND_A, S.PO4, np.full_like(leaf, -1), 16, 0.1).any()
    with pytest.raises(m.MembxError):
        g.pair_histogram(S.KIND_W, 1, leaf, 16, 0.1)     # water has one bead
    with pytest.raises(m.MembxError):
        g.pair_histogram(S.KIND_A, S.PO4, leaf, 0, 0.1)
    with pytest.raises(m.MembxError):
        g.pair_histogram(S.KIND_A, S.PO4, leaf, 16, -1.0)
    g.close()
