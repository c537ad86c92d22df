"""membx_energies_noalloc (the energy query for callers that cannot
allocate) against membx_energies through the C-ABI: the same kernels with
the partials in the library's static device array, so the results must be
identical bit for bit.  Two calls in a row, the second on a smaller system,
so that the second reads nothing the first left behind."""
import ctypes as C

import numpy as np
import pytest

from paper_2005_08348_amd import systems as S

pytestmark = pytest.mark.gpu


def _both(g):
    from paper_2005_08348_amd import membx as M
    L = M.lib()
    ea, eb = M.Energy(), M.Energy()
    ra = L.membx_energies(g.h, C.byref(ea))
    rb = L.membx_energies_noalloc(g.h, C.byref(eb))
    assert ra == 0 and rb == 0, (ra, rb, L.membx_last_error(g.h))
    return ea, eb


def _same(ea, eb):
    from paper_2005_08348_amd import membx as M
    for name, _ in M.Energy._fields_:
        a, b = getattr(ea, name), getattr(eb, name)
        if hasattr(a, "__len__"):
            assert list(a) == list(b), name
        else:
            assert a == b, (name, a, b)


def test_noalloc_energies_equal_arena_energies():
    from paper_2005_08348_amd import membx as M
    big = M.System(S.make("c1"), precision="mixed")
    big.minimize(60)
    big.md_step(7)
    ea, eb = _both(big)
    _same(ea, eb)
    assert ea.n_pairs_in_cutoff > 1_000_000
    big.close()
    small = M.System(S.make("c0"), precision="fp64")
    small.minimize(30)
    small.md_step(3)
    ea2, eb2 = _both(small)
    _same(ea2, eb2)
    assert 0 < ea2.n_pairs_in_cutoff < 100_000
    # a repeat on the small system reads the same
    _, eb3 = _both(small)
    _same(eb2, eb3)
    small.close()


def test_noalloc_rejects_null_handle():
    from paper_2005_08348_amd import membx as M
    e = M.Energy()
    assert M.lib().membx_energies_noalloc(None, C.byref(e)) == M.E_INVAL
