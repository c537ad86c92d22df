"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function include/membx.h declares, and validates descriptors."""
import numpy as np
import pytest

from paper_2005_08348_amd import membx as M
from paper_2005_08348_amd import systems as S


def test_exports_every_declared_symbol():
    names = M.header_symbols()
    assert len(names) >= 15
    L = M.lib()
    for n in names:
        assert hasattr(L, n), n


def test_arena_size_scales_with_system():
    b0 = M.arena_bytes(S.make("c0"), "mixed")
    b64 = M.arena_bytes(S.make("c0"), "fp64")
    assert 0 < b0 < b64


def test_descriptor_validation():
    s = S.make("c0")
    bad = s.copy()
    bad.box = np.array([2.0, 2.0, 2.0])        # smaller than 3 (r_cut + skin)
    with pytest.raises(M.MembxError) as e:
        M.arena_bytes(bad)
    assert e.value.code == M.E_INVAL
    bad = s.copy()
    bad.mol_kind = bad.mol_kind.copy()
    bad.mol_kind[0] = 99
    with pytest.raises(M.MembxError):
        M.arena_bytes(bad)
    with pytest.raises(M.MembxError):
        M.arena_bytes(s, lanes_per_bead=3)
    # a family whose kinds differ in their number of beads is rejected (the
    # 8-bead sterol beside the 12-bead lipids) ...
    k = S.standard_kinds()
    k[S.KIND_C].family = 0
    bad = s.copy()
    bad.kinds = k
    with pytest.raises(M.MembxError):
        M.arena_bytes(bad)
    # ... one whose kinds differ only in bonded terms (the sterol padded to
    # 12 slots with dummy beads) is a topology-changing family, accepted
    assert M.arena_bytes(S.make("topo")) > 0


def test_no_cpu_fallback():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        M.System(S.make("c0"))


def test_list_capacity_rounds_to_the_list_tiling():
    """The neighbour list is tiled in rows of 64 / lanes_per_bead beads, so a
    requested capacity is rounded up to a multiple of 8 entries: 97..104
    give the arena of 104, and 105 a larger one."""
    s = S.make("c0")
    b = [M.arena_bytes(s, "mixed", list_capacity=k) for k in (97, 100, 104, 105)]
    assert b[0] == b[1] == b[2] < b[3]
