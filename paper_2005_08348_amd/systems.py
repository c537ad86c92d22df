"""Seeded synthetic membrane systems (input generation only).

This module builds the inputs that both the GPU library and the CPU oracle
consume: molecule kinds (bead types, charges, masses, bonded topology, swap
family), the molecule list, bead coordinates and velocities, the box and the
force-field and integrator settings.  It performs none of the method's
arithmetic (no energies, forces, integration or Metropolis tests): it only
places beads on jittered lattices and draws seeded random numbers.

Workloads follow the paper's test system (a 1:1 two-lipid Martini bilayer
with ~0.64 nm^2 per lipid and Martini water, Section 3) scaled to the sizes
this project benchmarks:

* ``c0``  64 lipids (A:B 32:32) + 640 W, box 4.53 x 4.53 x 9.0 nm
* ``c1``  4096 lipids (A:B:C 1639:1638:819) + 50 000 W, 36.2 x 36.2 x 10 nm
* ``c3``  49 152 lipids (A:B:C:D 30:30:20:20) + 590 000 W, 125.4 x 125.4 x 11 nm
* ``job`` serving jobs of a requested size built like ``c1``

Kinds: A is a 12-bead saturated lipid (NC3 +1, PO4 -1, GL1, GL2, two 4-bead
tails); B is A with the third bead of each tail unsaturated; D is A with a -1
head charge; C is an 8-bead sterol-like molecule; W is one water bead.
A, B and D form swap family 0 (identical topology); C and W never swap.
``topo`` (C0's shape) puts A and S12, the sterol padded to 12 bead slots
with four dummy beads, in one family: a topology-changing exchange.

Coordinates lie in [0, L) per axis and are rounded to float32-representable
values, as are the box lengths and velocities, so that a float32 and a
float64 consumer start from bit-identical inputs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Bead types: 0 Q (charged head), 1 N (glycerol / sterol polar),
# 2 C (saturated tail, sterol ring/tail), 3 U (unsaturated tail), 4 W (water).
TYPE_Q, TYPE_N, TYPE_C, TYPE_U, TYPE_W = 0, 1, 2, 3, 4
N_TYPES = 5
# a bead with no Lennard-Jones interaction (a sixth type, only in systems
# with topology-changing exchanges, whose epsilon row and column are zero)
TYPE_DUMMY = 5
EPS_LEVELS = (5.6, 5.0, 4.5, 4.0, 3.5, 3.1, 2.7, 2.3, 2.0)  # kJ/mol
SIGMA = 0.47  # nm
MASS = 72.0  # amu
KB = 0.00831446261815324  # kJ/mol/K (used only to draw initial velocities)

SEEDS = {"c0": 200508348000, "c1": 200508348001, "c2": 200508348002,
         "c3": 200508348003, "mix": 200508348010, "topo": 200508348020}
PO4 = 1   # bead index of the phosphate in the lipid kinds A, B and D


@dataclass
class Kind:
    name: str
    types: list
    charges: list
    bonds: list = field(default_factory=list)    # (i, j, b0 nm, k kJ/mol/nm^2)
    angles: list = field(default_factory=list)   # (i, j, k, theta0 deg, k kJ/mol)
    family: int = -1
    masses: list | None = None

    def __post_init__(self):
        if self.masses is None:
            self.masses = [MASS] * len(self.types)

    @property
    def n(self):
        return len(self.types)


@dataclass
class System:
    """A complete simulation input.  All arrays are numpy, float64 unless noted."""
    name: str
    kinds: list              # list[Kind]
    mol_kind: np.ndarray     # int32 [n_mols]
    pos: np.ndarray          # [N, 3] in [0, L)
    vel: np.ndarray          # [N, 3]
    box: np.ndarray          # [3]
    eps: np.ndarray          # [nt, nt] LJ epsilon
    sigma: np.ndarray        # [nt, nt] LJ sigma
    rc: float = 1.1
    eps_r: float = 15.0
    eps_rf: float = math.inf
    dt: float = 0.02
    temperature: float = 323.0
    gamma: float = 1.0
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n_beads(self):
        return int(self.pos.shape[0])

    @property
    def n_mols(self):
        return int(self.mol_kind.shape[0])

    def mol_first(self):
        sizes = np.array([self.kinds[k].n for k in self.mol_kind], dtype=np.int64)
        first = np.zeros(len(sizes), dtype=np.int64)
        if len(sizes):
            first[1:] = np.cumsum(sizes)[:-1]
        return first, sizes

    def copy(self):
        import copy as _c
        return _c.deepcopy(self)


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


# ---------------------------------------------------------------- kinds
def lipid_kind(name, tail3_type, head_charge, family=0):
    types = [TYPE_Q, TYPE_Q, TYPE_N, TYPE_N,
             TYPE_C, TYPE_C, tail3_type, TYPE_C,
             TYPE_C, TYPE_C, tail3_type, TYPE_C]
    charges = [head_charge, -1.0, 0.0, 0.0] + [0.0] * 8
    # 0 NC3 1 PO4 2 GL1 3 GL2 4 C1A 5 C2A 6 C3A 7 C4A 8 C1B 9 C2B 10 C3B 11 C4B
    bl = [(0, 1), (1, 2), (2, 3), (2, 4), (4, 5), (5, 6), (6, 7),
          (3, 8), (8, 9), (9, 10), (10, 11)]
    bonds = [(i, j, 0.47, 1250.0) for i, j in bl]
    al = [(1, 2, 4), (2, 4, 5), (4, 5, 6), (5, 6, 7),
          (3, 8, 9), (8, 9, 10), (9, 10, 11)]
    angles = [(i, j, k, 180.0, 25.0) for i, j, k in al]
    return Kind(name, types, charges, bonds, angles, family)


def sterol_kind():
    # 0 P0, 1..4 ring R1..R4, 5..7 tail T5..T7
    types = [TYPE_N] + [TYPE_C] * 7
    charges = [0.0] * 8
    d = 0.47 * math.sqrt(2.0)
    bonds = [(0, 1, 0.47, 1250.0),
             (1, 2, 0.47, 5000.0), (2, 3, 0.47, 5000.0), (3, 4, 0.47, 5000.0),
             (4, 1, 0.47, 5000.0), (1, 3, d, 5000.0), (2, 4, d, 5000.0),
             (3, 5, 0.47, 1250.0), (5, 6, 0.47, 1250.0), (6, 7, 0.47, 1250.0)]
    angles = [(0, 1, 3, 180.0, 25.0), (1, 3, 5, 180.0, 25.0),
              (3, 5, 6, 180.0, 25.0), (5, 6, 7, 180.0, 25.0)]
    return Kind("C", types, charges, bonds, angles, -1)


def sterol12_kind(family=0):
    """The sterol padded to the lipids' 12 bead slots for a topology-changing
    exchange family with them: slots 0-7 the sterol, slots 8-11 dummy beads
    (type TYPE_DUMMY: no Lennard-Jones, no charge) held by a chain of bonds
    from slot 3, the way the lipid's second tail hangs from its GL2.  In an
    exchange with a lipid the dummies become a tail and four lipid beads
    become sterol beads or vanish."""
    st = sterol_kind()
    types = list(st.types) + [TYPE_DUMMY] * 4
    charges = list(st.charges) + [0.0] * 4
    bonds = list(st.bonds) + [(3, 8, 0.47, 1250.0), (8, 9, 0.47, 1250.0),
                              (9, 10, 0.47, 1250.0), (10, 11, 0.47, 1250.0)]
    angles = list(st.angles) + [(8, 9, 10, 180.0, 25.0), (9, 10, 11, 180.0, 25.0)]
    return Kind("S12", types, charges, bonds, angles, family)


def water_kind():
    return Kind("W", [TYPE_W], [0.0], [], [], -1)


def standard_kinds():
    """Kind list in id order A, B, C, D, W."""
    return [lipid_kind("A", TYPE_C, +1.0), lipid_kind("B", TYPE_U, +1.0),
            sterol_kind(), lipid_kind("D", TYPE_C, -1.0), water_kind()]


KIND_A, KIND_B, KIND_C, KIND_D, KIND_W = 0, 1, 2, 3, 4


def epsilon_matrix(rng):
    """Symmetric type x type epsilon from a seeded draw of level indices
    (upper triangle in row-major order, level = floor(9 u))."""
    eps = np.zeros((N_TYPES, N_TYPES))
    for i in range(N_TYPES):
        for j in range(i, N_TYPES):
            lvl = min(int(math.floor(9.0 * rng.random())), 8)
            eps[i, j] = eps[j, i] = EPS_LEVELS[lvl]
    return eps


def largest_remainder(total, fractions):
    raw = [total * f for f in fractions]
    counts = [int(math.floor(r)) for r in raw]
    rem = total - sum(counts)
    order = sorted(range(len(fractions)), key=lambda i: (-(raw[i] - counts[i]), i))
    for i in order[:rem]:
        counts[i] += 1
    return counts


def _grid_dims(n):
    """Factor n lipids per leaflet into nx >= ny with nx ~ 2 ny when possible."""
    best = None
    for ny in range(1, int(math.isqrt(n)) + 1):
        if n % ny:
            continue
        nx = n // ny
        score = abs(math.log(nx / ny) - math.log(2.0))
        if best is None or score < best[0]:
            best = (score, nx, ny)
    return best[1], best[2]


# ---------------------------------------------------------------- bilayer
def _lipid_template(kind_id, d, s=0.235):
    """Local coordinates (u, w, z) of a molecule with its head at z=0 and the
    tails pointing to -z.  u is the GL1->GL2 direction."""
    if kind_id == KIND_C:
        a = 0.33
        return np.array([
            [0.0, 0.0, -2.0 * d], [0.0, 0.0, -2.6 * d], [a, 0.0, -3.2 * d],
            [0.0, 0.0, -3.8 * d], [-a, 0.0, -3.2 * d], [0.0, 0.0, -4.6 * d],
            [0.0, 0.0, -5.3 * d], [0.0, 0.0, -6.0 * d]])
    return np.array([
        [0.0, 0.0, 0.0], [0.0, 0.0, -d],
        [-s, 0.0, -2 * d], [s, 0.0, -2 * d],
        [-s, 0.0, -3 * d], [-s, 0.0, -4 * d], [-s, 0.0, -5 * d], [-s, 0.0, -6 * d],
        [s, 0.0, -3 * d], [s, 0.0, -4 * d], [s, 0.0, -5 * d], [s, 0.0, -6 * d]])


def bilayer(name, n_per_leaflet, fractions, n_water, box_xy, box_z, seed,
            kinds=None, jitter=0.05, wobble_deg=10.0, demix=False, lipid_kinds=None):
    """Two-leaflet bilayer on an nx x ny grid per leaflet, kinds assigned by a
    seeded permutation with largest-remainder counts, water on a jittered
    lattice filling the rest of the periodic box.  ``demix``: each leaflet
    is instead filled column by column (along x) in kind order, so that each
    kind forms one stripe (a far-from-mixed start).  ``lipid_kinds``: the
    kind of each fraction (default 0, 1, 2, ...)."""
    rng = np.random.default_rng(seed)
    kinds = kinds if kinds is not None else standard_kinds()
    eps = epsilon_matrix(rng)
    n_lip = 2 * n_per_leaflet
    lipid_kinds = list(lipid_kinds) if lipid_kinds is not None else list(range(len(fractions)))
    counts = largest_remainder(n_lip, fractions)
    assign = np.concatenate([np.full(c, k, dtype=np.int32)
                             for k, c in zip(lipid_kinds, counts)])
    assign = assign[rng.permutation(n_lip)]
    Lx = float(np.float32(box_xy))
    Ly = Lx
    Lz = float(np.float32(box_z))
    nx, ny = _grid_dims(n_per_leaflet)
    if demix:
        per_leaf = largest_remainder(n_per_leaflet, fractions)
        stripe = np.concatenate([np.full(c, k, dtype=np.int32)
                                 for k, c in zip(lipid_kinds, per_leaf)])
        sites = np.arange(n_per_leaflet)
        order = np.lexsort((sites // nx, sites % nx))   # by column x, then row
        leaf_assign = np.empty(n_per_leaflet, dtype=np.int32)
        leaf_assign[order] = stripe
        assign = np.concatenate([leaf_assign, leaf_assign])
        counts = [2 * c for c in per_leaf]
    ax, ay = Lx / nx, Ly / ny
    area = Lx * Ly
    # depth step: fit the bilayer and a water slab of density ~8.36 /nm^3
    h_w = n_water / (area * 8.36) if n_water else 0.0
    d = (Lz - h_w - 3 * 0.47) / 12.0
    d = min(0.47, max(0.38, d))
    zmid = 0.5 * Lz
    head_up = zmid + 0.235 + 6 * d
    head_lo = zmid - 0.235 - 6 * d
    along_y = ay >= ax
    pos, mol_kind = [], []
    wob = math.radians(wobble_deg)
    for leaf in (0, 1):
        for s_idx in range(n_per_leaflet):
            lid = leaf * n_per_leaflet + s_idx
            k = int(assign[lid])
            ix, iy = s_idx % nx, s_idx // nx
            cx, cy = (ix + 0.5) * ax, (iy + 0.5) * ay
            if leaf == 1:  # stagger the lower leaflet
                cx += 0.5 * ax
            base = 0.5 * math.pi if along_y else 0.0
            phi = base + (math.pi if rng.random() < 0.5 else 0.0) \
                + rng.uniform(-wob, wob)
            tpl = _lipid_template(k, d)
            c, s = math.cos(phi), math.sin(phi)
            u, w, z = tpl[:, 0], tpl[:, 1], tpl[:, 2]
            px = cx + c * u - s * w
            py = cy + s * u + c * w
            pz = head_up + z if leaf == 0 else head_lo - z
            p = np.stack([px, py, pz], axis=1)
            p += rng.uniform(-jitter, jitter, size=p.shape)
            pos.append(p)
            mol_kind.append(k)
    # water: jittered lattice over the slab [head_up + 0.47, head_lo - 0.47 + Lz)
    if n_water:
        z0 = head_up + 0.47
        hz = (head_lo - 0.47 + Lz) - z0
        a = (area * hz / n_water) ** (1.0 / 3.0)
        nwx = max(1, int(round(Lx / a)))
        nwy = max(1, int(round(Ly / a)))
        nwz = int(math.ceil(n_water / (nwx * nwy)))
        while nwx * nwy * nwz < n_water:
            nwz += 1
        gx, gy, gz = Lx / nwx, Ly / nwy, hz / nwz
        n_full = (n_water // (nwx * nwy)) * nwx * nwy
        idx = np.arange(nwx * nwy * nwz)
        keep = np.concatenate([idx[:n_full],
                               n_full + np.sort(rng.permutation(len(idx) - n_full)
                                                [:n_water - n_full])])
        ix = keep % nwx
        iy = (keep // nwx) % nwy
        iz = keep // (nwx * nwy)
        wp = np.stack([(ix + 0.5) * gx, (iy + 0.5) * gy, z0 + (iz + 0.5) * gz], axis=1)
        wp += rng.uniform(-jitter, jitter, size=wp.shape)
        pos.append(wp)
        mol_kind += [KIND_W] * n_water
    pos = np.concatenate(pos, axis=0)
    box = np.array([Lx, Ly, Lz])
    pos = np.mod(pos, box)
    pos = _f32(pos)
    pos = np.where(pos >= box, 0.0, pos)  # float32 rounding can land on L
    temperature = 323.0
    masses = np.concatenate([np.asarray(kinds[k].masses) for k in mol_kind])
    sig = np.sqrt(KB * temperature / masses)
    vel = _f32(rng.standard_normal(pos.shape) * sig[:, None])
    sysm = System(name=name, kinds=kinds, mol_kind=np.asarray(mol_kind, dtype=np.int32),
                  pos=pos, vel=vel, box=box, eps=eps,
                  sigma=np.full((N_TYPES, N_TYPES), SIGMA), seed=int(seed),
                  temperature=temperature)
    # leaflet of each molecule (0 upper, 1 lower, -1 water): a structural
    # label of the build, used by the mixing observable
    leaflet = np.concatenate([np.zeros(n_per_leaflet, dtype=np.int32),
                              np.ones(n_per_leaflet, dtype=np.int32),
                              np.full(n_water, -1, dtype=np.int32)])
    sysm.meta = {"n_lipids": n_lip, "kind_counts": counts, "n_water": n_water,
                 "grid": (nx, ny), "depth_step": d, "leaflet": leaflet}
    return sysm


def make(config, seed=None, **kw):
    """Named workloads.  ``seed`` defaults to the workload's fixed seed."""
    if config == "c0":
        return bilayer("c0", 32, [0.5, 0.5], 640, 4.53, 9.0,
                       SEEDS["c0"] if seed is None else seed, **kw)
    if config in ("c1", "c2"):
        return bilayer(config, 2048, [0.4, 0.4, 0.2], 50000, 36.2, 10.0,
                       SEEDS[config] if seed is None else seed, **kw)
    if config == "c3":
        return bilayer("c3", 24576, [0.3, 0.3, 0.2, 0.2], 590000, 125.4, 11.0,
                       SEEDS["c3"] if seed is None else seed, **kw)
    if config == "topo":
        # topology-changing exchanges: C0's shape with lipid A and the
        # 12-slot sterol S12 in one swap family (S12 takes kind slot 1)
        kinds = standard_kinds()
        kinds[KIND_B] = sterol12_kind()
        s = bilayer("topo", 32, [0.5, 0.5], 640, 4.53, 9.0,
                    SEEDS["topo"] if seed is None else seed, kinds=kinds,
                    lipid_kinds=[KIND_A, KIND_B], **kw)
        eps = np.zeros((N_TYPES + 1, N_TYPES + 1))
        eps[:N_TYPES, :N_TYPES] = s.eps
        s.eps = eps
        s.sigma = np.full((N_TYPES + 1, N_TYPES + 1), SIGMA)
        return s
    if config == "mix":
        # the paper's mixing test in shape: 400 lipids, 1:1 of a neutral lipid
        # (A) and its anionic twin (D, head charge -1), water, far-from-mixed
        # stripes unless demix=False
        kw.setdefault("demix", True)
        return bilayer("mix", 200, [0.5, 0.5], 4000, 11.31, 9.0,
                       SEEDS["mix"] if seed is None else seed, lipid_kinds=[KIND_A, KIND_D], **kw)
    raise ValueError(f"unknown config {config!r}")


def serving_job(job_index, n_target, seed):
    """One serving job (built like c1) with about ``n_target`` beads."""
    rng = np.random.default_rng(seed)
    n = max(32, int(round(2048 * n_target / 95876)))
    nx, ny = _grid_dims(n)
    while nx / ny > 4.0:   # avoid degenerate strips: round n to a nicer number
        n += 1
        nx, ny = _grid_dims(n)
    xc = rng.uniform(0.0, 0.3)
    frac = [(1 - xc) / 2, (1 - xc) / 2, xc]
    n_w = int(round(50000 * n / 2048))
    L = math.sqrt(0.64 * n)
    s = bilayer(f"job{job_index}", n, frac, n_w, L, 10.0, seed)
    s.meta["job"] = job_index
    return s


def serving_jobs(n_jobs=48, n_min=1400, n_max=250000, base_seed=200508348100):
    rng = np.random.default_rng(base_seed)
    sizes = np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=n_jobs))
    return [serving_job(j, float(sizes[j]), base_seed + j) for j in range(n_jobs)]


# ---------------------------------------------------------------- toys
def custom(name, kinds, mol_kind, pos, box, eps, vel=None, seed=1, **kw):
    pos = _f32(np.asarray(pos, dtype=np.float64))
    box = _f32(np.asarray(box, dtype=np.float64))
    if vel is None:
        vel = np.zeros_like(pos)
    s = System(name=name, kinds=kinds, mol_kind=np.asarray(mol_kind, dtype=np.int32),
               pos=pos, vel=_f32(vel), box=box, eps=np.asarray(eps, dtype=np.float64),
               sigma=np.full(np.asarray(eps).shape, SIGMA), seed=seed)
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def topo_exchange_toy(nmol=216, box=4.8, seed=13):
    """A fluid of three-bead molecules of two kinds in one swap family whose
    bonded terms differ (a topology-changing exchange with moderate energy
    changes, so that exchanges are accepted): P is a chain h-s-t (bonds
    0.47 nm, 1250 kJ/mol/nm^2, an angle at s) with s and t of type C; Q has
    s and t of type U, bonds of 0.50 nm and 800 kJ/mol/nm^2 and no angle."""
    kp = Kind("P", [TYPE_N, TYPE_C, TYPE_C], [0.0, 0.0, 0.0],
              [(0, 1, 0.47, 1250.0), (1, 2, 0.47, 1250.0)], [(0, 1, 2, 180.0, 25.0)], 0)
    kq = Kind("Q", [TYPE_N, TYPE_U, TYPE_U], [0.0, 0.0, 0.0],
              [(0, 1, 0.50, 800.0), (1, 2, 0.50, 800.0)], [], 0)
    eps = np.full((N_TYPES + 1, N_TYPES + 1), 3.5)
    eps[TYPE_C, TYPE_C] = 4.5
    eps[TYPE_C, TYPE_U] = eps[TYPE_U, TYPE_C] = 4.0
    eps[TYPE_N, TYPE_C] = eps[TYPE_C, TYPE_N] = 3.1
    eps[TYPE_N, TYPE_U] = eps[TYPE_U, TYPE_N] = 4.0
    eps[TYPE_DUMMY, :] = 0.0
    eps[:, TYPE_DUMMY] = 0.0
    rng = np.random.default_rng(seed)
    n = int(math.ceil(nmol ** (1 / 3)))
    a = box / n
    pts = [(i, j, k) for i in range(n) for j in range(n) for k in range(n)][:nmol]
    pos = []
    for p in pts:
        hd = (np.array(p) + 0.2) * a
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        pos += [hd, hd + 0.47 * u, hd + 0.94 * u]
    pos = np.mod(np.array(pos), box)
    mk = np.array([i % 2 for i in range(nmol)], dtype=np.int32)
    masses = np.full(3 * nmol, MASS)
    sig = np.sqrt(KB * 323.0 / masses)
    vel = rng.standard_normal(pos.shape) * sig[:, None]
    s = custom("topo_toy", [kp, kq], mk, pos, [box] * 3, eps, vel=vel, seed=seed)
    s.sigma = np.full(eps.shape, SIGMA)
    return s


def twin_exchange_toy(m_per_region=8, n_q=8, seed=7):
    """2 m_per_region one-bead molecules of two kinds P and Q with identical
    parameters in one swap family, without interactions, split into two
    regions (meta["leaflet"]: the first m_per_region molecules 0, the rest
    1), all n_q molecules of kind Q in region 0 first.  Every exchange then
    has dU = 0, so the kinds perform the proposal chain alone."""
    kp = Kind("P", [TYPE_N], [0.0], [], [], 0)
    kq = Kind("Q", [TYPE_N], [0.0], [], [], 0)
    n = 2 * m_per_region
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, 6.0, size=(n, 3))
    mk = np.zeros(n, dtype=np.int32)
    mk[:n_q] = 1
    s = custom("twin", [kp, kq], mk, pos, [6.0, 6.0, 6.0], np.zeros((N_TYPES, N_TYPES)), seed=seed)
    s.meta["leaflet"] = np.repeat(np.array([0, 1], dtype=np.int32), m_per_region)
    return s


def two_lipid_toy(r, type_a=TYPE_C, type_b=TYPE_U, eps=None, box=6.0):
    """Two 2-bead molecules [h, s] of kinds X (s of type a) and Y (s of type b)
    in one swap family, plus a fixed bead E at distance r from X.s.  Y sits
    more than the cutoff away from X and E, so exchanging the kinds changes
    only the X.s-E pair."""
    kx = Kind("X", [TYPE_N, type_a], [0.0, 0.0], [(0, 1, 0.47, 1250.0)], [], 0)
    ky = Kind("Y", [TYPE_N, type_b], [0.0, 0.0], [(0, 1, 0.47, 1250.0)], [], 0)
    ke = Kind("E", [TYPE_W], [0.0], [], [], -1)
    if eps is None:
        eps = np.full((N_TYPES, N_TYPES), 2.0)
        eps[type_a, TYPE_W] = eps[TYPE_W, type_a] = 5.6
        eps[type_b, TYPE_W] = eps[TYPE_W, type_b] = 3.1
    c = box / 2
    pos = [[c - 1.0, 1.0, 1.0], [c - 1.0 + 0.47, 1.0, 1.0],            # X: h, s
           [c - 1.0, 1.0 + box / 2, 1.0 + box / 2],                     # Y.h
           [c - 1.0 + 0.47, 1.0 + box / 2, 1.0 + box / 2],              # Y.s
           [c - 1.0 + 0.47 + r, 1.0, 1.0]]                              # E
    return custom("toy2", [kx, ky, ke], [0, 1, 2], pos, [box, box, box], eps)
