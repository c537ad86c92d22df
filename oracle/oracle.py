"""ctypes wrapper of the float64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg.  The product path never imports it.

The wrapper only marshals arrays; every step of the computation is in
oracle.c.  It takes the same seeded input description as the GPU library
(``paper_2005_08348_amd.systems.System``) but reads only its raw fields
(kinds, molecules, coordinates, parameters) and converts them itself.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "oracle.c")

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def build(force=False):
    """Compile oracle.c with gcc (plain -O2, no FMA contraction; OpenMP runs
    the slabs of the nonbonded loop and the sampled forces on several
    threads, with results independent of the thread count)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-fopenmp",
           "-shared", "-o", tmp, SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        L.o_create.restype = C.c_void_p
        L.o_create.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, _i32p,
                               _i32p, _i32p, _f64p, _f64p,
                               _i32p, _i32p, _f64p, _f64p,
                               C.c_int, _i32p,
                               C.c_int, _f64p, _f64p,
                               _f64p, C.c_double, C.c_double, C.c_double,
                               C.c_double, C.c_double, C.c_double, C.c_uint64,
                               _f64p, _f64p]
        L.o_destroy.argtypes = [C.c_void_p]
        L.o_n.argtypes = [C.c_void_p]
        L.o_n.restype = C.c_int
        L.o_get_state.argtypes = [C.c_void_p, _f64p, _f64p, _f64p, _i32p, _i64p]
        L.o_set_state.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.o_energy_forces.argtypes = [C.c_void_p, C.c_void_p, _f64p, C.c_int]
        L.o_energy_forces.restype = C.c_long
        L.o_forces_on.argtypes = [C.c_void_p, C.c_int, _i32p, _f64p, _f64p]
        L.o_pairset.argtypes = [C.c_void_p, C.c_double, C.c_void_p, C.c_long, C.c_int]
        L.o_pairset.restype = C.c_long
        L.o_md_step.argtypes = [C.c_void_p, C.c_int]
        L.o_refresh_forces.argtypes = [C.c_void_p]
        L.o_minimize.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double]
        L.o_delta_u_pair.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.o_delta_u_pair.restype = C.c_double
        L.o_delta_u_full.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.o_delta_u_full.restype = C.c_double
        L.o_swap_batch.argtypes = [C.c_void_p, C.c_int, C.c_int, _i32p, _i32p, _i32p,
                                   _f64p, _f64p, _i32p]
        L.o_swap_batch.restype = C.c_int
        L.o_mdas_cycle.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int,
                                   C.POINTER(C.c_double), C.POINTER(C.c_int),
                                   C.POINTER(C.c_double), _i32p]
        L.o_mdas_cycle.restype = C.c_int
        L.o_pairs_delta_u.argtypes = [C.c_void_p, C.c_int, _i32p]
        L.o_pairs_delta_u.restype = C.c_double
        L.o_pair_histogram.argtypes = [C.c_void_p, C.c_int, C.c_int, _i32p, C.c_int, C.c_double,
                                       _i64p]
        L.o_set_ensemble.argtypes = [C.c_void_p, C.c_int, C.c_double, _i32p]
        L.o_set_exchange_regions.argtypes = [C.c_void_p, C.c_int, _i32p]
        L.o_virial.argtypes = [C.c_void_p, _f64p, C.c_int]
        L.o_set_barostat.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double, C.c_double]
        L.o_set_barostat_pr.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double, C.c_double]
        L.o_barostat_state.argtypes = [C.c_void_p, _f64p]
        L.o_barostat_state.restype = C.c_double
        L.o_set_box_velocity.argtypes = [C.c_void_p, _f64p]
        L.o_get_box.argtypes = [C.c_void_p, _f64p]
        L.o_sc_lj.argtypes = [C.c_double] * 6 + [_f64p]
        L.o_sc_energy.argtypes = [C.c_void_p, C.c_int, _i32p, C.c_double]
        L.o_sc_energy.restype = C.c_double
        L.o_set_mdas_path.argtypes = [C.c_void_p, C.c_int, C.c_double]
        L.o_gamma_mt.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_int64, C.c_int, _f64p]
        L.o_vr_alpha.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double, C.c_int64, C.c_int,
                                 _f64p]
        L.o_philox.argtypes = [_u32p, _u32p, _u32p]
        L.o_gauss3.argtypes = [_u32p, _f64p]
        L.o_pair_term.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_double,
                                  C.c_double, _f64p]
        L.o_hybrid_energy_forces.argtypes = [C.c_void_p, C.c_int, _i32p, C.c_double, _f64p]
        L.o_hybrid_energy_forces.restype = C.c_double
        L.o_threads.argtypes = [C.c_int]
        L.o_threads.restype = C.c_int
        _lib = L
    return _lib


def threads(n=0):
    """threads of the oracle's parallel loops (n <= 0: query only)"""
    return lib().o_threads(int(n))


def philox(ctr, key):
    out = np.zeros(4, dtype=np.uint32)
    lib().o_philox(np.asarray(ctr, dtype=np.uint32), np.asarray(key, dtype=np.uint32), out)
    return out


def gauss3(words):
    g = np.zeros(3)
    lib().o_gauss3(np.asarray(words, dtype=np.uint32), g)
    return g


def sc_lj(c6, c12, r2, mu, delta, rc):
    """the soft-core LJ term of one pair: (energy, -dV/dr / r)"""
    out = np.zeros(2)
    lib().o_sc_lj(c6, c12, r2, mu, delta, rc, out)
    return out[0], out[1]


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(-1))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))


BAR = 16.6054   # bar per kJ mol^-1 nm^-3


class Oracle:
    """Float64 CPU reference of one system (see oracle.c for the definitions)."""

    def __init__(self, system, pos=None, vel=None):
        s = system
        kinds = s.kinds
        kn = _i32([k.n for k in kinds])
        ktype = _i32([t for k in kinds for t in k.types])
        kq = _f64([q for k in kinds for q in k.charges])
        km = _f64([m for k in kinds for m in k.masses])
        kfam = _i32([k.family for k in kinds])
        knb = _i32([len(k.bonds) for k in kinds])
        bij = _i32([[b[0], b[1]] for k in kinds for b in k.bonds] or [0])
        bb0 = _f64([b[2] for k in kinds for b in k.bonds] or [0])
        bk = _f64([b[3] for k in kinds for b in k.bonds] or [0])
        kna = _i32([len(k.angles) for k in kinds])
        aijk = _i32([[a[0], a[1], a[2]] for k in kinds for a in k.angles] or [0])
        ath = _f64([a[3] for k in kinds for a in k.angles] or [0])
        akk = _f64([a[4] for k in kinds for a in k.angles] or [0])
        self.system = s
        self.n = s.n_beads
        self.nm = s.n_mols
        x = _f64(s.pos if pos is None else pos)
        v = _f64(s.vel if vel is None else vel)
        self._keep = (kn, ktype, kq, km, kfam, knb, bij, bb0, bk, kna, aijk, ath, akk)
        self.h = lib().o_create(len(kinds), kn, ktype, kq, km, kfam, knb, bij, bb0, bk,
                                kna, aijk, ath, akk, s.n_mols, _i32(s.mol_kind),
                                s.eps.shape[0], _f64(s.eps), _f64(s.sigma), _f64(s.box),
                                s.rc, s.eps_r, s.eps_rf, s.dt, s.temperature, s.gamma,
                                int(s.seed) & 0xFFFFFFFFFFFFFFFF, x, v)
        lib().o_refresh_forces(self.h)

    def __del__(self):
        if getattr(self, "h", None):
            lib().o_destroy(self.h)
            self.h = None

    # -- state
    def state(self):
        x = np.zeros(3 * self.n); v = np.zeros(3 * self.n); f = np.zeros(3 * self.n)
        mk = np.zeros(self.nm, dtype=np.int32); ctr = np.zeros(4, dtype=np.int64)
        lib().o_get_state(self.h, x, v, f, mk, ctr)
        return dict(pos=x.reshape(-1, 3), vel=v.reshape(-1, 3), force=f.reshape(-1, 3),
                    mol_kind=mk, step=int(ctr[0]), batch=int(ctr[1]), cycle=int(ctr[2]),
                    fe=int(ctr[3]))

    def set_state(self, pos=None, vel=None, mol_kind=None, counters=None):
        xs = _f64(pos) if pos is not None else None
        vs = _f64(vel) if vel is not None else None
        ms = _i32(mol_kind) if mol_kind is not None else None
        cs = np.ascontiguousarray(np.asarray(counters, dtype=np.int64)) if counters is not None else None
        p = lambda a: a.ctypes.data if a is not None else None
        lib().o_set_state(self.h, p(xs), p(vs), p(ms), p(cs))
        lib().o_refresh_forces(self.h)

    # -- evaluations
    def energy_forces(self, cells=True, forces=True):
        f = np.zeros(3 * self.n) if forces else None
        e = np.zeros(5)
        np_ = lib().o_energy_forces(self.h, f.ctypes.data if forces else None, e, int(cells))
        out = dict(lj=e[0], rf=e[1], bond=e[2], angle=e[3], kinetic=e[4], n_pairs=int(np_))
        out["potential"] = e[0] + e[1] + e[2] + e[3]
        out["total"] = out["potential"] + e[4]
        if forces:
            out["force"] = f.reshape(-1, 3)
        return out

    def set_barostat(self, nst, p_ref_bar=1.0, compressibility=3e-4, tau_p=12.0):
        """semi-isotropic stochastic cell rescaling every nst MD steps (0: off);
        pressure in bar, compressibility in 1/bar, tau_p in ps"""
        lib().o_set_barostat(self.h, int(nst), p_ref_bar / BAR, compressibility * BAR, tau_p)

    def set_barostat_pr(self, nst, p_ref_bar=1.0, compressibility=3e-4, tau_p=12.0):
        """semi-isotropic Parrinello-Rahman coupling every nst MD steps (0:
        off); pressure in bar, compressibility in 1/bar, tau_p in ps; the box
        velocity starts at zero"""
        lib().o_set_barostat_pr(self.h, int(nst), p_ref_bar / BAR, compressibility * BAR, tau_p)

    def barostat_state(self):
        """(box velocity [3] nm/ps, P0 V + W/2 |dL/dt|^2 in kJ/mol)"""
        bv = np.zeros(3)
        h = lib().o_barostat_state(self.h, bv)
        return bv, h

    def set_box_velocity(self, bv):
        lib().o_set_box_velocity(self.h, _f64(bv))

    def set_mdas_path(self, path, delta=0.05):
        """MDAS lambda path: 0 linear (Eq. 2), 1 soft-core LJ (Eq. 4, delta nm^2)"""
        lib().o_set_mdas_path(self.h, int(path), float(delta))

    def sc_energy(self, pairs, lam):
        """U at lambda on the soft-core path for exchanging pairs [(X, Y), ...]"""
        pr = _i32(pairs)
        return lib().o_sc_energy(self.h, len(pr) // 2, pr, float(lam))

    def hybrid_energy_forces(self, pairs, lam):
        """U(lambda) and F(lambda) on the MDAS path in force (linear, or
        soft-core after set_mdas_path(1)) for exchanging pairs [(X, Y), ...]"""
        pr = _i32(pairs)
        f = np.zeros(3 * self.n)
        u = lib().o_hybrid_energy_forces(self.h, len(pr) // 2, pr, float(lam), f)
        return u, f.reshape(-1, 3)

    def box(self):
        b = np.zeros(3)
        lib().o_get_box(self.h, b)
        return b

    def virial(self, cells=True):
        """W_aa (kJ/mol), sum m v_a^2 (kJ/mol), the pressure tensor diagonal
        P_aa = (sum m v_a^2 + W_aa) / V in bar, and the sum of |term| of W_aa
        (an error scale for reduced-precision evaluations)"""
        w = np.zeros(9)
        lib().o_virial(self.h, w, int(cells))
        vol = float(np.prod(self.box()))
        return dict(w=w[:3].copy(), mv2=w[3:6].copy(), pressure=(w[3:6] + w[:3]) / vol * BAR,
                    w_abs=w[6:].copy())

    def forces_on(self, beads):
        sel = _i32(beads)
        f = np.zeros(3 * len(sel)); nc = np.zeros(len(sel))
        lib().o_forces_on(self.h, len(sel), sel, f, nc)
        return f.reshape(-1, 3), nc

    def pairset(self, rlist, cells=True):
        n = lib().o_pairset(self.h, rlist, None, 0, int(cells))
        out = np.zeros(2 * max(n, 1), dtype=np.int32)
        lib().o_pairset(self.h, rlist, out.ctypes.data, n, int(cells))
        return out[:2 * n].reshape(-1, 2)

    def pair_term(self, ti, tj, qi, qj, r2):
        out = np.zeros(3)
        lib().o_pair_term(self.h, ti, tj, qi, qj, r2, out)
        return out  # vlj, vrf, fscal

    # -- dynamics and moves
    def md_step(self, n):
        lib().o_md_step(self.h, int(n))

    def minimize(self, n_iter, alpha=1e-4, cap=0.01):
        lib().o_minimize(self.h, int(n_iter), alpha, cap)

    def delta_u_pair(self, X, Y):
        return lib().o_delta_u_pair(self.h, int(X), int(Y))

    def delta_u_full(self, X, Y):
        return lib().o_delta_u_full(self.h, int(X), int(Y))

    def swap_batch(self, n_trials, draw_cap=None):
        cap = 64 * n_trials if draw_cap is None else draw_cap
        d = np.zeros(n_trials, dtype=np.int32); X = np.zeros_like(d); Y = np.zeros_like(d)
        du = np.zeros(n_trials); u = np.zeros(n_trials); acc = np.zeros(n_trials, dtype=np.int32)
        k = lib().o_swap_batch(self.h, n_trials, cap, d, X, Y, du, u, acc)
        return dict(draw=d[:k], X=X[:k], Y=Y[:k], du=du[:k], u=u[:k], accept=acc[:k].astype(bool))

    def mdas_cycle(self, n_pairs, K, M):
        w = C.c_double(); acc = C.c_int(); u = C.c_double()
        pairs = np.zeros(2 * max(n_pairs, 1), dtype=np.int32)
        k = lib().o_mdas_cycle(self.h, n_pairs, K, M, C.byref(w), C.byref(acc), C.byref(u), pairs)
        return dict(work=w.value, accept=bool(acc.value), u=u.value,
                    pairs=pairs[:2 * k].reshape(-1, 2))

    def set_ensemble(self, ensemble, tau_t=1.0, kind_group=None):
        """0: Langevin BAOAB; 1: velocity Verlet + stochastic velocity
        rescaling of the coupling groups kind_group[n_kinds] (0/1)"""
        nk = len(self.system.kinds)
        kg = np.zeros(nk, dtype=np.int32) if kind_group is None else _i32(kind_group)
        if len(kg) != nk:
            raise ValueError("kind_group needs one entry per molecule kind")
        lib().o_set_ensemble(self.h, int(ensemble), float(tau_t), kg)

    def set_exchange_regions(self, mode, region=None):
        """exchange partners: 0 anywhere in the family, 1 within the region
        (leaflet) of X, 2 in the other region; region[n_mols] 0/1"""
        rg = np.zeros(self.nm, dtype=np.int32) if region is None else _i32(region)
        if len(rg) != self.nm:
            raise ValueError("region needs one entry per molecule")
        lib().o_set_exchange_regions(self.h, int(mode), rg)

    def gamma_mt(self, group, a, ctr0, n):
        """the thermostat's Gamma(a, 1) draws at step counters ctr0 .. ctr0 + n - 1"""
        out = np.zeros(n)
        lib().o_gamma_mt(self.h, int(group), float(a), int(ctr0), int(n), out)
        return out

    def vr_alpha(self, group, K, nf, ctr0, n):
        """the thermostat's velocity factors for kinetic energy K of a group
        with nf degrees of freedom, at step counters ctr0 .. ctr0 + n - 1"""
        out = np.zeros(n)
        lib().o_vr_alpha(self.h, int(group), float(K), float(nf), int(ctr0), int(n), out)
        return out

    def pair_histogram(self, kind, po4, leaflet, n_bins, bin_width):
        """lateral PO4-PO4 pair counts per bin (unordered pairs, same leaflet)"""
        out = np.zeros(int(n_bins), dtype=np.int64)
        lib().o_pair_histogram(self.h, int(kind), int(po4), _i32(leaflet), int(n_bins),
                               float(bin_width), out)
        return out

    def pairs_delta_u(self, pairs):
        p = _i32(pairs)
        return lib().o_pairs_delta_u(self.h, len(p) // 2, p)
