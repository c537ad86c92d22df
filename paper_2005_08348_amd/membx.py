"""Python binding of the membx C-ABI (include/membx.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libmembx.so.  PyTorch supplies the device arena (a uint8 tensor)
and the caller's stream.  There is no CPU fallback: constructing a
``System`` without the built library or without a GPU raises.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmembx.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "membx.h")

OK, E_INVAL, E_NOMEM, E_DEVICE, E_LIST_OVERFLOW, E_NONFINITE, E_STATE, E_SKIN = range(8)
FP64, MIXED = 0, 1
_STATUS = {0: "OK", 1: "E_INVAL", 2: "E_NOMEM", 3: "E_DEVICE", 4: "E_LIST_OVERFLOW",
           5: "E_NONFINITE", 6: "E_STATE", 7: "E_SKIN"}


class MembxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"membx {_STATUS.get(code, code)}: {msg}")
        self.code = code


class Kind(C.Structure):
    _fields_ = [("n_beads", C.c_int32), ("bead_type", C.POINTER(C.c_int32)),
                ("bead_charge", C.POINTER(C.c_double)), ("bead_mass", C.POINTER(C.c_double)),
                ("n_bonds", C.c_int32), ("bond_ij", C.POINTER(C.c_int32)),
                ("bond_b0", C.POINTER(C.c_double)), ("bond_k", C.POINTER(C.c_double)),
                ("n_angles", C.c_int32), ("angle_ijk", C.POINTER(C.c_int32)),
                ("angle_theta0", C.POINTER(C.c_double)), ("angle_k", C.POINTER(C.c_double)),
                ("swap_family", C.c_int32)]


class Desc(C.Structure):
    _fields_ = [("n_kinds", C.c_int32), ("kinds", C.POINTER(Kind)),
                ("n_mols", C.c_int32), ("mol_kind", C.POINTER(C.c_int32)),
                ("pos", C.POINTER(C.c_double)), ("vel", C.POINTER(C.c_double)),
                ("box", C.c_double * 3), ("n_types", C.c_int32),
                ("lj_epsilon", C.POINTER(C.c_double)), ("lj_sigma", C.POINTER(C.c_double)),
                ("r_cut", C.c_double), ("eps_r", C.c_double), ("eps_rf", C.c_double),
                ("dt", C.c_double), ("temperature", C.c_double), ("gamma", C.c_double),
                ("seed", C.c_uint64), ("precision", C.c_int32),
                ("skin", C.c_double), ("skin_max", C.c_double),
                ("rebuild_interval", C.c_int32), ("lanes_per_bead", C.c_int32),
                ("list_capacity", C.c_int32), ("max_trials", C.c_int32),
                ("max_pairs", C.c_int32), ("skin_inner", C.c_double),
                ("prune_interval", C.c_int32)]


class Energy(C.Structure):
    _fields_ = [("lj", C.c_double), ("rf", C.c_double), ("bond", C.c_double),
                ("angle", C.c_double), ("kinetic", C.c_double), ("potential", C.c_double),
                ("total", C.c_double), ("n_pairs_in_cutoff", C.c_int64),
                ("fe_count", C.c_int64), ("step", C.c_int64), ("batch", C.c_int64),
                ("cycle", C.c_int64), ("n_rebuilds", C.c_int64),
                ("n_skin_violations", C.c_int64),
                ("max_displacement", C.c_double), ("n_list_entries", C.c_int64),
                ("virial", C.c_double * 3), ("mv2", C.c_double * 3), ("pressure", C.c_double * 3),
                ("list_retests", C.c_int64)]


class Request(C.Structure):
    _fields_ = [("minimize_iters", C.c_int32),
                ("md_cycles", C.c_int32), ("md_steps", C.c_int32), ("mdas_cycles", C.c_int32),
                ("mdas_pairs", C.c_int32), ("mdas_k", C.c_int32), ("mdas_m", C.c_int32),
                ("count_pairs", C.c_int32)]


class JobResult(C.Structure):
    _fields_ = [("job_id", C.c_int64), ("status", C.c_int32), ("n_cycles", C.c_int32),
                ("mdas_accepted", C.c_int32), ("n_beads", C.c_int32),
                ("submit_s", C.c_double), ("admit_s", C.c_double), ("finish_s", C.c_double),
                ("cycle_ms_p50", C.c_double), ("cycle_ms_p99", C.c_double),
                ("cycle_ms_max", C.c_double), ("md_steps", C.c_int64), ("fe_count", C.c_int64),
                ("pairs_in_cutoff", C.c_int64), ("potential", C.c_double),
                ("pair_interactions", C.c_int64)]


class Trial(C.Structure):
    _fields_ = [("draw", C.c_int32), ("mol_x", C.c_int32), ("mol_y", C.c_int32),
                ("accepted", C.c_int32), ("delta_u", C.c_double), ("u", C.c_double)]


_lib = None


def header_symbols():
    """Names of the functions include/membx.h declares."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int32_t|const char\*)\s+(membx_\w+)\(", txt, re.M)))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run "
                               "`python -m paper_2005_08348_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u64, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
        sig = {
            "membx_sys_bytes": ([C.POINTER(Desc), C.POINTER(u64)], i32),
            "membx_sys_create": ([C.POINTER(Desc), vp, u64, vp, C.POINTER(vp)], i32),
            "membx_sys_destroy": ([vp], i32),
            "membx_md_step": ([vp, i64], i32),
            "membx_mc_swap_trials": ([vp, i32, C.POINTER(i32), C.POINTER(i32), vp], i32),
            "membx_mdas_cycle": ([vp, i32, i32, i32, C.POINTER(dp), C.POINTER(i32), vp], i32),
            "membx_energies": ([vp, C.POINTER(Energy)], i32),
            "membx_energies_noalloc": ([vp, C.POINTER(Energy)], i32),
            "membx_get_state": ([vp, vp, vp, vp, vp], i32),
            "membx_set_state": ([vp, vp, vp, vp, vp], i32),
            "membx_forces": ([vp, vp], i32),
            "membx_pairset_export": ([vp, vp, i64, C.POINTER(i64)], i32),
            "membx_pair_histogram": ([vp, i32, i32, vp, i32, dp, vp], i32),
            "membx_minimize": ([vp, i32, dp, dp], i32),
            "membx_set_tuning": ([vp, dp, i32, i32, dp, i32], i32),
            "membx_autotune": ([vp, i32, C.POINTER(dp), C.POINTER(i32), C.POINTER(i32),
                                C.POINTER(dp), C.POINTER(i32)], i32),
            "membx_set_graphs": ([vp, i32], i32),
            "membx_set_ensemble": ([vp, i32, dp, vp], i32),
            "membx_set_exchange_regions": ([vp, i32, vp], i32),
            "membx_set_barostat": ([vp, i32, dp, dp, dp], i32),
            "membx_set_barostat_pr": ([vp, i32, dp, dp, dp], i32),
            "membx_barostat_state": ([vp, vp, vp, C.POINTER(dp)], i32),
            "membx_get_box": ([vp, vp], i32),
            "membx_set_mdas_path": ([vp, i32, dp], i32),
            "membx_kernel_timing": ([vp, i32], i32),
            "membx_kernel_time": ([vp, C.POINTER(i64), C.POINTER(dp)], i32),
            "membx_kernel_bench": ([vp, i32, C.POINTER(dp)], i32),
            "membx_server_create": ([vp, u64, C.POINTER(vp)], i32),
            "membx_server_submit": ([vp, vp, C.POINTER(Request), C.POINTER(i64)], i32),
            "membx_server_poll": ([vp, C.POINTER(JobResult), i32, C.POINTER(i32), C.POINTER(i32),
                                   C.POINTER(i32)], i32),
            "membx_server_cycle_times": ([vp, C.POINTER(C.c_float), i64, C.POINTER(i64)], i32),
            "membx_server_cycle_pairs": ([vp, C.POINTER(C.c_double), i64, C.POINTER(i64)], i32),
            "membx_server_destroy": ([vp], i32),
            "membx_server_last_error": ([vp], C.c_char_p),
            "membx_last_error": ([vp], C.c_char_p),
            "membx_status": ([vp], i32),
            "membx_calib_copy": ([vp, vp, vp, u64], i32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class _DescBuilder:
    """Keeps the numpy buffers a membx_desc points to alive."""

    def __init__(self, system, precision, skin, skin_max, rebuild_interval, lanes_per_bead,
                 list_capacity, max_trials, max_pairs, skin_inner=0.0, prune_interval=0):
        s = system
        self.keep = []
        kinds = (Kind * len(s.kinds))()
        for q, k in enumerate(s.kinds):
            t = np.ascontiguousarray(k.types, dtype=np.int32)
            ch = np.ascontiguousarray(k.charges, dtype=np.float64)
            ms = np.ascontiguousarray(k.masses, dtype=np.float64)
            bij = np.ascontiguousarray([[b[0], b[1]] for b in k.bonds] or [[0, 0]], dtype=np.int32)
            b0 = np.ascontiguousarray([b[2] for b in k.bonds] or [0.0])
            bk = np.ascontiguousarray([b[3] for b in k.bonds] or [0.0])
            aijk = np.ascontiguousarray([[a[0], a[1], a[2]] for a in k.angles] or [[0, 0, 0]],
                                        dtype=np.int32)
            ath = np.ascontiguousarray([a[3] for a in k.angles] or [0.0])
            ak = np.ascontiguousarray([a[4] for a in k.angles] or [0.0])
            self.keep += [t, ch, ms, bij, b0, bk, aijk, ath, ak]
            kinds[q] = Kind(k.n, _p(t, C.c_int32), _p(ch, C.c_double), _p(ms, C.c_double),
                            len(k.bonds), _p(bij, C.c_int32), _p(b0, C.c_double), _p(bk, C.c_double),
                            len(k.angles), _p(aijk, C.c_int32), _p(ath, C.c_double),
                            _p(ak, C.c_double), k.family)
        self.kinds = kinds
        mk = np.ascontiguousarray(s.mol_kind, dtype=np.int32)
        pos = np.ascontiguousarray(s.pos, dtype=np.float64).reshape(-1)
        vel = np.ascontiguousarray(s.vel, dtype=np.float64).reshape(-1)
        eps = np.ascontiguousarray(s.eps, dtype=np.float64).reshape(-1)
        sig = np.ascontiguousarray(s.sigma, dtype=np.float64).reshape(-1)
        self.keep += [mk, pos, vel, eps, sig]
        d = Desc()
        d.n_kinds = len(s.kinds)
        d.kinds = C.cast(kinds, C.POINTER(Kind))
        d.n_mols = len(mk)
        d.mol_kind = _p(mk, C.c_int32)
        d.pos = _p(pos, C.c_double)
        d.vel = _p(vel, C.c_double)
        for a in range(3):
            d.box[a] = float(s.box[a])
        d.n_types = int(s.eps.shape[0])
        d.lj_epsilon = _p(eps, C.c_double)
        d.lj_sigma = _p(sig, C.c_double)
        d.r_cut = s.rc
        d.eps_r = s.eps_r
        d.eps_rf = s.eps_rf if math.isfinite(s.eps_rf) else 0.0
        d.dt = s.dt
        d.temperature = s.temperature
        d.gamma = s.gamma
        d.seed = int(s.seed) & 0xFFFFFFFFFFFFFFFF
        d.precision = precision
        d.skin = skin
        d.skin_max = skin_max
        d.rebuild_interval = rebuild_interval
        d.lanes_per_bead = lanes_per_bead
        d.list_capacity = list_capacity
        d.max_trials = max_trials
        d.max_pairs = max_pairs
        d.skin_inner = skin_inner
        d.prune_interval = prune_interval
        self.desc = d


def _check(rc, h=None):
    if rc != OK:
        msg = lib().membx_last_error(h).decode() if h else ""
        raise MembxError(rc, msg)


def arena_bytes(system, precision="mixed", **tuning):
    prec = MIXED if precision == "mixed" else FP64
    b = _DescBuilder(system, prec, *_tuning(tuning))
    n = C.c_uint64()
    _check(lib().membx_sys_bytes(C.byref(b.desc), C.byref(n)))
    return int(n.value)


def _tuning(t):
    return (t.get("skin", 0.0), t.get("skin_max", 0.0), t.get("rebuild_interval", 0),
            t.get("lanes_per_bead", 0), t.get("list_capacity", 0), t.get("max_trials", 0),
            t.get("max_pairs", 0), t.get("skin_inner", 0.0), t.get("prune_interval", 0))


class System:
    """One membrane system resident on the GPU."""

    def __init__(self, system, precision="mixed", device="cuda:0", stream=None, **tuning):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("membx needs a GPU (no CPU fallback)")
        self.torch = torch
        self.device = torch.device(device)
        self.precision = precision
        prec = MIXED if precision == "mixed" else FP64
        self._b = _DescBuilder(system, prec, *_tuning(tuning))
        n = C.c_uint64()
        _check(lib().membx_sys_bytes(C.byref(self._b.desc), C.byref(n)))
        self.arena_bytes = int(n.value)
        with torch.cuda.device(self.device):
            self.arena = torch.empty(self.arena_bytes + 256, dtype=torch.uint8, device=self.device)
            st = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.stream = st
            h = C.c_void_p()
            _check(lib().membx_sys_create(C.byref(self._b.desc), C.c_void_p(self.arena.data_ptr()),
                                          self.arena_bytes + 256, C.c_void_p(st.cuda_stream),
                                          C.byref(h)))
        self.h = h
        self.n = system.n_beads
        self.nm = system.n_mols
        self.system = system

    def close(self):
        if getattr(self, "h", None):
            lib().membx_sys_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ dynamics
    def md_step(self, n=1):
        _check(lib().membx_md_step(self.h, int(n)), self.h)

    def swap_trials(self, n, results=True):
        if not results:
            _check(lib().membx_mc_swap_trials(self.h, int(n), None, None, None), self.h)
            return None
        na, nacc = C.c_int32(), C.c_int32()
        out = (Trial * int(n))()
        _check(lib().membx_mc_swap_trials(self.h, int(n), C.byref(na), C.byref(nacc), out), self.h)
        k = na.value
        return dict(draw=np.array([out[t].draw for t in range(k)], dtype=np.int32),
                    X=np.array([out[t].mol_x for t in range(k)], dtype=np.int32),
                    Y=np.array([out[t].mol_y for t in range(k)], dtype=np.int32),
                    accept=np.array([bool(out[t].accepted) for t in range(k)]),
                    du=np.array([out[t].delta_u for t in range(k)]),
                    u=np.array([out[t].u for t in range(k)]),
                    n_accepted=int(nacc.value))

    def mdas_cycle(self, n_pairs, k_increments, m_steps, results=True):
        if not results:
            _check(lib().membx_mdas_cycle(self.h, n_pairs, k_increments, m_steps, None, None,
                                          None), self.h)
            return None
        w, acc = C.c_double(), C.c_int32()
        pairs = np.zeros(2 * n_pairs, dtype=np.int32)
        _check(lib().membx_mdas_cycle(self.h, n_pairs, k_increments, m_steps, C.byref(w),
                                      C.byref(acc), pairs.ctypes.data_as(C.c_void_p)), self.h)
        pairs = pairs.reshape(-1, 2)
        return dict(work=w.value, accept=bool(acc.value), pairs=pairs[pairs[:, 0] >= 0])

    def minimize(self, n_iter, alpha=1e-4, max_step=0.01):
        _check(lib().membx_minimize(self.h, int(n_iter), float(alpha), float(max_step)), self.h)

    # -------------------------------------------------------------- queries
    def energies(self, check=True):
        e = Energy()
        rc = lib().membx_energies(self.h, C.byref(e))
        if check:
            _check(rc, self.h)
        out = {k: getattr(e, k) for k, _ in Energy._fields_}
        for k in ("virial", "mv2", "pressure"):
            out[k] = np.array(out[k][:], dtype=np.float64)
        out["status"] = rc
        return out

    def state(self):
        x = np.zeros(3 * self.n); v = np.zeros(3 * self.n)
        mk = np.zeros(self.nm, dtype=np.int32); ctr = np.zeros(3, dtype=np.int64)
        _check(lib().membx_get_state(self.h, x.ctypes.data_as(C.c_void_p),
                                     v.ctypes.data_as(C.c_void_p), mk.ctypes.data_as(C.c_void_p),
                                     ctr.ctypes.data_as(C.c_void_p)), self.h)
        return dict(pos=x.reshape(-1, 3), vel=v.reshape(-1, 3), mol_kind=mk,
                    step=int(ctr[0]), batch=int(ctr[1]), cycle=int(ctr[2]))

    def set_state(self, pos=None, vel=None, mol_kind=None, counters=None):
        keep = []

        def ptr(a, dt):
            if a is None:
                return None
            a = np.ascontiguousarray(a, dtype=dt).reshape(-1)
            keep.append(a)
            return a.ctypes.data_as(C.c_void_p)
        _check(lib().membx_set_state(self.h, ptr(pos, np.float64), ptr(vel, np.float64),
                                     ptr(mol_kind, np.int32), ptr(counters, np.int64)), self.h)

    def forces(self):
        f = np.zeros(3 * self.n)
        _check(lib().membx_forces(self.h, f.ctypes.data_as(C.c_void_p)), self.h)
        return f.reshape(-1, 3)

    def pairset(self):
        n = C.c_int64()
        _check(lib().membx_pairset_export(self.h, None, 0, C.byref(n)), self.h)
        out = np.zeros(2 * max(n.value, 1), dtype=np.int32)
        _check(lib().membx_pairset_export(self.h, out.ctypes.data_as(C.c_void_p), n.value,
                                          C.byref(n)), self.h)
        return out[:2 * n.value].reshape(-1, 2)

    def pair_histogram(self, kind, po4, leaflet, n_bins, bin_width):
        """lateral pair counts of bead po4 of the molecules of one kind within
        each leaflet (leaflet[n_mols]: 0/1, -1 skips), bins of bin_width"""
        lf = np.ascontiguousarray(leaflet, dtype=np.int32)
        if lf.shape != (self.nm,):
            raise ValueError("leaflet must have one entry per molecule")
        out = np.zeros(int(n_bins), dtype=np.int64)
        _check(lib().membx_pair_histogram(self.h, int(kind), int(po4), lf.ctypes.data_as(C.c_void_p),
                                          int(n_bins), float(bin_width),
                                          out.ctypes.data_as(C.c_void_p)), self.h)
        return out

    def status(self):
        return lib().membx_status(self.h)

    # --------------------------------------------------------------- tuning
    def set_barostat(self, nst, p_ref_bar=1.0, compressibility=3e-4, tau_p=12.0):
        """semi-isotropic pressure coupling every nst MD steps (0: off)"""
        _check(lib().membx_set_barostat(self.h, int(nst), float(p_ref_bar), float(compressibility),
                                        float(tau_p)), self.h)

    def set_barostat_pr(self, nst, p_ref_bar=1.0, compressibility=3e-4, tau_p=12.0):
        """semi-isotropic Parrinello-Rahman coupling every nst MD steps (0: off)"""
        _check(lib().membx_set_barostat_pr(self.h, int(nst), float(p_ref_bar), float(compressibility),
                                           float(tau_p)), self.h)

    def barostat_state(self, set_box_vel=None):
        """(box velocity [3] nm/ps, P0 V + W/2 |dL/dt|^2 kJ/mol); set_box_vel
        replaces the box velocity first"""
        bv, hb = np.zeros(3), C.c_double()
        sv = None if set_box_vel is None else np.ascontiguousarray(set_box_vel, dtype=np.float64)
        _check(lib().membx_barostat_state(self.h, None if sv is None else sv.ctypes.data_as(C.c_void_p),
                                          bv.ctypes.data_as(C.c_void_p), C.byref(hb)), self.h)
        return bv, hb.value

    def set_mdas_path(self, path, delta=0.05):
        """MDAS lambda path: 0 linear (Eq. 2), 1 soft-core LJ (Eq. 4, delta nm^2)"""
        _check(lib().membx_set_mdas_path(self.h, int(path), float(delta)), self.h)

    def box(self):
        b = np.zeros(3)
        _check(lib().membx_get_box(self.h, b.ctypes.data_as(C.c_void_p)), self.h)
        return b

    def set_exchange_regions(self, mode, region=None):
        """exchange partners: 0 anywhere in X's family (other kind), 1 other
        kind within X's region, 2 any family member in the other region;
        region[n_mols] 0/1 for exchangeable molecules (others ignored)"""
        rg = None
        if region is not None:
            rg = np.ascontiguousarray(region, dtype=np.int32)
            if rg.shape != (self.nm,):
                raise ValueError("region needs one entry per molecule")
        _check(lib().membx_set_exchange_regions(self.h, int(mode),
                                                None if rg is None else rg.ctypes.data_as(C.c_void_p)),
               self.h)

    def set_ensemble(self, ensemble, tau_t=1.0, kind_group=None):
        """0: Langevin BAOAB; 1: velocity Verlet + stochastic velocity
        rescaling with coupling time tau_t (ps) of the groups kind_group[n_kinds]
        (0/1; None: one group)"""
        kg = None
        if kind_group is not None:
            kg = np.ascontiguousarray(kind_group, dtype=np.int32)
            if kg.shape != (len(self.system.kinds),):
                raise ValueError("kind_group needs one entry per molecule kind")
        _check(lib().membx_set_ensemble(self.h, int(ensemble), float(tau_t),
                                        None if kg is None else kg.ctypes.data_as(C.c_void_p)),
               self.h)

    def set_tuning(self, skin, rebuild_interval, lanes_per_bead, skin_inner=0.0, prune_interval=0):
        _check(lib().membx_set_tuning(self.h, float(skin), int(rebuild_interval),
                                      int(lanes_per_bead), float(skin_inner), int(prune_interval)),
               self.h)

    def autotune(self, n_steps=200):
        sk, R, l, si, pr = C.c_double(), C.c_int32(), C.c_int32(), C.c_double(), C.c_int32()
        _check(lib().membx_autotune(self.h, int(n_steps), C.byref(sk), C.byref(R), C.byref(l),
                                    C.byref(si), C.byref(pr)), self.h)
        return dict(skin=sk.value, rebuild_interval=R.value, lanes_per_bead=l.value,
                    skin_inner=si.value, prune_interval=pr.value)

    def set_graphs(self, enable):
        _check(lib().membx_set_graphs(self.h, int(bool(enable))), self.h)

    def kernel_timing(self, enable):
        _check(lib().membx_kernel_timing(self.h, int(bool(enable))), self.h)

    def kernel_time(self):
        n, ms = C.c_int64(), C.c_double()
        _check(lib().membx_kernel_time(self.h, C.byref(n), C.byref(ms)), self.h)
        return int(n.value), float(ms.value)

    def kernel_bench(self, n_launch=200):
        """mean duration (ms) of the nonbonded kernel over n_launch graph-replayed launches"""
        ms = C.c_double()
        _check(lib().membx_kernel_bench(self.h, int(n_launch), C.byref(ms)), self.h)
        return ms.value

    def calib_copy(self, dst, src, nbytes):
        _check(lib().membx_calib_copy(self.h, C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()),
                                      int(nbytes)), self.h)


class Server:
    """Many membrane systems resident in one device arena (C-ABI serving loop).

    ``submit`` queues a job (a system plus a request); ``poll`` advances every
    job without blocking and returns the results of jobs that finished."""

    def __init__(self, budget_bytes, device="cuda:0"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("membx needs a GPU (no CPU fallback)")
        self.device = torch.device(device)
        self.arena = torch.empty(int(budget_bytes) + 256, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        h = C.c_void_p()
        rc = lib().membx_server_create(C.c_void_p(self.arena.data_ptr()), int(budget_bytes) + 256,
                                       C.byref(h))
        if rc:
            raise MembxError(rc, "server creation failed")
        self.h = h
        self._keep = {}

    def _err(self, rc):
        if rc:
            raise MembxError(rc, lib().membx_server_last_error(self.h).decode())

    def submit(self, system, minimize_iters=100, md_cycles=4, md_steps=50, mdas_cycles=20,
               mdas_pairs=8, mdas_k=50, mdas_m=1, count_pairs=False, precision="mixed", **tuning):
        b = _DescBuilder(system, MIXED if precision == "mixed" else FP64, *_tuning(tuning))
        rq = Request(minimize_iters, md_cycles, md_steps, mdas_cycles, mdas_pairs, mdas_k, mdas_m,
                     int(bool(count_pairs)))
        jid = C.c_int64()
        self._err(lib().membx_server_submit(self.h, C.byref(b.desc), C.byref(rq), C.byref(jid)))
        return int(jid.value)

    def poll(self, cap=64):
        out = (JobResult * cap)()
        n, nr, nw = C.c_int32(), C.c_int32(), C.c_int32()
        self._err(lib().membx_server_poll(self.h, out, cap, C.byref(n), C.byref(nr), C.byref(nw)))
        res = [{k: getattr(out[q], k) for k, _ in JobResult._fields_} for q in range(n.value)]
        return res, nr.value, nw.value

    def cycle_times(self):
        n = C.c_int64()
        self._err(lib().membx_server_cycle_times(self.h, None, 0, C.byref(n)))
        buf = (C.c_float * max(1, n.value))()
        self._err(lib().membx_server_cycle_times(self.h, buf, n.value, C.byref(n)))
        return np.frombuffer(buf, dtype=np.float32, count=n.value).copy()

    def cycle_pairs(self):
        n = C.c_int64()
        self._err(lib().membx_server_cycle_pairs(self.h, None, 0, C.byref(n)))
        buf = (C.c_double * max(1, n.value))()
        self._err(lib().membx_server_cycle_pairs(self.h, buf, n.value, C.byref(n)))
        return np.frombuffer(buf, dtype=np.float64, count=n.value).copy()

    def close(self):
        if getattr(self, "h", None):
            lib().membx_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
