"""Pins of the oracle's Parrinello-Rahman pressure coupling (the paper's
barostat, Methods): semi-isotropic, box velocity kicked by the pressure
every coupling interval, box moved, coordinates scaled with it and peculiar
velocities scaled against it.

* An ideal gas without friction whose three axes carry the same kinetic
  energy keeps a cubic box, and since each bead's velocity component along
  an axis scales as 1 / L, its pressure is 2 K0 L0^2 / L^5.  The box then
  obeys the one-dimensional equation W L'' = 2 K0 L0^2 / L^3 - P0 L^2, solved
  here to 1e-11 by scipy's Runge-Kutta: the oracle's box follows it with an
  error that halves with the coupling interval (a first-order scheme).
* Small oscillations of that gas (compressibility 3 / (5 P0), a monatomic
  gas without heat exchange) have the period tau_p: the property the box
  mass W = 3 tau_p^2 L / (4 pi^2 beta) is chosen for.
* A membrane (C0) without thermostat conserves the extended energy
  K + U + P0 V + W/2 |dL/dt|^2 up to an error that halves with the step.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from paper_2005_08348_amd import systems as S

MASS_W = 72.0


def _gas(L0=4.0, m=20, seed=3):
    """3 m free beads; velocities in triples (a, b, c), (b, c, a), (c, a, b)
    so that sum m v_a^2 is the same on every axis."""
    rng = np.random.default_rng(seed)
    n = 3 * m
    k = S.Kind("W", [S.TYPE_W], [0.0], [], [], -1)
    base = rng.normal(0, 0.3, size=(m, 3))
    vel = np.concatenate([base, np.roll(base, 1, axis=1), np.roll(base, 2, axis=1)])
    pos = rng.uniform(0, L0, size=(n, 3))
    eps = np.zeros((S.N_TYPES, S.N_TYPES))
    s = S.custom("gas", [k], [0] * n, pos, [L0, L0, L0], eps, vel=vel, seed=5)
    s.gamma = 0.0
    return s


def _box_run(oracle_mod, s, p0_bar, beta_bar, tau, dt, T):
    s = s.copy()
    s.dt = dt
    o = oracle_mod.Oracle(s)
    o.set_barostat_pr(1, p_ref_bar=p0_bar, compressibility=beta_bar, tau_p=tau)
    Ls = [o.box()[0]]
    for _ in range(int(round(T / dt))):
        o.md_step(1)
        b = o.box()
        assert abs(b[0] - b[1]) < 1e-12 * b[0] and abs(b[0] - b[2]) < 1e-9 * b[0]
        Ls.append(b[0])
    return np.asarray(Ls)


def _gas_energy_per_axis(s):
    v = s.vel.astype(np.float64)
    ka = 0.5 * MASS_W * (v ** 2).sum(axis=0)
    assert np.allclose(ka, ka[0], rtol=1e-12)
    return ka[0]


def test_pr_ideal_gas_box_follows_its_equation(oracle_mod):
    s = _gas()
    ka, L0 = _gas_energy_per_axis(s), float(s.box[0])
    p_init = 2.0 * ka / L0 ** 3
    p0 = 0.5 * p_init                       # the gas expands by about 30%
    p0_bar = p0 * oracle_mod.BAR
    beta_bar, tau, T = 3.0 / (5.0 * p0_bar), 2.0, 4.0
    w = 3.0 * tau ** 2 * L0 / (4.0 * math.pi ** 2 * beta_bar * oracle_mod.BAR)

    def rhs(t, y):
        return [y[1], (2.0 * ka * L0 ** 2 / y[0] ** 3 - p0 * y[0] ** 2) / w]

    errs = []
    for dt in (0.01, 0.005):
        Ls = _box_run(oracle_mod, s, p0_bar, beta_bar, tau, dt, T)
        ts = np.arange(len(Ls)) * dt
        ref = solve_ivp(rhs, (0.0, T), [L0, 0.0], t_eval=ts, rtol=1e-11, atol=1e-12).y[0]
        assert ref.max() - L0 > 1.0                       # a large excursion
        errs.append(np.abs(Ls - ref).max())
    print("box error at dt 0.01 / 0.005: %.3e / %.3e nm" % tuple(errs))
    assert 1.8 < errs[0] / errs[1] < 2.2
    assert errs[1] < 0.01


def test_pr_small_oscillation_period_is_tau_p(oracle_mod):
    s = _gas()
    ka, L0 = _gas_energy_per_axis(s), float(s.box[0])
    p0 = 2.0 * ka / L0 ** 3 / 1.02          # 2% off equilibrium
    p0_bar = p0 * oracle_mod.BAR
    tau = 2.0
    Ls = _box_run(oracle_mod, s, p0_bar, 3.0 / (5.0 * p0_bar), tau, 0.005, 3 * tau)
    x = Ls - Ls.mean()
    dt = 0.005
    up = [i * dt - x[i] * dt / (x[i + 1] - x[i]) for i in range(len(x) - 1) if x[i] < 0 <= x[i + 1]]
    periods = np.diff(up)
    print("periods", periods)
    assert len(periods) >= 2
    assert np.all(np.abs(periods / tau - 1.0) < 0.005)


@pytest.fixture(scope="module")
def c0_nve(oracle_mod):
    c0 = S.make("c0")
    o = oracle_mod.Oracle(c0)
    o.minimize(60)
    s = c0.copy()
    s.pos = o.state()["pos"] % c0.box
    s.gamma = 0.0
    return s


def test_pr_conserves_extended_energy(oracle_mod, c0_nve):
    """C0 under 300 bar of tension, tau_p = 1 ps, coupled every step, 1 ps
    without thermostat: the box grows by several percent, and the extended
    energy's largest excursion halves with the step and stays below 6% of
    the energy the box exchanged."""
    out = []
    for dt in (0.01, 0.005):
        s = c0_nve.copy()
        s.dt = dt
        o = oracle_mod.Oracle(s)
        o.set_barostat_pr(1, p_ref_bar=-300.0, compressibility=3e-4, tau_p=1.0)

        def h():
            e = o.energy_forces(forces=False)
            _, hb = o.barostat_state()
            return e["potential"] + e["kinetic"] + hb, hb

        h0, hb0 = h()
        dh, dhb = [], []
        for _ in range(int(round(1.0 / dt))):
            o.md_step(1)
            a, b = h()
            dh.append(a - h0)
            dhb.append(b - hb0)
        box = o.box()
        assert box[2] > 1.03 * s.box[2] and box[0] > 1.03 * s.box[0]
        out.append((np.abs(dh).max(), np.abs(dhb).max()))
    print("max |dH| %.2f / %.2f kJ/mol, box energy exchanged %.1f" % (out[0][0], out[1][0], out[1][1]))
    assert 1.7 < out[0][0] / out[1][0] < 2.4
    assert out[1][0] < 0.06 * out[1][1]
