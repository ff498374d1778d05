"""Pins of the oracle's NTC/VHS collision stage: per-cell conservation of
momentum and energy, and the equilibrium collision rate against the closed
form of the VHS <sigma_T c_r> averaged over the Maxwellian relative-speed
distribution."""
import math

import numpy as np
import pytest

from paper_2607_08195_amd import workloads as W
from oracle import Oracle, STAGE_SORT, STAGE_COLLIDE, STAGE_MOVE

KB = 1.380649e-23


def _cell_totals(p, nt):
    c = p["cell"]
    v = p["v"]
    mom = np.zeros((nt, 3))
    en = np.zeros(nt)
    np.add.at(mom, c, v)
    np.add.at(en, c, (v * v).sum(axis=1))
    absm = np.zeros(nt)
    np.add.at(absm, c, np.abs(v).sum(axis=1))
    return mom, en, absm


def test_collision_conserves_momentum_and_energy_fp64():
    wl = W.closed_box(n_hex=4, kind=W.BC_SPECULAR, ppc=40, vel_fp32=0)
    o = Oracle(wl)
    for _ in range(3):
        o.step_stages(STAGE_MOVE | STAGE_SORT)
        before = o.particles()
        o.lib.oracle_step_stages(o.h, STAGE_COLLIDE)  # same cells, collide only
        after = o.particles()
        assert np.array_equal(before["pid"], after["pid"])
        m0, e0, a0 = _cell_totals(before, o.nt)
        m1, e1, _ = _cell_totals(after, o.nt)
        assert o.pair_counts()[1].sum() > 100
        assert (np.abs(m1 - m0).max(axis=1) <= 1e-12 * a0).all()
        assert (np.abs(e1 - e0) <= 1e-12 * e0).all()


def sigma_c_eq(sp, T):
    """VHS <sigma_T c_r> at equilibrium temperature T:
    2 sqrt(pi) d^2 sqrt(2 k T_ref / m_r) (T/T_ref)^(1-omega)."""
    mr = sp.mass / 2
    return 2 * math.sqrt(math.pi) * sp.d_ref ** 2 * math.sqrt(2 * KB * sp.T_ref / mr) * \
        (T / sp.T_ref) ** (1 - sp.omega)


def test_sigma_c_eq_value():
    # argon at 273 K: 2.9395e-16 m^3/s
    assert abs(sigma_c_eq(W.Species(), 273.0) / 2.9395e-16 - 1) < 2e-4


@pytest.mark.parametrize("vel_fp32", [0, 1])
def test_equilibrium_collision_rate(vel_fp32):
    """Accepted collisions in an equilibrium closed box equal
    sum_cells 1/2 N(N-1) F_N <sigma c> dt / V to 3 sigma (Poisson), over
    >= 1e6 collisions."""
    wl = W.closed_box(n_hex=6, kind=W.BC_SPECULAR, ppc=20, vel_fp32=vel_fp32)
    o = Oracle(wl)
    sp, run = wl.species, wl.run
    vol = o.volumes()
    sc = sigma_c_eq(sp, run.T0)
    acc = 0
    exp = 0.0
    steps = 0
    while acc < 1_000_000:
        o.step(1)
        steps += 1
        N = np.diff(np.searchsorted(o.particles()["cell"], np.arange(o.nt + 1)))
        exp += (0.5 * N * (N - 1) * run.F_N * sc * run.dt / vol).sum()
        acc += int(o.pair_counts()[1].sum())
    z = (acc - exp) / math.sqrt(exp)
    assert abs(z) < 3.0, (acc, exp, z, steps)
