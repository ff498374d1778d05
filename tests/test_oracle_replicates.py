"""Calibration of the statistical parity criterion on the oracle alone: two
sets of eight oracle replicates of the CPU-finishable cavity (6^3 x 6 tets,
Kn = 1, 20 particles per cell, FP64, 500 steps with the last 300 sampled),
seeded from disjoint sets, pass it (the criterion does not reject two
samples of one distribution), and replicates whose walls are 1 % warmer
fail it in the temperature field (it detects a small physical
difference)."""
import numpy as np
import pytest

from paper_2607_08195_amd import workloads as W
from oracle import Oracle
import replicates as RP


def _cfg0(seed, Tw=None):
    wl = W.cavity_small()
    wl.run.seed = seed
    if Tw is not None:
        wl.boundaries = [W.Boundary(b.kind, Tw, b.u) for b in wl.boundaries]
    return wl


def _fields(runs, wl):
    V = Oracle(wl, fill=False).volumes()
    return np.array([RP.cell_fields(s, wl.species.mass, wl.run.F_N, V, n) for s, n in runs])


@pytest.fixture(scope="module")
def reps():
    wls = [_cfg0(100 + r) for r in range(8)] + [_cfg0(200 + r) for r in range(8)] + \
          [_cfg0(300 + r, Tw=276.0) for r in range(8)]
    runs = RP.oracle_replicates(wls, 500)
    assert all(n == 300 for _, n in runs)
    wl = _cfg0(0)
    return _fields(runs[:8], wl), _fields(runs[8:16], wl), _fields(runs[16:], wl)


def test_disjoint_seed_replicates_pass(reps):
    a, b, _ = reps
    zs = RP.field_z(a, b)
    assert RP.check_fields(zs) == {}
    zn, _ = RP.replicate_z(a, b)
    s = RP.z_summary(zn)
    assert s["n"] > 0.99 * a.shape[1] * 14
    assert s["frac_gt3"] <= 0.01 and 0.8 <= s["mean_z2"] <= 1.25, s


def test_warmer_walls_fail_in_temperature(reps):
    a, _, c = reps
    bad = RP.check_fields(RP.field_z(a, c))
    assert "T" in bad, bad
