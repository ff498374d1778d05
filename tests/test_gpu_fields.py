"""Macroscopic fields of long runs against the oracle within the sampling
noise: the CPU-finishable cavity (6^3 x 6 tets, Kn = 1, 20 particles per
cell, FP64 velocities, seed 0), 200 unsampled steps, then six batches of 50
sampled steps on both sides.  Per region of 2 x 2 x 2 hexes (48 tets) and
batch, density, velocity and temperature from the region's summed moments;
per region and field the GPU's and the oracle's batch means must agree
within the noise estimated from the batch-to-batch spread (z = difference /
combined standard error: mean z^2 below 3, no |z| above 6).  Over hundreds
of steps one flipped acceptance (the device's and the host's FP64 powers
may differ in the last bit) decorrelates the two runs, so this is the
statistical form of parity."""
import numpy as np
import pytest

from paper_2607_08195_amd import workloads as W
from oracle import Oracle
from statutil import fields_from_sums

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_08195_amd import dsmc
    return dsmc


def _regions(wl, o):
    xyz, tets = wl.mesh.xyz, o.tets()
    cen = xyz[tets].mean(axis=1)
    ijk = np.minimum((cen * 3).astype(int), 2)
    return ijk[:, 0] * 9 + ijk[:, 1] * 3 + ijk[:, 2]


def _batch_fields(sums, reg, vol, wl, blen):
    out = []
    for r in range(27):
        sel = reg == r
        f = fields_from_sums(sums[sel].sum(axis=0), wl.species.mass, wl.run.F_N, vol[sel].sum(), blen)
        out.append([f["n"], f["u"][0], f["u"][1], f["u"][2], f["T"]])
    return np.array(out)


def test_cavity_small_fields_within_sampling_noise(D):
    wl = W.cavity_small()
    wl.run.n_ss = 200
    o = Oracle(wl)
    g = D.Simulation(wl)
    reg = _regions(wl, o)
    vol = o.volumes()
    o.step(200)
    g.step(200)
    go, gg = [], []
    po = pg = 0.0
    for _ in range(6):
        o.step(50)
        g.step(50)
        so = o.sums(0)
        sg, ns = g.sums(D.SAMPLE_STEADY)
        go.append(_batch_fields(so - po, reg, vol, wl, 50))
        gg.append(_batch_fields(sg - pg, reg, vol, wl, 50))
        po, pg = so, sg
    go, gg = np.array(go), np.array(gg)          # [batch, region, field]
    mo, mg = go.mean(axis=0), gg.mean(axis=0)
    se = np.sqrt(go.var(axis=0, ddof=1) / 6 + gg.var(axis=0, ddof=1) / 6)
    # velocity fields are near zero in parts of the cavity: floor the noise
    # estimate at a small fraction of the thermal speed and density scales
    floor = np.array([1e-4 * mo[:, 0].mean(), 0.05, 0.05, 0.05, 0.05])
    z = (mg - mo) / np.maximum(se, floor)
    assert np.mean(z * z) < 3.0, (np.mean(z * z), np.abs(z).max())
    assert np.abs(z).max() < 6.0, np.abs(z).max()
    # the lid drives the flow: the top regions move with +x
    top = [r for r in range(27) if (r // 3) % 3 == 2]
    assert (mo[top, 1] > 0).all() and (mg[top, 1] > 0).all()
