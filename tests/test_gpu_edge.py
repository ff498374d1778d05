"""Degenerate inputs of the per-step path, through the C ABI, against the
oracle:
  * an empty particle store: steps leave it empty, sums, pair counts and
    counters stay zero and the fields are NaN;
  * a freestream filling an empty box: the injected particles match the
    oracle's (cells and (cell, pid) order bit-exact, positions and
    velocities to the single-step criteria) step after step;
  * a single particle bouncing between diffuse walls for many steps (no
    collision partner; every re-emission draw must agree);
  * the smallest closed mesh the workloads build, one hex split into 6 tets.
"""
import numpy as np
import pytest

from paper_2607_08195_amd import workloads as W
from oracle import Oracle
from parity_util import compare_particles, compare_sums

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_08195_amd import dsmc
    return dsmc


def _empty(n=0):
    return (np.zeros((n, 3)), np.zeros((n, 3)), np.zeros(n, np.int32), np.zeros(n, np.uint32))


def test_empty_store_steps(D):
    wl = W.cavity(n_hex=3, Kn=0.1, ppc=10, vel_fp32=1)
    wl.run.n_ss = 0
    g = D.Simulation(wl, fill=False, capacity=4096)
    x, v, c, p = _empty()
    g.set_state(x, v, c, p, 0, 0)
    g.step(3)
    st = g.state()
    assert st["n"] == 0 and st["step"] == 3
    sums, ns = g.sums(D.SAMPLE_STEADY)
    assert ns == 3 and not sums.any()
    nc, na = g.pair_counts()
    assert not nc.any() and not na.any()
    assert np.isnan(g.fields(D.SAMPLE_STEADY)).all()
    s = g.stats()
    assert s["n_particles"] == 0 and s["hops"] == 0 and s["wall_hits"] == 0 and s["lost"] == 0
    g.close()


def test_inflow_into_empty_box_matches_oracle(D):
    wl = W.open_box(n=(6, 4, 4), ppc=8, vel_fp32=1)
    wl.run.n0 = 0.0
    wl.run.n_ss = 0
    o = Oracle(wl)
    assert o.np == 0
    g = D.Simulation(wl, capacity=40000)
    assert g.state()["n"] == 0
    for k in range(5):
        o.step(1)
        g.step(1)
        compare_particles(g.state(), o.particles(), 1, L0=4.0, ctx=f"step {k + 1}")
        gc, ga = g.pair_counts()
        oc, oa = o.pair_counts()
        assert np.array_equal(gc, oc) and np.array_equal(ga, oa)
    assert o.np > 0
    compare_sums(g.sums(D.SAMPLE_STEADY)[0], o.sums(0))
    g.close()


@pytest.mark.parametrize("vel_fp32", [0, 1])
def test_single_particle_matches_oracle(D, vel_fp32):
    wl = W.cavity(n_hex=2, Kn=1.0, ppc=5, vel_fp32=vel_fp32, lid_speed=300.0)
    wl.run.n_ss = 0
    st = Oracle(wl).particles()
    one = (st["x"][3:4], st["v"][3:4], st["cell"][3:4], st["pid"][3:4])
    o = Oracle(wl, fill=False)
    o.set_particles(*one, 0, 1)
    g = D.Simulation(wl, fill=False, capacity=64)
    g.set_state(*one, 0, 1)
    for k in range(40):
        o.step(1)
        g.step(1)
        compare_particles(g.state(), o.particles(), vel_fp32, ctx=f"step {k + 1}")
    c0 = o.counters()
    assert g.stats()["wall_hits"] == c0["wall_hits"] > 0
    compare_sums(g.sums(D.SAMPLE_STEADY)[0], o.sums(0))
    g.close()


def test_one_hex_mesh_matches_oracle(D):
    wl = W.cavity(n_hex=1, Kn=0.2, ppc=40, vel_fp32=1, lid_speed=100.0)
    wl.run.n_ss = 0
    o = Oracle(wl)
    g = D.Simulation(wl)
    for k in range(6):
        o.step(1)
        g.step(1)
        compare_particles(g.state(), o.particles(), 1, ctx=f"step {k + 1}")
        gc, ga = g.pair_counts()
        oc, oa = o.pair_counts()
        assert np.array_equal(gc, oc) and np.array_equal(ga, oa)
    compare_sums(g.sums(D.SAMPLE_STEADY)[0], o.sums(0))
    g.close()
