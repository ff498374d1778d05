"""Failure handling of the oracle's tracker (the bounded hop loop of the
face-to-face tracking): a particle whose position lies in no cell (a
non-finite coordinate) crosses faces without ever finding its exit time and
is deleted at the hop limit and counted as lost; the other particles keep
finite positions."""
import numpy as np

from paper_2607_08195_amd import workloads as W
from oracle import Oracle


def _cavity():
    wl = W.cavity(n_hex=4, Kn=1.0, ppc=10, vel_fp32=0)
    o = Oracle(wl)
    return wl, o


def test_non_finite_position_is_lost_at_the_hop_limit():
    wl, o = _cavity()
    st = o.particles()
    n = len(st["pid"])
    x = st["x"].copy()
    x[17, 1] = np.nan
    o.set_particles(x, st["v"], st["cell"], st["pid"], o.step_index, o.next_pid)
    h0 = o.counters()["hops"]
    o.step(1)
    c = o.counters()
    assert c["lost"] == 1
    assert c["hops"] - h0 > 1000
    p = o.particles()
    assert len(p["pid"]) == n - 1 and st["pid"][17] not in set(p["pid"].tolist())
    assert np.isfinite(p["x"]).all()
