"""Batched cases, graph-captured stepping and the kernel-schedule autotuner.

* A batch context advances several independent cavities (different Kn,
  lid speed, mesh size and generator key) in one set of launches; each
  case must match the CPU oracle run of that case alone: the initial fill
  (positions bitwise, velocities through Box-Muller's libm calls within
  1e-12), and after steps the cell indices, (cell, pid) order and pair
  counts bit-exactly with positions and velocities to the single-step
  criteria.
* The same with nitrogen: each case's rotational energies and rotational
  sums match its own oracle run.
* dsmc_graph_step gives the same particle state as dsmc_step, bit for bit,
  for even and odd step counts, on a single case and on a batch, with
  freestream inflow, and after the particle count has grown past the count
  the graphs were captured with.
* The autotuner's choice does not change results: a context stepped through
  the autotuner's trials matches one stepped the same number of steps with
  the default schedule, bit for bit.
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


def _cases(vel_fp32=0):
    specs = [(3, 0.05, 150.0), (5, 0.5, 30.0), (4, 0.01, 200.0), (2, 1.0, 80.0)]
    out = []
    for k, (n, Kn, lid) in enumerate(specs):
        wl = W.cavity(n_hex=n, Kn=Kn, ppc=12, lid_speed=lid, seed=7, vel_fp32=vel_fp32)
        wl.run.case_id = 10 + k
        wl.run.n_ss = 0
        out.append(wl)
    return out


def _split(st, begin, k):
    m = (st["cell"] >= begin[k]) & (st["cell"] < begin[k + 1])
    return dict(n=int(m.sum()), x=st["x"][m], v=st["v"][m], cell=st["cell"][m] - begin[k], pid=st["pid"][m])


@pytest.mark.parametrize("vel_fp32", [0, 1])
def test_batch_cases_match_oracle(D, vel_fp32):
    cases = _cases(vel_fp32)
    g = D.Simulation(cases)
    begin = g.case_cells()
    assert len(begin) == len(cases) + 1 and begin[-1] == g.nt
    oracles = [Oracle(wl) for wl in cases]
    st = g.state()
    for k, o in enumerate(oracles):
        gk = _split(st, begin, k)
        ok = o.particles()
        assert np.array_equal(gk["x"], ok["x"]), f"fill positions of case {k}"
        compare_particles(gk, ok, vel_fp32, ctx=f"fill case {k}")
    for step in range(3):
        g.step(1)
        for o in oracles:
            o.step(1)
        st = g.state()
        nc, na = g.pair_counts()
        for k, o in enumerate(oracles):
            compare_particles(_split(st, begin, k), o.particles(), vel_fp32, ctx=f"case {k} step {step + 1}")
            oc, oa = o.pair_counts()
            assert np.array_equal(nc[begin[k]:begin[k + 1]], oc) and np.array_equal(na[begin[k]:begin[k + 1]], oa)
    sums, ns = g.sums(D.SAMPLE_STEADY)
    f = g.fields(D.SAMPLE_STEADY)
    for k, o in enumerate(oracles):
        assert ns == o.n_steady == 3
        compare_sums(sums[begin[k]:begin[k + 1]], o.sums(0))
        fo = o.fields(0)
        fk = f[begin[k]:begin[k + 1]]
        assert np.array_equal(np.isnan(fk), np.isnan(fo))
        scale = np.nanmax(np.abs(fo), axis=0, keepdims=True)
        assert np.all(np.nan_to_num(np.abs(fk - fo)) <= 1e-10 * scale), f"fields of case {k}"
    g.close()


def test_batch_rotating_gas_cases_match_oracle(D):
    """The batch of test_batch_cases_match_oracle with nitrogen (two
    rotational degrees of freedom): each case's rotational energies at the
    fill and after three steps within 1e-12 relative (or of k T0) of the
    oracle run of that case alone, cells, order and pair counts exact, the
    rotational sums within 1e-12 of their column scale."""
    KB = 1.380649e-23
    n2 = W.Species(mass=4.65e-26, d_ref=4.17e-10, omega=0.74, T_ref=273.0, alpha=1.0, dof_rot=2, z_rot=2.59)
    cases = _cases(0)
    for wl in cases:
        wl.species = n2
    g = D.Simulation(cases)
    begin = g.case_cells()
    oracles = [Oracle(wl) for wl in cases]

    def check(ctx):
        st = g.state()
        for k, o in enumerate(oracles):
            m = (st["cell"] >= begin[k]) & (st["cell"] < begin[k + 1])
            ok = o.particles()
            compare_particles(_split(st, begin, k), ok, 0, ctx=f"{ctx} case {k}")
            d = np.abs(st["ir"][m] - ok["ir"])
            lim = 1e-12 * np.maximum(np.abs(ok["ir"]), KB * cases[k].run.T0)
            assert np.all(d <= lim), f"{ctx} case {k}: rotational energies off by {d.max():.3e}"

    check("fill")
    for step in range(3):
        g.step(1)
        for o in oracles:
            o.step(1)
    check("after 3 steps")
    nc, na = g.pair_counts()
    rs, _ = g.rot_sums(D.SAMPLE_STEADY)
    for k, o in enumerate(oracles):
        oc, oa = o.pair_counts()
        assert np.array_equal(nc[begin[k]:begin[k + 1]], oc) and np.array_equal(na[begin[k]:begin[k + 1]], oa)
        compare_sums(rs[begin[k]:begin[k + 1]], o.rot_sums(0))
    assert sum(int(o.pair_counts()[1].sum()) for o in oracles) > 0
    g.close()


def _stream():
    import torch
    return torch.cuda.Stream()


@pytest.mark.parametrize("sort", [1, 3])
@pytest.mark.parametrize("batch", [False, True])
@pytest.mark.parametrize("n", [4, 5])
def test_graph_step_equals_eager(D, batch, n, sort):
    wl = _cases(1) if batch else W.cavity(n_hex=6, Kn=0.1, ppc=20, jitter=0.1, vel_fp32=1)
    a = D.Simulation(wl, stream=_stream())
    b = D.Simulation(wl, stream=_stream())
    for sim in (a, b):
        sim.set_tuning(15, 3, sort)
    a.step(n)
    b.graph_step(n)
    sa, sb = a.state(), b.state()
    for k in ["cell", "pid", "x", "v"]:
        assert np.array_equal(sa[k], sb[k]), k
    assert sa["step"] == sb["step"] == n
    # a second call replays the captured graphs
    a.step(6)
    b.graph_step(6)
    sa, sb = a.state(), b.state()
    assert np.array_equal(sa["x"], sb["x"]) and np.array_equal(sa["v"], sb["v"])
    assert np.array_equal(a.sums(D.SAMPLE_STEADY)[0], b.sums(D.SAMPLE_STEADY)[0])
    a.close()
    b.close()


@pytest.mark.parametrize("sort", [1, 3])
def test_graph_step_inflow_and_growth(D, sort):
    """Graph stepping with freestream inflow (grids over the whole store) and
    after the particle count grows past the count the graphs were captured
    with (they are captured again), bit-equal to ordinary stepping."""
    wl = W.open_box(n=(6, 4, 4), ppc=8, vel_fp32=1)
    a = D.Simulation(wl, stream=_stream(), capacity=60000)
    b = D.Simulation(wl, stream=_stream(), capacity=60000)
    for sim in (a, b):
        sim.set_tuning(15, 3, sort)
    a.step(4)
    b.graph_step(4)
    sa, sb = a.state(), b.state()
    assert sa["n"] == sb["n"] and all(np.array_equal(sa[k], sb[k]) for k in ["cell", "pid", "x", "v"])
    a.close()
    b.close()
    small = W.cavity(n_hex=5, Kn=0.1, ppc=10, vel_fp32=1, jitter=0.1)
    big = D.Simulation(W.cavity(n_hex=5, Kn=0.1, ppc=30, vel_fp32=1, jitter=0.1)).state()
    a = D.Simulation(small, stream=_stream(), capacity=100000)
    b = D.Simulation(small, stream=_stream(), capacity=100000)
    for sim in (a, b):
        sim.set_tuning(15, 3, sort)
    a.step(2)
    b.graph_step(2)
    for sim in (a, b):
        sim.set_state(big["x"], big["v"], big["cell"], big["pid"], 2, int(big["pid"].max()) + 1)
    a.step(4)
    b.graph_step(4)
    sa, sb = a.state(), b.state()
    assert sa["n"] == sb["n"] == big["n"]
    for k in ["cell", "pid", "x", "v"]:
        assert np.array_equal(sa[k], sb[k]), k
    a.close()
    b.close()


def test_autotune_keeps_results(D):
    wl = W.cavity(n_hex=8, Kn=0.1, ppc=20, jitter=0.1, vel_fp32=1)
    a = D.Simulation(wl)
    b = D.Simulation(wl)
    t = a.autotune(trial_steps=2)
    assert t["move"] in (1, 2, 4, 5, 6, 7, 12, 13, 14, 15, 16, 17) and t["collide"] in (0, 1, 2, 3, 4)
    assert t["sort"] in (0, 1, 2, 3)
    assert t["move_ms"] > 0 and t["collide_ms"] > 0 and t["sort_ms"] > 0
    steps = a.state(particles=False)["step"]
    # the deferred sort is tried only with the three-face move and an
    # LDS-ranked collide
    n_sorts = 4 if t["move"] == 15 and t["collide"] in (1, 2, 3, 4) else 3
    assert steps == 12 * 3 + 5 * 3 + n_sorts * 3
    b.step(steps)
    sa, sb = a.state(), b.state()
    for k in ["cell", "pid", "x", "v"]:
        assert np.array_equal(sa[k], sb[k]), k
    a.close()
    b.close()


def test_batch_refuses_inflow(D):
    wl = W.open_box(n=(4, 3, 3), ppc=4, vel_fp32=1)
    with pytest.raises(D.DsmcError):
        D.Simulation([wl, wl])
    g = D.Simulation(W.cavity(n_hex=2, Kn=1.0, ppc=4))
    with pytest.raises(D.DsmcError):
        g.dig_enable([1])
    g.close()


def _prim_close(a, b, wl, rel):
    cs = np.sqrt(1.380649e-23 / wl.species.mass * wl.run.T0)
    assert np.all(np.abs(a[:, 0] - b[:, 0]) <= rel * np.abs(b[:, 0])), "density"
    du = np.abs(a[:, 1:4] - b[:, 1:4])
    assert np.all(du <= rel * np.maximum(np.abs(b[:, 1:4]), cs)), f"velocity max {du.max():.3e}"
    assert np.all(np.abs(a[:, 4] - b[:, 4]) <= rel * np.abs(b[:, 4])), "temperature"


def test_batch_coupling_matches_oracle_per_case(D):
    """DIG coupling on a batch with cases 0 and 2 coupled and 1 and 3 left
    to plain DSMC: two cycles with DSMC steps between them, started from the
    oracle's state after a window of steps.  Each case against the oracle
    run of that case alone (coupled or not): cells, (cell, pid) order and
    particle counts exact, clone positions to 1e-12, velocities to 1e-9 of
    the largest, the kept macroscopic state M^k to 1e-10 (the criteria of
    the single-case cycle; the solve runs a fixed n_m iterations, eps_m = 0,
    so the batch-wide stopping test does not couple the cases)."""
    _batch_coupling_check(D, _cases(0), [1, 0, 1, 0])


def test_batch_coupling_open_case(D):
    """A batch coupling a closed cavity and a diffuse box with a vacuum
    outflow face: the closed case's solve is rescaled to its particles' mass,
    the open one's is not, each as the oracle run of the case alone."""
    cav = W.cavity(n_hex=3, Kn=0.05, ppc=12, lid_speed=150.0, seed=7, vel_fp32=0)
    box = W.closed_box(n_hex=3, kind=W.BC_DIFFUSE, Kn=0.05, ppc=12, vel_fp32=0, seed=7)
    box.boundaries = list(box.boundaries)
    box.boundaries[1] = W.Boundary(W.BC_OUTFLOW, 273.0)
    for k, wl in enumerate((cav, box)):
        wl.run.case_id = 30 + k
        wl.run.n_ss = 0
    _batch_coupling_check(D, [cav, box], [1, 1])


def _batch_coupling_check(D, cases, on):
    for wl in cases:
        wl.run.ewma_on = 1
        wl.run.n_a = 50
    oracles = [Oracle(wl) for wl in cases]
    for o in oracles:
        o.step(40)
    nt = [o.nt for o in oracles]
    begin = np.concatenate([[0], np.cumsum(nt)])
    sts = [o.particles() for o in oracles]
    g = D.Simulation(cases, fill=False, capacity=4 * sum(o.np for o in oracles) + 100000)
    assert np.array_equal(g.case_cells(), begin)
    cat = np.concatenate
    g.set_state(cat([s_["x"] for s_ in sts]), cat([s_["v"] for s_ in sts]),
                cat([s_["cell"] + begin[k] for k, s_ in enumerate(sts)]), cat([s_["pid"] for s_ in sts]),
                oracles[0].step_index, 0, cat([o.smax() for o in oracles]))
    g.set_sums(D.SAMPLE_EWMA, cat([o.sums(1) for o in oracles]), cat([o.ewma_counts() for o in oracles]))
    g.set_sums(D.SAMPLE_STEADY, cat([o.sums(0) for o in oracles]))
    g.dig_enable(on)
    kw = dict(kn_max=0.93, passes=3, n_m=40, eps_m=0.0, cfl=0.5, feedback=1, unconverged=1)
    changed = 0
    for cycle in range(2):
        rg = g.dig_couple(**kw)
        assert rg["iters"] == 40 and not rg["failed"]
        st = g.state()
        mprev = g.dig_get("mprev")
        for k, o in enumerate(oracles):
            n0 = o.np
            if on[k]:
                ro = o.dig_couple(**kw)
                assert ro["iters"] == 40 and not ro["failed"]
                changed += o.np != n0
            gk, ok = _split(st, begin, k), o.particles()
            ctx = f"cycle {cycle} case {k}"
            assert gk["n"] == o.np, ctx
            assert np.array_equal(gk["cell"], ok["cell"]) and np.array_equal(gk["pid"], ok["pid"]), ctx
            assert np.abs(gk["x"] - ok["x"]).max(initial=0.0) <= 1e-12, ctx
            assert np.abs(gk["v"] - ok["v"]).max(initial=0.0) <= 1e-9 * np.abs(ok["v"]).max(), ctx
            if on[k]:
                _prim_close(mprev[begin[k]:begin[k + 1]], o.mprev(), cases[k], 1e-10)
        g.step(3)
        for o in oracles:
            o.step(3)
        st = g.state()
        for k, o in enumerate(oracles):
            compare_particles(_split(st, begin, k), o.particles(), 0, ctx=f"after cycle {cycle} case {k}")
    assert changed > 0, "the feedback changed no particle count"
    g.close()


def test_ensemble64_smallest_cases_match_oracle(D):
    """The benchmark's 64-case ensemble (2.5M tets, 50M particles) advanced
    in one context, two steps with ordinary launches and two replayed from
    captured graphs; the eight smallest cases against the oracle run of each
    case alone (cells, order and pair counts exact, positions and velocities
    to the single-step criteria, sums and fields)."""
    cases = W.cavity_ensemble(64)
    for wl in cases:
        wl.run.n_ss = 0
    g = D.Simulation(cases, stream=_stream())
    begin = g.case_cells()
    g.step(2)
    g.graph_step(2)
    sizes = np.diff(begin)
    small = np.argsort(sizes, kind="stable")[:8]
    st = g.state()
    nc, na = g.pair_counts()
    sums, ns = g.sums(D.SAMPLE_STEADY)
    assert ns == 4
    for k in small:
        o = Oracle(cases[k])
        o.step(4)
        compare_particles(_split(st, begin, k), o.particles(), 1, ctx=f"case {k}")
        oc, oa = o.pair_counts()
        assert np.array_equal(nc[begin[k]:begin[k + 1]], oc) and np.array_equal(na[begin[k]:begin[k + 1]], oa)
        compare_sums(sums[begin[k]:begin[k + 1]], o.sums(0))
    g.close()


def _close(gk, ok, ctx, rel=1e-9):
    """Criteria of the coupled cycle: cells, order and counts exact; positions
    to 1e-11 m and velocities to `rel` of the largest speed (the solve's
    ulp-level differences carried through the feedback)."""
    assert gk["n"] == len(ok["pid"]), ctx
    assert np.array_equal(gk["cell"], ok["cell"]) and np.array_equal(gk["pid"], ok["pid"]), ctx
    assert np.abs(gk["x"] - ok["x"]).max(initial=0.0) <= 1e-11, ctx
    assert np.abs(gk["v"] - ok["v"]).max(initial=0.0) <= rel * np.abs(ok["v"]).max(), ctx


def test_ensemble64_half_coupled_smallest_cases_match_oracle(D):
    """The 64-case ensemble with the coupling step on half of the cases (four
    of the eight smallest among them) and a closure network attached: two
    ordinary and two graph-replayed steps, one coupling cycle, then two
    ordinary and two graph-replayed steps again.  The closure is evaluated on
    every cell and its gate set to zero tolerance, so every cell keeps its
    sampled HoT and the cycle is the oracle's.  Velocities are stored in
    FP64 here: the solve's ulp-level differences would otherwise turn into
    FP32 rounding flips.  The eight smallest cases against the oracle run of
    each case alone (coupled or not): cells, order and pair counts exact,
    positions to 1e-11 m, velocities and steady sums to 1e-9."""
    cases = W.cavity_ensemble(64, vel_fp32=0)
    for wl in cases:
        wl.run.n_ss = 0
        wl.run.ewma_on = 1
        wl.run.n_a = 50
    g = D.Simulation(cases, stream=_stream())
    begin = g.case_cells()
    small = np.argsort(np.diff(begin), kind="stable")[:8]
    on = (np.arange(len(cases)) % 2 == 1).astype(np.int32)
    for i, k in enumerate(small):
        on[k] = 1 - i % 2
    g.dig_enable(on)
    net = D.Mlp()
    net.init_weights(seed=3)
    g.set_closure(net, gate_tol=0.0)
    oracles = {int(k): Oracle(cases[k]) for k in small}
    kw = dict(kn_max=0.93, passes=3, n_m=20, eps_m=0.0, cfl=0.5, feedback=1, unconverged=1)
    g.step(2)
    g.graph_step(2)
    for o in oracles.values():
        o.step(4)
    r = g.dig_couple(**kw)
    assert r["iters"] == 20 and not r["failed"]
    assert r["n_closure"] == 0 and r["n_fallback"] > 0
    changed = 0
    for k, o in oracles.items():
        if on[k]:
            n0 = o.np
            o.dig_couple(**kw)
            changed += o.np != n0
    assert changed > 0
    st = g.state()
    for k, o in oracles.items():
        _close(_split(st, begin, k), o.particles(), f"coupled case {k}")
    g.step(2)
    g.graph_step(2)
    for o in oracles.values():
        o.step(4)
    st = g.state()
    nc, na = g.pair_counts()
    sums, ns = g.sums(D.SAMPLE_STEADY)
    assert ns == 8
    for k, o in oracles.items():
        _close(_split(st, begin, k), o.particles(), f"case {k}")
        oc, oa = o.pair_counts()
        assert np.array_equal(nc[begin[k]:begin[k + 1]], oc) and np.array_equal(na[begin[k]:begin[k + 1]], oa)
        compare_sums(sums[begin[k]:begin[k + 1]], o.sums(0), rel=1e-9)
    net.close()
    g.close()


def test_batch_coupling_with_no_case_enabled_changes_nothing(D):
    """All cases of a batch disabled: the coupling step runs its gate and
    leaves every particle, the local-accumulation flags and the particle
    count as they were."""
    cases = _cases(1)
    for wl in cases:
        wl.run.ewma_on = 1
        wl.run.n_a = 50
    g = D.Simulation(cases)
    g.step(20)
    st0 = g.state()
    g.dig_enable([0] * len(cases))
    r = g.dig_couple(kn_max=0.93, passes=3, n_m=20, eps_m=0.0, cfl=0.5, feedback=1, unconverged=1)
    assert not r["failed"] and r["np_after"] == r["np_before"] == st0["n"]
    st1 = g.state()
    for k in ["x", "v", "cell", "pid"]:
        assert np.array_equal(st0[k], st1[k]), k
    g.step(2)
    g.close()


def test_persistent_move_on_the_ensemble_equals_the_default(D):
    """The 64-case ensemble stepped with the persistent, XCD-sliced tile
    queue (move schedule 17) and with the default schedule: identical
    particle states, pair counts and sums after two ordinary and two
    graph-replayed steps (every schedule computes the same per-particle
    arithmetic; only which workgroup takes which tile differs)."""
    cases = W.cavity_ensemble(64)
    out = []
    for move in (15, 17):
        g = D.Simulation(cases, stream=_stream())
        t = g.tuning()
        g.set_tuning(move, t["collide"], t["sort"])
        g.step(2)
        g.graph_step(2)
        st = g.state()
        out.append((st, g.pair_counts(), g.sums(D.SAMPLE_STEADY)[0], g.stats()))
        g.close()
    (a, pa, sa, ca), (b, pb, sb, cb) = out
    for k in ["x", "v", "cell", "pid"]:
        assert np.array_equal(a[k], b[k]), k
    assert all(np.array_equal(x, y) for x, y in zip(pa, pb))
    assert np.array_equal(sa, sb)
    assert ca == cb
