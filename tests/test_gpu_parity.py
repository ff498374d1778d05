"""GPU path against the CPU oracle through the C ABI.

Single-step parity from an identical state (set from the oracle's own
state on both sides): bit-exact cell indices, (cell, pid) order and
per-cell candidate/accepted pair counts; positions within 1e-12 relative;
velocities within 1 float32 ulp (FP32 storage) or 1e-12 relative (FP64);
moment sums within 1e-12 relative; (sigma c)_max within 1e-15 relative (a
new maximum is an FP64 power, whose device and host results may differ in
the last bit).  Cases cover diffuse walls with a moving
lid, jittered irregular tets, specular walls, periodic plates, freestream
inflow/outflow, sparse cells (0-1 particles), dense chunks beyond the LDS
stage, VSS scattering (alpha = 1.4, 1.6) and the full 384,000-tet cavity in
the benchmark's configuration."""
import numpy as np
import pytest

from paper_2607_08195_amd import workloads as W
from oracle import Oracle
from parity_util import compare_particles, compare_sums

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dsmc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_08195_amd import dsmc as D
    return D


def _cases():
    c = {}
    c["cavity_6_fp64_kn1"] = (lambda: W.cavity(n_hex=6, Kn=1.0, ppc=20, vel_fp32=0), 10)
    c["cavity_8_fp32_jitter_kn0.1"] = (lambda: W.cavity(n_hex=8, Kn=0.1, ppc=30, jitter=0.1, vel_fp32=1), 5)
    c["specular_box"] = (lambda: W.closed_box(n_hex=5, kind=W.BC_SPECULAR, ppc=15, vel_fp32=1), 3)
    c["plates_periodic_couette"] = (lambda: W.plates(n=(3, 6, 3), U=300.0, T1=250.0, T2=350.0, ppc=25,
                                                     n0=3e19, vel_fp32=0), 4)
    c["open_box_inflow"] = (lambda: W.open_box(n=(6, 4, 4), ppc=12, vel_fp32=1), 6)
    c["sparse_ppc1"] = (lambda: W.cavity(n_hex=6, Kn=0.5, ppc=1, jitter=0.1, vel_fp32=1), 2)
    c["dense_ppc45"] = (lambda: W.cavity(n_hex=5, Kn=0.05, ppc=45, jitter=0.1, vel_fp32=1), 1)
    c["sphere_hypersonic"] = (lambda: W.sphere_flow(N=4, K=3, ppc=8, vel_fp32=1), 4)
    # VSS scattering (alpha != 1): deflection about the relative velocity
    c["vss_cavity_fp64_a1.4"] = (lambda: _vss(W.cavity(n_hex=6, Kn=0.5, ppc=20, vel_fp32=0), 1.4), 6)
    c["vss_dense_fp32_a1.6"] = (lambda: _vss(W.cavity(n_hex=5, Kn=0.05, ppc=45, jitter=0.1, vel_fp32=1), 1.6), 1)
    return c


def _vss(wl, alpha):
    wl.species.alpha = alpha
    wl.name += f"_vss{alpha}"
    return wl


CASES = _cases()


def _smax_close(a, b):
    d = np.abs(a - b) / np.abs(b)
    assert (d <= 1e-15).all(), f"(sigma c)_max: {int((d > 0).sum())} cells differ, max rel {d.max():.3e}"


def _one_step_parity(D, wl, presteps, steps=1, move=None, collide=None, sort=None):
    wl.run.n_ss = presteps
    o = Oracle(wl)
    o.step(presteps)
    st = o.particles()
    c0 = o.counters()
    g = D.Simulation(wl, fill=False, capacity=max(4 * o.np, 100000))
    g.set_state(st["x"], st["v"], st["cell"], st["pid"], o.step_index, o.next_pid, o.smax())
    if move is not None or collide is not None or sort is not None:
        t = g.tuning()
        g.set_tuning(t["move"] if move is None else move, t["collide"] if collide is None else collide,
                     t["sort"] if sort is None else sort)
    for _ in range(steps):
        o.step(1)
        g.step(1)
    gs = g.state()
    os_ = o.particles()
    info = compare_particles(gs, os_, wl.run.vel_fp32, ctx=wl.name)
    gc, ga = g.pair_counts()
    oc, oa = o.pair_counts()
    assert np.array_equal(gc, oc), "candidate pair counts differ"
    assert np.array_equal(ga, oa), "accepted pair counts differ"
    _smax_close(gs["smax"], o.smax())
    gsum, ns = g.sums(D.SAMPLE_STEADY)
    assert ns == o.n_steady == steps
    compare_sums(gsum, o.sums(0))
    c1 = o.counters()
    gstat = g.stats()
    for k in ["hops", "wall_hits", "injected", "removed", "lost"]:
        assert gstat[k] == c1[k] - c0[k], k
    assert gstat["step"] == o.step_index
    g.close()
    return info


@pytest.mark.parametrize("name", list(CASES))
def test_single_step_parity(dsmc, name):
    make, pre = CASES[name]
    wl = make()
    info = _one_step_parity(dsmc, wl, pre)
    print(name, info)


# every move schedule; the capped ones (12-14) park particles in flight
# after 4-6 exit tests and 15/16 test three faces after the first crossing,
# which these cases (several hops per step, diffuse, specular, periodic and
# open faces) exercise
MOVES = [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17]
MOVE_CASES = ["cavity_6_fp64_kn1", "specular_box", "plates_periodic_couette", "open_box_inflow", "sphere_hypersonic"]


@pytest.mark.parametrize("case", MOVE_CASES)
@pytest.mark.parametrize("move", MOVES)
def test_move_schedules_parity(dsmc, move, case):
    make, pre = CASES[case]
    wl = make()
    _one_step_parity(dsmc, wl, pre, steps=2, move=move)


# every collide schedule; the dense case puts more particles in a 64-cell
# chunk than the LDS of the smaller-chunk schedules holds (global fallback);
# the FP64 case stages double-precision velocities
@pytest.mark.parametrize("case", ["cavity_8_fp32_jitter_kn0.1", "dense_ppc45", "sparse_ppc1", "cavity_6_fp64_kn1",
                                  "vss_cavity_fp64_a1.4", "vss_dense_fp32_a1.6"])
@pytest.mark.parametrize("collide", [0, 1, 2, 3, 4])
def test_collide_schedules_parity(dsmc, collide, case):
    make, pre = CASES[case]
    _one_step_parity(dsmc, make(), pre, steps=2, collide=collide)


# every sort schedule with an LDS-staged and an LDS-ranked collide schedule:
# the fused form gathers inside the collide kernel (the dense case takes its
# global-memory path after the gather), with collide 0 it falls back to the
# gather kernel; the inflow case sorts injected particles too
@pytest.mark.parametrize("case", ["cavity_8_fp32_jitter_kn0.1", "dense_ppc45", "open_box_inflow", "cavity_6_fp64_kn1",
                                  "vss_dense_fp32_a1.6"])
@pytest.mark.parametrize("collide", [0, 3])
@pytest.mark.parametrize("sort", [0, 1, 2])
def test_sort_schedules_parity(dsmc, sort, collide, case):
    make, pre = CASES[case]
    _one_step_parity(dsmc, make(), pre, steps=2, collide=collide, sort=sort)


# deferred sort: the move reads the particles in the previous step's sorted
# order and writes them sorted, the collide kernel reaches them through the
# order; three steps, so that the second and third moves start from an order
# the sort computed (the first starts from the identity order)
@pytest.mark.parametrize("case", ["cavity_8_fp32_jitter_kn0.1", "dense_ppc45", "open_box_inflow", "cavity_6_fp64_kn1",
                                  "vss_dense_fp32_a1.6", "sphere_hypersonic", "plates_periodic_couette",
                                  "specular_box", "sparse_ppc1"])
@pytest.mark.parametrize("collide", [1, 2, 3, 4])
def test_deferred_sort_parity(dsmc, collide, case):
    make, pre = CASES[case]
    _one_step_parity(dsmc, make(), pre, steps=3, move=15, collide=collide, sort=3)


def test_deferred_sort_refuses_other_schedules(dsmc):
    g = dsmc.Simulation(W.cavity(n_hex=3, Kn=0.5, ppc=5, vel_fp32=1))
    for move, collide in [(12, 3), (15, 0), (17, 3)]:
        with pytest.raises(dsmc.DsmcError):
            g.set_tuning(move, collide, 3)
    # a move without the sort is refused (it would leave the store unsorted)
    with pytest.raises(dsmc.DsmcError):
        g.step_stages(1)
    g.close()


def test_deferred_sort_matches_gather_across_reads(dsmc):
    """Deferred stepping interleaved with state reads (which write the
    pending order out) and with surface sampling gives the states of the
    gather sort, bit for bit."""
    wl = W.cavity(n_hex=7, Kn=0.1, ppc=25, jitter=0.1, vel_fp32=1)
    a = dsmc.Simulation(wl)
    b = dsmc.Simulation(wl)
    a.set_tuning(15, 3, 1)
    b.set_tuning(15, 3, 3)
    a.surface_sampling(True)
    b.surface_sampling(True)
    for n in [1, 3, 2, 5]:
        a.step(n)
        b.step(n)
        sa, sb = a.state(), b.state()
        for k in ["cell", "pid", "x", "v"]:
            assert np.array_equal(sa[k], sb[k]), (n, k)
    assert np.array_equal(a.sums(dsmc.SAMPLE_STEADY)[0], b.sums(dsmc.SAMPLE_STEADY)[0])
    assert np.array_equal(a.surface()[0], b.surface()[0])
    a.close()
    b.close()


def test_three_steps_parity_fp64(dsmc):
    wl = W.cavity(n_hex=6, Kn=1.0, ppc=20, vel_fp32=0)
    _one_step_parity(dsmc, wl, 0, steps=3)


def test_init_fill_parity(dsmc):
    for wl in [W.cavity(n_hex=6, Kn=1.0, ppc=20, vel_fp32=0),
               W.cavity(n_hex=7, Kn=0.1, ppc=30, jitter=0.1, vel_fp32=1)]:
        o = Oracle(wl)
        g = dsmc.Simulation(wl)
        gs = g.state()
        os_ = o.particles()
        compare_particles(gs, os_, wl.run.vel_fp32, ctx="init " + wl.name)
        # positions involve no libm: bitwise equal
        assert np.array_equal(gs["x"], os_["x"])
        _smax_close(gs["smax"], o.smax())
        assert gs["next_pid"] == o.next_pid
        g.close()


def test_ewma_and_local_accumulation_parity(dsmc):
    wl = W.cavity(n_hex=6, Kn=0.5, ppc=20, vel_fp32=1, ewma_on=1, n_a=3)
    o = Oracle(wl)
    st = o.particles()
    g = dsmc.Simulation(wl, fill=False)
    g.set_state(st["x"], st["v"], st["cell"], st["pid"], o.step_index, o.next_pid, o.smax())
    flags = (np.arange(o.nt) % 3 == 0).astype(np.uint8)
    o.set_local_acc(flags)
    g.set_local_acc(flags)
    for _ in range(5):
        o.step(1)
        g.step(1)
    compare_particles(g.state(), o.particles(), 1)
    compare_sums(g.sums(dsmc.SAMPLE_EWMA)[0], o.sums(1))
    gf = g.fields(dsmc.SAMPLE_EWMA)
    of = o.fields(1)
    ok = np.isfinite(of)
    assert np.array_equal(ok, np.isfinite(gf))
    assert np.allclose(gf[ok], of[ok], rtol=1e-10, atol=0)
    g.close()


def test_determinism_run_twice(dsmc):
    wl = W.cavity(n_hex=8, Kn=0.1, ppc=30, jitter=0.1, vel_fp32=1)
    res = []
    for _ in range(2):
        g = dsmc.Simulation(wl)
        g.step(20)
        s = g.state()
        res.append((s, g.sums(dsmc.SAMPLE_STEADY)[0], g.stats()))
        g.close()
    a, b = res
    for k in ["x", "v", "cell", "pid", "smax"]:
        assert np.array_equal(a[0][k], b[0][k]), k
    assert np.array_equal(a[1], b[1])
    assert a[2] == b[2]


def test_capacity_overflow_reported(dsmc):
    wl = W.open_box(n=(6, 4, 4), ppc=12, vel_fp32=1)
    o = Oracle(wl, fill=True)
    g = dsmc.Simulation(wl, capacity=o.np + 10)
    with pytest.raises(dsmc.DsmcError) as e:
        for _ in range(5):
            g.step(1)
        g.sync()
    assert e.value.status == -5
    g.close()


def test_full_size_cavity_single_step(dsmc):
    """384,000 jittered tets, 11.52M particles, FP32 velocities: one step of
    the benchmark's kernels against the oracle from the oracle's initial
    state, compared on every particle and cell."""
    wl = W.cavity_large()
    info = _one_step_parity(dsmc, wl, 0)
    print("full size", info)


def test_full_size_vss_cavity_single_step(dsmc):
    """The same cavity with argon as a variable soft sphere (alpha = 1.40, the
    `cavity_vss` benchmark workload): one step of the VSS collide instance
    against the oracle on every particle and cell."""
    wl = W.cavity_large_vss()
    info = _one_step_parity(dsmc, wl, 0)
    print("full size vss", info)


def test_full_size_sphere_single_step(dsmc):
    """The hypersonic sphere at the benchmark's size (1,963,104 tets, 50M
    particles, FP32 velocities, inflow on five faces and outflow) with the
    schedules the autotuner chose for it (move defer5, collide global3k,
    sort fused): one step from the oracle's initial fill against the oracle,
    compared on every particle and cell."""
    wl = W.sphere_flow(N=22, K=16, grade=5.0, n_particles=50_000_000, vel_fp32=1)
    info = _one_step_parity(dsmc, wl, 0, move=7, collide=3, sort=2)
    print("full size sphere", info)


@pytest.mark.parametrize("case", ["cavity_6_fp64_kn1", "open_box_inflow", "sparse_ppc1"])
def test_instant_sums_match_oracle(dsmc, case):
    """DSMC_SAMPLE_INSTANT: zero until switched on, then the moment sums of
    the last step alone, step after step (1e-12 of the column scale), and
    the fields computed from them (NaN where a cell holds no particle),
    against the oracle's per-step sums and fields."""
    make, pre = CASES[case]
    wl = make()
    wl.run.n_ss = pre
    o = Oracle(wl)
    o.step(pre)
    st = o.particles()
    g = dsmc.Simulation(wl, fill=False, capacity=max(4 * o.np, 100000))
    g.set_state(st["x"], st["v"], st["cell"], st["pid"], o.step_index, o.next_pid, o.smax())
    s0, n0 = g.sums(dsmc.SAMPLE_INSTANT)
    assert n0 == 1 and not s0.any()
    g.instant_sampling(True)
    for k in range(2):
        o.step(1)
        g.step(1)
        gs, _ = g.sums(dsmc.SAMPLE_INSTANT)
        compare_sums(gs, o.sums(2))
        fg, fo = g.fields(dsmc.SAMPLE_INSTANT), o.fields(2)
        assert np.array_equal(np.isnan(fg), np.isnan(fo)), f"step {k}"
        scale = np.nanmax(np.abs(fo), axis=0, keepdims=True)
        assert np.all(np.nan_to_num(np.abs(fg - fo)) <= 1e-10 * scale), f"step {k}"
    g.instant_sampling(False)
    kept, _ = g.sums(dsmc.SAMPLE_INSTANT)
    g.step(1)
    assert np.array_equal(g.sums(dsmc.SAMPLE_INSTANT)[0], kept)
    g.close()
