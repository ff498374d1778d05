"""The coupling step of a rotating gas on the GPU against the CPU oracle
(section 2.2: eq. macro with the rotational energy equation and its
relaxation source, eq. thermal_conductivity_matrix; the paper's nitrogen),
through the C ABI.

Both sides start from one state: the oracle runs a window of DSMC steps with
the moving average on, then its particles (with I_r), (sigma c)_max and the
translational and rotational moving-average sums are loaded into the GPU
context.  Criteria (those of the monatomic coupling tests):
  * sampled state (18 columns, T_r and q_r included): bit-exact;
  * gate states, report counts, iterations, particle counts, cells and
    (cell, pid) order: exact;
  * residual: 1e-11 of the column's scale; solve and M^{k+1}: 1e-10
    relative (ulp-level differences of pow through a few hundred stable
    iterations);
  * feedback: positions bit-exact, velocities within one FP32 ulp or
    1e-12, rotational energies within 1e-12 relative.
The learned closure and the accelerated solve are refused for a rotating
gas.
"""
import numpy as np
import pytest

from paper_2607_08195_amd import workloads as W
from oracle import Oracle
from parity_util import compare_particles

pytestmark = pytest.mark.gpu

KB = 1.380649e-23


@pytest.fixture(scope="module")
def D():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_08195_amd import dsmc
    return dsmc


def _n2_cavity(vel_fp32=0, Kn=0.1, n_hex=6, ppc=20, jitter=0.0):
    sp = W.Species(mass=4.65e-26, d_ref=4.17e-10, omega=0.74, T_ref=273.0, alpha=1.0, dof_rot=2, z_rot=2.59)
    return W.cavity(n_hex=n_hex, Kn=Kn, ppc=ppc, vel_fp32=vel_fp32, jitter=jitter, lid_speed=80.0, species=sp)


def _pair(D, wl, steps, n_a=50):
    wl.run.ewma_on = 1
    wl.run.n_a = n_a
    o = Oracle(wl)
    o.step(steps)
    st = o.particles()
    g = D.Simulation(wl, fill=False, capacity=max(4 * o.np, 100000))
    g.set_state(st["x"], st["v"], st["cell"], st["pid"], o.step_index, o.next_pid, o.smax(), ir=st["ir"])
    g.set_sums(D.SAMPLE_EWMA, o.sums(1), o.ewma_counts())
    g.set_sums(D.SAMPLE_STEADY, o.sums(0))
    g.set_rot_sums(D.SAMPLE_EWMA, o.rot_sums(1))
    g.set_rot_sums(D.SAMPLE_STEADY, o.rot_sums(0))
    return o, g


def _nan_equal(a, b):
    return np.array_equal(np.isnan(a), np.isnan(b)) and np.array_equal(a[~np.isnan(a)], b[~np.isnan(b)])


def _rel_close(a, b, rel, what):
    d = np.abs(a - b)
    lim = rel * np.maximum(np.abs(b), np.abs(b).max(axis=0, keepdims=True) * 1e-6)
    assert np.all(d <= lim), f"{what}: max rel {np.max(d / np.maximum(np.abs(b), 1e-300)):.3e}"


def _col_close(a, b, rel, what):
    scale = np.abs(b).max(axis=0, keepdims=True) + 1e-300
    d = np.abs(a - b) / scale
    assert (d <= rel).all(), f"{what}: max {d.max():.3e}"


def _ir_close(g, o, ctx):
    d = np.abs(g["ir"] - o["ir"])
    assert np.all(d <= 1e-12 * np.abs(o["ir"]) + 1e-300), f"{ctx}: I_r max {d.max():.3e}"


@pytest.mark.parametrize("vel_fp32", [0, 1])
def test_couple_matches_oracle(D, vel_fp32):
    wl = _n2_cavity(vel_fp32=vel_fp32)
    o, g = _pair(D, wl, steps=40)
    kw = dict(kn_max=0.93, passes=3, n_m=60, eps_m=1e-8, cfl=0.5, feedback=1, unconverged=1)
    smp = o.dig_sampled()
    assert smp.shape[1] == 18
    rg = g.dig_couple(**kw)
    ro = o.dig_couple(**kw)
    assert _nan_equal(g.dig_get("sampled"), smp)
    for k in ["n_rejected", "n_reconstructed", "n_unreached", "iters", "converged", "failed", "np_before",
              "np_after", "fed_back"]:
        assert rg[k] == ro[k], (k, rg[k], ro[k])
    assert 0 < ro["n_rejected"] < o.nt, "the case should exercise the gate"
    assert ro["fed_back"] == 1
    assert abs(rg["residual"] - ro["residual"]) <= 1e-8 * max(ro["residual"], 1e-12)
    mp = g.dig_get("mprev")
    assert mp.shape == (o.nt, 6)
    _rel_close(mp, o.mprev(), 1e-10, "M^{k+1}")
    gs, os_ = g.state(), o.particles()
    compare_particles(gs, os_, vel_fp32, ctx="after feedback")
    _ir_close(gs, os_, "after feedback")
    g.close()


def test_residual_and_solve_match_oracle(D):
    wl = _n2_cavity(jitter=0.1)
    o, g = _pair(D, wl, steps=30)
    smp = o.dig_sampled()
    ok = np.isfinite(smp[:, 0]) & (smp[:, 0] > 0)
    assert ok.all()
    prim = np.concatenate([smp[:, :5], smp[:, 14:15]], axis=1)
    # out of rotational equilibrium, so the relaxation source is active
    prim[:, 5] = prim[:, 5] * 0.9
    rng = np.random.default_rng(5)
    sig = np.abs(smp[:, 5:14]).mean(axis=0)
    hot = np.concatenate([smp[:, 5:14], smp[:, 15:18]], axis=1) * 0.0
    hot[:, :9] = rng.normal(0, 1, (o.nt, 9)) * sig * 0.3
    hot[:, 9:] = rng.normal(0, 1, (o.nt, 3)) * np.abs(smp[:, 15:18]).mean(axis=0) * 0.3
    rg = g.dig_residual(prim, hot)
    ro = o.dig_residual(prim, hot)
    assert rg.shape == (o.nt, 6)
    _col_close(rg, ro, 1e-11, "residual")
    kw = dict(n_m=120, eps_m=0.0, cfl=0.5)
    pg, repg = g.dig_solve(prim, hot, **kw)
    po, repo = o.dig_solve(prim, hot, **kw)
    assert repg["iters"] == repo["iters"] == 120 and not repo["failed"]
    _rel_close(pg, po, 1e-10, "solve")
    # the relaxation moved T_r toward T
    assert np.abs(po[:, 5] / po[:, 4] - 1).mean() < np.abs(prim[:, 5] / prim[:, 4] - 1).mean()
    g.close()


@pytest.mark.parametrize("vel_fp32", [0, 1])
def test_feedback_matches_oracle(D, vel_fp32):
    wl = _n2_cavity(vel_fp32=vel_fp32, ppc=25)
    o, g = _pair(D, wl, steps=10)
    smp = o.dig_sampled()
    old = np.concatenate([smp[:, :5], smp[:, 14:15]], axis=1)
    new = old.copy()
    rng = np.random.default_rng(3)
    new[:, 0] *= 1.0 + 0.1 * rng.uniform(-1, 1, o.nt)
    new[:, 1:4] += 5.0 * rng.normal(size=(o.nt, 3))
    new[:, 4] *= 1.0 + 0.05 * rng.uniform(-1, 1, o.nt)
    new[:, 5] *= 1.0 + 0.08 * rng.uniform(-1, 1, o.nt)
    state = np.zeros(o.nt, np.int32)
    state[::7] = 2
    n_after = g.dig_feedback(old, new, state)
    o.dig_feedback(old, new, state)
    gs, os_ = g.state(), o.particles()
    assert n_after == len(os_["pid"])
    compare_particles(gs, os_, vel_fp32, ctx="feedback")
    _ir_close(gs, os_, "feedback")
    g.close()


def test_closure_and_accel_refused(D):
    wl = _n2_cavity(n_hex=3, ppc=5)
    g = D.Simulation(wl)
    g.step(3)
    with pytest.raises(D.DsmcError):
        g.dig_couple(accel=4)
    net = D.Mlp()
    with pytest.raises(D.DsmcError):
        g.set_closure(net)
    net.close()
    rep = g.dig_couple(n_m=5)
    assert not rep["failed"]
    g.close()
