"""What the learned closure gains over the sampled higher-order terms.

The network is trained on the fields the method itself samples: cavity runs
at several Knudsen numbers and lid speeds, each averaged over many steps so
that its HoT (sampled stress and heat flux minus NSF, per cell) is a
low-noise target.  On a held-out run (another Kn, lid speed and seed), the
HoT a coupling step would use after a short window of 100 steps is compared
with the same run's long-average HoT:
  * sampled: the short window's own HoT (what the method uses without the
    network);
  * learned: the network evaluated on the short window's gradients and Kn.
The test requires the learned closure to be closer to the long average than
the short-window sample (in the nondimensional units of the closure, rms
over cells), and prints both errors.  With the network attached to the
coupling step, its noise-aware gate (the network is taken where it lies
within three sampling-noise widths of the window's own HoT) selects the
network in a sizeable fraction of the cells, and the HoT the coupling step
then uses is closer to the long average than the window's sampled HoT.
"""
import numpy as np
import pytest

from paper_2607_08195_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_08195_amd import dsmc
    return dsmc


def _closure_pair(D, sim, sums):
    """Closure inputs/targets of one coupling evaluated on the given sums."""
    sim.set_sums(D.SAMPLE_EWMA, sums)
    sim.dig_couple(kn_max=1e9, passes=0, n_m=0, feedback=0)
    return sim.closure_data()


def _run(D, Kn, lid, seed, warm, long_steps, short_steps=100, n_hex=8, ppc=20, keep=False):
    wl = W.cavity(n_hex=n_hex, Kn=Kn, ppc=ppc, lid_speed=lid, seed=seed, vel_fp32=1, ewma_on=1,
                  n_a=short_steps, n_ss=warm)
    sim = D.Simulation(wl)
    sim.step(warm)
    # short window: the moving average over the last short_steps steps
    sim.step(short_steps)
    ewma, _ = sim.sums(D.SAMPLE_EWMA)
    sim.step(long_steps)
    acc, ns = sim.sums(D.SAMPLE_STEADY)
    x_s, t_s, v_s = _closure_pair(D, sim, ewma)
    x_l, t_l, v_l = _closure_pair(D, sim, acc / ns)
    if keep:
        return x_s, t_s, v_s & v_l, x_l, t_l, (sim, wl, ewma)
    sim.close()
    return x_s, t_s, v_s & v_l, x_l, t_l


def test_learned_closure_beats_short_window_samples(D):
    train_x, train_t = [], []
    for k, (Kn, lid) in enumerate([(0.05, 150.0), (0.1, 120.0), (0.07, 200.0), (0.15, 180.0), (0.05, 90.0)]):
        _, _, v, x_l, t_l = _run(D, Kn, lid, seed=k, warm=3000, long_steps=20000)
        train_x.append(x_l[v])
        train_t.append(t_l[v])
    x = np.concatenate(train_x)
    t = np.concatenate(train_t)
    scale = np.sqrt(np.mean(t ** 2, axis=0))
    net = D.Mlp()
    net.init_weights(seed=3)
    rep = net.train(x, t, steps=3000, batch=1024, lr=2e-3, seed=5)
    assert rep["loss_last"] < rep["loss_first"]
    # held-out run
    x_s, t_s, v, x_l, t_l, (sim, wl, ewma) = _run(D, 0.08, 140.0, seed=99, warm=3000, long_steps=20000, keep=True)
    y = net.forward(x_s[v])
    err_learned = np.sqrt(np.mean(((y - t_l[v]) / scale) ** 2))
    err_sampled = np.sqrt(np.mean(((t_s[v] - t_l[v]) / scale) ** 2))
    print(f"\nclosure vs long-average HoT (rms, per-component scaled): learned {err_learned:.4f}, "
          f"short-window sampled {err_sampled:.4f}, gain {err_sampled / err_learned:.2f}x; "
          f"train {x.shape[0]} cells, loss {rep['loss_first']:.3e} -> {rep['loss_last']:.3e}")
    assert err_learned < err_sampled
    # the gated closure inside the coupling step, on the short window
    from oracle import mlp_oracle as M
    sim.set_sums(D.SAMPLE_EWMA, ewma)
    sim.set_closure(net, gate_tol=3.0)
    r = sim.dig_couple(kn_max=1e9, passes=0, n_m=0, feedback=0)
    half = sim.dig_get("half")
    R = 1.380649e-23 / wl.species.mass
    t_g = M.closure_targets(sim.dig_get("hot"), half[:, 0], half[:, 4], R)
    err_gated = np.sqrt(np.mean(((t_g[v] - t_l[v]) / scale) ** 2))
    frac = r["n_closure"] / max(1, r["n_closure"] + r["n_fallback"])
    print(f"gated closure: network in {r['n_closure']} of {r['n_closure'] + r['n_fallback']} cells "
          f"({frac:.1%}), rms error {err_gated:.4f} against sampled {err_sampled:.4f}")
    assert frac > 0.2
    assert err_gated < err_sampled
    sim.set_closure(None)
    sim.close()
    net.close()
