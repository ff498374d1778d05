"""Pins of the MLP-closure oracle (FP64 forward, backward, Adam).

* forward: a small network evaluated in 50-digit scalar arithmetic (mpmath)
  unit by unit, and SiLU / sigmoid at tabulated points;
* backward: central finite differences of the FP64 loss for every
  parameter of a reduced network and a sample of the full 13-128-128-128-9
  network (1e-6 relative);
* Adam: the first step moves every parameter by lr g/(|g| + eps), the
  closed form of the bias-corrected moments after one step;
* bfloat16 rounding: exact values (ties to even) and the bound 2^-8;
* training a teacher-generated target drops the loss by an order of
  magnitude (an end-to-end check of the sign conventions);
* closure scaling and gate by hand.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import mlp_oracle as M


def _rand_params(layers, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    ps = []
    for i, o in zip(layers[:-1], layers[1:]):
        ps.append(rng.uniform(-1, 1, (i, o)).ravel() * scale / math.sqrt(i))
        ps.append(rng.uniform(-0.2, 0.2, o))
    return np.concatenate(ps)


def test_param_count():
    assert M.n_params() == 35977


def test_silu_tabulated():
    # sigmoid(1) = 1/(1+e^-1) = 0.7310585786300049, sigmoid(2) = 0.8807970779778823
    assert M.silu(np.array(1.0)) == pytest.approx(0.7310585786300049, rel=1e-15)
    assert M.silu(np.array(-1.0)) == pytest.approx(-0.2689414213699951, rel=1e-15)
    assert M.silu(np.array(2.0)) == pytest.approx(2 * 0.8807970779778823, rel=1e-15)
    assert M.silu_grad(np.array(0.0)) == 0.5
    # derivative against a central difference at a few points
    z = np.array([-3.0, -0.7, 0.2, 1.5, 4.0])
    h = 1e-6
    fd = (M.silu(z + h) - M.silu(z - h)) / (2 * h)
    assert np.allclose(M.silu_grad(z), fd, rtol=1e-8, atol=1e-10)


def test_forward_against_high_precision_scalar_evaluation():
    layers = (3, 4, 5, 2)
    p = _rand_params(layers, 1)
    x = np.random.default_rng(2).standard_normal((4, 3))
    y, _ = M.forward(p, x, layers=layers)
    mp.mp.dps = 50
    params = M.unpack(p, layers)
    for r in range(x.shape[0]):
        h = [mp.mpf(float(v)) for v in x[r]]
        for l, (W, b) in enumerate(params):
            z = []
            for o in range(W.shape[1]):
                acc = mp.mpf(float(b[o]))
                for i in range(W.shape[0]):
                    acc += h[i] * mp.mpf(float(W[i, o]))
                z.append(acc)
            h = [zz / (1 + mp.exp(-zz)) for zz in z] if l < len(params) - 1 else z
        for o in range(2):
            assert abs(float(h[o]) - y[r, o]) <= 1e-14 * max(1.0, abs(float(h[o])))


def _fd_check(layers, p, x, t, idx, h=1e-6):
    _, g = M.loss_and_grad(p, x, t, layers=layers)
    for k in idx:
        pp = p.copy(); pp[k] += h
        pm = p.copy(); pm[k] -= h
        lp = M.loss_and_grad(pp, x, t, layers=layers)[0]
        lm = M.loss_and_grad(pm, x, t, layers=layers)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), (k, fd, g[k])


def test_backward_against_finite_differences_small():
    layers = (5, 7, 6, 4, 3)
    p = _rand_params(layers, 3)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((6, 5))
    t = rng.standard_normal((6, 3))
    _fd_check(layers, p, x, t, range(M.n_params(layers)))


def test_backward_against_finite_differences_full_sample():
    p = _rand_params(M.LAYERS, 5)
    rng = np.random.default_rng(6)
    x = rng.standard_normal((5, 13))
    t = 0.1 * rng.standard_normal((5, 9))
    n = M.n_params()
    idx = np.unique(np.concatenate([rng.integers(0, n, 300), [0, 1663, 1664, 1791, n - 10, n - 1]]))
    _fd_check(M.LAYERS, p, x, t, idx)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(7)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    g[3] = 0.0
    p1, m, v = M.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    assert np.allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert p1[3] == p[3]
    # the bias corrections of step 2 with a constant gradient keep the step at lr
    p2, _, _ = M.adam_step(p1, g, m, v, 2, lr=1e-3)
    assert np.allclose(p2 - p1, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-15)


def test_bf16_rounding():
    v = np.array([1.0, 1 + 2**-8, 1 + 3 * 2**-8, math.pi, -2.5, 0.0, 1e-40, 65280.0, 1 + 2**-7])
    r = M.bf16_round(v)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1 + 2**-6
    assert r[3] == 3.140625 and r[4] == -2.5 and r[5] == 0.0 and r[7] == 65280.0 and r[8] == 1 + 2**-7
    x = np.random.default_rng(8).standard_normal(10000) * 10
    assert np.all(np.abs(M.bf16_round(x) - x) <= 2**-8 * np.abs(x))


def test_training_reduces_a_teacher_loss():
    rng = np.random.default_rng(9)
    teacher = _rand_params(M.LAYERS, 10, scale=1.5)
    x = rng.standard_normal((512, 13))
    t, _ = M.forward(teacher, x)
    p = _rand_params(M.LAYERS, 11)
    batches = [rng.integers(0, 512, 64) for _ in range(300)]
    _, losses = M.train(p, x, t, batches, lr=3e-3)
    assert np.mean(losses[-20:]) < 0.1 * np.mean(losses[:5])


def test_bf16_contract_close_to_fp64():
    p = _rand_params(M.LAYERS, 12)
    rng = np.random.default_rng(13)
    x = rng.standard_normal((64, 13))
    t = rng.standard_normal((64, 9))
    y64, _ = M.forward(p, x)
    y16, _ = M.forward(p, x, bf16=True)
    assert np.linalg.norm(y16 - y64) <= 2e-2 * np.linalg.norm(y64)
    _, g64 = M.loss_and_grad(p, x, t)
    _, g16 = M.loss_and_grad(p, x, t, bf16=True)
    assert np.linalg.norm(g16 - g64) <= 3e-2 * np.linalg.norm(g64)


def test_closure_scaling_and_gate_by_hand():
    R = 208.0
    T = np.array([300.0])
    gu = np.arange(9, dtype=float)[None, :] * 100.0
    gT = np.array([[10.0, -20.0, 30.0]])
    lam = np.array([1e-3])
    x = M.closure_inputs(gu, gT, T, np.array([0.5]), lam, R)
    cs = math.sqrt(R * 300.0)
    assert x[0, 1] == pytest.approx(1e-3 * 100.0 / cs)
    assert x[0, 10] == pytest.approx(1e-3 * -20.0 / 300.0)
    assert x[0, 12] == 0.5
    hot = np.array([[1.0, 2, 3, 4, 5, 6, 7, 8, 9]])
    y = M.closure_targets(hot, np.array([2.0]), T, R)
    p = 2.0 * R * 300.0
    assert y[0, 5] == pytest.approx(6 / p) and y[0, 8] == pytest.approx(9 / (p * cs))
    use, e = M.gate(np.array([[0.0] * 9, [1.0] * 9]), np.array([[0.0] * 9, [1.0] * 8 + [1.5]]),
                    np.array([[0.0] * 9, [3.0] + [0.0] * 8]), tol=0.2)
    assert use.tolist() == [True, True] and e[1] == pytest.approx(0.5 / 3.0)
    use, _ = M.gate(np.array([[np.nan] * 9]), np.zeros((1, 9)), np.ones((1, 9)), tol=0.2)
    assert not use[0]
    # the sampling noise widens the denominator: 14.5 / n added to |s|^2
    use, e = M.gate(np.array([[1.0] + [0.0] * 8]), np.zeros((1, 9)), np.array([[0.3, 0.4] + [0.0] * 7]), tol=1.0,
                    n_samples=np.array([14.5 / 0.75]))
    assert e[0] == pytest.approx(1.0) and use[0]


def test_gate_noise_constant_is_the_sampling_variance_of_a_maxwellian():
    """The gate's noise model: the nondimensional stress and heat flux
    (eq. dsmc_temperatures, over p and p sqrt(RT)) estimated from n
    particles of a Maxwellian at rest have zero mean and E|.|^2 = 14.5 / n
    to leading order (Gaussian moments: normal stresses 4/3, shear
    stresses 1, heat fluxes 5/2 each)."""
    from statutil import fields_from_sums
    rng = np.random.default_rng(12)
    n, reps = 400, 3000
    m, kT = 6.63e-26, 1.380649e-23 * 273.0
    cs = math.sqrt(kT / m)
    tot = 0.0
    for _ in range(reps):
        v = rng.standard_normal((n, 3)) * cs
        S = np.concatenate([[n], v.sum(0), (v * v).sum(0), [(v[:, 0] * v[:, 1]).sum(), (v[:, 0] * v[:, 2]).sum(),
                            (v[:, 1] * v[:, 2]).sum()], (v * (v * v).sum(1, keepdims=True)).sum(0)])
        f = fields_from_sums(S, m, 1.0, 1.0, 1)
        p = f["n"] * 1.380649e-23 * f["T"]
        sig = f["sig"][[0, 1, 2, 0, 0, 1], [0, 1, 2, 1, 2, 2]] / p
        q = f["q"] / (p * math.sqrt(1.380649e-23 * f["T"] / m))
        tot += (sig ** 2).sum() + (q ** 2).sum()
    est = tot / reps * n
    assert abs(est / M.NOISE_PER_PARTICLE - 1) < 0.05, est
