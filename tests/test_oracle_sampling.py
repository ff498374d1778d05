"""Pins of the oracle's sampling: cell fields of eq. (dsmc_temperatures)
against a direct two-pass central-moment computation on hand-built particle
sets; the exponential moving average (eq. exponential_average_moments_ch3)
and the steady average (eq. steady_average_moments_ch3) against their
closed forms."""
import numpy as np
import pytest

from paper_2607_08195_amd import workloads as W
from oracle import Oracle, STAGE_SORT, STAGE_SAMPLE

KB = 1.380649e-23


def _one_cell_sim(n_a=1000, ewma=0, n_ss=0):
    wl = W.closed_box(n_hex=1, kind=W.BC_SPECULAR, vel_fp32=0)
    wl.run.n_ss = n_ss
    wl.run.n_a = n_a
    wl.run.ewma_on = ewma
    return wl, Oracle(wl, fill=False)


def _centroid(wl, o, c):
    return wl.mesh.xyz[o.tets()[c]].mean(axis=0)


def _direct_fields(v, m, FN, V):
    N = len(v)
    u = v.mean(axis=0)
    c = v - u
    c2 = (c * c).sum(axis=1)
    rho = m * FN * N / V
    T = m * c2.mean() / (3 * KB)
    P = np.einsum("pi,pj->ij", c, c) / N
    sig = rho * (P - np.eye(3) * c2.mean() / 3)
    q = rho / 2 * (c * c2[:, None]).mean(axis=0)
    return rho, u, T, sig, q


@pytest.mark.parametrize("case", ["two", "symmetric", "random"])
def test_fields_match_direct_central_moments(case):
    wl, o = _one_cell_sim()
    rng = np.random.default_rng(11)
    if case == "two":
        v = np.array([[300.0, -20.0, 5.0], [-100.0, 40.0, 15.0]])
    elif case == "symmetric":
        base = rng.normal(size=(5, 3)) * 200
        v = np.concatenate([base, -base]) + np.array([30.0, -10.0, 5.0])
    else:
        v = rng.normal(size=(37, 3)) * 250 + np.array([50.0, 0.0, -20.0])
    n = len(v)
    x = np.tile(_centroid(wl, o, 0), (n, 1))
    o.set_particles(x, v, np.zeros(n, np.int32), np.arange(n, dtype=np.uint32), 0, n)
    o.step_stages(STAGE_SORT | STAGE_SAMPLE)
    f = o.fields(0)[0]
    rho, u, T, sig, q = _direct_fields(v, wl.species.mass, wl.run.F_N, o.volumes()[0])
    assert np.isclose(f[1], rho, rtol=1e-14)
    assert np.allclose(f[2:5], u, rtol=1e-12, atol=1e-12 * np.abs(v).max())
    assert np.isclose(f[5], T, rtol=1e-12)
    sig6 = [sig[0, 0], sig[1, 1], sig[2, 2], sig[0, 1], sig[0, 2], sig[1, 2]]
    scale_s = rho * (v * v).sum(axis=1).mean()
    assert np.allclose(f[6:12], sig6, rtol=0, atol=1e-12 * scale_s)
    scale_q = rho * (np.abs(v) ** 3).sum(axis=1).mean()
    assert np.allclose(f[12:15], q, rtol=0, atol=1e-12 * scale_q)
    # the symmetric set about its mean has zero heat flux
    if case == "symmetric":
        assert np.abs(f[12:15]).max() <= 1e-12 * scale_q


def test_empty_cell_fields_are_nan():
    wl, o = _one_cell_sim()
    x = np.tile(_centroid(wl, o, 0), (3, 1))
    o.set_particles(x, np.ones((3, 3)), np.zeros(3, np.int32), np.arange(3, dtype=np.uint32), 0, 3)
    o.step_stages(STAGE_SORT | STAGE_SAMPLE)
    f = o.fields(0)
    assert not np.isnan(f[0]).any()
    assert np.isnan(f[1:]).all()


def _set_velocity(o, wl, v):
    n = len(v)
    x = np.tile(_centroid(wl, o, 0), (n, 1))
    o.set_particles(x, v, np.zeros(n, np.int32), np.arange(n, dtype=np.uint32), o.step_index, n)


def test_ewma_constant_then_unit_step():
    n_a = 10
    wl, o = _one_cell_sim(n_a=n_a, ewma=1)
    A = np.array([[100.0, 0, 0], [-50.0, 0, 0]])
    B = np.array([[300.0, 10, 0], [-20.0, 0, 0], [5.0, 5, 5]])
    _set_velocity(o, wl, A)
    SA = None
    for m in range(1, 31):
        o.step_stages(STAGE_SORT | STAGE_SAMPLE)
        e = o.sums(1)[0]
        inst = o.sums(2)[0]
        if SA is None:
            SA = inst.copy()
        assert np.allclose(e, SA, rtol=1e-14)   # constant input stays constant
    _set_velocity(o, wl, B)
    for j in range(1, 40):
        o.step_stages(STAGE_SORT | STAGE_SAMPLE)
        SB = o.sums(2)[0]
        e = o.sums(1)[0]
        exp = SB + (SA - SB) * (1 - 1 / n_a) ** j
        assert np.allclose(e, exp, rtol=1e-12, atol=1e-12 * np.abs(SB).max())


def test_ewma_warmup_is_running_mean_and_local_accumulation_uncapped():
    n_a = 4
    wl, o = _one_cell_sim(n_a=n_a, ewma=1)
    rng = np.random.default_rng(2)
    hist = []
    for m in range(1, 13):
        _set_velocity(o, wl, rng.normal(size=(6, 3)) * 100)
        o.step_stages(STAGE_SORT | STAGE_SAMPLE)
        hist.append(o.sums(2)[0])
        e = o.sums(1)[0]
        if m <= n_a:
            assert np.allclose(e, np.mean(hist, axis=0), rtol=1e-13, atol=1e-9)
    # switch the cell to local accumulation: the average becomes cumulative
    o.set_local_acc(np.ones(o.nt, np.uint8))
    prev = o.sums(1)[0]
    mcount = 12
    for m in range(3):
        _set_velocity(o, wl, rng.normal(size=(6, 3)) * 100)
        o.step_stages(STAGE_SORT | STAGE_SAMPLE)
        mcount += 1
        S = o.sums(2)[0]
        exp = prev * (mcount - 1) / mcount + S / mcount
        assert np.allclose(o.sums(1)[0], exp, rtol=1e-13, atol=1e-9)
        prev = exp


def test_steady_average_is_arithmetic_mean_after_nss():
    n_ss = 5
    wl, o = _one_cell_sim(n_ss=n_ss)
    rng = np.random.default_rng(4)
    kept = []
    for m in range(1, 16):
        _set_velocity(o, wl, rng.normal(size=(5, 3)) * 100)
        o.step_stages(STAGE_SORT | STAGE_SAMPLE)
        if m > n_ss:
            kept.append(o.sums(2)[0])
    assert o.n_steady == 15 - n_ss
    assert np.allclose(o.sums(0)[0], np.sum(kept, axis=0), rtol=1e-14)
