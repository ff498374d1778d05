"""Physics pins of the oracle (whole loop against closed forms):
Maxwellian invariance of a closed box, the diffuse re-emission moments,
free-molecular Couette stress and heat flux between diffuse plates, and a
freestream box with inflow/outflow staying uniform."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_2607_08195_amd import workloads as W
from oracle import Oracle
from statutil import KB, batch_stat, fields_from_sums


def test_maxwellian_invariance_closed_diffuse_box():
    wl = W.closed_box(n_hex=6, kind=W.BC_DIFFUSE, ppc=20, vel_fp32=1)
    o = Oracle(wl)
    m, T0 = wl.species.mass, wl.run.T0
    sig = math.sqrt(KB * T0 / m)
    for snap in range(3):
        o.step(40)
        v = o.particles()["v"]
        n = len(v)
        assert abs(n - 25920) == 0
        mean = v.mean(axis=0)
        assert (np.abs(mean) < 3.5 * sig / math.sqrt(n)).all()
        T = m * (v * v).sum(axis=1).mean() / (3 * KB)
        # var of v^2 sum = 6 sig^4 per particle
        assert abs(T - T0) < 3.5 * T0 * math.sqrt(6.0 / (9 * n))
        kurt = stats.kurtosis(v, axis=0, fisher=False)
        assert (np.abs(kurt - 3.0) < 3.5 * math.sqrt(24.0 / n)).all()
        speed = np.linalg.norm(v, axis=1) / sig
        edges = np.linspace(0, 4.5, 19)
        cdf = stats.chi(3).cdf(edges)
        exp = np.diff(np.concatenate([cdf, [1.0]])) * n
        obs = np.histogram(speed, np.concatenate([edges, [np.inf]]))[0]
        chi2 = ((obs - exp) ** 2 / exp).sum()
        assert stats.chi2.sf(chi2, len(exp) - 1) > 1e-3


def test_diffuse_reemission_moments():
    wl = W.cavity(n_hex=2, ppc=2, lid_speed=50.0)
    o = Oracle(wl, fill=False)
    m, Tw = wl.species.mass, 273.0
    xyz, tets = wl.mesh.xyz, o.tets()
    # a tet touching the lid y=1
    cent = xyz[tets].mean(axis=1)
    c = int(np.argmax(cent[:, 1]))
    x0 = cent[c].copy()
    x0[1] = 1.0 - 1e-7
    # make sure x0 is inside c
    N = 20000
    vs = np.zeros((N, 3))
    for k in range(N):
        cc, x, v = o.trace_one(x0, [0.0, 300.0, 0.0], c, k, 1, 1e-9)
        vs[k] = v
    vn = -vs[:, 1]                      # inward normal is -y
    assert (vn > 0).all()
    sd = math.sqrt(KB * Tw / m)
    exp_vn = math.sqrt(math.pi * KB * Tw / (2 * m))
    sd_vn = math.sqrt(2 * KB * Tw / m - exp_vn ** 2)
    assert abs(vn.mean() - exp_vn) < 3.5 * sd_vn / math.sqrt(N)
    assert abs(vs[:, 0].mean() - 50.0) < 3.5 * sd / math.sqrt(N)
    assert abs(vs[:, 2].mean()) < 3.5 * sd / math.sqrt(N)
    for comp in (0, 2):
        var = vs[:, comp].var()
        assert abs(var / sd ** 2 - 1) < 3.5 * math.sqrt(2.0 / N)


def _collisionless(wl):
    wl.species = W.Species(d_ref=1e-25)
    return wl


def _run_batches(o, wl, transient, nbatch, blen):
    o.step(transient)
    V = o.volumes().sum()
    out = []
    for b in range(nbatch):
        S = np.zeros(13)
        for _ in range(blen):
            o.step(1)
            S += o.sums(2).sum(axis=0)
        out.append(fields_from_sums(S, wl.species.mass, wl.run.F_N, V, blen))
    return out


@pytest.mark.slow
def test_free_molecular_heat_flux_between_plates():
    T1, T2 = 200.0, 400.0
    wl = _collisionless(W.plates(n=(2, 8, 2), T1=T1, T2=T2, ppc=60, periodic=False))
    o = Oracle(wl)
    m = wl.species.mass
    res = _run_batches(o, wl, 150, 24, 40)
    n = np.mean([r["n"] for r in res])
    qy, se = batch_stat([r["q"][1] for r in res])
    exp = 2 * KB * (T1 - T2) * n * math.sqrt(2 * KB / (math.pi * m)) * \
        math.sqrt(T1 * T2) / (math.sqrt(T1) + math.sqrt(T2))
    assert abs(qy - exp) < 3.5 * se + 0.01 * abs(exp), (qy, exp, se)
    ux, seu = batch_stat([r["u"] for r in res])
    assert (np.abs(ux) < 3.5 * seu + 1.0).all()


@pytest.mark.slow
def test_free_molecular_couette_stress():
    U, Tw = 200.0, 273.0
    wl = _collisionless(W.plates(n=(2, 8, 2), U=U, T1=Tw, T2=Tw, ppc=60, periodic=True))
    o = Oracle(wl)
    m = wl.species.mass
    res = _run_batches(o, wl, 150, 24, 40)
    rho = np.mean([r["rho"] for r in res])
    sxy, se = batch_stat([r["sig"][0, 1] for r in res])
    exp = -rho * U * math.sqrt(KB * Tw / (2 * math.pi * m))
    assert abs(sxy - exp) < 3.5 * se + 0.01 * abs(exp), (sxy, exp, se)
    T, seT = batch_stat([r["T"] for r in res])
    heat = m * U * U / (12 * KB)
    expT = Tw + heat
    # particles with |v_y| below H/t have not met a plate yet and still carry
    # the initial temperature: allow 10% of the viscous-heating term for them
    assert abs(T - expT) < 3.5 * seT + 0.1 * heat, (T, expT, seT)
    q, seq = batch_stat([r["q"] for r in res])
    assert abs(q[1]) < 3.5 * seq[1] + 1e-3 * abs(exp) * U
    # periodic motion keeps every particle
    assert o.counters()["lost"] == 0 and o.counters()["removed"] == 0


@pytest.mark.slow
@pytest.mark.parametrize("collide", [False, True])
def test_freestream_box_stays_uniform(collide):
    wl = W.open_box(n=(6, 4, 4), ppc=12, vel_fp32=1)
    if not collide:
        wl = _collisionless(wl)
    o = Oracle(wl)
    info = wl.info
    m = wl.species.mass
    # injected count per step against the closed-form inflow flux
    sp = wl.species
    beta = math.sqrt(2 * KB * info["T"] / m)
    areas = {0: 16.0, 2: 24.0, 3: 24.0, 4: 24.0, 5: 24.0}
    mean_per_step = 0.0
    for g, A in areas.items():
        s = (info["u"] if g == 0 else 0.0) / beta
        flux = info["n_inf"] * math.sqrt(KB * info["T"] / (2 * math.pi * m)) * \
            (math.exp(-s * s) + math.sqrt(math.pi) * s * (1 + math.erf(s)))
        mean_per_step += flux * A * wl.run.dt / wl.run.F_N
    inj0 = o.counters()["injected"]
    res = _run_batches(o, wl, 40, 8, 10)
    inj = o.counters()["injected"] - inj0
    nstep = 120
    exp_inj = mean_per_step * nstep
    assert abs(inj - exp_inj) < 3.5 * math.sqrt(exp_inj)
    n, sen = batch_stat([r["n"] for r in res])
    assert abs(n / info["n_inf"] - 1) < 3.5 * sen / info["n_inf"] + 0.01
    ux = np.mean([r["u"][0] for r in res])
    assert abs(ux / info["u"] - 1) < 0.01
    T = np.mean([r["T"] for r in res])
    assert abs(T / info["T"] - 1) < 0.02
