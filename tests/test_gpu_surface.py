"""Surface sampling through the C ABI against the oracle, from one state:
diffuse walls with a moving lid (parked-wall move schedule and the
per-particle one), specular walls, diffuse plates with periodic sides, and a
batch of cavities.  Hit counts per face exact; velocity- and energy-change
sums within 1e-12 of the column's largest magnitude (the device adds them
with atomics, in hit order); the sampled step count equal; the library's
fields (number flux, pressure, shear, heat flux) equal to the same formulas
evaluated on the oracle's sums within 1e-10.  With nitrogen, the rotational
energy each face receives and its rotational heat flux as well."""
import numpy as np
import pytest

from paper_2607_08195_amd import workloads as W
from oracle import Oracle
from parity_util import compare_particles

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_08195_amd import dsmc
    return dsmc


def _fields(wl, sums, ns):
    """Per-face fields from sums, as include/dsmc.h defines them."""
    xyz, bf = wl.mesh.xyz, wl.mesh.bfaces
    p, q, r = xyz[bf[:, 0]], xyz[bf[:, 1]], xyz[bf[:, 2]]
    n = np.cross(q - p, r - p)
    area = 0.5 * np.linalg.norm(n, axis=1)
    n = n / (2.0 * area[:, None])
    # out of the gas: away from the fourth vertex of the tet on the face
    tets = wl.mesh.tets
    opp = {}
    for t in range(len(tets)):
        for f in range(4):
            opp[tuple(sorted(np.delete(tets[t], f)))] = tets[t][f]
    far = xyz[[opp[tuple(sorted(b))] for b in bf]]
    n *= np.where(((far - p) * n).sum(axis=1) > 0, -1.0, 1.0)[:, None]
    m, FN = wl.species.mass, wl.run.F_N
    ta = area * ns * wl.run.dt
    dn = (sums[:, :3] * n).sum(axis=1)
    out = np.zeros((len(bf), 6))
    out[:, 0] = FN * sums[:, 4] / ta
    out[:, 1] = m * FN * dn / ta
    out[:, 2:5] = m * FN * (sums[:, :3] - dn[:, None] * n) / ta[:, None]
    out[:, 5] = m * FN * sums[:, 3] / ta
    return out


def _compare(gs, gf, gn, os_, on, wl, ctx):
    assert gn == on, ctx
    assert np.array_equal(gs[:, 4], os_[:, 4]), f"{ctx}: hit counts"
    assert os_[:, 4].sum() > 0, ctx
    scale = np.abs(os_).max(axis=0) + 1e-300
    assert np.all(np.abs(gs - os_) <= 1e-12 * scale), f"{ctx}: sums"
    fo = _fields(wl, os_, on)
    fs = np.abs(fo).max(axis=0) + 1e-300
    assert np.all(np.abs(gf - fo) <= 1e-10 * fs), f"{ctx}: fields"


CASES = {
    "cavity_lid_fp64": lambda: W.cavity(n_hex=5, Kn=0.5, ppc=20, vel_fp32=0, lid_speed=200.0),
    "cavity_lid_fp32_jitter": lambda: W.cavity(n_hex=6, Kn=0.1, ppc=20, jitter=0.1, vel_fp32=1, lid_speed=100.0),
    "specular_box": lambda: W.closed_box(n_hex=5, kind=W.BC_SPECULAR, ppc=15, vel_fp32=1),
    "plates_couette": lambda: W.plates(n=(3, 6, 3), U=300.0, T1=250.0, T2=350.0, ppc=25, n0=3e19, vel_fp32=0),
    "sphere_hypersonic": lambda: W.sphere_flow(N=4, K=3, ppc=8, vel_fp32=1),
}


@pytest.mark.parametrize("move", [None, 0])
@pytest.mark.parametrize("case", list(CASES))
def test_surface_sums_match_oracle(D, case, move):
    wl = CASES[case]()
    pre = 3
    wl.run.n_ss = pre + 1
    o = Oracle(wl)
    o.step(pre)
    st = o.particles()
    g = D.Simulation(wl, fill=False, capacity=max(4 * o.np, 100000))
    g.set_state(st["x"], st["v"], st["cell"], st["pid"], o.step_index, o.next_pid, o.smax())
    if move is not None:
        t = g.tuning()
        g.set_tuning(move, t["collide"], t["sort"])
    o.surface_sampling(True)
    g.surface_sampling(True)
    # the first step is not sampled (step index = n_ss), the next four are
    o.step(5)
    g.step(5)
    compare_particles(g.state(), o.particles(), wl.run.vel_fp32, ctx=case)
    gs, gf, gn = g.surface()
    os_, on = o.surface()
    assert on == 4
    _compare(gs, gf, gn, os_, on, wl, case)
    # stopped: further steps add nothing and the window is kept
    o.surface_sampling(False)
    g.surface_sampling(False)
    o.step(2)
    g.step(2)
    gs2, _, gn2 = g.surface()
    assert gn2 == gn and np.array_equal(gs2, gs)
    g.close()


@pytest.mark.parametrize("case", ["cavity_lid_fp64", "plates_couette", "sphere_hypersonic"])
def test_rotational_surface_sums_match_oracle(D, case):
    """Nitrogen (two rotational degrees of freedom): the rotational energy
    each face receives within 1e-12 of the largest magnitude, the
    translational sums and hit counts as above, and the rotational heat
    flux equal to F_N sum / (A t)."""
    wl = CASES[case]()
    wl.species = W.Species(mass=4.65e-26, d_ref=4.17e-10, omega=0.74, T_ref=273.0, alpha=1.0, dof_rot=2,
                           z_rot=2.59)
    pre = 3
    wl.run.n_ss = pre + 1
    o = Oracle(wl)
    o.step(pre)
    st = o.particles()
    g = D.Simulation(wl, fill=False, capacity=max(4 * o.np, 100000))
    g.set_state(st["x"], st["v"], st["cell"], st["pid"], o.step_index, o.next_pid, o.smax(), ir=st["ir"])
    o.surface_sampling(True)
    g.surface_sampling(True)
    o.step(5)
    g.step(5)
    gs, gf, gn = g.surface()
    os_, on = o.surface()
    _compare(gs, gf, gn, os_, on, wl, case)
    gr, qr, nr = g.surface_rot()
    orr, onr = o.surface_rot()
    assert nr == onr == on == 4
    assert np.abs(orr).max() > 0, case
    assert np.all(np.abs(gr - orr) <= 1e-12 * np.abs(orr).max()), f"{case}: rotational sums"
    xyz, bf = wl.mesh.xyz, wl.mesh.bfaces
    area = 0.5 * np.linalg.norm(np.cross(xyz[bf[:, 1]] - xyz[bf[:, 0]], xyz[bf[:, 2]] - xyz[bf[:, 0]]), axis=1)
    q_o = wl.run.F_N * orr / (area * on * wl.run.dt)
    assert np.all(np.abs(qr - q_o) <= 1e-10 * np.abs(q_o).max()), f"{case}: rotational heat flux"
    g.close()
    # a monatomic gas has no rotational surface sums
    a = D.Simulation(W.cavity(n_hex=2, Kn=0.5, ppc=5))
    with pytest.raises(D.DsmcError):
        a.surface_rot()
    a.close()


def test_surface_graph_steps_and_restart(D):
    """Graph-replayed steps sample the same sums as ordinary steps, and a
    graph captured with sampling off is not reused once it is on."""
    import torch
    wl = CASES["cavity_lid_fp32_jitter"]()
    wl.run.n_ss = 0
    a = D.Simulation(wl, stream=torch.cuda.Stream())
    b = D.Simulation(wl, stream=torch.cuda.Stream())
    a.graph_step(2)
    b.step(2)
    a.surface_sampling(True)
    b.surface_sampling(True)
    a.graph_step(4)
    b.step(4)
    sa, fa, na = a.surface()
    sb, fb, nb = b.surface()
    assert na == nb == 4
    assert np.array_equal(sa[:, 4], sb[:, 4]) and sa[:, 4].sum() > 0
    scale = np.abs(sb).max(axis=0) + 1e-300
    assert np.all(np.abs(sa - sb) <= 1e-12 * scale)
    # restarting clears the sums
    a.surface_sampling(True)
    s0, _, n0 = a.surface()
    assert n0 == 0 and not s0.any()
    a.close()
    b.close()


@pytest.mark.parametrize("gas", ["argon", "nitrogen"])
def test_surface_batch_matches_oracle_per_case(D, gas):
    """Three cavities of different size, Kn and lid speed in one batch: each
    case's slice of the surface sums against its own oracle run; with
    nitrogen also its rotational sums (within 1e-12 of the case's largest)
    and rotational heat flux (F_N of the case)."""
    specs = [(3, 0.05, 150.0), (4, 0.5, 30.0), (2, 1.0, 80.0)]
    cases = []
    for k, (n, Kn, lid) in enumerate(specs):
        wl = W.cavity(n_hex=n, Kn=Kn, ppc=12, lid_speed=lid, seed=7, vel_fp32=1)
        if gas == "nitrogen":
            wl.species = W.Species(mass=4.65e-26, d_ref=4.17e-10, omega=0.74, T_ref=273.0, alpha=1.0, dof_rot=2,
                                   z_rot=2.59)
        wl.run.case_id = 20 + k
        wl.run.n_ss = 0
        cases.append(wl)
    g = D.Simulation(cases)
    oracles = [Oracle(wl) for wl in cases]
    g.surface_sampling(True)
    for o in oracles:
        o.surface_sampling(True)
    g.step(3)
    for o in oracles:
        o.step(3)
    gs, gf, gn = g.surface()
    if gas == "nitrogen":
        gr, gq, gnr = g.surface_rot()
        assert gnr == gn
    b0 = 0
    for k, (o, wl) in enumerate(zip(oracles, cases)):
        os_, on = o.surface()
        nb = len(wl.mesh.bfaces)
        _compare(gs[b0:b0 + nb], gf[b0:b0 + nb], gn, os_, on, wl, f"case {k}")
        if gas == "nitrogen":
            orr, onr = o.surface_rot()
            assert onr == on and np.abs(orr).max() > 0
            r = gr[b0:b0 + nb]
            assert np.all(np.abs(r - orr) <= 1e-12 * np.abs(orr).max()), f"case {k}: rotational sums"
            xyz, bf = wl.mesh.xyz, wl.mesh.bfaces
            area = 0.5 * np.linalg.norm(np.cross(xyz[bf[:, 1]] - xyz[bf[:, 0]], xyz[bf[:, 2]] - xyz[bf[:, 0]]),
                                        axis=1)
            q_o = wl.run.F_N * orr / (area * on * wl.run.dt)
            assert np.all(np.abs(gq[b0:b0 + nb] - q_o) <= 1e-10 * np.abs(q_o).max()), f"case {k}: flux"
        b0 += nb
    assert b0 == len(gs)
    g.close()


def test_surface_off_by_default(D):
    """Without surface sampling switched on the sums stay empty: zero sums,
    zero fields and no sampled steps, also after steps."""
    wl = W.cavity(n_hex=3, Kn=0.5, ppc=10, vel_fp32=1)
    wl.run.n_ss = 0
    g = D.Simulation(wl)
    g.step(3)
    s, f, n = g.surface()
    assert n == 0 and not s.any() and not f.any()
    g.surface_sampling(False)          # stopping while off is allowed and changes nothing
    g.step(1)
    s, f, n = g.surface()
    assert n == 0 and not s.any()
    g.close()
