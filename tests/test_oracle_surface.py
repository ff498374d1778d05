"""Surface sampling of the oracle (the wall pressure, shear stress and heat
flux compared on the sphere in section 5) pinned to:
  * one wall interaction traced by hand: the face hit and the sums it gets
    (velocity change and energy change of that particle, one hit), for a
    diffuse and a specular wall, and nothing outside the sampled steps;
  * the equilibrium closed box: every wall feels the pressure n k T and the
    number flux n sqrt(kT / (2 pi m)), with no shear and no net heat flux;
  * free-molecular Couette flow between diffuse plates moving at -U/2 and
    +U/2: shear stress m Phi U on each plate (Phi = n sqrt(kT / (2 pi m))),
    in the direction of the other plate's motion, pressure n k T;
  * free-molecular heat transfer between plates at T1 and T2: number flux
    Phi = n sqrt(2k / (pi m)) sqrt(T1 T2) / (sqrt T1 + sqrt T2) on both, heat
    flux 2 k Phi (T2 - T1) into the colder plate; specular side walls take
    only normal momentum and no energy;
  * the same plates with two rotational degrees of freedom: rotational heat
    flux Phi k (T2 - T1) into the colder plate (k (T2 - T1) per hit).
"""
import math

import numpy as np

from paper_2607_08195_amd import workloads as W
from oracle import Oracle
from statutil import KB, batch_stat


def _collisionless(wl):
    wl.species = W.Species(d_ref=1e-25)
    return wl


def _face_geometry(wl):
    """Area and unit normal out of the (convex box) domain of every boundary face."""
    xyz, bf = wl.mesh.xyz, wl.mesh.bfaces
    p, q, r = xyz[bf[:, 0]], xyz[bf[:, 1]], xyz[bf[:, 2]]
    n = np.cross(q - p, r - p)
    area = 0.5 * np.linalg.norm(n, axis=1)
    n = n / (2.0 * area[:, None])
    centre = 0.5 * (xyz.min(axis=0) + xyz.max(axis=0))
    out = np.sign(((p + q + r) / 3.0 - centre) * n).sum(axis=1)
    n *= np.where(out < 0, -1.0, 1.0)[:, None]
    return area, n


def _group_fields(wl, sums, nsteps, group):
    """Number flux, pressure, shear vector and heat flux over the faces of a
    boundary group (a plane): summed sums over the group's area and time."""
    area, n = _face_geometry(wl)
    sel = wl.mesh.bgroup == group
    S = sums[sel].sum(axis=0)
    A = area[sel].sum()
    nrm = n[sel][0]
    assert np.allclose(n[sel], nrm)
    m, FN = wl.species.mass, wl.run.F_N
    t = nsteps * wl.run.dt
    dn = S[:3] @ nrm
    return dict(flux=FN * S[4] / (A * t), p=m * FN * dn / (A * t),
                tau=m * FN * (S[:3] - dn * nrm) / (A * t), q=m * FN * S[3] / (A * t))


def _batches(o, wl, groups, nbatch, blen):
    out = []
    for _ in range(nbatch):
        o.surface_sampling(True)
        o.step(blen)
        sums, ns = o.surface()
        assert ns == blen
        out.append({g: _group_fields(wl, sums, ns, g) for g in groups})
    return out


def test_single_hits_by_hand():
    wl = W.cavity(n_hex=2, ppc=2, lid_speed=50.0, vel_fp32=0)
    wl.run.n_ss = 0
    o = Oracle(wl, fill=False)
    xyz, tets = wl.mesh.xyz, o.tets()
    cent = xyz[tets].mean(axis=1)
    c = int(np.argmax(cent[:, 1]))          # a tet under the lid y = 1
    x0 = cent[c].copy()
    vin = np.array([10.0, 300.0, -20.0])
    # just past the lid: the re-emitted particle cannot reach another wall
    t = 1.1 * (1.0 - x0[1]) / vin[1]
    o.surface_sampling(True)
    cc, x, v = o.trace_one(x0, vin, c, 7, 1, t)
    sums, _ = o.surface()
    hit = np.nonzero(sums[:, 4])[0]
    assert len(hit) == 1 and sums[hit[0], 4] == 1.0
    b = hit[0]
    assert wl.mesh.bgroup[b] == 3            # the lid group
    assert np.array_equal(sums[b, :3], vin - v)
    assert sums[b, 3] == 0.5 * ((vin @ vin) - (v @ v))
    assert np.count_nonzero(sums) == np.count_nonzero(sums[b])
    # step index 0 is not after n_ss = 0: nothing is added
    o.surface_sampling(True)
    o.trace_one(x0, vin, c, 7, 0, t)
    assert not o.surface()[0].any()
    # a specular wall: the velocity change is the reflection's, no energy
    wl = W.closed_box(n_hex=2, kind=W.BC_SPECULAR, ppc=2, vel_fp32=0)
    wl.run.n_ss = 0
    o = Oracle(wl, fill=False)
    cent = wl.mesh.xyz[o.tets()].mean(axis=1)
    c = int(np.argmax(cent[:, 0]))
    o.surface_sampling(True)
    vin = np.array([400.0, 30.0, 5.0])
    cc, x, v = o.trace_one(cent[c], vin, c, 3, 1, 1e-3)
    sums, _ = o.surface()
    b = np.nonzero(sums[:, 4])[0]
    assert len(b) == 1
    assert np.array_equal(sums[b[0], :3], vin - v)
    assert abs(sums[b[0], 0] - 800.0) < 1e-9 and abs(sums[b[0], 1]) < 1e-9 and abs(sums[b[0], 2]) < 1e-9
    assert abs(sums[b[0], 3]) < 1e-9 * (vin @ vin)


def test_equilibrium_box_pressure_and_flux():
    wl = W.closed_box(n_hex=4, kind=W.BC_DIFFUSE, Kn=1.0, ppc=20, vel_fp32=0)
    o = Oracle(wl)
    m, T = wl.species.mass, wl.run.T0
    n = o.np * wl.run.F_N / 1.0
    groups = list(range(6))
    res = _batches(o, wl, groups, 20, 10)
    p_exp = n * KB * T
    flux_exp = n * math.sqrt(KB * T / (2 * math.pi * m))
    cbar = math.sqrt(8 * KB * T / (math.pi * m))
    for g in groups:
        p, se = batch_stat([r[g]["p"] for r in res])
        assert abs(p - p_exp) < 3.5 * se + 0.005 * p_exp, (g, p, p_exp, se)
        f, sef = batch_stat([r[g]["flux"] for r in res])
        assert abs(f - flux_exp) < 3.5 * sef + 0.005 * flux_exp, (g, f, flux_exp)
        tau, set_ = batch_stat([r[g]["tau"] for r in res])
        assert (np.abs(tau) < 3.5 * set_ + 1e-3 * p_exp).all(), (g, tau, set_)
        q, seq = batch_stat([r[g]["q"] for r in res])
        assert abs(q) < 3.5 * seq + 1e-3 * p_exp * cbar, (g, q, seq)


def test_free_molecular_couette_shear():
    U, Tw = 200.0, 273.0
    wl = _collisionless(W.plates(n=(2, 8, 2), U=U, T1=Tw, T2=Tw, ppc=60, periodic=True))
    o = Oracle(wl)
    m = wl.species.mass
    o.step(150)
    n = o.np * wl.run.F_N / 1.0
    res = _batches(o, wl, [2, 3], 24, 40)
    phi = n * math.sqrt(KB * Tw / (2 * math.pi * m))
    tau_exp = m * phi * U
    # the lower plate (y = 0, moving -U/2) is dragged towards +x, the upper one towards -x
    for g, sign in ((2, 1.0), (3, -1.0)):
        tau, se = batch_stat([r[g]["tau"] for r in res])
        assert abs(tau[0] - sign * tau_exp) < 3.5 * se[0] + 0.01 * tau_exp, (g, tau, tau_exp, se)
        assert abs(tau[2]) < 3.5 * se[2] + 0.01 * tau_exp
        p, sep = batch_stat([r[g]["p"] for r in res])
        assert abs(p - n * KB * Tw) < 3.5 * sep + 0.01 * n * KB * Tw, (g, p)


def test_free_molecular_heat_transfer_between_plates():
    T1, T2 = 200.0, 400.0
    wl = _collisionless(W.plates(n=(2, 8, 2), T1=T1, T2=T2, ppc=60, periodic=False, vel_fp32=0))
    o = Oracle(wl)
    m = wl.species.mass
    o.step(150)
    n = o.np * wl.run.F_N / 1.0
    res = _batches(o, wl, [0, 1, 2, 3, 4, 5], 24, 40)
    phi = n * math.sqrt(2 * KB / (math.pi * m)) * math.sqrt(T1 * T2) / (math.sqrt(T1) + math.sqrt(T2))
    q_exp = 2 * KB * phi * (T2 - T1)
    for g, sign in ((2, 1.0), (3, -1.0)):
        f, sef = batch_stat([r[g]["flux"] for r in res])
        assert abs(f - phi) < 3.5 * sef + 0.01 * phi, (g, f, phi)
        q, seq = batch_stat([r[g]["q"] for r in res])
        assert abs(q - sign * q_exp) < 3.5 * seq + 0.01 * abs(q_exp), (g, q, q_exp, seq)
    # specular side walls (groups 0, 1, 4, 5): normal momentum only, no energy
    for g in (0, 1, 4, 5):
        for r in res:
            assert np.all(np.abs(r[g]["tau"]) <= 1e-9 * abs(r[g]["p"]))
            assert abs(r[g]["q"]) <= 1e-9 * abs(r[g]["p"]) * 1e3


def test_free_molecular_rotational_heat_transfer_between_plates():
    """A collisionless gas with two rotational degrees of freedom between
    diffuse plates at T1 and T2: a molecule reaching a plate last left the
    other one, so it brings a rotational energy of mean k T_other and
    leaves with mean k T_plate; the rotational heat flux into the colder
    plate is Phi k (T2 - T1), half the translational 2 k Phi (T2 - T1) (the
    total (2 + d_r/2) k Phi (T2 - T1) of free-molecular heat transfer in a
    diatomic gas), the opposite into the hotter one; per hit the rotational
    energy left is k (T2 - T1) on average; specular side walls take none."""
    T1, T2 = 200.0, 400.0
    wl = W.plates(n=(2, 8, 2), T1=T1, T2=T2, ppc=60, periodic=False, vel_fp32=0)
    wl.species = W.Species(d_ref=1e-25, dof_rot=2, z_rot=2.59)
    o = Oracle(wl)
    m = wl.species.mass
    o.step(150)
    n = o.np * wl.run.F_N / 1.0
    area, _ = _face_geometry(wl)
    phi = n * math.sqrt(2 * KB / (math.pi * m)) * math.sqrt(T1 * T2) / (math.sqrt(T1) + math.sqrt(T2))
    qr_exp = KB * phi * (T2 - T1)
    qr = {2: [], 3: []}
    per_hit = {2: [], 3: []}
    for _ in range(24):
        o.surface_sampling(True)
        o.step(40)
        sums, ns = o.surface()
        rs, nr = o.surface_rot()
        assert ns == nr == 40
        t = ns * wl.run.dt
        for g in (0, 1, 4, 5):
            assert np.all(rs[wl.mesh.bgroup == g] == 0.0)
        for g in (2, 3):
            sel = wl.mesh.bgroup == g
            qr[g].append(wl.run.F_N * rs[sel].sum() / (area[sel].sum() * t))
            per_hit[g].append(rs[sel].sum() / sums[sel, 4].sum())
    for g, sign in ((2, 1.0), (3, -1.0)):
        q, se = batch_stat(qr[g])
        assert abs(q - sign * qr_exp) < 3.5 * se + 0.01 * qr_exp, (g, q, qr_exp, se)
        h, seh = batch_stat(per_hit[g])
        assert abs(h - sign * KB * (T2 - T1)) < 3.5 * seh + 0.01 * KB * (T2 - T1), (g, h, seh)


# --------------------------------------------------------------------------
# free-molecular flow over the sphere
# --------------------------------------------------------------------------
def _facet_force(xyz, tri, n, m, T, U, Tw):
    """Expected force of a drifting Maxwellian (number density n, temperature
    T, drift U) on flat facets, each with its own side facing the gas,
    re-emitted diffusely at rest at Tw (free-molecular closed forms: incident
    number, normal and tangential momentum fluxes of a drifting Maxwellian
    through a plane, plus the normal momentum of the half-range Maxwellian
    leaving the wall)."""
    from scipy.special import erf
    p, q, r = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    nv = np.cross(q - p, r - p)
    A = 0.5 * np.linalg.norm(nv, axis=1)
    nv /= (2.0 * A)[:, None]
    c = (p + q + r) / 3.0
    nv *= np.where((nv * c).sum(axis=1) < 0, -1.0, 1.0)[:, None]   # out of the body (sphere at the origin)
    beta = math.sqrt(m / (2 * KB * T))
    Un = nv @ U
    sn = -beta * Un                                   # speed ratio towards the facet
    e = np.exp(-sn * sn)
    ef = 1.0 + erf(sn)
    phi = n / (2 * math.sqrt(math.pi) * beta) * (e + math.sqrt(math.pi) * sn * ef)
    pi_ = n * m / (2 * beta * beta) * (sn / math.sqrt(math.pi) * e + (0.5 + sn * sn) * ef)
    pr = m * phi * math.sqrt(math.pi * KB * Tw / (2 * m))
    Ut = U[None, :] - Un[:, None] * nv
    F = A[:, None] * (-(pi_ + pr)[:, None] * nv + m * phi[:, None] * Ut)
    return F.sum(axis=0)


def _sphere_cd(s, Tw, T):
    return ((2 * s * s + 1) / (math.sqrt(math.pi) * s ** 3) * math.exp(-s * s)
            + (4 * s ** 4 + 4 * s * s - 1) / (2 * s ** 4) * math.erf(s)
            + 2 * math.sqrt(math.pi) / (3 * s) * math.sqrt(Tw / T))


def test_facet_force_reference_reproduces_the_sphere_drag():
    """The facet closed forms, summed over a fine tessellation of the
    sphere, give the free-molecular sphere drag coefficient."""
    mesh = W.sphere_box_mesh(N=48, K=1, lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0))
    tri = mesh.bfaces[mesh.bgroup == 6]
    m, T, Tw, n = W.Species().mass, 200.0, 300.0, 1e19
    for u in (300.0, 866.0, 2634.66):
        U = np.array([u, 0.0, 0.0])
        F = _facet_force(mesh.xyz, tri, n, m, T, U, Tw)
        s = u / math.sqrt(2 * KB * T / m)
        D = _sphere_cd(s, Tw, T) * 0.5 * n * m * u * u * math.pi * 0.25
        assert abs(F[0] / D - 1) < 2e-3, (u, F[0] / D)
        assert abs(F[1]) < 1e-5 * D and abs(F[2]) < 1e-5 * D


def test_free_molecular_sphere_drag():
    """Collisionless freestream (speed ratio 3, inflow on all six box faces)
    over the faceted sphere: the sampled drag and side forces against the
    facet closed forms for the same polyhedron."""
    u, T, Tw = 866.0, 200.0, 300.0
    wl = _collisionless(W.sphere_flow(N=4, K=3, u=u, T=T, Tw=Tw, ppc=10, outflow=False, vel_fp32=0))
    o = Oracle(wl)
    m = wl.species.mass
    n = wl.info["n_inf"]
    sel = wl.mesh.bgroup == 6
    ref = _facet_force(wl.mesh.xyz, wl.mesh.bfaces[sel], n, m, T, np.array([u, 0.0, 0.0]), Tw)
    forces = []
    for _ in range(10):
        o.surface_sampling(True)
        o.step(20)
        sums, ns = o.surface()
        forces.append(m * wl.run.F_N * sums[sel, :3].sum(axis=0) / (ns * wl.run.dt))
    F, se = batch_stat(forces)
    assert abs(F[0] - ref[0]) < 3.5 * se[0] + 0.003 * ref[0], (F, ref, se)
    for k in (1, 2):
        assert abs(F[k]) < 3.5 * se[k] + 0.003 * ref[0], (F, se)
    # the drag of the polyhedron is within a few per cent of the sphere's
    s = u / math.sqrt(2 * KB * T / m)
    D = _sphere_cd(s, Tw, T) * 0.5 * n * m * u * u * math.pi * 0.25
    assert abs(ref[0] / D - 1) < 0.05


def test_cavity_surface_sums_conserve_energy_and_momentum():
    """A closed lid-driven cavity at steady state: the gas's energy and
    momentum do not change, so what all walls receive sums to zero (the lid
    does work on the gas that the other walls take back as heat; the lid's
    drag is balanced by the other walls), within the batch noise, while the
    individual walls carry clearly nonzero shares."""
    wl = W.cavity(n_hex=4, Kn=0.1, ppc=20, lid_speed=300.0, vel_fp32=0)
    o = Oracle(wl)
    o.step(300)
    m, FN, dt = wl.species.mass, wl.run.F_N, wl.run.dt
    tot_e, tot_p, lid_e, lid_px = [], [], [], []
    for _ in range(12):
        o.surface_sampling(True)
        o.step(25)
        sums, ns = o.surface()
        t = ns * dt
        tot_e.append(m * FN * sums[:, 3].sum() / t)
        tot_p.append(m * FN * sums[:, :3].sum(axis=0) / t)
        lid = wl.mesh.bgroup == 3
        lid_e.append(m * FN * sums[lid, 3].sum() / t)
        lid_px.append(m * FN * sums[lid, 0].sum() / t)
    E, seE = batch_stat(tot_e)
    P, seP = batch_stat(tot_p)
    LE, seLE = batch_stat(lid_e)
    LP, seLP = batch_stat(lid_px)
    # the lid gives energy to the gas and is dragged back (-x) by it
    assert LE < -5 * seLE and LP < -5 * seLP, (LE, seLE, LP, seLP)
    assert abs(E) < 3.5 * seE + 0.02 * abs(LE), (E, seE, LE)
    assert (np.abs(P) < 3.5 * seP + 0.02 * abs(LP)).all(), (P, seP, LP)
