"""Seeded synthetic inputs: tetrahedral meshes, boundary tables and run
parameters for the lid-driven cavity (paper section 5.1), the free-molecular
plate problems used as pins, and an open box with freestream inflow.

This module holds no part of the method's arithmetic: it only builds input
arrays (vertex coordinates, tet connectivity, boundary triangles and their
groups) and the scalar parameters a caller passes in.  Both the GPU path and
the CPU oracle consume its output.

Gas and reference scales follow the paper's statement of the problem: the
global Knudsen number of eq. (kn_definition_stability) with L0 the cavity
side, and the mean collision time tau = mu/p of section 2.1; the time step is
a fixed fraction of tau.
"""
from dataclasses import dataclass, field
import itertools
import math

import numpy as np

KB = 1.380649e-23

# boundary kinds (same numbering as the C interfaces)
BC_DIFFUSE, BC_SPECULAR, BC_INFLOW, BC_OUTFLOW, BC_PERIODIC = 0, 1, 2, 3, 4


@dataclass
class Species:
    mass: float = 6.63e-26      # argon
    d_ref: float = 4.17e-10
    omega: float = 0.81
    T_ref: float = 273.0
    alpha: float = 1.0          # 1 = VHS
    dof_rot: int = 0            # rotational degrees of freedom (0 or 2)
    z_rot: float = 0.0          # rotational collision number
    # heat-flux relaxation coefficients A_tt, A_tr, A_rt, A_rr of a rotating
    # gas (the conductivity matrix of section 2.2); nitrogen's
    a_heat: tuple = (0.786, -0.201, -0.059, 0.842)

    def mu(self, T):
        """VHS/VSS viscosity at temperature T (power law in T with index
        omega, coefficient from the reference diameter; VSS scattering scales
        it by (alpha+1)(alpha+2)/(6 alpha), Bird 1994)."""
        m, d, w, a = self.mass, self.d_ref, self.omega, self.alpha
        mu_ref = 15.0 * math.sqrt(math.pi * m * KB * self.T_ref) / (
            2.0 * math.pi * d * d * (5.0 - 2.0 * w) * (7.0 - 2.0 * w)) * ((a + 1.0) * (a + 2.0) / (6.0 * a))
        return mu_ref * (T / self.T_ref) ** w


@dataclass
class Boundary:
    kind: int
    T: float = 273.0
    u: tuple = (0.0, 0.0, 0.0)
    n: float = 0.0              # inflow number density
    shift: tuple = (0.0, 0.0, 0.0)  # periodic translation onto the partner face


@dataclass
class Mesh:
    xyz: np.ndarray             # [nv,3] float64
    tets: np.ndarray            # [nt,4] int32
    bfaces: np.ndarray          # [nb,3] int32
    bgroup: np.ndarray          # [nb] int32
    bpartner: np.ndarray = None  # [nb] int32 or None
    h: float = 0.0

    @property
    def n_tets(self):
        return int(self.tets.shape[0])


@dataclass
class Run:
    n0: float
    T0: float
    u0: tuple
    F_N: float
    dt: float
    seed: int = 0
    case_id: int = 0
    vel_fp32: int = 1
    n_ss: int = 0
    n_a: int = 1000
    ewma_on: int = 0


@dataclass
class Workload:
    name: str
    mesh: Mesh
    species: Species
    boundaries: list
    run: Run
    steps: int = 1
    info: dict = field(default_factory=dict)


# ---------------------------------------------------------------------------
# Kuhn-split box
# ---------------------------------------------------------------------------
def _kuhn_tets(nx, ny, nz):
    """Each hex cell split into 6 tets along the main diagonal: for each
    permutation of the axes, walk from the min corner to the max corner."""
    vid = lambda i, j, k: (i * (ny + 1) + j) * (nz + 1) + k
    I, J, K = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    out = []
    for perm in itertools.permutations(range(3)):
        pts = [np.zeros(3, dtype=np.int64)]
        for ax in perm:
            p = pts[-1].copy()
            p[ax] += 1
            pts.append(p)
        out.append(np.stack([vid(I + p[0], J + p[1], K + p[2]) for p in pts], axis=1))
    # order: hex-major, then permutation
    tets = np.stack(out, axis=1).reshape(-1, 4)
    return tets.astype(np.int32)


def _box_boundary(tets, xyz, lo, hi, tol):
    """Exterior triangles (faces used by one tet) and their side group:
    0 x-, 1 x+, 2 y-, 3 y+, 4 z-, 5 z+."""
    faces = np.concatenate([tets[:, [1, 2, 3]], tets[:, [0, 2, 3]],
                            tets[:, [0, 1, 3]], tets[:, [0, 1, 2]]])
    key = np.sort(faces, axis=1)
    _, inv, cnt = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    ext = faces[cnt[inv.ravel()] == 1]
    c = xyz[ext].mean(axis=1)
    grp = np.full(len(ext), -1, dtype=np.int32)
    for ax in range(3):
        grp[np.abs(c[:, ax] - lo[ax]) < tol] = 2 * ax
        grp[np.abs(c[:, ax] - hi[ax]) < tol] = 2 * ax + 1
    assert (grp >= 0).all()
    return ext.astype(np.int32), grp


def kuhn_box(nx, ny, nz, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), jitter=0.0, seed=0,
             periodic_axes=(), grade=0.0):
    """Box [lo,hi] meshed as nx*ny*nz hexes x 6 Kuhn tets.  ``jitter`` moves
    interior vertices by uniform +-jitter*h per coordinate, vertices on one
    box face only tangentially, and leaves edge and corner vertices fixed; a
    vertex is redrawn while any of its tets falls below 5% of the nominal
    volume.  ``periodic_axes`` pairs the faces on opposite sides of the
    listed axes (translation partners); jitter must then be 0.  ``grade`` =
    b > 0 clusters the vertices towards both faces of every axis, after the
    jitter: s -> (1 + tanh(b (2s - 1)) / tanh(b)) / 2 for the fraction s of
    the box (the spacing at a face shrinks by b (1 - tanh(b)^2) / tanh(b),
    0.29 for b = 1.5); ``h`` is then the smallest spacing."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    n = np.array([nx, ny, nz])
    hv = (hi - lo) / n
    gi = [np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1)]
    I, J, K = np.meshgrid(*gi, indexing="ij")
    idx = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)
    xyz = lo + idx * hv
    # exact end coordinates
    for ax in range(3):
        xyz[idx[:, ax] == n[ax], ax] = hi[ax]
    tets = _kuhn_tets(nx, ny, nz)
    h = float(hv.min())
    if jitter > 0:
        assert not periodic_axes
        rng = np.random.default_rng(seed)
        on_face = (idx == 0) | (idx == n)          # per-axis boundary flags
        nbnd = on_face.sum(axis=1)
        movable = nbnd <= 1
        vol0 = np.prod(hv) / 6.0

        def vols(x):
            a, b, c, d = (x[tets[:, i]] for i in range(4))
            return np.abs(np.einsum("ij,ij->i", b - a, np.cross(c - a, d - a))) / 6.0

        base = xyz.copy()
        disp = rng.uniform(-jitter, jitter, size=xyz.shape) * hv
        disp[on_face] = 0.0                          # no normal motion on a box face
        disp[~movable] = 0.0
        xyz = base + disp
        for _ in range(100):
            bad_t = np.nonzero(vols(xyz) < 0.05 * vol0)[0]
            if len(bad_t) == 0:
                break
            bad_v = np.unique(tets[bad_t].ravel())
            bad_v = bad_v[movable[bad_v]]
            d = rng.uniform(-jitter, jitter, size=(len(bad_v), 3)) * hv
            d[on_face[bad_v]] = 0.0
            xyz[bad_v] = base[bad_v] + d
        else:
            raise RuntimeError("jitter could not reach the minimum tet volume")
    if grade > 0:
        assert not periodic_axes
        frac = (xyz - lo) / (hi - lo)
        mapped = 0.5 * (1.0 + np.tanh(grade * (2.0 * frac - 1.0)) / np.tanh(grade))
        on_end = (idx == 0) | (idx == n)
        mapped[on_end] = frac[on_end]  # box faces stay where they are
        xyz = lo + mapped * (hi - lo)
        first = 0.5 * (1.0 + np.tanh(grade * (2.0 / n - 1.0)) / np.tanh(grade))
        h = float((first * (hi - lo)).min())
    bfaces, bgroup = _box_boundary(tets, xyz, lo, hi, 1e-9 * float((hi - lo).max()))
    partner = None
    if periodic_axes:
        partner = np.full(len(bfaces), -1, dtype=np.int32)
        for ax in periodic_axes:
            for side_lo, side_hi in [(2 * ax, 2 * ax + 1)]:
                a = np.nonzero(bgroup == side_lo)[0]
                b = np.nonzero(bgroup == side_hi)[0]
                # map each vertex on the hi side to its translate on the lo side
                ka = np.sort(_grid_keys(idx[bfaces[a]], ax, n), axis=1)
                kb = np.sort(_grid_keys(idx[bfaces[b]], ax, n, to_lo=True), axis=1)
                da = {tuple(r): i for r, i in zip(ka.tolist(), a.tolist())}
                for r, i in zip(kb.tolist(), b.tolist()):
                    j = da[tuple(r)]
                    partner[i] = j
                    partner[j] = i
        assert (partner[np.isin(bgroup, [2 * a for a in periodic_axes] +
                                [2 * a + 1 for a in periodic_axes])] >= 0).all()
    return Mesh(xyz=np.ascontiguousarray(xyz), tets=np.ascontiguousarray(tets),
                bfaces=np.ascontiguousarray(bfaces), bgroup=np.ascontiguousarray(bgroup),
                bpartner=partner, h=h)


def _grid_keys(ijk, ax, n, to_lo=False):
    """Integer key of each face vertex with the periodic axis coordinate
    dropped (so a face and its translate share keys)."""
    ijk = ijk.copy()
    if to_lo:
        ijk[..., ax] = 0
    other = [a for a in range(3) if a != ax]
    return ijk[..., other[0]] * (n[other[1]] + 1) + ijk[..., other[1]]


# ---------------------------------------------------------------------------
# Mixed-element box
# ---------------------------------------------------------------------------
@dataclass
class MixedMesh:
    """Mesh of tetrahedra, pyramids, prisms and hexahedra (vertex lists in
    the local orders of include/dsmc.h) with boundary triangles and
    quadrilaterals."""
    xyz: np.ndarray             # [nv,3]
    cells: list                 # vertex-index lists of 4, 5, 6 or 8
    bfaces: list                # vertex-index lists of 3 or 4 (cyclic)
    bgroup: np.ndarray          # [nb]
    kind: np.ndarray            # [n_cells] 4, 5, 6, 8
    h: float = 0.0


def _default_kinds(i, j, k, n):
    """Layer of prisms at the bottom (z), then hexahedra, pyramids and
    tetrahedra side by side in x."""
    nx, ny, nz = n
    if k < max(1, nz // 4):
        return "prism"
    if i < nx // 3:
        return "hex"
    if i < (2 * nx) // 3:
        return "pyr"
    return "tet"


def mixed_box(nx, ny, nz, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), jitter=0.0, seed=0, kinds=None):
    """Box [lo,hi] on an nx*ny*nz grid of hexahedral blocks, each block one
    hexahedron, two prisms (split by the vertical plane through its
    (i,j)-(i+1,j+1) diagonal), six pyramids around a vertex at its centre,
    or the six Kuhn tetrahedra, chosen by kinds(i, j, k, (nx, ny, nz)).
    Boundary faces are the cells' faces on the box sides, grouped 0 x-,
    1 x+, 2 y-, 3 y+, 4 z-, 5 z+.  ``jitter`` moves interior grid vertices
    by uniform +-jitter*h per coordinate (box-face vertices tangentially)."""
    kinds = kinds or _default_kinds
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    n = np.array([nx, ny, nz])
    hv = (hi - lo) / n
    vid = lambda i, j, k: (i * (ny + 1) + j) * (nz + 1) + k
    gi = [np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1)]
    I, J, K = np.meshgrid(*gi, indexing="ij")
    idx = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)
    xyz = lo + idx * hv
    for ax in range(3):
        xyz[idx[:, ax] == n[ax], ax] = hi[ax]
    if jitter > 0:
        rng = np.random.default_rng(seed)
        on_face = (idx == 0) | (idx == n)
        movable = on_face.sum(axis=1) <= 1
        disp = rng.uniform(-jitter, jitter, size=xyz.shape) * hv
        disp[on_face] = 0.0
        disp[~movable] = 0.0
        xyz = xyz + disp
    pts = [p for p in xyz]
    cells, kind = [], []
    tri_faces = []   # candidate boundary faces of every cell (vertex lists)

    def add(v, faces):
        cells.append(v)
        kind.append(len(v))
        tri_faces.extend(faces)

    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                c = [vid(i, j, k), vid(i + 1, j, k), vid(i + 1, j + 1, k), vid(i, j + 1, k),
                     vid(i, j, k + 1), vid(i + 1, j, k + 1), vid(i + 1, j + 1, k + 1), vid(i, j + 1, k + 1)]
                quads = [[c[0], c[1], c[2], c[3]], [c[4], c[5], c[6], c[7]], [c[0], c[1], c[5], c[4]],
                         [c[1], c[2], c[6], c[5]], [c[2], c[3], c[7], c[6]], [c[3], c[0], c[4], c[7]]]
                t = kinds(i, j, k, (nx, ny, nz))
                if t == "hex":
                    add(c, quads)
                elif t == "prism":
                    a = [c[0], c[1], c[2], c[4], c[5], c[6]]
                    b = [c[0], c[2], c[3], c[4], c[6], c[7]]
                    add(a, [[a[0], a[1], a[2]], [a[3], a[4], a[5]], [a[0], a[1], a[4], a[3]],
                            [a[1], a[2], a[5], a[4]]])
                    add(b, [[b[0], b[1], b[2]], [b[3], b[4], b[5]], [b[1], b[2], b[5], b[4]],
                            [b[2], b[0], b[3], b[5]]])
                elif t == "pyr":
                    ctr = len(pts)
                    pts.append(np.mean(xyz[c], axis=0))
                    for q in quads:
                        add(q + [ctr], [q])
                elif t == "tet":
                    base = np.array([i, j, k])
                    for perm in itertools.permutations(range(3)):
                        p = base.copy()
                        v = [vid(*p)]
                        for ax in perm:
                            p = p.copy()
                            p[ax] += 1
                            v.append(vid(*p))
                        add(v, [[v[1], v[2], v[3]], [v[0], v[2], v[3]], [v[0], v[1], v[3]], [v[0], v[1], v[2]]])
                else:
                    raise ValueError(t)
    P = np.array(pts)
    tol = 1e-9 * float((hi - lo).max())
    bfaces, bgroup, seen = [], [], set()
    for f in tri_faces:
        q = P[f]
        for ax in range(3):
            for side, val in ((0, lo[ax]), (1, hi[ax])):
                if np.all(np.abs(q[:, ax] - val) < tol):
                    key = tuple(sorted(f))
                    if key not in seen:
                        seen.add(key)
                        bfaces.append(list(f))
                        bgroup.append(2 * ax + side)
    return MixedMesh(xyz=np.ascontiguousarray(P), cells=cells, bfaces=bfaces,
                     bgroup=np.array(bgroup, dtype=np.int32), kind=np.array(kind, dtype=np.int32),
                     h=float(hv.min()))


# ---------------------------------------------------------------------------
# Reference scales
# ---------------------------------------------------------------------------
def n0_from_kn(sp: Species, Kn, T0, L0=1.0):
    """Number density for a global Knudsen number (eq. kn_definition_stability):
    Kn = mu0/(p0 L0) sqrt(pi R T0 / 2)."""
    R = KB / sp.mass
    p0 = sp.mu(T0) * math.sqrt(math.pi * R * T0 / 2.0) / (Kn * L0)
    return p0 / (KB * T0)


def tau_from_kn(sp: Species, Kn, T0, L0=1.0):
    """Mean collision time tau = mu/p (section 2.1) at the reference state."""
    R = KB / sp.mass
    return Kn * L0 / math.sqrt(math.pi * R * T0 / 2.0)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------
def cavity(n_hex=6, Kn=1.0, ppc=20, jitter=0.0, lid_speed=50.0, T0=273.0, seed=0,
           vel_fp32=1, steps=500, n_ss=200, mesh_seed=0, ewma_on=0, n_a=1000, species=None, grade=0.0):
    """3D lid-driven cavity on [0,1]^3: all walls diffuse at T0, the y=1 lid
    moving at lid_speed in +x.  Initial equilibrium at rest (section 5.1).
    The gas is VHS argon unless `species` is given; ``grade`` refines the
    mesh towards the walls (kuhn_box)."""
    sp = Species() if species is None else species
    mesh = kuhn_box(n_hex, n_hex, n_hex, jitter=jitter, seed=mesh_seed, grade=grade)
    name = (f"cavity_{n_hex}^3x6_Kn{Kn:g}" + ("" if sp.alpha == 1.0 else f"_vss{sp.alpha:g}") +
            ("" if not sp.dof_rot else f"_rot{sp.dof_rot}") + ("" if grade == 0 else f"_grade{grade:g}"))
    wl = cavity_on_mesh(mesh, Kn=Kn, ppc=ppc, lid_speed=lid_speed, T0=T0, seed=seed, vel_fp32=vel_fp32,
                        steps=steps, n_ss=n_ss, ewma_on=ewma_on, n_a=n_a, species=sp, name=name)
    wl.info.update(n_hex=n_hex, jitter=jitter, grade=grade)
    return wl


def cavity_on_mesh(mesh, Kn=1.0, ppc=20, lid_speed=50.0, T0=273.0, seed=0, vel_fp32=1, steps=500, n_ss=200,
                   ewma_on=0, n_a=1000, species=None, n_cells=None, name="cavity"):
    """The lid-driven cavity of `cavity` on a given tetrahedral mesh of the
    unit cube (boundary groups 0 x-, 1 x+, 2 y-, 3 y+ (the lid), 4 z-,
    5 z+), ppc particles per cell on average over n_cells cells (default:
    the tetrahedra)."""
    sp = Species() if species is None else species
    n0 = n0_from_kn(sp, Kn, T0)
    dt = 0.2 * tau_from_kn(sp, Kn, T0)
    F_N = n0 * 1.0 / (ppc * (mesh.n_tets if n_cells is None else n_cells))
    bcs = [Boundary(BC_DIFFUSE, T0)] * 6
    bcs = list(bcs)
    bcs[3] = Boundary(BC_DIFFUSE, T0, (lid_speed, 0.0, 0.0))
    run = Run(n0=n0, T0=T0, u0=(0.0, 0.0, 0.0), F_N=F_N, dt=dt, seed=seed, vel_fp32=vel_fp32,
              n_ss=n_ss, n_a=n_a, ewma_on=ewma_on)
    return Workload(name, mesh, sp, bcs, run, steps, dict(Kn=Kn, ppc=ppc, lid_speed=lid_speed))


def cavity_large_vss(steps=20000, n_ss=10000):
    """The 40^3 x 6 cavity of cavity_large with argon as a variable soft
    sphere (d_ref = 4.11e-10 m, alpha = 1.40 at T_ref = 273 K; the same
    viscosity as the VHS argon, so the same n0 and dt within 0.1 %)."""
    return cavity(n_hex=40, Kn=0.1, ppc=30, jitter=0.1, vel_fp32=1, steps=steps, n_ss=n_ss,
                  species=Species(d_ref=4.11e-10, alpha=1.40))


def cavity_small():
    """Lid-driven cavity, 6^3 hexes x 6 tets (1,296 tets), Kn=1, 20 particles
    per cell, FP64 velocities, 500 steps with the last 300 sampled."""
    return cavity(n_hex=6, Kn=1.0, ppc=20, vel_fp32=0, steps=500, n_ss=200)


def cavity_large(steps=20000, n_ss=10000):
    """Lid-driven cavity, 40^3 hexes x 6 tets (384,000 tets) with +-10%
    vertex jitter, Kn=0.1, 30 particles per cell (11.52M particles), FP32
    velocities, FP64 positions and moments."""
    return cavity(n_hex=40, Kn=0.1, ppc=30, jitter=0.1, vel_fp32=1, steps=steps, n_ss=n_ss)


def cavity_large_n2(steps=20000, n_ss=10000):
    """cavity_large with the paper's gas: nitrogen (VHS, omega = 0.74,
    d_ref = 4.17e-10 m, m = 4.65e-26 kg) with two rotational degrees of
    freedom exchanged by Borgnakke-Larsen at Z_r = 2.59 (section 5.1)."""
    sp = Species(mass=4.65e-26, d_ref=4.17e-10, omega=0.74, T_ref=273.0, alpha=1.0, dof_rot=2, z_rot=2.59)
    return cavity(n_hex=40, Kn=0.1, ppc=30, jitter=0.1, vel_fp32=1, steps=steps, n_ss=n_ss, species=sp)


def cavity_ensemble(n_cases=64, seed=0, n_min=6, n_max=24, ppc=20, vel_fp32=1, case_seed=0):
    """Independent lid-driven cavities for batched stepping: per case (seeded)
    Kn log-uniform in [0.01, 1], lid speed uniform in [20, 200] m/s and a
    mesh of n^3 hexes x 6 tets with n uniform in [n_min, n_max]; case k has
    generator key (seed, k)."""
    rng = np.random.default_rng(case_seed)
    out = []
    for k in range(n_cases):
        Kn = float(10.0 ** rng.uniform(-2.0, 0.0))
        lid = float(rng.uniform(20.0, 200.0))
        n = int(rng.integers(n_min, n_max + 1))
        wl = cavity(n_hex=n, Kn=Kn, ppc=ppc, lid_speed=lid, seed=seed, vel_fp32=vel_fp32)
        wl.run.case_id = k
        wl.name = f"case{k}_" + wl.name
        out.append(wl)
    return out


def closed_box(n_hex=4, kind=BC_SPECULAR, Kn=1.0, ppc=20, T0=273.0, vel_fp32=0, seed=0,
               Tw=None):
    """Closed unit box at rest with all six walls of one kind."""
    sp = Species()
    mesh = kuhn_box(n_hex, n_hex, n_hex)
    n0 = n0_from_kn(sp, Kn, T0)
    dt = 0.2 * tau_from_kn(sp, Kn, T0)
    F_N = n0 / (ppc * mesh.n_tets)
    bcs = [Boundary(kind, T0 if Tw is None else Tw)] * 6
    run = Run(n0=n0, T0=T0, u0=(0.0, 0.0, 0.0), F_N=F_N, dt=dt, seed=seed, vel_fp32=vel_fp32)
    return Workload("closed_box", mesh, sp, list(bcs), run, 1)


def plates(n=(4, 8, 4), H=1.0, U=0.0, T1=273.0, T2=273.0, n0=1e18, ppc=20, dt=None,
           seed=0, periodic=True, vel_fp32=0):
    """Two diffuse plates at y=0 (T1, moving -U/2 in x) and y=H (T2, +U/2),
    periodic (or specular) in x and z.  Collisionless limit via a negligible
    cross-section is the caller's choice of species."""
    sp = Species()
    mesh = kuhn_box(*n, hi=(1.0, H, 1.0), periodic_axes=(0, 2) if periodic else ())
    F_N = n0 * H / (ppc * mesh.n_tets)
    side = BC_PERIODIC if periodic else BC_SPECULAR
    bcs = [Boundary(side, 0.0, shift=(1.0, 0.0, 0.0)), Boundary(side, 0.0, shift=(-1.0, 0.0, 0.0)),
           Boundary(BC_DIFFUSE, T1, (-U / 2, 0.0, 0.0)), Boundary(BC_DIFFUSE, T2, (U / 2, 0.0, 0.0)),
           Boundary(side, 0.0, shift=(0.0, 0.0, 1.0)), Boundary(side, 0.0, shift=(0.0, 0.0, -1.0))]
    T0 = 0.5 * (T1 + T2)
    if dt is None:
        dt = 0.25 * (H / n[1]) / math.sqrt(2 * KB * T0 / sp.mass)
    run = Run(n0=n0, T0=T0, u0=(0.0, 0.0, 0.0), F_N=F_N, dt=dt, seed=seed, vel_fp32=vel_fp32)
    return Workload("plates", mesh, sp, bcs, run, 1)


def open_box(n=(6, 4, 4), lo=(-2.0, -2.0, -2.0), hi=(4.0, 2.0, 2.0), T=200.0, u=2634.66,
             Kn=0.05, ppc=10, seed=0, vel_fp32=1, dt=None):
    """Box with freestream inflow on five faces (x-, y-, y+, z-, z+) and a
    vacuum outflow at x+, filled with the freestream; cross-section
    parameters are those of argon, Kn referred to a 1 m length."""
    sp = Species()
    mesh = kuhn_box(*n, lo=lo, hi=hi)
    n_inf = n0_from_kn(sp, Kn, T)
    vol = float(np.prod(np.asarray(hi) - np.asarray(lo)))
    F_N = n_inf * vol / (ppc * mesh.n_tets)
    if dt is None:
        dt = 0.2 * mesh.h / u
    inflow = Boundary(BC_INFLOW, T, (u, 0.0, 0.0), n=n_inf)
    bcs = [inflow, Boundary(BC_OUTFLOW, T), inflow, inflow, inflow, inflow]
    run = Run(n0=n_inf, T0=T, u0=(u, 0.0, 0.0), F_N=F_N, dt=dt, seed=seed, vel_fp32=vel_fp32)
    return Workload("open_box", mesh, sp, bcs, run, 1, dict(n_inf=n_inf, u=u, T=T))


# ---------------------------------------------------------------------------
# Sphere in a box
# ---------------------------------------------------------------------------
_HEX_QUADS = ((0, 1, 2, 3), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7))


def _split_quads(q):
    """Each quad (cyclic vertex ids) as two triangles along the diagonal
    through its lowest-id vertex (the same diagonal from either side)."""
    lo = np.argmin(q, axis=1)
    ac = (lo == 0) | (lo == 2)
    t1 = np.where(ac[:, None], q[:, [0, 1, 2]], q[:, [0, 1, 3]])
    t2 = np.where(ac[:, None], q[:, [0, 2, 3]], q[:, [1, 2, 3]])
    return t1, t2


def sphere_box_mesh(N=4, K=3, a=1.0, R=0.5, lo=(-2.0, -2.0, -2.0), hi=(4.0, 2.0, 2.0), grade=5.0):
    """Box [lo,hi] minus the sphere of radius R at the origin.  A cube
    [-a,a]^3 around the sphere carries a cubed-sphere O-grid (N x N cells on
    each cube face, K layers from the sphere to the cube, layer thickness
    growing geometrically by `grade` from the wall outwards); the rest of
    the box is Cartesian with the cube's spacing h = 2a/N (lo, hi on that
    lattice).  Every hex is split into 12 tets around its centroid, each quad
    face into two triangles along the diagonal through its lowest-id vertex
    (conforming between neighbours).  Boundary groups: 0 x-, 1 x+, 2 y-,
    3 y+, 4 z-, 5 z+, 6 sphere."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    h = 2.0 * a / N
    n = np.rint((hi - lo) / h).astype(int)
    assert np.allclose(lo + n * h, hi) and np.allclose(np.rint((-a - lo) / h), (-a - lo) / h)
    c0 = np.rint((-a - lo) / h).astype(int)          # lattice index of the cube's low corner
    c1 = c0 + N
    # lattice vertices outside the open cube
    I, J, Kk = np.meshgrid(np.arange(n[0] + 1), np.arange(n[1] + 1), np.arange(n[2] + 1), indexing="ij")
    lat = np.stack([I.ravel(), J.ravel(), Kk.ravel()], axis=1)
    inside = np.all((lat > c0) & (lat < c1), axis=1)
    lid = np.full(len(lat), -1, dtype=np.int64)
    keep = np.nonzero(~inside)[0]
    lid[keep] = np.arange(len(keep))
    xyz = [lo + lat[keep] * h]
    nv = len(keep)

    def lat_id(ijk):
        ijk = np.asarray(ijk)
        return lid[(ijk[..., 0] * (n[1] + 1) + ijk[..., 1]) * (n[2] + 1) + ijk[..., 2]]

    # cube-surface lattice points and their O-grid layers 0..K-1 (layer K is the point itself)
    on_cube = np.all((lat >= c0) & (lat <= c1), axis=1) & ~inside
    cube_pts = lat[on_cube]
    cube_index = np.full(len(lat), -1, dtype=np.int64)
    cube_index[np.nonzero(on_cube)[0]] = np.arange(len(cube_pts))
    P = lo + cube_pts * h
    d = P / np.linalg.norm(P, axis=1, keepdims=True)
    S = R * d
    r = grade ** (1.0 / max(K - 1, 1))
    dl = r ** np.arange(K)
    g = np.concatenate([[0.0], np.cumsum(dl) / dl.sum()])
    layers = np.stack([S + g[k] * (P - S) for k in range(K)], axis=1)   # [ncube, K, 3]
    xyz.append(layers.reshape(-1, 3))
    layer_base = nv
    nv += len(cube_pts) * K

    def oid(ijk, k):
        ci = cube_index[(ijk[..., 0] * (n[1] + 1) + ijk[..., 1]) * (n[2] + 1) + ijk[..., 2]]
        return np.where(k == K, lat_id(ijk), layer_base + ci * K + k)

    hexes = []
    # Cartesian cells outside the cube
    ci, cj, ck = np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]), indexing="ij")
    cells = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=1)
    cells = cells[~np.all((cells >= c0) & (cells < c1), axis=1)]
    corner = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0], [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]])
    hexes.append(np.stack([lat_id(cells + corner[v]) for v in range(8)], axis=1))
    # O-grid cells: on each cube face, N x N cells and K layers
    u, v = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    u, v = u.ravel(), v.ravel()
    for ax in range(3):
        a1, a2 = (ax + 1) % 3, (ax + 2) % 3
        for side in (c0[ax], c1[ax]):
            base = np.zeros((len(u), 3), dtype=np.int64)
            base[:, ax] = side
            base[:, a1] = c0[a1] + u
            base[:, a2] = c0[a2] + v
            e1 = np.zeros(3, dtype=np.int64); e1[a1] = 1
            e2 = np.zeros(3, dtype=np.int64); e2[a2] = 1
            quad = [base, base + e1, base + e1 + e2, base + e2]
            for k in range(K):
                hexes.append(np.stack([oid(q, np.full(len(u), k)) for q in quad] +
                                      [oid(q, np.full(len(u), k + 1)) for q in quad], axis=1))
    H = np.concatenate(hexes).astype(np.int64)
    assert (H >= 0).all()
    xyz = np.concatenate(xyz)
    cen = xyz[H].mean(axis=1)
    cid = nv + np.arange(len(H))
    xyz = np.concatenate([xyz, cen])
    tets = []
    for qd in _HEX_QUADS:
        t1, t2 = _split_quads(H[:, qd])
        tets.append(np.concatenate([cid[:, None], t1], axis=1))
        tets.append(np.concatenate([cid[:, None], t2], axis=1))
    tets = np.stack(tets, axis=1).reshape(-1, 4)
    # boundary triangles: the box's outer quads and the sphere's quads
    bq, bg = [], []
    for ax in range(3):
        a1, a2 = (ax + 1) % 3, (ax + 2) % 3
        p, q = np.meshgrid(np.arange(n[a1]), np.arange(n[a2]), indexing="ij")
        p, q = p.ravel(), q.ravel()
        for s_, side in enumerate((0, n[ax])):
            base = np.zeros((len(p), 3), dtype=np.int64)
            base[:, ax] = side
            base[:, a1] = p
            base[:, a2] = q
            e1 = np.zeros(3, dtype=np.int64); e1[a1] = 1
            e2 = np.zeros(3, dtype=np.int64); e2[a2] = 1
            bq.append(np.stack([lat_id(base), lat_id(base + e1), lat_id(base + e1 + e2), lat_id(base + e2)], axis=1))
            bg.append(np.full(len(p), 2 * ax + s_))
        for side in (c0[ax], c1[ax]):
            base = np.zeros((len(u), 3), dtype=np.int64)
            base[:, ax] = side
            base[:, a1] = c0[a1] + u
            base[:, a2] = c0[a2] + v
            e1 = np.zeros(3, dtype=np.int64); e1[a1] = 1
            e2 = np.zeros(3, dtype=np.int64); e2[a2] = 1
            z = np.zeros(len(u), dtype=np.int64)
            bq.append(np.stack([oid(base, z), oid(base + e1, z), oid(base + e1 + e2, z), oid(base + e2, z)], axis=1))
            bg.append(np.full(len(u), 6))
    BQ = np.concatenate(bq)
    BG = np.concatenate(bg)
    t1, t2 = _split_quads(BQ)
    bfaces = np.concatenate([t1, t2]).astype(np.int32)
    bgroup = np.concatenate([BG, BG]).astype(np.int32)
    return Mesh(xyz=np.ascontiguousarray(xyz), tets=np.ascontiguousarray(tets.astype(np.int32)),
                bfaces=np.ascontiguousarray(bfaces), bgroup=np.ascontiguousarray(bgroup), bpartner=None, h=h)


def sphere_flow(N=4, K=3, grade=5.0, T=200.0, u=2634.66, Kn=0.05, Tw=500.0, ppc=10, n_particles=None,
                seed=0, vel_fp32=1, dt=None, outflow=True, lo=(-2.0, -2.0, -2.0), hi=(4.0, 2.0, 2.0)):
    """Hypersonic flow over a sphere of diameter 1 m (Kn referred to the
    diameter) in the box [lo,hi]: freestream (T, u along +x) through the five
    faces other than x+, vacuum outflow at x+ (with outflow=False, inflow
    there too), diffuse sphere at Tw; filled with the freestream.  F_N gives
    ppc particles per tet on average, or n_particles in all."""
    sp = Species()
    mesh = sphere_box_mesh(N=N, K=K, grade=grade, lo=lo, hi=hi)
    n_inf = n0_from_kn(sp, Kn, T)
    vol = float(np.prod(np.asarray(hi) - np.asarray(lo))) - math.pi / 6.0
    total = n_particles if n_particles is not None else ppc * mesh.n_tets
    F_N = n_inf * vol / total
    if dt is None:
        dt = 0.2 * mesh.h / u
    inflow = Boundary(BC_INFLOW, T, (u, 0.0, 0.0), n=n_inf)
    bcs = [inflow, Boundary(BC_OUTFLOW, T) if outflow else inflow, inflow, inflow, inflow, inflow,
           Boundary(BC_DIFFUSE, Tw)]
    run = Run(n0=n_inf, T0=T, u0=(u, 0.0, 0.0), F_N=F_N, dt=dt, seed=seed, vel_fp32=vel_fp32)
    return Workload(f"sphere_N{N}K{K}", mesh, sp, bcs, run, 1,
                    dict(n_inf=n_inf, u=u, T=T, Tw=Tw, R=0.5, Kn=Kn))
