"""Mixed-element meshes (section 5.4: tetrahedral, pyramid, prism and
hexahedral cells) on the CPU: the library's decomposition
(dsmc_mesh_decompose, host code) against the oracle's own, and the oracle's
decomposition pinned by what the geometry fixes.

* Both decompositions give the same vertices (bitwise), tetrahedra, cell
  map, boundary triangles, groups and parents, on a jittered mesh of all
  four cell types.
* Volumes: on the regular grid a hexahedron's tetrahedra add up to h^3, a
  prism's to h^3/2, a pyramid's to h^3/6 (closed forms of the cells); on the
  jittered mesh they add up to the box.
* The tetrahedra tile each cell: points drawn uniformly in a regular hex
  block fall in exactly one tetrahedron of the cell(s) of that block
  (brute-force barycentric location).
* Conformity: every interior triangle belongs to exactly two tetrahedra and
  the exterior triangles are exactly the boundary triangles.
* The quadrilateral rule on hand examples; error paths of the library.
* A gas at rest in a closed diffuse box on the mixed mesh stays uniform:
  cell densities and temperatures of the original cells (sums of their
  tetrahedra) within sampling noise of n0 and T0.
"""
import numpy as np
import pytest

from paper_2607_08195_amd import workloads as W
import oracle.mixed as OM

KB = 1.380649e-23


@pytest.fixture(scope="module")
def D():
    from paper_2607_08195_amd import dsmc
    return dsmc


def _vol(xyz, tets):
    a, b, c, d = (xyz[tets[:, k]] for k in range(4))
    return np.einsum("ij,ij->i", b - a, np.cross(c - a, d - a)) / 6.0


@pytest.mark.parametrize("jitter", [0.0, 0.12])
def test_library_decomposition_equals_oracle(D, jitter):
    m = W.mixed_box(5, 4, 6, jitter=jitter, seed=3)
    g = D.decompose(m.xyz, m.cells, m.bfaces, m.bgroup)
    o = OM.decompose(m.xyz, m.cells, m.bfaces, m.bgroup)
    for k, a in zip(["xyz", "tets", "tet_cell", "bfaces", "bgroup", "bpartner", "bparent"], o):
        assert g[k].shape == a.shape and np.array_equal(g[k], a), k


def test_counts_and_cell_volumes_regular_grid():
    n, h = 6, 1.0 / 6
    m = W.mixed_box(n, n, n)
    xyz, tets, tc, bf, bg, bp, bpar = OM.decompose(m.xyz, m.cells, m.bfaces, m.bgroup)
    kinds = m.kind
    per = {4: 1, 5: 2, 6: 8, 8: 12}
    assert len(tets) == sum(per[k] for k in kinds)
    assert len(xyz) == len(m.xyz) + int(np.sum((kinds == 6) | (kinds == 8)))
    assert set(np.unique(kinds)) == {4, 5, 6, 8}
    v = np.abs(_vol(xyz, tets))
    assert v.min() > 0
    cv = np.bincount(tc, weights=v, minlength=len(m.cells))
    exact = {8: h ** 3, 6: h ** 3 / 2, 5: h ** 3 / 6, 4: h ** 3 / 6}
    for k, e in exact.items():
        sel = kinds == k
        assert np.allclose(cv[sel], e, rtol=1e-12, atol=0), k
    assert abs(cv.sum() - 1.0) < 1e-12


def test_jittered_volumes_and_conformity():
    m = W.mixed_box(6, 5, 4, jitter=0.15, seed=1)
    xyz, tets, tc, bf, bg, bp, bpar = OM.decompose(m.xyz, m.cells, m.bfaces, m.bgroup)
    v = _vol(xyz, tets)
    assert np.all(np.abs(v) > 0)
    assert abs(np.abs(v).sum() - 1.0) < 1e-12
    faces = np.concatenate([tets[:, [1, 2, 3]], tets[:, [0, 2, 3]], tets[:, [0, 1, 3]], tets[:, [0, 1, 2]]])
    key = np.sort(faces, axis=1)
    uniq, cnt = np.unique(key, axis=0, return_counts=True)
    assert cnt.max() == 2
    ext = {tuple(r) for r in uniq[cnt == 1].tolist()}
    bnd = {tuple(r) for r in np.sort(bf, axis=1).tolist()}
    assert ext == bnd
    # each original boundary face is covered by its triangles: quads by two
    nv = np.array([len(f) for f in m.bfaces])
    assert np.array_equal(np.bincount(bpar, minlength=len(m.bfaces)), np.where(nv == 4, 2, 1))
    assert np.array_equal(bg, m.bgroup[bpar])


def test_tetrahedra_tile_their_cells():
    n = 4
    m = W.mixed_box(n, n, n)
    xyz, tets, tc, bf, bg, bp, bpar = OM.decompose(m.xyz, m.cells, m.bfaces, m.bgroup)
    rng = np.random.default_rng(0)
    # cells of each block: the block of a cell is where its vertex mean lies
    cells_cen = np.array([m.xyz[c].mean(axis=0) if len(c) != 5 else
                          m.xyz[c[:4]].mean(axis=0) * 0.5 + xyz[c[4]] * 0.5 for c in m.cells])
    block_of_cell = np.floor(cells_cen * n).astype(int)
    A = xyz[tets[:, 0]]
    M = np.stack([xyz[tets[:, k]] - A for k in (1, 2, 3)], axis=2)   # [nt,3,3]
    Minv = np.linalg.inv(M)
    for _ in range(300):
        p = rng.uniform(0.0, 1.0, 3)
        lam = np.einsum("tij,tj->ti", Minv, p[None, :] - A)
        inside = np.all(lam >= -1e-12, axis=1) & (lam.sum(axis=1) <= 1 + 1e-12)
        hits = np.nonzero(inside)[0]
        assert len(hits) == 1, (p, hits)
        blk = np.floor(p * n).astype(int)
        assert np.array_equal(block_of_cell[tc[hits[0]]], blk)


def test_quad_rule_by_hand():
    assert OM.split_quad([5, 2, 7, 9]) == [(5, 2, 9), (2, 7, 9)]
    assert OM.split_quad([1, 8, 3, 4]) == [(1, 8, 3), (1, 3, 4)]
    assert OM.split_quad([6, 4, 0, 9]) == [(6, 4, 0), (6, 0, 9)]
    assert OM.split_quad([6, 4, 9, 0]) == [(6, 4, 0), (4, 9, 0)]


def test_library_rejects_bad_input(D):
    xyz = np.eye(4, 3) * 1.0
    with pytest.raises(D.DsmcError):
        D.decompose(xyz, [[0, 1, 2]], [], [])                      # three vertices
    with pytest.raises(D.DsmcError):
        D.decompose(xyz, [[0, 1, 2, 7]], [], [])                   # index out of range
    with pytest.raises(D.DsmcError):
        D.decompose(xyz, [[0, 1, 2, 3]], [[0, 1, 2, 3], [0, 1, 2, 3]], [0, 0], [1, 0])   # quad partners


def test_mixed_box_gas_at_rest_stays_uniform():
    from oracle import Oracle
    m = W.mixed_box(5, 5, 5, jitter=0.1, seed=2)
    xyz, tets, tc, bf, bg, bp, bpar = OM.decompose(m.xyz, m.cells, m.bfaces, m.bgroup)
    mesh = W.Mesh(xyz=xyz, tets=tets, bfaces=bf, bgroup=bg, bpartner=None, h=m.h)
    wl = W.cavity_on_mesh(mesh, Kn=0.5, ppc=60, lid_speed=0.0, vel_fp32=0, n_ss=20, n_cells=len(m.cells))
    o = Oracle(wl)
    o.step(120)
    f = OM.cell_fields(o, tc, len(m.cells), which=0)
    ns = o.n_steady
    assert ns == 100
    # cell counts per step are Poisson about n V / F_N; over ns correlated
    # steps the noise is bounded by that of one step
    cv = np.bincount(tc, weights=o.volumes(), minlength=len(m.cells))
    mean_n = wl.run.n0 * cv / wl.run.F_N
    z = (f[:, 0] / wl.run.n0 - 1.0) * np.sqrt(mean_n)
    assert np.all(np.abs(z) < 5), np.abs(z).max()
    assert abs(np.mean(f[:, 0]) / wl.run.n0 - 1) < 0.01
    assert abs(np.average(f[:, 5], weights=cv) / wl.run.T0 - 1) < 0.01
    assert np.abs(f[:, 2:5]).max() < 0.2 * np.sqrt(KB * wl.run.T0 / wl.species.mass)
