"""The sphere-in-a-box mesh generator: conforming (every interior triangle
shared by exactly two tets, the exterior triangles exactly the boundary
list), no degenerate tet, the tets filling the box minus the inscribed
polyhedron, the wall triangles' vertices on the sphere, and the oracle
building it (its own mesh checks) with the initial fill inside."""
import numpy as np
import pytest

from paper_2607_08195_amd import workloads as W
from oracle import Oracle


@pytest.mark.parametrize("N,K,grade", [(4, 3, 5.0), (6, 4, 2.0)])
def test_sphere_mesh_is_conforming(N, K, grade):
    m = W.sphere_box_mesh(N=N, K=K, grade=grade)
    xyz, T = m.xyz, m.tets
    a, b, c, d = (xyz[T[:, i]] for i in range(4))
    vol = np.abs(np.einsum("ij,ij->i", b - a, np.cross(c - a, d - a))) / 6.0
    assert vol.min() > 1e-3 * vol.max()
    faces = np.sort(np.concatenate([T[:, [1, 2, 3]], T[:, [0, 2, 3]], T[:, [0, 1, 3]], T[:, [0, 1, 2]]]), axis=1)
    u, cnt = np.unique(faces, axis=0, return_counts=True)
    assert cnt.max() == 2
    ext = {tuple(r) for r in u[cnt == 1]}
    assert ext == {tuple(r) for r in np.sort(m.bfaces, axis=1)} and len(ext) == len(m.bfaces)
    sph = m.bfaces[m.bgroup == 6]
    r = np.linalg.norm(xyz[sph.ravel()], axis=1)
    assert np.allclose(r, 0.5, rtol=0, atol=1e-12)
    # box volume minus the convex polyhedron spanned by the wall triangles
    # (tets from the centre to each triangle)
    p, q, s = xyz[sph[:, 0]], xyz[sph[:, 1]], xyz[sph[:, 2]]
    poly = np.abs(np.einsum("ij,ij->i", p, np.cross(q, s))).sum() / 6.0
    assert abs(vol.sum() - (96.0 - poly)) < 1e-9 * 96.0
    assert 0.9 * np.pi / 6 < poly < np.pi / 6
    # the groups of the box faces lie on their planes
    for g, (ax, v) in enumerate([(0, -2.0), (0, 4.0), (1, -2.0), (1, 2.0), (2, -2.0), (2, 2.0)]):
        assert np.all(xyz[m.bfaces[m.bgroup == g].ravel(), ax] == v)


def test_oracle_builds_the_sphere_flow():
    wl = W.sphere_flow(N=4, K=3, ppc=2)
    o = Oracle(wl)
    st = o.particles()
    assert len(st["pid"]) > 0
    # outside the inscribed polyhedron, whose facets lie close to the sphere
    assert np.all(np.linalg.norm(st["x"], axis=1) > 0.45)
    o.step(2)
    assert o.counters()["injected"] > 0
