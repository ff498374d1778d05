"""Mixed-element meshes for the oracle (test infrastructure only): the
tetrahedral mesh of a mesh of tetrahedra, pyramids, prisms and hexahedra
(the cell types of the space-station mesh of section 5.4), and the fields of
the original cells.

Written from the statement of the decomposition alone, cell by cell in
plain Python (no code shared with the library's decomposition):

* a quadrilateral face, vertices (a, b, c, d) in cyclic order, becomes the
  triangles (a, b, c), (a, c, d) if a or c carries the smallest vertex index
  of the four, else (a, b, d), (b, c, d);
* a tetrahedron stays; a pyramid (base v0 v1 v2 v3, apex v4) becomes the
  apex over each of its two base triangles;
* a prism (triangles v0 v1 v2 and v3 v4 v5) and a hexahedron (v0..v3 and
  v4..v7 above them) receive a new vertex at the mean of their vertices
  (each coordinate summed in local order, then divided by the vertex count)
  and one tetrahedron per face triangle with that vertex: for a prism the
  two triangles, then the quadrilaterals (0,1,4,3), (1,2,5,4), (2,0,3,5); for
  a hexahedron (0,1,2,3), (4,5,6,7), (0,1,5,4), (1,2,6,5), (2,3,7,6),
  (3,0,4,7);
* boundary triangles stay, boundary quadrilaterals split as above; the
  periodic partner of a triangle is the first triangle of its partner face.

Cell fields: the steady (or other) sums of a cell's tetrahedra added in
ascending tetrahedron order, over the sum of their volumes, through the
oracle's own field formulas (eq. dsmc_temperatures).
"""
import numpy as np

PRISM_TRIS = [(0, 1, 2), (3, 4, 5)]
PRISM_QUADS = [(0, 1, 4, 3), (1, 2, 5, 4), (2, 0, 3, 5)]
HEX_QUADS = [(0, 1, 2, 3), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7)]


def split_quad(q):
    a, b, c, d = (int(x) for x in q)
    smallest = min(a, b, c, d)
    if smallest in (a, c):
        return [(a, b, c), (a, c, d)]
    return [(a, b, d), (b, c, d)]


def decompose(xyz, cells, bfaces, bgroup, bpartner=None):
    """cells, bfaces: lists of vertex-index lists.  Returns (xyz, tets,
    tet_cell, btri, bgroup, bpartner, bparent) as numpy arrays."""
    pts = [tuple(float(v) for v in p) for p in np.asarray(xyz, float)]
    tets, tet_cell = [], []
    for c, v in enumerate(cells):
        v = [int(x) for x in v]
        if len(v) == 4:
            tets.append(tuple(v))
            tet_cell.append(c)
        elif len(v) == 5:
            for t in split_quad(v[:4]):
                tets.append(t + (v[4],))
                tet_cell.append(c)
        elif len(v) in (6, 8):
            mean = []
            for i in range(3):
                s = pts[v[0]][i]
                for j in range(1, len(v)):
                    s = s + pts[v[j]][i]
                mean.append(s / float(len(v)))
            ctr = len(pts)
            pts.append(tuple(mean))
            tris = []
            if len(v) == 6:
                tris += [tuple(v[k] for k in t) for t in PRISM_TRIS]
                for q in PRISM_QUADS:
                    tris += split_quad([v[k] for k in q])
            else:
                for q in HEX_QUADS:
                    tris += split_quad([v[k] for k in q])
            for t in tris:
                tets.append(t + (ctr,))
                tet_cell.append(c)
        else:
            raise ValueError(f"cell {c}: {len(v)} vertices")
    btri, bg, bp, bpar, first = [], [], [], [], []
    for b, f in enumerate(bfaces):
        first.append(len(btri))
        f = [int(x) for x in f]
        parts = [tuple(f)] if len(f) == 3 else split_quad(f)
        for t in parts:
            btri.append(t)
            bg.append(int(bgroup[b]))
            bp.append(-1 if bpartner is None or len(f) == 4 else int(bpartner[b]))
            bpar.append(b)
    bp = [first[p] if p >= 0 else -1 for p in bp]
    return (np.array(pts, dtype=np.float64), np.array(tets, dtype=np.int32), np.array(tet_cell, dtype=np.int32),
            np.array(btri, dtype=np.int32).reshape(-1, 3), np.array(bg, dtype=np.int32), np.array(bp, dtype=np.int32),
            np.array(bpar, dtype=np.int32))


def cell_fields(oracle, tet_cell, n_cells, which=0):
    """Fields [n_cells][15] of the original cells from the oracle's sums."""
    sums = oracle.sums(which)
    vol = oracle.volumes()
    agg = np.zeros((n_cells, sums.shape[1]))
    cv = np.zeros(n_cells)
    for t in range(len(tet_cell)):
        c = tet_cell[t]
        agg[c] = agg[c] + sums[t]
        cv[c] = cv[c] + vol[t]
    ns = oracle.n_steady if which == 0 else 1
    return oracle.fields_of_sums(agg, cv, ns)
