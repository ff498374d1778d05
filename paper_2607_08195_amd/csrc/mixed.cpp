// Mixed-element meshes (tetrahedra, pyramids, prisms, hexahedra; the cell
// types of the space-station mesh of section 5.4) turned into the
// tetrahedral mesh that the tracker, the collisions and the sampling work
// on.  Host code only.
//
// Every quadrilateral face is split along the diagonal through its vertex of
// smallest global index, so two cells sharing a quadrilateral (or a
// boundary quadrilateral and its cell) split it the same way and the
// tetrahedral mesh is conforming.  A pyramid becomes the two tetrahedra of
// its apex over the two base triangles; a prism or a hexahedron gets one
// new vertex at the mean of its vertices and one tetrahedron per face
// triangle (8 and 12).
#include <cstring>
#include <string>
#include <vector>

#include "dsmc.h"

namespace {

// faces of the cell types in their local vertex numbers (outward order not
// needed: the mesh builder orients every tetrahedron itself)
const int kPrismTris[2][3] = {{0, 1, 2}, {3, 4, 5}};
const int kPrismQuads[3][4] = {{0, 1, 4, 3}, {1, 2, 5, 4}, {2, 0, 3, 5}};
const int kHexQuads[6][4] = {{0, 1, 2, 3}, {4, 5, 6, 7}, {0, 1, 5, 4}, {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}};

// The two triangles of quadrilateral (a, b, c, d), given cyclically:
// (a, b, c), (a, c, d) when the smallest index is a or c, otherwise
// (a, b, d), (b, c, d).
void split_quad(const int32_t q[4], int32_t t[2][3]) {
    int m = 0;
    for (int k = 1; k < 4; ++k)
        if (q[k] < q[m]) m = k;
    if (m == 0 || m == 2) {
        t[0][0] = q[0]; t[0][1] = q[1]; t[0][2] = q[2];
        t[1][0] = q[0]; t[1][1] = q[2]; t[1][2] = q[3];
    } else {
        t[0][0] = q[0]; t[0][1] = q[1]; t[0][2] = q[3];
        t[1][0] = q[1]; t[1][1] = q[2]; t[1][2] = q[3];
    }
}

int tets_of(int nv) { return nv == 4 ? 1 : nv == 5 ? 2 : nv == 6 ? 8 : nv == 8 ? 12 : -1; }

struct Out {
    std::vector<double> xyz;
    std::vector<int32_t> tv, tcell, bv, bg, bp, bparent;
};

std::string decompose(const dsmc_mixed_mesh_desc* in, Out& o) {
    if (in->n_vertices < 0 || in->n_cells < 0 || in->n_bfaces < 0 || (in->n_vertices > 0 && !in->xyz) ||
        (in->n_cells > 0 && (!in->cell_nv || !in->cell_vtx)) ||
        (in->n_bfaces > 0 && (!in->bface_nv || !in->bface_vtx || !in->bface_group)))
        return "NULL or negative descriptor field";
    const int nv = in->n_vertices;
    o.xyz.assign(in->xyz, in->xyz + 3 * (size_t)nv);
    size_t off = 0;
    for (int c = 0; c < in->n_cells; ++c) {
        const int k = in->cell_nv[c];
        if (tets_of(k) < 0) return "cell " + std::to_string(c) + ": vertex count must be 4, 5, 6 or 8";
        const int32_t* v = in->cell_vtx + off;
        off += (size_t)k;
        for (int j = 0; j < k; ++j)
            if (v[j] < 0 || v[j] >= nv) return "cell " + std::to_string(c) + ": vertex index out of range";
        auto tet = [&](int32_t a, int32_t b, int32_t d, int32_t e) {
            o.tv.push_back(a); o.tv.push_back(b); o.tv.push_back(d); o.tv.push_back(e);
            o.tcell.push_back(c);
        };
        if (k == 4) {
            tet(v[0], v[1], v[2], v[3]);
        } else if (k == 5) {
            int32_t t[2][3];
            split_quad(v, t);
            tet(t[0][0], t[0][1], t[0][2], v[4]);
            tet(t[1][0], t[1][1], t[1][2], v[4]);
        } else {
            // the new vertex: coordinate-wise sum in local order, divided by k
            const int32_t ctr = (int32_t)(o.xyz.size() / 3);
            for (int i = 0; i < 3; ++i) {
                double s = in->xyz[3 * (size_t)v[0] + i];
                for (int j = 1; j < k; ++j) s = s + in->xyz[3 * (size_t)v[j] + i];
                o.xyz.push_back(s / (double)k);
            }
            const int nq = k == 6 ? 3 : 6;
            if (k == 6)
                for (int f = 0; f < 2; ++f) tet(v[kPrismTris[f][0]], v[kPrismTris[f][1]], v[kPrismTris[f][2]], ctr);
            for (int f = 0; f < nq; ++f) {
                const int* lq = k == 6 ? kPrismQuads[f] : kHexQuads[f];
                const int32_t q[4] = {v[lq[0]], v[lq[1]], v[lq[2]], v[lq[3]]};
                int32_t t[2][3];
                split_quad(q, t);
                tet(t[0][0], t[0][1], t[0][2], ctr);
                tet(t[1][0], t[1][1], t[1][2], ctr);
            }
        }
    }
    // boundary faces: triangles kept, quadrilaterals split as their cells
    // split them; periodic partners are carried for triangles only
    std::vector<int32_t> first(in->n_bfaces);
    off = 0;
    for (int b = 0; b < in->n_bfaces; ++b) {
        const int k = in->bface_nv[b];
        if (k != 3 && k != 4) return "boundary face " + std::to_string(b) + ": vertex count must be 3 or 4";
        const int32_t* v = in->bface_vtx + off;
        off += (size_t)k;
        for (int j = 0; j < k; ++j)
            if (v[j] < 0 || v[j] >= nv) return "boundary face " + std::to_string(b) + ": vertex index out of range";
        const int32_t p = in->bface_partner ? in->bface_partner[b] : -1;
        if (p >= in->n_bfaces) return "boundary face " + std::to_string(b) + ": partner out of range";
        if (p >= 0 && (k != 3 || in->bface_nv[p] != 3))
            return "boundary face " + std::to_string(b) + ": periodic partners must be triangles";
        first[b] = (int32_t)o.bg.size();
        if (k == 3) {
            o.bv.insert(o.bv.end(), v, v + 3);
            o.bg.push_back(in->bface_group[b]);
            o.bp.push_back(p);
            o.bparent.push_back(b);
        } else {
            int32_t t[2][3];
            split_quad(v, t);
            for (int h = 0; h < 2; ++h) {
                o.bv.insert(o.bv.end(), t[h], t[h] + 3);
                o.bg.push_back(in->bface_group[b]);
                o.bp.push_back(-1);
                o.bparent.push_back(b);
            }
        }
    }
    for (size_t i = 0; i < o.bp.size(); ++i)
        if (o.bp[i] >= 0) o.bp[i] = first[o.bp[i]];
    return "";
}

std::string g_mixed_error;

}  // namespace

extern "C" {

dsmc_status dsmc_mesh_decompose(const dsmc_mixed_mesh_desc* in, dsmc_tet_mesh_out* out) {
    if (!in || !out) return DSMC_E_INVALID;
    Out o;
    g_mixed_error = decompose(in, o);
    if (!g_mixed_error.empty()) return DSMC_E_MESH;
    const bool fill = out->xyz || out->tet_vtx || out->tet_cell || out->bface_vtx || out->bface_group ||
                      out->bface_partner || out->bface_parent;
    const int32_t nv = (int32_t)(o.xyz.size() / 3), nt = (int32_t)o.tcell.size(), nb = (int32_t)o.bg.size();
    if (fill && (out->n_vertices < nv || out->n_tets < nt || out->n_bfaces < nb)) {
        g_mixed_error = "output arrays smaller than the decomposed mesh";
        return DSMC_E_INVALID;
    }
    out->n_vertices = nv;
    out->n_tets = nt;
    out->n_bfaces = nb;
    if (out->xyz) std::memcpy(out->xyz, o.xyz.data(), sizeof(double) * o.xyz.size());
    if (out->tet_vtx) std::memcpy(out->tet_vtx, o.tv.data(), sizeof(int32_t) * o.tv.size());
    if (out->tet_cell) std::memcpy(out->tet_cell, o.tcell.data(), sizeof(int32_t) * o.tcell.size());
    if (out->bface_vtx) std::memcpy(out->bface_vtx, o.bv.data(), sizeof(int32_t) * o.bv.size());
    if (out->bface_group) std::memcpy(out->bface_group, o.bg.data(), sizeof(int32_t) * o.bg.size());
    if (out->bface_partner) std::memcpy(out->bface_partner, o.bp.data(), sizeof(int32_t) * o.bp.size());
    if (out->bface_parent) std::memcpy(out->bface_parent, o.bparent.data(), sizeof(int32_t) * o.bparent.size());
    return DSMC_OK;
}

const char* dsmc_mesh_error(void) { return g_mixed_error.c_str(); }

}  // extern "C"
