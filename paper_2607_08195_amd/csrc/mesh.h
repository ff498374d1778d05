// Host-side preprocessing of a tetrahedral mesh into the device mesh image.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace dsmcx {

constexpr double kBoltzmann = 1.380649e-23;

// One face slot of a tet: the outward plane (s n, s d) with n the cross
// product of the face's vertices taken in ascending global id, and the
// neighbour code: (tet << 2 | local face) inside, -1 - bface on the boundary.
struct HostMesh {
    int nv = 0, nt = 0, nb = 0, nf = 0;
    std::vector<double> xyz;        // [nv][3]
    std::vector<int32_t> tv;        // [nt][4] positively oriented
    std::vector<double> vol;        // [nt]
    std::vector<double> plane;      // [nt][4][4] outward (nx, ny, nz, d)
    std::vector<int32_t> nbr;       // [nt][4]
    // boundary faces
    std::vector<int32_t> bf_tet, bf_lf, bf_group, bf_partner;
    std::vector<int32_t> bf_vtx;    // [nb][3] ascending global ids
    std::vector<double> bf_frame;   // [nb][9] inward unit normal, t1, t2
    std::vector<double> bf_area;    // [nb]
    std::vector<double> bf_nraw;    // [nb][3] unnormalised face normal (p<q<r cross product)
    std::vector<double> bf_sign;    // [nb] +1 if bf_nraw points out of the domain
    // cell renumbering for locality: internal (device) id -> caller's id and back
    std::vector<int32_t> orig;      // [nt]
    std::vector<int32_t> inv;       // [nt]
};

// Returns an empty string on success, otherwise the reason the mesh is
// rejected (degenerate tet, face shared by >2 tets, unmatched boundary
// triangle, exterior face without a boundary triangle, bad group/partner).
std::string build_mesh(HostMesh& m, int nv, const double* xyz, int nt, const int32_t* tet,
                       int nb, const int32_t* bface, const int32_t* bgroup,
                       const int32_t* bpartner, int ngroups);

// Renumber the tets along a space-filling curve of their centroids (curve
// 1: Morton / Z-order, 2: Hilbert) so that cells close in space are close
// in memory; fills orig/inv.  Only internal numbering changes: every
// interface keeps the caller's ids.  With `group` (one value per tet,
// caller numbering), tets are ordered by group first, so each group stays
// contiguous.
void reorder_cells(HostMesh& m, const std::vector<int32_t>* group = nullptr, int curve = 1);

}  // namespace dsmcx
