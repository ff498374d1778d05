// Host mesh preprocessing: orientation, unique face planes, neighbour
// codes and boundary frames (face-based tracking of section 4.2 needs, per
// tet, the four face planes and what lies behind each face).
//
// Arithmetic contract (shared with any independent implementation, so that
// integer tracking decisions agree bit for bit):
//  * det = (b-a) . ((c-a) x (d-a)); det < 0 swaps local vertices 2 and 3;
//    volume = |det| / 6.
//  * local face f is opposite local vertex f.
//  * a face's plane uses its vertices sorted by global id p<q<r:
//    n = (q-p) x (r-p), d = n . p, unnormalised; a tet sees it with sign
//    s = +1 when n . o - d < 0 for its opposite vertex o (n points out).
//    The device stores (s n, s d), which yields bit-identical tests because
//    negation commutes with rounding.
//  * boundary frame: inward unit normal -s n / |n|, t1 = (q-p)/|q-p|,
//    t2 = n_in x t1.
#include "mesh.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace dsmcx {

namespace {

struct FaceKey {
    int32_t k[3];
    int32_t tet, lf;
};

inline bool key_less(const FaceKey& a, const FaceKey& b) {
    if (a.k[0] != b.k[0]) return a.k[0] < b.k[0];
    if (a.k[1] != b.k[1]) return a.k[1] < b.k[1];
    if (a.k[2] != b.k[2]) return a.k[2] < b.k[2];
    if (a.tet != b.tet) return a.tet < b.tet;
    return a.lf < b.lf;
}

inline bool key_eq(const int32_t* a, const int32_t* b) {
    return a[0] == b[0] && a[1] == b[1] && a[2] == b[2];
}

inline void sort_triple(int32_t* a) {
    if (a[0] > a[1]) std::swap(a[0], a[1]);
    if (a[1] > a[2]) std::swap(a[1], a[2]);
    if (a[0] > a[1]) std::swap(a[0], a[1]);
}

double orient(const double* a, const double* b, const double* c, const double* d) {
    double bx = b[0] - a[0], by = b[1] - a[1], bz = b[2] - a[2];
    double cx = c[0] - a[0], cy = c[1] - a[1], cz = c[2] - a[2];
    double dx = d[0] - a[0], dy = d[1] - a[1], dz = d[2] - a[2];
    double ex = cy * dz - cz * dy;
    double ey = cz * dx - cx * dz;
    double ez = cx * dy - cy * dx;
    return bx * ex + by * ey + bz * ez;
}

}  // namespace

std::string build_mesh(HostMesh& m, int nv, const double* xyz, int nt, const int32_t* tet,
                       int nb, const int32_t* bface, const int32_t* bgroup,
                       const int32_t* bpartner, int ngroups) {
    if (nv <= 0 || nt <= 0 || !xyz || !tet) return "empty mesh";
    if (nb < 0 || (nb > 0 && (!bface || !bgroup))) return "boundary arrays missing";
    m.nv = nv; m.nt = nt; m.nb = nb;
    m.xyz.assign(xyz, xyz + 3 * (size_t)nv);
    m.tv.resize(4 * (size_t)nt);
    m.vol.resize(nt);
    for (int t = 0; t < nt; ++t) {
        int32_t* q = &m.tv[4 * (size_t)t];
        for (int i = 0; i < 4; ++i) {
            q[i] = tet[4 * (size_t)t + i];
            if (q[i] < 0 || q[i] >= nv) return "tet vertex index out of range";
        }
        double det = orient(xyz + 3 * (size_t)q[0], xyz + 3 * (size_t)q[1], xyz + 3 * (size_t)q[2],
                            xyz + 3 * (size_t)q[3]);
        if (det < 0) { std::swap(q[2], q[3]); det = -det; }
        if (!(det > 0)) return "degenerate tet " + std::to_string(t);
        m.vol[t] = det / 6.0;
    }

    const size_t n4 = 4 * (size_t)nt;
    std::vector<FaceKey> keys(n4);
    for (int t = 0; t < nt; ++t)
        for (int f = 0; f < 4; ++f) {
            FaceKey& k = keys[4 * (size_t)t + f];
            int j = 0;
            for (int i = 0; i < 4; ++i)
                if (i != f) k.k[j++] = m.tv[4 * (size_t)t + i];
            sort_triple(k.k);
            k.tet = t;
            k.lf = f;
        }
    std::sort(keys.begin(), keys.end(), key_less);

    m.plane.assign(16 * (size_t)nt, 0.0);
    m.nbr.assign(n4, 0);
    const int32_t kUnmatched = INT32_MIN;
    std::vector<double> face_n;  // per exterior tet-face: raw normal for boundary frames
    int nf = 0, n_ext = 0;
    for (size_t i = 0; i < n4;) {
        size_t j = i + 1;
        while (j < n4 && key_eq(keys[j].k, keys[i].k)) ++j;
        if (j - i > 2) return "face shared by more than two tets";
        ++nf;
        const double* p = xyz + 3 * (size_t)keys[i].k[0];
        const double* q = xyz + 3 * (size_t)keys[i].k[1];
        const double* r = xyz + 3 * (size_t)keys[i].k[2];
        double ax = q[0] - p[0], ay = q[1] - p[1], az = q[2] - p[2];
        double bx = r[0] - p[0], by = r[1] - p[1], bz = r[2] - p[2];
        double nx = ay * bz - az * by;
        double ny = az * bx - ax * bz;
        double nz = ax * by - ay * bx;
        double d = nx * p[0] + ny * p[1] + nz * p[2];
        for (size_t e = i; e < j; ++e) {
            int t = keys[e].tet, f = keys[e].lf;
            const double* o = xyz + 3 * (size_t)m.tv[4 * (size_t)t + f];
            double test = (nx * o[0] + ny * o[1] + nz * o[2]) - d;
            double s = test < 0 ? 1.0 : -1.0;
            double* pl = &m.plane[16 * (size_t)t + 4 * f];
            pl[0] = s * nx; pl[1] = s * ny; pl[2] = s * nz; pl[3] = s * d;
            if (j - i == 2) {
                const FaceKey& o2 = keys[e == i ? i + 1 : i];
                m.nbr[4 * (size_t)t + f] = (o2.tet << 2) | o2.lf;
            } else {
                m.nbr[4 * (size_t)t + f] = kUnmatched;
                ++n_ext;
            }
        }
        i = j;
    }
    m.nf = nf;
    if (n_ext != nb) return "boundary triangle count differs from the exterior face count";
    if (nt >= (1 << 29)) return "too many tets";

    // exterior faces by sorted triple
    std::vector<FaceKey> ext;
    ext.reserve(n_ext);
    for (size_t i = 0; i < n4; ++i)
        if (m.nbr[i] == kUnmatched) {
            FaceKey k;
            int t = (int)(i / 4), f = (int)(i % 4);
            int j = 0;
            for (int v = 0; v < 4; ++v)
                if (v != f) k.k[j++] = m.tv[4 * (size_t)t + v];
            sort_triple(k.k);
            k.tet = t;
            k.lf = f;
            ext.push_back(k);
        }
    std::sort(ext.begin(), ext.end(), key_less);

    m.bf_tet.resize(nb); m.bf_lf.resize(nb); m.bf_group.resize(nb); m.bf_partner.resize(nb);
    m.bf_vtx.resize(3 * (size_t)nb); m.bf_frame.resize(9 * (size_t)nb); m.bf_area.resize(nb);
    m.bf_nraw.resize(3 * (size_t)nb); m.bf_sign.resize(nb);
    for (int b = 0; b < nb; ++b) {
        FaceKey k;
        for (int i = 0; i < 3; ++i) k.k[i] = bface[3 * (size_t)b + i];
        sort_triple(k.k);
        auto it = std::lower_bound(ext.begin(), ext.end(), k, [](const FaceKey& a, const FaceKey& x) {
            if (a.k[0] != x.k[0]) return a.k[0] < x.k[0];
            if (a.k[1] != x.k[1]) return a.k[1] < x.k[1];
            return a.k[2] < x.k[2];
        });
        if (it == ext.end() || !key_eq(it->k, k.k)) return "boundary triangle matches no exterior face";
        int g = bgroup[b];
        if (g < 0 || g >= ngroups) return "boundary group out of range";
        int t = it->tet, f = it->lf;
        if (m.nbr[4 * (size_t)t + f] != kUnmatched) return "boundary triangle listed twice";
        m.nbr[4 * (size_t)t + f] = -1 - b;
        m.bf_tet[b] = t; m.bf_lf[b] = f; m.bf_group[b] = g;
        m.bf_partner[b] = bpartner ? bpartner[b] : -1;
        if (m.bf_partner[b] >= nb) return "periodic partner out of range";
        for (int i = 0; i < 3; ++i) m.bf_vtx[3 * (size_t)b + i] = k.k[i];
        // raw plane normal in ascending-id order and the tet's sign
        const double* p = xyz + 3 * (size_t)k.k[0];
        const double* q = xyz + 3 * (size_t)k.k[1];
        const double* r = xyz + 3 * (size_t)k.k[2];
        double ax = q[0] - p[0], ay = q[1] - p[1], az = q[2] - p[2];
        double bx = r[0] - p[0], by = r[1] - p[1], bz = r[2] - p[2];
        double n[3] = {ay * bz - az * by, az * bx - ax * bz, ax * by - ay * bx};
        double sgn = (m.plane[16 * (size_t)t + 4 * f] == n[0] && m.plane[16 * (size_t)t + 4 * f + 1] == n[1] &&
                      m.plane[16 * (size_t)t + 4 * f + 2] == n[2]) ? 1.0 : -1.0;
        m.bf_sign[b] = sgn;
        for (int i = 0; i < 3; ++i) m.bf_nraw[3 * (size_t)b + i] = n[i];
        double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        m.bf_area[b] = 0.5 * nn;
        double* fr = &m.bf_frame[9 * (size_t)b];
        for (int i = 0; i < 3; ++i) fr[i] = (-sgn * n[i]) / nn;
        double al = std::sqrt(ax * ax + ay * ay + az * az);
        fr[3] = ax / al; fr[4] = ay / al; fr[5] = az / al;
        fr[6] = fr[1] * fr[5] - fr[2] * fr[4];
        fr[7] = fr[2] * fr[3] - fr[0] * fr[5];
        fr[8] = fr[0] * fr[4] - fr[1] * fr[3];
    }
    return std::string();
}

namespace {
inline uint64_t spread3(uint64_t v) {
    v &= 0x1FFFFFull;
    v = (v | (v << 32)) & 0x1F00000000FFFFull;
    v = (v | (v << 16)) & 0x1F0000FF0000FFull;
    v = (v | (v << 8)) & 0x100F00F00F00F00Full;
    v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

// Hilbert curve index of 21-bit coordinates (Skilling, "Programming the
// Hilbert curve", 2004: the axes are turned into the curve's transposed
// index by undoing the excess work of the Gray code level by level, then
// Gray-encoded; interleaving the transposed words gives the index).
inline uint64_t hilbert3(uint32_t x, uint32_t y, uint32_t z) {
    uint32_t X[3] = {x, y, z};
    const uint32_t M = 1u << 20;
    for (uint32_t Q = M; Q > 1; Q >>= 1) {
        const uint32_t P = Q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                const uint32_t t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    for (int i = 1; i < 3; ++i) X[i] ^= X[i - 1];
    uint32_t t = 0;
    for (uint32_t Q = M; Q > 1; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1;
    for (int i = 0; i < 3; ++i) X[i] ^= t;
    return (spread3(X[0]) << 2) | (spread3(X[1]) << 1) | spread3(X[2]);
}
}  // namespace

void reorder_cells(HostMesh& m, const std::vector<int32_t>* group, int curve) {
    const int nt = m.nt;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    std::vector<double> cen(3 * (size_t)nt);
    for (int t = 0; t < nt; ++t)
        for (int i = 0; i < 3; ++i) {
            double s = 0;
            for (int k = 0; k < 4; ++k) s += m.xyz[3 * (size_t)m.tv[4 * (size_t)t + k] + i];
            cen[3 * (size_t)t + i] = 0.25 * s;
            lo[i] = std::min(lo[i], cen[3 * (size_t)t + i]);
            hi[i] = std::max(hi[i], cen[3 * (size_t)t + i]);
        }
    double ext = 0;
    for (int i = 0; i < 3; ++i) ext = std::max(ext, hi[i] - lo[i]);
    if (!(ext > 0)) ext = 1;
    std::vector<uint64_t> key(nt);
    for (int t = 0; t < nt; ++t) {
        uint64_t k = 0;
        uint32_t qv[3];
        for (int i = 0; i < 3; ++i) {
            double q = (cen[3 * (size_t)t + i] - lo[i]) / ext * 2097151.0;
            uint64_t qi = (uint64_t)std::min(2097151.0, std::max(0.0, q));
            qv[i] = (uint32_t)qi;
            k |= spread3(qi) << i;
        }
        key[t] = curve == 2 ? hilbert3(qv[0], qv[1], qv[2]) : k;
    }
    m.orig.resize(nt);
    std::iota(m.orig.begin(), m.orig.end(), 0);
    std::stable_sort(m.orig.begin(), m.orig.end(), [&](int a, int b) {
        if (group && (*group)[a] != (*group)[b]) return (*group)[a] < (*group)[b];
        return key[a] < key[b];
    });
    m.inv.assign(nt, 0);
    for (int t = 0; t < nt; ++t) m.inv[m.orig[t]] = t;
    std::vector<int32_t> tv(4 * (size_t)nt), nbr(4 * (size_t)nt);
    std::vector<double> vol(nt), plane(16 * (size_t)nt);
    for (int t = 0; t < nt; ++t) {
        const int o = m.orig[t];
        for (int k = 0; k < 4; ++k) {
            tv[4 * (size_t)t + k] = m.tv[4 * (size_t)o + k];
            const int code = m.nbr[4 * (size_t)o + k];
            nbr[4 * (size_t)t + k] = code >= 0 ? ((m.inv[code >> 2] << 2) | (code & 3)) : code;
        }
        vol[t] = m.vol[o];
        for (int k = 0; k < 16; ++k) plane[16 * (size_t)t + k] = m.plane[16 * (size_t)o + k];
    }
    m.tv.swap(tv);
    m.nbr.swap(nbr);
    m.vol.swap(vol);
    m.plane.swap(plane);
    for (int b = 0; b < m.nb; ++b) m.bf_tet[b] = m.inv[m.bf_tet[b]];
}

}  // namespace dsmcx
