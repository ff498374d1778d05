// Device-side building blocks shared by the kernels: the counter-based
// generator, its transforms and the particle tracking step.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dsmcx {

#define DSMC_TWO_PI 6.283185307179586
#define DSMC_SQRT_PI 1.7724538509055159
#define DSMC_INV_SQRT2 0.7071067811865476
#define DSMC_MAX_HOPS 1000

// Stream purposes of the counter layout (subject, step, purpose<<24 | block, block>>24).
enum : uint32_t {
    kPurposeInit = 1,
    kPurposeWall = 2,
    kPurposeInjectCount = 3,
    kPurposeNtcCount = 4,
    kPurposePair = 5,
    kPurposeScatter = 6,
    kPurposeRecalibrate = 7,
    kPurposeMlp = 8,
    kPurposeInitCount = 9,
    kPurposeInject = 10,
    kPurposeInelasticI = 11,  // rotational exchange of the first partner of a pair (block = candidate)
    kPurposeInelasticJ = 12,  // and of the second
};

enum : int { kBcDiffuse = 0, kBcSpecular = 1, kBcInflow = 2, kBcOutflow = 3, kBcPeriodic = 4 };

struct Rand4 {
    uint32_t w[4];
};

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplications mixed with the other words and the key; the key
// advances by the two Weyl constants between rounds.
__device__ __forceinline__ Rand4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // each 64-bit product is one v_mad_u64_u32 (rather than a mul_hi and
        // a mul_lo, both quarter-rate)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    Rand4 o;
    o.w[0] = c0; o.w[1] = c1; o.w[2] = c2; o.w[3] = c3;
    return o;
}

struct RngKey {
    uint32_t k0, k1;
};

__device__ __forceinline__ Rand4 draw(RngKey key, uint32_t subject, uint32_t step, uint32_t purpose,
                                      uint64_t block) {
    return philox(subject, step, (purpose << 24) | (uint32_t)(block & 0xFFFFFFu), (uint32_t)(block >> 24),
                  key.k0, key.k1);
}

// Uniform in (0,1): 52 random bits k from two words, (k + 1/2) * 2^-52,
// exact in binary64 and never 0 or 1.
__device__ __forceinline__ double u01(uint32_t a, uint32_t b) {
    const uint64_t k = ((uint64_t)(a >> 6) << 26) | (uint64_t)(b >> 6);
    return ((double)k + 0.5) * 0x1p-52;
}

// Integer in [0, n) by 32x32 multiply-shift.
__device__ __forceinline__ uint32_t pick(uint32_t r, uint32_t n) {
    return (uint32_t)(((uint64_t)r * (uint64_t)n) >> 32);
}

__device__ __forceinline__ void box_muller(double u1, double u2, double& g1, double& g2) {
    const double r = sqrt(-2.0 * log(u1));
    const double a = DSMC_TWO_PI * u2;
    g1 = r * cos(a);
    g2 = r * sin(a);
}

template <class VT>
__device__ __forceinline__ double round_store(double x) {
    return (double)(VT)x;
}

// Boundary group constants on the device.
struct GroupDev {
    int kind;
    int pad;
    double beta;     // sqrt(2 k T / m)
    double sw;       // sqrt(k T / m)
    double u[3];
    double shift[3];
    double kT;       // k T (mean rotational energy of two degrees of freedom)
};

// Slot of a particle in its cell's histogram bin.  Lanes of a wave that
// land in the same cell are grouped (ballot rounds over the first pending
// lane's cell, at most kRankRounds groups); one atomic add per group,
// issued by its first lane together with the single adds of ungrouped
// lanes, then each member takes base + its rank within the group.  Must be
// called by every lane of the wave (uniform control flow).
constexpr int kRankRounds = 8;
__device__ __forceinline__ uint32_t bin_slot(int32_t* counts, int cell, bool active) {
    const int lane = threadIdx.x & 63;
    uint64_t pending = __ballot(active);
    int leader_of_mine = lane;
    uint64_t group = 0;
    for (int round = 0; round < kRankRounds && pending; ++round) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int c0 = __shfl(cell, leader, 64);
        const uint64_t same = __ballot(active && cell == c0) & pending;
        if ((same >> lane) & 1ull) {
            leader_of_mine = leader;
            group = same;
        }
        pending &= ~same;
    }
    int base = 0;
    if (active && (group == 0 || leader_of_mine == lane))
        base = atomicAdd(&counts[cell], group ? __popcll(group) : 1);
    const int gbase = __shfl(base, leader_of_mine, 64);
    return group ? (uint32_t)(gbase + __popcll(group & ((1ull << lane) - 1ull))) : (uint32_t)base;
}

// Per-case parameters when several independent cases share one mesh (a
// batch): time step, particle weight, initial state and generator key.
struct CaseDev {
    double dt, FN, n0, T0, sig, u0[3], smax0;
    uint32_t k0, k1;
    int32_t cell0;  // first cell of the case in the caller's numbering (cell subjects are case-local)
    int32_t pad;
};

struct MeshDev {
    int nt;
    const double4* plane;    // [nt*4] outward (s n, s d)
    const int32_t* nbr;      // [nt*4] (tet<<2|lf) or -1-bface
    const double* vol;       // [nt]
    const int32_t* bf_group; // [nb]
    const int32_t* bf_pcode; // [nb] periodic partner (tet<<2|lf) or -1
    const double* bf_frame;  // [nb][9]
    const GroupDev* groups;
    double mass;
    const int32_t* cell_case;  // [nt] case of each cell (batch), or null
    const CaseDev* cases;
    int nb;                    // boundary faces
    int n_ss;                  // surface sums are taken on steps after n_ss
    double* surf;              // [5][nb] surface sums, or null (surface sampling off)
    int rot;                   // 1: particles carry rotational energy (two degrees of freedom)
};

// Surface sampling at a wall interaction of boundary face bf that turned
// velocity a into b: the velocity change a - b (momentum given to the wall
// per unit mass), the energy change (|a|^2 - |b|^2) / 2 and the hit, added to
// the face's sums on sampled steps.
// dI: the rotational energy the molecule gives the wall (incident minus
// re-emitted I_r; a rotating gas only, sixth row).
__device__ __forceinline__ void surface_hit(const MeshDev& m, int bf, uint32_t step, double a0, double a1,
                                            double a2, double b0, double b1, double b2, double dI) {
    if (!m.surf || (int64_t)step <= (int64_t)m.n_ss) return;
    double* s = m.surf + bf;
    const size_t nb = (size_t)m.nb;
    unsafeAtomicAdd(s, a0 - b0);
    unsafeAtomicAdd(s + nb, a1 - b1);
    unsafeAtomicAdd(s + 2 * nb, a2 - b2);
    unsafeAtomicAdd(s + 3 * nb, 0.5 * ((a0 * a0 + a1 * a1 + a2 * a2) - (b0 * b0 + b1 * b1 + b2 * b2)));
    unsafeAtomicAdd(s + 4 * nb, 1.0);
    if (m.rot && dI != 0.0) unsafeAtomicAdd(s + 5 * nb, dI);
}

// Generator key and time step of the case that owns `cell` (batch mode).
__device__ __forceinline__ void case_params(const int32_t* cell_case, const CaseDev* cases, int cell, RngKey& key,
                                            double& dt) {
    if (cell_case) {
        const CaseDev& cs = cases[cell_case[cell]];
        key.k0 = cs.k0;
        key.k1 = cs.k1;
        dt = cs.dt;
    }
}

struct TraceOut {
    int status;   // 0 alive, 1 removed through an open face, 2 lost
    int hops;
    int walls;
};

// Face-to-face tracking of one particle for time t (the exit test is the
// same arithmetic as the plane contract: den = N.v, lambda = (D - N.x)/den
// over faces with den > 0 other than the entry face, clamped at 0, minimum
// with ties to the lowest local face).
template <class VT>
__device__ __forceinline__ TraceOut trace(const MeshDev& m, double& x0, double& x1, double& x2,
                                          double& v0, double& v1, double& v2, int& cell, int entry,
                                          uint32_t pid, uint32_t step, RngKey key, double t,
                                          double* ir = nullptr) {
    TraceOut out{0, 0, 0};
    int c = cell;
    int nhop = 0;
    int hits = 0;
    for (;;) {
        int fb = -1;
        double lb = 0.0;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            if (f == entry) continue;
            const double4 pl = m.plane[4 * c + f];
            const double den = fma(pl.z, v2, fma(pl.y, v1, pl.x * v0));
            if (den > 0) {
                double lam = (pl.w - fma(pl.z, x2, fma(pl.y, x1, pl.x * x0))) / den;
                if (lam < 0) lam = 0;
                if (fb < 0 || lam < lb) {
                    fb = f;
                    lb = lam;
                }
            }
        }
        if (fb < 0 || lb >= t) {
            x0 = fma(v0, t, x0);
            x1 = fma(v1, t, x1);
            x2 = fma(v2, t, x2);
            break;
        }
        x0 = fma(v0, lb, x0);
        x1 = fma(v1, lb, x1);
        x2 = fma(v2, lb, x2);
        t = t - lb;
        ++nhop;
        if (nhop > DSMC_MAX_HOPS) {
            out.status = 2;
            break;
        }
        const int code = m.nbr[4 * c + fb];
        if (code >= 0) {
            c = code >> 2;
            entry = code & 3;
            continue;
        }
        const int bf = -1 - code;
        const GroupDev& g = m.groups[m.bf_group[bf]];
        if (g.kind == kBcDiffuse) {
            const Rand4 r0 = draw(key, pid, step, kPurposeWall, (uint64_t)(2 * hits));
            const Rand4 r1 = draw(key, pid, step, kPurposeWall, (uint64_t)(2 * hits + 1));
            const double ua = u01(r0.w[0], r0.w[1]);
            const double ub = u01(r0.w[2], r0.w[3]);
            const double uc = u01(r1.w[0], r1.w[1]);
            const double vn = g.beta * sqrt(-log(ua));
            double g1, g2;
            box_muller(ub, uc, g1, g2);
            const double* fr = m.bf_frame + 9 * (size_t)bf;
            const double a0 = v0, a1 = v1, a2 = v2;
            v0 = round_store<VT>((vn * fr[0] + g.sw * (g1 * fr[3] + g2 * fr[6])) + g.u[0]);
            v1 = round_store<VT>((vn * fr[1] + g.sw * (g1 * fr[4] + g2 * fr[7])) + g.u[1]);
            v2 = round_store<VT>((vn * fr[2] + g.sw * (g1 * fr[5] + g2 * fr[8])) + g.u[2]);
            // the re-emitted molecule's rotation is in equilibrium at the wall
            const double Inew = ir ? -g.kT * log(u01(r1.w[2], r1.w[3])) : 0.0;
            surface_hit(m, bf, step, a0, a1, a2, v0, v1, v2, ir ? *ir - Inew : 0.0);
            if (ir) *ir = Inew;
            ++hits;
            ++out.walls;
            entry = fb;
        } else if (g.kind == kBcSpecular) {
            const double4 pl = m.plane[4 * c + fb];
            const double vn = pl.x * v0 + pl.y * v1 + pl.z * v2;
            const double nn = pl.x * pl.x + pl.y * pl.y + pl.z * pl.z;
            const double f2 = 2.0 * (vn / nn);
            const double a0 = v0, a1 = v1, a2 = v2;
            v0 = round_store<VT>(v0 - f2 * pl.x);
            v1 = round_store<VT>(v1 - f2 * pl.y);
            v2 = round_store<VT>(v2 - f2 * pl.z);
            surface_hit(m, bf, step, a0, a1, a2, v0, v1, v2, 0.0);
            ++out.walls;
            entry = fb;
        } else if (g.kind == kBcPeriodic) {
            x0 = x0 + g.shift[0];
            x1 = x1 + g.shift[1];
            x2 = x2 + g.shift[2];
            const int pc = m.bf_pcode[bf];
            c = pc >> 2;
            entry = pc & 3;
        } else {
            out.status = 1;
            break;
        }
    }
    out.hops = nhop;
    cell = c;
    return out;
}

// State of one particle being tracked by a lane of the batched move kernel.
struct Walker {
    double x0, x1, x2, v0, v1, v2, t;
    int c, entry, nhop, hits, walls;
    uint32_t pid;
    double ir;   // rotational energy (read and written only when the gas rotates)
};

// One exit test of a walker (and the crossing or boundary interaction it
// leads to).  Returns -1 while the walker is still in flight, 0 when it has
// used up its time (alive), 1 when it left through an open face, 2 when it
// exceeded the hop limit.  Faces are visited in ascending local index, the
// entry face skipped, so ties resolve to the lowest index as in trace().
// One face of the exit test, branch-free: lambda = (D - N.x) / (N.v) is
// computed for every face and kept only for a face other than the entry
// face with N.v > 0; clamped at 0; the running minimum keeps the lowest
// face index on ties because faces are visited in ascending order.
__device__ __forceinline__ void exit_candidate(const double4& pl, int f, const Walker& w, int& fb, double& lb) {
    const double den = fma(pl.z, w.v2, fma(pl.y, w.v1, pl.x * w.v0));
    double lam = (pl.w - fma(pl.z, w.x2, fma(pl.y, w.x1, pl.x * w.x0))) / den;
    lam = lam < 0 ? 0.0 : lam;
    const bool ok = (f != w.entry) && (den > 0);
    const bool take = ok && (fb < 0 || lam < lb);
    fb = take ? f : fb;
    lb = take ? lam : lb;
}

// Diffuse re-emission of a walker that has just reached boundary face bf
// through local face fb (the wall becomes its entry face).
template <class VT>
__device__ __forceinline__ void diffuse_reemit(const MeshDev& m, Walker& w, int bf, int fb, uint32_t step,
                                               RngKey key) {
    const GroupDev& g = m.groups[m.bf_group[bf]];
    const Rand4 r0 = draw(key, w.pid, step, kPurposeWall, (uint64_t)(2 * w.hits));
    const Rand4 r1 = draw(key, w.pid, step, kPurposeWall, (uint64_t)(2 * w.hits + 1));
    const double ua = u01(r0.w[0], r0.w[1]);
    const double ub = u01(r0.w[2], r0.w[3]);
    const double uc = u01(r1.w[0], r1.w[1]);
    const double vn = g.beta * sqrt(-log(ua));
    double g1, g2;
    box_muller(ub, uc, g1, g2);
    const double* fr = m.bf_frame + 9 * (size_t)bf;
    const double a0 = w.v0, a1 = w.v1, a2 = w.v2;
    w.v0 = round_store<VT>((vn * fr[0] + g.sw * (g1 * fr[3] + g2 * fr[6])) + g.u[0]);
    w.v1 = round_store<VT>((vn * fr[1] + g.sw * (g1 * fr[4] + g2 * fr[7])) + g.u[1]);
    w.v2 = round_store<VT>((vn * fr[2] + g.sw * (g1 * fr[5] + g2 * fr[8])) + g.u[2]);
    // the re-emitted molecule's rotation is in equilibrium at the wall
    const double Inew = m.rot ? -g.kT * log(u01(r1.w[2], r1.w[3])) : 0.0;
    surface_hit(m, bf, step, a0, a1, a2, w.v0, w.v1, w.v2, m.rot ? w.ir - Inew : 0.0);
    if (m.rot) w.ir = Inew;
    ++w.hits;
    ++w.walls;
    w.entry = fb;
}

constexpr int kHopWallPending = 3;

// Exit test over the three faces other than the entry face (entry >= 0),
// visited from the entry face onwards; a tie keeps the lower face index, as
// the ascending scan of exit_candidate does.
__device__ __forceinline__ void exit_candidate3(const double4& pl, int f, const Walker& w, int& fb, double& lb) {
    const double den = fma(pl.z, w.v2, fma(pl.y, w.v1, pl.x * w.v0));
    double lam = (pl.w - fma(pl.z, w.x2, fma(pl.y, w.x1, pl.x * w.x0))) / den;
    lam = lam < 0 ? 0.0 : lam;
    const bool take = (den > 0) && (fb < 0 || lam < lb || (lam == lb && f < fb));
    fb = take ? f : fb;
    lb = take ? lam : lb;
}

// With DEFER, reaching a diffuse wall stops the walker there and returns
// kHopWallPending (the re-emission is left to a later pass); the walker's
// entry holds the wall's local face.  FACE3 is for a walker that has
// entered its cell through a face (entry >= 0, as after any crossing or
// boundary event): it tests (and loads the planes of) the other three faces
// only, with the same result.
// SURF = false leaves out the surface sampling of specular faces (for a
// launch made while sampling is off: fewer live registers in the hop loop).
template <class VT, bool DEFER = false, bool FACE3 = false, bool SURF = true>
__device__ __forceinline__ int hop_once(const MeshDev& m, Walker& w, uint32_t step, RngKey key) {
    const int base = 4 * w.c;
    const int4 nb4 = *reinterpret_cast<const int4*>(m.nbr + base);
    int fb = -1;
    double lb = 0.0;
    double4 p0, p1, p2, p3;
    if (FACE3) {
        const int f1 = (w.entry + 1) & 3, f2 = (w.entry + 2) & 3, f3 = (w.entry + 3) & 3;
        p1 = m.plane[base + f1];
        p2 = m.plane[base + f2];
        p3 = m.plane[base + f3];
        exit_candidate3(p1, f1, w, fb, lb);
        exit_candidate3(p2, f2, w, fb, lb);
        exit_candidate3(p3, f3, w, fb, lb);
        // the exit face's plane in p0 (for a specular reflection)
        p0 = fb == f1 ? p1 : fb == f2 ? p2 : p3;
    } else {
        // all four planes and neighbour codes of the cell in flight at once
        p0 = m.plane[base + 0];
        p1 = m.plane[base + 1];
        p2 = m.plane[base + 2];
        p3 = m.plane[base + 3];
        exit_candidate(p0, 0, w, fb, lb);
        exit_candidate(p1, 1, w, fb, lb);
        exit_candidate(p2, 2, w, fb, lb);
        exit_candidate(p3, 3, w, fb, lb);
    }
    if (fb < 0 || lb >= w.t) {
        w.x0 = fma(w.v0, w.t, w.x0);
        w.x1 = fma(w.v1, w.t, w.x1);
        w.x2 = fma(w.v2, w.t, w.x2);
        return 0;
    }
    w.x0 = fma(w.v0, lb, w.x0);
    w.x1 = fma(w.v1, lb, w.x1);
    w.x2 = fma(w.v2, lb, w.x2);
    w.t = w.t - lb;
    ++w.nhop;
    if (w.nhop > DSMC_MAX_HOPS) return 2;
    const int code = fb == 0 ? nb4.x : fb == 1 ? nb4.y : fb == 2 ? nb4.z : nb4.w;
    if (code >= 0) {
        w.c = code >> 2;
        w.entry = code & 3;
        return -1;
    }
    const int bf = -1 - code;
    const GroupDev& g = m.groups[m.bf_group[bf]];
    if (g.kind == kBcDiffuse) {
        if (DEFER) {
            w.entry = fb;
            return kHopWallPending;
        }
        diffuse_reemit<VT>(m, w, bf, fb, step, key);
    } else if (g.kind == kBcSpecular) {
        const double4 pl = FACE3 ? p0 : fb == 0 ? p0 : fb == 1 ? p1 : fb == 2 ? p2 : p3;
        const double vn = pl.x * w.v0 + pl.y * w.v1 + pl.z * w.v2;
        const double nn = pl.x * pl.x + pl.y * pl.y + pl.z * pl.z;
        const double f2 = 2.0 * (vn / nn);
        const double a0 = w.v0, a1 = w.v1, a2 = w.v2;
        w.v0 = round_store<VT>(w.v0 - f2 * pl.x);
        w.v1 = round_store<VT>(w.v1 - f2 * pl.y);
        w.v2 = round_store<VT>(w.v2 - f2 * pl.z);
        if (SURF) surface_hit(m, bf, step, a0, a1, a2, w.v0, w.v1, w.v2, 0.0);
        ++w.walls;
        w.entry = fb;
    } else if (g.kind == kBcPeriodic) {
        w.x0 = w.x0 + g.shift[0];
        w.x1 = w.x1 + g.shift[1];
        w.x2 = w.x2 + g.shift[2];
        const int pc = m.bf_pcode[bf];
        w.c = pc >> 2;
        w.entry = pc & 3;
    } else {
        return 1;
    }
    return -1;
}

}  // namespace dsmcx
