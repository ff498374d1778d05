// Device data structures and kernel launch wrappers of the DSMC step.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"

namespace dsmcx {

constexpr double kBoltzmannDev = 1.380649e-23;
constexpr int kNMom = 13;               // S0, S1(3), S2(6), S3(3)
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanBlock = kScanThreads * kScanItems;
constexpr int kMoveBatch = 512;        // particles per wave in the move kernel
constexpr int kCollideLanes = 64;       // one wave, one lane per cell
constexpr int kCollideCap = 2048;       // particles of one 64-cell chunk staged in LDS
constexpr int kCollideCapG = 4096;      // particles of one chunk ranked in LDS (order-only variant)
constexpr int kInflowStride = 25;       // doubles per inflow face
enum { kScanPlain = 0, kScanCells = 1, kScanInject = 2, kScanInit = 3 };
enum { kFlagCapacity = 1 };
// move kernel variants (tuning choice)
enum { kMoveLane = 0, kMoveLaneW6 = 1, kMoveLaneW8 = 2, kMoveBatched = 3, kMoveDefer6 = 4, kMoveDefer8 = 5, kMoveDefer4 = 6,
       kMoveDefer5 = 7, kMoveRefill5 = 8, kMoveRefill6 = 9,
       kMovePool128 = 10, kMovePool256 = 11, kMoveCap4 = 12, kMoveCap5 = 13, kMoveCap6 = 14,
       kMoveFace3 = 15, kMoveFace3W8 = 16, kMovePersist = 17 };
enum { kCollideLds = 0, kCollideGlobal = 1, kCollideGlobal8 = 2, kCollideG3k = 3, kCollideG2k = 4 };
// sort: scatter by rank; gather (k_perm then k_gather); fused (k_perm, then
// the collide kernel gathers each chunk before colliding it; G-type collide
// schedules only, the others take the gather form); deferred (k_perm only:
// the collide kernel reaches the particles through the sorted order, and the
// next step's move reads them in that order and writes them sorted, so no
// pass of its own moves the particle store; three-face move and G-type
// collide schedules)
enum { kSortScatter = 0, kSortGather = 1, kSortFused = 2, kSortDeferred = 3 };
// how the collide kernel reaches the sorted particles: in place, gathered
// into the sorted buffer first (fused sort), or through the sorted order
enum { kGatherNone = 0, kGatherFused = 1, kGatherIndirect = 2 };

// Particle store: positions and velocities interleaved per particle (a
// scattered access then touches one cache line per quantity, not three),
// cells and ids in arrays of their own.
template <class VT>
struct PartDev {
    double* pos;      // [cap][3] positions, x y z of a particle adjacent
    VT* vel;          // [cap][3] velocities, interleaved likewise
    int32_t* cell;
    uint32_t* pid;
    double* ir;       // [cap] rotational energies (J), or null for a monatomic gas
};

// Device-resident scalars of the step (read by kernels, never by the host
// inside a step).
struct Scalars {
    int64_t np;         // particles in the sorted buffer
    int64_t n_entries;  // entries of the unsorted buffer (np + injected) to scatter
    int64_t n_steady;   // steps summed into the steady accumulator
    uint32_t step;      // current step index
    uint32_t next_pid;
    int32_t ninj;       // particles injected this step
    int32_t flags;
};

// Particles parked by the deferring move kernels (at a diffuse wall, or in
// flight after the capped number of exit tests).  The queue is split into
// kQueueParts parts; workgroup b pushes into part b % kQueueParts, whose
// counter lives on its own 256-byte line, so that the wave-aggregated
// atomics of a launch spread over many addresses instead of queueing on one.
constexpr int kQueueParts = 64;
constexpr int kQueueStride = 32;     // counters kQueueStride x 8 bytes apart
constexpr int kQueueMaxBatch = 4096; // largest particles-per-wave batch of any move kernel
// The persistent move's tile counters follow the queue counters in the same
// array, one per XCD slice, kQueueStride apart.
constexpr int kTileSlices = 8;
struct WallQueue {
    int32_t* idx;              // particle index
    double* t;                 // remaining time (negative: parked in flight)
    int32_t* meta;             // entry face | hits << 2 | hops << 12 | walls << 22
    unsigned long long* n;     // [kQueueParts * kQueueStride] entries per part
    int64_t part;              // entries per part
};
// Entries per part for a particle capacity: a part serves every
// kQueueParts-th workgroup, each of which owns at most 4 * kQueueMaxBatch
// particles, and the grids round up to 8 workgroups.
inline int64_t queue_part_size(int64_t cap) {
    return (cap + kQueueParts - 1) / kQueueParts + 2 * 4 * (int64_t)kQueueMaxBatch;
}

struct Counters {
    unsigned long long hops, walls, injected, removed, lost;
};

// Inflow faces: consts[j][25] = mean count, speed ratio a, beta, sigma,
// tangential mean (2), inward normal (3), t1 (3), t2 (3), vertices A,B,C (9),
// k T of the freestream.
struct InflowDev {
    int n;
    const int32_t* bface;   // boundary face index (generator subject)
    const int32_t* tcode;   // (tet << 2 | local face) owning the face
    const double* consts;
};

struct CollideParams {
    int nt;
    int n_ss, n_a, ewma_on;
    RngKey key;
    double FN, dt, K, ex;
    int vss;            // VSS scattering (alpha != 1); else isotropic VHS
    double inv_alpha;   // 1 / alpha
    int rot;            // rotational energy exchange (Borgnakke-Larsen) and sums
    double pinel;       // inelastic probability per partner (eq. inelastic_probability)
    double ex_bl;       // 1 / (5/2 - omega): the translational share's exponent
    double mass;        // molecular mass
    double* racc;       // [4][nt] steady rotational sums (sum I_r, sum v_i I_r), or null
    double* rewma;      // [4][nt] moving average of the rotational sums, or null
    double* rinst;      // [4][nt] rotational sums of the step alone, or null
    const double* vol;
    double* smax;
    int32_t* ncand;
    int32_t* nacc;
    double* acc;        // [13][nt] steady sums
    double* ewma;       // [13][nt] moving average
    double* inst;       // [13][nt] sums of the step alone, or null
    int32_t* ewma_m;    // [nt] samples seen
    const uint8_t* local_acc;
    const int32_t* orig;  // [nt] caller's cell id (generator subject)
    const int32_t* cell_case;  // batch: [nt] case of each cell, or null
    const CaseDev* cases;
};

void launch_begin(hipStream_t s, int32_t* counts, int nt, Scalars* sc, int do_sample, int n_ss,
                  unsigned long long* queue_n);
void launch_init_count(hipStream_t s, const double* vol, const int32_t* orig, int nt, double n0, double FN,
                       RngKey key, int32_t* counts, int32_t* counts_orig, const int32_t* cell_case,
                       const CaseDev* cases);
template <class VT>
void launch_init_fill(hipStream_t s, const int4* tv, const double* xyz, int nt, const int32_t* offsets,
                      const int32_t* orig, const int32_t* pid_base, PartDev<VT> p, RngKey key, double sig,
                      const double* u0, int64_t cap, Scalars* sc, const int32_t* cell_case, const CaseDev* cases,
                      double T0);
// batch: case-local particle ids (prefix minus the case's first prefix) and per-case (sigma c)_max
void launch_batch_pid_base(hipStream_t s, const int32_t* prefix, const int32_t* case_first, const int32_t* case_of_orig,
                           int nt, int32_t* out);
void launch_batch_smax(hipStream_t s, const int32_t* cell_case, const CaseDev* cases, int nt, double* smax);
template <class VT>
// With gperm (deferred sort, three-face schedule): slot k of p receives the
// moved particle gperm[k] of src; p.cell already holds the slots' cells.
void launch_move(hipStream_t s, const MeshDev& m, PartDev<VT> p, const Scalars* sc, int32_t* counts,
                 uint32_t* rank, Counters* ctr, RngKey key, double dt, int64_t np_bound, int variant, int batch,
                 WallQueue wq, PartDev<VT> src = PartDev<VT>{}, const int32_t* gperm = nullptr);
template <class VT>
void launch_move_walls(hipStream_t s, const MeshDev& m, PartDev<VT> p, const Scalars* sc, int32_t* counts,
                       uint32_t* rank, Counters* ctr, RngKey key, WallQueue wq);
bool move_parks_walls(int variant);
template <class VT>
void launch_gather(hipStream_t s, PartDev<VT> src, PartDev<VT> dst, const Scalars* sc, const int32_t* perm,
                   int64_t bound);
void launch_perm_identity(hipStream_t s, const int32_t* cell, const Scalars* sc, int32_t* perm, int32_t* dst_cell,
                          int64_t bound);
void launch_count(hipStream_t s, const int32_t* cell, const Scalars* sc, int32_t* counts, uint32_t* rank,
                  int64_t np_bound);
void launch_inject_count(hipStream_t s, const InflowDev& in, const Scalars* sc, RngKey key, int32_t* fcount);
template <class VT>
void launch_inject_emit(hipStream_t s, const MeshDev& m, const InflowDev& in, PartDev<VT> p, Scalars* sc,
                        const int32_t* foff, int32_t* counts, uint32_t* rank, Counters* ctr, RngKey key,
                        double dt, int64_t cap, int64_t max_inject);
void launch_scan(hipStream_t s, const int32_t* in, int64_t n, int32_t* out, int32_t* blocksums, Scalars* sc,
                 int mode);
template <class VT>
void launch_scatter(hipStream_t s, PartDev<VT> src, PartDev<VT> dst, const Scalars* sc, const int32_t* offsets,
                    const uint32_t* rank, int64_t bound, int64_t cap, int32_t* perm, int variant);
// gmode kGatherFused: p's slots are first gathered from src through
// sortperm; kGatherIndirect: slot d of the sorted order is particle
// sortperm[d] of p, with its cell in src.cell[d] (both G-type schedules only:
// collide_fuses_gather).
template <class VT>
void launch_collide_sample(hipStream_t s, PartDev<VT> p, const int32_t* offsets, const CollideParams& cp,
                           const Scalars* sc, int32_t* perm, int do_collide, int do_sample, int variant, int gmode,
                           PartDev<VT> src, const int32_t* sortperm);
bool collide_fuses_gather(int variant);
void launch_fields(hipStream_t s, const double* sums, int nt, double ns, double mass, double FN,
                   const double* vol, const int32_t* orig, double* out, const int32_t* cell_case,
                   const CaseDev* cases);
void launch_philox(hipStream_t s, const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out, int64_t n);
void launch_copy(hipStream_t s, const void* src, void* dst, size_t bytes);
void launch_line_reads(hipStream_t s, const void* table, uint32_t line_mask, int iters, int share, int blocks,
                       void* sink);
void launch_fill_i32(hipStream_t s, int32_t* p, int32_t v, int64_t n);
void launch_fill_f64(hipStream_t s, double* p, double v, int64_t n);

}  // namespace dsmcx
