// HIP kernels of the DSMC step for gfx950 (wave64, 256 CUs on 8 XCDs).
//
// Per step (paper section 2.1: move, then select and collide pairs per
// cell; sampling per eq. dsmc_temperatures after the collisions):
//   k_begin          clear cell histogram, advance the device step counter
//   k_move           face-to-face tracking of every particle + histogram
//   k_inject_*       freestream particles on inflow faces (count, emit+trace)
//   k_scan_*         exclusive prefix of the cell histogram -> cell offsets
//   k_scatter        counting-sort scatter into the other particle buffer
//   k_collide_sample one lane per cell: rank the cell's particles by pid,
//                    NTC/VHS collisions and FP64 moment sums, in LDS
#include "kernels.h"

namespace dsmcx {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
// Workgroups are dispatched round-robin over the 8 XCDs; remap so that each
// XCD walks one contiguous slice of the particle range (its L2 then holds
// the mesh neighbourhood of that slice).  gridDim.x is a multiple of 8.
__device__ __forceinline__ int64_t xcd_block() {
    const int64_t per = gridDim.x >> 3;
    return (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum four counters over the block and add them to global counters.
__device__ __forceinline__ void block_counters(int a, int b, int c, int d, unsigned long long* ga,
                                               unsigned long long* gb, unsigned long long* gc,
                                               unsigned long long* gd) {
    __shared__ int red[4][16];
    a = wave_sum(a); b = wave_sum(b); c = wave_sum(c); d = wave_sum(d);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { red[0][w] = a; red[1][w] = b; red[2][w] = c; red[3][w] = d; }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        int s[4] = {0, 0, 0, 0};
        for (int k = 0; k < nw; ++k)
            for (int j = 0; j < 4; ++j) s[j] += red[j][k];
        if (s[0]) atomicAdd(ga, (unsigned long long)s[0]);
        if (s[1]) atomicAdd(gb, (unsigned long long)s[1]);
        if (s[2]) atomicAdd(gc, (unsigned long long)s[2]);
        if (s[3]) atomicAdd(gd, (unsigned long long)s[3]);
    }
}

// Slot of a particle in its cell's histogram bin, aggregated over the
// workgroup: the lanes' destination cells go into an LDS hash table
// (open addressing, twice as many entries as lanes, so a probe always ends),
// each lane takes its rank among the workgroup's particles of that cell
// from an LDS counter, then one global atomic per distinct cell reserves the
// workgroup's run in the bin.  After a step at a mean free path of a few
// cells a wave's 64 particles land in about 44 different cells, a
// workgroup's 256 in about 110, so this issues half the global atomics of
// the per-wave grouping.  Every lane of the workgroup must call it (it
// synchronises the workgroup); blockDim.x <= kBinLanes.
constexpr int kBinLanes = 256;
constexpr int kBinTable = 2 * kBinLanes;
__device__ __forceinline__ uint32_t block_bin_slot(int32_t* counts, int cell, bool active) {
    __shared__ int hkey[kBinTable];
    __shared__ int hcnt[kBinTable];
    const int t = threadIdx.x;
    for (int e = t; e < kBinTable; e += blockDim.x) {
        hkey[e] = -1;
        hcnt[e] = 0;
    }
    __syncthreads();
    int h = 0, local = 0;
    if (active) {
        h = (int)(((uint32_t)cell * 2654435761u) >> 23);  // 9 bits: kBinTable = 512
        for (int probe = 0; probe < kBinTable; ++probe) {
            const int old = atomicCAS(&hkey[h], -1, cell);
            if (old == -1 || old == cell) break;
            h = (h + 1) & (kBinTable - 1);
        }
        local = atomicAdd(&hcnt[h], 1);
    }
    __syncthreads();
    // hcnt now holds each cell's count; the owner of an entry replaces it
    // by the bin offset the global atomic returns
    for (int e = t; e < kBinTable; e += blockDim.x) {
        const int key = hkey[e];
        if (key >= 0) hcnt[e] = atomicAdd(&counts[key], hcnt[e]);
    }
    __syncthreads();
    return active ? (uint32_t)(hcnt[h] + local) : 0u;
}

// Wave-aggregated push of the lanes with `park` set into a part of the
// parked-particle queue (one atomic per wave); by default the part of this
// workgroup.
__device__ __forceinline__ void queue_push(const WallQueue& q, bool park, int64_t i, double t, int meta,
                                           int part = -1) {
    const uint64_t pm = __ballot(park);
    if (!pm) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((unsigned long long)pm) - 1;
    if (part < 0) part = (int)(blockIdx.x % kQueueParts);
    int64_t base = 0;
    if (lane == leader)
        base = (int64_t)atomicAdd(q.n + (size_t)part * kQueueStride, (unsigned long long)__popcll(pm));
    base = __shfl(base, leader, 64);
    if (park) {
        const int64_t slot = part * q.part + base + __popcll(pm & ((1ull << lane) - 1ull));
        q.idx[slot] = (int32_t)i;
        q.t[slot] = t;
        q.meta[slot] = meta;
    }
}

// ---------------------------------------------------------------------------
// step bookkeeping
// ---------------------------------------------------------------------------
__global__ void k_begin(int32_t* counts, int nt, Scalars* sc, int do_sample, int n_ss, unsigned long long* queue_n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= nt) counts[i] = 0;
    if (i < kQueueParts + kTileSlices) queue_n[i * kQueueStride] = 0ull;
    if (i == 0) {
        const uint32_t s = sc->step + 1;
        sc->step = s;
        sc->ninj = 0;
        if (do_sample && (int64_t)s > (int64_t)n_ss) sc->n_steady += 1;
    }
}

// ---------------------------------------------------------------------------
// initial fill
// ---------------------------------------------------------------------------
__global__ void k_init_count(const double* vol, const int32_t* orig, int nt, double n0, double FN, RngKey key,
                             int32_t* counts, int32_t* counts_orig, const int32_t* cell_case, const CaseDev* cases) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    const int o = orig[t];
    int subj = o;
    if (cell_case) {
        const CaseDev& cs = cases[cell_case[t]];
        n0 = cs.n0;
        FN = cs.FN;
        key.k0 = cs.k0;
        key.k1 = cs.k1;
        subj = o - cs.cell0;
    }
    const double mean = (n0 * vol[t]) / FN;
    const Rand4 r = draw(key, (uint32_t)subj, 0u, kPurposeInitCount, 0);
    const int32_t cnt = (int32_t)floor(mean + u01(r.w[0], r.w[1]));
    counts[t] = cnt;
    counts_orig[o] = cnt;
}

template <class VT>
__global__ void k_init_fill(const int4* tv, const double* xyz, int nt, const int32_t* offsets,
                            const int32_t* orig, const int32_t* pid_base, PartDev<VT> p, RngKey key, double sig,
                            double u0x, double u0y, double u0z, int64_t cap, Scalars* sc, const int32_t* cell_case,
                            const CaseDev* cases, double T0) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    if (cell_case) {
        const CaseDev& cs = cases[cell_case[t]];
        key.k0 = cs.k0;
        key.k1 = cs.k1;
        T0 = cs.T0;
        sig = cs.sig;
        u0x = cs.u0[0];
        u0y = cs.u0[1];
        u0z = cs.u0[2];
    }
    const int4 q = tv[t];
    const double* A = xyz + 3 * (size_t)q.x;
    const double* B = xyz + 3 * (size_t)q.y;
    const double* C = xyz + 3 * (size_t)q.z;
    const double* D = xyz + 3 * (size_t)q.w;
    const int64_t a = offsets[t], b = offsets[t + 1];
    if (b > cap) {
        if (t == 0) atomicOr(&sc->flags, kFlagCapacity);
        return;
    }
    const int64_t pb = pid_base[orig[t]];
    for (int64_t k = a; k < b; ++k) {
        const uint32_t id = (uint32_t)(pb + (k - a));
        double u[8];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const Rand4 r = draw(key, id, 0u, kPurposeInit, (uint64_t)j);
            u[2 * j] = u01(r.w[0], r.w[1]);
            u[2 * j + 1] = u01(r.w[2], r.w[3]);
        }
        double s1 = u[0], s2 = u[1], s3 = u[2], tmp;
        if (s1 > s2) { tmp = s1; s1 = s2; s2 = tmp; }
        if (s2 > s3) { tmp = s2; s2 = s3; s3 = tmp; }
        if (s1 > s2) { tmp = s1; s1 = s2; s2 = tmp; }
        const double w0 = s1, w1 = s2 - s1, w2 = s3 - s2, w3 = 1.0 - s3;
        p.pos[3 * k] = ((w0 * A[0] + w1 * B[0]) + w2 * C[0]) + w3 * D[0];
        p.pos[3 * k + 1] = ((w0 * A[1] + w1 * B[1]) + w2 * C[1]) + w3 * D[1];
        p.pos[3 * k + 2] = ((w0 * A[2] + w1 * B[2]) + w2 * C[2]) + w3 * D[2];
        double g1, g2, g3, g4;
        box_muller(u[3], u[4], g1, g2);
        box_muller(u[5], u[6], g3, g4);
        p.vel[3 * k] = (VT)(u0x + sig * g1);
        p.vel[3 * k + 1] = (VT)(u0y + sig * g2);
        p.vel[3 * k + 2] = (VT)(u0z + sig * g3);
        p.cell[k] = t;
        p.pid[k] = id;
        if (p.ir) {
            // two rotational degrees of freedom: exponential with mean k T0
            const Rand4 r = draw(key, id, 0u, kPurposeInit, 4);
            p.ir[k] = -(kBoltzmannDev * T0) * log(u01(r.w[0], r.w[1]));
        }
    }
}

// Batch: particle ids restart at 0 in every case (prefix of the counts in
// the caller's numbering minus the prefix at the case's first cell).
__global__ void k_batch_pid_base(const int32_t* prefix, const int32_t* case_first, const int32_t* case_of_orig, int nt,
                                 int32_t* out) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= nt) return;
    out[o] = prefix[o] - prefix[case_first[case_of_orig[o]]];
}

__global__ void k_batch_smax(const int32_t* cell_case, const CaseDev* cases, int nt, double* smax) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < nt) smax[c] = cases[cell_case[c]].smax0;
}

// ---------------------------------------------------------------------------
// move
// ---------------------------------------------------------------------------
// One particle per lane, tracked to the end of its step.  WPE bounds the
// register budget (waves per SIMD) the compiler must fit.
template <class VT, int WPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void k_move_lane(MeshDev m, PartDev<VT> p, const Scalars* sc,
                                                      int32_t* counts, uint32_t* rank, Counters* ctr,
                                                      RngKey key, double dt) {
    const int64_t i = xcd_block() * 256 + threadIdx.x;
    const int64_t n = sc->np;
    int hops = 0, walls = 0, rem = 0, lost = 0, dest = -1;
    if (i < n) {
        Walker w;
        w.x0 = p.pos[3 * i]; w.x1 = p.pos[3 * i + 1]; w.x2 = p.pos[3 * i + 2];
        w.v0 = (double)p.vel[3 * i]; w.v1 = (double)p.vel[3 * i + 1]; w.v2 = (double)p.vel[3 * i + 2];
        w.c = p.cell[i]; w.pid = p.pid[i];
        RngKey kp = key;
        double dtp = dt;
        case_params(m.cell_case, m.cases, w.c, kp, dtp);
        w.t = dtp;
        w.entry = -1; w.nhop = 0; w.hits = 0; w.walls = 0;
        const uint32_t step = sc->step;
        int st;
        do {
            st = hop_once<VT>(m, w, step, kp);
        } while (st < 0);
        hops = w.nhop;
        walls = w.walls;
        p.pos[3 * i] = w.x0; p.pos[3 * i + 1] = w.x1; p.pos[3 * i + 2] = w.x2;
        if (w.walls) {
            p.vel[3 * i] = (VT)w.v0; p.vel[3 * i + 1] = (VT)w.v1; p.vel[3 * i + 2] = (VT)w.v2;
        }
        if (st == 0) {
            p.cell[i] = w.c;
            dest = w.c;
        } else {
            p.cell[i] = -1;
            rem = st == 1;
            lost = st == 2;
        }
    }
    const uint32_t slot = bin_slot(counts, dest, dest >= 0);
    if (dest >= 0) rank[i] = slot;
    block_counters(hops, walls, rem, lost, &ctr->hops, &ctr->walls, &ctr->removed, &ctr->lost);
}

// One particle per lane; a particle that reaches a diffuse wall is parked at
// the wall (position, cell and remaining time) in a queue, so the costly
// re-emission sampling does not diverge the hop loop.  k_move_walls then
// re-emits the queued particles and finishes their step.  With CAP > 0 a
// lane also stops after CAP exit tests and parks its particle in flight
// (velocity written back, remaining time queued with a negative sign): a
// wave then runs at most CAP iterations instead of the largest hop count of
// its 64 particles, and the few long tracks finish in k_move_walls on
// compacted waves.
// With GATHER the kernel also does the previous step's sort: lane i takes
// slot i of that sorted order, i.e. particle gperm[i] of src (its cell
// already in p.cell[i], written by the sort), and writes the moved particle
// to slot i of p, so the sorted buffer is never written separately.
template <class VT, int WPE, int CAP, bool FACE3 = false, bool SURF = true, bool GATHER = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void k_move_defer(
    MeshDev m, PartDev<VT> p, Scalars* sc, int32_t* counts, uint32_t* rank, Counters* ctr, RngKey key,
    double dt, WallQueue q, PartDev<VT> src, const int32_t* gperm) {
    const int64_t i = xcd_block() * 256 + threadIdx.x;
    const int64_t n = sc->np;
    // A workgroup past the last particle leaves at once (the grid of a
    // context with inflow covers the whole store); the test is uniform over
    // the workgroup, so no lane skips a barrier the others reach.
    if (xcd_block() * 256 >= n) return;
    int hops = 0, walls = 0, rem = 0, lost = 0, dest = -1;
    bool park = false;
    Walker w{};
    if (i < n) {
        if (GATHER) {
            const int64_t j = gperm[i];
            w.x0 = src.pos[3 * j]; w.x1 = src.pos[3 * j + 1]; w.x2 = src.pos[3 * j + 2];
            w.v0 = (double)src.vel[3 * j]; w.v1 = (double)src.vel[3 * j + 1]; w.v2 = (double)src.vel[3 * j + 2];
            w.c = p.cell[i]; w.pid = src.pid[j];
            if (src.ir) p.ir[i] = src.ir[j];
            p.pid[i] = w.pid;
        } else {
            w.x0 = p.pos[3 * i]; w.x1 = p.pos[3 * i + 1]; w.x2 = p.pos[3 * i + 2];
            w.v0 = (double)p.vel[3 * i]; w.v1 = (double)p.vel[3 * i + 1]; w.v2 = (double)p.vel[3 * i + 2];
            w.c = p.cell[i]; w.pid = p.pid[i];
        }
        RngKey kp = key;
        double dtp = dt;
        case_params(m.cell_case, m.cases, w.c, kp, dtp);
        w.t = dtp;
        w.entry = -1; w.nhop = 0; w.hits = 0; w.walls = 0;
        const uint32_t step = sc->step;
        // the first test (entry face unknown) over all four faces; with
        // FACE3 the later ones over the three faces other than the entry
        int st = hop_once<VT, true, false, SURF>(m, w, step, kp);
        for (int it = 1; st < 0 && (CAP == 0 || it < CAP); ++it)
            st = FACE3 ? hop_once<VT, true, true, SURF>(m, w, step, kp) : hop_once<VT, true, false, SURF>(m, w, step, kp);
        p.pos[3 * i] = w.x0; p.pos[3 * i + 1] = w.x1; p.pos[3 * i + 2] = w.x2;
        if (st == kHopWallPending) {
            park = true;
            p.cell[i] = w.c;
            // the velocity it reaches the wall with (surface sampling reads it)
            if (GATHER || w.walls) {
                p.vel[3 * i] = (VT)w.v0; p.vel[3 * i + 1] = (VT)w.v1; p.vel[3 * i + 2] = (VT)w.v2;
            }
        } else if (CAP > 0 && st < 0) {
            // in flight after CAP tests: the queued time carries a negative
            // sign (a parked particle always has time left, t > 0)
            park = true;
            p.cell[i] = w.c;
            p.vel[3 * i] = (VT)w.v0; p.vel[3 * i + 1] = (VT)w.v1; p.vel[3 * i + 2] = (VT)w.v2;
            w.t = -w.t;
        } else {
            hops = w.nhop;
            walls = w.walls;
            if (GATHER || w.walls) {
                p.vel[3 * i] = (VT)w.v0; p.vel[3 * i + 1] = (VT)w.v1; p.vel[3 * i + 2] = (VT)w.v2;
            }
            if (st == 0) {
                p.cell[i] = w.c;
                dest = w.c;
            } else {
                p.cell[i] = -1;
                rem = st == 1;
                lost = st == 2;
            }
        }
    }
    queue_push(q, park, i, w.t, (w.entry & 3) | (w.hits << 2) | (w.nhop << 12) | (w.walls << 22));
    {
        const uint32_t slot = block_bin_slot(counts, dest, dest >= 0);
        if (dest >= 0) rank[i] = slot;
    }
    block_counters(hops, walls, rem, lost, &ctr->hops, &ctr->walls, &ctr->removed, &ctr->lost);
}

// Persistent move with a device work queue of tiles.  A fixed grid (a whole
// number of workgroups per XCD, as many as the CUs hold at once) pulls
// tiles of 256 consecutive particles.  The tiles are dealt out in
// kTileSlices contiguous slices, one per XCD, each with its own counter on
// its own line; a workgroup takes tiles from its XCD's slice and, once that
// slice is empty, from the others in turn, so that each XCD's L2 keeps the
// mesh neighbourhood of its slice while the last tiles balance the load.
// Per particle the work is that of k_move_defer with FACE3; a tile's parked
// particles go to the queue part of its tile index, as those of a
// non-persistent workgroup of that index would.  The grid does not depend
// on the particle count (the tile count is read from the device), so a
// captured graph stays valid as the count changes.  Every workgroup leaves
// once all slice counters have passed their slice's end.
template <class VT, bool SURF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_move_persist(
    MeshDev m, PartDev<VT> p, Scalars* sc, int32_t* counts, uint32_t* rank, Counters* ctr, RngKey key,
    double dt, WallQueue q) {
    __shared__ int64_t s_tile;
    const int64_t n = sc->np;
    const int64_t ntiles = (n + 255) / 256;
    const uint32_t step = sc->step;
    unsigned long long* tile_ctr = q.n + (size_t)kQueueParts * kQueueStride;
    const int home = (int)(blockIdx.x % kTileSlices);
    int hops = 0, walls = 0, rem = 0, lost = 0;
    for (int k = 0; k < kTileSlices; ++k) {
        const int sl = (home + k) % kTileSlices;
        const int64_t lo = ntiles * sl / kTileSlices, hi = ntiles * (sl + 1) / kTileSlices;
        for (;;) {
            if (threadIdx.x == 0) {
                const int64_t t = lo + (int64_t)atomicAdd(tile_ctr + (size_t)sl * kQueueStride, 1ull);
                s_tile = t < hi ? t : -1;
            }
            __syncthreads();
            const int64_t tile = s_tile;
            __syncthreads();
            if (tile < 0) break;
            const int64_t i = tile * 256 + threadIdx.x;
            int dest = -1;
            bool park = false;
            Walker w{};
            if (i < n) {
                w.x0 = p.pos[3 * i]; w.x1 = p.pos[3 * i + 1]; w.x2 = p.pos[3 * i + 2];
                w.v0 = (double)p.vel[3 * i]; w.v1 = (double)p.vel[3 * i + 1]; w.v2 = (double)p.vel[3 * i + 2];
                w.c = p.cell[i]; w.pid = p.pid[i];
                RngKey kp = key;
                double dtp = dt;
                case_params(m.cell_case, m.cases, w.c, kp, dtp);
                w.t = dtp;
                w.entry = -1; w.nhop = 0; w.hits = 0; w.walls = 0;
                int st = hop_once<VT, true, false, SURF>(m, w, step, kp);
                while (st < 0) st = hop_once<VT, true, true, SURF>(m, w, step, kp);
                p.pos[3 * i] = w.x0; p.pos[3 * i + 1] = w.x1; p.pos[3 * i + 2] = w.x2;
                if (st == kHopWallPending) {
                    park = true;
                    p.cell[i] = w.c;
                    if (w.walls) {
                        p.vel[3 * i] = (VT)w.v0; p.vel[3 * i + 1] = (VT)w.v1; p.vel[3 * i + 2] = (VT)w.v2;
                    }
                } else {
                    hops += w.nhop;
                    walls += w.walls;
                    if (w.walls) {
                        p.vel[3 * i] = (VT)w.v0; p.vel[3 * i + 1] = (VT)w.v1; p.vel[3 * i + 2] = (VT)w.v2;
                    }
                    if (st == 0) {
                        p.cell[i] = w.c;
                        dest = w.c;
                    } else {
                        p.cell[i] = -1;
                        rem += st == 1;
                        lost += st == 2;
                    }
                }
            }
            queue_push(q, park, i, w.t, (w.entry & 3) | (w.hits << 2) | (w.nhop << 12) | (w.walls << 22),
                       (int)(tile % kQueueParts));
            // workgroup-uniform: every lane reaches it once per tile
            const uint32_t slot = block_bin_slot(counts, dest, dest >= 0);
            if (dest >= 0) rank[i] = slot;
        }
    }
    block_counters(hops, walls, rem, lost, &ctr->hops, &ctr->walls, &ctr->removed, &ctr->lost);
}

// Batched move with lane refill and parked diffuse walls: each wave owns
// `batch` consecutive particles; a lane whose particle is done (or parked)
// takes the next untouched particle of the batch.
template <class VT, int WPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void k_move_refill(
    MeshDev m, PartDev<VT> p, Scalars* sc, int32_t* counts, uint32_t* rank, Counters* ctr, RngKey key,
    double dt, WallQueue q, int batch) {
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1ull;
    const int64_t wv = xcd_block() * 4 + (threadIdx.x >> 6);
    const int64_t n = sc->np;
    const int64_t lo = wv * (int64_t)batch;
    const int64_t hi = min(lo + (int64_t)batch, n);
    const uint32_t step = sc->step;
    int hops = 0, walls = 0, rem = 0, lost = 0;
    int64_t next = lo + 64;
    int64_t i = lo + lane;
    bool active = i < hi;
    Walker w;
    w.x0 = w.x1 = w.x2 = w.v0 = w.v1 = w.v2 = w.t = 0.0;
    w.c = 0; w.entry = -1; w.nhop = 0; w.hits = 0; w.walls = 0; w.pid = 0;
    if (active) {
        w.x0 = p.pos[3 * i]; w.x1 = p.pos[3 * i + 1]; w.x2 = p.pos[3 * i + 2];
        w.v0 = (double)p.vel[3 * i]; w.v1 = (double)p.vel[3 * i + 1]; w.v2 = (double)p.vel[3 * i + 2];
        w.c = p.cell[i]; w.pid = p.pid[i]; w.t = dt;
    }
    while (__ballot(active) != 0ull) {
        int st = -1;
        if (active) st = hop_once<VT, true>(m, w, step, key);
        const bool done = active && st >= 0;
        const bool park = done && st == kHopWallPending;
        if (done) {
            p.pos[3 * i] = w.x0; p.pos[3 * i + 1] = w.x1; p.pos[3 * i + 2] = w.x2;
            if (park) {
                p.cell[i] = w.c;
                if (w.walls) {
                    p.vel[3 * i] = (VT)w.v0; p.vel[3 * i + 1] = (VT)w.v1; p.vel[3 * i + 2] = (VT)w.v2;
                }
            } else {
                if (w.walls) {
                    p.vel[3 * i] = (VT)w.v0; p.vel[3 * i + 1] = (VT)w.v1; p.vel[3 * i + 2] = (VT)w.v2;
                }
                if (st == 0) {
                    p.cell[i] = w.c;
                    rank[i] = (uint32_t)atomicAdd(&counts[w.c], 1);
                } else {
                    p.cell[i] = -1;
                    rem += st == 1;
                    lost += st == 2;
                }
                hops += w.nhop;
                walls += w.walls;
            }
        }
        queue_push(q, park, i, w.t, (w.entry & 3) | (w.hits << 2) | (w.nhop << 12) | (w.walls << 22));
        const uint64_t dm = __ballot(done);
        if (done) {
            const int64_t ni = next + __popcll(dm & below);
            active = ni < hi;
            if (active) {
                i = ni;
                w.x0 = p.pos[3 * i]; w.x1 = p.pos[3 * i + 1]; w.x2 = p.pos[3 * i + 2];
                w.v0 = (double)p.vel[3 * i]; w.v1 = (double)p.vel[3 * i + 1]; w.v2 = (double)p.vel[3 * i + 2];
                w.c = p.cell[i]; w.pid = p.pid[i]; w.t = dt;
                w.entry = -1; w.nhop = 0; w.hits = 0; w.walls = 0;
            }
        }
        next += __popcll(dm);
    }
    block_counters(hops, walls, rem, lost, &ctr->hops, &ctr->walls, &ctr->removed, &ctr->lost);
}

// Pooled move: each wave stages its batch of POOL consecutive particles in
// LDS with one coalesced load; its lanes take particles from the pool as they
// finish (so lanes stay busy although hop counts differ), leave the results
// in the pool, and the wave writes the pool back, with the histogram
// atomics, in one coalesced pass at the end.  Diffuse walls are parked for
// k_move_walls.
template <class VT, int WPE, int POOL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void k_move_pool(
    MeshDev m, PartDev<VT> p, Scalars* sc, int32_t* counts, uint32_t* rank, Counters* ctr, RngKey key,
    double dt, WallQueue q) {
    __shared__ double sx[4][POOL], sy[4][POOL], sz[4][POOL];
    __shared__ VT svx[4][POOL], svy[4][POOL], svz[4][POOL];
    __shared__ int32_t scell[4][POOL];
    __shared__ uint32_t spid[4][POOL];
    __shared__ uint8_t sstate[4][POOL];   // bit0: velocity changed, bit1: parked
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    const uint64_t below = (1ull << lane) - 1ull;
    const int64_t wv = xcd_block() * 4 + wid;
    const int64_t n = sc->np;
    const int64_t lo = wv * (int64_t)POOL;
    const int cnt = (int)max((int64_t)0, min((int64_t)POOL, n - lo));
    for (int k = lane; k < cnt; k += 64) {
        sx[wid][k] = p.pos[3 * (lo + k)]; sy[wid][k] = p.pos[3 * (lo + k) + 1]; sz[wid][k] = p.pos[3 * (lo + k) + 2];
        svx[wid][k] = p.vel[3 * (lo + k)]; svy[wid][k] = p.vel[3 * (lo + k) + 1]; svz[wid][k] = p.vel[3 * (lo + k) + 2];
        scell[wid][k] = p.cell[lo + k]; spid[wid][k] = p.pid[lo + k];
    }
    __syncthreads();
    const uint32_t step = sc->step;
    int hops = 0, walls = 0, rem = 0, lost = 0;
    int next = 64;
    int j = lane;
    bool active = j < cnt;
    Walker w;
    w.x0 = w.x1 = w.x2 = w.v0 = w.v1 = w.v2 = w.t = 0.0;
    w.c = 0; w.entry = -1; w.nhop = 0; w.hits = 0; w.walls = 0; w.pid = 0;
    if (active) {
        w.x0 = sx[wid][j]; w.x1 = sy[wid][j]; w.x2 = sz[wid][j];
        w.v0 = (double)svx[wid][j]; w.v1 = (double)svy[wid][j]; w.v2 = (double)svz[wid][j];
        w.c = scell[wid][j]; w.pid = spid[wid][j]; w.t = dt;
    }
    while (__ballot(active) != 0ull) {
        int st = -1;
        if (active) st = hop_once<VT, true>(m, w, step, key);
        const bool done = active && st >= 0;
        const bool park = done && st == kHopWallPending;
        if (done) {
            sx[wid][j] = w.x0; sy[wid][j] = w.x1; sz[wid][j] = w.x2;
            uint8_t flags = park ? 2 : 0;
            if (w.walls) {
                svx[wid][j] = (VT)w.v0; svy[wid][j] = (VT)w.v1; svz[wid][j] = (VT)w.v2;
                flags |= 1;
            }
            if (!park) {
                rem += st == 1;
                lost += st == 2;
                hops += w.nhop;
                walls += w.walls;
            }
            scell[wid][j] = (st == 0 || park) ? w.c : -1;
            sstate[wid][j] = flags;
        }
        queue_push(q, park, lo + j, w.t, (w.entry & 3) | (w.hits << 2) | (w.nhop << 12) | (w.walls << 22));
        const uint64_t dm = __ballot(done);
        if (done) {
            const int nj = next + __popcll(dm & below);
            active = nj < cnt;
            if (active) {
                j = nj;
                w.x0 = sx[wid][j]; w.x1 = sy[wid][j]; w.x2 = sz[wid][j];
                w.v0 = (double)svx[wid][j]; w.v1 = (double)svy[wid][j]; w.v2 = (double)svz[wid][j];
                w.c = scell[wid][j]; w.pid = spid[wid][j]; w.t = dt;
                w.entry = -1; w.nhop = 0; w.hits = 0; w.walls = 0;
            }
        }
        next += __popcll(dm);
    }
    // write the pool back: positions, changed velocities, cells, ranks
    for (int k = lane; k < cnt; k += 64) {
        const int64_t i = lo + k;
        const uint8_t f = sstate[wid][k];
        const int cc = scell[wid][k];
        p.pos[3 * i] = sx[wid][k]; p.pos[3 * i + 1] = sy[wid][k]; p.pos[3 * i + 2] = sz[wid][k];
        if (f & 1) {
            p.vel[3 * i] = svx[wid][k]; p.vel[3 * i + 1] = svy[wid][k]; p.vel[3 * i + 2] = svz[wid][k];
        }
        p.cell[i] = cc;
        if (!(f & 2) && cc >= 0) rank[i] = (uint32_t)atomicAdd(&counts[cc], 1);
    }
    block_counters(hops, walls, rem, lost, &ctr->hops, &ctr->walls, &ctr->removed, &ctr->lost);
}

// Takes queue entry e into the lane's walker: a particle parked at a diffuse
// wall is re-emitted there, one parked in flight resumes with its velocity.
template <class VT>
__device__ __forceinline__ int64_t queue_take(const MeshDev& m, const PartDev<VT>& p, const WallQueue& q, int64_t e,
                                              uint32_t step, RngKey key, Walker& w, RngKey& kp) {
    const int64_t i = q.idx[e];
    const int meta = q.meta[e];
    const double tq = q.t[e];
    w.x0 = p.pos[3 * i]; w.x1 = p.pos[3 * i + 1]; w.x2 = p.pos[3 * i + 2];
    w.c = p.cell[i]; w.pid = p.pid[i]; w.t = tq < 0 ? -tq : tq;
    w.entry = meta & 3; w.hits = (meta >> 2) & 1023; w.nhop = (meta >> 12) & 1023; w.walls = (meta >> 22) & 1023;
    if (m.rot) w.ir = p.ir[i];
    kp = key;
    double dtp = 0.0;
    case_params(m.cell_case, m.cases, w.c, kp, dtp);
    // a walker parked in flight carries a negative time; one parked at a
    // diffuse wall entered through a boundary face.  Both tests are made:
    // a non-finite time (a particle whose position lies in no cell) has no
    // usable sign, and only a boundary face may be re-emitted from.
    const int code = m.nbr[4 * w.c + w.entry];
    if (tq < 0 || code >= 0) {
        w.v0 = (double)p.vel[3 * i]; w.v1 = (double)p.vel[3 * i + 1]; w.v2 = (double)p.vel[3 * i + 2];
    } else {
        // surface sampling needs the velocity the particle reached the wall with
        if (m.surf) {
            w.v0 = (double)p.vel[3 * i]; w.v1 = (double)p.vel[3 * i + 1]; w.v2 = (double)p.vel[3 * i + 2];
        }
        diffuse_reemit<VT>(m, w, -1 - code, w.entry, step, kp);
    }
    return i;
}

// Finishes the step of the parked particles, one queue entry per lane at a
// time.  Workgroups take the queue parts round-robin (gridDim.x is a
// multiple of kQueueParts) and stride through their part.  (Refilling lanes
// from the queue as their particles finish was measured slower: the refill
// brings the scattered loads and the wall re-emission into every pass of
// the hop loop.)
template <class VT>
__global__ __launch_bounds__(256) void k_move_walls(MeshDev m, PartDev<VT> p, const Scalars* sc, int32_t* counts,
                                                   uint32_t* rank, Counters* ctr, RngKey key, WallQueue q) {
    const int part = (int)(blockIdx.x % kQueueParts);
    const int64_t nq = (int64_t)q.n[(size_t)part * kQueueStride];
    const int64_t stride = (int64_t)(gridDim.x / kQueueParts) * blockDim.x;
    const uint32_t step = sc->step;
    int hops = 0, walls = 0, rem = 0, lost = 0;
    for (int64_t k = (int64_t)(blockIdx.x / kQueueParts) * blockDim.x + threadIdx.x; k < nq; k += stride) {
        Walker w;
        RngKey kp;
        const int64_t i = queue_take<VT>(m, p, q, part * q.part + k, step, key, w, kp);
        int st;
        do {
            st = hop_once<VT, false, true>(m, w, step, kp);  // parked walkers have an entry face
        } while (st < 0);
        hops += w.nhop;
        walls += w.walls;
        p.pos[3 * i] = w.x0; p.pos[3 * i + 1] = w.x1; p.pos[3 * i + 2] = w.x2;
        p.vel[3 * i] = (VT)w.v0; p.vel[3 * i + 1] = (VT)w.v1; p.vel[3 * i + 2] = (VT)w.v2;
        if (m.rot) p.ir[i] = w.ir;
        if (st == 0) {
            p.cell[i] = w.c;
            rank[i] = (uint32_t)atomicAdd(&counts[w.c], 1);
        } else {
            p.cell[i] = -1;
            rem += st == 1;
            lost += st == 2;
        }
    }
    block_counters(hops, walls, rem, lost, &ctr->hops, &ctr->walls, &ctr->removed, &ctr->lost);
}

// Each wave owns a batch of `batch` consecutive particles.  A lane tracks
// one particle hop by hop; when its particle is done the lane writes it back
// and takes the next untouched particle of the batch, so lanes stay busy
// while hop counts differ from particle to particle.
template <class VT>
__global__ __launch_bounds__(256) void k_move(MeshDev m, PartDev<VT> p, const Scalars* sc,
                                             int32_t* counts, uint32_t* rank, Counters* ctr,
                                             RngKey key, double dt, int batch) {
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1ull;
    const int64_t wv = xcd_block() * 4 + (threadIdx.x >> 6);
    const int64_t n = sc->np;
    const int64_t lo = wv * (int64_t)batch;
    const int64_t hi = min(lo + (int64_t)batch, n);
    const uint32_t step = sc->step;
    int hops = 0, walls = 0, rem = 0, lost = 0;
    int64_t next = lo + 64;
    int64_t i = lo + lane;
    bool active = i < hi;
    Walker w;
    w.x0 = w.x1 = w.x2 = w.v0 = w.v1 = w.v2 = w.t = 0.0;
    w.c = 0; w.entry = -1; w.nhop = 0; w.hits = 0; w.walls = 0; w.pid = 0;
    if (active) {
        w.x0 = p.pos[3 * i]; w.x1 = p.pos[3 * i + 1]; w.x2 = p.pos[3 * i + 2];
        w.v0 = (double)p.vel[3 * i]; w.v1 = (double)p.vel[3 * i + 1]; w.v2 = (double)p.vel[3 * i + 2];
        w.c = p.cell[i]; w.pid = p.pid[i]; w.t = dt;
    }
    while (__ballot(active) != 0ull) {
        int st = -1;
        if (active) st = hop_once<VT>(m, w, step, key);
        const bool done = active && st >= 0;
        if (done) {
            p.pos[3 * i] = w.x0; p.pos[3 * i + 1] = w.x1; p.pos[3 * i + 2] = w.x2;
            if (w.walls) {
                p.vel[3 * i] = (VT)w.v0; p.vel[3 * i + 1] = (VT)w.v1; p.vel[3 * i + 2] = (VT)w.v2;
            }
            if (st == 0) {
                p.cell[i] = w.c;
                rank[i] = (uint32_t)atomicAdd(&counts[w.c], 1);
            } else {
                p.cell[i] = -1;
                rem += st == 1;
                lost += st == 2;
            }
            hops += w.nhop;
            walls += w.walls;
        }
        const uint64_t dm = __ballot(done);
        if (done) {
            const int64_t ni = next + __popcll(dm & below);
            active = ni < hi;
            if (active) {
                i = ni;
                w.x0 = p.pos[3 * i]; w.x1 = p.pos[3 * i + 1]; w.x2 = p.pos[3 * i + 2];
                w.v0 = (double)p.vel[3 * i]; w.v1 = (double)p.vel[3 * i + 1]; w.v2 = (double)p.vel[3 * i + 2];
                w.c = p.cell[i]; w.pid = p.pid[i]; w.t = dt;
                w.entry = -1; w.nhop = 0; w.hits = 0; w.walls = 0;
            }
        }
        next += __popcll(dm);
    }
    block_counters(hops, walls, rem, lost, &ctr->hops, &ctr->walls, &ctr->removed, &ctr->lost);
}

// Histogram of the current cells (sort without a preceding move).
__global__ void k_count(const int32_t* cell, const Scalars* sc, int32_t* counts, uint32_t* rank) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = i < sc->np ? cell[i] : -1;
    const uint32_t slot = bin_slot(counts, c, c >= 0);
    if (c >= 0) rank[i] = slot;
}

// ---------------------------------------------------------------------------
// freestream injection
// ---------------------------------------------------------------------------
__global__ void k_inject_count(const InflowDev in, const Scalars* sc, RngKey key, int32_t* fcount) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= in.n) return;
    const double* cst = in.consts + (size_t)kInflowStride * j;
    const Rand4 r = draw(key, (uint32_t)in.bface[j], sc->step, kPurposeInjectCount, 0);
    fcount[j] = (int32_t)floor(cst[0] + u01(r.w[0], r.w[1]));
}

// Normal speed ratio z > 0 with density proportional to z exp(-(z-a)^2).
__device__ double flux_normal(double a, RngKey key, uint32_t bf, uint32_t step, uint64_t k) {
    if (a == 0.0) {
        const Rand4 r = draw(key, bf, step, kPurposeInject, (k << 6) | 3u);
        return sqrt(-log(u01(r.w[0], r.w[1])));
    }
    for (int tr = 0; tr < 30; ++tr) {
        const Rand4 r0 = draw(key, bf, step, kPurposeInject, (k << 6) | (uint64_t)(3 + 2 * tr));
        const Rand4 r1 = draw(key, bf, step, kPurposeInject, (k << 6) | (uint64_t)(4 + 2 * tr));
        const double ua = u01(r0.w[0], r0.w[1]), ub = u01(r0.w[2], r0.w[3]);
        const double uc = u01(r1.w[0], r1.w[1]), ud = u01(r1.w[2], r1.w[3]);
        if (a > 0) {
            const double pa = (a * DSMC_SQRT_PI) / ((a * DSMC_SQRT_PI) + 1.0);
            double w;
            if (ua < pa) {
                double g1, g2;
                box_muller(ub, uc, g1, g2);
                w = g1 * DSMC_INV_SQRT2;
            } else {
                const double rr = sqrt(-log(ub));
                w = uc < 0.5 ? rr : -rr;
            }
            const double z = a + w;
            if (z > 0 && ud * (a + fabs(w)) < z) return z;
        } else {
            const double w = sqrt(a * a - log(ub));
            const double z = a + w;
            if (ud * w < z) return z;
        }
    }
    return a > 0 ? a : 0.5;
}

template <class VT>
__global__ __launch_bounds__(256) void k_inject_emit(MeshDev m, const InflowDev in, PartDev<VT> p,
                                                    Scalars* sc, const int32_t* foff, int32_t* counts,
                                                    uint32_t* rank, Counters* ctr, RngKey key, double dt,
                                                    int64_t cap) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = foff[in.n];
    int hops = 0, walls = 0, rem = 0, lost = 0, made = 0;
    if (idx < total) {
        // face j: the last with foff[j] <= idx
        int lo = 0, hi = in.n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (foff[mid] <= idx) lo = mid; else hi = mid - 1;
        }
        const int j = lo;
        const int64_t k = idx - foff[j];
        const double* cst = in.consts + (size_t)kInflowStride * j;
        const uint32_t bf = (uint32_t)in.bface[j];
        const uint32_t step = sc->step;
        const uint64_t kb = (uint64_t)k << 6;
        Rand4 r = draw(key, bf, step, kPurposeInject, kb | 0u);
        double r1 = u01(r.w[0], r.w[1]), r2 = u01(r.w[2], r.w[3]);
        if (r1 + r2 > 1.0) { r1 = 1.0 - r1; r2 = 1.0 - r2; }
        r = draw(key, bf, step, kPurposeInject, kb | 1u);
        const double ut = u01(r.w[0], r.w[1]);
        // freestream rotation in equilibrium at the freestream temperature
        double irot = p.ir ? -cst[24] * log(u01(r.w[2], r.w[3])) : 0.0;
        r = draw(key, bf, step, kPurposeInject, kb | 2u);
        double g1, g2;
        box_muller(u01(r.w[0], r.w[1]), u01(r.w[2], r.w[3]), g1, g2);
        const double z = flux_normal(cst[1], key, bf, step, (uint64_t)k);
        const double vn = cst[2] * z;
        const double vt1 = cst[3] * g1 + cst[4];
        const double vt2 = cst[3] * g2 + cst[5];
        const double* nin = cst + 6;
        const double* t1 = cst + 9;
        const double* t2 = cst + 12;
        const double* A = cst + 15;
        const double* B = cst + 18;
        const double* C = cst + 21;
        double x0 = (A[0] + r1 * (B[0] - A[0])) + r2 * (C[0] - A[0]);
        double x1 = (A[1] + r1 * (B[1] - A[1])) + r2 * (C[1] - A[1]);
        double x2 = (A[2] + r1 * (B[2] - A[2])) + r2 * (C[2] - A[2]);
        double v0 = round_store<VT>((vn * nin[0] + vt1 * t1[0]) + vt2 * t2[0]);
        double v1 = round_store<VT>((vn * nin[1] + vt1 * t1[1]) + vt2 * t2[1]);
        double v2 = round_store<VT>((vn * nin[2] + vt1 * t1[2]) + vt2 * t2[2]);
        const uint32_t pid = sc->next_pid + (uint32_t)idx;
        const int code = in.tcode[j];
        int c = code >> 2;
        made = 1;
        const TraceOut o = trace<VT>(m, x0, x1, x2, v0, v1, v2, c, code & 3, pid, step, key, ut * dt,
                                     p.ir ? &irot : nullptr);
        hops = o.hops;
        walls = o.walls;
        const int64_t slot = sc->np + idx;
        if (slot >= cap) {
            atomicOr(&sc->flags, kFlagCapacity);
        } else {
            p.pos[3 * slot] = x0; p.pos[3 * slot + 1] = x1; p.pos[3 * slot + 2] = x2;
            p.vel[3 * slot] = (VT)v0; p.vel[3 * slot + 1] = (VT)v1; p.vel[3 * slot + 2] = (VT)v2;
            p.pid[slot] = pid;
            if (p.ir) p.ir[slot] = irot;
            if (o.status == 0) {
                p.cell[slot] = c;
                rank[slot] = (uint32_t)atomicAdd(&counts[c], 1);
            } else {
                p.cell[slot] = -1;
                rem = o.status == 1;
                lost = o.status == 2;
            }
        }
    }
    block_counters(hops, walls, rem, lost, &ctr->hops, &ctr->walls, &ctr->removed, &ctr->lost);
    // injected count
    const int s = wave_sum(made);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd(&ctr->injected, (unsigned long long)s);
}

// ---------------------------------------------------------------------------
// exclusive scan of int32 counts[n] -> offsets[n+1]
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// block-wide exclusive scan over blockDim.x (<= 1024) threads; returns the
// exclusive prefix of v and writes the block total to *total.
__device__ __forceinline__ int block_excl_scan(int v, int* total) {
    __shared__ int ws[17];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int inc = wave_incl_scan(v);
    if (lane == 63) ws[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        const int nw = (blockDim.x + 63) >> 6;
        for (int k = 0; k < nw; ++k) {
            const int t = ws[k];
            ws[k] = acc;
            acc += t;
        }
        ws[16] = acc;
    }
    __syncthreads();
    const int res = ws[w] + inc - v;
    *total = ws[16];
    __syncthreads();
    return res;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int32_t* in, int64_t n,
                                                              int32_t* blocksums) {
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    int s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
        if (i < n) s += in[i];
    }
    int total;
    block_excl_scan(s, &total);
    if (threadIdx.x == 0) blocksums[blockIdx.x] = total;
}

// Single workgroup: exclusive scan of the block sums; the grand total
// updates the device scalars according to mode.
__global__ __launch_bounds__(1024) void k_scan_top(int32_t* blocksums, int nblk, Scalars* sc, int mode,
                                                   int32_t* tail) {
    int carry = 0;
    for (int base = 0; base < nblk; base += 1024) {
        const int i = base + threadIdx.x;
        const int v = i < nblk ? blocksums[i] : 0;
        int total;
        const int ex = block_excl_scan(v, &total);
        if (i < nblk) blocksums[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) {
        *tail = carry;
        if (mode == kScanCells) {
            const int64_t ninj = sc->ninj;
            sc->n_entries = sc->np + ninj;
            sc->next_pid += (uint32_t)ninj;
            sc->np = carry;
        } else if (mode == kScanInject) {
            sc->ninj = carry;
        } else if (mode == kScanInit) {
            sc->np = carry;
            sc->n_entries = carry;
            sc->next_pid = (uint32_t)carry;
        }
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(const int32_t* in, int64_t n,
                                                            const int32_t* blocksums, int32_t* out) {
    __shared__ int buf[kScanBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
        buf[k * kScanThreads + threadIdx.x] = i < n ? in[i] : 0;
    }
    __syncthreads();
    // each thread owns kScanItems consecutive entries
    int loc[kScanItems];
    int s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        loc[k] = s;
        s += buf[threadIdx.x * kScanItems + k];
    }
    int total;
    const int ex = block_excl_scan(s, &total);
    const int off = blocksums[blockIdx.x] + ex;
    __syncthreads();
    for (int k = 0; k < kScanItems; ++k) buf[threadIdx.x * kScanItems + k] = off + loc[k];
    __syncthreads();
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
        if (i < n) out[i] = buf[k * kScanThreads + threadIdx.x];
    }
}

// ---------------------------------------------------------------------------
// counting-sort scatter
// ---------------------------------------------------------------------------
// Copies particle i of src to slot d of dst (cell given).  Every load is
// issued before the first store: the two buffers never alias, but the
// compiler cannot know it and would otherwise order each load after the
// previous store.
template <class VT>
__device__ __forceinline__ void copy_particle(const PartDev<VT>& src, int64_t i, const PartDev<VT>& dst, int64_t d,
                                              int32_t cell) {
    const double x0 = src.pos[3 * i], x1 = src.pos[3 * i + 1], x2 = src.pos[3 * i + 2];
    const VT v0 = src.vel[3 * i], v1 = src.vel[3 * i + 1], v2 = src.vel[3 * i + 2];
    const uint32_t id = src.pid[i];
    dst.pos[3 * d] = x0;
    dst.pos[3 * d + 1] = x1;
    dst.pos[3 * d + 2] = x2;
    dst.vel[3 * d] = v0;
    dst.vel[3 * d + 1] = v1;
    dst.vel[3 * d + 2] = v2;
    dst.cell[d] = cell;
    dst.pid[d] = id;
    if (src.ir) dst.ir[d] = src.ir[i];
}

template <class VT>
__global__ __launch_bounds__(256) void k_scatter(PartDev<VT> src, PartDev<VT> dst, const Scalars* sc,
                                                const int32_t* offsets, const uint32_t* rank, int64_t cap) {
    const int64_t i = xcd_block() * 256 + threadIdx.x;
    if (i >= sc->n_entries || i >= cap) return;
    const int c = src.cell[i];
    if (c < 0) return;
    const int64_t d = (int64_t)offsets[c] + rank[i];
    copy_particle(src, i, dst, d, c);
}

// Gather form of the counting sort: k_perm writes, for every destination
// slot, the index of the particle that lands there and its cell (4-byte
// scattered stores); k_gather then fills the rest of the sorted buffer slot
// by slot (coalesced stores, gathered loads from the spatially local source
// buffer).
__global__ __launch_bounds__(256) void k_perm(const int32_t* cell, const Scalars* sc, const int32_t* offsets,
                                             const uint32_t* rank, int32_t* perm, int32_t* dst_cell, int64_t cap) {
    const int64_t i = xcd_block() * 256 + threadIdx.x;
    if (i >= sc->n_entries || i >= cap) return;
    const int c = cell[i];
    if (c < 0) return;
    const int64_t d = (int64_t)offsets[c] + rank[i];
    perm[d] = (int32_t)i;
    dst_cell[d] = c;  // the slot's cell, so that the gather need not load it
}

// The sorted order of a buffer that is already sorted: slot k holds
// particle k (deferred sort after a physical sort).
__global__ __launch_bounds__(256) void k_perm_identity(const int32_t* cell, const Scalars* sc, int32_t* perm,
                                                      int32_t* dst_cell) {
    const int64_t k = xcd_block() * 256 + threadIdx.x;
    if (k >= sc->np) return;
    perm[k] = (int32_t)k;
    dst_cell[k] = cell[k];
}

template <class VT>
__global__ __launch_bounds__(256) void k_gather(PartDev<VT> src, PartDev<VT> dst, const Scalars* sc,
                                               const int32_t* perm) {
    const int64_t k = xcd_block() * 256 + threadIdx.x;
    if (k >= sc->np) return;
    const int64_t i = perm[k];
    const double x0 = src.pos[3 * i], x1 = src.pos[3 * i + 1], x2 = src.pos[3 * i + 2];
    const VT v0 = src.vel[3 * i], v1 = src.vel[3 * i + 1], v2 = src.vel[3 * i + 2];
    const uint32_t id = src.pid[i];
    // positions are next read by the following step's move: stream them past
    // the L2 (velocities and ids stay cached for the collide kernel)
    __builtin_nontemporal_store(x0, &dst.pos[3 * k]);
    __builtin_nontemporal_store(x1, &dst.pos[3 * k + 1]);
    __builtin_nontemporal_store(x2, &dst.pos[3 * k + 2]);
    dst.vel[3 * k] = v0;
    dst.vel[3 * k + 1] = v1;
    dst.vel[3 * k + 2] = v2;
    dst.pid[k] = id;
    if (src.ir) dst.ir[k] = src.ir[i];
}

// ---------------------------------------------------------------------------
// collisions and sampling
// ---------------------------------------------------------------------------
// Access to the velocities of one cell in logical (pid) order.
template <class VT>
struct LdsCell {
    VT* v0; VT* v1; VT* v2;
    const uint16_t* ord;
    uint8_t* touch;
    int s0;
    __device__ __forceinline__ void get(int k, double& a, double& b, double& c) const {
        const int l = ord[s0 + k];
        a = (double)v0[l]; b = (double)v1[l]; c = (double)v2[l];
    }
    __device__ __forceinline__ void put(int k, double a, double b, double c) const {
        const int l = ord[s0 + k];
        v0[l] = (VT)a; v1[l] = (VT)b; v2[l] = (VT)c;
        touch[l] = 1;
    }
};

template <class VT>
struct GlobalCell {
    VT* v;                 // interleaved velocities of the particle store
    const int32_t* perm;   // logical -> physical
    int64_t s0;
    double* ir;            // rotational energies of the particle store (rotating gas)
    __device__ __forceinline__ void get(int k, double& a, double& b, double& c) const {
        const int64_t l = perm[s0 + k];
        a = (double)v[3 * l]; b = (double)v[3 * l + 1]; c = (double)v[3 * l + 2];
    }
    __device__ __forceinline__ void put(int k, double a, double b, double c) const {
        const int64_t l = perm[s0 + k];
        v[3 * l] = (VT)a; v[3 * l + 1] = (VT)b; v[3 * l + 2] = (VT)c;
    }
    __device__ __forceinline__ double getI(int k) const { return ir[perm[s0 + k]]; }
    __device__ __forceinline__ void putI(int k, double e) const { ir[perm[s0 + k]] = e; }
};

template <class VT>
struct LdsOrderCell {
    VT* v;                 // interleaved velocities of the particle store
    const uint16_t* ord;   // sorted position -> slot relative to the chunk start
    int s0;
    int64_t a;             // chunk start in the particle arrays
    __device__ __forceinline__ void get(int k, double& x, double& y, double& z) const {
        const int64_t l = a + ord[s0 + k];
        x = (double)v[3 * l]; y = (double)v[3 * l + 1]; z = (double)v[3 * l + 2];
    }
    __device__ __forceinline__ void put(int k, double x, double y, double z) const {
        const int64_t l = a + ord[s0 + k];
        v[3 * l] = (VT)x; v[3 * l + 1] = (VT)y; v[3 * l + 2] = (VT)z;
    }
    double* ir;            // rotational energies of the particle store (rotating gas)
    __device__ __forceinline__ double getI(int k) const { return ir[a + ord[s0 + k]]; }
    __device__ __forceinline__ void putI(int k, double e) const { ir[a + ord[s0 + k]] = e; }
};

// As LdsOrderCell for particles left where the move put them: the window's
// slot -> particle index table in LDS.
template <class VT>
struct LdsIndCell {
    VT* v;                 // interleaved velocities of the particle store
    const uint16_t* ord;   // sorted position -> slot relative to the window start
    const uint32_t* src;   // window slot -> particle index
    int s0;
    __device__ __forceinline__ void get(int k, double& x, double& y, double& z) const {
        const int64_t l = src[ord[s0 + k]];
        x = (double)v[3 * l]; y = (double)v[3 * l + 1]; z = (double)v[3 * l + 2];
    }
    __device__ __forceinline__ void put(int k, double x, double y, double z) const {
        const int64_t l = src[ord[s0 + k]];
        v[3 * l] = (VT)x; v[3 * l + 1] = (VT)y; v[3 * l + 2] = (VT)z;
    }
    double* ir;            // rotational energies of the particle store (rotating gas)
    __device__ __forceinline__ double getI(int k) const { return ir[src[ord[s0 + k]]]; }
    __device__ __forceinline__ void putI(int k, double e) const { ir[src[ord[s0 + k]]] = e; }
};

// Post-collision relative velocity g' (|g'| = |g| = c_r) from two uniform
// deviates R1 (deflection) and R2 (azimuth eps = 2 pi R2).  VHS: isotropic,
// cos(theta) = 2 R1 - 1 measured from the x axis, independent of g.  VSS
// (section 2.1, the model of Bird 1994): the deflection chi from g has
// cos(chi) = 2 R1^(1/alpha) - 1 and g' = cos(chi) g + sin(chi) c_r
// (cos(eps) e1 + sin(eps) e2) in the frame e1 = (0, g_z, -g_y) / g_yz,
// e2 = (g_yz^2, -g_x g_y, -g_x g_z) / (c_r g_yz), g_yz = |(g_y, g_z)|; with
// g along x (g_yz = 0) e1 and e2 are the y and z axes.  VSS is a template
// parameter so that the isotropic kernels keep their register budget.
template <bool VSS>
__device__ __forceinline__ void scatter_vhs_vss(const CollideParams& cp, double gx, double gy, double gz,
                                                double cr2, double R1, double R2, double& o0, double& o1,
                                                double& o2) {
    const double cr = sqrt(cr2);
    const double eps = DSMC_TWO_PI * R2;
    if (!VSS) {
        const double cx = 2.0 * R1 - 1.0;
        const double sx = sqrt(1.0 - cx * cx);
        o0 = cr * cx;
        o1 = cr * (sx * cos(eps));
        o2 = cr * (sx * sin(eps));
        return;
    }
    const double cc = 2.0 * pow(R1, cp.inv_alpha) - 1.0;
    const double sc = sqrt(1.0 - cc * cc);
    const double ce = cos(eps), se = sin(eps);
    const double gyz = sqrt(gy * gy + gz * gz);
    double e10 = 0.0, e11 = 1.0, e12 = 0.0, e20 = 0.0, e21 = 0.0, e22 = 1.0;
    if (gyz > 0.0) {
        e11 = gz / gyz;
        e12 = -gy / gyz;
        e20 = gyz / cr;
        e21 = -(gx * gy) / (cr * gyz);
        e22 = -(gx * gz) / (cr * gyz);
    }
    const double scr = sc * cr;
    o0 = cc * gx + scr * (se * e20 + ce * e10);
    o1 = cc * gy + scr * (se * e21 + ce * e11);
    o2 = cc * gz + scr * (se * e22 + ce * e12);
}

template <bool VSS, bool ROT = false, class Acc>
__device__ __forceinline__ void ntc_cell(const Acc& cv, int N, int c, const CollideParams& cp,
                                         uint32_t step, double* smax, int32_t* ncand, int32_t* nacc) {
    int M = 0, acc = 0;
    if (N >= 2) {
        const double sm = smax[c];
        uint32_t subj = (uint32_t)cp.orig[c];
        RngKey key = cp.key;
        double FN = cp.FN, dt = cp.dt;
        if (cp.cell_case) {
            const CaseDev& cs = cp.cases[cp.cell_case[c]];
            key.k0 = cs.k0;
            key.k1 = cs.k1;
            FN = cs.FN;
            dt = cs.dt;
            subj -= (uint32_t)cs.cell0;
        }
        const Rand4 r = draw(key, subj, step, kPurposeNtcCount, 0);
        const double Nd = (double)N;
        const double mean = ((((0.5 * Nd) * (Nd - 1.0)) * FN) * sm) * dt / cp.vol[c];
        M = (int)floor(mean + u01(r.w[0], r.w[1]));
        double seen = 0.0;
        // (sigma c)/(sigma c)_max = K cr2^ex / sm is first estimated in FP32
        // (hardware log2/exp2); when the estimate is below 1 and U lies
        // outside a relative band of 1e-3 around it, both the acceptance and
        // the (sigma c)_max update (only values above sm matter) are decided
        // without the FP64 power, and decided as the FP64 expression would.
        const float lk = log2f((float)cp.K) - log2f((float)sm), ex32 = (float)cp.ex;
        for (int k = 0; k < M; ++k) {
            const Rand4 w = draw(key, subj, step, kPurposePair, (uint64_t)k);
            const uint32_t i = pick(w.w[0], (uint32_t)N);
            uint32_t j = pick(w.w[1], (uint32_t)(N - 1));
            if (j >= i) ++j;
            const double U = u01(w.w[2], w.w[3]);
            double a0, a1, a2, b0, b1, b2;
            cv.get((int)i, a0, a1, a2);
            cv.get((int)j, b0, b1, b2);
            const double gx = a0 - b0, gy = a1 - b1, gz = a2 - b2;
            const double cr2 = gx * gx + gy * gy + gz * gz;
            const double est = (double)exp2f(fmaf(ex32, log2f((float)cr2), lk));
            const double lo = est * (1.0 - 1e-3), hi = est * (1.0 + 1e-3);
            bool take;
            if (hi < 1.0 && (U < lo || U >= hi)) {
                take = U < lo;
            } else {
                const double sc = cp.K * pow(cr2, cp.ex);
                if (sc > seen) seen = sc;
                take = U < sc / sm;
            }
            if (!take) continue;
            ++acc;
            const Rand4 q = draw(key, subj, step, kPurposeScatter, (uint64_t)k);
            double gp0, gp1, gp2;
            if constexpr (ROT) {
                // Borgnakke-Larsen, partner by partner: with probability
                // pinel the partner's rotational energy and the relative
                // translational energy E_t = m c_r^2 / 4 are pooled and the
                // translation keeps E_c R^(1/(5/2 - omega)) (two rotational
                // degrees of freedom); the relative velocity keeps its
                // direction and takes the new speed
                const double R1 = u01(q.w[0], q.w[1]), R2 = u01(q.w[2], q.w[3]);
                double Ii = cv.getI((int)i), Ij = cv.getI((int)j);
                double Et = (0.25 * cp.mass) * cr2;
                bool inel = false;
                const Rand4 ri = draw(key, subj, step, kPurposeInelasticI, (uint64_t)k);
                if (u01(ri.w[0], ri.w[1]) < cp.pinel) {
                    const double Ec = Et + Ii;
                    Et = Ec * pow(u01(ri.w[2], ri.w[3]), cp.ex_bl);
                    Ii = Ec - Et;
                    inel = true;
                }
                const Rand4 rj = draw(key, subj, step, kPurposeInelasticJ, (uint64_t)k);
                if (u01(rj.w[0], rj.w[1]) < cp.pinel) {
                    const double Ec = Et + Ij;
                    Et = Ec * pow(u01(rj.w[2], rj.w[3]), cp.ex_bl);
                    Ij = Ec - Et;
                    inel = true;
                }
                if (inel) {
                    cv.putI((int)i, Ii);
                    cv.putI((int)j, Ij);
                    const double cr2n = (4.0 * Et) / cp.mass;
                    const double f = sqrt(cr2n / cr2);
                    scatter_vhs_vss<VSS>(cp, gx * f, gy * f, gz * f, cr2n, R1, R2, gp0, gp1, gp2);
                } else {
                    scatter_vhs_vss<VSS>(cp, gx, gy, gz, cr2, R1, R2, gp0, gp1, gp2);
                }
            } else {
                scatter_vhs_vss<VSS>(cp, gx, gy, gz, cr2, u01(q.w[0], q.w[1]), u01(q.w[2], q.w[3]), gp0, gp1,
                                     gp2);
            }
            const double cm0 = 0.5 * (a0 + b0), cm1 = 0.5 * (a1 + b1), cm2 = 0.5 * (a2 + b2);
            const double h0 = 0.5 * gp0, h1 = 0.5 * gp1, h2 = 0.5 * gp2;
            cv.put((int)i, cm0 + h0, cm1 + h1, cm2 + h2);
            cv.put((int)j, cm0 - h0, cm1 - h1, cm2 - h2);
        }
        if (seen > sm) smax[c] = seen;
    }
    ncand[c] = M;
    nacc[c] = acc;
}

template <bool ROT = false, class Acc>
__device__ __forceinline__ void sample_cell(const Acc& cv, int N, int c, const CollideParams& cp,
                                            uint32_t step) {
    double S[kNMom];
#pragma unroll
    for (int k = 0; k < kNMom; ++k) S[k] = 0.0;
    for (int k = 0; k < N; ++k) {
        double vx, vy, vz;
        cv.get(k, vx, vy, vz);
        const double v2 = vx * vx + vy * vy + vz * vz;
        S[0] += 1.0;
        S[1] += vx; S[2] += vy; S[3] += vz;
        S[4] += vx * vx; S[5] += vy * vy; S[6] += vz * vz;
        S[7] += vx * vy; S[8] += vx * vz; S[9] += vy * vz;
        S[10] += vx * v2; S[11] += vy * v2; S[12] += vz * v2;
    }
    const int64_t nt = cp.nt;
    if (cp.inst) {
#pragma unroll
        for (int k = 0; k < kNMom; ++k) cp.inst[k * nt + c] = S[k];
    }
    if ((int64_t)step > (int64_t)cp.n_ss) {
#pragma unroll
        for (int k = 0; k < kNMom; ++k) cp.acc[k * nt + c] += S[k];
    }
    if (cp.ewma_on) {
        const int m = cp.ewma_m[c] + 1;
        cp.ewma_m[c] = m;
        const int n = (cp.local_acc[c] || m < cp.n_a) ? m : cp.n_a;
        const double wo = (double)(n - 1) / (double)n;
        const double wn = 1.0 / (double)n;
#pragma unroll
        for (int k = 0; k < kNMom; ++k) {
            double* e = cp.ewma + k * nt + c;
            *e = wo * *e + wn * S[k];
        }
    }
    if constexpr (ROT) {
        // rotational sums: sum I_r, sum v_i I_r (rotational temperature and
        // heat flux of eq. dsmc_temperatures), in the same particle order
        double Rr[4] = {0.0, 0.0, 0.0, 0.0};
        for (int k = 0; k < N; ++k) {
            double vx, vy, vz;
            cv.get(k, vx, vy, vz);
            const double I = cv.getI(k);
            Rr[0] += I;
            Rr[1] += vx * I; Rr[2] += vy * I; Rr[3] += vz * I;
        }
        if (cp.rinst) {
#pragma unroll
            for (int k = 0; k < 4; ++k) cp.rinst[k * nt + c] = Rr[k];
        }
        if ((int64_t)step > (int64_t)cp.n_ss) {
#pragma unroll
            for (int k = 0; k < 4; ++k) cp.racc[k * nt + c] += Rr[k];
        }
        if (cp.ewma_on) {
            const int m = cp.ewma_m[c];
            const int n = (cp.local_acc[c] || m < cp.n_a) ? m : cp.n_a;
            const double wo = (double)(n - 1) / (double)n;
            const double wn = 1.0 / (double)n;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                double* e = cp.rewma + k * nt + c;
                *e = wo * *e + wn * Rr[k];
            }
        }
    }
}

template <class VT, bool VSS>
__global__ __launch_bounds__(kCollideLanes) void k_collide_sample(PartDev<VT> p, const int32_t* offsets,
                                                                  CollideParams cp, const Scalars* sc,
                                                                  int32_t* perm, int do_collide,
                                                                  int do_sample) {
    __shared__ VT sv0[kCollideCap];
    __shared__ VT sv1[kCollideCap];
    __shared__ VT sv2[kCollideCap];
    __shared__ uint32_t spid[kCollideCap];
    __shared__ uint16_t sord[kCollideCap];
    __shared__ uint8_t stouch[kCollideCap];
    const int nt = cp.nt;
    const int lane = threadIdx.x;
    const int c0 = blockIdx.x * kCollideLanes;
    const int c = c0 + lane;
    const int cend = min(c0 + kCollideLanes, nt);
    const int64_t a = offsets[c0];
    const int64_t n = (int64_t)offsets[cend] - a;
    const uint32_t step = sc->step;
    if (n <= kCollideCap) {
#pragma unroll 4
        for (int64_t i = lane; i < n; i += kCollideLanes) {
            sv0[i] = p.vel[3 * (a + i)];
            sv1[i] = p.vel[3 * (a + i) + 1];
            sv2[i] = p.vel[3 * (a + i) + 2];
            spid[i] = p.pid[a + i];
            stouch[i] = 0;
        }
        __syncthreads();
        if (c < nt) {
            const int s0 = (int)(offsets[c] - a);
            const int N = offsets[c + 1] - offsets[c];
            // logical order: insertion sort of the cell's pids (sord maps the
            // sorted position to the staged slot)
            for (int k = 0; k < N; ++k) {
                const uint32_t key = spid[s0 + k];
                int j = k;
                while (j > 0 && spid[s0 + j - 1] > key) {
                    spid[s0 + j] = spid[s0 + j - 1];
                    sord[s0 + j] = sord[s0 + j - 1];
                    --j;
                }
                spid[s0 + j] = key;
                sord[s0 + j] = (uint16_t)(s0 + k);
            }
            LdsCell<VT> cv{sv0, sv1, sv2, sord, stouch, s0};
            if (do_collide) ntc_cell<VSS>(cv, N, c, cp, step, cp.smax, cp.ncand, cp.nacc);
            if (do_sample) sample_cell(cv, N, c, cp, step);
        }
        __syncthreads();
        for (int64_t i = lane; i < n; i += kCollideLanes) {
            if (stouch[i]) {
                p.vel[3 * (a + i)] = sv0[i];
                p.vel[3 * (a + i) + 1] = sv1[i];
                p.vel[3 * (a + i) + 2] = sv2[i];
            }
        }
    } else if (c < nt) {
        // dense chunk: logical order through a global permutation
        const int64_t s0 = offsets[c];
        const int N = offsets[c + 1] - offsets[c];
        for (int k = 0; k < N; ++k) {
            const uint32_t pk = p.pid[s0 + k];
            int r = 0;
            for (int q = 0; q < N; ++q) r += p.pid[s0 + q] < pk;
            perm[s0 + r] = (int32_t)(s0 + k);
        }
        GlobalCell<VT> cv{p.vel, perm, s0, nullptr};
        if (do_collide) ntc_cell<VSS>(cv, N, c, cp, step, cp.smax, cp.ncand, cp.nacc);
        if (do_sample) sample_cell(cv, N, c, cp, step);
    }
}

// Variant with only the pid ranking staged in LDS (6 bytes per particle,
// up to kCollideCapG per 64-cell chunk); the velocities stay in global
// memory and are reached through the logical order, so several waves fit on
// a CU.  Ranks are computed one particle per lane (independent LDS reads
// that pipeline), the collisions and sums one cell per lane.
// CAP bounds the LDS of a workgroup (6 bytes per particle), hence how many
// workgroups share a CU; a chunk of more than CAP particles takes the
// global-memory path.
// With FUSED, the chunk's slots of the sorted buffer p are first filled from
// the unsorted buffer src through the gather permutation (slot -> source
// index; k_perm has written the slots' cells): the sort's gather done by the
// workgroup that then collides the chunk, so that gathering one chunk
// overlaps the collisions of others and the velocities are read back from
// cache.  With IND (deferred sort) nothing is moved: slot d of the sorted
// order is particle sortperm[d] of p, its cell src.cell[d]; after the
// ranking the window's pid table is overwritten with those particle indices.
template <class VT, int WPE, int CAP, int GM, bool VSS, bool ROT = false>
__global__ __launch_bounds__(kCollideLanes) __attribute__((amdgpu_waves_per_eu(WPE))) void k_collide_sample_g(
    PartDev<VT> p, const int32_t* offsets, CollideParams cp, const Scalars* sc, int32_t* perm, int do_collide,
    int do_sample, PartDev<VT> src, const int32_t* sortperm) {
    constexpr bool FUSED = GM == kGatherFused;
    constexpr bool IND = GM == kGatherIndirect;
    __shared__ uint32_t spid[CAP];
    __shared__ uint16_t sord[CAP];
    __shared__ int32_t soff[kCollideLanes + 1];
    const int nt = cp.nt;
    const int lane = threadIdx.x;
    const int c0 = blockIdx.x * kCollideLanes;
    const int c = c0 + lane;
    const int64_t a = offsets[c0];
    soff[lane] = offsets[min(c0 + lane, nt)] - (int32_t)a;
    if (lane == 0) soff[kCollideLanes] = offsets[min(c0 + kCollideLanes, nt)] - (int32_t)a;
    const int64_t n = (int64_t)offsets[min(c0 + kCollideLanes, nt)] - a;
    const uint32_t step = sc->step;
    __syncthreads();  // soff is read by every lane below
    if (FUSED) {
        // kFuseBatch particles per lane in flight: all loads of a batch are
        // issued before its stores (the compiler cannot move a load of src
        // above a store to p, which might alias it)
        constexpr int kFuseBatch = 8;
        for (int64_t i0 = lane; i0 < n; i0 += kFuseBatch * kCollideLanes) {
            int64_t j[kFuseBatch];
            double x[kFuseBatch][3];
            VT v[kFuseBatch][3];
            uint32_t id[kFuseBatch];
#pragma unroll
            for (int b = 0; b < kFuseBatch; ++b) {
                const int64_t i = i0 + b * kCollideLanes;
                j[b] = i < n ? sortperm[a + i] : 0;
            }
#pragma unroll
            for (int b = 0; b < kFuseBatch; ++b) {
                if (i0 + b * kCollideLanes < n) {
                    x[b][0] = src.pos[3 * j[b]];
                    x[b][1] = src.pos[3 * j[b] + 1];
                    x[b][2] = src.pos[3 * j[b] + 2];
                    v[b][0] = src.vel[3 * j[b]];
                    v[b][1] = src.vel[3 * j[b] + 1];
                    v[b][2] = src.vel[3 * j[b] + 2];
                    id[b] = src.pid[j[b]];
                }
            }
#pragma unroll
            for (int b = 0; b < kFuseBatch; ++b) {
                const int64_t i = i0 + b * kCollideLanes;
                if (i < n) {
                    const int64_t d = a + i;
                    p.pos[3 * d] = x[b][0];
                    p.pos[3 * d + 1] = x[b][1];
                    p.pos[3 * d + 2] = x[b][2];
                    p.vel[3 * d] = v[b][0];
                    p.vel[3 * d + 1] = v[b][1];
                    p.vel[3 * d + 2] = v[b][2];
                    p.pid[d] = id[b];
                    if (n <= CAP) spid[i] = id[b];
                }
            }
        }
        __syncthreads();
    }
    // The chunk's cells are taken in windows of consecutive cells whose
    // particles fit in CAP (one window when the whole chunk fits): ranks in
    // LDS, then the window's cells one per lane.  A single cell with more
    // than CAP particles takes the global-memory path.
    for (int k0 = 0; k0 < kCollideLanes;) {
        int k1 = k0;
        while (k1 < kCollideLanes && soff[k1 + 1] - soff[k0] <= CAP) ++k1;
        const int w0 = soff[k0];
        if (k1 == k0) {
            // one cell beyond the LDS stage
            if (lane == 0 && c0 + k0 < nt) {
                const int cc = c0 + k0;
                const int64_t s0 = offsets[cc];
                const int N = offsets[cc + 1] - offsets[cc];
                for (int k = 0; k < N; ++k) {
                    const uint32_t pk = IND ? p.pid[sortperm[s0 + k]] : p.pid[s0 + k];
                    int r = 0;
                    for (int q = 0; q < N; ++q) r += (IND ? p.pid[sortperm[s0 + q]] : p.pid[s0 + q]) < pk;
                    perm[s0 + r] = IND ? sortperm[s0 + k] : (int32_t)(s0 + k);
                }
                GlobalCell<VT> cv{p.vel, perm, s0, p.ir};
                if (do_collide) ntc_cell<VSS, ROT>(cv, N, cc, cp, step, cp.smax, cp.ncand, cp.nacc);
                if (do_sample) sample_cell<ROT>(cv, N, cc, cp, step);
            }
            k0 = k0 + 1;
            continue;
        }
        const int wn = soff[k1] - w0;
        if (!FUSED || n > CAP) {
            if (k0 > 0) __syncthreads();  // the previous window's ranks are no longer read
#pragma unroll 4
            for (int i = lane; i < wn; i += kCollideLanes)
                spid[i] = IND ? p.pid[sortperm[a + w0 + i]] : p.pid[a + w0 + i];
        }
        __syncthreads();
        for (int i = lane; i < wn; i += kCollideLanes) {
            const int k = (IND ? src.cell[a + w0 + i] : p.cell[a + w0 + i]) - c0;
            const int s0 = soff[k] - w0;
            const int N = soff[k + 1] - soff[k];
            const uint32_t pk = spid[i];
            int r = 0;
#pragma unroll 4
            for (int q = 0; q < N; ++q) r += spid[s0 + q] < pk ? 1 : 0;
            sord[s0 + r] = (uint16_t)i;
        }
        __syncthreads();
        if constexpr (IND) {
            // the pids are ranked: the table now maps window slots to particles
#pragma unroll 4
            for (int i = lane; i < wn; i += kCollideLanes) spid[i] = (uint32_t)sortperm[a + w0 + i];
            __syncthreads();
            if (lane >= k0 && lane < k1 && c < nt) {
                const int s0 = soff[lane] - w0;
                const int N = soff[lane + 1] - soff[lane];
                LdsIndCell<VT> cv{p.vel, sord, spid, s0, p.ir};
                if (do_collide) ntc_cell<VSS, ROT>(cv, N, c, cp, step, cp.smax, cp.ncand, cp.nacc);
                if (do_sample) sample_cell<ROT>(cv, N, c, cp, step);
            }
        } else if (lane >= k0 && lane < k1 && c < nt) {
            const int s0 = soff[lane] - w0;
            const int N = soff[lane + 1] - soff[lane];
            LdsOrderCell<VT> cv{p.vel, sord, s0, a + w0, p.ir};
            if (do_collide) ntc_cell<VSS, ROT>(cv, N, c, cp, step, cp.smax, cp.ncand, cp.nacc);
            if (do_sample) sample_cell<ROT>(cv, N, c, cp, step);
        }
        k0 = k1;
    }
}

// ---------------------------------------------------------------------------
// fields from moment sums (eq. dsmc_temperatures over accumulated samples)
// ---------------------------------------------------------------------------
__global__ void k_fields(const double* sums, int nt, double ns, double mass, double FN, const double* vol,
                         const int32_t* orig, double* out, const int32_t* cell_case, const CaseDev* cases) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nt) return;
    if (cell_case) FN = cases[cell_case[c]].FN;
    double S[kNMom];
    for (int k = 0; k < kNMom; ++k) S[k] = sums[(int64_t)k * nt + c];
    double* o = out + 15 * (size_t)orig[c];
    if (!(S[0] > 0) || !(ns > 0)) {
        for (int k = 0; k < 15; ++k) o[k] = __builtin_nan("");
        return;
    }
    const double n = (FN * (S[0] / ns)) / vol[c];
    const double rho = mass * n;
    const double u0 = S[1] / S[0], u1 = S[2] / S[0], u2 = S[3] / S[0];
    const double Cxx = S[4] / S[0] - u0 * u0, Cyy = S[5] / S[0] - u1 * u1, Czz = S[6] / S[0] - u2 * u2;
    const double Cxy = S[7] / S[0] - u0 * u1, Cxz = S[8] / S[0] - u0 * u2, Cyz = S[9] / S[0] - u1 * u2;
    const double Ckk = Cxx + Cyy + Czz;
    o[0] = n; o[1] = rho; o[2] = u0; o[3] = u1; o[4] = u2;
    o[5] = (mass * Ckk) / (3.0 * kBoltzmannDev);
    o[6] = rho * (Cxx - Ckk / 3.0);
    o[7] = rho * (Cyy - Ckk / 3.0);
    o[8] = rho * (Czz - Ckk / 3.0);
    o[9] = rho * Cxy;
    o[10] = rho * Cxz;
    o[11] = rho * Cyz;
    const double S2kk = S[4] + S[5] + S[6];
    const double uu = u0 * u0 + u1 * u1 + u2 * u2;
    const double uS0 = u0 * S[4] + u1 * S[7] + u2 * S[8];
    const double uS1 = u0 * S[7] + u1 * S[5] + u2 * S[9];
    const double uS2 = u0 * S[8] + u1 * S[9] + u2 * S[6];
    o[12] = (rho / 2.0) * (((S[10] - 2.0 * uS0) - u0 * S2kk) + 2.0 * S[0] * u0 * uu) / S[0];
    o[13] = (rho / 2.0) * (((S[11] - 2.0 * uS1) - u1 * S2kk) + 2.0 * S[0] * u1 * uu) / S[0];
    o[14] = (rho / 2.0) * (((S[12] - 2.0 * uS2) - u2 * S2kk) + 2.0 * S[0] * u2 * uu) / S[0];
}

// ---------------------------------------------------------------------------
// utilities
// ---------------------------------------------------------------------------
__global__ void k_philox(const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Rand4 r = philox(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1);
    for (int k = 0; k < 4; ++k) out[4 * i + k] = r.w[k];
}

// Plain copy of n16 16-byte words: each thread moves four words, 256
// threads apart, all four loads issued before the stores.
__global__ __launch_bounds__(256) void k_copy16(const uint4* src, uint4* dst, int64_t n16) {
    const int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    uint4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + 256 * k < n16) v[k] = src[base + 256 * k];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + 256 * k < n16) dst[base + 256 * k] = v[k];
}

// Scattered 16-byte loads, one 128-byte line of the table per group of
// `share` consecutive lanes and iteration, lines drawn by a linear
// congruential sequence (calibration of the vector L1's line-access rate,
// the limit of gather-bound kernels).  The sum of the loaded words is
// stored only if it equals a constant, which keeps the loads.
__global__ __launch_bounds__(256) void k_line_reads(const uint4* tab, uint32_t line_mask, int iters, int share,
                                                    uint32_t* sink) {
    uint32_t h = ((blockIdx.x * 256u + threadIdx.x) / (uint32_t)share) * 2654435761u + 12345u;
    uint32_t acc = 0;
    for (int k = 0; k < iters; ++k) {
        h = h * 1664525u + 1013904223u;
        const uint4 a = tab[(size_t)((h >> 8) & line_mask) * 8];
        acc += a.x ^ a.w;
    }
    if (acc == 0x9e3779b9u) sink[0] = acc;
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_f64(double* p, double v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// explicit instantiations through launch wrappers
// ---------------------------------------------------------------------------
#define GRID(n, b) dim3((unsigned)(((n) + (b)-1) / (b)))

static inline unsigned grid8(int64_t n, int b) {
    int64_t g = (n + b - 1) / b;
    g = (g + 7) / 8 * 8;
    return (unsigned)(g > 0 ? g : 8);
}

void launch_begin(hipStream_t s, int32_t* counts, int nt, Scalars* sc, int do_sample, int n_ss,
                  unsigned long long* queue_n) {
    hipLaunchKernelGGL(k_begin, GRID(std::max(nt + 1, kQueueParts + kTileSlices), 256), dim3(256), 0, s, counts, nt, sc,
                       do_sample, n_ss, queue_n);
}

void launch_init_count(hipStream_t s, const double* vol, const int32_t* orig, int nt, double n0, double FN,
                       RngKey key, int32_t* counts, int32_t* counts_orig, const int32_t* cell_case,
                       const CaseDev* cases) {
    hipLaunchKernelGGL(k_init_count, GRID(nt, 256), dim3(256), 0, s, vol, orig, nt, n0, FN, key, counts,
                       counts_orig, cell_case, cases);
}

void launch_batch_pid_base(hipStream_t s, const int32_t* prefix, const int32_t* case_first, const int32_t* case_of_orig,
                           int nt, int32_t* out) {
    hipLaunchKernelGGL(k_batch_pid_base, GRID(nt, 256), dim3(256), 0, s, prefix, case_first, case_of_orig, nt, out);
}

void launch_batch_smax(hipStream_t s, const int32_t* cell_case, const CaseDev* cases, int nt, double* smax) {
    hipLaunchKernelGGL(k_batch_smax, GRID(nt, 256), dim3(256), 0, s, cell_case, cases, nt, smax);
}

template <class VT>
void launch_init_fill(hipStream_t s, const int4* tv, const double* xyz, int nt, const int32_t* offsets,
                      const int32_t* orig, const int32_t* pid_base, PartDev<VT> p, RngKey key, double sig,
                      const double* u0, int64_t cap, Scalars* sc, const int32_t* cell_case, const CaseDev* cases,
                      double T0) {
    hipLaunchKernelGGL(k_init_fill<VT>, GRID(nt, 128), dim3(128), 0, s, tv, xyz, nt, offsets, orig, pid_base, p,
                       key, sig, u0[0], u0[1], u0[2], cap, sc, cell_case, cases, T0);
}

// Workgroups of the persistent move: as many as the device holds at once
// (its occupancy on every CU), rounded down to a multiple of kTileSlices.
static int persist_grid() {
    static int cached = 0;
    if (cached) return cached;
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_move_persist<float, false>, 256, 0) != hipSuccess ||
        per_cu <= 0)
        per_cu = 4;
    const int g = cus * per_cu / kTileSlices * kTileSlices;
    cached = g > 0 ? g : kTileSlices;
    return cached;
}

template <class VT>
void launch_move(hipStream_t s, const MeshDev& m, PartDev<VT> p, const Scalars* sc, int32_t* counts,
                 uint32_t* rank, Counters* ctr, RngKey key, double dt, int64_t np_bound, int variant, int batch,
                 WallQueue wq, PartDev<VT> src, const int32_t* gperm) {
    if (gperm) {
        // the sort's gather folded into the move (three-face schedule)
        const dim3 g(grid8(np_bound, 256));
        if (m.surf)
            hipLaunchKernelGGL((k_move_defer<VT, 6, 0, true, true, true>), g, dim3(256), 0, s, m, p, (Scalars*)sc,
                               counts, rank, ctr, key, dt, wq, src, gperm);
        else
            hipLaunchKernelGGL((k_move_defer<VT, 7, 0, true, false, true>), g, dim3(256), 0, s, m, p, (Scalars*)sc,
                               counts, rank, ctr, key, dt, wq, src, gperm);
        return;
    }
    switch (variant) {
    case kMoveBatched: {
        const int b = batch > 0 ? batch : kMoveBatch;
        hipLaunchKernelGGL(k_move<VT>, dim3(grid8(np_bound, 4 * b)), dim3(256), 0, s, m, p, sc, counts, rank,
                           ctr, key, dt, b);
        break;
    }
    case kMoveLaneW8:
        hipLaunchKernelGGL((k_move_lane<VT, 8>), dim3(grid8(np_bound, 256)), dim3(256), 0, s, m, p, sc, counts,
                           rank, ctr, key, dt);
        break;
    case kMoveLaneW6:
        hipLaunchKernelGGL((k_move_lane<VT, 6>), dim3(grid8(np_bound, 256)), dim3(256), 0, s, m, p, sc, counts,
                           rank, ctr, key, dt);
        break;
    case kMoveDefer4:
    case kMoveDefer5:
    case kMoveDefer6:
    case kMoveDefer8: {
        const dim3 g(grid8(np_bound, 256));
        if (variant == kMoveDefer4)
            hipLaunchKernelGGL((k_move_defer<VT, 4, 0>), g, dim3(256), 0, s, m, p, (Scalars*)sc, counts, rank, ctr,
                               key, dt, wq, PartDev<VT>{}, nullptr);
        else if (variant == kMoveDefer5)
            hipLaunchKernelGGL((k_move_defer<VT, 5, 0>), g, dim3(256), 0, s, m, p, (Scalars*)sc, counts, rank, ctr,
                               key, dt, wq, PartDev<VT>{}, nullptr);
        else if (variant == kMoveDefer6)
            hipLaunchKernelGGL((k_move_defer<VT, 6, 0>), g, dim3(256), 0, s, m, p, (Scalars*)sc, counts, rank, ctr,
                               key, dt, wq, PartDev<VT>{}, nullptr);
        else
            hipLaunchKernelGGL((k_move_defer<VT, 8, 0>), g, dim3(256), 0, s, m, p, (Scalars*)sc, counts, rank, ctr,
                               key, dt, wq, PartDev<VT>{}, nullptr);
        break;
    }
    case kMoveFace3:
        if (m.surf)
            hipLaunchKernelGGL((k_move_defer<VT, 6, 0, true>), dim3(grid8(np_bound, 256)), dim3(256), 0, s, m, p,
                               (Scalars*)sc, counts, rank, ctr, key, dt, wq, PartDev<VT>{}, nullptr);
        else
            hipLaunchKernelGGL((k_move_defer<VT, 6, 0, true, false>), dim3(grid8(np_bound, 256)), dim3(256), 0, s,
                               m, p, (Scalars*)sc, counts, rank, ctr, key, dt, wq, PartDev<VT>{}, nullptr);
        break;
    case kMoveFace3W8:
        hipLaunchKernelGGL((k_move_defer<VT, 8, 0, true>), dim3(grid8(np_bound, 256)), dim3(256), 0, s, m, p,
                           (Scalars*)sc, counts, rank, ctr, key, dt, wq, PartDev<VT>{}, nullptr);
        break;
    case kMovePersist: {
        const dim3 g((unsigned)persist_grid());
        if (m.surf)
            hipLaunchKernelGGL((k_move_persist<VT, true>), g, dim3(256), 0, s, m, p, (Scalars*)sc, counts, rank, ctr,
                               key, dt, wq);
        else
            hipLaunchKernelGGL((k_move_persist<VT, false>), g, dim3(256), 0, s, m, p, (Scalars*)sc, counts, rank,
                               ctr, key, dt, wq);
        break;
    }
    case kMoveCap4:
    case kMoveCap5:
    case kMoveCap6: {
        const dim3 g(grid8(np_bound, 256));
        if (variant == kMoveCap4)
            hipLaunchKernelGGL((k_move_defer<VT, 6, 4, true>), g, dim3(256), 0, s, m, p, (Scalars*)sc, counts, rank,
                               ctr, key, dt, wq, PartDev<VT>{}, nullptr);
        else if (variant == kMoveCap5)
            hipLaunchKernelGGL((k_move_defer<VT, 6, 5, true>), g, dim3(256), 0, s, m, p, (Scalars*)sc, counts, rank,
                               ctr, key, dt, wq, PartDev<VT>{}, nullptr);
        else
            hipLaunchKernelGGL((k_move_defer<VT, 6, 6, true>), g, dim3(256), 0, s, m, p, (Scalars*)sc, counts, rank,
                               ctr, key, dt, wq, PartDev<VT>{}, nullptr);
        break;
    }
    case kMovePool128:
    case kMovePool256: {
        if (variant == kMovePool128)
            hipLaunchKernelGGL((k_move_pool<VT, 6, 128>), dim3(grid8(np_bound, 4 * 128)), dim3(256), 0, s, m, p,
                               (Scalars*)sc, counts, rank, ctr, key, dt, wq);
        else
            hipLaunchKernelGGL((k_move_pool<VT, 4, 256>), dim3(grid8(np_bound, 4 * 256)), dim3(256), 0, s, m, p,
                               (Scalars*)sc, counts, rank, ctr, key, dt, wq);
        break;
    }
    case kMoveRefill5:
    case kMoveRefill6: {
        const int b = batch > 0 ? batch : kMoveBatch;
        const dim3 g(grid8(np_bound, 4 * b));
        if (variant == kMoveRefill5)
            hipLaunchKernelGGL((k_move_refill<VT, 5>), g, dim3(256), 0, s, m, p, (Scalars*)sc, counts, rank, ctr, key,
                               dt, wq, b);
        else
            hipLaunchKernelGGL((k_move_refill<VT, 6>), g, dim3(256), 0, s, m, p, (Scalars*)sc, counts, rank, ctr, key,
                               dt, wq, b);
        break;
    }
    default:
        hipLaunchKernelGGL((k_move_lane<VT, 1>), dim3(grid8(np_bound, 256)), dim3(256), 0, s, m, p, sc, counts,
                           rank, ctr, key, dt);
        break;
    }
}

template <class VT>
void launch_move_walls(hipStream_t s, const MeshDev& m, PartDev<VT> p, const Scalars* sc, int32_t* counts,
                       uint32_t* rank, Counters* ctr, RngKey key, WallQueue wq) {
    hipLaunchKernelGGL(k_move_walls<VT>, dim3(1024), dim3(256), 0, s, m, p, sc, counts, rank, ctr, key, wq);
}

bool move_parks_walls(int variant) {
    return variant == kMoveDefer4 || variant == kMoveDefer5 || variant == kMoveDefer6 || variant == kMoveDefer8 ||
           variant == kMoveCap4 || variant == kMoveCap5 || variant == kMoveCap6 || variant == kMoveFace3 || variant == kMoveFace3W8 ||
           variant == kMovePool128 || variant == kMovePool256 || variant == kMoveRefill5 || variant == kMoveRefill6 ||
           variant == kMovePersist;
}

void launch_count(hipStream_t s, const int32_t* cell, const Scalars* sc, int32_t* counts, uint32_t* rank,
                  int64_t np_bound) {
    hipLaunchKernelGGL(k_count, GRID(np_bound > 0 ? np_bound : 1, 256), dim3(256), 0, s, cell, sc, counts,
                       rank);
}

void launch_inject_count(hipStream_t s, const InflowDev& in, const Scalars* sc, RngKey key, int32_t* fcount) {
    hipLaunchKernelGGL(k_inject_count, GRID(in.n, 256), dim3(256), 0, s, in, sc, key, fcount);
}

template <class VT>
void launch_inject_emit(hipStream_t s, const MeshDev& m, const InflowDev& in, PartDev<VT> p, Scalars* sc,
                        const int32_t* foff, int32_t* counts, uint32_t* rank, Counters* ctr, RngKey key,
                        double dt, int64_t cap, int64_t max_inject) {
    hipLaunchKernelGGL(k_inject_emit<VT>, GRID(max_inject > 0 ? max_inject : 1, 256), dim3(256), 0, s, m, in,
                       p, sc, foff, counts, rank, ctr, key, dt, cap);
}

void launch_scan(hipStream_t s, const int32_t* in, int64_t n, int32_t* out, int32_t* blocksums, Scalars* sc,
                 int mode) {
    const int nblk = (int)((n + kScanBlock - 1) / kScanBlock);
    const int nb = nblk > 0 ? nblk : 1;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanThreads), 0, s, in, n, blocksums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, blocksums, nb, sc, mode, out + n);
    hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kScanThreads), 0, s, in, n, blocksums, out);
}

template <class VT>
void launch_scatter(hipStream_t s, PartDev<VT> src, PartDev<VT> dst, const Scalars* sc, const int32_t* offsets,
                    const uint32_t* rank, int64_t bound, int64_t cap, int32_t* perm, int variant) {
    if (variant != kSortScatter) {
        hipLaunchKernelGGL(k_perm, dim3(grid8(bound, 256)), dim3(256), 0, s, src.cell, sc, offsets, rank, perm,
                           dst.cell, cap);
    } else {
        hipLaunchKernelGGL(k_scatter<VT>, dim3(grid8(bound, 256)), dim3(256), 0, s, src, dst, sc, offsets, rank, cap);
    }
}

template <class VT>
void launch_gather(hipStream_t s, PartDev<VT> src, PartDev<VT> dst, const Scalars* sc, const int32_t* perm,
                   int64_t bound) {
    hipLaunchKernelGGL(k_gather<VT>, dim3(grid8(bound, 256)), dim3(256), 0, s, src, dst, sc, perm);
}

void launch_perm_identity(hipStream_t s, const int32_t* cell, const Scalars* sc, int32_t* perm, int32_t* dst_cell,
                          int64_t bound) {
    hipLaunchKernelGGL(k_perm_identity, dim3(grid8(bound, 256)), dim3(256), 0, s, cell, sc, perm, dst_cell);
}

template <class VT, int WPE, int CAP, bool VSS, bool ROT>
static void launch_collide_g(hipStream_t s, int nchunk, PartDev<VT> p, const int32_t* offsets, const CollideParams& cp,
                             const Scalars* sc, int32_t* perm, int do_collide, int do_sample, int gmode,
                             PartDev<VT> src, const int32_t* sortperm) {
    if (gmode == kGatherIndirect) {
        hipLaunchKernelGGL((k_collide_sample_g<VT, WPE, CAP, kGatherIndirect, VSS, ROT>), dim3(nchunk),
                           dim3(kCollideLanes), 0, s, p, offsets, cp, sc, perm, do_collide, do_sample, src, sortperm);
    } else if constexpr (ROT) {
        // a rotating gas never takes the fused gather (the host refuses that schedule)
        hipLaunchKernelGGL((k_collide_sample_g<VT, WPE, CAP, kGatherNone, VSS, true>), dim3(nchunk),
                           dim3(kCollideLanes), 0, s, p, offsets, cp, sc, perm, do_collide, do_sample, src, sortperm);
    } else if (gmode == kGatherFused) {
        hipLaunchKernelGGL((k_collide_sample_g<VT, WPE, CAP, kGatherFused, VSS>), dim3(nchunk), dim3(kCollideLanes), 0,
                           s, p, offsets, cp, sc, perm, do_collide, do_sample, src, sortperm);
    } else {
        hipLaunchKernelGGL((k_collide_sample_g<VT, WPE, CAP, kGatherNone, VSS>), dim3(nchunk), dim3(kCollideLanes), 0,
                           s, p, offsets, cp, sc, perm, do_collide, do_sample, src, sortperm);
    }
}

bool collide_fuses_gather(int variant) {
    return variant == kCollideGlobal || variant == kCollideGlobal8 || variant == kCollideG3k || variant == kCollideG2k;
}

// Waves per SIMD the collide kernels are compiled for.  The chunk's pid
// table (18.7 KB of LDS at 3072 particles) already holds a one-wave
// workgroup to two waves per SIMD; the rotating gas's instances ask for two,
// so that the compiler keeps them within 256 registers (asked for more, they
// took 263 and ran at one wave per SIMD).
constexpr int collide_wpe(int w, bool rot) { return rot ? 2 : w; }

template <class VT, bool VSS, bool ROT>
static void launch_collide_v(hipStream_t s, PartDev<VT> p, const int32_t* offsets, const CollideParams& cp,
                             const Scalars* sc, int32_t* perm, int do_collide, int do_sample, int variant, int gmode,
                             PartDev<VT> src, const int32_t* sortperm) {
    const int nchunk = (cp.nt + kCollideLanes - 1) / kCollideLanes;
    if (variant == kCollideGlobal)
        launch_collide_g<VT, collide_wpe(4, ROT), kCollideCapG, VSS, ROT>(s, nchunk, p, offsets, cp, sc, perm, do_collide, do_sample,
                                                        gmode, src, sortperm);
    else if (variant == kCollideGlobal8)
        launch_collide_g<VT, collide_wpe(8, ROT), kCollideCapG, VSS, ROT>(s, nchunk, p, offsets, cp, sc, perm, do_collide, do_sample,
                                                        gmode, src, sortperm);
    else if (variant == kCollideG3k)
        launch_collide_g<VT, collide_wpe(4, ROT), 3072, VSS, ROT>(s, nchunk, p, offsets, cp, sc, perm, do_collide, do_sample, gmode, src,
                                                sortperm);
    else if (variant == kCollideG2k)
        launch_collide_g<VT, collide_wpe(4, ROT), 2048, VSS, ROT>(s, nchunk, p, offsets, cp, sc, perm, do_collide, do_sample, gmode, src,
                                                sortperm);
    else if constexpr (!ROT)
        hipLaunchKernelGGL((k_collide_sample<VT, VSS>), dim3(nchunk), dim3(kCollideLanes), 0, s, p, offsets, cp, sc,
                           perm, do_collide, do_sample);
}

template <class VT>
void launch_collide_sample(hipStream_t s, PartDev<VT> p, const int32_t* offsets, const CollideParams& cp,
                           const Scalars* sc, int32_t* perm, int do_collide, int do_sample, int variant, int gmode,
                           PartDev<VT> src, const int32_t* sortperm) {
    if (cp.rot) {
        if (cp.vss)
            launch_collide_v<VT, true, true>(s, p, offsets, cp, sc, perm, do_collide, do_sample, variant, gmode, src,
                                             sortperm);
        else
            launch_collide_v<VT, false, true>(s, p, offsets, cp, sc, perm, do_collide, do_sample, variant, gmode, src,
                                              sortperm);
    } else if (cp.vss) {
        launch_collide_v<VT, true, false>(s, p, offsets, cp, sc, perm, do_collide, do_sample, variant, gmode, src, sortperm);
    } else {
        launch_collide_v<VT, false, false>(s, p, offsets, cp, sc, perm, do_collide, do_sample, variant, gmode, src,
                                           sortperm);
    }
}

void launch_fields(hipStream_t s, const double* sums, int nt, double ns, double mass, double FN,
                   const double* vol, const int32_t* orig, double* out, const int32_t* cell_case,
                   const CaseDev* cases) {
    hipLaunchKernelGGL(k_fields, GRID(nt, 256), dim3(256), 0, s, sums, nt, ns, mass, FN, vol, orig, out, cell_case,
                       cases);
}

void launch_philox(hipStream_t s, const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out, int64_t n) {
    hipLaunchKernelGGL(k_philox, GRID(n, 256), dim3(256), 0, s, ctr, k0, k1, out, n);
}

void launch_copy(hipStream_t s, const void* src, void* dst, size_t bytes) {
    const int64_t n16 = (int64_t)(bytes / 16);
    if (n16 > 0)
        hipLaunchKernelGGL(k_copy16, dim3((unsigned)((n16 + 1023) / 1024)), dim3(256), 0, s, (const uint4*)src,
                           (uint4*)dst, n16);
}

void launch_line_reads(hipStream_t s, const void* table, uint32_t line_mask, int iters, int share, int blocks,
                       void* sink) {
    hipLaunchKernelGGL(k_line_reads, dim3((unsigned)blocks), dim3(256), 0, s, (const uint4*)table, line_mask, iters,
                       share, (uint32_t*)sink);
}

void launch_fill_i32(hipStream_t s, int32_t* p, int32_t v, int64_t n) {
    if (n > 0) hipLaunchKernelGGL(k_fill_i32, GRID(n, 256), dim3(256), 0, s, p, v, n);
}

void launch_fill_f64(hipStream_t s, double* p, double v, int64_t n) {
    if (n > 0) hipLaunchKernelGGL(k_fill_f64, GRID(n, 256), dim3(256), 0, s, p, v, n);
}

#define INSTANTIATE(VT)                                                                                      \
    template void launch_init_fill<VT>(hipStream_t, const int4*, const double*, int, const int32_t*,       \
                                       const int32_t*, const int32_t*, PartDev<VT>, RngKey, double,         \
                                       const double*, int64_t, Scalars*, const int32_t*, const CaseDev*,    \
                                       double);                                                             \
    template void launch_move<VT>(hipStream_t, const MeshDev&, PartDev<VT>, const Scalars*, int32_t*,       \
                                  uint32_t*, Counters*, RngKey, double, int64_t, int, int, WallQueue,       \
                                  PartDev<VT>, const int32_t*);                                             \
    template void launch_inject_emit<VT>(hipStream_t, const MeshDev&, const InflowDev&, PartDev<VT>,        \
                                         Scalars*, const int32_t*, int32_t*, uint32_t*, Counters*, RngKey,  \
                                         double, int64_t, int64_t);                                         \
    template void launch_scatter<VT>(hipStream_t, PartDev<VT>, PartDev<VT>, const Scalars*, const int32_t*, \
                                     const uint32_t*, int64_t, int64_t, int32_t*, int);                                           \
    template void launch_move_walls<VT>(hipStream_t, const MeshDev&, PartDev<VT>, const Scalars*, int32_t*,  \
                                        uint32_t*, Counters*, RngKey, WallQueue);                           \
    template void launch_gather<VT>(hipStream_t, PartDev<VT>, PartDev<VT>, const Scalars*, const int32_t*,  \
                                    int64_t);                                                               \
    template void launch_collide_sample<VT>(hipStream_t, PartDev<VT>, const int32_t*, const CollideParams&, \
                                            const Scalars*, int32_t*, int, int, int, int, PartDev<VT>,        \
                                            const int32_t*);

INSTANTIATE(float)
INSTANTIATE(double)

}  // namespace dsmcx
