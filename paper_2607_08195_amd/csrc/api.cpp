// C ABI of the DSMC library: context lifetime, device memory, the per-step
// launch sequence, state import/export and statistics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/dsmc.h"
#include "context.h"

using namespace dsmcx;

namespace {

enum Slot {
    kSlotBegin = 0, kSlotMove, kSlotWalls, kSlotInject, kSlotScan, kSlotScatter, kSlotGather, kSlotCollide, kNumSlots
};
// one slot per kernel (or per fixed kernel group) of the step
const char* kSlotNames[kNumSlots] = {"begin", "move", "move_walls", "inject", "scan", "sort_perm", "sort_gather",
                                     "collide_sample"};

std::string g_global_error;

}  // namespace

namespace dsmcx {

dsmc_status fail(dsmc_ctx c, dsmc_status s, const std::string& msg) {
    if (c) c->err = msg; else g_global_error = msg;
    return s;
}

void* dev_alloc(dsmc_ctx c, size_t bytes) {
    if (bytes == 0) bytes = 16;
    void* p = nullptr;
    if (c->has_alloc) {
        p = c->alloc.alloc(bytes, c->alloc.user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p) c->owned.push_back(p);
    return p;
}

void dev_free(dsmc_ctx c, void* p) {
    if (!p) return;
    auto it = std::find(c->owned.begin(), c->owned.end(), p);
    if (it != c->owned.end()) c->owned.erase(it);
    if (c->has_alloc) c->alloc.free(p, c->alloc.user); else hipFree(p);
}

dsmc_status sync_scalars(dsmc_ctx c, Scalars* out) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    Scalars s;
    HIP_TRY(c, hipMemcpy(&s, c->d_sc, sizeof s, hipMemcpyDeviceToHost));
    c->np_bound = s.np;
    if (out) *out = s;
    if (s.flags & kFlagCapacity) {
        c->broken = true;
        return fail(c, DSMC_E_CAPACITY, "particle store capacity exceeded");
    }
    return DSMC_OK;
}

}  // namespace dsmcx

namespace {

bool alloc_buf(dsmc_ctx c, Buf& b, int64_t cap, int vel64) {
    const size_t vs = vel64 ? sizeof(double) : sizeof(float);
    return alloc_n(c, b.pos, 3 * (size_t)cap) && (b.vel = dev_alloc(c, vs * 3 * (size_t)cap)) &&
           alloc_n(c, b.cell, cap) && alloc_n(c, b.pid, cap);
}

hipEvent_t get_event(dsmc_ctx c) {
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct Timed {
    dsmc_ctx c;
    int slot;
    hipEvent_t a = nullptr, b = nullptr;
    Timed(dsmc_ctx c_, int s) : c(c_), slot(s) {
        if (c->profiling && !c->capturing) {
            a = get_event(c);
            b = get_event(c);
            if (a) hipEventRecord(a, c->stream);
        }
    }
    ~Timed() {
        if (c->profiling && !c->capturing && a && b) {
            hipEventRecord(b, c->stream);
            c->ev_used.push_back({slot, {a, b}});
        }
    }
};

CollideParams collide_params(dsmc_ctx c) {
    CollideParams cp;
    cp.nt = c->nt; cp.n_ss = c->n_ss; cp.n_a = c->n_a; cp.ewma_on = c->ewma_on;
    cp.key = c->key; cp.FN = c->FN; cp.dt = c->dt; cp.K = c->K; cp.ex = c->ex;
    cp.vss = c->alpha != 1.0; cp.inv_alpha = 1.0 / c->alpha;
    cp.vol = c->d_vol; cp.smax = c->d_smax; cp.ncand = c->d_ncand; cp.nacc = c->d_nacc;
    cp.acc = c->d_acc; cp.ewma = c->d_ewma; cp.ewma_m = c->d_ewma_m; cp.local_acc = c->d_local;
    cp.inst = c->inst_on ? c->d_inst : nullptr;
    cp.orig = c->d_orig;
    cp.cell_case = c->d_cell_case;
    cp.cases = c->d_cases;
    cp.rot = c->dr ? 1 : 0;
    cp.pinel = c->pinel;
    cp.ex_bl = 1.0 / (2.5 - c->omega);
    cp.mass = c->mass;
    cp.racc = c->d_racc;
    cp.rewma = c->d_rewma;
    cp.rinst = c->dr && c->inst_on ? c->d_rinst : nullptr;
    return cp;
}

// The deferred sort needs the three-face move and an LDS-ranked collide.
bool deferred_ok(int move, int collide) { return move == kMoveFace3 && collide_fuses_gather(collide); }

}  // namespace

namespace dsmcx {

// Writes the pending sorted order of a deferred sort out to B and swaps, so
// that A is sorted by cell again (for calls that read or rebuild the store).
dsmc_status materialize(dsmc_ctx c) {
    if (!c->pending) return DSMC_OK;
    if (c->vel64)
        launch_gather<double>(c->stream, as_dev<double>(c->A), as_dev<double>(c->B), c->d_sc, c->d_sortperm,
                              c->np_bound);
    else
        launch_gather<float>(c->stream, as_dev<float>(c->A), as_dev<float>(c->B), c->d_sc, c->d_sortperm,
                             c->np_bound);
    std::swap(c->A, c->B);
    c->pending = false;
    HIP_TRY(c, hipGetLastError());
    return DSMC_OK;
}

}  // namespace dsmcx

namespace {

// Gives a sorted store the identity order, so that a deferred step can
// start from it.
void ensure_pending(dsmc_ctx c) {
    if (c->pending) return;
    launch_perm_identity(c->stream, c->A.cell, c->d_sc, c->d_sortperm, c->B.cell, c->np_bound);
    c->pending = true;
}

// One step with the deferred sort: the move reads the particles in the
// previous step's sorted order and writes them in it (k_move_defer's gather
// form, into B, which then becomes A); the sort only computes the new order;
// the collide kernel reaches the particles through it.
template <class VT>
dsmc_status run_step_deferred(dsmc_ctx c, bool inj, bool col, bool smp, int64_t need) {
    hipStream_t s = c->stream;
    if (!c->capturing) ensure_pending(c);
    PartDev<VT> a = as_dev<VT>(c->A), b = as_dev<VT>(c->B);
    {
        Timed t(c, kSlotBegin);
        launch_begin(s, c->d_counts, c->nt, c->d_sc, smp ? 1 : 0, c->n_ss, c->wq.n);
    }
    {
        Timed t(c, kSlotMove);
        launch_move<VT>(s, c->mesh, b, c->d_sc, c->d_counts, c->d_rank, c->d_ctr, c->key, c->dt,
                        c->capturing ? c->capture_bound : c->np_bound, c->move_variant, c->move_batch, c->wq, a,
                        c->d_sortperm);
    }
    std::swap(c->A, c->B);
    std::swap(a, b);
    {
        Timed t(c, kSlotWalls);
        launch_move_walls<VT>(s, c->mesh, a, c->d_sc, c->d_counts, c->d_rank, c->d_ctr, c->key, c->wq);
    }
    if (inj) {
        Timed t(c, kSlotInject);
        launch_inject_count(s, c->inflow, c->d_sc, c->key, c->d_fcount);
        launch_scan(s, c->d_fcount, c->inflow.n, c->d_foff, c->d_blocksums, c->d_sc, kScanInject);
        launch_inject_emit<VT>(s, c->mesh, c->inflow, a, c->d_sc, c->d_foff, c->d_counts, c->d_rank, c->d_ctr,
                               c->key, c->dt, c->cap, c->max_inject);
    }
    {
        Timed t(c, kSlotScan);
        launch_scan(s, c->d_counts, c->nt, c->d_offsets, c->d_blocksums, c->d_sc, kScanCells);
    }
    {
        Timed t(c, kSlotScatter);
        launch_scatter<VT>(s, a, b, c->d_sc, c->d_offsets, c->d_rank, need, c->cap, c->d_sortperm, kSortDeferred);
    }
    c->np_bound = need;
    {
        Timed t(c, kSlotCollide);
        const CollideParams cp = collide_params(c);
        launch_collide_sample<VT>(s, a, c->d_offsets, cp, c->d_sc, c->d_perm, col ? 1 : 0, smp ? 1 : 0,
                                  c->collide_variant, kGatherIndirect, b, c->d_sortperm);
    }
    c->pending = true;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        c->broken = true;
        return fail(c, DSMC_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    }
    return DSMC_OK;
}

template <class VT>
dsmc_status run_step(dsmc_ctx c, int mask) {
    const bool mv = mask & 1, inj = (mask & 2) && c->inflow.n > 0, srt = mask & 4, col = mask & 8,
               smp = mask & 16;
    if ((col || smp) && mv && !srt) return fail(c, DSMC_E_INVALID, "collide/sample after move needs sort");
    const bool defer = c->sort_variant == kSortDeferred && deferred_ok(c->move_variant, c->collide_variant) && mv &&
                       srt && (col || smp);
    if (!defer && c->pending) {
        // a partial step works on the sorted store
        dsmc_status st = materialize(c);
        if (st != DSMC_OK) return st;
    }
    // Under graph capture nothing may synchronise: grids cover the capture
    // bound and the kernels bound themselves by the device-side counts.
    const int64_t need = c->capturing ? c->capture_bound : c->np_bound + (inj ? c->max_inject : 0);
    if (!c->capturing && need > c->cap) {
        dsmc_status st = sync_scalars(c, nullptr);
        if (st != DSMC_OK) return st;
        if (c->np_bound + (inj ? c->max_inject : 0) > c->cap)
            return fail(c, DSMC_E_CAPACITY, "particle store capacity would be exceeded");
    }
    if (defer) return run_step_deferred<VT>(c, inj, col, smp, need);
    hipStream_t s = c->stream;
    PartDev<VT> a = as_dev<VT>(c->A), b = as_dev<VT>(c->B);
    bool fuse = false;  // the collide kernel gathers the sorted buffer
    {
        Timed t(c, kSlotBegin);
        launch_begin(s, c->d_counts, c->nt, c->d_sc, smp ? 1 : 0, c->n_ss, c->wq.n);
    }
    if (mv) {
        Timed t(c, kSlotMove);
        launch_move<VT>(s, c->mesh, a, c->d_sc, c->d_counts, c->d_rank, c->d_ctr, c->key, c->dt,
                        c->capturing ? c->capture_bound : c->np_bound, c->move_variant, c->move_batch, c->wq);
    }
    if (mv && move_parks_walls(c->move_variant)) {
        Timed t(c, kSlotWalls);
        launch_move_walls<VT>(s, c->mesh, a, c->d_sc, c->d_counts, c->d_rank, c->d_ctr, c->key, c->wq);
    }
    if (inj) {
        Timed t(c, kSlotInject);
        launch_inject_count(s, c->inflow, c->d_sc, c->key, c->d_fcount);
        launch_scan(s, c->d_fcount, c->inflow.n, c->d_foff, c->d_blocksums, c->d_sc, kScanInject);
        launch_inject_emit<VT>(s, c->mesh, c->inflow, a, c->d_sc, c->d_foff, c->d_counts, c->d_rank, c->d_ctr,
                               c->key, c->dt, c->cap, c->max_inject);
    }
    if (srt) {
        if (!mv && !inj)
            launch_count(s, a.cell, c->d_sc, c->d_counts, c->d_rank, c->capturing ? c->capture_bound : c->np_bound);
        {
            Timed t(c, kSlotScan);
            launch_scan(s, c->d_counts, c->nt, c->d_offsets, c->d_blocksums, c->d_sc, kScanCells);
        }
        {
            Timed t(c, kSlotScatter);
            launch_scatter<VT>(s, a, b, c->d_sc, c->d_offsets, c->d_rank, need, c->cap, c->d_sortperm, c->sort_variant);
        }
        fuse = c->sort_variant == kSortFused && (col || smp) && collide_fuses_gather(c->collide_variant);
        if (c->sort_variant != kSortScatter && !fuse) {
            Timed t(c, kSlotGather);
            launch_gather<VT>(s, a, b, c->d_sc, c->d_sortperm, need);
        }
        std::swap(c->A, c->B);
        a = as_dev<VT>(c->A);
        c->np_bound = need;
    }
    if (col || smp) {
        Timed t(c, kSlotCollide);
        const CollideParams cp = collide_params(c);
        launch_collide_sample<VT>(s, a, c->d_offsets, cp, c->d_sc, c->d_perm, col ? 1 : 0, smp ? 1 : 0,
                                  c->collide_variant, fuse ? kGatherFused : kGatherNone,
                                  fuse ? as_dev<VT>(c->B) : PartDev<VT>{}, c->d_sortperm);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        c->broken = true;
        return fail(c, DSMC_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    }
    return DSMC_OK;
}

dsmc_status step_any(dsmc_ctx c, int mask) {
    return c->vel64 ? run_step<double>(c, mask) : run_step<float>(c, mask);
}

// Schedules that carry the rotational energy of a rotating gas: the
// parked-wall move kernels (their main pass stops at diffuse walls, whose
// re-emission, rotation included, the walls pass makes), the LDS-ranked
// collide kernels and the scatter or gather sort.
bool rot_schedule_ok(int move, int collide, int sort) {
    const bool mv = move == kMoveDefer4 || move == kMoveDefer5 || move == kMoveDefer6 || move == kMoveDefer8 ||
                    move == kMoveCap4 || move == kMoveCap5 || move == kMoveCap6 || move == kMoveFace3 ||
                    move == kMoveFace3W8 || move == kMovePersist;
    const bool co = collide == kCollideGlobal || collide == kCollideGlobal8 || collide == kCollideG3k ||
                    collide == kCollideG2k;
    const bool so = sort == kSortScatter || sort == kSortGather || (sort == kSortDeferred && deferred_ok(move, collide));
    return mv && co && so;
}

// Move schedules that read the per-case tables of a batch (lane, parked-wall
// and capped parked-wall kernels).
bool move_reads_cases(int v) {
    return v == kMoveLane || v == kMoveLaneW6 || v == kMoveLaneW8 || v == kMoveDefer4 || v == kMoveDefer5 ||
           v == kMoveDefer6 || v == kMoveDefer8 || v == kMoveCap4 || v == kMoveCap5 || v == kMoveCap6 ||
           v == kMoveFace3 || v == kMoveFace3W8 || v == kMovePersist;
}

// Tuning overrides from the environment: DSMC_MOVE (lane, lane6, lane8,
// batched, defer4/5/6/8, face3, face3w8, cap4/5/6, refill5/6, pool128/256), DSMC_MOVE_BATCH,
// DSMC_REORDER (0/1), DSMC_SORT, DSMC_COLLIDE.
void read_tuning(dsmc_ctx c) {
    if (const char* v = std::getenv("DSMC_MOVE")) {
        std::string s(v);
        if (s == "lane") c->move_variant = kMoveLane;
        else if (s == "lane6") c->move_variant = kMoveLaneW6;
        else if (s == "lane8") c->move_variant = kMoveLaneW8;
        else if (s == "batched") c->move_variant = kMoveBatched;
        else if (s == "defer6") c->move_variant = kMoveDefer6;
        else if (s == "defer8") c->move_variant = kMoveDefer8;
        else if (s == "defer4") c->move_variant = kMoveDefer4;
        else if (s == "defer5") c->move_variant = kMoveDefer5;
        else if (s == "refill5") c->move_variant = kMoveRefill5;
        else if (s == "refill6") c->move_variant = kMoveRefill6;
        else if (s == "pool128") c->move_variant = kMovePool128;
        else if (s == "pool256") c->move_variant = kMovePool256;
        else if (s == "cap4") c->move_variant = kMoveCap4;
        else if (s == "cap5") c->move_variant = kMoveCap5;
        else if (s == "cap6") c->move_variant = kMoveCap6;
        else if (s == "face3") c->move_variant = kMoveFace3;
        else if (s == "face3w8") c->move_variant = kMoveFace3W8;
        else if (s == "persist") c->move_variant = kMovePersist;
    }
    if (const char* v = std::getenv("DSMC_MOVE_BATCH"))
        c->move_batch = std::min(kQueueMaxBatch, std::max(64, std::atoi(v) / 64 * 64));
    if (const char* v = std::getenv("DSMC_REORDER")) c->reorder = std::atoi(v);
    if (const char* v = std::getenv("DSMC_SORT")) {
        const std::string k(v);
        c->sort_variant = k == "scatter"  ? kSortScatter
                          : k == "fused"    ? kSortFused
                          : k == "deferred" ? kSortDeferred
                                            : kSortGather;
    }
    if (const char* v = std::getenv("DSMC_COLLIDE")) {
        std::string s(v);
        if (s == "lds") c->collide_variant = kCollideLds;
        else if (s == "global") c->collide_variant = kCollideGlobal;
        else if (s == "global8") c->collide_variant = kCollideGlobal8;
        else if (s == "global3k") c->collide_variant = kCollideG3k;
        else if (s == "global2k") c->collide_variant = kCollideG2k;
    }
}


int tuning_sig(dsmc_ctx c) {
    return c->move_variant | (c->collide_variant << 8) | (c->sort_variant << 12) | (c->mesh.surf ? 1 << 16 : 0) |
           (c->inst_on ? 1 << 17 : 0);
}

void drop_graph(dsmc_ctx_s::Graph& g) {
    if (g.exec) hipGraphExecDestroy(g.exec);
    if (g.graph) hipGraphDestroy(g.graph);
    g = dsmc_ctx_s::Graph{};
}

// Record two full steps (the buffers swap twice, so a replay leaves them as
// it found them) into a graph and instantiate it.  Without inflow the
// particle count cannot grow inside a step, so the grids cover the exact
// count at capture time (a replay with more particles captures again);
// with inflow they cover the whole store.  (Grids over the whole store of
// a closed cavity, twice its particles, cost about 1 ms per step of blocks
// that exit at once.)
dsmc_status capture_two_steps(dsmc_ctx c, dsmc_ctx_s::Graph& g) {
    drop_graph(g);
    if (c->inflow.n > 0) {
        c->capture_bound = c->cap;
    } else {
        dsmc_status st = sync_scalars(c, nullptr);
        if (st != DSMC_OK) return st;
        c->capture_bound = std::max<int64_t>(c->np_bound, 1);
    }
    if (c->sort_variant == kSortDeferred && deferred_ok(c->move_variant, c->collide_variant)) ensure_pending(c);
    const void* a_x = c->A.pos;
    HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    c->capturing = true;
    dsmc_status st = step_any(c, 31);
    if (st == DSMC_OK) st = step_any(c, 31);
    c->capturing = false;
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(c->stream, &graph);
    if (st != DSMC_OK) {
        if (graph) hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess || !graph) {
        c->broken = true;
        return fail(c, DSMC_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    g.graph = graph;
    HIP_TRY(c, hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0));
    g.a_x = a_x;
    g.sig = tuning_sig(c);
    g.bound = c->capture_bound;
    return DSMC_OK;
}

// Mean milliseconds per step of the given profile slots over `steps` steps.
dsmc_status time_slots(dsmc_ctx c, int steps, std::initializer_list<int> slots, double* ms) {
    dsmc_status st = step_any(c, 31);  // untimed warm-up with the candidate
    if (st != DSMC_OK) return st;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (auto& u : c->ev_used) {
        c->ev_pool.push_back(u.second.first);
        c->ev_pool.push_back(u.second.second);
    }
    c->ev_used.clear();
    c->profiling = true;
    for (int i = 0; i < steps && st == DSMC_OK; ++i) st = step_any(c, 31);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    double tot = 0;
    for (auto& u : c->ev_used) {
        float t = 0;
        for (int sl : slots)
            if (u.first == sl && hipEventElapsedTime(&t, u.second.first, u.second.second) == hipSuccess) tot += t;
    }
    c->profiling = false;
    *ms = tot / std::max(1, steps);
    return st;
}

template <class VT>
void fill_dispatch(dsmc_ctx c, double sig) {
    const int32_t* pid_base = c->d_cell_case ? c->d_counts_orig : c->d_cell_tmp;
    launch_init_fill<VT>(c->stream, c->d_tv, c->d_xyz, c->nt, c->d_offsets, c->d_orig, pid_base, as_dev<VT>(c->A),
                         c->key, sig, c->u0, c->cap, c->d_sc, c->d_cell_case, c->d_cases, c->T0);
}

// Cases of a batch: per-case run parameters, the case of every cell of the
// union mesh (caller numbering) and the first cell of each case.
struct BatchSpec {
    std::vector<dsmc_run_desc> runs;
    std::vector<int32_t> tet_case;
    std::vector<int32_t> cell0;
};

}  // namespace

// ===========================================================================
// Context construction shared by the single-case and the batch entry points.
// With a batch, `run` carries the batch-wide settings (velocity storage,
// sampling, capacity, stream, allocator, fill) and bs the per-case ones.
dsmc_status init_impl(dsmc_ctx* out, const dsmc_mesh_desc* mesh, const dsmc_species_desc* sp, int32_t n_bc,
                      const dsmc_boundary_desc* bcs, const dsmc_run_desc* run, const BatchSpec* bs) {
    if (!out) return fail(nullptr, DSMC_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!mesh || !sp || !run || (n_bc > 0 && !bcs) || n_bc < 0)
        return fail(nullptr, DSMC_E_INVALID, "NULL descriptor");
    if (!(sp->mass > 0) || !(sp->d_ref > 0) || !(sp->T_ref > 0) || !(sp->alpha > 0) || !(run->F_N > 0) ||
        !(run->dt > 0))
        return fail(nullptr, DSMC_E_INVALID, "non-positive physical parameter");
    if (!(sp->dof_rot == 0 || sp->dof_rot == 2) || (sp->dof_rot == 2 && !(sp->z_rot > 0)))
        return fail(nullptr, DSMC_E_INVALID, "rotational degrees of freedom must be 0 or 2 (with z_rot > 0)");
    if (run->n_a < 1) return fail(nullptr, DSMC_E_INVALID, "n_a must be >= 1");
    for (int g = 0; g < n_bc; ++g)
        if (bcs[g].kind < 0 || bcs[g].kind > 4) return fail(nullptr, DSMC_E_INVALID, "bad boundary kind");

    dsmc_ctx c = new dsmc_ctx_s();
    c->stream = (hipStream_t)run->hip_stream;
    if (run->allocator) {
        if (!run->allocator->alloc || !run->allocator->free) {
            delete c;
            return fail(nullptr, DSMC_E_INVALID, "allocator callbacks missing");
        }
        c->alloc = *run->allocator;
        c->has_alloc = true;
    }
    std::string merr = build_mesh(c->hm, mesh->n_vertices, mesh->xyz, mesh->n_tets, mesh->tet_vtx, mesh->n_bfaces,
                                  mesh->bface_vtx, mesh->bface_group, mesh->bface_partner, n_bc);
    if (!merr.empty()) {
        delete c;
        return fail(nullptr, DSMC_E_MESH, merr);
    }
    HostMesh& hm = c->hm;
    read_tuning(c);
    if (c->reorder) reorder_cells(hm, bs ? &bs->tet_case : nullptr, c->reorder);
    else {
        hm.orig.resize(hm.nt);
        std::iota(hm.orig.begin(), hm.orig.end(), 0);
        hm.inv = hm.orig;
    }
    c->nt = hm.nt;
    c->nb = hm.nb;
    for (int b = 0; b < hm.nb; ++b)
        if (bcs[hm.bf_group[b]].kind == DSMC_BC_PERIODIC && hm.bf_partner[b] < 0) {
            delete c;
            return fail(nullptr, DSMC_E_MESH, "periodic boundary face without partner");
        }

    c->mass = sp->mass; c->dref = sp->d_ref; c->omega = sp->omega; c->Tref = sp->T_ref;
    c->alpha = sp->alpha;
    c->dr = sp->dof_rot;
    c->zr = sp->z_rot;
    if (c->dr) {
        const double* a = sp->heat_relax;
        const bool zero = a[0] == 0.0 && a[1] == 0.0 && a[2] == 0.0 && a[3] == 0.0;
        const double dflt[4] = {0.786, -0.201, -0.059, 0.842};
        for (int k = 0; k < 4; ++k) c->a_heat[k] = zero ? dflt[k] : a[k];
        const double det = c->a_heat[0] * c->a_heat[3] - c->a_heat[1] * c->a_heat[2];
        if (!(std::isfinite(det) && det != 0.0)) {
            delete c;
            return fail(nullptr, DSMC_E_INVALID, "singular heat-flux relaxation matrix");
        }
    }
    {
        const double a = sp->alpha, w = sp->omega;
        c->pinel = c->dr ? ((a * (5.0 - 2.0 * w)) * (7.0 - 2.0 * w)) / ((((5.0 * (a + 1.0)) * (a + 2.0))) * c->zr)
                         : 0.0;
    }
    if (c->dr) {
        // the rotating gas runs the kernels that carry the rotational energy
        if (!rot_schedule_ok(c->move_variant, c->collide_variant, c->sort_variant)) {
            c->move_variant = kMoveFace3;
            c->collide_variant = kCollideG3k;
            c->sort_variant = kSortGather;
        }
    }
    const double mr = sp->mass / 2.0;
    c->K = ((M_PI * sp->d_ref) * sp->d_ref) * std::pow(((2.0 * kBoltzmann) * sp->T_ref) / mr, sp->omega - 0.5) /
           std::tgamma(2.5 - sp->omega);
    c->ex = 1.0 - sp->omega;
    c->FN = run->F_N; c->dt = run->dt; c->n0 = run->n0; c->T0 = run->T0;
    for (int i = 0; i < 3; ++i) c->u0[i] = run->u0[i];
    c->key = RngKey{(uint32_t)(run->seed & 0xFFFFFFFFu), run->case_id};
    c->vel64 = run->vel_fp64 ? 1 : 0;
    c->bcs.assign(bcs, bcs + n_bc);
    c->n_ss = run->n_ss; c->n_a = run->n_a; c->ewma_on = run->ewma_on ? 1 : 0;
    if (bs && !move_reads_cases(c->move_variant))
        c->move_variant = kMoveFace3;  // the batch tables are read by the lane and deferring kernels

    // expected particle count at n0 sizes the default capacity
    double fill_total = 0;
    for (int t = 0; t < hm.nt; ++t) {
        const dsmc_run_desc* rc = bs ? &bs->runs[bs->tet_case[t]] : run;
        fill_total += (rc->n0 * hm.vol[t]) / rc->F_N + 1.0;
    }
    c->cap = run->capacity > 0 ? run->capacity : std::max<int64_t>(1024, (int64_t)(2.0 * fill_total) + 1024);
    if (c->cap >= ((int64_t)1 << 31) - 1) {
        delete c;
        return fail(nullptr, DSMC_E_INVALID, "capacity above 2^31 - 1");
    }

    // ---- inflow faces --------------------------------------------------
    std::vector<int32_t> in_bf, in_tc;
    std::vector<double> in_cst;
    for (int b = 0; b < hm.nb; ++b) {
        const dsmc_boundary_desc& g = bcs[hm.bf_group[b]];
        if (g.kind != DSMC_BC_INFLOW) continue;
        if (bs) {
            delete c;
            return fail(nullptr, DSMC_E_INVALID, "freestream inflow is not supported in a batch");
        }
        const double* fr = &hm.bf_frame[9 * (size_t)b];
        const double* nin = fr;
        const double* t1 = fr + 3;
        const double* t2 = fr + 6;
        const double T = g.T;
        const double beta = std::sqrt(((2.0 * kBoltzmann) * T) / sp->mass);
        const double sig = std::sqrt((kBoltzmann * T) / sp->mass);
        const double un = g.u[0] * nin[0] + g.u[1] * nin[1] + g.u[2] * nin[2];
        const double a = un / beta;
        const double f1 = std::sqrt((kBoltzmann * T) / ((2.0 * M_PI) * sp->mass));
        const double f2 = std::exp(-(a * a)) + (DSMC_SQRT_PI * a) * (1.0 + std::erf(a));
        const double flux = (g.n * f1) * f2;
        const double mean = ((flux * hm.bf_area[b]) * run->dt) / run->F_N;
        double cst[kInflowStride];
        cst[0] = mean; cst[1] = a; cst[2] = beta; cst[3] = sig;
        cst[4] = g.u[0] * t1[0] + g.u[1] * t1[1] + g.u[2] * t1[2];
        cst[5] = g.u[0] * t2[0] + g.u[1] * t2[1] + g.u[2] * t2[2];
        for (int i = 0; i < 9; ++i) cst[6 + i] = fr[i];
        for (int v = 0; v < 3; ++v)
            for (int i = 0; i < 3; ++i) cst[15 + 3 * v + i] = hm.xyz[3 * (size_t)hm.bf_vtx[3 * (size_t)b + v] + i];
        cst[24] = kBoltzmann * T;
        in_cst.insert(in_cst.end(), cst, cst + kInflowStride);
        in_bf.push_back(b);
        in_tc.push_back((hm.bf_tet[b] << 2) | hm.bf_lf[b]);
        c->max_inject += (int64_t)std::floor(mean) + 1;
    }

    // ---- device allocations --------------------------------------------
    const int nt = hm.nt, nb = hm.nb;
    const int nblk_cells = (nt + kScanBlock) / kScanBlock + 1;
    const int nin = (int)in_bf.size();
    bool ok = alloc_n(c, c->d_plane, 4 * (size_t)nt) && alloc_n(c, c->d_nbr, 4 * (size_t)nt) &&
              alloc_n(c, c->d_vol, nt) && alloc_n(c, c->d_bf_group, nb + 1) && alloc_n(c, c->d_bf_pcode, nb + 1) &&
              alloc_n(c, c->d_bf_frame, 9 * (size_t)nb + 9) && alloc_n(c, c->d_groups, n_bc + 1) &&
              alloc_n(c, c->d_tv, nt) && alloc_n(c, c->d_xyz, 3 * (size_t)hm.nv) &&
              alloc_n(c, c->d_orig, nt) && alloc_n(c, c->d_cell_tmp, nt + 1) &&
              alloc_n(c, c->d_counts_orig, nt + 1) &&
              alloc_n(c, c->d_counts, nt + 1) && alloc_n(c, c->d_offsets, nt + 1) &&
              alloc_n(c, c->d_blocksums, std::max(nblk_cells, (nin + kScanBlock) / kScanBlock + 1)) &&
              alloc_n(c, c->d_smax, nt) && alloc_n(c, c->d_ncand, nt) && alloc_n(c, c->d_nacc, nt) &&
              alloc_n(c, c->d_acc, (size_t)kNMom * nt) && alloc_n(c, c->d_ewma, (size_t)kNMom * nt) &&
              alloc_n(c, c->d_ewma_m, nt) && alloc_n(c, c->d_local, nt) && alloc_n(c, c->d_sc, 1) &&
              alloc_n(c, c->d_ctr, 1) && alloc_n(c, c->d_fcount, nin + 1) && alloc_n(c, c->d_foff, nin + 1);
    int32_t* d_in_bf = nullptr;
    int32_t* d_in_tc = nullptr;
    double* d_in_cst = nullptr;
    ok = ok && alloc_n(c, d_in_bf, nin + 1) && alloc_n(c, d_in_tc, nin + 1) &&
         alloc_n(c, d_in_cst, (size_t)kInflowStride * nin + 1);
    if (c->dr)
        ok = ok && alloc_n(c, c->A.ir, c->cap) && alloc_n(c, c->B.ir, c->cap) &&
             alloc_n(c, c->d_racc, (size_t)4 * nt) && alloc_n(c, c->d_rewma, (size_t)4 * nt) &&
             alloc_n(c, c->d_rinst, (size_t)4 * nt);
    ok = ok && alloc_buf(c, c->A, c->cap, c->vel64) && alloc_buf(c, c->B, c->cap, c->vel64) &&
         alloc_n(c, c->d_rank, c->cap) && alloc_n(c, c->d_perm, c->cap) && alloc_n(c, c->d_sortperm, c->cap) &&
         alloc_n(c, c->wq.idx, kQueueParts * queue_part_size(c->cap)) &&
         alloc_n(c, c->wq.t, kQueueParts * queue_part_size(c->cap)) &&
         alloc_n(c, c->wq.meta, kQueueParts * queue_part_size(c->cap)) &&
         alloc_n(c, c->wq.n, (size_t)(kQueueParts + kTileSlices) * kQueueStride);
    c->wq.part = queue_part_size(c->cap);
    if (!ok) {
        dsmc_destroy(c);
        return fail(nullptr, DSMC_E_OOM, "device allocation failed");
    }

    // ---- uploads -------------------------------------------------------
    std::vector<int32_t> pcode(nb + 1, -1);
    for (int b = 0; b < nb; ++b) {
        const int p = hm.bf_partner[b];
        if (p >= 0) pcode[b] = (hm.bf_tet[p] << 2) | hm.bf_lf[p];
    }
    std::vector<GroupDev> groups(n_bc + 1);
    for (int g = 0; g < n_bc; ++g) {
        GroupDev& d = groups[g];
        d.kind = bcs[g].kind;
        d.pad = 0;
        d.beta = std::sqrt(((2.0 * kBoltzmann) * bcs[g].T) / sp->mass);
        d.sw = std::sqrt((kBoltzmann * bcs[g].T) / sp->mass);
        d.kT = kBoltzmann * bcs[g].T;
        for (int i = 0; i < 3; ++i) {
            d.u[i] = bcs[g].u[i];
            d.shift[i] = bcs[g].shift[i];
        }
    }
    hipStream_t s = c->stream;
#define UP(dst, src, bytes) HIP_TRY(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s))
    UP(c->d_plane, hm.plane.data(), sizeof(double) * 16 * (size_t)nt);
    UP(c->d_nbr, hm.nbr.data(), sizeof(int32_t) * 4 * (size_t)nt);
    UP(c->d_vol, hm.vol.data(), sizeof(double) * nt);
    if (nb) {
        UP(c->d_bf_group, hm.bf_group.data(), sizeof(int32_t) * nb);
        UP(c->d_bf_frame, hm.bf_frame.data(), sizeof(double) * 9 * (size_t)nb);
    }
    UP(c->d_bf_pcode, pcode.data(), sizeof(int32_t) * (nb + 1));
    UP(c->d_groups, groups.data(), sizeof(GroupDev) * (n_bc + 1));
    UP(c->d_tv, hm.tv.data(), sizeof(int32_t) * 4 * (size_t)nt);
    UP(c->d_xyz, hm.xyz.data(), sizeof(double) * 3 * (size_t)hm.nv);
    UP(c->d_orig, hm.orig.data(), sizeof(int32_t) * nt);
    if (nin) {
        UP(d_in_bf, in_bf.data(), sizeof(int32_t) * nin);
        UP(d_in_tc, in_tc.data(), sizeof(int32_t) * nin);
        UP(d_in_cst, in_cst.data(), sizeof(double) * in_cst.size());
    }
    Scalars sc0{};
    Counters ct0{};
    UP(c->d_sc, &sc0, sizeof sc0);
    UP(c->d_ctr, &ct0, sizeof ct0);
    HIP_TRY(c, hipStreamSynchronize(s));  // host vectors above are temporaries
    c->mesh.nt = nt;
    c->mesh.plane = c->d_plane;
    c->mesh.nbr = c->d_nbr;
    c->mesh.vol = c->d_vol;
    c->mesh.bf_group = c->d_bf_group;
    c->mesh.bf_pcode = c->d_bf_pcode;
    c->mesh.bf_frame = c->d_bf_frame;
    c->mesh.groups = c->d_groups;
    c->mesh.mass = sp->mass;
    c->mesh.nb = nb;
    c->mesh.n_ss = run->n_ss;
    c->mesh.surf = nullptr;
    c->mesh.rot = c->dr ? 1 : 0;
    c->inflow.n = nin;
    c->inflow.bface = d_in_bf;
    c->inflow.tcode = d_in_tc;
    c->inflow.consts = d_in_cst;

    // cell state
    const double eq = (((2.0 * DSMC_SQRT_PI) * sp->d_ref) * sp->d_ref) * std::sqrt(((2.0 * kBoltzmann) * sp->T_ref) / mr) *
                      std::pow(run->T0 / sp->T_ref, 1.0 - sp->omega);
    if (bs) {
        // per-case table; cell subjects and particle ids are case-local
        std::vector<CaseDev> cases(bs->runs.size());
        for (size_t k = 0; k < cases.size(); ++k) {
            const dsmc_run_desc& r = bs->runs[k];
            CaseDev& d = cases[k];
            d.dt = r.dt; d.FN = r.F_N; d.n0 = r.n0; d.T0 = r.T0;
            d.sig = std::sqrt((kBoltzmann * r.T0) / sp->mass);
            for (int i = 0; i < 3; ++i) d.u0[i] = r.u0[i];
            const double eqk = (((2.0 * DSMC_SQRT_PI) * sp->d_ref) * sp->d_ref) *
                               std::sqrt(((2.0 * kBoltzmann) * sp->T_ref) / mr) * std::pow(r.T0 / sp->T_ref, 1.0 - sp->omega);
            d.smax0 = 2.0 * eqk;
            d.k0 = (uint32_t)(r.seed & 0xFFFFFFFFu);
            d.k1 = r.case_id;
            d.cell0 = bs->cell0[k];
            d.pad = 0;
        }
        std::vector<int32_t> cc(nt), first(cases.size());
        for (int t = 0; t < nt; ++t) cc[t] = bs->tet_case[hm.orig[t]];
        for (size_t k = 0; k < cases.size(); ++k) first[k] = bs->cell0[k];
        bool okb = alloc_n(c, c->d_cases, cases.size()) && alloc_n(c, c->d_cell_case, nt) &&
                   alloc_n(c, c->d_case_of_orig, nt) && alloc_n(c, c->d_case_first, cases.size());
        if (!okb) {
            dsmc_destroy(c);
            return fail(nullptr, DSMC_E_OOM, "device allocation failed");
        }
        UP(c->d_cases, cases.data(), sizeof(CaseDev) * cases.size());
        UP(c->d_cell_case, cc.data(), sizeof(int32_t) * nt);
        UP(c->d_case_of_orig, bs->tet_case.data(), sizeof(int32_t) * nt);
        UP(c->d_case_first, first.data(), sizeof(int32_t) * first.size());
        HIP_TRY(c, hipStreamSynchronize(s));
        c->n_cases = (int)cases.size();
        c->case_cell0 = bs->cell0;
        c->mesh.cell_case = c->d_cell_case;
        c->mesh.cases = c->d_cases;
        launch_batch_smax(s, c->d_cell_case, c->d_cases, nt, c->d_smax);
    } else {
        launch_fill_f64(s, c->d_smax, 2.0 * eq, nt);
    }
    launch_fill_i32(s, c->d_ncand, 0, nt);
    launch_fill_i32(s, c->d_nacc, 0, nt);
    launch_fill_f64(s, c->d_acc, 0.0, (int64_t)kNMom * nt);
    launch_fill_f64(s, c->d_ewma, 0.0, (int64_t)kNMom * nt);
    if (c->dr) {
        launch_fill_f64(s, c->d_racc, 0.0, (int64_t)4 * nt);
        launch_fill_f64(s, c->d_rewma, 0.0, (int64_t)4 * nt);
        launch_fill_f64(s, c->d_rinst, 0.0, (int64_t)4 * nt);
    }
    launch_fill_i32(s, c->d_ewma_m, 0, nt);
    HIP_TRY(c, hipMemsetAsync(c->d_local, 0, nt, s));
    launch_fill_i32(s, c->d_offsets, 0, nt + 1);

    if (run->fill) {
        // counts per cell; particle ids follow the caller's cell order
        launch_init_count(s, c->d_vol, c->d_orig, nt, run->n0, run->F_N, c->key, c->d_counts, c->d_counts_orig,
                          c->d_cell_case, c->d_cases);
        launch_scan(s, c->d_counts_orig, nt, c->d_cell_tmp, c->d_blocksums, c->d_sc, kScanPlain);
        if (bs)  // particle ids restart in every case: base = prefix - prefix at the case's first cell
            launch_batch_pid_base(s, c->d_cell_tmp, c->d_case_first, c->d_case_of_orig, nt, c->d_counts_orig);
        launch_scan(s, c->d_counts, nt, c->d_offsets, c->d_blocksums, c->d_sc, kScanInit);
        const double sig = std::sqrt((kBoltzmann * run->T0) / sp->mass);
        if (c->vel64) fill_dispatch<double>(c, sig); else fill_dispatch<float>(c, sig);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        std::string m = std::string("kernel launch: ") + hipGetErrorString(e);
        dsmc_destroy(c);
        return fail(nullptr, DSMC_E_DEVICE, m);
    }
    dsmc_status st = sync_scalars(c, nullptr);
    if (st != DSMC_OK) {
        std::string m = c->err;
        dsmc_destroy(c);
        return fail(nullptr, st, m);
    }
    *out = c;
    return DSMC_OK;
}

extern "C" {

dsmc_status dsmc_init(dsmc_ctx* out, const dsmc_mesh_desc* mesh, const dsmc_species_desc* sp, int32_t n_bc,
                      const dsmc_boundary_desc* bcs, const dsmc_run_desc* run) {
    return init_impl(out, mesh, sp, n_bc, bcs, run, nullptr);
}

dsmc_status dsmc_batch_init(dsmc_ctx* out, int32_t n_cases, const dsmc_mesh_desc* meshes,
                            const dsmc_species_desc* sp, const int32_t* n_bc, const dsmc_boundary_desc* bcs,
                            const dsmc_run_desc* runs) {
    if (!out) return fail(nullptr, DSMC_E_INVALID, "out is NULL");
    *out = nullptr;
    if (n_cases < 1 || !meshes || !sp || !n_bc || !runs) return fail(nullptr, DSMC_E_INVALID, "bad batch arguments");
    BatchSpec bs;
    std::vector<double> xyz;
    std::vector<int32_t> tets, bfv, bgrp, bpart;
    int32_t nv = 0, nt = 0, nb = 0, ng = 0;
    std::vector<dsmc_boundary_desc> groups;
    for (int k = 0; k < n_cases; ++k) {
        const dsmc_mesh_desc& m = meshes[k];
        const dsmc_run_desc& r = runs[k];
        if (m.n_vertices <= 0 || m.n_tets <= 0 || !m.xyz || !m.tet_vtx || (m.n_bfaces > 0 && (!m.bface_vtx || !m.bface_group)))
            return fail(nullptr, DSMC_E_INVALID, "bad mesh of a batch case");
        if (!(r.F_N > 0) || !(r.dt > 0)) return fail(nullptr, DSMC_E_INVALID, "non-positive physical parameter");
        if (n_bc[k] < 0) return fail(nullptr, DSMC_E_INVALID, "bad boundary count");
        if ((int64_t)nt + m.n_tets >= ((int64_t)1 << 28)) return fail(nullptr, DSMC_E_INVALID, "batch too large");
        xyz.insert(xyz.end(), m.xyz, m.xyz + 3 * (size_t)m.n_vertices);
        for (int64_t i = 0; i < 4 * (int64_t)m.n_tets; ++i) tets.push_back(m.tet_vtx[i] + nv);
        for (int64_t i = 0; i < 3 * (int64_t)m.n_bfaces; ++i) bfv.push_back(m.bface_vtx[i] + nv);
        for (int64_t i = 0; i < m.n_bfaces; ++i) {
            bgrp.push_back(m.bface_group[i] + ng);
            const int32_t pp = m.bface_partner ? m.bface_partner[i] : -1;
            bpart.push_back(pp >= 0 ? pp + nb : -1);
        }
        for (int g = 0; g < n_bc[k]; ++g) groups.push_back(bcs[ng + g]);
        bs.runs.push_back(r);
        bs.cell0.push_back(nt);
        for (int t = 0; t < m.n_tets; ++t) bs.tet_case.push_back(k);
        nv += m.n_vertices;
        nt += m.n_tets;
        nb += m.n_bfaces;
        ng += n_bc[k];
    }
    dsmc_mesh_desc u{nv, xyz.data(), nt, tets.data(), nb, bfv.data(), bgrp.data(), bpart.data()};
    return init_impl(out, &u, sp, ng, groups.data(), &runs[0], &bs);
}

dsmc_status dsmc_batch_cases(dsmc_ctx c, int32_t* n_cases, int32_t* cell_begin) {
    if (!c || !n_cases) return fail(c, DSMC_E_INVALID, "bad arguments");
    const int n = std::max(1, c->n_cases);
    *n_cases = n;
    if (cell_begin) {
        for (int k = 0; k < n; ++k) cell_begin[k] = c->n_cases ? c->case_cell0[k] : 0;
        cell_begin[n] = c->nt;
    }
    return DSMC_OK;
}

dsmc_status dsmc_graph_step(dsmc_ctx c, int32_t n) {
    if (!c || n < 0) return fail(c, DSMC_E_INVALID, "bad arguments");
    if (c->broken) return fail(c, DSMC_E_INVALID, "context is in an error state");
    if (!c->stream) return fail(c, DSMC_E_INVALID, "graph stepping needs a non-null HIP stream");
    // a captured deferred step starts from a pending order (a state read may
    // have written it out since the last replay)
    if (n >= 2 && c->sort_variant == kSortDeferred && deferred_ok(c->move_variant, c->collide_variant))
        ensure_pending(c);
    int done = 0;
    while (done + 2 <= n) {
        dsmc_ctx_s::Graph* g = nullptr;
        for (auto& cand : c->graphs)
            if (cand.exec && cand.a_x == c->A.pos && cand.sig == tuning_sig(c) && c->np_bound <= cand.bound) g = &cand;
        if (!g) {
            g = (c->graphs[0].a_x == c->A.pos || !c->graphs[0].exec) ? &c->graphs[0] : &c->graphs[1];
            dsmc_status st = capture_two_steps(c, *g);
            if (st != DSMC_OK) return st;
        }
        HIP_TRY(c, hipGraphLaunch(g->exec, c->stream));
        done += 2;
        // without inflow the count cannot have grown; with it, unknown until
        // the next synchronising call
        if (c->inflow.n > 0) c->np_bound = c->cap;
    }
    if (done < n) return step_any(c, 31);
    return DSMC_OK;
}

dsmc_status dsmc_get_tuning(dsmc_ctx c, dsmc_tuning* t) {
    if (!c || !t) return fail(c, DSMC_E_INVALID, "bad arguments");
    t->move = c->move_variant;
    t->collide = c->collide_variant;
    t->sort = c->sort_variant;
    return DSMC_OK;
}

dsmc_status dsmc_set_tuning(dsmc_ctx c, const dsmc_tuning* t) {
    if (!c || !t) return fail(c, DSMC_E_INVALID, "bad arguments");
    const bool batch_ok = move_reads_cases(t->move);
    if (t->move < 0 || t->move > kMovePersist || t->collide < 0 || t->collide > kCollideG2k || t->sort < 0 ||
        t->sort > kSortDeferred || (c->n_cases && !batch_ok))
        return fail(c, DSMC_E_INVALID, "unknown or unsupported kernel variant");
    if (t->sort == kSortDeferred && !deferred_ok(t->move, t->collide))
        return fail(c, DSMC_E_INVALID, "the deferred sort needs the three-face move and an LDS-ranked collide");
    if (c->dr && !rot_schedule_ok(t->move, t->collide, t->sort))
        return fail(c, DSMC_E_INVALID, "a rotating gas needs a parked-wall move, LDS-ranked collide and scatter, "
                                       "gather or deferred sort schedule");
    if (t->sort != kSortDeferred) {
        dsmc_status st = materialize(c);
        if (st != DSMC_OK) return st;
    }
    c->move_variant = t->move;
    c->collide_variant = t->collide;
    c->sort_variant = t->sort;
    return DSMC_OK;
}

dsmc_status dsmc_autotune(dsmc_ctx c, int32_t trial_steps, dsmc_tuning* out) {
    if (!c || trial_steps < 1) return fail(c, DSMC_E_INVALID, "bad arguments");
    if (c->broken) return fail(c, DSMC_E_INVALID, "context is in an error state");
    const bool was_profiling = c->profiling;
    dsmc_tuning best{c->move_variant, c->collide_variant, c->sort_variant, 1e300, 1e300, 1e300};
    // moves and collides are timed with the plain gather sort
    if (c->sort_variant == kSortDeferred) {
        dsmc_status st = materialize(c);
        if (st != DSMC_OK) return st;
        c->sort_variant = kSortGather;
    }
    const int moves[] = {kMoveDefer4, kMoveDefer5, kMoveDefer6, kMoveDefer8, kMoveFace3, kMoveFace3W8, kMoveCap4,
                         kMoveCap5, kMoveCap6, kMoveLaneW6, kMoveLaneW8, kMovePersist};
    for (int v : moves) {
        if (c->dr && !rot_schedule_ok(v, c->collide_variant, c->sort_variant)) continue;
        c->move_variant = v;
        double ms = 0;
        dsmc_status st = time_slots(c, trial_steps, {kSlotMove, kSlotWalls}, &ms);
        if (st != DSMC_OK) return st;
        if (ms < best.move_ms) { best.move_ms = ms; best.move = v; }
    }
    c->move_variant = best.move;
    const int collides[] = {kCollideGlobal, kCollideGlobal8, kCollideG3k, kCollideG2k, kCollideLds};
    for (int v : collides) {
        if (c->dr && !rot_schedule_ok(c->move_variant, v, c->sort_variant)) continue;
        c->collide_variant = v;
        double ms = 0;
        dsmc_status st = time_slots(c, trial_steps, {kSlotCollide}, &ms);
        if (st != DSMC_OK) return st;
        if (ms < best.collide_ms) { best.collide_ms = ms; best.collide = v; }
    }
    c->collide_variant = best.collide;
    const int sorts[] = {kSortGather, kSortScatter, kSortFused, kSortDeferred};
    for (int v : sorts) {
        if (c->dr && !rot_schedule_ok(c->move_variant, c->collide_variant, v)) continue;
        if (v == kSortDeferred && !deferred_ok(c->move_variant, c->collide_variant)) continue;
        c->sort_variant = v;
        double ms = 0;
        // the fused form gathers inside the collide kernel and the deferred
        // one inside the move: compare the whole step
        dsmc_status st = time_slots(c, trial_steps,
                                    {kSlotMove, kSlotWalls, kSlotScan, kSlotScatter, kSlotGather, kSlotCollide}, &ms);
        if (st != DSMC_OK) return st;
        if (ms < best.sort_ms) { best.sort_ms = ms; best.sort = v; }
    }
    if (best.sort != kSortDeferred) {
        dsmc_status st = materialize(c);
        if (st != DSMC_OK) return st;
    }
    c->sort_variant = best.sort;
    c->profiling = was_profiling;
    if (out) *out = best;
    return DSMC_OK;
}

dsmc_status dsmc_step(dsmc_ctx c, int32_t n) {
    if (!c || n < 0) return fail(c, DSMC_E_INVALID, "bad arguments");
    if (c->broken) return fail(c, DSMC_E_INVALID, "context is in an error state");
    for (int i = 0; i < n; ++i) {
        dsmc_status s = step_any(c, 31);
        if (s != DSMC_OK) return s;
    }
    return DSMC_OK;
}

dsmc_status dsmc_step_stages(dsmc_ctx c, int32_t mask) {
    if (!c || mask < 0 || mask > 31) return fail(c, DSMC_E_INVALID, "bad arguments");
    if ((mask & 3) && !(mask & 4))
        return fail(c, DSMC_E_INVALID, "move or injection without the sort would leave the store unsorted");
    if (c->broken) return fail(c, DSMC_E_INVALID, "context is in an error state");
    return step_any(c, mask);
}

dsmc_status dsmc_sync(dsmc_ctx c) {
    if (!c) return fail(c, DSMC_E_INVALID, "NULL context");
    return sync_scalars(c, nullptr);
}

// The device array of an accumulator (INSTANT: allocated and cleared on
// first use).
static const double* accumulator(dsmc_ctx c, int32_t which) {
    if (which == DSMC_SAMPLE_STEADY) return c->d_acc;
    if (which == DSMC_SAMPLE_EWMA) return c->d_ewma;
    if (!c->d_inst) {
        if (!alloc_n(c, c->d_inst, (size_t)kNMom * c->nt)) return nullptr;
        launch_fill_f64(c->stream, c->d_inst, 0.0, (int64_t)kNMom * c->nt);
    }
    return c->d_inst;
}

dsmc_status dsmc_instant_sampling(dsmc_ctx c, int32_t on) {
    if (!c) return fail(c, DSMC_E_INVALID, "NULL context");
    if (c->broken) return fail(c, DSMC_E_INVALID, "context is in an error state");
    if (on && !accumulator(c, DSMC_SAMPLE_INSTANT)) return fail(c, DSMC_E_OOM, "device allocation failed");
    c->inst_on = on != 0;
    return sync_scalars(c, nullptr);
}

dsmc_status dsmc_sample(dsmc_ctx c, int32_t which, double* out, int32_t out_on_device) {
    if (!c || !out || (which != DSMC_SAMPLE_STEADY && which != DSMC_SAMPLE_EWMA && which != DSMC_SAMPLE_INSTANT))
        return fail(c, DSMC_E_INVALID, "bad arguments");
    Scalars sc;
    dsmc_status st = sync_scalars(c, &sc);
    if (st != DSMC_OK) return st;
    const double ns = which == DSMC_SAMPLE_STEADY ? (double)sc.n_steady : 1.0;
    const double* src = accumulator(c, which);
    if (!src) return fail(c, DSMC_E_OOM, "device allocation failed");
    double* dout = out;
    double* tmp = nullptr;
    if (!out_on_device) {
        if (!alloc_n(c, tmp, 15 * (size_t)c->nt)) return fail(c, DSMC_E_OOM, "device allocation failed");
        dout = tmp;
    }
    launch_fields(c->stream, src, c->nt, ns, c->mass, c->FN, c->d_vol, c->d_orig, dout, c->d_cell_case, c->d_cases);
    HIP_TRY(c, hipGetLastError());
    if (!out_on_device) {
        HIP_TRY(c, hipMemcpyAsync(out, tmp, sizeof(double) * 15 * (size_t)c->nt, hipMemcpyDeviceToHost, c->stream));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    dev_free(c, tmp);
    return DSMC_OK;
}

dsmc_status dsmc_surface_sampling(dsmc_ctx c, int32_t on) {
    if (!c) return fail(c, DSMC_E_INVALID, "bad arguments");
    if (c->broken) return fail(c, DSMC_E_INVALID, "context is in an error state");
    Scalars sc;
    dsmc_status st = sync_scalars(c, &sc);
    if (st != DSMC_OK) return st;
    if (on) {
        // five rows, and the rotational-energy row of a rotating gas
        if (!c->d_surf && !alloc_n(c, c->d_surf, 6 * (size_t)c->nb + 6))
            return fail(c, DSMC_E_OOM, "device allocation failed");
        launch_fill_f64(c->stream, c->d_surf, 0.0, 6 * (int64_t)c->nb + 6);
        HIP_TRY(c, hipGetLastError());
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        c->mesh.surf = c->d_surf;
        c->surf_from = sc.step;
        c->surf_to = -1;
    } else if (c->mesh.surf) {
        c->mesh.surf = nullptr;
        c->surf_to = sc.step;
    }
    return DSMC_OK;
}

dsmc_status dsmc_get_surface(dsmc_ctx c, double* sums, double* fields, int64_t* n_steps) {
    if (!c) return fail(c, DSMC_E_INVALID, "bad arguments");
    Scalars sc;
    dsmc_status st = sync_scalars(c, &sc);
    if (st != DSMC_OK) return st;
    const int nb = c->nb;
    std::vector<double> h(5 * (size_t)nb, 0.0);
    if (c->d_surf) HIP_TRY(c, hipMemcpy(h.data(), c->d_surf, sizeof(double) * h.size(), hipMemcpyDeviceToHost));
    const int64_t end = c->surf_to < 0 ? (int64_t)sc.step : c->surf_to;
    const int64_t from = std::max<int64_t>(c->surf_from, c->n_ss);
    const int64_t ns = c->d_surf && end > from ? end - from : 0;
    if (n_steps) *n_steps = ns;
    if (sums)
        for (int b = 0; b < nb; ++b)
            for (int k = 0; k < 5; ++k) sums[5 * (size_t)b + k] = h[(size_t)k * nb + b];
    if (fields) {
        // per face: F_N and dt of its case
        std::vector<CaseDev> cases(std::max(1, c->n_cases));
        if (c->n_cases)
            HIP_TRY(c, hipMemcpy(cases.data(), c->d_cases, sizeof(CaseDev) * c->n_cases, hipMemcpyDeviceToHost));
        for (int b = 0; b < nb; ++b) {
            double FN = c->FN, dt = c->dt;
            if (c->n_cases) {
                const int o = c->hm.orig[c->hm.bf_tet[b]];
                const int k = (int)(std::upper_bound(c->case_cell0.begin(), c->case_cell0.end(), o) -
                                    c->case_cell0.begin()) - 1;
                FN = cases[k].FN;
                dt = cases[k].dt;
            }
            double* f = fields + 6 * (size_t)b;
            const double ta = c->hm.bf_area[b] * ((double)ns * dt);
            if (!(ta > 0)) {
                for (int k = 0; k < 6; ++k) f[k] = 0.0;
                continue;
            }
            // outward unit normal (into the wall) = minus the inward one of the face frame
            const double* fr = &c->hm.bf_frame[9 * (size_t)b];
            const double n[3] = {-fr[0], -fr[1], -fr[2]};
            const double s = c->mass * FN / ta;
            const double d[3] = {h[b], h[(size_t)nb + b], h[2 * (size_t)nb + b]};
            const double dn = d[0] * n[0] + d[1] * n[1] + d[2] * n[2];
            f[0] = FN * h[4 * (size_t)nb + b] / ta;
            f[1] = s * dn;
            for (int i = 0; i < 3; ++i) f[2 + i] = s * (d[i] - dn * n[i]);
            f[5] = s * h[3 * (size_t)nb + b];
        }
    }
    return DSMC_OK;
}

dsmc_status dsmc_get_surface_rot(dsmc_ctx c, double* sums, double* qr, int64_t* n_steps) {
    if (!c) return fail(c, DSMC_E_INVALID, "bad arguments");
    if (!c->dr) return fail(c, DSMC_E_INVALID, "the gas has no rotational degrees of freedom");
    Scalars sc;
    dsmc_status st = sync_scalars(c, &sc);
    if (st != DSMC_OK) return st;
    const int nb = c->nb;
    std::vector<double> h((size_t)nb, 0.0);
    if (c->d_surf)
        HIP_TRY(c, hipMemcpy(h.data(), c->d_surf + 5 * (size_t)nb, sizeof(double) * nb, hipMemcpyDeviceToHost));
    const int64_t end = c->surf_to < 0 ? (int64_t)sc.step : c->surf_to;
    const int64_t from = std::max<int64_t>(c->surf_from, c->n_ss);
    const int64_t ns = c->d_surf && end > from ? end - from : 0;
    if (n_steps) *n_steps = ns;
    if (sums)
        for (int b = 0; b < nb; ++b) sums[b] = h[b];
    if (qr) {
        std::vector<CaseDev> cases(std::max(1, c->n_cases));
        if (c->n_cases)
            HIP_TRY(c, hipMemcpy(cases.data(), c->d_cases, sizeof(CaseDev) * c->n_cases, hipMemcpyDeviceToHost));
        for (int b = 0; b < nb; ++b) {
            double FN = c->FN, dt = c->dt;
            if (c->n_cases) {
                const int o = c->hm.orig[c->hm.bf_tet[b]];
                const int k = (int)(std::upper_bound(c->case_cell0.begin(), c->case_cell0.end(), o) -
                                    c->case_cell0.begin()) - 1;
                FN = cases[k].FN;
                dt = cases[k].dt;
            }
            const double ta = c->hm.bf_area[b] * ((double)ns * dt);
            qr[b] = ta > 0 ? FN * h[b] / ta : 0.0;
        }
    }
    return DSMC_OK;
}

dsmc_status dsmc_get_sums(dsmc_ctx c, int32_t which, double* out, int64_t* n_samples) {
    if (!c || !out || (which != DSMC_SAMPLE_STEADY && which != DSMC_SAMPLE_EWMA && which != DSMC_SAMPLE_INSTANT))
        return fail(c, DSMC_E_INVALID, "bad arguments");
    const double* src = accumulator(c, which);
    if (!src) return fail(c, DSMC_E_OOM, "device allocation failed");
    Scalars sc;
    dsmc_status st = sync_scalars(c, &sc);
    if (st != DSMC_OK) return st;
    std::vector<double> h((size_t)kNMom * c->nt);
    HIP_TRY(c, hipMemcpy(h.data(), src, sizeof(double) * h.size(), hipMemcpyDeviceToHost));
    for (int t = 0; t < c->nt; ++t)
        for (int k = 0; k < kNMom; ++k) out[(size_t)kNMom * c->hm.orig[t] + k] = h[(size_t)k * c->nt + t];
    if (n_samples) *n_samples = which == DSMC_SAMPLE_INSTANT ? 1 : sc.n_steady;
    return DSMC_OK;
}

dsmc_status dsmc_get_rot_sums(dsmc_ctx c, int32_t which, double* out, int64_t* n_samples) {
    if (!c || !out || (which != DSMC_SAMPLE_STEADY && which != DSMC_SAMPLE_EWMA && which != DSMC_SAMPLE_INSTANT))
        return fail(c, DSMC_E_INVALID, "bad arguments");
    if (!c->dr) return fail(c, DSMC_E_INVALID, "the gas has no rotational degrees of freedom");
    const double* src = which == DSMC_SAMPLE_STEADY ? c->d_racc : which == DSMC_SAMPLE_EWMA ? c->d_rewma : c->d_rinst;
    Scalars sc;
    dsmc_status st = sync_scalars(c, &sc);
    if (st != DSMC_OK) return st;
    std::vector<double> h((size_t)4 * c->nt);
    HIP_TRY(c, hipMemcpy(h.data(), src, sizeof(double) * h.size(), hipMemcpyDeviceToHost));
    for (int t = 0; t < c->nt; ++t)
        for (int k = 0; k < 4; ++k) out[(size_t)4 * c->hm.orig[t] + k] = h[(size_t)k * c->nt + t];
    if (n_samples) *n_samples = which == DSMC_SAMPLE_INSTANT ? 1 : sc.n_steady;
    return DSMC_OK;
}

dsmc_status dsmc_rot_sample(dsmc_ctx c, int32_t which, double* out) {
    if (!c || !out) return fail(c, DSMC_E_INVALID, "bad arguments");
    if (!c->dr) return fail(c, DSMC_E_INVALID, "the gas has no rotational degrees of freedom");
    std::vector<double> S((size_t)kNMom * c->nt), R((size_t)4 * c->nt);
    int64_t n_steady = 0;
    dsmc_status st = dsmc_get_sums(c, which, S.data(), &n_steady);
    if (st == DSMC_OK) st = dsmc_get_rot_sums(c, which, R.data(), nullptr);
    if (st != DSMC_OK) return st;
    const double ns = which == DSMC_SAMPLE_STEADY ? (double)n_steady : 1.0;
    std::vector<int32_t> cs;
    std::vector<double> fn(c->nt, c->FN);
    if (c->d_cell_case) {
        // per-case particle weights of a batch, in the caller's cell order
        cs.resize(c->nt);
        HIP_TRY(c, hipMemcpy(cs.data(), c->d_cell_case, sizeof(int32_t) * c->nt, hipMemcpyDeviceToHost));
        std::vector<CaseDev> cases(c->n_cases);
        HIP_TRY(c, hipMemcpy(cases.data(), c->d_cases, sizeof(CaseDev) * c->n_cases, hipMemcpyDeviceToHost));
        for (int t = 0; t < c->nt; ++t) fn[c->hm.orig[t]] = cases[cs[t]].FN;
    }
    for (int o = 0; o < c->nt; ++o) {
        const double* a = &S[(size_t)kNMom * o];
        const double* r = &R[(size_t)4 * o];
        double* q = out + 4 * (size_t)o;
        if (!(a[0] > 0) || !(ns > 0)) {
            for (int k = 0; k < 4; ++k) q[k] = std::nan("");
            continue;
        }
        q[0] = (2.0 * (r[0] / a[0])) / ((double)c->dr * kBoltzmann);
        const double f = fn[o] / (c->hm.vol[c->hm.inv[o]] * ns);
        for (int i = 0; i < 3; ++i) q[1 + i] = f * (r[1 + i] - (a[1 + i] / a[0]) * r[0]);
    }
    return DSMC_OK;
}

dsmc_status dsmc_sample_cells(dsmc_ctx c, int32_t which, int32_t n_cells, const int32_t* tet_cell, double* out) {
    if (!c || !tet_cell || !out || n_cells < 0) return fail(c, DSMC_E_INVALID, "bad arguments");
    if (c->n_cases) return fail(c, DSMC_E_INVALID, "cell fields of a batch: use dsmc_sample per case");
    for (int t = 0; t < c->nt; ++t)
        if (tet_cell[t] < 0 || tet_cell[t] >= n_cells) return fail(c, DSMC_E_INVALID, "tet_cell out of range");
    std::vector<double> S((size_t)kNMom * c->nt);
    int64_t n_steady = 0;
    dsmc_status st = dsmc_get_sums(c, which, S.data(), &n_steady);
    if (st != DSMC_OK) return st;
    // per cell: sums and volumes of its tetrahedra in ascending order, laid
    // out as the device accumulators are ([13][n_cells]) for the field kernel
    const int ne = std::max(n_cells, 1);
    std::vector<double> agg((size_t)kNMom * ne, 0.0), vol(ne, 0.0);
    std::vector<int32_t> ident(ne);
    std::iota(ident.begin(), ident.end(), 0);
    for (int t = 0; t < c->nt; ++t) {
        const int e = tet_cell[t];
        for (int k = 0; k < kNMom; ++k) agg[(size_t)k * ne + e] += S[(size_t)kNMom * t + k];
        vol[e] += c->hm.vol[c->hm.inv[t]];
    }
    double *d_agg = nullptr, *d_vol = nullptr, *d_out = nullptr;
    int32_t* d_id = nullptr;
    if (!alloc_n(c, d_agg, agg.size()) || !alloc_n(c, d_vol, (size_t)ne) || !alloc_n(c, d_out, 15 * (size_t)ne) ||
        !alloc_n(c, d_id, (size_t)ne)) {
        dev_free(c, d_agg); dev_free(c, d_vol); dev_free(c, d_out); dev_free(c, d_id);
        return fail(c, DSMC_E_OOM, "device allocation failed");
    }
    HIP_TRY(c, hipMemcpyAsync(d_agg, agg.data(), sizeof(double) * agg.size(), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(d_vol, vol.data(), sizeof(double) * ne, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(d_id, ident.data(), sizeof(int32_t) * ne, hipMemcpyHostToDevice, c->stream));
    const double ns = which == DSMC_SAMPLE_STEADY ? (double)n_steady : 1.0;
    launch_fields(c->stream, d_agg, n_cells, ns, c->mass, c->FN, d_vol, d_id, d_out, nullptr, nullptr);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipMemcpyAsync(out, d_out, sizeof(double) * 15 * (size_t)n_cells, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    dev_free(c, d_agg); dev_free(c, d_vol); dev_free(c, d_out); dev_free(c, d_id);
    return DSMC_OK;
}

dsmc_status dsmc_get_state(dsmc_ctx c, dsmc_state* st) {
    if (!c || !st) return fail(c, DSMC_E_INVALID, "bad arguments");
    if (st->x || st->v || st->cell || st->pid || st->ir) {
        dsmc_status s = materialize(c);
        if (s != DSMC_OK) return s;
    }
    Scalars sc;
    dsmc_status s = sync_scalars(c, &sc);
    if (s != DSMC_OK) return s;
    const int64_t n = sc.np;
    st->n_particles = n;
    st->step = sc.step;
    st->next_pid = sc.next_pid;
    if (st->smax) {
        std::vector<double> sm(c->nt);
        HIP_TRY(c, hipMemcpy(sm.data(), c->d_smax, sizeof(double) * c->nt, hipMemcpyDeviceToHost));
        for (int t = 0; t < c->nt; ++t) st->smax[c->hm.orig[t]] = sm[t];
    }
    double* ir_out = c->dr ? st->ir : nullptr;
    if (!st->x && !st->v && !st->cell && !st->pid && !ir_out) return DSMC_OK;
    std::vector<double> xs(3 * n), vs(3 * n), irs(ir_out ? n : 0);
    std::vector<int32_t> cell(n);
    std::vector<uint32_t> pid(n);
    HIP_TRY(c, hipMemcpy(xs.data(), c->A.pos, 24 * n, hipMemcpyDeviceToHost));
    if (ir_out) HIP_TRY(c, hipMemcpy(irs.data(), c->A.ir, 8 * n, hipMemcpyDeviceToHost));
    if (c->vel64) {
        HIP_TRY(c, hipMemcpy(vs.data(), c->A.vel, 24 * n, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> f(3 * n);
        HIP_TRY(c, hipMemcpy(f.data(), c->A.vel, 12 * n, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < 3 * n; ++i) vs[i] = f[i];
    }
    HIP_TRY(c, hipMemcpy(cell.data(), c->A.cell, 4 * n, hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(pid.data(), c->A.pid, 4 * n, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; ++i) cell[i] = c->hm.orig[cell[i]];
    std::vector<int64_t> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
        if (cell[a] != cell[b]) return cell[a] < cell[b];
        return pid[a] < pid[b];
    });
    for (int64_t k = 0; k < n; ++k) {
        const int64_t i = idx[k];
        if (st->x) { st->x[3 * k] = xs[3 * i]; st->x[3 * k + 1] = xs[3 * i + 1]; st->x[3 * k + 2] = xs[3 * i + 2]; }
        if (st->v) { st->v[3 * k] = vs[3 * i]; st->v[3 * k + 1] = vs[3 * i + 1]; st->v[3 * k + 2] = vs[3 * i + 2]; }
        if (st->cell) st->cell[k] = cell[i];
        if (st->pid) st->pid[k] = pid[i];
        if (ir_out) ir_out[k] = irs[i];
    }
    return DSMC_OK;
}

dsmc_status dsmc_set_state(dsmc_ctx c, const dsmc_state* st) {
    if (!c || !st || st->n_particles < 0 || (st->n_particles > 0 && (!st->x || !st->v || !st->cell || !st->pid)))
        return fail(c, DSMC_E_INVALID, "bad arguments");
    const int64_t n = st->n_particles;
    if (n > c->cap) return fail(c, DSMC_E_CAPACITY, "state larger than the particle store");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->pending = false;  // the store is rewritten sorted
    std::vector<int64_t> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    for (int64_t i = 0; i < n; ++i)
        if (st->cell[i] < 0 || st->cell[i] >= c->nt) return fail(c, DSMC_E_INVALID, "particle cell out of range");
    const std::vector<int32_t>& inv = c->hm.inv;
    std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
        const int32_t ca = inv[st->cell[a]], cb = inv[st->cell[b]];
        if (ca != cb) return ca < cb;
        return st->pid[a] < st->pid[b];
    });
    std::vector<double> xs(3 * n), vs(3 * n);
    std::vector<int32_t> cell(n), counts(c->nt + 1, 0);
    std::vector<uint32_t> pid(n);
    for (int64_t k = 0; k < n; ++k) {
        const int64_t i = idx[k];
        for (int j = 0; j < 3; ++j) {
            xs[3 * k + j] = st->x[3 * i + j];
            vs[3 * k + j] = st->v[3 * i + j];
        }
        cell[k] = inv[st->cell[i]]; pid[k] = st->pid[i];
        counts[cell[k] + 1]++;
    }
    for (int t = 0; t < c->nt; ++t) counts[t + 1] += counts[t];
    HIP_TRY(c, hipMemcpy(c->A.pos, xs.data(), 24 * n, hipMemcpyHostToDevice));
    if (c->vel64) {
        HIP_TRY(c, hipMemcpy(c->A.vel, vs.data(), 24 * n, hipMemcpyHostToDevice));
    } else {
        std::vector<float> f(3 * n);
        for (int64_t i = 0; i < 3 * n; ++i) f[i] = (float)vs[i];
        HIP_TRY(c, hipMemcpy(c->A.vel, f.data(), 12 * n, hipMemcpyHostToDevice));
    }
    HIP_TRY(c, hipMemcpy(c->A.cell, cell.data(), 4 * n, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->A.pid, pid.data(), 4 * n, hipMemcpyHostToDevice));
    if (c->dr) {
        // rotational energies in the same order (zero when the caller gives none)
        std::vector<double> irs(n, 0.0);
        if (st->ir)
            for (int64_t k = 0; k < n; ++k) irs[k] = st->ir[idx[k]];
        HIP_TRY(c, hipMemcpy(c->A.ir, irs.data(), 8 * n, hipMemcpyHostToDevice));
    }
    HIP_TRY(c, hipMemcpy(c->d_offsets, counts.data(), 4 * (c->nt + 1), hipMemcpyHostToDevice));
    if (st->smax) {
        std::vector<double> sm(c->nt);
        for (int t = 0; t < c->nt; ++t) sm[t] = st->smax[c->hm.orig[t]];
        HIP_TRY(c, hipMemcpy(c->d_smax, sm.data(), sizeof(double) * c->nt, hipMemcpyHostToDevice));
    }
    Scalars sc;
    HIP_TRY(c, hipMemcpy(&sc, c->d_sc, sizeof sc, hipMemcpyDeviceToHost));
    sc.np = n;
    sc.n_entries = n;
    sc.step = st->step;
    sc.next_pid = st->next_pid;
    sc.ninj = 0;
    HIP_TRY(c, hipMemcpy(c->d_sc, &sc, sizeof sc, hipMemcpyHostToDevice));
    c->np_bound = n;
    return DSMC_OK;
}

dsmc_status dsmc_get_pair_counts(dsmc_ctx c, int32_t* ncand, int32_t* nacc) {
    if (!c) return fail(c, DSMC_E_INVALID, "NULL context");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    std::vector<int32_t> h(c->nt);
    if (ncand) {
        HIP_TRY(c, hipMemcpy(h.data(), c->d_ncand, 4 * (size_t)c->nt, hipMemcpyDeviceToHost));
        for (int t = 0; t < c->nt; ++t) ncand[c->hm.orig[t]] = h[t];
    }
    if (nacc) {
        HIP_TRY(c, hipMemcpy(h.data(), c->d_nacc, 4 * (size_t)c->nt, hipMemcpyDeviceToHost));
        for (int t = 0; t < c->nt; ++t) nacc[c->hm.orig[t]] = h[t];
    }
    return DSMC_OK;
}

dsmc_status dsmc_stats(dsmc_ctx c, dsmc_counters* out) {
    if (!c || !out) return fail(c, DSMC_E_INVALID, "bad arguments");
    Scalars sc;
    dsmc_status st = sync_scalars(c, &sc);
    Counters ct;
    HIP_TRY(c, hipMemcpy(&ct, c->d_ctr, sizeof ct, hipMemcpyDeviceToHost));
    out->n_particles = sc.np;
    out->hops = (int64_t)ct.hops;
    out->wall_hits = (int64_t)ct.walls;
    out->injected = (int64_t)ct.injected;
    out->removed = (int64_t)ct.removed;
    out->lost = (int64_t)ct.lost;
    out->step = sc.step;
    return st;
}

dsmc_status dsmc_set_local_acc(dsmc_ctx c, const uint8_t* flags) {
    if (!c || !flags) return fail(c, DSMC_E_INVALID, "bad arguments");
    std::vector<uint8_t> f(c->nt);
    for (int t = 0; t < c->nt; ++t) f[t] = flags[c->hm.orig[t]] ? 1 : 0;
    HIP_TRY(c, hipMemcpyAsync(c->d_local, f.data(), c->nt, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return DSMC_OK;
}

dsmc_status dsmc_profile(dsmc_ctx c, int32_t enable) {
    if (!c) return fail(c, DSMC_E_INVALID, "NULL context");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (auto& u : c->ev_used) {
        c->ev_pool.push_back(u.second.first);
        c->ev_pool.push_back(u.second.second);
    }
    c->ev_used.clear();
    c->profiling = enable != 0;
    return DSMC_OK;
}

int32_t dsmc_profile_read(dsmc_ctx c, double* total_ms, int64_t* launches, int32_t max_slots) {
    if (!c) return -1;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return -1;
    std::vector<double> ms(kNumSlots, 0.0);
    std::vector<int64_t> cnt(kNumSlots, 0);
    for (auto& u : c->ev_used) {
        float t = 0;
        if (hipEventElapsedTime(&t, u.second.first, u.second.second) == hipSuccess) {
            ms[u.first] += t;
            cnt[u.first] += 1;
        }
    }
    for (int i = 0; i < std::min<int>(max_slots, kNumSlots); ++i) {
        if (total_ms) total_ms[i] = ms[i];
        if (launches) launches[i] = cnt[i];
    }
    return kNumSlots;
}

const char* dsmc_profile_name(int32_t slot) {
    return (slot >= 0 && slot < kNumSlots) ? kSlotNames[slot] : "";
}

dsmc_status dsmc_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t n) {
    if (!ctr || !key || !out || n < 0) return fail(nullptr, DSMC_E_INVALID, "bad arguments");
    if (n == 0) return DSMC_OK;
    uint32_t* d_in = nullptr;
    uint32_t* d_out = nullptr;
    if (hipMalloc(&d_in, 16 * n) != hipSuccess) return fail(nullptr, DSMC_E_OOM, "hipMalloc failed");
    if (hipMalloc(&d_out, 16 * n) != hipSuccess) {
        hipFree(d_in);
        return fail(nullptr, DSMC_E_OOM, "hipMalloc failed");
    }
    dsmc_status st = DSMC_OK;
    if (hipMemcpy(d_in, ctr, 16 * n, hipMemcpyHostToDevice) != hipSuccess) st = DSMC_E_DEVICE;
    if (st == DSMC_OK) {
        launch_philox(nullptr, d_in, key[0], key[1], d_out, n);
        if (hipGetLastError() != hipSuccess || hipMemcpy(out, d_out, 16 * n, hipMemcpyDeviceToHost) != hipSuccess)
            st = DSMC_E_DEVICE;
    }
    hipFree(d_in);
    hipFree(d_out);
    if (st != DSMC_OK) return fail(nullptr, st, "device Philox failed");
    return DSMC_OK;
}

dsmc_status dsmc_device_copy(dsmc_ctx c, void* dst, const void* src, size_t bytes) {
    if (!c || !dst || !src || (bytes % 16) != 0) return fail(c, DSMC_E_INVALID, "bad arguments (bytes % 16)");
    launch_copy(c->stream, src, dst, bytes);
    HIP_TRY(c, hipGetLastError());
    return DSMC_OK;
}

dsmc_status dsmc_device_line_reads(dsmc_ctx c, const void* table, size_t bytes, void* sink, int share, int iters,
                                   int blocks) {
    if (!c || !table || !sink || bytes < 128 || ((uintptr_t)table % 16) != 0 || ((uintptr_t)sink % 4) != 0)
        return fail(c, DSMC_E_INVALID, "bad arguments (table of at least 128 bytes, 16-byte aligned; sink)");
    if (share < 1 || share > 64 || (share & (share - 1)) != 0 || iters < 1 || iters > 4096 || blocks < 1 ||
        blocks > 65536)
        return fail(c, DSMC_E_INVALID, "bad arguments (share a power of two in [1, 64], iters, blocks)");
    uint64_t lines = 1;
    while (lines * 2 <= bytes / 128 && lines * 2 <= (1ull << 32)) lines *= 2;
    launch_line_reads(c->stream, table, (uint32_t)(lines - 1), iters, share, blocks, sink);
    HIP_TRY(c, hipGetLastError());
    return DSMC_OK;
}

const char* dsmc_last_error(dsmc_ctx c) { return c ? c->err.c_str() : g_global_error.c_str(); }

void dsmc_destroy(dsmc_ctx c) {
    if (!c) return;
    hipStreamSynchronize(c->stream);
    dsmcx::dig_release(c);
    for (auto& g : c->graphs) drop_graph(g);
    for (auto& u : c->ev_used) {
        hipEventDestroy(u.second.first);
        hipEventDestroy(u.second.second);
    }
    for (hipEvent_t e : c->ev_pool) hipEventDestroy(e);
    for (void* p : c->owned) {
        if (c->has_alloc) c->alloc.free(p, c->alloc.user); else hipFree(p);
    }
    delete c;
}

}  // extern "C"
