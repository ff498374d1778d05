// Private definition of the library context shared by the C ABI sources.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/dsmc.h"
#include "../../include/mlp.h"
#include "kernels.h"
#include "mesh.h"

namespace dsmcx {

struct Buf {
    double* pos = nullptr;  // [cap][3]
    void* vel = nullptr;    // [cap][3] float or double
    int32_t* cell = nullptr;
    uint32_t* pid = nullptr;
    double* ir = nullptr;   // [cap] rotational energies, or null (monatomic gas)
};

template <class VT>
PartDev<VT> as_dev(const Buf& b) {
    return PartDev<VT>{b.pos, (VT*)b.vel, b.cell, b.pid, b.ir};
}

struct DigState;  // coupling state, owned by the context
void dig_release(dsmc_ctx c);

}  // namespace dsmcx

struct dsmc_ctx_s {
    hipStream_t stream = nullptr;
    dsmc_allocator alloc{};
    bool has_alloc = false;
    std::vector<void*> owned;
    std::string err;
    bool broken = false;

    dsmcx::HostMesh hm;
    int nt = 0, nb = 0;
    // species / run
    double mass = 0, dref = 0, omega = 0, Tref = 0, K = 0, ex = 0;
    double alpha = 1;   // VSS scattering exponent (1: VHS)
    int dr = 0;         // rotational degrees of freedom (0 or 2)
    double zr = 0, pinel = 0;  // rotational collision number, inelastic probability
    double a_heat[4] = {0, 0, 0, 0};  // heat-flux relaxation matrix of a rotating gas
    double* d_racc = nullptr;   // [4][nt] rotational sums (steady), when dr > 0
    double* d_rewma = nullptr;  // [4][nt] moving average of the rotational sums
    double* d_rinst = nullptr;  // [4][nt] rotational sums of the last step
    double FN = 0, dt = 0, n0 = 0, T0 = 0, u0[3] = {0, 0, 0};
    dsmcx::RngKey key{0, 0};
    int vel64 = 0, n_ss = 0, n_a = 1000, ewma_on = 0;
    int64_t cap = 0;
    // device mesh
    dsmcx::MeshDev mesh{};
    double4* d_plane = nullptr;
    int32_t* d_nbr = nullptr;
    double* d_vol = nullptr;
    int32_t* d_bf_group = nullptr;
    int32_t* d_bf_pcode = nullptr;
    double* d_bf_frame = nullptr;
    dsmcx::GroupDev* d_groups = nullptr;
    // surface sampling: [5][nb] sums (mesh.surf points here while on) and the
    // step window (to < 0: still running)
    double* d_surf = nullptr;
    // instantaneous sums ([13][nt], the last sampled step) while on
    double* d_inst = nullptr;
    bool inst_on = false;
    int64_t surf_from = 0, surf_to = -1;
    int4* d_tv = nullptr;
    double* d_xyz = nullptr;
    int32_t* d_orig = nullptr;      // internal cell -> caller's cell id
    int32_t* d_cell_tmp = nullptr;  // [nt+1] scratch of the initial fill
    // inflow
    dsmcx::InflowDev inflow{};
    int32_t* d_fcount = nullptr;
    int32_t* d_foff = nullptr;
    int64_t max_inject = 0;
    // particles
    dsmcx::Buf A, B;
    uint32_t* d_rank = nullptr;
    int32_t* d_perm = nullptr;
    dsmcx::WallQueue wq{nullptr, nullptr, nullptr, nullptr, 0};
    // cells
    int32_t* d_counts = nullptr;
    int32_t* d_offsets = nullptr;
    int32_t* d_blocksums = nullptr;
    double* d_smax = nullptr;
    int32_t* d_ncand = nullptr;
    int32_t* d_nacc = nullptr;
    double* d_acc = nullptr;
    double* d_ewma = nullptr;
    int32_t* d_ewma_m = nullptr;
    uint8_t* d_local = nullptr;
    dsmcx::Scalars* d_sc = nullptr;
    dsmcx::Counters* d_ctr = nullptr;
    int32_t* d_counts_orig = nullptr;  // [nt] scratch of the initial fill
    // tuning choices
    int move_variant = dsmcx::kMoveFace3;
    int move_batch = 0;
    int collide_variant = dsmcx::kCollideG3k;
    int sort_variant = dsmcx::kSortGather;
    int32_t* d_sortperm = nullptr;
    int reorder = 2;  // cell order: 0 caller's, 1 Morton, 2 Hilbert
    // host view
    int64_t np_bound = 0;
    // profiling
    bool profiling = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_used;
    std::vector<hipEvent_t> ev_pool;
    // boundary table (copied at init) and the coupling state, built on first use
    std::vector<dsmc_boundary_desc> bcs;
    dsmcx::DigState* dig = nullptr;
    // batch of independent cases sharing the mesh (null / 0 for one case)
    dsmcx::CaseDev* d_cases = nullptr;
    int32_t* d_cell_case = nullptr;     // internal cell -> case
    int32_t* d_case_of_orig = nullptr;  // caller cell -> case
    int32_t* d_case_first = nullptr;    // case -> first caller cell
    int n_cases = 0;
    // captured two-step graphs, keyed by the particle buffer current at capture
    bool capturing = false;
    // deferred sort: A holds the particles where the last move left them and
    // d_sortperm / B.cell their sorted order (slot -> particle, slot -> cell)
    bool pending = false;
    // particle-grid bound of the steps being captured (see capture_two_steps)
    int64_t capture_bound = 0;
    struct Graph {
        const void* a_x = nullptr;
        int sig = -1;
        int64_t bound = 0;  // grids of the captured kernels cover this many particles
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
    } graphs[2];
    std::vector<int32_t> case_cell0;
    dsmc_mlp closure = nullptr;  // learned HoT closure of the coupling step (not owned)
    double gate_tol = 0.05;
};

namespace dsmcx {

dsmc_status fail(dsmc_ctx c, dsmc_status s, const std::string& msg);
void* dev_alloc(dsmc_ctx c, size_t bytes);
void dev_free(dsmc_ctx c, void* p);

template <class T>
bool alloc_n(dsmc_ctx c, T*& p, size_t n) {
    p = (T*)dev_alloc(c, sizeof(T) * n);
    return p != nullptr;
}

// Exact particle count and latched device flags (synchronises).
dsmc_status sync_scalars(dsmc_ctx c, Scalars* out);
// Physically sorts the store when a deferred sort left its order pending.
dsmc_status materialize(dsmc_ctx c);

}  // namespace dsmcx

#define HIP_TRY(ctx, call)                                                                            \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess) {                                                                       \
            if (ctx) (ctx)->broken = true;                                                            \
            return ::dsmcx::fail(ctx, DSMC_E_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
        }                                                                                             \
    } while (0)
