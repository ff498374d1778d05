// DIG coupling step on the device: sampled macroscopic state, least-squares
// gradients, NSF relations and higher-order terms, admissibility gate with
// reconstruction passes, finite-volume pseudo-time solve, particle feedback
// (section 3, Algorithm 1).  All arrays use the internal cell numbering.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace dsmcx {

constexpr int kDigNV = 5;        // primitive variables of a monatomic gas: rho, u(3), T
// A gas with rotational degrees of freedom carries rho, u(3), T_t, T_r (6
// primitives), sigma(6), q_t(3), q_r(3) (12 HoT) and 18 sampled values.
constexpr int kDigNVR = 6;
constexpr int kDigThreads = 256;
constexpr int kFbLanes = 64;     // one wave per cell in the feedback kernel

// What lies behind a tet face: kind | (neighbour cell or boundary group) << 3.
enum : int { kLinkInterior = 0, kLinkPeriodic = 1, kLinkWall = 2, kLinkSpecular = 3, kLinkInflow = 4, kLinkOutflow = 5 };

struct DigGroup {
    double T;
    double u[3];
    double rho;  // freestream mass density (inflow)
};

// Coupling parameters of one case of a batch (independent meshes joined in
// one context): reference state, particle weight, generator key, cell
// ranges (caller numbering and internal order) and the next particle id.
struct DigCase {
    double FN;
    double mu0, p0, kfac;  // reference Knudsen number mu0 / (p0 L0) kfac, kfac = sqrt(pi R T0 / 2)
    double T0, rho0, mass_scale;
    uint32_t k0, k1;
    int32_t cell0, cell_end;  // caller cells [cell0, cell_end)
    int32_t first, end;       // internal cells [first, end)
    int32_t enabled;          // 0: the case's particles are left as they are
    int32_t closed;           // no inflow or outflow face: the solve's mass is rescaled
    uint32_t next_pid;
};

struct DigGeom {
    int nt;
    const double* cen;     // [nt][3] centroid
    const double* fcen;    // [nt][4][3] face centroid
    const double* fnu;     // [nt][4][3] outward unit normal
    const double* farea;   // [nt][4]
    const double* fdx;     // [nt][4][3] centroid -> neighbour centroid (periodic: shifted) or -> face centroid
    const int32_t* flink;  // [nt][4]
    const double* lsq;     // [nt][9] inverse of the weighted least-squares normal matrix
    const double* vol;     // [nt]
    const DigGroup* groups;
    double mass, R, mu_ref, omega, T_ref;
    double FN;  // real molecules per particle
    const int32_t* cell_case;  // batch: internal cell -> case (null for one case)
    DigCase* cases;            // batch: per-case parameters
    int n_cases;
    int skip_idle;             // batch: the solve leaves out the cells of cases not coupled
    // rotating gas (dr = 2): rotational collision number, heat-flux
    // relaxation matrix (A_tt, A_tr, A_rt, A_rr) and R T0, the scale of the
    // rotational-energy residual in the convergence norm (per case in a batch)
    int dr;
    double zr;
    double a_heat[4];
    double ert;
};

struct DigCtl {
    double res0, res, dtmin;
    int conv, failed, iters;
    int n_rejected, n_reconstructed, n_unreached;
    int n_closure, n_fallback;
    double mass_scale;
};

// Arrays below are per cell with NV = 5 primitives and NH = 9 HoT for a
// monatomic gas, NV = 6 and NH = 12 for a rotating one.
struct DigWork {
    double* samp;     // [nt][14] rho, u(3), T, sigma(6), q(3) of the moving average (rotating: [nt][18],
                      // then T_r, q_r(3)); NaN without samples
    uint8_t* ok;      // [nt] cell has samples
    double* prim;     // [nt][NV] working state; M^{k+1} after the solve
    double* half;     // [nt][NV] M^{k+1/2} after the gate
    double* hot;      // [nt][NH] cell HoT
    double* hotf;     // [nt][4][NH] HoT carried by each cell face (the solve's closure)
    double* grad;     // [nt][NV][3] gradients of the primitives
    double* kn;       // [nt]
    uint8_t* avail;   // [nt]
    uint8_t* navail;  // [nt]
    double* nprim;    // [nt][NV] reconstruction candidates of one pass
    double* nhot;     // [nt][NH]
    int32_t* state;   // [nt] 0 admissible, 1 reconstructed, 2 unreached
    double* mprev;    // [nt][NV] M^k
    double* Rs;       // [nt][NV] residual
    double* dt;       // [nt] pseudo-time step
    double* U0;       // [nt][NV] conserved state at the start of an iteration
    double* stage;    // [nt][NV] stage state
    double* partial;  // [2 * blocks] reduction partials (blocks of the residual kernel: 4 lanes per cell)
    DigCtl* ctl;
    int32_t* fb_cnt;  // [nt] clones per cell, caller order
    int32_t* fb_off;  // [nt + 1]
    int32_t* fb_tgt;  // [nt] target count per internal cell
    float* cx;        // [nt][13] closure inputs
    float* ct;        // [nt][9] nondimensional sampled HoT
    float* cs;        // [nt][9] nondimensional sampled stress and heat flux
    float* cy;        // [nt][9] closure outputs
    uint8_t* cvalid;  // [nt]
};

// rewma [4][nt]: the rotational moving-average sums of a rotating gas (else null)
void launch_dig_sampled(hipStream_t s, const DigGeom& g, const double* ewma, const double* rewma, double FN, DigWork w);
void launch_dig_kn(hipStream_t s, const DigGeom& g, DigWork w, double kn_ref, double T0, double rho0, double L0);
void launch_dig_gradients(hipStream_t s, const DigGeom& g, const double* prim, double* grad, const DigCtl* ctl);
void launch_dig_hot(hipStream_t s, const DigGeom& g, DigWork w);
// Face HoT from cell HoT at prim (with `consistent`, corrected so that each
// face's viscous stress at prim is the average of its cells' NSF + HoT).
void launch_dig_face_hot(hipStream_t s, const DigGeom& g, const double* prim, const double* grad, const double* hot,
                         double* hotf, int consistent);
void launch_dig_gate(hipStream_t s, const DigGeom& g, DigWork w, double kn_max, int passes);
void launch_dig_ctl_reset(hipStream_t s, DigCtl* ctl);
void launch_dig_copy(hipStream_t s, const double* src, double* dst, int64_t n);
void launch_dig_residual(hipStream_t s, const DigGeom& g, const double* prim, const double* hotf, const double* grad,
                         double* Rs, DigWork w, int first, double cfl);
void launch_dig_iteration(hipStream_t s, const DigGeom& g, DigWork w, double cfl, double eps_m, int global_dt,
                          int it);
// Closed domain: scale the density of w.prim so that its total mass equals
// the particles' (n_particles F_N m).
void launch_dig_mass_rescale(hipStream_t s, const DigGeom& g, DigWork w, const Scalars* sc,
                             const int32_t* offsets);
// Batch: the next particle id of each case after its feedback clones.
void launch_dig_case_pids(hipStream_t s, const DigGeom& g, const DigWork& w);
// Batch: next particle id of each case = its largest id + 1.
void launch_dig_case_pid_init(hipStream_t s, const DigGeom& g, const int32_t* cell, const uint32_t* pid,
                              const Scalars* sc, int64_t bound);
// Anderson acceleration of the pseudo-time iteration (type II, Walker and
// Ni): the iteration G is applied as a fixed-point map to the primitive
// state x; with f = G(x) - x, the next state is G(x_k) - sum_i gamma_i dG_i,
// gamma minimising |f_k - sum_i gamma_i dF_i| in the norm weighted by
// 1/scale^2 per variable over the last m differences dF_i = f_{i+1} - f_i,
// dG_i = G(x_{i+1}) - G(x_i).
struct AaWork {
    double* x;      // [nt][5] input of the current application of G
    double* fprev;  // [nt][5] f of the previous application (then the current one)
    double* gprev;  // [nt][5] G of the previous application (then the current one)
    double* dF;     // [m][nt][5]
    double* dG;     // [m][nt][5]
    double* part;   // [blocks][2m + 1] block partials of the inner products
    double* red;    // [2m + 2] reduced inner products, then two fallback counts
                    // (used by alternate iterations)
    double* gam;    // [m] coefficients
    int m;
};
// f = gx - x into fprev (after dF_slot = f - fprev, dG_slot = gx - gprev
// unless first), gx into gprev; clears the fallback count red[2m + parity].
void launch_aa_diff(hipStream_t s, const DigGeom& g, const AaWork& a, const double* gx, int slot, int first,
                    int parity);
// red[i] = <dF_slot, dF_i> (i < cnt), red[m + i] = <f, dF_i>; weights w[5].
void launch_aa_dots(hipStream_t s, const DigGeom& g, const AaWork& a, int slot, int cnt, const double* w5);
// prim = gprev - sum_i gam_i dG_i cell by cell; a cell whose result is not
// physical (density or temperature <= 0) keeps gprev; red[2m + parity]
// counts them.
void launch_aa_update(hipStream_t s, const DigGeom& g, const AaWork& a, int cnt, double* prim, int parity);

// Newton-Krylov solve of the steady equations: pseudo-transient
// continuation (Kelley and Keyes 1998) with one GMRES(m) cycle per Newton
// step (Saad and Schultz 1986), Jacobian products by forward differences of
// the residual (Knoll and Keyes 2004), unknowns and equations scaled by
// NkScale, right preconditioning by the pseudo-time diagonal.
constexpr int kNkMaxKrylov = 100;
struct NkScale {
    double s[kDigNVR];  // rho0, rho0 a0 (3), rho0 a0^2 (energy, and rho e_r)
};
struct NkWork {
    double* V;     // [m + 1][nt][NV] Krylov basis
    double* w;     // [nt][NV] new direction
    double* U;     // [nt][NV] conserved state of the Newton iterate
    double* Ut;    // [nt][NV] trial state
    double* R0;    // [nt][NV] residual at U
    double* Rp;    // [nt][NV] residual at the perturbed state
    double* part;  // [m + 1][blocks] block partials
    double* red;   // reduced values, slots below
    double* y;     // [m] coefficients of the update
    int32_t* flag; // a trial or perturbed cell was not physical
    int m;
};
// Slots of NkWork::red: first and second Gram-Schmidt coefficients, |w|^2,
// |V/p|^2 and the finite-difference step of the next product, |b|^2 and
// |U/scale|^2 of the Newton step.
__host__ __device__ constexpr int kNkH1(int m) { return 0; }
__host__ __device__ constexpr int kNkH2(int m) { return m + 1; }
__host__ __device__ constexpr int kNkHn2(int m) { return 2 * m + 2; }
__host__ __device__ constexpr int kNkVs2(int m) { return 2 * m + 3; }
__host__ __device__ constexpr int kNkEps(int m) { return 2 * m + 4; }
__host__ __device__ constexpr int kNkBeta2(int m) { return 2 * m + 5; }
__host__ __device__ constexpr int kNkXr2(int m) { return 2 * m + 6; }
__host__ __device__ constexpr int kNkRedSize(int m) { return 2 * m + 7; }
// Residual and spectral sums at w.prim (w.Rs, w.dt = V / S), the stopping
// test of Newton step `it` (w.ctl), R0, U (from w.prim when it == 0), V_0 =
// -R0 / scale; |V_0|^2 and |U/scale|^2 into red.
void launch_nk_begin(hipStream_t s, const DigGeom& g, DigWork w, NkWork nk, NkScale sc, int it, double eps_m);
// V_0 /= sqrt(red[beta2]) and the finite-difference step of its product.
void launch_nk_scale(hipStream_t s, const DigGeom& g, DigWork w, NkWork nk, double cfl, double fd);
// Arnoldi step j: the product with V_j, two Gram-Schmidt passes (H column j
// = red[H1] + red[H2], |w|^2 in red[Hn2]), V_{j+1} and the next step.
void launch_nk_arnoldi(hipStream_t s, const DigGeom& g, DigWork w, NkWork nk, NkScale sc, int j, double cfl,
                       double fd);
// Trial state U + alpha P^-1 V y (y in nk.y, jn terms) into nk.Ut, w.stage.
void launch_nk_try(hipStream_t s, const DigGeom& g, DigWork w, NkWork nk, NkScale sc, int jn, double alpha,
                   double cfl);
// U = Ut, w.prim = w.stage.
void launch_nk_commit(hipStream_t s, const DigGeom& g, DigWork w, NkWork nk);

// Local-accumulation flags from the gate states (cases of a batch that are
// not coupled keep theirs).
void launch_dig_set_local(hipStream_t s, const DigGeom& g, const int32_t* state, uint8_t* local);
void launch_dig_fb_count(hipStream_t s, const DigGeom& g, DigWork w, const int32_t* offsets, const int32_t* orig,
                         const Scalars* sc, RngKey key);
template <class VT>
void launch_dig_fb_apply(hipStream_t s, const DigGeom& g, DigWork w, PartDev<VT> p, const int32_t* offsets, const int4* tv,
                         const double* xyz, const int32_t* orig, const Scalars* sc, RngKey key, int32_t* scratch,
                         uint32_t* bits, int nt, int64_t cap);
void launch_dig_count_all(hipStream_t s, const int32_t* cell, const Scalars* sc, int32_t* counts, uint32_t* rank,
                          int64_t bound);
void launch_fill_u8(hipStream_t s, uint8_t* p, uint8_t v, int64_t n);
void launch_dig_closure_prep(hipStream_t s, const DigGeom& g, DigWork w);
// ewma [13][nt] moving-average sums (row 0: mean particles per step), ewma_m
// [nt] samples taken, n_a the moving average's length
void launch_dig_closure_gate(hipStream_t s, const DigGeom& g, DigWork w, double tol, const double* ewma,
                             const int32_t* ewma_m, int n_a);

}  // namespace dsmcx
