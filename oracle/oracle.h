/*
 * Plain CPU oracle of the DSMC particle loop (test infrastructure only).
 *
 * This library is a slow, single-threaded, obviously-sequential statement of
 * what the GPU path computes.  It is used only by the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark; the product path never
 * links, loads or calls it.  It shares no code with the GPU library: both are
 * written independently from the paper (DSMC step splitting, section 2.1;
 * cell sampling, eq. dsmc_temperatures; exponential averaging,
 * eq. exponential_average_moments_ch3; steady average,
 * eq. steady_average_moments_ch3) and from the written arithmetic contracts
 * for geometry, random numbers and operation order.
 *
 * Units are SI.  Every floating-point operation is a separate IEEE binary64
 * operation (built with -ffp-contract=off, no fast-math).
 */
#ifndef DSMC_ORACLE_H
#define DSMC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct osim osim;

enum { O_BC_DIFFUSE = 0, O_BC_SPECULAR = 1, O_BC_INFLOW = 2, O_BC_OUTFLOW = 3, O_BC_PERIODIC = 4 };
enum { O_STAGE_MOVE = 1, O_STAGE_INJECT = 2, O_STAGE_SORT = 4, O_STAGE_COLLIDE = 8, O_STAGE_SAMPLE = 16 };

/* Philox4x32-10 block (counter ctr[4], key key[2]) -> out[4]. */
void oracle_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Build the simulation: mesh, boundary groups, species and run parameters.
 * Returns NULL on an invalid mesh (message via oracle_last_error()). */
osim* oracle_create(int nv, const double* xyz, int nt, const int* tet,
                    int nb, const int* bface, const int* bgroup, const int* bpartner,
                    int ng, const int* g_kind, const double* g_T, const double* g_u,
                    const double* g_n, const double* g_shift,
                    double mass, double d_ref, double omega, double T_ref,
                    double F_N, double dt, uint32_t seed, uint32_t case_id,
                    int vel_fp32, int n_ss, int n_a, int ewma_on);
const char* oracle_last_error(void);
void oracle_destroy(osim*);

/* Initial equilibrium fill at (n0, T0, u0); also sets (sigma c)_max. */
int oracle_init_fill(osim*, double n0, double T0, const double* u0);

/* Advance n steps (all stages), or one step restricted to a stage mask. */
int oracle_step(osim*, int n);
int oracle_step_stages(osim*, int mask);

/* State in (cell, pid) order. */
int64_t oracle_num_particles(const osim*);
void oracle_get_particles(const osim*, double* x, double* v, int* cell, uint32_t* pid);
/* ir[np]: rotational energies (J) when the gas rotates (NULL: zero). */
int oracle_set_particles(osim*, int64_t np, const double* x, const double* v,
                         const int* cell, const uint32_t* pid, uint32_t step, uint32_t next_pid,
                         const double* ir);
/* VSS scattering exponent (section 2.1; 1, the default, is VHS).  Also
 * scales the viscosity the continuum side uses.  -1 unless alpha > 0. */
int oracle_set_alpha(osim*, double alpha);
/* Rotational degrees of freedom d_r (0 or 2) and rotational collision
 * number Z_r (section 2.1, eq. inelastic_probability); call after
 * oracle_set_alpha and before the fill.  -1 on other values. */
int oracle_set_rotation(osim*, int dr, double zr);
double oracle_inelastic_probability(const osim*);
/* Rotational energies in (cell, pid) order (nothing for a monatomic gas). */
void oracle_get_rotation(const osim*, double* ir);
/* Rotational sums [nt][4] = sum I_r, sum v_i I_r (0 steady, 1 moving
 * average, 2 last step) and fields [nt][4] = T_r, q_r (eq. dsmc_temperatures). */
void oracle_get_rot_sums(const osim*, int which, double* out);
void oracle_rot_fields(const osim*, int which, double* out);
/* Viscosity of the species at temperature T (VHS/VSS power law). */
double oracle_viscosity(const osim*, double T);
void oracle_get_smax(const osim*, double* out);
void oracle_set_smax(osim*, const double* in);
uint32_t oracle_step_index(const osim*);

/* Surface sampling of the wall interactions (diffuse and specular faces):
 * on = 1 clears the sums and starts, 0 stops.  oracle_get_surface copies
 * the sums [nb][5] (boundary faces in input order: sum of v_in - v_out (3),
 * of (|v_in|^2 - |v_out|^2)/2, hits) and returns the number of sampled
 * steps (steps after n_ss inside the on window). */
int oracle_surface_sampling(osim*, int on);
int64_t oracle_get_surface(const osim*, double* sums);
/* A rotating gas: the rotational energy given to each boundary face,
 * sums[nb] (incident minus re-emitted I_r at every diffuse re-emission);
 * returns the sampled step count (0 and nothing copied for a monatomic
 * gas). */
int64_t oracle_get_surface_rot(const osim*, double* sums);
uint32_t oracle_next_pid(const osim*);

/* Per-cell candidate / accepted pair counts of the last collide stage. */
void oracle_get_pair_counts(const osim*, int* ncand, int* nacc);
/* counters: hops, wall hits, injected, removed (outflow), lost */
void oracle_get_counters(const osim*, int64_t out[5]);

/* Moment sums [nt][13]: S0, S1(3), S2(xx,yy,zz,xy,xz,yz), S3(3).
 * which: 0 steady accumulator (sum over sampled steps), 1 EWMA, 2 last step. */
void oracle_get_sums(const osim*, int which, double* out);
int64_t oracle_num_steady(const osim*);
/* Replace the steady (0) or moving-average (1) sums [nt][13]. */
void oracle_set_sums(osim*, int which, const double* in);
/* Per-cell numbers of moving-average samples taken. */
void oracle_get_ewma_counts(const osim*, int* out);
void oracle_set_local_acc(osim*, const unsigned char* flags);
/* fields [nt][15]: n, rho, u(3), T, sigma(xx,yy,zz,xy,xz,yz), q(3) */
void oracle_fields(const osim*, int which, double* out);
void oracle_fields_of_sums(const osim*, const double* sums, const double* vol, int n, double ns, double* out);

/* Geometry accessors for the tests. */
void oracle_get_volumes(const osim*, double* vol);
void oracle_get_neighbours(const osim*, int* nbr /* [nt][4], -1-bface on the boundary */);
void oracle_get_tets(const osim*, int* tv /* [nt][4] reoriented */);
int oracle_num_faces(const osim*);

/* Trace one particle for time t from (x, v) in cell with the given pid/step;
 * returns the final cell (-1 if deleted) and writes x, v. */
int oracle_trace_one(osim*, double* x, double* v, int cell, uint32_t pid, uint32_t step, double t);

/* ------------------------------------------------------------------ */
/* DIG coupling (paper sections 2.2 and 3, Algorithm 1).               */
/* ------------------------------------------------------------------ */
typedef struct {
    double kn_max;  /* admissibility threshold on the cell Knudsen number */
    int passes;     /* neighbour reconstruction passes */
    int n_m;        /* maximum macroscopic iterations */
    double eps_m;   /* relative residual tolerance */
    double cfl;     /* pseudo-time CFL number */
    double L0;      /* reference length of the Knudsen number */
    int feedback;   /* 1: adjust the particles to the macroscopic solution */
    int global_dt;  /* 1: one pseudo-time step for all cells (conservative) */
    int warm_start; /* 1: the solve starts from M^k instead of M^{k+1/2} */
    int unconverged; /* 1: feed back also a solve that stopped at n_m */
    int solver;     /* 0: three-stage pseudo-time marching; 1: Newton-Krylov
                       (n_m counts Newton steps, cfl is the initial
                       pseudo-time CFL number of the continuation) */
    int krylov;     /* GMRES steps per Newton step (0: 40) */
} odig_params;

typedef struct {
    int iters;
    double residual;   /* last relative density residual */
    int converged;
    int failed;        /* non-physical state: feedback skipped */
    int n_rejected;    /* cells failing the admissibility criterion */
    int n_reconstructed;
    int n_unreached;
    int64_t np_before, np_after;
    int fed_back;      /* the particles were adjusted */
    int krylov_steps;  /* Newton-Krylov solve: GMRES steps in all */
} odig_report;

/* Reference state (n0, T0, u0) used by the admissibility criterion and as the
 * initial macroscopic state; set by oracle_init_fill or explicitly. */
void oracle_set_reference(osim*, double n0, double T0, const double* u0);

/* A rotating gas (d_r = 2) couples through the polyatomic equations of
 * section 2.2: primitives [nt][6] = rho, u(3), T_t, T_r; HoT [nt][12] =
 * sigma(6), q_t(3), q_r(3); the heat conductivities from the relaxation
 * matrix A (eq. thermal_conductivity_matrix), set here (A_tt, A_tr, A_rt,
 * A_rr; the default is the nitrogen matrix 0.786, -0.201, -0.059, 0.842).
 * The arrays below are [nt][5] and [nt][9] for a monatomic gas. */
int oracle_set_heat_relaxation(osim*, const double* a);

/* Sampled macroscopic state of every cell from the moving-average sums:
 * out[nt][14] = rho, u(3), T, sigma(6), q(3) (rotating gas: [nt][18], then
 * T_r, q_r(3)); NaN for cells without samples. */
void oracle_dig_sampled(osim*, double* out);
/* Least-squares gradients of u and T: grad[nt][12] = du_i/dx_j (row-major),
 * dT/dx_j (rotating gas: [nt][15], then dT_r/dx_j), from the primitives. */
void oracle_dig_gradients(osim*, const double* prim, double* grad);
/* NSF stress and heat flux from prim and its gradients: out[nt][9] (rotating
 * gas: [nt][12], sigma, q_t, q_r). */
void oracle_dig_nsf(osim*, const double* prim, const double* grad, double* out);
/* Cell Knudsen number Kn_Delta for prim: out[nt]. */
void oracle_dig_kn_cell(osim*, const double* prim, double L0, double* out);
/* Admissibility gate + reconstruction passes on (prim[nt][5], hot[nt][9]) in
 * place; state[nt] out: 0 admissible, 1 reconstructed, 2 unreached (kept
 * the previous macroscopic state, HoT = 0). */
void oracle_dig_gate(osim*, double* prim, double* hot, const double* kn, double kn_max, int passes, int* state);
/* Macroscopic synthetic solve from prim (in/out) with frozen hot. */
int oracle_dig_solve(osim*, double* prim, const double* hot, const odig_params*, odig_report*);
/* HoT of every cell face hotf[nt][4][9] from cell HoT at prim: averaged to
 * the faces, and with `consistent` corrected so that at prim each face's
 * viscous stress is the average of the two cells' NSF + HoT. */
void oracle_dig_face_hot(osim*, const double* prim, const double* hot, int consistent, double* hotf);
/* Residual at prim with given face HoT hotf[nt][4][9]: out[nt][5]. */
void oracle_dig_residual_faces(osim*, const double* prim, const double* hotf, double* out);
/* Residual of the discrete macroscopic equations at prim: out[nt][5]. */
void oracle_dig_residual(osim*, const double* prim, const double* hot, double* out);
/* Particle feedback from (prim_old -> prim_new) on cells with state <= 1. */
void oracle_dig_feedback(osim*, const double* prim_old, const double* prim_new, const int* state);
/* One outer coupling cycle after the DSMC steps of the window. */
int oracle_dig_couple(osim*, const odig_params*, odig_report*);
void oracle_get_mprev(const osim*, double* out);

#ifdef __cplusplus
}
#endif
#endif
