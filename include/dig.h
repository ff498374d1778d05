/*
 * dig.h — C ABI of the DIG coupling step on top of a dsmc_ctx.
 *
 * One outer cycle of the paper's Algorithm 1 (section 3): after a window of
 * DSMC steps, the moving-average sums of every cell give the sampled
 * low-order state M^{k+1/2} = (rho, u, T) (eq. sampled_macro_state_ch3) and
 * the sampled stress and heat flux; the higher-order terms (HoT) are their
 * difference from the NSF relations evaluated with that state and its
 * gradients (eq. nsf_heat_flux, eq. hot_extraction_ch3).  Cells whose local
 * Knudsen number (eq. cell_kn_stability) exceeds the threshold are rebuilt
 * from admissible face neighbours over several passes and switch to local
 * accumulation (section 3.2).  The macroscopic equations (eq. macro,
 * monatomic) are then solved towards steady state with the HoT frozen
 * (eq. hot_used_in_macro_solver_ch3), stopping at the relative residual
 * eps_m or after n_m iterations, and the particles are adjusted to the new
 * state M^{k+1} (Algorithm 1, feedback step).
 *
 * The paper leaves the finite-volume discretisation and the particle
 * feedback map to other work; this library implements:
 *  - cell-centred finite volumes on the tets with weighted least-squares
 *    gradients (weights 1/|dx|^2 over face neighbours; a diffuse wall
 *    contributes its velocity and temperature at the face centroid),
 *    linear face reconstruction, a central inviscid flux with scalar
 *    dissipation scaled by min(1, max(Mach, 0.05)), NSF viscous fluxes from
 *    averaged gradients with a jump correction along the centroid connector
 *    plus the face average of the frozen HoT, no-slip walls (wall HoT from
 *    the adjacent cell), Dirichlet freestream at inflow faces and zero
 *    gradient at outflow faces;
 *  - explicit three-stage pseudo-time marching (stage weights 1/3, 1/2, 1)
 *    with the local step cfl V / sum_f A (|u.n| + c + viscous rate);
 *  - feedback per admissible or reconstructed cell: velocities shifted and
 *    scaled, v' = u_new + sqrt(T_new / T_old) (v - u_old); particle count
 *    set to floor(rho_new V / (F_N m) + U) (V the cell volume, m the
 *    molecular mass: unchanged when rho_new equals the density the cell's
 *    particles carry) by deleting particles chosen one at a time among the
 *    remaining (pid order) or by cloning random particles to uniform
 *    positions in the cell with new pids; re-sorted; only after a solve
 *    that converged (dig_params.unconverged).
 *
 * Conventions are those of dsmc.h: status codes, SI units, host arrays in
 * the caller's cell numbering ([n_tets][k] row-major), calls synchronise
 * the context's stream.  Random numbers of the feedback use generator
 * purpose 7 with the caller's cell id as subject and the current step.
 */
#ifndef DSMC_DIG_H
#define DSMC_DIG_H

#include "dsmc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double kn_max;      /* admissibility threshold on Kn_Delta (eq. cell_kn_stability) */
    int32_t passes;     /* neighbour reconstruction passes (section 3.2) */
    int32_t n_m;        /* maximum macroscopic iterations (Algorithm 1) */
    double eps_m;       /* relative residual tolerance of the macroscopic solve */
    double cfl;         /* pseudo-time CFL number */
    double L0;          /* reference length of the Knudsen number, m */
    int32_t feedback;   /* 1: adjust the particles to M^{k+1} */
    int32_t global_dt;  /* 1: one pseudo-time step for all cells */
    int32_t warm_start; /* 1: the solve starts from the previous macroscopic
                           solution M^k (same steady target), 0: from M^{k+1/2} */
    int32_t accel;      /* 0: plain pseudo-time iterations; m > 0: Anderson
                           mixing of the iterates over the last m (<= 64)
                           differences (one host synchronisation per
                           iteration; same steady solution) */
    int32_t unconverged; /* 0 (default): the closed-domain mass rescale and
                           the particle feedback follow only a solve that
                           reached eps_m; 1: also a solve that stopped at
                           n_m iterations (never one that failed) */
    int32_t solver;     /* 0: three-stage pseudo-time marching (n_m
                           iterations); 1: Newton-Krylov solve of the same
                           steady equations (n_m Newton steps; cfl is the
                           initial CFL number of its pseudo-transient
                           continuation; not with accel, global_dt or a
                           batch) */
    int32_t krylov;     /* GMRES steps per Newton step, 0 (default 40) to 100 */
} dig_params;

typedef struct {
    int32_t iters;           /* completed macroscopic iterations */
    double residual;         /* last density residual norm over the first one */
    int32_t converged;       /* residual <= eps_m reached */
    int32_t failed;          /* a non-physical state appeared: feedback skipped */
    int32_t n_rejected;      /* cells failing the admissibility criterion */
    int32_t n_reconstructed; /* rejected cells rebuilt from neighbours */
    int32_t n_unreached;     /* rejected cells keeping M^k with zero HoT */
    int64_t np_before, np_after;
    int32_t n_closure;       /* cells whose HoT came from the learned closure (mlp.h) */
    int32_t n_fallback;      /* cells with samples that kept the sampled HoT */
    int32_t fed_back;        /* 1: the particles were adjusted to M^{k+1} */
    int32_t krylov_steps;    /* Newton-Krylov solve: GMRES steps (residual
                                evaluations of Jacobian products) in all */
} dig_report;

/* One coupling cycle (Algorithm 1) on the context's current moving-average
 * sums and particles.  Skips the solve and the feedback when every cell is
 * rejected; skips the feedback when the solve fails or, unless
 * params->unconverged, when it did not reach eps_m within n_m iterations
 * (the report says which, and fed_back whether the particles changed).
 * The solution of a solve that did not fail becomes M^k, the state kept for
 * unreached cells and the warm start of the next cycle.  Sets the local
 * accumulation flags of rejected cells.  DSMC_E_CAPACITY if the clones of
 * the feedback would overflow the particle store (state left unchanged).
 *
 * A gas with two rotational degrees of freedom (dsmc_species_desc.dof_rot)
 * couples through the polyatomic equations of section 2.2: the primitives
 * are rho, u(3), T_t, T_r; the total energy includes e_r = (d_r/2) R T_r
 * and a sixth equation carries rho e_r with the rotational heat flux and
 * the relaxation source (d_r/2) rho R (T - T_r) / (Z_r tau), T = (3 T_t +
 * d_r T_r)/(3 + d_r), tau = mu(T_t)/p_t (eq. macro); the NSF heat fluxes are
 * -kappa_t grad T_t and -kappa_r grad T_r with (kappa_t, kappa_r) = (mu R /
 * 2) A^{-1} (5, d_r) (eq. thermal_conductivity_matrix, A from the species);
 * the HoT include q_r; the solve's convergence norm adds the
 * rotational-energy residual divided by R T0 to the density residual; the
 * feedback scales each particle's I_r by T_r^{k+1}/T_r^{k+1/2}.  The
 * learned closure and params->accel are refused for it (DSMC_E_INVALID). */
dsmc_status dig_couple(dsmc_ctx ctx, const dig_params* params, dig_report* report);

/* Batch contexts (dsmc_batch_init): one call couples every enabled case at
 * once (with the pseudo-time marching: params->solver = 1 is refused).  Each case uses its own reference state (n0, T0) for the Knudsen
 * number, its own F_N, generator key and case-local cell subjects and
 * particle ids (a case's next id starts at its largest id + 1 when the
 * coupling state is first built), and its own closed-domain mass rescale,
 * so an enabled case reproduces the single-case cycle of that case.  The
 * pseudo-time solve runs over all cells together: its stopping test (eps_m)
 * and, with global_dt or accel, its step and mixing coefficients are
 * batch-wide, so only with eps_m = 0, local steps and accel = 0 is each
 * case's solve the one its own context would make.  Report counts are
 * batch totals.  All cases are enabled until dig_batch_enable says
 * otherwise. */

/* Per-cell arrays of the last dig_couple, in caller cell order (widths of a
 * rotating gas in brackets):
 *  DIG_OUT_SAMPLED [n][14] rho, u(3), T, sigma(6), q(3) of the moving average
 *                          ([n][18]: then T_r, q_r(3)); NaN: no samples
 *  DIG_OUT_HALF    [n][5]  M^{k+1/2} after the gate and reconstruction ([n][6]: rho, u, T_t, T_r)
 *  DIG_OUT_NEW     [n][5]  M^{k+1} from the macroscopic solve ([n][6])
 *  DIG_OUT_HOT     [n][9]  frozen HoT (sigma xx,yy,zz,xy,xz,yz; q) after reconstruction
 *                          ([n][12]: sigma, q_t, q_r)
 *  DIG_OUT_KN      [n]     Kn_Delta of the sampled state (inf: no samples)
 *  DIG_OUT_STATE   [n]     int32: 0 admissible, 1 reconstructed, 2 unreached
 *  DIG_OUT_MPREV   [n][5]  the state M^k kept for unreached cells ([n][6]) */
enum {
    DIG_OUT_SAMPLED = 0, DIG_OUT_HALF = 1, DIG_OUT_NEW = 2, DIG_OUT_HOT = 3,
    DIG_OUT_KN = 4, DIG_OUT_STATE = 5, DIG_OUT_MPREV = 6
};
dsmc_status dig_get(dsmc_ctx ctx, int32_t which, void* out);

/* Residual of the discrete macroscopic equations (eq. macro with frozen
 * HoT) at prim[n][5] = rho, u(3), T: out[n][5] = sum over the cell's faces
 * of the numerical flux times the face area (mass, momentum, energy); a
 * rotating gas: prim[n][6] = rho, u(3), T_t, T_r, hot[n][12], out[n][6]
 * with rho e_r last, less the cell volume times its relaxation source. */
dsmc_status dig_residual(dsmc_ctx ctx, const double* prim, const double* hot, double* out);

/* Macroscopic solve alone from prim[n][5] (in/out) with frozen hot[n][9]
 * (rotating gas: [n][6] and [n][12]); uses n_m, eps_m, cfl, global_dt,
 * accel, solver and krylov of params.  With solver = 1 (Newton-Krylov) the
 * steady state is the marching's (the same discrete equations), n_m counts
 * Newton steps and report->krylov_steps the GMRES steps; a perturbed or
 * updated state that stays non-physical after ten halvings ends the solve
 * with report->failed.  Both solvers take their stopping test on the
 * density residual (a rotating gas adds its rotational-energy residual)
 * against its value at the start, which a warm start from a near solution
 * makes strict. */
dsmc_status dig_solve(dsmc_ctx ctx, double* prim, const double* hot, const dig_params* params,
                      dig_report* report);

/* Particle feedback alone: from prim_old[n][5] to prim_new[n][5] on cells
 * with state[n] <= 1; re-sorts.  A rotating gas takes [n][6] and scales
 * the rotational energies by the ratio of T_r; a clone takes the rotational
 * energy of the particle it copies.  DSMC_E_CAPACITY as for dig_couple. */
dsmc_status dig_feedback(dsmc_ctx ctx, const double* prim_old, const double* prim_new, const int32_t* state,
                         int64_t* np_after);

/* Batch contexts: enabled[n_cases] (nonzero: coupled) selects the cases
 * whose particles and local-accumulation flags dig_couple and dig_feedback
 * change; the others keep stepping as plain DSMC.  DSMC_E_INVALID on a
 * single-case context or a NULL array. */
dsmc_status dig_batch_enable(dsmc_ctx ctx, const int32_t* enabled);

/* Replace the sums of an accumulator (DSMC_SAMPLE_STEADY or
 * DSMC_SAMPLE_EWMA) by sums[n][13] (layout of dsmc_get_sums); restarts or
 * checkpoints the moving average.  For the moving average, counts[n] (may be
 * NULL to keep the current ones) are the per-cell numbers of samples taken,
 * which set its weights. */
dsmc_status dsmc_set_sums(dsmc_ctx ctx, int32_t which, const double* sums, const int32_t* counts);

/* The same for the rotational sums of a rotating gas: sums[n][4] (layout
 * of dsmc_get_rot_sums).  DSMC_E_INVALID for a monatomic gas. */
dsmc_status dsmc_set_rot_sums(dsmc_ctx ctx, int32_t which, const double* sums);

#ifdef __cplusplus
}
#endif
#endif /* DSMC_DIG_H */
