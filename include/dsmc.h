/*
 * dsmc.h — C ABI of the MI355X (gfx950) DSMC particle loop.
 *
 * The library advances a direct simulation Monte Carlo gas on an
 * unstructured tetrahedral mesh, one time step at a time, following the
 * step splitting of the paper's section 2.1 (particles are moved, then
 * pairs are selected and collided within each cell) and the cell sampling
 * of eq. (dsmc_temperatures), with the moving average of
 * eq. (exponential_average_moments_ch3) and the steady average of
 * eq. (steady_average_moments_ch3) from section 3.1.  Particle state is the
 * (x, v; N_eff) of eq. (dsmc_particle_state) for a monatomic gas.
 *
 * Conventions
 *  - Every call returns a dsmc_status: 0 on success, negative on error.
 *    No C++ exception crosses this boundary.  dsmc_last_error() gives a
 *    message for the last failing call on a context.
 *  - Units are SI (m, s, kg, K).  Host pointers are plain C arrays in the
 *    row-major layouts stated per argument.
 *  - Input descriptors are borrowed for the duration of the call only: the
 *    library copies what it needs.  Output buffers belong to the caller.
 *  - A context owns all device memory it allocates (through the caller's
 *    allocator when one is given) and releases it in dsmc_destroy().
 *  - Work is enqueued asynchronously on the context's HIP stream.  Calls
 *    that return host data synchronise that stream.  Device-side faults
 *    (capacity overflow) are latched and reported by the next
 *    synchronising call (dsmc_stats, dsmc_get_state, dsmc_sample,
 *    dsmc_sync).  After DSMC_E_CAPACITY or DSMC_E_DEVICE only
 *    dsmc_destroy() is valid.
 *  - One context per host thread; distinct contexts are independent.
 */
#ifndef DSMC_H
#define DSMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dsmc_ctx_s* dsmc_ctx;

typedef enum {
    DSMC_OK = 0,
    DSMC_E_INVALID = -1,       /* bad argument or call order */
    DSMC_E_MESH = -2,          /* degenerate tet, unmatched boundary triangle, non-manifold face */
    DSMC_E_OOM = -3,           /* device allocation failed */
    DSMC_E_DEVICE = -4,        /* HIP runtime error */
    DSMC_E_CAPACITY = -5       /* particle store would overflow */
    /* Particles lost to the hop limit are counted (dsmc_counters.lost), and
     * a coupling solve that stops short of its tolerance is reported
     * (dig_report.converged); neither is an error status. */
} dsmc_status;

/* Tetrahedral mesh (paper section 4.1: cells and faces of the local mesh).
 * xyz      [n_vertices][3]  vertex coordinates (m)
 * tet_vtx  [n_tets][4]      vertex indices, any orientation
 * bface_vtx   [n_bfaces][3] boundary triangles (each must match exactly one
 *                           exterior tet face)
 * bface_group [n_bfaces]    index into the boundary table of dsmc_init
 * bface_partner [n_bfaces]  periodic partner triangle, or -1; may be NULL */
typedef struct {
    int32_t n_vertices;
    const double* xyz;
    int32_t n_tets;
    const int32_t* tet_vtx;
    int32_t n_bfaces;
    const int32_t* bface_vtx;
    const int32_t* bface_group;
    const int32_t* bface_partner;
} dsmc_mesh_desc;

/* Variable hard / soft sphere species (paper section 5: VHS collision
 * model, power-law viscosity index omega; section 2.1: VSS).  The total
 * cross-section is the VHS one of d_ref for every alpha.  alpha = 1 scatters
 * isotropically (VHS); otherwise the deflection chi from the pre-collision
 * relative velocity has cos(chi) = 2 R^(1/alpha) - 1 with R uniform and a
 * uniform azimuth (VSS, Bird 1994), and the viscosity the continuum side
 * uses is the VHS value times (alpha+1)(alpha+2)/(6 alpha).  alpha must be
 * positive (DSMC_E_INVALID otherwise).
 * Rotation (section 2.1, eq. dsmc_particle_state): with dof_rot = 2 every
 * particle carries a rotational energy I_r, drawn from the equilibrium
 * distribution (exponential, mean k T) at the fill (T0), at diffuse walls
 * (T of the wall) and at inflow faces (T of the freestream); after an
 * accepted collision each partner in turn, with probability
 * alpha (5 - 2 omega)(7 - 2 omega) / (5 (alpha + 1)(alpha + 2) z_rot)
 * (eq. inelastic_probability), pools its I_r with the relative
 * translational energy E_t = m c_r^2 / 4 and keeps the share
 * E_t = E_c R^(1 / (5/2 - omega)) for translation (Borgnakke-Larsen for two
 * rotational degrees of freedom), the relative velocity keeping its
 * direction.  dof_rot = 0 (monatomic) leaves all of this out.  Other values,
 * or z_rot <= 0 with dof_rot = 2, are DSMC_E_INVALID.  A rotating gas runs
 * the parked-wall move schedules (4-7, 12-17), the LDS-ranked collide
 * schedules (1-4) and the scatter, gather or deferred sort (0, 1, 3); the
 * coupling step (dig.h) solves the polyatomic synthetic equations for it,
 * with the heat conductivities from heat_relax = (A_tt, A_tr, A_rt, A_rr),
 * the relaxation matrix of eq. thermal_conductivity_matrix (all zero:
 * nitrogen's 0.786, -0.201, -0.059, 0.842; a singular matrix is
 * DSMC_E_INVALID); surface sampling adds the rotational energy exchanged
 * at diffuse walls (dsmc_get_surface_rot). */
typedef struct {
    double mass;     /* kg */
    double d_ref;    /* reference diameter, m */
    double omega;    /* viscosity index */
    double T_ref;    /* reference temperature of d_ref, K */
    double alpha;    /* VSS scattering exponent; 1 = VHS */
    int32_t dof_rot; /* rotational degrees of freedom: 0 or 2 */
    double z_rot;    /* rotational collision number (dof_rot = 2) */
    double heat_relax[4]; /* heat-flux relaxation matrix A (dof_rot = 2), row-major */
} dsmc_species_desc;

typedef enum {
    DSMC_BC_DIFFUSE = 0,   /* full accommodation at (T, u) (paper section 5) */
    DSMC_BC_SPECULAR = 1,  /* mirror reflection */
    DSMC_BC_INFLOW = 2,    /* freestream (n, T, u) enters; leaving particles are removed */
    DSMC_BC_OUTFLOW = 3,   /* vacuum: leaving particles are removed */
    DSMC_BC_PERIODIC = 4   /* translate by shift onto the partner triangle */
} dsmc_bc_kind;

typedef struct {
    int32_t kind;     /* dsmc_bc_kind */
    double T;         /* wall or freestream temperature, K */
    double u[3];      /* wall or freestream velocity, m/s */
    double n;         /* freestream number density (INFLOW), m^-3 */
    double shift[3];  /* translation onto the partner face (PERIODIC), m */
} dsmc_boundary_desc;

/* Optional device allocator; alloc returns NULL on failure. */
typedef struct {
    void* (*alloc)(size_t bytes, void* user);
    void (*free)(void* ptr, void* user);
    void* user;
} dsmc_allocator;

typedef struct {
    double n0;            /* initial number density, m^-3 */
    double T0;            /* initial temperature, K */
    double u0[3];         /* initial bulk velocity, m/s */
    double F_N;           /* real molecules per simulation particle (N_eff) */
    double dt;            /* time step, s */
    uint64_t seed;        /* low 32 bits key the generator */
    uint32_t case_id;     /* second key word of the generator */
    int32_t vel_fp64;     /* 1: store velocities in FP64; 0: FP32 storage */
    int32_t n_ss;         /* steps discarded before the steady average */
    int32_t n_a;          /* effective samples of the moving average */
    int32_t ewma_on;      /* 1: keep the moving-average accumulator */
    int32_t fill;         /* 1: equilibrium fill at (n0, T0, u0); 0: empty */
    int64_t capacity;     /* particle store size; 0 chooses 2x the count at n0 */
    void* hip_stream;     /* hipStream_t to enqueue on; NULL = null stream */
    const dsmc_allocator* allocator; /* NULL = hipMalloc / hipFree */
} dsmc_run_desc;

/* Build the device mesh image, boundary tables and particle store, and
 * (with run->fill) perform the initial equilibrium fill.  On success *out
 * is a new context; on failure *out is NULL and the status says why. */
dsmc_status dsmc_init(dsmc_ctx* out, const dsmc_mesh_desc* mesh, const dsmc_species_desc* species,
                      int32_t n_bc, const dsmc_boundary_desc* bcs, const dsmc_run_desc* run);

/* Advance n_steps time steps: move (with boundary interactions) ->
 * freestream injection -> counting sort by cell -> NTC collisions ->
 * sampling.  Asynchronous. */
dsmc_status dsmc_step(dsmc_ctx ctx, int32_t n_steps);

/* One step restricted to the stages in mask (1 move, 2 inject, 4 sort,
 * 8 collide, 16 sample); for stage-level testing.  A mask with move or
 * injection must include the sort (DSMC_E_INVALID otherwise). */
dsmc_status dsmc_step_stages(dsmc_ctx ctx, int32_t mask);

/* Accumulators: STEADY sums every step after n_ss, EWMA is the moving
 * average, INSTANT holds the sums of the last sampled step alone (kept only
 * while switched on by dsmc_instant_sampling; zero before). */
enum { DSMC_SAMPLE_STEADY = 0, DSMC_SAMPLE_EWMA = 1, DSMC_SAMPLE_INSTANT = 2 };

/* on = 1: from the next step on, every sampled step also stores its own
 * moment sums (DSMC_SAMPLE_INSTANT; 104 bytes per cell and step); 0 stops
 * (the last sums are kept).  Synchronises. */
dsmc_status dsmc_instant_sampling(dsmc_ctx ctx, int32_t on);

/* Cell fields from an accumulator (eq. dsmc_temperatures over the sampled
 * steps): out[n_tets][15] = n, rho, u(3), T, sigma(xx,yy,zz,xy,xz,yz),
 * q(3).  Cells without samples give NaN.  out is a host pointer unless
 * out_on_device is 1.  Synchronises. */
dsmc_status dsmc_sample(dsmc_ctx ctx, int32_t which, double* out, int32_t out_on_device);

/* Raw moment sums out[n_tets][13] = S0, S1(3), S2(xx,yy,zz,xy,xz,yz), S3(3)
 * of an accumulator, and the number of steps summed (steady; 1 for
 * INSTANT) into *n_samples.  Synchronises. */
dsmc_status dsmc_get_sums(dsmc_ctx ctx, int32_t which, double* out, int64_t* n_samples);

/* Rotational sums of a rotating gas: out[n_tets][4] = sum of I_r and of
 * v_i I_r (i = x, y, z) of an accumulator (layout and sample count of
 * dsmc_get_sums); dsmc_rot_sample gives the rotational temperature and heat
 * flux of eq. (dsmc_temperatures) out[n_tets][4] = T_r = 2 <I_r> / (d_r k),
 * q_r,i = (N_eff / V) sum (v_i - u_i) I_r per sampled step (NaN without
 * samples).  Host arrays; synchronise; DSMC_E_INVALID for a monatomic gas. */
dsmc_status dsmc_get_rot_sums(dsmc_ctx ctx, int32_t which, double* out, int64_t* n_samples);
dsmc_status dsmc_rot_sample(dsmc_ctx ctx, int32_t which, double* out);

/* Mixed-element meshes (section 5.4: tetrahedral, pyramid ("pentahedral"),
 * triangular-prism and hexahedral cells).  The step works on tetrahedra:
 * dsmc_mesh_decompose turns a mixed mesh into a conforming tetrahedral one
 * for dsmc_init, and dsmc_sample_cells gives the fields of the original
 * cells from the sums of their tetrahedra.
 *
 * cell_nv[c] = 4, 5, 6 or 8 vertices, listed in cell_vtx one cell after the
 * other in these local orders: tetrahedron v0..v3; pyramid base v0 v1 v2 v3
 * (cyclic) and apex v4; prism triangles v0 v1 v2 and v3 v4 v5 with v3 over
 * v0, v4 over v1, v5 over v2; hexahedron v0 v1 v2 v3 (cyclic) and v4..v7
 * over them.  Boundary faces: bface_nv[b] = 3 or 4 vertices (cyclic) in
 * bface_vtx, a group each, periodic partners (bface_partner, may be NULL)
 * only between triangles.
 *
 * Decomposition: a quadrilateral face (a, b, c, d) is split into (a, b, c),
 * (a, c, d) when a or c has the smallest vertex index of the four, else
 * into (a, b, d), (b, c, d), so neighbours split a shared face alike; a
 * pyramid becomes its apex over its two base triangles; a prism or a
 * hexahedron gets a new vertex at the mean of its vertices (coordinate-wise
 * sum in local order, divided by the vertex count; new vertices numbered
 * after the input ones in cell order) and one tetrahedron per face
 * triangle with it: the two triangles first, then the quadrilaterals
 * (v0 v1 v4 v3), (v1 v2 v5 v4), (v2 v0 v3 v5) of a prism, and (v0 v1 v2
 * v3), (v4 v5 v6 v7), (v0 v1 v5 v4), (v1 v2 v6 v5), (v2 v3 v7 v6), (v3 v0
 * v4 v7) of a hexahedron.  Tetrahedra come in cell order (tet_cell: the
 * cell of each), boundary triangles in face order (bface_parent: the face
 * of each).  Cells must be convex (star-shaped from their vertex mean);
 * dsmc_init checks the result as any tetrahedral mesh.
 *
 * Call with every output array NULL to get the counts, then with arrays of
 * at least those sizes (n_vertices, n_tets, n_bfaces set to their
 * capacities).  DSMC_E_MESH on a bad cell or face (dsmc_mesh_error says
 * which); DSMC_E_INVALID for NULL arguments or short arrays.  Host only. */
typedef struct {
    int32_t n_vertices;
    const double* xyz;           /* [n_vertices][3] */
    int32_t n_cells;
    const int32_t* cell_nv;      /* [n_cells] */
    const int32_t* cell_vtx;     /* sum of cell_nv entries */
    int32_t n_bfaces;
    const int32_t* bface_nv;     /* [n_bfaces] */
    const int32_t* bface_vtx;    /* sum of bface_nv entries */
    const int32_t* bface_group;  /* [n_bfaces] */
    const int32_t* bface_partner; /* [n_bfaces] or NULL */
} dsmc_mixed_mesh_desc;

typedef struct {
    int32_t n_vertices, n_tets, n_bfaces; /* capacities in, counts out */
    double* xyz;            /* [n_vertices][3]: the input vertices, then the new ones */
    int32_t* tet_vtx;       /* [n_tets][4] */
    int32_t* tet_cell;      /* [n_tets] */
    int32_t* bface_vtx;     /* [n_bfaces][3] */
    int32_t* bface_group;   /* [n_bfaces] */
    int32_t* bface_partner; /* [n_bfaces], -1 where none */
    int32_t* bface_parent;  /* [n_bfaces] */
} dsmc_tet_mesh_out;

dsmc_status dsmc_mesh_decompose(const dsmc_mixed_mesh_desc* in, dsmc_tet_mesh_out* out);
const char* dsmc_mesh_error(void);

/* Fields of the cells of a mixed mesh: the moment sums of each cell's
 * tetrahedra (tet_cell[n_tets] from dsmc_mesh_decompose, caller's tet
 * numbering) added in ascending tetrahedron order, over the sum of their
 * volumes, through the formulas of dsmc_sample: out[n_cells][15] (NaN for
 * a cell without samples).  Host arrays; synchronises.  DSMC_E_INVALID for
 * a cell index out of range or a batch context. */
dsmc_status dsmc_sample_cells(dsmc_ctx ctx, int32_t which, int32_t n_cells, const int32_t* tet_cell, double* out);

/* Surface sampling (the wall pressure, shear stress and heat flux the
 * paper compares on the sphere, section 5): every interaction of a particle
 * with a diffuse or specular boundary face on a step after n_ss adds, for
 * that face, the velocity change v_in - v_out, the kinetic-energy change
 * (|v_in|^2 - |v_out|^2) / 2 (per unit mass) and one hit.  on = 1 clears
 * the sums and starts sampling, 0 stops it (sums kept); off by default.
 * Synchronises.  The sums are added with device atomics, so their rounding
 * depends on the order of the hits (the hit counts are exact). */
dsmc_status dsmc_surface_sampling(dsmc_ctx ctx, int32_t on);

/* Surface sums and fields of the boundary faces (input order) over the
 * *n_steps sampled steps (steps after n_ss inside the on window):
 * sums[n_bfaces][5] = sum of v_in - v_out (3), of the energy change, hits;
 * fields[n_bfaces][6] = number flux F_N hits / (A t), pressure
 * m F_N (S.n) / (A t), shear stress m F_N (S - (S.n) n) / (A t) (3),
 * heat flux m F_N E / (A t), with S the velocity-change sum, E the energy
 * sum, n the unit normal out of the gas, A the face area, t = n_steps dt
 * (F_N and dt of the face's case in a batch; zeros without sampled steps).
 * Either pointer may be NULL.  Synchronises. */
dsmc_status dsmc_get_surface(dsmc_ctx ctx, double* sums, double* fields, int64_t* n_steps);

/* Rotational part of the surface sums of a rotating gas (the rotational
 * heat flux the paper compares on the sphere, section 5): every diffuse
 * re-emission adds to its face the incident molecule's rotational energy
 * minus the re-emitted one's (J; specular faces keep it).  sums[n_bfaces] =
 * that sum, qr[n_bfaces] = the rotational heat flux into the wall F_N sum /
 * (A t) (W/m^2), over the *n_steps sampled steps of dsmc_get_surface; the
 * sums are added with device atomics.  Either pointer may be NULL.
 * DSMC_E_INVALID for a monatomic gas.  Synchronises. */
dsmc_status dsmc_get_surface_rot(dsmc_ctx ctx, double* sums, double* qr, int64_t* n_steps);

/* Particle state.  dsmc_get_state fills n_particles, step and next_pid; the
 * arrays (host, may be NULL) receive the particles in (cell, pid) order:
 * x[n][3], v[n][3] (FP64), cell[n], pid[n], ir[n] the rotational energies
 * (J; untouched for a monatomic gas), and smax[n_tets] the per-cell
 * (sigma_T c_r)_max.  dsmc_set_state replaces the state (particles in any
 * order, ir in the same order or NULL for zero rotational energy); smax may
 * be NULL to keep the current values. */
typedef struct {
    int64_t n_particles;
    double* x;
    double* v;
    int32_t* cell;
    uint32_t* pid;
    double* smax;
    uint32_t step;
    uint32_t next_pid;
    double* ir;
} dsmc_state;

dsmc_status dsmc_get_state(dsmc_ctx ctx, dsmc_state* state);
dsmc_status dsmc_set_state(dsmc_ctx ctx, const dsmc_state* state);

/* Per-cell candidate and accepted pair counts of the last collide stage
 * (host arrays [n_tets]).  Synchronises. */
dsmc_status dsmc_get_pair_counts(dsmc_ctx ctx, int32_t* ncand, int32_t* nacc);

/* Cumulative counters.  Synchronises and reports latched device errors. */
typedef struct {
    int64_t n_particles;
    int64_t hops;        /* face events (crossings and boundary interactions) */
    int64_t wall_hits;   /* diffuse and specular reflections */
    int64_t injected;
    int64_t removed;     /* left through inflow/outflow faces */
    int64_t lost;        /* exceeded the hop limit and were deleted */
    uint32_t step;
} dsmc_counters;
dsmc_status dsmc_stats(dsmc_ctx ctx, dsmc_counters* out);

/* Wait for all work enqueued on the context; reports latched errors. */
dsmc_status dsmc_sync(dsmc_ctx ctx);

/* Per-cell local-accumulation flags (host array [n_tets] of 0/1): flagged
 * cells average their moving-average accumulator cumulatively
 * (section 3.2). */
dsmc_status dsmc_set_local_acc(dsmc_ctx ctx, const uint8_t* flags);

/* Per-kernel timing of the step's kernels with HIP events on the context's
 * stream.  dsmc_profile(ctx, 1) starts recording (and resets), 0 stops.
 * dsmc_profile_read writes for each kernel slot: total milliseconds and
 * launch count; names via dsmc_profile_name.  Returns the slot count. */
dsmc_status dsmc_profile(dsmc_ctx ctx, int32_t enable);
int32_t dsmc_profile_read(dsmc_ctx ctx, double* total_ms, int64_t* launches, int32_t max_slots);
const char* dsmc_profile_name(int32_t slot);

/* Philox4x32-10 evaluated on the device for n counters ctr[n][4] under
 * key[2]; out[n][4] (host arrays).  Known-answer check of the generator. */
dsmc_status dsmc_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t n);

/* Plain device copy of `bytes` between two device buffers on the context
 * stream (HBM bandwidth calibration of the traffic counters). */
dsmc_status dsmc_device_copy(dsmc_ctx ctx, void* dst, const void* src, size_t bytes);

/* Scattered reads for calibrating the vector L1's line-access rate (the
 * limit of the move kernel's geometry gathers), on the context stream:
 * `blocks` workgroups of 256 lanes; per iteration each group of `share`
 * consecutive lanes loads 16 bytes from the start of one pseudo-randomly
 * chosen 128-byte line among the first 2^k lines of `table` (2^k the
 * largest power of two with 128 * 2^k <= bytes), so one wave instruction
 * touches 64 / share lines; `iters` iterations per lane.  table: device
 * memory, at least 128 bytes, 16-byte aligned, read only.  sink: 4 bytes of
 * device memory, written only if the sum of the loaded words equals a fixed
 * constant.  DSMC_E_INVALID for null pointers, a short or misaligned table,
 * share not a power of two in [1, 64], iters outside [1, 4096] or blocks
 * outside [1, 65536] (at most about 7e10 loads, a fraction of a second). */
dsmc_status dsmc_device_line_reads(dsmc_ctx ctx, const void* table, size_t bytes, void* sink, int share, int iters,
                                   int blocks);

/* ---- batches, graphs and kernel schedules ------------------------------ */

/* Many independent cases in one context (a batch): the cases' meshes are
 * joined into one mesh whose cells never touch across cases, so every
 * kernel launch of a step advances all cases at once.  meshes[n_cases],
 * n_bc[n_cases] and runs[n_cases] are per case; bcs holds the boundary
 * tables of all cases one after the other (case k's groups are numbered
 * from 0 in its own mesh).  Per case: n0, T0, u0, F_N, dt, seed and case_id
 * (the generator key (seed, case_id), cell subjects and particle ids are
 * case-local, so each case evolves as it would in a context of its own).
 * Batch-wide, from runs[0]: vel_fp64, n_ss, n_a, ewma_on, fill, capacity,
 * hip_stream, allocator.  Freestream inflow is not available for a batch
 * (DSMC_E_INVALID); the coupling step is (dig.h: dig_couple over the cases
 * that dig_batch_enable selects).  Every other call works on the joined
 * mesh: cells are numbered case after case in the callers' order
 * (dsmc_batch_cases gives the first cell of each case). */
dsmc_status dsmc_batch_init(dsmc_ctx* out, int32_t n_cases, const dsmc_mesh_desc* meshes,
                            const dsmc_species_desc* species, const int32_t* n_bc,
                            const dsmc_boundary_desc* bcs, const dsmc_run_desc* runs);
/* *n_cases (1 for a plain context) and cell_begin[n_cases + 1]: case k owns
 * cells cell_begin[k] .. cell_begin[k+1]-1 (cell_begin may be NULL). */
dsmc_status dsmc_batch_cases(dsmc_ctx ctx, int32_t* n_cases, int32_t* cell_begin);

/* Advance n_steps full steps through a captured HIP graph: two steps are
 * recorded once (per particle-buffer parity and kernel schedule) and
 * replayed; an odd remainder runs as an ordinary step.  With freestream
 * inflow the kernel grids cover the whole particle store; without it they
 * cover the particle count at capture time (a step cannot add particles),
 * and a replay that finds more particles than that (after feedback clones)
 * captures again.  The kernels bound themselves by the device counts.
 * Needs a non-null hip_stream.  Results equal dsmc_step's. */
dsmc_status dsmc_graph_step(dsmc_ctx ctx, int32_t n_steps);

/* Kernel schedule: move 0 lane, 1 lane (6 waves/SIMD), 2 lane (8),
 * 3 batched, 4/5/6/7 parked-wall at 6/8/4/5 waves/SIMD, 8/9 refill,
 * 10/11 pooled, 15 (default) / 16 parked-wall at 6 / 8 waves/SIMD testing
 * only the three faces other than the entry face after the first test,
 * 12/13/14 as 15 and also parking particles still in flight after 4/5/6
 * exit tests, 17 persistent: the work of 15 done by a fixed grid (as many
 * workgroups as the device holds at once) pulling tiles of 256 particles
 * from a device work queue dealt out in one contiguous slice per XCD
 * (a workgroup drains its XCD's slice, then takes tiles from the others);
 * collide 0 LDS-staged
 * velocities, 1/2 LDS-ranked at 4/8 waves/SIMD (chunks up to 4096
 * particles in LDS), 3/4 LDS-ranked with chunks up to 3072/2048 particles
 * (more workgroups per CU); sort 0 scatter, 1 gather, 2 gather done by
 * the collide kernel chunk by chunk (collide 1-4; with collide 0 it acts as
 * 1).  The autotuner's sort_ms includes the collide kernel.
 * Every schedule gives the same results.  A batch accepts only move 0-2
 * and 4-7, 12-17. */
typedef struct {
    int32_t move, collide, sort;
    double move_ms, collide_ms, sort_ms;  /* per step, filled by dsmc_autotune */
} dsmc_tuning;
dsmc_status dsmc_get_tuning(dsmc_ctx ctx, dsmc_tuning* t);
dsmc_status dsmc_set_tuning(dsmc_ctx ctx, const dsmc_tuning* t);
/* Time each move, collide and sort schedule over trial_steps real steps
 * (after one warm-up step each) on the current workload and keep the
 * fastest; the simulation advances by those steps. */
dsmc_status dsmc_autotune(dsmc_ctx ctx, int32_t trial_steps, dsmc_tuning* chosen);

const char* dsmc_last_error(dsmc_ctx ctx);
void dsmc_destroy(dsmc_ctx ctx);

#ifdef __cplusplus
}
#endif
#endif /* DSMC_H */
