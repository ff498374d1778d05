/*
 * Internal definitions of the CPU oracle (test infrastructure only), shared
 * by its translation units.
 */
#ifndef DSMC_ORACLE_INTERNAL_H
#define DSMC_ORACLE_INTERNAL_H
#include "oracle.h"

#define KB 1.380649e-23
#define TWO_PI 6.283185307179586
#define SQRT_PI 1.7724538509055159
#define INV_SQRT2 0.7071067811865476
#define MAX_HOPS 1000
#define NMOM 13

enum { P_INIT = 1, P_WALL = 2, P_INJCOUNT = 3, P_NTCCOUNT = 4, P_PAIR = 5, P_SCATTER = 6,
       P_INITCOUNT = 9, P_INJECT = 10, P_INELASTIC_I = 11, P_INELASTIC_J = 12 };
#define NROT 4  /* rotational sums per cell: sum I_r, sum v_i I_r */

struct osim {
    /* species */
    double m, dref, omega, Tref, K, ex;
    double alpha;       /* VSS scattering exponent; 1 is VHS (isotropic) */
    int dr;             /* rotational degrees of freedom: 0 (monatomic) or 2 */
    double zr, pinel;   /* rotational collision number; inelastic probability */
    /* run */
    double FN, dt;
    uint32_t seed, case_id;
    int vel_fp32, n_ss, n_a, ewma_on;
    /* mesh */
    int nv, nt, nb, nf;
    double* xyz;
    int* tv;          /* [nt][4] reoriented */
    double* vol;      /* [nt] */
    int* tf_face;     /* [nt][4] face id */
    double* tf_s;     /* [nt][4] +1 if the face normal points out of this tet */
    int* tf_nbr;      /* [nt][4] neighbour tet, or -1-bface */
    int* tf_nlf;      /* [nt][4] neighbour's local face index */
    double* fn;       /* [nf][3] unnormalised face normal */
    double* fd;       /* [nf] plane offset */
    int* fvert;       /* [nf][3] sorted global vertex ids */
    int* bf_tet; int* bf_lf; int* bf_group; int* bf_partner; int* bf_face;
    double* bf_nin; double* bf_t1; double* bf_t2; double* bf_area;
    /* groups */
    int ng; int* g_kind; double* g_T; double* g_u; double* g_n; double* g_shift;
    /* per inflow face */
    double* in_mean; double* in_a; double* in_beta; double* in_sig; double* in_ut1; double* in_ut2;
    /* particles, kept in (cell, pid) order after the sort stage */
    int64_t np, cap;
    double* x; double* v; int* cell; uint32_t* pid;
    double* ir;         /* rotational energy (J) of each particle when dr > 0 */
    uint32_t next_pid, step;
    /* per cell */
    double* smax; int* ncand; int* nacc; int64_t* start;
    double* acc; int64_t n_steady;
    double* ewma; int* ewma_m; unsigned char* local_acc;
    double* inst;
    double* racc; double* rewma; double* rinst;  /* [nt][NROT] when dr > 0 */
    /* counters */
    int64_t hops, walls, injected, removed, lost;
    /* surface sampling: [nb][5] sums of (v_in - v_out), (|v_in|^2 - |v_out|^2)/2
     * and hits over the sampled steps while on; window start and end steps */
    double* surf;
    double* rsurf; /* [nb] rotational energy given to each face (rotating gas) */
    int surf_on;
    int64_t surf_from, surf_to;
    /* reference state of the run (initial fill) and DIG coupling state */
    double ref_n, ref_T, ref_u[3];
    double* cen;    /* [nt][3] cell centroids */
    double* fcen;   /* [nt][4][3] face centroids */
    double* fnu;    /* [nt][4][3] outward unit normals */
    double* farea;  /* [nt][4] face areas */
    double* lsq;    /* [nt][9] inverse least-squares matrix (zero when singular) */
    double* mprev;  /* [nt][5] rho, u(3), T (monatomic) or [nt][6] rho, u(3), T_t, T_r
                       of the last macroscopic solution */
    double a_heat[4]; /* heat-flux relaxation coefficients A_tt, A_tr, A_rt, A_rr */
    int dig_ready;
};


/* shared helpers */
void o_draw(const osim* s, uint32_t subject, uint32_t step, uint32_t purpose, uint64_t block, uint32_t out[4]);
double o_u01(uint32_t a, uint32_t b);
uint32_t o_pick(uint32_t r, uint32_t n);
double o_to_store(const osim* s, double x);
void o_sort(osim* s);
void o_reserve(osim* s, int64_t need);
void o_set_err(const char* m);

#endif
