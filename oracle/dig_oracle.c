/*
 * Plain CPU oracle of the DIG coupling step (test infrastructure only).
 *
 * Follows the paper's section 3 and Algorithm 1: after a window of DSMC
 * steps, the moving-average sums give the sampled low-order state M^{k+1/2}
 * (eq. sampled_macro_state_ch3) and the sampled stress and heat flux; the
 * higher-order terms are their difference from the NSF relations evaluated
 * with the same state and its gradients (eq. nsf_heat_flux,
 * eq. hot_extraction_ch3); cells whose local Knudsen number
 * (eq. cell_kn_stability) exceeds the threshold (criterion) are rebuilt from
 * admissible face neighbours with equal weights over several passes
 * (section 3.2); the macroscopic equations (eq. macro) are solved
 * towards steady state with the HoT frozen (eq. hot_used_in_macro_solver_ch3)
 * until the residual falls below eps_m or n_m iterations; the particles are
 * then adjusted to the new state M^{k+1}; in a closed domain the density of
 * M^{k+1} is first scaled so that its total mass equals the particles'.
 *
 * The finite-volume discretisation and the feedback map are not given in the
 * paper (they are delegated to its references); the readings implemented
 * here are: cell-centred finite volumes with
 * least-squares gradients, linear face reconstruction, a central flux with
 * low-Mach-scaled scalar dissipation, NSF + frozen HoT viscous fluxes (the
 * HoT carried per face so that the sampled state is consistent) and
 * local pseudo-time stepping; feedback by velocity shift-and-scale and
 * clone/delete to the density ratio.
 *
 * A gas with rotational degrees of freedom (d_r = 2) takes the polyatomic
 * form of eq. (macro): the primitives are rho, u, T_t, T_r; the total
 * energy includes e_r = (d_r/2) R T_r; a fifth equation carries rho e_r
 * with the rotational heat flux q_r and the relaxation source
 * (d_r/2) rho R (T - T_r) / (Z_r tau), T = (3 T_t + d_r T_r)/(3 + d_r),
 * tau = mu/p_t; the heat conductivities come from the relaxation matrix
 * (eq. thermal_conductivity_matrix) with q_t = -kappa_t grad T_t and
 * q_r = -kappa_r grad T_r (eq. nsf_heat_flux); the sampled state takes T_r
 * and q_r of eq. (dsmc_temperatures), the HoT q_r too; the feedback scales
 * the rotational energies by T_r^{k+1}/T_r^{k+1/2}.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle_internal.h"

#define GAMMA (5.0 / 3.0)
#define M_CUT 0.05
#define P_RECAL 7
#define NVX 6  /* primitive variables at most: rho, u(3), T_t, T_r */
#define NHX 12 /* HoT at most: sigma(6), q_t(3), q_r(3) */
#define GS (3 * NVX) /* gradient stride per cell */

/* primitive and HoT counts: 5 and 9 for a monatomic gas, 6 and 12 with rotation */
static int nv_of(const osim* s) { return s->dr ? 6 : 5; }
static int nh_of(const osim* s) { return s->dr ? 12 : 9; }

enum { L_INTERIOR = 0, L_PERIODIC = 1, L_WALL = 2, L_SPECULAR = 3, L_INFLOW = 4, L_OUTFLOW = 5 };

/* Reference viscosity of the VHS/VSS molecule (Bird 1994, the model that
 * section 2.1 cites): the hard-sphere-like Chapman-Enskog value times
 * (alpha+1)(alpha+2)/(6 alpha), which is exactly 1 for VHS scattering. */
static double mu_ref_of(const osim* s) {
    double w = s->omega, a = s->alpha;
    double vss = ((a + 1.0) * (a + 2.0)) / (6.0 * a);
    return 15.0 * sqrt(M_PI * s->m * KB * s->Tref) / (2.0 * M_PI * s->dref * s->dref * (5.0 - 2.0 * w) * (7.0 - 2.0 * w)) *
           vss;
}
static double mu_of(const osim* s, double T) { return mu_ref_of(s) * pow(T / s->Tref, s->omega); }
double oracle_viscosity(const osim* s, double T) { return mu_of(s, T); }
static double kappa_of(const osim* s, double mu) { return 15.0 * KB * mu / (4.0 * s->m); }

/* Heat conductivities of a rotating gas (eq. thermal_conductivity_matrix):
 * (kappa_t, kappa_r) = (mu R / 2) A^{-1} (5, d_r), R = k/m. */
static void kappas_of(const osim* s, double mu, double* kt, double* kr) {
    const double* A = s->a_heat;
    double det = A[0] * A[3] - A[1] * A[2];
    double f = (mu * (KB / s->m)) / 2.0;
    *kt = f * ((A[3] * 5.0 - A[1] * (double)s->dr) / det);
    *kr = f * ((A[0] * (double)s->dr - A[2] * 5.0) / det);
}

int oracle_set_heat_relaxation(osim* s, const double* a) {
    double det = a[0] * a[3] - a[1] * a[2];
    if (!(isfinite(det) && det != 0.0)) return -1;
    for (int k = 0; k < 4; ++k) s->a_heat[k] = a[k];
    return 0;
}

/* ratio of specific heats of the frozen gas, (5 + d_r)/(3 + d_r) */
static double gamma_of(const osim* s) { return s->dr ? (5.0 + s->dr) / (3.0 + s->dr) : GAMMA; }

void oracle_set_reference(osim* s, double n0, double T0, const double* u0) {
    s->ref_n = n0;
    s->ref_T = T0;
    for (int i = 0; i < 3; ++i) s->ref_u[i] = u0 ? u0[i] : 0.0;
    if (s->mprev)
        for (int c = 0; c < s->nt; ++c) {
            double* m = s->mprev + nv_of(s) * (size_t)c;
            m[0] = s->m * n0; m[1] = s->ref_u[0]; m[2] = s->ref_u[1]; m[3] = s->ref_u[2]; m[4] = T0;
            if (s->dr) m[5] = T0;
        }
}

/* What lies behind local face f of cell c: kind, neighbour cell, and the
 * vector from c's centroid to the neighbour centroid (periodic: shifted into
 * c's frame) or to the face centroid (boundaries). */
static int face_link(const osim* s, int c, int f, int* nb, double dx[3]) {
    int k = 4 * c + f;
    int code = s->tf_nbr[k];
    const double* xc = s->cen + 3 * (size_t)c;
    if (code >= 0) {
        *nb = code;
        for (int i = 0; i < 3; ++i) dx[i] = s->cen[3 * (size_t)code + i] - xc[i];
        return L_INTERIOR;
    }
    int bf = -1 - code;
    int g = s->bf_group[bf];
    *nb = -1;
    switch (s->g_kind[g]) {
    case O_BC_PERIODIC: {
        int pt = s->bf_tet[s->bf_partner[bf]];
        *nb = pt;
        for (int i = 0; i < 3; ++i) dx[i] = (s->cen[3 * (size_t)pt + i] - s->g_shift[3 * g + i]) - xc[i];
        return L_PERIODIC;
    }
    case O_BC_DIFFUSE:
        for (int i = 0; i < 3; ++i) dx[i] = s->fcen[12 * (size_t)c + 3 * f + i] - xc[i];
        return L_WALL;
    case O_BC_SPECULAR:
        for (int i = 0; i < 3; ++i) dx[i] = s->fcen[12 * (size_t)c + 3 * f + i] - xc[i];
        return L_SPECULAR;
    case O_BC_INFLOW:
        for (int i = 0; i < 3; ++i) dx[i] = s->fcen[12 * (size_t)c + 3 * f + i] - xc[i];
        return L_INFLOW;
    default:
        for (int i = 0; i < 3; ++i) dx[i] = s->fcen[12 * (size_t)c + 3 * f + i] - xc[i];
        return L_OUTFLOW;
    }
}

static int face_group(const osim* s, int c, int f) { return s->bf_group[-1 - s->tf_nbr[4 * c + f]]; }

static void geometry(osim* s) {
    if (s->dig_ready) return;
    int nt = s->nt;
    s->cen = (double*)malloc(sizeof(double) * 3 * (size_t)nt);
    s->fcen = (double*)malloc(sizeof(double) * 12 * (size_t)nt);
    s->fnu = (double*)malloc(sizeof(double) * 12 * (size_t)nt);
    s->farea = (double*)malloc(sizeof(double) * 4 * (size_t)nt);
    s->lsq = (double*)malloc(sizeof(double) * 9 * (size_t)nt);
    s->mprev = (double*)malloc(sizeof(double) * NVX * (size_t)nt);
    for (int c = 0; c < nt; ++c) {
        const int* q = s->tv + 4 * c;
        for (int i = 0; i < 3; ++i) {
            double a = s->xyz[3 * q[0] + i], b = s->xyz[3 * q[1] + i];
            double d = s->xyz[3 * q[2] + i], e = s->xyz[3 * q[3] + i];
            s->cen[3 * (size_t)c + i] = (((a + b) + d) + e) * 0.25;
        }
        for (int f = 0; f < 4; ++f) {
            int v[3], j = 0;
            for (int k = 0; k < 4; ++k)
                if (k != f) v[j++] = q[k];
            for (int i = 0; i < 3; ++i)
                s->fcen[12 * (size_t)c + 3 * f + i] =
                    ((s->xyz[3 * v[0] + i] + s->xyz[3 * v[1] + i]) + s->xyz[3 * v[2] + i]) / 3.0;
            const double* n = s->fn + 3 * s->tf_face[4 * c + f];
            double sg = s->tf_s[4 * c + f];
            double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
            for (int i = 0; i < 3; ++i) s->fnu[12 * (size_t)c + 3 * f + i] = (sg * n[i]) / nn;
            s->farea[4 * (size_t)c + f] = 0.5 * nn;
        }
    }
    for (int c = 0; c < nt; ++c) {
        double A[3][3] = {{0}};
        for (int f = 0; f < 4; ++f) {
            int nb;
            double dx[3];
            int kind = face_link(s, c, f, &nb, dx);
            if (kind != L_INTERIOR && kind != L_PERIODIC && kind != L_WALL) continue;
            double w = 1.0 / (dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) A[i][j] += w * dx[i] * dx[j];
        }
        double* L = s->lsq + 9 * (size_t)c;
        double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                     A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                     A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
        double tr = (A[0][0] + A[1][1] + A[2][2]) / 3.0;
        if (!(fabs(det) > 1e-10 * tr * tr * tr)) {
            for (int k = 0; k < 9; ++k) L[k] = 0.0;
            continue;
        }
        L[0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / det;
        L[1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
        L[2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
        L[3] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / det;
        L[4] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
        L[5] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
        L[6] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / det;
        L[7] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
        L[8] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
    }
    s->dig_ready = 1;
    oracle_set_reference(s, s->ref_n, s->ref_T, s->ref_u);
}

/* Least-squares gradients of all primitives: g[nt][NVX][3]. At a diffuse
 * wall the far value is the wall velocity and temperature (both
 * temperatures of a rotating gas: full accommodation) and the cell's own
 * density; specular, inflow and outflow faces do not contribute. */
static void gradients(osim* s, const double* prim, double* g) {
    int nv = nv_of(s);
    for (int c = 0; c < s->nt; ++c) {
        const double* pc = prim + nv * (size_t)c;
        double b[NVX][3];
        memset(b, 0, sizeof b);
        for (int f = 0; f < 4; ++f) {
            int nb;
            double dx[3];
            int kind = face_link(s, c, f, &nb, dx);
            double far[NVX];
            if (kind == L_INTERIOR || kind == L_PERIODIC) {
                memcpy(far, prim + nv * (size_t)nb, sizeof(double) * nv);
            } else if (kind == L_WALL) {
                int grp = face_group(s, c, f);
                far[0] = pc[0];
                far[1] = s->g_u[3 * grp]; far[2] = s->g_u[3 * grp + 1]; far[3] = s->g_u[3 * grp + 2];
                far[4] = s->g_T[grp];
                far[5] = s->g_T[grp];
            } else {
                continue;
            }
            double w = 1.0 / (dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]);
            for (int v = 0; v < nv; ++v) {
                double dphi = far[v] - pc[v];
                for (int i = 0; i < 3; ++i) b[v][i] += w * dx[i] * dphi;
            }
        }
        const double* L = s->lsq + 9 * (size_t)c;
        for (int v = 0; v < nv; ++v)
            for (int i = 0; i < 3; ++i)
                g[GS * (size_t)c + 3 * v + i] = L[3 * i] * b[v][0] + L[3 * i + 1] * b[v][1] + L[3 * i + 2] * b[v][2];
    }
}

/* gradients of u, T (and T_r) of a cell in the public layout */
static int grad_width(const osim* s) { return s->dr ? 15 : 12; }

void oracle_dig_gradients(osim* s, const double* prim, double* grad) {
    geometry(s);
    int gw = grad_width(s);
    double* g = (double*)malloc(sizeof(double) * GS * (size_t)s->nt);
    gradients(s, prim, g);
    for (int c = 0; c < s->nt; ++c)
        for (int k = 0; k < gw; ++k) grad[gw * (size_t)c + k] = g[GS * (size_t)c + 3 + k];
    free(g);
}

/* NSF stress (xx,yy,zz,xy,xz,yz) and heat flux from a velocity gradient
 * gu[i][j] = du_i/dx_j and a temperature gradient gT at temperature T
 * (the translational one of a rotating gas, whose rotational heat flux
 * -kappa_r grad T_r follows from gTr). */
static void nsf_local(const osim* s, double T, const double* gu, const double* gT, const double* gTr, double* out) {
    double mu = mu_of(s, T);
    double div = gu[0] + gu[4] + gu[8];
    const int ii[6] = {0, 1, 2, 0, 0, 1}, jj[6] = {0, 1, 2, 1, 2, 2};
    for (int k = 0; k < 6; ++k) {
        double e = gu[3 * ii[k] + jj[k]] + gu[3 * jj[k] + ii[k]];
        if (k < 3) e -= (2.0 / 3.0) * div;
        out[k] = -mu * e;
    }
    if (s->dr) {
        double kt, kr;
        kappas_of(s, mu, &kt, &kr);
        for (int j = 0; j < 3; ++j) out[6 + j] = -kt * gT[j];
        for (int j = 0; j < 3; ++j) out[9 + j] = -kr * gTr[j];
    } else {
        double kap = kappa_of(s, mu);
        for (int j = 0; j < 3; ++j) out[6 + j] = -kap * gT[j];
    }
}

void oracle_dig_nsf(osim* s, const double* prim, const double* grad, double* out) {
    int nv = nv_of(s), nh = nh_of(s), gw = grad_width(s);
    for (int c = 0; c < s->nt; ++c) {
        const double* gc = grad + gw * (size_t)c;
        nsf_local(s, prim[nv * (size_t)c + 4], gc, gc + 9, gc + 12, out + nh * (size_t)c);
    }
}

static int samp_width(const osim* s) { return s->dr ? 18 : 14; }

void oracle_dig_sampled(osim* s, double* out) {
    int sw = samp_width(s);
    double* f = (double*)malloc(sizeof(double) * 15 * (size_t)s->nt);
    double* r = (double*)malloc(sizeof(double) * 4 * (size_t)s->nt);
    oracle_fields(s, 1, f);
    if (s->dr) oracle_rot_fields(s, 1, r);
    for (int c = 0; c < s->nt; ++c) {
        const double* a = f + 15 * (size_t)c;
        double* o = out + sw * (size_t)c;
        for (int k = 0; k < 14; ++k) o[k] = a[1 + k];
        if (s->dr)
            for (int k = 0; k < 4; ++k) o[14 + k] = r[4 * (size_t)c + k];
    }
    free(f); free(r);
}

void oracle_dig_kn_cell(osim* s, const double* prim, double L0, double* out) {
    double T0 = s->ref_T;
    double p0 = s->ref_n * KB * T0;
    double R = KB / s->m;
    double kn = mu_of(s, T0) / (p0 * L0) * sqrt(M_PI * R * T0 / 2.0);
    double rho0 = s->m * s->ref_n;
    int nv = nv_of(s);
    for (int c = 0; c < s->nt; ++c) {
        double rho = prim[nv * (size_t)c], T = prim[nv * (size_t)c + 4];
        double lam = kn * pow(T / T0, s->omega - 0.5) / (rho / rho0);
        double dc = 2.0 * cbrt(3.0 * s->vol[c] / (4.0 * M_PI)) / L0;
        double k = lam / dc;
        out[c] = (rho > 0 && T > 0 && isfinite(k)) ? k : INFINITY;
    }
}

void oracle_dig_gate(osim* s, double* prim, double* hot, const double* kn, double kn_max, int passes, int* state) {
    geometry(s);
    int nt = s->nt, nv = nv_of(s), nh = nh_of(s);
    unsigned char* avail = (unsigned char*)malloc((size_t)nt);
    unsigned char* next = (unsigned char*)malloc((size_t)nt);
    double* np = (double*)malloc(sizeof(double) * nv * (size_t)nt);
    double* nhot = (double*)malloc(sizeof(double) * nh * (size_t)nt);
    for (int c = 0; c < nt; ++c) {
        int ok = kn[c] <= kn_max;
        for (int v = 0; v < nv && ok; ++v) ok = isfinite(prim[nv * (size_t)c + v]);
        avail[c] = (unsigned char)ok;
        state[c] = ok ? 0 : 2;
    }
    for (int p = 0; p < passes; ++p) {
        memcpy(next, avail, (size_t)nt);
        for (int c = 0; c < nt; ++c) {
            if (avail[c]) continue;
            int cnt = 0;
            double sp[NVX] = {0}, sh[NHX] = {0};
            for (int f = 0; f < 4; ++f) {
                int nb;
                double dx[3];
                int kind = face_link(s, c, f, &nb, dx);
                if ((kind != L_INTERIOR && kind != L_PERIODIC) || !avail[nb]) continue;
                ++cnt;
                for (int v = 0; v < nv; ++v) sp[v] += prim[nv * (size_t)nb + v];
                for (int v = 0; v < nh; ++v) sh[v] += hot[nh * (size_t)nb + v];
            }
            if (!cnt) continue;
            for (int v = 0; v < nv; ++v) np[nv * (size_t)c + v] = sp[v] / cnt;
            for (int v = 0; v < nh; ++v) nhot[nh * (size_t)c + v] = sh[v] / cnt;
            next[c] = 1;
            state[c] = 1;
        }
        for (int c = 0; c < nt; ++c)
            if (next[c] && !avail[c]) {
                memcpy(prim + nv * (size_t)c, np + nv * (size_t)c, sizeof(double) * nv);
                memcpy(hot + nh * (size_t)c, nhot + nh * (size_t)c, sizeof(double) * nh);
            }
        memcpy(avail, next, (size_t)nt);
    }
    for (int c = 0; c < nt; ++c)
        if (state[c] == 2) {
            memcpy(prim + nv * (size_t)c, s->mprev + nv * (size_t)c, sizeof(double) * nv);
            for (int v = 0; v < nh; ++v) hot[nh * (size_t)c + v] = 0.0;
        }
    free(avail); free(next); free(np); free(nhot);
}

/* ---------------------------------------------------------------------- */
/* Finite-volume residual                                                   */
/* ---------------------------------------------------------------------- */
static void cons_of(const osim* s, const double* P, double* U) {
    double R = KB / s->m;
    double uu = P[1] * P[1] + P[2] * P[2] + P[3] * P[3];
    U[0] = P[0];
    U[1] = P[0] * P[1]; U[2] = P[0] * P[2]; U[3] = P[0] * P[3];
    if (s->dr) {
        /* total energy with e_r = (d_r/2) R T_r, and rho e_r (eq. energy_definitions) */
        double er = (0.5 * s->dr) * R * P[5];
        U[4] = P[0] * ((1.5 * R * P[4] + 0.5 * uu) + er);
        U[5] = P[0] * er;
    } else {
        U[4] = P[0] * (1.5 * R * P[4] + 0.5 * uu);
    }
}

static int prim_of(const osim* s, const double* U, double* P) {
    double R = KB / s->m;
    if (!(U[0] > 0)) return 0;
    P[0] = U[0];
    P[1] = U[1] / U[0]; P[2] = U[2] / U[0]; P[3] = U[3] / U[0];
    double uu = P[1] * P[1] + P[2] * P[2] + P[3] * P[3];
    if (s->dr) {
        double er = U[5] / U[0];
        P[4] = ((U[4] / U[0] - 0.5 * uu) - er) / (1.5 * R);
        P[5] = er / ((0.5 * s->dr) * R);
        return P[4] > 0 && isfinite(P[4]) && P[5] > 0 && isfinite(P[5]);
    }
    P[4] = (U[4] / U[0] - 0.5 * uu) / (1.5 * R);
    return P[4] > 0 && isfinite(P[4]);
}

/* inviscid flux F(P).n; the pressure is the translational one, rho R T_t */
static void flux_of(const osim* s, const double* P, const double* n, double* F) {
    double R = KB / s->m;
    double un = P[1] * n[0] + P[2] * n[1] + P[3] * n[2];
    double p = P[0] * R * P[4];
    double uu = P[1] * P[1] + P[2] * P[2] + P[3] * P[3];
    F[0] = P[0] * un;
    for (int i = 0; i < 3; ++i) F[1 + i] = P[0] * P[1 + i] * un + p * n[i];
    if (s->dr) {
        double er = (0.5 * s->dr) * R * P[5];
        double E = (1.5 * R * P[4] + 0.5 * uu) + er;
        F[4] = (P[0] * E + p) * un;
        F[5] = P[0] * er * un;
    } else {
        double E = 1.5 * R * P[4] + 0.5 * uu;
        F[4] = (P[0] * E + p) * un;
    }
}

/* acoustic spectral radius |u.n| + c (pseudo-time step), c of the frozen gas */
static double acoustic_speed(const osim* s, const double* P, const double* n) {
    double R = KB / s->m;
    return fabs(P[1] * n[0] + P[2] * n[1] + P[3] * n[2]) + sqrt(gamma_of(s) * R * P[4]);
}

/* dissipation speed: |u.n| + theta c with theta = min(1, max(M, M_cut)) */
static double wave_speed(const osim* s, const double* P, const double* n) {
    double R = KB / s->m;
    double c = sqrt(gamma_of(s) * R * P[4]);
    double un = fabs(P[1] * n[0] + P[2] * n[1] + P[3] * n[2]);
    double u = sqrt(P[1] * P[1] + P[2] * P[2] + P[3] * P[3]);
    double th = u / c;
    if (th < M_CUT) th = M_CUT;
    if (th > 1.0) th = 1.0;
    return un + th * c;
}

/* Face gradients of u, T (and T_r): the base gradient (gb, [NVX][3]) plus
 * the correction that makes its component along the connector dx equal the
 * difference quotient of far - near. */
static void face_grad(const osim* s, const double* gb, const double* far, const double* near, const double* dx,
                      double dl, double* gu, double* gT, double* gTr) {
    int nv = nv_of(s);
    for (int v = 1; v < nv; ++v) {
        double gf[3], ga = 0.0;
        for (int j = 0; j < 3; ++j) {
            gf[j] = gb[3 * v + j];
            ga += gf[j] * dx[j] / dl;
        }
        double jump = (far[v] - near[v]) / dl - ga;
        for (int j = 0; j < 3; ++j) gf[j] += jump * dx[j] / dl;
        if (v < 4)
            for (int j = 0; j < 3; ++j) gu[3 * (v - 1) + j] = gf[j];
        else if (v == 4)
            for (int j = 0; j < 3; ++j) gT[j] = gf[j];
        else
            for (int j = 0; j < 3; ++j) gTr[j] = gf[j];
    }
}

/* the state a diffuse wall imposes on the gradients: the cell's density,
 * the wall's velocity and temperature (both temperatures) */
static void wall_state(const osim* s, const double* Pc, int grp, double* w) {
    w[0] = Pc[0];
    w[1] = s->g_u[3 * grp]; w[2] = s->g_u[3 * grp + 1]; w[3] = s->g_u[3 * grp + 2];
    w[4] = s->g_T[grp];
    w[5] = s->g_T[grp];
}

/* HoT carried by each cell face [nt][4][nh]: the cell HoT averaged to the
 * face (the cell's own at a diffuse wall); with `consistent`, plus the
 * difference between the cell NSF stresses (cell gradients, cell T)
 * averaged to the face and the face NSF stress of the viscous flux (face
 * gradients, face T), both at the state prim.  At prim the viscous stress of
 * every face is then the average of the two cells' NSF + HoT, i.e. of their
 * sampled stresses (the coupling step's HoT). */
static void face_hot(osim* s, const double* prim, const double* g, const double* hot, int consistent, double* hotf) {
    int nv = nv_of(s), nh = nh_of(s);
    for (int c = 0; c < s->nt; ++c) {
        const double* Pc = prim + nv * (size_t)c;
        const double* gc = g + GS * (size_t)c;
        double nc[NHX];
        nsf_local(s, Pc[4], gc + 3, gc + 12, gc + 15, nc);
        for (int f = 0; f < 4; ++f) {
            int nb;
            double dx[3];
            int kind = face_link(s, c, f, &nb, dx);
            double* h = hotf + 4 * nh * (size_t)c + nh * f;
            double dl = sqrt(dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]);
            double gu[9], gT[3], gTr[3], vf[NHX];
            if (kind == L_INTERIOR || kind == L_PERIODIC) {
                const double* Pn = prim + nv * (size_t)nb;
                const double* gn = g + GS * (size_t)nb;
                double gavg[GS], nn[NHX];
                for (int k = 0; k < 3 * nv; ++k) gavg[k] = 0.5 * (gc[k] + gn[k]);
                face_grad(s, gavg, Pn, Pc, dx, dl, gu, gT, gTr);
                nsf_local(s, 0.5 * (Pc[4] + Pn[4]), gu, gT, gTr, vf);
                nsf_local(s, Pn[4], gn + 3, gn + 12, gn + 15, nn);
                for (int k = 0; k < nh; ++k) {
                    h[k] = 0.5 * (hot[nh * (size_t)c + k] + hot[nh * (size_t)nb + k]);
                    if (consistent) h[k] += 0.5 * (nc[k] + nn[k]) - vf[k];
                }
            } else if (kind == L_WALL) {
                int grp = face_group(s, c, f);
                double wallv[NVX];
                wall_state(s, Pc, grp, wallv);
                face_grad(s, gc, wallv, Pc, dx, dl, gu, gT, gTr);
                nsf_local(s, s->g_T[grp], gu, gT, gTr, vf);
                for (int k = 0; k < nh; ++k) {
                    h[k] = hot[nh * (size_t)c + k];
                    if (consistent) h[k] += nc[k] - vf[k];
                }
            } else {
                for (int k = 0; k < nh; ++k) h[k] = 0.0;
            }
        }
    }
}

/* Viscous part of a face flux: stress, its work with the face velocity uf
 * and the heat fluxes (both into the energy, q_r also into rho e_r). */
static void add_viscous(const osim* s, const double* vis, const double* n, const double* uf, double* F) {
    double S[3][3] = {{vis[0], vis[3], vis[4]}, {vis[3], vis[1], vis[5]}, {vis[4], vis[5], vis[2]}};
    double work = 0.0;
    for (int i = 0; i < 3; ++i) {
        double sn = S[i][0] * n[0] + S[i][1] * n[1] + S[i][2] * n[2];
        F[1 + i] += sn;
        work += sn * uf[i];
    }
    F[4] += work + (vis[6] * n[0] + vis[7] * n[1] + vis[8] * n[2]);
    if (s->dr) {
        double qr = vis[9] * n[0] + vis[10] * n[1] + vis[11] * n[2];
        F[4] += qr;
        F[5] += qr;
    }
}

/* viscous diffusion rate of the pseudo-time step at a face: the largest of
 * the momentum and thermal diffusivities, times 2 / dl */
static double viscous_rate(const osim* s, double T, double rho, double dl) {
    double R = KB / s->m;
    double mu = mu_of(s, T);
    double dmom = 4.0 * mu / (3.0 * rho), d = dmom;
    if (s->dr) {
        double kt, kr;
        kappas_of(s, mu, &kt, &kr);
        double dt_ = kt / (1.5 * rho * R), dr_ = kr / ((0.5 * s->dr) * rho * R);
        if (dt_ > d) d = dt_;
        if (dr_ > d) d = dr_;
    } else {
        double dth = kappa_of(s, mu) / (1.5 * rho * R);
        if (dth > d) d = dth;
    }
    return 2.0 * d / dl;
}

/* rotational relaxation (eq. macro): the source of rho e_r,
 * (d_r/2) rho R (T - T_r) / (Z_r tau), T = (3 T_t + d_r T_r)/(3 + d_r),
 * tau = mu(T_t) / p_t; *rate = 1 / (Z_r tau) */
static double relax_source(const osim* s, const double* P, double* rate) {
    double R = KB / s->m;
    double T = (3.0 * P[4] + s->dr * P[5]) / (3.0 + s->dr);
    double tau = mu_of(s, P[4]) / (P[0] * R * P[4]);
    *rate = 1.0 / (s->zr * tau);
    return (((0.5 * s->dr) * P[0]) * R) * (T - P[5]) * *rate;
}

/* residual R[nt][nv] = sum over faces of (flux . n) A (minus V times the
 * relaxation source in the rho e_r equation), and the sum over faces of
 * (spectral radius) A plus V times the relaxation rate for the pseudo-time
 * step: spec[nt] */
static void residual_all(osim* s, const double* prim, const double* hotf, const double* g, double* Rs, double* spec) {
    double R = KB / s->m;
    int nv = nv_of(s), nh = nh_of(s);
    for (int c = 0; c < s->nt; ++c) {
        const double* Pc = prim + nv * (size_t)c;
        const double* gc = g + GS * (size_t)c;
        double* Rc = Rs + nv * (size_t)c;
        for (int v = 0; v < nv; ++v) Rc[v] = 0.0;
        double sp = 0.0;
        for (int f = 0; f < 4; ++f) {
            int nb;
            double dx[3];
            int kind = face_link(s, c, f, &nb, dx);
            const double* n = s->fnu + 12 * (size_t)c + 3 * f;
            const double* xf = s->fcen + 12 * (size_t)c + 3 * f;
            const double* xc = s->cen + 3 * (size_t)c;
            const double* hf = hotf + 4 * nh * (size_t)c + nh * f;
            double A = s->farea[4 * (size_t)c + f];
            double F[NVX] = {0};
            double lam = 0.0, lamv = 0.0;
            if (kind == L_INTERIOR || kind == L_PERIODIC) {
                const double* Pn = prim + nv * (size_t)nb;
                const double* gn = g + GS * (size_t)nb;
                /* neighbour centroid in c's frame and face reconstruction */
                double rc[3], rn[3];
                for (int i = 0; i < 3; ++i) {
                    rc[i] = xf[i] - xc[i];
                    rn[i] = xf[i] - (xc[i] + dx[i]);
                }
                double PL[NVX], PR[NVX];
                for (int v = 0; v < nv; ++v) {
                    PL[v] = Pc[v] + (gc[3 * v] * rc[0] + gc[3 * v + 1] * rc[1] + gc[3 * v + 2] * rc[2]);
                    PR[v] = Pn[v] + (gn[3 * v] * rn[0] + gn[3 * v + 1] * rn[1] + gn[3 * v + 2] * rn[2]);
                }
                int pos = PL[0] > 0 && PL[4] > 0 && PR[0] > 0 && PR[4] > 0;
                if (s->dr) pos = pos && PL[5] > 0 && PR[5] > 0;
                if (!pos) {
                    memcpy(PL, Pc, sizeof(double) * nv);
                    memcpy(PR, Pn, sizeof(double) * nv);
                }
                double FL[NVX], FR[NVX], UL[NVX], UR[NVX];
                flux_of(s, PL, n, FL);
                flux_of(s, PR, n, FR);
                cons_of(s, PL, UL);
                cons_of(s, PR, UR);
                double aL = wave_speed(s, PL, n), aR = wave_speed(s, PR, n);
                double lam_d = aL > aR ? aL : aR;
                for (int v = 0; v < nv; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * lam_d * (UR[v] - UL[v]);
                double sL = acoustic_speed(s, PL, n), sR = acoustic_speed(s, PR, n);
                lam = sL > sR ? sL : sR;
                /* viscous: averaged gradients corrected along the centroid connector */
                double d2 = dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2];
                double dl = sqrt(d2);
                double gu[9], gT[3], gTr[3], gavg[GS];
                for (int k = 0; k < 3 * nv; ++k) gavg[k] = 0.5 * (gc[k] + gn[k]);
                face_grad(s, gavg, Pn, Pc, dx, dl, gu, gT, gTr);
                double Tf = 0.5 * (Pc[4] + Pn[4]);
                double rf = 0.5 * (Pc[0] + Pn[0]);
                double vis[NHX];
                nsf_local(s, Tf, gu, gT, gTr, vis);
                for (int k = 0; k < nh; ++k) vis[k] += hf[k];
                double uf[3] = {0.5 * (Pc[1] + Pn[1]), 0.5 * (Pc[2] + Pn[2]), 0.5 * (Pc[3] + Pn[3])};
                add_viscous(s, vis, n, uf, F);
                lamv = viscous_rate(s, Tf, rf, dl);
            } else if (kind == L_WALL || kind == L_SPECULAR) {
                double p = Pc[0] * R * Pc[4];
                for (int i = 0; i < 3; ++i) F[1 + i] = p * n[i];
                lam = acoustic_speed(s, Pc, n);
                if (kind == L_WALL) {
                    int grp = face_group(s, c, f);
                    const double* uw = s->g_u + 3 * grp;
                    double Tw = s->g_T[grp];
                    double d2 = dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2];
                    double dl = sqrt(d2);
                    double wallv[NVX];
                    wall_state(s, Pc, grp, wallv);
                    double gu[9], gT[3], gTr[3];
                    face_grad(s, gc, wallv, Pc, dx, dl, gu, gT, gTr);
                    double vis[NHX];
                    nsf_local(s, Tw, gu, gT, gTr, vis);
                    for (int k = 0; k < nh; ++k) vis[k] += hf[k];
                    add_viscous(s, vis, n, uw, F);
                    lamv = viscous_rate(s, Tw, Pc[0], dl);
                }
            } else if (kind == L_INFLOW) {
                int grp = face_group(s, c, f);
                double PR[NVX] = {s->m * s->g_n[grp], s->g_u[3 * grp], s->g_u[3 * grp + 1], s->g_u[3 * grp + 2],
                                  s->g_T[grp], s->g_T[grp]};
                double FL[NVX], FR[NVX], UL[NVX], UR[NVX];
                flux_of(s, Pc, n, FL);
                flux_of(s, PR, n, FR);
                cons_of(s, Pc, UL);
                cons_of(s, PR, UR);
                double aL = wave_speed(s, Pc, n), aR = wave_speed(s, PR, n);
                double lam_d = aL > aR ? aL : aR;
                for (int v = 0; v < nv; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * lam_d * (UR[v] - UL[v]);
                double sL = acoustic_speed(s, Pc, n), sR = acoustic_speed(s, PR, n);
                lam = sL > sR ? sL : sR;
            } else {
                flux_of(s, Pc, n, F);
                lam = acoustic_speed(s, Pc, n);
            }
            for (int v = 0; v < nv; ++v) Rc[v] += F[v] * A;
            sp += (lam + lamv) * A;
        }
        if (s->dr) {
            double rate;
            double src = relax_source(s, Pc, &rate);
            Rc[5] -= s->vol[c] * src;
            sp += s->vol[c] * rate;
        }
        spec[c] = sp;
    }
}

void oracle_dig_residual_faces(osim* s, const double* prim, const double* hotf, double* out) {
    geometry(s);
    double* g = (double*)malloc(sizeof(double) * GS * (size_t)s->nt);
    double* spec = (double*)malloc(sizeof(double) * (size_t)s->nt);
    gradients(s, prim, g);
    residual_all(s, prim, hotf, g, out, spec);
    free(g); free(spec);
}

void oracle_dig_face_hot(osim* s, const double* prim, const double* hot, int consistent, double* hotf) {
    geometry(s);
    double* g = (double*)malloc(sizeof(double) * GS * (size_t)s->nt);
    gradients(s, prim, g);
    face_hot(s, prim, g, hot, consistent, hotf);
    free(g);
}

void oracle_dig_residual(osim* s, const double* prim, const double* hot, double* out) {
    geometry(s);
    double* g = (double*)malloc(sizeof(double) * GS * (size_t)s->nt);
    double* spec = (double*)malloc(sizeof(double) * (size_t)s->nt);
    double* hotf = (double*)malloc(sizeof(double) * 4 * NHX * (size_t)s->nt);
    gradients(s, prim, g);
    face_hot(s, prim, g, hot, 0, hotf);
    residual_all(s, prim, hotf, g, out, spec);
    free(g); free(spec); free(hotf);
}

/* Pseudo-time marching to steady state: three-stage Runge-Kutta
 * (stage coefficients 1/3, 1/2, 1) with a local (or global) step
 * cfl V / (sum_f A (|u.n| + c + viscous rate) + V relaxation rate); stops
 * when the density residual norm (with rotation: together with the
 * rotational-energy residual over R T0) falls below eps_m times its first
 * value or after n_m iterations. */
static int solve_faces(osim* s, double* prim, const double* hotf, const odig_params* prm, odig_report* rep) {
    int nt = s->nt, nv = nv_of(s);
    const double alpha[3] = {1.0 / 3.0, 0.5, 1.0};
    double* g = (double*)malloc(sizeof(double) * GS * (size_t)nt);
    double* Rs = (double*)malloc(sizeof(double) * nv * (size_t)nt);
    double* spec = (double*)malloc(sizeof(double) * (size_t)nt);
    double* dt = (double*)malloc(sizeof(double) * (size_t)nt);
    double* U0 = (double*)malloc(sizeof(double) * nv * (size_t)nt);
    double* stage = (double*)malloc(sizeof(double) * nv * (size_t)nt);
    double res0 = 0.0, res = 0.0;
    int it = 0, conv = 0, failed = 0;
    for (it = 0; it < prm->n_m && !failed; ++it) {
        memcpy(stage, prim, sizeof(double) * nv * (size_t)nt);
        for (int c = 0; c < nt; ++c) cons_of(s, prim + nv * (size_t)c, U0 + nv * (size_t)c);
        for (int k = 0; k < 3 && !failed; ++k) {
            gradients(s, stage, g);
            residual_all(s, stage, hotf, g, Rs, spec);
            if (k == 0) {
                /* the density residual norm; a rotating gas adds its
                 * rotational-energy residual in mass units, R_er / (R T0) */
                double acc = 0.0, ert = (KB / s->m) * s->ref_T;
                for (int c = 0; c < nt; ++c) {
                    double r0 = Rs[nv * (size_t)c];
                    acc += r0 * r0;
                    if (s->dr) {
                        double r5 = Rs[nv * (size_t)c + 5] / ert;
                        acc += r5 * r5;
                    }
                }
                res = sqrt(acc);
                if (it == 0) res0 = res;
                if (!(res0 > 0) || res <= prm->eps_m * res0) {
                    conv = 1;
                    break;
                }
                double dtg = INFINITY;
                for (int c = 0; c < nt; ++c) {
                    dt[c] = prm->cfl * s->vol[c] / spec[c];
                    if (dt[c] < dtg) dtg = dt[c];
                }
                if (prm->global_dt)
                    for (int c = 0; c < nt; ++c) dt[c] = dtg;
            }
            for (int c = 0; c < nt; ++c) {
                double U[NVX];
                for (int v = 0; v < nv; ++v)
                    U[v] = U0[nv * (size_t)c + v] - alpha[k] * dt[c] / s->vol[c] * Rs[nv * (size_t)c + v];
                if (!prim_of(s, U, stage + nv * (size_t)c)) failed = 1;
            }
        }
        if (conv || failed) break;
        memcpy(prim, stage, sizeof(double) * nv * (size_t)nt);
    }
    if (rep) {
        rep->iters = it;
        rep->residual = res0 > 0 ? res / res0 : 0.0;
        rep->converged = conv;
        rep->failed = failed;
    }
    free(g); free(Rs); free(spec); free(dt); free(U0); free(stage);
    return failed ? -1 : 0;
}

/* ---------------------------------------------------------------------- */
/* Newton-Krylov solve of the same steady equations                         */
/* ---------------------------------------------------------------------- */
/* The steady discrete equations R(U) = 0 of the marching above, solved by
 * Newton's method with pseudo-transient continuation (Kelley and Keyes,
 * SIAM J. Numer. Anal. 35, 1998): step k solves
 *     (diag(S_c) / c_k + J(U_k)) dU = -R(U_k)
 * approximately, S_c being the sum that sets the local pseudo-time step of
 * the marching (V_c / dtau_c = S_c / cfl), and c_k the pseudo-time CFL
 * number, grown by the ratio of successive residual norms (switched
 * evolution relaxation, Mulder and van Leer, J. Comput. Phys. 59, 1985)
 * from the caller's cfl, within [cfl, NK_CFL_MAX], and at least halved
 * after a step whose linear solve left more than NK_LIN_POOR of its initial
 * residual (the linear system at that CFL number is beyond one GMRES
 * cycle).  The linear system is
 * solved by one cycle of at most m steps of GMRES (Saad and Schultz, SIAM J.
 * Sci. Stat. Comput. 7, 1986) from zero, with classical Gram-Schmidt applied
 * twice, Givens rotations, and a stop at NK_ETA of the initial linear
 * residual; products with the Jacobian are forward differences of the
 * residual (Knoll and Keyes, J. Comput. Phys. 193, 2004).  Unknowns and
 * equations are scaled by the reference state (density rho0, momentum
 * rho0 a0, energies rho0 a0^2, a0^2 = R T0), and the preconditioner on the
 * right divides cell c's unknowns by S_c (1 + 1/c_k) (the pseudo-time
 * operator's diagonal).  An update that leaves a cell non-physical is
 * halved, at most NK_HALVINGS times; then the solve fails.  The stopping test is
 * that of the marching (density residual, with rotation the rotational
 * energy residual too, against eps_m times its first value), taken at the
 * start of each Newton step; iters counts the updates made. */
#define NK_ETA 0.05
#define NK_CFL_MAX 1e8
#define NK_FD 1e-7
#define NK_HALVINGS 10
#define NK_LIN_POOR 0.5

static double conv_norm(const osim* s, const double* Rs) {
    int nv = nv_of(s);
    double acc = 0.0, ert = (KB / s->m) * s->ref_T;
    for (int c = 0; c < s->nt; ++c) {
        double r0 = Rs[nv * (size_t)c];
        acc += r0 * r0;
        if (s->dr) {
            double r5 = Rs[nv * (size_t)c + 5] / ert;
            acc += r5 * r5;
        }
    }
    return sqrt(acc);
}

static int solve_nk(osim* s, double* prim, const double* hotf, const odig_params* prm, odig_report* rep) {
    const int nt = s->nt, nv = nv_of(s);
    const size_t n = (size_t)nv * nt;
    const int m = prm->krylov > 0 ? prm->krylov : 40;
    const double R = KB / s->m;
    const double rho0 = s->m * s->ref_n, a2 = R * s->ref_T, a0 = sqrt(a2);
    double sc[NVX];
    sc[0] = rho0;
    sc[1] = sc[2] = sc[3] = rho0 * a0;
    sc[4] = sc[5] = rho0 * a2;
    double* g = (double*)malloc(sizeof(double) * GS * (size_t)nt);
    double* R0 = (double*)malloc(sizeof(double) * n);
    double* Rp = (double*)malloc(sizeof(double) * n);
    double* spec = (double*)malloc(sizeof(double) * (size_t)nt);
    double* specp = (double*)malloc(sizeof(double) * (size_t)nt);
    double* pc = (double*)malloc(sizeof(double) * (size_t)nt);
    double* U = (double*)malloc(sizeof(double) * n);
    double* Ut = (double*)malloc(sizeof(double) * n);
    double* Pt = (double*)malloc(sizeof(double) * n);
    double* V = (double*)malloc(sizeof(double) * n * (size_t)(m + 1));
    double* w = (double*)malloc(sizeof(double) * n);
    double* z = (double*)malloc(sizeof(double) * n);
    double* H = (double*)calloc((size_t)(m + 1) * m, sizeof(double));
    double* cs = (double*)malloc(sizeof(double) * m);
    double* sn = (double*)malloc(sizeof(double) * m);
    double* gv = (double*)malloc(sizeof(double) * (m + 1));
    double* y = (double*)malloc(sizeof(double) * m);
    double* h = (double*)malloc(sizeof(double) * (m + 1));
    for (int c = 0; c < nt; ++c) cons_of(s, prim + nv * (size_t)c, U + nv * (size_t)c);
    double res0 = 0.0, res = 0.0, cfl = prm->cfl, bprev = 0.0, lin = 0.0;
    int k = 0, conv = 0, failed = 0, nkry = 0;
    for (k = 0; k < prm->n_m; ++k) {
        gradients(s, prim, g);
        residual_all(s, prim, hotf, g, R0, spec);
        res = conv_norm(s, R0);
        if (k == 0) res0 = res;
        if (!(res0 > 0) || res <= prm->eps_m * res0) {
            conv = 1;
            break;
        }
        /* right-hand side -R in scaled units, its norm, the CFL number */
        double beta = 0.0;
        for (size_t e = 0; e < n; ++e) {
            V[e] = -R0[e] / sc[e % nv];
            beta += V[e] * V[e];
        }
        beta = sqrt(beta);
        if (k > 0) {
            double f = bprev / beta;
            if (lin > NK_LIN_POOR && f > 0.5) f = 0.5;
            cfl = cfl * f;
            if (cfl < prm->cfl) cfl = prm->cfl;
            if (cfl > NK_CFL_MAX) cfl = NK_CFL_MAX;
        }
        bprev = beta;
        for (int c = 0; c < nt; ++c) pc[c] = spec[c] * (1.0 + 1.0 / cfl);
        double xr = 0.0;
        for (size_t e = 0; e < n; ++e) {
            double x = U[e] / sc[e % nv];
            xr += x * x;
        }
        xr = sqrt(xr / (double)n);
        for (size_t e = 0; e < n; ++e) V[e] = V[e] / beta;
        memset(H, 0, sizeof(double) * (size_t)(m + 1) * m);
        gv[0] = beta;
        int jn = 0;
        for (int j = 0; j < m; ++j) {
            const double* vj = V + n * (size_t)j;
            /* w = B v_j: the preconditioned direction in U, a forward
             * difference of the residual along it, the pseudo-time diagonal */
            double vn = 0.0;
            for (int c = 0; c < nt; ++c)
                for (int v = 0; v < nv; ++v) {
                    double q = vj[nv * (size_t)c + v] / pc[c];
                    vn += q * q;
                }
            vn = sqrt(vn / (double)n);
            double eps = NK_FD * (1.0 + xr) / vn;
            int ok = 1;
            for (int c = 0; c < nt && ok; ++c) {
                for (int v = 0; v < nv; ++v) {
                    size_t e = nv * (size_t)c + v;
                    Ut[e] = U[e] + eps * (sc[v] * vj[e] / pc[c]);
                }
                ok = prim_of(s, Ut + nv * (size_t)c, Pt + nv * (size_t)c);
            }
            if (!ok) {
                failed = 1;
                break;
            }
            gradients(s, Pt, g);
            residual_all(s, Pt, hotf, g, Rp, specp);
            for (int c = 0; c < nt; ++c)
                for (int v = 0; v < nv; ++v) {
                    size_t e = nv * (size_t)c + v;
                    double du = sc[v] * vj[e] / pc[c];
                    w[e] = ((Rp[e] - R0[e]) / eps + spec[c] / cfl * du) / sc[v];
                }
            /* classical Gram-Schmidt, twice */
            for (int pass = 0; pass < 2; ++pass) {
                for (int i = 0; i <= j; ++i) {
                    const double* vi = V + n * (size_t)i;
                    double d = 0.0;
                    for (size_t e = 0; e < n; ++e) d += vi[e] * w[e];
                    h[i] = d;
                }
                for (size_t e = 0; e < n; ++e) {
                    double t = w[e];
                    for (int i = 0; i <= j; ++i) t -= h[i] * V[n * (size_t)i + e];
                    w[e] = t;
                }
                for (int i = 0; i <= j; ++i) H[i * m + j] += h[i];
            }
            double hn = 0.0;
            for (size_t e = 0; e < n; ++e) hn += w[e] * w[e];
            hn = sqrt(hn);
            H[(j + 1) * m + j] = hn;
            if (hn > 0)
                for (size_t e = 0; e < n; ++e) V[n * (size_t)(j + 1) + e] = w[e] / hn;
            /* the earlier rotations, then a new one that zeroes H[j+1][j] */
            for (int i = 0; i < j; ++i) {
                double a = H[i * m + j], b = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * b;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
            }
            double a = H[j * m + j], b = H[(j + 1) * m + j];
            double r = sqrt(a * a + b * b);
            cs[j] = r > 0 ? a / r : 1.0;
            sn[j] = r > 0 ? b / r : 0.0;
            H[j * m + j] = r;
            H[(j + 1) * m + j] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            jn = j + 1;
            ++nkry;
            if (fabs(gv[j + 1]) <= NK_ETA * beta || !(hn > 0)) break;
        }
        if (failed) break;
        lin = fabs(gv[jn]) / beta;
        /* y from the triangular system, z = V y, dU = preconditioned z */
        for (int i = jn - 1; i >= 0; --i) {
            double t = gv[i];
            for (int l = i + 1; l < jn; ++l) t -= H[i * m + l] * y[l];
            y[i] = t / H[i * m + i];
        }
        for (size_t e = 0; e < n; ++e) {
            double t = 0.0;
            for (int i = 0; i < jn; ++i) t += y[i] * V[n * (size_t)i + e];
            z[e] = t;
        }
        double alpha = 1.0;
        int accepted = 0;
        for (int tries = 0; tries <= NK_HALVINGS && !accepted; ++tries) {
            int ok = 1;
            for (int c = 0; c < nt && ok; ++c) {
                for (int v = 0; v < nv; ++v) {
                    size_t e = nv * (size_t)c + v;
                    Ut[e] = U[e] + alpha * (sc[v] * z[e] / pc[c]);
                }
                ok = prim_of(s, Ut + nv * (size_t)c, Pt + nv * (size_t)c);
            }
            if (ok)
                accepted = 1;
            else
                alpha = 0.5 * alpha;
        }
        if (!accepted) {
            failed = 1;
            break;
        }
        memcpy(U, Ut, sizeof(double) * n);
        memcpy(prim, Pt, sizeof(double) * n);
    }
    if (rep) {
        rep->iters = k;
        rep->residual = res0 > 0 ? res / res0 : 0.0;
        rep->converged = conv;
        rep->failed = failed;
        rep->krylov_steps = nkry;
    }
    free(g); free(R0); free(Rp); free(spec); free(specp); free(pc); free(U); free(Ut); free(Pt); free(V);
    free(w); free(z); free(H); free(cs); free(sn); free(gv); free(y); free(h);
    return failed ? -1 : 0;
}

static int solve_any(osim* s, double* prim, const double* hotf, const odig_params* prm, odig_report* rep) {
    return prm->solver == 1 ? solve_nk(s, prim, hotf, prm, rep) : solve_faces(s, prim, hotf, prm, rep);
}

/* The solve with the cell HoT averaged to the faces. */
int oracle_dig_solve(osim* s, double* prim, const double* hot, const odig_params* prm, odig_report* rep) {
    geometry(s);
    double* g = (double*)malloc(sizeof(double) * GS * (size_t)s->nt);
    double* hotf = (double*)malloc(sizeof(double) * 4 * NHX * (size_t)s->nt);
    gradients(s, prim, g);
    face_hot(s, prim, g, hot, 0, hotf);
    int rc = solve_any(s, prim, hotf, prm, rep);
    free(g); free(hotf);
    return rc;
}

/* ---------------------------------------------------------------------- */
/* Particle feedback                                                        */
/* ---------------------------------------------------------------------- */
/* Per admissible or reconstructed cell with particles: velocities shifted
 * and scaled from (u, T) of M^{k+1/2} to those of M^{k+1} (a rotating gas:
 * T_t, and the rotational energies scaled by the ratio of T_r); the
 * particle count set from the new density, floor(rho_new V / (F_N m) + U),
 * which leaves it unchanged when rho_new equals the cell's particle
 * density. */
static int fb_valid(const osim* s, const double* a, const double* b) {
    int ok = a[0] > 0 && b[0] > 0 && a[4] > 0 && b[4] > 0;
    if (s->dr) ok = ok && a[5] > 0 && b[5] > 0;
    return ok;
}

void oracle_dig_feedback(osim* s, const double* po, const double* pn, const int* state) {
    int nt = s->nt, nv = nv_of(s);
    int64_t cap_new = s->np;
    /* worst case growth is bounded per cell by the density ratio; count first */
    int* target = (int*)malloc(sizeof(int) * (size_t)nt);
    uint32_t w[4];
    for (int c = 0; c < nt; ++c) {
        int N = (int)(s->start[c + 1] - s->start[c]);
        target[c] = N;
        if (state[c] > 1 || N == 0) continue;
        const double* a = po + nv * (size_t)c;
        const double* b = pn + nv * (size_t)c;
        if (!fb_valid(s, a, b)) continue;
        o_draw(s, (uint32_t)c, s->step, P_RECAL, 0, w);
        target[c] = (int)floor(b[0] * s->vol[c] / (s->FN * s->m) + o_u01(w[0], w[1]));
        if (target[c] > N) cap_new += target[c] - N;
    }
    o_reserve(s, cap_new);
    int64_t np0 = s->np;
    for (int c = 0; c < nt; ++c) {
        int64_t a0 = s->start[c];
        int N = (int)(s->start[c + 1] - a0);
        if (state[c] > 1 || N == 0) continue;
        const double* a = po + nv * (size_t)c;
        const double* b = pn + nv * (size_t)c;
        if (!fb_valid(s, a, b)) continue;
        double scale = sqrt(b[4] / a[4]);
        for (int64_t p = a0; p < a0 + N; ++p)
            for (int i = 0; i < 3; ++i)
                s->v[3 * p + i] = o_to_store(s, b[1 + i] + scale * (s->v[3 * p + i] - a[1 + i]));
        if (s->dr) {
            double rs = b[5] / a[5];
            for (int64_t p = a0; p < a0 + N; ++p) s->ir[p] = rs * s->ir[p];
        }
        int T = target[c];
        if (T < N) {
            /* delete N - T particles chosen one by one among the remaining
             * (logical pid order) */
            int64_t* live = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
            for (int k = 0; k < N; ++k) live[k] = a0 + k;
            int rem = N;
            for (int k = 0; k < N - T; ++k) {
                o_draw(s, (uint32_t)c, s->step, P_RECAL, (uint64_t)(2 + 2 * k), w);
                int idx = (int)o_pick(w[0], (uint32_t)rem);
                s->cell[live[idx]] = -1;
                memmove(live + idx, live + idx + 1, sizeof(int64_t) * (size_t)(rem - idx - 1));
                --rem;
            }
            free(live);
        } else if (T > N) {
            const int* q = s->tv + 4 * c;
            for (int k = 0; k < T - N; ++k) {
                uint32_t w2[4];
                o_draw(s, (uint32_t)c, s->step, P_RECAL, (uint64_t)(2 + 2 * k), w);
                o_draw(s, (uint32_t)c, s->step, P_RECAL, (uint64_t)(3 + 2 * k), w2);
                int src = (int)o_pick(w[0], (uint32_t)N);
                double u1 = o_u01(w[2], w[3]), u2 = o_u01(w2[0], w2[1]), u3 = o_u01(w2[2], w2[3]), t;
                if (u1 > u2) { t = u1; u1 = u2; u2 = t; }
                if (u2 > u3) { t = u2; u2 = u3; u3 = t; }
                if (u1 > u2) { t = u1; u1 = u2; u2 = t; }
                double wt[4] = {u1, u2 - u1, u3 - u2, 1.0 - u3};
                int64_t d = s->np++;
                for (int i = 0; i < 3; ++i) {
                    double xi = wt[0] * s->xyz[3 * q[0] + i];
                    xi = xi + wt[1] * s->xyz[3 * q[1] + i];
                    xi = xi + wt[2] * s->xyz[3 * q[2] + i];
                    xi = xi + wt[3] * s->xyz[3 * q[3] + i];
                    s->x[3 * d + i] = xi;
                    s->v[3 * d + i] = s->v[3 * (a0 + src) + i];
                }
                s->cell[d] = c;
                s->pid[d] = s->next_pid++;
                if (s->dr) s->ir[d] = s->ir[a0 + src];
            }
        }
    }
    (void)np0;
    free(target);
    o_sort(s);
}

/* No freestream or outflow boundary: the particle mass is fixed. */
static int closed_domain(const osim* s) {
    for (int g = 0; g < s->ng; ++g)
        if (s->g_kind[g] == O_BC_INFLOW || s->g_kind[g] == O_BC_OUTFLOW) return 0;
    return 1;
}

int oracle_dig_couple(osim* s, const odig_params* prm, odig_report* rep) {
    geometry(s);
    int nt = s->nt, nv = nv_of(s), nh = nh_of(s), sw = samp_width(s), gw = grad_width(s);
    odig_report r;
    memset(&r, 0, sizeof r);
    r.np_before = s->np;
    double* smp = (double*)malloc(sizeof(double) * sw * (size_t)nt);
    double* prim = (double*)malloc(sizeof(double) * nv * (size_t)nt);
    double* half = (double*)malloc(sizeof(double) * nv * (size_t)nt);
    double* grad = (double*)malloc(sizeof(double) * gw * (size_t)nt);
    double* nsf = (double*)malloc(sizeof(double) * nh * (size_t)nt);
    double* hot = (double*)malloc(sizeof(double) * nh * (size_t)nt);
    double* kn = (double*)malloc(sizeof(double) * (size_t)nt);
    int* state = (int*)malloc(sizeof(int) * (size_t)nt);
    oracle_dig_sampled(s, smp);
    for (int c = 0; c < nt; ++c) {
        const double* a = smp + sw * (size_t)c;
        double* p = prim + nv * (size_t)c;
        int ok = isfinite(a[0]) && a[0] > 0;
        for (int v = 0; v < 5; ++v) p[v] = ok ? a[v] : s->mprev[nv * (size_t)c + v];
        if (s->dr) p[5] = ok ? a[14] : s->mprev[nv * (size_t)c + 5];
    }
    oracle_dig_kn_cell(s, prim, prm->L0, kn);
    for (int c = 0; c < nt; ++c)
        if (!(isfinite(smp[sw * (size_t)c]) && smp[sw * (size_t)c] > 0)) kn[c] = INFINITY;
    oracle_dig_gradients(s, prim, grad);
    oracle_dig_nsf(s, prim, grad, nsf);
    for (int c = 0; c < nt; ++c) {
        const double* a = smp + sw * (size_t)c;
        double* h = hot + nh * (size_t)c;
        const double* q = nsf + nh * (size_t)c;
        int ok = isfinite(a[0]) && a[0] > 0;
        for (int k = 0; k < 9; ++k) h[k] = ok ? a[5 + k] - q[k] : 0.0;
        if (s->dr)
            for (int k = 0; k < 3; ++k) h[9 + k] = ok ? a[15 + k] - q[9 + k] : 0.0;
    }
    oracle_dig_gate(s, prim, hot, kn, prm->kn_max, prm->passes, state);
    for (int c = 0; c < nt; ++c) {
        r.n_rejected += state[c] != 0;
        r.n_reconstructed += state[c] == 1;
        r.n_unreached += state[c] == 2;
    }
    memcpy(half, prim, sizeof(double) * nv * (size_t)nt);
    /* face HoT consistent with M^{k+1/2} */
    double* gf = (double*)malloc(sizeof(double) * GS * (size_t)nt);
    double* hotf = (double*)malloc(sizeof(double) * 4 * NHX * (size_t)nt);
    gradients(s, half, gf);
    face_hot(s, half, gf, hot, 1, hotf);
    /* the steady solve may start from the previous macroscopic solution */
    if (prm->warm_start) memcpy(prim, s->mprev, sizeof(double) * nv * (size_t)nt);
    if (r.n_rejected < nt) {
        solve_any(s, prim, hotf, prm, &r);
        /* only the solution of the synthetic equations is fed back: a solve
         * that stopped short of eps_m leaves the particles unchanged unless
         * the caller asks otherwise */
        int adjust = !r.failed && (r.converged || prm->unconverged);
        if (adjust && closed_domain(s)) {
            /* a closed domain keeps the mass of its particles */
            double mp = (double)s->np * s->FN * s->m, mfv = 0.0;
            for (int c = 0; c < nt; ++c) mfv += prim[nv * (size_t)c] * s->vol[c];
            double f = mp / mfv;
            for (int c = 0; c < nt; ++c) prim[nv * (size_t)c] = prim[nv * (size_t)c] * f;
        }
        if (adjust && prm->feedback) {
            oracle_dig_feedback(s, half, prim, state);
            r.fed_back = 1;
        }
        if (!r.failed) memcpy(s->mprev, prim, sizeof(double) * nv * (size_t)nt);
    }
    for (int c = 0; c < nt; ++c) s->local_acc[c] = state[c] != 0;
    r.np_after = s->np;
    if (rep) *rep = r;
    free(smp); free(prim); free(half); free(grad); free(nsf); free(hot); free(kn); free(state); free(gf); free(hotf);
    return r.failed ? -1 : 0;
}

void oracle_get_mprev(const osim* s, double* out) {
    if (s->mprev) memcpy(out, s->mprev, sizeof(double) * nv_of(s) * (size_t)s->nt);
}
