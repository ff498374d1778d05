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
 * (section 3.2); the macroscopic equations (eq. macro, monatomic) are solved
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
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle_internal.h"

#define GAMMA (5.0 / 3.0)
#define M_CUT 0.05
#define P_RECAL 7
#define NV 5 /* primitive variables: rho, u(3), T */

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

void oracle_set_reference(osim* s, double n0, double T0, const double* u0) {
    s->ref_n = n0;
    s->ref_T = T0;
    for (int i = 0; i < 3; ++i) s->ref_u[i] = u0 ? u0[i] : 0.0;
    if (s->mprev)
        for (int c = 0; c < s->nt; ++c) {
            double* m = s->mprev + NV * (size_t)c;
            m[0] = s->m * n0; m[1] = s->ref_u[0]; m[2] = s->ref_u[1]; m[3] = s->ref_u[2]; m[4] = T0;
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
    s->mprev = (double*)malloc(sizeof(double) * NV * (size_t)nt);
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

/* Least-squares gradients of all five primitives: g[nt][5][3]. At a diffuse
 * wall the far value is the wall velocity and temperature and the cell's own
 * density; specular, inflow and outflow faces do not contribute. */
static void gradients5(osim* s, const double* prim, double* g) {
    for (int c = 0; c < s->nt; ++c) {
        const double* pc = prim + NV * (size_t)c;
        double b[NV][3];
        memset(b, 0, sizeof b);
        for (int f = 0; f < 4; ++f) {
            int nb;
            double dx[3];
            int kind = face_link(s, c, f, &nb, dx);
            double far[NV];
            if (kind == L_INTERIOR || kind == L_PERIODIC) {
                memcpy(far, prim + NV * (size_t)nb, sizeof far);
            } else if (kind == L_WALL) {
                int grp = face_group(s, c, f);
                far[0] = pc[0];
                far[1] = s->g_u[3 * grp]; far[2] = s->g_u[3 * grp + 1]; far[3] = s->g_u[3 * grp + 2];
                far[4] = s->g_T[grp];
            } else {
                continue;
            }
            double w = 1.0 / (dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]);
            for (int v = 0; v < NV; ++v) {
                double dphi = far[v] - pc[v];
                for (int i = 0; i < 3; ++i) b[v][i] += w * dx[i] * dphi;
            }
        }
        const double* L = s->lsq + 9 * (size_t)c;
        for (int v = 0; v < NV; ++v)
            for (int i = 0; i < 3; ++i)
                g[15 * (size_t)c + 3 * v + i] = L[3 * i] * b[v][0] + L[3 * i + 1] * b[v][1] + L[3 * i + 2] * b[v][2];
    }
}

void oracle_dig_gradients(osim* s, const double* prim, double* grad) {
    geometry(s);
    double* g = (double*)malloc(sizeof(double) * 15 * (size_t)s->nt);
    gradients5(s, prim, g);
    for (int c = 0; c < s->nt; ++c) {
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) grad[12 * (size_t)c + 3 * i + j] = g[15 * (size_t)c + 3 * (1 + i) + j];
        for (int j = 0; j < 3; ++j) grad[12 * (size_t)c + 9 + j] = g[15 * (size_t)c + 12 + j];
    }
    free(g);
}

/* NSF stress (xx,yy,zz,xy,xz,yz) and heat flux from a velocity gradient
 * gu[i][j] = du_i/dx_j and a temperature gradient gT at temperature T. */
static void nsf_local(const osim* s, double T, const double* gu, const double* gT, double* out) {
    double mu = mu_of(s, T);
    double kap = kappa_of(s, mu);
    double div = gu[0] + gu[4] + gu[8];
    const int ii[6] = {0, 1, 2, 0, 0, 1}, jj[6] = {0, 1, 2, 1, 2, 2};
    for (int k = 0; k < 6; ++k) {
        double e = gu[3 * ii[k] + jj[k]] + gu[3 * jj[k] + ii[k]];
        if (k < 3) e -= (2.0 / 3.0) * div;
        out[k] = -mu * e;
    }
    for (int j = 0; j < 3; ++j) out[6 + j] = -kap * gT[j];
}

void oracle_dig_nsf(osim* s, const double* prim, const double* grad, double* out) {
    for (int c = 0; c < s->nt; ++c)
        nsf_local(s, prim[NV * (size_t)c + 4], grad + 12 * (size_t)c, grad + 12 * (size_t)c + 9, out + 9 * (size_t)c);
}

void oracle_dig_sampled(osim* s, double* out) {
    double* f = (double*)malloc(sizeof(double) * 15 * (size_t)s->nt);
    oracle_fields(s, 1, f);
    for (int c = 0; c < s->nt; ++c) {
        const double* a = f + 15 * (size_t)c;
        double* o = out + 14 * (size_t)c;
        for (int k = 0; k < 14; ++k) o[k] = a[1 + k];
    }
    free(f);
}

void oracle_dig_kn_cell(osim* s, const double* prim, double L0, double* out) {
    double T0 = s->ref_T;
    double p0 = s->ref_n * KB * T0;
    double R = KB / s->m;
    double kn = mu_of(s, T0) / (p0 * L0) * sqrt(M_PI * R * T0 / 2.0);
    double rho0 = s->m * s->ref_n;
    for (int c = 0; c < s->nt; ++c) {
        double rho = prim[NV * (size_t)c], T = prim[NV * (size_t)c + 4];
        double lam = kn * pow(T / T0, s->omega - 0.5) / (rho / rho0);
        double dc = 2.0 * cbrt(3.0 * s->vol[c] / (4.0 * M_PI)) / L0;
        double k = lam / dc;
        out[c] = (rho > 0 && T > 0 && isfinite(k)) ? k : INFINITY;
    }
}

void oracle_dig_gate(osim* s, double* prim, double* hot, const double* kn, double kn_max, int passes, int* state) {
    geometry(s);
    int nt = s->nt;
    unsigned char* avail = (unsigned char*)malloc((size_t)nt);
    unsigned char* next = (unsigned char*)malloc((size_t)nt);
    double* np = (double*)malloc(sizeof(double) * NV * (size_t)nt);
    double* nh = (double*)malloc(sizeof(double) * 9 * (size_t)nt);
    for (int c = 0; c < nt; ++c) {
        int ok = kn[c] <= kn_max;
        for (int v = 0; v < NV && ok; ++v) ok = isfinite(prim[NV * (size_t)c + v]);
        avail[c] = (unsigned char)ok;
        state[c] = ok ? 0 : 2;
    }
    for (int p = 0; p < passes; ++p) {
        memcpy(next, avail, (size_t)nt);
        for (int c = 0; c < nt; ++c) {
            if (avail[c]) continue;
            int cnt = 0;
            double sp[NV] = {0}, sh[9] = {0};
            for (int f = 0; f < 4; ++f) {
                int nb;
                double dx[3];
                int kind = face_link(s, c, f, &nb, dx);
                if ((kind != L_INTERIOR && kind != L_PERIODIC) || !avail[nb]) continue;
                ++cnt;
                for (int v = 0; v < NV; ++v) sp[v] += prim[NV * (size_t)nb + v];
                for (int v = 0; v < 9; ++v) sh[v] += hot[9 * (size_t)nb + v];
            }
            if (!cnt) continue;
            for (int v = 0; v < NV; ++v) np[NV * (size_t)c + v] = sp[v] / cnt;
            for (int v = 0; v < 9; ++v) nh[9 * (size_t)c + v] = sh[v] / cnt;
            next[c] = 1;
            state[c] = 1;
        }
        for (int c = 0; c < nt; ++c)
            if (next[c] && !avail[c]) {
                memcpy(prim + NV * (size_t)c, np + NV * (size_t)c, sizeof(double) * NV);
                memcpy(hot + 9 * (size_t)c, nh + 9 * (size_t)c, sizeof(double) * 9);
            }
        memcpy(avail, next, (size_t)nt);
    }
    for (int c = 0; c < nt; ++c)
        if (state[c] == 2) {
            memcpy(prim + NV * (size_t)c, s->mprev + NV * (size_t)c, sizeof(double) * NV);
            for (int v = 0; v < 9; ++v) hot[9 * (size_t)c + v] = 0.0;
        }
    free(avail); free(next); free(np); free(nh);
}

/* ---------------------------------------------------------------------- */
/* Finite-volume residual                                                   */
/* ---------------------------------------------------------------------- */
static void cons_of(const osim* s, const double* P, double* U) {
    double R = KB / s->m;
    double uu = P[1] * P[1] + P[2] * P[2] + P[3] * P[3];
    U[0] = P[0];
    U[1] = P[0] * P[1]; U[2] = P[0] * P[2]; U[3] = P[0] * P[3];
    U[4] = P[0] * (1.5 * R * P[4] + 0.5 * uu);
}

static int prim_of(const osim* s, const double* U, double* P) {
    double R = KB / s->m;
    if (!(U[0] > 0)) return 0;
    P[0] = U[0];
    P[1] = U[1] / U[0]; P[2] = U[2] / U[0]; P[3] = U[3] / U[0];
    double uu = P[1] * P[1] + P[2] * P[2] + P[3] * P[3];
    P[4] = (U[4] / U[0] - 0.5 * uu) / (1.5 * R);
    return P[4] > 0 && isfinite(P[4]);
}

/* inviscid flux F(P).n */
static void flux_of(const osim* s, const double* P, const double* n, double* F) {
    double R = KB / s->m;
    double un = P[1] * n[0] + P[2] * n[1] + P[3] * n[2];
    double p = P[0] * R * P[4];
    double uu = P[1] * P[1] + P[2] * P[2] + P[3] * P[3];
    double E = 1.5 * R * P[4] + 0.5 * uu;
    F[0] = P[0] * un;
    for (int i = 0; i < 3; ++i) F[1 + i] = P[0] * P[1 + i] * un + p * n[i];
    F[4] = (P[0] * E + p) * un;
}

/* acoustic spectral radius |u.n| + c (pseudo-time step) */
static double acoustic_speed(const osim* s, const double* P, const double* n) {
    double R = KB / s->m;
    return fabs(P[1] * n[0] + P[2] * n[1] + P[3] * n[2]) + sqrt(GAMMA * R * P[4]);
}

/* dissipation speed: |u.n| + theta c with theta = min(1, max(M, M_cut)) */
static double wave_speed(const osim* s, const double* P, const double* n) {
    double R = KB / s->m;
    double c = sqrt(GAMMA * R * P[4]);
    double un = fabs(P[1] * n[0] + P[2] * n[1] + P[3] * n[2]);
    double u = sqrt(P[1] * P[1] + P[2] * P[2] + P[3] * P[3]);
    double th = u / c;
    if (th < M_CUT) th = M_CUT;
    if (th > 1.0) th = 1.0;
    return un + th * c;
}

/* Face gradients of u and T: the base gradient (gb, [5][3]) plus the
 * correction that makes its component along the connector dx equal the
 * difference quotient of far - near. */
static void face_grad(const double* gb, const double* far, const double* near, const double* dx, double dl,
                      double* gu, double* gT) {
    for (int v = 1; v < NV; ++v) {
        double gf[3], ga = 0.0;
        for (int j = 0; j < 3; ++j) {
            gf[j] = gb[3 * v + j];
            ga += gf[j] * dx[j] / dl;
        }
        double jump = (far[v] - near[v]) / dl - ga;
        for (int j = 0; j < 3; ++j) gf[j] += jump * dx[j] / dl;
        if (v < 4)
            for (int j = 0; j < 3; ++j) gu[3 * (v - 1) + j] = gf[j];
        else
            for (int j = 0; j < 3; ++j) gT[j] = gf[j];
    }
}

/* HoT carried by each cell face [nt][4][9]: the cell HoT averaged to the
 * face (the cell's own at a diffuse wall); with `consistent`, plus the
 * difference between the cell NSF stresses (cell gradients, cell T)
 * averaged to the face and the face NSF stress of the viscous flux (face
 * gradients, face T), both at the state prim.  At prim the viscous stress of
 * every face is then the average of the two cells' NSF + HoT, i.e. of their
 * sampled stresses (the coupling step's HoT). */
static void face_hot(osim* s, const double* prim, const double* g, const double* hot, int consistent, double* hotf) {
    for (int c = 0; c < s->nt; ++c) {
        const double* Pc = prim + NV * (size_t)c;
        const double* gc = g + 15 * (size_t)c;
        double nc[9];
        nsf_local(s, Pc[4], gc + 3, gc + 12, nc);
        for (int f = 0; f < 4; ++f) {
            int nb;
            double dx[3];
            int kind = face_link(s, c, f, &nb, dx);
            double* h = hotf + 36 * (size_t)c + 9 * f;
            double dl = sqrt(dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]);
            double gu[9], gT[3], vf[9];
            if (kind == L_INTERIOR || kind == L_PERIODIC) {
                const double* Pn = prim + NV * (size_t)nb;
                const double* gn = g + 15 * (size_t)nb;
                double gavg[15], nn[9];
                for (int k = 0; k < 15; ++k) gavg[k] = 0.5 * (gc[k] + gn[k]);
                face_grad(gavg, Pn, Pc, dx, dl, gu, gT);
                nsf_local(s, 0.5 * (Pc[4] + Pn[4]), gu, gT, vf);
                nsf_local(s, Pn[4], gn + 3, gn + 12, nn);
                for (int k = 0; k < 9; ++k) {
                    h[k] = 0.5 * (hot[9 * (size_t)c + k] + hot[9 * (size_t)nb + k]);
                    if (consistent) h[k] += 0.5 * (nc[k] + nn[k]) - vf[k];
                }
            } else if (kind == L_WALL) {
                int grp = face_group(s, c, f);
                double wallv[NV] = {Pc[0], s->g_u[3 * grp], s->g_u[3 * grp + 1], s->g_u[3 * grp + 2], s->g_T[grp]};
                face_grad(gc, wallv, Pc, dx, dl, gu, gT);
                nsf_local(s, s->g_T[grp], gu, gT, vf);
                for (int k = 0; k < 9; ++k) {
                    h[k] = hot[9 * (size_t)c + k];
                    if (consistent) h[k] += nc[k] - vf[k];
                }
            } else {
                for (int k = 0; k < 9; ++k) h[k] = 0.0;
            }
        }
    }
}

/* residual R[nt][5] = sum over faces of (flux . n) A, and the sum over faces
 * of (spectral radius) A for the pseudo-time step: spec[nt] */
static void residual_all(osim* s, const double* prim, const double* hotf, const double* g, double* Rs, double* spec) {
    double R = KB / s->m;
    for (int c = 0; c < s->nt; ++c) {
        const double* Pc = prim + NV * (size_t)c;
        const double* gc = g + 15 * (size_t)c;
        double* Rc = Rs + NV * (size_t)c;
        for (int v = 0; v < NV; ++v) Rc[v] = 0.0;
        double sp = 0.0;
        for (int f = 0; f < 4; ++f) {
            int nb;
            double dx[3];
            int kind = face_link(s, c, f, &nb, dx);
            const double* n = s->fnu + 12 * (size_t)c + 3 * f;
            const double* xf = s->fcen + 12 * (size_t)c + 3 * f;
            const double* xc = s->cen + 3 * (size_t)c;
            double A = s->farea[4 * (size_t)c + f];
            double F[NV] = {0};
            double lam = 0.0, lamv = 0.0;
            if (kind == L_INTERIOR || kind == L_PERIODIC) {
                const double* Pn = prim + NV * (size_t)nb;
                const double* gn = g + 15 * (size_t)nb;
                /* neighbour centroid in c's frame and face reconstruction */
                double rc[3], rn[3];
                for (int i = 0; i < 3; ++i) {
                    rc[i] = xf[i] - xc[i];
                    rn[i] = xf[i] - (xc[i] + dx[i]);
                }
                double PL[NV], PR[NV];
                for (int v = 0; v < NV; ++v) {
                    PL[v] = Pc[v] + (gc[3 * v] * rc[0] + gc[3 * v + 1] * rc[1] + gc[3 * v + 2] * rc[2]);
                    PR[v] = Pn[v] + (gn[3 * v] * rn[0] + gn[3 * v + 1] * rn[1] + gn[3 * v + 2] * rn[2]);
                }
                if (!(PL[0] > 0 && PL[4] > 0 && PR[0] > 0 && PR[4] > 0)) {
                    memcpy(PL, Pc, sizeof PL);
                    memcpy(PR, Pn, sizeof PR);
                }
                double FL[NV], FR[NV], UL[NV], UR[NV];
                flux_of(s, PL, n, FL);
                flux_of(s, PR, n, FR);
                cons_of(s, PL, UL);
                cons_of(s, PR, UR);
                double aL = wave_speed(s, PL, n), aR = wave_speed(s, PR, n);
                double lam_d = aL > aR ? aL : aR;
                for (int v = 0; v < NV; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * lam_d * (UR[v] - UL[v]);
                double sL = acoustic_speed(s, PL, n), sR = acoustic_speed(s, PR, n);
                lam = sL > sR ? sL : sR;
                /* viscous: averaged gradients corrected along the centroid connector */
                double d2 = dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2];
                double dl = sqrt(d2);
                double gu[9], gT[3], gavg[15];
                for (int k = 0; k < 15; ++k) gavg[k] = 0.5 * (gc[k] + gn[k]);
                face_grad(gavg, Pn, Pc, dx, dl, gu, gT);
                double Tf = 0.5 * (Pc[4] + Pn[4]);
                double rf = 0.5 * (Pc[0] + Pn[0]);
                double vis[9];
                nsf_local(s, Tf, gu, gT, vis);
                for (int k = 0; k < 9; ++k) vis[k] += hotf[36 * (size_t)c + 9 * f + k];
                double uf[3] = {0.5 * (Pc[1] + Pn[1]), 0.5 * (Pc[2] + Pn[2]), 0.5 * (Pc[3] + Pn[3])};
                double S[3][3] = {{vis[0], vis[3], vis[4]}, {vis[3], vis[1], vis[5]}, {vis[4], vis[5], vis[2]}};
                double work = 0.0;
                for (int i = 0; i < 3; ++i) {
                    double sn = S[i][0] * n[0] + S[i][1] * n[1] + S[i][2] * n[2];
                    F[1 + i] += sn;
                    work += sn * uf[i];
                }
                F[4] += work + (vis[6] * n[0] + vis[7] * n[1] + vis[8] * n[2]);
                double mu = mu_of(s, Tf);
                double dmom = 4.0 * mu / (3.0 * rf), dth = kappa_of(s, mu) / (1.5 * rf * R);
                lamv = 2.0 * (dmom > dth ? dmom : dth) / dl;
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
                    double wallv[NV] = {Pc[0], uw[0], uw[1], uw[2], Tw};
                    double gu[9], gT[3];
                    face_grad(gc, wallv, Pc, dx, dl, gu, gT);
                    double vis[9];
                    nsf_local(s, Tw, gu, gT, vis);
                    for (int k = 0; k < 9; ++k) vis[k] += hotf[36 * (size_t)c + 9 * f + k];
                    double S[3][3] = {{vis[0], vis[3], vis[4]}, {vis[3], vis[1], vis[5]}, {vis[4], vis[5], vis[2]}};
                    double work = 0.0;
                    for (int i = 0; i < 3; ++i) {
                        double sn = S[i][0] * n[0] + S[i][1] * n[1] + S[i][2] * n[2];
                        F[1 + i] += sn;
                        work += sn * uw[i];
                    }
                    F[4] += work + (vis[6] * n[0] + vis[7] * n[1] + vis[8] * n[2]);
                    double mu = mu_of(s, Tw);
                    double dmom = 4.0 * mu / (3.0 * Pc[0]), dth = kappa_of(s, mu) / (1.5 * Pc[0] * R);
                    lamv = 2.0 * (dmom > dth ? dmom : dth) / dl;
                }
            } else if (kind == L_INFLOW) {
                int grp = face_group(s, c, f);
                double PR[NV] = {s->m * s->g_n[grp], s->g_u[3 * grp], s->g_u[3 * grp + 1], s->g_u[3 * grp + 2],
                                 s->g_T[grp]};
                double FL[NV], FR[NV], UL[NV], UR[NV];
                flux_of(s, Pc, n, FL);
                flux_of(s, PR, n, FR);
                cons_of(s, Pc, UL);
                cons_of(s, PR, UR);
                double aL = wave_speed(s, Pc, n), aR = wave_speed(s, PR, n);
                double lam_d = aL > aR ? aL : aR;
                for (int v = 0; v < NV; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * lam_d * (UR[v] - UL[v]);
                double sL = acoustic_speed(s, Pc, n), sR = acoustic_speed(s, PR, n);
                lam = sL > sR ? sL : sR;
            } else {
                flux_of(s, Pc, n, F);
                lam = acoustic_speed(s, Pc, n);
            }
            for (int v = 0; v < NV; ++v) Rc[v] += F[v] * A;
            sp += (lam + lamv) * A;
        }
        spec[c] = sp;
    }
}

void oracle_dig_residual_faces(osim* s, const double* prim, const double* hotf, double* out) {
    geometry(s);
    double* g = (double*)malloc(sizeof(double) * 15 * (size_t)s->nt);
    double* spec = (double*)malloc(sizeof(double) * (size_t)s->nt);
    gradients5(s, prim, g);
    residual_all(s, prim, hotf, g, out, spec);
    free(g); free(spec);
}

void oracle_dig_face_hot(osim* s, const double* prim, const double* hot, int consistent, double* hotf) {
    geometry(s);
    double* g = (double*)malloc(sizeof(double) * 15 * (size_t)s->nt);
    gradients5(s, prim, g);
    face_hot(s, prim, g, hot, consistent, hotf);
    free(g);
}

void oracle_dig_residual(osim* s, const double* prim, const double* hot, double* out) {
    geometry(s);
    double* g = (double*)malloc(sizeof(double) * 15 * (size_t)s->nt);
    double* spec = (double*)malloc(sizeof(double) * (size_t)s->nt);
    double* hotf = (double*)malloc(sizeof(double) * 36 * (size_t)s->nt);
    gradients5(s, prim, g);
    face_hot(s, prim, g, hot, 0, hotf);
    residual_all(s, prim, hotf, g, out, spec);
    free(g); free(spec); free(hotf);
}

/* Pseudo-time marching to steady state: three-stage Runge-Kutta
 * (stage coefficients 1/3, 1/2, 1) with a local (or global) step
 * cfl V / sum_f A (|u.n| + c + viscous rate); stops when the density
 * residual norm falls below eps_m times its first value or after n_m
 * iterations. */
static int solve_faces(osim* s, double* prim, const double* hotf, const odig_params* prm, odig_report* rep) {
    int nt = s->nt;
    const double alpha[3] = {1.0 / 3.0, 0.5, 1.0};
    double* g = (double*)malloc(sizeof(double) * 15 * (size_t)nt);
    double* Rs = (double*)malloc(sizeof(double) * NV * (size_t)nt);
    double* spec = (double*)malloc(sizeof(double) * (size_t)nt);
    double* dt = (double*)malloc(sizeof(double) * (size_t)nt);
    double* U0 = (double*)malloc(sizeof(double) * NV * (size_t)nt);
    double* stage = (double*)malloc(sizeof(double) * NV * (size_t)nt);
    double res0 = 0.0, res = 0.0;
    int it = 0, conv = 0, failed = 0;
    for (it = 0; it < prm->n_m && !failed; ++it) {
        memcpy(stage, prim, sizeof(double) * NV * (size_t)nt);
        for (int c = 0; c < nt; ++c) cons_of(s, prim + NV * (size_t)c, U0 + NV * (size_t)c);
        for (int k = 0; k < 3 && !failed; ++k) {
            gradients5(s, stage, g);
            residual_all(s, stage, hotf, g, Rs, spec);
            if (k == 0) {
                double acc = 0.0;
                for (int c = 0; c < nt; ++c) acc += Rs[NV * (size_t)c] * Rs[NV * (size_t)c];
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
                double U[NV];
                for (int v = 0; v < NV; ++v)
                    U[v] = U0[NV * (size_t)c + v] - alpha[k] * dt[c] / s->vol[c] * Rs[NV * (size_t)c + v];
                if (!prim_of(s, U, stage + NV * (size_t)c)) failed = 1;
            }
        }
        if (conv || failed) break;
        memcpy(prim, stage, sizeof(double) * NV * (size_t)nt);
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

/* The solve with the cell HoT averaged to the faces. */
int oracle_dig_solve(osim* s, double* prim, const double* hot, const odig_params* prm, odig_report* rep) {
    geometry(s);
    double* g = (double*)malloc(sizeof(double) * 15 * (size_t)s->nt);
    double* hotf = (double*)malloc(sizeof(double) * 36 * (size_t)s->nt);
    gradients5(s, prim, g);
    face_hot(s, prim, g, hot, 0, hotf);
    int rc = solve_faces(s, prim, hotf, prm, rep);
    free(g); free(hotf);
    return rc;
}

/* ---------------------------------------------------------------------- */
/* Particle feedback                                                        */
/* ---------------------------------------------------------------------- */
/* Per admissible or reconstructed cell with particles: velocities shifted
 * and scaled from (u, T) of M^{k+1/2} to those of M^{k+1}; the particle
 * count set from the new density, floor(rho_new V / (F_N m) + U), which
 * leaves it unchanged when rho_new equals the cell's particle density. */
void oracle_dig_feedback(osim* s, const double* po, const double* pn, const int* state) {
    int nt = s->nt;
    int64_t cap_new = s->np;
    /* worst case growth is bounded per cell by the density ratio; count first */
    int* target = (int*)malloc(sizeof(int) * (size_t)nt);
    uint32_t w[4];
    for (int c = 0; c < nt; ++c) {
        int N = (int)(s->start[c + 1] - s->start[c]);
        target[c] = N;
        if (state[c] > 1 || N == 0) continue;
        const double* a = po + NV * (size_t)c;
        const double* b = pn + NV * (size_t)c;
        if (!(a[0] > 0 && b[0] > 0 && a[4] > 0 && b[4] > 0)) continue;
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
        const double* a = po + NV * (size_t)c;
        const double* b = pn + NV * (size_t)c;
        if (!(a[0] > 0 && b[0] > 0 && a[4] > 0 && b[4] > 0)) continue;
        double scale = sqrt(b[4] / a[4]);
        for (int64_t p = a0; p < a0 + N; ++p)
            for (int i = 0; i < 3; ++i)
                s->v[3 * p + i] = o_to_store(s, b[1 + i] + scale * (s->v[3 * p + i] - a[1 + i]));
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
    int nt = s->nt;
    odig_report r;
    memset(&r, 0, sizeof r);
    r.np_before = s->np;
    double* smp = (double*)malloc(sizeof(double) * 14 * (size_t)nt);
    double* prim = (double*)malloc(sizeof(double) * NV * (size_t)nt);
    double* half = (double*)malloc(sizeof(double) * NV * (size_t)nt);
    double* grad = (double*)malloc(sizeof(double) * 12 * (size_t)nt);
    double* nsf = (double*)malloc(sizeof(double) * 9 * (size_t)nt);
    double* hot = (double*)malloc(sizeof(double) * 9 * (size_t)nt);
    double* kn = (double*)malloc(sizeof(double) * (size_t)nt);
    int* state = (int*)malloc(sizeof(int) * (size_t)nt);
    oracle_dig_sampled(s, smp);
    for (int c = 0; c < nt; ++c) {
        const double* a = smp + 14 * (size_t)c;
        int ok = isfinite(a[0]) && a[0] > 0;
        for (int v = 0; v < NV; ++v) prim[NV * (size_t)c + v] = ok ? a[v] : s->mprev[NV * (size_t)c + v];
    }
    oracle_dig_kn_cell(s, prim, prm->L0, kn);
    for (int c = 0; c < nt; ++c)
        if (!(isfinite(smp[14 * (size_t)c]) && smp[14 * (size_t)c] > 0)) kn[c] = INFINITY;
    oracle_dig_gradients(s, prim, grad);
    oracle_dig_nsf(s, prim, grad, nsf);
    for (int c = 0; c < nt; ++c) {
        const double* a = smp + 14 * (size_t)c;
        int ok = isfinite(a[0]) && a[0] > 0;
        for (int k = 0; k < 9; ++k) hot[9 * (size_t)c + k] = ok ? a[5 + k] - nsf[9 * (size_t)c + k] : 0.0;
    }
    oracle_dig_gate(s, prim, hot, kn, prm->kn_max, prm->passes, state);
    for (int c = 0; c < nt; ++c) {
        r.n_rejected += state[c] != 0;
        r.n_reconstructed += state[c] == 1;
        r.n_unreached += state[c] == 2;
    }
    memcpy(half, prim, sizeof(double) * NV * (size_t)nt);
    /* face HoT consistent with M^{k+1/2} */
    double* g5 = (double*)malloc(sizeof(double) * 15 * (size_t)nt);
    double* hotf = (double*)malloc(sizeof(double) * 36 * (size_t)nt);
    gradients5(s, half, g5);
    face_hot(s, half, g5, hot, 1, hotf);
    /* the steady solve may start from the previous macroscopic solution */
    if (prm->warm_start) memcpy(prim, s->mprev, sizeof(double) * NV * (size_t)nt);
    if (r.n_rejected < nt) {
        solve_faces(s, prim, hotf, prm, &r);
        /* only the solution of the synthetic equations is fed back: a solve
         * that stopped short of eps_m leaves the particles unchanged unless
         * the caller asks otherwise */
        int adjust = !r.failed && (r.converged || prm->unconverged);
        if (adjust && closed_domain(s)) {
            /* a closed domain keeps the mass of its particles */
            double mp = (double)s->np * s->FN * s->m, mfv = 0.0;
            for (int c = 0; c < nt; ++c) mfv += prim[NV * (size_t)c] * s->vol[c];
            double f = mp / mfv;
            for (int c = 0; c < nt; ++c) prim[NV * (size_t)c] = prim[NV * (size_t)c] * f;
        }
        if (adjust && prm->feedback) {
            oracle_dig_feedback(s, half, prim, state);
            r.fed_back = 1;
        }
        if (!r.failed) memcpy(s->mprev, prim, sizeof(double) * NV * (size_t)nt);
    }
    for (int c = 0; c < nt; ++c) s->local_acc[c] = state[c] != 0;
    r.np_after = s->np;
    if (rep) *rep = r;
    free(smp); free(prim); free(half); free(grad); free(nsf); free(hot); free(kn); free(state); free(g5); free(hotf);
    return r.failed ? -1 : 0;
}

void oracle_get_mprev(const osim* s, double* out) {
    if (s->mprev) memcpy(out, s->mprev, sizeof(double) * NV * (size_t)s->nt);
}
