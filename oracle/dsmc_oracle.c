/*
 * Plain CPU oracle of the DSMC particle loop.  TEST INFRASTRUCTURE ONLY:
 * called by tests/, the smoke check and the benchmark's CPU-baseline leg;
 * never by the product path.  Single-threaded, written for clarity, not
 * speed.  Shares no code with the GPU library.
 *
 * What it follows:
 *  - DSMC step splitting (paper, section 2.1): particles are moved, then
 *    pairs are selected inside each cell and collided.  Move is face-to-face
 *    tracking through the tetrahedra (section 4.2, face-based tracking).
 *  - Collisions: Bird's no-time-counter pair selection with the variable
 *    hard sphere model (section 2.1 and the gas model of section 5); the
 *    selection formula itself is not printed in the paper and is the
 *    standard NTC expression.  Scattering is isotropic (VHS) or, with a
 *    VSS exponent alpha != 1, Bird's variable soft sphere deflection law
 *    (section 2.1 names the VSS model).
 *  - Rotational energy (paper section 2.1, eq. dsmc_particle_state and
 *    eq. inelastic_probability) for a gas with two rotational degrees of
 *    freedom: every particle carries I_r, drawn from the equilibrium
 *    distribution at the local temperature when it is created (fill,
 *    inflow) or re-emitted by a diffuse wall; after an accepted collision
 *    each partner in turn exchanges energy with the pair's relative
 *    translation with probability P_inelastic (Borgnakke-Larsen, applied
 *    particle by particle); the cells also sum I_r and v I_r (rotational
 *    temperature and heat flux of eq. dsmc_temperatures).
 *  - Cell sampling: eq. (dsmc_temperatures); the exponential moving average
 *    eq. (exponential_average_moments_ch3) and the steady average
 *    eq. (steady_average_moments_ch3) of section 3.1; cells in local
 *    accumulation (section 3.2) average cumulatively.
 *  - The geometry, random-number and operation-order conventions of this
 *    file are fixed, so that an independent implementation can agree
 *    bit-for-bit on integer outcomes (the exit test's dot products and the
 *    free-flight advance use fused multiply-adds, the only contraction).
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle_internal.h"

static char g_err[512];
const char* oracle_last_error(void) { return g_err; }
static void set_err(const char* m) { snprintf(g_err, sizeof g_err, "%s", m); }

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11).                               */
/* ------------------------------------------------------------------ */
void oracle_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(const osim* s, uint32_t subject, uint32_t step, uint32_t purpose, uint64_t block,
                 uint32_t out[4]) {
    uint32_t ctr[4] = {subject, step, (purpose << 24) | (uint32_t)(block & 0xFFFFFFu),
                       (uint32_t)(block >> 24)};
    uint32_t key[2] = {s->seed, s->case_id};
    oracle_philox(ctr, key, out);
}

/* uniform in (0,1): 52 bits k, (k + 1/2) 2^-52 */
static double u01(uint32_t a, uint32_t b) {
    uint64_t k = ((uint64_t)(a >> 6) << 26) | (uint64_t)(b >> 6);
    return ((double)k + 0.5) * 0x1p-52;
}

/* integer in [0, n) by multiply-shift */
static uint32_t pick(uint32_t r, uint32_t n) { return (uint32_t)(((uint64_t)r * n) >> 32); }

static void box_muller(double u1, double u2, double* g1, double* g2) {
    double r = sqrt(-2.0 * log(u1));
    double a = TWO_PI * u2;
    *g1 = r * cos(a);
    *g2 = r * sin(a);
}

static double to_store(const osim* s, double x) { return s->vel_fp32 ? (double)(float)x : x; }

/* ------------------------------------------------------------------ */
/* Mesh preprocessing                                                   */
/* ------------------------------------------------------------------ */
typedef struct { int k[3]; int tet, lf; } fkey;

static int cmp_fkey(const void* a, const void* b) {
    const fkey* x = (const fkey*)a; const fkey* y = (const fkey*)b;
    for (int i = 0; i < 3; ++i) {
        if (x->k[i] < y->k[i]) return -1;
        if (x->k[i] > y->k[i]) return 1;
    }
    if (x->tet != y->tet) return x->tet < y->tet ? -1 : 1;
    return x->lf < y->lf ? -1 : (x->lf > y->lf);
}

static void sort3(int* a) {
    int t;
    if (a[0] > a[1]) { t = a[0]; a[0] = a[1]; a[1] = t; }
    if (a[1] > a[2]) { t = a[1]; a[1] = a[2]; a[2] = t; }
    if (a[0] > a[1]) { t = a[0]; a[0] = a[1]; a[1] = t; }
}

static int cmp3(const int* a, const int* b) {
    for (int i = 0; i < 3; ++i) {
        if (a[i] < b[i]) return -1;
        if (a[i] > b[i]) return 1;
    }
    return 0;
}

/* (b-a) . ((c-a) x (d-a)) */
static double det_tet(const double* a, const double* b, const double* c, const double* d) {
    double bx = b[0] - a[0], by = b[1] - a[1], bz = b[2] - a[2];
    double cx = c[0] - a[0], cy = c[1] - a[1], cz = c[2] - a[2];
    double dx = d[0] - a[0], dy = d[1] - a[1], dz = d[2] - a[2];
    double ex = cy * dz - cz * dy;
    double ey = cz * dx - cx * dz;
    double ez = cx * dy - cy * dx;
    return bx * ex + by * ey + bz * ez;
}

void oracle_destroy(osim* s) {
    if (!s) return;
    void* ptrs[] = {s->xyz, s->tv, s->vol, s->tf_face, s->tf_s, s->tf_nbr, s->tf_nlf, s->fn, s->fd,
                    s->fvert, s->bf_tet, s->bf_lf, s->bf_group, s->bf_partner, s->bf_face,
                    s->bf_nin, s->bf_t1, s->bf_t2, s->bf_area, s->g_kind, s->g_T, s->g_u, s->g_n,
                    s->g_shift, s->in_mean, s->in_a, s->in_beta, s->in_sig, s->in_ut1, s->in_ut2,
                    s->x, s->v, s->cell, s->pid, s->smax, s->ncand, s->nacc, s->start, s->acc,
                    s->ewma, s->ewma_m, s->local_acc, s->inst, s->cen, s->fcen, s->fnu, s->farea,
                    s->lsq, s->mprev, s->surf, s->rsurf, s->ir, s->racc, s->rewma, s->rinst};
    for (size_t i = 0; i < sizeof ptrs / sizeof ptrs[0]; ++i) free(ptrs[i]);
    free(s);
}

osim* oracle_create(int nv, const double* xyz, int nt, const int* tet,
                    int nb, const int* bface, const int* bgroup, const int* bpartner,
                    int ng, const int* g_kind, const double* g_T, const double* g_u,
                    const double* g_n, const double* g_shift,
                    double mass, double d_ref, double omega, double T_ref,
                    double F_N, double dt, uint32_t seed, uint32_t case_id,
                    int vel_fp32, int n_ss, int n_a, int ewma_on) {
    osim* s = (osim*)calloc(1, sizeof(osim));
    s->m = mass; s->dref = d_ref; s->omega = omega; s->Tref = T_ref;
    s->alpha = 1.0;
    s->FN = F_N; s->dt = dt; s->seed = seed; s->case_id = case_id;
    s->vel_fp32 = vel_fp32; s->n_ss = n_ss; s->n_a = n_a; s->ewma_on = ewma_on;
    s->nv = nv; s->nt = nt; s->nb = nb; s->ng = ng;

    /* VHS: sigma_T c_r = K (c_r^2)^(1-omega), m_r = m/2 */
    double mr = mass / 2.0;
    s->K = ((M_PI * d_ref) * d_ref) * pow(((2.0 * KB) * T_ref) / mr, omega - 0.5) / tgamma(2.5 - omega);
    s->ex = 1.0 - omega;

    s->xyz = (double*)malloc(sizeof(double) * 3 * (size_t)nv);
    memcpy(s->xyz, xyz, sizeof(double) * 3 * (size_t)nv);
    s->tv = (int*)malloc(sizeof(int) * 4 * (size_t)nt);
    s->vol = (double*)malloc(sizeof(double) * (size_t)nt);
    for (int t = 0; t < nt; ++t) {
        int* q = s->tv + 4 * t;
        for (int i = 0; i < 4; ++i) {
            q[i] = tet[4 * t + i];
            if (q[i] < 0 || q[i] >= nv) { set_err("tet vertex out of range"); oracle_destroy(s); return NULL; }
        }
        double det = det_tet(xyz + 3 * q[0], xyz + 3 * q[1], xyz + 3 * q[2], xyz + 3 * q[3]);
        if (det < 0) { int tmp = q[2]; q[2] = q[3]; q[3] = tmp; det = -det; }
        if (!(det > 0)) { set_err("degenerate tet"); oracle_destroy(s); return NULL; }
        s->vol[t] = det / 6.0;
    }

    /* unique faces by sorted vertex triple */
    size_t n4 = 4 * (size_t)nt;
    fkey* keys = (fkey*)malloc(sizeof(fkey) * n4);
    for (int t = 0; t < nt; ++t)
        for (int f = 0; f < 4; ++f) {
            fkey* k = keys + 4 * t + f;
            int j = 0;
            for (int i = 0; i < 4; ++i)
                if (i != f) k->k[j++] = s->tv[4 * t + i];
            sort3(k->k);
            k->tet = t; k->lf = f;
        }
    qsort(keys, n4, sizeof(fkey), cmp_fkey);
    s->tf_face = (int*)malloc(sizeof(int) * n4);
    s->tf_s = (double*)malloc(sizeof(double) * n4);
    s->tf_nbr = (int*)malloc(sizeof(int) * n4);
    s->tf_nlf = (int*)malloc(sizeof(int) * n4);
    s->fn = (double*)malloc(sizeof(double) * 3 * n4);
    s->fd = (double*)malloc(sizeof(double) * n4);
    s->fvert = (int*)malloc(sizeof(int) * 3 * n4);
    int nf = 0;
    int next = 0;
    for (size_t i = 0; i < n4;) {
        size_t j = i + 1;
        while (j < n4 && cmp3(keys[j].k, keys[i].k) == 0) ++j;
        if (j - i > 2) { set_err("face shared by more than two tets"); free(keys); oracle_destroy(s); return NULL; }
        int id = nf++;
        const double* p = xyz + 3 * keys[i].k[0];
        const double* q = xyz + 3 * keys[i].k[1];
        const double* r = xyz + 3 * keys[i].k[2];
        double ax = q[0] - p[0], ay = q[1] - p[1], az = q[2] - p[2];
        double bx = r[0] - p[0], by = r[1] - p[1], bz = r[2] - p[2];
        double nx = ay * bz - az * by;
        double ny = az * bx - ax * bz;
        double nz = ax * by - ay * bx;
        s->fn[3 * id] = nx; s->fn[3 * id + 1] = ny; s->fn[3 * id + 2] = nz;
        s->fd[id] = nx * p[0] + ny * p[1] + nz * p[2];
        memcpy(s->fvert + 3 * id, keys[i].k, sizeof(int) * 3);
        for (size_t e = i; e < j; ++e) {
            int t = keys[e].tet, f = keys[e].lf;
            const double* o = xyz + 3 * s->tv[4 * t + f];
            double test = (nx * o[0] + ny * o[1] + nz * o[2]) - s->fd[id];
            s->tf_face[4 * t + f] = id;
            s->tf_s[4 * t + f] = test < 0 ? 1.0 : -1.0;
            if (j - i == 2) {
                const fkey* other = &keys[e == i ? i + 1 : i];
                s->tf_nbr[4 * t + f] = other->tet;
                s->tf_nlf[4 * t + f] = other->lf;
            } else {
                s->tf_nbr[4 * t + f] = -1 - 0x3fffffff; /* unmatched marker, fixed below */
                s->tf_nlf[4 * t + f] = -1;
                ++next;
            }
        }
        i = j;
    }
    s->nf = nf;
    free(keys);

    /* boundary faces */
    if (next != nb) { set_err("boundary face count does not match exterior faces"); oracle_destroy(s); return NULL; }
    s->bf_tet = (int*)malloc(sizeof(int) * (size_t)(nb ? nb : 1));
    s->bf_lf = (int*)malloc(sizeof(int) * (size_t)(nb ? nb : 1));
    s->bf_group = (int*)malloc(sizeof(int) * (size_t)(nb ? nb : 1));
    s->bf_partner = (int*)malloc(sizeof(int) * (size_t)(nb ? nb : 1));
    s->bf_face = (int*)malloc(sizeof(int) * (size_t)(nb ? nb : 1));
    s->bf_nin = (double*)malloc(sizeof(double) * 3 * (size_t)(nb ? nb : 1));
    s->bf_t1 = (double*)malloc(sizeof(double) * 3 * (size_t)(nb ? nb : 1));
    s->bf_t2 = (double*)malloc(sizeof(double) * 3 * (size_t)(nb ? nb : 1));
    s->bf_area = (double*)malloc(sizeof(double) * (size_t)(nb ? nb : 1));
    {
        /* index exterior tet-faces by their sorted triple */
        fkey* ext = (fkey*)malloc(sizeof(fkey) * (size_t)(nb ? nb : 1));
        int ne = 0;
        for (int t = 0; t < nt; ++t)
            for (int f = 0; f < 4; ++f)
                if (s->tf_nbr[4 * t + f] == -1 - 0x3fffffff) {
                    memcpy(ext[ne].k, s->fvert + 3 * s->tf_face[4 * t + f], sizeof(int) * 3);
                    ext[ne].tet = t; ext[ne].lf = f; ++ne;
                }
        qsort(ext, (size_t)ne, sizeof(fkey), cmp_fkey);
        for (int b = 0; b < nb; ++b) {
            int k[3] = {bface[3 * b], bface[3 * b + 1], bface[3 * b + 2]};
            sort3(k);
            int lo = 0, hi = ne - 1, found = -1;
            while (lo <= hi) {
                int mid = (lo + hi) / 2;
                int c = cmp3(ext[mid].k, k);
                if (c == 0) { found = mid; break; }
                if (c < 0) lo = mid + 1; else hi = mid - 1;
            }
            if (found < 0 || bgroup[b] < 0 || bgroup[b] >= ng) {
                set_err("boundary triangle matches no exterior face (or bad group)");
                free(ext); oracle_destroy(s); return NULL;
            }
            int t = ext[found].tet, f = ext[found].lf;
            if (s->tf_nbr[4 * t + f] != -1 - 0x3fffffff) {
                set_err("boundary triangle listed twice"); free(ext); oracle_destroy(s); return NULL;
            }
            s->tf_nbr[4 * t + f] = -1 - b;
            s->bf_tet[b] = t; s->bf_lf[b] = f; s->bf_group[b] = bgroup[b];
            s->bf_partner[b] = bpartner ? bpartner[b] : -1;
            int id = s->tf_face[4 * t + f];
            s->bf_face[b] = id;
            const double* n = s->fn + 3 * id;
            double sg = s->tf_s[4 * t + f];
            double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
            s->bf_area[b] = 0.5 * nn;
            double* nin = s->bf_nin + 3 * b;
            for (int i = 0; i < 3; ++i) nin[i] = (-sg * n[i]) / nn;
            const double* p = xyz + 3 * s->fvert[3 * id];
            const double* q = xyz + 3 * s->fvert[3 * id + 1];
            double ax = q[0] - p[0], ay = q[1] - p[1], az = q[2] - p[2];
            double al = sqrt(ax * ax + ay * ay + az * az);
            double* t1 = s->bf_t1 + 3 * b;
            t1[0] = ax / al; t1[1] = ay / al; t1[2] = az / al;
            double* t2 = s->bf_t2 + 3 * b;
            t2[0] = nin[1] * t1[2] - nin[2] * t1[1];
            t2[1] = nin[2] * t1[0] - nin[0] * t1[2];
            t2[2] = nin[0] * t1[1] - nin[1] * t1[0];
        }
        free(ext);
    }

    s->g_kind = (int*)malloc(sizeof(int) * (size_t)(ng ? ng : 1));
    s->g_T = (double*)malloc(sizeof(double) * (size_t)(ng ? ng : 1));
    s->g_u = (double*)malloc(sizeof(double) * 3 * (size_t)(ng ? ng : 1));
    s->g_n = (double*)malloc(sizeof(double) * (size_t)(ng ? ng : 1));
    s->g_shift = (double*)malloc(sizeof(double) * 3 * (size_t)(ng ? ng : 1));
    for (int g = 0; g < ng; ++g) {
        s->g_kind[g] = g_kind[g]; s->g_T[g] = g_T[g]; s->g_n[g] = g_n ? g_n[g] : 0.0;
        for (int i = 0; i < 3; ++i) {
            s->g_u[3 * g + i] = g_u[3 * g + i];
            s->g_shift[3 * g + i] = g_shift ? g_shift[3 * g + i] : 0.0;
        }
    }
    for (int b = 0; b < nb; ++b)
        if (s->g_kind[s->bf_group[b]] == O_BC_PERIODIC) {
            int pb = s->bf_partner[b];
            if (pb < 0 || pb >= nb) { set_err("periodic face without partner"); oracle_destroy(s); return NULL; }
        }

    /* inflow face constants */
    s->in_mean = (double*)calloc((size_t)(nb ? nb : 1), sizeof(double));
    s->in_a = (double*)calloc((size_t)(nb ? nb : 1), sizeof(double));
    s->in_beta = (double*)calloc((size_t)(nb ? nb : 1), sizeof(double));
    s->in_sig = (double*)calloc((size_t)(nb ? nb : 1), sizeof(double));
    s->in_ut1 = (double*)calloc((size_t)(nb ? nb : 1), sizeof(double));
    s->in_ut2 = (double*)calloc((size_t)(nb ? nb : 1), sizeof(double));
    for (int b = 0; b < nb; ++b) {
        int g = s->bf_group[b];
        if (s->g_kind[g] != O_BC_INFLOW) continue;
        double T = s->g_T[g];
        const double* u = s->g_u + 3 * g;
        const double* nin = s->bf_nin + 3 * b;
        const double* t1 = s->bf_t1 + 3 * b;
        const double* t2 = s->bf_t2 + 3 * b;
        double beta = sqrt(((2.0 * KB) * T) / mass);
        double sig = sqrt((KB * T) / mass);
        double un = u[0] * nin[0] + u[1] * nin[1] + u[2] * nin[2];
        double a = un / beta;
        double f1 = sqrt((KB * T) / ((2.0 * M_PI) * mass));
        double f2 = exp(-(a * a)) + (SQRT_PI * a) * (1.0 + erf(a));
        double flux = (s->g_n[g] * f1) * f2;
        s->in_mean[b] = ((flux * s->bf_area[b]) * dt) / F_N;
        s->in_a[b] = a; s->in_beta[b] = beta; s->in_sig[b] = sig;
        s->in_ut1[b] = u[0] * t1[0] + u[1] * t1[1] + u[2] * t1[2];
        s->in_ut2[b] = u[0] * t2[0] + u[1] * t2[1] + u[2] * t2[2];
    }

    size_t ntz = (size_t)nt;
    s->smax = (double*)calloc(ntz, sizeof(double));
    s->ncand = (int*)calloc(ntz, sizeof(int));
    s->nacc = (int*)calloc(ntz, sizeof(int));
    s->start = (int64_t*)calloc(ntz + 1, sizeof(int64_t));
    s->acc = (double*)calloc(ntz * NMOM, sizeof(double));
    s->ewma = (double*)calloc(ntz * NMOM, sizeof(double));
    s->inst = (double*)calloc(ntz * NMOM, sizeof(double));
    s->ewma_m = (int*)calloc(ntz, sizeof(int));
    s->local_acc = (unsigned char*)calloc(ntz, 1);
    s->cap = 0;
    return s;
}

static void reserve(osim* s, int64_t need) {
    if (need <= s->cap) return;
    int64_t c = s->cap ? s->cap : 1024;
    while (c < need) c *= 2;
    s->x = (double*)realloc(s->x, sizeof(double) * 3 * (size_t)c);
    s->v = (double*)realloc(s->v, sizeof(double) * 3 * (size_t)c);
    s->cell = (int*)realloc(s->cell, sizeof(int) * (size_t)c);
    s->pid = (uint32_t*)realloc(s->pid, sizeof(uint32_t) * (size_t)c);
    if (s->dr) s->ir = (double*)realloc(s->ir, sizeof(double) * (size_t)c);
    s->cap = c;
}

/* ------------------------------------------------------------------ */
/* Sort by (cell, pid), dropping deleted particles (cell < 0).          */
/* ------------------------------------------------------------------ */
static const osim* g_sort_sim;
static int cmp_particle(const void* a, const void* b) {
    int64_t i = *(const int64_t*)a, j = *(const int64_t*)b;
    const osim* s = g_sort_sim;
    if (s->cell[i] != s->cell[j]) return s->cell[i] < s->cell[j] ? -1 : 1;
    if (s->pid[i] != s->pid[j]) return s->pid[i] < s->pid[j] ? -1 : 1;
    return 0;
}

static void stage_sort(osim* s) {
    int64_t n = 0;
    int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(s->np ? s->np : 1));
    for (int64_t i = 0; i < s->np; ++i)
        if (s->cell[i] >= 0) idx[n++] = i;
    g_sort_sim = s;
    qsort(idx, (size_t)n, sizeof(int64_t), cmp_particle);
    double* x = (double*)malloc(sizeof(double) * 3 * (size_t)(s->cap ? s->cap : 1));
    double* v = (double*)malloc(sizeof(double) * 3 * (size_t)(s->cap ? s->cap : 1));
    int* c = (int*)malloc(sizeof(int) * (size_t)(s->cap ? s->cap : 1));
    uint32_t* p = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(s->cap ? s->cap : 1));
    double* ir = s->dr ? (double*)malloc(sizeof(double) * (size_t)(s->cap ? s->cap : 1)) : NULL;
    for (int64_t k = 0; k < n; ++k) {
        int64_t i = idx[k];
        memcpy(x + 3 * k, s->x + 3 * i, sizeof(double) * 3);
        memcpy(v + 3 * k, s->v + 3 * i, sizeof(double) * 3);
        c[k] = s->cell[i]; p[k] = s->pid[i];
        if (ir) ir[k] = s->ir[i];
    }
    free(s->x); free(s->v); free(s->cell); free(s->pid); free(idx);
    s->x = x; s->v = v; s->cell = c; s->pid = p; s->np = n;
    if (ir) { free(s->ir); s->ir = ir; }
    for (int t = 0; t <= s->nt; ++t) s->start[t] = 0;
    for (int64_t k = 0; k < n; ++k) s->start[s->cell[k] + 1]++;
    for (int t = 0; t < s->nt; ++t) s->start[t + 1] += s->start[t];
}

/* ------------------------------------------------------------------ */
/* Initial fill                                                        */
/* ------------------------------------------------------------------ */
int oracle_init_fill(osim* s, double n0, double T0, const double* u0) {
    int64_t total = 0;
    int* cnt = (int*)malloc(sizeof(int) * (size_t)s->nt);
    uint32_t w[4];
    for (int t = 0; t < s->nt; ++t) {
        double mean = (n0 * s->vol[t]) / s->FN;
        draw(s, (uint32_t)t, 0, P_INITCOUNT, 0, w);
        cnt[t] = (int)floor(mean + u01(w[0], w[1]));
        total += cnt[t];
    }
    reserve(s, total);
    double sig = sqrt((KB * T0) / s->m);
    int64_t k = 0;
    for (int t = 0; t < s->nt; ++t) {
        const int* q = s->tv + 4 * t;
        for (int j = 0; j < cnt[t]; ++j, ++k) {
            uint32_t id = (uint32_t)k;
            double u[8];
            for (int b = 0; b < 4; ++b) {
                draw(s, id, 0, P_INIT, (uint64_t)b, w);
                u[2 * b] = u01(w[0], w[1]);
                u[2 * b + 1] = u01(w[2], w[3]);
            }
            double a = u[0], b = u[1], c = u[2], tmp;
            if (a > b) { tmp = a; a = b; b = tmp; }
            if (b > c) { tmp = b; b = c; c = tmp; }
            if (a > b) { tmp = a; a = b; b = tmp; }
            double wts[4] = {a, b - a, c - b, 1.0 - c};
            for (int i = 0; i < 3; ++i) {
                double xi = wts[0] * s->xyz[3 * q[0] + i];
                xi = xi + wts[1] * s->xyz[3 * q[1] + i];
                xi = xi + wts[2] * s->xyz[3 * q[2] + i];
                xi = xi + wts[3] * s->xyz[3 * q[3] + i];
                s->x[3 * k + i] = xi;
            }
            double g1, g2, g3, g4;
            box_muller(u[3], u[4], &g1, &g2);
            box_muller(u[5], u[6], &g3, &g4);
            s->v[3 * k] = to_store(s, u0[0] + sig * g1);
            s->v[3 * k + 1] = to_store(s, u0[1] + sig * g2);
            s->v[3 * k + 2] = to_store(s, u0[2] + sig * g3);
            s->cell[k] = t;
            s->pid[k] = id;
            if (s->dr) {
                /* two rotational degrees of freedom: exponential with mean k T0 */
                draw(s, id, 0, P_INIT, 4, w);
                s->ir[k] = -(KB * T0) * log(u01(w[0], w[1]));
            }
        }
    }
    free(cnt);
    s->np = total;
    s->next_pid = (uint32_t)total;
    s->step = 0;
    s->ref_n = n0; s->ref_T = T0;
    for (int i = 0; i < 3; ++i) s->ref_u[i] = u0[i];
    /* (sigma c)_max = 2 <sigma_T c_r> at equilibrium T0 */
    double mr = s->m / 2.0;
    double eq = (((2.0 * SQRT_PI) * s->dref) * s->dref) * sqrt(((2.0 * KB) * s->Tref) / mr) *
                pow(T0 / s->Tref, 1.0 - s->omega);
    for (int t = 0; t < s->nt; ++t) s->smax[t] = 2.0 * eq;
    stage_sort(s);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Move: face-to-face tracking with boundary interactions               */
/* ------------------------------------------------------------------ */
/* Surface sampling: one wall interaction at boundary face bf that turned
 * velocity a into b adds the velocity change a - b (the momentum given to
 * the wall per unit mass), the kinetic-energy change (|a|^2 - |b|^2)/2 and
 * one hit to the face's sums, on the steps after n_ss while sampling is on
 * (the stress and heat flux a surface receives: section 5, sphere surface
 * pressure, shear stress and heat flux). */
static void surface_hit(osim* s, int bf, uint32_t step, const double* a, const double* b, double dI) {
    if (!s->surf_on || (int64_t)step <= (int64_t)s->n_ss) return;
    double* q = s->surf + 5 * (size_t)bf;
    q[0] += a[0] - b[0];
    q[1] += a[1] - b[1];
    q[2] += a[2] - b[2];
    q[3] += 0.5 * ((a[0] * a[0] + a[1] * a[1] + a[2] * a[2]) - (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]));
    q[4] += 1.0;
    /* a rotating gas: the rotational energy the molecule leaves at the wall */
    if (s->rsurf) s->rsurf[bf] += dI;
}

/* n . a with fused multiply-adds, n0 a0 first: the rounding the tracking
 * below uses for its exit test (the paper fixes none). */
static double dot_fused(const double* n, const double* a) {
    return fma(n[2], a[2], fma(n[1], a[1], n[0] * a[0]));
}

/* returns 0 alive, 1 removed through an open boundary, 2 lost */
static int trace(osim* s, double* x, double* v, double* ir, int* cellp, int entry, uint32_t pid, uint32_t step,
                 double t) {
    int c = *cellp;
    int nhop = 0, hits = 0;
    for (;;) {
        int fb = -1;
        double lb = 0.0;
        for (int f = 0; f < 4; ++f) {
            if (f == entry) continue;
            int k = 4 * c + f;
            const double* n = s->fn + 3 * s->tf_face[k];
            double d = s->fd[s->tf_face[k]];
            double sg = s->tf_s[k];
            double den = sg * dot_fused(n, v);
            if (den > 0) {
                double lam = (sg * (d - dot_fused(n, x))) / den;
                if (lam < 0) lam = 0;
                if (fb < 0 || lam < lb) { fb = f; lb = lam; }
            }
        }
        if (fb < 0 || lb >= t) {
            for (int i = 0; i < 3; ++i) x[i] = fma(v[i], t, x[i]);
            break;
        }
        for (int i = 0; i < 3; ++i) x[i] = fma(v[i], lb, x[i]);
        t = t - lb;
        s->hops++;
        if (++nhop > MAX_HOPS) { s->lost++; *cellp = c; return 2; }
        int k = 4 * c + fb;
        int nb = s->tf_nbr[k];
        if (nb >= 0) { c = nb; entry = s->tf_nlf[k]; continue; }
        int bf = -1 - nb;
        int g = s->bf_group[bf];
        switch (s->g_kind[g]) {
        case O_BC_DIFFUSE: {
            uint32_t w[4];
            double u[4];
            draw(s, pid, step, P_WALL, (uint64_t)(2 * hits), w);
            u[0] = u01(w[0], w[1]); u[1] = u01(w[2], w[3]);
            draw(s, pid, step, P_WALL, (uint64_t)(2 * hits + 1), w);
            u[2] = u01(w[0], w[1]); u[3] = u01(w[2], w[3]);
            double Tw = s->g_T[g];
            double beta = sqrt(((2.0 * KB) * Tw) / s->m);
            double sw = sqrt((KB * Tw) / s->m);
            double vn = beta * sqrt(-log(u[0]));
            double g1, g2;
            box_muller(u[1], u[2], &g1, &g2);
            const double* nin = s->bf_nin + 3 * bf;
            const double* t1 = s->bf_t1 + 3 * bf;
            const double* t2 = s->bf_t2 + 3 * bf;
            const double* uw = s->g_u + 3 * g;
            const double vin[3] = {v[0], v[1], v[2]};
            for (int i = 0; i < 3; ++i) {
                double tang = sw * (g1 * t1[i] + g2 * t2[i]);
                v[i] = to_store(s, (vn * nin[i] + tang) + uw[i]);
            }
            /* the re-emitted molecule's rotation is in equilibrium at the wall */
            double inew = ir ? -(KB * Tw) * log(u01(w[2], w[3])) : 0.0;
            surface_hit(s, bf, step, vin, v, ir ? *ir - inew : 0.0);
            if (ir) *ir = inew;
            ++hits;
            s->walls++;
            entry = fb;
            break;
        }
        case O_BC_SPECULAR: {
            const double* n = s->fn + 3 * s->tf_face[k];
            double vn = n[0] * v[0] + n[1] * v[1] + n[2] * v[2];
            double nn = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
            double f2 = 2.0 * (vn / nn);
            const double vin[3] = {v[0], v[1], v[2]};
            for (int i = 0; i < 3; ++i) v[i] = to_store(s, v[i] - f2 * n[i]);
            surface_hit(s, bf, step, vin, v, 0.0);
            s->walls++;
            entry = fb;
            break;
        }
        case O_BC_PERIODIC: {
            int pb = s->bf_partner[bf];
            const double* sh = s->g_shift + 3 * g;
            for (int i = 0; i < 3; ++i) x[i] = x[i] + sh[i];
            c = s->bf_tet[pb];
            entry = s->bf_lf[pb];
            break;
        }
        default: /* inflow and outflow faces remove the particle */
            s->removed++;
            *cellp = c;
            return 1;
        }
    }
    *cellp = c;
    return 0;
}

int oracle_trace_one(osim* s, double* x, double* v, int cell, uint32_t pid, uint32_t step, double t) {
    int c = cell;
    int st = trace(s, x, v, NULL, &c, -1, pid, step, t);
    return st == 0 ? c : -1;
}

static void stage_move(osim* s) {
    for (int64_t i = 0; i < s->np; ++i) {
        if (s->cell[i] < 0) continue;
        int c = s->cell[i];
        int st = trace(s, s->x + 3 * i, s->v + 3 * i, s->dr ? s->ir + i : NULL, &c, -1, s->pid[i], s->step, s->dt);
        s->cell[i] = st == 0 ? c : -1;
    }
}

/* ------------------------------------------------------------------ */
/* Freestream injection                                                 */
/* ------------------------------------------------------------------ */
/* Normal speed ratio z > 0 with density proportional to z exp(-(z-a)^2):
 * rejection from the envelope (a + |w|) exp(-w^2), w = z - a (a > 0), or
 * from the truncated Rayleigh w exp(-w^2), w > -a (a < 0). */
static double flux_normal(const osim* s, double a, uint32_t bf, uint32_t step, uint64_t k) {
    uint32_t w[4];
    if (a == 0.0) {
        draw(s, bf, step, P_INJECT, (k << 6) | 3u, w);
        return sqrt(-log(u01(w[0], w[1])));
    }
    for (int tr = 0; tr < 30; ++tr) {
        double u[4];
        draw(s, bf, step, P_INJECT, (k << 6) | (uint64_t)(3 + 2 * tr), w);
        u[0] = u01(w[0], w[1]); u[1] = u01(w[2], w[3]);
        draw(s, bf, step, P_INJECT, (k << 6) | (uint64_t)(4 + 2 * tr), w);
        u[2] = u01(w[0], w[1]); u[3] = u01(w[2], w[3]);
        if (a > 0) {
            double pa = (a * SQRT_PI) / ((a * SQRT_PI) + 1.0);
            double wv;
            if (u[0] < pa) {
                double g1, g2;
                box_muller(u[1], u[2], &g1, &g2);
                wv = g1 * INV_SQRT2;
            } else {
                double r = sqrt(-log(u[1]));
                wv = u[2] < 0.5 ? r : -r;
            }
            double z = a + wv;
            if (z > 0 && u[3] * (a + fabs(wv)) < z) return z;
        } else {
            double wv = sqrt(a * a - log(u[1]));
            double z = a + wv;
            if (u[3] * wv < z) return z;
        }
    }
    return a > 0 ? a : 0.5;
}

static void stage_inject(osim* s) {
    uint32_t w[4];
    for (int b = 0; b < s->nb; ++b) {
        int g = s->bf_group[b];
        if (s->g_kind[g] != O_BC_INFLOW) continue;
        draw(s, (uint32_t)b, s->step, P_INJCOUNT, 0, w);
        int n = (int)floor(s->in_mean[b] + u01(w[0], w[1]));
        const double* nin = s->bf_nin + 3 * b;
        const double* t1 = s->bf_t1 + 3 * b;
        const double* t2 = s->bf_t2 + 3 * b;
        int fid = s->bf_face[b];
        const double* A = s->xyz + 3 * s->fvert[3 * fid];
        const double* B = s->xyz + 3 * s->fvert[3 * fid + 1];
        const double* C = s->xyz + 3 * s->fvert[3 * fid + 2];
        for (int k = 0; k < n; ++k) {
            uint64_t kb = (uint64_t)k << 6;
            draw(s, (uint32_t)b, s->step, P_INJECT, kb | 0u, w);
            double r1 = u01(w[0], w[1]), r2 = u01(w[2], w[3]);
            if (r1 + r2 > 1.0) { r1 = 1.0 - r1; r2 = 1.0 - r2; }
            draw(s, (uint32_t)b, s->step, P_INJECT, kb | 1u, w);
            double ut = u01(w[0], w[1]);
            draw(s, (uint32_t)b, s->step, P_INJECT, kb | 2u, w);
            double g1, g2;
            box_muller(u01(w[0], w[1]), u01(w[2], w[3]), &g1, &g2);
            double z = flux_normal(s, s->in_a[b], (uint32_t)b, s->step, (uint64_t)k);
            double vn = s->in_beta[b] * z;
            double vt1 = s->in_sig[b] * g1 + s->in_ut1[b];
            double vt2 = s->in_sig[b] * g2 + s->in_ut2[b];
            double x[3], v[3];
            for (int i = 0; i < 3; ++i) {
                x[i] = (A[i] + r1 * (B[i] - A[i])) + r2 * (C[i] - A[i]);
                v[i] = to_store(s, (vn * nin[i] + vt1 * t1[i]) + vt2 * t2[i]);
            }
            uint32_t id = s->next_pid++;
            s->injected++;
            int c = s->bf_tet[b];
            double irot = 0.0;
            if (s->dr) {
                /* freestream rotation in equilibrium at the freestream temperature */
                draw(s, (uint32_t)b, s->step, P_INJECT, kb | 1u, w);
                irot = -(KB * s->g_T[g]) * log(u01(w[2], w[3]));
            }
            int st = trace(s, x, v, s->dr ? &irot : NULL, &c, s->bf_lf[b], id, s->step, ut * s->dt);
            if (st != 0) continue;
            reserve(s, s->np + 1);
            memcpy(s->x + 3 * s->np, x, sizeof x);
            memcpy(s->v + 3 * s->np, v, sizeof v);
            s->cell[s->np] = c;
            s->pid[s->np] = id;
            if (s->dr) s->ir[s->np] = irot;
            s->np++;
        }
    }
}

/* ------------------------------------------------------------------ */
/* NTC collisions, VHS / VSS                                            */
/* ------------------------------------------------------------------ */
/* Post-collision relative velocity g' (|g'| = |g| = c_r) from the two
 * uniform deviates R1 (deflection) and R2 (azimuth).
 * VHS (alpha = 1): g' is isotropic, cos(theta) = 2 R1 - 1 about the x axis,
 * independent of g.
 * VSS (section 2.1 cites Bird 1994 for the model): the deflection chi from g
 * obeys b/d = cos(chi/2)^(1/alpha) with (b/d)^2 uniform, so
 * cos(chi) = 2 R1^(1/alpha) - 1; g' is g turned by chi at azimuth
 * eps = 2 pi R2, in the frame (g/c_r, e1, e2) with
 *   e1 = (0, g_z, -g_y) / g_yz,   e2 = (g_yz^2, -g_x g_y, -g_x g_z) / (c_r g_yz),
 *   g_yz = sqrt(g_y^2 + g_z^2),
 * that is g' = cos(chi) g + sin(chi) c_r (sin(eps) e2 + cos(eps) e1), Bird's
 * rotation written as a frame.  When g_yz = 0 (g along x), e1 = y, e2 = z. */
static void scatter(const osim* s, double gx, double gy, double gz, double cr2, double R1, double R2,
                    double gp[3]) {
    double cr = sqrt(cr2);
    double eps = TWO_PI * R2;
    if (s->alpha == 1.0) {
        double cx = 2.0 * R1 - 1.0;
        double sx = sqrt(1.0 - cx * cx);
        gp[0] = cr * cx;
        gp[1] = cr * (sx * cos(eps));
        gp[2] = cr * (sx * sin(eps));
        return;
    }
    double cc = 2.0 * pow(R1, 1.0 / s->alpha) - 1.0;
    double sc = sqrt(1.0 - cc * cc);
    double ce = cos(eps), se = sin(eps);
    double gyz = sqrt(gy * gy + gz * gz);
    double e1[3], e2[3];
    if (gyz > 0.0) {
        e1[0] = 0.0; e1[1] = gz / gyz; e1[2] = -gy / gyz;
        e2[0] = gyz / cr; e2[1] = -(gx * gy) / (cr * gyz); e2[2] = -(gx * gz) / (cr * gyz);
    } else {
        e1[0] = 0.0; e1[1] = 1.0; e1[2] = 0.0;
        e2[0] = 0.0; e2[1] = 0.0; e2[2] = 1.0;
    }
    double g[3] = {gx, gy, gz};
    for (int d = 0; d < 3; ++d) gp[d] = cc * g[d] + (sc * cr) * (se * e2[d] + ce * e1[d]);
}

static void stage_collide(osim* s) {
    uint32_t w[4];
    for (int c = 0; c < s->nt; ++c) {
        int64_t a = s->start[c];
        int N = (int)(s->start[c + 1] - a);
        s->ncand[c] = 0; s->nacc[c] = 0;
        if (N < 2) continue;
        double* v = s->v + 3 * a;
        double smax = s->smax[c];
        draw(s, (uint32_t)c, s->step, P_NTCCOUNT, 0, w);
        double Nd = (double)N;
        double mean = ((((0.5 * Nd) * (Nd - 1.0)) * s->FN) * smax) * s->dt / s->vol[c];
        int M = (int)floor(mean + u01(w[0], w[1]));
        double seen = 0.0;
        int acc = 0;
        for (int k = 0; k < M; ++k) {
            draw(s, (uint32_t)c, s->step, P_PAIR, (uint64_t)k, w);
            uint32_t i = pick(w[0], (uint32_t)N);
            uint32_t j = pick(w[1], (uint32_t)(N - 1));
            if (j >= i) ++j;
            double U = u01(w[2], w[3]);
            double* vi = v + 3 * i;
            double* vj = v + 3 * j;
            double gx = vi[0] - vj[0], gy = vi[1] - vj[1], gz = vi[2] - vj[2];
            double cr2 = gx * gx + gy * gy + gz * gz;
            double sc = s->K * pow(cr2, s->ex);
            if (sc > seen) seen = sc;
            if (!(U < sc / smax)) continue;
            ++acc;
            draw(s, (uint32_t)c, s->step, P_SCATTER, (uint64_t)k, w);
            double R1 = u01(w[0], w[1]), R2 = u01(w[2], w[3]);
            double gp[3];
            if (s->dr) {
                /* Borgnakke-Larsen, particle by particle: with probability
                 * P_inelastic a partner's rotational energy and the relative
                 * translational energy E_t = m_r c_r^2 / 2 (m_r = m/2) are
                 * pooled into E_c and split again; the translational share
                 * E_t / E_c of a molecule with two rotational degrees of
                 * freedom follows Beta(5/2 - omega, 1), whose inverse
                 * distribution function gives E_t = E_c R^(1/(5/2 - omega)). */
                double* Ii = s->ir + a + i;
                double* Ij = s->ir + a + j;
                double Et = (0.25 * s->m) * cr2;
                double ex = 1.0 / (2.5 - s->omega);
                int inel = 0;
                uint32_t wi[4];
                draw(s, (uint32_t)c, s->step, P_INELASTIC_I, (uint64_t)k, wi);
                if (u01(wi[0], wi[1]) < s->pinel) {
                    double Ec = Et + *Ii;
                    Et = Ec * pow(u01(wi[2], wi[3]), ex);
                    *Ii = Ec - Et;
                    inel = 1;
                }
                draw(s, (uint32_t)c, s->step, P_INELASTIC_J, (uint64_t)k, wi);
                if (u01(wi[0], wi[1]) < s->pinel) {
                    double Ec = Et + *Ij;
                    Et = Ec * pow(u01(wi[2], wi[3]), ex);
                    *Ij = Ec - Et;
                    inel = 1;
                }
                if (inel) {
                    /* the relative velocity keeps its direction (the VSS
                     * deflection is taken from it) and takes the new speed */
                    double cr2n = (4.0 * Et) / s->m;
                    double f = sqrt(cr2n / cr2);
                    scatter(s, gx * f, gy * f, gz * f, cr2n, R1, R2, gp);
                } else {
                    scatter(s, gx, gy, gz, cr2, R1, R2, gp);
                }
            } else {
                scatter(s, gx, gy, gz, cr2, R1, R2, gp);
            }
            for (int d = 0; d < 3; ++d) {
                double cm = 0.5 * (vi[d] + vj[d]);
                double hg = 0.5 * gp[d];
                vi[d] = to_store(s, cm + hg);
                vj[d] = to_store(s, cm - hg);
            }
        }
        if (seen > smax) s->smax[c] = seen;
        s->ncand[c] = M;
        s->nacc[c] = acc;
    }
}

/* ------------------------------------------------------------------ */
/* Sampling: moment sums, steady accumulator and moving average         */
/* ------------------------------------------------------------------ */
static void stage_sample(osim* s) {
    int steady = (int64_t)s->step > (int64_t)s->n_ss;
    for (int c = 0; c < s->nt; ++c) {
        double S[NMOM], Rs[NROT];
        for (int k = 0; k < NMOM; ++k) S[k] = 0.0;
        for (int k = 0; k < NROT; ++k) Rs[k] = 0.0;
        for (int64_t p = s->start[c]; p < s->start[c + 1]; ++p) {
            double vx = s->v[3 * p], vy = s->v[3 * p + 1], vz = s->v[3 * p + 2];
            double v2 = vx * vx + vy * vy + vz * vz;
            S[0] += 1.0;
            S[1] += vx; S[2] += vy; S[3] += vz;
            S[4] += vx * vx; S[5] += vy * vy; S[6] += vz * vz;
            S[7] += vx * vy; S[8] += vx * vz; S[9] += vy * vz;
            S[10] += vx * v2; S[11] += vy * v2; S[12] += vz * v2;
            if (s->dr) {
                double I = s->ir[p];
                Rs[0] += I;
                Rs[1] += vx * I; Rs[2] += vy * I; Rs[3] += vz * I;
            }
        }
        memcpy(s->inst + NMOM * (size_t)c, S, sizeof S);
        if (s->dr) memcpy(s->rinst + NROT * (size_t)c, Rs, sizeof Rs);
        if (steady) {
            for (int k = 0; k < NMOM; ++k) s->acc[NMOM * (size_t)c + k] += S[k];
            if (s->dr)
                for (int k = 0; k < NROT; ++k) s->racc[NROT * (size_t)c + k] += Rs[k];
        }
        if (s->ewma_on) {
            int m = ++s->ewma_m[c];
            int n = (s->local_acc[c] || m < s->n_a) ? m : s->n_a;
            double wo = (double)(n - 1) / (double)n;
            double wn = 1.0 / (double)n;
            for (int k = 0; k < NMOM; ++k) {
                double* e = s->ewma + NMOM * (size_t)c + k;
                *e = wo * *e + wn * S[k];
            }
            if (s->dr)
                for (int k = 0; k < NROT; ++k) {
                    double* e = s->rewma + NROT * (size_t)c + k;
                    *e = wo * *e + wn * Rs[k];
                }
        }
    }
    if (steady) s->n_steady++;
}

/* ------------------------------------------------------------------ */
int oracle_step_stages(osim* s, int mask) {
    s->step++;
    if (mask & O_STAGE_MOVE) stage_move(s);
    if (mask & O_STAGE_INJECT) stage_inject(s);
    if (mask & O_STAGE_SORT) stage_sort(s);
    if (mask & O_STAGE_COLLIDE) stage_collide(s);
    if (mask & O_STAGE_SAMPLE) stage_sample(s);
    return 0;
}

int oracle_step(osim* s, int n) {
    for (int i = 0; i < n; ++i) oracle_step_stages(s, 31);
    return 0;
}

int64_t oracle_num_particles(const osim* s) { return s->np; }

void oracle_get_particles(const osim* s, double* x, double* v, int* cell, uint32_t* pid) {
    if (x) memcpy(x, s->x, sizeof(double) * 3 * (size_t)s->np);
    if (v) memcpy(v, s->v, sizeof(double) * 3 * (size_t)s->np);
    if (cell) memcpy(cell, s->cell, sizeof(int) * (size_t)s->np);
    if (pid) memcpy(pid, s->pid, sizeof(uint32_t) * (size_t)s->np);
}

int oracle_set_particles(osim* s, int64_t np, const double* x, const double* v, const int* cell,
                         const uint32_t* pid, uint32_t step, uint32_t next_pid, const double* ir) {
    reserve(s, np);
    for (int64_t i = 0; i < np; ++i)
        if (cell[i] < 0 || cell[i] >= s->nt) { set_err("particle cell out of range"); return -1; }
    if (s->dr)
        for (int64_t i = 0; i < np; ++i) s->ir[i] = ir ? ir[i] : 0.0;
    memcpy(s->x, x, sizeof(double) * 3 * (size_t)np);
    for (int64_t i = 0; i < 3 * np; ++i) s->v[i] = to_store(s, v[i]);
    memcpy(s->cell, cell, sizeof(int) * (size_t)np);
    memcpy(s->pid, pid, sizeof(uint32_t) * (size_t)np);
    s->np = np;
    s->step = step;
    s->next_pid = next_pid;
    stage_sort(s);
    return 0;
}

/* Rotational degrees of freedom (0 or 2) and rotational collision number;
 * the inelastic probability is eq. (inelastic_probability) with the
 * species' VSS exponent and viscosity index (call after oracle_set_alpha
 * and before the fill). */
int oracle_set_rotation(osim* s, int dr, double zr) {
    if (!(dr == 0 || dr == 2) || (dr && !(zr > 0.0))) {
        set_err("rotational degrees of freedom must be 0 or 2, with a positive collision number");
        return -1;
    }
    s->dr = dr;
    s->zr = zr;
    double a = s->alpha, w = s->omega;
    s->pinel = dr ? ((a * (5.0 - 2.0 * w)) * (7.0 - 2.0 * w)) / ((((5.0 * (a + 1.0)) * (a + 2.0))) * zr) : 0.0;
    /* nitrogen's heat-flux relaxation matrix until set otherwise */
    s->a_heat[0] = 0.786; s->a_heat[1] = -0.201; s->a_heat[2] = -0.059; s->a_heat[3] = 0.842;
    if (dr) {
        size_t ntz = (size_t)s->nt;
        s->ir = (double*)realloc(s->ir, sizeof(double) * (size_t)(s->cap ? s->cap : 1));
        for (int64_t i = 0; i < s->cap; ++i) s->ir[i] = 0.0;
        free(s->racc); free(s->rewma); free(s->rinst);
        s->racc = (double*)calloc(ntz * NROT, sizeof(double));
        s->rewma = (double*)calloc(ntz * NROT, sizeof(double));
        s->rinst = (double*)calloc(ntz * NROT, sizeof(double));
    }
    return 0;
}

double oracle_inelastic_probability(const osim* s) { return s->pinel; }

void oracle_get_rotation(const osim* s, double* ir) {
    if (s->dr && ir) memcpy(ir, s->ir, sizeof(double) * (size_t)s->np);
}

/* Rotational sums out[nt][4] = sum I_r, sum v_i I_r of an accumulator
 * (0 steady, 1 moving average, 2 last step). */
void oracle_get_rot_sums(const osim* s, int which, double* out) {
    const double* src = which == 0 ? s->racc : which == 1 ? s->rewma : s->rinst;
    if (s->dr) memcpy(out, src, sizeof(double) * NROT * (size_t)s->nt);
}

/* Rotational temperature and heat flux out[nt][4] (eq. dsmc_temperatures):
 * T_r = 2 <I_r> / (d_r k), q_r,i = (N_eff / V) sum (v_i - u_i) I_r per
 * sample; NaN where the cell has no samples. */
void oracle_rot_fields(const osim* s, int which, double* out) {
    const double* S = which == 0 ? s->acc : which == 1 ? s->ewma : s->inst;
    const double* R = which == 0 ? s->racc : which == 1 ? s->rewma : s->rinst;
    double ns = which == 0 ? (double)s->n_steady : 1.0;
    for (int c = 0; c < s->nt; ++c) {
        const double* a = S + NMOM * (size_t)c;
        const double* r = R + NROT * (size_t)c;
        double* o = out + 4 * (size_t)c;
        if (!s->dr || !(a[0] > 0) || !(ns > 0)) {
            for (int k = 0; k < 4; ++k) o[k] = NAN;
            continue;
        }
        o[0] = (2.0 * (r[0] / a[0])) / ((double)s->dr * KB);
        double f = s->FN / (s->vol[c] * ns);
        for (int i = 0; i < 3; ++i) o[1 + i] = f * (r[1 + i] - (a[1 + i] / a[0]) * r[0]);
    }
}

int oracle_set_alpha(osim* s, double alpha) {
    if (!(alpha > 0.0)) {
        set_err("alpha must be positive");
        return -1;
    }
    s->alpha = alpha;
    return 0;
}

void oracle_get_smax(const osim* s, double* out) { memcpy(out, s->smax, sizeof(double) * (size_t)s->nt); }
void oracle_set_smax(osim* s, const double* in) { memcpy(s->smax, in, sizeof(double) * (size_t)s->nt); }
uint32_t oracle_step_index(const osim* s) { return s->step; }

int oracle_surface_sampling(osim* s, int on) {
    if (on) {
        if (!s->surf) s->surf = (double*)malloc(sizeof(double) * 5 * (size_t)(s->nb ? s->nb : 1));
        if (!s->surf) { set_err("out of memory"); return -1; }
        memset(s->surf, 0, sizeof(double) * 5 * (size_t)(s->nb ? s->nb : 1));
        if (s->dr) {
            if (!s->rsurf) s->rsurf = (double*)malloc(sizeof(double) * (size_t)(s->nb ? s->nb : 1));
            if (!s->rsurf) { set_err("out of memory"); return -1; }
            memset(s->rsurf, 0, sizeof(double) * (size_t)(s->nb ? s->nb : 1));
        }
        s->surf_on = 1;
        s->surf_from = s->step;
        s->surf_to = -1;
    } else if (s->surf_on) {
        s->surf_on = 0;
        s->surf_to = s->step;
    }
    return 0;
}

int64_t oracle_get_surface_rot(const osim* s, double* sums) {
    if (!s->rsurf) return 0;
    if (sums) memcpy(sums, s->rsurf, sizeof(double) * (size_t)s->nb);
    int64_t end = s->surf_to < 0 ? (int64_t)s->step : s->surf_to;
    int64_t from = s->surf_from > s->n_ss ? s->surf_from : s->n_ss;
    return end > from ? end - from : 0;
}

int64_t oracle_get_surface(const osim* s, double* sums) {
    if (!s->surf) return 0;
    if (sums) memcpy(sums, s->surf, sizeof(double) * 5 * (size_t)s->nb);
    int64_t end = s->surf_to < 0 ? (int64_t)s->step : s->surf_to;
    int64_t from = s->surf_from > s->n_ss ? s->surf_from : s->n_ss;
    return end > from ? end - from : 0;
}
uint32_t oracle_next_pid(const osim* s) { return s->next_pid; }

void oracle_get_pair_counts(const osim* s, int* ncand, int* nacc) {
    memcpy(ncand, s->ncand, sizeof(int) * (size_t)s->nt);
    memcpy(nacc, s->nacc, sizeof(int) * (size_t)s->nt);
}

void oracle_get_counters(const osim* s, int64_t out[5]) {
    out[0] = s->hops; out[1] = s->walls; out[2] = s->injected; out[3] = s->removed; out[4] = s->lost;
}

void oracle_get_sums(const osim* s, int which, double* out) {
    const double* src = which == 0 ? s->acc : which == 1 ? s->ewma : s->inst;
    memcpy(out, src, sizeof(double) * NMOM * (size_t)s->nt);
}

int64_t oracle_num_steady(const osim* s) { return s->n_steady; }

void oracle_get_ewma_counts(const osim* s, int* out) { memcpy(out, s->ewma_m, sizeof(int) * (size_t)s->nt); }

void oracle_set_sums(osim* s, int which, const double* in) {
    double* dst = which == 0 ? s->acc : s->ewma;
    memcpy(dst, in, sizeof(double) * NMOM * (size_t)s->nt);
}

void oracle_set_local_acc(osim* s, const unsigned char* flags) {
    memcpy(s->local_acc, flags, (size_t)s->nt);
}

/* Fields from a sum set over ns samples (eq. dsmc_temperatures, with the
 * cell mean taken over all sampled particles). */
/* Fields of one set of moment sums S (eq. dsmc_temperatures): number
 * density, density, velocity, temperature, stress, heat flux; NaN without
 * samples. */
static void fields_of(const double* S, double ns, double FN, double m, double vol, double* o) {
    if (!(S[0] > 0) || !(ns > 0)) {
        for (int k = 0; k < 15; ++k) o[k] = NAN;
        return;
    }
    double nbar = S[0] / ns;
    double n = (FN * nbar) / vol;
    double rho = m * n;
    double u[3] = {S[1] / S[0], S[2] / S[0], S[3] / S[0]};
    /* C_ij = S2_ij/S0 - u_i u_j, order xx, yy, zz, xy, xz, yz */
    const int ii[6] = {0, 1, 2, 0, 0, 1}, jj[6] = {0, 1, 2, 1, 2, 2};
    double C[6];
    for (int k = 0; k < 6; ++k) C[k] = S[4 + k] / S[0] - u[ii[k]] * u[jj[k]];
    double Ckk = C[0] + C[1] + C[2];
    double T = (m * Ckk) / (3.0 * KB);
    o[0] = n; o[1] = rho; o[2] = u[0]; o[3] = u[1]; o[4] = u[2]; o[5] = T;
    for (int k = 0; k < 6; ++k) o[6 + k] = rho * (C[k] - (k < 3 ? Ckk / 3.0 : 0.0));
    /* full second-moment matrix entries S2_ij */
    double M2[3][3] = {{S[4], S[7], S[8]}, {S[7], S[5], S[9]}, {S[8], S[9], S[6]}};
    double S2kk = S[4] + S[5] + S[6];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < 3; ++i) {
        double uS = u[0] * M2[i][0] + u[1] * M2[i][1] + u[2] * M2[i][2];
        double br = ((S[10 + i] - 2.0 * uS) - u[i] * S2kk) + 2.0 * S[0] * u[i] * uu;
        o[12 + i] = (rho / 2.0) * br / S[0];
    }
}

void oracle_fields(const osim* s, int which, double* out) {
    const double* src = which == 0 ? s->acc : which == 1 ? s->ewma : s->inst;
    double ns = which == 0 ? (double)s->n_steady : 1.0;
    for (int c = 0; c < s->nt; ++c) fields_of(src + NMOM * (size_t)c, ns, s->FN, s->m, s->vol[c], out + 15 * (size_t)c);
}

/* The same fields of n given sets of sums [n][13] over the given volumes
 * (cells made of several tetrahedra). */
void oracle_fields_of_sums(const osim* s, const double* sums, const double* vol, int n, double ns, double* out) {
    for (int c = 0; c < n; ++c) fields_of(sums + NMOM * (size_t)c, ns, s->FN, s->m, vol[c], out + 15 * (size_t)c);
}

void oracle_get_volumes(const osim* s, double* vol) { memcpy(vol, s->vol, sizeof(double) * (size_t)s->nt); }
void oracle_get_neighbours(const osim* s, int* nbr) { memcpy(nbr, s->tf_nbr, sizeof(int) * 4 * (size_t)s->nt); }
void oracle_get_tets(const osim* s, int* tv) { memcpy(tv, s->tv, sizeof(int) * 4 * (size_t)s->nt); }
int oracle_num_faces(const osim* s) { return s->nf; }

void o_draw(const osim* s, uint32_t subject, uint32_t step, uint32_t purpose, uint64_t block, uint32_t out[4]) {
    draw(s, subject, step, purpose, block, out);
}
double o_u01(uint32_t a, uint32_t b) { return u01(a, b); }
uint32_t o_pick(uint32_t r, uint32_t n) { return pick(r, n); }
double o_to_store(const osim* s, double x) { return to_store(s, x); }
void o_sort(osim* s) { stage_sort(s); }
void o_reserve(osim* s, int64_t need) { reserve(s, need); }
void o_set_err(const char* m) { set_err(m); }
