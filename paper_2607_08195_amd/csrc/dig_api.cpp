// C ABI of the DIG coupling step (section 3, Algorithm 1): geometry of the
// macroscopic finite-volume solver, the coupling cycle and its parts.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <string>
#include <utility>
#include <vector>

#include "../../include/dig.h"
#include "context.h"
#include "dig.h"
#include "mlp.h"

namespace dsmcx {

struct DigState {
    DigGeom g{};
    DigWork w{};
    int nblk = 0;
    AaWork aa{};  // Anderson history, allocated at the first accelerated solve
    NkWork nk{};  // Krylov basis and work of the Newton-Krylov solve, allocated at its first use
    bool closed = true;  // no inflow or outflow boundary: the solve's mass is rescaled to the particles'
};

void dig_release(dsmc_ctx c) {
    // device arrays belong to the context's allocation list
    delete c->dig;
    c->dig = nullptr;
}

namespace {

constexpr int kPollEvery = 16;  // iterations between convergence polls

struct HostGeom {
    std::vector<double> cen, fcen, fnu, farea, fdx, lsq;
    std::vector<int32_t> flink;
};

// Centroids, face centroids, outward unit normals and areas, the link of
// every tet face (neighbour across an interior or periodic face, boundary
// group otherwise) with the connector dx, and the inverse of the weighted
// least-squares matrix sum_f w dx dx^T (w = 1/|dx|^2) over the faces that
// carry a gradient value (interior, periodic, diffuse wall).
void build_geometry(const HostMesh& m, const std::vector<dsmc_boundary_desc>& bcs, HostGeom& G) {
    const int nt = m.nt;
    G.cen.assign(3 * (size_t)nt, 0.0);
    G.fcen.assign(12 * (size_t)nt, 0.0);
    G.fnu.assign(12 * (size_t)nt, 0.0);
    G.farea.assign(4 * (size_t)nt, 0.0);
    G.fdx.assign(12 * (size_t)nt, 0.0);
    G.lsq.assign(9 * (size_t)nt, 0.0);
    G.flink.assign(4 * (size_t)nt, 0);
    const double* X = m.xyz.data();
    for (int c = 0; c < nt; ++c) {
        const int32_t* q = &m.tv[4 * (size_t)c];
        for (int i = 0; i < 3; ++i) {
            const double a = X[3 * (size_t)q[0] + i], b = X[3 * (size_t)q[1] + i];
            const double d = X[3 * (size_t)q[2] + i], e = X[3 * (size_t)q[3] + i];
            G.cen[3 * (size_t)c + i] = (((a + b) + d) + e) * 0.25;
        }
        for (int f = 0; f < 4; ++f) {
            int v[3], j = 0;
            for (int k = 0; k < 4; ++k)
                if (k != f) v[j++] = q[k];
            for (int i = 0; i < 3; ++i)
                G.fcen[12 * (size_t)c + 3 * f + i] =
                    ((X[3 * (size_t)v[0] + i] + X[3 * (size_t)v[1] + i]) + X[3 * (size_t)v[2] + i]) / 3.0;
            const double* pl = &m.plane[16 * (size_t)c + 4 * f];
            const double nn = std::sqrt(pl[0] * pl[0] + pl[1] * pl[1] + pl[2] * pl[2]);
            for (int i = 0; i < 3; ++i) G.fnu[12 * (size_t)c + 3 * f + i] = pl[i] / nn;
            G.farea[4 * (size_t)c + f] = 0.5 * nn;
        }
    }
    for (int c = 0; c < nt; ++c) {
        const double* xc = &G.cen[3 * (size_t)c];
        for (int f = 0; f < 4; ++f) {
            const int code = m.nbr[4 * (size_t)c + f];
            double* dx = &G.fdx[12 * (size_t)c + 3 * f];
            const double* xf = &G.fcen[12 * (size_t)c + 3 * f];
            int32_t link;
            if (code >= 0) {
                const int nb = code >> 2;
                for (int i = 0; i < 3; ++i) dx[i] = G.cen[3 * (size_t)nb + i] - xc[i];
                link = kLinkInterior | (nb << 3);
            } else {
                const int bf = -1 - code;
                const int grp = m.bf_group[bf];
                const dsmc_boundary_desc& b = bcs[grp];
                if (b.kind == DSMC_BC_PERIODIC) {
                    const int pt = m.bf_tet[m.bf_partner[bf]];
                    for (int i = 0; i < 3; ++i) dx[i] = (G.cen[3 * (size_t)pt + i] - b.shift[i]) - xc[i];
                    link = kLinkPeriodic | (pt << 3);
                } else {
                    for (int i = 0; i < 3; ++i) dx[i] = xf[i] - xc[i];
                    const int kind = b.kind == DSMC_BC_DIFFUSE    ? kLinkWall
                                     : b.kind == DSMC_BC_SPECULAR ? kLinkSpecular
                                     : b.kind == DSMC_BC_INFLOW   ? kLinkInflow
                                                                  : kLinkOutflow;
                    link = kind | (grp << 3);
                }
            }
            G.flink[4 * (size_t)c + f] = link;
        }
        double A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        for (int f = 0; f < 4; ++f) {
            const int kind = G.flink[4 * (size_t)c + f] & 7;
            if (kind != kLinkInterior && kind != kLinkPeriodic && kind != kLinkWall) continue;
            const double* dx = &G.fdx[12 * (size_t)c + 3 * f];
            const double w = 1.0 / (dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) A[i][j] += w * dx[i] * dx[j];
        }
        double* L = &G.lsq[9 * (size_t)c];
        const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                           A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                           A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
        const double tr = (A[0][0] + A[1][1] + A[2][2]) / 3.0;
        if (!(std::fabs(det) > 1e-10 * tr * tr * tr)) continue;  // rank-deficient stencil: zero gradient
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
}

// Viscosity of the VHS/VSS gas at T_ref (Chapman-Enskog first
// approximation); VSS scattering multiplies the VHS value by
// (alpha+1)(alpha+2)/(6 alpha), exactly 1 at alpha = 1 (Bird 1994).
double mu_ref_of(dsmc_ctx c) {
    const double w = c->omega, a = c->alpha;
    return 15.0 * std::sqrt(M_PI * c->mass * kBoltzmann * c->Tref) /
           (2.0 * M_PI * c->dref * c->dref * (5.0 - 2.0 * w) * (7.0 - 2.0 * w)) * (((a + 1.0) * (a + 2.0)) / (6.0 * a));
}

template <class T>
dsmc_status upload(dsmc_ctx c, T* dst, const std::vector<T>& src) {
    HIP_TRY(c, hipMemcpyAsync(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, c->stream));
    return DSMC_OK;
}

int dig_nv(dsmc_ctx c) { return c->dr ? kDigNVR : kDigNV; }
int dig_nh(dsmc_ctx c) { return c->dr ? 12 : 9; }
int dig_ns(dsmc_ctx c) { return c->dr ? 18 : 14; }

dsmc_status ensure(dsmc_ctx c) {
    if (c->dig) return DSMC_OK;
    HostGeom G;
    build_geometry(c->hm, c->bcs, G);
    const int nt = c->nt;
    const int ng = (int)c->bcs.size();
    DigState* d = new DigState();
    d->nblk = (nt + kDigThreads - 1) / kDigThreads;
    double *cen, *fcen, *fnu, *farea, *fdx, *lsq;
    int32_t* flink;
    DigGroup* groups;
    DigWork& w = d->w;
    // widths per cell: primitives, HoT, sampled values (rotating gas: 6, 12, 18)
    const size_t nv = dig_nv(c), nh = dig_nh(c), ns = dig_ns(c);
    bool ok = alloc_n(c, cen, G.cen.size()) && alloc_n(c, fcen, G.fcen.size()) && alloc_n(c, fnu, G.fnu.size()) &&
              alloc_n(c, farea, G.farea.size()) && alloc_n(c, fdx, G.fdx.size()) && alloc_n(c, lsq, G.lsq.size()) &&
              alloc_n(c, flink, G.flink.size()) && alloc_n(c, groups, ng + 1);
    ok = ok && alloc_n(c, w.samp, ns * nt) && alloc_n(c, w.ok, nt) && alloc_n(c, w.prim, nv * nt) &&
         alloc_n(c, w.half, nv * nt) && alloc_n(c, w.hot, nh * nt) && alloc_n(c, w.hotf, 4 * nh * nt) &&
         alloc_n(c, w.grad, 3 * nv * nt) && alloc_n(c, w.kn, nt) && alloc_n(c, w.avail, nt) &&
         alloc_n(c, w.navail, nt) && alloc_n(c, w.nprim, nv * nt) && alloc_n(c, w.nhot, nh * nt) &&
         alloc_n(c, w.state, nt) && alloc_n(c, w.mprev, nv * nt) && alloc_n(c, w.Rs, nv * nt) &&
         alloc_n(c, w.dt, nt) && alloc_n(c, w.U0, nv * nt) && alloc_n(c, w.stage, nv * nt) &&
         alloc_n(c, w.partial, 8 * (size_t)d->nblk) && alloc_n(c, w.ctl, 1) && alloc_n(c, w.fb_cnt, nt) &&
         alloc_n(c, w.fb_off, nt + 1) && alloc_n(c, w.fb_tgt, nt) && alloc_n(c, w.cx, 13 * (size_t)nt) &&
         alloc_n(c, w.ct, 9 * (size_t)nt) && alloc_n(c, w.cs, 9 * (size_t)nt) && alloc_n(c, w.cy, 9 * (size_t)nt) &&
         alloc_n(c, w.cvalid, nt);
    if (!ok) {
        delete d;
        return fail(c, DSMC_E_OOM, "device allocation of the coupling state failed");
    }
    std::vector<DigGroup> hg(ng + 1);
    for (int g = 0; g < ng; ++g) {
        hg[g].T = c->bcs[g].T;
        for (int i = 0; i < 3; ++i) hg[g].u[i] = c->bcs[g].u[i];
        hg[g].rho = c->mass * c->bcs[g].n;
    }
    // Batch: per-case reference state, particle weight, key and cell ranges
    // (the cases are contiguous in both numberings).
    const int ncase = c->n_cases;
    std::vector<CaseDev> cd(std::max(1, ncase));
    std::vector<DigCase> dc(ncase);
    std::vector<int32_t> case_of(nt, 0);
    if (ncase) {
        if (hipStreamSynchronize(c->stream) != hipSuccess ||
            hipMemcpy(cd.data(), c->d_cases, sizeof(CaseDev) * ncase, hipMemcpyDeviceToHost) != hipSuccess) {
            delete d;
            return fail(c, DSMC_E_DEVICE, "reading the case table failed");
        }
        const double R = kBoltzmann / c->mass;
        for (int k = 0; k < ncase; ++k) {
            DigCase& q = dc[k];
            const double T0 = cd[k].T0;
            q.FN = cd[k].FN;
            q.p0 = cd[k].n0 * kBoltzmann * T0;
            q.mu0 = mu_ref_of(c) * std::pow(T0 / c->Tref, c->omega);
            q.kfac = std::sqrt(M_PI * R * T0 / 2.0);
            q.T0 = T0;
            q.rho0 = c->mass * cd[k].n0;
            q.mass_scale = 1.0;
            q.k0 = cd[k].k0;
            q.k1 = cd[k].k1;
            q.cell0 = c->case_cell0[k];
            q.cell_end = k + 1 < ncase ? c->case_cell0[k + 1] : nt;
            q.first = nt;
            q.end = 0;
            q.enabled = 1;
            q.closed = 1;
            q.next_pid = 0;
        }
        for (int t = 0; t < nt; ++t) {
            const int o = c->hm.orig[t];
            const int k = (int)(std::upper_bound(c->case_cell0.begin(), c->case_cell0.end(), o) - c->case_cell0.begin()) - 1;
            case_of[t] = k;
            dc[k].first = std::min(dc[k].first, t);
            dc[k].end = std::max(dc[k].end, t + 1);
        }
        // a case with an inflow or outflow face is open
        for (int b = 0; b < c->nb; ++b) {
            const int kind = c->bcs[c->hm.bf_group[b]].kind;
            if (kind == DSMC_BC_INFLOW || kind == DSMC_BC_OUTFLOW) dc[case_of[c->hm.bf_tet[b]]].closed = 0;
        }
        for (const DigCase& q : dc)
            if (q.end - q.first != q.cell_end - q.cell0) {
                delete d;
                return fail(c, DSMC_E_INVALID, "batch cases are not contiguous in the internal cell order");
            }
        if (!alloc_n(c, d->g.cases, ncase)) {
            delete d;
            return fail(c, DSMC_E_OOM, "device allocation of the coupling state failed");
        }
    }
    std::vector<double> mprev(nv * nt);
    for (int t = 0; t < nt; ++t) {
        double* p = &mprev[nv * t];
        const CaseDev& q = cd[case_of[t]];
        p[0] = c->mass * (ncase ? q.n0 : c->n0);
        p[1] = ncase ? q.u0[0] : c->u0[0];
        p[2] = ncase ? q.u0[1] : c->u0[1];
        p[3] = ncase ? q.u0[2] : c->u0[2];
        p[4] = ncase ? q.T0 : c->T0;
        if (nv == 6) p[5] = p[4];
    }
    dsmc_status st = DSMC_OK;
    if (ncase) st = upload(c, d->g.cases, dc);
    if (st == DSMC_OK) st = upload(c, cen, G.cen);
    if (st == DSMC_OK) st = upload(c, fcen, G.fcen);
    if (st == DSMC_OK) st = upload(c, fnu, G.fnu);
    if (st == DSMC_OK) st = upload(c, farea, G.farea);
    if (st == DSMC_OK) st = upload(c, fdx, G.fdx);
    if (st == DSMC_OK) st = upload(c, lsq, G.lsq);
    if (st == DSMC_OK) st = upload(c, flink, G.flink);
    if (st == DSMC_OK) st = upload(c, groups, hg);
    if (st == DSMC_OK) st = upload(c, w.mprev, mprev);
    if (st == DSMC_OK) {
        launch_fill_i32(c->stream, w.state, 0, nt);
        launch_dig_ctl_reset(c->stream, w.ctl);
        if (hipStreamSynchronize(c->stream) != hipSuccess) st = fail(c, DSMC_E_DEVICE, "coupling state upload failed");
    }
    if (st != DSMC_OK) {
        delete d;
        return st;
    }
    DigGeom& g = d->g;
    g.nt = nt;
    g.cen = cen; g.fcen = fcen; g.fnu = fnu; g.farea = farea; g.fdx = fdx; g.flink = flink; g.lsq = lsq;
    g.vol = c->d_vol;
    g.groups = groups;
    g.mass = c->mass;
    g.R = kBoltzmann / c->mass;
    g.mu_ref = mu_ref_of(c);
    g.omega = c->omega;
    g.T_ref = c->Tref;
    g.FN = c->FN;
    g.cell_case = ncase ? c->d_cell_case : nullptr;
    g.n_cases = ncase;
    g.dr = c->dr;
    g.zr = c->zr;
    for (int k = 0; k < 4; ++k) g.a_heat[k] = c->a_heat[k];
    g.ert = g.R * c->T0;
    for (const dsmc_boundary_desc& b : c->bcs) d->closed = d->closed && b.kind != DSMC_BC_INFLOW && b.kind != DSMC_BC_OUTFLOW;
    // a batch rescales its closed cases (per case, in the kernel)
    for (const DigCase& q : dc) d->closed = d->closed || q.closed;
    if (ncase) {
        // next particle id of each case: its largest id + 1
        Scalars sc;
        if ((st = sync_scalars(c, &sc)) != DSMC_OK) {
            delete d;
            return st;
        }
        launch_dig_case_pid_init(c->stream, g, c->A.cell, c->A.pid, c->d_sc, sc.np);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) {
            delete d;
            return fail(c, DSMC_E_DEVICE, "case id scan failed");
        }
    }
    c->dig = d;
    return DSMC_OK;
}

DigCtl read_ctl(dsmc_ctx c, dsmc_status* st) {
    DigCtl h{};
    *st = DSMC_OK;
    if (hipStreamSynchronize(c->stream) != hipSuccess ||
        hipMemcpy(&h, c->dig->w.ctl, sizeof h, hipMemcpyDeviceToHost) != hipSuccess) {
        c->broken = true;
        *st = fail(c, DSMC_E_DEVICE, "reading the coupling control block failed");
    }
    return h;
}

dsmc_status check_params(dsmc_ctx c, const dig_params* p) {
    if (!p) return fail(c, DSMC_E_INVALID, "params is NULL");
    if (p->passes < 0 || p->n_m < 0 || !(p->cfl > 0) || !(p->L0 > 0) || !(p->eps_m >= 0) || p->accel < 0)
        return fail(c, DSMC_E_INVALID, "bad coupling parameters");
    if (p->solver != 0 && p->solver != 1) return fail(c, DSMC_E_INVALID, "solver must be 0 or 1");
    if (p->krylov < 0 || p->krylov > kNkMaxKrylov) return fail(c, DSMC_E_INVALID, "krylov must be in [0, 100]");
    if (p->solver == 1 && (p->accel > 0 || p->global_dt))
        return fail(c, DSMC_E_INVALID, "the Newton-Krylov solve takes neither accel nor global_dt");
    if (p->solver == 1 && c->dig && c->dig->g.n_cases > 0)
        return fail(c, DSMC_E_INVALID, "the Newton-Krylov solve is not available for a batch");
    return DSMC_OK;
}

// Pseudo-time marching from w.prim with w.hot frozen; fills the solve part
// of the report.
constexpr int kAaDepthMax = 64;

// History of depth m for the accelerated solve (kept for later solves).
dsmc_status ensure_aa(dsmc_ctx c, int m) {
    DigState* d = c->dig;
    if (d->aa.m >= m) return DSMC_OK;
    const size_t n = 5 * (size_t)c->nt;
    AaWork& a = d->aa;
    for (double* q : {a.x, a.fprev, a.gprev, a.dF, a.dG, a.part, a.red, a.gam}) dev_free(c, q);
    a = AaWork{};
    const bool ok = alloc_n(c, a.x, n) && alloc_n(c, a.fprev, n) && alloc_n(c, a.gprev, n) &&
                    alloc_n(c, a.dF, n * m) && alloc_n(c, a.dG, n * m) &&
                    alloc_n(c, a.part, (size_t)d->nblk * (2 * m + 1)) && alloc_n(c, a.red, 2 * (size_t)m + 2) &&
                    alloc_n(c, a.gam, m);
    if (!ok) return fail(c, DSMC_E_OOM, "device allocation of the acceleration history failed");
    a.m = m;
    return DSMC_OK;
}

// Solves the m x m system (H + lambda I) gam = b by Cholesky (lambda a
// small multiple of the largest diagonal entry); false if H is not usable.
bool solve_small(int n, int ld, const std::vector<double>& H, const std::vector<double>& b, std::vector<double>& x) {
    double dmax = 0.0;
    for (int i = 0; i < n; ++i) dmax = std::max(dmax, H[i * ld + i]);
    if (!(dmax > 0) || !std::isfinite(dmax)) return false;
    std::vector<double> L(n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) {
            double v = H[i * ld + j] + (i == j ? 1e-10 * dmax : 0.0);
            for (int k = 0; k < j; ++k) v -= L[i * n + k] * L[j * n + k];
            if (i == j) {
                if (!(v > 0)) return false;
                L[i * n + i] = std::sqrt(v);
            } else {
                L[i * n + j] = v / L[j * n + j];
            }
        }
    std::vector<double> y(n);
    for (int i = 0; i < n; ++i) {
        double v = b[i];
        for (int k = 0; k < i; ++k) v -= L[i * n + k] * y[k];
        y[i] = v / L[i * n + i];
    }
    x.assign(n, 0.0);
    for (int i = n - 1; i >= 0; --i) {
        double v = y[i];
        for (int k = i + 1; k < n; ++k) v -= L[k * n + i] * x[k];
        x[i] = v / L[i * n + i];
    }
    for (double v : x)
        if (!std::isfinite(v)) return false;
    return true;
}

// Pseudo-time iteration accelerated by Anderson mixing of depth m: one
// synchronisation per iteration, which brings back the inner products, the
// control block and the fallback count of the previous mixing step.
dsmc_status run_solve_aa(dsmc_ctx c, const dig_params* p, dig_report* r, int m) {
    DigState* d = c->dig;
    hipStream_t s = c->stream;
    dsmc_status st = ensure_aa(c, m);
    if (st != DSMC_OK) return st;
    AaWork& a = d->aa;
    const double R = kBoltzmann / c->mass;
    const double rho = c->mass * c->n0, cs2 = R * c->T0, T2 = c->T0 * c->T0;
    const double w5[5] = {1.0 / (rho * rho), 1.0 / cs2, 1.0 / cs2, 1.0 / cs2, 1.0 / T2};
    const size_t n = 5 * (size_t)c->nt;
    std::vector<double> H((size_t)m * m, 0.0), red(2 * (size_t)m + 2, 0.0), b(m), gam(m, 0.0), bs;
    int cnt = 0, made = 0;  // stored differences, differences made since the last restart
    bool fresh = true;      // the next application of G starts a new history
    bool mixed = false;     // the previous iteration ended with a mixing step
    DigCtl h{};
    launch_dig_ctl_reset(s, d->w.ctl);
    for (int it = 0; it < p->n_m; ++it) {
        const int par = it & 1;
        HIP_TRY(c, hipMemcpyAsync(a.x, d->w.prim, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        launch_dig_iteration(s, d->g, d->w, p->cfl, p->eps_m, p->global_dt ? 1 : 0, it);
        const int slot = fresh ? 0 : made % m;
        launch_aa_diff(s, d->g, a, d->w.prim, slot, fresh ? 1 : 0, par);
        const int ncnt = fresh ? 0 : std::min(cnt + 1, m);
        if (ncnt > 0) launch_aa_dots(s, d->g, a, slot, ncnt, w5);
        HIP_TRY(c, hipMemcpyAsync(red.data(), a.red, sizeof(double) * (2 * m + 2), hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipMemcpyAsync(&h, d->w.ctl, sizeof h, hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipStreamSynchronize(s));
        HIP_TRY(c, hipGetLastError());
        if (h.conv || h.failed) break;
        if (fresh) {
            fresh = false;
            cnt = made = 0;
            mixed = false;
            continue;  // G(x_0) is the next state
        }
        ++made;
        cnt = ncnt;
        if (mixed && red[2 * m + (par ^ 1)] > 0) {
            // cells of the previous mixing step fell back to G(x): restart
            fresh = true;
            mixed = false;
            continue;
        }
        for (int i = 0; i < cnt; ++i) {
            H[(size_t)slot * m + i] = red[i];
            H[(size_t)i * m + slot] = red[i];
            b[i] = red[m + i];
        }
        bs.assign(b.begin(), b.begin() + cnt);
        if (!solve_small(cnt, m, H, bs, gam)) {
            fresh = true;  // the history is degenerate: plain step, new history
            mixed = false;
            continue;
        }
        HIP_TRY(c, hipMemcpyAsync(a.gam, gam.data(), sizeof(double) * cnt, hipMemcpyHostToDevice, s));
        launch_aa_update(s, d->g, a, cnt, d->w.prim, par);
        mixed = true;
    }
    HIP_TRY(c, hipGetLastError());
    h = read_ctl(c, &st);
    if (st != DSMC_OK) return st;
    r->iters = h.iters;
    r->residual = h.res0 > 0 ? h.res / h.res0 : 0.0;
    r->converged = h.conv;
    r->failed = h.failed;
    return DSMC_OK;
}

constexpr int kNkDefaultKrylov = 40;
constexpr double kNkEta = 0.05;      // GMRES stops at this fraction of its initial residual
constexpr double kNkCflMax = 1e8;    // largest pseudo-time CFL number of the continuation
constexpr double kNkFd = 1e-7;       // relative size of the finite-difference step
constexpr int kNkHalvings = 10;      // halvings of an update that leaves a cell non-physical
constexpr double kNkLinPoor = 0.5;   // a linear solve that leaves more than this halves the CFL number

dsmc_status ensure_nk(dsmc_ctx c, int m) {
    DigState* d = c->dig;
    if (d->nk.m >= m) return DSMC_OK;
    NkWork& k = d->nk;
    for (double* q : {k.V, k.w, k.U, k.Ut, k.R0, k.Rp, k.part, k.red, k.y}) dev_free(c, q);
    dev_free(c, k.flag);
    k = NkWork{};
    const size_t n = (size_t)dig_nv(c) * c->nt;
    const size_t nblk = ((size_t)c->nt + kDigThreads - 1) / kDigThreads;
    const bool ok = alloc_n(c, k.V, n * (m + 1)) && alloc_n(c, k.w, n) && alloc_n(c, k.U, n) && alloc_n(c, k.Ut, n) &&
                    alloc_n(c, k.R0, n) && alloc_n(c, k.Rp, n) && alloc_n(c, k.part, nblk * (m + 1)) &&
                    alloc_n(c, k.red, (size_t)kNkRedSize(m)) && alloc_n(c, k.y, (size_t)m) && alloc_n(c, k.flag, 1);
    if (!ok) return fail(c, DSMC_E_OOM, "device allocation of the Krylov basis failed");
    k.m = m;
    return DSMC_OK;
}

// Newton-Krylov solve from w.prim with w.hotf frozen (the steady equations
// of the marching): pseudo-transient continuation with the CFL number
// grown by the ratio of successive residual norms from p->cfl (within
// [p->cfl, kNkCflMax]) and at least halved after a step whose linear solve
// left more than kNkLinPoor of its initial residual; each Newton step runs one cycle of at most m GMRES
// steps from zero on the scaled, right-preconditioned system
// (S/cfl + J) dU = -R, stopping at kNkEta of its initial residual; an
// update that leaves a cell non-physical is halved up to kNkHalvings
// times, then the solve fails.  The stopping test is the marching's (the
// density residual norm, with rotation the rotational-energy residual too,
// against eps_m times its first value), taken at the start of each Newton
// step; iters counts the updates.  Host round trips: one per Newton step,
// one per GMRES step and one per trial update.
dsmc_status run_solve_nk(dsmc_ctx c, const dig_params* p, dig_report* r) {
    DigState* d = c->dig;
    hipStream_t s = c->stream;
    const int m = p->krylov > 0 ? p->krylov : kNkDefaultKrylov;
    dsmc_status st = ensure_nk(c, m);
    if (st != DSMC_OK) return st;
    NkWork& nk = d->nk;
    const int nv = dig_nv(c);
    const double n = (double)nv * c->nt;
    const double R = kBoltzmann / c->mass;
    const double rho0 = c->mass * c->n0, a2 = R * c->T0, a0 = std::sqrt(a2);
    NkScale sc{};
    sc.s[0] = rho0;
    sc.s[1] = sc.s[2] = sc.s[3] = rho0 * a0;
    sc.s[4] = sc.s[5] = rho0 * a2;
    std::vector<double> red((size_t)kNkRedSize(m)), H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), y(m);
    launch_dig_ctl_reset(s, d->w.ctl);
    double cfl = p->cfl, bprev = 0.0, lin = 0.0;
    bool failed = false;
    DigCtl h{};
    int k = 0, nkry = 0;
    // DSMC_NK_TRACE=1: one line per Newton step on stderr
    const char* tr = std::getenv("DSMC_NK_TRACE");
    const bool trace = tr && tr[0] == '1';
    auto fetch = [&](int32_t* flag) -> dsmc_status {
        HIP_TRY(c, hipMemcpyAsync(red.data(), nk.red, sizeof(double) * red.size(), hipMemcpyDeviceToHost, s));
        if (flag) HIP_TRY(c, hipMemcpyAsync(flag, nk.flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipStreamSynchronize(s));
        HIP_TRY(c, hipGetLastError());
        return DSMC_OK;
    };
    for (k = 0; k < p->n_m; ++k) {
        launch_nk_begin(s, d->g, d->w, nk, sc, k, p->eps_m);
        HIP_TRY(c, hipMemcpyAsync(&h, d->w.ctl, sizeof h, hipMemcpyDeviceToHost, s));
        if ((st = fetch(nullptr)) != DSMC_OK) return st;
        if (h.conv) break;
        const double beta = std::sqrt(red[kNkBeta2(m)]);
        if (k > 0) {
            double f = bprev / beta;
            if (lin > kNkLinPoor && f > 0.5) f = 0.5;
            cfl = std::min(kNkCflMax, std::max(p->cfl, cfl * f));
        }
        bprev = beta;
        HIP_TRY(c, hipMemsetAsync(nk.flag, 0, sizeof(int32_t), s));
        launch_nk_scale(s, d->g, d->w, nk, cfl, kNkFd);
        std::fill(H.begin(), H.end(), 0.0);
        gv[0] = beta;
        int jn = 0;
        for (int j = 0; j < m; ++j) {
            launch_nk_arnoldi(s, d->g, d->w, nk, sc, j, cfl, kNkFd);
            int32_t flag = 0;
            if ((st = fetch(&flag)) != DSMC_OK) return st;
            if (flag) {
                failed = true;
                break;
            }
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = (0.0 + red[kNkH1(m) + i]) + red[kNkH2(m) + i];
            const double hn = std::sqrt(red[kNkHn2(m)]);
            H[(size_t)(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                const double a = H[(size_t)i * m + j], b = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * b;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
            }
            const double a = H[(size_t)j * m + j], b = H[(size_t)(j + 1) * m + j];
            const double rr = std::sqrt(a * a + b * b);
            cs[j] = rr > 0 ? a / rr : 1.0;
            sn[j] = rr > 0 ? b / rr : 0.0;
            H[(size_t)j * m + j] = rr;
            H[(size_t)(j + 1) * m + j] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            jn = j + 1;
            ++nkry;
            if (std::fabs(gv[j + 1]) <= kNkEta * beta || !(hn > 0)) break;
        }
        if (trace)
            std::fprintf(stderr, "nk step %d: density residual %.3e of the first, |b| %.4e, cfl %.3e, gmres %d, "
                         "linear residual %.3e\n", k, h.res0 > 0 ? h.res / h.res0 : 0.0, beta, cfl, jn,
                         std::fabs(gv[jn]) / beta);
        if (failed) break;
        lin = std::fabs(gv[jn]) / beta;
        for (int i = jn - 1; i >= 0; --i) {
            double t = gv[i];
            for (int l = i + 1; l < jn; ++l) t -= H[(size_t)i * m + l] * y[l];
            y[i] = t / H[(size_t)i * m + i];
        }
        HIP_TRY(c, hipMemcpyAsync(nk.y, y.data(), sizeof(double) * jn, hipMemcpyHostToDevice, s));
        double alpha = 1.0;
        bool accepted = false;
        for (int tries = 0; tries <= kNkHalvings && !accepted; ++tries) {
            HIP_TRY(c, hipMemsetAsync(nk.flag, 0, sizeof(int32_t), s));
            launch_nk_try(s, d->g, d->w, nk, sc, jn, alpha, cfl);
            int32_t flag = 0;
            HIP_TRY(c, hipMemcpyAsync(&flag, nk.flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            HIP_TRY(c, hipStreamSynchronize(s));
            if (!flag)
                accepted = true;
            else
                alpha = 0.5 * alpha;
        }
        if (!accepted) {
            failed = true;
            break;
        }
        launch_nk_commit(s, d->g, d->w, nk);
    }
    HIP_TRY(c, hipGetLastError());
    h = read_ctl(c, &st);
    if (st != DSMC_OK) return st;
    r->iters = k;
    r->residual = h.res0 > 0 ? h.res / h.res0 : 0.0;
    r->converged = h.conv;
    r->failed = failed ? 1 : 0;
    r->krylov_steps = nkry;
    return DSMC_OK;
}

dsmc_status run_solve(dsmc_ctx c, const dig_params* p, dig_report* r) {
    if (p->solver == 1) return run_solve_nk(c, p, r);
    if (p->accel > 0) return run_solve_aa(c, p, r, std::min(p->accel, kAaDepthMax));
    DigState* d = c->dig;
    launch_dig_ctl_reset(c->stream, d->w.ctl);
    dsmc_status st = DSMC_OK;
    DigCtl h{};
    for (int it = 0; it < p->n_m; ++it) {
        launch_dig_iteration(c->stream, d->g, d->w, p->cfl, p->eps_m, p->global_dt ? 1 : 0, it);
        if ((it + 1) % kPollEvery == 0 && it + 1 < p->n_m) {
            HIP_TRY(c, hipGetLastError());
            h = read_ctl(c, &st);
            if (st != DSMC_OK) return st;
            if (h.conv || h.failed) break;
        }
    }
    HIP_TRY(c, hipGetLastError());
    h = read_ctl(c, &st);
    if (st != DSMC_OK) return st;
    r->iters = h.iters;
    r->residual = h.res0 > 0 ? h.res / h.res0 : 0.0;
    r->converged = h.conv;
    r->failed = h.failed;
    return DSMC_OK;
}

template <class VT>
dsmc_status feedback_t(dsmc_ctx c) {
    DigState* d = c->dig;
    hipStream_t s = c->stream;
    const int nt = c->nt;
    launch_dig_fb_count(s, d->g, d->w, c->d_offsets, c->d_orig, c->d_sc, c->key);
    launch_scan(s, d->w.fb_cnt, nt, d->w.fb_off, c->d_blocksums, c->d_sc, kScanInject);
    HIP_TRY(c, hipGetLastError());
    Scalars sc;
    dsmc_status st = sync_scalars(c, &sc);
    if (st != DSMC_OK) return st;
    const int64_t bound = sc.np + sc.ninj;
    if (bound > c->cap) {
        sc.ninj = 0;
        HIP_TRY(c, hipMemcpy(c->d_sc, &sc, sizeof sc, hipMemcpyHostToDevice));
        return fail(c, DSMC_E_CAPACITY, "feedback clones would exceed the particle store");
    }
    PartDev<VT> a = as_dev<VT>(c->A), b = as_dev<VT>(c->B);
    launch_dig_fb_apply<VT>(s, d->g, d->w, a, c->d_offsets, c->d_tv, c->d_xyz, c->d_orig, c->d_sc, c->key, c->d_perm,
                            c->d_rank, nt, c->cap);
    launch_dig_case_pids(s, d->g, d->w);
    // counting sort of the survivors and the clones
    launch_fill_i32(s, c->d_counts, 0, nt + 1);
    launch_dig_count_all(s, a.cell, c->d_sc, c->d_counts, c->d_rank, bound);
    launch_scan(s, c->d_counts, nt, c->d_offsets, c->d_blocksums, c->d_sc, kScanCells);
    launch_scatter<VT>(s, a, b, c->d_sc, c->d_offsets, c->d_rank, bound, c->cap, c->d_sortperm, c->sort_variant);
    if (c->sort_variant != kSortScatter) launch_gather<VT>(s, a, b, c->d_sc, c->d_sortperm, bound);
    std::swap(c->A, c->B);
    c->np_bound = bound;
    HIP_TRY(c, hipGetLastError());
    return sync_scalars(c, nullptr);
}

dsmc_status run_feedback(dsmc_ctx c) { return c->vel64 ? feedback_t<double>(c) : feedback_t<float>(c); }

// host [nt][k] in caller order <-> device [nt][k] in internal order
template <class T>
dsmc_status to_device(dsmc_ctx c, T* dst, const T* src, int k) {
    const int nt = c->nt;
    std::vector<T> h((size_t)k * nt);
    for (int t = 0; t < nt; ++t)
        for (int j = 0; j < k; ++j) h[(size_t)k * t + j] = src[(size_t)k * c->hm.orig[t] + j];
    HIP_TRY(c, hipMemcpyAsync(dst, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return DSMC_OK;
}

template <class T>
dsmc_status to_host(dsmc_ctx c, T* dst, const T* src, int k) {
    const int nt = c->nt;
    std::vector<T> h((size_t)k * nt);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(h.data(), src, sizeof(T) * h.size(), hipMemcpyDeviceToHost));
    for (int t = 0; t < nt; ++t)
        for (int j = 0; j < k; ++j) dst[(size_t)k * c->hm.orig[t] + j] = h[(size_t)k * t + j];
    return DSMC_OK;
}

dsmc_status usable(dsmc_ctx c) {
    if (!c) return fail(c, DSMC_E_INVALID, "NULL context");
    if (c->broken) return fail(c, DSMC_E_INVALID, "context is in an error state");
    // the feedback and the batch tables read the store sorted by cell
    dsmc_status st = materialize(c);
    if (st != DSMC_OK) return st;
    return ensure(c);
}

}  // namespace
}  // namespace dsmcx

using namespace dsmcx;

extern "C" {

dsmc_status dig_couple(dsmc_ctx c, const dig_params* p, dig_report* rep) {
    dsmc_status st = usable(c);
    if (st != DSMC_OK) return st;
    if ((st = check_params(c, p)) != DSMC_OK) return st;
    if (c->dr && (c->closure || p->accel > 0))
        return fail(c, DSMC_E_INVALID, "the learned closure and the accelerated solve are monatomic");
    DigState* d = c->dig;
    const int nv = dig_nv(c);
    hipStream_t s = c->stream;
    const int nt = c->nt;
    Scalars sc;
    if ((st = sync_scalars(c, &sc)) != DSMC_OK) return st;
    dig_report r{};
    r.np_before = sc.np;
    // reference state of the Knudsen number (eq. cell_kn_stability)
    const double T0 = c->T0;
    const double p0 = c->n0 * kBoltzmann * T0;
    const double R = kBoltzmann / c->mass;
    const double mu0 = d->g.mu_ref * std::pow(T0 / c->Tref, c->omega);
    const double kn_ref = mu0 / (p0 * p->L0) * std::sqrt(M_PI * R * T0 / 2.0);
    const double rho0 = c->mass * c->n0;

    launch_dig_ctl_reset(s, d->w.ctl);
    launch_dig_sampled(s, d->g, c->d_ewma, c->dr ? c->d_rewma : nullptr, c->FN, d->w);
    launch_dig_kn(s, d->g, d->w, kn_ref, T0, rho0, p->L0);
    launch_dig_gradients(s, d->g, d->w.prim, d->w.grad, nullptr);
    launch_dig_hot(s, d->g, d->w);
    launch_dig_closure_prep(s, d->g, d->w);
    if (c->closure) {
        launch_mlp_forward(s, mlp_handle_view(c->closure), d->w.cx, nullptr, nt, d->w.cy);
        launch_dig_closure_gate(s, d->g, d->w, c->gate_tol, c->d_ewma, c->d_ewma_m, c->n_a);
    }
    launch_dig_gate(s, d->g, d->w, p->kn_max, p->passes);
    launch_dig_copy(s, d->w.prim, d->w.half, nv * (int64_t)nt);
    // the solve's face HoT, consistent with M^{k+1/2}
    launch_dig_gradients(s, d->g, d->w.half, d->w.grad, nullptr);
    launch_dig_face_hot(s, d->g, d->w.half, d->w.grad, d->w.hot, d->w.hotf, 1);
    if (p->warm_start) launch_dig_copy(s, d->w.mprev, d->w.prim, nv * (int64_t)nt);
    HIP_TRY(c, hipGetLastError());
    DigCtl h = read_ctl(c, &st);
    if (st != DSMC_OK) return st;
    r.n_rejected = h.n_rejected;
    r.n_reconstructed = h.n_reconstructed;
    r.n_unreached = h.n_unreached;
    r.n_closure = h.n_closure;
    r.n_fallback = h.n_fallback;
    if (r.n_rejected < nt) {
        d->g.skip_idle = c->n_cases ? 1 : 0;
        st = run_solve(c, p, &r);
        d->g.skip_idle = 0;
        if (st != DSMC_OK) return st;
        // Algorithm 1 feeds back the solution of the synthetic equations: a
        // solve that stopped short of eps_m leaves the particles as they are
        // unless the caller asks otherwise
        const bool adjust = !r.failed && (r.converged || p->unconverged);
        if (adjust && d->closed) launch_dig_mass_rescale(s, d->g, d->w, c->d_sc, c->d_offsets);
        if (adjust && p->feedback) {
            if ((st = run_feedback(c)) != DSMC_OK) {
                if (rep) *rep = r;
                return st;
            }
            r.fed_back = 1;
        }
        if (!r.failed) launch_dig_copy(s, d->w.prim, d->w.mprev, nv * (int64_t)nt);
    }
    launch_dig_set_local(s, d->g, d->w.state, c->d_local);
    HIP_TRY(c, hipGetLastError());
    if ((st = sync_scalars(c, &sc)) != DSMC_OK) return st;
    r.np_after = sc.np;
    if (rep) *rep = r;
    return DSMC_OK;
}

dsmc_status dig_get(dsmc_ctx c, int32_t which, void* out) {
    dsmc_status st = usable(c);
    if (st != DSMC_OK) return st;
    if (!out) return fail(c, DSMC_E_INVALID, "out is NULL");
    const DigWork& w = c->dig->w;
    switch (which) {
    case DIG_OUT_SAMPLED: return to_host(c, (double*)out, w.samp, dig_ns(c));
    case DIG_OUT_HALF: return to_host(c, (double*)out, w.half, dig_nv(c));
    case DIG_OUT_NEW: return to_host(c, (double*)out, w.prim, dig_nv(c));
    case DIG_OUT_HOT: return to_host(c, (double*)out, w.hot, dig_nh(c));
    case DIG_OUT_KN: return to_host(c, (double*)out, w.kn, 1);
    case DIG_OUT_STATE: return to_host(c, (int32_t*)out, w.state, 1);
    case DIG_OUT_MPREV: return to_host(c, (double*)out, w.mprev, dig_nv(c));
    default: return fail(c, DSMC_E_INVALID, "unknown coupling output");
    }
}

dsmc_status dig_residual(dsmc_ctx c, const double* prim, const double* hot, double* out) {
    dsmc_status st = usable(c);
    if (st != DSMC_OK) return st;
    if (!prim || !hot || !out) return fail(c, DSMC_E_INVALID, "NULL array");
    DigState* d = c->dig;
    if ((st = to_device(c, d->w.stage, prim, dig_nv(c))) != DSMC_OK) return st;
    if ((st = to_device(c, d->w.nhot, hot, dig_nh(c))) != DSMC_OK) return st;
    launch_dig_ctl_reset(c->stream, d->w.ctl);
    launch_dig_gradients(c->stream, d->g, d->w.stage, d->w.grad, d->w.ctl);
    launch_dig_face_hot(c->stream, d->g, d->w.stage, d->w.grad, d->w.nhot, d->w.hotf, 0);
    launch_dig_residual(c->stream, d->g, d->w.stage, d->w.hotf, d->w.grad, d->w.Rs, d->w, 0, 1.0);
    HIP_TRY(c, hipGetLastError());
    return to_host(c, out, d->w.Rs, dig_nv(c));
}

dsmc_status dig_solve(dsmc_ctx c, double* prim, const double* hot, const dig_params* p, dig_report* rep) {
    dsmc_status st = usable(c);
    if (st != DSMC_OK) return st;
    if ((st = check_params(c, p)) != DSMC_OK) return st;
    if (!prim || !hot) return fail(c, DSMC_E_INVALID, "NULL array");
    if (c->dr && p->accel > 0) return fail(c, DSMC_E_INVALID, "the accelerated solve is monatomic");
    DigState* d = c->dig;
    if ((st = to_device(c, d->w.prim, (const double*)prim, dig_nv(c))) != DSMC_OK) return st;
    if ((st = to_device(c, d->w.hot, hot, dig_nh(c))) != DSMC_OK) return st;
    launch_dig_gradients(c->stream, d->g, d->w.prim, d->w.grad, nullptr);
    launch_dig_face_hot(c->stream, d->g, d->w.prim, d->w.grad, d->w.hot, d->w.hotf, 0);
    dig_report r{};
    if ((st = run_solve(c, p, &r)) != DSMC_OK) return st;
    if ((st = to_host(c, prim, d->w.prim, dig_nv(c))) != DSMC_OK) return st;
    if (rep) *rep = r;
    return DSMC_OK;
}

dsmc_status dig_feedback(dsmc_ctx c, const double* prim_old, const double* prim_new, const int32_t* state,
                         int64_t* np_after) {
    dsmc_status st = usable(c);
    if (st != DSMC_OK) return st;
    if (!prim_old || !prim_new || !state) return fail(c, DSMC_E_INVALID, "NULL array");
    DigState* d = c->dig;
    if ((st = to_device(c, d->w.half, prim_old, dig_nv(c))) != DSMC_OK) return st;
    if ((st = to_device(c, d->w.prim, prim_new, dig_nv(c))) != DSMC_OK) return st;
    if ((st = to_device(c, d->w.state, state, 1)) != DSMC_OK) return st;
    if ((st = run_feedback(c)) != DSMC_OK) return st;
    if (np_after) {
        Scalars sc;
        if ((st = sync_scalars(c, &sc)) != DSMC_OK) return st;
        *np_after = sc.np;
    }
    return DSMC_OK;
}

dsmc_status dig_batch_enable(dsmc_ctx c, const int32_t* enabled) {
    dsmc_status st = usable(c);
    if (st != DSMC_OK) return st;
    if (!c->n_cases || !enabled) return fail(c, DSMC_E_INVALID, "not a batch context or NULL array");
    std::vector<DigCase> h(c->n_cases);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(h.data(), c->dig->g.cases, sizeof(DigCase) * h.size(), hipMemcpyDeviceToHost));
    for (int k = 0; k < c->n_cases; ++k) h[k].enabled = enabled[k] != 0;
    HIP_TRY(c, hipMemcpy(c->dig->g.cases, h.data(), sizeof(DigCase) * h.size(), hipMemcpyHostToDevice));
    return DSMC_OK;
}

dsmc_status dig_set_closure(dsmc_ctx c, dsmc_mlp net, double gate_tol) {
    if (!c || !(gate_tol >= 0)) return fail(c, DSMC_E_INVALID, "bad arguments");
    if (c->dr && net) return fail(c, DSMC_E_INVALID, "the learned closure predicts monatomic HoT");
    c->closure = net;
    c->gate_tol = gate_tol;
    return DSMC_OK;
}

dsmc_status dig_closure_data(dsmc_ctx c, float* x, float* t, uint8_t* valid) {
    dsmc_status st = usable(c);
    if (st != DSMC_OK) return st;
    const DigWork& w = c->dig->w;
    if (x && (st = to_host(c, x, w.cx, 13)) != DSMC_OK) return st;
    if (t && (st = to_host(c, t, w.ct, 9)) != DSMC_OK) return st;
    if (valid && (st = to_host(c, valid, w.cvalid, 1)) != DSMC_OK) return st;
    return DSMC_OK;
}

dsmc_status dsmc_set_rot_sums(dsmc_ctx c, int32_t which, const double* sums) {
    if (!c || !sums || (which != DSMC_SAMPLE_STEADY && which != DSMC_SAMPLE_EWMA))
        return fail(c, DSMC_E_INVALID, "bad arguments");
    if (c->broken) return fail(c, DSMC_E_INVALID, "context is in an error state");
    if (!c->dr) return fail(c, DSMC_E_INVALID, "the gas has no rotational degrees of freedom");
    const int nt = c->nt;
    std::vector<double> h((size_t)4 * nt);
    for (int t = 0; t < nt; ++t)
        for (int k = 0; k < 4; ++k) h[(size_t)k * nt + t] = sums[(size_t)4 * c->hm.orig[t] + k];
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(which == DSMC_SAMPLE_STEADY ? c->d_racc : c->d_rewma, h.data(), sizeof(double) * h.size(),
                         hipMemcpyHostToDevice));
    return DSMC_OK;
}

dsmc_status dsmc_set_sums(dsmc_ctx c, int32_t which, const double* sums, const int32_t* counts) {
    if (!c || !sums || (which != DSMC_SAMPLE_STEADY && which != DSMC_SAMPLE_EWMA))
        return fail(c, DSMC_E_INVALID, "bad arguments");
    if (c->broken) return fail(c, DSMC_E_INVALID, "context is in an error state");
    const int nt = c->nt;
    std::vector<double> h((size_t)kNMom * nt);
    for (int t = 0; t < nt; ++t)
        for (int k = 0; k < kNMom; ++k) h[(size_t)k * nt + t] = sums[(size_t)kNMom * c->hm.orig[t] + k];
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(which == DSMC_SAMPLE_STEADY ? c->d_acc : c->d_ewma, h.data(), sizeof(double) * h.size(),
                         hipMemcpyHostToDevice));
    if (which == DSMC_SAMPLE_EWMA && counts) {
        std::vector<int32_t> m(nt);
        for (int t = 0; t < nt; ++t) m[t] = counts[c->hm.orig[t]];
        HIP_TRY(c, hipMemcpy(c->d_ewma_m, m.data(), sizeof(int32_t) * nt, hipMemcpyHostToDevice));
    }
    return DSMC_OK;
}

}  // extern "C"
