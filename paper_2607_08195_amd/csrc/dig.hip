// Kernels of the DIG coupling step (section 3, Algorithm 1).
//
//   k_dig_sampled   moving-average sums -> sampled (rho, u, T, sigma, q)
//   k_dig_kn        local Knudsen number of eq. cell_kn_stability
//   k_dig_grad      weighted least-squares gradients of the primitives
//   k_dig_hot       NSF stress / heat flux and HoT = sampled - NSF
//   k_dig_gate_*    admissibility gate and Jacobi reconstruction passes
//   k_dig_save / k_dig_residual / k_dig_check / k_dig_update / k_dig_commit
//                   one three-stage pseudo-time iteration of the
//                   finite-volume macroscopic equations with frozen HoT
//   k_dig_fb_*      particle feedback: target counts, shift-scale,
//                   delete / clone
//
// One thread per cell except the feedback apply kernel (one wave per cell).
// Per-cell arithmetic is written as a fixed sequence of IEEE binary64
// operations (the library is built with contraction off).
#include "dig.h"

namespace dsmcx {

namespace {

constexpr double kGamma = 5.0 / 3.0;
constexpr double kMachCut = 0.05;

// Per-cell widths: NV primitives (5, or 6 with rotation), NH HoT (9 or 12),
// NS sampled values (14 or 18).
template <int NV> struct Widths {
    static constexpr int NH = NV == 6 ? 12 : 9;
    static constexpr int NS = NV == 6 ? 18 : 14;
    static constexpr int NG = 3 * NV;
};

__device__ __forceinline__ bool stopped(const DigCtl* ctl) { return ctl != nullptr && (ctl->conv | ctl->failed); }

__device__ __forceinline__ double mu_of(const DigGeom& g, double T) { return g.mu_ref * pow(T / g.T_ref, g.omega); }
__device__ __forceinline__ double kappa_of(const DigGeom& g, double mu) {
    return 15.0 * kBoltzmannDev * mu / (4.0 * g.mass);
}
// Translational and rotational conductivities of a rotating gas
// (eq. thermal_conductivity_matrix): (mu R / 2) A^{-1} (5, d_r).
__device__ __forceinline__ void kappas_of(const DigGeom& g, double mu, double& kt, double& kr) {
    const double det = g.a_heat[0] * g.a_heat[3] - g.a_heat[1] * g.a_heat[2];
    const double f = (mu * g.R) / 2.0;
    kt = f * ((g.a_heat[3] * 5.0 - g.a_heat[1] * (double)g.dr) / det);
    kr = f * ((g.a_heat[0] * (double)g.dr - g.a_heat[2] * 5.0) / det);
}
// ratio of specific heats of the frozen gas
template <int NV>
__device__ __forceinline__ double gamma_of(const DigGeom& g) {
    if constexpr (NV == 6) return (5.0 + g.dr) / (3.0 + g.dr);
    return kGamma;
}

// NSF stress (xx,yy,zz,xy,xz,yz) and Fourier heat flux (eq. nsf_heat_flux)
// from gu[i][j] = du_i/dx_j and gT at temperature T; with rotation the
// translational and rotational heat fluxes from gT and gTr.
template <int NV>
__device__ void nsf_local(const DigGeom& g, double T, const double* gu, const double* gT, const double* gTr,
                          double* out) {
    const double mu = mu_of(g, T);
    const double div = gu[0] + gu[4] + gu[8];
    const int ii[6] = {0, 1, 2, 0, 0, 1}, jj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        double e = gu[3 * ii[k] + jj[k]] + gu[3 * jj[k] + ii[k]];
        if (k < 3) e -= (2.0 / 3.0) * div;
        out[k] = -mu * e;
    }
    if constexpr (NV == 6) {
        double kt, kr;
        kappas_of(g, mu, kt, kr);
#pragma unroll
        for (int j = 0; j < 3; ++j) out[6 + j] = -kt * gT[j];
#pragma unroll
        for (int j = 0; j < 3; ++j) out[9 + j] = -kr * gTr[j];
    } else {
        const double kap = kappa_of(g, mu);
#pragma unroll
        for (int j = 0; j < 3; ++j) out[6 + j] = -kap * gT[j];
    }
}

template <int NV>
__device__ __forceinline__ void cons_of(const DigGeom& g, const double* P, double* U) {
    const double uu = P[1] * P[1] + P[2] * P[2] + P[3] * P[3];
    U[0] = P[0];
    U[1] = P[0] * P[1];
    U[2] = P[0] * P[2];
    U[3] = P[0] * P[3];
    if constexpr (NV == 6) {
        // total energy with e_r = (d_r/2) R T_r, and rho e_r (eq. energy_definitions)
        const double er = (0.5 * g.dr) * g.R * P[5];
        U[4] = P[0] * ((1.5 * g.R * P[4] + 0.5 * uu) + er);
        U[5] = P[0] * er;
    } else {
        U[4] = P[0] * (1.5 * g.R * P[4] + 0.5 * uu);
    }
}

template <int NV>
__device__ __forceinline__ bool prim_of(const DigGeom& g, const double* U, double* P) {
    if (!(U[0] > 0)) return false;
    P[0] = U[0];
    P[1] = U[1] / U[0];
    P[2] = U[2] / U[0];
    P[3] = U[3] / U[0];
    const double uu = P[1] * P[1] + P[2] * P[2] + P[3] * P[3];
    if constexpr (NV == 6) {
        const double er = U[5] / U[0];
        P[4] = ((U[4] / U[0] - 0.5 * uu) - er) / (1.5 * g.R);
        P[5] = er / ((0.5 * g.dr) * g.R);
        return P[4] > 0 && isfinite(P[4]) && P[5] > 0 && isfinite(P[5]);
    }
    P[4] = (U[4] / U[0] - 0.5 * uu) / (1.5 * g.R);
    return P[4] > 0 && isfinite(P[4]);
}

// Inviscid flux F(P).n of eq. macro (pressure rho R T_t).
template <int NV>
__device__ __forceinline__ void flux_of(const DigGeom& g, const double* P, const double* n, double* F) {
    const double un = P[1] * n[0] + P[2] * n[1] + P[3] * n[2];
    const double p = P[0] * g.R * P[4];
    const double uu = P[1] * P[1] + P[2] * P[2] + P[3] * P[3];
    F[0] = P[0] * un;
#pragma unroll
    for (int i = 0; i < 3; ++i) F[1 + i] = P[0] * P[1 + i] * un + p * n[i];
    if constexpr (NV == 6) {
        const double er = (0.5 * g.dr) * g.R * P[5];
        const double E = (1.5 * g.R * P[4] + 0.5 * uu) + er;
        F[4] = (P[0] * E + p) * un;
        F[5] = P[0] * er * un;
    } else {
        const double E = 1.5 * g.R * P[4] + 0.5 * uu;
        F[4] = (P[0] * E + p) * un;
    }
}

template <int NV>
__device__ __forceinline__ double acoustic_speed(const DigGeom& g, const double* P, const double* n) {
    return fabs(P[1] * n[0] + P[2] * n[1] + P[3] * n[2]) + sqrt(gamma_of<NV>(g) * g.R * P[4]);
}

// Dissipation speed |u.n| + theta c, theta = min(1, max(Mach, 0.05)).
template <int NV>
__device__ __forceinline__ double wave_speed(const DigGeom& g, const double* P, const double* n) {
    const double c = sqrt(gamma_of<NV>(g) * g.R * P[4]);
    const double un = fabs(P[1] * n[0] + P[2] * n[1] + P[3] * n[2]);
    const double u = sqrt(P[1] * P[1] + P[2] * P[2] + P[3] * P[3]);
    double th = u / c;
    if (th < kMachCut) th = kMachCut;
    if (th > 1.0) th = 1.0;
    return un + th * c;
}

// Central flux with scalar dissipation between states L and R.
template <int NV>
__device__ __forceinline__ void central_flux(const DigGeom& g, const double* PL, const double* PR, const double* n,
                                             double* F, double& lam) {
    double FL[NV], FR[NV], UL[NV], UR[NV];
    flux_of<NV>(g, PL, n, FL);
    flux_of<NV>(g, PR, n, FR);
    cons_of<NV>(g, PL, UL);
    cons_of<NV>(g, PR, UR);
    const double aL = wave_speed<NV>(g, PL, n), aR = wave_speed<NV>(g, PR, n);
    const double lam_d = aL > aR ? aL : aR;
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * lam_d * (UR[v] - UL[v]);
    const double sL = acoustic_speed<NV>(g, PL, n), sR = acoustic_speed<NV>(g, PR, n);
    lam = sL > sR ? sL : sR;
}

// Face gradients of u and T (and T_r): base gradients plus the correction
// that makes their component along the connector dx equal the difference
// quotient.
template <int NV>
__device__ __forceinline__ void face_gradients(const double* gbase, const double* far, const double* near,
                                               const double* dx, double dl, double* gu, double* gT, double* gTr) {
#pragma unroll
    for (int v = 1; v < NV; ++v) {
        double gf[3], ga = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            gf[j] = gbase[3 * v + j];
            ga += gf[j] * dx[j] / dl;
        }
        const double jump = (far[v] - near[v]) / dl - ga;
#pragma unroll
        for (int j = 0; j < 3; ++j) gf[j] += jump * dx[j] / dl;
        if (v < 4) {
#pragma unroll
            for (int j = 0; j < 3; ++j) gu[3 * (v - 1) + j] = gf[j];
        } else if (v == 4) {
#pragma unroll
            for (int j = 0; j < 3; ++j) gT[j] = gf[j];
        } else {
#pragma unroll
            for (int j = 0; j < 3; ++j) gTr[j] = gf[j];
        }
    }
}

// Momentum and energy parts of the viscous flux: (sigma + q).n with the
// face velocity uf doing work; a rotating gas's q_r also enters rho e_r.
template <int NV>
__device__ __forceinline__ void add_viscous(const double* vis, const double* n, const double* uf, double* F) {
    const double S[3][3] = {{vis[0], vis[3], vis[4]}, {vis[3], vis[1], vis[5]}, {vis[4], vis[5], vis[2]}};
    double work = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double sn = S[i][0] * n[0] + S[i][1] * n[1] + S[i][2] * n[2];
        F[1 + i] += sn;
        work += sn * uf[i];
    }
    F[4] += work + (vis[6] * n[0] + vis[7] * n[1] + vis[8] * n[2]);
    if constexpr (NV == 6) {
        const double qr = vis[9] * n[0] + vis[10] * n[1] + vis[11] * n[2];
        F[4] += qr;
        F[5] += qr;
    }
}

template <int NV>
__device__ __forceinline__ double viscous_rate(const DigGeom& g, double T, double rho, double dl) {
    const double mu = mu_of(g, T);
    if constexpr (NV == 6) {
        double kt, kr;
        kappas_of(g, mu, kt, kr);
        double d = 4.0 * mu / (3.0 * rho);
        const double dt_ = kt / (1.5 * rho * g.R), dr_ = kr / ((0.5 * g.dr) * rho * g.R);
        if (dt_ > d) d = dt_;
        if (dr_ > d) d = dr_;
        return 2.0 * d / dl;
    }
    const double dmom = 4.0 * mu / (3.0 * rho), dth = kappa_of(g, mu) / (1.5 * rho * g.R);
    return 2.0 * (dmom > dth ? dmom : dth) / dl;
}

// Rotational relaxation source of rho e_r (eq. macro):
// (d_r/2) rho R (T - T_r) / (Z_r tau), T = (3 T_t + d_r T_r)/(3 + d_r),
// tau = mu(T_t)/p_t; rate = 1/(Z_r tau).
__device__ __forceinline__ double relax_source(const DigGeom& g, const double* P, double& rate) {
    const double T = (3.0 * P[4] + g.dr * P[5]) / (3.0 + g.dr);
    const double tau = mu_of(g, P[4]) / (P[0] * g.R * P[4]);
    rate = 1.0 / (g.zr * tau);
    return (((0.5 * g.dr) * P[0]) * g.R) * (T - P[5]) * rate;
}

__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ void block_sum_min(double s, double m, double* out_s, double* out_m) {
    __shared__ double ss[kDigThreads], sm[kDigThreads];
    const int t = threadIdx.x;
    ss[t] = s;
    sm[t] = m;
    __syncthreads();
    for (int o = kDigThreads / 2; o > 0; o >>= 1) {
        if (t < o) {
            ss[t] += ss[t + o];
            sm[t] = fmin(sm[t], sm[t + o]);
        }
        __syncthreads();
    }
    if (t == 0) {
        *out_s = ss[0];
        *out_m = sm[0];
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// sampled state (eq. sampled_macro_state_ch3 with the cell formulas of
// eq. dsmc_temperatures applied to the moving-average sums)
// ---------------------------------------------------------------------------
template <int NV>
__global__ void k_dig_sampled(DigGeom g, const double* ewma, const double* rewma, double FN, DigWork w) {
    constexpr int NS = Widths<NV>::NS;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nt) return;
    const int nt = g.nt;
    double S[kNMom];
#pragma unroll
    for (int k = 0; k < kNMom; ++k) S[k] = ewma[(int64_t)k * nt + c];
    double* o = w.samp + NS * (size_t)c;
    double* P = w.prim + NV * (size_t)c;
    if (!(S[0] > 0)) {
        for (int k = 0; k < NS; ++k) o[k] = __builtin_nan("");
        for (int v = 0; v < NV; ++v) P[v] = w.mprev[NV * (size_t)c + v];
        w.ok[c] = 0;
        return;
    }
    if (g.cases) FN = g.cases[g.cell_case[c]].FN;
    const double n = (FN * (S[0] / 1.0)) / g.vol[c];
    const double rho = g.mass * n;
    const double u0 = S[1] / S[0], u1 = S[2] / S[0], u2 = S[3] / S[0];
    const double Cxx = S[4] / S[0] - u0 * u0, Cyy = S[5] / S[0] - u1 * u1, Czz = S[6] / S[0] - u2 * u2;
    const double Cxy = S[7] / S[0] - u0 * u1, Cxz = S[8] / S[0] - u0 * u2, Cyz = S[9] / S[0] - u1 * u2;
    const double Ckk = Cxx + Cyy + Czz;
    const double T = (g.mass * Ckk) / (3.0 * kBoltzmannDev);
    o[0] = rho; o[1] = u0; o[2] = u1; o[3] = u2; o[4] = T;
    o[5] = rho * (Cxx - Ckk / 3.0);
    o[6] = rho * (Cyy - Ckk / 3.0);
    o[7] = rho * (Czz - Ckk / 3.0);
    o[8] = rho * Cxy;
    o[9] = rho * Cxz;
    o[10] = rho * Cyz;
    const double S2kk = S[4] + S[5] + S[6];
    const double uu = u0 * u0 + u1 * u1 + u2 * u2;
    const double uS0 = u0 * S[4] + u1 * S[7] + u2 * S[8];
    const double uS1 = u0 * S[7] + u1 * S[5] + u2 * S[9];
    const double uS2 = u0 * S[8] + u1 * S[9] + u2 * S[6];
    o[11] = (rho / 2.0) * (((S[10] - 2.0 * uS0) - u0 * S2kk) + 2.0 * S[0] * u0 * uu) / S[0];
    o[12] = (rho / 2.0) * (((S[11] - 2.0 * uS1) - u1 * S2kk) + 2.0 * S[0] * u1 * uu) / S[0];
    o[13] = (rho / 2.0) * (((S[12] - 2.0 * uS2) - u2 * S2kk) + 2.0 * S[0] * u2 * uu) / S[0];
    if constexpr (NV == 6) {
        // rotational temperature and heat flux of the same sums
        const double r0 = rewma[c], r1 = rewma[(int64_t)nt + c], r2 = rewma[2 * (int64_t)nt + c],
                     r3 = rewma[3 * (int64_t)nt + c];
        o[14] = (2.0 * (r0 / S[0])) / ((double)g.dr * kBoltzmannDev);
        const double f = FN / (g.vol[c] * 1.0);
        o[15] = f * (r1 - (S[1] / S[0]) * r0);
        o[16] = f * (r2 - (S[2] / S[0]) * r0);
        o[17] = f * (r3 - (S[3] / S[0]) * r0);
    }
    const bool ok = isfinite(rho) && rho > 0;
    for (int v = 0; v < 5; ++v) P[v] = ok ? o[v] : w.mprev[NV * (size_t)c + v];
    if constexpr (NV == 6) P[5] = ok ? o[14] : w.mprev[NV * (size_t)c + 5];
    w.ok[c] = ok ? 1 : 0;
}

// Kn_Delta = (Kn (T/T0)^(omega-1/2) / (rho/rho0)) / (d_c / L0), d_c = 2 (3V/4pi)^(1/3)
// (eq. cell_kn_stability); infinite for cells without samples.
template <int NV>
__global__ void k_dig_kn(DigGeom g, DigWork w, double kn_ref, double T0, double rho0, double L0) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nt) return;
    const double rho = w.prim[NV * (size_t)c], T = w.prim[NV * (size_t)c + 4];
    if (g.cases) {
        const DigCase& k = g.cases[g.cell_case[c]];
        kn_ref = k.mu0 / (k.p0 * L0) * k.kfac;
        T0 = k.T0;
        rho0 = k.rho0;
    }
    const double lam = kn_ref * pow(T / T0, g.omega - 0.5) / (rho / rho0);
    const double dc = 2.0 * cbrt(3.0 * g.vol[c] / (4.0 * M_PI)) / L0;
    const double k = lam / dc;
    const bool fin = rho > 0 && T > 0 && isfinite(k);
    w.kn[c] = (w.ok[c] && fin) ? k : __builtin_inf();
}

// Weighted least squares over face neighbours: a diffuse wall contributes
// its velocity and temperature (both temperatures of a rotating gas) and the
// cell's own density at the face centroid; specular, inflow and outflow
// faces contribute nothing.  Batch, inside the coupling step's solve: cells
// of cases that are not coupled are left out (cases share no faces, so no
// coupled cell reads them).
__device__ __forceinline__ bool idle_cell(const DigGeom& g, int c) {
    return g.skip_idle && !g.cases[g.cell_case[c]].enabled;
}

// One lane per (cell, face), four consecutive lanes per cell: each lane
// forms its face's weighted difference terms; the cell's sums are taken over
// the four lanes in face order (a face without a value adds +0, which leaves
// the sum unchanged), and each lane writes a quarter of the gradient.
template <int NV>
__global__ __launch_bounds__(kDigThreads) void k_dig_grad(DigGeom g, const double* prim, double* grad, const DigCtl* ctl) {
    if (stopped(ctl)) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = (int)(t >> 2), f = (int)(t & 3);
    const bool live = c < g.nt && !idle_cell(g, c);
    double tb[NV][3];
#pragma unroll
    for (int v = 0; v < NV; ++v) tb[v][0] = tb[v][1] = tb[v][2] = 0.0;
    if (live) {
        const int link = g.flink[4 * (size_t)c + f];
        const int kind = link & 7, idx = link >> 3;
        const bool inner = kind == kLinkInterior || kind == kLinkPeriodic;
        if (inner || kind == kLinkWall) {
            double pc[NV], far[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) pc[v] = prim[NV * (size_t)c + v];
            if (inner) {
#pragma unroll
                for (int v = 0; v < NV; ++v) far[v] = prim[NV * (size_t)idx + v];
            } else {
                const DigGroup& gr = g.groups[idx];
                far[0] = pc[0];
                far[1] = gr.u[0]; far[2] = gr.u[1]; far[3] = gr.u[2];
                far[4] = gr.T;
                if constexpr (NV == 6) far[5] = gr.T;
            }
            const double* dx = g.fdx + 12 * (size_t)c + 3 * f;
            const double d0 = dx[0], d1 = dx[1], d2 = dx[2];
            const double wgt = 1.0 / (d0 * d0 + d1 * d1 + d2 * d2);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double dphi = far[v] - pc[v];
                tb[v][0] = wgt * d0 * dphi;
                tb[v][1] = wgt * d1 * dphi;
                tb[v][2] = wgt * d2 * dphi;
            }
        }
    }
    const int q0 = (int)(threadIdx.x & 63) & ~3;
    double b[NV][3];
#pragma unroll
    for (int v = 0; v < NV; ++v) b[v][0] = b[v][1] = b[v][2] = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int i = 0; i < 3; ++i) b[v][i] += __shfl(tb[v][i], q0 + k, 64);
    if (!live) return;
    const double* L = g.lsq + 9 * (size_t)c;
    double* o = grad + 3 * NV * (size_t)c;
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int i = 0; i < 3; ++i)
            if ((3 * v + i) % 4 == f) o[3 * v + i] = L[3 * i] * b[v][0] + L[3 * i + 1] * b[v][1] + L[3 * i + 2] * b[v][2];
}

// HoT = (sigma, q)_sampled - (sigma, q)_NSF at the sampled state
// (eq. hot_extraction_ch3); zero for cells without samples.
template <int NV>
__global__ void k_dig_hot(DigGeom g, DigWork w) {
    constexpr int NH = Widths<NV>::NH, NS = Widths<NV>::NS;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nt) return;
    const double* gr = w.grad + 3 * NV * (size_t)c;
    double nsf[NH];
    nsf_local<NV>(g, w.prim[NV * (size_t)c + 4], gr + 3, gr + 12, gr + 15, nsf);
    const bool ok = w.ok[c];
    const double* a = w.samp + NS * (size_t)c;
#pragma unroll
    for (int k = 0; k < 9; ++k) w.hot[NH * (size_t)c + k] = ok ? a[5 + k] - nsf[k] : 0.0;
    if constexpr (NV == 6) {
#pragma unroll
        for (int k = 0; k < 3; ++k) w.hot[NH * (size_t)c + 9 + k] = ok ? a[15 + k] - nsf[9 + k] : 0.0;
    }
}

// The state a diffuse wall imposes: the cell's density, the wall's velocity
// and temperature (both temperatures).
template <int NV>
__device__ __forceinline__ void wall_state(const DigGroup& gr, const double* Pc, double* wv) {
    wv[0] = Pc[0];
    wv[1] = gr.u[0]; wv[2] = gr.u[1]; wv[3] = gr.u[2];
    wv[4] = gr.T;
    if constexpr (NV == 6) wv[5] = gr.T;
}

// HoT carried by each cell face: the cell HoT averaged to the face (the
// cell's own at a diffuse wall); with `consistent`, plus the cell NSF
// stresses averaged to the face minus the face NSF stress of the viscous
// flux, both at prim, so that at prim each face's viscous stress is the
// average of its cells' NSF + HoT.
template <int NV>
__global__ void k_dig_face_hot(DigGeom g, const double* prim, const double* grad, const double* hot, double* hotf,
                               int consistent) {
    constexpr int NH = Widths<NV>::NH, NG = Widths<NV>::NG;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nt) return;
    double Pc[NV], gc[NG], nc[NH];
    for (int v = 0; v < NV; ++v) Pc[v] = prim[NV * (size_t)c + v];
    for (int k = 0; k < NG; ++k) gc[k] = grad[NG * (size_t)c + k];
    nsf_local<NV>(g, Pc[4], gc + 3, gc + 12, gc + 15, nc);
    for (int f = 0; f < 4; ++f) {
        const int link = g.flink[4 * c + f];
        const int kind = link & 7, idx = link >> 3;
        const size_t fo = 12 * (size_t)c + 3 * f;
        const double dx[3] = {g.fdx[fo], g.fdx[fo + 1], g.fdx[fo + 2]};
        const double dl = sqrt(dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]);
        double* h = hotf + 4 * NH * (size_t)c + NH * f;
        double gu[9], gT[3], gTr[3], vf[NH];
        if (kind == kLinkInterior || kind == kLinkPeriodic) {
            const int nb = idx;
            double Pn[NV], gn[NG], gavg[NG], nn[NH];
            for (int v = 0; v < NV; ++v) Pn[v] = prim[NV * (size_t)nb + v];
            for (int k = 0; k < NG; ++k) gn[k] = grad[NG * (size_t)nb + k];
            for (int k = 0; k < NG; ++k) gavg[k] = 0.5 * (gc[k] + gn[k]);
            face_gradients<NV>(gavg, Pn, Pc, dx, dl, gu, gT, gTr);
            nsf_local<NV>(g, 0.5 * (Pc[4] + Pn[4]), gu, gT, gTr, vf);
            nsf_local<NV>(g, Pn[4], gn + 3, gn + 12, gn + 15, nn);
            for (int k = 0; k < NH; ++k) {
                double v = 0.5 * (hot[NH * (size_t)c + k] + hot[NH * (size_t)nb + k]);
                if (consistent) v += 0.5 * (nc[k] + nn[k]) - vf[k];
                h[k] = v;
            }
        } else if (kind == kLinkWall) {
            const DigGroup& gr = g.groups[idx];
            double wallv[NV];
            wall_state<NV>(gr, Pc, wallv);
            face_gradients<NV>(gc, wallv, Pc, dx, dl, gu, gT, gTr);
            nsf_local<NV>(g, gr.T, gu, gT, gTr, vf);
            for (int k = 0; k < NH; ++k) {
                double v = hot[NH * (size_t)c + k];
                if (consistent) v += nc[k] - vf[k];
                h[k] = v;
            }
        } else {
            for (int k = 0; k < NH; ++k) h[k] = 0.0;
        }
    }
}

// Admissibility (criterion on Kn_Delta) and availability of every cell.
template <int NV>
__global__ void k_dig_gate_init(DigGeom g, DigWork w, double kn_max) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nt) return;
    bool ok = w.kn[c] <= kn_max;
    for (int v = 0; v < NV && ok; ++v) ok = isfinite(w.prim[NV * (size_t)c + v]);
    w.avail[c] = ok ? 1 : 0;
    w.navail[c] = ok ? 1 : 0;
    w.state[c] = ok ? 0 : 2;
}

// One reconstruction pass: every unavailable cell with available face
// neighbours takes their equal-weight mean of M and HoT.  Results become
// visible to neighbours only in the next pass (k_dig_gate_commit).
template <int NV>
__global__ void k_dig_gate_pass(DigGeom g, DigWork w) {
    constexpr int NH = Widths<NV>::NH;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nt || w.avail[c]) return;
    int cnt = 0;
    double sp[NV], sh[NH];
#pragma unroll
    for (int v = 0; v < NV; ++v) sp[v] = 0.0;
#pragma unroll
    for (int v = 0; v < NH; ++v) sh[v] = 0.0;
    for (int f = 0; f < 4; ++f) {
        const int link = g.flink[4 * c + f];
        const int kind = link & 7, nb = link >> 3;
        if ((kind != kLinkInterior && kind != kLinkPeriodic) || !w.avail[nb]) continue;
        ++cnt;
#pragma unroll
        for (int v = 0; v < NV; ++v) sp[v] += w.prim[NV * (size_t)nb + v];
#pragma unroll
        for (int v = 0; v < NH; ++v) sh[v] += w.hot[NH * (size_t)nb + v];
    }
    if (!cnt) return;
#pragma unroll
    for (int v = 0; v < NV; ++v) w.nprim[NV * (size_t)c + v] = sp[v] / cnt;
#pragma unroll
    for (int v = 0; v < NH; ++v) w.nhot[NH * (size_t)c + v] = sh[v] / cnt;
    w.navail[c] = 1;
    w.state[c] = 1;
}

template <int NV>
__global__ void k_dig_gate_commit(DigGeom g, DigWork w) {
    constexpr int NH = Widths<NV>::NH;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nt) return;
    if (w.navail[c] && !w.avail[c]) {
        for (int v = 0; v < NV; ++v) w.prim[NV * (size_t)c + v] = w.nprim[NV * (size_t)c + v];
        for (int v = 0; v < NH; ++v) w.hot[NH * (size_t)c + v] = w.nhot[NH * (size_t)c + v];
        w.avail[c] = 1;
    }
}

// Unreached cells keep M^k with zero HoT; counts of the report.
template <int NV>
__global__ void k_dig_gate_final(DigGeom g, DigWork w) {
    constexpr int NH = Widths<NV>::NH;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    int rej = 0, rec = 0, unr = 0;
    if (c < g.nt) {
        const int st = w.state[c];
        rej = st != 0;
        rec = st == 1;
        unr = st == 2;
        if (st == 2) {
            for (int v = 0; v < NV; ++v) w.prim[NV * (size_t)c + v] = w.mprev[NV * (size_t)c + v];
            for (int v = 0; v < NH; ++v) w.hot[NH * (size_t)c + v] = 0.0;
        }
    }
    rej = wave_sum_i(rej);
    rec = wave_sum_i(rec);
    unr = wave_sum_i(unr);
    if ((threadIdx.x & 63) == 0) {
        if (rej) atomicAdd(&w.ctl->n_rejected, rej);
        if (rec) atomicAdd(&w.ctl->n_reconstructed, rec);
        if (unr) atomicAdd(&w.ctl->n_unreached, unr);
    }
}

__global__ void k_dig_ctl_reset(DigCtl* ctl) {
    ctl->res0 = 0.0;
    ctl->res = 0.0;
    ctl->dtmin = 0.0;
    ctl->conv = 0;
    ctl->failed = 0;
    ctl->iters = 0;
    ctl->n_rejected = 0;
    ctl->n_reconstructed = 0;
    ctl->n_unreached = 0;
    ctl->n_closure = 0;
    ctl->n_fallback = 0;
    ctl->mass_scale = 1.0;
}

__global__ void k_dig_copy(const double* src, double* dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// finite-volume residual: R_c = sum_f (F_inviscid + F_viscous).n A_f
// (minus V times the relaxation source in the rho e_r equation)
// ---------------------------------------------------------------------------
// One lane per (cell, face), four consecutive lanes per cell: each lane
// computes its face's flux; the cell's sums are then formed from the four
// lanes' terms in face order (the order of a loop over the faces), so that
// four times as many lanes keep the gathered neighbour loads in flight.
template <int NV>
__global__ __launch_bounds__(kDigThreads) void k_dig_residual(DigGeom g, const double* prim, const double* hotf,
                                                              const double* grad, double* Rs, DigWork w, int first,
                                                              double cfl) {
    constexpr int NH = Widths<NV>::NH, NG = Widths<NV>::NG;
    if (stopped(w.ctl)) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = (int)(t >> 2), f = (int)(t & 3);
    const bool live = c < g.nt && !idle_cell(g, c);
    double FA[NV], SA = 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) FA[v] = 0.0;
    double Pc[NV];
    if (live) {
        double gc[NG];
#pragma unroll
        for (int v = 0; v < NV; ++v) Pc[v] = prim[NV * (size_t)c + v];
#pragma unroll
        for (int k = 0; k < NG; ++k) gc[k] = grad[NG * (size_t)c + k];
        const double xc[3] = {g.cen[3 * (size_t)c], g.cen[3 * (size_t)c + 1], g.cen[3 * (size_t)c + 2]};
        const int link = g.flink[4 * (size_t)c + f];
        const int kind = link & 7, idx = link >> 3;
        const bool inner = kind == kLinkInterior || kind == kLinkPeriodic;
        // the neighbour's state and gradients are requested with the face's
        // geometry (a face without a neighbour cell reads its own cell's,
        // unused)
        const size_t nb = inner ? (size_t)idx : (size_t)c;
        double Pn[NV], gn[NG];
#pragma unroll
        for (int v = 0; v < NV; ++v) Pn[v] = prim[NV * nb + v];
#pragma unroll
        for (int k = 0; k < NG; ++k) gn[k] = grad[NG * nb + k];
        const size_t fo = 12 * (size_t)c + 3 * f;
        const double n[3] = {g.fnu[fo], g.fnu[fo + 1], g.fnu[fo + 2]};
        const double dx[3] = {g.fdx[fo], g.fdx[fo + 1], g.fdx[fo + 2]};
        const double A = g.farea[4 * (size_t)c + f];
        double F[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) F[v] = 0.0;
        double lam = 0.0, lamv = 0.0;
        if (inner) {
            const double xf[3] = {g.fcen[fo], g.fcen[fo + 1], g.fcen[fo + 2]};
            double rc[3], rn[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                rc[i] = xf[i] - xc[i];
                rn[i] = xf[i] - (xc[i] + dx[i]);
            }
            double PL[NV], PR[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                PL[v] = Pc[v] + (gc[3 * v] * rc[0] + gc[3 * v + 1] * rc[1] + gc[3 * v + 2] * rc[2]);
                PR[v] = Pn[v] + (gn[3 * v] * rn[0] + gn[3 * v + 1] * rn[1] + gn[3 * v + 2] * rn[2]);
            }
            bool pos = PL[0] > 0 && PL[4] > 0 && PR[0] > 0 && PR[4] > 0;
            if constexpr (NV == 6) pos = pos && PL[5] > 0 && PR[5] > 0;
            if (!pos) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    PL[v] = Pc[v];
                    PR[v] = Pn[v];
                }
            }
            central_flux<NV>(g, PL, PR, n, F, lam);
            const double d2 = dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2];
            const double dl = sqrt(d2);
            double gavg[NG];
#pragma unroll
            for (int k = 3; k < NG; ++k) gavg[k] = 0.5 * (gc[k] + gn[k]);
            double gu[9], gT[3], gTr[3];
            face_gradients<NV>(gavg, Pn, Pc, dx, dl, gu, gT, gTr);
            const double Tf = 0.5 * (Pc[4] + Pn[4]);
            const double rf = 0.5 * (Pc[0] + Pn[0]);
            double vis[NH];
            nsf_local<NV>(g, Tf, gu, gT, gTr, vis);
            const double* hf = hotf + 4 * NH * (size_t)c + NH * f;
#pragma unroll
            for (int k = 0; k < NH; ++k) vis[k] += hf[k];
            const double uf[3] = {0.5 * (Pc[1] + Pn[1]), 0.5 * (Pc[2] + Pn[2]), 0.5 * (Pc[3] + Pn[3])};
            add_viscous<NV>(vis, n, uf, F);
            lamv = viscous_rate<NV>(g, Tf, rf, dl);
        } else if (kind == kLinkWall || kind == kLinkSpecular) {
            const double p = Pc[0] * g.R * Pc[4];
#pragma unroll
            for (int i = 0; i < 3; ++i) F[1 + i] = p * n[i];
            lam = acoustic_speed<NV>(g, Pc, n);
            if (kind == kLinkWall) {
                const DigGroup& gr = g.groups[idx];
                const double d2 = dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2];
                const double dl = sqrt(d2);
                double wallv[NV];
                wall_state<NV>(gr, Pc, wallv);
                double gu[9], gT[3], gTr[3];
                face_gradients<NV>(gc, wallv, Pc, dx, dl, gu, gT, gTr);
                double vis[NH];
                nsf_local<NV>(g, gr.T, gu, gT, gTr, vis);
                const double* hf = hotf + 4 * NH * (size_t)c + NH * f;
#pragma unroll
                for (int k = 0; k < NH; ++k) vis[k] += hf[k];
                add_viscous<NV>(vis, n, gr.u, F);
                lamv = viscous_rate<NV>(g, gr.T, Pc[0], dl);
            }
        } else if (kind == kLinkInflow) {
            const DigGroup& gr = g.groups[idx];
            double PR[NV];
            PR[0] = gr.rho; PR[1] = gr.u[0]; PR[2] = gr.u[1]; PR[3] = gr.u[2]; PR[4] = gr.T;
            if constexpr (NV == 6) PR[5] = gr.T;
            central_flux<NV>(g, Pc, PR, n, F, lam);
        } else {
            flux_of<NV>(g, Pc, n, F);
            lam = acoustic_speed<NV>(g, Pc, n);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) FA[v] = F[v] * A;
        SA = (lam + lamv) * A;
    }
    // the cell's sums over its four lanes, in face order (every lane of the
    // wave takes part in the exchange)
    const int q0 = (int)(threadIdx.x & 63) & ~3;
    double Rc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Rc[v] = 0.0;
    double sp = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int v = 0; v < NV; ++v) Rc[v] += __shfl(FA[v], q0 + k, 64);
        sp += __shfl(SA, q0 + k, 64);
    }
    double r2 = 0.0, dtc = __builtin_inf();
    if (live && f == 0) {
        if constexpr (NV == 6) {
            double rate;
            const double src = relax_source(g, Pc, rate);
            Rc[5] -= g.vol[c] * src;
            sp += g.vol[c] * rate;
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) Rs[NV * (size_t)c + v] = Rc[v];
        if (first) {
            dtc = cfl * g.vol[c] / sp;
            w.dt[c] = dtc;
            r2 = Rc[0] * Rc[0];
            if constexpr (NV == 6) {
                // the rotational-energy residual in mass units, R_er / (R T0)
                const double ert = g.cases ? g.R * g.cases[g.cell_case[c]].T0 : g.ert;
                const double r5 = Rc[5] / ert;
                r2 = r2 + r5 * r5;
            }
        }
    }
    if (first) block_sum_min(r2, dtc, &w.partial[2 * blockIdx.x], &w.partial[2 * blockIdx.x + 1]);
}

// Density residual norm (with rotation: and the rotational-energy residual),
// first-iteration reference, convergence test and the smallest local step
// (single workgroup).
__global__ __launch_bounds__(kDigThreads) void k_dig_check(DigWork w, int nblk, int it, double eps_m) {
    if (stopped(w.ctl)) return;
    double s = 0.0, m = __builtin_inf();
    for (int b = threadIdx.x; b < nblk; b += kDigThreads) {
        s += w.partial[2 * b];
        m = fmin(m, w.partial[2 * b + 1]);
    }
    __shared__ double tot, mn;
    block_sum_min(s, m, &tot, &mn);
    __syncthreads();
    if (threadIdx.x == 0) {
        DigCtl* ctl = w.ctl;
        const double res = sqrt(tot);
        ctl->res = res;
        if (it == 0) ctl->res0 = res;
        const double res0 = ctl->res0;
        if (!(res0 > 0) || res <= eps_m * res0) ctl->conv = 1;
        ctl->dtmin = mn;
    }
}

template <int NV>
__global__ void k_dig_save(DigGeom g, DigWork w) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nt || stopped(w.ctl) || idle_cell(g, c)) return;
    double P[NV], U[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        P[v] = w.prim[NV * (size_t)c + v];
        w.stage[NV * (size_t)c + v] = P[v];
    }
    cons_of<NV>(g, P, U);
#pragma unroll
    for (int v = 0; v < NV; ++v) w.U0[NV * (size_t)c + v] = U[v];
}

// Stage update U = U0 - alpha dt / V R(stage).
template <int NV>
__global__ void k_dig_update(DigGeom g, DigWork w, double alpha, int global_dt) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nt || stopped(w.ctl) || idle_cell(g, c)) return;
    const double dtc = global_dt ? w.ctl->dtmin : w.dt[c];
    double U[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v)
        U[v] = w.U0[NV * (size_t)c + v] - alpha * dtc / g.vol[c] * w.Rs[NV * (size_t)c + v];
    double P[NV];
    if (prim_of<NV>(g, U, P)) {
#pragma unroll
        for (int v = 0; v < NV; ++v) w.stage[NV * (size_t)c + v] = P[v];
    } else {
        if (U[0] > 0) {
#pragma unroll
            for (int v = 0; v < NV; ++v) w.stage[NV * (size_t)c + v] = P[v];
        }
        atomicOr(&w.ctl->failed, 1);
    }
}

template <int NV>
__global__ void k_dig_commit(DigGeom g, DigWork w) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nt || stopped(w.ctl)) return;
    if (c == 0) w.ctl->iters += 1;
    if (idle_cell(g, c)) return;
#pragma unroll
    for (int v = 0; v < NV; ++v) w.prim[NV * (size_t)c + v] = w.stage[NV * (size_t)c + v];
}

template <int NV>
__global__ __launch_bounds__(kDigThreads) void k_dig_mass_partial(DigGeom g, DigWork w) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const double m = c < g.nt ? w.prim[NV * (size_t)c] * g.vol[c] : 0.0;
    block_sum_min(m, 0.0, &w.partial[2 * blockIdx.x], &w.partial[2 * blockIdx.x + 1]);
}

__global__ __launch_bounds__(kDigThreads) void k_dig_mass_factor(DigGeom g, DigWork w, int nblk, const Scalars* sc) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kDigThreads) s += w.partial[2 * b];
    __shared__ double tot, dummy;
    block_sum_min(s, 0.0, &tot, &dummy);
    __syncthreads();
    if (threadIdx.x == 0) {
        const double mp = (double)sc->np * g.FN * g.mass;
        w.ctl->mass_scale = mp / tot;
    }
}

template <int NV>
__global__ void k_dig_mass_apply(DigGeom g, DigWork w) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < g.nt) w.prim[NV * (size_t)c] = w.prim[NV * (size_t)c] * w.ctl->mass_scale;
}

__global__ void k_dig_set_local(DigGeom g, const int32_t* state, uint8_t* local) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nt || (g.cases && !g.cases[g.cell_case[c]].enabled)) return;
    local[c] = state[c] != 0 ? 1 : 0;
}

// ---------------------------------------------------------------------------
// particle feedback (Algorithm 1: particles adjusted to M^{k+1})
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool fb_valid(const DigGeom& g, const double* a, const double* b) {
    bool ok = a[0] > 0 && b[0] > 0 && a[4] > 0 && b[4] > 0;
    if (g.dr) ok = ok && a[5] > 0 && b[5] > 0;
    return ok;
}

// Target count floor(rho_new V / (F_N m) + U) of each cell (unchanged when
// rho_new is the cell's particle density); clone counts in the caller's
// cell order (new pids follow that order).
__global__ void k_dig_fb_count(DigGeom g, DigWork w, const int32_t* offsets, const int32_t* orig, const Scalars* sc,
                               RngKey key) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nt) return;
    const int N = offsets[c + 1] - offsets[c];
    int T = N;
    const int nv = g.dr ? kDigNVR : kDigNV;
    const double* a = w.half + nv * (size_t)c;
    const double* b = w.prim + nv * (size_t)c;
    double FN = g.FN;
    uint32_t subject = (uint32_t)orig[c];
    bool on = true;
    if (g.cases) {
        const DigCase& k = g.cases[g.cell_case[c]];
        FN = k.FN;
        key.k0 = k.k0;
        key.k1 = k.k1;
        subject -= (uint32_t)k.cell0;
        on = k.enabled != 0;
    }
    if (on && w.state[c] <= 1 && N > 0 && fb_valid(g, a, b)) {
        const Rand4 r = draw(key, subject, sc->step, kPurposeRecalibrate, 0);
        double t = floor(b[0] * g.vol[c] / (FN * g.mass) + u01(r.w[0], r.w[1]));
        if (!(t < 1073741824.0)) t = 1073741824.0;
        T = (int)t;
    }
    w.fb_tgt[c] = T;
    w.fb_cnt[orig[c]] = T > N ? T - N : 0;
}

// One wave per cell: shift-scale the velocities, rank the particles by pid,
// then delete (one at a time among the remaining, in pid order) or clone.
template <class VT>
__global__ __launch_bounds__(kFbLanes) void k_dig_fb_apply(DigGeom g, DigWork w, PartDev<VT> p, const int32_t* offsets,
                                                           const int4* tv, const double* xyz, const int32_t* orig,
                                                           const Scalars* sc, RngKey key, int32_t* scratch,
                                                           uint32_t* bits, int64_t cap) {
    const int c = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t a0 = offsets[c];
    const int N = offsets[c + 1] - (int)a0;
    const int nv = g.dr ? kDigNVR : kDigNV;
    const double* a = w.half + nv * (size_t)c;
    const double* b = w.prim + nv * (size_t)c;
    uint32_t subject = (uint32_t)orig[c];
    uint32_t next_pid = sc->next_pid;
    int64_t pid_off = 0;
    if (g.cases) {
        const DigCase& k = g.cases[g.cell_case[c]];
        if (!k.enabled) return;
        key.k0 = k.k0;
        key.k1 = k.k1;
        subject -= (uint32_t)k.cell0;
        next_pid = k.next_pid;
        pid_off = w.fb_off[k.cell0];
    }
    if (w.state[c] > 1 || N == 0 || !fb_valid(g, a, b)) return;
    const double scale = sqrt(b[4] / a[4]);
    for (int i = lane; i < N; i += kFbLanes) {
        const int64_t k = a0 + i;
        p.vel[3 * k] = (VT)(b[1] + scale * ((double)p.vel[3 * k] - a[1]));
        p.vel[3 * k + 1] = (VT)(b[2] + scale * ((double)p.vel[3 * k + 1] - a[2]));
        p.vel[3 * k + 2] = (VT)(b[3] + scale * ((double)p.vel[3 * k + 2] - a[3]));
    }
    if (g.dr && p.ir) {
        // rotational energies scaled by the ratio of the rotational temperatures
        const double rs = b[5] / a[5];
        for (int i = lane; i < N; i += kFbLanes) p.ir[a0 + i] = rs * p.ir[a0 + i];
    }
    // logical (pid) order of the cell
    for (int i = lane; i < N; i += kFbLanes) {
        const uint32_t me = p.pid[a0 + i];
        int r = 0;
        for (int j = 0; j < N; ++j) r += p.pid[a0 + j] < me ? 1 : 0;
        scratch[a0 + r] = (int32_t)(a0 + i);
    }
    __syncthreads();
    const int T = w.fb_tgt[c];
    const uint32_t step = sc->step;
    if (T < N) {
        // Live ranks as a bitmap (in the cell's slice of `bits`); each lane
        // owns a contiguous run of words and keeps its live count in a
        // register, so a deletion touches one lane's words only.
        const int nw = (N + 31) >> 5;
        const int wpl = (nw + kFbLanes - 1) / kFbLanes;
        uint32_t* words = bits + a0;
        int cnt = 0;
        for (int j = 0; j < wpl; ++j) {
            const int wi = lane * wpl + j;
            if (wi < nw) {
                const uint32_t word = (wi < nw - 1 || (N & 31) == 0) ? 0xFFFFFFFFu : ((1u << (N & 31)) - 1u);
                words[wi] = word;
                cnt += __popc(word);
            }
        }
        int rem = N;
        for (int k = 0; k < N - T; ++k) {
            const Rand4 r = draw(key, subject, step, kPurposeRecalibrate, (uint64_t)(2 + 2 * k));
            const int idx = (int)pick(r.w[0], (uint32_t)rem);
            int inc = cnt;
            for (int o = 1; o < kFbLanes; o <<= 1) {
                const int y = __shfl_up(inc, o, kFbLanes);
                if (lane >= o) inc += y;
            }
            const int exc = inc - cnt;
            if (idx >= exc && idx < inc) {
                int need = idx - exc;
                for (int j = 0; j < wpl; ++j) {
                    const int wi = lane * wpl + j;
                    if (wi >= nw) break;
                    const uint32_t word = words[wi];
                    const int pc = __popc(word);
                    if (need < pc) {
                        int bit = 0;
                        for (; bit < 32; ++bit)
                            if ((word >> bit) & 1u) {
                                if (need == 0) break;
                                --need;
                            }
                        words[wi] = word & ~(1u << bit);
                        p.cell[scratch[a0 + wi * 32 + bit]] = -1;
                        break;
                    }
                    need -= pc;
                }
                --cnt;
            }
            --rem;
        }
    } else if (T > N) {
        const int4 q = tv[c];
        const double* A = xyz + 3 * (size_t)q.x;
        const double* B = xyz + 3 * (size_t)q.y;
        const double* C = xyz + 3 * (size_t)q.z;
        const double* D = xyz + 3 * (size_t)q.w;
        const int64_t base = sc->np + w.fb_off[orig[c]];
        const uint32_t pid0 = next_pid + (uint32_t)(w.fb_off[orig[c]] - pid_off);
        for (int k = lane; k < T - N; k += kFbLanes) {
            const Rand4 r1 = draw(key, subject, step, kPurposeRecalibrate, (uint64_t)(2 + 2 * k));
            const Rand4 r2 = draw(key, subject, step, kPurposeRecalibrate, (uint64_t)(3 + 2 * k));
            const int src = (int)pick(r1.w[0], (uint32_t)N);
            const int64_t si = scratch[a0 + src];
            double u1 = u01(r1.w[2], r1.w[3]), u2 = u01(r2.w[0], r2.w[1]), u3 = u01(r2.w[2], r2.w[3]), t;
            if (u1 > u2) { t = u1; u1 = u2; u2 = t; }
            if (u2 > u3) { t = u2; u2 = u3; u3 = t; }
            if (u1 > u2) { t = u1; u1 = u2; u2 = t; }
            const double w0 = u1, w1 = u2 - u1, w2 = u3 - u2, w3 = 1.0 - u3;
            const int64_t d = base + k;
            if (d >= cap) continue;
            p.pos[3 * d] = ((w0 * A[0] + w1 * B[0]) + w2 * C[0]) + w3 * D[0];
            p.pos[3 * d + 1] = ((w0 * A[1] + w1 * B[1]) + w2 * C[1]) + w3 * D[1];
            p.pos[3 * d + 2] = ((w0 * A[2] + w1 * B[2]) + w2 * C[2]) + w3 * D[2];
            p.vel[3 * d] = p.vel[3 * si];
            p.vel[3 * d + 1] = p.vel[3 * si + 1];
            p.vel[3 * d + 2] = p.vel[3 * si + 2];
            p.cell[d] = c;
            p.pid[d] = pid0 + (uint32_t)k;
            if (p.ir) p.ir[d] = p.ir[si];
        }
    }
}

// Histogram of the cells of the sorted particles and of the entries
// appended after them (feedback clones).
__global__ void k_dig_count_all(const int32_t* cell, const Scalars* sc, int32_t* counts, uint32_t* rank) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = i < sc->np + sc->ninj ? cell[i] : -1;
    const uint32_t slot = bin_slot(counts, c, c >= 0);
    if (c >= 0) rank[i] = slot;
}

__global__ void k_fill_u8(uint8_t* p, uint8_t v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// learned closure: inputs, targets and the gate against the sampled HoT
// ---------------------------------------------------------------------------
// Per cell with samples: lambda = Kn_Delta d_c (local mean free path);
// inputs lambda du_i/dx_j / sqrt(RT), lambda dT/dx_j / T, Kn_Delta; targets
// HoT / p and HoT_q / (p sqrt(RT)); the sampled stress and heat flux in the
// same units (the gate's scale).
__global__ void k_dig_closure_prep(DigGeom g, DigWork w) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nt) return;
    const double* P = w.prim + kDigNV * (size_t)c;
    const double kn = w.kn[c];
    const double rho = P[0], T = P[4];
    const bool valid = w.ok[c] && isfinite(kn) && rho > 0 && T > 0;
    float* x = w.cx + 13 * (size_t)c;
    float* t = w.ct + 9 * (size_t)c;
    float* sc = w.cs + 9 * (size_t)c;
    w.cvalid[c] = valid ? 1 : 0;
    if (!valid) {
        for (int k = 0; k < 13; ++k) x[k] = 0.f;
        for (int k = 0; k < 9; ++k) t[k] = sc[k] = 0.f;
        return;
    }
    const double dc = 2.0 * cbrt(3.0 * g.vol[c] / (4.0 * M_PI));
    const double lam = kn * dc;
    const double cs = sqrt(g.R * T);
    const double p = rho * g.R * T;
    const double* gr = w.grad + 15 * (size_t)c;
    for (int k = 0; k < 9; ++k) x[k] = (float)(lam * gr[3 + k] / cs);
    for (int k = 0; k < 3; ++k) x[9 + k] = (float)(lam * gr[12 + k] / T);
    x[12] = (float)kn;
    const double* h = w.hot + 9 * (size_t)c;
    const double* a = w.samp + 14 * (size_t)c;
    for (int k = 0; k < 6; ++k) {
        t[k] = (float)(h[k] / p);
        sc[k] = (float)(a[5 + k] / p);
    }
    for (int k = 6; k < 9; ++k) {
        t[k] = (float)(h[k] / (p * cs));
        sc[k] = (float)(a[5 + k] / (p * cs));
    }
}

// Take the network's HoT where its distance to the sampled HoT is at most
// tol times max(sqrt(|sampled stress, heat flux|^2 + noise^2), 1e-3), the
// noise being the sampling error of that nondimensional vector over the
// moving average's particle samples: 14.5 / (mean particles per step x
// min(samples taken, n_a)) (Gaussian moments: 3 x 4/3 + 3 x 1 + 3 x 5/2
// per particle).
__global__ void k_dig_closure_gate(DigGeom g, DigWork w, double tol, const double* ewma, const int32_t* ewma_m,
                                   int n_a) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    int used = 0, fell = 0;
    if (c < g.nt && w.cvalid[c]) {
        const float* y = w.cy + 9 * (size_t)c;
        const float* t = w.ct + 9 * (size_t)c;
        const float* sc = w.cs + 9 * (size_t)c;
        double d2 = 0.0, s2 = 0.0;
        for (int k = 0; k < 9; ++k) {
            const double d = (double)y[k] - (double)t[k];
            d2 += d * d;
            s2 += (double)sc[k] * (double)sc[k];
        }
        const int mc = ewma_m[c] < n_a ? ewma_m[c] : n_a;
        const double ns = ewma[c] * (double)mc;
        if (ns > 0) s2 += 14.5 / ns;
        const double e = sqrt(d2) / fmax(sqrt(s2), 1e-3);
        if (isfinite(e) && e <= tol) {
            const double* P = w.prim + kDigNV * (size_t)c;
            const double p = P[0] * g.R * P[4];
            const double cs = sqrt(g.R * P[4]);
            double* h = w.hot + 9 * (size_t)c;
            for (int k = 0; k < 6; ++k) h[k] = (double)y[k] * p;
            for (int k = 6; k < 9; ++k) h[k] = (double)y[k] * (p * cs);
            used = 1;
        } else {
            fell = 1;
        }
    }
    used = wave_sum_i(used);
    fell = wave_sum_i(fell);
    if ((threadIdx.x & 63) == 0) {
        if (used) atomicAdd(&w.ctl->n_closure, used);
        if (fell) atomicAdd(&w.ctl->n_fallback, fell);
    }
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
static inline dim3 cells_grid(int64_t n) { return dim3((unsigned)((n + kDigThreads - 1) / kDigThreads)); }

// Kernels of the coupling step come in a monatomic (5 primitives) and a
// rotating (6) instance; the launchers pick by the gas.
#define DIG_NV(g, kernel) ((g).dr ? (kernel<kDigNVR>) : (kernel<kDigNV>))

void launch_dig_sampled(hipStream_t s, const DigGeom& g, const double* ewma, const double* rewma, double FN,
                        DigWork w) {
    hipLaunchKernelGGL(DIG_NV(g, k_dig_sampled), cells_grid(g.nt), dim3(kDigThreads), 0, s, g, ewma, rewma, FN, w);
}

void launch_dig_kn(hipStream_t s, const DigGeom& g, DigWork w, double kn_ref, double T0, double rho0, double L0) {
    hipLaunchKernelGGL(DIG_NV(g, k_dig_kn), cells_grid(g.nt), dim3(kDigThreads), 0, s, g, w, kn_ref, T0, rho0, L0);
}

void launch_dig_gradients(hipStream_t s, const DigGeom& g, const double* prim, double* grad, const DigCtl* ctl) {
    hipLaunchKernelGGL(DIG_NV(g, k_dig_grad), cells_grid(4 * (int64_t)g.nt), dim3(kDigThreads), 0, s, g, prim, grad,
                       ctl);
}

void launch_dig_hot(hipStream_t s, const DigGeom& g, DigWork w) {
    hipLaunchKernelGGL(DIG_NV(g, k_dig_hot), cells_grid(g.nt), dim3(kDigThreads), 0, s, g, w);
}

void launch_dig_gate(hipStream_t s, const DigGeom& g, DigWork w, double kn_max, int passes) {
    const dim3 gr = cells_grid(g.nt), bl(kDigThreads);
    hipLaunchKernelGGL(DIG_NV(g, k_dig_gate_init), gr, bl, 0, s, g, w, kn_max);
    for (int p = 0; p < passes; ++p) {
        hipLaunchKernelGGL(DIG_NV(g, k_dig_gate_pass), gr, bl, 0, s, g, w);
        hipLaunchKernelGGL(DIG_NV(g, k_dig_gate_commit), gr, bl, 0, s, g, w);
    }
    hipLaunchKernelGGL(DIG_NV(g, k_dig_gate_final), gr, bl, 0, s, g, w);
}

void launch_dig_ctl_reset(hipStream_t s, DigCtl* ctl) {
    hipLaunchKernelGGL(k_dig_ctl_reset, dim3(1), dim3(1), 0, s, ctl);
}

void launch_dig_copy(hipStream_t s, const double* src, double* dst, int64_t n) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_dig_copy, cells_grid(n), dim3(kDigThreads), 0, s, src, dst, n);
}

void launch_dig_residual(hipStream_t s, const DigGeom& g, const double* prim, const double* hotf, const double* grad,
                         double* Rs, DigWork w, int first, double cfl) {
    hipLaunchKernelGGL(DIG_NV(g, k_dig_residual), cells_grid(4 * (int64_t)g.nt), dim3(kDigThreads), 0, s, g, prim,
                       hotf, grad, Rs, w, first, cfl);
}

void launch_dig_face_hot(hipStream_t s, const DigGeom& g, const double* prim, const double* grad, const double* hot,
                         double* hotf, int consistent) {
    hipLaunchKernelGGL(DIG_NV(g, k_dig_face_hot), cells_grid(g.nt), dim3(kDigThreads), 0, s, g, prim, grad, hot, hotf,
                       consistent);
}

// One pseudo-time iteration: three stages with weights 1/3, 1/2, 1; the
// convergence test and the step size come from the first stage.
void launch_dig_iteration(hipStream_t s, const DigGeom& g, DigWork w, double cfl, double eps_m, int global_dt,
                          int it) {
    const dim3 gr = cells_grid(g.nt), grq = cells_grid(4 * (int64_t)g.nt), bl(kDigThreads);
    const int nblk = (int)grq.x;  // partials of the residual kernel
    const double alpha[3] = {1.0 / 3.0, 0.5, 1.0};
    hipLaunchKernelGGL(DIG_NV(g, k_dig_save), gr, bl, 0, s, g, w);
    for (int k = 0; k < 3; ++k) {
        hipLaunchKernelGGL(DIG_NV(g, k_dig_grad), grq, bl, 0, s, g, (const double*)w.stage, w.grad,
                           (const DigCtl*)w.ctl);
        hipLaunchKernelGGL(DIG_NV(g, k_dig_residual), grq, bl, 0, s, g, (const double*)w.stage,
                           (const double*)w.hotf, (const double*)w.grad, w.Rs, w, k == 0 ? 1 : 0, cfl);
        if (k == 0) hipLaunchKernelGGL(k_dig_check, dim3(1), bl, 0, s, w, nblk, it, eps_m);
        hipLaunchKernelGGL(DIG_NV(g, k_dig_update), gr, bl, 0, s, g, w, alpha[k], global_dt);
    }
    hipLaunchKernelGGL(DIG_NV(g, k_dig_commit), gr, bl, 0, s, g, w);
}

// ---------------------------------------------------------------------------
// Anderson acceleration of the pseudo-time iteration
// ---------------------------------------------------------------------------
__global__ void k_aa_diff(int n, const double* x, const double* gx, double* fprev, double* gprev, double* dF,
                          double* dG, int first, double* flag_clear) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e == 0) *flag_clear = 0.0;
    if (e >= n) return;
    const double gv = gx[e];
    const double f = gv - x[e];
    if (!first) {
        dF[e] = f - fprev[e];
        dG[e] = gv - gprev[e];
    }
    fprev[e] = f;
    gprev[e] = gv;
}

// Block (x, y): the weighted inner product of column y (y < cnt: the new
// difference dF_slot with dF_y; otherwise f with dF_{y - cnt}) over the
// block's cells; then a fixed-order reduction over the x blocks.
constexpr int kAaMaxDepth = 64;
__global__ __launch_bounds__(kDigThreads) void k_aa_dots(int nt, const double* f, const double* dF, int slot,
                                                          int cnt, int m, double w0, double w1, double w2, double w3,
                                                          double w4, double* part) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    const int col = y < cnt ? y : y - cnt;
    const double wv[kDigNV] = {w0, w1, w2, w3, w4};
    const size_t n = (size_t)nt * kDigNV;
    const double* lhs = y < cnt ? dF + (size_t)slot * n : f;
    double sum = 0.0;
    if (c < nt) {
        const double* d = dF + (size_t)col * n + kDigNV * (size_t)c;
        const double* l = lhs + kDigNV * (size_t)c;
#pragma unroll
        for (int v = 0; v < kDigNV; ++v) sum += (l[v] * wv[v]) * d[v];
    }
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
    __shared__ double red[kDigThreads / 64];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kDigThreads / 64; ++k) t += red[k];
        part[(size_t)blockIdx.x * (2 * m + 1) + (y < cnt ? y : m + col)] = t;
    }
}

__global__ __launch_bounds__(kDigThreads) void k_aa_reduce(const double* part, int nblk, int m, int cnt,
                                                            double* out) {
    const int i = blockIdx.x;  // 0..2cnt-1
    const int idx = i < cnt ? i : m + (i - cnt);
    double sum = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kDigThreads) sum += part[(size_t)b * (2 * m + 1) + idx];
    __shared__ double red[kDigThreads];
    red[threadIdx.x] = sum;
    __syncthreads();
    for (int o = kDigThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[idx] = red[0];
}

__global__ void k_aa_update(int nt, const double* gprev, const double* dG, const double* gam, int cnt,
                            double* prim, double* flag) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nt) return;
    const size_t n = (size_t)nt * kDigNV;
    double x[kDigNV];
#pragma unroll
    for (int v = 0; v < kDigNV; ++v) {
        double t = gprev[kDigNV * (size_t)c + v];
        for (int i = 0; i < cnt; ++i) t -= gam[i] * dG[(size_t)i * n + kDigNV * (size_t)c + v];
        x[v] = t;
    }
    const bool ok = x[0] > 0 && x[4] > 0 && isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]) && isfinite(x[3]) &&
                    isfinite(x[4]);
    if (!ok) {
        atomicAdd(flag, 1.0);
#pragma unroll
        for (int v = 0; v < kDigNV; ++v) x[v] = gprev[kDigNV * (size_t)c + v];
    }
#pragma unroll
    for (int v = 0; v < kDigNV; ++v) prim[kDigNV * (size_t)c + v] = x[v];
}

void launch_aa_diff(hipStream_t s, const DigGeom& g, const AaWork& a, const double* gx, int slot, int first,
                    int parity) {
    const int n = kDigNV * g.nt;
    const size_t off = (size_t)slot * n;
    hipLaunchKernelGGL(k_aa_diff, dim3((n + 255) / 256), dim3(256), 0, s, n, (const double*)a.x, gx, a.fprev,
                       a.gprev, a.dF + off, a.dG + off, first, a.red + 2 * a.m + parity);
}

void launch_aa_dots(hipStream_t s, const DigGeom& g, const AaWork& a, int slot, int cnt, const double* w5) {
    const dim3 gr = cells_grid(g.nt), bl(kDigThreads);
    hipLaunchKernelGGL(k_aa_dots, dim3(gr.x, 2 * cnt), bl, 0, s, g.nt, (const double*)a.fprev, (const double*)a.dF,
                       slot, cnt, a.m, w5[0], w5[1], w5[2], w5[3], w5[4], a.part);
    hipLaunchKernelGGL(k_aa_reduce, dim3(2 * cnt), bl, 0, s, (const double*)a.part, (int)gr.x, a.m, cnt, a.red);
}

void launch_aa_update(hipStream_t s, const DigGeom& g, const AaWork& a, int cnt, double* prim, int parity) {
    hipLaunchKernelGGL(k_aa_update, cells_grid(g.nt), dim3(kDigThreads), 0, s, g.nt, (const double*)a.gprev,
                       (const double*)a.dG, (const double*)a.gam, cnt, prim, a.red + 2 * a.m + parity);
}

// ---------------------------------------------------------------------------
// Newton-Krylov solve (pseudo-transient continuation, one GMRES cycle per
// Newton step, Jacobian products by forward differences of the residual)
// ---------------------------------------------------------------------------
// One lane per cell.  Unknowns and equations are scaled per variable by
// NkScale; the right preconditioner divides cell c's unknowns by
// p_c = S_c (1 + 1/cfl), S_c = V_c / dt_c the sum that sets the marching's
// local step (the residual kernel's dt at CFL number 1).  Inner products are
// reduced in a fixed order: wave, then the block's four waves, then
// k_nk_reduce over the blocks.

// Per-column block partials: column i's value of this lane is added over the
// block and written to part[i * nblk + block].
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ void nk_block_column(double (*red)[kDigThreads / 64], int i, double v) {
    v = wave_sum_d(v);
    if ((threadIdx.x & 63) == 0) red[i][threadIdx.x >> 6] = v;
}

__device__ __forceinline__ void nk_block_store(double (*red)[kDigThreads / 64], int ncol, double* part) {
    __syncthreads();
    for (int i = threadIdx.x; i < ncol; i += blockDim.x)
        part[(size_t)i * gridDim.x + blockIdx.x] = ((red[i][0] + red[i][1]) + red[i][2]) + red[i][3];
}

// Columns 0..j of the block partials of <V_i, w> (V pointing at this lane's
// cell in basis vector 0, vectors n apart): loads of four vectors at a time,
// each dot in the order of the variables.
template <int NV>
__device__ __forceinline__ void nk_block_dots(double (*red)[kDigThreads / 64], const double* __restrict__ V,
                                              size_t n, int j, const double* wv, bool live) {
    int i = 0;
    for (; i + 4 <= j + 1; i += 4) {
        double d[4] = {0.0, 0.0, 0.0, 0.0};
        if (live) {
            double a[4][NV];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int v = 0; v < NV; ++v) a[q][v] = V[(size_t)(i + q) * n + v];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int v = 0; v < NV; ++v) d[q] += a[q][v] * wv[v];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) nk_block_column(red, i + q, d[q]);
    }
    for (; i <= j; ++i) {
        double d = 0.0;
        if (live) {
#pragma unroll
            for (int v = 0; v < NV; ++v) d += V[(size_t)i * n + v] * wv[v];
        }
        nk_block_column(red, i, d);
    }
}

// Fixed-order sum over the blocks of column blockIdx.x into out[blockIdx.x].
__global__ __launch_bounds__(kDigThreads) void k_nk_reduce(const double* part, int nblk, double* out) {
    const double* p = part + (size_t)blockIdx.x * nblk;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kDigThreads) s += p[b];
    __shared__ double tot, dummy;
    block_sum_min(s, 0.0, &tot, &dummy);
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = tot;
}

// The finite-difference step of the next product from the reduced
// sum of squares of the preconditioned direction and that of the state.
__global__ __launch_bounds__(kDigThreads) void k_nk_reduce_eps(const double* part, int nblk, double* red, int m,
                                                                double n, double fd) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kDigThreads) s += part[b];
    __shared__ double tot, dummy;
    block_sum_min(s, 0.0, &tot, &dummy);
    __syncthreads();
    if (threadIdx.x == 0) {
        red[kNkVs2(m)] = tot;
        const double vn = sqrt(tot / n), xr = sqrt(red[kNkXr2(m)] / n);
        red[kNkEps(m)] = fd * (1.0 + xr) / vn;
    }
}

// Start of a Newton step: R0 = the residual just computed; U from the
// primitives on the first step; V_0 = -R0 / scale; partials of |V_0|^2 and
// |U / scale|^2.
template <int NV>
__global__ __launch_bounds__(kDigThreads) void k_nk_start(DigGeom g, DigWork w, NkWork nk, NkScale sc, int first) {
    __shared__ double red[2][kDigThreads / 64];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    double b2 = 0.0, x2 = 0.0;
    if (c < g.nt) {
        double U[NV];
        if (first) {
            double P[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) P[v] = w.prim[NV * (size_t)c + v];
            cons_of<NV>(g, P, U);
#pragma unroll
            for (int v = 0; v < NV; ++v) nk.U[NV * (size_t)c + v] = U[v];
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) U[v] = nk.U[NV * (size_t)c + v];
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const size_t e = NV * (size_t)c + v;
            const double r = w.Rs[e];
            nk.R0[e] = r;
            const double b = -r / sc.s[v];
            nk.V[e] = b;
            b2 += b * b;
            const double x = U[v] / sc.s[v];
            x2 += x * x;
        }
    }
    nk_block_column(red, 0, b2);
    nk_block_column(red, 1, x2);
    nk_block_store(red, 2, nk.part);
}

// V_0 /= beta; partial of |V_0 / p|^2 (the next finite-difference step).
template <int NV>
__global__ __launch_bounds__(kDigThreads) void k_nk_scale(DigGeom g, DigWork w, NkWork nk, double cfl) {
    __shared__ double red[1][kDigThreads / 64];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    double q2 = 0.0;
    if (c < g.nt) {
        const double beta = sqrt(nk.red[kNkBeta2(nk.m)]);
        const double pc = g.vol[c] / w.dt[c] * (1.0 + 1.0 / cfl);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const size_t e = NV * (size_t)c + v;
            const double x = nk.V[e] / beta;
            nk.V[e] = x;
            const double q = x / pc;
            q2 += q * q;
        }
    }
    nk_block_column(red, 0, q2);
    nk_block_store(red, 1, nk.part);
}

// The state perturbed along the preconditioned direction V_j, as
// primitives in w.stage; a cell that is not physical sets the flag.
template <int NV>
__global__ __launch_bounds__(kDigThreads) void k_nk_perturb(DigGeom g, DigWork w, NkWork nk, NkScale sc, int j,
                                                            double cfl) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nt) return;
    const double eps = nk.red[kNkEps(nk.m)];
    const double pc = g.vol[c] / w.dt[c] * (1.0 + 1.0 / cfl);
    const double* vj = nk.V + (size_t)j * NV * g.nt;
    double U[NV], P[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const size_t e = NV * (size_t)c + v;
        U[v] = nk.U[e] + eps * (sc.s[v] * vj[e] / pc);
    }
    if (!prim_of<NV>(g, U, P)) atomicOr(nk.flag, 1);
#pragma unroll
    for (int v = 0; v < NV; ++v) w.stage[NV * (size_t)c + v] = P[v];
}

// w = scaled ((R(U + eps d) - R(U)) / eps + S / cfl d), d the preconditioned
// V_j; partials of <V_i, w>, i <= j (the first Gram-Schmidt pass).
template <int NV>
__global__ __launch_bounds__(kDigThreads) void k_nk_matvec(DigGeom g, DigWork w, NkWork nk, NkScale sc, int j,
                                                           double cfl) {
    __shared__ double red[kNkMaxKrylov + 1][kDigThreads / 64];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = c < g.nt;
    const size_t n = (size_t)NV * g.nt;
    double wv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) wv[v] = 0.0;
    if (live) {
        const double eps = nk.red[kNkEps(nk.m)];
        const double sp = g.vol[c] / w.dt[c];
        const double pc = sp * (1.0 + 1.0 / cfl);
        const double* vj = nk.V + (size_t)j * n;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const size_t e = NV * (size_t)c + v;
            const double du = sc.s[v] * vj[e] / pc;
            wv[v] = ((nk.Rp[e] - nk.R0[e]) / eps + sp / cfl * du) / sc.s[v];
            nk.w[e] = wv[v];
        }
    }
    nk_block_dots<NV>(red, nk.V + NV * (size_t)c, n, j, wv, live);
    nk_block_store(red, j + 1, nk.part);
}

// w -= sum_{i <= j} h_i V_i with h = red[off ...]; then partials of the next
// pass's <V_i, w> (norm = 0) or of |w|^2 (norm = 1).
template <int NV>
__global__ __launch_bounds__(kDigThreads) void k_nk_orth(DigGeom g, NkWork nk, int j, int off, int norm) {
    __shared__ double red[kNkMaxKrylov + 1][kDigThreads / 64];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = c < g.nt;
    const size_t n = (size_t)NV * g.nt;
    // the basis, the coefficients and w do not overlap: loads of several
    // basis vectors can be in flight before w is written back
    const double* __restrict__ V = nk.V + NV * (size_t)c;
    const double* __restrict__ h = nk.red + off;
    double* __restrict__ W = nk.w + NV * (size_t)c;
    double wv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) wv[v] = 0.0;
    if (live) {
#pragma unroll
        for (int v = 0; v < NV; ++v) wv[v] = W[v];
        // each element subtracts h_i V_i[e] in ascending i
        int i = 0;
        for (; i + 4 <= j + 1; i += 4) {
            double a[4][NV];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int v = 0; v < NV; ++v) a[q][v] = V[(size_t)(i + q) * n + v];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double hq = h[i + q];
#pragma unroll
                for (int v = 0; v < NV; ++v) wv[v] -= hq * a[q][v];
            }
        }
        for (; i <= j; ++i) {
            const double hi = h[i];
#pragma unroll
            for (int v = 0; v < NV; ++v) wv[v] -= hi * V[(size_t)i * n + v];
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) W[v] = wv[v];
    }
    if (norm) {
        double d = 0.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) d += wv[v] * wv[v];
        nk_block_column(red, 0, d);
        nk_block_store(red, 1, nk.part);
        return;
    }
    nk_block_dots<NV>(red, V, n, j, wv, live);
    nk_block_store(red, j + 1, nk.part);
}

// V_{j+1} = w / |w| (when |w| > 0); partial of |V_{j+1} / p|^2.
template <int NV>
__global__ __launch_bounds__(kDigThreads) void k_nk_normalize(DigGeom g, DigWork w, NkWork nk, int j, double cfl) {
    __shared__ double red[1][kDigThreads / 64];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    double q2 = 0.0;
    const double hn = sqrt(nk.red[kNkHn2(nk.m)]);
    if (c < g.nt && hn > 0) {
        const size_t n = (size_t)NV * g.nt;
        const double pc = g.vol[c] / w.dt[c] * (1.0 + 1.0 / cfl);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const size_t e = NV * (size_t)c + v;
            const double x = nk.w[e] / hn;
            nk.V[(size_t)(j + 1) * n + e] = x;
            const double q = x / pc;
            q2 += q * q;
        }
    }
    nk_block_column(red, 0, q2);
    nk_block_store(red, 1, nk.part);
}

// Trial state U + alpha dU, dU the preconditioned sum_{i < jn} y_i V_i, into
// nk.Ut and (as primitives) w.stage; a cell that is not physical sets the
// flag.
template <int NV>
__global__ __launch_bounds__(kDigThreads) void k_nk_try(DigGeom g, DigWork w, NkWork nk, NkScale sc, int jn,
                                                        double alpha, double cfl) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nt) return;
    const size_t n = (size_t)NV * g.nt;
    const double pc = g.vol[c] / w.dt[c] * (1.0 + 1.0 / cfl);
    const double* __restrict__ V = nk.V + NV * (size_t)c;
    const double* __restrict__ y = nk.y;
    // z = sum_{i < jn} y_i V_i, each element in ascending i, four basis
    // vectors in flight
    double z[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) z[v] = 0.0;
    int i = 0;
    for (; i + 4 <= jn; i += 4) {
        double a[4][NV];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int v = 0; v < NV; ++v) a[q][v] = V[(size_t)(i + q) * n + v];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int v = 0; v < NV; ++v) z[v] += y[i + q] * a[q][v];
    }
    for (; i < jn; ++i)
#pragma unroll
        for (int v = 0; v < NV; ++v) z[v] += y[i] * V[(size_t)i * n + v];
    double U[NV], P[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const size_t e = NV * (size_t)c + v;
        U[v] = nk.U[e] + alpha * (sc.s[v] * z[v] / pc);
        nk.Ut[e] = U[v];
    }
    if (!prim_of<NV>(g, U, P)) atomicOr(nk.flag, 1);
#pragma unroll
    for (int v = 0; v < NV; ++v) w.stage[NV * (size_t)c + v] = P[v];
}

template <int NV>
__global__ void k_nk_commit(DigGeom g, DigWork w, NkWork nk) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nt) return;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const size_t e = NV * (size_t)c + v;
        nk.U[e] = nk.Ut[e];
        w.prim[e] = w.stage[e];
    }
}

void launch_nk_begin(hipStream_t s, const DigGeom& g, DigWork w, NkWork nk, NkScale sc, int it, double eps_m) {
    const dim3 gr = cells_grid(g.nt), grq = cells_grid(4 * (int64_t)g.nt), bl(kDigThreads);
    hipLaunchKernelGGL(DIG_NV(g, k_dig_grad), grq, bl, 0, s, g, (const double*)w.prim, w.grad, (const DigCtl*)nullptr);
    hipLaunchKernelGGL(DIG_NV(g, k_dig_residual), grq, bl, 0, s, g, (const double*)w.prim, (const double*)w.hotf,
                       (const double*)w.grad, w.Rs, w, 1, 1.0);
    hipLaunchKernelGGL(k_dig_check, dim3(1), bl, 0, s, w, (int)grq.x, it, eps_m);
    hipLaunchKernelGGL(DIG_NV(g, k_nk_start), gr, bl, 0, s, g, w, nk, sc, it == 0 ? 1 : 0);
    hipLaunchKernelGGL(k_nk_reduce, dim3(2), bl, 0, s, (const double*)nk.part, (int)gr.x, nk.red + kNkBeta2(nk.m));
}

void launch_nk_scale(hipStream_t s, const DigGeom& g, DigWork w, NkWork nk, double cfl, double fd) {
    const dim3 gr = cells_grid(g.nt), bl(kDigThreads);
    hipLaunchKernelGGL(DIG_NV(g, k_nk_scale), gr, bl, 0, s, g, w, nk, cfl);
    hipLaunchKernelGGL(k_nk_reduce_eps, dim3(1), bl, 0, s, (const double*)nk.part, (int)gr.x, nk.red, nk.m,
                       (double)(g.dr ? kDigNVR : kDigNV) * g.nt, fd);
}

void launch_nk_arnoldi(hipStream_t s, const DigGeom& g, DigWork w, NkWork nk, NkScale sc, int j, double cfl,
                       double fd) {
    const dim3 gr = cells_grid(g.nt), grq = cells_grid(4 * (int64_t)g.nt), bl(kDigThreads);
    const int nblk = (int)gr.x, m = nk.m;
    hipLaunchKernelGGL(DIG_NV(g, k_nk_perturb), gr, bl, 0, s, g, w, nk, sc, j, cfl);
    hipLaunchKernelGGL(DIG_NV(g, k_dig_grad), grq, bl, 0, s, g, (const double*)w.stage, w.grad,
                       (const DigCtl*)nullptr);
    hipLaunchKernelGGL(DIG_NV(g, k_dig_residual), grq, bl, 0, s, g, (const double*)w.stage, (const double*)w.hotf,
                       (const double*)w.grad, nk.Rp, w, 0, 1.0);
    hipLaunchKernelGGL(DIG_NV(g, k_nk_matvec), gr, bl, 0, s, g, w, nk, sc, j, cfl);
    hipLaunchKernelGGL(k_nk_reduce, dim3(j + 1), bl, 0, s, (const double*)nk.part, nblk, nk.red + kNkH1(m));
    hipLaunchKernelGGL(DIG_NV(g, k_nk_orth), gr, bl, 0, s, g, nk, j, kNkH1(m), 0);
    hipLaunchKernelGGL(k_nk_reduce, dim3(j + 1), bl, 0, s, (const double*)nk.part, nblk, nk.red + kNkH2(m));
    hipLaunchKernelGGL(DIG_NV(g, k_nk_orth), gr, bl, 0, s, g, nk, j, kNkH2(m), 1);
    hipLaunchKernelGGL(k_nk_reduce, dim3(1), bl, 0, s, (const double*)nk.part, nblk, nk.red + kNkHn2(m));
    hipLaunchKernelGGL(DIG_NV(g, k_nk_normalize), gr, bl, 0, s, g, w, nk, j, cfl);
    hipLaunchKernelGGL(k_nk_reduce_eps, dim3(1), bl, 0, s, (const double*)nk.part, nblk, nk.red, m,
                       (double)(g.dr ? kDigNVR : kDigNV) * g.nt, fd);
}

void launch_nk_try(hipStream_t s, const DigGeom& g, DigWork w, NkWork nk, NkScale sc, int jn, double alpha,
                   double cfl) {
    hipLaunchKernelGGL(DIG_NV(g, k_nk_try), cells_grid(g.nt), dim3(kDigThreads), 0, s, g, w, nk, sc, jn, alpha, cfl);
}

void launch_nk_commit(hipStream_t s, const DigGeom& g, DigWork w, NkWork nk) {
    hipLaunchKernelGGL(DIG_NV(g, k_nk_commit), cells_grid(g.nt), dim3(kDigThreads), 0, s, g, w, nk);
}

// Batch: one workgroup per case sums its FV mass over its internal cells in
// a fixed order; the factor matches the case's particle mass.
__global__ __launch_bounds__(kDigThreads) void k_dig_mass_cases(DigGeom g, DigWork w, const int32_t* offsets) {
    DigCase& k = g.cases[blockIdx.x];
    double m = 0.0;
    for (int c = k.first + (int)threadIdx.x; c < k.end; c += kDigThreads)
        m += w.prim[(g.dr ? kDigNVR : kDigNV) * (size_t)c] * g.vol[c];
    __shared__ double tot, dummy;
    block_sum_min(m, 0.0, &tot, &dummy);
    __syncthreads();
    if (threadIdx.x == 0) {
        const double mp = (double)(offsets[k.end] - offsets[k.first]) * k.FN * g.mass;
        k.mass_scale = k.enabled && k.closed && tot > 0 ? mp / tot : 1.0;
    }
}

__global__ void k_dig_mass_apply_cases(DigGeom g, DigWork w) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const size_t nv = g.dr ? kDigNVR : kDigNV;
    if (c < g.nt) w.prim[nv * (size_t)c] = w.prim[nv * (size_t)c] * g.cases[g.cell_case[c]].mass_scale;
}

__global__ void k_dig_case_pids(DigGeom g, DigWork w) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= g.n_cases) return;
    DigCase& d = g.cases[k];
    if (d.enabled) d.next_pid += (uint32_t)(w.fb_off[d.cell_end] - w.fb_off[d.cell0]);
}

__global__ void k_dig_case_pid_init(DigGeom g, const int32_t* cell, const uint32_t* pid, const Scalars* sc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sc->np) return;
    const int c = cell[i];
    if (c >= 0) atomicMax(&g.cases[g.cell_case[c]].next_pid, pid[i] + 1u);
}

void launch_dig_mass_rescale(hipStream_t s, const DigGeom& g, DigWork w, const Scalars* sc,
                             const int32_t* offsets) {
    const dim3 gr = cells_grid(g.nt), bl(kDigThreads);
    if (g.cases) {
        hipLaunchKernelGGL(k_dig_mass_cases, dim3(g.n_cases), bl, 0, s, g, w, offsets);
        hipLaunchKernelGGL(k_dig_mass_apply_cases, gr, bl, 0, s, g, w);
        return;
    }
    hipLaunchKernelGGL(DIG_NV(g, k_dig_mass_partial), gr, bl, 0, s, g, w);
    hipLaunchKernelGGL(k_dig_mass_factor, dim3(1), bl, 0, s, g, w, (int)gr.x, sc);
    hipLaunchKernelGGL(DIG_NV(g, k_dig_mass_apply), gr, bl, 0, s, g, w);
}

void launch_dig_case_pids(hipStream_t s, const DigGeom& g, const DigWork& w) {
    if (g.cases) hipLaunchKernelGGL(k_dig_case_pids, dim3((g.n_cases + 63) / 64), dim3(64), 0, s, g, w);
}

void launch_dig_case_pid_init(hipStream_t s, const DigGeom& g, const int32_t* cell, const uint32_t* pid,
                              const Scalars* sc, int64_t bound) {
    if (!g.cases || bound <= 0) return;
    hipLaunchKernelGGL(k_dig_case_pid_init, dim3((unsigned)((bound + 255) / 256)), dim3(256), 0, s, g, cell, pid, sc);
}

void launch_dig_set_local(hipStream_t s, const DigGeom& g, const int32_t* state, uint8_t* local) {
    hipLaunchKernelGGL(k_dig_set_local, cells_grid(g.nt), dim3(kDigThreads), 0, s, g, state, local);
}

void launch_dig_fb_count(hipStream_t s, const DigGeom& g, DigWork w, const int32_t* offsets, const int32_t* orig,
                         const Scalars* sc, RngKey key) {
    hipLaunchKernelGGL(k_dig_fb_count, cells_grid(g.nt), dim3(kDigThreads), 0, s, g, w, offsets, orig, sc, key);
}

template <class VT>
void launch_dig_fb_apply(hipStream_t s, const DigGeom& g, DigWork w, PartDev<VT> p, const int32_t* offsets,
                         const int4* tv, const double* xyz, const int32_t* orig, const Scalars* sc, RngKey key,
                         int32_t* scratch, uint32_t* bits, int nt, int64_t cap) {
    hipLaunchKernelGGL(k_dig_fb_apply<VT>, dim3((unsigned)nt), dim3(kFbLanes), 0, s, g, w, p, offsets, tv, xyz, orig,
                       sc, key, scratch, bits, cap);
}

void launch_dig_count_all(hipStream_t s, const int32_t* cell, const Scalars* sc, int32_t* counts, uint32_t* rank,
                          int64_t bound) {
    hipLaunchKernelGGL(k_dig_count_all, cells_grid(bound > 0 ? bound : 1), dim3(kDigThreads), 0, s, cell, sc, counts,
                       rank);
}

void launch_dig_closure_prep(hipStream_t s, const DigGeom& g, DigWork w) {
    hipLaunchKernelGGL(k_dig_closure_prep, cells_grid(g.nt), dim3(kDigThreads), 0, s, g, w);
}

void launch_dig_closure_gate(hipStream_t s, const DigGeom& g, DigWork w, double tol, const double* ewma,
                             const int32_t* ewma_m, int n_a) {
    hipLaunchKernelGGL(k_dig_closure_gate, cells_grid(g.nt), dim3(kDigThreads), 0, s, g, w, tol, ewma, ewma_m, n_a);
}

void launch_fill_u8(hipStream_t s, uint8_t* p, uint8_t v, int64_t n) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_u8, cells_grid(n), dim3(kDigThreads), 0, s, p, v, n);
}

template void launch_dig_fb_apply<float>(hipStream_t, const DigGeom&, DigWork, PartDev<float>, const int32_t*, const int4*,
                                         const double*, const int32_t*, const Scalars*, RngKey, int32_t*, uint32_t*,
                                         int, int64_t);
template void launch_dig_fb_apply<double>(hipStream_t, const DigGeom&, DigWork, PartDev<double>, const int32_t*, const int4*,
                                          const double*, const int32_t*, const Scalars*, RngKey, int32_t*, uint32_t*,
                                          int, int64_t);

}  // namespace dsmcx
