"""Independent replicates and the field z-test of the statistical parity
criterion (test-side only).

Over hundreds of steps a DSMC trajectory is chaotic, so two correct
implementations agree only in distribution.  The criterion compares the
per-cell time-averaged fields of R replicates from one implementation with
R replicates from the other, every replicate seeded from a set disjoint from
all others: per cell and field, z = (mean_a - mean_b) / sqrt(s_a^2/R +
s_b^2/R).  With R = 8 the sample variances carry 7 degrees of freedom each,
so z follows Welch's t distribution (Satterthwaite's degrees of freedom,
about 14) rather than the normal one; each z is therefore mapped through its
t tail probability onto the standard normal scale before the two
summaries are taken: the fraction of |z| > 3 (0.27 % expected) and the mean
of z^2 (1 expected).

Fields per cell (eq. dsmc_temperatures over the steady window): number
density, velocity (3), temperature, stress (xx, yy, zz, xy, xz, yz) and heat
flux (3) — 14 columns.
"""
import os
from concurrent.futures import ProcessPoolExecutor
import multiprocessing as mp

import numpy as np

KB = 1.380649e-23
FIELD_NAMES = ["n", "ux", "uy", "uz", "T", "sxx", "syy", "szz", "sxy", "sxz", "syz", "qx", "qy", "qz"]


def cell_fields(S, m, FN, V, ns):
    """Fields of per-cell moment sums S[nc, 13] over ns samples (cells of
    volume V[nc]); rows without samples are NaN."""
    S = np.asarray(S, dtype=np.float64)
    S0 = S[:, 0]
    with np.errstate(invalid="ignore", divide="ignore"):
        u = S[:, 1:4] / S0[:, None]
        M2 = np.empty((len(S), 3, 3))
        M2[:, 0, 0], M2[:, 1, 1], M2[:, 2, 2] = S[:, 4], S[:, 5], S[:, 6]
        M2[:, 0, 1] = M2[:, 1, 0] = S[:, 7]
        M2[:, 0, 2] = M2[:, 2, 0] = S[:, 8]
        M2[:, 1, 2] = M2[:, 2, 1] = S[:, 9]
        M2 /= S0[:, None, None]
        C = M2 - u[:, :, None] * u[:, None, :]
        n = FN * S0 / ns / V
        rho = m * n
        tr = np.trace(C, axis1=1, axis2=2)
        T = m * tr / (3 * KB)
        sig = rho[:, None, None] * (C - np.eye(3)[None] * (tr / 3)[:, None, None])
        S3 = S[:, 10:13] / S0[:, None]
        trM = np.trace(M2, axis1=1, axis2=2)
        q = rho[:, None] / 2 * (S3 - 2 * np.einsum("cij,cj->ci", M2, u) - u * trM[:, None]
                                + 2 * u * (u * u).sum(1, keepdims=True))
    out = np.column_stack([n, u, T, sig[:, 0, 0], sig[:, 1, 1], sig[:, 2, 2], sig[:, 0, 1], sig[:, 0, 2],
                           sig[:, 1, 2], q])
    out[S0 <= 0] = np.nan
    return out


def _oracle_run(args):
    from oracle import Oracle
    wl, steps = args
    o = Oracle(wl)
    o.step(steps)
    return o.sums(0), int(o.n_steady)


def oracle_replicates(workloads, steps, workers=None):
    """Steady sums and sample counts of one oracle run per workload, in
    worker processes started fresh (no state inherited from a process that
    may hold a GPU context)."""
    workers = workers or max(1, min(16, os.cpu_count() or 1, len(workloads)))
    if workers == 1:
        return [_oracle_run((w, steps)) for w in workloads]
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_oracle_run, [(w, steps) for w in workloads]))


def replicate_z(fa, fb):
    """fa, fb: [R, nc, nf] per-replicate fields.  Returns the normal-scale z
    of every cell-field where both sides have samples and spread, as a flat
    array, and the raw Welch z of the same entries."""
    from scipy import stats
    fa, fb = np.asarray(fa), np.asarray(fb)
    ra, rb = fa.shape[0], fb.shape[0]
    ok = np.isfinite(fa).all(axis=0) & np.isfinite(fb).all(axis=0)
    ma, mb = fa.mean(axis=0), fb.mean(axis=0)
    va, vb = fa.var(axis=0, ddof=1) / ra, fb.var(axis=0, ddof=1) / rb
    se2 = va + vb
    ok &= se2 > 0
    z = (ma[ok] - mb[ok]) / np.sqrt(se2[ok])
    df = se2[ok] ** 2 / (va[ok] ** 2 / (ra - 1) + vb[ok] ** 2 / (rb - 1))
    p = stats.t.sf(np.abs(z), df)
    zn = np.sign(z) * stats.norm.isf(p)
    return zn, z


def z_summary(zn):
    return dict(n=int(zn.size), frac_gt3=float((np.abs(zn) > 3).mean()), mean_z2=float((zn * zn).mean()),
                max_abs=float(np.abs(zn).max()))


def check_fields(zn_by_field, frac_max=0.01, lo=0.8, hi=1.25):
    """The statistical parity criterion per field: at most frac_max of the
    cells with |z| > 3 and the mean of z^2 in [lo, hi].  zn_by_field maps a
    field name to its normal-scale z values.  Returns the failures."""
    bad = {}
    for name, zn in zn_by_field.items():
        s = z_summary(zn)
        if s["frac_gt3"] > frac_max or not (lo <= s["mean_z2"] <= hi):
            bad[name] = s
    return bad


def field_z(fa, fb):
    """Normal-scale z per field name from per-replicate fields [R, nc, 14]."""
    return {name: replicate_z(fa[:, :, j:j + 1], fb[:, :, j:j + 1])[0] for j, name in enumerate(FIELD_NAMES)}
