"""Statistics helpers for the physics pins (test-side only)."""
import numpy as np

KB = 1.380649e-23


def fields_from_sums(S, m, FN, V, ns):
    """Fields of a set of moment sums S[13] accumulated over ns samples in a
    region of volume V (central moments from raw sums)."""
    S0 = S[0]
    u = S[1:4] / S0
    M2 = np.array([[S[4], S[7], S[8]], [S[7], S[5], S[9]], [S[8], S[9], S[6]]]) / S0
    C = M2 - np.outer(u, u)
    n = FN * S0 / ns / V
    rho = m * n
    T = m * np.trace(C) / (3 * KB)
    sig = rho * (C - np.eye(3) * np.trace(C) / 3)
    S3 = S[10:13] / S0
    q = rho / 2 * (S3 - 2 * M2 @ u - u * np.trace(M2) + 2 * u * (u @ u))
    return dict(n=n, rho=rho, u=u, T=T, sig=sig, q=q)


def batch_stat(values):
    """Mean and standard error of the mean from batch values."""
    v = np.asarray(values, dtype=float)
    return v.mean(axis=0), v.std(axis=0, ddof=1) / np.sqrt(len(v))
