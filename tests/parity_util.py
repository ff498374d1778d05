"""Helpers of the GPU-vs-oracle parity tests."""
import numpy as np


def f32_ulp(a):
    return np.spacing(np.abs(a).astype(np.float32)).astype(np.float64)


def compare_particles(g, o, vel_fp32, L0=1.0, ctx=""):
    """Bit-exact cell indices and (cell, pid) order; positions within 1e-12
    relative to max(|x|, L0); velocities within 1 float32 ulp (FP32 storage)
    or 1e-12 relative to the speed (FP64 storage)."""
    assert g["n"] == len(o["pid"]), f"{ctx}: particle count {g['n']} vs {len(o['pid'])}"
    assert np.array_equal(g["cell"], o["cell"]), f"{ctx}: cells differ at {np.nonzero(g['cell'] != o['cell'])[0][:10]}"
    assert np.array_equal(g["pid"], o["pid"]), f"{ctx}: order differs"
    dx = np.abs(g["x"] - o["x"])
    lim = 1e-12 * np.maximum(np.abs(o["x"]), L0)
    bad = dx > lim
    assert not bad.any(), f"{ctx}: {bad.sum()} position components off, max {dx.max():.3e}"
    dv = np.abs(g["v"] - o["v"])
    if vel_fp32:
        lim = f32_ulp(o["v"])
    else:
        lim = 1e-12 * np.maximum(np.linalg.norm(o["v"], axis=1, keepdims=True), 1.0)
    bad = dv > lim
    assert not bad.any(), f"{ctx}: {bad.sum()} velocity components off, max {dv.max():.3e}"
    return dict(max_dx=float(dx.max()) if dx.size else 0.0, exact_x=float((dx == 0).mean()) if dx.size else 1.0,
                exact_v=float((dv == 0).mean()) if dv.size else 1.0)


def compare_sums(gs, os_, rel=1e-12):
    scale = np.abs(os_).max(axis=0, keepdims=True) + 1e-300
    d = np.abs(gs - os_) / scale
    assert (d <= rel).all(), f"sums differ: max rel {d.max():.3e}"
