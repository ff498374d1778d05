"""Plain FP64 statement of the MLP closure (test infrastructure only).

The closure maps 13 nondimensional inputs per cell (the nine velocity
gradients and three temperature gradients scaled by the local mean free
path, and Kn_Delta) through three hidden layers of 128 SiLU units to the
nine nondimensional higher-order terms (six stresses over p, three heat
fluxes over p sqrt(RT)).  It is trained by mean-squared error with Adam.
Nothing here is used by the product path; tests and the benchmark's
baseline leg call it to check the GPU kernels.

Parameters are one flat vector: for each layer l = 1..4, W_l[in][out]
row-major, then b_l[out].

`bf16=True` evaluates the same network with the GPU kernels' precision
contract: inputs, weights, every hidden activation fed to the next layer and
every pre-activation gradient fed to a product are rounded to bfloat16
(round to nearest, ties to even); all products and sums are then exact-ish
(FP64 here), and bias gradients use the unrounded pre-activation gradients.
"""
import numpy as np

LAYERS = (13, 128, 128, 128, 9)


def n_params(layers=LAYERS):
    return sum(i * o + o for i, o in zip(layers[:-1], layers[1:]))


def unpack(p, layers=LAYERS):
    out, k = [], 0
    for i, o in zip(layers[:-1], layers[1:]):
        W = p[k:k + i * o].reshape(i, o)
        k += i * o
        b = p[k:k + o]
        k += o
        out.append((W, b))
    assert k == p.size
    return out


def bf16_round(x):
    """Nearest bfloat16 value of x (ties to even), returned as float64.
    bfloat16 keeps the top 16 bits of the IEEE binary32 pattern."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if np.any(nan):
        out = np.where(nan, np.nan, out)
    return out


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def silu_grad(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def forward(p, x, bf16=False, layers=LAYERS):
    """Returns the outputs y[n][9] and the cache of the backward pass."""
    q = bf16_round if bf16 else (lambda a: a)
    params = unpack(np.asarray(p, np.float64), layers)
    h = q(np.asarray(x, np.float64))
    hs, zs = [h], []
    for l, (W, b) in enumerate(params):
        z = h @ q(W) + b
        zs.append(z)
        if l < len(params) - 1:
            h = q(silu(z))
            hs.append(h)
        else:
            h = z
    return h, (hs, zs)


def loss_and_grad(p, x, t, bf16=False, layers=LAYERS):
    """Mean-squared error over all n*9 outputs and its gradient (flat)."""
    q = bf16_round if bf16 else (lambda a: a)
    params = unpack(np.asarray(p, np.float64), layers)
    y, (hs, zs) = forward(p, x, bf16, layers)
    t = np.asarray(t, np.float64)
    n = y.shape[0]
    loss = float(np.mean((y - t) ** 2))
    dz = 2.0 * (y - t) / (n * y.shape[1])
    grads = []
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        dzq = q(dz)
        dW = hs[l].T @ dzq
        db = dz.sum(axis=0)
        grads.append((dW, db))
        if l > 0:
            dh = dzq @ q(W).T
            dz = dh * silu_grad(zs[l - 1])
    grads.reverse()
    flat = np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])
    return loss, flat


def adam_step(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) at 1-based step; returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def train(p, x, t, batches, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, bf16=False):
    """Adam over the given list of index batches, from parameters p."""
    p = np.array(p, np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    losses = []
    for k, idx in enumerate(batches):
        loss, g = loss_and_grad(p, x[idx], t[idx], bf16)
        losses.append(loss)
        p, m, v = adam_step(p, g, m, v, k + 1, lr, b1, b2, eps)
    return p, losses


def closure_inputs(grad_u, grad_T, T, kn, lam, R):
    """Nondimensional inputs: lam du_i/dx_j / sqrt(RT) (9), lam dT/dx_j / T
    (3), Kn_Delta; lam is the local mean free path in metres."""
    cs = np.sqrt(R * T)
    a = lam[:, None] * grad_u / cs[:, None]
    b = lam[:, None] * grad_T / T[:, None]
    return np.concatenate([a, b, kn[:, None]], axis=1)


def closure_targets(hot, rho, T, R):
    """Nondimensional HoT: stresses over p, heat fluxes over p sqrt(RT)."""
    p = rho * R * T
    cs = np.sqrt(R * T)
    return np.concatenate([hot[:, :6] / p[:, None], hot[:, 6:] / (p * cs)[:, None]], axis=1)


# Expected squared norm of the nondimensional (sigma/p, q/(p sqrt(RT)))
# estimated from one Maxwellian particle: 3 x 4/3 (normal stresses) + 3 x 1
# (shear stresses) + 3 x 5/2 (heat fluxes), from the Gaussian moments.
NOISE_PER_PARTICLE = 14.5


def gate(mlp_out, sampled_hot_nd, sampled_stress_nd, tol, n_samples=None):
    """Per cell: use the MLP when its distance to the sampled HoT is at most
    tol times max(sqrt(|sampled stress and heat flux|^2 + noise^2), 1e-3)
    and finite, the noise being the sampling error of that vector for
    n_samples particle samples (14.5 / n_samples; none when n_samples is
    None): a network within the sample's own noise of it is accepted."""
    s2 = np.sum(np.asarray(sampled_stress_nd, dtype=np.float64) ** 2, axis=1)
    if n_samples is not None:
        n = np.asarray(n_samples, dtype=np.float64)
        s2 = s2 + np.where(n > 0, NOISE_PER_PARTICLE / np.where(n > 0, n, 1.0), 0.0)
    e = np.linalg.norm(mlp_out - sampled_hot_nd, axis=1) / np.maximum(np.sqrt(s2), 1e-3)
    return np.isfinite(e) & (e <= tol), e
