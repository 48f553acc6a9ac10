"""FP64 oracle of the learned warm start: a message-passing network that predicts the
correction from the first guess y_n (Algorithm 1, first line) to the converged
positions x_{n+1} of a cell.

TEST INFRASTRUCTURE ONLY (see the package header).  The paper gives no network; this
module writes out, in plain NumPy, the network that the GPU library implements, so
that its inference, its gradients and its optimiser step can be checked element by
element.  Definitions:

Frame (Kabsch / orthogonal Procrustes).  With masses m_i, mass-weighted centroids
x_c of x_n and X_c of the rest mesh X, and C = sum_i m_i (x_i - x_c)(X_i - X_c)^T,
R = U diag(1, 1, det(U V^T)) V^T from the SVD C = U S V^T: the rotation that best
maps the centred rest shape onto the centred current shape.

Scales.  v_c = mass-weighted mean velocity; a_c = sum F / sum m; the de-meaned force
F'_i = F_i - m_i a_c; F_rms = sqrt(mean_i |F'_i|^2); mean mass m_bar; the
displacement scale of the cell s = h^2 (F_rms + F0) / m_bar with a force floor F0.

Node features (12), all in the cell frame:
  [0:3]  (R^T (x_i - x_c) - (X_i - X_c)) / l_shape       shape deviation
  [3:6]  R^T (v_i - v_c) h / s                            velocity
  [6:9]  R^T F'_i h^2 / (m_i s)                           force
  [9:12] (X_i - X_c) / rho, rho = max_i |X_i - X_c|       place on the rest shape

Network (residual GraphSAGE with mean aggregation over mesh neighbours N(i)):
  h = relu(W_e f + b_e);  for each of the L layers:
      a_i = mean_{j in N(i)} h_j,  z = W_s h + W_n a + b,  h <- h + relu(z)
  o = W_d h + b_d  (3 outputs per node), and the correction is delta_i = s R o_i.

Loss (training on solver trajectories): the mean over cells, nodes and components of
(o_i - t_i)^2 with the target t_i = R^T (x_{n+1,i} - y_{n,i}) / s.

Flat parameter vector (float): W_e [H][12], b_e [H]; per layer W_s [H][H], W_n [H][H],
b [H]; then W_d [3][H], b_d [3] -- row-major, H = hidden width.

Optimiser: Adam (Kingma & Ba 2015) with bias correction.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

N_FEAT = 12


@dataclass
class NetConfig:
    hidden: int = 64
    layers: int = 4
    force_floor: float = 1.0        # F0, force units
    shape_scale: float = 0.1        # l_shape, length units


def param_count(cfg: NetConfig) -> int:
    H = cfg.hidden
    return H * N_FEAT + H + cfg.layers * (2 * H * H + H) + 3 * H + 3


def unpack(theta: np.ndarray, cfg: NetConfig) -> dict:
    """Views of the flat parameter vector in the documented order."""
    H, k = cfg.hidden, 0
    p = {}

    def take(name, shape):
        nonlocal k
        size = int(np.prod(shape))
        p[name] = theta[k:k + size].reshape(shape)
        k += size

    take("We", (H, N_FEAT))
    take("be", (H,))
    for l in range(cfg.layers):
        take(f"Ws{l}", (H, H))
        take(f"Wn{l}", (H, H))
        take(f"b{l}", (H,))
    take("Wd", (3, H))
    take("bd", (3,))
    assert k == theta.size
    return p


def init_params(cfg: NetConfig, seed: int) -> np.ndarray:
    """He-style initial weights (biases zero, output layer scaled down)."""
    rng = np.random.default_rng(seed)
    theta = np.zeros(param_count(cfg))
    p = unpack(theta, cfg)
    H = cfg.hidden
    p["We"][:] = rng.standard_normal((H, N_FEAT)) * np.sqrt(2.0 / N_FEAT)
    for l in range(cfg.layers):
        p[f"Ws{l}"][:] = rng.standard_normal((H, H)) * np.sqrt(1.0 / H)
        p[f"Wn{l}"][:] = rng.standard_normal((H, H)) * np.sqrt(1.0 / H)
    p["Wd"][:] = rng.standard_normal((3, H)) * np.sqrt(1.0 / H) * 0.1
    return theta


def neighbour_mean_matrix(n: int, tris: np.ndarray):
    """Sparse operator A with (A h)_i = mean of h_j over the mesh neighbours j of i,
    built from the triangle list (each triangle edge joins two neighbours)."""
    import scipy.sparse as sp
    t = np.asarray(tris, np.int64)
    r = np.concatenate([t[:, 0], t[:, 1], t[:, 2], t[:, 1], t[:, 2], t[:, 0]])
    c = np.concatenate([t[:, 1], t[:, 2], t[:, 0], t[:, 0], t[:, 1], t[:, 2]])
    A = sp.coo_matrix((np.ones(r.size), (r, c)), shape=(n, n)).tocsr()
    A.data[:] = 1.0                              # each directed edge once
    deg = np.asarray(A.sum(axis=1)).ravel()
    return sp.diags(1.0 / deg) @ A


def kabsch(X: np.ndarray, x: np.ndarray, m: np.ndarray):
    """Rotation R (rest -> current) and the two mass-weighted centroids."""
    w = m / m.sum()
    xc, Xc = w @ x, w @ X
    C = (m[:, None] * (x - xc)).T @ (X - Xc)
    U, _, Vt = np.linalg.svd(C)
    d = np.sign(np.linalg.det(U @ Vt))
    R = U @ np.diag([1.0, 1.0, d]) @ Vt
    return R, xc, Xc


def features(X, x, v, F, m, h, cfg: NetConfig):
    """Node features [n, 12], the frame R and the displacement scale s of one cell."""
    R, xc, Xc = kabsch(X, x, m)
    w = m / m.sum()
    vc = w @ v
    ac = F.sum(axis=0) / m.sum()
    Fd = F - m[:, None] * ac
    Frms = np.sqrt(np.mean(np.sum(Fd * Fd, axis=1)))
    s = h * h * (Frms + cfg.force_floor) / m.mean()
    rho = np.max(np.linalg.norm(X - Xc, axis=1))
    f = np.empty((len(X), N_FEAT))
    f[:, 0:3] = ((x - xc) @ R - (X - Xc)) / cfg.shape_scale       # rows: R^T (x_i - x_c)
    f[:, 3:6] = ((v - vc) @ R) * (h / s)
    f[:, 6:9] = (Fd @ R) * (h * h / s) / m[:, None]
    f[:, 9:12] = (X - Xc) / rho
    return f, R, s


def relu(z):
    return np.maximum(z, 0.0)


def forward(theta, f, Amean, cfg: NetConfig):
    """Outputs o [n, 3] and the activations the backward pass needs."""
    p = unpack(theta, cfg)
    z0 = f @ p["We"].T + p["be"]
    h = relu(z0)
    cache = {"f": f, "z0": z0, "h": [h], "a": [], "z": []}
    for l in range(cfg.layers):
        a = Amean @ h
        z = h @ p[f"Ws{l}"].T + a @ p[f"Wn{l}"].T + p[f"b{l}"]
        h = h + relu(z)
        cache["a"].append(a)
        cache["z"].append(z)
        cache["h"].append(h)
    o = h @ p["Wd"].T + p["bd"]
    return o, cache


def backward(theta, cache, dO, Amean, cfg: NetConfig) -> np.ndarray:
    """Gradient of sum(dO * o) with respect to the flat parameters (chain rule through
    the layers in reverse order)."""
    p = unpack(theta, cfg)
    g = np.zeros_like(theta)
    q = unpack(g, cfg)
    hL = cache["h"][-1]
    q["Wd"][:] = dO.T @ hL
    q["bd"][:] = dO.sum(axis=0)
    dh = dO @ p["Wd"]
    for l in reversed(range(cfg.layers)):
        z, a, hin = cache["z"][l], cache["a"][l], cache["h"][l]
        dz = dh * (z > 0)
        q[f"Ws{l}"][:] = dz.T @ hin
        q[f"Wn{l}"][:] = dz.T @ a
        q[f"b{l}"][:] = dz.sum(axis=0)
        da = dz @ p[f"Wn{l}"]
        dh = dh + dz @ p[f"Ws{l}"] + Amean.T @ da
    dz0 = dh * (cache["z0"] > 0)
    q["We"][:] = dz0.T @ cache["f"]
    q["be"][:] = dz0.sum(axis=0)
    return g


def target(R, s, delta):
    """t_i = R^T delta_i / s for the world-frame correction delta = x_{n+1} - y_n."""
    return (delta @ R) / s


def loss_and_grad(theta, cells, Amean, cfg: NetConfig):
    """Mean squared error over all cells, nodes and components, and its gradient.
    cells: list of (features, target) pairs of equal node count."""
    n_tot = sum(f.shape[0] for f, _ in cells) * 3
    L = 0.0
    g = np.zeros_like(theta)
    for f, t in cells:
        o, cache = forward(theta, f, Amean, cfg)
        r = o - t
        L += np.sum(r * r)
        g += backward(theta, cache, 2.0 * r / n_tot, Amean, cfg)
    return L / n_tot, g


def predict_delta(theta, X, x, v, F, m, h, Amean, cfg: NetConfig):
    """World-frame correction delta_i = s R o_i for one cell."""
    f, R, s = features(X, x, v, F, m, h, cfg)
    o, _ = forward(theta, f, Amean, cfg)
    return s * (o @ R.T)


@dataclass
class Adam:
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8


def adam_update(theta, g, mom, vel, t: int, opt: Adam):
    """One Adam step (t counts from 1); returns the new (theta, mom, vel)."""
    mom = opt.beta1 * mom + (1.0 - opt.beta1) * g
    vel = opt.beta2 * vel + (1.0 - opt.beta2) * g * g
    mhat = mom / (1.0 - opt.beta1 ** t)
    vhat = vel / (1.0 - opt.beta2 ** t)
    return theta - opt.lr * mhat / (np.sqrt(vhat) + opt.eps), mom, vel


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 value (ties to even), returned as float64."""
    a32 = np.ascontiguousarray(a, np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
