"""Oracle of the learned T2 starting guess, FP64, plain NumPy.

Test infrastructure only: nothing in the library imports this module.

The paper starts CCSD from the MP1 amplitudes (Eq. 21).  The learned guess
keeps that starting point and adds a per-amplitude correction predicted by a
small multilayer perceptron from quantities that exist before the first
iteration:

    t2_0[i,j,a,b] = t_MP1[i,j,a,b] + y_mu + y_sigma * net(norm(x[i,j,a,b])),
    t1_0 = 0,

where x is the feature vector below, norm(x) = (x - mu) * inv_sigma, and net is
an MLP with three hidden layers of width H (256 in the library) and SiLU
activations (silu(z) = z / (1 + exp(-z))):

    h1 = silu(W1 norm(x) + b1),  h2 = silu(W2 h1 + b2),  h3 = silu(W3 h2 + b3),
    net = w4 . h3 + b4.

Training minimises the mean squared error between net(norm(x)) and the
standardised target (t_CCSD - t_MP1 - y_mu) / y_sigma over sampled amplitudes.
The CCSD equations decide the final answer; the guess only changes the number
of iterations.

Features of amplitude (i, j, a, b), with K[i,a,j,b] = (ia|jb) and
D = e_i + e_j - e_a - e_b.  Every feature is unchanged under
(i, j, a, b) -> (j, i, b, a), so the guess keeps the symmetry
t_ij^ab = t_ji^ba of the exact amplitudes:
     0  K[i,a,j,b] / D             (the MP1 amplitude t_ij^ab)
     1  K[i,b,j,a] / D             (its exchange partner t_ij^ba)
     2  K[i,a,j,b]
     3  K[i,b,j,a]
     4  1 / D
     5  D
     6  e_i + e_j                  7  |e_i - e_j|
     8  e_a + e_b                  9  |e_a - e_b|
    10  |B_ia| |B_jb|              (|B_pq| = Euclidean norm over Q of B[Q,p,q])
    11  |B_ib| |B_ja|
    12  1 if i == j else 0
    13  1 if a == b else 0
    14  (ii|aa) + (jj|bb)
    15  (ii|bb) + (jj|aa)

Model blob (FP32, the layout the library reads): 64 header floats
[mu(16), inv_sigma(16), y_mu, y_sigma, zeros], then the trainable parameters
W1[H][16], b1[H], W2[H][H], b2[H], W3[H][H], b3[H], w4[H], b4, zero padding to
a multiple of 64 floats.
"""
from __future__ import annotations

import dataclasses

import numpy as np

NFEAT = 16
HEADER = 64


def pair_features(B: np.ndarray, eps_occ: np.ndarray, eps_vir: np.ndarray) -> np.ndarray:
    """All features as X[i,j,a,b,f] (FP64), from the definitions above."""
    o, v = eps_occ.size, eps_vir.size
    Bov = B[:, :o, o:]
    K = np.einsum("Qia,Qjb->iajb", Bov, Bov)
    D = (eps_occ[:, None, None, None] + eps_occ[None, :, None, None]
         - eps_vir[None, None, :, None] - eps_vir[None, None, None, :])
    Kd = K.transpose(0, 2, 1, 3)                 # [i,j,a,b] = (ia|jb)
    Kx = K.transpose(0, 2, 3, 1)                 # [i,j,a,b] = (ib|ja)
    nrm = np.sqrt(np.einsum("Qia,Qia->ia", Bov, Bov))
    diag_o = np.einsum("Qii->Qi", B[:, :o, :o])
    diag_v = np.einsum("Qaa->Qa", B[:, o:, o:])
    J = diag_o.T @ diag_v                        # J[i,a] = (ii|aa)
    X = np.empty((o, o, v, v, NFEAT))
    X[..., 0] = Kd / D
    X[..., 1] = Kx / D
    X[..., 2] = Kd
    X[..., 3] = Kx
    X[..., 4] = 1.0 / D
    X[..., 5] = D
    eo_i, eo_j = eps_occ[:, None, None, None], eps_occ[None, :, None, None]
    ev_a, ev_b = eps_vir[None, None, :, None], eps_vir[None, None, None, :]
    X[..., 6] = eo_i + eo_j + 0 * ev_a
    X[..., 7] = np.abs(eo_i - eo_j) + 0 * ev_a
    X[..., 8] = ev_a + ev_b + 0 * eo_i
    X[..., 9] = np.abs(ev_a - ev_b) + 0 * eo_i
    X[..., 10] = nrm[:, None, :, None] * nrm[None, :, None, :]
    X[..., 11] = nrm[:, None, None, :] * nrm[None, :, :, None]
    X[..., 12] = np.eye(o)[:, :, None, None]
    X[..., 13] = np.eye(v)[None, None, :, :]
    X[..., 14] = J[:, None, :, None] + J[None, :, None, :]
    X[..., 15] = J[:, None, None, :] + J[None, :, :, None]
    return X


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


@dataclasses.dataclass
class Model:
    mu: np.ndarray
    inv_sigma: np.ndarray
    y_mu: float
    y_sigma: float
    W1: np.ndarray
    b1: np.ndarray
    W2: np.ndarray
    b2: np.ndarray
    W3: np.ndarray
    b3: np.ndarray
    w4: np.ndarray
    b4: float

    PARAMS = ("W1", "b1", "W2", "b2", "W3", "b3", "w4", "b4")


def n_params(H: int) -> int:
    n = H * NFEAT + H + 2 * (H * H + H) + H + 1
    return (n + 63) // 64 * 64


def unpack(blob: np.ndarray, H: int = 256) -> Model:
    """Model from a flat blob in the layout of the module docstring."""
    b = np.asarray(blob, dtype=np.float64)
    hdr = b[:HEADER]
    p = b[HEADER:]
    shapes = [(H, NFEAT), (H,), (H, H), (H,), (H, H), (H,), (H,), ()]
    vals = []
    off = 0
    for s in shapes:
        n = int(np.prod(s)) if s else 1
        vals.append(p[off:off + n].reshape(s) if s else float(p[off]))
        off += n
    return Model(hdr[:16].copy(), hdr[16:32].copy(), float(hdr[32]), float(hdr[33]),
                 *[v.copy() if isinstance(v, np.ndarray) else v for v in vals])


def pack(m: Model) -> np.ndarray:
    H = m.b1.size
    hdr = np.zeros(HEADER)
    hdr[:16], hdr[16:32], hdr[32], hdr[33] = m.mu, m.inv_sigma, m.y_mu, m.y_sigma
    p = np.zeros(n_params(H))
    flat = np.concatenate([m.W1.ravel(), m.b1, m.W2.ravel(), m.b2, m.W3.ravel(), m.b3, m.w4,
                           [m.b4]])
    p[:flat.size] = flat
    return np.concatenate([hdr, p])


def forward(m: Model, X: np.ndarray):
    """Network output net(norm(x)) for rows of X [n, 16] and the cache for backward."""
    xn = (X - m.mu) * m.inv_sigma
    z1 = xn @ m.W1.T + m.b1
    h1 = silu(z1)
    z2 = h1 @ m.W2.T + m.b2
    h2 = silu(z2)
    z3 = h2 @ m.W3.T + m.b3
    h3 = silu(z3)
    y = h3 @ m.w4 + m.b4
    return y, (xn, z1, h1, z2, h2, z3, h3)


def predict_correction(m: Model, X: np.ndarray) -> np.ndarray:
    """t2_0 - t_MP1 for rows of X."""
    y, _ = forward(m, X)
    return m.y_mu + m.y_sigma * y


def loss_and_grad(m: Model, X: np.ndarray, target: np.ndarray):
    """L = mean_n (net(norm(x_n)) - s_n)^2 with s = (target - y_mu) / y_sigma, and dL/dparams
    by the chain rule (returned as a Model whose parameter fields hold gradients)."""
    n = X.shape[0]
    y, (xn, z1, h1, z2, h2, z3, h3) = forward(m, X)
    s = (target - m.y_mu) / m.y_sigma
    r = y - s
    L = float(np.mean(r * r))
    dy = 2.0 * r / n
    g = dataclasses.replace(m)
    g.w4 = h3.T @ dy
    g.b4 = float(dy.sum())
    dz3 = np.outer(dy, m.w4) * dsilu(z3)
    g.W3 = dz3.T @ h2
    g.b3 = dz3.sum(axis=0)
    dz2 = (dz3 @ m.W3) * dsilu(z2)
    g.W2 = dz2.T @ h1
    g.b2 = dz2.sum(axis=0)
    dz1 = (dz2 @ m.W2) * dsilu(z1)
    g.W1 = dz1.T @ xn
    g.b1 = dz1.sum(axis=0)
    return L, g


def adam_step(p: np.ndarray, g: np.ndarray, m1: np.ndarray, m2: np.ndarray, step: int,
              lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """Adam (Kingma and Ba 2015) on flat arrays; step counts from 1.  Updates in place."""
    m1 *= beta1
    m1 += (1 - beta1) * g
    m2 *= beta2
    m2 += (1 - beta2) * g * g
    mh = m1 / (1 - beta1 ** step)
    vh = m2 / (1 - beta2 ** step)
    p -= lr * mh / (np.sqrt(vh) + eps)


# ---------------------------------------------------------------- training
MASK64 = (1 << 64) - 1


def splitmix64(z: int) -> int:
    """Output function of splitmix64 (Steele, Lea and Flood, OOPSLA 2014) at
    counter value z: add the golden-gamma increment, then two xor-shift-multiply
    rounds and a final xor-shift, all modulo 2^64."""
    z = (z + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def minibatch_rows(seed: int, step: int, batch: int, n: int) -> np.ndarray:
    """Rows of the minibatch of Adam step `step` (counted from 1): row k is
    splitmix64(seed XOR splitmix64(step * 2^32 + k)) mod n."""
    return np.array([splitmix64((seed ^ splitmix64(((step << 32) | k) & MASK64)) & MASK64) % n
                     for k in range(batch)], dtype=np.int64)


def gradient_vector(m: Model, g: Model) -> np.ndarray:
    """Trainable part of the blob layout holding the gradient fields of g."""
    return pack(dataclasses.replace(g, mu=m.mu, inv_sigma=m.inv_sigma, y_mu=m.y_mu,
                                    y_sigma=m.y_sigma))[HEADER:]


def train(blob: np.ndarray, X: np.ndarray, Y: np.ndarray, step0: int, nsteps: int, batch: int,
          lr: float, seed: int, m1: np.ndarray | None = None, m2: np.ndarray | None = None):
    """nsteps Adam steps on the trainable part of blob (FP64 copy), each on the
    minibatch drawn by minibatch_rows; returns (blob, m1, m2, losses)."""
    b = np.array(blob, dtype=np.float64)
    H = 256
    P = n_params(H)
    m1 = np.zeros(P) if m1 is None else np.array(m1, dtype=np.float64)
    m2 = np.zeros(P) if m2 is None else np.array(m2, dtype=np.float64)
    losses = []
    for k in range(nsteps):
        t = step0 + k + 1
        rows = minibatch_rows(seed, t, batch, X.shape[0])
        m = unpack(b, H)
        L, g = loss_and_grad(m, X[rows], Y[rows])
        losses.append(L)
        p = b[HEADER:]
        adam_step(p, gradient_vector(m, g), m1, m2, t, lr)
        b[HEADER:] = p
    return b, m1, m2, losses
