"""Message-passing warm start for the pressure-correction solve (FP64).

Not in the paper: a small graph network on the P1 mesh graph predicts a
correction to the previous pressure correction, used only as the initial
guess of the Jacobi-PCG solve (which still converges to the same residual
tolerance).  Definition:

Per-node inputs (X, [N, 6]), for K the pressure matrix with diagonal D:
  r     = b_phi - K phi_prev,  s = D^{-1} r,  sigma = rms(s) (1 if zero)
  x0 = s / sigma
  x1 = (D^{-1} b_phi) / rms(D^{-1} b_phi)            (0 if zero)
  x2 = phi_prev / rms(phi_prev)                        (0 if zero)
  x3..x5 = coordinates mapped to [-1, 1] by the mesh bounding box (0 if absent)
Edge weights on the off-diagonal CSR entries of K: w_ij = -K_ij / K_ii.
Network (hidden width 32, 3 message-passing layers):
  h0 = relu(X We^T + ce)
  a_l = Agg(h_{l-1}),  Agg(h)_i = sum_{j != i} w_ij h_j
  z_l = h_{l-1} Ws_l^T + a_l Wn_l^T + c_l,  h_l = h_{l-1} + relu(z_l)
  delta = h_3 wd + cd
Guess: phi_prev + sigma * delta.  Training target: (phi - phi_prev) / sigma,
and one of two losses, averaged over samples:
  mse    mean over nodes of (delta - target)^2;
  knorm  (delta - target)^T K (delta - target) / target^T K target, the
         K-norm (energy norm) of the guess error relative to that of
         phi_prev.  sigma cancels.  With phi the solution of K phi = b_phi,
         J(x) - J(phi) = 1/2 ||x - phi||_K^2 for J the CG energy below, so
         this loss is (J(guess) - J(phi)) / (J(phi_prev) - J(phi)): the
         quantity the guard compares and the error norm CG reduces.  A
         sample whose target has zero K-norm (phi_prev already exact up to
         a constant) has loss 0 and no gradient.
The solve starts from the guess only if its CG energy 1/2 x^T K x - b^T x
is below that of the plain start (phi_prev, or 0; guarded_start); PCG then
runs to the same tolerance.
Adam (beta1 0.9, beta2 0.999, eps 1e-8), bias-corrected.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

N_IN = 6
HID = 32
LAYERS = 3
PARAM_SHAPES = [("We", (HID, N_IN)), ("ce", (HID,)),
                ("Ws", (LAYERS, HID, HID)), ("Wn", (LAYERS, HID, HID)), ("c", (LAYERS, HID)),
                ("wd", (HID,)), ("cd", (1,))]


def init_params(seed=0):
    rng = np.random.default_rng(seed)
    P = {}
    P["We"] = rng.normal(0, np.sqrt(2.0 / N_IN), (HID, N_IN))
    P["ce"] = np.zeros(HID)
    P["Ws"] = rng.normal(0, np.sqrt(1.0 / HID), (LAYERS, HID, HID)) * 0.5
    P["Wn"] = rng.normal(0, np.sqrt(1.0 / HID), (LAYERS, HID, HID)) * 0.5
    P["c"] = np.zeros((LAYERS, HID))
    P["wd"] = np.zeros(HID)
    P["cd"] = np.zeros(1)
    return P


def edge_weights(K):
    """CSR matrix W with W_ij = -K_ij / K_ii for j != i."""
    K = K.tocsr()
    d = K.diagonal()
    W = sp.diags(1.0 / d) @ K
    W = W.tocsr()
    W.setdiag(0.0)
    W.eliminate_zeros()
    return -W


def _rms(v):
    return float(np.sqrt(np.mean(v * v)))


def features(K, b_phi, phi_prev, coords):
    d = K.diagonal()
    r = b_phi - K @ phi_prev
    s = r / d
    sigma = _rms(s)
    if sigma == 0.0:
        sigma = 1.0
    N = b_phi.size
    X = np.zeros((N, N_IN))
    X[:, 0] = s / sigma
    bd = b_phi / d
    rb = _rms(bd)
    X[:, 1] = bd / rb if rb > 0 else 0.0
    rp = _rms(phi_prev)
    X[:, 2] = phi_prev / rp if rp > 0 else 0.0
    lo = coords.min(axis=0)
    hi = coords.max(axis=0)
    for a in range(coords.shape[1]):
        span = hi[a] - lo[a]
        X[:, 3 + a] = 2.0 * (coords[:, a] - lo[a]) / span - 1.0 if span > 0 else 0.0
    return X, sigma


def forward(P, X, W):
    cache = {"X": X, "z": [], "h": [], "a": []}
    z0 = X @ P["We"].T + P["ce"]
    h = np.maximum(z0, 0.0)
    cache["z0"] = z0
    cache["h"].append(h)
    for l in range(LAYERS):
        a = W @ h
        z = h @ P["Ws"][l].T + a @ P["Wn"][l].T + P["c"][l]
        h = h + np.maximum(z, 0.0)
        cache["a"].append(a)
        cache["z"].append(z)
        cache["h"].append(h)
    delta = h @ P["wd"] + P["cd"][0]
    return delta, cache


def loss(delta, target, kind="mse", K=None):
    e = delta - target
    if kind == "mse":
        return float(np.mean(e * e))
    if kind != "knorm":
        raise ValueError(kind)
    den = float(target @ (K @ target))
    return float(e @ (K @ e)) / den if den > 0 else 0.0


def loss_seed(delta, target, kind="mse", K=None):
    """d loss / d delta."""
    e = delta - target
    if kind == "mse":
        return 2.0 * e / delta.size
    if kind != "knorm":
        raise ValueError(kind)
    den = float(target @ (K @ target))
    return 2.0 * (K @ e) / den if den > 0 else np.zeros_like(e)


def backward(P, cache, delta, target, W, kind="mse", K=None):
    """Gradients of loss(delta, target, kind, K) with respect to every
    parameter (K: the pressure matrix, for the K-norm loss)."""
    G = {k: np.zeros(s) for k, s in PARAM_SHAPES}
    gd = loss_seed(delta, target, kind, K)
    h3 = cache["h"][LAYERS]
    G["wd"] = h3.T @ gd
    G["cd"] = np.array([gd.sum()])
    gh = np.outer(gd, P["wd"])
    WT = W.T.tocsr()
    for l in reversed(range(LAYERS)):
        hprev = cache["h"][l]
        gz = gh * (cache["z"][l] > 0.0)
        G["Ws"][l] = gz.T @ hprev
        G["Wn"][l] = gz.T @ cache["a"][l]
        G["c"][l] = gz.sum(axis=0)
        gh = gh + gz @ P["Ws"][l] + WT @ (gz @ P["Wn"][l])
    gz0 = gh * (cache["z0"] > 0.0)
    G["We"] = gz0.T @ cache["X"]
    G["ce"] = gz0.sum(axis=0)
    return G


class Adam:
    def __init__(self, P, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = {k: np.zeros_like(v) for k, v in P.items()}
        self.v = {k: np.zeros_like(v) for k, v in P.items()}
        self.t = 0

    def step(self, P, G):
        self.t += 1
        for k in P:
            self.m[k] = self.b1 * self.m[k] + (1 - self.b1) * G[k]
            self.v[k] = self.b2 * self.v[k] + (1 - self.b2) * G[k] * G[k]
            mh = self.m[k] / (1 - self.b1 ** self.t)
            vh = self.v[k] / (1 - self.b2 ** self.t)
            P[k] = P[k] - self.lr * mh / (np.sqrt(vh) + self.eps)
        return P


def predict_guess(P, K, b_phi, phi_prev, coords):
    X, sigma = features(K, b_phi, phi_prev, coords)
    delta, _ = forward(P, X, edge_weights(K))
    return phi_prev + sigma * delta


def energy(K, b, x):
    """The functional CG minimises: J(x) = 1/2 x^T K x - b^T x."""
    return 0.5 * (x @ (K @ x)) - b @ x


def guarded_start(K, b_phi, plain, guess):
    """The guess is used only if its CG energy is lower than that of the
    plain start `plain` (phi_prev, or zeros); otherwise PCG starts from
    `plain`.  J(x) - J(x*) = 1/2 ||x - x*||_K^2, the error norm CG reduces."""
    j_g = energy(K, b_phi, guess)
    j_p = energy(K, b_phi, plain)
    if np.isfinite(j_g) and j_g < j_p:
        return guess, True
    return plain, False
