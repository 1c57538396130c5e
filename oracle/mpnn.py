"""CPU FP64 reference of the learned edge-criticality surrogate.

TEST INFRASTRUCTURE (see the package docstring): plain NumPy, FP64, one
operation per line of the model's definition; shares no code with the GPU
kernels.

Model (2 message-passing layers, hidden width H = 32, about 5k parameters):
    A1 = N X,                  N = D^-1 A (row-normalised adjacency of G)
    H1 = relu(X Ws1 + A1 Wn1 + b1)
    A2 = N H1
    H2 = relu(H1 Ws2 + A2 Wn2 + b2)
    for each candidate edge e = (p, q):
        z_e = [ |H2_p - H2_q| , H2_p * H2_q , f_e ]          (2H + 4)
        g_e = z_e Wh1 + bh1
        yhat_e = relu(g_e) . wh2 + bh2
    loss = mean_e (yhat_e - y_e)^2
The parameters live in one flat vector in the order of ``LAYOUT``.

Node features (8): 1, log D_G, log D_T, log deg_G, log deg_T, log |x_p|^2,
and the log local energies sum_q w_pq |x_p - x_q|^2 / D_p on G and on T, of a
cheap smoothed block x.  Edge features (4): log w, log of the cheap score
w |x_p - x_q|^2, and the min and max of log D_T at the two ends.  Both are
standardised with stored means and inverse standard deviations.
"""
from __future__ import annotations

import numpy as np

F_IN = 8
HID = 32
F_EDGE = 4
Z = 2 * HID + F_EDGE
TINY = 1e-30

LAYOUT = [
    ("Ws1", (F_IN, HID)), ("Wn1", (F_IN, HID)), ("b1", (HID,)),
    ("Ws2", (HID, HID)), ("Wn2", (HID, HID)), ("b2", (HID,)),
    ("Wh1", (Z, HID)), ("bh1", (HID,)), ("wh2", (HID,)), ("bh2", (1,)),
]


def n_params() -> int:
    return int(sum(np.prod(s) for _, s in LAYOUT))


def unpack(theta):
    out, o = {}, 0
    for name, shape in LAYOUT:
        c = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + c], dtype=np.float64).reshape(shape)
        o += c
    return out


def pack(d) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in LAYOUT])


def norm_adjacency(n, u, v, w):
    import scipy.sparse as sp

    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    A = sp.coo_matrix((np.concatenate([w, w]), (np.concatenate([u, v]), np.concatenate([v, u]))),
                      shape=(n, n)).tocsr()
    d = np.asarray(A.sum(axis=1)).reshape(-1)
    return A, d


def raw_features(n, u, v, w, tree_mask, xc, cand):
    """Unstandardised node (n x 8) and candidate-edge (ne x 4) features."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    t = np.asarray(tree_mask, dtype=bool)
    xc = np.asarray(xc, dtype=np.float64)
    dG = np.zeros(n)
    dT = np.zeros(n)
    cG = np.zeros(n)
    cT = np.zeros(n)
    eG = np.zeros(n)
    eT = np.zeros(n)
    diff2 = np.sum((xc[u] - xc[v]) ** 2, axis=1)
    for arr, vals, mask in ((dG, w, None), (cG, np.ones_like(w), None), (eG, w * diff2, None),
                            (dT, w, t), (cT, np.ones_like(w), t), (eT, w * diff2, t)):
        sel = slice(None) if mask is None else mask
        np.add.at(arr, u[sel], vals[sel])
        np.add.at(arr, v[sel], vals[sel])
    nf = np.stack([np.ones(n), np.log(dG), np.log(dT), np.log(cG), np.log(cT),
                   np.log(np.sum(xc * xc, axis=1) + TINY), np.log(eG / dG + TINY), np.log(eT / dT + TINY)], axis=1)
    c = np.asarray(cand, dtype=np.int64)
    lp, lq = np.log(dT[u[c]]), np.log(dT[v[c]])
    ef = np.stack([np.log(w[c]), np.log(w[c] * diff2[c] + TINY), np.minimum(lp, lq), np.maximum(lp, lq)], axis=1)
    return nf, ef


def standardise(nf, ef, norm):
    """norm = [node means (8), node inverse stds (8), edge means (4), edge inverse stds (4)]."""
    norm = np.asarray(norm, dtype=np.float64)
    nm, ns = norm[:F_IN], norm[F_IN:2 * F_IN]
    em, es = norm[2 * F_IN:2 * F_IN + F_EDGE], norm[2 * F_IN + F_EDGE:]
    nf2 = (nf - nm) * ns
    nf2[:, 0] = 1.0
    return nf2, (ef - em) * es


def forward(theta, A, d, X, u, v, cand, ef):
    P = unpack(theta)
    Nx = (A @ X) / d[:, None]
    P1 = X @ P["Ws1"] + Nx @ P["Wn1"] + P["b1"]
    H1 = np.maximum(P1, 0.0)
    A2 = (A @ H1) / d[:, None]
    P2 = H1 @ P["Ws2"] + A2 @ P["Wn2"] + P["b2"]
    H2 = np.maximum(P2, 0.0)
    c = np.asarray(cand, dtype=np.int64)
    p, q = np.asarray(u, dtype=np.int64)[c], np.asarray(v, dtype=np.int64)[c]
    zz = np.concatenate([np.abs(H2[p] - H2[q]), H2[p] * H2[q], ef], axis=1)
    G = zz @ P["Wh1"] + P["bh1"]
    Ah = np.maximum(G, 0.0)
    yhat = Ah @ P["wh2"] + P["bh2"][0]
    cache = dict(Nx=Nx, P1=P1, H1=H1, A2=A2, P2=P2, H2=H2, p=p, q=q, zz=zz, G=G, Ah=Ah)
    return yhat, cache


def loss(yhat, y) -> float:
    return float(np.mean((yhat - y) ** 2))


def backward(theta, A, d, X, y, yhat, cache):
    """Gradient of the mean squared error with respect to theta (flat)."""
    P = unpack(theta)
    ne = yhat.shape[0]
    dy = 2.0 * (yhat - y) / ne
    gr = {}
    gr["wh2"] = cache["Ah"].T @ dy
    gr["bh2"] = np.array([np.sum(dy)])
    dG = np.outer(dy, P["wh2"]) * (cache["G"] > 0)
    gr["Wh1"] = cache["zz"].T @ dG
    gr["bh1"] = np.sum(dG, axis=0)
    dz = dG @ P["Wh1"].T
    H2, p, q = cache["H2"], cache["p"], cache["q"]
    sgn = np.sign(H2[p] - H2[q])
    dH2 = np.zeros_like(H2)
    np.add.at(dH2, p, dz[:, :HID] * sgn + dz[:, HID:2 * HID] * H2[q])
    np.add.at(dH2, q, -dz[:, :HID] * sgn + dz[:, HID:2 * HID] * H2[p])
    dP2 = dH2 * (cache["P2"] > 0)
    gr["Ws2"] = cache["H1"].T @ dP2
    gr["Wn2"] = cache["A2"].T @ dP2
    gr["b2"] = np.sum(dP2, axis=0)
    # the transpose of N = D^-1 A is A D^-1
    dH1 = dP2 @ P["Ws2"].T + A.T @ ((dP2 @ P["Wn2"].T) / d[:, None])
    dP1 = dH1 * (cache["P1"] > 0)
    gr["Ws1"] = X.T @ dP1
    gr["Wn1"] = cache["Nx"].T @ dP1
    gr["b1"] = np.sum(dP1, axis=0)
    return pack(gr)


def adam_step(theta, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, 2015) with bias correction; step counts from 1."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed: int) -> np.ndarray:
    """He-style initial weights, zero biases (seeded)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = {}
    for name, shape in LAYOUT:
        if len(shape) == 2:
            d[name] = rng.standard_normal(shape) * np.sqrt(2.0 / shape[0])
        elif name == "wh2":
            d[name] = rng.standard_normal(shape) * np.sqrt(1.0 / shape[0])
        else:
            d[name] = np.zeros(shape)
    return pack(d)
