"""Training and inference driver of the selector's cost model.

All arithmetic of the network (forward, backward, Adam) runs in the
library's HIP kernels (csrc/mlp.hip); this module only moves data.  Inputs
are standardised with the training set's mean and deviation; for inference
the standardisation is folded into the first layer
(W1' = W1 / sigma, b1' = b1 - (mu / sigma) W1), an exact identity, so raw
device features go straight into the forward kernel.
"""
from __future__ import annotations

import json

import numpy as np

from . import ewahthr as E

NI, H = 16, 64


def _unpack(p, k):
    o = 0
    W1 = p[o:o + NI * H].reshape(NI, H); o += NI * H
    b1 = p[o:o + H]; o += H
    rest = p[o:]
    return W1, b1, rest


def fold_standardisation(p: np.ndarray, k: int, mu: np.ndarray, sigma: np.ndarray) -> np.ndarray:
    W1, b1, rest = _unpack(np.asarray(p, dtype=np.float64), k)
    W1f = W1 / sigma[:, None]
    b1f = b1 - (mu / sigma) @ W1
    return np.concatenate([W1f.ravel(), b1f, rest]).astype(np.float32)


def standardiser(X: np.ndarray):
    mu = X.mean(axis=0).astype(np.float64)
    sd = X.std(axis=0).astype(np.float64)
    sd[sd < 1e-6] = 1.0
    mu[-1] = 0.0          # constant input stays 1
    sd[-1] = 1.0
    return mu, sd


def train(X: np.ndarray, Y: np.ndarray, epochs: int = 60, batch: int = 1024, lr: float = 2e-3, seed: int = 1,
          log=None):
    """Fit the MLP on standardised features X [n, 16] and targets Y [n, K] on the GPU.
    Returns (model dict with folded weights, loss history)."""
    import torch
    n, k = Y.shape
    mu, sd = standardiser(X)
    Xs = ((X - mu) / sd).astype(np.float32)
    Xs[:, -1] = 1.0
    ym = Y.mean()
    Yc = (Y - ym).astype(np.float32)      # targets as given (the caller centres per query if it wants relative costs)
    net = E.MLP(k, seed)
    rng = np.random.default_rng(seed)
    dX = torch.empty((n, NI), dtype=torch.float32, device="cuda")
    dY = torch.empty((n, k), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    hist = []
    for ep in range(epochs):
        perm = rng.permutation(n)
        dX.copy_(torch.from_numpy(Xs[perm]))
        dY.copy_(torch.from_numpy(Yc[perm]))
        tot, nb = 0.0, 0
        for s in range(0, n, batch):
            b = min(batch, n - s)
            net.train_step(dX.data_ptr() + 4 * NI * s, dY.data_ptr() + 4 * k * s, b, lr, loss.data_ptr(), stream)
            if nb % 8 == 0:
                tot += float(loss.item())
            nb += 1
        hist.append(tot / max(1, (nb + 7) // 8))
        if log and (ep % 10 == 0 or ep == epochs - 1):
            log(f"epoch {ep}: mse {hist[-1]:.4f}")
    p = net.get_params()
    net.free()
    model = {"kind": "mlp", "n_out": k, "mu": mu.tolist(), "sigma": sd.tolist(), "y_mean": float(ym),
             "params_raw": p.astype(float).tolist(),
             "params_folded": fold_standardisation(p, k, mu, sd).astype(float).tolist()}
    return model, hist


class Predictor:
    """Inference on device with folded weights: features (device) -> predicted log-times (device)."""

    def __init__(self, model: dict, seed: int = 1):
        self.k = int(model["n_out"])
        self.net = E.MLP(self.k, seed)
        self.net.set_params(np.asarray(model["params_folded"], dtype=np.float32))

    def forward(self, feat_ptr: int, n: int, pred_ptr: int, stream=None):
        self.net.forward(feat_ptr, n, pred_ptr, stream)

    def free(self):
        self.net.free()


def save(model: dict, path: str):
    with open(path, "w") as f:
        json.dump(model, f)


def load(path: str) -> dict:
    with open(path) as f:
        return json.load(f)
