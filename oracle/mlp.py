"""The learned insertion proposal, written plainly in FP64 (test infrastructure only).

Network 352 -> 128 -> 128 -> 128 with ReLU between layers.  The 128 outputs are two
groups of 64 logits: the bin of the creator time tau_s and the bin of the pair
length l = (tau_e - tau_s) mod beta, each on 64 equal bins of [0, beta).  Loss
per sample: -log softmax(z_tau)[t_tau] - log softmax(z_l)[t_l]; the batch loss is
the mean.

With quantize=True the forward and backward pass round to BF16 at the points where
the device stores BF16:
- the weights;
- the hidden activations after ReLU;
- the output gradient and the masked hidden gradients that enter the next
  products.
Everything else is FP64.  With quantize=False it is the plain FP64 network, which
the finite-difference pins check.

Features of (configuration without the pair, flavor f), 352 entries:
- one-hot f (F entries);
- k_g / 32 for every flavor g (F entries);
- for every flavor g and each of 32 equal time bins b, the number of creators minus
  annihilators of g before the bin centre (b + 1/2) beta / 32 (32 F entries);
- zeros up to 352.

Insertion density of a pair:

    q(tau_s, l) = (1 - eps) p_tau(bin tau_s) (64 / beta) p_l(bin l) (64 / beta) + eps / beta^2
"""
from __future__ import annotations

import numpy as np

IN, H, OUT, BINS, TBINS = 352, 128, 128, 64, 32


def bf16(x):
    """Round to the nearest BF16 value (ties to even) via the float32 bit pattern."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def features(cre, ann, f: int, beta: float, exclude=None) -> np.ndarray:
    """Features of flavor f proposing into the configuration (cre, ann), leaving out the
    pair exclude = (flavor, creator label, annihilator label) if given."""
    F = len(cre)
    x = np.zeros(IN)
    x[f] = 1.0
    for g in range(F):
        k = len(cre[g]) - (1 if exclude is not None and exclude[0] == g else 0)
        x[F + g] = k / 32.0
    for g in range(F):
        for b in range(TBINS):
            tb = (b + 0.5) * beta / TBINS
            cnt = 0
            for q, t in enumerate(cre[g]):
                if not (exclude is not None and exclude[0] == g and exclude[1] == q) and t < tb:
                    cnt += 1
            for q, t in enumerate(ann[g]):
                if not (exclude is not None and exclude[0] == g and exclude[2] == q) and t < tb:
                    cnt -= 1
            x[2 * F + g * TBINS + b] = cnt
    return x


def _softmax(z):
    e = np.exp(z - z.max(axis=-1, keepdims=True))
    return e / e.sum(axis=-1, keepdims=True)


class Network:
    """Ws = [W1 (128 x 352), W2 (128 x 128), W3 (128 x 128)] (output-major), bs = biases."""

    def __init__(self, Ws, bs, quantize: bool = True):
        self.q = quantize
        rnd = bf16 if quantize else (lambda a: np.asarray(a, dtype=np.float64))
        self.W = [rnd(np.asarray(W, dtype=np.float64)) for W in Ws]
        self.b = [np.asarray(b, dtype=np.float64) for b in bs]
        self.rnd = rnd

    def forward(self, X):
        X = np.asarray(X, dtype=np.float64)
        Z1 = np.maximum(X @ self.W[0].T + self.b[0], 0.0)
        H1 = self.rnd(Z1)
        Z2 = np.maximum(H1 @ self.W[1].T + self.b[1], 0.0)
        H2 = self.rnd(Z2)
        Z3 = H2 @ self.W[2].T + self.b[2]
        return dict(X=X, Z1=Z1, H1=H1, Z2=Z2, H2=H2, Z3=Z3)

    def loss(self, X, T):
        Z3 = self.forward(X)["Z3"]
        lt = np.log(_softmax(Z3[:, :BINS]))
        ll = np.log(_softmax(Z3[:, BINS:]))
        n = len(T)
        return float(-(lt[np.arange(n), T[:, 0]] + ll[np.arange(n), T[:, 1]]).mean())

    def gradients(self, X, T):
        """(dWs, dbs, loss) of the mean loss."""
        a = self.forward(X)
        n = len(T)
        P = np.concatenate([_softmax(a["Z3"][:, :BINS]), _softmax(a["Z3"][:, BINS:])], axis=1)
        Y = np.zeros_like(P)
        Y[np.arange(n), T[:, 0]] = 1.0
        Y[np.arange(n), BINS + T[:, 1]] = 1.0
        dZ3 = (P - Y) / n
        loss = float(-(np.log(P[np.arange(n), T[:, 0]]) + np.log(P[np.arange(n), BINS + T[:, 1]])).mean())
        dZ3q = self.rnd(dZ3)
        dW3 = dZ3q.T @ a["H2"]
        db3 = dZ3.sum(axis=0)
        dZ2 = (dZ3q @ self.W[2]) * (a["Z2"] > 0)
        dZ2q = self.rnd(dZ2)
        dW2 = dZ2q.T @ a["H1"]
        db2 = dZ2.sum(axis=0)
        dZ1 = (dZ2q @ self.W[1]) * (a["Z1"] > 0)
        dZ1q = self.rnd(dZ1)
        dW1 = dZ1q.T @ a["X"]
        db1 = dZ1.sum(axis=0)
        return [dW1, dW2, dW3], [db1, db2, db3], loss


def logq(z, ts: float, length: float, beta: float, eps: float) -> float:
    """log q(tau_s, l) for one row of logits z (128 values)."""
    pt = _softmax(np.asarray(z[:BINS], dtype=np.float64))
    pl = _softmax(np.asarray(z[BINS:], dtype=np.float64))
    bs = min(int(ts / beta * BINS), BINS - 1)
    bl = min(int(length / beta * BINS), BINS - 1)
    d = BINS / beta
    return float(np.log((1.0 - eps) * pt[bs] * d * pl[bl] * d + eps / beta ** 2))
