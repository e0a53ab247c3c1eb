"""CPU oracle of the learned refinement predictor (TEST INFRASTRUCTURE ONLY).

Plain FP64 numpy, written from the predictor's definition (a per-block MLP that
maps an 8x8 average pool of every field to refine / keep / coarsen logits):

* features: the block's synchronised node values, averaged over 8 x 8 bins of
  (bs-1)/8 nodes per direction (the last node row and column, shared with the
  neighbour, is not used); bins in x-fastest order, fields outer;
* normalisation per field: x_hat = (x - mean_f) / std_f;
* layers 256 -> 64 -> 64 -> 3 (nf*64 inputs), GELU(z) = z/2 (1 + erf(z/sqrt 2));
* loss: class-weighted softmax cross-entropy, divided by the sum of the weights of
  the batch's labels;
* Adam: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, p -= lr (m/(1-b1^t)) / (sqrt(v/(1-b2^t)) + eps);
* labels at horizon H from the method's own grids: a block of G^n at level l is
  'refine' (0) if any block of G^{n+H} finer than l overlaps it, 'coarsen' (2) if it
  lies inside a block of G^{n+H} coarser than l, else 'keep' (1).

Parameter vector layout (shared with the library): W1[nin][64], b1[64], W2[64][64],
b2[64], W3[64][3], b3[3], row-major.

parity unpinned beyond: gradients by central differences, Adam's first step, the
softmax-CE gradient identities and GELU values (see tests).
"""
from __future__ import annotations

import math

import numpy as np

HID = 64
NOUT = 3
REFINE, KEEP, COARSEN = 0, 1, 2


def n_params(nin: int) -> int:
    return nin * HID + HID + HID * HID + HID + HID * NOUT + NOUT


def unpack(p, nin):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + nin * HID].reshape(nin, HID); o += nin * HID
    b1 = p[o:o + HID]; o += HID
    W2 = p[o:o + HID * HID].reshape(HID, HID); o += HID * HID
    b2 = p[o:o + HID]; o += HID
    W3 = p[o:o + HID * NOUT].reshape(HID, NOUT); o += HID * NOUT
    b3 = p[o:o + NOUT]; o += NOUT
    assert o == len(p)
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])


_erf = np.vectorize(math.erf)


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def pool_features(blocks, bs: int, nf: int, dim: int = 2):
    """blocks: [n][nf][bs^2] synchronised values -> [n][nf*64] bin averages (FP64)."""
    assert dim == 2
    w = (bs - 1) // 8
    n = blocks.shape[0]
    out = np.zeros((n, nf * 64))
    b = blocks.reshape(n, nf, bs, bs)
    for f in range(nf):
        for by in range(8):
            for bx in range(8):
                s = np.zeros(n)
                for y in range(by * w, by * w + w):
                    for x in range(bx * w, bx * w + w):
                        s = s + b[:, f, y, x]
                out[:, f * 64 + by * 8 + bx] = s / (w * w)
    return out


def normalise(x, mean, std, nf):
    x = np.asarray(x, dtype=np.float64).copy()
    for f in range(nf):
        x[:, f * 64:(f + 1) * 64] = (x[:, f * 64:(f + 1) * 64] - mean[f]) / std[f]
    return x


def forward(p, x, nin):
    W1, b1, W2, b2, W3, b3 = unpack(p, nin)
    z1 = x @ W1 + b1
    a1 = gelu(z1)
    z2 = a1 @ W2 + b2
    a2 = gelu(z2)
    z3 = a2 @ W3 + b3
    return z3, (x, z1, a1, z2, a2)


def loss_and_grad(p, x, y, classw, nin):
    """Weighted softmax cross-entropy and its gradient w.r.t. the parameter vector."""
    z3, (x, z1, a1, z2, a2) = forward(p, x, nin)
    y = np.asarray(y, dtype=np.int64)
    zmax = z3.max(axis=1, keepdims=True)
    e = np.exp(z3 - zmax)
    prob = e / e.sum(axis=1, keepdims=True)
    w = np.asarray(classw, dtype=np.float64)[y]
    W = w.sum()
    loss = float(np.sum(w * -np.log(prob[np.arange(len(y)), y])) / W)
    dz3 = prob.copy()
    dz3[np.arange(len(y)), y] -= 1.0
    dz3 = dz3 * (w / W)[:, None]
    W1, b1, W2, b2, W3, b3 = unpack(p, nin)
    dW3 = a2.T @ dz3
    db3 = dz3.sum(axis=0)
    dz2 = (dz3 @ W3.T) * gelu_grad(z2)
    dW2 = a1.T @ dz2
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2.T) * gelu_grad(z1)
    dW1 = x.T @ dz1
    db1 = dz1.sum(axis=0)
    return loss, pack(dW1, db1, dW2, db2, dW3, db3)


class Adam:
    def __init__(self, n, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, p, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return p - self.lr * mh / (np.sqrt(vh) + self.eps)


def horizon_labels(lv_now, co_now, lv_later, co_later, dim=2):
    """Label every block of the grid at step n from the grid H steps later."""
    later = {}
    for l, c in zip(lv_later, co_later):
        later[(int(l),) + tuple(int(v) for v in c)] = True
    jmax = max(int(np.max(lv_now)), int(np.max(lv_later)))
    out = np.zeros(len(lv_now), dtype=np.int8)
    for i, (l, c) in enumerate(zip(lv_now, co_now)):
        l = int(l)
        c = tuple(int(v) for v in c)
        # a coarser block of the later grid containing this one?
        inside_coarser = False
        for L in range(1, l):
            anc = (L,) + tuple(v >> (l - L) for v in c)
            if anc in later:
                inside_coarser = True
        # a finer block of the later grid inside this one?
        finer = False
        for L in range(l + 1, jmax + 1):
            s = L - l
            rng = [range(v << s, (v + 1) << s) for v in c]
            for cc in np.array(np.meshgrid(*rng, indexing="ij")).reshape(dim, -1).T:
                if (L,) + tuple(int(v) for v in cc) in later:
                    finer = True
                    break
            if finer:
                break
        out[i] = REFINE if finer else (COARSEN if inside_coarser else KEEP)
    return out
