"""Oracle for the extraction-threshold model (TEST INFRASTRUCTURE ONLY).

FP64 numpy reference of the 8 -> 64 -> 64 -> 1 GELU network that chooses how
many minima a round pulls, with the same parameter layout as the GPU blob
(W1[8][64], b1[64], W2[64][64], b2[64], w3[64], b3, mu[8], sd[8], scale;
weights input-major).  GELU is the exact x * Phi(x) (Hendrycks & Gimpel 2016);
weights are rounded to bfloat16 (round to nearest even) before use, as on the
GPU.  Also: the zero-waste label of a traced round.
"""
import math

import numpy as np

F, H = 8, 64
PARAMS = F * H + H + H * H + H + H + 1
BLOB = PARAMS + 2 * F + 1


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even)."""
    a = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    a = a + np.uint64(0x7FFF) + ((a >> np.uint64(16)) & np.uint64(1))
    return (a.astype(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32)


def gelu(x):
    erf = np.vectorize(math.erf)
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def unpack(blob):
    b = np.asarray(blob, dtype=np.float64)
    o = 0
    W1 = b[o:o + F * H].reshape(F, H); o += F * H
    b1 = b[o:o + H]; o += H
    W2 = b[o:o + H * H].reshape(H, H); o += H * H
    b2 = b[o:o + H]; o += H
    w3 = b[o:o + H]; o += H
    b3 = b[o]; o += 1
    mu = b[o:o + F]; o += F
    sd = b[o:o + F]; o += F
    return W1, b1, W2, b2, w3, b3, mu, sd, b[o]


def rounded(blob):
    """Blob with its weights (not the normalisation) rounded to bfloat16."""
    out = np.array(blob, dtype=np.float64)
    out[:PARAMS] = bf16_round(np.asarray(blob[:PARAMS], np.float32)).astype(np.float64)
    return out


def forward(blob, X):
    """y for every row of X (n x 8), in float64, with the weights as given."""
    W1, b1, W2, b2, w3, b3, mu, sd, _ = unpack(blob)
    x = (np.asarray(X, np.float64) - mu) / sd
    h1 = gelu(x @ W1 + b1)
    h2 = gelu(h1 @ W2 + b2)
    return h2 @ w3 + b3


def loss(blob, X, Y):
    e = forward(blob, X) - np.asarray(Y, np.float64)
    return float(np.mean(e * e))


def grad_fd(blob, X, Y, eps=1e-6):
    """Central finite differences of the loss with respect to each master
    weight, evaluated at the bfloat16-rounded weights (the GPU treats the
    rounding as identity in its backward pass)."""
    base = rounded(blob)
    g = np.zeros(PARAMS)
    for p in range(PARAMS):
        a = base.copy()
        b = base.copy()
        a[p] += eps
        b[p] -= eps
        g[p] = (loss(a, X, Y) - loss(b, X, Y)) / (2 * eps)
    return g


def zero_waste_label(keys, ids, dist):
    """log2 of the longest prefix of a traced round's keys (in order) that
    already equal their final distances; UINT64_MAX keys end the list."""
    k = 0
    for key, v in zip(keys, ids):
        if key == np.uint64(0xFFFFFFFFFFFFFFFF) or dist[v] != key:
            break
        k += 1
    return math.log2(max(k, 1))
