"""Float64 reference of the learned prefilter -- TEST INFRASTRUCTURE ONLY.

Only ``tests/`` and the ``cpu_baseline`` leg of ``bench.py`` may use it.

The prefilter ranks database sequences for a query by a predicted
Smith-Waterman score, then rescores the best-ranked fraction exactly (the
method's learned growth; the paper itself only runs the exhaustive search,
Background "database similarity search").  Definitions, in plain numpy:

* Dipeptide counts of a sequence: c[20 a + b] = number of positions i with
  (code(s_i), code(s_i+1)) = (a, b), over the 20 standard residues (codes
  0..19 of the protein alphabet); a pair that involves any other symbol
  (B, Z, X, *) is not counted.  Frequencies f = c / (L - 1) for L >= 2, else 0.
* Pair features x[k] = f_q[k] * f_t[k] for k < 400 and
  x[400] = ln(max(1, min(L_q, L_t))); normalised z = (x - mu) / sigma with the
  training set's per-feature mean and population standard deviation
  (sigma = 1 where the deviation is 0).
* Network 401 -> 256 (ReLU) -> 256 (ReLU) -> 1:
      h1 = relu(W1 z + b1), h2 = relu(W2 h1 + b2), yhat = w3 . h2 + b3.
* Target y = ln(1 + S), loss = mean over the batch of (yhat - y)^2.
* Adam (Kingma & Ba, 2015) with bias correction:
      m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
      theta -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

``loss_and_grads_bf16`` is the same computation with the operands of the
matrix products rounded to bfloat16 (round to nearest, ties to even) where a
bfloat16 GEMM takes them; products and sums stay in float64.
"""
from __future__ import annotations

import numpy as np

NSTD = 20          # standard residues
NDIP = NSTD * NSTD
NIN = NDIP + 1     # 400 dipeptide products + log length
NH = 256

SHAPES = [("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("w3", (NH,)), ("b3", (1,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


# ------------------------------------------------------------------ features

def codes(seq, alphabet: str) -> np.ndarray:
    """Symbol codes of a sequence (ASCII bytes), case-insensitive."""
    lut = np.full(256, -1, dtype=np.int64)
    for k, ch in enumerate(alphabet):
        lut[ord(ch.upper())] = k
        lut[ord(ch.lower())] = k
    b = np.frombuffer(bytes(seq), dtype=np.uint8)
    c = lut[b]
    if (c < 0).any():
        raise ValueError(f"symbol at position {int(np.argmax(c < 0))} is not in the alphabet")
    return c


def dipeptide_counts(seq, alphabet: str) -> np.ndarray:
    c = codes(seq, alphabet)
    if len(c) < 2:
        return np.zeros(NDIP, dtype=np.int64)
    a, b = c[:-1], c[1:]
    ok = (a < NSTD) & (b < NSTD)
    return np.bincount(NSTD * a[ok] + b[ok], minlength=NDIP).astype(np.int64)


def frequencies(seq, alphabet: str) -> np.ndarray:
    L = len(bytes(seq))
    if L < 2:
        return np.zeros(NDIP)
    return dipeptide_counts(seq, alphabet) / float(L - 1)


def pair_features(fq: np.ndarray, Lq: int, ft: np.ndarray, Lt: int) -> np.ndarray:
    x = np.empty(NIN)
    x[:NDIP] = fq * ft
    x[NDIP] = np.log(max(1, min(int(Lq), int(Lt))))
    return x


def norm_stats(X: np.ndarray):
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    sd = np.where(sd > 0, sd, 1.0)
    return mu, sd


# ------------------------------------------------------------------ network

def unflatten(theta: np.ndarray) -> dict:
    P, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        P[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return P


def flatten(P: dict) -> np.ndarray:
    return np.concatenate([np.asarray(P[n], dtype=np.float64).ravel() for n, _ in SHAPES])


def relu(x):
    return np.maximum(x, 0.0)


def forward(P: dict, Z: np.ndarray) -> np.ndarray:
    h1 = relu(Z @ P["W1"].T + P["b1"])
    h2 = relu(h1 @ P["W2"].T + P["b2"])
    return h2 @ P["w3"] + P["b3"][0]


def loss_and_grads(P: dict, Z: np.ndarray, y: np.ndarray):
    """MSE loss and its gradient with respect to every parameter (float64)."""
    B = Z.shape[0]
    z1 = Z @ P["W1"].T + P["b1"]
    h1 = relu(z1)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = relu(z2)
    yhat = h2 @ P["w3"] + P["b3"][0]
    r = yhat - y
    loss = float(np.mean(r * r))
    d = 2.0 * r / B
    G = {"w3": h2.T @ d, "b3": np.array([d.sum()])}
    dz2 = np.outer(d, P["w3"]) * (z2 > 0)
    G["W2"] = dz2.T @ h1
    G["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ P["W2"]) * (z1 > 0)
    G["W1"] = dz1.T @ Z
    G["b1"] = dz1.sum(axis=0)
    return loss, G


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even), returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def loss_and_grads_bf16(P: dict, Z: np.ndarray, y: np.ndarray):
    """As loss_and_grads with bfloat16 operands in the five matrix products:
    Z, W1 (layer 1), h1, W2 (layer 2), dz2 and W2 (backward to h1), dz2 and
    h1 (dW2), dz1 and Z (dW1).  Layer 3, the loss and the bias sums use the
    float values."""
    B = Z.shape[0]
    Zb, W1b, W2b = bf16(Z), bf16(P["W1"]), bf16(P["W2"])
    z1 = Zb @ W1b.T + P["b1"]
    h1 = bf16(relu(z1))
    z2 = h1 @ W2b.T + P["b2"]
    h2 = relu(z2)
    yhat = h2 @ P["w3"] + P["b3"][0]
    r = yhat - y
    loss = float(np.mean(r * r))
    d = 2.0 * r / B
    G = {"w3": h2.T @ d, "b3": np.array([d.sum()])}
    dz2 = np.outer(d, P["w3"]) * (z2 > 0)
    G["b2"] = dz2.sum(axis=0)
    dz2b = bf16(dz2)
    G["W2"] = dz2b.T @ h1
    dz1 = (dz2b @ W2b) * (h1 > 0)
    G["b1"] = dz1.sum(axis=0)
    G["W1"] = bf16(dz1).T @ Zb
    return loss, G


def adam_step(theta: np.ndarray, g: np.ndarray, m: np.ndarray, v: np.ndarray, t: int,
              lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step (t counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------------ search

def predict(P: dict, mu: np.ndarray, sd: np.ndarray, query, db_seqs, alphabet: str) -> np.ndarray:
    """Predicted ln(1 + S) of query against every database sequence (plain, unfolded)."""
    fq = frequencies(query, alphabet)
    Lq = len(bytes(query))
    X = np.stack([pair_features(fq, Lq, frequencies(d, alphabet), len(bytes(d))) for d in db_seqs])
    return forward(P, (X - mu) / sd)


def predict_folded(P: dict, mu: np.ndarray, sd: np.ndarray, query, db_seqs, alphabet: str, rnd=None):
    """The same predictions through the query-folded first layer:
        W1 z = (W1 diag(f_q / sd)) f_t + (b1 - W1 (mu / sd)) + W1[:, 400] z_400
    (exact algebra).  rnd, when given (for example bf16), rounds the operands
    of the two matrix products: the folded weights, the database
    frequencies, the hidden activations and W2."""
    r = rnd if rnd is not None else (lambda a: np.asarray(a, dtype=np.float64))
    fq = frequencies(query, alphabet)
    Lq = len(bytes(query))
    W1 = P["W1"]
    A = r(W1[:, :NDIP] * (fq / sd[:NDIP])[None, :])
    c = P["b1"] - W1[:, :NDIP] @ (mu[:NDIP] / sd[:NDIP])
    w1x = W1[:, NDIP] / sd[NDIP]
    F = r(np.stack([frequencies(d, alphabet) for d in db_seqs]))
    z400 = np.array([(np.log(max(1, min(Lq, len(bytes(d))))) - mu[NDIP]) for d in db_seqs])
    h1 = r(relu(F @ A.T + c + np.outer(z400, w1x)))
    h2 = relu(h1 @ r(P["W2"]).T + P["b2"])
    return h2 @ P["w3"] + P["b3"][0]


def recall_at_k(found_idx, true_idx) -> float:
    """|found top-k  intersect  true top-k| / k, averaged over queries."""
    found_idx = np.asarray(found_idx)
    true_idx = np.asarray(true_idx)
    k = true_idx.shape[1]
    return float(np.mean([len(set(a[a >= 0]) & set(b[b >= 0])) / k for a, b in zip(found_idx, true_idx)]))
