"""Pins of the float64 prefilter oracle (oracle/mlp.py) against facts that do
not come from the oracle itself: brute-force dipeptide counting, closed-form
networks, central finite differences, Adam's closed forms and bfloat16
rounding of exactly representable cases."""
import re

import numpy as np
import pytest

import seqgen
from oracle import mlp

ALPHA = seqgen.PROTEIN_ALPHABET


def _brute_counts(s: str) -> np.ndarray:
    # count every dipeptide of standard residues by overlapping string search
    std = ALPHA[:20]
    out = np.zeros(400, dtype=np.int64)
    up = s.upper()
    for a in range(20):
        for b in range(20):
            out[20 * a + b] = len(re.findall(f"(?={re.escape(std[a] + std[b])})", up))
    return out


@pytest.mark.parametrize("s", ["", "A", "AA", "AAAA", "ARNDARND", "wYwYw", "AXAB*AZAA", "CCXCC"])
def test_dipeptide_counts_brute(s):
    assert np.array_equal(mlp.dipeptide_counts(s.encode(), ALPHA), _brute_counts(s))


def test_dipeptide_counts_random_and_total():
    rng = np.random.default_rng(3)
    for L in (2, 17, 300):
        s = seqgen.to_str(seqgen.random_protein(rng, L))
        c = mlp.dipeptide_counts(s.encode(), ALPHA)
        assert np.array_equal(c, _brute_counts(s))
        assert c.sum() == L - 1                       # all residues standard
        assert np.isclose(mlp.frequencies(s.encode(), ALPHA).sum(), 1.0)


def test_bad_symbol():
    with pytest.raises(ValueError):
        mlp.dipeptide_counts(b"AR1N", ALPHA)


def test_pair_features_closed_form():
    f = mlp.frequencies(b"ARAR", ALPHA)   # AR twice, RA once
    x = mlp.pair_features(f, 4, f, 9)
    ar, ra = 20 * 0 + 1, 20 * 1 + 0
    assert np.isclose(x[ar], (2 / 3) ** 2) and np.isclose(x[ra], (1 / 3) ** 2)
    assert np.isclose(x[400], np.log(4)) and np.count_nonzero(x[:400]) == 2
    assert mlp.pair_features(f, 0, f, 5)[400] == 0.0


def _zero_params():
    return {n: np.zeros(s) for n, s in mlp.SHAPES}


def test_forward_closed_forms():
    Z = np.zeros((3, 401))
    Z[:, 0] = [-1.3, 0.7, 2.0]
    P = _zero_params()
    P["b3"][0] = 2.5
    assert np.allclose(mlp.forward(P, Z), 2.5)
    # a single path z0 -> relu -> relu -> output: yhat = max(z0, 0)
    P = _zero_params()
    P["W1"][0, 0] = 1.0
    P["W2"][0, 0] = 1.0
    P["w3"][0] = 1.0
    assert np.allclose(mlp.forward(P, Z), [0.0, 0.7, 2.0])
    # biases enter before the ReLU: relu(z0 - 1) then relu(. + 0.5)
    P["b1"][0] = -1.0
    P["b2"][0] = 0.5
    assert np.allclose(mlp.forward(P, Z), [0.5, 0.5, 1.5])


def test_loss_closed_form():
    P = _zero_params()
    P["b3"][0] = 1.0
    Z = np.random.default_rng(0).normal(size=(5, 401))
    y = np.array([0.0, 1.0, 2.0, 3.0, 4.0])
    loss, G = mlp.loss_and_grads(P, Z, y)
    assert np.isclose(loss, np.mean((1.0 - y) ** 2))
    assert np.isclose(G["b3"][0], 2 * np.mean(1.0 - y))
    assert np.allclose(G["W1"], 0) and np.allclose(G["w3"], 0)


def _random_params(rng, scale=1.0):
    P = {}
    for n, s in mlp.SHAPES:
        fan = s[1] if len(s) == 2 else mlp.NH
        P[n] = rng.normal(scale=scale * np.sqrt(2.0 / fan), size=s)
    return P


def test_gradients_central_differences():
    rng = np.random.default_rng(11)
    P = _random_params(rng)
    Z = rng.normal(size=(16, 401))
    y = rng.normal(loc=3.0, size=16)
    _, G = mlp.loss_and_grads(P, Z, y)
    theta = mlp.flatten(P)
    g = mlp.flatten(G)
    h = 1e-6
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in mlp.SHAPES])
    picks = np.concatenate([rng.integers(offs[i], offs[i + 1], size=60) for i in range(len(offs) - 1)])
    num = []
    for i in picks:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        lp, _ = mlp.loss_and_grads(mlp.unflatten(tp), Z, y)
        lm, _ = mlp.loss_and_grads(mlp.unflatten(tm), Z, y)
        num.append((lp - lm) / (2 * h))
    num = np.array(num)
    ana = g[picks]
    rel = np.linalg.norm(num - ana) / np.linalg.norm(ana)
    assert rel < 1e-6, rel


def test_bf16_rounding_exact_cases():
    u = 2.0 ** -7    # unit in the last place of bfloat16 at 1.0
    vals = np.array([1.0, 1 + u / 2, 1 + u + u / 2, 1 + u / 4, -3.0, 0.0, 1 + u * 0.75])
    want = np.array([1.0, 1.0, 1 + 2 * u, 1.0, -3.0, 0.0, 1 + u])
    assert np.array_equal(mlp.bf16(vals), want)


def test_bf16_grads_close_to_float64():
    rng = np.random.default_rng(5)
    P = _random_params(rng)
    Z = rng.normal(size=(64, 401))
    y = rng.normal(loc=3.0, size=64)
    _, G = mlp.loss_and_grads(P, Z, y)
    _, Gb = mlp.loss_and_grads_bf16(P, Z, y)
    a, b = mlp.flatten(G), mlp.flatten(Gb)
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 2e-2


def test_adam_closed_forms():
    rng = np.random.default_rng(2)
    theta = rng.normal(size=50)
    g = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    # first step: the bias corrections cancel, the step is lr * g / (|g| + eps)
    t1, m, v = mlp.adam_step(theta, g, m, v, 1, lr=1e-3)
    assert np.allclose(t1 - theta, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    # a constant gradient keeps the corrected moments at g and g^2: same step every time
    th = t1
    for t in range(2, 7):
        nth, m, v = mlp.adam_step(th, g, m, v, t, lr=1e-3)
        assert np.allclose(nth - th, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-15)
        th = nth


def test_norm_stats_standardise():
    X = np.random.default_rng(1).normal(loc=5, scale=3, size=(500, 401))
    X[:, 7] = 2.0
    mu, sd = mlp.norm_stats(X)
    Zs = (X - mu) / sd
    assert np.allclose(Zs.mean(0), 0, atol=1e-12)
    assert np.allclose(np.delete(Zs.std(0), 7), 1)
    assert sd[7] == 1.0


def test_recall():
    assert mlp.recall_at_k([[1, 2, 3]], [[3, 2, 1]]) == 1.0
    assert mlp.recall_at_k([[1, 2, 9], [4, 5, 6]], [[1, 2, 3], [7, 8, 9]]) == pytest.approx((2 / 3) / 2)


def test_folded_prediction_equals_plain_network():
    rng = np.random.default_rng(21)
    P = _random_params(rng)
    P["b1"] = rng.normal(scale=0.1, size=256)
    q = seqgen.random_protein(rng, 300)
    db = [seqgen.random_protein(rng, L) for L in (2, 30, 300, 1000)] + [q]
    X = np.stack([mlp.pair_features(mlp.frequencies(bytes(q), ALPHA), 300, mlp.frequencies(bytes(d), ALPHA), len(d))
                  for d in db])
    mu, sd = mlp.norm_stats(X)
    sd = sd + 0.5
    a = mlp.predict(P, mu, sd, bytes(q), [bytes(d) for d in db], ALPHA)
    b = mlp.predict_folded(P, mu, sd, bytes(q), [bytes(d) for d in db], ALPHA)
    assert np.allclose(a, b, rtol=0, atol=1e-9)
    c = mlp.predict_folded(P, mu, sd, bytes(q), [bytes(d) for d in db], ALPHA, rnd=mlp.bf16)
    assert np.max(np.abs(c - a)) < 0.1
