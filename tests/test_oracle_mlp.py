"""Pins for the float64 network reference: finite differences, softmax, GELU closed form,
BF16 rounding against its definition."""

import math

import numpy as np

import seeded_inputs
from oracle import mlp


def small_params(seed=3):
    return seeded_inputs.mlp_init(12, 8, 3, 5, seed)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    params = {k: v.astype(np.float64) for k, v in small_params().items()}
    for k in params:
        if k.startswith("b"):
            params[k] = rng.normal(size=params[k].shape) * 0.1
    x = rng.normal(size=(6, 12))
    y = rng.integers(0, 5, 6)
    grads = mlp.gradients(params, x, y, depth=3)
    eps = 1e-6
    for name in params:
        flat = params[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp = mlp.loss(params, x, y, 3)
            flat[idx] = old - eps
            lm = mlp.loss(params, x, y, 3)
            flat[idx] = old
            num = (lp - lm) / (2 * eps)
            assert abs(num - grads[name].reshape(-1)[idx]) < 1e-7 + 1e-5 * abs(num), (name, idx)


def test_gelu_closed_form_values():
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    # gelu(x) - gelu(-x) = x (since erf is odd)
    for v in (0.3, 1.7, 4.0):
        assert abs(mlp.gelu(np.array([v]))[0] - mlp.gelu(np.array([-v]))[0] - v) < 1e-12
    # gelu'(0) = 1/2
    assert abs(mlp.gelu_grad(np.array([0.0]))[0] - 0.5) < 1e-15


def test_softmax_rows_sum_to_one():
    rng = np.random.default_rng(1)
    p = mlp.softmax(rng.normal(size=(7, 11)) * 5)
    assert np.allclose(p.sum(axis=1), 1.0)


def test_bf16_rounding_definition():
    # bfloat16 keeps the top 16 bits of a float32; ties go to the even 16-bit pattern
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, 3.14159, -2.5e-3], dtype=np.float32)
    r = mlp.bf16_round(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                     # halfway between 1 and 1 + 2^-7: ties to even (1.0)
    assert r[2] == np.float32(1.0 + 2 ** -6)  # halfway, rounds up to the even pattern
    assert r[3] == 1.0
    for v, w in zip(vals, r):
        assert abs(float(w) - float(v)) <= abs(float(v)) * 2 ** -8


def test_init_is_seeded_and_bounded():
    a = seeded_inputs.mlp_init(4096, 512, 3, 11, 42)
    b = seeded_inputs.mlp_init(4096, 512, 3, 11, 42)
    assert all(np.array_equal(a[k], b[k]) for k in a)
    assert np.abs(a["W0"]).max() <= 1 / math.sqrt(4096)
    assert abs(float(a["W1"].mean())) < 1e-3
    assert sum(v.size for v in a.values()) == 4096 * 512 + 512 + 2 * (512 * 512 + 512) + 512 * 11 + 11


def _float_rows(m):
    """Rows of the exact channel rep (A + B sqrt2) / sqrt2^e in float64, computed directly."""
    a = np.array(m.A, dtype=np.float64)
    b = np.array(m.B, dtype=np.float64)
    return (a + b * math.sqrt(2.0)) / math.sqrt(2.0) ** m.e


def test_features_pins():
    """The canonical features: invariant under left Cliffords; as a 4^n x 4^n matrix orthogonal up to
    float32 rounding (a signed row permutation of an orthogonal matrix); each row equal, up to sign,
    to a row of the target evaluated directly; the identity gives a permutation matrix."""
    from oracle import zmat
    for n, k, seed in ((1, 4, 1), (2, 5, 2), (3, 4, 3)):
        tw = seeded_inputs.target_words(n, k, seed)
        u = zmat.target_from_words(n, tw.paulis, tw.clifford)
        f = mlp.features(u)
        d = zmat.clifford_from_word(n, seeded_inputs.random_clifford_word(n, 40 + seed))
        assert np.array_equal(f, mlp.features(d @ u))
        r = 4 ** n
        fm = f.astype(np.float64).reshape(r, r)
        assert np.allclose(fm @ fm.T, np.eye(r), atol=1e-5)
        rows = _float_rows(u)
        for i in range(r):
            assert min(np.abs(rows - s * fm[i]).max(axis=1).min() for s in (1, -1)) < 1e-6
    ident = mlp.features(zmat.ZMat.identity(2)).reshape(16, 16)
    assert sorted(ident.sum(axis=0).tolist()) == [1.0] * 16 and set(np.unique(ident)) == {0.0, 1.0}
