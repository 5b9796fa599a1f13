"""The screening oracle against facts: complex-step derivatives of the loss,
closed forms, Adam's first step, and the pair bound against brute force."""
import numpy as np

from oracle import rimp2_oracle as O
from oracle import screen_oracle as S
import pins


def rand_params(seed, scale=0.3):
    return np.random.default_rng(seed).standard_normal(S.NP) * scale


def test_gradient_matches_complex_step():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((9, 4))
    t = rng.standard_normal(9)
    p = rand_params(2)
    _, g = S.loss_grad(x, t, p)
    h = 1e-30
    for q in list(range(0, S.NP, 37)) + [S.NP - 1, S.NP - 2, 255, 256]:
        pc = p.astype(np.complex128)
        pc[q] += 1j * h
        d = S.loss(x, t, pc).imag / h
        assert abs(d - g[q]) <= 1e-12 * max(1.0, abs(d)), (q, d, g[q])


def test_zero_weights_closed_form():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((5, 4))
    t = rng.standard_normal(5)
    p = np.zeros(S.NP)
    p[-1] = 0.7
    assert np.allclose(S.forward(x, p), 0.7)
    L, g = S.loss_grad(x, t, p)
    assert abs(L - np.mean((0.7 - t) ** 2)) < 1e-15
    assert abs(g[-1] - 2 * np.mean(0.7 - t)) < 1e-15
    assert np.all(g[:-1 - S.H] == 0)   # everything before W3 gets no gradient through zero weights


def test_adam_first_step():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 0.0])
    p1, m, v = S.adam(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    # step 1: m_hat = g, v_hat = g^2, so the move is -lr g / (|g| + eps)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8))


def test_bound_holds_for_every_pair():
    for seed in range(3):
        B, eo, ev = pins.tiny_inputs(5, 6, 7, 200 + seed)
        e = O.fragment(B, eo, ev, gamma=False, density=False)["e_pair"]
        bd = S.pair_bound(B, eo, ev)
        assert np.all(np.abs(e) <= bd * (1 + 1e-12))


def test_features_definition():
    B, eo, ev = pins.tiny_inputs(3, 4, 5, 7)
    r = np.array([[0.0, 0, 0], [3.0, 4.0, 0], [0, 0, 1.0]])
    f = S.pair_features(B, eo, r).reshape(3, 3, 4)
    assert abs(f[0, 1, 0] - 0.5) < 1e-15 and abs(f[1, 0, 0] - 0.5) < 1e-15
    assert abs(np.exp(f[1, 2, 1]) - np.linalg.norm(B[1])) < 1e-13
    assert abs(f[2, 0, 3] - (eo[2] + eo[0]) / 10) < 1e-15
