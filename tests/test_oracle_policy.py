"""Oracle pins for the policy-in-the-loop step: BF16 rounding, the two-layer
perceptron and the level draw.

References: torch's own float32 -> bfloat16 conversion; numpy FP64 matrix
products on the decoded BF16 operands; level frequencies against softmax(z)
(chi-square); the inverse-distribution rule on a two-level case worked by hand
from the Philox word (itself pinned by the known-answer vectors).
"""
import math

import numpy as np
import torch
from scipy import stats

import workloads as W


def bf16_to_f64(bits):
    return (np.asarray(bits, np.uint32) << 16).view(np.float32).astype(np.float64)


def test_bf16_rounding_matches_torch(oracle_lib):
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 4000), rng.normal(0, 1e-3, 1000), [0.0, 1.0, -2.5, 1 + 2**-8]])
    x = x.astype(np.float32).astype(np.float64)          # float32-exact inputs: no double rounding
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([oracle_lib.bf16_round(v) for v in x])
    assert np.array_equal(got, ref)
    bits = W.bf16_bits(x)
    assert np.array_equal(bf16_to_f64(bits), ref)


def test_mlp_logits_match_numpy(oracle_lib):
    o = oracle_lib
    spec = W.policy_station()
    c = o.OracleClass(spec)
    H = 64
    weights = W.policy_weights(spec.n_ports, hidden=H, std=0.2, seed=3)
    w1, b1, w2, b2 = [bf16_to_f64(w) for w in weights]
    rng = np.random.default_rng(4)
    for trial in range(5):
        obs = rng.uniform(-1, 1, spec.obs_dim).astype(np.float32).astype(np.float64)
        logits, k = c.policy(H, weights, obs, 9, trial, 3)
        x = torch.tensor(obs, dtype=torch.float32).to(torch.bfloat16).double().numpy()
        h = np.tanh(x @ w1.reshape(spec.obs_dim, H) + b1)
        hb = torch.tensor(h, dtype=torch.float32).to(torch.bfloat16).double().numpy()
        ref = hb @ w2.reshape(H, -1) + b2
        bound = 2.0**-8 * (np.abs(w2.reshape(H, -1)).sum(axis=0)) + 1e-12
        assert np.all(np.abs(logits - ref) <= bound)
        assert np.all((k >= 0) & (k <= 10))


def test_levels_follow_softmax(oracle_lib):
    """With W1 = 0 the logits are the bias b2; the chosen levels must then follow
    softmax(b2) per port."""
    o = oracle_lib
    spec = W.splitter_tree(1, 4, 1000.0, 1000.0)
    c = o.OracleClass(spec)
    H = 8
    L1 = spec.n_levels + 1
    w1 = np.zeros((spec.obs_dim, H), np.uint16)
    b1 = np.zeros(H, np.uint16)
    w2 = np.zeros((H, spec.n_ports * L1), np.uint16)
    z = np.linspace(-1.5, 1.5, L1)
    b2 = W.bf16_bits(np.tile(z, spec.n_ports))
    zb = bf16_to_f64(b2)[:L1]
    p = np.exp(zb - zb.max())
    p /= p.sum()
    obs = np.zeros(spec.obs_dim)
    counts = np.zeros((spec.n_ports, L1))
    n = 6000
    for i in range(n):
        _, k = c.policy(H, (w1, b1, w2, b2), obs, 12, i % 50, i // 50)
        counts[np.arange(spec.n_ports), k] += 1
    for port in range(spec.n_ports):
        chi = ((counts[port] - n * p) ** 2 / (n * p)).sum()
        assert stats.chi2.sf(chi, L1 - 1) > 1e-4, (port, counts[port], n * p)


def test_tiny_perceptron_hand_worked(oracle_lib):
    """Two ports, levels {0, 1}, two hidden units, every operand a BF16 value,
    worked by hand (pins the weight layouts, where tanh and the two BF16
    roundings sit, and which logit belongs to which port and level):

      obs x = (0.5, 0.25, 0.3, 0, ...); 0.3 rounds to BF16 0.30078125
      W1 [feature][hidden]: W1[0][0] = 1, W1[1][0] = 2, W1[0][1] = -2, W1[2][1] = 4;
      b1 = (0, 0.25)
        a0 = 0.5 + 0.5 = 1                    h0 = bf16(tanh 1)        = 0.76171875
        a1 = -1 + 4 * 0.30078125 + 0.25 = 0.453125
                                              h1 = bf16(tanh 0.453125) = 0.423828125
        (no rounding of x would give a1 = 0.45, h1 = 0.421875)
      W2 [hidden][port * 2 + level] = ((2, -1, 0.5, 0), (0.5, 4, 0, -3)); b2 = (0, 64, 64, -1)
        z = (2 h0 + 0.5 h1, 64 - h0 + 4 h1, 64 + 0.5 h0, -1 - 3 h1)
          = (1.7353515625, 64.93359375, 64.380859375, -2.271484375)
    Softmax gives port 0's level 1 and port 1's level 0 all but e^-60 of the
    probability, so those are the levels drawn."""
    o = oracle_lib
    spec = W.single_transformer(2, 1000.0).replace(n_levels=1)
    assert spec.obs_dim == 16
    c = o.OracleClass(spec)
    H = 2
    w1 = np.zeros((16, H))
    w1[0, 0], w1[1, 0], w1[0, 1], w1[2, 1] = 1.0, 2.0, -2.0, 4.0
    b1 = np.array([0.0, 0.25])
    w2 = np.array([[2.0, -1.0, 0.5, 0.0], [0.5, 4.0, 0.0, -3.0]])
    b2 = np.array([0.0, 64.0, 64.0, -1.0])
    weights = tuple(W.bf16_bits(a.ravel()) for a in (w1, b1, w2, b2))
    obs = np.zeros(16)
    obs[:3] = (0.5, 0.25, 0.3)
    for env, g in ((0, 0), (5, 123), (77, 9999)):
        logits, k = c.policy(H, weights, obs, 21, env, g)
        assert list(logits) == [1.7353515625, 64.93359375, 64.380859375, -2.271484375]
        assert list(k) == [1, 0]


def test_inverse_distribution_two_levels(oracle_lib):
    """Levels {0, 1} with logits (0, ln 3) (bias only): p = (1/4, 3/4), so the
    level is 0 exactly when u < 1/4, u = (top 24 bits of word (port / 16) mod 4
    of Philox (env, g, port mod 16 + 16 (port / 64), 3) + 1/2) 2^-24 -- ports 16
    apart share a call; the margin is |1/4 - u|.  40 ports: words 0, 1 and 2."""
    o = oracle_lib
    n_ports = 40
    spec = W.single_transformer(n_ports, 1000.0).replace(n_levels=1)
    c = o.OracleClass(spec)
    H = 2
    w1 = np.zeros((spec.obs_dim, H), np.uint16)
    b1 = np.zeros(H, np.uint16)
    w2 = np.zeros((H, 2 * n_ports), np.uint16)
    b2 = np.zeros(2 * n_ports)
    b2[1::2] = math.log(3.0)
    b2bits = W.bf16_bits(b2)
    z1 = bf16_to_f64(b2bits)[1]            # ln 3 rounded to BF16
    p0 = 1.0 / (1.0 + math.exp(z1))
    seed = 0x1234_5678_9ABC
    zeros = 0
    for env, g in [(e, t) for e in range(0, 40, 3) for t in range(0, 500, 37)]:
        _, k, margin = c.policy(H, (w1, b1, w2, b2bits), np.zeros(spec.obs_dim), seed, env, g, with_margin=True)
        for port in range(n_ports):
            w = o.philox([env, g, port % 16 + 16 * (port // 64), 3], [seed & 0xFFFFFFFF, seed >> 32])
            u = ((int(w[(port // 16) % 4]) >> 8) + 0.5) * 2.0**-24
            assert k[port] == (0 if u < p0 else 1), (env, g, port, u, k[port])
            assert abs(margin[port] - abs(p0 - u)) < 1e-12
            zeros += k[port] == 0
    assert 0.2 < zeros / (n_ports * 14 * 14) < 0.3
