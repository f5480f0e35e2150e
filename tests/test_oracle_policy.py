"""Oracle pins for the policy-in-the-loop step: BF16 rounding, the two-layer
perceptron and the Gumbel-max draw.

References: torch's own float32 -> bfloat16 conversion; numpy FP64 matrix
products on the decoded BF16 operands; the Gumbel-max property that
argmax(z + Gumbel) is distributed as softmax(z).
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


def test_gumbel_argmax_is_softmax_sampling(oracle_lib):
    """With W1 = 0 the logits are the bias b2; the chosen levels must then follow
    softmax(b2) per port (Gumbel-max)."""
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
