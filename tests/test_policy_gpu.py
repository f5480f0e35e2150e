"""GPU parity of the policy-in-the-loop rollout, teacher-forced against the oracle:

* logits of the BF16 matrix-core MLP equal the oracle's FP64 products on the same
  BF16 operands, within the bound of one BF16 rounding flip per hidden unit;
* every sampled level equals the oracle's draw on the oracle's own observation,
  except where the uniform of the draw lies within 1e-3 of a boundary of the
  softmax distribution function (such flips are counted and must stay rare);
* the environment, replayed in the oracle on the GPU's levels, matches exactly
  (integers) and within the FP tolerances (rewards, observations).
"""
import numpy as np
import pytest
import torch

import workloads as W
from tests import parity as PY

pytestmark = pytest.mark.gpu

TIE = 1e-3
H = 256


@pytest.fixture(scope="module")
def cxm():
    from paper_2507_01522_amd import cx
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    return cx


def bf16_f64(bits):
    return (np.asarray(bits, np.uint32) << 16).view(np.float32).astype(np.float64)


def hidden_abs(weights, x, hidden):
    """|h| of the oracle's hidden layer (numpy), used only to size the tolerance."""
    w1, b1 = bf16_f64(weights[0]).reshape(-1, hidden), bf16_f64(weights[1])
    xb = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).double().numpy()
    return np.abs(np.tanh(xb @ w1 + b1))


def check_levels(o, spec, weights, obs_in, levels, seed, env_ids, g0, hidden=H):
    """obs_in [T][E][obs_dim] (oracle), levels [T][E][N] (GPU). Returns flip count."""
    c = o.OracleClass(spec)
    T, E = levels.shape[:2]
    flips = 0
    for t in range(T):
        for e in range(E):
            _, k, margin = c.policy(hidden, weights, obs_in[t, e], seed, int(env_ids[e]), g0 + t, with_margin=True)
            bad = levels[t, e] != k
            if bad.any():
                assert np.all(margin[bad] < TIE), (
                    f"step {t} env {env_ids[e]}: levels {levels[t, e][bad]} vs oracle {k[bad]}, "
                    f"margins {margin[bad]}")
                flips += int(bad.sum())
    return flips


def teacher_forced(o, spec, weights, seed, gout, env_ids, T, g0=0, start=None, hidden=H):
    """Replay the GPU's levels in the oracle and check rewards, done flags and
    every level against the oracle's policy on the oracle's observations."""
    E, N, dim = len(env_ids), spec.n_ports, spec.obs_dim
    c = o.OracleClass(spec)
    bs = o.BatchState([c], np.zeros(E, np.int32), env_ids=env_ids)
    if start is not None:
        start(bs)
    obs0 = np.stack([c.observe(_env_state(bs, e, N)) for e in range(E)])
    act = gout["actions"]
    ref = o.rollout(bs, seed, T, mode=0, act_in=act, want_obs=True)
    PY.compare_rollout({"actions": act, "reward": gout["reward"], "done": gout["done"]}, ref, [spec],
                       np.zeros(E, np.int32), check_obs=False)
    obs_in = np.concatenate([obs0[None], ref["obs"][:-1].reshape(T - 1, E, dim)]) if T > 1 else obs0[None]
    flips = check_levels(o, spec, weights, obs_in, act.reshape(T, E, N), seed, env_ids, g0, hidden)
    assert flips <= max(2, T * E * N // 2000), f"{flips} near-tie flips"
    return ref, bs


def _env_state(bs, e, N):
    class S:
        pass
    s = S()
    sl = slice(e * N, (e + 1) * N)
    s.dwell = np.ascontiguousarray(bs.dwell[sl])
    s.soc = np.ascontiguousarray(bs.soc[sl])
    s.e_rem = np.ascontiguousarray(bs.e_rem[sl])
    s.cap = np.ascontiguousarray(bs.cap[sl])
    s.p_last = np.ascontiguousarray(bs.p_last[sl])
    s.batt = np.ascontiguousarray(bs.batt[2 * e:2 * e + 2])
    s.user = np.ascontiguousarray(bs.user[sl])
    s.t_day = bs.t_day
    return s


def test_policy_logits_match_oracle(cxm, oracle_lib):
    """197 observations (rollout records and uniform noise, a ragged last tile)."""
    spec = W.policy_station()
    weights = W.policy_weights(spec.n_ports, hidden=H, std=0.2, seed=7)
    env = cxm.Env(spec, n_envs=8, seed=5)
    env.set_policy(H, weights)
    rec = env.rollout(4, cxm.ACT_RANDOM)["obs"].reshape(-1, spec.obs_dim)
    rng = np.random.default_rng(1)
    noise = torch.from_numpy(rng.uniform(-1.5, 1.5, (165, spec.obs_dim)).astype(np.float32)).cuda()
    obs = torch.cat([rec, noise]).contiguous()
    z = env.policy_logits(obs).cpu().numpy().astype(np.float64)
    x = obs.cpu().numpy().astype(np.float64)
    c = oracle_lib.OracleClass(spec)
    ref = np.stack([c.policy(H, weights, x[i], 5, 0, 0)[0] for i in range(len(x))])
    w2 = np.abs(bf16_f64(weights[2]).reshape(H, -1))
    s = hidden_abs(weights, x, H) @ w2                     # sum_j |h_j w2_jo| per row
    bound = 2.0**-7 * s + 1e-5 * (s + np.abs(bf16_f64(weights[3]))) + 1e-6
    err = np.abs(z - ref)
    assert np.all(err <= bound), f"worst {np.max(err / bound):.3g} x bound"
    # rounding flips are rare: typical errors sit at the FP32 accumulation level
    assert np.median(err / (s + 1e-12)) < 1e-5


@pytest.mark.parametrize("out_mode", ["act_reward", "full"])
def test_policy_rollout_teacher_forced(cxm, oracle_lib, out_mode):
    """40 envs x 300 steps (the day boundary at 288), levels from the MLP."""
    spec = W.policy_station()
    weights = W.policy_weights(spec.n_ports, hidden=H, std=0.2, seed=11)
    E, T, seed = 40, 300, 21
    env = cxm.Env(spec, n_envs=E, seed=seed)
    env.set_policy(H, weights)
    om = cxm.OUT_FULL if out_mode == "full" else cxm.OUT_ACT_REWARD
    g = PY.to_np(env.rollout(T, cxm.ACT_POLICY, om))
    ref, bs = teacher_forced(oracle_lib, spec, weights, seed, g, np.arange(E), T)
    if out_mode == "full":
        PY.compare_obs(g["obs"], ref["obs"], [spec], np.zeros(E, np.int32))
    PY.compare_state(env.state_arrays(), bs, [spec], np.zeros(E, np.int32))
    assert g["done"][287].all() and g["done"].sum() == E
    assert len(np.unique(g["actions"])) == spec.n_levels + 1


POLICY_CLASSES = {
    # 8 and 16 ports on aligned splitters (SIMPLE, 8 and 16 slots): the fused rollout with 1 and
    # 2 slots per lane; 40 ports under one transformer (padded to 64 slots): two kernels per step
    "split2x4": (lambda: W.splitter_tree(2, 4, 60.0, 120.0), 64, 4),
    "fan16": (lambda: W.fanout4_tree(16, 2), 96, 10),
    "flat40": (lambda: W.single_transformer(40, 600.0), 256, 7),
}


@pytest.mark.parametrize("name", list(POLICY_CLASSES))
def test_policy_classes_teacher_forced(cxm, oracle_lib, name):
    """Other station sizes, hidden sizes and level counts (hidden 64 and 96:
    padded hidden tiles; 5 and 8 levels: a padded level tile): 37 envs (a
    ragged last block) x 300 steps replayed in the oracle, and every record
    and the final state equal to the rollout that allocates nothing (two
    kernels per step), bit for bit."""
    make_spec, hidden, n_levels = POLICY_CLASSES[name]
    spec = make_spec().replace(n_levels=n_levels)
    weights = W.policy_weights(spec.n_ports, hidden=hidden, n_levels=n_levels, std=0.2, seed=31)
    E, T, seed = 37, 300, 17
    envs = []
    for _ in range(2):
        e = cxm.Env(spec, n_envs=E, seed=seed)
        e.set_policy(hidden, weights)
        envs.append(e)
    g = PY.to_np(envs[0].rollout(T, cxm.ACT_POLICY, cxm.OUT_FULL))
    ref, bs = teacher_forced(oracle_lib, spec, weights, seed, g, np.arange(E), T, hidden=hidden)
    PY.compare_obs(g["obs"], ref["obs"], [spec], np.zeros(E, np.int32))
    PY.compare_state(envs[0].state_arrays(), bs, [spec], np.zeros(E, np.int32))
    b = PY.to_np(envs[1].rollout_policy_noalloc(T, cxm.OUT_FULL))
    for k in g:
        assert np.array_equal(g[k], b[k]), k
    assert envs[0].get_state() == envs[1].get_state()


def test_policy_modes_agree_and_split(cxm):
    """FULL and ACT_REWARD give the same levels and rewards; 100 + 200 steps
    equal 300; three one-step calls equal a 3-step rollout."""
    spec = W.policy_station()
    weights = W.policy_weights(spec.n_ports, hidden=H, std=0.2, seed=11)
    E, seed = 70, 4

    def make():
        e = cxm.Env(spec, n_envs=E, seed=seed)
        e.set_policy(H, weights)
        return e

    a = PY.to_np(make().rollout(300, cxm.ACT_POLICY, cxm.OUT_FULL))
    b = PY.to_np(make().rollout(300, cxm.ACT_POLICY, cxm.OUT_ACT_REWARD))
    for k in ("actions", "reward", "done"):
        assert np.array_equal(a[k], b[k]), k
    env = make()
    c1 = PY.to_np(env.rollout(100, cxm.ACT_POLICY, cxm.OUT_FULL))
    c2 = PY.to_np(env.rollout(200, cxm.ACT_POLICY, cxm.OUT_FULL))
    for k in a:
        assert np.array_equal(a[k], np.concatenate([c1[k], c2[k]])), k
    env = make()
    steps = [PY.to_np(env.step(cxm.ACT_POLICY)) for _ in range(3)]
    for k in a:
        assert np.array_equal(a[k][:3], np.concatenate([s[k] for s in steps])), k


def test_policy_after_random_start(cxm, oracle_lib):
    """The policy starts from a state reached by 150 random steps (occupied
    ports, mid-day): the start observation comes from the observation kernel."""
    spec = W.policy_station()
    weights = W.policy_weights(spec.n_ports, hidden=H, std=0.2, seed=12)
    E, seed = 33, 8
    env = cxm.Env(spec, n_envs=E, seed=seed)
    env.set_policy(H, weights)
    env.rollout(150, cxm.ACT_RANDOM, cxm.OUT_REWARD)
    g = PY.to_np(env.rollout(20, cxm.ACT_POLICY, cxm.OUT_ACT_REWARD))

    def start(bs):
        oracle_lib.rollout(bs, seed, 150, want_obs=False, want_act=False)

    teacher_forced(oracle_lib, spec, weights, seed, g, np.arange(E), 20, g0=150, start=start)


def test_observe_equals_last_record(cxm):
    """cx_observe of the state after a rollout equals the rollout's last
    observation record bit for bit (uneven classes, padded trees)."""
    specs = W.mixture_classes()[:6]
    ec = np.repeat(np.arange(6), 9).astype(np.int32)
    env = cxm.Env(specs, env_class=ec, seed=3)
    out = env.rollout(37, cxm.ACT_RANDOM, cxm.OUT_FULL)
    assert torch.equal(env.observe(), out["obs"][-1])
    env.reset()
    z = torch.empty_like(out["obs"][0])
    env.reset(z)
    assert torch.equal(env.observe(), z)


def test_policy_full_size_sampled(cxm, oracle_lib):
    """1,048,576 stations of 32 ports, 8 steps in the production launch shape;
    64 sampled stations replayed in the oracle."""
    spec = W.policy_station()
    weights = W.policy_weights(spec.n_ports, hidden=H, std=0.2, seed=13)
    E, T, seed = 1 << 20, 8, 5
    env = cxm.Env(spec, n_envs=E, seed=seed)
    env.set_policy(H, weights)
    out = env.rollout(T, cxm.ACT_POLICY, cxm.OUT_ACT_REWARD)
    rng = np.random.default_rng(3)
    ids = np.sort(np.concatenate([rng.choice(E, 62, replace=False), [0, E - 1]]))
    ids = np.unique(ids)
    N = spec.n_ports
    cols = (ids[:, None] * N + np.arange(N)).ravel()
    g = {"actions": out["actions"][:, torch.from_numpy(cols).cuda()].cpu().numpy(),
         "reward": out["reward"][:, torch.from_numpy(ids).cuda()].cpu().numpy(),
         "done": out["done"][:, torch.from_numpy(ids).cuda()].cpu().numpy()}
    teacher_forced(oracle_lib, spec, weights, seed, g, ids, T)


def test_policy_across_segments(cxm, oracle_lib):
    """5,600,000 stations of 32 ports: one step's observations pass 4 GiB, so
    the fused rollout runs the class as two segments; stations on both sides
    of the cut, at block edges and at the ends replayed in the oracle."""
    spec = W.policy_station()
    weights = W.policy_weights(spec.n_ports, hidden=H, std=0.2, seed=14)
    n, T, seed = 5_600_000, 3, 19
    chunk = ((1 << 32) - 1) // (4 * spec.obs_dim)
    chunk -= chunk % 64
    assert chunk < n
    env = cxm.Env(spec, n_envs=n, seed=seed)
    env.set_policy(H, weights)
    out = env.rollout(T, cxm.ACT_POLICY, cxm.OUT_ACT_REWARD)
    ids = np.array([0, 1, 31, 32, chunk - 33, chunk - 1, chunk, chunk + 1, chunk + 32, n - 33, n - 2, n - 1],
                   np.int64)
    N = spec.n_ports
    cols = (ids[:, None] * N + np.arange(N)).ravel()
    g = {"actions": out["actions"][:, torch.from_numpy(cols).cuda()].cpu().numpy(),
         "reward": out["reward"][:, torch.from_numpy(ids).cuda()].cpu().numpy(),
         "done": out["done"][:, torch.from_numpy(ids).cuda()].cpu().numpy()}
    del out
    teacher_forced(oracle_lib, spec, weights, seed, g, ids, T)


def test_policy_invalid(cxm):
    spec = W.policy_station()
    weights = W.policy_weights(spec.n_ports, hidden=H, seed=1)
    env = cxm.Env(spec, n_envs=4, seed=1)
    with pytest.raises(cxm.CxError):
        env.rollout(2, cxm.ACT_POLICY, cxm.OUT_REWARD)          # no policy yet
    with pytest.raises(cxm.CxError):
        env.set_policy(48, W.policy_weights(spec.n_ports, hidden=48, seed=1))
    big = W.splitter_tree(4, 16, 60.0, 500.0)                   # 64 ports: obs longer than 256
    with pytest.raises(cxm.CxError):
        cxm.Env(big, n_envs=2, seed=1).set_policy(H, W.policy_weights(big.n_ports, hidden=H, seed=1))
    specs = W.mixture_classes()[:2]
    multi = cxm.Env(specs, env_class=np.array([0, 1], np.int32), seed=1)
    with pytest.raises(cxm.CxError):
        multi.set_policy(H, W.policy_weights(specs[0].n_ports, hidden=H, seed=1))
    env.set_policy(H, weights)
    env.set_policy(H, weights)                                  # replacing a policy is allowed
    out = env.rollout(2, cxm.ACT_POLICY, cxm.OUT_REWARD)
    assert out["reward"].shape == (2, 4)
