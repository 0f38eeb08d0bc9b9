"""The learned layout search (Section III-C, Algorithm 1) on the host: the
networks' gradients against finite differences, action masking, the paper's
sandbox (reward for reproducing the ALTO encoding), the reward cache, the
reward model's filtering and elastic early stopping."""
import math

import numpy as np
import pytest

import oracle
from paper_2509_00280_amd import agent


def _fd_check(forward_loss, params, grads, rng, count=12, h=1e-6):
    for _ in range(count):
        k = int(rng.integers(len(params)))
        p = params[k]
        i = tuple(int(rng.integers(s)) for s in p.shape)
        old = p[i]
        p[i] = old + h
        up = forward_loss()
        p[i] = old - h
        dn = forward_loss()
        p[i] = old
        num = (up - dn) / (2 * h)
        assert abs(num - grads[k][i]) <= 1e-5 * max(1.0, abs(num)), (k, i, num, grads[k][i])


def test_qnet_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    net = agent.QNet(3, 6, 8, rng)
    for p in net.params:
        p += rng.standard_normal(p.shape) * 0.05  # biases off zero: no ReLU kinks at 0
    x = rng.integers(0, 2, size=(4, 3, 6)).astype(np.float32)
    dq = rng.standard_normal((4, 3))

    def loss():
        return float((net.forward(x) * dq).sum())

    net.forward(x, keep=True)
    _fd_check(loss, net.params, net.backward(dq), rng)


def test_reward_model_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    m = agent.RewardModel(10, 7, rng)
    for p in m.params:
        p += rng.standard_normal(p.shape) * 0.05
    x = rng.standard_normal((5, 10))
    dy = rng.standard_normal(5)

    def loss():
        return float((m.forward(x) * dy).sum())

    m.forward(x, keep=True)
    _fd_check(loss, m.params, m.backward(dy), rng)


def test_every_episode_ends_in_a_valid_interleaving():
    lbits = [3, 2, 2, 1]
    seen = []

    def reward(layout):
        counts = np.bincount(layout, minlength=len(lbits))
        assert list(counts) == lbits  # the mask keeps every mode at exactly l(n) bits
        seen.append(tuple(layout))
        return 1.0 + 0.1 * layout.index(3) / len(layout)

    res = agent.relate_search(reward, lbits, episodes=60, seed=2, model_warmup=10 ** 9)
    assert seen and len(set(seen)) == len(seen)  # the cache measures a layout once
    assert list(np.bincount(res.best_layout, minlength=4)) == lbits
    assert res.evaluations == len(seen) and res.evaluations + res.cache_hits + res.imagined == res.episodes


def test_sandbox_reproduces_the_alto_encoding():
    """The paper's sandbox (Section IV-A): reward for reproducing the ALTO encoding."""
    dims = (8, 4, 4, 2)
    target = list(oracle.alto_layout(dims))
    lbits = list(oracle.bit_lengths(dims))
    L = len(target)

    def reward(layout):
        return math.exp(sum(int(a == b) for a, b in zip(layout, target)) / L)

    calls = []

    def measured(layout):
        calls.append(tuple(layout))
        return reward(layout)

    # sandbox mode measures nothing real: the reward model is left out
    res = agent.relate_search(measured, lbits, episodes=2000, seed=0, model_warmup=10 ** 9)
    found = calls.index(tuple(target)) + 1
    greedy = agent.greedy_layout(res.policy, lbits)
    print(f"episodes {res.episodes}, measured {res.evaluations}, target at measurement {found}, greedy {greedy}")
    assert res.best_layout == target and res.best_reward == pytest.approx(math.e)
    # uniform sampling without repeats needs 841 of the 1680 interleavings
    # (Eq. (1): 8!/(3!2!2!1!)) on average; the learned policy far fewer
    assert found < 420
    # and the trained policy alone reproduces most of the encoding
    assert sum(int(a == b) for a, b in zip(greedy, target)) >= 6


def test_elastic_stop_on_a_flat_reward():
    res = agent.relate_search(lambda layout: 1.0, [4, 3, 2], episodes=200, seed=3, model_warmup=10 ** 9)
    # the best reward never improves after the first episode: the search ends once
    # the patience window ceil(E_max * eps) has shrunk below the episodes since then
    assert res.stopped_early and res.episodes < 200
    eps = max(0.1, (0.1) ** (res.episodes / 100))
    assert res.episodes - 1 >= math.ceil(200 * eps)


def test_reward_model_filters_once_accurate():
    lbits = [4, 4, 3]
    rng = np.random.default_rng(5)
    w = rng.standard_normal((3, 11)) * 0.05

    def reward(layout):
        return float(np.exp((w * agent.layout_to_state(layout, 3)).sum()))

    res = agent.relate_search(reward, lbits, episodes=400, seed=4)
    assert res.model_trusted_at is not None and res.imagined > 0
    # the best layout was measured, never imagined
    assert res.best_reward == pytest.approx(reward(res.best_layout))


def test_greedy_rollout_is_valid():
    rng = np.random.default_rng(6)
    net = agent.QNet(3, 7, 16, rng)
    lay = agent.greedy_layout(net, [3, 2, 2])
    assert list(np.bincount(lay, minlength=3)) == [3, 2, 2]
