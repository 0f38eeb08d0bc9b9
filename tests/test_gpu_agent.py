"""The learned layout search (Section III-C, Algorithm 1) with our GPU MTTKRP
as its environment: every encoding it reaches is exact, and MTTKRP on the
best one matches the oracle."""
import numpy as np
import pytest

import oracle
from paper_2509_00280_amd import agent, synth
from _gpu_helpers import check_encoding, factors_dev, mttkrp_error, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spt():
    import torch
    assert torch.cuda.is_available()
    from paper_2509_00280_amd import spt as _spt
    _spt.lib()
    return _spt


def test_agent_search_on_the_gpu_environment(spt):
    import torch
    t = synth.distinct_coo(7, (300, 200, 64), 30_000, [("zipf", 1.2), ("zipf", 1.2), "uniform"], "u01")
    F = synth.normal_factors(8, t.dims, 16)
    c, v = to_dev(t)
    Fd = factors_dev(F)
    reward, alto, alto_ms, lbits = agent.gpu_environment(t.dims, c, v, Fd, iters=2, repeats=3)
    assert alto == list(oracle.alto_layout(t.dims)) and alto_ms > 0
    assert lbits == oracle.bit_lengths(t.dims)
    res = agent.relate_search(reward, lbits, episodes=150, seed=5, max_evaluations=30)
    print(f"episodes {res.episodes} measured {res.evaluations} best speedup over ALTO {res.best_reward:.4f}", flush=True)
    assert list(np.bincount(res.best_layout, minlength=3)) == lbits and res.evaluations >= 1
    h = spt.encode(t.dims, c, v, layout=res.best_layout)
    check_encoding(h, t, layout=res.best_layout)
    for mode in range(3):
        out = spt.mttkrp(h, Fd, mode)
        torch.cuda.synchronize()
        err, bad = mttkrp_error(t, F, mode, out.cpu().numpy())
        assert bad == 0 and err <= 1e-4
    # the reward is relative to ALTO: ALTO measured again is about 1 (timing noise aside)
    assert 0.7 < reward(alto) < 1.4
