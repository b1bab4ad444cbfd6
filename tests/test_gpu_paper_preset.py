"""The paper's own workload on the GPU: the Sec. IV-B uncertainty model with
RK4, no obstacle, at every sample count of Table I.  Each row equals the
reference (FP64, same seeded inputs) and its statistics fall in the band of
the paper's printed row; at 350,000 samples the minimum safe headways of
Sec. VI-C.  The paper's random stream is unstated, so the comparison with
its numbers is statistical."""
import json
import os

import numpy as np
import pytest

from paper_2604_27193_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_results.json")


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2604_27193_amd import binding
    binding.lib()
    return binding


def test_table_I_rows(B, orc):
    gold = json.load(open(GOLD))
    risk = tuple(gold["headways"]["risk"])
    threads = orc.host_threads()
    sigma = 12.2
    for row in gold["table_I"]["rows"]:
        n = row["n"]
        d = W.paper_preset(n, seed=2026)
        st = B.reduce(B.rollout(d), risk=risk)
        if n <= 100_000:
            ref = orc.reduce(orc.run(d, threads=threads), risk=risk)
            for k in ("n", "n_stop", "n_horizon"):
                assert st[k] == ref[k], (n, k)
            assert abs(st["mean_dist"] - ref["mean_dist"]) <= 1e-12 * ref["mean_dist"]
            assert abs(st["sd_dist"] - ref["sd_dist"]) <= 1e-10 * ref["sd_dist"]
            for a, b in zip(st["headway"], ref["headway"]):
                assert abs(a - b) <= 1e-12 * b, n
        # two independent estimates of the same mean / sd
        se_mean = np.sqrt(2.0) * sigma / np.sqrt(n)
        se_sd = np.sqrt(2.0) * sigma / np.sqrt(2.0 * n)
        assert abs(st["mean_dist"] - row["mean"]) <= 4 * se_mean + 0.1, (n, st["mean_dist"])
        assert abs(st["sd_dist"] - row["sd"]) <= 4 * se_sd + 0.1, (n, st["sd_dist"])
        if n == 350_000:
            h, want = st["headway"], gold["headways"]["h0"]
            assert abs(h[0] - want[0]) < 1.0 and abs(h[1] - want[1]) < 1.5
            # the 0.1 % tail is the most sensitive to the parts of the uncertainty
            # model the paper leaves open (the same band as the reference's pin)
            assert abs(h[2] - want[2]) < 6.0
            print(f"paper preset 350k: mean {st['mean_dist']:.3f} sd {st['sd_dist']:.3f} "
                  f"headways {[round(x, 2) for x in h]}")
