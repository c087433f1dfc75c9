"""The V-cycle launch timer and the launch-shape autotuner (GPU).

* aao_profile_vcycle reports one labelled in-situ and one stand-alone time
  per kernel launch of a V-cycle (down and up kernels per tiled level, one
  tail), bracketing the time of the whole cycle;
* aao_autotune picks one of its candidates, never changes the cycle's
  arithmetic beyond rounding (multigrid output against the oracle), and
  reads its choice back from the cache file instead of timing again.
"""
import numpy as np
import pytest

from gpu_util import announce, rel_err, require_gpu
from oracle import allatonce, multigrid, tableau

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_profile_vcycle_labels_and_times():
    require_gpu()
    from paper_2609_16863_amd import HeatProblem
    n, s, nt = 256, 3, 8
    hp = HeatProblem(2, n, s, nt, 1.0, precision="fp32")
    nodes, tail = hp.mg_levels()
    announce("profile_vcycle")
    for count in (1, nt):
        launches, total = hp.profile_vcycle(count=count, reps=5)
        labels = [lab for lab, _, _ in launches]
        want = [f"k_down2d@{l}" for l in range(tail)] + [f"k_tail_fast@{tail}"] + \
               [f"k_up2d@{l}" for l in reversed(range(tail))]
        assert labels == want, (labels, want)
        situ = [u for _, u, _ in launches]
        alone = [u for _, _, u in launches]
        assert all(u > 0 for u in situ) and all(u > 0 for u in alone)
        # the graph-replayed cycle costs at most the in-situ launches (which
        # add an event between every two of them) and at least its longest
        # launch; the sum of the launches alone is no bound (replayed alone,
        # each pays the dispatch latency that back-to-back launches hide)
        assert max(alone) <= 1.2 * total and total <= 1.2 * sum(situ), (alone, total, sum(situ))


def test_autotune_choice_cache_and_parity(tmp_path):
    require_gpu()
    from paper_2609_16863_amd import HeatProblem
    n, s, nt = 150, 2, 16
    cache = tmp_path / "tune.txt"
    hp = HeatProblem(2, n, s, nt, 1.0, precision="fp32", schur="mgrit", mgrit_cf=4)
    announce("autotune")
    t = hp.autotune(reps=3, cache=cache)
    assert t["from_cache"] == 0
    assert t["tall_min_b"] in (1, 8, 1 << 30) and t["tail_extend"] in (0, 1)
    assert t["blocks"] == [1, 4, 16]
    assert all(v > 0 for row in t["us"] for v, w in zip(row, t["weight"]) if w > 0)
    # the chosen candidate has the least weighted time
    cost = [sum(w * u for w, u in zip(t["weight"], row)) for row in t["us"]]
    chosen = [c for c in range(6) if (1, 8, 1 << 30)[c % 3] == t["tall_min_b"] and int(c < 3) == t["tail_extend"]]
    assert cost[chosen[0]] == min(cost)
    # a second handle of the same shape reads the cache
    hp2 = HeatProblem(2, n, s, nt, 1.0, precision="fp32", schur="mgrit", mgrit_cf=4)
    t2 = hp2.autotune(reps=3, cache=cache)
    assert t2["from_cache"] == 1
    assert (t2["tall_min_b"], t2["tail_extend"]) == (t["tall_min_b"], t["tail_extend"])
    # tuned cycles are still the oracle's cycle (FP32 rounding)
    p = allatonce.Problem(n, 2, s, nt, 1.0)
    L, _ = tableau.crout(p.A)
    H = multigrid.Hierarchy(p.K(), n, 2, p.tau * L[0, 0], multigrid.COARSE_MAX)
    r = np.random.default_rng(2).standard_normal((nt, p.N)).astype(np.float32)
    z = hp.apply_mg(torch.from_numpy(r).cuda().reshape(-1), 0).cpu().numpy().reshape(nt, p.N)
    ref = np.stack([multigrid.solve(H, b.astype(np.float64), 1, 0.8, 2, 2) for b in r[[0, nt - 1]]])
    assert rel_err(z[[0, nt - 1]], ref) <= 2e-5
