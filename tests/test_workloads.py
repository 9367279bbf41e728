"""The paper's nine int32 distributions follow its recipe (its experimental setup): range, shape, repeats."""
import numpy as np

import workloads


def test_paper_distributions_recipe():
    n = 200_000
    d = {name: workloads.make(name, np.int32, n, 42) for name in workloads.PAPER_DISTRIBUTIONS}
    for name, x in d.items():
        assert x.dtype == np.int32 and x.size == n, name
        assert x.min() >= -10**9 and x.max() <= 10**9, name
    assert abs(np.mean(d["paper_uniform"])) < 1e7
    assert abs(np.std(d["paper_normal"].astype(np.float64)) / 1e8 - 1) < 0.02
    e = d["paper_exponential"].astype(np.float64) + 1e9  # Exp(1e9) before the shift
    assert abs(np.median(e) / (1e9 * np.log(2)) - 1) < 0.02
    assert (d["paper_exponential"] == 10**9).mean() > 0.1  # the clip at 2e9 catches e^-2 of the mass
    p = (d["paper_power"].astype(np.float64) + 1e9) / 2e9  # power(a=0.5): CDF x^0.5
    assert abs(np.mean(p < 0.25) - 0.5) < 0.01
    b = (d["paper_beta"].astype(np.float64) + 1e9) / 2e9
    assert abs(b.mean() - 2 / 7) < 0.005  # Beta(2, 5) mean
    assert abs((d["paper_sparse"] == 0).mean() - 0.9) < 0.001
    c = d["paper_clustered"].astype(np.float64)
    centres = np.linspace(-1e9, 1e9, 10)
    assert np.median(np.min(np.abs(c[:, None] - centres[None, :]), axis=1)) < 1e8
    ns = d["paper_nearly_sorted"]
    assert 0.80 < np.mean(np.diff(ns.astype(np.int64)) >= 0) < 0.95  # ramp with 10 % replaced
    assert abs(np.unique(d["paper_duplicates"]).size / n - 0.1) < 0.01
    # reproducible from the seed
    assert np.array_equal(workloads.make("paper_beta", np.int32, 1000, 7), workloads.make("paper_beta", np.int32, 1000, 7))
