"""Host-side logic of the bench and the workload generators (no GPU)."""
import numpy as np
import pytest

import bench
from workloads import gen


def test_taylor_flop_count_small_orders():
    # order 0: no powers, one column with only the value product and FMA into d/du, then 3 subtractions
    assert bench.taylor_flops_per_particle(0) == 0 + 3 + 6
    # order 1: powers 2; columns (0,0) top 1: 4+3, (0,1): 3+4, (1,0): 3+4; + 6
    assert bench.taylor_flops_per_particle(1) == 2 + (4 + 3) + (3 + 4) + (3 + 4) + 6


def test_roofline_picks_the_binding_roof():
    r = bench._roofline(nbytes=8e12 * 0.5, flops=78.6e12 * 0.1, ms=1000.0, kernel="k")
    assert r["bound"] == "hbm" and abs(r["frac"] - 0.5) < 1e-12 and r["other_roof"]["bound"] == "alu"
    r = bench._roofline(nbytes=8e12 * 0.1, flops=78.6e12 * 0.3, ms=1000.0, kernel="k")
    assert r["bound"] == "alu" and abs(r["frac"] - 0.3) < 1e-12


def test_frac_errors_over_several_boxes():
    ref0 = np.array([[1.0, 0.0, 0.0], [0.0, 2.0, 0.0]])
    ref1 = np.array([[0.0, 0.0, 4.0]])
    acc = np.zeros((5, 3), np.float32)
    acc[1] = [1.0 + 1e-3, 0, 0]
    acc[2] = [0, 2.0, 0]
    acc[4] = [0, 0, 4.0 * (1 + 1e-2)]
    med, p99, n = bench.frac_errors(acc, [(np.array([1, 2]), ref0), (np.array([4]), ref1)])
    assert n == 3
    assert med == pytest.approx(np.median([1e-3, 0.0, 1e-2]), rel=1e-4)


def test_oracle_sample_covers_boxes_and_grows():
    w = gen.workload("batched", n_boxes=3, lo=8 ** 3, hi=10 ** 3)
    base, parts = bench.oracle_sample(w.boxes, 0, 0.2, 2, m_fixed=300)
    assert len(parts) == 3
    offs = np.cumsum([0] + [b.n for b in w.boxes])
    for k, (idx, ref) in enumerate(parts):
        assert np.all((idx >= offs[k]) & (idx < offs[k + 1]))
        assert len(np.unique(idx)) == len(idx) and ref.shape == (len(idx), 3)
    assert base["cores"] == 2 and base["kind"] == "oracle" and base["single_core"]["cores"] == 1


def test_taylor_coefficients_scale_with_degree():
    T = gen.taylor_coefficients(4000, 4, seed=1, amp=2.0, r0=3.0)
    assert T.shape == (4000, 35)
    start = 0
    for n in range(5):
        cnt = (n + 1) * (n + 2) // 2
        sd = T[:, start:start + cnt].std()
        assert sd == pytest.approx(2.0 * 3.0 ** -n, rel=0.05)
        start += cnt


def test_sample_sinks_distinct_and_sorted():
    s = gen.sample_sinks(1000, 100, seed=5)
    assert len(np.unique(s)) == 100 and np.all(np.diff(s) > 0) and s.max() < 1000
    assert np.array_equal(gen.sample_sinks(50, 100), np.arange(50))
