"""The throughput convention (GFLOP/s = 2 m n k / t) reproduces the rates the
paper prints in Tables I and II (tests/golden/paper_rates.txt)."""
import os

from paper_1608_05265_amd.workloads import gflops_rate

HERE = os.path.dirname(os.path.abspath(__file__))


def test_paper_rates():
    rows = 0
    with open(os.path.join(HERE, "golden", "paper_rates.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            m, n, k, t, printed, _src = line.split()
            rate = gflops_rate(int(m), int(n), int(k), float(t))
            # the printed rates carry three decimals, sometimes rounded and
            # sometimes truncated (2.5436 appears as 2.543): within one unit
            # of the last printed digit
            assert abs(rate - float(printed)) < 1e-3, line
            rows += 1
    assert rows == 4
