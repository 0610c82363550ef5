"""Pin of the oracle's divided difference of the logarithm, (ln b_i - ln b_j) / (b_i - b_j),
the off-diagonal factor of the principal-direction tangent (Appendix B; finite at coalescing
eigenvalues, where it tends to 1 / b_j).

The reference is computed from the same double inputs in 50-digit decimal arithmetic
(Python's decimal module: ln and division correctly rounded at that precision), so it is
independent of the oracle's two branches (a 7-term series of log1p(x)/x for |x| < 1e-3 with
x = b_i / b_j - 1, long-double log1p beyond). Gaps straddle the branch switch and reach down
to a few ulps; a wrong series coefficient (x^2 / 4 for x^2 / 3, say) would be off by ~1e-7
at the switch.
"""
from decimal import Decimal, getcontext

import numpy as np
import pytest

getcontext().prec = 50


def exact(bi_m1, bj_m1):
    bi = Decimal(1) + Decimal(bi_m1)
    bj = Decimal(1) + Decimal(bj_m1)
    if bi == bj:
        return Decimal(1) / bj
    return (bi.ln() - bj.ln()) / (bi - bj)


GAPS = [0.0, 1e-16, 3e-15, 1e-12, 1e-9, 1e-6, 1e-4, 5e-4, 9.9e-4, 1.01e-3, 3e-3, 1e-2, 0.1, 0.5, 2.0]
BASES = [-0.6, -2e-2, -1e-4, 0.0, 3e-7, 1e-3, 2e-2, 0.4, 3.0]


@pytest.mark.parametrize("bj_m1", BASES)
def test_log_divdiff_matches_50_digit_reference(oracle_lib, bj_m1):
    worst = 0.0
    for gap in GAPS:
        for sign in (1.0, -1.0):
            bi_m1 = (1.0 + bj_m1) * (1.0 + sign * gap) - 1.0
            if 1.0 + bi_m1 <= 0.0:
                continue
            got = oracle_lib.log_divdiff(bi_m1, bj_m1)
            ref = exact(bi_m1, bj_m1)
            rel = abs(Decimal(got) - ref) / abs(ref)
            worst = max(worst, float(rel))
            assert rel <= Decimal("4e-16"), (bi_m1, bj_m1, got, ref)
    assert worst <= 4e-16


def test_log_divdiff_symmetric_and_limit(oracle_lib):
    rng = np.random.default_rng(7)
    for _ in range(200):
        a, b = rng.uniform(-0.5, 2.0, 2)
        b = a + rng.choice([0.0, 1e-14, 1e-8, 1e-4, 1e-2]) * rng.choice([-1.0, 1.0])
        x, y = oracle_lib.log_divdiff(a, b), oracle_lib.log_divdiff(b, a)
        assert abs(x - y) <= 4e-16 * abs(x), (a, b, x, y)
    for b in (-0.5, 0.0, 1e-3, 1.0):
        assert abs(oracle_lib.log_divdiff(b, b) - 1.0 / (1.0 + b)) <= 2e-16 / (1.0 + b)
