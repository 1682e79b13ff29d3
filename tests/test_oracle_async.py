"""Pins of the asynchrony layer (Sec. 3.2 Eq. (7)-(8), Table 1; Sec. 4 CAA / SAA)."""
import os
from fractions import Fraction

import numpy as np
import pytest

from workloads import gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "at_coefficients_table1.txt")


def table1():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        parts = line.split()
        order, level = int(parts[0]), parts[1]
        num = [int(x) for x in parts[2:6]]
        den, den_fixed = int(parts[6]), int(parts[7])
        shift = 0 if level == "k" else int(level.split("+")[1])
        rows.append((order, shift, num, den, den_fixed, "MISPRINT" in parts))
    return rows


def poly(num, k):
    return sum(c * k**p for p, c in enumerate(num))


@pytest.mark.parametrize("k", range(0, 6))
def test_at_weights_match_table1(orc, k):
    """Eq. (8) solved by the oracle equals Table 1 (with its one misprinted denominator corrected)."""
    for order, shift, num, den, den_fixed, misprint in table1():
        c = orc.at_coeffs(order, k)
        expect = Fraction(poly(num, k), den_fixed)
        assert c[shift] == float(expect), (order, shift, k, c[shift], expect)
        if misprint and k >= 1:
            # the printed /6 would break sum c = 1 (zeta = 0 row of Eq. (8))
            printed = [Fraction(poly(n2, k), d2) for (o2, s2, n2, d2, _, _) in table1() if o2 == order]
            assert sum(printed) != 1


def test_at2_explicit_form(orc):
    """Sec. 3.2 writes the second-order AT flux as (k+1) f^{n-k} - k f^{n-k-1}."""
    for k in range(8):
        np.testing.assert_array_equal(orc.at_coeffs(2, k), [k + 1, -k])


@pytest.mark.parametrize("q", range(1, 7))
@pytest.mark.parametrize("k", range(0, 6))
def test_eq8_residuals_vanish_exactly(orc, q, k):
    c = [Fraction(x).limit_denominator(10**6) for x in orc.at_coeffs(q, k)]
    for x, y in zip(c, orc.at_coeffs(q, k)):
        assert float(x) == y
    for z in range(q):
        res = sum(cl * Fraction(-(k + l)) ** z for l, cl in enumerate(c))
        assert res == (1 if z == 0 else 0)


def test_zero_delay_weights_are_synchronous(orc):
    for q in range(1, 7):
        c = orc.at_coeffs(q, 0)
        assert c[0] == 1.0 and np.all(c[1:] == 0.0)


def test_splitmix64_published_vector(orc):
    """SplitMix64 from state 0 gives 0xE220A8397B1DCDAF as its first output."""
    assert orc.lib().or_splitmix64(0) == 0xE220A8397B1DCDAF


def _cfg(orc, mode, L=3, pmf=(0.3, 0.4, 0.3), n_pe=16, seed=2502, schedule=None):
    case, _ = gen.case_c0(E=64, n_pe=n_pe, mode=mode, pmf=pmf, seed=seed)
    case["async"]["L"] = L
    case["disc"]["order_p"] = 2
    if schedule is not None:
        case["async"]["schedule"] = schedule
    return orc.Config(case)


@pytest.mark.parametrize("pmf", [(0.3, 0.4, 0.3), (0.5, 0.3, 0.2), (0.8, 0.1, 0.1)])
def test_saa_binning_matches_probability_sets(orc, pmf):
    """Sec. 4.2: [0,1] is cut into bins of widths p_k; the delay frequencies follow the set."""
    cfg = _cfg(orc, "saa", pmf=pmf)
    lib = orc.lib()
    counts = np.zeros(3)
    n_if = 16
    for n in range(4000):
        for i in range(n_if):
            counts[lib.or_raw_delay(cfg.ref(), n_if, n, i)] += 1
    freq = counts / counts.sum()
    np.testing.assert_allclose(freq, pmf, atol=0.01)


def test_saa_bin_edges(orc):
    """The drawn number decides the bin by left-closed intervals."""
    lib = orc.lib()
    cfg = _cfg(orc, "saa", pmf=(0.3, 0.4, 0.3))
    for n in range(50):
        for i in range(16):
            u = lib.or_saa_uniform(2502, n, i, 16)
            assert 0.0 <= u < 1.0
            k = lib.or_raw_delay(cfg.ref(), 16, n, i)
            assert k == (0 if u < 0.3 else 1 if u < 0.3 + 0.4 else 2)


def test_caa_schedule(orc):
    """Sec. 4.1: the delay grows by one level per step and resets when n % L == 0."""
    cfg = _cfg(orc, "caa", L=3)
    lib = orc.lib()
    assert [lib.or_raw_delay(cfg.ref(), 16, n, 5) for n in range(9)] == [0, 1, 2, 0, 1, 2, 0, 1, 2]


def test_startup_clamp(orc):
    """Levels before n = 0 do not exist: a delay is clamped to k <= n - q + 1."""
    sched = np.full((1, 16), 2, dtype=np.int8)
    cfg = _cfg(orc, "schedule", schedule=sched)   # q = N_p + 1 = 3
    lib = orc.lib()
    got = [lib.or_eff_delay(cfg.ref(), 16, n, 0) for n in range(6)]
    assert got == [0, 0, 0, 1, 2, 2]
