"""Pins of the buffer-element stencils of Eq. (11): the temporal one (every Legendre mode of the
neighbour across a delayed PE interface extrapolated from q past levels with the weights of Eq. (8))
and the hybrid spatio-temporal one of the end of Sec. 3.3 (mode j from q_j = max(1, q - j) levels:
in nodal values, each node's level-n value from delayed values at all the element's nodes, older
levels contributing only the low modes)."""
import math

import numpy as np
import pytest
from numpy.polynomial import legendre as L

from workloads import gen


def buffer(orc, q, k, levels, hybrid):
    """levels: [q][V][M] modal data of levels n-k, n-k-1, ..."""
    levels = np.ascontiguousarray(levels, dtype=np.float64)
    _, V, M = levels.shape
    out = np.zeros((V, M))
    assert orc.lib().or_at_buffer(q, k, V, M, int(hybrid), orc._dptr(levels), orc._dptr(out)) == 0
    return out


@pytest.mark.parametrize("q", [2, 3, 4, 5])
@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_each_mode_uses_exactly_its_levels(orc, q, k):
    """Mode j of the hybrid stencil is exact for data polynomial in time of degree q_j - 1 and not
    for degree q_j (so it uses exactly q_j = max(1, q - j) levels); the temporal stencil is exact to
    degree q - 1 in every mode.  Level n - k - l sits at time -(k + l), level n at 0."""
    M, V = q, 2
    rng = np.random.default_rng(10 * q + k)
    t = -(k + np.arange(q, dtype=float))
    for hybrid in (False, True):
        for extra in (0, 1):
            coef = rng.normal(size=(V, M, q + 1))
            lv = np.zeros((q, V, M))
            exact = np.zeros((V, M))
            for j in range(M):
                deg = (max(1, q - j) if hybrid else q) - 1 + extra
                for v in range(V):
                    p = coef[v, j, : deg + 1]
                    lv[:, v, j] = np.polynomial.polynomial.polyval(t, p)
                    exact[v, j] = p[0]
            out = buffer(orc, q, k, lv, hybrid)
            if extra == 0:
                # the weights grow like k^q: cancellation of the level values, not of the result
                np.testing.assert_allclose(out, exact, rtol=0, atol=1e-12 * np.abs(lv).max() * (k + q) ** q)
            elif k > 0:
                err = np.abs(out - exact)
                assert np.all(err.max(axis=0) > 1e-6), (hybrid, err)   # every mode misses one degree more
            else:
                np.testing.assert_array_equal(out, lv[0])              # k = 0: the current level itself


def local_error(orc, E, order_p, k, hybrid, cfl=0.1, lam=1.0 + math.sqrt(1.4 / 0.8)):
    """Error of the buffer element's level-n modes formed from exact past levels of the entropy wave
    rho = 1 + 0.2 sin 2 pi (x - t), L2 over all elements of a periodic mesh (the DG Courant step)."""
    q = order_p + 1
    dt = gen.default_dt(cfl, 1.0 / E, lam, order_p)
    fn = lambda t: (lambda x: np.array([gen.entropy_wave_exact(x, t)]))
    lv = np.stack([gen.project(fn(-(k + l) * dt), E, order_p, 0.0, 1.0)[:, 0, :] for l in range(q)])   # [q][E][M]
    exact = gen.project(fn(0.0), E, order_p, 0.0, 1.0)[:, 0, :]
    out = buffer(orc, q, k, lv.transpose(0, 1, 2), hybrid)   # the elements play the role of variables
    err = out - exact
    return math.sqrt(np.sum(err**2 * (2.0 / (2 * np.arange(q) + 1))[None, :]) * 0.5 / E)


@pytest.mark.parametrize("order_p", [1, 2, 3])
@pytest.mark.parametrize("k", [1, 2])
def test_buffer_stencils_reach_order_q_on_the_entropy_wave(orc, order_p, k):
    """With dt ~ dx the temporal stencil's error is O(dt^q) and the hybrid one's O(dt^(q-j) dx^j) in
    mode j: both converge at order q = N_p + 1 (the hybrid with a larger constant, about
    (dx/dt)^N_p times at the DG Courant step), while one level fewer in every mode loses an order."""
    Es = [8, 16, 32, 64]
    q = order_p + 1
    for hybrid in (False, True):
        errs = np.array([local_error(orc, E, order_p, k, hybrid) for E in Es])
        rates = np.log2(errs[:-1] / errs[1:])
        assert abs(rates[-1] - q) < 0.15, (hybrid, errs, rates)


def hybrid_case(E, order_p, stencil, mode, t_end, cfl):
    case, w0 = gen.case_c0(E=E, order_p=order_p, n_pe=8, mode=mode, k_pre=0.0, cfl=cfl, pmf=(1 / 3, 1 / 3, 1 / 3))
    case["async"].update(L=3, at_stencil=stencil)
    case["disc"].update(limiter=1, indicator="all")
    steps = int(math.ceil(t_end / case["disc"]["dt"]))
    case["disc"]["dt"] = t_end / steps
    return case, w0, steps


def run(orc, case, w0, steps):
    s = orc.OracleSolver(case, w0, steps + 1)
    s.step(steps)
    w = s.state()
    s.close()
    return w


def l2_rho(e, order_p, E):
    M = order_p + 1
    return math.sqrt(np.sum(e[:, 0, :] ** 2 * (2.0 / (2 * np.arange(M) + 1))[None, :]) * 0.5 / E)


def test_hybrid_adg_keeps_the_order_of_the_delay_error(orc):
    """The whole solver on the entropy wave with the limiter on every cell (the accuracy-test setting
    of the simple WENO limiter) and CAA delays k = n mod 3 at 8 PE interfaces: the error the delays
    add (ADG against the synchronous run) converges at N_p + 1 = 3 with either buffer stencil."""
    order_p, t_end, cfl = 2, 0.1, 0.05
    Es = [16, 32, 64]
    d = {"temporal": [], "hybrid": []}
    for E in Es:
        case, w0, steps = hybrid_case(E, order_p, "temporal", "sync", t_end, cfl)
        sa = run(orc, case, w0, steps)
        for st in d:
            case, w0, steps = hybrid_case(E, order_p, st, "caa", t_end, cfl)
            d[st].append(l2_rho(run(orc, case, w0, steps) - sa, order_p, E))
    for st, errs in d.items():
        rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
        assert rates[-1] > order_p + 1 - 0.3, (st, errs, rates)


def test_hybrid_conserves_and_k0_is_synchronous(orc):
    """Cell means are kept by the limiter, so the hybrid run conserves mass, momentum and energy; with
    every delay 0 it is the synchronous run bit for bit."""
    case, w0, steps = hybrid_case(32, 2, "hybrid", "caa", 0.05, 0.05)
    w = run(orc, case, w0, steps)
    for v in range(3):
        assert abs(w[:, v, 0].sum() - w0[:, v, 0].sum()) <= 1e-13 * abs(w0[:, v, 0]).sum()
    sync, _, _ = hybrid_case(32, 2, "temporal", "sync", 0.05, 0.05)
    zero, _, _ = hybrid_case(32, 2, "hybrid", "saa", 0.05, 0.05)
    zero["async"]["pmf"] = [1.0, 0.0, 0.0]
    np.testing.assert_array_equal(run(orc, zero, w0, steps), run(orc, sync, w0, steps))
