"""Integration pins of the oracle's ADG time step (Sec. 3.1-3.3, Sec. 4)."""
import math

import numpy as np
import pytest
from numpy.polynomial import legendre as L

from workloads import gen


def run(orc, case, w0, steps):
    s = orc.OracleSolver(case, w0, steps + 1)
    s.step(steps)
    return s.state()


def test_zero_delays_reproduce_synchronous_dg_bitwise(orc):
    """Sec. 3.2: with k = 0 the AT flux is the synchronous flux, so ADG is SA exactly."""
    case, w0 = gen.case_c0(E=96, n_pe=6, mode="sync")
    ref = run(orc, case, w0, 60)
    case_saa = dict(case, **{"async": dict(case["async"], mode="saa", pmf=[1.0, 0.0], L=2)})
    np.testing.assert_array_equal(run(orc, case_saa, w0, 60), ref)
    case_caa = dict(case, **{"async": dict(case["async"], mode="caa", L=1)})
    np.testing.assert_array_equal(run(orc, case_caa, w0, 60), ref)


def test_delays_change_the_solution_slightly(orc):
    case, w0 = gen.case_c0(E=96, n_pe=6, mode="sync")
    ref = run(orc, case, w0, 60)
    case["async"]["mode"] = "saa"
    w = run(orc, case, w0, 60)
    d = np.abs(w - ref).max()
    assert 0 < d < 1e-4


@pytest.mark.parametrize("mode", ["saa", "caa"])
def test_conservation_and_mass_fractions_under_delays(orc, mode):
    """Single-valued PE-interface fluxes keep mass, momentum, energy and total species exactly."""
    case, w0 = gen.case_c0(E=128, n_pe=8, mode=mode)
    w = run(orc, case, w0, 200)
    tot0 = w0[:, :, 0].sum(0)
    tot = w[:, :, 0].sum(0)
    for v in range(3):
        assert abs(tot[v] - tot0[v]) <= 1e-13 * abs(tot0[v])
    assert abs(tot[3] + tot[4] - tot0[3] - tot0[4]) <= 1e-13 * abs(tot0[3] + tot0[4])
    assert tot[4] > tot0[4] + 1e-3, "reaction must have consumed reactant"
    np.testing.assert_allclose(w[:, 3:, :].sum(1), w[:, 0, :], rtol=0, atol=1e-13)


def test_uniform_state_stays_uniform_under_delays(orc):
    """sum_l c^l = 1, so delayed fluxes of a uniform state cancel exactly."""
    case, _ = gen.case_c0(E=40, n_pe=5, mode="saa", k_pre=0.0)
    w0 = np.zeros((40, 5, 3))
    w0[:, :, 0] = gen.onestep_conserved(1.3, 0.7, 2.0, 0.4, case["physics"])[:, None].T
    w = run(orc, case, w0, 50)
    np.testing.assert_allclose(w, w0, rtol=0, atol=1e-14 * np.abs(w0).max())


def entropy_error(orc, E, order_p, mode, at_order, t_end=0.2, cfl=0.2, pmf=(0.5, 0.5)):
    case, w0 = gen.case_c0(E=E, order_p=order_p, n_pe=8, mode=mode, k_pre=0.0, cfl=cfl,
                           at_order=at_order, pmf=pmf)
    steps = int(math.ceil(t_end / case["disc"]["dt"]))
    case["disc"]["dt"] = t_end / steps
    w = run(orc, case, w0, steps)
    exact = gen.project(lambda x: np.array([gen.entropy_wave_exact(x, t_end)]), E, order_p, 0.0, 1.0)[:, 0, :]
    err = w[:, 0, :] - exact
    M = order_p + 1
    # L2 norm through the orthogonality of the modes: int P_j^2 = 2/(2j+1)
    return math.sqrt(np.sum(err**2 * (2.0 / (2 * np.arange(M) + 1))[None, :]) * 0.5 / E)


@pytest.mark.parametrize("order_p", [1, 2])
@pytest.mark.parametrize("mode", ["sync", "saa"])
def test_design_order_on_the_exact_entropy_wave(orc, order_p, mode):
    """N_p + 1 order on an exact Euler solution, kept under delays with AT order N_p + 1 (Eq. (8))."""
    Es = [16, 32, 64]
    errs = [entropy_error(orc, E, order_p, mode, 0) for E in Es]
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > order_p + 1 - 0.3, (errs, rates)


def test_plain_delayed_flux_loses_accuracy(orc):
    """With q = 1 (the plain delayed flux) the error is far larger and the order drops.

    Its O(dt) error sits at the 8 PE interfaces only, so the L2 rate is about 3/2."""
    Es = [16, 32, 64]
    at = [entropy_error(orc, E, 2, "saa", 0) for E in Es]
    plain = [entropy_error(orc, E, 2, "saa", 1) for E in Es]
    rate_plain = math.log2(plain[-2] / plain[-1])
    rate_at = math.log2(at[-2] / at[-1])
    assert plain[-1] > 10 * at[-1]
    assert rate_plain < 2.0 and rate_at > 2.7


def test_error_grows_linearly_with_the_number_of_pes(orc):
    """Sec. 5.1: the AT error scales with the number of PEs (ensemble over seeds)."""
    E, steps = 128, 120
    case, w0 = gen.case_c0(E=E, n_pe=2, mode="sync", k_pre=0.0)
    ref = run(orc, case, w0, steps)
    means = []
    Ps = [2, 4, 8, 16]
    for P in Ps:
        errs = []
        for seed in range(8):
            c2, _ = gen.case_c0(E=E, n_pe=P, mode="saa", k_pre=0.0, seed=100 + seed)
            errs.append(np.abs(run(orc, c2, w0, steps)[:, 0, 0] - ref[:, 0, 0]).mean())
        means.append(np.mean(errs))
    slope = np.polyfit(np.log(Ps), np.log(means), 1)[0]
    assert 0.7 < slope < 1.3, (means, slope)


def test_delay_moments_order_the_error(orc):
    """Sec. 5.1: larger delay moments give larger error (set-3 < set-2 < set-1 by mean delay)."""
    E, steps = 96, 100
    case, w0 = gen.case_c0(E=E, n_pe=8, mode="sync", k_pre=0.0, cfl=0.1)
    ref = run(orc, case, w0, steps)
    out = []
    for pmf in [(0.8, 0.1, 0.1), (0.5, 0.3, 0.2), (0.3, 0.4, 0.3)]:
        errs = []
        for seed in range(6):
            c2, _ = gen.case_c0(E=E, n_pe=8, mode="saa", k_pre=0.0, seed=7 + seed, pmf=pmf, cfl=0.1)
            errs.append(np.abs(run(orc, c2, w0, steps)[:, 0, 0] - ref[:, 0, 0]).mean())
        out.append(np.mean(errs))
    assert out[0] < out[1] < out[2], out


@pytest.mark.parametrize("e_act,q_heat", [(0.0, 0.0), (3.0, 0.0)])
def test_zero_d_reactor_closed_form(orc, e_act, q_heat):
    """Uniform state, u = 0, no heat release: rho Y_R = rho Y0 exp(-K exp(-Ea/T) t), T = p/rho."""
    K, T, t_end = 5.0, 1.25, 0.4
    case, _ = gen.case_c0(E=8, n_pe=2, mode="sync")
    case["physics"].update(k_pre=K, e_act=e_act, q_heat=q_heat)
    steps = 400
    case["disc"]["dt"] = t_end / steps
    rho, p = 0.8, 0.8 * T
    w0 = np.zeros((8, 5, 3))
    w0[:, :, 0] = gen.onestep_conserved(rho, 0.0, p, 1.0, case["physics"])[:, None].T
    w = run(orc, case, w0, steps)
    exact = rho * math.exp(-K * math.exp(-e_act / T) * t_end)
    assert abs(w[0, 3, 0] - exact) < 1e-8 * rho
    np.testing.assert_allclose(w[:, 3, 0], w[0, 3, 0], rtol=1e-15)
    assert np.all(np.abs(w[:, :, 1:]) < 1e-15)


def test_rankine_hugoniot_shock_speed(orc):
    """A pressure-ratio-30 shock (gamma = 1.2, no reaction) travels at the Rankine-Hugoniot speed."""
    E, length, x0 = 256, 16.0, 4.0
    case, w0 = gen.case_c2(E=E, order_p=2, length=length, shock_x=x0, n_pe=4, mode="sync", k_pre=0.0,
                           cfl=0.4)
    case["physics"]["q_heat"] = 0.0
    rho2, u2, p2, s = gen.rh_post_shock(1.2, 30.0)
    phys = case["physics"]

    def fn(x):
        left = x < x0
        return gen.onestep_conserved(np.where(left, rho2, 1.0), np.where(left, u2, 0.0),
                                     np.where(left, p2, 1.0), 1.0, phys)

    w0 = gen._fix_density_modes(gen.project(fn, E, 2, 0.0, length))
    t_end = 1.2
    steps = int(math.ceil(t_end / case["disc"]["dt"]))
    case["disc"]["dt"] = t_end / steps
    w = run(orc, case, w0, steps)
    rho = w[:, 0, 0]
    u = w[:, 1, 0] / rho
    p = 0.2 * (w[:, 2, 0] - 0.5 * rho * u * u)
    x = (np.arange(E) + 0.5) * length / E
    i = np.where(p > 0.5 * (p2 + 1.0))[0].max()
    xs = x[i] + (p[i] - 0.5 * (p2 + 1)) / (p[i] - p[i + 1]) * (x[i + 1] - x[i])
    dx = length / E
    assert abs(xs - (x0 + s * t_end)) < 2 * dx, (xs, x0 + s * t_end)
    plateau = (x > x0 + s * t_end - 3.0) & (x < x0 + s * t_end - 1.0)
    # post-shock plateau: start-up noise of a strong moving shock stays at the percent level
    assert abs(p[plateau].mean() - p2) < 5e-3 * p2 and abs(rho[plateau].mean() - rho2) < 5e-3 * rho2
    np.testing.assert_allclose(p[plateau], p2, rtol=0.05)
    # jump condition s [w] = [f] on the measured plateau values
    assert abs(s * (rho[plateau].mean() - 1.0) - rho[plateau].mean() * u[plateau].mean()) < 1e-2 * rho2 * u2


def test_flux_consistency(orc):
    rng = np.random.default_rng(0)
    for flux in ("rusanov", "hllc"):
        case, _ = gen.case_c2(E=16, order_p=2, length=16.0, n_pe=2, k_pre=1.0)
        case["disc"]["flux"] = flux
        cfg = orc.Config(case)
        for _ in range(20):
            w = np.array(gen.onestep_conserved(np.array(rng.uniform(0.5, 5)), np.array(rng.uniform(-3, 3)),
                                               np.array(rng.uniform(0.5, 30)), np.array(rng.uniform(0, 1)),
                                               case["physics"]), dtype=float)
            f = orc.call_vec("or_conv_flux", cfg, w, nout=5)
            fh = orc.call_vec("or_num_flux", cfg, w, w, nout=5)
            if flux == "rusanov":
                np.testing.assert_array_equal(fh, f)
            else:
                np.testing.assert_allclose(fh, f, rtol=1e-14, atol=1e-14 * np.abs(f).max())


def test_hllc_keeps_a_stationary_contact(orc):
    case, _ = gen.case_c2(E=16, order_p=2, length=16.0, n_pe=2, k_pre=1.0)
    cfg = orc.Config(case)
    wl = np.array(gen.onestep_conserved(np.array(3.0), np.array(0.0), np.array(2.0), np.array(1.0), case["physics"]), float)
    wr = np.array(gen.onestep_conserved(np.array(0.5), np.array(0.0), np.array(2.0), np.array(0.0), case["physics"]), float)
    fh = orc.call_vec("or_num_flux", cfg, wl, wr, nout=5)
    np.testing.assert_allclose(fh, [0, 2.0, 0, 0, 0], atol=1e-14)
    case["disc"]["flux"] = "rusanov"
    fr = orc.call_vec("or_num_flux", orc.Config(case), wl, wr, nout=5)
    assert abs(fr[0]) > 0.1, "Rusanov smears the contact; HLLC does not"
