"""Pins of the detailed-chemistry physics (Sec. 2, Eq. (2)-(3)) of the oracle."""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

from workloads import gen


@pytest.fixture(scope="module")
def mech():
    return gen.synthetic_mechanism(1747, dt=1e-10)


def cfg_for(orc, mech, E=8, order_p=1, viscous=1, bc="periodic", **kw):
    case, w0 = gen.case_c1(E=E, order_p=order_p, mech=mech, viscous=viscous, n_pe=2, mode="sync", **kw)
    case["disc"]["bc"] = bc
    return orc.Config(case), case, w0


def thermo(orc, cfg, i, T):
    cp, h, s = (np.zeros(1) for _ in range(3))
    orc.lib().or_species_thermo(cfg.ref(), i, T, orc._dptr(cp), orc._dptr(h), orc._dptr(s))
    return cp[0], h[0], s[0]


def test_nasa_thermo_is_self_consistent(orc, mech):
    """dh/dT = cp and ds/dT = cp/T (h = R T h_RT, s = R s_R), by centred differences."""
    cfg, _, _ = cfg_for(orc, mech)
    for i in range(9):
        for T in (400.0, 1000.0, 2500.0):
            d = 1e-3 * T
            cp, _, _ = thermo(orc, cfg, i, T)
            _, hp, sp = thermo(orc, cfg, i, T + d)
            _, hm, sm = thermo(orc, cfg, i, T - d)
            dh = ((T + d) * hp - (T - d) * hm) / (2 * d)
            ds = (sp - sm) / (2 * d)
            assert abs(dh - cp) < 1e-6 * cp
            assert abs(ds - cp / T) < 1e-6 * cp / T


def state(mech, T, Y=None, rho=0.3, u=0.0):
    Y = gen.premix_mass_fractions(mech) if Y is None else Y
    e = gen._mixture_e(mech, Y, T)
    return np.concatenate([[rho, rho * u, rho * (e + 0.5 * u * u)], rho * Y])


def test_temperature_newton_round_trip(orc, mech):
    cfg, _, _ = cfg_for(orc, mech)
    lib = orc.lib()
    for T in np.linspace(300.0, 3500.0, 17):
        w = state(mech, T, u=37.0)
        out = np.zeros(1)
        it = orc.C.c_int()
        assert lib.or_temperature(cfg.ref(), orc._dptr(w), orc._dptr(out), orc.C.byref(it)) == 0
        assert abs(out[0] - T) < 1e-12 * T
        assert it.value <= 12


def rates(orc, cfg, w, nr=21):
    kf, kr, q = np.zeros(nr), np.zeros(nr), np.zeros(nr)
    assert orc.lib().or_reaction_rates(cfg.ref(), orc._dptr(w), orc._dptr(kf), orc._dptr(kr), orc._dptr(q)) == 0
    return kf, kr, q


def test_production_rates_conserve_mass_and_elements(orc, mech):
    cfg, _, _ = cfg_for(orc, mech)
    rng = np.random.default_rng(5)
    for T in (900.0, 1500.0, 2500.0):
        Y = rng.uniform(0.01, 1.0, size=9)
        Y /= Y.sum()
        w = state(mech, T, Y)
        s = orc.call_vec("or_source", cfg, w, nout=12)
        assert np.all(s[:3] == 0.0)
        scale = np.abs(s[3:]).max()
        assert abs(s[3:].sum()) < 1e-13 * scale
        wdot = s[3:] / mech["W"]
        for el in range(3):
            assert abs(np.dot(mech["composition"][:, el], wdot)) < 1e-12 * np.abs(wdot).max()


def test_arrhenius_parameters_recovered(orc, mech):
    """ln k_f is linear in (1, ln T, 1/T): fitting three temperatures returns (ln A, b, -Ea/Ru)."""
    cfg, _, _ = cfg_for(orc, mech)
    Ts = np.array([800.0, 1300.0, 2100.0, 2900.0])
    lnk = np.array([np.log(rates(orc, cfg, state(mech, T))[0]) for T in Ts])
    X = np.stack([np.ones_like(Ts), np.log(Ts), 1.0 / Ts], axis=1)
    for r in range(21):
        coef, *_ = np.linalg.lstsq(X, lnk[:, r], rcond=None)
        assert abs(coef[0] - math.log(mech["A"][r])) < 1e-8 * max(1, abs(math.log(mech["A"][r])))
        assert abs(coef[1] - mech["b"][r]) < 1e-8
        assert abs(coef[2] + mech["Ea"][r] / gen.RU) < 1e-6 * max(1.0, mech["Ea"][r] / gen.RU)


def test_van_t_hoff(orc, mech):
    """d ln K_c / dT = (Delta H - Delta nu Ru T) / (Ru T^2) with K_c = k_f / k_r."""
    cfg, _, _ = cfg_for(orc, mech)
    nu = (mech["nu_r"] - mech["nu_f"]).astype(float)
    for T in (900.0, 1600.0, 2600.0):
        d = 1e-3 * T
        lnKp = np.log(np.divide(*rates(orc, cfg, state(mech, T + d))[:2]))
        lnKm = np.log(np.divide(*rates(orc, cfg, state(mech, T - d))[:2]))
        h = np.array([thermo(orc, cfg, i, T)[1] for i in range(9)])   # h/(Ru T)
        dH_RT = nu @ h
        expect = (dH_RT - nu.sum(axis=1)) / T
        np.testing.assert_allclose((lnKp - lnKm) / (2 * d), expect, rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("r", [0, 4, 11, 19])
def test_zero_net_rate_at_helmholtz_minimum(orc, mech, r):
    """At fixed T and V the equilibrium composition minimises sum_i n_i (mu_i - Ru T); there
    the oracle's net rate of progress of the reaction vanishes."""
    cfg, _, _ = cfg_for(orc, mech)
    T, V = 1400.0, 1.0
    nu = (mech["nu_r"][r] - mech["nu_f"][r]).astype(float)
    g = np.array([thermo(orc, cfg, i, T)[1] - thermo(orc, cfg, i, T)[2] for i in range(9)])
    n0 = np.full(9, 2.0)

    def F(xi):
        n = n0 + xi * nu
        c = n / V
        return float(np.sum(n * (g + np.log(c * gen.RU * T / gen.P_ATM) - 1.0)))

    lo = max(-(n0[i] / nu[i]) for i in range(9) if nu[i] > 0) + 1e-9
    hi = min(-(n0[i] / nu[i]) for i in range(9) if nu[i] < 0) - 1e-9
    # stationary point of F: dF/dxi = sum_i nu_i (g_i + ln(c_i Ru T / p0)) = 0 (F is convex)
    dF = lambda xi: float(np.sum(nu * (g + np.log((n0 + xi * nu) / V * gen.RU * T / gen.P_ATM))))
    xi = brentq(dF, lo, hi, xtol=1e-15, rtol=1e-15)
    assert F(xi) <= min(F(xi - 1e-6), F(xi + 1e-6))
    n = n0 + xi * nu
    Y = n * mech["W"] / np.sum(n * mech["W"])
    rho = np.sum(n * mech["W"]) / V
    w = state(mech, T, Y, rho=rho)
    kf, kr, q = rates(orc, cfg, w)
    fwd = kf[r] * np.prod((n / V) ** mech["nu_f"][r])
    assert abs(q[r]) < 1e-6 * fwd, (q[r], fwd)


def test_ldg_gradient_is_exact_for_a_global_polynomial(orc, mech):
    """Central traces of a continuous degree-N_p polynomial are exact, so q = dw/dx exactly."""
    order_p, E = 3, 6
    cfg, case, _ = cfg_for(orc, mech, E=E, order_p=order_p, bc="transmissive")
    a = np.random.default_rng(2).normal(size=(12, order_p + 1))
    fn = lambda x: np.array([np.polynomial.polynomial.polyval(x / 0.01, a[v]) for v in range(12)])
    dfn = lambda x: np.array([np.polynomial.polynomial.polyval(x / 0.01, np.polynomial.polynomial.polyder(a[v])) / 0.01
                              for v in range(12)])
    w = gen.project(fn, E, order_p, 0.0, 0.01)
    q = np.zeros_like(w)
    assert orc.lib().or_gradient_sync(cfg.ref(), orc._dptr(w), orc._dptr(q)) == 0
    np.testing.assert_allclose(q, gen.project(dfn, E, order_p, 0.0, 0.01), rtol=1e-9, atol=1e-9 * np.abs(q).max())


def test_thermal_diffusion_decay_rate(orc, mech):
    """A small isobaric temperature mode decays at chi k^2, chi = kappa/(rho cp) = mu/(rho Pr)."""
    mech0 = dict(mech, A=np.zeros_like(mech["A"]))
    Lx, E, order_p = 1e-4, 16, 3
    case, _ = gen.case_c1(E=E, order_p=order_p, mech=mech0, n_pe=2, mode="sync", Lx=Lx)
    eps, T0 = 5.0, 1000.0
    w0 = gen.project(lambda x: gen.ignition_state(mech0, x, Lx, T_mean=T0, T_amp=eps), E, order_p, 0.0, Lx)
    w0 = gen._fix_density_modes(w0)
    rho0 = w0[:, 0, 0].mean()
    Y = gen.premix_mass_fractions(mech0)
    cp = sum(Y[i] * gen.RU / mech0["W"][i] * gen._nasa_cp_R(mech0["nasa7"][i], T0) for i in range(9))
    mu = mech0["mu_ref"] * (T0 / mech0["T_ref"]) ** mech0["mu_exp"]
    chi = mu / (rho0 * mech0["prandtl"])
    sigma = chi * (2 * np.pi / Lx) ** 2
    t_end = 0.4 / sigma
    steps = 1500
    case["disc"]["dt"] = t_end / steps
    s = orc.OracleSolver(case, w0, steps + 1)
    s.step(steps)
    w = s.state()
    x = (np.arange(E) + 0.5) * Lx / E
    cfg = orc.Config(case)
    gam = cp / (cp - gen.RU * np.sum(Y / mech0["W"]))

    def amp(ww):
        # entropy perturbation p'/p - gamma rho'/rho: acoustic modes carry none of it
        rho = ww[:, 0, 0]
        p = np.array([orc.call_vec("or_pressure", cfg, ww[e, :, 0], nout=1)[0] for e in range(E)])
        sig = p / p.mean() - gam * rho / rho.mean()
        return np.abs(np.sum((sig - sig.mean()) * np.exp(-2j * np.pi * x / Lx)))

    rate = -math.log(amp(w) / amp(w0)) / t_end
    assert abs(rate / sigma - 1.0) < 0.01, rate / sigma
