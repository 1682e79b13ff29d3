"""Pins of the oracle's diffusive flux (Sec. 2, Eq. (2)-(3)): viscous stress, species diffusion and
the enthalpy carried by diffusion, each against linear theory of a small mode on a periodic domain.

Transport reading: mu = mu_ref (T/T_ref)^mu_exp, k = mu cp/Pr, unit Lewis number, so every species has
rho D = k/cp = mu/Pr and the diffusive mass flux is J_i = -rho D dY_i/dx; the heat flux is
-k dT/dx + sum_i h_i J_i and the stress 4/3 mu du/dx (no bulk viscosity).
"""
import math

import numpy as np
import pytest

from workloads import gen


def _rate(a0, a1, t):
    return -math.log(a1 / a0) / t


def _fourier(vals, x, Lx):
    return np.abs(np.sum((vals - vals.mean()) * np.exp(-2j * np.pi * x / Lx)))


def test_acoustic_attenuation(orc):
    """A right-running sound wave in the inert premix decays at k^2/2 (4 nu/3 + (gamma - 1) chi)
    (classical absorption, Stokes hypothesis): pins the 4/3 of the viscous stress."""
    mech = gen.synthetic_mechanism(1747, dt=1e-10)
    mech0 = dict(mech, A=np.zeros_like(mech["A"]))
    Lx, E, order_p, T0 = 1e-4, 16, 3, 1000.0
    Y = gen.premix_mass_fractions(mech0)
    W = 1.0 / np.sum(Y / mech0["W"])
    rho0 = gen.P_ATM * W / (gen.RU * T0)
    cp = sum(Y[i] * gen.RU / mech0["W"][i] * gen._nasa_cp_R(mech0["nasa7"][i], T0) for i in range(9))
    R = gen.RU / W
    gam = cp / (cp - R)
    a0 = math.sqrt(gam * R * T0)
    eps = 1e-5

    def fn(x):
        s = eps * np.sin(2 * np.pi * x / Lx)
        rho = rho0 * (1.0 + s)
        u = a0 * s
        T = T0 * (1.0 + (gam - 1.0) * s)
        e = gen._mixture_e(mech0, Y, T)
        return np.vstack([rho, rho * u, rho * (e + 0.5 * u * u), rho[None, :] * Y[:, None]])

    case, _ = gen.case_c1(E=E, order_p=order_p, mech=mech0, n_pe=2, mode="sync", Lx=Lx)
    w0 = gen._fix_density_modes(gen.project(fn, E, order_p, 0.0, Lx))
    mu = mech0["mu_ref"] * (T0 / mech0["T_ref"]) ** mech0["mu_exp"]
    nu = mu / rho0
    chi = mu / (rho0 * mech0["prandtl"])
    k = 2 * np.pi / Lx
    alpha = 0.5 * k * k * (4.0 / 3.0 * nu + (gam - 1.0) * chi)
    t_end = 0.4 / alpha
    steps = 2000
    case["disc"]["dt"] = t_end / steps
    s = orc.OracleSolver(case, w0, steps + 1)
    s.step(steps)
    w = s.state()
    s.close()
    cfg = orc.Config(case)
    x = (np.arange(E) + 0.5) * Lx / E

    def riemann(ww):
        p = np.array([orc.call_vec("or_pressure", cfg, ww[e, :, 0], nout=1)[0] for e in range(E)])
        u = ww[:, 1, 0] / ww[:, 0, 0]
        return _fourier(p + rho0 * a0 * u, x, Lx)

    rate = _rate(riemann(w0), riemann(w), t_end)
    # with a stress of mu u_x (no 4/3) the rate would be 15 % lower
    assert abs(rate / alpha - 1.0) < 0.01, rate / alpha


def _binary_mechanism(dhf=0.0):
    """Two species of equal molecular weight and equal heat capacity (test input data), an inert
    channel X1 <-> X2 with A = 0; dhf (J/mol) is the formation-enthalpy difference h_2 - h_1."""
    base = gen.synthetic_mechanism(1747, dt=1e-10)
    z = base["names"].index("Z")
    a = base["nasa7"][z].copy()
    nasa = np.stack([a, a])
    nasa[1, 5] += dhf / gen.RU
    W = np.array([base["W"][z], base["W"][z]])
    return {"n_species": 2, "n_reactions": 1, "names": ["X1", "X2"], "W": W, "nasa7": nasa,
            "nu_f": np.array([[1, 0]], dtype=np.int32), "nu_r": np.array([[0, 1]], dtype=np.int32),
            "A": np.zeros(1), "b": np.zeros(1), "Ea": np.zeros(1), "Ru": gen.RU, "p_ref": gen.P_ATM,
            "mu_ref": 1.8e-5, "T_ref": 300.0, "mu_exp": 0.7, "prandtl": 0.7, "T_guess": 1500.0}


def _binary_run(orc, mech, steps=1500, eps=0.05):
    Lx, E, order_p, T0 = 1e-4, 16, 3, 1000.0
    rho0 = gen.P_ATM * mech["W"][0] / (gen.RU * T0)

    def fn(x):
        y1 = 0.5 + eps * np.sin(2 * np.pi * x / Lx)
        Y = np.vstack([y1, 1.0 - y1])
        rho = np.full_like(x, rho0)
        e = sum(Y[i] * gen.RU / mech["W"][i] * T0 * (gen._nasa_h_RT(mech["nasa7"][i], T0) - 1.0) for i in range(2))
        return np.vstack([rho, 0.0 * rho, rho * e, rho[None, :] * Y])

    case = {
        "name": "binary_exchange",
        "physics": gen.detailed_physics(mech, 1),
        "disc": {"order_p": order_p, "n_quad": 0, "n_elem": E, "x_left": 0.0, "x_right": Lx, "bc": "periodic",
                 "flux": "rusanov", "limiter": 0, "dt": 1.0},
        "async": {"n_pe": 2, "pe_offsets": None, "mode": "sync", "L": 1, "pmf": [1.0], "seed": 0, "at_order": 0},
    }
    w0 = gen._fix_density_modes(gen.project(fn, E, order_p, 0.0, Lx))
    mu = mech["mu_ref"] * (T0 / mech["T_ref"]) ** mech["mu_exp"]
    D = mu / (mech["prandtl"] * rho0)
    sigma = D * (2 * np.pi / Lx) ** 2
    t_end = 0.4 / sigma
    case["disc"]["dt"] = t_end / steps
    s = orc.OracleSolver(case, w0, steps + 1)
    s.step(steps)
    w = s.state()
    s.close()
    x = (np.arange(E) + 0.5) * Lx / E
    cfg = orc.Config(case)
    temps = []
    for e in range(E):
        out = np.zeros(1)
        it = orc.C.c_int()
        assert orc.lib().or_temperature(cfg.ref(), orc._dptr(w[e, :, 0].copy()), orc._dptr(out), orc.C.byref(it)) == 0
        temps.append(out[0])
    rate = _rate(_fourier(w0[:, 3, 0], x, Lx), _fourier(w[:, 3, 0], x, Lx), t_end)
    return rate / sigma, np.array(temps), w, T0


def test_binary_species_exchange_decays_at_D_k2(orc):
    """Two species alike in every thermodynamic property: a composition mode is pure diffusion,
    decaying at D k^2 with rho D = mu/Pr (pins the sign and size of J_i = -rho D dY_i/dx)."""
    ratio, T, w, T0 = _binary_run(orc, _binary_mechanism(0.0))
    assert abs(ratio - 1.0) < 0.01, ratio
    assert np.abs(T - T0).max() < 1e-8 * T0
    assert np.abs(w[:, 1, :]).max() < 1e-12 * np.abs(w[:, 0, 0]).max()


@pytest.mark.parametrize("dhf", [-3.0e4, 5.0e4])
def test_enthalpy_carried_by_diffusion_keeps_the_mixture_isothermal(orc, dhf):
    """With different formation enthalpies the exchange mode moves energy; the enthalpy flux
    sum_i h_i J_i in the heat flux carries exactly that energy, so T stays uniform (without it the
    mode would heat or cool the gas by about dhf Y'/(W c_v) ~ 10 K here)."""
    ratio, T, w, T0 = _binary_run(orc, _binary_mechanism(dhf))
    assert abs(ratio - 1.0) < 0.01, ratio
    assert np.abs(T - T0).max() < 1e-6, np.abs(T - T0).max()
