"""Seeded synthetic workloads for the ADG solver (inputs only).

Every function returns plain Python / numpy data: a *case* dictionary (physics,
discretisation and delay-model parameters, in the units the solver expects) and
an initial modal state ``w0`` of shape [E][V][M] (element, conserved variable,
Legendre mode).  The oracle and the HIP library both consume exactly these
arrays; nothing here evaluates the DG operator, the fluxes, the limiter or the
AT combination.

Workload shapes follow the paper's two experiments (arXiv 2501.01747, Sec. 5):
auto-ignition of a lean premixture with a 9-species / 21-reaction mechanism on
a periodic domain with emulated PEs and delays up to 3, and a propagating
detonation with the limiter on a transmissive domain.  The paper's mechanisms,
Cantera and SDToolbox are not available, so the chemistry is a seeded synthetic
mechanism with the same species and reaction counts, and the detonation uses a
one-step Arrhenius model.

Seeds: delays 2501 + config index, mechanism 1747, batch sampler 42, arrivals 7.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from numpy.polynomial import legendre as npleg

RU = 8.31446261815324      # J/(mol K)
P_ATM = 101325.0           # Pa
WENO_GAMMA = (0.001, 0.998, 0.001)
WENO_EPS = 1e-6


# ----------------------------------------------------------------------------- helpers

def project(fn, E: int, order_p: int, x_left: float, x_right: float, n_pts: int | None = None) -> np.ndarray:
    """Modal Legendre coefficients (P_j(1) = 1) of the L2 projection of ``fn`` per element.

    ``fn(x)`` maps an array of positions to an array [V, len(x)] of conserved
    variables.  Uses numpy's Gauss-Legendre rule with 2 (N_p + 3) points.
    """
    M = order_p + 1
    n_pts = n_pts or 2 * (order_p + 3)
    xi, wq = npleg.leggauss(n_pts)
    dx = (x_right - x_left) / E
    centers = x_left + (np.arange(E) + 0.5) * dx
    x = centers[:, None] + 0.5 * dx * xi[None, :]            # [E, n_pts]
    vals = np.asarray(fn(x.reshape(-1)))                     # [V, E*n_pts]
    V = vals.shape[0]
    vals = vals.reshape(V, E, n_pts)
    P = np.stack([npleg.legval(xi, np.eye(M)[j]) for j in range(M)])  # [M, n_pts]
    coef = np.einsum("ven,jn,n->evj", vals, P, wq) * ((2 * np.arange(M) + 1) / 2.0)[None, None, :]
    return np.ascontiguousarray(coef)


def _fix_density_modes(w: np.ndarray) -> np.ndarray:
    """Make rho's modes equal to the sum of the rho Y_i modes (sum Y_i = 1)."""
    w = w.copy()
    w[:, 0, :] = w[:, 3:, :].sum(axis=1)
    return w


def default_dt(cfl: float, dx: float, lam: float, order_p: int) -> float:
    """DG Courant number convention: dt = CFL dx / ((2 N_p + 1) lambda)."""
    return cfl * dx / ((2 * order_p + 1) * lam)


def uniform_pe_offsets(E: int, P: int) -> list[int]:
    return [(p * E) // P for p in range(P + 1)]


# ------------------------------------------------------------------ one-step reactive Euler

def onestep_physics(gamma=1.4, q_heat=1.0, e_act=10.0, k_pre=1e4) -> dict:
    return {"model": "onestep", "n_species": 2, "gamma": gamma, "q_heat": q_heat,
            "e_act": e_act, "k_pre": k_pre, "viscous": 0}


def onestep_conserved(rho, u, p, yr, phys):
    """(rho, rho u, rho E, rho Y_R, rho Y_P) with rho E = rho u^2/2 + p/(g-1) + q rho Y_R."""
    g, q = phys["gamma"], phys["q_heat"]
    rho, u, p, yr = np.broadcast_arrays(rho, u, p, yr)
    return np.stack([rho, rho * u, 0.5 * rho * u * u + p / (g - 1.0) + q * rho * yr,
                     rho * yr, rho * (1.0 - yr)])


def case_c0(E=512, order_p=2, steps=500, n_pe=8, mode="saa", pmf=(0.5, 0.5), seed=2501,
            cfl=0.2, at_order=0, k_pre=1e4):
    """Smooth reacting wave: rho = 1 + 0.2 sin(2 pi x), u = 1, p = 1, Y_R = 1 on periodic [0,1].

    gamma = 1.4, one-step K = 1e4, Ea = 10, q = 1; Rusanov flux, no limiter; SAA delays in {0,1}.
    """
    phys = onestep_physics(1.4, 1.0, 10.0, k_pre)
    dx = 1.0 / E
    lam0 = 1.0 + math.sqrt(1.4 * 1.0 / 0.8)
    dt = default_dt(cfl, dx, lam0, order_p)
    case = {
        "name": "c0_onestep_euler",
        "physics": phys,
        "disc": {"order_p": order_p, "n_quad": 0, "n_elem": E, "x_left": 0.0, "x_right": 1.0,
                 "bc": "periodic", "flux": "rusanov", "limiter": 0, "dt": dt,
                 "weno_gamma": WENO_GAMMA, "weno_eps": WENO_EPS},
        "async": {"n_pe": n_pe, "pe_offsets": None, "mode": mode, "L": len(pmf), "pmf": list(pmf),
                  "seed": seed, "at_order": at_order},
        "steps": steps,
        "cfl": cfl,
    }
    w0 = project(lambda x: onestep_conserved(1.0 + 0.2 * np.sin(2 * np.pi * x), 1.0, 1.0, 1.0, phys),
                 E, order_p, 0.0, 1.0)
    return case, _fix_density_modes(w0)


def entropy_wave_exact(x, t):
    """Exact entropy wave of the non-reacting Euler equations (density only moves)."""
    return 1.0 + 0.2 * np.sin(2 * np.pi * (x - t))


def rh_post_shock(gamma: float, p_ratio: float):
    """Post-shock (rho, u, p) behind a normal shock moving right into (1, 0, 1); and its speed."""
    a1 = math.sqrt(gamma)
    M2 = 1.0 + (p_ratio - 1.0) * (gamma + 1.0) / (2.0 * gamma)
    s = math.sqrt(M2) * a1
    rho2 = (gamma + 1.0) * M2 / ((gamma - 1.0) * M2 + 2.0)
    u2 = s * (1.0 - 1.0 / rho2)
    return rho2, u2, p_ratio, s


def cj_speed(gamma: float, q: float) -> float:
    """Chapman-Jouguet speed of the one-step model into (1, 0, 1)."""
    a = (gamma * gamma - 1.0) * q / 2.0
    return math.sqrt(gamma + a) + math.sqrt(a)


def znd_rate_constant(gamma: float, q: float, e_act: float, half_length: float = 1.0) -> float:
    """Pre-exponential K that gives the CJ detonation a ZND half-reaction length ``half_length``.

    Steady ZND structure in the shock frame (upstream (1, 0, 1), speed D_CJ): the
    Rayleigh line and the Hugoniot with partial heat release give the specific
    volume as a function of the reaction progress; the progress obeys
    u dlam/dx = K (1 - lam) exp(-Ea / T).  Input-shaping only.
    """
    from scipy.integrate import quad

    D = cj_speed(gamma, q)

    def v_of(lam):
        a = D * D * (gamma + 1.0)
        b = 2.0 * gamma * (1.0 + D * D)
        c = 2.0 * gamma + (gamma - 1.0) * D * D + 2.0 * (gamma - 1.0) * q * lam
        disc = max(b * b - 4.0 * a * c, 0.0)
        return (b - math.sqrt(disc)) / (2.0 * a)

    def integrand(lam):
        v = v_of(lam)
        p = 1.0 + D * D * (1.0 - v)
        T = p * v
        return D * v / ((1.0 - lam) * math.exp(-e_act / T))

    val, _ = quad(integrand, 0.0, 0.5)
    return val / half_length


def case_c2(E=8192, order_p=3, steps=200, n_pe=64, mode="saa", L=4, seed=2503, length=256.0,
            shock_x=16.0, cfl=0.1, lam_ref=10.0, k_pre=None, at_order=0):
    """Reacting shock with the limiter: one-step gamma = 1.2, q = 50, Ea = 25, HLLC, KXRCF + AT-WENO.

    Left of ``shock_x``: post-shock state of a pressure-ratio-30 shock (unreacted, Y_R = 1);
    right: (rho, u, p, Y_R) = (1, 0, 1, 1).  Transmissive ends.  Delays uniform in {0..L-1}.
    """
    gamma, q, ea = 1.2, 50.0, 25.0
    if k_pre is None:
        k_pre = znd_rate_constant(gamma, q, ea)
    phys = onestep_physics(gamma, q, ea, k_pre)
    dx = length / E
    dt = default_dt(cfl, dx, lam_ref, order_p)
    rho2, u2, p2, _ = rh_post_shock(gamma, 30.0)

    def fn(x):
        left = x < shock_x
        return onestep_conserved(np.where(left, rho2, 1.0), np.where(left, u2, 0.0),
                                 np.where(left, p2, 1.0), 1.0, phys)

    case = {
        "name": "c2_detonation_weno",
        "physics": phys,
        "disc": {"order_p": order_p, "n_quad": 0, "n_elem": E, "x_left": 0.0, "x_right": length,
                 "bc": "transmissive", "flux": "hllc", "limiter": 1, "dt": dt,
                 "weno_gamma": WENO_GAMMA, "weno_eps": WENO_EPS},
        "async": {"n_pe": n_pe, "pe_offsets": None, "mode": mode, "L": L, "pmf": [1.0 / L] * L,
                  "seed": seed, "at_order": at_order},
        "steps": steps,
        "cfl": cfl,
    }
    w0 = project(fn, E, order_p, 0.0, length)
    return case, _fix_density_modes(w0)


# ------------------------------------------------------------------ synthetic detailed chemistry

_ELEMENT_W = {"A": 1.008e-3, "B": 15.999e-3, "Z": 28.014e-3}
# name, (n_A, n_B, n_Z), class for the formation enthalpy draw (J/mol)
_SPECIES = [
    ("A2", (2, 0, 0), (0.0, 0.0)),
    ("B2", (0, 2, 0), (0.0, 0.0)),
    ("A", (1, 0, 0), (2.0e5, 2.4e5)),
    ("B", (0, 1, 0), (2.2e5, 2.6e5)),
    ("AB", (1, 1, 0), (2.5e4, 4.5e4)),
    ("A2B", (2, 1, 0), (-2.6e5, -2.2e5)),
    ("AB2", (1, 2, 0), (0.5e4, 2.0e4)),
    ("A2B2", (2, 2, 0), (-1.5e5, -1.2e5)),
    ("Z", (0, 0, 1), (0.0, 0.0)),
]
# further species of the same two elements, for mechanisms of more than 9 species
_SPECIES_EXTRA = [
    ("A3", (3, 0, 0), (1.1e5, 1.5e5)),
    ("B3", (0, 3, 0), (1.3e5, 1.6e5)),
    ("A3B", (3, 1, 0), (-0.9e5, -0.5e5)),
    ("AB3", (1, 3, 0), (0.2e5, 0.6e5)),
    ("A2B3", (2, 3, 0), (-1.0e5, -0.6e5)),
    ("A3B2", (3, 2, 0), (-1.6e5, -1.2e5)),
    ("A4", (4, 0, 0), (0.8e5, 1.2e5)),
]
T0 = 298.15


def _nasa_cp_R(a, T):
    return a[0] + a[1] * T + a[2] * T**2 + a[3] * T**3 + a[4] * T**4


def _nasa_h_RT(a, T):
    return a[0] + a[1] * T / 2 + a[2] * T**2 / 3 + a[3] * T**3 / 4 + a[4] * T**4 / 5 + a[5] / T


def _nasa_s_R(a, T):
    return a[0] * np.log(T) + a[1] * T + a[2] * T**2 / 2 + a[3] * T**3 / 3 + a[4] * T**4 / 4 + a[6]


def synthetic_mechanism(seed: int = 1747, n_reactions: int = 21, dt: float = 8.0e-10,
                        p: float = P_ATM, species: list[str] | None = None) -> dict:
    """9 species over two reactive elements and an inert diluent, 21 reversible reactions
    (`species`: other species by name, from the 9 and a few larger molecules of the same elements;
    A2, B2 and Z are needed for the premix).

    * NASA-7 single-range thermo: a1..a5 drawn and redrawn until cp(T) is
      non-decreasing on [200, 4000] K; a6, a7 set the formation enthalpy and the
      standard entropy at 298.15 K drawn per species class.
    * Reactions: atom-balanced 2 <-> 2 and 2 <-> 1 channels among the 8 reactive
      species, drawn without replacement; A log-uniform in [1e6, 1e14] cm^3/(mol s)
      (converted to SI), b uniform in [-1, 2], Ea uniform in [0, 2e5] J/mol.
    * Stiffness rejection: a draw is kept only if every pseudo-first-order rate
      k c_tot^(order-1) (both directions) stays below 0.2/dt on [900, 3000] K at
      pressure p; otherwise the parameters (then the channel) are redrawn.
    """
    rng = np.random.default_rng(seed)
    catalogue = {sp[0]: sp for sp in _SPECIES + _SPECIES_EXTRA}
    table = _SPECIES if species is None else [catalogue[n] for n in species]
    ns = len(table)
    W = np.array([sum(n * _ELEMENT_W[el] for n, el in zip(comp, "ABZ")) for _, comp, _ in table])
    comp = np.array([c for _, c, _ in table], dtype=np.int64)
    nasa = np.zeros((ns, 7))
    Tg = np.linspace(200.0, 4000.0, 400)
    for i, (name, c, (hlo, hhi)) in enumerate(table):
        atoms = sum(c)
        while True:
            a = np.array([rng.uniform(2.5, 3.5) + 0.6 * (atoms - 1),
                          rng.uniform(0.0, 1.5e-3),
                          rng.uniform(-3e-7, 3e-7),
                          rng.uniform(-3e-11, 3e-11),
                          rng.uniform(-1e-15, 1e-15)])
            cp = _nasa_cp_R(a, Tg)
            dcp = a[1] + 2 * a[2] * Tg + 3 * a[3] * Tg**2 + 4 * a[4] * Tg**3
            if np.all(dcp >= 0.0) and cp.max() < 3.0 + 4.0 * atoms:
                break
        hf = rng.uniform(hlo, hhi) if hhi != hlo else hlo
        s0 = rng.uniform(110.0, 150.0) + 25.0 * (atoms - 1)
        nasa[i, :5] = a
        nasa[i, 5] = hf / RU - T0 * (a[0] + a[1] * T0 / 2 + a[2] * T0**2 / 3 + a[3] * T0**3 / 4 + a[4] * T0**4 / 5)
        nasa[i, 6] = s0 / RU - (a[0] * math.log(T0) + a[1] * T0 + a[2] * T0**2 / 2 + a[3] * T0**3 / 3
                                 + a[4] * T0**4 / 4)
    reactive = [i for i in range(ns) if comp[i, 2] == 0]
    channels = []
    pairs = list(itertools.combinations_with_replacement(reactive, 2))
    for lhs in pairs:
        cl = comp[lhs[0]] + comp[lhs[1]]
        for rhs in pairs:
            if sorted(rhs) <= sorted(lhs):
                continue
            if np.array_equal(comp[rhs[0]] + comp[rhs[1]], cl):
                channels.append((lhs, rhs))
        for k in reactive:
            if np.array_equal(comp[k], cl):
                channels.append((lhs, (k,)))
    order = rng.permutation(len(channels))
    Tcheck = np.linspace(900.0, 3000.0, 64)
    nu_f = np.zeros((n_reactions, ns), dtype=np.int32)
    nu_r = np.zeros((n_reactions, ns), dtype=np.int32)
    A = np.zeros(n_reactions)
    b = np.zeros(n_reactions)
    Ea = np.zeros(n_reactions)
    g_RT = np.stack([_nasa_h_RT(nasa[i], Tcheck) - _nasa_s_R(nasa[i], Tcheck) for i in range(ns)])
    ctot = p / (RU * Tcheck)
    limit = 0.2 / dt
    r = 0
    for ch in order:
        if r == n_reactions:
            break
        lhs, rhs = channels[ch]
        nf = np.zeros(ns, dtype=np.int32)
        nr = np.zeros(ns, dtype=np.int32)
        for i in lhs:
            nf[i] += 1
        for i in rhs:
            nr[i] += 1
        dnu = int(nr.sum() - nf.sum())
        dG = ((nr - nf)[:, None] * g_RT).sum(axis=0)
        Kc = np.exp(-dG) * (P_ATM / (RU * Tcheck)) ** dnu
        for _ in range(200):
            A_cgs = 10.0 ** rng.uniform(6.0, 14.0)
            bb = rng.uniform(-1.0, 2.0)
            ea = rng.uniform(0.0, 2.0e5)
            A_si = A_cgs * 1e-6 ** (nf.sum() - 1)
            kf = A_si * Tcheck**bb * np.exp(-ea / (RU * Tcheck))
            kr = kf / Kc
            pf = kf * ctot ** (nf.sum() - 1)
            pr = kr * ctot ** (nr.sum() - 1)
            if np.all(pf < limit) and np.all(pr < limit) and np.all(np.isfinite(pr)):
                nu_f[r], nu_r[r], A[r], b[r], Ea[r] = nf, nr, A_si, bb, ea
                r += 1
                break
    if r < n_reactions:
        raise RuntimeError("synthetic mechanism: not enough admissible channels")
    return {"n_species": ns, "n_reactions": n_reactions, "names": [s[0] for s in table],
            "W": W, "nasa7": nasa, "nu_f": nu_f, "nu_r": nu_r, "A": A, "b": b, "Ea": Ea,
            "Ru": RU, "p_ref": P_ATM, "mu_ref": 1.8e-5, "T_ref": 300.0, "mu_exp": 0.7,
            "prandtl": 0.7, "T_guess": 1500.0, "composition": comp}


def premix_mass_fractions(mech: dict, phi: float = 0.4895, radical_x: float = 1e-4) -> np.ndarray:
    """Fuel A2 : oxidiser B2 : diluent Z = 2 phi : 1 : 3.76 by moles, plus a trace of every radical."""
    names = mech["names"]
    X = np.full(len(names), radical_x)
    X[names.index("A2")] = 2.0 * phi
    X[names.index("B2")] = 1.0
    X[names.index("Z")] = 3.76
    X /= X.sum()
    Y = X * mech["W"]
    return Y / Y.sum()


def _mixture_e(mech, Y, T):
    """Mixture internal energy per mass (input shaping: converts the initial T to rho E)."""
    e = 0.0
    for i in range(mech["n_species"]):
        e = e + Y[i] * RU / mech["W"][i] * T * (_nasa_h_RT(mech["nasa7"][i], T) - 1.0)
    return e


def _frozen_sound_speed(mech, Y, T):
    cp = sum(Y[i] * RU / mech["W"][i] * _nasa_cp_R(mech["nasa7"][i], T) for i in range(mech["n_species"]))
    R = RU * sum(Y[i] / mech["W"][i] for i in range(mech["n_species"]))
    return np.sqrt(cp / (cp - R) * R * T)


def detailed_physics(mech: dict, viscous: int = 1) -> dict:
    return {"model": "detailed", "n_species": mech["n_species"], "viscous": viscous, "mech": mech}


def ignition_state(mech, x, Lx, T_mean=1000.0, T_amp=50.0, phase=0.0, p=P_ATM, u=0.0):
    Y = premix_mass_fractions(mech)
    T = T_mean + T_amp * np.sin(2 * np.pi * x / Lx + phase)
    Wmix = 1.0 / np.sum(Y / mech["W"])
    rho = p * Wmix / (RU * T)
    e = _mixture_e(mech, Y, T)
    rhoE = rho * (e + 0.5 * u * u)
    return np.vstack([rho, rho * u, rhoE, rho[None, :] * Y[:, None]])


def case_c1(E=2048, order_p=3, steps=200, n_pe=16, mode="saa", pmf=(0.3, 0.4, 0.3), seed=2502,
            Lx=0.01, cfl=0.04, at_order=0, mech=None, viscous=1, phase=0.0):
    """Spontaneous-ignition shape: periodic 1 cm, p = 1 atm, u = 0, T = 1000 + 50 sin(2 pi x/Lx) K."""
    dx = Lx / E
    if mech is None:
        mech = synthetic_mechanism(1747, dt=default_dt(cfl, dx, 750.0, order_p))
    Y = premix_mass_fractions(mech)
    lam0 = float(_frozen_sound_speed(mech, Y, 1050.0))
    dt = default_dt(cfl, dx, lam0, order_p)
    case = {
        "name": "c1_ignition_ns",
        "physics": detailed_physics(mech, viscous),
        "disc": {"order_p": order_p, "n_quad": 0, "n_elem": E, "x_left": 0.0, "x_right": Lx,
                 "bc": "periodic", "flux": "rusanov", "limiter": 0, "dt": dt,
                 "weno_gamma": WENO_GAMMA, "weno_eps": WENO_EPS},
        "async": {"n_pe": n_pe, "pe_offsets": None, "mode": mode, "L": len(pmf), "pmf": list(pmf),
                  "seed": seed, "at_order": at_order},
        "steps": steps,
        "cfl": cfl,
    }
    w0 = project(lambda x: ignition_state(mech, x, Lx, phase=phase), E, order_p, 0.0, Lx)
    return case, _fix_density_modes(w0)


def c1_mechanism(cfl=0.04, Lx=0.01):
    """The mechanism of the ignition workload (screened against its time step)."""
    return synthetic_mechanism(1747, dt=default_dt(cfl, Lx / 2048, 750.0, 3))


def diffusive_dt(mech, dx, order_p, c_visc=0.05, T=1050.0):
    """Explicit time-step limit of the LDG diffusion terms: c_visc dx^2 / (D (N_p+1)^4), with D the
    largest of the momentum and heat diffusivities (4/3 nu, nu/Pr) of the premix at T and 1 atm."""
    Y = premix_mass_fractions(mech)
    Wmix = 1.0 / np.sum(Y / mech["W"])
    rho = P_ATM * Wmix / (RU * T)
    mu = mech["mu_ref"] * (T / mech["T_ref"]) ** mech["mu_exp"]
    D = mu / rho * max(4.0 / 3.0, 1.0 / mech["prandtl"])
    return c_visc * dx * dx / (D * (order_p + 1) ** 4)


def case_c3(n_inst=4096, seed=42, e_range=(128, 4096), orders=(2, 3), pe_range=(4, 32), pmf=(0.3, 0.4, 0.3),
            cfl=0.04, Lx=0.01, steps=200, delay_seed=2504, mech=None):
    """Batched ignition instances: element counts log-uniform in e_range, N_p uniform over `orders`,
    PE counts uniform in pe_range, SAA delays k in {0, 1, 2} with `pmf`, IC phase uniform in
    [0, 2 pi).  Every instance uses the ignition mechanism; its time step is the Courant step of its
    own mesh, capped at the step the mechanism was screened against and at the diffusive limit.
    Yields (case, w0)."""
    rng = np.random.default_rng(seed)
    mech = mech if mech is not None else c1_mechanism(cfl, Lx)
    dt_chem = default_dt(cfl, Lx / 2048, 750.0, 3)
    lo, hi = math.log(e_range[0]), math.log(e_range[1])
    for i in range(n_inst):
        E = int(round(math.exp(rng.uniform(lo, hi))))
        order_p = int(rng.choice(orders))
        n_pe = min(int(rng.integers(pe_range[0], pe_range[1] + 1)), E)
        phase = float(rng.uniform(0.0, 2.0 * math.pi))
        case, w0 = case_c1(E=E, order_p=order_p, steps=steps, n_pe=n_pe, pmf=pmf,
                           seed=(delay_seed << 20) + i, Lx=Lx, cfl=cfl, mech=mech, phase=phase)
        case["disc"]["dt"] = min(case["disc"]["dt"], dt_chem, diffusive_dt(mech, Lx / E, order_p))
        case["name"] = "c3_batched_ignition"
        yield case, w0


IGNITION_CFL = {1: 0.1, 2: 0.08, 3: 0.04, 4: 0.01}
SHOCK_CFL = {1: 0.1, 2: 0.05, 3: 0.0125, 4: 0.00625}


def case_shock(E, order_p, n_pe=64, L=4, seed=2503):
    """Reacting shock of the detonation workload at its resolution (dx = 1/32): domain E/32 long,
    shock one sixteenth of the way in (on an element face: E a multiple of 16).  The Courant
    number shrinks with the order (no positivity limiter: the high orders need the margin)."""
    if E % 16:
        raise ValueError("E must be a multiple of 16")
    length = E / 32.0
    return case_c2(E=E, order_p=order_p, n_pe=min(n_pe, E), L=L, seed=seed, length=length,
                   shock_x=length / 16.0, cfl=SHOCK_CFL[order_p])


def c4_requests(n, rate, seed=42, arrival_seed=7, e_range=(256, 65536), steps_range=(100, 2000),
                mech=None, delay_seed=2505):
    """Served stream: Poisson arrivals at `rate` requests/s (all at t = 0 when rate is None), half
    ignition requests (Navier-Stokes, detailed chemistry, 1 cm, 16 PEs, SAA k <= 2) and half reacting
    shocks (one-step Euler with the limiter, 64 PEs, k <= 3); element counts log-uniform in e_range,
    N_p uniform in {1..4}, step counts uniform in steps_range.  Yields dicts with keys
    rid, kind, case, w0, steps, arrival."""
    rng = np.random.default_rng(seed)
    arr = np.random.default_rng(arrival_seed)
    mech = mech if mech is not None else c1_mechanism()
    lo, hi = math.log(e_range[0]), math.log(e_range[1])
    t = 0.0
    for i in range(n):
        if rate:
            t += float(arr.exponential(1.0 / rate))
        kind = "ignition" if rng.random() < 0.5 else "shock"
        E = int(round(math.exp(rng.uniform(lo, hi))))
        order_p = int(rng.integers(1, 5))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        phase = float(rng.uniform(0.0, 2.0 * math.pi)) if kind == "ignition" else 0.0
        if kind == "shock":
            E = max(e_range[0], 16 * int(round(E / 16)))
        case, w0 = c4_request(kind, E, order_p, steps, (delay_seed << 20) + i, mech=mech, phase=phase)
        yield {"rid": i, "kind": kind, "case": case, "w0": w0, "steps": steps, "arrival": t}


def c4_request(kind, E, order_p, steps, seed, mech=None, phase=0.0):
    """One request of the served stream: an ignition solve (Navier-Stokes, detailed chemistry, 1 cm,
    16 PEs, SAA k <= 2, time step capped by the mechanism's screening step and the diffusive limit)
    or a reacting shock (one-step Euler with the limiter at dx = 1/32, 64 PEs, k <= 3; E a multiple
    of 16)."""
    if kind == "ignition":
        mech = mech if mech is not None else c1_mechanism()
        dt_chem = default_dt(0.04, 0.01 / 2048, 750.0, 3)
        case, w0 = case_c1(E=E, order_p=order_p, steps=steps, n_pe=min(16, E), seed=seed,
                           cfl=IGNITION_CFL[order_p], mech=mech, phase=phase)
        case["disc"]["dt"] = min(case["disc"]["dt"], dt_chem, diffusive_dt(mech, 0.01 / E, order_p))
    else:
        case, w0 = case_shock(E, order_p, seed=seed)
    case["name"] = "c4_" + kind
    return case, w0


def dof(case: dict) -> int:
    d = case["disc"]
    return d["n_elem"] * (d["order_p"] + 1) * (3 + case["physics"]["n_species"])
