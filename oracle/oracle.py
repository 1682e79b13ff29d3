"""ADG oracle: Python access to the plain FP64 C oracle — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  The product path (``paper_2501_01747_amd``)
never touches it.

The oracle follows the paper (arXiv 2501.01747) step by step: Sec. 3.1 DG/LDG,
Sec. 3.2 AT fluxes (Eq. (7)-(8)), Sec. 3.3 (AT-)WENO limiter (Eq. (9)-(11)),
Sec. 4 CAA/SAA delays.  See the header of each C file for its pins.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = ["or_basis.c", "or_physics.c", "or_limiter.c", "or_solver.c"]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

ONESTEP, DETAILED = 0, 1
PERIODIC, TRANSMISSIVE = 0, 1
RUSANOV, HLLC = 0, 1
SYNC, CAA, SAA, SCHEDULE = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle with plain gcc (no contraction, no vectorisation hints)."""
    if force or not os.path.exists(_LIB_PATH):
        srcs = [os.path.join(_HERE, s) for s in _SRC]
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-D_GNU_SOURCE", "-Wall", "-Wno-unused-function", "-o", tmp] + srcs + ["-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class OrConfig(C.Structure):
    _fields_ = [
        ("model", C.c_int32), ("n_species", C.c_int32), ("viscous", C.c_int32),
        ("gamma", C.c_double), ("q_heat", C.c_double), ("e_act", C.c_double), ("k_pre", C.c_double),
        ("n_reactions", C.c_int32),
        ("W", C.POINTER(C.c_double)), ("nasa7", C.POINTER(C.c_double)),
        ("nu_f", C.POINTER(C.c_int32)), ("nu_r", C.POINTER(C.c_int32)),
        ("A", C.POINTER(C.c_double)), ("b", C.POINTER(C.c_double)), ("Ea", C.POINTER(C.c_double)),
        ("Ru", C.c_double), ("p_ref", C.c_double),
        ("mu_ref", C.c_double), ("T_ref", C.c_double), ("mu_exp", C.c_double), ("prandtl", C.c_double),
        ("T_guess", C.c_double),
        ("order_p", C.c_int32), ("n_quad", C.c_int32), ("n_elem", C.c_int32),
        ("x_left", C.c_double), ("x_right", C.c_double),
        ("bc", C.c_int32), ("flux", C.c_int32), ("limiter", C.c_int32),
        ("indicator", C.c_int32), ("tvb_m", C.c_double),
        ("weno_gamma", C.c_double * 3), ("weno_eps", C.c_double),
        ("dt", C.c_double), ("rk", C.c_int32),
        ("n_pe", C.c_int32), ("pe_offsets", C.POINTER(C.c_int32)),
        ("mode", C.c_int32), ("L", C.c_int32), ("pmf", C.POINTER(C.c_double)),
        ("seed", C.c_uint64),
        ("schedule", C.POINTER(C.c_int8)), ("schedule_steps", C.c_int32),
        ("at_order", C.c_int32), ("at_stencil", C.c_int32),
    ]


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = C.CDLL(_LIB_PATH)
        P = C.POINTER
        d, i32, i64, u64 = C.c_double, C.c_int32, C.c_int64, C.c_uint64
        cfgp = P(OrConfig)
        sig = {
            "or_create": (C.c_int, [cfgp, P(d), i32, P(C.c_void_p)]),
            "or_step": (C.c_int, [C.c_void_p, i32]),
            "or_get_state": (C.c_int, [C.c_void_p, P(d)]),
            "or_get_step": (i64, [C.c_void_p]),
            "or_get_flags": (C.c_int, [C.c_void_p, P(C.c_int8)]),
            "or_total_flags": (i64, [C.c_void_p]),
            "or_error": (C.c_char_p, [C.c_void_p]),
            "or_destroy": (None, [C.c_void_p]),
            "or_n_interfaces": (i32, [C.c_void_p]),
            "or_legendre": (d, [C.c_int, d]),
            "or_legendre_deriv": (d, [C.c_int, C.c_int, d]),
            "or_gauss_legendre": (None, [C.c_int, P(d), P(d)]),
            "or_at_coeffs": (C.c_int, [C.c_int, C.c_int, P(d)]),
            "or_at_buffer": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, P(d), P(d)]),
            "or_splitmix64": (u64, [u64]),
            "or_saa_uniform": (d, [u64, i64, i32, i32]),
            "or_raw_delay": (C.c_int, [cfgp, i32, i64, i32]),
            "or_eff_delay": (C.c_int, [cfgp, i32, i64, i32]),
            "or_conv_flux": (C.c_int, [cfgp, P(d), P(d)]),
            "or_source": (C.c_int, [cfgp, P(d), P(d)]),
            "or_num_flux": (C.c_int, [cfgp, P(d), P(d), P(d)]),
            "or_wave_speed": (C.c_int, [cfgp, P(d), P(d), P(d)]),
            "or_temperature": (C.c_int, [cfgp, P(d), P(d), P(C.c_int)]),
            "or_pressure": (C.c_int, [cfgp, P(d), P(d)]),
            "or_species_thermo": (None, [cfgp, C.c_int, d, P(d), P(d), P(d)]),
            "or_reaction_rates": (C.c_int, [cfgp, P(d), P(d), P(d), P(d)]),
            "or_diff_flux": (C.c_int, [cfgp, P(d), P(d), P(d)]),
            "or_char_matrices": (C.c_int, [cfgp, P(d), P(d), P(d)]),
            "or_weno_cell": (C.c_int, [cfgp, P(d), P(d), P(d), P(d)]),
            "or_beta_matrix": (None, [C.c_int, P(d)]),
            "or_translation": (None, [C.c_int, C.c_int, P(d)]),
            "or_rhs_sync": (C.c_int, [cfgp, P(d), P(d)]),
            "or_gradient_sync": (C.c_int, [cfgp, P(d), P(d)]),
            "or_indicator": (C.c_int, [cfgp, P(d), P(d), P(d), C.c_int, C.c_int]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Config:
    """Owns the numpy arrays an ``OrConfig`` points to (keeps them alive)."""

    def __init__(self, case: dict):
        self._keep = []
        c = OrConfig()
        phys, disc, asy = case["physics"], case["disc"], case["async"]
        c.model = DETAILED if phys["model"] == "detailed" else ONESTEP
        c.n_species = int(phys["n_species"])
        c.viscous = int(phys.get("viscous", 0))
        c.gamma = float(phys.get("gamma", 1.4))
        c.q_heat = float(phys.get("q_heat", 0.0))
        c.e_act = float(phys.get("e_act", 0.0))
        c.k_pre = float(phys.get("k_pre", 0.0))
        if c.model == DETAILED:
            mech = phys["mech"]
            c.n_reactions = int(mech["n_reactions"])
            c.W = self._d(mech["W"])
            c.nasa7 = self._d(mech["nasa7"])
            c.nu_f = self._i(mech["nu_f"])
            c.nu_r = self._i(mech["nu_r"])
            c.A = self._d(mech["A"])
            c.b = self._d(mech["b"])
            c.Ea = self._d(mech["Ea"])
            c.Ru = float(mech["Ru"])
            c.p_ref = float(mech["p_ref"])
            c.mu_ref = float(mech["mu_ref"])
            c.T_ref = float(mech["T_ref"])
            c.mu_exp = float(mech["mu_exp"])
            c.prandtl = float(mech["prandtl"])
            c.T_guess = float(mech["T_guess"])
        c.order_p = int(disc["order_p"])
        c.n_quad = int(disc.get("n_quad", 0))
        c.n_elem = int(disc["n_elem"])
        c.x_left = float(disc["x_left"])
        c.x_right = float(disc["x_right"])
        c.bc = TRANSMISSIVE if disc.get("bc", "periodic") == "transmissive" else PERIODIC
        c.flux = HLLC if disc.get("flux", "rusanov") == "hllc" else RUSANOV
        c.limiter = int(disc.get("limiter", 0))
        c.rk = {"ssprk3": 0, "rk2": 1, "lserk4": 2}[disc.get("rk", "ssprk3")]
        c.indicator = {"kxrcf": 0, "minmod": 1, "all": 2}[disc.get("indicator", "kxrcf")]
        c.tvb_m = float(disc.get("tvb_m", 0.0))
        g = disc.get("weno_gamma", (0.001, 0.998, 0.001))
        c.weno_gamma[0], c.weno_gamma[1], c.weno_gamma[2] = g
        c.weno_eps = float(disc.get("weno_eps", 1e-6))
        c.dt = float(disc["dt"])
        c.n_pe = int(asy["n_pe"])
        if asy.get("pe_offsets") is not None:
            c.pe_offsets = self._i(asy["pe_offsets"])
        c.mode = {"sync": SYNC, "caa": CAA, "saa": SAA, "schedule": SCHEDULE}[asy.get("mode", "sync")]
        c.L = int(asy.get("L", 1))
        if asy.get("pmf") is not None:
            c.pmf = self._d(asy["pmf"])
        c.seed = int(asy.get("seed", 0)) & (2**64 - 1)
        if asy.get("schedule") is not None:
            sch = np.ascontiguousarray(asy["schedule"], dtype=np.int8)
            self._keep.append(sch)
            c.schedule = sch.ctypes.data_as(C.POINTER(C.c_int8))
            c.schedule_steps = int(sch.shape[0])
        c.at_order = int(asy.get("at_order", 0))
        c.at_stencil = {"temporal": 0, "hybrid": 1}[asy.get("at_stencil", "temporal")]
        self.c = c
        self.V = 3 + c.n_species
        self.M = c.order_p + 1
        self.E = c.n_elem

    def _d(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        self._keep.append(a)
        return _dptr(a)

    def _i(self, a):
        a = np.ascontiguousarray(a, dtype=np.int32)
        self._keep.append(a)
        return a.ctypes.data_as(C.POINTER(C.c_int32))

    def ref(self):
        return C.byref(self.c)


class OracleSolver:
    """Stateful oracle run: ``step(n)``, ``state()`` in [E][V][M] layout."""

    def __init__(self, case: dict, w0: np.ndarray, max_steps: int):
        self.cfg = Config(case)
        w0 = np.ascontiguousarray(w0, dtype=np.float64)
        assert w0.shape == (self.cfg.E, self.cfg.V, self.cfg.M), w0.shape
        h = C.c_void_p()
        rc = lib().or_create(self.cfg.ref(), _dptr(w0), int(max_steps), C.byref(h))
        if rc != 0:
            raise ValueError(f"or_create failed ({rc})")
        self.h = h

    def step(self, n: int):
        rc = lib().or_step(self.h, int(n))
        if rc != 0:
            raise RuntimeError("oracle step failed: " + lib().or_error(self.h).decode())

    def state(self) -> np.ndarray:
        w = np.empty((self.cfg.E, self.cfg.V, self.cfg.M))
        lib().or_get_state(self.h, _dptr(w))
        return w

    def flags(self) -> np.ndarray:
        f = np.empty(self.cfg.E, dtype=np.int8)
        lib().or_get_flags(self.h, f.ctypes.data_as(C.POINTER(C.c_int8)))
        return f

    def total_flags(self) -> int:
        return int(lib().or_total_flags(self.h))

    @property
    def n(self) -> int:
        return int(lib().or_get_step(self.h))

    @property
    def n_interfaces(self) -> int:
        return int(lib().or_n_interfaces(self.h))

    def close(self):
        if getattr(self, "h", None):
            lib().or_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


def run(case: dict, w0: np.ndarray, n_steps: int) -> np.ndarray:
    s = OracleSolver(case, w0, max_steps=max(n_steps, 1))
    s.step(n_steps)
    w = s.state()
    s.close()
    return w


# ---- thin accessors used by the pin tests -------------------------------------------

def vec(a):
    return _dptr(np.ascontiguousarray(a, dtype=np.float64))


def at_coeffs(q: int, k: int) -> np.ndarray:
    c = np.zeros(q)
    rc = lib().or_at_coeffs(q, k, _dptr(c))
    assert rc == 0
    return c


def gauss_legendre(n: int):
    x, w = np.zeros(n), np.zeros(n)
    lib().or_gauss_legendre(n, _dptr(x), _dptr(w))
    return x, w


def call_vec(name: str, cfg: Config, *arrays, nout: int, out_shape=None):
    """Call ``name(cfg, in..., out)`` for a function with one output vector."""
    ins = [np.ascontiguousarray(a, dtype=np.float64) for a in arrays]
    out = np.zeros(nout if out_shape is None else int(np.prod(out_shape)))
    rc = getattr(lib(), name)(cfg.ref(), *[_dptr(a) for a in ins], _dptr(out))
    if rc not in (None, 0):
        raise ValueError(f"{name} failed ({rc})")
    return out if out_shape is None else out.reshape(out_shape)
