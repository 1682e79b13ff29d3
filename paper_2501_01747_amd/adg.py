"""ctypes binding of the ADG C ABI (include/adg.h): argument marshalling only.

Every function here calls the identically named entry point of ``libadg.so``;
all arithmetic runs in the HIP kernels.  PyTorch provides the device workspace
and the stream.  The module raises ``ImportError`` when the library is missing:
there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libadg.so")

ADG_OK, ADG_ERR_ARG, ADG_ERR_NOMEM, ADG_ERR_HIP, ADG_ERR_STATE, ADG_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5
ONESTEP, DETAILED = 0, 1
PERIODIC, TRANSMISSIVE = 0, 1
RUSANOV, HLLC = 0, 1
SYNC, CAA, SAA, SCHEDULE = 0, 1, 2, 3
HOST, DEVICE = 0, 1
FP64, MIXED_FP32, MIXED_BF16 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "mixed": MIXED_FP32, "bf16": MIXED_BF16}
KXRCF, MINMOD, ALL_CELLS = 0, 1, 2
AT_TEMPORAL, AT_HYBRID = 0, 1
SSPRK3, RK2, LSERK4 = 0, 1, 2
PROFILE_CLASSES = ("stage",)
BATCH_PROFILE_CLASSES = ("detailed_stage", "onestep_stage")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
_lib = C.CDLL(LIB_PATH)


class Mechanism(C.Structure):
    _fields_ = [
        ("n_species", C.c_int32), ("n_reactions", C.c_int32),
        ("W", C.POINTER(C.c_double)), ("nasa7", C.POINTER(C.c_double)),
        ("nu_f", C.POINTER(C.c_int32)), ("nu_r", C.POINTER(C.c_int32)),
        ("A", C.POINTER(C.c_double)), ("b", C.POINTER(C.c_double)), ("Ea", C.POINTER(C.c_double)),
        ("Ru", C.c_double), ("p_ref", C.c_double),
        ("mu_ref", C.c_double), ("T_ref", C.c_double), ("mu_exp", C.c_double), ("prandtl", C.c_double),
        ("T_guess", C.c_double),
    ]


class Physics(C.Structure):
    _fields_ = [
        ("model", C.c_int32), ("n_species", C.c_int32), ("viscous", C.c_int32),
        ("gamma", C.c_double), ("q_heat", C.c_double), ("e_act", C.c_double), ("k_pre", C.c_double),
        ("mech", C.POINTER(Mechanism)),
    ]


class Discretization(C.Structure):
    _fields_ = [
        ("order_p", C.c_int32), ("n_quad", C.c_int32), ("n_elem", C.c_int32),
        ("x_left", C.c_double), ("x_right", C.c_double),
        ("bc", C.c_int32), ("flux", C.c_int32), ("limiter", C.c_int32),
        ("indicator", C.c_int32), ("tvb_m", C.c_double),
        ("weno_gamma", C.c_double * 3), ("weno_eps", C.c_double),
        ("dt", C.c_double), ("rk", C.c_int32), ("precision", C.c_int32),
    ]


class Async(C.Structure):
    _fields_ = [
        ("n_pe", C.c_int32), ("pe_offsets", C.POINTER(C.c_int32)),
        ("mode", C.c_int32), ("L", C.c_int32), ("pmf", C.POINTER(C.c_double)),
        ("seed", C.c_uint64),
        ("schedule", C.POINTER(C.c_int8)), ("schedule_steps", C.c_int32),
        ("at_order", C.c_int32), ("at_stencil", C.c_int32),
    ]


_P = C.POINTER
_sig = {
    "adg_workspace_bytes": (C.c_size_t, [_P(Physics), _P(Discretization), _P(Async)]),
    "adg_create": (C.c_int32, [_P(Physics), _P(Discretization), _P(Async), C.c_void_p, C.c_size_t,
                               C.c_void_p, _P(C.c_void_p)]),
    "adg_create_noalloc": (C.c_int32, [_P(Physics), _P(Discretization), _P(Async), C.c_void_p, _P(C.c_void_p)]),
    "adg_set_state": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32]),
    "adg_step": (C.c_int32, [C.c_void_p, C.c_int32]),
    "adg_get_state": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32]),
    "adg_sync": (C.c_int32, [C.c_void_p]),
    "adg_get_flags": (C.c_int32, [C.c_void_p, _P(C.c_int8), _P(C.c_int64)]),
    "adg_step_count": (C.c_int64, [C.c_void_p]),
    "adg_n_interfaces": (C.c_int32, [C.c_void_p]),
    "adg_profile": (C.c_int32, [C.c_void_p, C.c_int32, _P(C.c_double), _P(C.c_int64), C.c_int32]),
    "adg_set_graph": (C.c_int32, [C.c_void_p, C.c_int32]),
    "adg_graph_replays": (C.c_int64, [C.c_void_p]),
    "adg_set_kernel_config": (C.c_int32, [C.c_void_p, C.c_int32]),
    "adg_autotune": (C.c_int32, [C.c_void_p, C.c_int32, _P(C.c_int32)]),
    "adg_destroy": (None, [C.c_void_p]),
    "adg_last_error": (C.c_char_p, [C.c_void_p]),
    "adg_batch_header_bytes": (C.c_size_t, [C.c_int32, C.c_int64]),
    "adg_batch_instance_bytes": (C.c_size_t, [_P(Physics), _P(Discretization), _P(Async)]),
    "adg_batch_create": (C.c_int32, [C.c_int32, C.c_int64, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                                     _P(C.c_void_p)]),
    "adg_batch_add": (C.c_int32, [C.c_void_p, _P(Physics), _P(Discretization), _P(Async), C.c_void_p, C.c_int64,
                                  C.c_int32, C.c_int64, _P(C.c_int32)]),
    "adg_batch_remove": (C.c_int32, [C.c_void_p, C.c_int32]),
    "adg_batch_step": (C.c_int32, [C.c_void_p, C.c_int32]),
    "adg_batch_poll": (C.c_int32, [C.c_void_p, _P(C.c_int64), _P(C.c_int32)]),
    "adg_batch_get_state": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_int32]),
    "adg_batch_set_graph": (C.c_int32, [C.c_void_p, C.c_int32]),
    "adg_batch_profile": (C.c_int32, [C.c_void_p, C.c_int32, _P(C.c_double), _P(C.c_int64), C.c_int32]),
    "adg_batch_autotune": (C.c_int32, [C.c_void_p, C.c_int32, _P(C.c_int32)]),
    "adg_batch_set_kernel_config": (C.c_int32, [C.c_void_p, C.c_int32]),
    "adg_batch_set_group_streams": (C.c_int32, [C.c_void_p, C.c_int32]),
    "adg_batch_active": (C.c_int32, [C.c_void_p]),
    "adg_batch_free_bytes": (C.c_int64, [C.c_void_p]),
    "adg_batch_destroy": (None, [C.c_void_p]),
    "adg_batch_last_error": (C.c_char_p, [C.c_void_p]),
}
for _name, (_res, _args) in _sig.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args
    globals()[_name] = _fn

EXPORTED = tuple(_sig)


class AdgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ADG error {code}: {msg}")
        self.code = code


class Problem:
    """ABI structs built from a case dictionary; keeps the arrays they point to alive."""

    def __init__(self, case: dict):
        self._keep = []
        phys, disc, asy = case["physics"], case["disc"], case["async"]
        p = Physics()
        p.model = DETAILED if phys["model"] == "detailed" else ONESTEP
        p.n_species = int(phys["n_species"])
        p.viscous = int(phys.get("viscous", 0))
        p.gamma = float(phys.get("gamma", 1.4))
        p.q_heat = float(phys.get("q_heat", 0.0))
        p.e_act = float(phys.get("e_act", 0.0))
        p.k_pre = float(phys.get("k_pre", 0.0))
        if p.model == DETAILED:
            m = phys["mech"]
            mc = Mechanism()
            mc.n_species = int(m["n_species"])
            mc.n_reactions = int(m["n_reactions"])
            mc.W, mc.nasa7 = self._d(m["W"]), self._d(m["nasa7"])
            mc.nu_f, mc.nu_r = self._i(m["nu_f"]), self._i(m["nu_r"])
            mc.A, mc.b, mc.Ea = self._d(m["A"]), self._d(m["b"]), self._d(m["Ea"])
            mc.Ru, mc.p_ref = float(m["Ru"]), float(m["p_ref"])
            mc.mu_ref, mc.T_ref, mc.mu_exp = float(m["mu_ref"]), float(m["T_ref"]), float(m["mu_exp"])
            mc.prandtl, mc.T_guess = float(m["prandtl"]), float(m["T_guess"])
            self._keep.append(mc)
            p.mech = C.pointer(mc)
        d = Discretization()
        d.order_p = int(disc["order_p"])
        d.n_quad = int(disc.get("n_quad", 0))
        d.n_elem = int(disc["n_elem"])
        d.x_left, d.x_right = float(disc["x_left"]), float(disc["x_right"])
        d.bc = TRANSMISSIVE if disc.get("bc", "periodic") == "transmissive" else PERIODIC
        d.flux = HLLC if disc.get("flux", "rusanov") == "hllc" else RUSANOV
        d.limiter = int(disc.get("limiter", 0))
        d.indicator = {"kxrcf": KXRCF, "minmod": MINMOD, "all": ALL_CELLS}[disc.get("indicator", "kxrcf")]
        d.tvb_m = float(disc.get("tvb_m", 0.0))
        g = disc.get("weno_gamma", (0.001, 0.998, 0.001))
        d.weno_gamma[0], d.weno_gamma[1], d.weno_gamma[2] = g
        d.weno_eps = float(disc.get("weno_eps", 1e-6))
        d.dt = float(disc["dt"])
        d.rk = {"ssprk3": SSPRK3, "rk2": RK2, "lserk4": LSERK4}[disc.get("rk", "ssprk3")]
        d.precision = PRECISIONS[disc.get("precision", "fp64")]
        a = Async()
        a.n_pe = int(asy["n_pe"])
        if asy.get("pe_offsets") is not None:
            a.pe_offsets = self._i(asy["pe_offsets"])
        a.mode = {"sync": SYNC, "caa": CAA, "saa": SAA, "schedule": SCHEDULE}[asy.get("mode", "sync")]
        a.L = int(asy.get("L", 1))
        if asy.get("pmf") is not None:
            a.pmf = self._d(asy["pmf"])
        a.seed = int(asy.get("seed", 0)) & (2**64 - 1)
        if asy.get("schedule") is not None:
            sch = np.ascontiguousarray(asy["schedule"], dtype=np.int8)
            self._keep.append(sch)
            a.schedule = sch.ctypes.data_as(C.POINTER(C.c_int8))
            a.schedule_steps = int(sch.shape[0])
        a.at_order = int(asy.get("at_order", 0))
        a.at_stencil = {"temporal": AT_TEMPORAL, "hybrid": AT_HYBRID}[asy.get("at_stencil", "temporal")]
        self.phys, self.disc, self.asyn = p, d, a
        self.E = d.n_elem
        self.V = 3 + p.n_species
        self.M = d.order_p + 1

    def _d(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        self._keep.append(x)
        return x.ctypes.data_as(C.POINTER(C.c_double))

    def _i(self, x):
        x = np.ascontiguousarray(x, dtype=np.int32)
        self._keep.append(x)
        return x.ctypes.data_as(C.POINTER(C.c_int32))

    def workspace_bytes(self) -> int:
        return int(adg_workspace_bytes(C.byref(self.phys), C.byref(self.disc), C.byref(self.asyn)))


class Solver:
    """One ADG problem on the current HIP device: torch owns the workspace, the
    library runs every step on the current torch stream."""

    def __init__(self, case: dict, device: str = "cuda", noalloc: bool = False):
        """noalloc: place the solver in the library's static device scratch (adg_create_noalloc)
        instead of a torch workspace."""
        import torch

        self.problem = Problem(case)
        h = C.c_void_p()
        if noalloc:
            self.workspace = None
            self.stream = torch.cuda.current_stream(torch.device(device))
            rc = adg_create_noalloc(C.byref(self.problem.phys), C.byref(self.problem.disc),
                                    C.byref(self.problem.asyn), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        else:
            nbytes = self.problem.workspace_bytes()
            if nbytes == 0:
                raise AdgError(ADG_ERR_ARG, "invalid problem description")
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
            base = self.workspace.data_ptr()
            self._ws_ptr = (base + 255) & ~255
            self.stream = torch.cuda.current_stream(self.workspace.device)
            rc = adg_create(C.byref(self.problem.phys), C.byref(self.problem.disc), C.byref(self.problem.asyn),
                            C.c_void_p(self._ws_ptr), C.c_size_t(nbytes), C.c_void_p(self.stream.cuda_stream),
                            C.byref(h))
        if rc != ADG_OK:
            raise AdgError(rc, adg_last_error(None).decode())
        self.h = h
        self.shape = (self.problem.E, self.problem.V, self.problem.M)

    def _check(self, rc):
        if rc != ADG_OK:
            raise AdgError(rc, adg_last_error(self.h).decode())

    def set_state(self, w):
        import torch

        if isinstance(w, torch.Tensor):
            assert w.is_cuda and w.dtype == torch.float64 and tuple(w.shape) == self.shape
            w = w.contiguous()
            self._check(adg_set_state(self.h, C.c_void_p(w.data_ptr()), w.numel(), DEVICE))
        else:
            w = np.ascontiguousarray(w, dtype=np.float64)
            assert w.shape == self.shape, (w.shape, self.shape)
            self._check(adg_set_state(self.h, w.ctypes.data_as(C.c_void_p), w.size, HOST))

    def step(self, n: int = 1):
        self._check(adg_step(self.h, int(n)))

    def state(self) -> np.ndarray:
        w = np.empty(self.shape)
        self._check(adg_get_state(self.h, w.ctypes.data_as(C.c_void_p), w.size, HOST))
        return w

    def state_device(self, out):
        self._check(adg_get_state(self.h, C.c_void_p(out.data_ptr()), out.numel(), DEVICE))

    def sync(self):
        self._check(adg_sync(self.h))

    def flags(self):
        f = np.empty(self.problem.E, dtype=np.int8)
        tot = C.c_int64()
        self._check(adg_get_flags(self.h, f.ctypes.data_as(C.POINTER(C.c_int8)), C.byref(tot)))
        return f, int(tot.value)

    def step_count(self) -> int:
        return int(adg_step_count(self.h))

    @property
    def n_interfaces(self) -> int:
        return int(adg_n_interfaces(self.h))

    def set_graph(self, steps_per_graph: int):
        self._check(adg_set_graph(self.h, int(steps_per_graph)))

    @property
    def graph_replays(self) -> int:
        return int(adg_graph_replays(self.h))

    def autotune(self, n_reps: int = 20) -> int:
        """Pick the stage kernel's work decomposition by timing (state unchanged)."""
        c = C.c_int32(0)
        self._check(adg_autotune(self.h, int(n_reps), C.byref(c)))
        return c.value

    def set_kernel_config(self, config: int):
        """Use stage-kernel work decomposition `config` (adg_autotune's numbering)."""
        self._check(adg_set_kernel_config(self.h, int(config)))

    def profile(self, n_steps: int) -> dict:
        k = len(PROFILE_CLASSES)
        ms = (C.c_double * k)()
        cnt = (C.c_int64 * k)()
        self._check(adg_profile(self.h, int(n_steps), ms, cnt, k))
        return {name: (ms[i], int(cnt[i])) for i, name in enumerate(PROFILE_CLASSES)}

    def close(self):
        if getattr(self, "h", None):
            adg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent instances advanced together (adg_batch_*): torch owns
    the workspace (header + heap of ``heap_bytes``), the library places
    instances in it and runs every step on the current torch stream."""

    def __init__(self, max_instances: int, max_elements: int, heap_bytes: int, precision: str = "fp64",
                 device: str = "cuda"):
        import torch

        prec = PRECISIONS[precision]
        hdr = int(adg_batch_header_bytes(int(max_instances), int(max_elements)))
        if hdr == 0:
            raise AdgError(ADG_ERR_ARG, "invalid batch capacity")
        nbytes = hdr + int(heap_bytes)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        self._ws_ptr = (self.workspace.data_ptr() + 255) & ~255
        self.stream = torch.cuda.current_stream(self.workspace.device)
        h = C.c_void_p()
        rc = adg_batch_create(int(max_instances), int(max_elements), prec, C.c_void_p(self._ws_ptr),
                              C.c_size_t(nbytes), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != ADG_OK:
            raise AdgError(rc, "adg_batch_create failed")
        self.h = h
        self.max_instances = int(max_instances)
        self.shapes = {}

    @staticmethod
    def instance_bytes(case: dict) -> int:
        p = Problem(case)
        return int(adg_batch_instance_bytes(C.byref(p.phys), C.byref(p.disc), C.byref(p.asyn)))

    def _check(self, rc):
        if rc != ADG_OK:
            raise AdgError(rc, adg_batch_last_error(self.h).decode())

    def add(self, case: dict, w0, n_steps: int = 0) -> int:
        """Admit an instance; raises AdgError with code ADG_ERR_NOMEM when it does not fit."""
        p = Problem(case)
        shape = (p.E, p.V, p.M)
        slot = C.c_int32(-1)
        import torch

        if isinstance(w0, torch.Tensor):
            assert w0.is_cuda and w0.dtype == torch.float64 and tuple(w0.shape) == shape
            w0 = w0.contiguous()
            rc = adg_batch_add(self.h, C.byref(p.phys), C.byref(p.disc), C.byref(p.asyn), C.c_void_p(w0.data_ptr()),
                               w0.numel(), DEVICE, int(n_steps), C.byref(slot))
        else:
            w = np.ascontiguousarray(w0, dtype=np.float64)
            assert w.shape == shape, (w.shape, shape)
            rc = adg_batch_add(self.h, C.byref(p.phys), C.byref(p.disc), C.byref(p.asyn),
                               w.ctypes.data_as(C.c_void_p), w.size, HOST, int(n_steps), C.byref(slot))
        self._check(rc)
        self.shapes[slot.value] = shape
        return slot.value

    def remove(self, slot: int):
        self._check(adg_batch_remove(self.h, int(slot)))
        self.shapes.pop(slot, None)

    def step(self, n: int = 1):
        self._check(adg_batch_step(self.h, int(n)))

    def poll(self):
        """(steps, state_err) per slot; steps is -1 for empty slots."""
        st = np.empty(self.max_instances, dtype=np.int64)
        er = np.empty(self.max_instances, dtype=np.int32)
        self._check(adg_batch_poll(self.h, st.ctypes.data_as(C.POINTER(C.c_int64)),
                                   er.ctypes.data_as(C.POINTER(C.c_int32))))
        return st, er

    def state(self, slot: int) -> np.ndarray:
        w = np.empty(self.shapes[slot])
        self._check(adg_batch_get_state(self.h, int(slot), w.ctypes.data_as(C.c_void_p), w.size, HOST))
        return w

    def state_device(self, slot: int, out):
        self._check(adg_batch_get_state(self.h, int(slot), C.c_void_p(out.data_ptr()), out.numel(), DEVICE))

    def set_graph(self, steps_per_graph: int):
        self._check(adg_batch_set_graph(self.h, int(steps_per_graph)))

    def autotune(self, n_reps: int = 5) -> int:
        """Pick the batched kernel's tile size by timing (state unchanged)."""
        c = C.c_int32(0)
        self._check(adg_batch_autotune(self.h, int(n_reps), C.byref(c)))
        return c.value

    def set_decomposition(self, config: int):
        """Use the batched kernel's work decomposition `config` (autotune's numbering)."""
        self._check(adg_batch_set_kernel_config(self.h, int(config)))

    def set_group_streams(self, streams: int):
        """Spread each stage's group launches over `streams` streams (1..4)."""
        self._check(adg_batch_set_group_streams(self.h, int(streams)))

    def profile(self, n_steps: int) -> dict:
        k = len(BATCH_PROFILE_CLASSES)
        ms = (C.c_double * k)()
        cnt = (C.c_int64 * k)()
        self._check(adg_batch_profile(self.h, int(n_steps), ms, cnt, k))
        return {name: (ms[i], int(cnt[i])) for i, name in enumerate(BATCH_PROFILE_CLASSES)}

    @property
    def active(self) -> int:
        return int(adg_batch_active(self.h))

    @property
    def free_bytes(self) -> int:
        return int(adg_batch_free_bytes(self.h))

    def close(self):
        if getattr(self, "h", None):
            adg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
