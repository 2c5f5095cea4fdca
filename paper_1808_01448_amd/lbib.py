"""ctypes binding of the gfx950 LB-IB adhesion library (include/lbib.h).

Argument marshalling only: every step of the time loop runs in the library's HIP kernels.
PyTorch provides device memory for the kernel-level entry points and the HIP stream the
simulation is enqueued on.  If the shared library has not been built, importing the
binding's functions raises immediately: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "liblbib.so")

OK, E_INVALID, E_STATE, E_NOMEM, E_DEVICE, E_NUMERIC, E_UNSUPPORTED, E_FULL = 0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "OK", -1: "E_INVALID", -2: "E_STATE", -3: "E_NOMEM", -4: "E_DEVICE", -5: "E_NUMERIC",
                -6: "E_UNSUPPORTED", -7: "E_FULL"}
FP64, FP32, FP16, BF16, FP16_NEQ, BF16_NEQ = 0, 1, 2, 3, 4, 5
POOL_RUNNING, POOL_FINISHED, POOL_FAILED = 0, 1, 2


class LbibError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class LatticeDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("tau", C.c_double), ("re", C.c_double),
                ("drive", C.c_int32), ("precision", C.c_int32), ("seed", C.c_uint64)]


class ParticleDesc(C.Structure):
    _fields_ = [("shape", C.c_int32), ("a_major", C.c_double), ("b_minor", C.c_double), ("xc", C.c_double),
                ("yc", C.c_double), ("theta0", C.c_double), ("rho_p", C.c_double), ("n_markers", C.c_int32)]


class LigandDesc(C.Structure):
    _fields_ = [("rho_l_num", C.c_int32), ("rho_l_den", C.c_int32), ("sigma_hat", C.c_double),
                ("sigma_star_ratio", C.c_double), ("y_cr_hat", C.c_double), ("y_eq_ratio", C.c_double),
                ("k_f", C.c_double), ("k_r0", C.c_double), ("kbt_hat", C.c_double), ("hamaker_hat", C.c_double)]


class ReceptorDesc(C.Structure):
    _fields_ = [("wall", C.c_int32), ("density", C.c_double)]


class ParticleState(C.Structure):
    _fields_ = [("step", C.c_int64), ("xc", C.c_double), ("yc", C.c_double), ("theta", C.c_double),
                ("ux", C.c_double), ("uy", C.c_double), ("omega", C.c_double), ("fx", C.c_double),
                ("fy", C.c_double), ("torque", C.c_double), ("fx_hydro", C.c_double), ("fy_hydro", C.c_double),
                ("m_hydro", C.c_double), ("fx_bond", C.c_double), ("fy_bond", C.c_double), ("m_bond", C.c_double),
                ("fy_wall", C.c_double), ("gap", C.c_double), ("n_bonds", C.c_int32), ("n_probing", C.c_int32)]


STATE_FIELDS = [n for n, _ in ParticleState._fields_]

REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, 3


class RequestResult(C.Structure):
    _fields_ = [("id", C.c_int64), ("state", C.c_int32), ("slot", C.c_int32), ("steps", C.c_int64),
                ("steps_done", C.c_int64), ("bytes", C.c_int64), ("t_arrival", C.c_double), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double), ("final_state", ParticleState)]

_P = C.c_void_p
_D = C.POINTER(C.c_double)
_U8 = C.POINTER(C.c_uint8)
_I64 = C.POINTER(C.c_int64)

_SIGS = {
    "lbib_abi_version": (C.c_int, []),
    "lbib_create": (C.c_int, [C.POINTER(LatticeDesc), _P, C.POINTER(_P)]),
    "lbib_particle_add": (C.c_int, [_P, C.POINTER(ParticleDesc), C.POINTER(C.c_int32)]),
    "lbib_ligands_set": (C.c_int, [_P, C.c_int32, C.POINTER(LigandDesc)]),
    "lbib_receptors_set": (C.c_int, [_P, C.POINTER(ReceptorDesc)]),
    "lbib_init": (C.c_int, [_P]),
    "lbib_step": (C.c_int, [_P, C.c_int64]),
    "lbib_sync": (C.c_int, [_P]),
    "lbib_step_count": (C.c_int, [_P, _I64]),
    "lbib_read_particle": (C.c_int, [_P, C.c_int32, C.POINTER(ParticleState)]),
    "lbib_read_bonds": (C.c_int, [_P, C.c_int32, _U8, _U8, C.c_int32]),
    "lbib_read_markers": (C.c_int, [_P, C.c_int32, _D, _D, C.c_int32]),
    "lbib_read_field": (C.c_int, [_P, C.c_int32, _D, C.c_int64]),
    "lbib_write_populations": (C.c_int, [_P, _D, C.c_int64]),
    "lbib_write_particle": (C.c_int, [_P, C.c_int32, _D]),
    "lbib_write_bonds": (C.c_int, [_P, C.c_int32, _U8, C.c_int32]),
    "lbib_trace_enable": (C.c_int, [_P, C.c_int32, C.c_int64]),
    "lbib_read_trace": (C.c_int, [_P, C.c_int32, C.POINTER(ParticleState), C.c_int64, _I64]),
    "lbib_save": (C.c_int, [_P, _P, _I64]),
    "lbib_load": (C.c_int, [_P, _P, C.c_int64]),
    "lbib_kernel_timing": (C.c_int, [_P, C.c_int32]),
    "lbib_set_overlap": (C.c_int, [_P, C.c_int32]),
    "lbib_set_layout": (C.c_int, [_P, C.c_int32]),
    "lbib_get_layout": (C.c_int, [_P, C.POINTER(C.c_int32)]),
    "lbib_kernel_time": (C.c_int, [_P, C.c_int32, _D, _I64]),
    "lbib_bytes_per_update": (C.c_int, [_P, _I64]),
    "lbib_last_error": (C.c_char_p, [_P]),
    "lbib_destroy": (None, [_P]),
    "lbib_kernel_philox": (C.c_int, [_P, _P, _P, C.c_int64, _P]),
    "lbib_kernel_mls": (C.c_int, [_P, C.c_int64, C.c_int32, C.c_int32, _P, _P, _P, _P, _P]),
    "lbib_kernel_bonds": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, C.c_int32, C.c_int32, _D, C.c_uint64,
                                    C.c_uint32, _P]),
    "lbib_bandwidth_probe": (C.c_int, [C.c_int64, C.c_int32, _P, _D]),
    "lbib_solve_static": (C.c_int, [C.POINTER(LatticeDesc), C.POINTER(ParticleDesc), C.POINTER(LigandDesc),
                                    C.c_int64, _P, _I64, _P, _P, _P]),
    "lbib_pool_create": (C.c_int, [C.c_int32, C.c_int64, C.c_int32, _P, C.POINTER(_P)]),
    "lbib_pool_footprint": (C.c_int, [C.POINTER(LatticeDesc), C.POINTER(ParticleDesc), _I64]),
    "lbib_pool_add": (C.c_int, [_P, C.POINTER(LatticeDesc), C.POINTER(ParticleDesc), C.POINTER(LigandDesc),
                                C.c_int64, C.POINTER(C.c_int32)]),
    "lbib_pool_step": (C.c_int, [_P, C.c_int64]),
    "lbib_pool_poll": (C.c_int, [_P, C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int32)]),
    "lbib_pool_status": (C.c_int, [_P, C.c_int32, _I64, C.POINTER(C.c_int32)]),
    "lbib_pool_read_particle": (C.c_int, [_P, C.c_int32, C.POINTER(ParticleState)]),
    "lbib_pool_read_bonds": (C.c_int, [_P, C.c_int32, _U8, _U8, C.c_int32]),
    "lbib_pool_read_field": (C.c_int, [_P, C.c_int32, C.c_int32, _D, C.c_int64]),
    "lbib_pool_trace_enable": (C.c_int, [_P, C.c_int32, C.c_int64]),
    "lbib_pool_read_trace": (C.c_int, [_P, C.c_int32, C.POINTER(ParticleState), C.c_int64, _I64]),
    "lbib_pool_remove": (C.c_int, [_P, C.c_int32]),
    "lbib_pool_usage": (C.c_int, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), _I64]),
    "lbib_pool_kernel_timing": (C.c_int, [_P, C.c_int32]),
    "lbib_pool_kernel_time": (C.c_int, [_P, C.c_int32, _D, _I64]),
    "lbib_pool_set_config": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32]),
    "lbib_pool_get_config": (C.c_int, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "lbib_pool_autotune": (C.c_int, [_P, C.c_int32, _D]),
    "lbib_pool_last_error": (C.c_char_p, [_P]),
    "lbib_pool_destroy": (None, [_P]),
    "lbib_server_create": (C.c_int, [C.c_int32, C.c_int64, C.c_int32, C.c_int32, C.c_int32, _P, C.POINTER(_P)]),
    "lbib_server_submit": (C.c_int, [_P, C.POINTER(LatticeDesc), C.POINTER(ParticleDesc), C.POINTER(LigandDesc),
                                     C.c_int64, C.c_double, _I64]),
    "lbib_server_progress": (C.c_int, [_P, C.POINTER(C.c_int32)]),
    "lbib_server_take_completed": (C.c_int, [_P, _I64, C.c_int32, C.POINTER(C.c_int32)]),
    "lbib_server_result": (C.c_int, [_P, C.c_int64, C.POINTER(RequestResult)]),
    "lbib_server_release": (C.c_int, [_P, C.c_int64]),
    "lbib_server_set_trace": (C.c_int, [_P, C.c_int64]),
    "lbib_server_read_trace": (C.c_int, [_P, C.c_int64, C.POINTER(ParticleState), C.c_int64, _I64]),
    "lbib_server_read_bonds": (C.c_int, [_P, C.c_int64, _U8, _U8, C.c_int32]),
    "lbib_server_stats": (C.c_int, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), _I64, _I64]),
    "lbib_server_pool": (_P, [_P]),
    "lbib_server_clock": (C.c_double, [_P]),
    "lbib_server_last_error": (C.c_char_p, [_P]),
    "lbib_server_destroy": (None, [_P]),
}
EXPORTED = tuple(_SIGS)

_lib = None


def lib():
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int, handle=None, pool: bool = False, server: bool = False):
    if status != OK:
        L = lib()
        err = L.lbib_server_last_error if server else L.lbib_pool_last_error if pool else L.lbib_last_error
        msg = err(handle)
        raise LbibError(status, msg.decode() if msg else "")


def _stream_ptr(stream):
    if stream is None:
        return None
    return C.c_void_p(int(stream.cuda_stream if hasattr(stream, "cuda_stream") else stream))


def _ptr(t):
    """Device pointer of a torch tensor."""
    return C.c_void_p(t.data_ptr())


def particle_entries(w: dict) -> list:
    """(particle, ligand) descriptor pairs of a workload: the single form ("particle",
    "ligand") or the list form ("particles": [{"particle": ..., "ligand": ...}, ...])."""
    if "particles" in w:
        return [(e["particle"], e["ligand"]) for e in w["particles"]]
    if w.get("particle") is not None:
        return [(w["particle"], w["ligand"])]
    return []


def _lattice_desc(lat: dict) -> LatticeDesc:
    return LatticeDesc(int(lat["nx"]), int(lat["ny"]), float(lat["tau"]), float(lat["re"]), int(lat.get("drive", 0)),
                       int(lat.get("precision", FP64)), int(lat.get("seed", 0)))


def _particle_desc(part: dict) -> ParticleDesc:
    return ParticleDesc(int(part["shape"]), float(part["a_major"]), float(part["b_minor"]), float(part["xc"]),
                        float(part["yc"]), float(part["theta0"]), float(part["rho_p"]), int(part["n_markers"]))


def _ligand_desc(g: dict) -> LigandDesc:
    return LigandDesc(int(g["rho_l_num"]), int(g["rho_l_den"]), float(g["sigma_hat"]), float(g["sigma_star_ratio"]),
                      float(g["y_cr_hat"]), float(g["y_eq_ratio"]), float(g["k_f"]), float(g["k_r0"]),
                      float(g["kbt_hat"]), float(g["hamaker_hat"]))


def _state_dtype() -> np.dtype:
    kinds = {C.c_int64: np.int64, C.c_int32: np.int32, C.c_double: np.float64}
    dt = np.dtype([(n, kinds[t]) for n, t in ParticleState._fields_], align=True)
    assert dt.itemsize == C.sizeof(ParticleState)
    return dt


def _trace_array(buf, count: int) -> np.ndarray:
    """Records as float64 [count, 20] in the field order of STATE_FIELDS."""
    a = np.frombuffer(buf, dtype=_state_dtype(), count=count)
    out = np.empty((count, len(STATE_FIELDS)))
    for c, n in enumerate(STATE_FIELDS):
        out[:, c] = a[n]
    return out


# ----------------------------------------------------------------------------------------
# Simulation handle
# ----------------------------------------------------------------------------------------

class Sim:
    """One simulation: lattice, at most one particle, ligands, receptors."""

    def __init__(self, workload: dict, stream=None, *, init: bool = True, layout: int = 2):
        L = lib()
        lat = workload["lattice"]
        self.workload = workload
        self.nx, self.ny = int(lat["nx"]), int(lat["ny"])
        self.precision = int(lat.get("precision", FP64))
        d = _lattice_desc(lat)
        self._h = C.c_void_p()
        self.stream = stream
        _check(L.lbib_create(C.byref(d), _stream_ptr(stream), C.byref(self._h)))
        self.nl = 0
        self.nls = []
        try:
            for part, lig in particle_entries(workload):
                pd = _particle_desc(part)
                pid = C.c_int32()
                self._call(L.lbib_particle_add, C.byref(pd), C.byref(pid))
                self.nls.append(int(part["n_markers"]))
                ld = _ligand_desc(lig)
                self._call(L.lbib_ligands_set, pid.value, C.byref(ld))
            if self.nls:
                self.nl = self.nls[0]
                r = workload.get("receptor", {"wall": 0, "density": 1.0})
                rd = ReceptorDesc(int(r["wall"]), float(r["density"]))
                self._call(L.lbib_receptors_set, C.byref(rd))
            self._call(L.lbib_set_layout, int(layout))
            if init:
                self._call(L.lbib_init)
        except Exception:
            self.close()
            raise

    def _call(self, fn, *args):
        _check(fn(self._h, *args), self._h)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().lbib_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- time loop ---------------------------------------------------------------------
    def init(self):
        self._call(lib().lbib_init)

    def step(self, n: int = 1):
        self._call(lib().lbib_step, int(n))

    def sync(self):
        self._call(lib().lbib_sync)

    @property
    def steps(self) -> int:
        v = C.c_int64()
        self._call(lib().lbib_step_count, C.byref(v))
        return v.value

    @property
    def bytes_per_update(self) -> int:
        v = C.c_int64()
        self._call(lib().lbib_bytes_per_update, C.byref(v))
        return v.value

    # -- reads ---------------------------------------------------------------------------
    def particle(self, pid: int = 0) -> dict:
        s = ParticleState()
        self._call(lib().lbib_read_particle, pid, C.byref(s))
        return {n: getattr(s, n) for n in STATE_FIELDS}

    def bonds(self, pid: int = 0):
        nl = self.nls[pid]
        b = np.zeros(nl, np.uint8)
        lg = np.zeros(nl, np.uint8)
        self._call(lib().lbib_read_bonds, pid, b.ctypes.data_as(_U8), lg.ctypes.data_as(_U8), nl)
        return b, lg

    def markers(self, pid: int = 0):
        nl = self.nls[pid]
        X = np.zeros((nl, 2))
        n = np.zeros((nl, 2))
        self._call(lib().lbib_read_markers, pid, X.ctypes.data_as(_D), n.ctypes.data_as(_D), nl)
        return X, n

    def field(self, which: int) -> np.ndarray:
        shape = (9, self.ny, self.nx) if which == 3 else (self.ny, self.nx)
        out = np.zeros(shape)
        self._call(lib().lbib_read_field, int(which), out.ctypes.data_as(_D), out.size)
        return out

    @property
    def f(self) -> np.ndarray:
        return self.field(3)

    def fields(self):
        return self.field(0), self.field(1), self.field(2)

    # -- writes --------------------------------------------------------------------------
    def write_populations(self, f: np.ndarray):
        f = np.ascontiguousarray(f, np.float64)
        assert f.shape == (9, self.ny, self.nx)
        self._call(lib().lbib_write_populations, f.ctypes.data_as(_D), f.size)

    def write_particle(self, state12, pid: int = 0):
        v = np.ascontiguousarray(state12, np.float64)
        assert v.shape == (12,)
        self._call(lib().lbib_write_particle, pid, v.ctypes.data_as(_D))

    def write_bonds(self, bonded, pid: int = 0):
        b = np.ascontiguousarray(bonded, np.uint8)
        self._call(lib().lbib_write_bonds, pid, b.ctypes.data_as(_U8), len(b))

    # -- trace ---------------------------------------------------------------------------
    def trace_enable(self, capacity: int, pid: int = 0):
        self._call(lib().lbib_trace_enable, pid, int(capacity))

    def trace(self, capacity: int, pid: int = 0) -> np.ndarray:
        """Recorded states as a float64 array [count, 20] in the field order of STATE_FIELDS."""
        buf = (ParticleState * max(1, capacity))()
        cnt = C.c_int64()
        self._call(lib().lbib_read_trace, pid, buf, int(capacity), C.byref(cnt))
        return _trace_array(buf, cnt.value)

    # -- checkpoints ---------------------------------------------------------------------
    def save(self) -> bytes:
        size = C.c_int64()
        self._call(lib().lbib_save, None, C.byref(size))
        buf = C.create_string_buffer(size.value)
        self._call(lib().lbib_save, buf, C.byref(size))
        return buf.raw[: size.value]

    def load(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        self._call(lib().lbib_load, buf, len(blob))

    @property
    def pull(self) -> bool:
        """True when the population buffers use the pull layout."""
        v = C.c_int32()
        self._call(lib().lbib_get_layout, C.byref(v))
        return bool(v.value)

    def set_overlap(self, mode):
        """0 / False: serial; 1 / True: overlapped with a particle launch per step (one particle)
        or chained split phase (several); 2 (default): overlapped with one resident particle
        launch over a call's steps (one particle), the one-launch split phase (several); 3: the
        split particle phase in order on one stream; 4: several particles' split phase as one
        launch (workgroups claim their particles, no co-residency needed); 5: that launch on a
        single workgroup (its fallback path every step; for testing)."""
        self._call(lib().lbib_set_overlap, int(mode))

    # -- timing --------------------------------------------------------------------------
    def kernel_timing(self, enable=True):
        """True: time all three kernels; False: off; an int: bit mask of the kernels to time."""
        mask = 7 if enable is True else 0 if enable is False else int(enable)
        self._call(lib().lbib_kernel_timing, mask)

    def kernel_time(self, kernel: int):
        """(total milliseconds, launches) of kernel 0 (lattice sweep: all nodes, or the nodes
        outside the particle's box), 1 (particle phase) or 2 (sweep of the box)."""
        ms = C.c_double()
        n = C.c_int64()
        self._call(lib().lbib_kernel_time, int(kernel), C.byref(ms), C.byref(n))
        return ms.value, n.value


# ----------------------------------------------------------------------------------------
# Pool of simulations stepped together
# ----------------------------------------------------------------------------------------

class Pool:
    """Many independent simulations (one particle each) stepped with one particle-phase launch
    and one sweep launch per time step.  Members join with add() and leave with remove().
    The whole memory budget is allocated on the device when the pool is created."""

    def __init__(self, precision: int = FP32, budget_bytes: int = 16 << 30, max_members: int = 4096, stream=None):
        self._h = C.c_void_p()
        self.stream = stream
        self.precision = int(precision)
        self._shape = {}
        _check(lib().lbib_pool_create(self.precision, int(budget_bytes), int(max_members), _stream_ptr(stream),
                                      C.byref(self._h)), None, pool=True)

    def _call(self, fn, *args):
        _check(fn(self._h, *args), self._h, pool=True)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().lbib_pool_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @staticmethod
    def footprint(workload: dict) -> int:
        v = C.c_int64()
        _check(lib().lbib_pool_footprint(C.byref(_lattice_desc(workload["lattice"])),
                                         C.byref(_particle_desc(workload["particle"])), C.byref(v)), None, pool=True)
        return v.value

    def add(self, workload: dict, n_steps: int) -> int:
        """Add a simulation (lattice + particle + ligands) to run n_steps steps; returns its slot."""
        lat, part = workload["lattice"], workload["particle"]
        slot = C.c_int32()
        self._call(lib().lbib_pool_add, C.byref(_lattice_desc(lat)), C.byref(_particle_desc(part)),
                   C.byref(_ligand_desc(workload["ligand"])), int(n_steps), C.byref(slot))
        self._shape[slot.value] = (int(lat["nx"]), int(lat["ny"]), int(part["n_markers"]))
        return slot.value

    def remove(self, slot: int):
        self._call(lib().lbib_pool_remove, int(slot))
        self._shape.pop(slot, None)

    def step(self, n: int = 1):
        self._call(lib().lbib_pool_step, int(n))

    def poll(self, capacity: int = 65536) -> list:
        """Wait for the enqueued steps; slots that finished or failed since the last poll."""
        buf = (C.c_int32 * max(1, capacity))()
        cnt = C.c_int32()
        self._call(lib().lbib_pool_poll, buf, int(capacity), C.byref(cnt))
        return [buf[k] for k in range(cnt.value)]

    def status(self, slot: int):
        """(steps done, state) with state POOL_RUNNING / POOL_FINISHED / POOL_FAILED."""
        n = C.c_int64()
        st = C.c_int32()
        self._call(lib().lbib_pool_status, int(slot), C.byref(n), C.byref(st))
        return n.value, st.value

    def last_error(self) -> str:
        m = lib().lbib_pool_last_error(self._h)
        return m.decode() if m else ""

    def usage(self):
        """(members, running, bytes in use)."""
        m, r, b = C.c_int32(), C.c_int32(), C.c_int64()
        self._call(lib().lbib_pool_usage, C.byref(m), C.byref(r), C.byref(b))
        return m.value, r.value, b.value

    def particle(self, slot: int) -> dict:
        s = ParticleState()
        self._call(lib().lbib_pool_read_particle, int(slot), C.byref(s))
        return {n: getattr(s, n) for n in STATE_FIELDS}

    def bonds(self, slot: int):
        nl = self._shape[slot][2]
        b = np.zeros(nl, np.uint8)
        lg = np.zeros(nl, np.uint8)
        self._call(lib().lbib_pool_read_bonds, int(slot), b.ctypes.data_as(_U8), lg.ctypes.data_as(_U8), nl)
        return b, lg

    def field(self, slot: int, which: int) -> np.ndarray:
        nx, ny, _ = self._shape[slot]
        out = np.zeros((9, ny, nx) if which == 3 else (ny, nx))
        self._call(lib().lbib_pool_read_field, int(slot), int(which), out.ctypes.data_as(_D), out.size)
        return out

    def trace_enable(self, slot: int, capacity: int):
        self._call(lib().lbib_pool_trace_enable, int(slot), int(capacity))

    def trace(self, slot: int, capacity: int) -> np.ndarray:
        buf = (ParticleState * max(1, capacity))()
        cnt = C.c_int64()
        self._call(lib().lbib_pool_read_trace, int(slot), buf, int(capacity), C.byref(cnt))
        return _trace_array(buf, cnt.value)

    def set_config(self, tile_x: int = 256, tiles_per_block: int = 4, graph_steps: int = 0):
        self._call(lib().lbib_pool_set_config, int(tile_x), int(tiles_per_block), int(graph_steps))

    def config(self):
        """(tile_x, tiles_per_block, graph_steps)."""
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        self._call(lib().lbib_pool_get_config, C.byref(a), C.byref(b), C.byref(c))
        return a.value, b.value, c.value

    def autotune(self, steps_per_trial: int = 20) -> float:
        """Pick the fastest sweep launch shape (and graph replay) on real steps; returns the
        best time per step in microseconds."""
        v = C.c_double()
        self._call(lib().lbib_pool_autotune, int(steps_per_trial), C.byref(v))
        return v.value

    def kernel_timing(self, enable: bool):
        self._call(lib().lbib_pool_kernel_timing, 1 if enable else 0)

    def kernel_time(self, kernel: int):
        """(total milliseconds, launches) of kernel 0 (pool sweep) or 1 (pool particle phase)."""
        ms = C.c_double()
        n = C.c_int64()
        self._call(lib().lbib_pool_kernel_time, int(kernel), C.byref(ms), C.byref(n))
        return ms.value, n.value


# ----------------------------------------------------------------------------------------
# Server: continuous batching of adhesion solves
# ----------------------------------------------------------------------------------------

class Server:
    """Requests (one adhesion solve each) queue in arrival order and join a pool as slots and
    memory free up; progress() runs one scheduling round (admit, step a chunk, collect)."""

    def __init__(self, precision: int = FP32, budget_bytes: int = 16 << 30, max_members: int = 4096,
                 chunk_steps: int = 200, max_bypass: int = 8, stream=None):
        self._h = C.c_void_p()
        self.stream = stream
        _check(lib().lbib_server_create(int(precision), int(budget_bytes), int(max_members), int(chunk_steps),
                                        int(max_bypass), _stream_ptr(stream), C.byref(self._h)), None, server=True)

    def _call(self, fn, *args):
        _check(fn(self._h, *args), self._h, server=True)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().lbib_server_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def clock(self) -> float:
        return lib().lbib_server_clock(self._h)

    def submit(self, workload: dict, n_steps: int, arrival_s: float = -1.0) -> int:
        rid = C.c_int64()
        self._call(lib().lbib_server_submit, C.byref(_lattice_desc(workload["lattice"])),
                   C.byref(_particle_desc(workload["particle"])), C.byref(_ligand_desc(workload["ligand"])),
                   int(n_steps), float(arrival_s), C.byref(rid))
        return rid.value

    def progress(self) -> int:
        n = C.c_int32()
        self._call(lib().lbib_server_progress, C.byref(n))
        return n.value

    def take_completed(self, capacity: int = 65536) -> list:
        buf = (C.c_int64 * max(1, capacity))()
        n = C.c_int32()
        self._call(lib().lbib_server_take_completed, buf, int(capacity), C.byref(n))
        return [buf[k] for k in range(n.value)]

    def result(self, rid: int) -> dict:
        r = RequestResult()
        self._call(lib().lbib_server_result, int(rid), C.byref(r))
        out = {n: getattr(r, n) for n, _ in RequestResult._fields_ if n != "final_state"}
        out["final_state"] = {n: getattr(r.final_state, n) for n in STATE_FIELDS}
        return out

    def release(self, rid: int):
        self._call(lib().lbib_server_release, int(rid))

    def set_trace(self, capacity: int):
        """Requests admitted from now on record their first `capacity` steps (0: off)."""
        self._call(lib().lbib_server_set_trace, int(capacity))

    def trace(self, rid: int, capacity: int) -> np.ndarray:
        """A completed request's records as float64 [count, 20] (field order of STATE_FIELDS)."""
        buf = (ParticleState * max(1, capacity))()
        cnt = C.c_int64()
        self._call(lib().lbib_server_read_trace, int(rid), buf, int(capacity), C.byref(cnt))
        return _trace_array(buf, cnt.value)

    def bonds(self, rid: int, n_markers: int):
        """A completed request's (bonded, ligand) flags after its last step."""
        b = np.zeros(n_markers, np.uint8)
        lg = np.zeros(n_markers, np.uint8)
        self._call(lib().lbib_server_read_bonds, int(rid), b.ctypes.data_as(_U8), lg.ctypes.data_as(_U8),
                   int(n_markers))
        return b, lg

    def stats(self):
        """(queued, running, bytes in use, chunks stepped)."""
        q, r, b, c = C.c_int32(), C.c_int32(), C.c_int64(), C.c_int64()
        self._call(lib().lbib_server_stats, C.byref(q), C.byref(r), C.byref(b), C.byref(c))
        return q.value, r.value, b.value, c.value


# ----------------------------------------------------------------------------------------
# Kernel-level entry points (torch tensors on the GPU)
# ----------------------------------------------------------------------------------------

def philox(ctr, key, stream=None):
    """ctr: uint32-compatible int32 tensor [n, 4]; key [n, 2] -> [n, 4] (as int32 bit patterns)."""
    import torch

    n = ctr.shape[0]
    out = torch.empty((n, 4), dtype=torch.int32, device=ctr.device)
    _check(lib().lbib_kernel_philox(_ptr(ctr), _ptr(key), _ptr(out), n, _stream_ptr(stream)))
    return out


def mls(pts, nx: int, ny: int, stream=None):
    """pts: float64 [n, 2] -> (node int32 [n, 9, 2], phi, psix, psiy float64 [n, 9])."""
    import torch

    n = pts.shape[0]
    dev = pts.device
    node = torch.empty((n, 9, 2), dtype=torch.int32, device=dev)
    phi = torch.empty((n, 9), dtype=torch.float64, device=dev)
    psx = torch.empty_like(phi)
    psy = torch.empty_like(phi)
    _check(lib().lbib_kernel_mls(_ptr(pts), n, nx, ny, _ptr(node), _ptr(phi), _ptr(psx), _ptr(psy),
                                 _stream_ptr(stream)))
    return node, phi, psx, psy


def bonds(ligand, d, b_in, step, params, seed: int, pid: int = 0, stream=None):
    """Batched bond update: ligand/b_in uint8 [sets, nl], d float64 [sets, nl], step int64 [sets];
    params = (y_cr, y_eq, sigma, sigma_star, k_f, k_r0, kBT).  Returns (b_out, n_bonds, n_probing)."""
    import torch

    sets, nl = d.shape
    dev = d.device
    b_out = torch.empty((sets, nl), dtype=torch.uint8, device=dev)
    nb = torch.empty(sets, dtype=torch.int32, device=dev)
    npr = torch.empty(sets, dtype=torch.int32, device=dev)
    p = (C.c_double * 7)(*[float(x) for x in params])
    _check(lib().lbib_kernel_bonds(_ptr(ligand), _ptr(d), _ptr(b_in), _ptr(b_out), _ptr(step), _ptr(nb), _ptr(npr),
                                   nl, sets, p, int(seed), int(pid), _stream_ptr(stream)))
    return b_out, nb, npr


def bandwidth_probe(nbytes: int, iters: int = 10, stream=None) -> float:
    v = C.c_double()
    _check(lib().lbib_bandwidth_probe(int(nbytes), int(iters), _stream_ptr(stream), C.byref(v)))
    return v.value


def solve_static_bytes(workload: dict) -> int:
    """Bytes of the population buffers lbib_solve_static needs for this lattice."""
    v = C.c_int64(0)
    _check(lib().lbib_solve_static(C.byref(_lattice_desc(workload["lattice"])),
                                   C.byref(_particle_desc(workload["particle"])),
                                   C.byref(_ligand_desc(workload["ligand"])), 0, None, C.byref(v), None, None,
                                   None))
    return v.value


def solve_static(workload: dict, n_steps: int, stream=None):
    """The allocation-free solve (lbib_solve_static): n_steps steps of the workload's single
    particle with the serial schedule.  The device buffers it is given (populations, trace,
    bonds) are torch tensors allocated here, as a caller with its own memory would provide
    them.  Returns (trace float64 [n_steps, 20] in the field order of STATE_FIELDS, bond
    flags uint8 [n_markers])."""
    import torch

    need = solve_static_bytes(workload)
    pops = torch.empty(need, dtype=torch.uint8, device="cuda")
    rec = C.sizeof(ParticleState)
    tr = torch.empty(max(1, n_steps) * rec, dtype=torch.uint8, device="cuda")
    nl = int(workload["particle"]["n_markers"])
    bd = torch.empty(nl, dtype=torch.uint8, device="cuda")
    v = C.c_int64(need)
    st = _stream_ptr(stream)
    if stream is not None:
        stream.wait_stream(torch.cuda.current_stream())
    _check(lib().lbib_solve_static(C.byref(_lattice_desc(workload["lattice"])),
                                   C.byref(_particle_desc(workload["particle"])),
                                   C.byref(_ligand_desc(workload["ligand"])), int(n_steps), _ptr(pops), C.byref(v),
                                   _ptr(tr), _ptr(bd), st))
    raw = tr.cpu().numpy().tobytes()
    return _trace_array(raw, int(n_steps)), bd.cpu().numpy()
