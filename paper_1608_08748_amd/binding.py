"""Thin ctypes binding of libmhdchem.so (include/mhdchem.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch provides the device workspace and the stream.  Importing this module
does not touch the GPU; creating a ``Box`` does (it allocates the workspace).
"""
import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmhdchem.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mhdchem.h")

MHD_OK, MHD_EINVAL, MHD_ENOMEM, MHD_EDEVICE, MHD_ECFL, MHD_ENONPHYS, MHD_ETOOLARGE = 0, -1, -2, -3, -4, -5, -6
NOALLOC_MAX_CELLS = 16777216   # MHD_NOALLOC_MAX_CELLS
FP64, FP32_MIXED = 0, 1
STAGE_NONADV, STAGE_ADV, STAGE_TAIL, STAGE_NONADV_RHS, STAGE_ADV_RHS = 1, 2, 3, 4, 5
FIELDS = ("rho", "mx", "my", "mz", "E", "e", "bx", "by", "bz", "h2", "hp")
NFIELDS = len(FIELDS)      # conserved fields (hp = rho_H+, zero without the ionisation network)
NPRIM = 10                 # primitive fields: rho, vx, vy, vz, p, bx_f, by_f, bz_f, x_h2, x_hp
KCLASSES = ("setup", "nonadv_face", "nonadv_update", "adv_face", "adv_update", "tail", "reduce", "poisson")
NKCLASS = len(KCLASSES)

# chemistry unit map: 5 H nuclei per cm^3 per unit density, T_u = 5000 K,
# t_u = L_u / v_u with L_u = 256 pc and v_u = sqrt(k_B T_u / m_H)
_KB, _MH, _PC = 1.380649e-16, 1.6735575e-24, 3.0856775814913673e18
DEFAULT_UNITS = (5.0, 5000.0, 256.0 * _PC / (_KB * 5000.0 / _MH) ** 0.5)


class MhdParams(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("gamma", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("theta", ctypes.c_double),
        ("chemistry", ctypes.c_int32),
        ("cooling", ctypes.c_int32),
        ("ionisation", ctypes.c_int32),
        ("grav_G", ctypes.c_double),
        ("n_unit_cm3", ctypes.c_double),
        ("T_unit_K", ctypes.c_double),
        ("t_unit_s", ctypes.c_double),
        ("stream", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
    ]


class ServerParams(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("gamma", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("theta", ctypes.c_double),
        ("chemistry", ctypes.c_int32),
        ("cooling", ctypes.c_int32),
        ("n_unit_cm3", ctypes.c_double),
        ("T_unit_K", ctypes.c_double),
        ("t_unit_s", ctypes.c_double),
        ("max_slots", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("persistent", ctypes.c_int32),
        ("max_workgroups", ctypes.c_int32),
    ]


class Request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("steps", ctypes.c_int32), ("keep_state", ctypes.c_int32),
                ("borrow", ctypes.c_int32)]


class Completion(ctypes.Structure):
    _fields_ = [
        ("id", ctypes.c_uint64),
        ("status", ctypes.c_int32),
        ("steps", ctypes.c_int32),
        ("t_submit", ctypes.c_double),
        ("t_admit", ctypes.c_double),
        ("t_done", ctypes.c_double),
        ("totals", ctypes.c_double * NFIELDS),
        ("cells", ctypes.c_int64),
        ("bytes", ctypes.c_size_t),
    ]


class MhdError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__("%s: %s (status %d)" % (what, strerror(status), status))


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def exported_names():
    """Function names declared in include/mhdchem.h."""
    with open(HEADER) as f:
        txt = f.read()
    return sorted(set(re.findall(r"\b(mhd_[a-z0-9_]+)\s*\(", txt)))


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmhdchem.so is not built (run python -m paper_1608_08748_amd.build); "
                          "there is no fallback path")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(MhdParams)
    B = ctypes.c_void_p
    sig = {
        "mhd_workspace_bytes": ([P], ctypes.c_size_t),
        "mhd_create": ([P, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
        "mhd_init_state": ([B, _D], ctypes.c_int),
        "mhd_set_state": ([B, _D], ctypes.c_int),
        "mhd_get_state": ([B, _D], ctypes.c_int),
        "mhd_get_potential": ([B, _D], ctypes.c_int),
        "mhd_cfl_dt": ([B, _D], ctypes.c_int),
        "mhd_step": ([B, ctypes.c_double], ctypes.c_int),
        "mhd_step_cfl": ([B], ctypes.c_int),
        "mhd_conserved_totals": ([B, _D], ctypes.c_int),
        "mhd_conserved_totals_noalloc": ([ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                          ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
        "mhd_debug_stage": ([B, ctypes.c_int, ctypes.c_double], ctypes.c_int),
        "mhd_destroy": ([B], ctypes.c_int),
        "mhd_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "mhd_set_timing": ([B, ctypes.c_int], ctypes.c_int),
        "mhd_get_timing": ([B, _D, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
        "mhd_server_reserved_bytes": ([], ctypes.c_size_t),
        "mhd_server_box_bytes": ([ctypes.POINTER(ServerParams), ctypes.POINTER(ctypes.c_int32)], ctypes.c_size_t),
        "mhd_server_create": ([ctypes.POINTER(ServerParams), ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
        "mhd_server_submit": ([B, ctypes.POINTER(Request), _D, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
        "mhd_server_progress": ([B, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "mhd_server_poll": ([B, ctypes.POINTER(Completion), ctypes.c_int, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "mhd_server_result": ([B, ctypes.c_uint64, _D, ctypes.c_size_t], ctypes.c_int),
        "mhd_server_memory": ([B, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                               ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "mhd_server_destroy": ([B], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def strerror(status):
    return lib().mhd_strerror(int(status)).decode()


def _check(status, what):
    if status != MHD_OK:
        raise MhdError(status, what)


def gravity_G(units=None):
    """Gravitational constant in code units, G_cgs n_u m_H t_u^2 (density unit
    n_u m_H g cm^-3, time unit t_u s): about 0.845 for the default units."""
    nu, Tu, tu = units if units is not None else DEFAULT_UNITS
    return 6.6743e-8 * nu * _MH * tu * tu


def make_params(shape, precision=FP64, gamma=5.0 / 3.0, cfl=0.3, theta=1.0, chemistry=True, units=None,
                cooling=False, grav_G=0.0, ionisation=False):
    nz, ny, nx = shape
    p = MhdParams()
    p.n[0], p.n[1], p.n[2] = nx, ny, nz
    p.gamma, p.cfl, p.precision, p.theta = gamma, cfl, precision, theta
    p.chemistry = 1 if chemistry else 0
    p.cooling = 1 if cooling else 0
    p.grav_G = float(grav_G)
    p.ionisation = 1 if ionisation else 0
    p.n_unit_cm3, p.T_unit_K, p.t_unit_s = units if units is not None else DEFAULT_UNITS
    return p


def workspace_bytes(params):
    return lib().mhd_workspace_bytes(ctypes.byref(params))


class Box:
    """One periodic box on one GPU.  shape = (nz, ny, nx)."""

    def __init__(self, shape, precision=FP64, gamma=5.0 / 3.0, cfl=0.3, theta=1.0, chemistry=True,
                 units=None, device="cuda", stream=None, workspace=None, cooling=False, grav_G=0.0,
                 ionisation=False):
        import torch
        self.shape = tuple(int(s) for s in shape)
        self.p = make_params(self.shape, precision, gamma, cfl, theta, chemistry, units, cooling, grav_G, ionisation)
        nbytes = workspace_bytes(self.p)
        if nbytes == 0:
            raise MhdError(MHD_EINVAL, "mhd_workspace_bytes")
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.ws = workspace
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.ws.device)
        self.p.stream = self.stream.cuda_stream
        self.p.workspace = self.ws.data_ptr()
        self.p.workspace_bytes = self.ws.numel() * self.ws.element_size()
        h = ctypes.c_void_p()
        _check(lib().mhd_create(ctypes.byref(self.p), ctypes.byref(h)), "mhd_create")
        self.h = h

    @property
    def ncell(self):
        return self.shape[0] * self.shape[1] * self.shape[2]

    def init_state(self, W):
        W = np.ascontiguousarray(W, dtype=np.float64)
        assert W.shape == (NPRIM,) + self.shape
        _check(lib().mhd_init_state(self.h, W.ctypes.data_as(_D)), "mhd_init_state")

    def set_state(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        assert U.shape == (NFIELDS,) + self.shape
        _check(lib().mhd_set_state(self.h, U.ctypes.data_as(_D)), "mhd_set_state")

    def get_state(self):
        U = np.empty((NFIELDS,) + self.shape, dtype=np.float64)
        _check(lib().mhd_get_state(self.h, U.ctypes.data_as(_D)), "mhd_get_state")
        return U

    def potential(self):
        """Gravitational potential of the current density (boxes with grav_G > 0)."""
        phi = np.empty(self.shape, dtype=np.float64)
        _check(lib().mhd_get_potential(self.h, phi.ctypes.data_as(_D)), "mhd_get_potential")
        return phi

    def cfl_dt(self):
        dt = ctypes.c_double()
        _check(lib().mhd_cfl_dt(self.h, ctypes.byref(dt)), "mhd_cfl_dt")
        return dt.value

    def step(self, dt):
        _check(lib().mhd_step(self.h, float(dt)), "mhd_step")

    def step_cfl(self):
        _check(lib().mhd_step_cfl(self.h), "mhd_step_cfl")

    def totals(self):
        out = np.zeros(NFIELDS, dtype=np.float64)
        _check(lib().mhd_conserved_totals(self.h, out.ctypes.data_as(_D)), "mhd_conserved_totals")
        return out

    def debug_stage(self, stage, dt):
        _check(lib().mhd_debug_stage(self.h, int(stage), float(dt)), "mhd_debug_stage")

    def set_timing(self, enable):
        _check(lib().mhd_set_timing(self.h, 1 if enable else 0), "mhd_set_timing")

    def get_timing(self):
        """{class name: (ms total, launches)} since timing was enabled."""
        ms = np.zeros(NKCLASS, dtype=np.float64)
        cnt = np.zeros(NKCLASS, dtype=np.int64)
        _check(lib().mhd_get_timing(self.h, ms.ctypes.data_as(_D),
                                    cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))), "mhd_get_timing")
        return {KCLASSES[i]: (float(ms[i]), int(cnt[i])) for i in range(NKCLASS)}

    def run(self, steps):
        """steps x {dt = cfl_dt(); step(dt)}; returns the dt list."""
        dts = []
        for _ in range(steps):
            dt = self.cfl_dt()
            self.step(dt)
            dts.append(dt)
        return dts

    def close(self):
        if getattr(self, "h", None):
            lib().mhd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def conserved_totals_noalloc(state, precision, out, stream=None):
    """mhd_conserved_totals_noalloc on device tensors: state (MHD_NFIELDS, nz,
    ny, nx), float64 for FP64 or float32 for FP32_MIXED, contiguous; out: 11
    float64 on the same device.  Asynchronous on the stream (default: the
    current one)."""
    import torch
    assert state.is_cuda and out.is_cuda and state.is_contiguous() and out.is_contiguous()
    assert state.dim() == 4 and state.shape[0] == NFIELDS and out.dtype == torch.float64 and out.numel() >= NFIELDS
    assert state.dtype == (torch.float64 if precision == FP64 else torch.float32)
    nz, ny, nx = state.shape[1:]
    n = (ctypes.c_int32 * 3)(nx, ny, nz)
    s = stream if stream is not None else torch.cuda.current_stream(state.device)
    return lib().mhd_conserved_totals_noalloc(ctypes.c_void_p(state.data_ptr()), int(precision), n,
                                              ctypes.c_void_p(s.cuda_stream), ctypes.c_void_p(out.data_ptr()))


def server_params(precision=FP32_MIXED, gamma=5.0 / 3.0, cfl=0.3, theta=1.0, chemistry=True, units=None,
                  max_slots=64, cooling=False, persistent=True, max_workgroups=0):
    p = ServerParams()
    p.precision, p.gamma, p.cfl, p.theta = precision, gamma, cfl, theta
    p.chemistry = 1 if chemistry else 0
    p.cooling = 1 if cooling else 0
    p.n_unit_cm3, p.T_unit_K, p.t_unit_s = units if units is not None else DEFAULT_UNITS
    p.max_slots = max_slots
    p.persistent = 1 if persistent else 0
    p.max_workgroups = max_workgroups
    return p


def server_box_bytes(params, shape):
    nz, ny, nx = shape
    n = (ctypes.c_int32 * 3)(nx, ny, nz)
    return lib().mhd_server_box_bytes(ctypes.byref(params), n)


class Server:
    """Continuous-batching server of many boxes on one GPU; ``budget_bytes`` of
    device memory hold every box in flight (plus the fixed launch-table area)."""

    def __init__(self, budget_bytes, max_slots=64, precision=FP32_MIXED, device="cuda", stream=None, **phys):
        import torch
        self.p = server_params(precision=precision, max_slots=max_slots, **phys)
        total = int(budget_bytes) + lib().mhd_server_reserved_bytes()
        self.ws = torch.empty(total, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.ws.device)
        self.p.stream = self.stream.cuda_stream
        self.p.workspace = self.ws.data_ptr()
        self.p.workspace_bytes = total
        h = ctypes.c_void_p()
        _check(lib().mhd_server_create(ctypes.byref(self.p), ctypes.byref(h)), "mhd_server_create")
        self.h = h
        self.shapes = {}
        self.held = {}      # borrowed request states, kept alive until their completion is polled

    def box_bytes(self, shape):
        return server_box_bytes(self.p, shape)

    def submit(self, W, steps, keep_state=False, borrow=False):
        """Queue a request.  borrow=True lends W to the server instead of
        copying it (the array is held here until its completion is polled;
        pinned host memory makes the upload a single DMA)."""
        W = np.ascontiguousarray(W, dtype=np.float64)
        shape = W.shape[1:]
        r = Request()
        r.n[0], r.n[1], r.n[2] = shape[2], shape[1], shape[0]
        r.steps = int(steps)
        r.keep_state = 1 if keep_state else 0
        r.borrow = 1 if borrow else 0
        rid = ctypes.c_uint64()
        _check(lib().mhd_server_submit(self.h, ctypes.byref(r), W.ctypes.data_as(_D), ctypes.byref(rid)),
               "mhd_server_submit")
        self.shapes[rid.value] = tuple(shape)
        if borrow:
            self.held[rid.value] = W
        return rid.value

    def progress(self):
        na, npend = ctypes.c_int(), ctypes.c_int()
        _check(lib().mhd_server_progress(self.h, ctypes.byref(na), ctypes.byref(npend)), "mhd_server_progress")
        return na.value, npend.value

    def poll(self, cap=1024):
        buf = (Completion * cap)()
        n = ctypes.c_int()
        _check(lib().mhd_server_poll(self.h, buf, cap, ctypes.byref(n)), "mhd_server_poll")
        out = []
        for k in range(n.value):
            c = buf[k]
            self.held.pop(c.id, None)
            out.append(dict(id=c.id, status=c.status, steps=c.steps, t_submit=c.t_submit, t_admit=c.t_admit,
                            t_done=c.t_done, totals=np.array(c.totals[:]), cells=c.cells, bytes=c.bytes))
        return out

    def result(self, rid):
        shape = self.shapes[rid]
        U = np.empty((NFIELDS,) + shape, dtype=np.float64)
        _check(lib().mhd_server_result(self.h, ctypes.c_uint64(rid), U.ctypes.data_as(_D), U.size),
               "mhd_server_result")
        return U

    def memory(self):
        u, pk, cap = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().mhd_server_memory(self.h, ctypes.byref(u), ctypes.byref(pk), ctypes.byref(cap)),
               "mhd_server_memory")
        return u.value, pk.value, cap.value

    def close(self):
        if getattr(self, "h", None):
            lib().mhd_server_destroy(self.h)   # waits for the server's stream
            self.h = None
        self.held = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
