"""ctypes loader for the plain FP64 CPU oracle (``mhd_oracle.c``).

Test infrastructure only: the test suite, the smoke check and the
CPU-baseline leg of the benchmark load this module; the HIP library never
does.  It shares nothing with the GPU path except the seeded input
generators, which hold none of the method's arithmetic.

State arrays are float64 of shape (11, nz, ny, nx) in field order
rho, mx, my, mz, E, e, bx, by, bz, h2, hp (x fastest in memory).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mhd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FIELDS = ("rho", "mx", "my", "mz", "E", "e", "bx", "by", "bz", "h2")
NF = 11


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("theta", ctypes.c_double),
        ("chemistry", ctypes.c_int), ("cooling", ctypes.c_int), ("ionisation", ctypes.c_int),
        ("grav_G", ctypes.c_double),
        ("n_unit", ctypes.c_double), ("T_unit", ctypes.c_double), ("t_unit", ctypes.c_double),
    ]


def build(force=True):
    """Compile the oracle with gcc (plain FP64, no FMA contraction, OpenMP)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def _p(a):
    return a.ctypes.data_as(_D)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(Params)
        for name, args, res in [
            ("orc_parabola", [_D, _D], None),
            ("orc_avg_right", [_D, ctypes.c_double], ctypes.c_double),
            ("orc_avg_left", [_D, ctypes.c_double], ctypes.c_double),
            ("orc_eigen", [ctypes.c_double] * 7 + [_D, _D, _D], None),
            ("orc_riemann_face", [_D, _D, _D, _D] + [ctypes.c_double] * 4 + [_D], None),
            ("orc_nonadv_stage", [P, _D, ctypes.c_double], None),
            ("orc_adv_stage", [P, _D, ctypes.c_double], None),
            ("orc_nonadv_rhs", [P, _D, ctypes.c_double, _D], None),
            ("orc_adv_rhs", [P, _D, ctypes.c_double, _D], None),
            ("orc_k1_base", [ctypes.c_double], ctypes.c_double),
            ("orc_k2", [ctypes.c_double], ctypes.c_double),
            ("orc_k3", [ctypes.c_double], ctypes.c_double),
            ("orc_k4", [], ctypes.c_double),
            ("orc_chem_cell", [P] + [ctypes.c_double] * 4 + [_D], ctypes.c_double),
            ("orc_ncrit", [ctypes.c_double], ctypes.c_double),
            ("orc_lh2", [ctypes.c_double], ctypes.c_double),
            ("orc_ll2", [ctypes.c_double] * 3, ctypes.c_double),
            ("orc_ln_ll3", [ctypes.c_double] * 2, ctypes.c_double),
            ("orc_heat_cool", [P] + [ctypes.c_double] * 3 + [_D], ctypes.c_double),
            ("orc_cooling", [P, _D, ctypes.c_double], None),
            ("orc_potential", [P, _D, _D], None),
            ("orc_gamma_cell", [P] + [ctypes.c_double] * 3, ctypes.c_double),
            ("orc_k5", [], ctypes.c_double),
            ("orc_k6", [ctypes.c_double], ctypes.c_double),
            ("orc_k7", [ctypes.c_double], ctypes.c_double),
            ("orc_k8", [ctypes.c_double], ctypes.c_double),
            ("orc_chem_cell_ion", [P] + [ctypes.c_double] * 5 + [_D, _D, _D], None),
            ("orc_heat_cool_ion", [P] + [ctypes.c_double] * 4 + [_D], ctypes.c_double),
            ("orc_stencil_factor", [ctypes.c_int, ctypes.c_int], ctypes.c_double),
            ("orc_clamp_h2", [P, _D], None),
            ("orc_chemistry", [P, _D, ctypes.c_double], None),
            ("orc_regularise", [P, _D], None),
            ("orc_cell_speed", [P, _D, ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_double),
            ("orc_cfl_dt", [P, _D], ctypes.c_double),
            ("orc_step", [P, _D, ctypes.c_double], None),
            ("orc_totals", [P, _D, _D], None),
            ("orc_prim_to_cons", [P, _D, _D], None),
            ("orc_max_divb", [P, _D], ctypes.c_double),
            ("orc_num_threads", [], ctypes.c_int),
        ]:
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


# default chemistry unit map: 5 H nuclei cm^-3 per unit density, T_u = 5000 K,
# t_u = L_u / v_u with L_u = 256 pc and v_u = sqrt(k_B T_u / m_H)
def default_units():
    kB = 1.380649e-16
    mH = 1.6735575e-24
    pc = 3.0856775814913673e18
    T_u = 5000.0
    v_u = (kB * T_u / mH) ** 0.5
    return 5.0, T_u, 256.0 * pc / v_u


def gravity_G(units=None):
    """G in code units, G_cgs n_u m_H t_u^2 (density unit n_u m_H g cm^-3, time unit t_u s)."""
    nu, Tu, tu = units if units is not None else default_units()
    return 6.6743e-8 * nu * 1.6735575e-24 * tu * tu


def make_params(shape, gamma=5.0 / 3.0, cfl=0.3, theta=1.0, chemistry=True, units=None, cooling=False, grav_G=0.0,
                ionisation=False):
    nz, ny, nx = shape
    nu, Tu, tu = units if units is not None else default_units()
    return Params(nx, ny, nz, gamma, cfl, theta, 1 if chemistry else 0, 1 if cooling else 0,
                  1 if ionisation else 0, float(grav_G), nu, Tu, tu)


def _check_state(U):
    assert U.dtype == np.float64 and U.flags.c_contiguous and U.ndim == 4 and U.shape[0] == NF


def prim_to_cons(P, W):
    W = np.ascontiguousarray(W, dtype=np.float64)
    U = np.empty((NF,) + W.shape[1:], dtype=np.float64)
    lib().orc_prim_to_cons(ctypes.byref(P), _p(W), _p(U))
    return U


def cfl_dt(P, U):
    _check_state(U)
    return lib().orc_cfl_dt(ctypes.byref(P), _p(U))


def step(P, U, dt):
    """One full operator-split step, in place."""
    _check_state(U)
    lib().orc_step(ctypes.byref(P), _p(U), float(dt))
    return U


def nonadv_stage(P, U, dt):
    _check_state(U)
    lib().orc_nonadv_stage(ctypes.byref(P), _p(U), float(dt))
    return U


def adv_stage(P, U, dt):
    _check_state(U)
    lib().orc_adv_stage(ctypes.byref(P), _p(U), float(dt))
    return U


def nonadv_rhs(P, U, dt):
    _check_state(U)
    inc = np.zeros_like(U)
    lib().orc_nonadv_rhs(ctypes.byref(P), _p(U), float(dt), _p(inc))
    return inc


def adv_rhs(P, U, dt):
    _check_state(U)
    inc = np.zeros_like(U)
    lib().orc_adv_rhs(ctypes.byref(P), _p(U), float(dt), _p(inc))
    return inc


def clamp_h2(P, U):
    lib().orc_clamp_h2(ctypes.byref(P), _p(U))
    return U


def chemistry(P, U, dt):
    lib().orc_chemistry(ctypes.byref(P), _p(U), float(dt))
    return U


def cooling(P, U, dt):
    """Heating/cooling stage (explicit Euler), in place."""
    _check_state(U)
    lib().orc_cooling(ctypes.byref(P), _p(U), float(dt))
    return U


def heat_cool(P, rho, e, h2):
    """Gamma - Lambda (erg cm^-3 s^-1) and the terms (Gamma1, Gamma4, Lambda2, Lambda3, T)."""
    out = np.zeros(5)
    r = lib().orc_heat_cool(ctypes.byref(P), float(rho), float(e), float(h2), _p(out))
    return r, out


def potential(P, rho):
    """Gravitational potential of the density field (Poisson stage)."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    phi = np.empty_like(rho)
    lib().orc_potential(ctypes.byref(P), _p(rho), _p(phi))
    return phi


def gamma_cell(P, rho, h2, hp):
    return lib().orc_gamma_cell(ctypes.byref(P), float(rho), float(h2), float(hp))


def ion_rates(T):
    L = lib()
    return L.orc_k5(), L.orc_k6(T), L.orc_k7(T), L.orc_k8(T)


def chem_cell_ion(P, rho, e, h2, hp, dt):
    """One cell of the chemistry with reactions 1-8: (h2', hp', rates)."""
    a, b = ctypes.c_double(), ctypes.c_double()
    rates = np.zeros(9)
    lib().orc_chem_cell_ion(ctypes.byref(P), float(rho), float(e), float(h2), float(hp), float(dt),
                            ctypes.byref(a), ctypes.byref(b), _p(rates))
    return a.value, b.value, dict(zip(("k1b", "k2", "k3", "k4", "k5", "k6", "k7", "k8", "T"), rates))


def heat_cool_ion(P, rho, e, h2, hp):
    out = np.zeros(7)
    r = lib().orc_heat_cool_ion(ctypes.byref(P), float(rho), float(e), float(h2), float(hp), _p(out))
    return r, out


def regularise(P, U):
    lib().orc_regularise(ctypes.byref(P), _p(U))
    return U


def totals(P, U):
    out = np.zeros(NF, dtype=np.float64)
    lib().orc_totals(ctypes.byref(P), _p(U), _p(out))
    return out


def max_divb(P, U):
    return lib().orc_max_divb(ctypes.byref(P), _p(U))


def parabola(q5):
    q = np.ascontiguousarray(q5, dtype=np.float64)
    out = np.zeros(4)
    lib().orc_parabola(_p(q), _p(out))
    return out


def avg_right(par, y):
    par = np.ascontiguousarray(par, dtype=np.float64)
    return lib().orc_avg_right(_p(par), float(y))


def avg_left(par, y):
    par = np.ascontiguousarray(par, dtype=np.float64)
    return lib().orc_avg_left(_p(par), float(y))


def eigen(rho, p, bn, bt1, bt2, gamma=5.0 / 3.0, eps=1e-12):
    lam = np.zeros(6)
    R = np.zeros(36)
    L = np.zeros(36)
    lib().orc_eigen(rho, p, bn, bt1, bt2, gamma, eps, _p(lam), _p(R), _p(L))
    return lam, R.reshape(6, 6), L.reshape(6, 6)


def riemann_face(cl, cr, parl, parr, bn, gamma=5.0 / 3.0, eps=1e-12, ydx=0.0):
    """cl, cr: (rho, vn, vt1, vt2, Bt1, Bt2, p); parl, parr: (6, 4) parabolas."""
    cl = np.ascontiguousarray(cl, dtype=np.float64)
    cr = np.ascontiguousarray(cr, dtype=np.float64)
    pl = np.ascontiguousarray(parl, dtype=np.float64).reshape(24)
    pr = np.ascontiguousarray(parr, dtype=np.float64).reshape(24)
    out = np.zeros(6)
    lib().orc_riemann_face(_p(cl), _p(cr), _p(pl), _p(pr), bn, gamma, eps, ydx, _p(out))
    return out


def chem_cell(P, rho, e, h2, dt):
    rates = np.zeros(7)
    h2n = lib().orc_chem_cell(ctypes.byref(P), rho, e, h2, dt, _p(rates))
    return h2n, dict(zip(("k1b", "k2", "k3", "k4", "C", "D", "T"), rates))


def k_rates(T):
    L = lib()
    return L.orc_k1_base(T), L.orc_k2(T), L.orc_k3(T), L.orc_k4()


def num_threads():
    return lib().orc_num_threads()


def run(P, U, steps):
    """steps x {dt = cfl_dt; step(dt)}; returns the list of dt used."""
    dts = []
    for _ in range(steps):
        dt = cfl_dt(P, U)
        step(P, U, dt)
        dts.append(dt)
    return dts
