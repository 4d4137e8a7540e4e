"""The C-ABI library loads and exports every entry point include/mhdchem.h
declares; host-only calls validate arguments.  No device work."""
import ctypes

import pytest

from paper_1608_08748_amd import binding


def test_every_declared_symbol_is_exported():
    L = binding.lib()
    names = binding.exported_names()
    assert "mhd_step" in names and "mhd_cfl_dt" in names and "mhd_conserved_totals" in names
    for n in names:
        assert hasattr(L, n), n


def test_workspace_bytes_scales_with_cells_and_precision():
    p64 = binding.make_params((8, 8, 8), precision=binding.FP64)
    p32 = binding.make_params((8, 8, 8), precision=binding.FP32_MIXED)
    big = binding.make_params((16, 16, 16), precision=binding.FP64)
    w64, w32, wb = (binding.workspace_bytes(p) for p in (p64, p32, big))
    assert w64 > w32 > 0
    assert 7 * w64 < wb < 9 * w64
    # three state copies of 10 fields are the floor
    assert w64 >= 3 * 10 * 512 * 8


@pytest.mark.parametrize("field,value", [("gamma", 1.0), ("cfl", 0.0), ("theta", -1.0), ("precision", 7),
                                         ("chemistry", 2), ("cooling", 2)])
def test_invalid_parameters_rejected(field, value):
    p = binding.make_params((4, 4, 4))
    setattr(p, field, value)
    assert binding.workspace_bytes(p) == 0
    h = ctypes.c_void_p()
    assert binding.lib().mhd_create(ctypes.byref(p), ctypes.byref(h)) == binding.MHD_EINVAL


def test_bad_dims_rejected():
    p = binding.make_params((4, 4, 4))
    p.n[1] = 0
    assert binding.workspace_bytes(p) == 0
    p = binding.make_params((2048, 2048, 2048))
    assert binding.workspace_bytes(p) == 0


def test_missing_or_small_workspace():
    p = binding.make_params((4, 4, 4))
    h = ctypes.c_void_p()
    assert binding.lib().mhd_create(ctypes.byref(p), ctypes.byref(h)) == binding.MHD_ENOMEM
    buf = ctypes.create_string_buffer(1 << 20)
    p.workspace = ctypes.addressof(buf)
    p.workspace_bytes = 16
    assert binding.lib().mhd_create(ctypes.byref(p), ctypes.byref(h)) == binding.MHD_ENOMEM


def test_null_box_and_bad_dt_rejected():
    L = binding.lib()
    assert L.mhd_step(None, 1e-3) == binding.MHD_EINVAL
    assert L.mhd_cfl_dt(None, None) == binding.MHD_EINVAL


def test_strerror():
    for s in (0, -1, -2, -3, -4, -5):
        assert binding.strerror(s)
    assert binding.strerror(-99) == "unknown status"


def test_gravity_parameters_validated():
    ok = binding.make_params((8, 16, 32), grav_G=0.8)
    base = binding.make_params((8, 16, 32))
    assert binding.workspace_bytes(ok) > binding.workspace_bytes(base) > 0
    for shape, G in (((8, 16, 24), 0.8), ((8, 16, 2048), 0.8), ((8, 8, 8), -1.0), ((8, 8, 8), float("nan")),
                     ((8, 8, 8), float("inf"))):
        p = binding.make_params(shape, grav_G=G)
        assert binding.workspace_bytes(p) == 0, (shape, G)
    # without gravity any shape is fine
    assert binding.workspace_bytes(binding.make_params((8, 16, 24))) > 0


def test_gravity_constant_in_code_units():
    # G n_u m_H t_u^2 with n_u = 5 cm^-3, t_u = 256 pc / sqrt(k_B 5000 K / m_H)
    assert abs(binding.gravity_G() - 0.84486) < 1e-4


def _host_bound_box(**kw):
    """A box bound to a host buffer standing in for the workspace: mhd_create
    only records the pointer, and the calls below return before any device
    work."""
    p = binding.make_params((8, 8, 8), **kw)
    need = binding.workspace_bytes(p)
    buf = ctypes.create_string_buffer(need + 256)
    addr = (ctypes.addressof(buf) + 255) & ~255
    p.workspace, p.workspace_bytes = addr, need
    h = ctypes.c_void_p()
    assert binding.lib().mhd_create(ctypes.byref(p), ctypes.byref(h)) == binding.MHD_OK
    return h, buf


def test_host_side_argument_checks():
    L = binding.lib()
    h, buf = _host_bound_box()
    phi = (ctypes.c_double * 512)()
    # no self-gravity on this machine
    assert L.mhd_get_potential(h, phi) == binding.MHD_EINVAL
    # unknown stage selector
    assert L.mhd_debug_stage(h, 99, 1e-3) == binding.MHD_EINVAL
    # a step must be finite and positive
    for dt in (0.0, -1.0, float("nan"), float("inf")):
        assert L.mhd_step(h, dt) == binding.MHD_EINVAL, dt
    # unaligned workspace
    p = binding.make_params((8, 8, 8))
    p.workspace, p.workspace_bytes = ctypes.addressof(buf) | 8, binding.workspace_bytes(p)
    h2 = ctypes.c_void_p()
    assert L.mhd_create(ctypes.byref(p), ctypes.byref(h2)) == binding.MHD_EINVAL
    assert L.mhd_destroy(h) == binding.MHD_OK


def test_ionisation_parameters_validated():
    base = binding.workspace_bytes(binding.make_params((8, 8, 8)))
    ion = binding.workspace_bytes(binding.make_params((8, 8, 8), ionisation=True))
    # one more primitive (gamma_eff) and one more ADV flux per direction
    assert ion > base
    p = binding.make_params((8, 8, 8), ionisation=True)
    p.ionisation = 2
    assert binding.workspace_bytes(p) == 0
    p = binding.make_params((8, 8, 8), ionisation=True, units=(0.0, 5000.0, 1e15))
    assert binding.workspace_bytes(p) == 0
    assert binding.NFIELDS == 11 and binding.NPRIM == 10
