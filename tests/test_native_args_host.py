"""Host checks of the binding's argument validation: every wrapper compares
tensor extents with what the kernels will touch and raises before a pointer
reaches the library.  Run on CPU tensors: a size mismatch must raise
ValueError; correctly sized CPU tensors get as far as the device check
(TypeError), so nothing is launched either way."""
import ctypes

import pytest
import torch

from paper_2204_06633_amd import native

f64 = torch.float64


class _Orb:
    """Stand-in orbit handle (the calls below never reach the library)."""
    ref = ctypes.byref(native.lr_orbits())


def _z(*shape):
    return torch.zeros(shape, dtype=f64)


def _batch(n=3, h_extent=100, out_extent=60):
    b = object.__new__(native.Batch)
    b.templates = [(0, 10, 0, 5, 0)] * n
    b.c = native.lr_batch()
    b.c.h_extent = h_extent
    b.c.out_extent = out_extent
    b.channels, b.rows = "AET", 3
    return b


def test_project_links_sizes():
    args = dict(orb=_Orb(), t0_h=0.0, dt=10.0, order=25, y_start=20, n_y=50)
    with pytest.raises(ValueError, match="hc"):
        native.project_links(hp=_z(100), hc=_z(99), sky=_z(2), **args)
    with pytest.raises(ValueError, match="sky"):
        native.project_links(hp=_z(100), hc=_z(100), sky=_z(3), **args)
    with pytest.raises(ValueError, match="y has shape"):
        native.project_links(hp=_z(100), hc=_z(100), sky=_z(2), y=_z(6, 49), **args)
    with pytest.raises(TypeError):
        native.project_links(hp=_z(100), hc=_z(100), sky=_z(2), y=_z(6, 50), **args)


def test_tdi_sizes():
    with pytest.raises(ValueError, match="y must be"):
        native.tdi_combine(_Orb(), 0.0, 10.0, _z(5, 80), 2, 25, "XYZ", 20, 40)
    with pytest.raises(ValueError, match="out has shape"):
        native.tdi_combine(_Orb(), 0.0, 10.0, _z(6, 80), 2, 25, "XYZAET", 20, 40, out=_z(3, 40))
    with pytest.raises(TypeError):
        native.tdi_combine(_Orb(), 0.0, 10.0, _z(6, 80), 2, 25, "XYZAET", 20, 40, out=_z(6, 40))
    with pytest.raises(ValueError, match="g_out must be"):
        native.tdi_adjoint(_Orb(), 0.0, 10.0, 80, 2, 25, "XYZAET", 20, _z(3, 40))
    with pytest.raises(ValueError, match="g_y has shape"):
        native.tdi_adjoint(_Orb(), 0.0, 10.0, 80, 2, 25, "AET", 20, _z(3, 40), g_y=_z(6, 79))
    with pytest.raises(TypeError):
        native.tdi_adjoint(_Orb(), 0.0, 10.0, 80, 2, 25, "AET", 20, _z(3, 40), g_y=_z(6, 80))


def test_project_adjoint_sizes():
    a = dict(orb=_Orb(), t0_h=0.0, dt=10.0, order=25, y_start=20)
    with pytest.raises(ValueError, match="g_y must be"):
        native.project_adjoint(n_h=100, hp=None, hc=None, sky=_z(2), g_y=_z(5, 50),
                               want_sky=False, **a)
    with pytest.raises(ValueError, match="g_hp"):
        native.project_adjoint(n_h=100, hp=None, hc=None, sky=_z(2), g_y=_z(6, 50),
                               want_sky=False, g_hp=_z(99), **a)
    with pytest.raises(ValueError, match="hp"):
        native.project_adjoint(n_h=100, hp=_z(98), hc=_z(100), sky=_z(2), g_y=_z(6, 50), **a)
    with pytest.raises(ValueError, match="g_sky"):
        native.project_adjoint(n_h=100, hp=_z(100), hc=_z(100), sky=_z(2), g_y=_z(6, 50),
                               g_sky=_z(3), **a)
    with pytest.raises(TypeError):
        native.project_adjoint(n_h=100, hp=_z(100), hc=_z(100), sky=_z(2), g_y=_z(6, 50), **a)


def test_loglike_sizes():
    with pytest.raises(ValueError, match="data"):
        native.loglike(_z(3, 10), _z(3, 9), 1.0)
    with pytest.raises(ValueError, match="g_h"):
        native.loglike(_z(3, 10), _z(3, 10), 1.0, g_h=_z(29))
    with pytest.raises(TypeError):
        native.loglike(_z(3, 10), _z(3, 10), 1.0)


def test_batch_sizes():
    b = _batch()
    with pytest.raises(ValueError, match="hp"):
        b.response(_z(99), _z(100), _z(3, 2))
    with pytest.raises(ValueError, match="sky"):
        b.response(_z(100), _z(100), _z(2, 2))
    with pytest.raises(ValueError, match="out"):
        b.response(_z(100), _z(100), _z(3, 2), out=_z(59))
    with pytest.raises(TypeError):
        b.response(_z(100), _z(100), _z(3, 2), out=_z(60))
    with pytest.raises(ValueError, match="g_out"):
        b.adjoint(_z(100), _z(100), _z(3, 2), _z(59))
    with pytest.raises(ValueError, match="g_hc"):
        b.adjoint(_z(100), _z(100), _z(3, 2), _z(60), g_hc=_z(50))
    with pytest.raises(ValueError, match="g_sky"):
        b.adjoint(_z(100), _z(100), _z(3, 2), _z(60), g_sky=_z(2, 2))
    with pytest.raises(ValueError, match="needs hp"):
        b.adjoint(None, None, _z(3, 2), _z(60))
    with pytest.raises(TypeError):
        b.adjoint(None, None, _z(3, 2), _z(60), want_sky=False)
    with pytest.raises(ValueError, match="data"):
        b.loglike(_z(60), _z(10), 1.0)
    with pytest.raises(ValueError, match="loglike"):
        b.loglike(_z(60), _z(60), 1.0, ll=_z(2))
    with pytest.raises(TypeError):
        b.loglike(_z(60), _z(60), 1.0)


def test_waveform_sizes():
    with pytest.raises(ValueError, match="params"):
        native.gb_polarizations(_z(2, 7), 0, 10, 1.0)
    with pytest.raises(ValueError, match="hp must be"):
        native.gb_polarizations(_z(2, 8), 0, 10, 1.0, hp=_z(2, 9), hc=_z(2, 9))
    with pytest.raises(TypeError):
        native.gb_polarizations(_z(2, 8), 0, 10, 1.0)
    with pytest.raises(ValueError, match="params"):
        native.gb_polarizations_adjoint(_z(3, 8), 0, 1.0, _z(2, 10), _z(2, 10))
    with pytest.raises(ValueError, match="g_params"):
        native.gb_polarizations_adjoint(_z(2, 8), 0, 1.0, _z(2, 10), _z(2, 10),
                                        g_params=_z(2, 7))
    with pytest.raises(TypeError):
        native.gb_polarizations_adjoint(_z(2, 8), 0, 1.0, _z(2, 10), _z(2, 10))


def test_fd_plan_sizes():
    n_bins = native.fd_length(5000) // 2 + 1
    with pytest.raises(ValueError, match="channels"):
        native.FdPlan(_z(4, 5000), _z(n_bins), _z(n_bins), 10.0)
    with pytest.raises(ValueError, match="w_ae"):
        native.FdPlan(_z(3, 5000), _z(n_bins - 1), _z(n_bins), 10.0)
    with pytest.raises(ValueError, match="w_t"):
        native.FdPlan(_z(3, 5000), _z(n_bins), _z(n_bins + 1), 10.0)
    with pytest.raises(TypeError):
        native.FdPlan(_z(3, 5000), _z(n_bins), _z(n_bins), 10.0)
