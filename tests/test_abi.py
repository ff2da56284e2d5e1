"""The C-ABI library loads and exports every entry point declared in
include/vdc.h; argument checks that fail before any device call (no GPU)."""
import ctypes
import os
import re

import pytest

from paper_2307_13483_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "vdc.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(vdc_\w+)\s*\(", txt, re.M)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("vdc_model2d_create", "vdc_solve", "vdc_solve_plain", "vdc_level_shift",
              "vdc_matvec", "vdc_workspace_size", "vdc_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2307_13483_amd import vdc
    L = vdc.lib()
    for n in _declared():
        assert hasattr(L, n), n
    assert "gfx950" in vdc.version()


def test_invalid_model_rejected_before_device_work():
    from paper_2307_13483_amd import vdc
    p = inputs.base_params()
    for bad in (dict(Ng=0), dict(Nu=2000)):
        with pytest.raises(vdc.VdcError) as e:
            vdc.Model2D(p, bad.get("Ng", 4), bad.get("Nu", 4))
        assert e.value.code == vdc.VDC_ERR_INVALID_ARG
    q = dict(p, B1e=0.0)
    with pytest.raises(vdc.VdcError) as e:
        vdc.Model2D(q, 4, 4)
    assert e.value.code == vdc.VDC_ERR_INVALID_ARG
    assert "B" in vdc.lib().vdc_last_error().decode()


def test_null_arguments_rejected():
    from paper_2307_13483_amd import vdc
    L = vdc.lib()
    assert L.vdc_model2d_create(None, None) == vdc.VDC_ERR_INVALID_ARG
    assert L.vdc_level_shift(None, 1, None, None, None) == vdc.VDC_ERR_INVALID_ARG
    assert L.vdc_model_destroy(None) == vdc.VDC_OK
    for f in (L.vdc_batch_launch, L.vdc_batch_capture, L.vdc_batch_replay):
        assert f(None, None) == vdc.VDC_ERR_INVALID_ARG
    assert L.vdc_batch_info(None, None, None) == vdc.VDC_ERR_INVALID_ARG
    assert L.vdc_batch_kernel_times(None, None, None) == vdc.VDC_ERR_INVALID_ARG
    assert L.vdc_batch_destroy(None) == vdc.VDC_OK


def test_invalid_co2_model_rejected_before_device_work():
    from paper_2307_13483_amd import vdc
    p = inputs.co2like_params()
    for bad in (dict(s=4, x=4, y=32, a=2), dict(s=0, x=4, y=4, a=2)):
        with pytest.raises(vdc.VdcError) as e:
            vdc.Co2Model(p, bad)
        assert e.value.code == vdc.VDC_ERR_INVALID_ARG
    with pytest.raises(vdc.VdcError) as e:
        vdc.Co2Model(dict(p, omega_b=0.0), dict(s=4, x=4, y=4, a=2))
    assert e.value.code == vdc.VDC_ERR_INVALID_ARG
    assert vdc.lib().vdc_co2_create(None, None) == vdc.VDC_ERR_INVALID_ARG
    assert vdc.lib().vdc_co2_destroy(None) == vdc.VDC_OK


@pytest.mark.parametrize("name,value", [("kappa1", float("nan")), ("omega_u", float("inf")),
                                        ("A2o", float("nan")), ("gap", 1.7e308),
                                        ("lam", float("-inf"))])
def test_nonfinite_parameter_rejected_before_device_work(name, value):
    """A NaN or infinite model parameter, or one whose derived state energy
    E_2 = E_1 + gap overflows, is a call error (VDC_ERR_INVALID_ARG) raised by
    the host checks of vdc_model2d_create, before any device call."""
    from paper_2307_13483_amd import vdc
    p = dict(inputs.base_params())
    p[name] = value
    if name == "gap":
        p["E1"] = 1.7e308
    with pytest.raises(vdc.VdcError) as e:
        vdc.Model2D(p, 4, 4)
    assert e.value.code == vdc.VDC_ERR_INVALID_ARG
