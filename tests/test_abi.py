"""CPU-side checks of the C-ABI library: it loads, exports every entry point
declared in include/tdo.h, and host-only queries validate their arguments."""
import ctypes
import os
import re

import pytest

from oracle import ansatz as oa
from paper_2502_20723_amd import synth, tdo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    src = open(os.path.join(ROOT, "include", "tdo.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tdo_[a-z_0-9]+)\s*\(", src)))


def test_header_lists_the_binding_exports():
    assert set(declared_entry_points()) == set(tdo.EXPORTS)


def test_library_loads_and_exports_every_declared_symbol():
    lib = tdo.lib()
    for name in declared_entry_points():
        assert hasattr(lib, name), name


@pytest.mark.parametrize("name", ["ising_n4", "ising_n8", "xyz_n16", "ising_n32", "batched_uneven"])
def test_num_params_matches_layout(name):
    a = synth.WORKLOADS[name]["arch"]
    P = tdo.num_params(a)
    assert P == synth.num_params(a)
    assert P == oa.num_params(oa.Arch(**a))


def test_invalid_arch_is_rejected():
    bad = [dict(d=48, heads=4, layers=1, mlp=64), dict(d=64, heads=3, layers=1, mlp=64),
           dict(d=64, heads=2, layers=1, mlp=64), dict(d=64, heads=4, layers=0, mlp=64),
           dict(d=64, heads=4, layers=1, mlp=40), dict(d=64, heads=4, layers=1, mlp=64, c1=32),
           dict(d=64, heads=4, layers=1, mlp=64, act=1)]
    for a in bad:
        with pytest.raises(tdo.TdoError):
            tdo.num_params(a)
        assert tdo.lib().tdo_last_error().decode() != ""


def test_new_entry_points_validate_before_any_device_call():
    """Argument checks of the update, SR and observable calls happen on the host,
    before anything is launched, so they run without a GPU."""
    L = tdo.lib()
    st = None
    assert L.tdo_sgd_step(-1, None, None, 0.1, st) != 0
    assert "P=" in L.tdo_last_error().decode()
    assert L.tdo_sgd_step(0, None, None, 0.1, st) == 0                      # nothing to do
    assert L.tdo_adam_step(4, None, None, None, None, 0, 1e-3, 0.9, 0.999, 1e-8, st) != 0
    assert "t=0" in L.tdo_last_error().decode()
    assert L.tdo_adam_step(4, None, None, None, None, 1, 1e-3, 1.0, 0.999, 1e-8, st) != 0
    assert L.tdo_adam_step(4, None, None, None, None, 1, 1e-3, 0.9, 0.999, 0.0, st) != 0
    assert L.tdo_sr_solve(None, None, 4, 10, None, None, 1e-3, 10, None, None, st) != 0
    assert "ctx" in L.tdo_last_error().decode()
    arch = tdo.arch_t(dict(d=16, heads=2, layers=1, mlp=64))
    assert L.tdo_observables(None, ctypes.byref(arch), None, 4, None, 0, 0, None, None, None, None, st) != 0
    assert L.tdo_purity(None, ctypes.byref(arch), None, 4, None, None, 1, 0, None, st) != 0
    assert L.tdo_sample_diag(None, ctypes.byref(arch), None, 4, 1, None, None, 0, None, 1, 0, None, st) != 0
    assert L.tdo_log_rho_jacobian(None, ctypes.byref(arch), None, 4, None, 1, 0, None, st) != 0


def test_arch_fields_and_status_codes():
    """c1 = d and c1 = 0 (its default) describe the same network; the header's
    TDO_ENONFINITE and TDO_ACT_RELU_FFN are the binding's values."""
    a = dict(d=64, heads=4, layers=2, mlp=256)
    assert tdo.num_params(dict(a, c1=64)) == tdo.num_params(a) == oa.num_params(oa.Arch(**a))
    src = open(os.path.join(ROOT, "include", "tdo.h")).read()
    assert re.search(r"#define TDO_ENONFINITE \((-?\d+)\)", src).group(1) == str(tdo.TDO_ENONFINITE)
    assert re.search(r"#define TDO_ACT_RELU_FFN (\d+)", src).group(1) == str(tdo.TDO_ACT_RELU_FFN)
