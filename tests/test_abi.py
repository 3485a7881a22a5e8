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
           dict(d=64, heads=4, layers=1, mlp=40)]
    for a in bad:
        with pytest.raises(tdo.TdoError):
            tdo.num_params(a)
        assert tdo.lib().tdo_last_error().decode() != ""
