"""CPU-side checks of the C-ABI library: it loads without a GPU, exports every
entry point that include/memd.h declares, and the binding's constants match
the header.  No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "memd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(memd_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("memd_init_lattice", "memd_set_permittivity", "memd_initial_gauss_solve",
                     "memd_step", "memd_forces", "memd_energy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1309_7859_amd import memd
    lib = memd.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert lib.memd_version() == 1


def test_status_codes_match_header():
    from paper_1309_7859_amd import memd
    text = open(HEADER).read()
    codes = dict((k, int(v)) for k, v in re.findall(r"(MEMD_E[A-Z]+|MEMD_OK)\s*=\s*(-?\d+)", text))
    assert codes["MEMD_OK"] == memd.OK
    assert codes["MEMD_EINVAL"] == memd.EINVAL
    assert codes["MEMD_ENONNEUTRAL"] == memd.ENONNEUTRAL
    assert codes["MEMD_EUNSTABLE"] == memd.EUNSTABLE
    assert codes["MEMD_ESTATE"] == memd.ESTATE
    assert codes["MEMD_ENOCONV"] == memd.ENOCONV
    assert codes["MEMD_EDEVICE"] == memd.EDEVICE
    assert codes["MEMD_ESIZE"] == memd.ESIZE
    for k, v in re.findall(r"(MEMD_EPS_[A-Z]+)\s*=\s*(\d+)", text):
        assert getattr(memd, k[len("MEMD_"):]) == int(v)
    lib = memd.load()
    assert lib.memd_strerror(memd.ENONNEUTRAL).decode() == "charges are not neutral"


def test_params_struct_layout():
    from paper_1309_7859_amd import memd
    # int, pad, 3 doubles, 3 ints (+pad): the C layout on x86-64
    assert ctypes.sizeof(memd.memd_params) == 48
    assert memd.memd_params.a.offset == 8
    assert memd.memd_params.precision.offset == 32
    assert ctypes.sizeof(memd.memd_energy_t) == 40


def test_binding_refuses_missing_library(tmp_path, monkeypatch):
    from paper_1309_7859_amd import memd
    monkeypatch.setattr(memd, "_lib", None)
    monkeypatch.setattr(memd, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(RuntimeError):
        memd.load()
