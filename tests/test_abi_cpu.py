"""Host-side checks of the C ABI library: it loads without a GPU, exports every
entry point that include/pyhea.h declares, and the binding covers them all."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pyhea.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pyhea_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libpath():
    from paper_2411_18906_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2411_18906_amd import build_lib
        build_lib.build()
    return binding.LIB_PATH


def test_header_declares_the_four_entry_points():
    names = _declared()
    for n in ["pyhea_sro_eval", "pyhea_mc_run", "pyhea_mc_batch", "pyhea_serve_submit"]:
        assert n in names


def test_library_exports_every_declared_symbol(libpath):
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True,
                         check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing


def test_library_loads_and_binding_covers_header(libpath):
    from paper_2411_18906_amd import binding
    L = binding.lib()
    for n in _declared():
        assert hasattr(L, n)
    assert sorted(binding.EXPORTS) == _declared()
    assert binding.pyhea_version() >= 10000


def test_host_side_validation_without_gpu(libpath):
    """Descriptor validation happens on the host, before any device call."""
    from paper_2411_18906_amd import binding as b
    L = b.lib()
    bad = [b.make_lattice(3, (4, 4, 4), 4, 2),      # unknown lattice
           b.make_lattice(b.FCC, (4, 4, 4), 9, 2),  # too many species
           b.make_lattice(b.FCC, (4, 4, 4), 4, 5),  # too many shells
           b.make_lattice(b.FCC, (2, 2, 1), 4, 2),  # offset (0,0,2) maps a site onto itself
           b.make_lattice(b.FCC, (0, 4, 4), 4, 2)]
    for lat in bad:
        code = L.pyhea_sro_eval(ctypes.byref(lat), ctypes.c_void_p(1), None, None, None, None, None)
        assert code == b.EINVAL
        assert L.pyhea_last_error().decode()
    assert L.pyhea_tune_force(99) == b.EINVAL
    assert L.pyhea_tune_force(-1) == b.OK
