"""The C-ABI library loads and exports every function include/psc.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "psc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(psc_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["psc_amg_build", "psc_pcg_solve", "psc_fcg_solve", "psc_hier_info", "psc_vcycle_apply",
                 "psc_net_create", "psc_net_train", "psc_pairs_collect", "psc_last_error", "psc_hier_free"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2406_19754_amd", "libpsc.so"))
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_loads_without_gpu():
    from paper_2406_19754_amd import psc
    assert psc.net_param_count() == 7809
    assert psc.lib().psc_last_error() is not None
