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


def _c_layout(type_name, fields):
    """sizeof and offsetof of a header struct, from a C program compiled here."""
    import subprocess
    import tempfile
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "psc.h"', 'int main(void) {',
             f'  printf("%zu\\n", sizeof({type_name}));']
    lines += [f'  printf("%zu\\n", offsetof({type_name}, {f}));' for f in fields]
    lines += ['  return 0;', '}']
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "layout.c"), os.path.join(d, "layout")
        open(src, "w").write("\n".join(lines) + "\n")
        subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), [int(x) for x in out[1:]]


def test_binding_structs_match_the_header_layout():
    from paper_2406_19754_amd import psc
    for cls, name in [(psc.AmgOpts, "psc_amg_opts"), (psc.HierStats, "psc_hier_stats")]:
        fields = [f[0] for f in cls._fields_]
        size, offs = _c_layout(name, fields)
        assert ctypes.sizeof(cls) == size, name
        assert [getattr(cls, f).offset for f in fields] == offs, name


def test_net_load_rejects_bad_files_before_any_device_call(tmp_path):
    """psc_net_load checks the file on the host first: a missing file, bad
    magic, a header for another network and a truncated file all return
    PSC_ERR_IO and a NULL handle (no GPU is touched on these paths)."""
    import struct
    from paper_2406_19754_amd import psc
    L = psc.lib()
    npar = psc.net_param_count()

    def load(path):
        h = ctypes.c_void_p(123)
        st = L.psc_net_load(os.fsencode(str(path)), None, ctypes.byref(h))
        return st, h.value

    def header(magic=b"PSCNET01", hb=40, np_=npar, ch=16, k=3, flags=1, t=5):
        return magic + struct.pack("<6Iq", hb, np_, ch, k, flags, 0, t)

    cases = {
        "missing": None,
        "magic": header(magic=b"NOTANET!") + bytes(12 * npar),
        "params": header(np_=npar + 1) + bytes(12 * npar),
        "channels": header(ch=8) + bytes(12 * npar),
        "flags": header(flags=2) + bytes(12 * npar),
        "truncated": header() + bytes(12 * npar - 4),
        "trailing": header() + bytes(12 * npar + 4),
        "short": b"PSCNET",
    }
    for name, blob in cases.items():
        path = tmp_path / name
        if blob is not None:
            path.write_bytes(blob)
        st, h = load(path)
        assert st == psc.ERR_IO, (name, st)
        assert h is None, name
        assert L.psc_last_error()


def test_shipped_network_checkpoint_header():
    """The trained 128^3 network ships in the checkpoint format psc_net_load reads."""
    import struct
    from paper_2406_19754_amd import psc
    path = os.path.join(ROOT, "paper_2406_19754_amd", "weights", "net_poisson128.ckpt")
    blob = open(path, "rb").read()
    hb, npar, ch, k, flags, _, t = struct.unpack("<6Iq", blob[8:40])
    assert blob[:8] == b"PSCNET01" and hb == 40 and npar == psc.net_param_count() and ch == 16 and k == 3
    assert len(blob) == 40 + 4 * npar * (3 if flags & 1 else 1)
