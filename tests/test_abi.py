"""The C-ABI library loads and exports every function include/mfm.h declares (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mfm.h")
LIB = os.path.join(ROOT, "paper_1712_01294_amd", "libmfm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mfm_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1712_01294_amd import build
        build.build()
    return C.CDLL(LIB)


def test_header_declares_the_pass_calls():
    names = declared_functions()
    for f in ("mfm_create", "mfm_destroy", "mfm_build_neighbours", "mfm_solve_h", "mfm_gradients",
              "mfm_hydro_fluxes", "mfm_step", "mfm_get_counters"):
        assert f in names


def test_every_declared_symbol_is_exported(lib):
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_binding_lists_every_export():
    from paper_1712_01294_amd import mfm
    assert set(declared_functions()) <= set(mfm.EXPORTS)


def test_status_strings_are_host_only(lib):
    lib.mfm_status_str.restype = C.c_char_p
    lib.mfm_status_str.argtypes = [C.c_int]
    assert lib.mfm_status_str(0) == b"ok"
    assert b"capacity" in lib.mfm_status_str(-6)
    assert lib.mfm_status_str(123) == b"unknown status"


def test_create_rejects_bad_parameters_before_touching_the_device(lib):
    from paper_1712_01294_amd import mfm
    lib.mfm_create.argtypes = [C.POINTER(mfm.Params), C.c_int64, C.POINTER(C.c_void_p)]
    good = mfm.Config(gamma=5 / 3, box=(1, 1, 1))
    h = C.c_void_p()
    for bad in (dict(gamma=1.0), dict(n_ngb=10.0), dict(box=(1, 0, 1)), dict(beta=0.0),
                dict(precision=7), dict(scheme=7)):
        cfg = mfm.Config(**{**good.__dict__, **bad})
        assert lib.mfm_create(C.byref(cfg.c()), 1000, C.byref(h)) == -1
        assert not h.value
    assert lib.mfm_create(C.byref(good.c()), 0, C.byref(h)) == -1
    assert lib.mfm_create(None, 10, C.byref(h)) == -1


def test_binding_structs_match_the_header_layout(tmp_path):
    """sizeof and every field offset of the three structs, from a C compile of the header."""
    import shutil
    import subprocess
    from paper_1712_01294_amd import mfm
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"mfm_params": mfm.Params, "mfm_particles": mfm.Particles, "mfm_counters": mfm.Counters}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mfm.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines += ['return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                       text=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)
