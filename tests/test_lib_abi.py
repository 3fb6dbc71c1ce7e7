"""The C-ABI library loads and exports every symbol its header declares (CPU;
no compute calls)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(fn_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ["fn_nll", "fn_nll_async", "fn_model_create", "fn_fit", "fn_norm", "fn_eval", "fn_events_check"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1710_08826_amd import _lib
    lib = _lib.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_python_prototypes_cover_header():
    from paper_1710_08826_amd import _lib
    assert set(declared_functions()) <= set(_lib.PROTOTYPES)


def test_version_and_error_string():
    from paper_1710_08826_amd import _lib
    lib = _lib.load()
    assert lib.fn_version() >= 10000
    assert isinstance(lib.fn_last_error(), bytes)


def test_null_arguments_rejected_without_gpu():
    """Argument checks run before any device call."""
    from paper_1710_08826_amd import _lib
    lib = _lib.load()
    assert lib.fn_model_create(None, b"{}", None) == _lib.FN_E_INVALID
    assert lib.fn_nll(None, None, None, 0, 0, None, None, None) == _lib.FN_E_INVALID
    assert lib.fn_model_info(None, None, None, None) == _lib.FN_E_INVALID
    assert b"NULL" in lib.fn_last_error()


def test_missing_library_fails_loudly(tmp_path):
    from paper_1710_08826_amd import _lib
    with pytest.raises(RuntimeError):
        _lib._lib, saved = None, _lib._lib
        try:
            _lib.load(str(tmp_path / "nope.so"))
        finally:
            _lib._lib = saved


def test_struct_layouts_match_header(tmp_path):
    """sizeof/offsetof of the request/result structs, compiled from the C
    header with gcc, equal the ctypes mirrors in the binding."""
    import subprocess
    from paper_1710_08826_amd import api
    src = tmp_path / "s.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "fitnll.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu\\n", sizeof(fn_request), sizeof(fn_result),'
                   ' offsetof(fn_request, arrival_s), offsetof(fn_result, t_done), offsetof(fn_result, theta));'
                   'return 0;}\n')
    exe = tmp_path / "s"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    got = [int(v) for v in out]
    want = [C.sizeof(api._Request), C.sizeof(api._Result), api._Request.arrival_s.offset,
            api._Result.t_done.offset, api._Result.theta.offset]
    assert got == want


def test_model_kernels_compile_for_gfx950_without_a_device():
    """The structure-specialized kernels of amplitude models are compiled at
    run time; the same compilation runs here on the CPU for gfx950."""
    import json
    import synth
    from paper_1710_08826_amd import _lib
    lib = _lib.load()
    for free in (False, True):
        d = synth.dalitz_desc(free_lineshapes=free)
        assert lib.fn_model_check_compile(json.dumps(d).encode(), b"gfx950") == _lib.FN_OK, lib.fn_last_error()
        # the events passes with two events per thread and loop iteration
        d["events_per_thread"] = 2
        assert lib.fn_model_check_compile(json.dumps(d).encode(), b"gfx950") == _lib.FN_OK, lib.fn_last_error()
        d["events_per_thread"] = 3
        assert lib.fn_model_check_compile(json.dumps(d).encode(), None) == _lib.FN_E_INVALID
    d = synth.td4_desc()
    d["events_per_thread"] = 2
    assert lib.fn_model_check_compile(json.dumps(d).encode(), None) == _lib.FN_E_INVALID
    # a two-resonance model in one pair with spins 0 and 2 only
    d = synth.dalitz_desc()
    d["resonances"] = [{"pair": "13", "L": 0, "m0": 1.43, "w0": 0.27}, {"pair": "13", "L": 2, "m0": 1.43, "w0": 0.1}]
    assert lib.fn_model_check_compile(json.dumps(d).encode(), None) == _lib.FN_OK, lib.fn_last_error()
    # the time-dependent three- and four-body models
    for d in (synth.tddp3_desc(), synth.td4_desc(), synth.td4_split_desc()):
        assert lib.fn_model_check_compile(json.dumps(d).encode(), b"gfx950") == _lib.FN_OK, lib.fn_last_error()
    bad = synth.dalitz_desc()
    bad["resonances"][0]["pair"] = "14"
    assert lib.fn_model_check_compile(json.dumps(bad).encode(), None) == _lib.FN_E_INVALID
    assert lib.fn_model_check_compile(b"{not json", None) == _lib.FN_E_INVALID
