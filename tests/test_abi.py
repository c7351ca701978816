"""C ABI checks that need no GPU: the library loads, exports every function
include/reap_spgemm.h declares, and rejects bad arguments before any device
call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "reap_spgemm.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(reap_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2004_13907_amd import _capi, build
    if build.is_stale():
        build.build()
    return _capi.load()


def test_header_declares_the_four_entry_points():
    names = _declared()
    for n in ("reap_spgemm_create", "reap_spgemm_symbolic", "reap_spgemm_numeric", "reap_spgemm_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2004_13907_amd import _capi
    names = _declared()
    assert sorted(_capi.EXPORTED) == names
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(lib):
    for s in range(8):
        assert lib.reap_status_string(s) != b"unknown status"
    assert lib.reap_status_string(99) == b"unknown status"
    assert lib.reap_version() == b"0.2.0"


def test_null_arguments_rejected_without_gpu(lib):
    from paper_2004_13907_amd import _capi
    assert lib.reap_spgemm_create(None, 1, 0, None, None) == _capi.REAP_ERR_INVALID_ARG
    h = ctypes.c_void_p()
    assert lib.reap_spgemm_create(ctypes.byref(h), 7, 0, None, None) == _capi.REAP_ERR_INVALID_ARG
    assert not h.value
    assert lib.reap_spgemm_create(ctypes.byref(h), 1, 5, None, None) == _capi.REAP_ERR_INVALID_ARG
    assert lib.reap_spgemm_symbolic(None, None, None, None, None, None, None) == _capi.REAP_ERR_INVALID_ARG
    assert lib.reap_spgemm_numeric(None, None, None, None, None, None) == _capi.REAP_ERR_INVALID_ARG
    assert lib.reap_spgemm_destroy(None) == _capi.REAP_OK
    assert lib.reap_spgemm_bin_stats(None, None) == _capi.REAP_ERR_INVALID_ARG
    assert lib.reap_spgemm_phase_times(None, None, 0) == _capi.REAP_ERR_INVALID_ARG


def test_struct_layout_matches_header(tmp_path):
    """Size and field offsets of every ctypes struct equal the C header's,
    as compiled by the host C compiler."""
    import shutil
    import subprocess
    from paper_2004_13907_amd import _capi
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = [_capi.reap_csr_t, _capi.reap_options_t, _capi.reap_bin_stats_t]
    lines = ['#include "reap_spgemm.h"', "#include <stddef.h>", "#include <stdio.h>", "int main(void) {"]
    for st in structs:
        name = st.__name__
        lines.append('printf("%%s %%zu\\n", "%s", sizeof(%s));' % (name, name))
        for f, _ in st._fields_:
            lines.append('printf("%%s.%%s %%zu\\n", "%s", "%s", offsetof(%s, %s));' % (name, f, name, f))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cc, "-I", inc, "-o", str(exe), str(src)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                      text=True).stdout.splitlines())
    for st in structs:
        name = st.__name__
        assert int(got[name]) == ctypes.sizeof(st), name
        for f, _ in st._fields_:
            assert int(got["%s.%s" % (name, f)]) == getattr(st, f).offset, (name, f)


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2004_13907_amd import _capi
    monkeypatch.setattr(_capi, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_capi, "_lib", None)
    with pytest.raises(RuntimeError):
        _capi.load()


def test_create_without_a_device_fails_cleanly(lib):
    """With no GPU visible, create returns REAP_ERR_HIP, leaves the handle
    NULL, and destroy(NULL) is accepted (the CPU tier's view of the plan's
    error path; allocation failures are forced by the test_fail_alloc hook in
    the GPU tests)."""
    torch = pytest.importorskip("torch")
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is visible")
    from paper_2004_13907_amd import _capi
    h = ctypes.c_void_p()
    opts = _capi.reap_options_t()
    opts.test_fail_alloc = 1
    st = lib.reap_spgemm_create(ctypes.byref(h), _capi.REAP_F64, _capi.REAP_I32, None, ctypes.byref(opts))
    assert st == _capi.REAP_ERR_HIP and not h.value
    assert lib.reap_spgemm_destroy(None) == _capi.REAP_OK
    size = ctypes.c_size_t(0)
    assert lib.reap_spgemm_workspace_query(None, 1, None, None, ctypes.byref(size)) == _capi.REAP_ERR_INVALID_ARG
