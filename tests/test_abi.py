"""The C-ABI library loads and exports every symbol include/ahf.h declares
(CPU only: no compute call is made)."""
import ctypes as C
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ahf.h")
LIB = os.path.join(ROOT, "paper_0904_3662_amd", "libahf.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(ahf_[a-z_]+)\s*\(", text))
    # function-pointer typedefs are not functions
    return sorted(n for n in names if not n.endswith("_fn"))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_0904_3662_amd import build
        build.build()
    return C.CDLL(LIB)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("ahf_build_hierarchy", "ahf_label_refinements", "ahf_level_get",
              "ahf_hierarchy_order", "ahf_ctx_create"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_export():
    from paper_0904_3662_amd import ahf
    assert sorted(ahf.EXPORTS) == declared_functions()


def test_null_arguments_are_rejected_without_a_device(lib):
    lib.ahf_last_error.restype = C.c_char_p
    lib.ahf_hierarchy_num_levels.argtypes = [C.c_void_p, C.POINTER(C.c_uint32)]
    out = C.c_uint32(7)
    assert lib.ahf_hierarchy_num_levels(None, C.byref(out)) == -1
    assert out.value == 0
    assert b"NULL" in lib.ahf_last_error()
    lib.ahf_build_hierarchy.argtypes = [C.c_void_p] * 5
    h = C.c_void_p(1)
    assert lib.ahf_build_hierarchy(None, None, None, None, C.byref(h)) == -1
    assert h.value is None
    lib.ahf_hierarchy_free.argtypes = [C.c_void_p]
    lib.ahf_hierarchy_free(None)
    # the batch entry points check their arguments before touching a device
    lib.ahf_batch_create.argtypes = [C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p,
                                     C.c_uint32, C.c_uint32, C.c_void_p, C.c_void_p]
    b = C.c_void_p(1)
    assert lib.ahf_batch_create(None, 1, None, None, 4, 0, None, C.byref(b)) == -1
    assert b.value is None
    lib.ahf_batch_run.argtypes = [C.c_void_p, C.c_void_p]
    assert lib.ahf_batch_run(None, None) == -1
    lib.ahf_batch_wait.argtypes = [C.c_void_p]
    assert lib.ahf_batch_wait(None) == -1
    lib.ahf_batch_hierarchy.argtypes = [C.c_void_p, C.c_uint32, C.c_void_p]
    assert lib.ahf_batch_hierarchy(None, 0, C.byref(b)) == -1
    lib.ahf_batch_destroy.argtypes = [C.c_void_p]
    lib.ahf_batch_destroy(None)


def test_ctx_create_without_a_gpu_fails_cleanly():
    # run in a child so that a HIP runtime without devices cannot disturb this process
    code = (
        "import ctypes as C, sys\n"
        f"L = C.CDLL({LIB!r})\n"
        "class D(C.Structure):\n"
        "    _fields_=[('s',C.c_uint32),('d',C.c_int32),('a',C.c_void_p),('f',C.c_void_p),('u',C.c_void_p)]\n"
        "d = D(C.sizeof(D), 0, None, None, None)\n"
        "h = C.c_void_p()\n"
        "L.ahf_ctx_create.argtypes=[C.POINTER(D), C.POINTER(C.c_void_p)]\n"
        "rc = L.ahf_ctx_create(C.byref(d), C.byref(h))\n"
        "print(rc)\n"
    )
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().splitlines()[-1] == str(-3)


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    from paper_0904_3662_amd import ahf
    monkeypatch.setattr(ahf, "LIB_PATH", str(tmp_path / "libahf.so"))
    monkeypatch.setattr(ahf, "_lib", None)
    with pytest.raises(RuntimeError):
        ahf.load()
