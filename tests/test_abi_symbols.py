"""The C-ABI library loads on the host and exports every declared entry point
(no compute call: there may be no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h")]
LIB = os.path.join(ROOT, "paper_1607_00693_amd", "libstomsfem.so")


def declared_functions():
    names = []
    for h in HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(stomsfem_[A-Za-z0-9_]+)\s*\(", src, re.M):
            names.append(m.group(1))
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("stomsfem_upscale", "stomsfem_coarse_solve", "stomsfem_coef_bumps"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"
    lib.stomsfem_version.restype = ctypes.c_int
    assert lib.stomsfem_version() == 1


def test_binding_fails_loudly_without_the_library(tmp_path, monkeypatch):
    # the product path has no CPU fallback: a missing library is an error
    from paper_1607_00693_amd import stomsfem

    monkeypatch.setattr(stomsfem, "_lib", None)
    monkeypatch.setattr(stomsfem, "LIB_PATH", str(tmp_path / "libstomsfem.so"))
    with pytest.raises(RuntimeError, match="missing"):
        stomsfem.lib()
    with pytest.raises(RuntimeError, match="missing"):
        stomsfem.version()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_validation_without_gpu():
    # argument checks run on the host before anything touches a device
    lib = ctypes.CDLL(LIB)
    lib.stomsfem_coarse_solve.restype = ctypes.c_int
    rc = lib.stomsfem_coarse_solve(ctypes.c_int32(0), ctypes.c_int32(3), ctypes.c_int64(1), None, None, None, None,
                                   None, None, None)
    assert rc == -1  # EINVAL: ncx < 1
    lib.stomsfem_last_error.restype = ctypes.c_char_p
    assert b"bad sizes" in lib.stomsfem_last_error()
    lib.stomsfem_autotune.restype = ctypes.c_int
    assert lib.stomsfem_autotune(None, ctypes.c_int32(1), None, None) == -1
    lib.stomsfem_plan_create.restype = ctypes.c_int
    assert lib.stomsfem_plan_create(None, ctypes.c_int32(0), None) == -1
    # oversampling / Petrov-Galerkin entry points
    lib.stomsfem_upscale_os.restype = ctypes.c_int
    assert lib.stomsfem_upscale_os(None, ctypes.c_int32(4), None) == -1
    assert b"NULL batch" in lib.stomsfem_last_error()
    lib.stomsfem_coarse_solve_pg.restype = ctypes.c_int
    rc = lib.stomsfem_coarse_solve_pg(ctypes.c_int32(65), ctypes.c_int32(3), ctypes.c_int64(1), None, None, None,
                                      None, None, None, None)
    assert rc == -1 and b"ncx <= 64" in lib.stomsfem_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_model_file_rejections_and_counters_on_host(tmp_path):
    # rejected before any device work: missing file, foreign file, wrong ABI version
    import struct

    from paper_1607_00693_amd import stomsfem

    with pytest.raises(stomsfem.StomsfemError) as e:
        stomsfem.model_load(str(tmp_path / "nothing.bin"))
    assert e.value.code == stomsfem.EINVAL
    junk = tmp_path / "junk.bin"
    junk.write_bytes(b"not a model file at all" * 10)
    with pytest.raises(stomsfem.StomsfemError) as e:
        stomsfem.model_load(str(junk))
    assert e.value.code == stomsfem.EVERSION
    old = tmp_path / "old.bin"
    old.write_bytes(b"STOMSFEM" + struct.pack("<II", 999, 3) + bytes(200))
    with pytest.raises(stomsfem.StomsfemError) as e:
        stomsfem.model_load(str(old))
    assert e.value.code == stomsfem.EVERSION
    stomsfem.stats_reset()
    assert all(v == 0 for v in stomsfem.stats_get().values())


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_noalloc_coarse_solve_validates_on_the_host():
    # the entry point for callers that cannot allocate checks its arguments
    # before touching a device: bad sizes, and a mesh beyond the coarse LDS window
    lib = ctypes.CDLL(LIB)
    f = lib.stomsfem_coarse_solve_noalloc
    f.restype = ctypes.c_int
    lib.stomsfem_last_error.restype = ctypes.c_char_p
    args = [None] * 7
    assert f(ctypes.c_int32(0), ctypes.c_int32(3), ctypes.c_int64(1), *args) == -1
    assert b"bad sizes" in lib.stomsfem_last_error()
    assert f(ctypes.c_int32(2000), ctypes.c_int32(3), ctypes.c_int64(1), *args) == -1
    assert f(ctypes.c_int32(3), ctypes.c_int32(3), ctypes.c_int64(-1), *args) == -1
