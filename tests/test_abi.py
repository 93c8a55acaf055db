"""The C-ABI library loads and exports every entry point that
include/vfstokes.h declares (no compute calls: no GPU needed)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")
LIB = os.path.join(ROOT, "paper_1010_2832_amd", "libvfstokes.so")


def declared_symbols():
    names = set()
    for f in os.listdir(HEADER_DIR):
        if not f.endswith(".h"):
            continue
        text = open(os.path.join(HEADER_DIR, f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        for m in re.finditer(r"\b(vfs_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "libvfstokes.so is not built"
    lib = ctypes.CDLL(LIB)
    names = declared_symbols()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    from paper_1010_2832_amd import vfstokes
    assert set(declared_symbols()) <= set(vfstokes.EXPORTED)


def test_create_error_without_device_is_reported():
    """Creating a context either succeeds (GPU present) or fails with a
    message, never silently."""
    from paper_1010_2832_amd import vfstokes
    try:
        ctx = vfstokes.Context(2, (4, 4), 0.25)
        ctx.close()
    except vfstokes.VfsError as e:
        assert str(e)


def test_invalid_arguments_rejected_before_any_device_work():
    from paper_1010_2832_amd import vfstokes
    for args in ((4, 8, 8, 1, 0.1), (2, 0, 8, 1, 0.1), (2, 8, 8, 1, -1.0), (2, 8, 8, 1, float("nan"))):
        try:
            vfstokes.vfs_create(*args)
            raise AssertionError("expected failure")
        except vfstokes.VfsError as e:
            assert e.code == vfstokes.VFS_EINVAL
