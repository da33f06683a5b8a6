"""CPU checks of the boundary: the built library loads and exports every
function the public header declares; the binding refuses to run without it."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bem.h")
LIB = os.path.join(ROOT, "paper_0908_0673_amd", "libbem.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w]+\s*\**\s*(bem_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_four_entry_points():
    names = declared()
    for n in ("bem_mesh_load", "bem_tree_build", "bem_matvec", "bem_solve"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbem.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_the_same_symbols():
    import paper_0908_0673_amd as bem

    assert sorted(bem.EXPORTED) == declared()


def test_binding_fails_loudly_without_library(tmp_path):
    import paper_0908_0673_amd as bem

    with pytest.raises(ImportError):
        bem._lib = None
        try:
            bem.load_library(str(tmp_path / "missing.so"))
        finally:
            bem._lib = None


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_0908_0673_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt and "bem_oracle" not in txt, f


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbem.so not built")
def test_server_options_are_checked_before_any_device_work():
    """Bad serving options are refused with BEM_EINVAL, and with no usable
    device the server reports BEM_EDEVICE (no host fallback)."""
    import paper_0908_0673_amd as bem

    L = bem.load_library()
    h = ctypes.c_void_p()
    o = bem._ServerOpts()
    o.lanes = -1
    assert L.bem_server_create(ctypes.byref(o), ctypes.byref(h)) == bem.BEM_EINVAL
    o.lanes, o.max_batch_rhs = 1, -3
    assert L.bem_server_create(ctypes.byref(o), ctypes.byref(h)) == bem.BEM_EINVAL
    o.max_batch_rhs, o.helmholtz_B = 1, -1
    assert L.bem_server_create(ctypes.byref(o), ctypes.byref(h)) == bem.BEM_EINVAL
    o.helmholtz_B = 0
    o.max_batch_rhs, o.device = 1, 1 << 20  # no such device
    assert L.bem_server_create(ctypes.byref(o), ctypes.byref(h)) == bem.BEM_EDEVICE
    assert not h.value
