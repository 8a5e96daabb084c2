"""The C-ABI library loads on a machine without a GPU, exports every declared entry point,
and rejects invalid arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "frpca.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1810_06825_amd import binding

    if not os.path.exists(binding.LIB_PATH):
        from paper_1810_06825_amd.build import build_library

        build_library()
    return binding.load()


def declared_entry_points():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(frpca_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_entry_points()
    for required in ("frpca_create", "frpca_run", "frpca_backward", "frpca_destroy", "frpca_get_info",
                     "frpca_last_error", "frpca_set_values"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    from paper_1810_06825_amd import binding

    names = declared_entry_points()
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(binding.exported_symbols()) == names


def test_options_struct_matches_header():
    """The ctypes mirror of frpca_opts lists the header's fields in the header's order."""
    from paper_1810_06825_amd import binding

    text = open(HEADER).read()
    body = re.search(r"typedef struct \{(.*?)\} frpca_opts;", text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"^\s*(?:int|double|size_t)\s+(\w+);", body, re.M)
    assert fields == [f[0] for f in binding.FrpcaOpts._fields_]


def test_invalid_arguments_rejected_without_gpu(lib):
    from paper_1810_06825_amd import binding

    h = ctypes.c_void_p()
    o = binding.FrpcaOpts()
    assert lib.frpca_create(ctypes.byref(h), 0, 5, 0, None, None, None, ctypes.byref(o), None) == binding.FRPCA_EINVAL
    assert h.value is None
    assert "m, n" in binding.frpca_last_error(None)
    assert lib.frpca_create(ctypes.byref(h), 4, 5, -1, None, None, None, ctypes.byref(o), None) == binding.FRPCA_EINVAL
    assert lib.frpca_create(ctypes.byref(h), 4, 5, 3, None, None, None, ctypes.byref(o), None) == binding.FRPCA_EINVAL
    o.rank_tol = 2.0
    assert lib.frpca_create(ctypes.byref(h), 4, 5, 0, 1, None, None, ctypes.byref(o), None) == binding.FRPCA_EINVAL
    for call in (lambda: lib.frpca_run(None, 5, 3, 2, 1, None, None, None),
                 lambda: lib.frpca_backward(None, None, None, None, None),
                 lambda: lib.frpca_adjoint(None, 5, None, None, None, None, None, None, None),
                 lambda: lib.frpca_set_values(None, None),
                 lambda: lib.frpca_spmm(None, 0, 4, None, 0, 4, None, 0, 4)):
        assert call() == binding.FRPCA_EINVAL
    assert lib.frpca_destroy(None) == binding.FRPCA_OK


def test_binding_raises_on_error(lib):
    from paper_1810_06825_amd import binding

    with pytest.raises(binding.FrpcaError) as ei:
        binding.frpca_create(0, 1, 0, None, None, None)
    assert ei.value.code == binding.FRPCA_EINVAL


def test_product_path_has_no_oracle_dependency():
    # the package never imports the oracle (test infrastructure only)
    pkg = os.path.join(ROOT, "paper_1810_06825_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", src, flags=re.M), f
