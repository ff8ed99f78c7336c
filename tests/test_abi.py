"""Host-side checks of the C ABI (no GPU needed): the library loads and exports every
function include/lesmi.h declares, and the binding's parameter struct matches the header."""
import ctypes
import re

from paper_2212_12365_amd import lesmi


def test_library_exports_every_declared_function():
    lib = lesmi.load()
    names = lesmi.header_functions()
    assert {"les_init_grid", "les_residual", "les_step", "les_sgs_viscosity"} <= set(names)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_params_struct_layout_matches_header():
    text = open(lesmi.HEADER).read()
    body = text[text.index("typedef struct {", text.index("les_closure;")):text.index("} les_params;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"\b(int|double)\s+([^;]+);", body)
    declared = []
    for typ, names in fields:
        for nm in names.split(","):
            nm = nm.strip()
            base = re.match(r"[a-z_0-9]+", nm).group(0)
            dims = [int(x) for x in re.findall(r"\[(\d+)\]", nm)]
            count = 1
            for d in dims:
                count *= d
            declared.append((base, typ, count))
    ours = []
    for name, ctype in lesmi.les_params._fields_:
        base = "int" if ctype in (ctypes.c_int,) or getattr(ctype, "_type_", None) is ctypes.c_int \
            else "double"
        count = getattr(ctype, "_length_", 1)
        ours.append((name, base, count))
    assert declared == ours


def test_oversized_grid_is_rejected_before_any_device_call():
    """Grids whose per-node planes would overflow the kernels' 32-bit offsets are refused by
    les_init_grid's parameter check, which runs before any HIP call (no GPU here)."""
    import numpy as np
    import synthetic as sy
    lib = lesmi.load()
    text = open(lesmi.HEADER).read()
    limit = int(re.search(r"#define LES_MAX_NODES (\d+)LL", text).group(1))
    assert limit == (2 ** 31 - 1) // 11
    dummy = np.zeros(3)
    for n in [(581, 581, 579), (1200, 600, 300), (4096, 4096, 16)]:
        assert n[0] * n[1] * n[2] > limit
        for p in (sy.jet_params(n), sy.box_params(n, np.zeros((3, 3)))):
            s = lesmi.make_params(p)
            h = ctypes.c_void_p(1)
            rc = lib.les_init_grid(ctypes.byref(s),
                                   dummy.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   ctypes.byref(h))
            assert rc == lesmi.LES_EINVAL
            assert not h.value


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built library the binding raises at once: there is no fallback path that
    would compute anything elsewhere."""
    import pytest
    monkeypatch.setattr(lesmi, "LIB_PATH", str(tmp_path / "liblesmi.so"))
    monkeypatch.setattr(lesmi, "_lib", None)
    with pytest.raises(RuntimeError, match="is not built"):
        lesmi.load()
