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
