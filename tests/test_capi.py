"""Host-side checks of the C ABI: the library loads and exports every function
that include/pixelsne.h declares, the ctypes layouts match, and argument
validation rejects bad calls before any device work (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pixelsne.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pixelsne3?_[a-z_A-Z0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def psne():
    from paper_1611_02568_amd import pixelsne
    pixelsne.load()
    return pixelsne


def test_every_declared_symbol_is_exported(psne):
    names = _declared()
    assert len(names) >= 15
    lib = C.CDLL(psne.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding declares a signature for exactly these functions
    assert sorted(psne.SIGNATURES) == names


def test_params_layout_matches(psne):
    p = psne.default_params()
    assert p.struct_size == C.sizeof(psne.Params)
    assert (p.theta, p.eta, p.exaggeration, p.exag_iters, p.mom_switch) == (0.5, 200.0, 12.0, 250, 250)
    assert (p.mom0, p.mom1, p.min_gain, p.eps, p.init_sigma) == (0.5, 0.8, 0.01, 1e-6, 1e-4)
    assert (p.reorder_every, p.reorder_growth, p.data_order, p.graphs) == (100, 2.0, 1, 1)


def _init(psne, X, n, D, u, w, h, **kw):
    p = psne.default_params(**kw)
    return psne.load().pixelsne_init_ex(X, n, D, u, w, h, C.byref(p))


@pytest.mark.parametrize("args,frag", [
    ((10, 4, 3.0, 512, 512), "device pointer"),        # host pointer for X
    ((1, 4, 3.0, 512, 512), "n must be"),
    ((10, 0, 3.0, 512, 512), "D must be"),
    ((10, 4, -1.0, 512, 512), "perplexity"),
    ((10, 4, 5.0, 512, 512), "k = floor"),             # k = 15 > n - 1
    ((10, 4, 3.0, 512, 256), "square"),
    ((10, 4, 3.0, 500, 500), "power of two"),
    ((10, 4, 3.0, 1, 1), "screen size"),
])
def test_init_validation(psne, args, frag):
    X = np.zeros((10, 4), np.float32)
    h = _init(psne, X.ctypes.data, *args)
    assert not h
    assert frag in psne.load().pixelsne_last_error().decode()


@pytest.mark.parametrize("kw,frag", [({"theta": 1.0}, "theta"), ({"precision": 7}, "precision"),
                                     ({"com_mode": 3}, "com_mode"), ({"struct_size": 8}, "struct_size"),
                                     ({"eta": 0.0}, "eta"), ({"reorder_growth": 0.5}, "reorder_growth"),
                                     ({"reorder_every": -1}, "reorder_every"),
                                     ({"attract_blocks_per_cu": 17}, "attract_blocks_per_cu"),
                                     ({"attract_help_blocks_per_cu": -1},
                                      "attract_help_blocks_per_cu"),
                                     ({"attract_blocks_per_cu": 0,
                                       "attract_help_blocks_per_cu": 0}, "both 0"),
                                     ({"attract_fork": 3}, "attract_fork")])
def test_params_validation(psne, kw, frag):
    X = np.zeros((10, 4), np.float32)
    assert not _init(psne, X.ctypes.data, 10, 4, 3.0, 512, 512, **kw)
    assert frag in psne.load().pixelsne_last_error().decode()


def test_null_context_calls(psne):
    lib = psne.load()
    assert lib.pixelsne_step(None, 1) == psne.PSNE_E_INVAL
    assert lib.pixelsne_get_Y(None, None, 0) == psne.PSNE_E_INVAL
    lib.pixelsne_destroy(None)
    assert lib.pixelsne_knn(None, 10, 4, 0, 20, None, None, None) == psne.PSNE_E_INVAL
    assert lib.pixelsne_perplexity(None, 10, 5, -2.0, None, None, None) == psne.PSNE_E_INVAL
    assert lib.pixelsne_kl(None, None) == psne.PSNE_E_INVAL
    assert lib.pixelsne_knn2d(None, None) == psne.PSNE_E_INVAL
    assert lib.pixelsne_neighborhood_precision(None, None, 10, None, 1, None) == psne.PSNE_E_INVAL


def test_null_context_calls_3d(psne):
    lib = psne.load()
    assert lib.pixelsne3_step(None, 1) == psne.PSNE_E_INVAL
    assert lib.pixelsne3_get_Y(None, None, 0) == psne.PSNE_E_INVAL
    assert lib.pixelsne3_kl(None, None) == psne.PSNE_E_INVAL
    assert lib.pixelsne3_gradient(None, 1.0, None, None, None, None, None, None) == psne.PSNE_E_INVAL
    lib.pixelsne3_destroy(None)


@pytest.mark.parametrize("kw,r,n,frag", [
    ({}, 64, 10, "device pointers"),                            # host CSR pointers
    ({"precision": 0}, 64, 10, "FP64"),
    ({"com_mode": 1}, 64, 10, "FP64"),
    ({"tree": 1}, 64, 10, "FP64"),
    ({}, 2048, 10, "power of two in [2, 1024]"),
    ({}, 48, 10, "power of two in [2, 1024]"),
    ({}, 64, 1, "n must be"),
    ({"theta": 1.0}, 64, 10, "theta"),
])
def test_init3_validation(psne, kw, r, n, frag):
    kw = dict({"precision": 1}, **kw)
    p = psne.default_params(**kw)
    rp = np.zeros(n + 1, np.int64)
    col = np.zeros(4, np.int32)
    val = np.zeros(4)
    h = psne.load().pixelsne3_init_with_P(n, 4, rp.ctypes.data, col.ctypes.data, val.ctypes.data,
                                          r, C.byref(p))
    assert not h
    assert frag in psne.load().pixelsne_last_error().decode()


def test_struct_layouts_match_header(psne, tmp_path):
    """Every struct the binding mirrors has the header's size and field
    offsets, as a C compiler lays them out (gcc on the header itself)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = [("pixelsne_params", psne.Params), ("pixelsne_stats", psne.Stats),
               ("pixelsne_pass_times", psne.PassTimes),
               ("pixelsne_refine_result", psne.RefineResult)]
    lines = ["#include <stddef.h>", "#include <stdio.h>", f'#include "{HEADER}"',
             "int main(void) {"]
    for cname, cls in structs:
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in cls._fields_:
            lines.append(f'    printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-o", str(exe), str(src)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True,
                               text=True).stdout.splitlines():
        name, key, val = line.split()
        got[(name, key)] = int(val)
    for cname, cls in structs:
        assert got[(cname, "size")] == C.sizeof(cls), cname
        for field, _ in cls._fields_:
            assert got[(cname, field)] == getattr(cls, field).offset, (cname, field)


def test_enum_constants_match_header(psne):
    """Every PSNE_* enumerator of the header has the value the binding uses
    (the binding's name drops the prefix, except for the status codes)."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    values = {}
    for body in re.findall(r"\benum\s*\{(.*?)\}", src, flags=re.S):
        for name, val in re.findall(r"\b(PSNE_[A-Z0-9_]+)\s*=\s*(-?\d+)", body):
            values[name] = int(val)
    assert len(values) >= 20
    for name, val in values.items():
        py = name if name.startswith(("PSNE_OK", "PSNE_E_")) else name[len("PSNE_"):]
        assert getattr(psne, py) == val, (name, getattr(psne, py, None), val)


def _c_kind(decl):
    """The ABI kind of a C declaration ("const double* s" -> "ptr")."""
    decl = decl.strip()
    if "*" in decl:
        return "ptr"
    words = [w for w in decl.replace("const ", "").split() if w]
    base = words[0]
    return {"int32_t": "i32", "int64_t": "i64", "uint64_t": "u64", "double": "f64",
            "float": "f32", "int": "i32", "psne_status": "i32", "void": "void"}[base]


def _py_kind(t):
    if t is None:
        return "void"
    if t in (C.c_void_p, C.c_char_p) or (isinstance(t, type) and issubclass(t, C._Pointer)):
        return "ptr"
    return {C.c_int32: "i32", C.c_int: "i32", C.c_int64: "i64", C.c_uint64: "u64",
            C.c_double: "f64", C.c_float: "f32"}[t]


def test_signatures_match_header(psne):
    """Each declared function's return and parameter kinds (pointer, 32/64-bit
    integer, float, double) equal the binding's restype and argtypes."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    protos = re.findall(r"([A-Za-z_][\w\s\*]*?)\b(pixelsne3?_\w+)\s*\(([^)]*)\)\s*;", src)
    seen = set()
    for ret, name, params in protos:
        params = params.strip()
        args = [] if params in ("", "void") else [p for p in params.split(",")]
        restype, argtypes = psne.SIGNATURES[name]
        ret_kind = "ptr" if "*" in ret else _c_kind(ret.split()[-1])
        assert _py_kind(restype) == ret_kind, (name, "return")
        assert [_c_kind(a) for a in args] == [_py_kind(t) for t in argtypes], name
        seen.add(name)
    assert seen == set(psne.SIGNATURES)


def test_c_program_links_and_calls(psne, tmp_path):
    """A C program built against the header and linked with the library (no
    Python in between) reads the defaults and gets a clean refusal for a bad
    call, which does no device work."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use.c"
    src.write_text(
        f'#include "{HEADER}"\n'
        "#include <stdio.h>\n"
        "int main(void) {\n"
        "    pixelsne_params p;\n"
        "    pixelsne_default_params(&p);\n"
        "    pixelsne_ctx* c = pixelsne_init(NULL, 1, 4, 3.0, 512, 512);\n"
        '    printf("%g %d %d %s\\n", p.theta, p.exag_iters, c == NULL,\n'
        "           pixelsne_last_error());\n"
        "    return 0;\n"
        "}\n")
    lib = os.path.dirname(psne.LIB_PATH)
    exe = tmp_path / "use"
    subprocess.run([cc, "-std=c11", "-o", str(exe), str(src), f"-L{lib}", "-lpixelsne",
                    f"-Wl,-rpath,{lib}"], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    assert out[:3] == ["0.5", "250", "1"]
    assert " ".join(out[3:]).startswith("n must be")
