"""CPU-side checks of the C ABI: the library loads, exports every symbol the header
declares, and the host-only calls validate their inputs.  No device work."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ptlm.h")

pt = pytest.importorskip("paper_2103_01767_amd")


def header_functions():
    text = open(HEADER).read()
    return re.findall(r"^(?:ptlm_status|void|const char\*|ptlm_handle\*)\s+(ptlm_\w+)\s*\(", text, re.M)


def test_every_declared_symbol_is_exported_and_bound():
    names = header_functions()
    assert len(names) >= 15
    lib = ctypes.CDLL(pt.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(pt.EXPORTS)


def header_enum_values():
    """name -> value of every enumerator the header defines"""
    text = open(HEADER).read()
    out = {}
    for body in re.findall(r"typedef enum\s*\{([^}]*)\}", text):
        for name, val in re.findall(r"(PTLM_\w+)\s*=\s*(-?\d+)", body):
            out[name] = int(val)
    return out


def test_binding_constants_match_the_header():
    """The binding's status codes, metric / mode / GGN codes and transform names carry the
    header's values."""
    e = header_enum_values()
    for name in ("PTLM_OK", "PTLM_ENOTACCEPTED", "PTLM_EINVAL", "PTLM_EWORKSPACE", "PTLM_EHIP", "PTLM_ENUMERIC"):
        assert getattr(pt, name) == e[name], name
    assert (pt.GAUSS, pt.POISSON) == (e["PTLM_GAUSS"], e["PTLM_POISSON"])
    assert (pt.OBJECT, pt.JOINT) == (e["PTLM_OBJECT"], e["PTLM_JOINT"])
    assert (pt.GGN_MAGNITUDE, pt.GGN_INTENSITY) == (e["PTLM_GGN_MAGNITUDE"], e["PTLM_GGN_INTENSITY"])
    transforms = {k: v for k, v in e.items() if k.startswith("PTLM_TRANSFORM_")}
    assert len(pt.TRANSFORMS) == len(transforms)
    for name, value in transforms.items():
        assert pt.TRANSFORMS[value] == name[len("PTLM_TRANSFORM_"):].lower(), name


def _ws(desc, pos):
    n = ctypes.c_size_t(0)
    st = pt.lib().ptlm_workspace_bytes(ctypes.byref(desc), pos.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n))
    return st, n.value


def test_workspace_validation():
    pos = np.array([[0, 0], [8, 8], [16, 0]], np.int32)
    d = pt.ptlm_desc(48, 40, 32, 16, 3, pt.GAUSS, pt.JOINT, 1e-8)
    st, n = _ws(d, pos)
    assert st == pt.PTLM_OK and n > 3 * 32 * 16 * 8
    for bad in ([17, 0], [0, 25], [-1, 0]):
        p2 = pos.copy()
        p2[2] = bad
        assert _ws(d, p2)[0] == pt.PTLM_EINVAL
        assert b"position 2" in pt.lib().ptlm_last_error()
    for field, val in (("my", 48), ("mx", 24), ("K", 0), ("metric", 7), ("mode", 3), ("background", 0.0),
                       ("ggn", 2), ("seg_len", -1)):
        d2 = pt.ptlm_desc(48, 40, 32, 16, 3, pt.GAUSS, pt.JOINT, 1e-8)
        setattr(d2, field, val)
        assert _ws(d2, pos)[0] == pt.PTLM_EINVAL, field
    # the intensity-based GGN keeps the square root of its weight per measurement, as Poisson does
    d_int = pt.ptlm_desc(48, 40, 32, 16, 3, pt.GAUSS, pt.JOINT, 1e-8, pt.GGN_INTENSITY)
    d_poi = pt.ptlm_desc(48, 40, 32, 16, 3, pt.POISSON, pt.JOINT, 1e-8)
    n_int, n_poi = _ws(d_int, pos)[1], _ws(d_poi, pos)[1]
    assert n_int == n_poi >= n + 3 * 32 * 16 * 4
    # more positions need more workspace (stored phasor field grows with K)
    many = np.array([[i % 17, i % 25] for i in range(40)], np.int32)
    d3 = pt.ptlm_desc(48, 40, 32, 16, 40, pt.GAUSS, pt.JOINT, 1e-8)
    assert _ws(d3, many)[1] > n
    # seg_len caps the segment count: fewer probe partials and strips to hold
    d4 = pt.ptlm_desc(48, 40, 32, 16, 40, pt.GAUSS, pt.JOINT, 1e-8)
    d4.seg_len = 10
    assert _ws(d4, many)[0] == pt.PTLM_OK and _ws(d4, many)[1] < _ws(d3, many)[1]


def test_large_probe_shapes():
    """48, 96 and 256 are planned as square probes only; 256 x 256 adds per-workgroup transform tiles."""
    pos = np.array([[0, 0], [16, 16], [32, 0]], np.int32)
    d = pt.ptlm_desc(300, 300, 256, 256, 3, pt.GAUSS, pt.JOINT, 1e-8)
    st, n = _ws(d, pos)
    assert st == pt.PTLM_OK
    # phasor field + probe slots + transform tiles: at least 3 * 3 tiles of 512 KiB
    assert n >= 9 * 256 * 256 * 8
    for side in (48, 96):
        d1 = pt.ptlm_desc(300, 300, side, side, 3, pt.GAUSS, pt.JOINT, 1e-8)
        assert _ws(d1, pos)[0] == pt.PTLM_OK
    for my, mx in ((256, 128), (128, 256), (256, 64), (48, 96), (96, 32), (48, 16)):
        d2 = pt.ptlm_desc(300, 300, my, mx, 3, pt.GAUSS, pt.JOINT, 1e-8)
        assert _ws(d2, pos)[0] == pt.PTLM_EINVAL


def test_create_rejects_small_workspace():
    pos = np.array([[0, 0]], np.int32)
    d = pt.ptlm_desc(16, 16, 16, 16, 1, pt.GAUSS, pt.OBJECT, 1e-8)
    h = ctypes.c_void_p()
    st = pt.lib().ptlm_create(ctypes.byref(d), pos.ctypes.data_as(ctypes.c_void_p), None, 0, None, ctypes.byref(h))
    assert st == pt.PTLM_EWORKSPACE and not h.value


def test_default_params_are_the_papers():
    p = pt.default_params()
    assert (p.mu0, p.mu_min, p.kappa, p.nu, p.rho_min, p.beta) == (1e-5, 1e-8, 4.0, 1.0, 1e-4, 0.1)
    assert p.cg_max == 10 and p.scaling == 0 and p.precond == 0


def test_batch_workspace_validation():
    descs = (pt.ptlm_desc * 2)(pt.ptlm_desc(40, 40, 16, 16, 2, pt.GAUSS, pt.JOINT, 1e-8),
                               pt.ptlm_desc(100, 100, 48, 48, 2, pt.GAUSS, pt.JOINT, 1e-8))
    p0 = np.array([[0, 0], [10, 10]], np.int32)
    p1 = np.array([[0, 0], [52, 52]], np.int32)
    ptrs = (ctypes.c_void_p * 2)(p0.ctypes.data_as(ctypes.c_void_p), p1.ctypes.data_as(ctypes.c_void_p))
    n = ctypes.c_size_t(0)
    assert pt.lib().ptlm_batch_workspace_bytes(2, descs, ptrs, ctypes.byref(n)) == pt.PTLM_OK
    # at least the two problems' own workspaces
    one = [_ws(descs[i], p)[1] for i, p in enumerate((p0, p1))]
    assert n.value >= sum(one)
    p1[1] = [53, 0]  # outside the 100 x 100 object for a 48 x 48 probe
    assert pt.lib().ptlm_batch_workspace_bytes(2, descs, ptrs, ctypes.byref(n)) == pt.PTLM_EINVAL
    assert b"problem 1" in pt.lib().ptlm_last_error()
    assert pt.lib().ptlm_batch_workspace_bytes(0, descs, ptrs, ctypes.byref(n)) == pt.PTLM_EINVAL


def test_struct_mirrors_match_the_header(tmp_path):
    """The ctypes mirrors of the header's structs have its sizes and field offsets (the library
    writes the LM state in place, so a shorter or shifted mirror would be overrun or misread)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    mirrors = {"ptlm_desc": pt.ptlm_desc, "ptlm_lm_params": pt.ptlm_lm_params, "ptlm_lm_state": pt.ptlm_lm_state,
               "ptlm_cnn_desc": pt.ptlm_cnn_desc}
    lines = []
    for cname, py in mirrors.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in py._fields_:
            cfield = "lambda" if fname == "lambda_" else fname
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, cfield))
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "ptlm.h"\nint main(void) {\n'
                   + "\n".join(lines) + "\nreturn 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    seen = 0
    for ln in out:
        if not ln:
            continue
        cname, field, val = ln.split()
        py = mirrors[cname]
        want = ctypes.sizeof(py) if field == "size" else getattr(py, field).offset
        assert int(val) == want, (cname, field, int(val), want)
        seen += 1
    assert seen == sum(len(p._fields_) + 1 for p in mirrors.values())


def test_binding_fails_loudly_without_the_library(tmp_path):
    """Without the built HIP library the binding refuses to import (no silent CPU path)."""
    import shutil
    import subprocess
    import sys
    pkg = tmp_path / "paper_2103_01767_amd"
    pkg.mkdir()
    shutil.copy(os.path.join(ROOT, "paper_2103_01767_amd", "__init__.py"), pkg / "__init__.py")
    r = subprocess.run([sys.executable, "-c", "import paper_2103_01767_amd"], cwd=str(tmp_path),
                       env={**os.environ, "PYTHONPATH": str(tmp_path)}, capture_output=True, text=True)
    assert r.returncode != 0
    assert "libptlm.so is not built" in r.stderr
