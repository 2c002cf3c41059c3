"""The ctypes binding matches include/streamconv.h: every struct's size and
field offsets (from a C program compiled against the header with the host
compiler) and the enum constants the binding mirrors."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

from paper_2204_07064_amd import _native as n

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "streamconv.h")

STRUCTS = [("sc_node", n.ScNode), ("sc_model_info", n.ScModelInfo), ("sc_op_profile", n.ScOpProfile),
           ("sc_server_config", n.ScServerConfig), ("sc_server_stats", n.ScServerStats)]


def _c_layout(tmp_path):
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "streamconv.h"', "int main(void) {"]
    for cname, py in STRUCTS:
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for field, _ in py._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, field, cname, field))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, stdout=subprocess.PIPE, text=True).stdout
    return {tuple(ln.split()[:2]): int(ln.split()[2]) for ln in out.splitlines()}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_struct_layouts_match_header(tmp_path):
    c = _c_layout(tmp_path)
    for cname, py in STRUCTS:
        assert c[(cname, "size")] == ctypes.sizeof(py), cname
        for field, _ in py._fields_:
            assert c[(cname, field)] == getattr(py, field).offset, (cname, field)


def _header_constants():
    text = open(HEADER).read()
    return {m.group(1): int(m.group(2)) for m in re.finditer(r"\b(SC_[A-Z0-9_]+)\s*=\s*(-?\d+)u?\b", text)}


def test_enum_constants_match_header():
    h = _header_constants()
    for name in ("SC_MODEL_NO_FUSION", "SC_MODEL_NO_MFMA", "SC_MODEL_NO_TWIN", "SC_MODEL_NO_WIN",
                 "SC_MODEL_NO_SPLIT", "SC_MODEL_NO_OUT_FUSION", "SC_MODEL_NO_CONVT_FUSION", "SC_MODEL_NO_INPUT_DIRECT", "SC_MODEL_NO_PAIR_FUSION", "SC_FLAG_WARMUP_MASK",
                 "SC_PENDING",
                 "SC_SUBMIT_DISCARD", "SC_OK"):
        assert getattr(n, name) == h[name], name
    for code, label in n.STATUS.items():
        assert h[label] == code, label
    assert n.PRECISION == {"fp32": h["SC_FP32"], "bf16": h["SC_BF16"], "fp8": h["SC_FP8E4M3"]}
    assert n.OPS == {"input": h["SC_OP_INPUT"], "conv": h["SC_OP_CONV"], "convt": h["SC_OP_CONVT"],
                     "add": h["SC_OP_ADD"]}
    # the no-alloc path's scratch size, as the header defines it
    m = re.search(r"#define\s+SC_NOALLOC_SCRATCH_BYTES\s+\((\d+)u \* (\d+)u \* (\d+)u\)", open(HEADER).read())
    assert m and int(m.group(1)) * int(m.group(2)) * int(m.group(3)) == n.SC_NOALLOC_SCRATCH_BYTES
    # option bits are distinct powers of two
    opts = [h[k] for k in h if k.startswith("SC_MODEL_NO_")]
    assert len(set(opts)) == len(opts) and all(o & (o - 1) == 0 for o in opts)


def _prototypes():
    """name -> (return type text, parameter count) of every function the header declares."""
    text = re.sub(r"/\*.*?\*/", " ", open(HEADER).read(), flags=re.S)
    protos = {}
    for m in re.finditer(r"([A-Za-z_][A-Za-z0-9_ \*]*?)\b([a-z_][a-z0-9_]*)\s*\(([^;{]*?)\)\s*;", text):
        ret, name, params = m.group(1).strip(), m.group(2), m.group(3).strip()
        if name not in n.EXPORTS:
            continue
        count = 0 if params in ("", "void") else params.count(",") + 1
        protos[name] = (ret, count)
    return protos


def test_function_signatures_match_header():
    protos = _prototypes()
    L = n.lib() if os.path.exists(n.LIB_PATH) else None
    if L is None:
        pytest.skip("library not built")
    assert sorted(protos) == sorted(n.EXPORTS)
    for name, (ret, count) in protos.items():
        f = getattr(L, name)
        assert len(f.argtypes) == count, (name, count, f.argtypes)
        if ret.endswith("void") and "*" not in ret:
            assert f.restype is None, name
        elif ret == "sc_status" or ret.endswith("int32_t"):
            assert f.restype is ctypes.c_int32, name
        elif ret.endswith("int64_t"):
            assert f.restype is ctypes.c_int64, name
        elif "char" in ret:
            assert f.restype is ctypes.c_char_p, name
