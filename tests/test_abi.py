"""CPU checks of the C ABI: the built library loads and exports every function
include/pic.h declares; the binding's structs match the header's layout."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pic.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"\b(pic_[a-z_]+)\s*\(", src)))


def _lib():
    from paper_1503_00276_amd import pic

    if not os.path.exists(pic.LIB_PATH):
        pytest.skip("libpic.so not built (run __graft_entry__.build())")
    return pic, ctypes.CDLL(pic.LIB_PATH)


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["pic_create", "pic_load_particles", "pic_step", "pic_diag", "pic_batch_step"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    pic, L = _lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert set(pic.EXPORTED) == set(_declared())


def _c_layout(tmp_path, struct, fields):
    """sizeof and offsetof of a header struct, as the C compiler lays it out."""
    src = tmp_path / "layout.c"
    body = "".join(f'  printf("{f} %zu\\n", offsetof({struct}, {f}));\n' for f in fields)
    src.write_text(
        "#include <stdio.h>\n#include <stddef.h>\n#include \"pic.h\"\n"
        f"int main(void) {{\n  printf(\"size %zu\\n\", sizeof({struct}));\n{body}  return 0;\n}}\n"
    )
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True)
    return {k: int(v) for k, v in (line.split() for line in out.strip().splitlines())}


@pytest.mark.parametrize("struct", ["pic_config", "pic_info"])
def test_struct_layout_matches_header(tmp_path, struct):
    pic, _ = _lib()
    cls = getattr(pic, struct)
    names = [f[0] for f in cls._fields_]
    lay = _c_layout(tmp_path, struct, names)
    assert lay["size"] == ctypes.sizeof(cls)
    for n in names:
        assert lay[n] == getattr(cls, n).offset, n


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_1503_00276_amd import pic

    monkeypatch.setattr(pic, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(pic, "_lib", None)
    with pytest.raises(ImportError):
        pic.lib()
