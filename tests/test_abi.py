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


@pytest.mark.parametrize("struct", ["pic_config", "pic_info", "pic_tune"])
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


def _create_status(pic, **kw):
    base = dict(ndim=2, nx=(16, 16), dx=(0.2, 0.2), dt=0.1, shape_order=1)
    base.update(kw)
    cfg = pic.Config(**base)
    L = pic.lib()
    h = ctypes.c_void_p()
    c = cfg.c()
    rc = L.pic_create(ctypes.byref(c), None, ctypes.byref(h))
    if rc == 0:
        L.pic_destroy(h)
    return rc


@pytest.mark.parametrize("kw,why", [
    (dict(ndim=4), "dimension"),
    (dict(shape_order=4), "shape order"),
    (dict(shape_order=0), "shape order"),
    (dict(nx=(0, 16)), "empty axis"),
    (dict(dx=(-0.2, 0.2)), "negative cell"),
    (dict(dt=0.15), "Courant: 0.15*sqrt(2)/0.2 > 1"),
    (dict(dt=0.0), "zero step"),
    (dict(dt=float("nan")), "nan step"),
    (dict(capacity=-5), "negative capacity"),
    (dict(tile=(3, 16)), "tile smaller than slack + 2"),
    (dict(tile=(16, 13)), "ragged remainder 3 smaller than slack + 2 = 4"),
    (dict(accumulator=7), "unknown accumulator"),
    (dict(sort_interval=-1), "negative interval"),
    (dict(ndim=3, nx=(64, 64, 64), dx=(0.2, 0.2, 0.2), dt=0.1, shape_order=3, tile=(64, 64, 64)),
     "explicit tile that cannot fit the LDS"),
])
def test_invalid_configuration_rejected_on_host(kw, why):
    """Invalid configurations fail with PIC_E_INVALID before any HIP call,
    so this runs without a GPU."""
    pic, _ = _lib()
    assert _create_status(pic, **kw) == pic.PIC_E_INVALID, why


def test_null_arguments_rejected():
    pic, _ = _lib()
    L = pic.lib()
    assert L.pic_create(None, None, None) == pic.PIC_E_INVALID
    assert L.pic_step(None, 1) == pic.PIC_E_INVALID
    assert L.pic_diag(None, 0, None, 0, None) == pic.PIC_E_INVALID
    assert L.pic_destroy(None) == 0
    assert L.pic_batch_destroy(None) == 0
    assert L.pic_last_error(None) == b"null context"
    assert L.pic_autotune(None, None) == pic.PIC_E_INVALID
    assert L.pic_batch_autotune(None, None) == pic.PIC_E_INVALID
    assert L.pic_batch_get_info(None, 0, None) == pic.PIC_E_INVALID


def test_tristan_needs_linear_shape():
    pic, _ = _lib()
    assert _create_status(pic, shape_order=2, deposit=pic.PIC_DEPOSIT_TRISTAN) == pic.PIC_E_INVALID
    assert _create_status(pic, shape_order=1, deposit=7) == pic.PIC_E_INVALID


def test_bench_refuses_more_than_one_gpu():
    """bench.py is a one-GPU benchmark: --gpus above 1 exits before touching a
    GPU, with a message."""
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
