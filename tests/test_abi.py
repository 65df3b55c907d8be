"""The C-ABI library loads and exports every function include/ffv.h declares
(no GPU needed: nothing is called)."""
import ctypes
import os
import re

from paper_2112_10603_amd import ffv

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "ffv.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ffv_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_binding_exports():
    assert declared_functions() == sorted(ffv.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(ffv.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name


def test_default_opts_and_null_args():
    L = ffv.lib()
    o = ffv.ffv_opts()
    L.ffv_default_opts(ctypes.byref(o))
    assert o.abi_version == ffv.FFV_ABI_VERSION and o.precision == ffv.FFV_FP32
    h = ctypes.c_void_p()
    assert L.ffv_create_net(None, ctypes.byref(o), ctypes.byref(h)) == -1
    assert b"null" in L.ffv_last_error()
    o.abi_version = 99
    assert L.ffv_create_net(b"x.ffvw", ctypes.byref(o), ctypes.byref(h)) == -1
    assert L.ffv_interpolate(None, None, 1, None, 1, None) == -1


def test_bad_weights_file_rejected(tmp_path):
    """A corrupted payload fails the SHA-256 check before any device work."""
    from synth.weights import write_weights_file
    p = write_weights_file(str(tmp_path / "w.ffvw"), seed=0)
    raw = bytearray(open(p, "rb").read())
    raw[-10] ^= 0xFF
    bad = tmp_path / "bad.ffvw"
    bad.write_bytes(bytes(raw))
    L = ffv.lib()
    o = ffv.ffv_opts()
    L.ffv_default_opts(ctypes.byref(o))
    h = ctypes.c_void_p()
    assert L.ffv_create_net(str(bad).encode(), ctypes.byref(o), ctypes.byref(h)) == -5
    assert b"checksum" in L.ffv_last_error()
    assert L.ffv_create_net(b"/nonexistent.ffvw", ctypes.byref(o), ctypes.byref(h)) == -5
