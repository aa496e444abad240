"""CPU: the LDS probe library (the measured LDS rates behind the decode
kernel's roofline) loads, exports its two calls, and counts the bytes a
launch moves: distinct bank-conflict-free accesses only."""
import ctypes as C
import os

ROOT = os.path.join(os.path.dirname(__file__), "..")


def test_probe_library_exports_and_byte_count():
    L = C.CDLL(os.path.join(ROOT, "paper_2403_18901_amd", "libgdg_probe.so"))
    assert hasattr(L, "lds_probe_launch")
    L.lds_probe_bytes.argtypes = [C.c_int, C.c_int, C.c_int]
    L.lds_probe_bytes.restype = C.c_double
    # 32 KiB per workgroup: 32 / 16 / 8 distinct slots per thread for 4 / 8 / 16 bytes
    assert L.lds_probe_bytes(0, 2, 3) == 2 * 256 * 16 * 3 * 4
    assert L.lds_probe_bytes(1, 2, 3) == 2 * 256 * 16 * 3 * 8
    assert L.lds_probe_bytes(2, 2, 3) == 2 * 256 * 8 * 3 * 16
    assert L.lds_probe_bytes(3, 2, 3) == 2 * 256 * 16 * 3 * 4
    # 16 KiB: 16 / 8 / 4 slots
    assert L.lds_probe_bytes(4, 1, 1) == 256 * 16 * 4
    assert L.lds_probe_bytes(5, 1, 1) == 256 * 8 * 8
    assert L.lds_probe_bytes(6, 1, 1) == 256 * 4 * 16
    L.lds_probe_launch.argtypes = [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p]
    assert L.lds_probe_launch(7, 1, 1, C.c_void_p(16), None) == -1   # bad mode, no launch
    assert L.lds_probe_launch(0, 0, 1, C.c_void_p(16), None) == -1
