"""CPU: the entry points added for the comparator, the warm start and the
chained launch reject missing arguments with GDG_EINVAL and an error text,
before touching the device (no GPU is needed for these calls)."""
import ctypes as C

import pytest

EINVAL = -22


def _lib():
    import paper_2403_18901_amd.gdg as G
    return G.lib()


def test_new_entry_points_reject_null_arguments():
    L = _lib()
    N = None
    assert L.gdg_decode_osd(N, 4, N, 0, 10, 1, 10, 0, N, N, N, N, N, N) == EINVAL
    assert b"null window" in L.gdg_last_error()
    assert L.gdg_link_windows(N, N) == EINVAL
    assert L.gdg_window_edge_slots(N, N) == EINVAL
    assert L.gdg_decode_batch_warm(N, 4, N, 0, N, 0, N, 0, N, N, N, N, 0, N, N) == EINVAL
    assert L.gdg_decode_chain(N, N, N, 11, 4, N, N, N, N, N, N, N, 0, N, N, N) == EINVAL
    assert b"first window" in L.gdg_last_error()
    # zero items is a no-op once the first window is there; negative sizes are refused
    assert L.gdg_decode_chain(N, N, N, 0, 4, N, N, N, N, N, N, N, 0, N, N, N) == EINVAL


@pytest.mark.parametrize("n_shots", [-1])
def test_decode_entry_points_reject_negative_sizes(n_shots):
    L = _lib()
    assert L.gdg_decode_batch_warm(None, n_shots, None, 0, None, 0, None, 0, None, None, None,
                                   None, 0, None, None) == EINVAL
    assert L.gdg_decode_osd(None, n_shots, None, 0, 10, 1, 10, 0, None, None, None, None, None,
                            None) == EINVAL
