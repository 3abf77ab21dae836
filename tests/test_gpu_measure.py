"""GPU test of the measurement helper that the bench's read ceiling uses."""

import ctypes as C

import pytest

pytestmark = pytest.mark.gpu


def test_stream_read_sums_every_element():
    import torch

    from paper_1709_05660_amd import _lib
    L = _lib.lib()
    n = 3 * 1000 * 1000 + 2   # not a multiple of the grid: exercises the tail loop
    x = torch.arange(n, dtype=torch.float64, device="cuda")
    out = torch.empty(L.fsi_stream_read_blocks(), dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream()
    rc = L.fsi_stream_read(C.c_void_p(x.data_ptr()), n, C.c_void_p(out.data_ptr()),
                           C.c_void_p(st.cuda_stream))
    assert rc == 0
    torch.cuda.synchronize()
    assert float(out.sum()) == pytest.approx(n * (n - 1) / 2, rel=1e-12)
