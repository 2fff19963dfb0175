"""fd_cfl_dt_static (no workspace, nothing allocated) against fd_cfl_dt, through the C ABI:
two calls in a row on the same device, the second on a smaller grid, each with the
same bits as the workspace form."""
import ctypes as C

import numpy as np
import pytest
import torch

from workloads import layered_velocity, smooth_velocity

pytestmark = pytest.mark.gpu

api = pytest.importorskip("paper_2506_02486_amd.api")
from paper_2506_02486_amd import _lib  # noqa: E402


def test_static_scratch_cfl_matches_workspace_form():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    torch.cuda.set_device(0)
    L = api.lib()
    cases = [smooth_velocity(96, 70, 50, seed=2, sigma=3.0),   # vmax 4500 at the model's max
             layered_velocity(20, 9, 13, seed=1)]               # smaller, and a different vmax
    seen = []
    for v in cases:
        nz, ny, nx = v.shape
        g = api.Grid(nx, ny, nz, (10.0, 12.0, 9.0))
        vt = g.zeros()
        g.interior(vt).copy_(torch.from_numpy(v))
        ws = torch.full((2,), -1, dtype=torch.int32, device="cuda")
        out_ws = (C.c_double(), C.c_double())
        out_st = (C.c_double(), C.c_double())
        s = torch.cuda.current_stream().cuda_stream
        assert L.fd_cfl_dt(g.ref, vt.data_ptr(), 0.4, ws.data_ptr(), C.byref(out_ws[0]),
                           C.byref(out_ws[1]), s) == 0
        assert L.fd_cfl_dt_static(g.ref, vt.data_ptr(), 0.4, C.byref(out_st[0]),
                                  C.byref(out_st[1]), s) == 0
        assert out_st[0].value == out_ws[0].value == float(np.float32(v.max()))
        assert out_st[1].value == out_ws[1].value == 0.4 * 9.0 / float(np.float32(v.max()))
        seen.append(out_st[0].value)
        # the Python binding gives the same numbers
        assert api.cfl_dt_static(g, vt, 0.4) == api.cfl_dt(g, vt, 0.4)
    assert seen[0] != seen[1]  # the second call did not keep the first call's maximum
    # a model with a non-positive velocity is refused by both forms alike
    g = api.Grid(8, 8, 8)
    bad = g.zeros()
    g.interior(bad).fill_(1500.0)
    g.interior(bad)[3, 3, 3] = -1.0
    d0, d1 = C.c_double(), C.c_double()
    assert L.fd_cfl_dt_static(g.ref, bad.data_ptr(), 0.4, C.byref(d0), C.byref(d1),
                              torch.cuda.current_stream().cuda_stream) == _lib.FD_EINVAL
