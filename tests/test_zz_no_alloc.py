"""The allocation-free clustering entry point (gid_cluster_frame_noalloc),
called through the C ABI, against the allocating one (gid_cluster_frame):
identical cluster count, centres, colours and ids, on two calls in a row (the
second on a smaller frame, so stale scratch contents of the first would show)."""
import ctypes
from ctypes import POINTER, byref, c_double, c_int32, c_void_p

import numpy as np
import pytest

from scenes import make_clip

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


def _call(torch, lib, fn, frame, k_max):
    H, W = frame.shape[1:]
    f = torch.from_numpy(np.ascontiguousarray(frame)).cuda()
    ids = torch.full((H, W), 255, dtype=torch.uint8, device="cuda")
    cols = np.full(3 * k_max, np.nan)
    cen = np.full(3 * k_max, np.nan)
    k = c_int32(-1)
    stream = c_void_p(torch.cuda.current_stream().cuda_stream)
    st = getattr(lib, fn)(c_void_p(f.data_ptr()), W, H, k_max, 0.2, stream, c_void_p(ids.data_ptr()),
                          cols.ctypes.data_as(POINTER(c_double)), cen.ctypes.data_as(POINTER(c_double)), byref(k))
    assert st == 0, (fn, st)
    n = k.value
    return ids.cpu().numpy(), cols[:3 * n].reshape(n, 3), cen[:3 * n].reshape(n, 3)


def test_noalloc_equals_allocating_entry_point_on_two_calls(torch):
    import paper_1908_01961_amd as G
    lib = G.load_library()
    for fn in ("gid_cluster_frame", "gid_cluster_frame_noalloc"):
        getattr(lib, fn).restype = c_int32
        getattr(lib, fn).argtypes = [c_void_p, c_int32, c_int32, c_int32, c_double, c_void_p, c_void_p,
                                     POINTER(c_double), POINTER(c_double), POINTER(c_int32)]
    big = make_clip(640, 480, 8, 1, 4242, gt=False).frames[0]
    small = make_clip(97, 61, 3, 1, 4243, gt=False).frames[0]
    for frame, k_max in ((big, 10), (small, 6)):
        a = _call(torch, lib, "gid_cluster_frame", frame, k_max)
        b = _call(torch, lib, "gid_cluster_frame_noalloc", frame, k_max)
        print(f"[gpu-case] no-alloc {frame.shape[2]}x{frame.shape[1]} k_max {k_max}: {len(a[1])} clusters",
              flush=True)
        assert len(a[1]) == len(b[1]) > 0
        assert np.array_equal(a[0], b[0])
        assert np.array_equal(a[2], b[2])
        assert np.array_equal(a[1], b[1])     # same kernels, same reduction order
