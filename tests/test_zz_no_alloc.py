"""fcm_histogram_noalloc, the histogram entry point that allocates nothing
(its workspace is a fixed device array), against fcm_histogram through the C
ABI: bit-identical normalised histograms on two calls in a row, the second
with a smaller input, for several instances and for one (which spreads its
counts over 16 copies); more instances than the array holds are refused
before any GPU work."""
import ctypes

import numpy as np
import pytest

from paper_1601_00072_amd import _lib as L
from phantom import PhantomParams, phantom

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    L.load()
    return torch, torch.device("cuda:0")


def call(fn, torch, x, sizes):
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    out = torch.full((len(sizes), 256), -1.0, dtype=torch.float32, device=x.device)
    st = torch.cuda.current_stream(x.device)
    rc = fn(ctypes.c_void_p(x.data_ptr()), off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(sizes),
            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(st.cuda_stream))
    assert rc == L.FCM_OK, rc
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("shapes", [
    [(300, 257), (64, 64), (1, 13), (40, 41, 42), (517, 3)],   # several instances, ragged sizes
    [(96, 128, 128)],                                           # one instance: 16 counter copies
])
def test_noalloc_histogram_matches_allocating_entry_point(torch_dev, shapes):
    torch, dev = torch_dev
    lib = L.load()
    print("CASE histogram noalloc", shapes, flush=True)
    xs = [phantom(PhantomParams(shape=s, seed=70 + i)).ravel() for i, s in enumerate(shapes)]
    flat = np.concatenate(xs)
    buf = torch.zeros(flat.size + 16, dtype=torch.uint8, device=dev)
    buf[3:3 + flat.size] = torch.from_numpy(flat).to(dev)   # misaligned start
    x = buf[3:3 + flat.size]
    sizes = [a.size for a in xs]
    ref = call(lib.fcm_histogram, torch, x, sizes)
    got = call(lib.fcm_histogram_noalloc, torch, x, sizes)
    assert torch.equal(got, ref)
    # the second call, on a smaller input, starts from clean counters
    small = sizes[:-1] if len(sizes) > 1 else [sizes[0] // 3]
    n2 = int(sum(small))
    ref2 = call(lib.fcm_histogram, torch, x[:n2], small)
    got2 = call(lib.fcm_histogram_noalloc, torch, x[:n2], small)
    assert torch.equal(got2, ref2)
    # and both agree with the integer counts
    off = np.concatenate([[0], np.cumsum(small)])
    for i in range(len(small)):
        want = np.bincount(flat[off[i]:off[i + 1]], minlength=256) / float(small[i])
        assert np.array_equal(got2[i].cpu().numpy(), want.astype(np.float32))


def test_noalloc_histogram_refuses_more_instances_than_its_array(torch_dev):
    torch, dev = torch_dev
    lib = L.load()
    x = torch.zeros(2048, dtype=torch.uint8, device=dev)
    out = torch.zeros((1025, 256), dtype=torch.float32, device=dev)
    off = np.arange(1026, dtype=np.int64)
    rc = lib.fcm_histogram_noalloc(ctypes.c_void_p(x.data_ptr()), off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   1025, ctypes.c_void_p(out.data_ptr()), None)
    assert rc == L.FCM_EINVAL
    assert b"1024" in lib.fcm_last_error()
