"""The allocation-free reconstruction entry point, called through the C ABI:
its output equals iwpp_morph_recon_u8's (and the oracle's) on two calls in a
row, the second smaller than the first, and an image beyond its static work
area is refused before anything is launched."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1209_3314_amd import synth
from tests.gpu_util import announce, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def abi():
    torch, iw = require_gpu()
    from paper_1209_3314_amd import _lib

    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.iwpp_create(0, None, ctypes.byref(h)) == _lib.IWPP_OK
    yield torch, lib, h, _lib
    torch.cuda.synchronize()
    lib.iwpp_destroy(h)


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream(0).cuda_stream)


def _run(abi, fn_name, J, I, conn):
    torch, lib, h, _lib = abi
    d = torch.device("cuda", 0)
    Jd, Id = torch.from_numpy(J).to(d), torch.from_numpy(I).to(d)
    out = torch.full_like(Id, 7)  # not the result anywhere: the call must write every pixel
    hgt, wid = I.shape
    rc = getattr(lib, fn_name)(h, Jd.data_ptr(), Id.data_ptr(), out.data_ptr(), hgt, wid, conn, _stream(torch))
    assert rc == _lib.IWPP_OK, lib.iwpp_last_error(h).decode()
    torch.cuda.synchronize()
    st = _lib.Stats()
    assert lib.iwpp_get_stats(h, ctypes.byref(st)) == _lib.IWPP_OK
    assert st.status == 0
    return out.cpu().numpy(), st


@pytest.mark.parametrize("shape,conn,seed", [((2048, 3000), 8, 41), ((300, 257), 4, 42)])
def test_noalloc_equals_the_allocating_call(abi, shape, conn, seed):
    """Run as listed: the first case fills the static area with a larger
    image's lists, flags and border columns; the second, smaller one must not
    be affected by what it left."""
    h, w = shape
    J, I = synth.mr_inputs(h, w, seed=seed, n_disks=max(4, h * w // 6500), radius=(5, 20), offset=40)
    announce("noalloc mr", h, w, conn)
    got, st = _run(abi, "iwpp_morph_recon_u8_noalloc", J, I, conn)
    announce("alloc mr", h, w, conn)
    ref, st_ref = _run(abi, "iwpp_morph_recon_u8", J, I, conn)
    assert np.array_equal(got, ref)
    assert st.rounds == st_ref.rounds and st.items == st_ref.items
    assert np.array_equal(got, oracle.mr_fh(J, I, conn))


def test_noalloc_twice_in_a_row_then_smaller(abi):
    """Two calls back to back on one stream (no synchronisation between them),
    the second on a smaller image, each equal to the oracle."""
    torch, lib, h, _lib = abi
    d = torch.device("cuda", 0)
    cases = []
    for (hh, ww, seed) in [(1500, 1800, 43), (700, 333, 44)]:
        J, I = synth.mr_inputs(hh, ww, seed=seed, n_disks=max(4, hh * ww // 6500), radius=(5, 20), offset=32)
        Jd, Id = torch.from_numpy(J).to(d), torch.from_numpy(I).to(d)
        cases.append((J, I, Jd, Id, torch.zeros_like(Id)))
    announce("noalloc back to back")
    for J, I, Jd, Id, out in cases:
        hh, ww = I.shape
        rc = lib.iwpp_morph_recon_u8_noalloc(h, Jd.data_ptr(), Id.data_ptr(), out.data_ptr(), hh, ww, 8, _stream(torch))
        assert rc == _lib.IWPP_OK, lib.iwpp_last_error(h).decode()
    torch.cuda.synchronize()
    for J, I, Jd, Id, out in cases:
        assert np.array_equal(out.cpu().numpy(), oracle.mr_fh(J, I, 8))


def test_noalloc_in_place(abi):
    """out may alias the marker, as for the allocating call."""
    torch, lib, h, _lib = abi
    d = torch.device("cuda", 0)
    J, I = synth.mr_inputs(513, 640, seed=45, n_disks=30, radius=(5, 20), offset=32)
    Jd, Id = torch.from_numpy(J).to(d), torch.from_numpy(I).to(d)
    announce("noalloc in place")
    rc = lib.iwpp_morph_recon_u8_noalloc(h, Jd.data_ptr(), Id.data_ptr(), Jd.data_ptr(), 513, 640, 8, _stream(torch))
    assert rc == _lib.IWPP_OK
    torch.cuda.synchronize()
    assert np.array_equal(Jd.cpu().numpy(), oracle.mr_fh(J, I, 8))


def test_noalloc_refuses_images_beyond_its_area(abi):
    """20480 x 20480 is 102,400 tiles of 64 x 64, above what the static area
    holds: IWPP_EINVAL before any launch."""
    torch, lib, h, _lib = abi
    d = torch.device("cuda", 0)
    n = 20480
    I = torch.zeros((n, n), dtype=torch.uint8, device=d)
    J = torch.zeros((n, n), dtype=torch.uint8, device=d)
    out = torch.zeros((n, n), dtype=torch.uint8, device=d)
    announce("noalloc oversize")
    rc = lib.iwpp_morph_recon_u8_noalloc(h, J.data_ptr(), I.data_ptr(), out.data_ptr(), n, n, 8, _stream(torch))
    assert rc == _lib.IWPP_EINVAL
    msg = lib.iwpp_last_error(h).decode()
    assert "static area" in msg and "102400 tiles" in msg
    torch.cuda.synchronize()
    assert int(out.max()) == 0  # nothing ran


def test_noalloc_whole_slide_tile(abi):
    """The 16384 x 16384 reconstruction workload (65,536 tiles, within the
    area), 4-connected: equal to the allocating call's output byte for byte."""
    torch, lib, h, _lib = abi
    J, I = synth.workload_mr_16k()
    d = torch.device("cuda", 0)
    Jd, Id = torch.from_numpy(J).to(d), torch.from_numpy(I).to(d)
    a, b = torch.zeros_like(Id), torch.ones_like(Id)
    announce("noalloc 16384^2 conn 4")
    assert lib.iwpp_morph_recon_u8_noalloc(h, Jd.data_ptr(), Id.data_ptr(), a.data_ptr(), 16384, 16384, 4,
                                           _stream(torch)) == _lib.IWPP_OK
    assert lib.iwpp_morph_recon_u8(h, Jd.data_ptr(), Id.data_ptr(), b.data_ptr(), 16384, 16384, 4,
                                   _stream(torch)) == _lib.IWPP_OK
    torch.cuda.synchronize()
    assert torch.equal(a, b)
