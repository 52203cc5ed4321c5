"""The library's own argument checks, called through the C ABI directly
(bypassing the Python binding's checks): every bad argument returns
IWPP_EINVAL with a message, before anything is enqueued, so the output
buffers keep their contents."""
import ctypes

import pytest

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


def _bufs(torch, shape=(64, 80)):
    d = torch.device("cuda", 0)
    J = torch.zeros(shape, dtype=torch.uint8, device=d)
    I = torch.full(shape, 9, dtype=torch.uint8, device=d)
    out = torch.full(shape, 77, dtype=torch.uint8, device=d)
    B = torch.ones(shape, dtype=torch.uint8, device=d)
    sq = torch.full(shape, 5, dtype=torch.int32, device=d)
    nr = torch.full(shape, 6, dtype=torch.int32, device=d)
    return J, I, out, B, sq, nr


def _expect_einval(lib, h, _lib, rc, words):
    assert rc == _lib.IWPP_EINVAL
    msg = lib.iwpp_last_error(h).decode()
    assert all(w in msg for w in words), msg


def test_recon_argument_errors(abi):
    torch, lib, h, _lib = abi
    J, I, out, _, _, _ = _bufs(torch)
    H, W = J.shape
    announce("abi recon errors")
    f = lib.iwpp_morph_recon_u8
    assert f(None, J.data_ptr(), I.data_ptr(), out.data_ptr(), H, W, 8, None) == _lib.IWPP_EINVAL
    _expect_einval(lib, h, _lib, f(h, None, I.data_ptr(), out.data_ptr(), H, W, 8, None), ["NULL"])
    _expect_einval(lib, h, _lib, f(h, J.data_ptr(), None, out.data_ptr(), H, W, 8, None), ["NULL"])
    _expect_einval(lib, h, _lib, f(h, J.data_ptr(), I.data_ptr(), None, H, W, 8, None), ["NULL"])
    _expect_einval(lib, h, _lib, f(h, J.data_ptr(), I.data_ptr(), out.data_ptr(), H, W, 5, None), ["conn"])
    _expect_einval(lib, h, _lib, f(h, J.data_ptr(), I.data_ptr(), out.data_ptr(), 0, W, 8, None), ["height"])
    _expect_einval(lib, h, _lib, f(h, J.data_ptr(), I.data_ptr(), out.data_ptr(), H, -3, 8, None), ["width"])
    # out aliasing the mask, or overlapping the marker without being it
    _expect_einval(lib, h, _lib, f(h, J.data_ptr(), I.data_ptr(), I.data_ptr(), H, W, 8, None), ["alias mask"])
    big = torch.zeros(2 * H * W, dtype=torch.uint8, device=J.device)  # marker = first half; out 5 bytes in
    _expect_einval(lib, h, _lib, f(h, big.data_ptr(), I.data_ptr(), big.data_ptr() + 5, H, W, 8, None), ["overlap"])
    # a width beyond the 32-bit band addressing (checked before any access)
    _expect_einval(lib, h, _lib, f(h, J.data_ptr(), I.data_ptr(), out.data_ptr(), 1, (1 << 25) + 1, 8, None),
                   ["width"])
    torch.cuda.synchronize()
    assert int(out.min()) == 77 and int(out.max()) == 77  # nothing ran


def test_edt_argument_errors(abi):
    torch, lib, h, _lib = abi
    _, _, _, B, sq, nr = _bufs(torch)
    H, W = B.shape
    announce("abi edt errors")
    f = lib.iwpp_edt
    assert f(None, B.data_ptr(), sq.data_ptr(), nr.data_ptr(), H, W, 8, None) == _lib.IWPP_EINVAL
    _expect_einval(lib, h, _lib, f(h, None, sq.data_ptr(), nr.data_ptr(), H, W, 8, None), ["NULL"])
    _expect_einval(lib, h, _lib, f(h, B.data_ptr(), None, nr.data_ptr(), H, W, 8, None), ["NULL"])
    _expect_einval(lib, h, _lib, f(h, B.data_ptr(), sq.data_ptr(), None, H, W, 8, None), ["NULL"])
    _expect_einval(lib, h, _lib, f(h, B.data_ptr(), sq.data_ptr(), nr.data_ptr(), H, W, 5, None), ["conn"])
    _expect_einval(lib, h, _lib, f(h, B.data_ptr(), sq.data_ptr(), nr.data_ptr(), H, 0, 8, None), ["height"])
    # sqdist and nearest the same buffer; an output over the input
    _expect_einval(lib, h, _lib, f(h, B.data_ptr(), sq.data_ptr(), sq.data_ptr(), H, W, 8, None), ["alias"])
    _expect_einval(lib, h, _lib, f(h, sq.data_ptr(), sq.data_ptr() + 4, nr.data_ptr(), H, W, 8, None), ["alias"])
    # sides beyond the int32 distance limit (checked before any access)
    _expect_einval(lib, h, _lib, f(h, B.data_ptr(), sq.data_ptr(), nr.data_ptr(), 1, 46341, 8, None), ["46340"])
    torch.cuda.synchronize()
    assert int(sq.min()) == 5 and int(sq.max()) == 5 and int(nr.min()) == 6 and int(nr.max()) == 6


def test_batch_argument_errors(abi):
    torch, lib, h, _lib = abi
    J, I, out, B, sq, nr = _bufs(torch)
    H, W = J.shape
    announce("abi batch errors")
    Job = _lib.Job
    ok_mr = Job(_lib.IWPP_OP_RECON, 8, H, W, J.data_ptr(), I.data_ptr(), out.data_ptr(), None)
    ok_edt = Job(_lib.IWPP_OP_EDT, 8, H, W, B.data_ptr(), None, sq.data_ptr(), nr.data_ptr())
    jobs = (Job * 2)(ok_mr, ok_edt)
    _expect_einval(lib, h, _lib, lib.iwpp_run_batch(h, jobs, 0, None), ["at least one job"])
    _expect_einval(lib, h, _lib, lib.iwpp_run_batch(h, None, 2, None), ["at least one job"])
    bad = (Job * 2)(ok_mr, Job(7, 8, H, W, B.data_ptr(), None, sq.data_ptr(), nr.data_ptr()))
    _expect_einval(lib, h, _lib, lib.iwpp_run_batch(h, bad, 2, None), ["job 1", "op"])
    # the second job writes into the first job's output
    bad = (Job * 2)(ok_mr, Job(_lib.IWPP_OP_RECON, 8, H, W, J.data_ptr(), I.data_ptr(), out.data_ptr(), None))
    _expect_einval(lib, h, _lib, lib.iwpp_run_batch(h, bad, 2, None), ["overlaps"])
    # a reconstruction job with an EDT output
    bad = (Job * 1)(Job(_lib.IWPP_OP_RECON, 8, H, W, J.data_ptr(), I.data_ptr(), out.data_ptr(), nr.data_ptr()))
    _expect_einval(lib, h, _lib, lib.iwpp_run_batch(h, bad, 1, None), ["job 0"])
    torch.cuda.synchronize()
    assert int(out.min()) == 77 and int(sq.min()) == 5


def test_context_argument_errors(abi):
    torch, lib, h, _lib = abi
    announce("abi context errors")
    opt = _lib.Options()
    opt.mr_max_sweeps = -1
    _expect_einval(lib, h, _lib, lib.iwpp_set_options(h, ctypes.byref(opt)), ["negative"])
    assert lib.iwpp_set_options(h, None) == _lib.IWPP_EINVAL
    assert lib.iwpp_get_stats(h, None) == _lib.IWPP_EINVAL
    assert lib.iwpp_round_times(h, None, 4, None) == _lib.IWPP_EINVAL
    out = ctypes.c_void_p()
    assert lib.iwpp_create(-1, None, ctypes.byref(out)) == _lib.IWPP_EINVAL
    assert "no HIP device" in lib.iwpp_last_error(None).decode()
    assert lib.iwpp_create(0, None, None) == _lib.IWPP_EINVAL
    bad = _lib.Options()
    bad.persistent_blocks = -2
    assert lib.iwpp_create(0, ctypes.byref(bad), ctypes.byref(out)) == _lib.IWPP_EINVAL
    lib.iwpp_destroy(None)  # NULL is allowed
