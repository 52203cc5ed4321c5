"""MI355X-native irregular wavefront propagation (IWPP), after Teodoro et al.,
"Efficient Irregular Wavefront Propagation Algorithms on Hybrid CPU-GPU
Machines" (arXiv 1209.3314).

Thin Python binding over the C ABI of ``include/iwpp.h`` (``libiwpp.so``):
argument checks and marshalling only.  PyTorch provides the device memory and
the stream; every step of the computation runs in the library's HIP kernels.
There is no CPU fallback: the calls raise if the library or a GPU is missing.

    morph_recon(marker, mask, conn=8, out=None) -> uint8 tensor   (Sec. 2.1)
    morph_recon_erode(marker, mask, conn=8, out=None) -> uint8     (the dual)
    edt(binary, conn=8) -> (sqdist int32, nearest int32)         (Sec. 2.2)
"""
from __future__ import annotations

import ctypes
import threading

from . import _lib

__all__ = ["Context", "BatchGraph", "Server", "IwppError", "morph_recon", "morph_recon_erode", "edt", "last_stats"]


class IwppError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"iwpp error {code}: {msg}")
        self.code = code


def _torch():
    import torch

    return torch


def _check_image(t, name: str, dtype, device=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D (height, width)")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous (row stride == width)")


class Context:
    """One library context (scratch memory, counters) on one device.

    Calls on a context must not overlap; the module-level functions use one
    context per device and the current torch stream."""

    def __init__(self, device: int = 0, mr_list_capacity: int = 0, mr_max_sweeps: int = 0,
                 persistent_blocks: int = 0, profile: bool = False, mr_seed_sweeps: int = 0, wg_waves: int = 0,
                 stage_depth: int = 0, mr_seed_strip: int = 0):
        lib = _lib.load()
        opt = _options(mr_list_capacity=mr_list_capacity, mr_max_sweeps=mr_max_sweeps,
                       persistent_blocks=persistent_blocks, profile=profile, mr_seed_sweeps=mr_seed_sweeps,
                       wg_waves=wg_waves, stage_depth=stage_depth, mr_seed_strip=mr_seed_strip)
        h = ctypes.c_void_p()
        rc = lib.iwpp_create(int(device), ctypes.byref(opt), ctypes.byref(h))
        if rc != _lib.IWPP_OK:
            raise IwppError(rc, lib.iwpp_last_error(None).decode())
        self._lib = lib
        self._h = h
        self.device = int(device)
        self.options = {"mr_list_capacity": int(mr_list_capacity), "mr_max_sweeps": int(mr_max_sweeps),
                        "persistent_blocks": int(persistent_blocks), "profile": bool(profile),
                        "mr_seed_sweeps": int(mr_seed_sweeps), "wg_waves": int(wg_waves),
                        "stage_depth": int(stage_depth), "mr_seed_strip": int(mr_seed_strip)}

    def set_options(self, **kw) -> None:
        """Change tuning options (same names as the constructor) for later
        calls; options not named keep their value.  Results never depend on
        them."""
        unknown = set(kw) - set(self.options)
        if unknown:
            raise TypeError(f"unknown options {sorted(unknown)}")
        new = dict(self.options, **kw)
        rc = self._lib.iwpp_set_options(self._h, ctypes.byref(_options(**new)))
        if rc != _lib.IWPP_OK:
            self._err(rc)
        self.options = new

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.iwpp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, rc: int):
        raise IwppError(rc, self._lib.iwpp_last_error(self._h).decode())

    def _stream(self, device):
        return ctypes.c_void_p(_torch().cuda.current_stream(device).cuda_stream)

    def morph_recon(self, marker, mask, conn: int = 8, out=None):
        torch = _torch()
        _check_image(mask, "mask", torch.uint8)
        _check_image(marker, "marker", torch.uint8, mask.device)
        if marker.shape != mask.shape:
            raise ValueError("marker and mask must have the same shape")
        if conn not in (4, 8):
            raise ValueError("conn must be 4 or 8")
        if out is None:
            out = torch.empty_like(mask)
        else:
            _check_image(out, "out", torch.uint8, mask.device)
            if out.shape != mask.shape:
                raise ValueError("out must have the shape of mask")
        h, w = mask.shape
        rc = self._lib.iwpp_morph_recon_u8(self._h, marker.data_ptr(), mask.data_ptr(), out.data_ptr(),
                                           h, w, conn, self._stream(mask.device))
        if rc != _lib.IWPP_OK:
            self._err(rc)
        return out

    def morph_recon_erode(self, marker, mask, conn: int = 8, out=None):
        """Reconstruction by erosion rho*_I(J) (the dual of morph_recon; a
        marker below the mask is raised to it first)."""
        torch = _torch()
        _check_image(mask, "mask", torch.uint8)
        _check_image(marker, "marker", torch.uint8, mask.device)
        if marker.shape != mask.shape:
            raise ValueError("marker and mask must have the same shape")
        if conn not in (4, 8):
            raise ValueError("conn must be 4 or 8")
        if out is None:
            out = torch.empty_like(mask)
        else:
            _check_image(out, "out", torch.uint8, mask.device)
            if out.shape != mask.shape:
                raise ValueError("out must have the shape of mask")
        h, w = mask.shape
        rc = self._lib.iwpp_morph_recon_erode_u8(self._h, marker.data_ptr(), mask.data_ptr(), out.data_ptr(),
                                                 h, w, conn, self._stream(mask.device))
        if rc != _lib.IWPP_OK:
            self._err(rc)
        return out

    def morph_recon_queue(self, marker, mask, conn: int = 8, mode: str = "staged", capacity: int = 0,
                          seed_sweeps: int = 0, out=None):
        """Reconstruction by dilation with the paper's pixel queue
        (iwpp_morph_recon_queue_u8): the same result as morph_recon, for
        comparing queue designs.  `mode` is how items enter a round's queue:
        "naive", "ballot" or "staged"; `capacity` bounds each queue (0 = never
        overflows); `seed_sweeps` is the seed pass's sweep iterations per
        tile (0 = default)."""
        torch = _torch()
        _check_image(mask, "mask", torch.uint8)
        _check_image(marker, "marker", torch.uint8, mask.device)
        if marker.shape != mask.shape:
            raise ValueError("marker and mask must have the same shape")
        if conn not in (4, 8):
            raise ValueError("conn must be 4 or 8")
        if mode not in _lib.QUEUE_MODES:
            raise ValueError(f"mode must be one of {sorted(_lib.QUEUE_MODES)}")
        if out is None:
            out = torch.empty_like(mask)
        else:
            _check_image(out, "out", torch.uint8, mask.device)
            if out.shape != mask.shape:
                raise ValueError("out must have the shape of mask")
        q = _lib.QueueOptions(_lib.QUEUE_MODES[mode], int(seed_sweeps), int(capacity))
        h, w = mask.shape
        rc = self._lib.iwpp_morph_recon_queue_u8(self._h, marker.data_ptr(), mask.data_ptr(), out.data_ptr(), h, w,
                                                 conn, ctypes.byref(q), self._stream(mask.device))
        if rc != _lib.IWPP_OK:
            self._err(rc)
        return out

    def morph_recon_noalloc(self, marker, mask, out, conn: int = 8):
        """morph_recon through iwpp_morph_recon_u8_noalloc: no device memory is
        allocated, neither by the library (its work area is a static device
        array) nor here (`out` is required).  Calls on one device must not
        overlap."""
        torch = _torch()
        _check_image(mask, "mask", torch.uint8)
        _check_image(marker, "marker", torch.uint8, mask.device)
        _check_image(out, "out", torch.uint8, mask.device)
        if marker.shape != mask.shape or out.shape != mask.shape:
            raise ValueError("marker, mask and out must have the same shape")
        if conn not in (4, 8):
            raise ValueError("conn must be 4 or 8")
        h, w = mask.shape
        rc = self._lib.iwpp_morph_recon_u8_noalloc(self._h, marker.data_ptr(), mask.data_ptr(), out.data_ptr(),
                                                   h, w, conn, self._stream(mask.device))
        if rc != _lib.IWPP_OK:
            self._err(rc)
        return out

    def edt(self, binary, conn: int = 8, out=None):
        torch = _torch()
        _check_image(binary, "binary", torch.uint8)
        if conn not in (4, 8):
            raise ValueError("conn must be 4 or 8")
        h, w = binary.shape
        if out is None:
            sq = torch.empty((h, w), dtype=torch.int32, device=binary.device)
            nr = torch.empty((h, w), dtype=torch.int32, device=binary.device)
        else:
            sq, nr = out
            _check_image(sq, "sqdist", torch.int32, binary.device)
            _check_image(nr, "nearest", torch.int32, binary.device)
        rc = self._lib.iwpp_edt(self._h, binary.data_ptr(), sq.data_ptr(), nr.data_ptr(), h, w, conn,
                                self._stream(binary.device))
        if rc != _lib.IWPP_OK:
            self._err(rc)
        return sq, nr

    def edt_exact(self, binary, out=None):
        """The exact Euclidean distance transform (iwpp_edt_exact): exact
        squared distances and, per pixel, a feature at exactly that distance."""
        torch = _torch()
        _check_image(binary, "binary", torch.uint8)
        h, w = binary.shape
        if out is None:
            sq = torch.empty((h, w), dtype=torch.int32, device=binary.device)
            nr = torch.empty((h, w), dtype=torch.int32, device=binary.device)
        else:
            sq, nr = out
            _check_image(sq, "sqdist", torch.int32, binary.device)
            _check_image(nr, "nearest", torch.int32, binary.device)
        rc = self._lib.iwpp_edt_exact(self._h, binary.data_ptr(), sq.data_ptr(), nr.data_ptr(), h, w,
                                      self._stream(binary.device))
        if rc != _lib.IWPP_OK:
            self._err(rc)
        return sq, nr

    def run_batch(self, jobs: list) -> None:
        """Run many images in few launches (see iwpp_run_batch).  Each job is a
        dict: reconstruction ``{"op": "recon", "marker", "mask", "out", "conn"}``
        or EDT ``{"op": "edt", "binary", "sqdist", "nearest", "conn"}`` with
        tensors on this context's device (outputs preallocated)."""
        arr, dev = _marshal_jobs(jobs)
        rc = self._lib.iwpp_run_batch(self._h, arr, len(jobs), self._stream(dev))
        if rc != _lib.IWPP_OK:
            self._err(rc)

    def batch_graph(self, jobs: list) -> "BatchGraph":
        """Capture `jobs` (same form as run_batch) into a replayable HIP graph.
        The graph keeps reading and writing the jobs' tensors: keep them alive
        and in place while the graph is used."""
        arr, dev = _marshal_jobs(jobs)
        g = ctypes.c_void_p()
        rc = self._lib.iwpp_batch_graph_create(self._h, arr, len(jobs), ctypes.byref(g))
        if rc != _lib.IWPP_OK:
            self._err(rc)
        return BatchGraph(self, g, dev, [t for j in jobs for t in j.values() if not isinstance(t, (int, str))])

    def profile_read(self) -> list:
        """(kernel name, device ms) for every launch since the last read, in
        launch order (needs ``profile=True``); synchronises."""
        buf = (_lib.KernelTime * 4096)()
        n = ctypes.c_int32()
        rc = self._lib.iwpp_profile_read(self._h, buf, 4096, ctypes.byref(n))
        if rc != _lib.IWPP_OK:
            self._err(rc)
        return [(_lib.KERNEL_NAMES.get(buf[i].kernel, str(buf[i].kernel)), float(buf[i].ms)) for i in range(n.value)]

    def round_times(self) -> list:
        """Device time (us) of each phase of the last call's persistent kernel:
        reconstruction [seed pass, round 1, ...], EDT [step 1, ...]."""
        buf = (ctypes.c_double * 512)()
        n = ctypes.c_int32()
        rc = self._lib.iwpp_round_times(self._h, buf, 512, ctypes.byref(n))
        if rc != _lib.IWPP_OK:
            self._err(rc)
        return [float(buf[i]) for i in range(n.value)]

    def round_work(self) -> list:
        """(device us, tiles visited) of each phase of the last call's
        persistent kernel, phases as in round_times."""
        buf = (ctypes.c_double * 256)()
        tiles = (ctypes.c_int64 * 256)()
        n = ctypes.c_int32()
        rc = self._lib.iwpp_round_work(self._h, buf, tiles, 256, ctypes.byref(n))
        if rc != _lib.IWPP_OK:
            self._err(rc)
        return [(float(buf[i]), int(tiles[i])) for i in range(n.value)]

    def stats(self) -> dict:
        st = _lib.Stats()
        rc = self._lib.iwpp_get_stats(self._h, ctypes.byref(st))
        if rc != _lib.IWPP_OK:
            self._err(rc)
        return _stats_dict(st)


OPTION_NAMES = ("mr_list_capacity", "mr_max_sweeps", "persistent_blocks", "profile", "mr_seed_sweeps", "wg_waves",
                "stage_depth", "mr_seed_strip")


def _options(mr_list_capacity=0, mr_max_sweeps=0, persistent_blocks=0, profile=False, mr_seed_sweeps=0,
             wg_waves=0, stage_depth=0, mr_seed_strip=0):
    opt = _lib.Options()
    opt.mr_list_capacity = int(mr_list_capacity)
    opt.mr_max_sweeps = int(mr_max_sweeps)
    opt.persistent_blocks = int(persistent_blocks)
    opt.profile = 1 if profile else 0
    opt.mr_seed_sweeps = int(mr_seed_sweeps)
    opt.wg_waves = int(wg_waves)
    opt.stage_depth = int(stage_depth)
    opt.mr_seed_strip = int(mr_seed_strip)
    return opt


def _marshal_jobs(jobs: list):
    torch = _torch()
    if not jobs:
        raise ValueError("empty batch")
    arr = (_lib.Job * len(jobs))()
    dev = None
    for i, j in enumerate(jobs):
        conn = int(j.get("conn", 8))
        if conn not in (4, 8):
            raise ValueError(f"job {i}: conn must be 4 or 8")
        if j["op"] in ("recon", "erode"):
            _check_image(j["mask"], f"job {i} mask", torch.uint8, dev)
            dev = j["mask"].device
            _check_image(j["marker"], f"job {i} marker", torch.uint8, dev)
            _check_image(j["out"], f"job {i} out", torch.uint8, dev)
            if not (j["marker"].shape == j["mask"].shape == j["out"].shape):
                raise ValueError(f"job {i}: shapes differ")
            h, w = j["mask"].shape
            op = _lib.IWPP_OP_RECON if j["op"] == "recon" else _lib.IWPP_OP_RECON_ERODE
            arr[i] = _lib.Job(op, conn, h, w, j["marker"].data_ptr(), j["mask"].data_ptr(), j["out"].data_ptr(), None)
        elif j["op"] == "edt":
            _check_image(j["binary"], f"job {i} binary", torch.uint8, dev)
            dev = j["binary"].device
            _check_image(j["sqdist"], f"job {i} sqdist", torch.int32, dev)
            _check_image(j["nearest"], f"job {i} nearest", torch.int32, dev)
            if not (j["binary"].shape == j["sqdist"].shape == j["nearest"].shape):
                raise ValueError(f"job {i}: shapes differ")
            h, w = j["binary"].shape
            arr[i] = _lib.Job(_lib.IWPP_OP_EDT, conn, h, w, j["binary"].data_ptr(), None,
                              j["sqdist"].data_ptr(), j["nearest"].data_ptr())
        else:
            raise ValueError(f"job {i}: op must be 'recon', 'erode' or 'edt'")
    return arr, dev


class BatchGraph:
    """A batch captured into a HIP graph (iwpp_batch_graph_create): one launch
    replays every kernel of every job on the given (or current) stream."""

    def __init__(self, ctx: Context, handle, device, keep: list):
        self._lib = ctx._lib
        self._ctx = ctx
        self._h = handle
        self.device = device
        self._keep = keep  # the tensors the graph reads and writes

    def launch(self, stream=None) -> None:
        torch = _torch()
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        rc = self._lib.iwpp_batch_graph_launch(self._h, ctypes.c_void_p(s.cuda_stream))
        if rc != _lib.IWPP_OK:
            raise IwppError(rc, self._lib.iwpp_last_error(self._ctx._h).decode())

    def round_times(self) -> list:
        """Device time (us) of each phase of the last persistent kernel of the
        last replay (the graph's last group); [] before the first replay."""
        buf = (ctypes.c_double * 512)()
        n = ctypes.c_int32()
        rc = self._lib.iwpp_batch_graph_round_times(self._h, buf, 512, ctypes.byref(n))
        if rc != _lib.IWPP_OK:
            raise IwppError(rc, self._lib.iwpp_last_error(self._ctx._h).decode())
        return [float(buf[i]) for i in range(n.value)]

    def stats(self) -> dict:
        st = _lib.Stats()
        rc = self._lib.iwpp_batch_graph_stats(self._h, ctypes.byref(st))
        if rc != _lib.IWPP_OK:
            raise IwppError(rc, self._lib.iwpp_last_error(self._ctx._h).decode())
        return _stats_dict(st)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.iwpp_batch_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_host(t, name: str, dtype):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if t.device.type != "cpu":
        raise ValueError(f"{name} must be a host (CPU) tensor")
    if t.dim() != 2 or not t.is_contiguous():
        raise ValueError(f"{name} must be 2-D and contiguous")


class Server:
    """A request loop on a context (iwpp_server_*): jobs with HOST tensors
    (pinned memory lets copies overlap compute) are admitted against a device
    memory budget, run in continuous batches and copied back; with
    ``resident=True`` jobs come with tensors already on the context's device
    and nothing is copied.  While it runs, the context's other calls raise
    (busy)."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int = 0, scratch_bytes: int = 0, max_inflight: int = 0,
                 max_batch: int = 0, resident: bool = False):
        o = _lib.ServerOptions()
        o.hbm_budget_bytes = int(hbm_budget_bytes)
        o.scratch_bytes = int(scratch_bytes)
        o.max_inflight = int(max_inflight)
        o.max_batch = int(max_batch)
        o.resident = 1 if resident else 0
        self.resident = bool(resident)
        h = ctypes.c_void_p()
        rc = ctx._lib.iwpp_server_start(ctx._h, ctypes.byref(o), ctypes.byref(h))
        if rc != _lib.IWPP_OK:
            ctx._err(rc)
        self._ctx = ctx
        self._lib = ctx._lib
        self._h = h
        self._keep = {}  # ticket -> tensors the job reads or writes

    def _err(self, rc):
        raise IwppError(rc, self._lib.iwpp_last_error(self._ctx._h).decode())

    def submit(self, job: dict, arrival_ns: int = 0, stream=None) -> int:
        """Queue a job: ``{"op": "recon" or "erode", "marker", "mask", "out", "conn"}`` or
        ``{"op": "edt", "binary", "sqdist", "nearest", "conn"}`` with CPU
        tensors (device tensors of the context's device for a resident
        server); `arrival_ns` on time.monotonic_ns()'s clock (0 = now).  The
        job waits for the work queued on `stream` (default: torch's current
        stream of the context's device) before the submit."""
        torch = _torch()
        if stream is None:
            stream = torch.cuda.current_stream(torch.device("cuda", self._ctx.device))
        conn = int(job.get("conn", 8))
        if self.resident:
            dev = torch.device("cuda", self._ctx.device)
            check = lambda t, name, dtype: _check_image(t, name, dtype, dev)  # noqa: E731
        else:
            check = _check_host
        if job["op"] in ("recon", "erode"):
            for k in ("marker", "mask", "out"):
                check(job[k], k, torch.uint8)
            if not (job["marker"].shape == job["mask"].shape == job["out"].shape):
                raise ValueError("shapes differ")
            h, w = job["mask"].shape
            op = _lib.IWPP_OP_RECON if job["op"] == "recon" else _lib.IWPP_OP_RECON_ERODE
            j = _lib.Job(op, conn, h, w, job["marker"].data_ptr(), job["mask"].data_ptr(), job["out"].data_ptr(), None)
            keep = (job["marker"], job["mask"], job["out"])
        elif job["op"] == "edt":
            check(job["binary"], "binary", torch.uint8)
            check(job["sqdist"], "sqdist", torch.int32)
            check(job["nearest"], "nearest", torch.int32)
            if not (job["binary"].shape == job["sqdist"].shape == job["nearest"].shape):
                raise ValueError("shapes differ")
            h, w = job["binary"].shape
            j = _lib.Job(_lib.IWPP_OP_EDT, conn, h, w, job["binary"].data_ptr(), None, job["sqdist"].data_ptr(),
                         job["nearest"].data_ptr())
            keep = (job["binary"], job["sqdist"], job["nearest"])
        else:
            raise ValueError("op must be 'recon', 'erode' or 'edt'")
        t = ctypes.c_uint64()
        rc = self._lib.iwpp_server_submit(self._h, ctypes.byref(j), int(arrival_ns), ctypes.c_void_p(stream.cuda_stream),
                                          ctypes.byref(t))
        if rc != _lib.IWPP_OK:
            self._err(rc)
        self._keep[t.value] = keep
        return t.value

    def poll(self, ticket: int):
        """(state, latency_ms): state is one of _lib.JOB_*; latency -1 until done."""
        s = ctypes.c_int32()
        lat = ctypes.c_double()
        rc = self._lib.iwpp_server_poll(self._h, int(ticket), ctypes.byref(s), ctypes.byref(lat))
        if rc != _lib.IWPP_OK:
            self._err(rc)
        if s.value in (_lib.JOB_DONE, _lib.JOB_FAILED):
            self._keep.pop(int(ticket), None)
        return s.value, lat.value

    def drain(self, timeout_ms: int = -1) -> None:
        rc = self._lib.iwpp_server_drain(self._h, int(timeout_ms))
        if rc != _lib.IWPP_OK:
            self._err(rc)

    def stats(self) -> dict:
        st = _lib.ServerStats()
        rc = self._lib.iwpp_server_get_stats(self._h, ctypes.byref(st))
        if rc != _lib.IWPP_OK:
            self._err(rc)
        return {n: getattr(st, n) for n, _ in _lib.ServerStats._fields_ if n != "reserved"}

    def stop(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            h, self._h = self._h, ctypes.c_void_p()
            rc = self._lib.iwpp_server_stop(h)
            self._keep.clear()
            if rc != _lib.IWPP_OK:
                self._err(rc)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.stop()

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass


def _stats_dict(st) -> dict:
    return {"status": st.status, "op": st.op, "seeds": st.seeds, "items": st.items, "sweeps": st.sweeps,
            "rounds": st.rounds, "updates": st.updates, "overflow_restarts": st.overflow_restarts}


_contexts: dict = {}
_ctx_lock = threading.Lock()


def _default_ctx(device) -> Context:
    idx = device.index if device.index is not None else _torch().cuda.current_device()
    with _ctx_lock:
        c = _contexts.get(idx)
        if c is None:
            c = Context(idx)
            _contexts[idx] = c
        return c


def morph_recon(marker, mask, conn: int = 8, out=None):
    """Grayscale reconstruction by dilation rho_I(J) of `mask` from `marker`
    (uint8 GPU tensors of one shape); bit-exact."""
    _check_image(mask, "mask", _torch().uint8)
    return _default_ctx(mask.device).morph_recon(marker, mask, conn, out)


def morph_recon_erode(marker, mask, conn: int = 8, out=None):
    """Reconstruction by erosion rho*_I(J) of `mask` from `marker` (uint8 GPU
    tensors of one shape), the dual of morph_recon; bit-exact."""
    _check_image(mask, "mask", _torch().uint8)
    return _default_ctx(mask.device).morph_recon_erode(marker, mask, conn, out)


def edt(binary, conn: int = 8, out=None):
    """Propagation EDT of a uint8 GPU image (0 = feature).  Returns int32
    (squared distance, nearest feature index y*W+x); -1 if no feature."""
    _check_image(binary, "binary", _torch().uint8)
    return _default_ctx(binary.device).edt(binary, conn, out)


def last_stats(device=0) -> dict:
    """Counters of the last call on the default context of `device`."""
    torch = _torch()
    return _default_ctx(torch.device("cuda", device) if isinstance(device, int) else device).stats()
