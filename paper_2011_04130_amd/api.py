"""Torch-facing wrapper of the C ABI: device buffers are torch tensors.

Bit strings are int64 tensors holding the LSB-first 64-bit words (torch has
no general uint64 arithmetic; only the bit pattern matters).  Samples are
uint8 tensors.  Every call runs on the tensors' device, on torch's current
stream for that device unless a stream is given.
"""
from __future__ import annotations

import ctypes

import numpy as np

from ._lib import (MODEL_FIT, MODEL_GIVEN, MODEL_QUANTUM, PATH_AUTO, PLAN_ESTIMATE, PLAN_GRAPH,
                   PLAN_TUNE, U_MODEL_ARGMAX, Block, MeOpts, MeResult, PlanInfo, QrngError, Served,
                   ServerCfg, ServerStats, check, kernel_names, load_library)


def _words(bits: int) -> int:
    return (bits + 63) // 64


def _stream(torch, device, stream):
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """A libqrng context on one GPU (tables, workspace, seed cache)."""

    def __init__(self, device: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libqrng needs a ROCm GPU; none is visible")
        self._torch = torch
        self._lib = load_library()
        self.device = int(device)
        h = ctypes.c_void_p()
        check(self._lib.qrng_create(ctypes.byref(h), self.device))
        self._h = h
        self._seeds = {}

    # -- lifetime ---------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.qrng_destroy(self._h)
            self._h = None
            self._seeds.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ----------------------------------------------------------
    def _dev_tensor(self, t, name, dtype=None):
        torch = self._torch
        if not isinstance(t, torch.Tensor):
            raise TypeError("%s must be a torch tensor" % name)
        if t.device.type != "cuda" or t.device.index != self.device:
            raise ValueError("%s must live on cuda:%d" % (name, self.device))
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        if dtype is not None and t.dtype != dtype:
            raise TypeError("%s must have dtype %s" % (name, dtype))
        return ctypes.c_void_p(t.data_ptr())

    def _out(self, y, m):
        torch = self._torch
        if y is None:
            return torch.empty(max(_words(m), 1), dtype=torch.int64,
                               device="cuda:%d" % self.device)
        if y.numel() * y.element_size() < _words(m) * 8:
            raise ValueError("output buffer too small for %d bits" % m)
        return y

    # -- kernel timing --------------------------------------------------------
    def profile(self, on: bool = True) -> None:
        """Bracket every kernel launch with HIP events on its own stream."""
        check(self._lib.qrng_profile_enable(self._h, 1 if on else 0))

    def profile_reset(self) -> None:
        check(self._lib.qrng_profile_reset(self._h))

    def profile_read(self) -> dict:
        """{kernel: (launches, total_ms)} since the last reset."""
        out = {}
        for kid, name in enumerate(kernel_names()):
            cnt, ms = ctypes.c_uint64(), ctypes.c_double()
            check(self._lib.qrng_profile_query(self._h, kid, ctypes.byref(cnt), ctypes.byref(ms)))
            if cnt.value:
                out[name] = (int(cnt.value), float(ms.value))
        return out

    def issue_rates(self, clock_ghz: float = 2.4, stream=None) -> dict:
        """{instruction: cycles per wave64 instruction per SIMD}, measured on
        the device by the library's probe kernels (4.0 = the nominal rate)."""
        import torch
        n = 8
        buf = (ctypes.c_double * n)()
        check(self._lib.qrng_profile_issue_rates(self._h, float(clock_ghz), buf, n,
                                                 _stream(torch, self.device, stream)))
        out = {}
        for i in range(n):
            nm = self._lib.qrng_profile_issue_op_name(i)
            if nm:
                out[nm.decode()] = round(float(buf[i]), 3)
        return out

    # -- Sec. II ------------------------------------------------------------
    def minentropy(self, samples, sample_bits: int = 8, model: int = MODEL_FIT,
                   mu: float = 0.0, sigma: float = 0.0, u_mode: int = U_MODEL_ARGMAX,
                   stream=None, want_counts: bool = False, subset_seed: int = 0,
                   keep_thr: int = 0) -> dict:
        """Sec. II estimate of 1-byte samples (synchronous); keep_thr > 0
        estimates on the random subset qrng_minentropy_subset keeps."""
        torch = self._torch
        p = self._dev_tensor(samples, "samples", torch.uint8)
        opts = MeOpts(sample_bits, model, mu, sigma, u_mode, 0)
        res = MeResult()
        counts = (ctypes.c_uint64 * (1 << sample_bits))() if want_counts else None
        check(self._lib.qrng_minentropy_subset(self._h, p, samples.numel(), ctypes.byref(opts),
                                               subset_seed, keep_thr, ctypes.byref(res), counts,
                                               _stream(torch, self.device, stream)))
        out = res.as_dict()
        if want_counts:
            out["counts"] = list(counts)
        return out

    # -- Sec. III.B ---------------------------------------------------------
    def hash(self, x, n: int, seed, m: int, y=None, path: int = PATH_AUTO, stream=None):
        """y = T x mod 2 for one block (returns the int64 word tensor y)."""
        torch = self._torch
        xp = self._dev_tensor(x, "x")
        sp = self._dev_tensor(seed, "seed")
        if x.numel() * x.element_size() < _words(n) * 8:
            raise ValueError("x holds fewer than n bits")
        if m and seed.numel() * seed.element_size() < _words(n + m - 1) * 8:
            raise ValueError("seed holds fewer than n+m-1 bits")
        y = self._out(y, m)
        yp = self._dev_tensor(y, "y")
        check(self._lib.qrng_toeplitz_hash(self._h, xp, n, sp, m, yp, path,
                                           _stream(torch, self.device, stream)))
        return y

    def hash_noalloc(self, x, n: int, seed, m: int, y, path: int = PATH_AUTO, stream=None):
        """As hash(), through the entry point that allocates nothing (its
        intermediate buffers live in a fixed per-device scratch array); y is
        required, since this call must not allocate either."""
        torch = self._torch
        xp = self._dev_tensor(x, "x")
        sp = self._dev_tensor(seed, "seed")
        if x.numel() * x.element_size() < _words(n) * 8:
            raise ValueError("x holds fewer than n bits")
        if m and seed.numel() * seed.element_size() < _words(n + m - 1) * 8:
            raise ValueError("seed holds fewer than n+m-1 bits")
        if y is None or y.numel() * y.element_size() < _words(m) * 8:
            raise ValueError("y must hold ceil(m/64) words")
        yp = self._dev_tensor(y, "y")
        check(self._lib.qrng_toeplitz_hash_noalloc(self._h, xp, n, sp, m, yp, path,
                                                   _stream(torch, self.device, stream)))
        return y

    def register_seed(self, seed, L: int, stream=None) -> int:
        """Register L seed bits; their transforms are computed now, on
        `stream` (torch's current stream by default), after the work that
        filled the seed."""
        sp = self._dev_tensor(seed, "seed")
        if seed.numel() * seed.element_size() < _words(L) * 8:
            raise ValueError("seed holds fewer than L bits")
        sid = ctypes.c_uint32()
        check(self._lib.qrng_seed_register(self._h, sp, L, ctypes.byref(sid),
                                           _stream(self._torch, self.device, stream)))
        self._seeds[sid.value] = seed  # keep the memory alive while registered
        return sid.value

    def unregister_seed(self, seed_id: int) -> None:
        check(self._lib.qrng_seed_unregister(self._h, seed_id))
        self._seeds.pop(seed_id, None)

    def hash_seeded(self, x, n: int, seed_id: int, m: int, y=None, path: int = PATH_AUTO,
                    stream=None):
        torch = self._torch
        xp = self._dev_tensor(x, "x")
        if x.numel() * x.element_size() < _words(n) * 8:
            raise ValueError("x holds fewer than n bits")
        y = self._out(y, m)
        yp = self._dev_tensor(y, "y")
        check(self._lib.qrng_toeplitz_hash_seeded(self._h, xp, n, seed_id, m, yp, path,
                                                  _stream(torch, self.device, stream)))
        return y

    def hash_fft64(self, x, n: int, seed, m: int, y=None, err_out=None, stream=None):
        """The paper's float64 circulant method on the device (returns y).

        err_out: float64 tensor of >= 1 element (receives the largest distance
        of a kept value from its integer)."""
        torch = self._torch
        xp = self._dev_tensor(x, "x")
        sp = self._dev_tensor(seed, "seed")
        if x.numel() * x.element_size() < _words(n) * 8:
            raise ValueError("x holds fewer than n bits")
        if m and seed.numel() * seed.element_size() < _words(n + m - 1) * 8:
            raise ValueError("seed holds fewer than n+m-1 bits")
        y = self._out(y, m)
        yp = self._dev_tensor(y, "y")
        ep = self._dev_tensor(err_out, "err_out") if err_out is not None else None
        check(self._lib.qrng_toeplitz_hash_fft64(self._h, xp, n, sp, m, yp, ep,
                                                 _stream(torch, self.device, stream)))
        return y

    def modified_hash(self, x, n: int, seed, m: int, y=None, path: int = PATH_AUTO,
                      stream=None):
        """Sec. III.D: y = (A, I_m) x mod 2 with an (n-1)-bit seed (returns y)."""
        torch = self._torch
        xp = self._dev_tensor(x, "x")
        sp = self._dev_tensor(seed, "seed")
        if x.numel() * x.element_size() < _words(n) * 8:
            raise ValueError("x holds fewer than n bits")
        if seed.numel() * seed.element_size() < _words(max(n - 1, 1)) * 8:
            raise ValueError("seed holds fewer than n-1 bits")
        y = self._out(y, m)
        yp = self._dev_tensor(y, "y")
        check(self._lib.qrng_modified_toeplitz_hash(self._h, xp, n, sp, m, yp, path,
                                                    _stream(torch, self.device, stream)))
        return y

    def modified_hash_seeded(self, x, n: int, seed_id: int, m: int, y=None,
                             path: int = PATH_AUTO, stream=None):
        """modified_hash with a registered seed (its first n-1 bits)."""
        torch = self._torch
        xp = self._dev_tensor(x, "x")
        if x.numel() * x.element_size() < _words(n) * 8:
            raise ValueError("x holds fewer than n bits")
        y = self._out(y, m)
        yp = self._dev_tensor(y, "y")
        check(self._lib.qrng_modified_toeplitz_hash_seeded(self._h, xp, n, seed_id, m, yp, path,
                                                           _stream(torch, self.device, stream)))
        return y

    def extract(self, samples, seed_id: int, m_cap: int, y=None, m_out=None, me_out=None,
                model: int = MODEL_FIT, mu: float = 0.0, sigma: float = 0.0,
                u_mode: int = U_MODEL_ARGMAX, log2_inv_eps: float = 0.0,
                path: int = PATH_AUTO, stream=None):
        """Asynchronous min-entropy -> m -> hash of 8-bit samples, all on the device.

        m_out: int64 tensor of >= 1 element (receives m); me_out: uint8 tensor
        of >= sizeof(qrng_me_result) bytes (receives the estimate).  Returns y.
        """
        torch = self._torch
        sp = self._dev_tensor(samples, "samples", torch.uint8)
        y = self._out(y, m_cap)
        yp = self._dev_tensor(y, "y")
        mp = self._dev_tensor(m_out, "m_out") if m_out is not None else None
        if me_out is not None and me_out.numel() * me_out.element_size() < ctypes.sizeof(MeResult):
            raise ValueError("me_out too small")
        rp = self._dev_tensor(me_out, "me_out") if me_out is not None else None
        opts = MeOpts(8, model, mu, sigma, u_mode, 0)
        check(self._lib.qrng_extract(self._h, sp, samples.numel(), ctypes.byref(opts),
                                     log2_inv_eps, seed_id, m_cap, yp, mp, rp, path,
                                     _stream(torch, self.device, stream)))
        return y

    @staticmethod
    def me_result_from_bytes(buf) -> dict:
        """Decode a qrng_me_result read back from device memory (uint8 tensor)."""
        raw = bytes(buf.cpu().numpy().tobytes()[: ctypes.sizeof(MeResult)])
        return MeResult.from_buffer_copy(raw).as_dict()

    # -- Sec. III.E ---------------------------------------------------------
    def hash_strided(self, x_pool, n: int, x_stride_words: int, seed_id: int, m: int, y_pool,
                     y_stride_words: int, nblocks: int, path: int = PATH_AUTO, stream=None):
        """Equal blocks at constant strides (a long sequence cut into blocks)."""
        torch = self._torch
        if nblocks and (x_pool.numel() * x_pool.element_size() // 8
                        < (nblocks - 1) * x_stride_words + _words(n)):
            raise ValueError("x_pool too small")
        if nblocks and (y_pool.numel() * y_pool.element_size() // 8
                        < (nblocks - 1) * y_stride_words + _words(m)):
            raise ValueError("y_pool too small")
        xp = self._dev_tensor(x_pool, "x_pool")
        yp = self._dev_tensor(y_pool, "y_pool")
        check(self._lib.qrng_toeplitz_hash_strided(self._h, xp, n, x_stride_words, seed_id, m, yp,
                                                   y_stride_words, nblocks, path,
                                                   _stream(torch, self.device, stream)))
        return y_pool

    @staticmethod
    def _block_records(blocks, x_pool, y_pool):
        """Checked qrng_block records (numpy) for (x_word_off, n, m, y_word_off, seed_id) rows."""
        import numpy as np
        a = np.asarray(blocks, dtype=np.uint64).reshape(-1, 5)
        xw = x_pool.numel() * x_pool.element_size() // 8
        yw = y_pool.numel() * y_pool.element_size() // 8
        words = lambda b: (b + np.uint64(63)) // np.uint64(64)
        bad = (a[:, 0] + words(a[:, 1]) > xw) | (a[:, 3] + words(a[:, 2]) > yw)
        if bad.any():
            raise ValueError("block %d lies outside its pool" % int(np.flatnonzero(bad)[0]))
        rec = np.zeros(len(a), dtype=np.dtype([("x", "<u8"), ("n", "<u8"), ("m", "<u8"),
                                               ("y", "<u8"), ("sid", "<u4"), ("flags", "<u4")]))
        rec["x"], rec["n"], rec["m"], rec["y"], rec["sid"] = a[:, 0], a[:, 1], a[:, 2], a[:, 3], a[:, 4]
        assert rec.dtype.itemsize == ctypes.sizeof(Block)
        return rec

    def block_records(self, blocks, x_pool, y_pool):
        """qrng_block records of (x_word_off, n, m, y_word_off, seed_id) rows as
        a uint8 device tensor, for hash_batched (offsets checked against the
        pools here, on the host)."""
        rec = self._block_records(blocks, x_pool, y_pool)
        return self._torch.from_numpy(rec.view(np.uint8).copy()).to("cuda:%d" % self.device)

    def hash_batched(self, blocks_dev, x_pool, y_pool, seed_ids=None, path: int = PATH_AUTO,
                     stream=None):
        """Blocks described in device memory (blocks_dev: uint8 tensor of
        qrng_block records, e.g. from block_records; seed_ids: optional int32
        device tensor of one seed id per block).  Graph-capturable."""
        torch = self._torch
        nb = blocks_dev.numel() * blocks_dev.element_size() // ctypes.sizeof(Block)
        bp = self._dev_tensor(blocks_dev, "blocks_dev")
        sp = None
        if seed_ids is not None:
            if seed_ids.numel() < nb or seed_ids.element_size() != 4:
                raise ValueError("seed_ids holds fewer than one 32-bit id per block")
            sp = self._dev_tensor(seed_ids, "seed_ids")
        xp = self._dev_tensor(x_pool, "x_pool")
        yp = self._dev_tensor(y_pool, "y_pool")
        check(self._lib.qrng_toeplitz_hash_batched(self._h, bp, nb, xp, sp, yp, path,
                                                   _stream(torch, self.device, stream)))
        return y_pool

    def batched_rejected(self, stream=None) -> int:
        """Descriptors the last hash_batched call skipped as invalid."""
        c = ctypes.c_uint32()
        check(self._lib.qrng_toeplitz_hash_batched_rejected(
            self._h, ctypes.byref(c), _stream(self._torch, self.device, stream)))
        return int(c.value)

    def hash_batched_host(self, blocks, x_pool, y_pool, path: int = PATH_AUTO, stream=None):
        """blocks: (k, 5) integer array or iterable of
        (x_word_off, n, m, y_word_off, seed_id), in host memory."""
        torch = self._torch
        rec = self._block_records(blocks, x_pool, y_pool)
        arr = rec.ctypes.data_as(ctypes.POINTER(Block))
        xp = self._dev_tensor(x_pool, "x_pool")
        yp = self._dev_tensor(y_pool, "y_pool")
        check(self._lib.qrng_toeplitz_hash_batched_host(self._h, arr, len(rec), xp, yp, path,
                                                        _stream(torch, self.device, stream)))
        return y_pool

    # -- uneven batches fixed once ---------------------------------------------
    def plan(self, blocks, x_pool, y_pool, m_out=None, me_out=None, estimate: bool = False,
             graph: bool = False, tune: bool = False, model: int = MODEL_FIT, mu: float = 0.0,
             sigma: float = 0.0, u_mode: int = U_MODEL_ARGMAX, log2_inv_eps: float = 0.0,
             path: int = PATH_AUTO, stream=None) -> "Plan":
        """A qrng_plan over (x_word_off, n, m, y_word_off, seed_id) rows.

        With estimate=True, m is each block's cap and m_out (int64 tensor of
        len(blocks)) receives the output lengths; me_out (uint8 tensor of
        len(blocks) * sizeof(qrng_me_result) bytes) the estimates.
        """
        torch = self._torch
        rec = self._block_records(blocks, x_pool, y_pool)
        k = len(rec)
        xp = self._dev_tensor(x_pool, "x_pool")
        yp = self._dev_tensor(y_pool, "y_pool")
        mp = rp = None
        if m_out is not None:
            if m_out.numel() * m_out.element_size() < 8 * k:
                raise ValueError("m_out holds fewer than len(blocks) lengths")
            mp = self._dev_tensor(m_out, "m_out")
        if me_out is not None:
            if me_out.numel() * me_out.element_size() < k * ctypes.sizeof(MeResult):
                raise ValueError("me_out too small")
            rp = self._dev_tensor(me_out, "me_out")
        flags = (PLAN_ESTIMATE if estimate else 0) | (PLAN_GRAPH if graph else 0) | \
                (PLAN_TUNE if tune else 0)
        opts = MeOpts(8, model, mu, sigma, u_mode, 0)
        h = ctypes.c_void_p()
        check(self._lib.qrng_plan_create(self._h, rec.ctypes.data_as(ctypes.POINTER(Block)), k,
                                         xp, yp, mp, rp, ctypes.byref(opts), log2_inv_eps, path,
                                         flags, _stream(torch, self.device, stream),
                                         ctypes.byref(h)))
        return Plan(self, h, (x_pool, y_pool, m_out, me_out))

    def server(self, seed_id: int, window_samples: int, block_bits: int = 0,
               ring_bits: int = 1 << 30, window_slots: int = 4, max_queue: int = 1 << 16,
               model: int = MODEL_FIT, mu: float = 0.0, sigma: float = 0.0,
               u_mode: int = U_MODEL_ARGMAX, log2_inv_eps: float = 0.0,
               path: int = PATH_AUTO) -> "Server":
        """A qrng_server (continuous batching over windows of raw samples)."""
        cfg = ServerCfg(window_samples, block_bits, ring_bits, window_slots, max_queue, seed_id,
                        path, MeOpts(8, model, mu, sigma, u_mode, 0), log2_inv_eps)
        h = ctypes.c_void_p()
        check(self._lib.qrng_server_create(self._h, ctypes.byref(cfg), ctypes.byref(h)))
        return Server(self, h)

    def tune_export(self) -> str:
        n = ctypes.c_uint64()
        check(self._lib.qrng_tune_export(self._h, None, 0, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value + 1)
        check(self._lib.qrng_tune_export(self._h, buf, n.value + 1, ctypes.byref(n)))
        return buf.value.decode()

    def tune_import(self, text: str) -> None:
        check(self._lib.qrng_tune_import(self._h, text.encode()))

    def tune_save(self, path: str) -> None:
        with open(path, "w") as f:
            f.write(self.tune_export())

    def tune_load(self, path: str) -> None:
        with open(path) as f:
            self.tune_import(f.read())


class Plan:
    """An uneven batch fixed once (see Context.plan); keeps its buffers alive."""

    def __init__(self, ctx: Context, handle, keep):
        self._ctx = ctx
        self._h = handle
        self._keep = keep

    def execute(self, stream=None) -> None:
        torch = self._ctx._torch
        check(self._ctx._lib.qrng_plan_execute(self._h, _stream(torch, self._ctx.device, stream)))

    def info(self) -> dict:
        i = PlanInfo()
        check(self._ctx._lib.qrng_plan_query(self._h, ctypes.byref(i)))
        return i.as_dict()

    def close(self) -> None:
        if getattr(self, "_h", None) and getattr(self._ctx, "_h", None):
            self._ctx._lib.qrng_plan_destroy(self._h)
        self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop on one context (see Context.server)."""

    def __init__(self, ctx: Context, handle):
        self._ctx = ctx
        self._h = handle
        self._lib = ctx._lib

    def feed(self, samples, stream=None) -> None:
        torch = self._ctx._torch
        p = self._ctx._dev_tensor(samples, "samples", torch.uint8)
        check(self._lib.qrng_server_feed(self._h, p, _stream(torch, self._ctx.device, stream)))

    def try_feed(self, samples, stream=None) -> bool:
        """feed(), but False instead of an error when every slot is busy."""
        torch = self._ctx._torch
        p = self._ctx._dev_tensor(samples, "samples", torch.uint8)
        st = self._lib.qrng_server_feed(self._h, p, _stream(torch, self._ctx.device, stream))
        if st == -5:
            return False
        check(st)
        return True

    def submit(self, bits: int) -> int:
        rid = ctypes.c_uint64()
        check(self._lib.qrng_server_submit(self._h, bits, ctypes.byref(rid)))
        return rid.value

    def submit_many(self, bits):
        """Queue many requests (numpy-convertible sizes); returns the
        accepted ids as a uint64 array (shorter if the queue filled)."""
        import numpy as np
        b = np.ascontiguousarray(np.asarray(bits, dtype=np.uint64))
        ids = np.empty(len(b), dtype=np.uint64)
        n = ctypes.c_uint32()
        check(self._lib.qrng_server_submit_many(self._h, b.ctypes.data, len(b), ids.ctypes.data,
                                                ctypes.byref(n)))
        return ids[: n.value]

    def release_many(self, ids) -> None:
        import numpy as np
        a = np.ascontiguousarray(np.asarray(ids, dtype=np.uint64))
        check(self._lib.qrng_server_release_many(self._h, a.ctypes.data, len(a)))

    def poll_array(self, cap: int = 1 << 16):
        """Completed requests as a numpy structured array (fields of qrng_served)."""
        import numpy as np
        dt = np.dtype([("request_id", "<u8"), ("bits", "<u8"), ("ring_word", "<u8"),
                       ("window", "<u8"), ("first_block", "<u8"), ("blocks", "<u4"),
                       ("status", "<i4"), ("m_block", "<u8")])
        assert dt.itemsize == ctypes.sizeof(Served)
        out = np.empty(cap, dtype=dt)
        n = ctypes.c_uint32()
        check(self._lib.qrng_server_poll(self._h, out.ctypes.data_as(ctypes.POINTER(Served)), cap,
                                         ctypes.byref(n)))
        return out[: n.value]

    def step(self) -> int:
        n = ctypes.c_uint32()
        check(self._lib.qrng_server_step(self._h, ctypes.byref(n)))
        return n.value

    def poll(self, cap: int = 4096) -> list:
        arr = (Served * cap)()
        n = ctypes.c_uint32()
        check(self._lib.qrng_server_poll(self._h, arr, cap, ctypes.byref(n)))
        return [arr[i].as_dict() for i in range(n.value)]

    def release(self, request_id: int) -> None:
        check(self._lib.qrng_server_release(self._h, request_id))

    def read(self, request_id: int, bits: int, out=None, stream=None):
        """A completed request's output bits as an int64 word tensor."""
        torch = self._ctx._torch
        if out is None:
            out = torch.empty((bits + 63) // 64, dtype=torch.int64,
                              device="cuda:%d" % self._ctx.device)
        if out.numel() * out.element_size() < (bits + 63) // 64 * 8:
            raise ValueError("output buffer too small")
        p = self._ctx._dev_tensor(out, "out")
        check(self._lib.qrng_server_read(self._h, request_id, p,
                                         _stream(torch, self._ctx.device, stream)))
        return out

    def ring_ptr(self) -> int:
        p = ctypes.c_void_p()
        check(self._lib.qrng_server_ring(self._h, ctypes.byref(p)))
        return p.value

    def window_estimate_ptr(self, window: int) -> int:
        s, e = ctypes.c_void_p(), ctypes.c_void_p()
        check(self._lib.qrng_server_window(self._h, window, ctypes.byref(s), ctypes.byref(e)))
        return e.value

    def stats(self) -> dict:
        st = ServerStats()
        check(self._lib.qrng_server_query(self._h, ctypes.byref(st)))
        return st.as_dict()

    def close(self) -> None:
        if getattr(self, "_h", None) and getattr(self._ctx, "_h", None):
            self._lib.qrng_server_destroy(self._h)
        self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


__all__ = ["Context", "Plan", "Server", "QrngError"]
