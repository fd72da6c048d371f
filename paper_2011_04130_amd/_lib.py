"""ctypes declarations of the C ABI in include/qrng.h (no torch needed)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libqrng.so")

OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, EBUSY = 0, -1, -2, -3, -4, -5
PATH_AUTO, PATH_DIRECT, PATH_NTT, PATH_MFMA = 0, 1, 2, 3
U_MODEL_ARGMAX, U_BOTH_ARGMAX, U_ALL = 0, 1, 2
MODEL_FIT, MODEL_GIVEN, MODEL_QUANTUM = 0, 1, 2
PLAN_ESTIMATE, PLAN_GRAPH, PLAN_TUNE = 1, 2, 4

_NAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE",
          EUNSUPPORTED: "EUNSUPPORTED", EBUSY: "EBUSY"}


class QrngError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_NAMES.get(status, str(status)), msg))
        self.status = status


class MeOpts(ctypes.Structure):
    _fields_ = [("sample_bits", ctypes.c_int32), ("model", ctypes.c_int32),
                ("mu", ctypes.c_double), ("sigma", ctypes.c_double),
                ("u_mode", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class MeResult(ctypes.Structure):
    _fields_ = [("mu_hat", ctypes.c_double), ("sigma_hat", ctypes.c_double),
                ("h_min", ctypes.c_double), ("h_actual", ctypes.c_double),
                ("d_u", ctypes.c_double), ("delta_h_m", ctypes.c_double),
                ("h_mod", ctypes.c_double), ("argmax_model", ctypes.c_uint32),
                ("argmax_empirical", ctypes.c_uint32), ("samples", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class Block(ctypes.Structure):
    _fields_ = [("x_word_off", ctypes.c_uint64), ("n", ctypes.c_uint64),
                ("m", ctypes.c_uint64), ("y_word_off", ctypes.c_uint64),
                ("seed_id", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("blocks", ctypes.c_uint32), ("classes", ctypes.c_uint32),
                ("launches", ctypes.c_uint32), ("graph", ctypes.c_uint32),
                ("workspace_bytes", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerCfg(ctypes.Structure):
    _fields_ = [("window_samples", ctypes.c_uint64), ("block_bits", ctypes.c_uint64),
                ("ring_bits", ctypes.c_uint64), ("window_slots", ctypes.c_uint32),
                ("max_queue", ctypes.c_uint32), ("seed_id", ctypes.c_uint32),
                ("path", ctypes.c_int32), ("opts", MeOpts), ("log2_inv_eps", ctypes.c_double)]


class Served(ctypes.Structure):
    _fields_ = [("request_id", ctypes.c_uint64), ("bits", ctypes.c_uint64),
                ("ring_word", ctypes.c_uint64), ("window", ctypes.c_uint64),
                ("first_block", ctypes.c_uint64), ("blocks", ctypes.c_uint32),
                ("status", ctypes.c_int32), ("m_block", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in
                ("block_bits", "blocks_per_window", "windows_fed", "windows_used",
                 "blocks_hashed", "bits_served", "queued", "in_flight", "ring_free_bits",
                 "m_block")]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None

# every symbol the header declares
EXPORTS = ["qrng_version", "qrng_last_error", "qrng_create", "qrng_destroy",
           "qrng_minentropy", "qrng_minentropy_subset", "qrng_output_bits",
           "qrng_toeplitz_hash", "qrng_toeplitz_hash_noalloc",
           "qrng_seed_register", "qrng_seed_unregister", "qrng_toeplitz_hash_seeded",
           "qrng_modified_toeplitz_hash", "qrng_modified_toeplitz_hash_seeded",
           "qrng_toeplitz_hash_fft64",
           "qrng_toeplitz_hash_batched", "qrng_toeplitz_hash_batched_rejected",
           "qrng_toeplitz_hash_batched_host", "qrng_toeplitz_hash_strided", "qrng_extract",
           "qrng_plan_create", "qrng_plan_execute", "qrng_plan_query", "qrng_plan_destroy",
           "qrng_tune_export", "qrng_tune_import",
           "qrng_server_create", "qrng_server_feed", "qrng_server_submit",
           "qrng_server_submit_many", "qrng_server_release_many", "qrng_server_step",
           "qrng_server_poll", "qrng_server_release", "qrng_server_read", "qrng_server_ring",
           "qrng_server_window",
           "qrng_server_query", "qrng_server_destroy",
           "qrng_profile_enable", "qrng_profile_kernel_name",
           "qrng_profile_query", "qrng_profile_reset",
           "qrng_profile_issue_rates", "qrng_profile_issue_op_name"]


def load_library(path: str | None = None):
    """Load libqrng.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise OSError("libqrng.so is not built (%s); run python -m paper_2011_04130_amd.build" % p)
    lib = ctypes.CDLL(p)
    vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    lib.qrng_version.restype = ctypes.c_char_p
    lib.qrng_last_error.restype = ctypes.c_char_p
    lib.qrng_create.argtypes = [ctypes.POINTER(vp), i32]
    lib.qrng_create.restype = i32
    lib.qrng_destroy.argtypes = [vp]
    lib.qrng_destroy.restype = None
    lib.qrng_minentropy.argtypes = [vp, vp, u64, ctypes.POINTER(MeOpts),
                                    ctypes.POINTER(MeResult), ctypes.POINTER(u64), vp]
    lib.qrng_minentropy.restype = i32
    lib.qrng_minentropy_subset.argtypes = [vp, vp, u64, ctypes.POINTER(MeOpts), u64, u32,
                                           ctypes.POINTER(MeResult), ctypes.POINTER(u64), vp]
    lib.qrng_minentropy_subset.restype = i32
    lib.qrng_output_bits.argtypes = [u64, i32, ctypes.c_double, ctypes.c_double,
                                     ctypes.POINTER(u64)]
    lib.qrng_output_bits.restype = i32
    lib.qrng_toeplitz_hash.argtypes = [vp, vp, u64, vp, u64, vp, i32, vp]
    lib.qrng_toeplitz_hash.restype = i32
    lib.qrng_toeplitz_hash_noalloc.argtypes = [vp, vp, u64, vp, u64, vp, i32, vp]
    lib.qrng_toeplitz_hash_noalloc.restype = i32
    lib.qrng_seed_register.argtypes = [vp, vp, u64, ctypes.POINTER(u32), vp]
    lib.qrng_seed_register.restype = i32
    lib.qrng_seed_unregister.argtypes = [vp, u32]
    lib.qrng_seed_unregister.restype = i32
    lib.qrng_toeplitz_hash_seeded.argtypes = [vp, vp, u64, u32, u64, vp, i32, vp]
    lib.qrng_toeplitz_hash_seeded.restype = i32
    lib.qrng_toeplitz_hash_fft64.argtypes = [vp, vp, u64, vp, u64, vp, vp, vp]
    lib.qrng_toeplitz_hash_fft64.restype = i32
    lib.qrng_modified_toeplitz_hash.argtypes = [vp, vp, u64, vp, u64, vp, i32, vp]
    lib.qrng_modified_toeplitz_hash.restype = i32
    lib.qrng_modified_toeplitz_hash_seeded.argtypes = [vp, vp, u64, u32, u64, vp, i32, vp]
    lib.qrng_modified_toeplitz_hash_seeded.restype = i32
    lib.qrng_toeplitz_hash_batched.argtypes = [vp, vp, u32, vp, vp, vp, i32, vp]
    lib.qrng_toeplitz_hash_batched.restype = i32
    lib.qrng_toeplitz_hash_batched_rejected.argtypes = [vp, ctypes.POINTER(u32), vp]
    lib.qrng_toeplitz_hash_batched_rejected.restype = i32
    lib.qrng_toeplitz_hash_batched_host.argtypes = [vp, ctypes.POINTER(Block), u32, vp, vp,
                                                    i32, vp]
    lib.qrng_toeplitz_hash_batched_host.restype = i32
    lib.qrng_toeplitz_hash_strided.argtypes = [vp, vp, u64, u64, u32, u64, vp, u64, u32, i32,
                                               vp]
    lib.qrng_toeplitz_hash_strided.restype = i32
    lib.qrng_extract.argtypes = [vp, vp, u64, ctypes.POINTER(MeOpts), ctypes.c_double, u32,
                                 u64, vp, vp, vp, i32, vp]
    lib.qrng_extract.restype = i32
    lib.qrng_plan_create.argtypes = [vp, ctypes.POINTER(Block), u32, vp, vp, vp, vp,
                                     ctypes.POINTER(MeOpts), ctypes.c_double, i32, u32, vp,
                                     ctypes.POINTER(vp)]
    lib.qrng_plan_create.restype = i32
    lib.qrng_plan_execute.argtypes = [vp, vp]
    lib.qrng_plan_execute.restype = i32
    lib.qrng_plan_query.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    lib.qrng_plan_query.restype = i32
    lib.qrng_plan_destroy.argtypes = [vp]
    lib.qrng_plan_destroy.restype = None
    lib.qrng_tune_export.argtypes = [vp, ctypes.c_char_p, u64, ctypes.POINTER(u64)]
    lib.qrng_tune_export.restype = i32
    lib.qrng_tune_import.argtypes = [vp, ctypes.c_char_p]
    lib.qrng_tune_import.restype = i32
    lib.qrng_server_create.argtypes = [vp, ctypes.POINTER(ServerCfg), ctypes.POINTER(vp)]
    lib.qrng_server_feed.argtypes = [vp, vp, vp]
    lib.qrng_server_submit.argtypes = [vp, u64, ctypes.POINTER(u64)]
    lib.qrng_server_step.argtypes = [vp, ctypes.POINTER(u32)]
    lib.qrng_server_submit_many.argtypes = [vp, vp, u32, vp, ctypes.POINTER(u32)]
    lib.qrng_server_release_many.argtypes = [vp, vp, u32]
    lib.qrng_server_poll.argtypes = [vp, ctypes.POINTER(Served), u32, ctypes.POINTER(u32)]
    lib.qrng_server_release.argtypes = [vp, u64]
    lib.qrng_server_read.argtypes = [vp, u64, vp, vp]
    lib.qrng_server_ring.argtypes = [vp, ctypes.POINTER(vp)]
    lib.qrng_server_window.argtypes = [vp, u64, ctypes.POINTER(vp), ctypes.POINTER(vp)]
    lib.qrng_server_query.argtypes = [vp, ctypes.POINTER(ServerStats)]
    for f in ("create", "feed", "submit", "submit_many", "step", "poll", "release",
              "release_many", "read", "ring", "window", "query"):
        getattr(lib, "qrng_server_" + f).restype = i32
    lib.qrng_server_destroy.argtypes = [vp]
    lib.qrng_server_destroy.restype = None
    lib.qrng_profile_enable.argtypes = [vp, i32]
    lib.qrng_profile_enable.restype = i32
    lib.qrng_profile_kernel_name.argtypes = [i32]
    lib.qrng_profile_kernel_name.restype = ctypes.c_char_p
    lib.qrng_profile_query.argtypes = [vp, i32, ctypes.POINTER(u64),
                                       ctypes.POINTER(ctypes.c_double)]
    lib.qrng_profile_query.restype = i32
    lib.qrng_profile_reset.argtypes = [vp]
    lib.qrng_profile_reset.restype = i32
    lib.qrng_profile_issue_rates.argtypes = [vp, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                             i32, vp]
    lib.qrng_profile_issue_rates.restype = i32
    lib.qrng_profile_issue_op_name.argtypes = [i32]
    lib.qrng_profile_issue_op_name.restype = ctypes.c_char_p
    if path is None:
        _lib = lib
    return lib


def check(status: int) -> None:
    if status != OK:
        msg = load_library().qrng_last_error().decode(errors="replace")
        raise QrngError(status, msg)


def kernel_names() -> list:
    """Kernel classes the timing hooks report, in id order."""
    lib = load_library()
    out, i = [], 0
    while True:
        nm = lib.qrng_profile_kernel_name(i)
        if not nm:
            return out
        out.append(nm.decode())
        i += 1


def version() -> str:
    return load_library().qrng_version().decode()


def output_bits(n: int, sample_bits: int, h_mod: float, log2_inv_eps: float = 0.0) -> int:
    """m = n H/N - 2 log2(1/eps) with H in whole bits per sample (host only)."""
    out = ctypes.c_uint64()
    check(load_library().qrng_output_bits(n, sample_bits, h_mod, log2_inv_eps,
                                          ctypes.byref(out)))
    return int(out.value)
