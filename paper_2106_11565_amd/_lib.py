"""ctypes binding of libflinng.so (argument marshalling only).

Every step of the query path runs in the HIP library; this module only turns
numpy arrays / torch tensors into the C structs of include/flinng.h.  torch is
used for device memory and streams.  If the library is not built, importing
raises: there is no fallback path.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libflinng.so")

SRP_F32, SRP_BF16, MINHASH_U32, MINHASH_U64 = 0, 1, 2, 3
OK, EINVAL, ENOMEM, EDEVICE, EBUSY, ETIMEDOUT, ESTATE = 0, -22, -12, -5, -16, -110, -77

c_u32, c_u64, c_i64, c_vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p


class FlinngError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"flinng error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("family", c_u32), ("dim", c_u32), ("K", c_u32), ("L", c_u32),
                ("R", c_u32), ("B", c_u32), ("bucket_bits", c_u32),
                ("reserved", c_u32), ("seed", c_u64)]


class Input(ctypes.Structure):
    _fields_ = [("values", c_vp), ("offsets", c_vp), ("count", c_u64),
                ("on_device", c_u32), ("reserved", c_u32)]


class Text(ctypes.Structure):
    _fields_ = [("symbols", c_vp), ("offsets", c_vp), ("count", c_u64), ("key", c_u64),
                ("gram", c_u32), ("radix", c_u32), ("on_device", c_u32), ("reserved", c_u32)]


class IndexInfo(ctypes.Structure):
    _fields_ = [("N", c_u64), ("list_entries", c_u64), ("device_bytes", c_u64),
                ("family", c_u32), ("dim", c_u32), ("K", c_u32), ("L", c_u32),
                ("R", c_u32), ("B", c_u32), ("bucket_bits", c_u32),
                ("cell_id_bytes", c_u32), ("srp_rechecked", c_u64),
                ("srp_exact", c_u64)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("mem_budget", c_u64), ("max_inflight", c_u32), ("max_batch", c_u32),
                ("max_queue", c_u32), ("persistent", c_u32), ("linger_ns", c_u64)]


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", c_u64), ("completed", c_u64), ("rejected", c_u64),
                ("batches", c_u64), ("queries", c_u64), ("wall_s", ctypes.c_double),
                ("qps", ctypes.c_double), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
                ("mean_batch", ctypes.c_double), ("peak_mem_bytes", c_u64)]


class Theory(ctypes.Structure):
    _fields_ = [("B", c_u32), ("R", c_u32), ("K", c_u32), ("L", c_u32), ("t", c_u32),
                ("conditions_met", c_u32), ("R_real", ctypes.c_double), ("p", ctypes.c_double),
                ("q", ctypes.c_double), ("one_minus_p", ctypes.c_double),
                ("gamma", ctypes.c_double), ("m_paper", ctypes.c_double),
                ("t_real", ctypes.c_double), ("t_over_m_low", ctypes.c_double),
                ("t_over_m_high", ctypes.c_double), ("alpha", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is not built; run `python -m paper_2106_11565_amd.build` "
                "(the HIP library is required: there is no CPU fallback)")
        # one HIP runtime per process: the device pointers and streams handed
        # to the library come from torch, so torch's runtime is loaded first
        # and the library binds to it (same soname)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        sig = {
            "flinng_build": (ctypes.c_int, [P(Params), P(Input), c_vp, P(c_vp)]),
            "flinng_build_text": (ctypes.c_int, [P(Params), P(Text), c_vp, P(c_vp)]),
            "flinng_query_text": (ctypes.c_int, [c_vp, P(Text), c_u32, c_vp, c_vp, c_u32, c_u32, c_vp]),
            "flinng_serve_submit_text": (ctypes.c_int, [c_vp, c_u32, P(Text), c_u32, c_vp, c_vp,
                                                        P(c_u64)]),
            "flinng_query": (ctypes.c_int, [c_vp, P(Input), c_u32, c_vp, c_vp, c_u32, c_u32, c_vp]),
            "flinng_query_codes": (ctypes.c_int, [c_vp, c_vp, c_u64, c_u32, c_vp, c_vp, c_u32, c_vp, c_vp]),
            "flinng_query_noalloc": (ctypes.c_int, [c_vp, P(Input), c_u32, c_vp, c_vp, c_u32, c_vp]),
            "flinng_query_threshold": (ctypes.c_int, [c_vp, P(Input), c_u32, c_u32, c_vp, c_vp, c_u32,
                                                      c_vp]),
            "flinng_theory_params": (ctypes.c_int, [c_u64, ctypes.c_double, ctypes.c_double,
                                                    ctypes.c_double, P(Theory)]),
            "flinng_index_free": (None, [c_vp]),
            "flinng_index_insert": (ctypes.c_int, [c_vp, P(Input), c_vp]),
            "flinng_index_get_info": (ctypes.c_int, [c_vp, P(IndexInfo)]),
            "flinng_last_error": (ctypes.c_char_p, []),
            "flinng_debug_hash": (ctypes.c_int, [c_vp, P(Input), c_vp, c_u32, c_vp]),
            "flinng_debug_counts": (ctypes.c_int, [c_vp, P(Input), c_vp, c_u32, c_vp]),
            "flinng_debug_projections": (ctypes.c_int, [c_vp, P(Input), c_vp, c_vp, c_u32, c_vp]),
            "flinng_index_export": (ctypes.c_int, [c_vp, c_vp, c_vp, c_vp, c_vp]),
            "flinng_serve_create": (ctypes.c_int, [P(c_vp), c_u32, P(ServeConfig), P(c_vp)]),
            "flinng_serve_submit": (ctypes.c_int, [c_vp, c_u32, P(Input), c_u32, P(c_u64)]),
            "flinng_serve_submit_to": (ctypes.c_int, [c_vp, c_u32, P(Input), c_u32, c_vp, c_vp,
                                                      P(c_u64)]),
            "flinng_serve_wait": (ctypes.c_int, [c_vp, c_u64, c_vp, c_vp, c_i64]),
            "flinng_serve_poll": (ctypes.c_int, [c_vp, c_u64]),
            "flinng_serve_stats_get": (ctypes.c_int, [c_vp, P(ServeStats)]),
            "flinng_serve_stats_reset": (ctypes.c_int, [c_vp]),
            "flinng_serve_destroy": (None, [c_vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc):
    if rc != OK:
        msg = lib().flinng_last_error()
        raise FlinngError(rc, msg.decode() if msg else "")
    return rc


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def make_input(data, family):
    """Marshal dense rows or (items, offsets) into an Input.  Returns (Input,
    keepalive).  numpy arrays are host inputs; CUDA torch tensors are device
    inputs (data_ptr)."""
    keep = []
    inp = Input()
    if family in (SRP_F32, SRP_BF16):
        want = np.float32 if family == SRP_F32 else np.uint16
        if _is_torch(data):
            assert data.is_cuda and data.dim() == 2 and data.is_contiguous()
            inp.values, inp.count, inp.on_device = data.data_ptr(), data.shape[0], 1
            keep.append(data)
        else:
            a = np.ascontiguousarray(data, dtype=want)
            assert a.ndim == 2
            inp.values, inp.count, inp.on_device = a.ctypes.data, a.shape[0], 0
            keep.append(a)
    else:
        items, offs = data
        want = np.uint64 if family == MINHASH_U64 else np.uint32
        if _is_torch(items) and not _is_torch(offs):
            # device items with host offsets (accepted by the server only)
            assert items.is_cuda
            of = np.ascontiguousarray(offs, dtype=np.uint64)
            inp.values, inp.offsets = items.data_ptr(), of.ctypes.data
            inp.count, inp.on_device = of.shape[0] - 1, 2
            keep += [items, of]
        elif _is_torch(items):
            assert items.is_cuda and offs.is_cuda
            inp.values, inp.offsets = items.data_ptr(), offs.data_ptr()
            inp.count, inp.on_device = offs.shape[0] - 1, 1
            keep += [items, offs]
        else:
            it = np.ascontiguousarray(items, dtype=want)
            of = np.ascontiguousarray(offs, dtype=np.uint64)
            if it.size == 0:
                it = np.zeros(1, dtype=want)
            inp.values, inp.offsets = it.ctypes.data, of.ctypes.data
            inp.count, inp.on_device = of.shape[0] - 1, 0
            keep += [it, of]
    return inp, keep


def make_text(seqs, gram, radix, key):
    """Marshal symbol sequences (symbols uint8, offsets) into a Text.  numpy
    arrays are host inputs; CUDA torch tensors are device inputs.  Returns
    (Text, keepalive)."""
    sym, offs = seqs
    t = Text(gram=gram, radix=radix, key=int(key) & (2**64 - 1), reserved=0)
    keep = []
    if _is_torch(sym):
        assert sym.is_cuda and offs.is_cuda
        t.symbols, t.offsets, t.count, t.on_device = sym.data_ptr(), offs.data_ptr(), offs.shape[0] - 1, 1
        keep += [sym, offs]
    else:
        s = np.ascontiguousarray(sym, dtype=np.uint8)
        o = np.ascontiguousarray(offs, dtype=np.uint64)
        if s.size == 0:
            s = np.zeros(1, dtype=np.uint8)
        t.symbols, t.offsets, t.count, t.on_device = s.ctypes.data, o.ctypes.data, o.shape[0] - 1, 0
        keep += [s, o]
    return t, keep


def current_stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
