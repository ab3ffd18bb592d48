"""Python binding of libhd, the C-ABI declared in include/hd.h.

Argument marshalling only: host arrays are numpy, device buffers are torch
tensors (PyTorch supplies device memory and HIP streams; every step of the
decode runs in the library's own kernels).  The functions keep the C names
without the ``hd_`` prefix.  When libhd.so is missing this module raises at
import time -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhd.so")

OK, ERR_ARG, ERR_INFEASIBLE, ERR_SYMBOL, ERR_CORRUPT, ERR_NOMEM, ERR_DEVICE, ERR_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6, -7
MODE_GAP, MODE_SELF_SYNC = 0, 1

# Header declarations (name -> (restype, argtypes)); the CPU test suite checks
# that this list, include/hd.h and the library's exports agree.
_vp, _u32, _u64, _sz = C.c_void_p, C.c_uint32, C.c_uint64, C.c_size_t
SIGNATURES = {
    "hd_build_codebook": (C.c_int, [_vp, _u32, _u32, _vp, _vp]),
    "hd_encode_ref": (C.c_int, [_vp, _u64, _vp, _vp, _u32, _u32, _vp, _vp, _u64, _vp, _u64, _vp, _u64, _vp]),
    "hd_table_create": (C.c_int, [_vp, _vp, _u32, _u32, _u32, _vp, C.POINTER(_vp)]),
    "hd_table_destroy": (None, [_vp]),
    "hd_table_lds_bytes": (_sz, [_vp]),
    "hd_decode_workspace_size": (C.c_int, [_vp, C.c_int, _vp, C.POINTER(_sz)]),
    "hd_decode": (C.c_int, [_vp, _vp, C.c_int, _vp, _vp, _sz, _vp]),
    "hd_decode_prepare": (C.c_int, [_vp, C.c_int, _vp, _vp, _sz, _vp]),
    "hd_decode_run": (C.c_int, [_vp, _vp, C.c_int, _vp, _vp, _sz, _vp]),
    "hd_decode_sync_points": (C.c_int, [_vp, _vp, _sz, _vp, _vp]),
    "hd_decode_batch_workspace_size": (C.c_int, [_vp, _u32, C.c_int, C.POINTER(_sz)]),
    "hd_decode_batch": (C.c_int, [_vp, _u32, _vp, C.c_int, _vp, _vp, _sz, _vp]),
    "hd_autotune": (C.c_int, [_vp, C.c_int, _vp, _vp, _sz, _vp, _vp, _vp]),
    "hd_decode_cr_classes_workspace_size": (C.c_int, [_vp, C.POINTER(_sz)]),
    "hd_decode_cr_classes": (C.c_int, [_vp, _vp, _vp, _sz, _vp, _vp]),
    "hd_decode_status": (C.c_int, [_vp, _vp]),
    "hd_decode_status_bits": (_u32, [_vp, _vp]),
    "hd_decode_noalloc": (C.c_int, [_vp, _vp, C.c_int, _vp, _vp, _vp]),
    "hd_lorenzo_workspace_size": (_sz, [_u32, _u32, _u32]),
    "hd_histogram": (C.c_int, [_vp, _u64, _u32, _vp, _vp]),
    "hd_codebook_workspace_size": (_sz, [_u32]),
    "hd_build_codebook_device": (C.c_int, [_vp, _u32, _u32, _vp, _vp, _vp, _sz, _vp]),
    "hd_encode_workspace_size": (_sz, [_u64, _u32, _vp]),
    "hd_encode_plan": (C.c_int, [_vp, _u64, _vp, _u32, _vp, _sz, _vp]),
    "hd_encode_bits": (C.c_int, [_vp, C.POINTER(_u64), _vp]),
    "hd_encode_write": (C.c_int, [_vp, _u64, _vp, _vp, _u32, _vp, _vp, _u64, _vp, _u64, _vp, _u64, _vp, _sz, _vp]),
    "hd_lorenzo_reconstruct": (C.c_int, [_vp, _u32, _u32, _u32, _u32, _vp, _vp, _u64, C.c_double, _vp, _vp, _vp,
                                         _sz, _vp]),
    "hd_stream_layout": (C.c_int, [_u64, _u64, _u32, _u32, _vp, _vp]),
    "hd_status_str": (C.c_char_p, [C.c_int]),
    "hd_server_create": (C.c_int, [_sz, _u32, _u32, C.POINTER(_vp)]),
    "hd_server_destroy": (None, [_vp]),
    "hd_server_submit": (C.c_int, [_vp, _vp, C.POINTER(_u64)]),
    "hd_server_poll": (C.c_int, [_vp, _vp, _u32, C.POINTER(_u32)]),
    "hd_server_result": (C.c_int, [_vp, _u64, C.POINTER(_vp), C.POINTER(C.c_int), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double)]),
    "hd_server_release": (C.c_int, [_vp, _u64]),
    "hd_server_stats": (C.c_int, [_vp, C.POINTER(_u64), C.POINTER(_u64), C.POINTER(_u64), C.POINTER(_u64),
                                  C.POINTER(_u64)]),
}


class HDError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_str(status)} ({status})")
        self.status = status


class Layout(C.Structure):
    _fields_ = [("subseq_bits", C.c_uint32), ("chunk_subseqs", C.c_uint32), ("symbol_bytes", C.c_uint32)]


class StreamInfo(C.Structure):
    _fields_ = [("n_symbols", C.c_uint64), ("n_bits", C.c_uint64), ("n_words", C.c_uint64),
                ("n_subseq", C.c_uint64), ("n_chunks", C.c_uint64), ("subseq_bits", C.c_uint32),
                ("chunk_subseqs", C.c_uint32), ("alphabet_size", C.c_uint32), ("max_len", C.c_uint32),
                ("symbol_bytes", C.c_uint32), ("reserved", C.c_uint32)]


class Tune(C.Structure):
    _fields_ = [("waves_per_group", C.c_uint32), ("stage_symbols", C.c_uint32),
                ("groups_per_cu", C.c_uint32), ("reserved", C.c_uint32)]


class CrClasses(C.Structure):
    _fields_ = [("t_high", C.c_uint32), ("launches", C.c_uint32), ("classify_us", C.c_double),
                ("tiles", C.c_uint32 * 17),
                ("stage_symbols", C.c_uint32 * 17), ("waves_per_group", C.c_uint32 * 17)]


class DStream(C.Structure):
    _fields_ = [("words", C.c_void_p), ("gap", C.c_void_p), ("chunk_offsets", C.c_void_p),
                ("info", StreamInfo), ("table", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2201_09118_amd.build` "
                              "(hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


lib()   # fail loudly at import when the extension is missing


def status_str(st: int) -> str:
    return lib().hd_status_str(int(st)).decode()


def _check(st, what):
    if st != OK:
        raise HDError(st, what)


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _dev_ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _out_ptr(ds, out):
    """Device pointer of a decode output tensor, checked against the stream's
    symbol width and length (a short or narrower tensor would be overrun)."""
    w = int(ds.info.symbol_bytes) or 2
    n = int(ds.info.n_symbols)
    if out is None:
        if n:
            raise ValueError("decode output is None")
        return None
    if out.element_size() != w or out.numel() < n or not out.is_contiguous():
        raise ValueError(f"decode output must be a contiguous tensor of >= {n} elements of {w} bytes")
    return _dev_ptr(out)


def _stream_handle(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


# ----------------------------------------------------------------- host ---

def build_codebook(hist: np.ndarray, L: int):
    """hist uint64[A] -> (lengths uint8[A], codes uint32[A])."""
    hist = np.ascontiguousarray(hist, dtype=np.uint64)
    A = hist.size
    ln = np.zeros(A, np.uint8)
    cd = np.zeros(A, np.uint32)
    _check(lib().hd_build_codebook(_np_ptr(hist), A, L, _np_ptr(ln), _np_ptr(cd)), "hd_build_codebook")
    return ln, cd


@dataclass
class HostStream:
    words: np.ndarray
    gap: np.ndarray
    chunk_offsets: np.ndarray      # uint64[n_chunks + 1]
    info: StreamInfo

    @property
    def n_symbols(self):
        return int(self.info.n_symbols)

    @property
    def n_bits(self):
        return int(self.info.n_bits)


_WIDTH_OF = {np.dtype(np.uint8): 1, np.dtype(np.uint16): 2, np.dtype(np.uint32): 4}


def encode_ref(syms: np.ndarray, lengths: np.ndarray, codes: np.ndarray, L: int,
               S: int = 128, Cc: int = 32) -> HostStream:
    """hd_encode_ref; uint8 and uint32 symbol arrays keep their width, others are taken as uint16."""
    syms = np.asarray(syms)
    if syms.dtype not in _WIDTH_OF:
        syms = syms.astype(np.uint16)
    syms = np.ascontiguousarray(syms)
    lengths = np.ascontiguousarray(lengths, dtype=np.uint8)
    codes = np.ascontiguousarray(codes, dtype=np.uint32)
    lay = Layout(S, Cc, _WIDTH_OF[syms.dtype])
    info = StreamInfo()
    L_ = lib()
    _check(L_.hd_encode_ref(_np_ptr(syms), syms.size, _np_ptr(lengths), _np_ptr(codes), lengths.size, L,
                            C.byref(lay), None, 0, None, 0, None, 0, C.byref(info)), "hd_encode_ref(size)")
    words = np.zeros(info.n_words, np.uint32)
    gap = np.zeros(info.n_subseq, np.uint8)
    cc = np.zeros(info.n_chunks + 1, np.uint64)
    _check(L_.hd_encode_ref(_np_ptr(syms), syms.size, _np_ptr(lengths), _np_ptr(codes), lengths.size, L,
                            C.byref(lay), _np_ptr(words), words.size, _np_ptr(gap), gap.size, _np_ptr(cc),
                            cc.size, C.byref(info)), "hd_encode_ref")
    return HostStream(words, gap, cc, info)


# --------------------------------------------------------------- device ---

class Table:
    """Device decode table (hd_table_create / hd_table_destroy)."""

    def __init__(self, lengths: np.ndarray, codes: np.ndarray, L: int, lut_bits: int = 0, stream=None):
        lengths = np.ascontiguousarray(lengths, dtype=np.uint8)
        codes = np.ascontiguousarray(codes, dtype=np.uint32)
        self._h = C.c_void_p()
        _check(lib().hd_table_create(_np_ptr(lengths), _np_ptr(codes), lengths.size, L, lut_bits,
                                     _stream_handle(stream), C.byref(self._h)), "hd_table_create")
        self.A, self.L = lengths.size, L

    @property
    def handle(self):
        return self._h

    @property
    def lds_bytes(self) -> int:
        return int(lib().hd_table_lds_bytes(self._h))

    def close(self):
        if self._h:
            lib().hd_table_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class DeviceStream:
    """A stream resident in device memory (torch tensors) plus its table."""
    words: object          # torch int32 tensor (bit pattern of the uint32 units)
    gap: object            # torch uint8 tensor or None
    chunk_offsets: object  # torch int64 tensor (n_chunks + 1 entries) or None
    info: StreamInfo
    table: Table

    @classmethod
    def from_host(cls, hs: HostStream, table: Table, device="cuda", with_gap=True):
        import torch
        w = torch.from_numpy(hs.words.view(np.int32)).to(device)
        g = torch.from_numpy(hs.gap).to(device) if with_gap else None
        c = torch.from_numpy(hs.chunk_offsets.view(np.int64)).to(device) if with_gap else None
        info = StreamInfo()
        C.pointer(info)[0] = hs.info
        return cls(w, g, c, info, table)

    def as_c(self) -> DStream:
        d = DStream()
        d.words = self.words.data_ptr() if self.words is not None and self.words.numel() else None
        d.gap = self.gap.data_ptr() if self.gap is not None and self.gap.numel() else None
        d.chunk_offsets = (self.chunk_offsets.data_ptr()
                           if self.chunk_offsets is not None and self.chunk_offsets.numel() else None)
        d.info = self.info
        d.table = self.table.handle
        return d

    @property
    def n_symbols(self):
        return int(self.info.n_symbols)


def _tune_ptr(tune):
    if tune is None:
        return None
    if isinstance(tune, dict):
        tune = Tune(tune.get("waves_per_group", 0), tune.get("stage_symbols", 0),
                    tune.get("groups_per_cu", 0), 0)
    return C.byref(tune)


def decode_workspace_size(ds: DeviceStream, mode: int = MODE_GAP, tune=None) -> int:
    d = ds.as_c()
    n = C.c_size_t()
    _check(lib().hd_decode_workspace_size(C.byref(d), mode, _tune_ptr(tune), C.byref(n)),
           "hd_decode_workspace_size")
    return int(n.value)


def alloc_workspace(nbytes: int, device="cuda"):
    import torch
    return torch.empty(max(256, nbytes), dtype=torch.uint8, device=device)


def decode(ds: DeviceStream, out, mode: int = MODE_GAP, tune=None, workspace=None, stream=None):
    """Enqueues hd_decode; returns the workspace (for decode_status)."""
    d = ds.as_c()
    if workspace is None:
        workspace = alloc_workspace(decode_workspace_size(ds, mode, tune), out.device)
    _check(lib().hd_decode(C.byref(d), _out_ptr(ds, out), mode, _tune_ptr(tune), _dev_ptr(workspace),
                           workspace.numel(), _stream_handle(stream)), "hd_decode")
    return workspace


def decode_prepare(ds: DeviceStream, workspace, mode: int = MODE_GAP, tune=None, stream=None):
    d = ds.as_c()
    _check(lib().hd_decode_prepare(C.byref(d), mode, _tune_ptr(tune), _dev_ptr(workspace), workspace.numel(),
                                   _stream_handle(stream)), "hd_decode_prepare")


def decode_run(ds: DeviceStream, out, workspace, mode: int = MODE_GAP, tune=None, stream=None):
    d = ds.as_c()
    _check(lib().hd_decode_run(C.byref(d), _out_ptr(ds, out), mode, _tune_ptr(tune), _dev_ptr(workspace),
                               workspace.numel(), _stream_handle(stream)), "hd_decode_run")


def decode_sync_points(ds: DeviceStream, workspace, gap_out, stream=None):
    """Copies the sync points found by a self-sync decode into gap_out (uint8 device tensor)."""
    d = ds.as_c()
    _check(lib().hd_decode_sync_points(C.byref(d), _dev_ptr(workspace), workspace.numel(), _dev_ptr(gap_out),
                                       _stream_handle(stream)), "hd_decode_sync_points")


def decode_batch_workspace_size(streams, mode: int = MODE_GAP) -> int:
    arr = (DStream * len(streams))(*[s.as_c() for s in streams])
    n = C.c_size_t()
    _check(lib().hd_decode_batch_workspace_size(arr, len(streams), mode, C.byref(n)),
           "hd_decode_batch_workspace_size")
    return int(n.value)


def decode_batch(streams, outs, mode: int = MODE_GAP, tunes=None, workspace=None, stream=None):
    """Enqueues hd_decode_batch; tunes is None or one Tune/dict per stream."""
    arr = (DStream * len(streams))(*[s.as_c() for s in streams])
    optrs = (C.c_void_p * len(outs))(*[o.data_ptr() if o.numel() else None for o in outs])
    tptr = None
    if tunes is not None:
        ts = [t if isinstance(t, Tune) else Tune(t.get("waves_per_group", 0), t.get("stage_symbols", 0),
                                                  t.get("groups_per_cu", 0), 0) for t in tunes]
        tptr = (Tune * len(ts))(*ts)
    if workspace is None:
        workspace = alloc_workspace(decode_batch_workspace_size(streams, mode), outs[0].device)
    _check(lib().hd_decode_batch(arr, len(streams), optrs, mode, tptr, _dev_ptr(workspace),
                                 workspace.numel(), _stream_handle(stream)), "hd_decode_batch")
    return workspace


def autotune(ds: DeviceStream, out, workspace=None, mode: int = MODE_GAP, stream=None):
    """hd_autotune on a sample stream -> (Tune, milliseconds of the fastest decode_run)."""
    d = ds.as_c()
    if workspace is None:
        workspace = alloc_workspace(decode_workspace_size(ds, mode), out.device)
    best = Tune()
    ms = C.c_float()
    _check(lib().hd_autotune(C.byref(d), mode, _out_ptr(ds, out), _dev_ptr(workspace), workspace.numel(),
                             _stream_handle(stream), C.byref(best), C.byref(ms)), "hd_autotune")
    return best, float(ms.value)


def decode_cr_classes(ds: DeviceStream, out, workspace=None, stream=None):
    """hd_decode_cr_classes (the paper's Algorithm 2 as an ablation); returns
    (workspace, report dict)."""
    d = ds.as_c()
    if workspace is None:
        n = C.c_size_t()
        _check(lib().hd_decode_cr_classes_workspace_size(C.byref(d), C.byref(n)),
               "hd_decode_cr_classes_workspace_size")
        workspace = alloc_workspace(int(n.value), out.device)
    rep = CrClasses()
    _check(lib().hd_decode_cr_classes(C.byref(d), _dev_ptr(out), _dev_ptr(workspace), workspace.numel(),
                                      _stream_handle(stream), C.byref(rep)), "hd_decode_cr_classes")
    used = [c for c in range(17) if rep.tiles[c]]
    return workspace, {"t_high": rep.t_high, "launches": rep.launches, "classify_us": rep.classify_us,
                       "classes": {c + 1: {"tiles": rep.tiles[c], "stage_symbols": rep.stage_symbols[c],
                                           "waves_per_group": rep.waves_per_group[c]} for c in used}}


def histogram(syms, A: int, hist=None, stream=None):
    """hd_histogram of a uint16-sized device tensor into an int64 device tensor of A bins."""
    import torch
    if hist is None:
        hist = torch.empty(A, dtype=torch.int64, device=syms.device)
    _check(lib().hd_histogram(_dev_ptr(syms) if syms.numel() else None, syms.numel(), A, _dev_ptr(hist),
                              _stream_handle(stream)), "hd_histogram")
    return hist


def build_codebook_device(hist, L: int, lengths=None, codes=None, workspace=None, stream=None):
    """hd_build_codebook_device: (lengths uint8[A], codes int32[A], workspace) device tensors from an
    int64 device histogram of A bins; the status bits are read with decode_status_bits(workspace)."""
    import torch
    A = hist.numel()
    dev = hist.device
    if lengths is None:
        lengths = torch.empty(A, dtype=torch.uint8, device=dev)
    if codes is None:
        codes = torch.empty(A, dtype=torch.int32, device=dev)
    if lengths.numel() < A or codes.numel() < A or lengths.element_size() != 1 or codes.element_size() != 4:
        raise ValueError("lengths / codes must hold A uint8 / 32-bit entries")
    if workspace is None:
        nb = int(lib().hd_codebook_workspace_size(L))
        if nb == 0:
            raise HDError(ERR_ARG, "hd_codebook_workspace_size")
        workspace = alloc_workspace(nb, dev)
    _check(lib().hd_build_codebook_device(_dev_ptr(hist), A, L, _dev_ptr(lengths), _dev_ptr(codes),
                                          _dev_ptr(workspace), workspace.numel(), _stream_handle(stream)),
           "hd_build_codebook_device")
    return lengths, codes, workspace


@dataclass
class DeviceEncoded:
    words: object
    gap: object
    chunk_offsets: object
    n_symbols: int
    n_bits: int
    S: int
    C: int


def encode_device(syms, lengths, codes, L: int, S: int = 128, chunk: int = 32, workspace=None, stream=None):
    """Device encode of a uint16-sized device tensor with a codebook given as
    device tensors (lengths uint8[A], codes int32[A]): plan, read the total
    bits (one host wait), allocate, write.  Returns a DeviceEncoded."""
    import torch
    n = syms.numel()
    A = lengths.numel()
    lay = Layout(S, chunk)
    if workspace is None:
        nb = lib().hd_encode_workspace_size(n, L, C.byref(lay))
        if nb == 0:
            raise HDError(ERR_ARG, "hd_encode_workspace_size")
        workspace = alloc_workspace(nb, syms.device)
    sp = _dev_ptr(syms) if n else None
    _check(lib().hd_encode_plan(sp, n, _dev_ptr(lengths), A, _dev_ptr(workspace), workspace.numel(),
                                _stream_handle(stream)), "hd_encode_plan")
    bits = C.c_uint64()
    _check(lib().hd_encode_bits(_dev_ptr(workspace), C.byref(bits), _stream_handle(stream)), "hd_encode_bits")
    B = int(bits.value)
    info = stream_layout(n, B, A, L, S, chunk)
    K, M, NW = int(info.n_subseq), int(info.n_chunks), int(info.n_words)
    words = torch.empty(NW, dtype=torch.int32, device=syms.device)
    gap = torch.empty(max(K, 1), dtype=torch.uint8, device=syms.device)
    cc = torch.empty(M + 1, dtype=torch.int64, device=syms.device)
    _check(lib().hd_encode_write(sp, n, _dev_ptr(lengths), _dev_ptr(codes), A, C.byref(lay), _dev_ptr(words), NW,
                                 _dev_ptr(gap), K, _dev_ptr(cc), M, _dev_ptr(workspace), workspace.numel(),
                                 _stream_handle(stream)), "hd_encode_write")
    return DeviceEncoded(words, gap[:K], cc, n, B, S, chunk), workspace


def stream_layout(n_symbols: int, n_bits: int, A: int, L: int, S: int = 128, chunk: int = 32) -> StreamInfo:
    """hd_stream_layout: the stream-format sizes (StreamInfo) of n_symbols coded in n_bits bits."""
    info = StreamInfo()
    lay = Layout(S, chunk)
    _check(lib().hd_stream_layout(n_symbols, n_bits, A, L, C.byref(lay), C.byref(info)), "hd_stream_layout")
    return info


def lorenzo_workspace_size(shape) -> int:
    ni, nj, nk = (int(v) for v in shape)
    return int(lib().hd_lorenzo_workspace_size(ni, nj, nk))


def lorenzo_reconstruct(codes, shape, radius: int, outlier_idx, outlier_val, eb: float, out, q_out=None,
                        workspace=None, stream=None):
    """Enqueues hd_lorenzo_reconstruct.  codes: uint16-sized device tensor (int16
    or uint16) of prod(shape) codes; outlier_idx: int64 device tensor of ascending
    flat indices (or None); outlier_val: int32 device tensor; out: float32 device
    tensor; q_out: optional int32 device tensor.  Returns the workspace."""
    ni, nj, nk = (int(v) for v in shape)
    n_out = 0 if outlier_idx is None else int(outlier_idx.numel())
    if workspace is None:
        workspace = alloc_workspace(lorenzo_workspace_size(shape), out.device)
    _check(lib().hd_lorenzo_reconstruct(_dev_ptr(codes), ni, nj, nk, int(radius),
                                        _dev_ptr(outlier_idx) if n_out else None,
                                        _dev_ptr(outlier_val) if n_out else None, n_out, float(eb),
                                        _dev_ptr(out), _dev_ptr(q_out), _dev_ptr(workspace), workspace.numel(),
                                        _stream_handle(stream)), "hd_lorenzo_reconstruct")
    return workspace


def decode_status(workspace, stream=None) -> int:
    return int(lib().hd_decode_status(_dev_ptr(workspace), _stream_handle(stream)))


def decode_status_bits(workspace, stream=None) -> int:
    return int(lib().hd_decode_status_bits(_dev_ptr(workspace), _stream_handle(stream)))


NOALLOC_SCRATCH_BYTES = 32 << 20   # HD_NOALLOC_SCRATCH_BYTES


def decode_noalloc(ds: DeviceStream, out, status, mode: int = MODE_GAP, tune=None, stream=None):
    """Enqueues hd_decode_noalloc; status is a one-element int32/uint32 device tensor that
    receives the raw status bits."""
    d = ds.as_c()
    _check(lib().hd_decode_noalloc(C.byref(d), _out_ptr(ds, out), mode, _tune_ptr(tune), _dev_ptr(status),
                                   _stream_handle(stream)), "hd_decode_noalloc")


class Server:
    """hd_server_*: continuous-batching decode server over an HBM budget."""

    def __init__(self, hbm_budget: int, n_streams: int = 4, max_batch: int = 64):
        self._h = C.c_void_p()
        _check(lib().hd_server_create(hbm_budget, n_streams, max_batch, C.byref(self._h)), "hd_server_create")
        self._keep = {}

    def submit(self, ds: DeviceStream) -> int:
        d = ds.as_c()
        rid = C.c_uint64()
        _check(lib().hd_server_submit(self._h, C.byref(d), C.byref(rid)), "hd_server_submit")
        self._keep[rid.value] = ds          # buffers and table stay alive until completion
        return rid.value

    def poll(self, cap: int = 4096):
        ids = (C.c_uint64 * cap)()
        n = C.c_uint32()
        _check(lib().hd_server_poll(self._h, ids, cap, C.byref(n)), "hd_server_poll")
        return [ids[i] for i in range(n.value)]

    def result(self, rid: int):
        """(device pointer, status, t_submit, t_done) of a completed request."""
        p = C.c_void_p()
        st = C.c_int()
        t0 = C.c_double()
        t1 = C.c_double()
        _check(lib().hd_server_result(self._h, rid, C.byref(p), C.byref(st), C.byref(t0), C.byref(t1)),
               "hd_server_result")
        return p.value, st.value, t0.value, t1.value

    def release(self, rid: int):
        _check(lib().hd_server_release(self._h, rid), "hd_server_release")
        self._keep.pop(rid, None)

    def stats(self):
        v = [C.c_uint64() for _ in range(5)]
        _check(lib().hd_server_stats(self._h, *[C.byref(x) for x in v]), "hd_server_stats")
        return dict(zip(("batches", "done", "queued", "arena_used", "arena_peak"), (x.value for x in v)))

    def close(self):
        if self._h:
            lib().hd_server_destroy(self._h)
            self._h = C.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
