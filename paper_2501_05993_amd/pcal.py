"""ctypes binding of libpcal (include/pcal.h): argument marshalling only.

Every step of the extraction runs in the library's HIP kernels; this module
passes device pointers, sizes and stream handles through.  PyTorch provides
device memory and streams.  torch is imported before the library is loaded
so that libpcal resolves ``libamdhip64.so.7`` to the HIP runtime torch already
loaded (one runtime per process: torch's stream handles are valid in it).

There is no CPU fallback: if ``libpcal.so`` is missing, loading fails.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np
import torch  # noqa: F401  (must precede loading libpcal, see module docstring)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpcal.so")

OK, EINVAL, ENOMEM, EHIP, EAGAIN, ESTATE, ENOTSUP = 0, -1, -2, -3, -4, -5, -6
METHOD_AUTO, METHOD_PERIOD_FOLD, METHOD_LUT, METHOD_OSC, METHOD_CFO, METHOD_MCO, METHOD_DFR_EF = 0, 1, 2, 3, 4, 5, 6
RESET_OVERLAP = 2  # pcal_results_async: finish the integration, take the next in the other lane (two streams)
PREC_F64, PREC_MIXED, PREC_F32, PREC_F16, PREC_Q17 = 0, 1, 2, 3, 4

_i64 = ctypes.c_int64


class Info(ctypes.Structure):
    _fields_ = [(n, _i64) for n in (
        "ntones", "rotator_period", "joint_period", "fold_period", "method", "precision",
        "samples_total", "samples_integ", "block_threads", "row_vectors", "col_tiles",
        "lds_positions", "device_bytes", "period_vectors", "tile_vectors", "target_blocks")]

    def as_dict(self) -> dict:
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class Launch(ctypes.Structure):
    _fields_ = [(n, _i64) for n in (
        "grid", "threads", "lds_bytes", "head_bytes", "nvec", "tail_bytes", "rows_total",
        "rows_per_group", "q0", "head_q", "tail_q", "groups_per_wg", "extra_groups", "odd_start")]

    def as_dict(self) -> dict:
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class PcalError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__("%s failed: %s (%d)%s" % (what, strerror(code), code,
                                                   (" -- " + last_error()) if code == EHIP else ""))


_lib = None

_SIGS = {
    "pcal_create": ([_i64, _i64, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "pcal_create_ex": ([_i64, _i64, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                        ctypes.c_void_p], ctypes.c_int),
    "pcal_extract": ([ctypes.c_void_p, ctypes.c_void_p, _i64, ctypes.c_void_p], ctypes.c_int),
    "pcal_extract_timed": ([ctypes.c_void_p, ctypes.c_void_p, _i64, ctypes.c_void_p, ctypes.c_void_p,
                            ctypes.c_void_p], ctypes.c_int),
    "pcal_results": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "pcal_spectrum": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "pcal_results_async": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int], ctypes.c_int),
    "pcal_sync": ([ctypes.c_void_p], ctypes.c_int),
    "pcal_flush": ([ctypes.c_void_p], ctypes.c_int),
    "pcal_bins": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "pcal_pulse": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
                   ctypes.c_int),
    "pcal_bandpass": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "pcal_refine": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "pcal_reset": ([ctypes.c_void_p], ctypes.c_int),
    "pcal_destroy": ([ctypes.c_void_p], ctypes.c_int),
    "pcal_num_tones": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "pcal_info": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "pcal_plan": ([_i64, _i64, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p],
                  ctypes.c_int),
    "pcal_plan_launch": ([_i64, _i64, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, _i64,
                          _i64, ctypes.c_void_p], ctypes.c_int),
    "pcal_batch_create": ([ctypes.c_int, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "pcal_batch_add": ([ctypes.c_void_p, _i64, _i64, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "pcal_batch_handle": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "pcal_batch_extract": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                            ctypes.c_void_p], ctypes.c_int),
    "pcal_batch_results": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                            ctypes.c_void_p], ctypes.c_int),
    "pcal_batch_spectra": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
                           ctypes.c_int),
    "pcal_batch_reset": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "pcal_batch_size": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "pcal_batch_destroy": ([ctypes.c_void_p], ctypes.c_int),
    "pcal_server_create": ([_i64, ctypes.c_int, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "pcal_server_open": ([ctypes.c_void_p, _i64, _i64, _i64, ctypes.c_int, ctypes.c_int, _i64, ctypes.c_void_p],
                         ctypes.c_int),
    "pcal_server_close": ([ctypes.c_void_p, ctypes.c_int], ctypes.c_int),
    "pcal_server_submit": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
                           ctypes.c_int),
    "pcal_server_step": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "pcal_server_poll": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
                         ctypes.c_int),
    "pcal_server_result": ([ctypes.c_void_p, ctypes.c_int, _i64, ctypes.c_void_p, ctypes.c_void_p,
                            ctypes.c_void_p], ctypes.c_int),
    "pcal_server_spectrum": ([ctypes.c_void_p, ctypes.c_int, _i64, ctypes.c_void_p, ctypes.c_void_p],
                             ctypes.c_int),
    "pcal_server_stats": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "pcal_server_destroy": ([ctypes.c_void_p], ctypes.c_int),
    "pcal_server_start": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "pcal_server_stop": ([ctypes.c_void_p], ctypes.c_int),
    "pcal_server_loop_stats": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int], ctypes.c_int),
    "pcal_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "pcal_read_probe": ([ctypes.c_void_p, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                         ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "pcal_last_error": ([], ctypes.c_char_p),
    "pcal_extract_noalloc": ([_i64, _i64, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, _i64, ctypes.c_void_p,
                              ctypes.c_void_p], ctypes.c_int),
}


def lib():
    """The loaded libpcal (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libpcal.so is not built (%s); run paper_2501_05993_amd/build.py" % LIB_PATH)
        l = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(l, name)
            f.argtypes = args
            f.restype = res
        _lib = l
    return _lib


def strerror(code: int) -> str:
    return lib().pcal_strerror(code).decode()


def last_error() -> str:
    return lib().pcal_last_error().decode()


def _check(code: int, what: str) -> None:
    if code != OK:
        raise PcalError(code, what)


def read_probe(data, out, blocks: int, threads: int, stream=None, events=None) -> None:
    """Streaming-read reference pass over a contiguous device tensor (pcal_read_probe).

    out: int64 device tensor of at least blocks * threads / 64 elements (the
    XOR of the 64-bit words each wave read); events: optional (start, stop)
    torch.cuda.Event pair, already recorded once, stamped with the kernel's own
    start and end."""
    if not (isinstance(data, torch.Tensor) and data.is_cuda and data.is_contiguous()):
        raise ValueError("read_probe needs a contiguous device tensor")
    if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.int64
            and out.numel() >= blocks * threads // 64):
        raise ValueError("out needs blocks * threads / 64 int64 elements on the device")
    e0, e1 = (None, None) if events is None else \
        (ctypes.c_void_p(int(e.cuda_event)) if e is not None else None for e in events)
    _check(lib().pcal_read_probe(ctypes.c_void_p(data.data_ptr()), data.numel() * data.element_size(), blocks,
                                 threads, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(_stream_handle(stream)),
                                 e0, e1), "pcal_read_probe")


def extract_noalloc(fs: int, f_comb: int, f_offset: int, nbits: int, data, nsamples: int, out,
                    sideband: int = 1, stream=None) -> None:
    """One integration without any allocation (pcal_extract_noalloc): data is a device tensor (or a raw
    device address) of packed samples, out a float64 device tensor of 4N + 1 elements receiving
    amp, phase, Re C, Im C and the delay.  Asynchronous on stream."""
    N = fs // f_comb if f_comb > 0 else 0
    if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.float64 and out.is_contiguous()
            and out.numel() >= 4 * N + 1):
        raise ValueError("out needs 4N + 1 contiguous float64 elements on the device")
    ptr = data.data_ptr() if isinstance(data, torch.Tensor) else int(data)
    if isinstance(data, torch.Tensor) and nsamples * nbits > data.numel() * data.element_size() * 8:
        raise ValueError("tensor holds fewer than nsamples samples")
    _check(lib().pcal_extract_noalloc(fs, f_comb, f_offset, nbits, sideband, ctypes.c_void_p(ptr), nsamples,
                                      ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(_stream_handle(stream))),
           "pcal_extract_noalloc")


def plan(fs: int, f_comb: int, f_offset: int, nbits: int, method: int = METHOD_AUTO,
         precision: int = PREC_F64) -> dict:
    info = Info()
    _check(lib().pcal_plan(fs, f_comb, f_offset, nbits, method, precision, ctypes.byref(info)), "pcal_plan")
    return info.as_dict()


def plan_launch(fs: int, f_comb: int, f_offset: int, nbits: int, nsamples: int, addr_low: int = 0,
                samples_before: int = 0, method: int = METHOD_AUTO, precision: int = PREC_F64) -> dict:
    out = Launch()
    _check(lib().pcal_plan_launch(fs, f_comb, f_offset, nbits, method, precision, addr_low, samples_before,
                                  nsamples, ctypes.byref(out)), "pcal_plan_launch")
    return out.as_dict()


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class PCal:
    """One stream's extraction state (a pcal_t handle)."""

    def __init__(self, fs: int, f_comb: int, f_offset: int, nbits: int, sideband: int = 1,
                 method: int = METHOD_AUTO, precision: int = PREC_F64):
        self._h = ctypes.c_void_p()
        _check(lib().pcal_create_ex(fs, f_comb, f_offset, nbits, sideband, method, precision,
                                    ctypes.byref(self._h)), "pcal_create")
        self.fs, self.f_comb, self.f_offset, self.nbits, self.sideband = fs, f_comb, f_offset, nbits, sideband
        self.ntones = fs // f_comb

    @property
    def handle(self) -> int:
        return self._h.value

    def extract(self, data, nsamples: Optional[int] = None, stream=None, byte_offset: int = 0,
                events=None) -> None:
        """Enqueue packed samples held in a device tensor (or at a raw device address).

        events: optional (start, stop) torch.cuda.Event pair, already recorded once
        (so that they exist), which pcal_extract_timed stamps with the kernel's
        own start and end."""
        if isinstance(data, torch.Tensor):
            if not data.is_cuda:
                raise ValueError("extract needs device memory")
            if not data.is_contiguous():
                raise ValueError("extract needs a contiguous tensor")
            ptr = data.data_ptr() + byte_offset
            avail = data.numel() * data.element_size() - byte_offset
            if nsamples is None:
                nsamples = avail * (8 // self.nbits)
            if nsamples * self.nbits > avail * 8:
                raise ValueError("tensor holds fewer than nsamples samples")
        else:
            ptr = int(data) + byte_offset
            if nsamples is None:
                raise ValueError("nsamples is required with a raw pointer")
        if events is None:
            _check(lib().pcal_extract(self._h, ctypes.c_void_p(ptr), nsamples,
                                      ctypes.c_void_p(_stream_handle(stream))), "pcal_extract")
        else:
            e0, e1 = (ctypes.c_void_p(int(e.cuda_event)) if e is not None else None for e in events)
            _check(lib().pcal_extract_timed(self._h, ctypes.c_void_p(ptr), nsamples,
                                            ctypes.c_void_p(_stream_handle(stream)), e0, e1),
                   "pcal_extract_timed")

    def results(self) -> Tuple[np.ndarray, np.ndarray, float]:
        amp = np.zeros(self.ntones)
        phase = np.zeros(self.ntones)
        delay = np.zeros(1)
        _check(lib().pcal_results(self._h, amp.ctypes.data, phase.ctypes.data, delay.ctypes.data),
               "pcal_results")
        return amp, phase, float(delay[0])

    def results_async(self, host_out, reset=False) -> None:
        """Enqueue finalize + copy into host_out (4N+1 doubles, ideally pinned); see pcal_results_async.
        reset: False, True, or RESET_OVERLAP (pipelined integrations on two streams in turn)."""
        ptr = host_out.data_ptr() if isinstance(host_out, torch.Tensor) else host_out.ctypes.data
        flag = RESET_OVERLAP if reset == RESET_OVERLAP else (1 if reset else 0)
        _check(lib().pcal_results_async(self._h, ctypes.c_void_p(ptr), flag), "pcal_results_async")

    def sync(self) -> None:
        _check(lib().pcal_sync(self._h), "pcal_sync")

    def flush(self) -> None:
        """Enqueue a pending finalize now (non-blocking); see pcal_flush."""
        _check(lib().pcal_flush(self._h), "pcal_flush")

    def spectrum(self) -> np.ndarray:
        re = np.zeros(self.ntones)
        im = np.zeros(self.ntones)
        _check(lib().pcal_spectrum(self._h, re.ctypes.data, im.ctypes.data), "pcal_spectrum")
        return re + 1j * im

    def bins(self, integer: bool = False):
        re = np.zeros(self.ntones)
        im = np.zeros(self.ntones)
        ib = np.zeros(self.ntones, dtype=np.int64) if integer else None
        _check(lib().pcal_bins(self._h, re.ctypes.data, im.ctypes.data, ib.ctypes.data if integer else None),
               "pcal_bins")
        return (re + 1j * im, ib) if integer else re + 1j * im

    def pulse(self):
        """(P[b] complex [N], delay_s, peak_bin, offset_bins, peak_power) of the current integration."""
        re = np.zeros(self.ntones)
        im = np.zeros(self.ntones)
        delay = ctypes.c_double()
        peak = np.zeros(3)
        _check(lib().pcal_pulse(self._h, re.ctypes.data, im.ctypes.data, ctypes.byref(delay), peak.ctypes.data),
               "pcal_pulse")
        return re + 1j * im, delay.value, int(peak[0]), float(peak[1]), float(peak[2])

    def bandpass(self):
        """(amp[N], phase[N] corrected for the pulse's group delay, that delay in s)."""
        amp = np.zeros(self.ntones)
        ph = np.zeros(self.ntones)
        delay = ctypes.c_double()
        _check(lib().pcal_bandpass(self._h, amp.ctypes.data, ph.ctypes.data, ctypes.byref(delay)), "pcal_bandpass")
        return amp, ph, delay.value

    def refine(self, iters: int):
        """(delays[iters + 1] in s, intercept in rad, rms residual in rad) of the multi-pass refinement."""
        d = np.zeros(iters + 1)
        r = np.zeros(2)
        _check(lib().pcal_refine(self._h, iters, d.ctypes.data, r.ctypes.data), "pcal_refine")
        return d, float(r[0]), float(r[1])

    def reset(self) -> None:
        _check(lib().pcal_reset(self._h), "pcal_reset")

    def info(self) -> dict:
        info = Info()
        _check(lib().pcal_info(self._h, ctypes.byref(info)), "pcal_info")
        return info.as_dict()

    def close(self) -> None:
        if self._h and self._h.value:
            _check(lib().pcal_destroy(self._h), "pcal_destroy")
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class PCalBatch:
    """Many streams extracted by one launch (pcal_batch_*)."""

    def __init__(self, max_streams: int, precision: int = PREC_F64):
        self._b = ctypes.c_void_p()
        _check(lib().pcal_batch_create(max_streams, precision, ctypes.byref(self._b)), "pcal_batch_create")
        self.ntones = []

    def add(self, fs: int, f_comb: int, f_offset: int, nbits: int, sideband: int = 1) -> int:
        i = ctypes.c_int()
        _check(lib().pcal_batch_add(self._b, fs, f_comb, f_offset, nbits, sideband, ctypes.byref(i)),
               "pcal_batch_add")
        self.ntones.append(fs // f_comb)
        return i.value

    def member_info(self, i: int) -> dict:
        h = ctypes.c_void_p()
        _check(lib().pcal_batch_handle(self._b, i, ctypes.byref(h)), "pcal_batch_handle")
        info = Info()
        _check(lib().pcal_info(h, ctypes.byref(info)), "pcal_info")
        return info.as_dict()

    @staticmethod
    def _ids(ids):
        return np.ascontiguousarray(np.asarray(ids, dtype=np.int32))

    def extract(self, ids, datas, nsamples, stream=None) -> None:
        """datas: device tensors (or raw addresses); nsamples: samples per chunk."""
        idv = self._ids(ids)
        ptrs = np.ascontiguousarray(np.asarray([d.data_ptr() if isinstance(d, torch.Tensor) else int(d)
                                                for d in datas], dtype=np.uint64))
        ns = np.ascontiguousarray(np.asarray(nsamples, dtype=np.int64))
        _check(lib().pcal_batch_extract(self._b, idv.size, idv.ctypes.data, ptrs.ctypes.data, ns.ctypes.data,
                                        ctypes.c_void_p(_stream_handle(stream))), "pcal_batch_extract")

    def _split(self, ids, flat):
        out, o = [], 0
        for i in ids:
            n = self.ntones[i]
            out.append(flat[o:o + n])
            o += n
        return out

    def results(self, ids):
        idv = self._ids(ids)
        tot = sum(self.ntones[i] for i in ids)
        amp = np.zeros(tot)
        ph = np.zeros(tot)
        d = np.zeros(len(ids))
        _check(lib().pcal_batch_results(self._b, idv.size, idv.ctypes.data, amp.ctypes.data, ph.ctypes.data,
                                        d.ctypes.data), "pcal_batch_results")
        return self._split(ids, amp), self._split(ids, ph), d

    def spectra(self, ids):
        idv = self._ids(ids)
        tot = sum(self.ntones[i] for i in ids)
        re = np.zeros(tot)
        im = np.zeros(tot)
        _check(lib().pcal_batch_spectra(self._b, idv.size, idv.ctypes.data, re.ctypes.data, im.ctypes.data),
               "pcal_batch_spectra")
        return self._split(ids, re + 1j * im)

    def reset(self, ids) -> None:
        idv = self._ids(ids)
        _check(lib().pcal_batch_reset(self._b, idv.size, idv.ctypes.data), "pcal_batch_reset")

    def close(self) -> None:
        if self._b and self._b.value:
            _check(lib().pcal_batch_destroy(self._b), "pcal_batch_destroy")
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class PCalServer:
    """Served form (pcal_server_t): many live streams under one device-memory budget,
    continuously batched."""

    def __init__(self, mem_budget_bytes: int, max_streams: int, precision: int = PREC_F64):
        self._s = ctypes.c_void_p()
        _check(lib().pcal_server_create(mem_budget_bytes, max_streams, precision, ctypes.byref(self._s)),
               "pcal_server_create")
        self.ntones = {}
        self._poll_sid = np.zeros(4096, dtype=np.int32)
        self._poll_int = np.zeros(4096, dtype=np.int64)
        # poll and step run once per turn of a serving loop: their arguments are made once
        self._poll_args = (self._poll_sid.size, self._poll_sid.ctypes.data, self._poll_int.ctypes.data)
        self._n = ctypes.c_int()
        self._dispatched = ctypes.c_int64()
        self._resident = False

    def open(self, fs: int, f_comb: int, f_offset: int, nbits: int, integration_samples: int,
             sideband: int = 1) -> int:
        """Stream id; raises PcalError(EAGAIN) when the memory budget cannot admit it."""
        sid = ctypes.c_int()
        _check(lib().pcal_server_open(self._s, fs, f_comb, f_offset, nbits, sideband, integration_samples,
                                      ctypes.byref(sid)), "pcal_server_open")
        self.ntones[sid.value] = fs // f_comb
        return sid.value

    def close_stream(self, sid: int) -> None:
        _check(lib().pcal_server_close(self._s, sid), "pcal_server_close")
        self.ntones.pop(sid, None)

    def submit(self, sids, ptrs, nsamples) -> None:
        """Queue chunks: sids, raw device addresses (or tensors) and sample counts, one per chunk."""
        n = len(sids)
        if len(ptrs) != n or len(nsamples) != n:
            raise ValueError("sids, ptrs and nsamples differ in length")
        if n == 0:
            return
        if isinstance(sids, np.ndarray) and isinstance(ptrs, np.ndarray) and isinstance(nsamples, np.ndarray):
            # arrays: their own memory, converted only where the element type differs
            sv = np.ascontiguousarray(sids, dtype=np.int32)
            pv = np.ascontiguousarray(ptrs, dtype=np.uint64)
            nv = np.ascontiguousarray(nsamples, dtype=np.int64)
            _check(lib().pcal_server_submit(self._s, n, sv.ctypes.data, pv.ctypes.data, nv.ctypes.data),
                   "pcal_server_submit")
            return
        # plain ctypes arrays: cheaper to build than numpy arrays and their ctypes views
        sv = (ctypes.c_int32 * n)(*(sids.tolist() if isinstance(sids, np.ndarray) else sids))
        pv = (ctypes.c_uint64 * n)(*(ptrs.tolist() if isinstance(ptrs, np.ndarray) else
                                     [p.data_ptr() if isinstance(p, torch.Tensor) else int(p) for p in ptrs]))
        nv = (ctypes.c_int64 * n)(*(nsamples.tolist() if isinstance(nsamples, np.ndarray) else nsamples))
        _check(lib().pcal_server_submit(self._s, n, ctypes.addressof(sv), ctypes.addressof(pv),
                                        ctypes.addressof(nv)), "pcal_server_submit")

    def step(self, stream=None) -> int:
        n = self._dispatched
        # the device-resident loop launches nothing on the caller's stream
        handle = None if self._resident and stream is None else _stream_handle(stream)
        _check(lib().pcal_server_step(self._s, handle, ctypes.byref(n)), "pcal_server_step")
        return n.value

    def poll(self):
        """[(sid, integration), ...] whose results have reached the host."""
        n = self._n
        _check(lib().pcal_server_poll(self._s, *self._poll_args, ctypes.byref(n)), "pcal_server_poll")
        k = n.value
        if k == 0:
            return []
        return list(zip(self._poll_sid[:k].tolist(), self._poll_int[:k].tolist()))

    def result(self, sid: int, integration: int):
        N = self.ntones[sid]
        amp = np.zeros(N)
        ph = np.zeros(N)
        d = np.zeros(1)
        _check(lib().pcal_server_result(self._s, sid, integration, amp.ctypes.data, ph.ctypes.data,
                                        d.ctypes.data), "pcal_server_result")
        return amp, ph, float(d[0])

    def spectrum(self, sid: int, integration: int) -> np.ndarray:
        N = self.ntones[sid]
        re = np.zeros(N)
        im = np.zeros(N)
        _check(lib().pcal_server_spectrum(self._s, sid, integration, re.ctypes.data, im.ctypes.data),
               "pcal_server_spectrum")
        return re + 1j * im

    def start(self, workgroups: int = 64, stream=None) -> None:
        """Switch to the device-resident loop: one persistent kernel on `stream` (pcal_server_start)."""
        _check(lib().pcal_server_start(self._s, workgroups, ctypes.c_void_p(_stream_handle(stream))),
               "pcal_server_start")
        self._resident = True

    def stop(self) -> None:
        """Leave the device-resident loop once the published work has ended (pcal_server_stop)."""
        _check(lib().pcal_server_stop(self._s), "pcal_server_stop")
        self._resident = False

    LOOP_STATS = ("chunks_published", "tasks_run", "tasks_published", "descriptor_reads_from_host",
                  "scheduler_rounds", "finalizes", "relaunches", "idle_rounds", "wait_ns", "descriptor_ns",
                  "fold_ns", "count_finalize_ns", "finalize_ns")

    def loop_stats(self) -> dict:
        """Counters of the device-resident loop (pcal_server_loop_stats), by name."""
        out = np.zeros(len(self.LOOP_STATS), dtype=np.int64)
        _check(lib().pcal_server_loop_stats(self._s, out.ctypes.data, out.size), "pcal_server_loop_stats")
        return {k: int(v) for k, v in zip(self.LOOP_STATS, out)}

    def stats(self) -> dict:
        q = ctypes.c_int64()
        f = ctypes.c_int()
        b = ctypes.c_int64()
        _check(lib().pcal_server_stats(self._s, ctypes.byref(q), ctypes.byref(f), ctypes.byref(b)),
               "pcal_server_stats")
        return {"queued_samples": q.value, "inflight_finalizes": f.value, "device_bytes": b.value}

    def close(self) -> None:
        if self._s and self._s.value:
            _check(lib().pcal_server_destroy(self._s), "pcal_server_destroy")
            self._s = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
