"""ctypes binding of libnufds (argument marshalling only).

Every step of the reconstruction runs in the library's HIP kernels; this module
only converts Python values to the C ABI declared in include/nufds.h and passes
device pointers and streams of torch tensors.  It never computes a result
itself and raises if the library is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnufds.so")

OK = 0
ERR_INVALID_ARG = 1
ERR_UNSUPPORTED = 2
ERR_OUT_OF_MEMORY = 3
ERR_HIP = 4
ERR_BUSY = 5

C64 = 0
C128 = 1

FLAG_CONVERGING = 1
FLAG_NO_STRETCH = 2
FLAG_NO_REMAP = 4


class View(ctypes.Structure):
    _fields_ = [("center_x", ctypes.c_double), ("center_y", ctypes.c_double),
                ("pitch_x", ctypes.c_double), ("pitch_y", ctypes.c_double),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("pad", ctypes.c_double), ("frt_size_x", ctypes.c_int32), ("frt_size_y", ctypes.c_int32),
                ("oversample", ctypes.c_int32), ("map_model", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("sx", ctypes.c_int32), ("sy", ctypes.c_int32),
                ("mx", ctypes.c_int32), ("my", ctypes.c_int32), ("kcx", ctypes.c_int32), ("kcy", ctypes.c_int32),
                ("dfx", ctypes.c_double), ("dfy", ctypes.c_double), ("dox", ctypes.c_double),
                ("doy", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("image_size", ctypes.c_double), ("xlo", ctypes.c_double), ("xhi", ctypes.c_double),
                ("ylo", ctypes.c_double), ("yhi", ctypes.c_double), ("padx", ctypes.c_double),
                ("pady", ctypes.c_double), ("workspace_bytes", ctypes.c_uint64), ("map_bytes", ctypes.c_uint64),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32), ("fcx0", ctypes.c_int32),
                ("fcxn", ctypes.c_int32), ("oversample", ctypes.c_int32), ("map_model", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("ms", ctypes.c_double), ("bytes", ctypes.c_uint64)]


class ServerOptions(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("max_frt_size", ctypes.c_int32), ("max_view_size", ctypes.c_int32),
                ("max_inflight", ctypes.c_int32), ("max_workspace_bytes", ctypes.c_uint64)]


class NufdsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libnufds status {status}: {msg}")
        self.status = status


_lib: Optional[ctypes.CDLL] = None

# name -> (restype, argtypes): every entry point of include/nufds.h
_SIGNATURES = {
    "nufds_plan_geometry": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_double, ctypes.POINTER(View), ctypes.c_uint32,
                                           ctypes.POINTER(Options), ctypes.POINTER(PlanInfo)]),
    "nufds_plan_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(View),
                                         ctypes.c_int, ctypes.c_uint32]),
    "nufds_plan_create_ex": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_double, ctypes.c_double,
                                            ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(View),
                                            ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(Options)]),
    "nufds_plan_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(PlanInfo)]),
    "nufds_execute": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "nufds_debug_copy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_uint64), ctypes.c_void_p]),
    "nufds_set_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "nufds_get_timings": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(KernelTime), ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32)]),
    "nufds_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "nufds_synth_hologram": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_void_p,
                                            ctypes.c_void_p]),
    "nufds_spectrum_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_double, ctypes.c_double,
                                             ctypes.c_int32, ctypes.c_int32, ctypes.c_int, ctypes.c_uint32,
                                             ctypes.c_void_p, ctypes.c_void_p]),
    "nufds_spectrum_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "nufds_execute_spectrum": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "nufds_server_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ServerOptions)]),
    "nufds_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.POINTER(View),
                                           ctypes.c_uint32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "nufds_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_double)]),
    "nufds_server_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]),
    "nufds_server_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "nufds_stack_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_double, ctypes.c_double,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                          ctypes.c_int32, ctypes.c_int, ctypes.c_uint32]),
    "nufds_stack_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(PlanInfo)]),
    "nufds_stack_execute": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.c_void_p]),
    "nufds_stack_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "nufds_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "nufds_last_error": (ctypes.c_char_p, []),
}


def load() -> ctypes.CDLL:
    """Load libnufds.so from the package directory; raise if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libnufds.so not found at {LIB_PATH}; build it with "
                           "python -m paper_2410_13474_amd.build_lib")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int) -> None:
    if status != OK:
        lib = load()
        raise NufdsError(status, lib.nufds_last_error().decode())


def _view(view) -> Optional[View]:
    if view is None:
        return None
    if isinstance(view, View):
        return view
    return View(float(view.get("center_x", 0.0)), float(view.get("center_y", 0.0)),
                float(view.get("pitch_x", 0.0)), float(view.get("pitch_y", 0.0)),
                int(view["nx"]), int(view["ny"]))


MAP_MODELS = {"exact": 0, "paper": 1}


def _options(pad, frt_size, oversample=None, map_model=None) -> Optional[Options]:
    if pad is None and frt_size is None and oversample is None and map_model is None:
        return None
    fx, fy = frt_size if frt_size is not None else (0, 0)
    return Options(-1.0 if pad is None else float(pad), int(fx), int(fy), int(oversample or 0),
                   MAP_MODELS[map_model or "exact"])


def plan_geometry(wavelength, pitch, nx, ny, z, view=None, flags=0, pad=None, frt_size=None,
                  oversample=None, map_model=None) -> dict:
    """Host-only geometry of a plan (no GPU touched): sizes, K_c, M, pitches."""
    lib = load()
    info = PlanInfo()
    v = _view(view)
    o = _options(pad, frt_size, oversample, map_model)
    _check(lib.nufds_plan_geometry(float(wavelength), float(pitch), int(nx), int(ny), float(z),
                                   ctypes.byref(v) if v is not None else None, int(flags),
                                   ctypes.byref(o) if o is not None else None, ctypes.byref(info)))
    return info.as_dict()


def _stream_handle(stream) -> ctypes.c_void_p:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """A reconstruction plan bound to the current device.

    ``precision`` is "c64" (complex64 data, float64 maps and phases) or "c128".
    ``view`` is None (full view) or a dict with center_x, center_y, pitch_x,
    pitch_y (<= 0: Delta_F) and nx, ny.
    """

    def __init__(self, wavelength, pitch, nx, ny, z, view=None, precision="c64", flags=0, pad=None,
                 frt_size=None, oversample=None, map_model=None):
        lib = load()
        self._lib = lib
        self.precision = {"c64": C64, "c128": C128}[precision]
        handle = ctypes.c_void_p()
        v = _view(view)
        o = _options(pad, frt_size, oversample, map_model)
        vp = ctypes.byref(v) if v is not None else None
        if o is None:
            st = lib.nufds_plan_create(ctypes.byref(handle), float(wavelength), float(pitch), int(nx), int(ny),
                                       float(z), vp, self.precision, int(flags))
        else:
            st = lib.nufds_plan_create_ex(ctypes.byref(handle), float(wavelength), float(pitch), int(nx),
                                          int(ny), float(z), vp, self.precision, int(flags), ctypes.byref(o))
        _check(st)
        self._h = handle
        info = PlanInfo()
        _check(lib.nufds_plan_info(self._h, ctypes.byref(info)))
        self.info = info.as_dict()

    @property
    def dtype(self):
        import torch
        return torch.complex64 if self.precision == C64 else torch.complex128

    def execute_spectrum(self, spectrum: "Spectrum", out, stream=None) -> None:
        """Enqueue the reconstruction from a cached spectrum (no forward FFT) into ``out``."""
        i = self.info
        if out.dtype != self.dtype or tuple(out.shape) != (i["sy"], i["sx"]) or not out.is_contiguous():
            raise ValueError("out must be a contiguous tensor of the plan's output shape and precision")
        _check(self._lib.nufds_execute_spectrum(self._h, spectrum._h, ctypes.c_void_p(out.data_ptr()),
                                                _stream_handle(stream)))

    def execute(self, hologram, out, stream=None) -> None:
        """Enqueue the reconstruction of device tensor ``hologram`` into ``out``."""
        import torch
        i = self.info
        if hologram.dtype != self.dtype or out.dtype != self.dtype:
            raise TypeError("tensor dtypes must match the plan precision")
        if tuple(hologram.shape) != (i["ny"], i["nx"]) or tuple(out.shape) != (i["sy"], i["sx"]):
            raise ValueError("tensor shapes do not match the plan")
        if not (hologram.is_cuda and out.is_cuda and hologram.is_contiguous() and out.is_contiguous()):
            raise ValueError("tensors must be contiguous device tensors")
        _check(self._lib.nufds_execute(self._h, ctypes.c_void_p(hologram.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))

    def __call__(self, hologram, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((self.info["sy"], self.info["sx"]), dtype=self.dtype, device=hologram.device)
        self.execute(hologram, out, stream)
        return out

    def debug_copy(self, which: int, stream=None):
        """Copy an internal buffer (1 spectrum, 2 FrT F, 3 map table) into a new device tensor."""
        import torch
        n = ctypes.c_uint64()
        _check(self._lib.nufds_debug_copy(self._h, int(which), None, ctypes.byref(n), None))
        i = self.info
        if which == 3:
            dst = torch.empty(int(n.value) // 8, dtype=torch.float64, device="cuda")
        else:
            f = i["oversample"]
            shape = (f * i["ny"], f * i["nx"]) if which == 1 else (i["my"], i["mx"])
            dst = torch.empty(shape, dtype=self.dtype, device="cuda")
        _check(self._lib.nufds_debug_copy(self._h, int(which), ctypes.c_void_p(dst.data_ptr()),
                                          ctypes.byref(n), _stream_handle(stream)))
        return dst

    def set_timing(self, n_executes: int = 1) -> None:
        """Record HIP events around every kernel of the next ``n_executes`` executes (0: off)."""
        _check(self._lib.nufds_set_timing(self._h, int(n_executes)))

    def timings(self) -> list:
        """[(name, ms, algorithmic bytes)] for each recorded launch, in launch order."""
        n = ctypes.c_int32()
        _check(self._lib.nufds_get_timings(self._h, None, 0, ctypes.byref(n)))
        arr = (KernelTime * max(1, n.value))()
        _check(self._lib.nufds_get_timings(self._h, arr, n.value, ctypes.byref(n)))
        return [(arr[i].name.decode(), float(arr[i].ms), int(arr[i].bytes)) for i in range(n.value)]

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.nufds_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def synth_hologram(points, nx, ny, pitch, wavelength, out, stream=None) -> None:
    """Point-source hologram on the GPU into device tensor ``out`` ([ny, nx] complex64/128).

    ``points``: float64 array (P, 5) of x, y, z, amplitude, phase (host).
    """
    import numpy as np
    import torch
    lib = load()
    pts = np.ascontiguousarray(points, dtype=np.float64)
    if pts.ndim != 2 or pts.shape[1] != 5:
        raise ValueError("points must be (P, 5)")
    prec = C64 if out.dtype == torch.complex64 else C128
    if tuple(out.shape) != (ny, nx) or not out.is_contiguous():
        raise ValueError("out must be a contiguous [ny, nx] tensor")
    _check(lib.nufds_synth_hologram(pts.ctypes.data_as(ctypes.c_void_p), int(pts.shape[0]), int(nx), int(ny),
                                    float(pitch), float(wavelength), prec, ctypes.c_void_p(out.data_ptr()),
                                    _stream_handle(stream)))


class Spectrum:
    """The forward FFT of one hologram, cached on the device (computed when constructed)."""

    def __init__(self, hologram, wavelength, pitch, flags=0, stream=None):
        import torch
        lib = load()
        self._lib = lib
        if hologram.dtype not in (torch.complex64, torch.complex128):
            raise TypeError("hologram must be complex64 or complex128")
        if not (hologram.is_cuda and hologram.is_contiguous() and hologram.dim() == 2):
            raise ValueError("hologram must be a contiguous 2-D device tensor")
        self.precision = C64 if hologram.dtype == torch.complex64 else C128
        self.ny, self.nx = int(hologram.shape[0]), int(hologram.shape[1])
        self.wavelength, self.pitch, self.flags = float(wavelength), float(pitch), int(flags)
        handle = ctypes.c_void_p()
        _check(lib.nufds_spectrum_create(ctypes.byref(handle), self.wavelength, self.pitch, self.nx, self.ny,
                                         self.precision, self.flags, ctypes.c_void_p(hologram.data_ptr()),
                                         _stream_handle(stream)))
        self._h = handle

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.nufds_spectrum_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Partial-view server over cached spectra: submit() queues, wait() returns the latency in ms."""

    def __init__(self, precision="c64", max_frt_size=8192, max_view_size=4096, max_inflight=4,
                 max_workspace_bytes=0):
        lib = load()
        self._lib = lib
        self.precision = {"c64": C64, "c128": C128}[precision]
        opt = ServerOptions(self.precision, int(max_frt_size), int(max_view_size), int(max_inflight),
                            int(max_workspace_bytes))
        handle = ctypes.c_void_p()
        _check(lib.nufds_server_create(ctypes.byref(handle), ctypes.byref(opt)))
        self._h = handle

    def submit(self, spectrum: Spectrum, z, out, view=None, flags=0) -> int:
        """Queue one view of ``spectrum`` at distance ``z`` into device tensor ``out``; returns a ticket."""
        v = _view(view)
        if not (out.is_cuda and out.is_contiguous()):
            raise ValueError("out must be a contiguous device tensor")
        t = ctypes.c_uint64()
        _check(self._lib.nufds_server_submit(self._h, spectrum._h, float(z), ctypes.byref(v) if v is not None else None,
                                             int(flags), ctypes.c_void_p(out.data_ptr()), ctypes.byref(t)))
        return int(t.value)

    def poll(self, ticket: int):
        """(state, latency_ms): state 0 queued/running, 1 done, 2 failed."""
        st, lat = ctypes.c_int32(), ctypes.c_double()
        _check(self._lib.nufds_server_poll(self._h, int(ticket), ctypes.byref(st), ctypes.byref(lat)))
        return int(st.value), float(lat.value)

    def wait(self, ticket: int) -> float:
        """Block until the request ends; returns its latency in ms (raises on a failed request)."""
        lat = ctypes.c_double()
        _check(self._lib.nufds_server_wait(self._h, int(ticket), ctypes.byref(lat)))
        return float(lat.value)

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.nufds_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Stack:
    """Full views of one hologram at several depths sharing the z-independent stages (one FFT of the
    hologram, stretch-gather and inverse DFT per execute; chirp, DFT and output gather per depth)."""

    def __init__(self, wavelength, pitch, nx, ny, zs, precision="c64", flags=0):
        lib = load()
        self._lib = lib
        self.precision = {"c64": C64, "c128": C128}[precision]
        zs = [float(z) for z in zs]
        arr = (ctypes.c_double * max(1, len(zs)))(*zs)
        handle = ctypes.c_void_p()
        _check(lib.nufds_stack_create(ctypes.byref(handle), float(wavelength), float(pitch), int(nx), int(ny), arr,
                                      len(zs), self.precision, int(flags)))
        self._h = handle
        self.zs = zs
        self.infos = []
        for i in range(len(zs)):
            info = PlanInfo()
            _check(lib.nufds_stack_info(self._h, i, ctypes.byref(info)))
            self.infos.append(info.as_dict())

    @property
    def dtype(self):
        import torch
        return torch.complex64 if self.precision == C64 else torch.complex128

    def execute(self, hologram, outs, stream=None) -> None:
        """Enqueue every depth of the stack from device tensor ``hologram`` into ``outs`` (one per depth)."""
        i0 = self.infos[0]
        if hologram.dtype != self.dtype or tuple(hologram.shape) != (i0["ny"], i0["nx"]):
            raise ValueError("hologram must match the stack's precision and size")
        if len(outs) != len(self.zs):
            raise ValueError("one output per depth")
        for o, info in zip(outs, self.infos):
            if o.dtype != self.dtype or tuple(o.shape) != (info["sy"], info["sx"]) or not (o.is_cuda and
                                                                                          o.is_contiguous()):
                raise ValueError("outputs must be contiguous device tensors of each depth's shape and precision")
        if not (hologram.is_cuda and hologram.is_contiguous()):
            raise ValueError("hologram must be a contiguous device tensor")
        ptrs = (ctypes.c_void_p * len(outs))(*[o.data_ptr() for o in outs])
        _check(self._lib.nufds_stack_execute(self._h, ctypes.c_void_p(hologram.data_ptr()), ptrs,
                                             _stream_handle(stream)))

    def __call__(self, hologram, outs=None, stream=None):
        import torch
        if outs is None:
            outs = [torch.empty((i["sy"], i["sx"]), dtype=self.dtype, device=hologram.device) for i in self.infos]
        self.execute(hologram, outs, stream)
        return outs

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.nufds_stack_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
