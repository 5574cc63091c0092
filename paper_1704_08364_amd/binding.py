"""ctypes binding of libbst.so (include/bst.h) -- argument marshalling only.

Every step of the computation runs in the library's HIP kernels; torch only
provides device memory and the current stream. If the library has not been
built, importing works but every call raises BstNativeMissing: there is no
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# BST_LIBRARY selects another build of the same library (for instance the
# host-sanitizer build of `python -m paper_1704_08364_amd.build --host-sanitize`).
LIB_PATH = os.environ.get("BST_LIBRARY") or os.path.join(_HERE, "libbst.so")

BST_OK = 0
STATUS_NAMES = {
    0: "BST_OK", 1: "BST_E_NULL", 2: "BST_E_SHAPE", 3: "BST_E_ANGLES", 4: "BST_E_PARAM",
    5: "BST_E_WORKSPACE", 6: "BST_E_NOMEM", 7: "BST_E_DEVICE", 8: "BST_E_UNSUPPORTED",
    9: "BST_E_BATCH", 10: "BST_E_ALIAS",
}
FILTERS = {"none": 0, "ramp": 1}
TAPERS = {"deapod": 0, "none": 1, "kaiser": 2, "kb": 2, "keys": 3}
INTERPS = {"linear": 0, "keys": 1}
ANGULARS = {"linear": 0, "tent": 1}
APODIZATIONS = {"ramlak": 0, "shepp": 1, "hann": 2, "cosine": 3}
DTYPES = {"f32": 0, "f64": 1}

# Every symbol include/bst.h declares, with its ctypes signature.
_P = C.c_void_p
_I = C.c_int32
_S = C.c_size_t


class bst_params(C.Structure):
    _fields_ = [
        ("n_det", C.c_int32), ("n_angles", C.c_int32), ("n_out", C.c_int32),
        ("angles", C.POINTER(C.c_double)),
        ("pad_radial", C.c_int32), ("pad_cart", C.c_int32),
        ("filter", C.c_int32), ("taper", C.c_int32), ("taper_beta", C.c_double),
        ("max_batch", C.c_int32), ("device", C.c_int32), ("adjoint", C.c_int32),
        ("apodization", C.c_int32), ("center_shift", C.c_double),
        ("interp", C.c_int32), ("monopole_width", C.c_double), ("angular", C.c_int32),
        ("dtype", C.c_int32), ("gather_slices", C.c_int32),
    ]


SIGNATURES = {
    "bst_params_default": (None, [C.POINTER(bst_params), _I, _I, _I]),
    "bst_validate": (C.c_int, [C.POINTER(bst_params)]),
    "bst_query_workspace": (C.c_int, [C.POINTER(bst_params), _I, C.POINTER(_S)]),
    "bst_query_max_batch": (C.c_int, [C.POINTER(bst_params), _S, C.POINTER(_I)]),
    "bst_plan": (C.c_int, [C.POINTER(bst_params), C.POINTER(_P)]),
    "bst_workspace_size": (C.c_int, [_P, _I, C.POINTER(_S)]),
    "bst_backproject": (C.c_int, [_P, _P, _P, _I, _P, _S, _P]),
    "bst_backproject_timed": (C.c_int, [_P, _P, _P, _I, _P, _S, _P, C.POINTER(_P)]),
    "bst_backproject_noalloc": (C.c_int, [_P, _P, _P, _I, _P]),
    "bst_backproject_counts": (C.c_int, [_P, _P, _P, _P, _P, _I, _P, _S, _P]),
    "bst_backproject_bruteforce": (C.c_int, [_P, _P, _P, _I, _P]),
    "bst_project": (C.c_int, [_P, _P, _P, _I, _P, _S, _P]),
    "bst_ramp_filter": (C.c_int, [_P, _P, _P, _I, _P]),
    "bst_backproject_f64": (C.c_int, [_P, _P, _P, _I, _P, _S, _P]),
    "bst_project_f64": (C.c_int, [_P, _P, _P, _I, _P, _S, _P]),
    "bst_debug_spectrum": (C.c_int, [_P, _P, _P, _P, _I, _P, _S, _P]),
    "bst_destroy": (C.c_int, [_P]),
    "bst_status_string": (C.c_char_p, [C.c_int]),
    "bst_debug_check": (C.c_int, [_I, C.POINTER(C.c_uint32)]),
    "bst_last_error_string": (C.c_char_p, []),
    "bst_event_create": (C.c_int, [C.POINTER(_P)]),
    "bst_event_destroy": (C.c_int, [_P]),
    "bst_event_elapsed_ms": (C.c_int, [_P, _P, C.POINTER(C.c_float)]),
    "bst_stream_synchronize": (C.c_int, [_P]),
    "bst_batch_create": (C.c_int, [C.POINTER(bst_params), _I, C.POINTER(_I), C.POINTER(_I), C.POINTER(_P)]),
    "bst_batch_workspace_size": (C.c_int, [_P, C.POINTER(_S)]),
    "bst_batch_classes": (C.c_int, [_P, C.POINTER(_I)]),
    "bst_batch_tune": (C.c_int, [_P, _P, C.POINTER(C.c_int64), _P, C.POINTER(C.c_int64), _P, _S, _P]),
    "bst_batch_backproject": (C.c_int, [_P, _P, C.POINTER(C.c_int64), _P, C.POINTER(C.c_int64), _P, _S, _P]),
    "bst_batch_destroy": (C.c_int, [_P]),
}


class BstNativeMissing(RuntimeError):
    pass


class BstError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        name = STATUS_NAMES.get(status, str(status))
        msg = f"{where}: {name}"
        if detail:
            msg += f" ({detail})"
        super().__init__(msg)


_lib = None


def lib():
    """The loaded library; raises BstNativeMissing when it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise BstNativeMissing(
                f"{LIB_PATH} is missing: build it with `python -m paper_1704_08364_amd.build`")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


def _check(status: int, where: str):
    if status != BST_OK:
        L = lib()
        detail = L.bst_last_error_string().decode() if status == 7 else L.bst_status_string(status).decode()
        raise BstError(status, where, detail)


def make_params(n_det: int, n_angles: int, n_out: Optional[int] = None, *, pad_radial: int = 2,
                pad_cart: int = 2, filter: str = "ramp", taper: str = "deapod",
                taper_beta: float = 8.0, max_batch: int = 1, device: int = 0,
                angles: Optional[Sequence[float]] = None, adjoint: bool = False,
                apodization: str = "ramlak", center_shift: float = 0.0, interp: str = "linear",
                monopole_width: float = 0.0, angular: str = "linear", gather_slices: int = 0,
                dtype: str = "f32"):
    """bst_params plus the ctypes array that backs `angles` (keep both alive).
    interp='keys' (cubic radial interpolation) pairs with taper='keys';
    monopole_width > 0 (filter='none' only) subtracts a Gaussian monopole of that
    width (units of t, detector in [-1, 1)) and adds its backprojection back;
    angular='tent' (uniform angles, linear interp) widens the angular kernel at
    small radii, which makes plan.project a close Radon approximation.
    gather_slices (0 = default) sets the slices per block of the gather kernel;
    results do not depend on it. dtype='f64' makes a plan of the FP64
    gradient-check path (float64 sinograms and images)."""
    p = bst_params()
    lib().bst_params_default(C.byref(p), n_det, n_angles, n_det if n_out is None else n_out)
    p.pad_radial = pad_radial
    p.pad_cart = pad_cart
    p.filter = FILTERS[filter] if isinstance(filter, str) else int(filter)
    p.taper = TAPERS[taper] if isinstance(taper, str) else int(taper)
    p.taper_beta = taper_beta
    p.max_batch = max_batch
    p.device = device
    p.adjoint = 1 if adjoint else 0
    p.apodization = APODIZATIONS[apodization] if isinstance(apodization, str) else int(apodization)
    p.center_shift = center_shift
    p.interp = INTERPS[interp] if isinstance(interp, str) else int(interp)
    p.monopole_width = monopole_width
    p.angular = ANGULARS[angular] if isinstance(angular, str) else int(angular)
    p.gather_slices = int(gather_slices)
    p.dtype = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    keep = None
    if angles is not None:
        arr = np.ascontiguousarray(np.asarray(angles, dtype=np.float64))
        keep = (C.c_double * arr.size)(*arr.tolist())
        p.angles = C.cast(keep, C.POINTER(C.c_double))
    return p, keep


def query_workspace(params: bst_params, batch: int) -> int:
    out = C.c_size_t(0)
    _check(lib().bst_query_workspace(C.byref(params), batch, C.byref(out)), "bst_query_workspace")
    return int(out.value)


def query_max_batch(params: bst_params, budget_bytes: int) -> int:
    """Largest batch whose sinograms, images and workspace fit in budget_bytes
    (0 when not even one slice fits)."""
    out = C.c_int32(0)
    st = lib().bst_query_max_batch(C.byref(params), int(budget_bytes), C.byref(out))
    if st not in (BST_OK, 6):  # 6: BST_E_NOMEM, nothing fits
        _check(st, "bst_query_max_batch")
    return int(out.value)


def _stream_ptr(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _dev_tensor(t, name: str, dtype, shape_tail):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape[-len(shape_tail):]) != tuple(shape_tail):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected [..., {shape_tail}]")
    return t


def _out_tensor(out, name: str, shape, device, dtype=None):
    """A caller-supplied output: float32 (float64 for FP64 plans), contiguous,
    exactly `shape`, on the plan's device. The library writes shape-many
    elements and receives no size, so anything smaller would be written past
    its end."""
    import torch
    _dev_tensor(out, name, dtype or torch.float32, shape[1:])
    if tuple(out.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(out.shape)}, expected {tuple(shape)}")
    if out.device != device:
        raise ValueError(f"{name} is on {out.device}, the plan's data on {device}")
    return out


def _keep_alive(stream, *tensors):
    """Tensors the kernels use on `stream` while they may be freed or reused by
    the caching allocator of another stream: tell the allocator."""
    import torch
    if stream is None or stream == torch.cuda.current_stream(stream.device):
        return
    for t in tensors:
        if t is not None:
            t.record_stream(stream)


class Event:
    """A HIP event made by the library (for per-kernel timing)."""

    def __init__(self):
        h = C.c_void_p()
        _check(lib().bst_event_create(C.byref(h)), "bst_event_create")
        self.handle = h

    def elapsed_ms(self, stop: "Event") -> float:
        ms = C.c_float(0.0)
        _check(lib().bst_event_elapsed_ms(self.handle, stop.handle, C.byref(ms)), "bst_event_elapsed_ms")
        return float(ms.value)

    def __del__(self):
        try:
            if self.handle:
                lib().bst_event_destroy(self.handle)
        except Exception:
            pass


class Plan:
    """A bst_plan on one device. Sinograms are float32 [B][V][n] (or [V][n]),
    images float32 [B][N][N]; float64 for plans of dtype 'f64' (backproject
    and project only)."""

    def __init__(self, n_det: int, n_angles: int, n_out: Optional[int] = None, **kw):
        self.params, self._angles_keep = make_params(n_det, n_angles, n_out, **kw)
        self.n = n_det
        self.V = n_angles
        self.N = n_det if n_out is None else n_out
        self.max_batch = self.params.max_batch
        self.device = self.params.device
        self.M = (self.params.pad_radial or 2) * n_det
        self.G = (self.params.pad_cart or 2) * self.N
        self.f64 = self.params.dtype == DTYPES["f64"]
        h = C.c_void_p()
        _check(lib().bst_plan(C.byref(self.params), C.byref(h)), "bst_plan")
        self.handle = h

    @property
    def torch_dtype(self):
        import torch
        return torch.float64 if self.f64 else torch.float32

    def close(self):
        if getattr(self, "handle", None):
            _check(lib().bst_destroy(self.handle), "bst_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_size(self, batch: int) -> int:
        out = C.c_size_t(0)
        _check(lib().bst_workspace_size(self.handle, batch, C.byref(out)), "bst_workspace_size")
        return int(out.value)

    def workspace(self, batch: int):
        import torch
        return torch.empty(max(self.workspace_size(batch), 1), dtype=torch.uint8,
                           device=f"cuda:{self.device}")

    def _prep(self, sino, dtype=None):
        import torch
        sino = _dev_tensor(sino, "sino", dtype or torch.float32, (self.V, self.n))
        batched = sino.dim() == 3
        s3 = sino if batched else sino.unsqueeze(0)
        return s3, batched

    def backproject(self, sino, out=None, workspace=None, stream=None, events=None):
        import torch
        s3, batched = self._prep(sino, self.torch_dtype)
        B = s3.shape[0]
        if out is None:
            out = torch.empty(B, self.N, self.N, dtype=self.torch_dtype, device=s3.device)
        o3 = _out_tensor(out if out.dim() == 3 or batched else out.unsqueeze(0), "out", (B, self.N, self.N),
                         s3.device, self.torch_dtype)
        if workspace is None:
            workspace = self.workspace(B)
        _keep_alive(stream, s3, o3, workspace)
        sp = _stream_ptr(stream)
        if self.f64:
            if events is not None:
                raise ValueError("per-kernel events are for float32 plans")
            st = lib().bst_backproject_f64(self.handle, s3.data_ptr(), o3.data_ptr(), B, workspace.data_ptr(),
                                           workspace.numel(), sp)
            _check(st, "bst_backproject_f64")
        elif events is None:
            st = lib().bst_backproject(self.handle, s3.data_ptr(), o3.data_ptr(), B,
                                       workspace.data_ptr(), workspace.numel(), sp)
            _check(st, "bst_backproject")
        else:
            arr = (C.c_void_p * 4)(*[e.handle for e in events])
            st = lib().bst_backproject_timed(self.handle, s3.data_ptr(), o3.data_ptr(), B,
                                             workspace.data_ptr(), workspace.numel(), sp, arr)
            _check(st, "bst_backproject_timed")
        return o3 if batched else o3[0]

    def backproject_counts(self, counts, flat, dark, out=None, workspace=None, stream=None):
        """BST of raw counts with per-slice flat/dark fields [B][n] (normalised on load)."""
        import torch
        c3, batched = self._prep(counts)
        B = c3.shape[0]
        flat = _dev_tensor(flat, "flat", torch.float32, (self.n,)).reshape(-1, self.n)
        dark = _dev_tensor(dark, "dark", torch.float32, (self.n,)).reshape(-1, self.n)
        if flat.shape[0] != B or dark.shape[0] != B:
            raise ValueError("flat and dark need one row of n values per slice")
        if out is None:
            out = torch.empty(B, self.N, self.N, dtype=torch.float32, device=c3.device)
        o3 = _out_tensor(out if out.dim() == 3 or batched else out.unsqueeze(0), "out", (B, self.N, self.N),
                         c3.device)
        if workspace is None:
            workspace = self.workspace(B)
        _keep_alive(stream, c3, flat, dark, o3, workspace)
        _check(lib().bst_backproject_counts(self.handle, c3.data_ptr(), flat.data_ptr(), dark.data_ptr(),
                                            o3.data_ptr(), B, workspace.data_ptr(), workspace.numel(),
                                            _stream_ptr(stream)), "bst_backproject_counts")
        return o3 if batched else o3[0]

    def bruteforce(self, sino, out=None, stream=None):
        import torch
        s3, batched = self._prep(sino)
        B = s3.shape[0]
        if out is None:
            out = torch.empty(B, self.N, self.N, dtype=torch.float32, device=s3.device)
        o3 = _out_tensor(out if out.dim() == 3 or batched else out.unsqueeze(0), "out", (B, self.N, self.N),
                         s3.device)
        _keep_alive(stream, s3, o3)
        _check(lib().bst_backproject_bruteforce(self.handle, s3.data_ptr(), o3.data_ptr(), B,
                                                _stream_ptr(stream)), "bst_backproject_bruteforce")
        return o3 if batched else o3[0]

    def ramp_filter(self, sino, out=None, stream=None):
        """The brute-force FBP's ramp filter (Kak-Slaney kernel, linear
        convolution) of float32 [B][V][n] sinograms."""
        import torch
        s3, batched = self._prep(sino)
        B = s3.shape[0]
        if out is None:
            out = torch.empty_like(s3)
        o3 = _out_tensor(out if out.dim() == 3 or batched else out.unsqueeze(0), "out", (B, self.V, self.n),
                         s3.device)
        _keep_alive(stream, s3, o3)
        _check(lib().bst_ramp_filter(self.handle, s3.data_ptr(), o3.data_ptr(), B, _stream_ptr(stream)),
               "bst_ramp_filter")
        return o3 if batched else o3[0]

    def debug_spectrum(self, sino, workspace=None, stream=None):
        """(complex64 [B][V][M/2] polar spectrum dt*K*Y, float32 [B][V] dt*Y[0])."""
        import torch
        s3, batched = self._prep(sino)
        B = s3.shape[0]
        spec = torch.empty(B, self.V, self.M // 2, dtype=torch.complex64, device=s3.device)
        dc = torch.empty(B, self.V, dtype=torch.float32, device=s3.device)
        if workspace is None:
            workspace = self.workspace(B)
        _keep_alive(stream, s3, spec, dc, workspace)
        _check(lib().bst_debug_spectrum(self.handle, s3.data_ptr(), spec.data_ptr(), dc.data_ptr(), B,
                                        workspace.data_ptr(), workspace.numel(), _stream_ptr(stream)),
               "bst_debug_spectrum")
        return (spec, dc) if batched else (spec[0], dc[0])

    def project(self, img, out=None, workspace=None, stream=None):
        import torch
        img = _dev_tensor(img, "img", self.torch_dtype, (self.N, self.N))
        i3 = img if img.dim() == 3 else img.unsqueeze(0)
        B = i3.shape[0]
        if out is None:
            out = torch.empty(B, self.V, self.n, dtype=self.torch_dtype, device=i3.device)
        o3 = _out_tensor(out if out.dim() == 3 or img.dim() == 3 else out.unsqueeze(0), "out",
                         (B, self.V, self.n), i3.device, self.torch_dtype)
        if workspace is None:
            workspace = self.workspace(B)
        _keep_alive(stream, i3, o3, workspace)
        fn, name = (lib().bst_project_f64, "bst_project_f64") if self.f64 else (lib().bst_project, "bst_project")
        _check(fn(self.handle, i3.data_ptr(), o3.data_ptr(), B, workspace.data_ptr(), workspace.numel(),
                  _stream_ptr(stream)), name)
        return o3 if img.dim() == 3 else o3[0]


class Batch:
    """Uneven-size batch (bst_batch_*): sinograms of sizes (n_i, V_i) packed in
    one float32 device buffer, images in another, run as one graph launch."""

    def __init__(self, sizes, device: int = 0, **kw):
        """sizes: sequence of (n_det, n_angles); other parameters as for Plan."""
        self.sizes = [(int(n), int(v)) for n, v in sizes]
        self.count = len(self.sizes)
        self.params, self._keep = make_params(self.sizes[0][0], self.sizes[0][1], device=device, **kw)
        n_arr = (C.c_int32 * self.count)(*[n for n, _ in self.sizes])
        v_arr = (C.c_int32 * self.count)(*[v for _, v in self.sizes])
        h = C.c_void_p()
        _check(lib().bst_batch_create(C.byref(self.params), self.count, n_arr, v_arr, C.byref(h)),
               "bst_batch_create")
        self.handle = h
        self.device = device
        self.sino_off, self.img_off = [], []
        so = io = 0
        for n, v in self.sizes:
            self.sino_off.append(so)
            self.img_off.append(io)
            so += v * n
            io += n * n
        self.sino_elems, self.img_elems = so, io
        self._so = (C.c_int64 * self.count)(*self.sino_off)
        self._io = (C.c_int64 * self.count)(*self.img_off)

    def close(self):
        if getattr(self, "handle", None):
            lib().bst_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def classes(self) -> int:
        out = C.c_int32()
        _check(lib().bst_batch_classes(self.handle, C.byref(out)), "bst_batch_classes")
        return int(out.value)

    def workspace(self):
        import torch
        out = C.c_size_t()
        _check(lib().bst_batch_workspace_size(self.handle, C.byref(out)), "bst_batch_workspace_size")
        return torch.empty(max(int(out.value), 1), dtype=torch.uint8, device=f"cuda:{self.device}")

    def _args(self, sinos, imgs, workspace):
        import torch
        _dev_tensor(sinos, "sinos", torch.float32, (self.sino_elems,))
        _dev_tensor(imgs, "imgs", torch.float32, (self.img_elems,))
        return (self.handle, sinos.data_ptr(), self._so, imgs.data_ptr(), self._io,
                workspace.data_ptr(), workspace.numel())

    def tune(self, sinos, imgs, workspace, stream=None):
        _check(lib().bst_batch_tune(*self._args(sinos, imgs, workspace), _stream_ptr(stream)), "bst_batch_tune")

    def backproject(self, sinos, imgs, workspace, stream=None):
        _check(lib().bst_batch_backproject(*self._args(sinos, imgs, workspace), _stream_ptr(stream)),
               "bst_batch_backproject")
        return imgs

    def sino_view(self, sinos, i):
        n, v = self.sizes[i]
        return sinos[self.sino_off[i]:self.sino_off[i] + v * n].view(v, n)

    def img_view(self, imgs, i):
        n, _ = self.sizes[i]
        return imgs[self.img_off[i]:self.img_off[i] + n * n].view(n, n)
