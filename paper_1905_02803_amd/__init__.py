"""Python binding of the MI355X pencil 3D R2C / C2R FFT library (libpencilfft.so).

Argument marshalling only: every step of a transform runs in the library's
HIP kernels; PyTorch supplies device memory and streams.  The functions named
``pf_*`` mirror the C ABI in include/pencilfft.h one to one; ``Plan`` wraps a
plan handle for convenience.  There is no fallback: if the library is not
built, importing the binding's functions raises.

Layouts (C order, slowest index first; Table 1 of the paper):
  real X-pencil            [nz][ny][nx]
  Z-pencil, stride1 = 1    [nxh][ny][nz]  complex, nxh = nx // 2 + 1
  Z-pencil, stride1 = 0    [nz][ny][nxh]  complex
Forward and backward are unnormalised: btran(ftran(u)) = nx*ny*nz * u.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpencilfft.so")

PF_OK = 0
PF_EINVAL = -1
PF_EUNSUPPORTED = -2
PF_EALIGN = -3
PF_EALIAS = -4
PF_ENOMEM = -5
PF_EWORKSPACE = -6
PF_EHIP = -7
PF_ETIMEOUT = -8

PF_F32, PF_F64 = 0, 1
PF_PLAIN, PF_MFMA_FP16X2, PF_MFMA_BF16X2 = 0, 1, 2
PF_THIRD_FFT, PF_THIRD_EMPTY, PF_THIRD_CHEB = 0, 1, 2
PF_PENCIL_X, PF_PENCIL_Y, PF_PENCIL_Z = 0, 1, 2
PF_DIR_FORWARD, PF_DIR_BACKWARD = 0, 1
PF_BATCH_SERIAL, PF_BATCH_FUSED, PF_BATCH_GRAPH, PF_BATCH_STREAMS = 0, 1, 2, 4
PF_BATCH_NSTREAMS = 4
PF_WS_BLOCKED, PF_WS_TRANSPOSED = 0, 1
PF_PROBE_COPY, PF_PROBE_TILES, PF_PROBE_TILES_INPLACE = 0, 1, 2

EXPORTED = (
    "pf_layout_init", "pf_check", "pf_query_dims", "pf_setup", "pf_get_dims", "pf_workspace_bytes",
    "pf_set_workspace", "pf_ftran_r2c", "pf_btran_c2r", "pf_destroy", "pf_strerror", "pf_num_passes",
    "pf_run_pass", "pf_pass_name", "pf_pass_bytes", "pf_set_timing", "pf_get_timing", "pf_copy",
    "pf_batch_setup", "pf_batch_offset", "pf_batch_bytes", "pf_batch_set_mode", "pf_batch_ftran_r2c",
    "pf_batch_btran_c2r", "pf_batch_destroy", "pf_spectral_step", "pf_exec_noalloc", "pf_check_status",
    "pf_probe", "pf_pass_kernel", "pf_workspace_layout",
)


class PfError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {pf_strerror(code)} (code {code})")
        self.code = code


class pf_layout(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int) for name in (
        "m1", "m2", "stride1", "useeven", "precision", "math", "inplace", "third", "share_only", "r1", "r2",
        "fused_xy")]


class pf_tune(ctypes.Structure):
    _fields_ = [("radix_order", ctypes.c_int * 3), ("tile", ctypes.c_int * 3)]


@dataclass
class Layout:
    """Plan options; field meanings as in include/pencilfft.h."""
    m1: int = 1
    m2: int = 1
    stride1: int = 1
    useeven: int = 0
    precision: int = PF_F32
    math: int = PF_PLAIN
    inplace: int = 0
    third: int = PF_THIRD_FFT
    share_only: int = 0
    r1: int = 0
    r2: int = 0
    fused_xy: int = 0

    def c(self) -> pf_layout:
        return pf_layout(*[int(getattr(self, f[0])) for f in pf_layout._fields_])


_lib = None
_ip3 = ctypes.c_int * 3


def lib():
    """Load libpencilfft.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1905_02803_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
        lp = ctypes.POINTER(pf_layout)
        ip = ctypes.POINTER(ctypes.c_int)
        sig = {
            "pf_layout_init": (None, [lp]),
            "pf_check": (i, [i, i, i, lp]),
            "pf_query_dims": (i, [i, i, i, lp, i, i, i, ip, ip, ip]),
            "pf_setup": (i, [i, i, i, lp, ctypes.POINTER(vp)]),
            "pf_get_dims": (i, [vp, i, i, i, ip, ip, ip]),
            "pf_workspace_bytes": (sz, [vp]),
            "pf_set_workspace": (i, [vp, vp, sz]),
            "pf_ftran_r2c": (i, [vp, vp, vp, vp]),
            "pf_btran_c2r": (i, [vp, vp, vp, vp]),
            "pf_exec_noalloc": (i, [vp, i, vp, vp, vp]),
            "pf_check_status": (i, [vp]),
            "pf_probe": (i, [i, vp, vp, sz, vp]),
            "pf_destroy": (i, [vp]),
            "pf_strerror": (ctypes.c_char_p, [i]),
            "pf_num_passes": (i, [vp, i]),
            "pf_run_pass": (i, [vp, i, i, vp, vp, vp]),
            "pf_pass_name": (ctypes.c_char_p, [vp, i, i]),
            "pf_pass_kernel": (ctypes.c_char_p, [vp, i, i]),
            "pf_workspace_layout": (i, [vp, i]),
            "pf_pass_bytes": (ctypes.c_double, [vp, i, i]),
            "pf_set_timing": (i, [vp, i]),
            "pf_copy": (i, [vp, vp, sz, vp]),
            "pf_get_timing": (i, [vp, i, i, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong)]),
            "pf_batch_setup": (i, [i, ip, lp, ctypes.POINTER(pf_tune), ctypes.POINTER(vp)]),
            "pf_batch_offset": (sz, [vp, i, i]),
            "pf_batch_bytes": (sz, [vp, i]),
            "pf_batch_set_mode": (i, [vp, i]),
            "pf_batch_ftran_r2c": (i, [vp, vp, vp, vp]),
            "pf_batch_btran_c2r": (i, [vp, vp, vp, vp]),
            "pf_batch_destroy": (i, [vp]),
            "pf_spectral_step": (i, [vp, vp, vp, vp, i, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _raise(code: int, what: str) -> None:
    if code != PF_OK:
        raise PfError(code, what)


# ---- one-to-one wrappers of the C ABI -------------------------------------

def pf_strerror(code: int) -> str:
    return lib().pf_strerror(int(code)).decode()


def pf_layout_init() -> Layout:
    c = pf_layout()
    lib().pf_layout_init(ctypes.byref(c))
    return Layout(*[getattr(c, f[0]) for f in pf_layout._fields_])


def pf_check(nx: int, ny: int, nz: int, layout: Layout | None = None) -> int:
    """Host-only validation; returns the status code (0 = accepted)."""
    c = (layout or Layout()).c()
    return int(lib().pf_check(nx, ny, nz, ctypes.byref(c)))


def pf_query_dims(nx, ny, nz, layout, pencil, r1=0, r2=0):
    """Host-only Table 1 block of rank (r1, r2): (start, size, order) along (X, Y, Z)."""
    c = (layout or Layout()).c()
    st, sz, od = _ip3(), _ip3(), _ip3()
    _raise(lib().pf_query_dims(nx, ny, nz, ctypes.byref(c), pencil, r1, r2, st, sz, od), "pf_query_dims")
    return tuple(st), tuple(sz), tuple(od)


def pf_setup(nx: int, ny: int, nz: int, layout: Layout | None = None) -> int:
    c = (layout or Layout()).c()
    h = ctypes.c_void_p()
    _raise(lib().pf_setup(nx, ny, nz, ctypes.byref(c), ctypes.byref(h)), "pf_setup")
    return h.value


def pf_destroy(h) -> None:
    _raise(lib().pf_destroy(h), "pf_destroy")


def pf_ftran_r2c(h, in_ptr: int, out_ptr: int, stream: int = 0) -> None:
    _raise(lib().pf_ftran_r2c(h, in_ptr, out_ptr, stream), "pf_ftran_r2c")


def pf_btran_c2r(h, in_ptr: int, out_ptr: int, stream: int = 0) -> None:
    _raise(lib().pf_btran_c2r(h, in_ptr, out_ptr, stream), "pf_btran_c2r")


PF_NOALLOC_MAX_BYTES = 256 << 20


def pf_exec_noalloc(h, direction: int, in_ptr: int, out_ptr: int, stream: int = 0) -> None:
    """Transform with the library's static device scratch as the workspace (no allocation)."""
    _raise(lib().pf_exec_noalloc(h, direction, in_ptr, out_ptr, stream), "pf_exec_noalloc")


def pf_probe(kind: int, dst_ptr: int, src_ptr: int, nbytes: int, stream: int = 0) -> None:
    """Bandwidth probe kernels (PF_PROBE_*): copies in the transform passes' access shapes."""
    _raise(lib().pf_probe(kind, dst_ptr, src_ptr, nbytes, stream), "pf_probe")


def pf_check_status(h) -> None:
    """Wait for the device; raise PfError(PF_ETIMEOUT) if a fused pass of the plan hit its wait bound."""
    _raise(lib().pf_check_status(h), "pf_check_status")


def pf_run_pass(h, direction: int, pass_index: int, in_ptr: int, out_ptr: int, stream: int = 0) -> None:
    _raise(lib().pf_run_pass(h, direction, pass_index, in_ptr, out_ptr, stream), "pf_run_pass")


def pf_workspace_bytes(h) -> int:
    return int(lib().pf_workspace_bytes(h))


def pf_set_workspace(h, ptr: int, nbytes: int) -> None:
    _raise(lib().pf_set_workspace(h, ptr, nbytes), "pf_set_workspace")


def pf_num_passes(h, direction: int) -> int:
    return int(lib().pf_num_passes(h, direction))


def pf_pass_name(h, direction: int, pass_index: int) -> str:
    return lib().pf_pass_name(h, direction, pass_index).decode()


def pf_pass_kernel(h, direction: int, pass_index: int) -> str:
    return lib().pf_pass_kernel(h, direction, pass_index).decode()


def pf_workspace_layout(h, direction: int) -> int:
    r = lib().pf_workspace_layout(h, direction)
    _raise(r if r < 0 else 0, "pf_workspace_layout")
    return r


def pf_pass_bytes(h, direction: int, pass_index: int) -> float:
    return float(lib().pf_pass_bytes(h, direction, pass_index))


def pf_set_timing(h, enable: bool) -> None:
    _raise(lib().pf_set_timing(h, int(bool(enable))), "pf_set_timing")


def pf_get_timing(h, direction: int, pass_index: int):
    ms = ctypes.c_double()
    n = ctypes.c_longlong()
    _raise(lib().pf_get_timing(h, direction, pass_index, ctypes.byref(ms), ctypes.byref(n)), "pf_get_timing")
    return ms.value, n.value


def pf_copy(dst_ptr: int, src_ptr: int, nbytes: int, stream: int = 0) -> None:
    """Plain device copy (the HBM roofline probe)."""
    _raise(lib().pf_copy(dst_ptr, src_ptr, nbytes, stream), "pf_copy")


def pf_get_dims(h, pencil, r1=0, r2=0):
    st, sz, od = _ip3(), _ip3(), _ip3()
    _raise(lib().pf_get_dims(h, pencil, r1, r2, st, sz, od), "pf_get_dims")
    return tuple(st), tuple(sz), tuple(od)


# ---- convenience wrapper ----------------------------------------------------

def _stream_handle(stream) -> int:
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


class Plan:
    """A plan for one grid; tensors in, tensors out, on torch's current stream."""

    def __init__(self, nx: int, ny: int, nz: int, layout: Layout | None = None, **opts):
        self.layout = layout or Layout(**opts)
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.nxh = self.nx // 2 + 1
        self.handle = pf_setup(self.nx, self.ny, self.nz, self.layout)

    # shapes and dtypes
    @property
    def real_dtype(self):
        import torch

        return torch.float64 if self.layout.precision == PF_F64 else torch.float32

    @property
    def complex_dtype(self):
        import torch

        return torch.complex128 if self.layout.precision == PF_F64 else torch.complex64

    def _block_shape(self, pencil):
        """C shape of rank (r1, r2)'s block of a pencil (share-only plans), slowest first."""
        _, size, order = pf_query_dims(self.nx, self.ny, self.nz, self.layout, pencil, self.layout.r1,
                                       self.layout.r2)
        return (size[order[2]], size[order[1]], size[order[0]])

    @property
    def real_shape(self):
        if self.layout.share_only:
            return self._block_shape(PF_PENCIL_X)
        return (self.nz, self.ny, self.nx)

    @property
    def complex_shape(self):
        if self.layout.share_only:
            return self._block_shape(PF_PENCIL_Z)
        if self.layout.stride1:
            return (self.nxh, self.ny, self.nz)
        return (self.nz, self.ny, self.nxh)

    def empty_real(self, device="cuda"):
        import torch

        return torch.empty(self.real_shape, dtype=self.real_dtype, device=device)

    def empty_complex(self, device="cuda"):
        import torch

        return torch.empty(self.complex_shape, dtype=self.complex_dtype, device=device)

    def _check_tensor(self, t, shape, dtype, what):
        if not t.is_cuda or t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError(f"{what} must be a contiguous {dtype} CUDA tensor of shape {shape}, got "
                             f"{t.dtype} {tuple(t.shape)} on {t.device}")

    def ftran(self, u, out=None, stream=None):
        """Forward R2C: real [nz][ny][nx] -> complex Z-pencil (returned)."""
        self._check_tensor(u, self.real_shape, self.real_dtype, "input")
        if out is None:
            out = self.empty_complex(u.device)
        self._check_tensor(out, self.complex_shape, self.complex_dtype, "output")
        pf_ftran_r2c(self.handle, u.data_ptr(), out.data_ptr(), _stream_handle(stream))
        return out

    def btran(self, U, out=None, stream=None):
        """Backward C2R: complex Z-pencil -> real [nz][ny][nx] (unnormalised)."""
        self._check_tensor(U, self.complex_shape, self.complex_dtype, "input")
        if out is None:
            out = self.empty_real(U.device)
        self._check_tensor(out, self.real_shape, self.real_dtype, "output")
        pf_btran_c2r(self.handle, U.data_ptr(), out.data_ptr(), _stream_handle(stream))
        return out

    @property
    def inplace_bytes(self) -> int:
        """Bytes an in-place buffer must hold: max(real, complex) of the plan's arrays."""
        rs = 8 if self.layout.precision == PF_F64 else 4
        nreal = nc = 1
        for v in self.real_shape:
            nreal *= v
        for v in self.complex_shape:
            nc *= v
        return max(nreal * rs, nc * 2 * rs)

    @staticmethod
    def _check_buffer(t, nbytes, what):
        """A contiguous CUDA tensor, 16-byte aligned, whose storage holds nbytes from its data pointer."""
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{what} must be a contiguous CUDA tensor, got {tuple(t.shape)} on {t.device}")
        if t.data_ptr() % 16:
            raise ValueError(f"{what} must be 16-byte aligned")
        st = t.untyped_storage()
        have = st.data_ptr() + st.nbytes() - t.data_ptr()
        if have < nbytes:
            raise ValueError(f"{what} holds {have} bytes from its data pointer, the plan needs {nbytes}")

    def ftran_inplace(self, buf, stream=None):
        """In-place forward on a buffer tensor holding max(real, complex) bytes."""
        self._check_buffer(buf, self.inplace_bytes, "in-place buffer")
        pf_ftran_r2c(self.handle, buf.data_ptr(), buf.data_ptr(), _stream_handle(stream))
        return buf

    def btran_inplace(self, buf, stream=None):
        """In-place backward on a buffer tensor holding max(real, complex) bytes."""
        self._check_buffer(buf, self.inplace_bytes, "in-place buffer")
        pf_btran_c2r(self.handle, buf.data_ptr(), buf.data_ptr(), _stream_handle(stream))
        return buf

    def run_pass(self, direction, index, src, dst, stream=None):
        pf_run_pass(self.handle, direction, index, src.data_ptr(), dst.data_ptr(), _stream_handle(stream))
        return dst

    @property
    def workspace_bytes(self) -> int:
        return pf_workspace_bytes(self.handle)

    def num_passes(self, direction: int) -> int:
        return pf_num_passes(self.handle, direction)

    def pass_name(self, direction: int, index: int) -> str:
        return pf_pass_name(self.handle, direction, index)

    def pass_kernel(self, direction: int, index: int) -> str:
        return pf_pass_kernel(self.handle, direction, index)

    def workspace_layout(self, direction: int) -> int:
        return pf_workspace_layout(self.handle, direction)

    def pass_bytes(self, direction: int, index: int) -> float:
        return pf_pass_bytes(self.handle, direction, index)

    def set_timing(self, enable: bool) -> None:
        pf_set_timing(self.handle, enable)

    def get_timing(self, direction: int, index: int):
        return pf_get_timing(self.handle, direction, index)

    def dims(self, pencil, r1=0, r2=0):
        return pf_get_dims(self.handle, pencil, r1, r2)

    def destroy(self) -> None:
        if getattr(self, "handle", None):
            pf_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def pf_spectral_step(h, in_ptr: int, spec_ptr: int, out_ptr: int, adjoint: int = 0, stream: int = 0) -> None:
    _raise(lib().pf_spectral_step(h, in_ptr, spec_ptr, out_ptr, int(adjoint), stream), "pf_spectral_step")


def spectral_step(plan, u, spec=None, adjoint: bool = False, stream=None):
    """The plan's spectral step L (or its adjoint) on a real [nz][ny][nx] CUDA tensor (not differentiable;
    see SpectralStep)."""
    import torch

    plan._check_tensor(u, plan.real_shape, plan.real_dtype, "input")
    if spec is None:
        spec = plan.empty_complex(u.device)
    out = torch.empty_like(u)
    pf_spectral_step(plan.handle, u.data_ptr(), spec.data_ptr(), out.data_ptr(), int(adjoint), _stream_handle(stream))
    return out


def _spectral_function():
    import torch

    class SpectralStep(torch.autograd.Function):
        """Differentiable spectral step: forward L u, backward L^T g (both hand-written GPU passes)."""

        @staticmethod
        def forward(ctx, u, plan):
            ctx.plan = plan
            return spectral_step(plan, u.contiguous())

        @staticmethod
        def backward(ctx, g):
            return spectral_step(ctx.plan, g.contiguous(), adjoint=True), None

    return SpectralStep


def spectral_step_autograd(u, plan):
    """L u with gradients through the hand-written adjoint."""
    global _SPEC_FN
    if _SPEC_FN is None:
        _SPEC_FN = _spectral_function()
    return _SPEC_FN.apply(u, plan)


_SPEC_FN = None


def pf_batch_setup(dims, layout: Layout | None = None, tune=None) -> int:
    """dims: sequence of (nx, ny, nz); tune: None or a sequence of ((rx, ry, rz), (tx, ty, tz)) per transform."""
    n = len(dims)
    flat = (ctypes.c_int * (3 * n))(*[int(v) for d in dims for v in d])
    c = (layout or Layout()).c()
    tp = None
    if tune is not None:
        arr = (pf_tune * n)()
        for i, (ro, tl) in enumerate(tune):
            arr[i].radix_order[:] = [int(v) for v in ro]
            arr[i].tile[:] = [int(v) for v in tl]
        tp = arr
    h = ctypes.c_void_p()
    _raise(lib().pf_batch_setup(n, flat, ctypes.byref(c), tp, ctypes.byref(h)), "pf_batch_setup")
    return h.value


def pf_batch_offset(h, which: int, i: int) -> int:
    v = lib().pf_batch_offset(h, which, i)
    if v == ctypes.c_size_t(-1).value:
        raise PfError(PF_EINVAL, "pf_batch_offset")
    return v


def pf_batch_bytes(h, which: int) -> int:
    return lib().pf_batch_bytes(h, which)


def pf_batch_set_mode(h, mode: int) -> None:
    _raise(lib().pf_batch_set_mode(h, mode), "pf_batch_set_mode")


def pf_batch_ftran_r2c(h, in_ptr: int, out_ptr: int, stream: int = 0) -> None:
    _raise(lib().pf_batch_ftran_r2c(h, in_ptr, out_ptr, stream), "pf_batch_ftran_r2c")


def pf_batch_btran_c2r(h, in_ptr: int, out_ptr: int, stream: int = 0) -> None:
    _raise(lib().pf_batch_btran_c2r(h, in_ptr, out_ptr, stream), "pf_batch_btran_c2r")


def pf_batch_destroy(h) -> None:
    _raise(lib().pf_batch_destroy(h), "pf_batch_destroy")


class Batch:
    """Many 3D transforms of different sizes; user arrays are two flat device buffers (REAL, COMPLEX)."""

    def __init__(self, dims, layout: Layout | None = None, tune=None, mode: int = PF_BATCH_FUSED):
        self.dims = [tuple(int(v) for v in d) for d in dims]
        self.layout = layout or Layout()
        self.handle = pf_batch_setup(self.dims, self.layout, tune)
        self.set_mode(mode)

    def set_mode(self, mode: int) -> None:
        pf_batch_set_mode(self.handle, mode)
        self.mode = mode

    @property
    def real_dtype(self):
        import torch

        return torch.float64 if self.layout.precision == PF_F64 else torch.float32

    @property
    def complex_dtype(self):
        import torch

        return torch.complex128 if self.layout.precision == PF_F64 else torch.complex64

    def empty(self, which: int, device="cuda"):
        """A flat byte-sized buffer for REAL (0) or COMPLEX (1) data, 256-byte aligned by torch's allocator."""
        import torch

        return torch.empty(pf_batch_bytes(self.handle, which), dtype=torch.uint8, device=device)

    def view(self, buf, which: int, i: int):
        """Transform i's array inside a batch buffer: [nz][ny][nx] real or its Z-pencil complex."""
        nx, ny, nz = self.dims[i]
        off = pf_batch_offset(self.handle, which, i)
        if which == 0:
            shape, dt = (nz, ny, nx), self.real_dtype
        else:
            nxh = nx // 2 + 1
            shape, dt = ((nxh, ny, nz) if self.layout.stride1 else (nz, ny, nxh)), self.complex_dtype
        n = shape[0] * shape[1] * shape[2] * dt.itemsize
        return buf[off:off + n].view(dt).view(shape)

    def ftran(self, real_buf, complex_buf, stream=None):
        pf_batch_ftran_r2c(self.handle, real_buf.data_ptr(), complex_buf.data_ptr(), _stream_handle(stream))
        return complex_buf

    def btran(self, complex_buf, real_buf, stream=None):
        pf_batch_btran_c2r(self.handle, complex_buf.data_ptr(), real_buf.data_ptr(), _stream_handle(stream))
        return real_buf

    def destroy(self) -> None:
        if getattr(self, "handle", None):
            pf_batch_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def workspace_to_half_spectrum(ws, nx: int, ny: int, nz: int):
    """View a workspace buffer (the layout between passes, see pf_run_pass) as [nz][ny][nxh].

    Pure index permutation for tests; ws is a tensor of the plan's complex dtype
    with nz * nkb * ny * B elements.
    """
    nxh = nx // 2 + 1
    B = 128 // ws.element_size()
    nkb = (nxh + B - 1) // B
    w = ws[: nz * nkb * ny * B].reshape(nz, nkb, ny, B).permute(0, 2, 1, 3).reshape(nz, ny, nkb * B)
    return w[:, :, :nxh]


def transposed_workspace_to_half_spectrum(ws, nx: int, ny: int, nz: int):
    """View a transposed workspace (PF_WS_TRANSPOSED: [nz][nxh][ny]) as [nz][ny][nxh]; for tests."""
    nxh = nx // 2 + 1
    return ws[: nz * nxh * ny].reshape(nz, nxh, ny).permute(0, 2, 1)


def half_spectrum_to_workspace(U, ws):
    """Inverse of workspace_to_half_spectrum: scatter U[nz][ny][nxh] into the workspace layout."""
    nz, ny, nxh = U.shape
    B = 128 // ws.element_size()
    nkb = (nxh + B - 1) // B
    w = ws[: nz * nkb * ny * B].reshape(nz, nkb, ny, B)
    full = U.new_zeros((nz, ny, nkb * B))
    full[:, :, :nxh] = U
    w.copy_(full.reshape(nz, ny, nkb, B).permute(0, 2, 1, 3))
    return ws
