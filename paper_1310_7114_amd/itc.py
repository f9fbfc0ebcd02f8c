"""Python binding of libitc_lattice.so: argument marshalling only.

Every step of the clustering runs in the HIP kernels behind the C ABI
(include/itc_lattice.h). PyTorch supplies device memory and the current
stream. There is no CPU fallback: if the library or a GPU is missing, the
calls raise.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
# the in-tree library; ITC_LIB_PATH names another build of it (the host-sanitized one of the ABI tests)
LIB_PATH = os.environ.get("ITC_LIB_PATH") or os.path.join(_PKG, "libitc_lattice.so")

ITC_U8, ITC_F32, ITC_F64 = 0, 1, 2
ITC_FIT_NONFINITE_SUMS, ITC_FIT_NONFINITE_STEP, ITC_FIT_NONFINITE_D = 1, 2, 4
ITC_MAX_CODEVECTORS = 1024
STATUS = {0: "ITC_OK", 1: "ITC_E_NULL", 2: "ITC_E_ARG", 3: "ITC_E_UNSUPPORTED", 4: "ITC_E_DEVICE"}


class ItcError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{STATUS.get(status, status)}: {detail}")
        self.status = status
        self.detail = detail


class Desc(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("width", ctypes.c_int32), ("pitch", ctypes.c_int64),
                ("weight_dtype", ctypes.c_int32), ("real_dtype", ctypes.c_int32),
                ("weight_scale", ctypes.c_double), ("sigma", ctypes.c_double),
                ("radius", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Batch(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("desc", ctypes.POINTER(Desc)),
                ("weight_off", ctypes.POINTER(ctypes.c_int64)), ("map_off", ctypes.POINTER(ctypes.c_int64)),
                ("M", ctypes.POINTER(ctypes.c_int32)), ("w_off", ctypes.POINTER(ctypes.c_int64)),
                ("iters", ctypes.POINTER(ctypes.c_int32))]


class VolumeDesc(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("radius", ctypes.c_int32), ("row_pitch", ctypes.c_int64), ("slice_pitch", ctypes.c_int64),
                ("weight_dtype", ctypes.c_int32), ("reserved", ctypes.c_int32), ("weight_scale", ctypes.c_double),
                ("sigma", ctypes.c_double)]


_lib = None
_P = ctypes.c_void_p
_DP = ctypes.POINTER(Desc)

# name -> (restype, argtypes)
SIGNATURES = {
    "itc_lattice_radius": (ctypes.c_int32, [_DP]),
    "itc_lattice_plane_elems": (ctypes.c_int64, [_DP]),
    "itc_lattice_maps_bytes": (ctypes.c_size_t, [_DP]),
    "itc_lattice_precompute": (ctypes.c_int, [_DP, _P, _P, _P, _P]),
    "itc_lattice_fit": (ctypes.c_int, [_DP, _P, _P, ctypes.c_int32, _P, ctypes.c_int32, ctypes.c_double,
                                       _P, _P, _P, _P]),
    "itc_lattice_fit_wide": (ctypes.c_int, [_DP, _P, _P, ctypes.c_int32, _P, ctypes.c_int32, ctypes.c_double,
                                            _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "itc_lattice_fit_wide_work_bytes": (ctypes.c_size_t, [ctypes.c_int32]),
    "itc_lattice_divergence": (ctypes.c_int, [_DP, _P, _P, ctypes.c_int32, _P, _P, _P]),
    "itc_lattice_divergence_backward": (ctypes.c_int, [_DP, _P, _P, ctypes.c_int32, _P, _P, _P, _P, _P]),
    "itc_lattice_plan_create": (ctypes.c_int, [ctypes.POINTER(Batch), ctypes.POINTER(ctypes.c_void_p)]),
    "itc_lattice_precompute_batched": (ctypes.c_int, [_P, _P, _P, _P]),
    "itc_lattice_fit_batched": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, _P, _P, _P, _P, _P, _P]),
    "itc_lattice_run_batched": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_double, _P, _P, _P, _P, _P, _P]),
    "itc_lattice_divergence_backward_batched": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "itc_lattice_chamfer": (ctypes.c_int, [_DP, _P, ctypes.c_int32, ctypes.c_int32, _P, _P]),
    "itc_lattice_label": (ctypes.c_int, [_DP, _P, ctypes.c_int32, _P, _P, _P]),
    "itc_lattice_recursive_maps_bytes": (ctypes.c_size_t, [_DP]),
    "itc_volume_maps_bytes": (ctypes.c_size_t, [ctypes.POINTER(VolumeDesc)]),
    "itc_volume_work_bytes": (ctypes.c_size_t, [ctypes.POINTER(VolumeDesc)]),
    "itc_volume_precompute": (ctypes.c_int, [ctypes.POINTER(VolumeDesc), _P, _P, _P, _P, _P]),
    "itc_volume_fit": (ctypes.c_int, [ctypes.POINTER(VolumeDesc), _P, _P, ctypes.c_int32, _P, ctypes.c_int32,
                                      ctypes.c_double, _P, _P, _P, _P]),
    "itc_lattice_recursive_work_bytes": (ctypes.c_size_t, [_DP]),
    "itc_lattice_precompute_recursive": (ctypes.c_int, [_DP, _P, _P, _P, _P, _P]),
    "itc_lattice_label_batched": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "itc_lattice_literal_work_bytes": (ctypes.c_size_t, [_DP, ctypes.c_int32, ctypes.c_double, ctypes.c_int32]),
    "itc_lattice_literal_fit": (ctypes.c_int, [_DP, _P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, _P,
                                               ctypes.c_int32, ctypes.c_double, _P, _P, _P, _P, _P]),
    "itc_lattice_literal_fit_noalloc": (ctypes.c_int, [_DP, _P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                                       _P, ctypes.c_int32, ctypes.c_double, _P, _P, _P, _P]),
    "itc_lattice_literal_density_work_bytes": (ctypes.c_size_t, [_DP, ctypes.c_int32, ctypes.c_double,
                                                                 ctypes.c_int32]),
    "itc_lattice_literal_fit_density": (ctypes.c_int, [_DP, _P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                                       _P, ctypes.c_int32, ctypes.c_double, _P, _P, _P, _P, _P]),
    "itc_lattice_chamfer_batched": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_int32, _P, _P]),
    "itc_lattice_plan_size": (ctypes.c_int32, [_P]),
    "itc_lattice_plan_conv_classes": (ctypes.c_int32, [_P]),
    "itc_lattice_plan_conv_launches": (ctypes.c_int32, [_P]),
    "itc_lattice_plan_conv_class": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, _P]),
    "itc_lattice_plan_set_conv_shape": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "itc_lattice_plan_destroy": (None, [_P]),
    "itc_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "itc_last_error": (ctypes.c_char_p, []),
}


def load(path: str = LIB_PATH):
    """Loads the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        raise ItcError(status, load().itc_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


_WDT = {torch.uint8: ITC_U8, torch.float32: ITC_F32, torch.float64: ITC_F64}
_RDT = {torch.float32: ITC_F32, torch.float64: ITC_F64}


def radius_for(sigma: float) -> int:
    """Default truncation radius ceil(3 sigma)."""
    return int(math.ceil(3.0 * sigma - 1e-12))


def make_desc(H: int, W: int, sigma: float, weight_dtype=torch.uint8, real_dtype=torch.float32,
              scale: float = 1.0, radius: int = 0, pitch: Optional[int] = None) -> Desc:
    return Desc(int(H), int(W), int(W if pitch is None else pitch), _WDT[weight_dtype], _RDT[real_dtype],
                float(scale), float(sigma), int(radius), 0)


def maps_bytes(desc: Desc) -> int:
    n = load().itc_lattice_maps_bytes(ctypes.byref(desc))
    if n == 0:
        raise ItcError(2, load().itc_last_error().decode())
    return int(n)


def plane_elems(desc: Desc) -> int:
    return int(load().itc_lattice_plane_elems(ctypes.byref(desc)))


MAP_PANEL = 16  # columns per panel of a map plane


def panel_view(flat: torch.Tensor, H: int, W: int) -> torch.Tensor:
    """An (H, W) strided view of one map plane stored in panels of 16 columns
    (element (u, v) at ((v // 16) * H + u) * 16 + v % 16); the panels are a
    (panels, H, 16) array, so the view is a permute and reshape (no arithmetic)."""
    npan = (W + MAP_PANEL - 1) // MAP_PANEL
    return flat[: npan * H * MAP_PANEL].view(npan, H, MAP_PANEL).permute(1, 0, 2).reshape(H, npan * MAP_PANEL)[:, :W]


@dataclass
class Maps:
    """Device maps of one image: buffer (bytes), S_X, and the descriptor."""
    desc: Desc
    buf: torch.Tensor
    s_x: torch.Tensor
    real_dtype: torch.dtype

    def planes(self):
        """(A, M_u, M_v) as (H, W) tensors read out of the panel layout of the map buffer."""
        H, W = self.desc.height, self.desc.width
        n = plane_elems(self.desc)
        esz = torch.finfo(self.real_dtype).bits // 8
        flat = self.buf[: 3 * n * esz].view(self.real_dtype)
        return tuple(panel_view(flat[i * n:(i + 1) * n], H, W) for i in range(3))


def alloc_maps(desc: Desc, device="cuda") -> torch.Tensor:
    return torch.empty(maps_bytes(desc), dtype=torch.uint8, device=device)


def precompute(weights: torch.Tensor, sigma: float, scale: float = 1.0, radius: int = 0,
               real_dtype=torch.float32, out: Optional[Maps] = None) -> Maps:
    """Convolution maps A, M_u, M_v and S_X of a (H, W) weight image on the GPU."""
    if weights.dim() != 2:
        raise ValueError("weights must be (H, W)")
    if weights.stride(1) != 1:
        weights = weights.contiguous()
    H, W = weights.shape
    desc = make_desc(H, W, sigma, weights.dtype, real_dtype, scale, radius, pitch=weights.stride(0))
    if out is None:
        out = Maps(desc, alloc_maps(desc, weights.device),
                   torch.empty(1, dtype=torch.float64, device=weights.device), real_dtype)
    _check(load().itc_lattice_precompute(ctypes.byref(desc), _ptr(weights), _ptr(out.buf), _ptr(out.s_x),
                                         _stream()))
    out.desc = desc
    return out


def fit(maps: Maps, w_init: torch.Tensor, iters: int, theta: float = -1.0, trace: bool = True,
        w_out: Optional[torch.Tensor] = None):
    """Runs `iters` sweeps; returns (W, D trace or None, iterations done tensor)."""
    w_init = w_init.to(maps.real_dtype).contiguous()
    M = int(w_init.shape[0])
    if w_out is None:
        w_out = torch.empty_like(w_init)
    d_trace = torch.full((iters + 1,), float("nan"), dtype=torch.float64, device=w_init.device) if trace else None
    done = torch.zeros(1, dtype=torch.int32, device=w_init.device)
    _check(load().itc_lattice_fit(ctypes.byref(maps.desc), _ptr(maps.buf), _ptr(maps.s_x), M, _ptr(w_init),
                                  int(iters), float(theta), _ptr(w_out), _ptr(d_trace), _ptr(done), _stream()))
    return w_out, d_trace, done


def fit_wide_work_bytes(M: int) -> int:
    return int(load().itc_lattice_fit_wide_work_bytes(int(M)))


def fit_wide(maps: Maps, w_init: torch.Tensor, iters: int, theta: float = -1.0, trace: bool = True,
             w_out: Optional[torch.Tensor] = None, work: Optional[torch.Tensor] = None):
    """fit() over several workgroups, one launch per sweep (FP32 maps); `work`
    (uint8, fit_wide_work_bytes(M) bytes) is allocated when not given.
    Returns (W, D trace or None, iterations done tensor)."""
    w_init = w_init.to(torch.float32).contiguous()
    M = int(w_init.shape[0])
    if w_out is None:
        w_out = torch.empty_like(w_init)
    if work is None:
        work = torch.empty(fit_wide_work_bytes(M), dtype=torch.uint8, device=w_init.device)
    d_trace = torch.full((iters + 1,), float("nan"), dtype=torch.float64, device=w_init.device) if trace else None
    done = torch.zeros(1, dtype=torch.int32, device=w_init.device)
    _check(load().itc_lattice_fit_wide(ctypes.byref(maps.desc), _ptr(maps.buf), _ptr(maps.s_x), M, _ptr(w_init),
                                       int(iters), float(theta), _ptr(w_out), _ptr(d_trace), _ptr(done),
                                       _ptr(work), int(work.numel()), _stream()))
    return w_out, d_trace, done


def divergence(maps: Maps, w: torch.Tensor) -> torch.Tensor:
    """D of eq. (1) for codebook w, as a 1-element float64 device tensor."""
    w = w.to(maps.real_dtype).contiguous()
    d = torch.empty(1, dtype=torch.float64, device=w.device)
    _check(load().itc_lattice_divergence(ctypes.byref(maps.desc), _ptr(maps.buf), _ptr(maps.s_x),
                                         int(w.shape[0]), _ptr(w), _ptr(d), _stream()))
    return d


def divergence_backward(maps: Maps, w: torch.Tensor, grad_d: torch.Tensor, want_w=True, want_weights=True):
    """(dL/dw [M,2], dL/dh [H,W]) for dL/dD = grad_d (1-element float64 device tensor)."""
    w = w.to(maps.real_dtype).contiguous()
    gw = torch.empty_like(w) if want_w else None
    gI = torch.empty((maps.desc.height, maps.desc.width), dtype=maps.real_dtype, device=w.device) \
        if want_weights else None
    _check(load().itc_lattice_divergence_backward(ctypes.byref(maps.desc), _ptr(maps.buf), _ptr(maps.s_x),
                                                  int(w.shape[0]), _ptr(w), _ptr(grad_d.to(torch.float64)),
                                                  _ptr(gw), _ptr(gI), _stream()))
    return gw, gI


def chamfer(x: torch.Tensor, a: int = 3, b: int = 4, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Chamfer distance transform of a (H, W) binary uint8 device image: float32 (H, W) of exact
    integer chamfer costs (orthogonal step a, diagonal step b); T / a approximates pixels."""
    if x.dim() != 2 or x.dtype != torch.uint8:
        raise ValueError("x must be a (H, W) uint8 tensor")
    if x.stride(1) != 1:
        x = x.contiguous()
    H, W = x.shape
    desc = make_desc(H, W, 1.0, torch.uint8, torch.float32, 1.0, 0, pitch=x.stride(0))
    if out is None:
        out = torch.empty((H, x.stride(0)), dtype=torch.float32, device=x.device)
    _check(load().itc_lattice_chamfer(ctypes.byref(desc), _ptr(x), int(a), int(b), _ptr(out), _stream()))
    return out[:, :W]


def precompute_recursive(weights: torch.Tensor, sigma: float, scale: float = 1.0,
                         work: Optional[torch.Tensor] = None) -> Maps:
    """Maps A, M_u, M_v and S_X with the recursive Gaussian of width sigma (any sigma >= 0.5)."""
    if weights.dim() != 2:
        raise ValueError("weights must be (H, W)")
    if weights.stride(1) != 1:
        weights = weights.contiguous()
    H, W = weights.shape
    desc = make_desc(H, W, sigma, weights.dtype, torch.float32, scale, 1, pitch=weights.stride(0))
    nm = load().itc_lattice_recursive_maps_bytes(ctypes.byref(desc))
    nw = load().itc_lattice_recursive_work_bytes(ctypes.byref(desc))
    if nm == 0 or nw == 0:
        raise ItcError(2, load().itc_last_error().decode())
    if work is None or work.numel() < nw:
        work = torch.empty(nw, dtype=torch.uint8, device=weights.device)
    out = Maps(desc, torch.empty(nm, dtype=torch.uint8, device=weights.device),
               torch.empty(1, dtype=torch.float64, device=weights.device), torch.float32)
    _check(load().itc_lattice_precompute_recursive(ctypes.byref(desc), _ptr(weights), _ptr(out.buf),
                                                   _ptr(out.s_x), _ptr(work), _stream()))
    return out


class VolumeMaps:
    """Device maps A, M_s, M_u, M_v of a volume (FP32, each D x H x W) and S_X."""

    def __init__(self, desc, buf, s_x):
        self.desc, self.buf, self.s_x = desc, buf, s_x

    def planes(self):
        n = self.desc.depth * self.desc.height * self.desc.width
        f = self.buf[: 16 * n].view(torch.float32)
        shape = (self.desc.depth, self.desc.height, self.desc.width)
        return [f[i * n:(i + 1) * n].view(shape) for i in range(4)]


def volume_precompute(vol: torch.Tensor, sigma: float, scale: float = 1.0, radius: int = 0,
                      work: Optional[torch.Tensor] = None) -> VolumeMaps:
    """Maps of a (D, H, W) weight volume (3-D lattice)."""
    if vol.dim() != 3:
        raise ValueError("vol must be (D, H, W)")
    if vol.stride(2) != 1:
        vol = vol.contiguous()
    D, H, W = vol.shape
    desc = VolumeDesc(int(D), int(H), int(W), int(radius), int(vol.stride(1)), int(vol.stride(0)),
                      _WDT[vol.dtype], 0, float(scale), float(sigma))
    nm = load().itc_volume_maps_bytes(ctypes.byref(desc))
    nw = load().itc_volume_work_bytes(ctypes.byref(desc))
    if nm == 0 or nw == 0:
        raise ItcError(2, load().itc_last_error().decode())
    if work is None or work.numel() < nw:
        work = torch.empty(nw, dtype=torch.uint8, device=vol.device)
    out = VolumeMaps(desc, torch.empty(nm, dtype=torch.uint8, device=vol.device),
                     torch.empty(1, dtype=torch.float64, device=vol.device))
    _check(load().itc_volume_precompute(ctypes.byref(desc), _ptr(vol), _ptr(out.buf), _ptr(out.s_x), _ptr(work),
                                        _stream()))
    return out


def volume_fit(maps: VolumeMaps, w_init: torch.Tensor, iters: int, theta: float = -1.0, trace: bool = True):
    """Sweeps of eq. (4) on a volume: (W (M, 3) float32, D trace or None, sweeps done tensor)."""
    w_init = w_init.to(torch.float32).contiguous()
    M = int(w_init.shape[0])
    w_out = torch.empty_like(w_init)
    d_trace = torch.full((iters + 1,), float("nan"), dtype=torch.float64, device=w_init.device) if trace else None
    done = torch.zeros(1, dtype=torch.int32, device=w_init.device)
    _check(load().itc_volume_fit(ctypes.byref(maps.desc), _ptr(maps.buf), _ptr(maps.s_x), M, _ptr(w_init),
                                 int(iters), float(theta), _ptr(w_out), _ptr(d_trace), _ptr(done), _stream()))
    return w_out, d_trace, done


def label(weights: torch.Tensor, w: torch.Tensor, scale: float = 1.0, out: Optional[torch.Tensor] = None,
          real_dtype=torch.float32) -> torch.Tensor:
    """Segments: int32 (H, W) index of the nearest codevector for pixels of weight > 0, -1 elsewhere."""
    if weights.dim() != 2:
        raise ValueError("weights must be (H, W)")
    if weights.stride(1) != 1:
        weights = weights.contiguous()
    H, W = weights.shape
    desc = make_desc(H, W, 1.0, weights.dtype, real_dtype, scale, 0, pitch=weights.stride(0))
    w = w.to(real_dtype).contiguous()
    if out is None:
        out = torch.empty((H, weights.stride(0)), dtype=torch.int32, device=weights.device)
    _check(load().itc_lattice_label(ctypes.byref(desc), _ptr(weights), int(w.shape[0]), _ptr(w), _ptr(out),
                                    _stream()))
    return out[:, :W]


def fit_literal(weights: torch.Tensor, w_init: torch.Tensor, xi: float, omega: float, iters: int,
                theta: float = -1.0, scale: float = 1.0, radius_xi: int = 0, radius_omega: int = 0,
                trace: bool = True, work: Optional[torch.Tensor] = None):
    """Algorithm 1 with eq. (6) on the lattice. w_init: (M, 2) int32 lattice points (u, v).
    Returns (W int32 (M, 2), D trace or None, sweeps done tensor)."""
    if weights.dim() != 2:
        raise ValueError("weights must be (H, W)")
    if weights.stride(1) != 1:
        weights = weights.contiguous()
    H, W = weights.shape
    desc = make_desc(H, W, xi, weights.dtype, torch.float32, scale, radius_xi, pitch=weights.stride(0))
    w_init = w_init.to(torch.int32).contiguous()
    M = int(w_init.shape[0])
    nb = load().itc_lattice_literal_work_bytes(ctypes.byref(desc), M, float(omega), int(radius_omega))
    if nb == 0:
        raise ItcError(2, "invalid Algorithm 1 parameters: " + load().itc_last_error().decode())
    if work is None or work.numel() < nb:
        work = torch.empty(nb, dtype=torch.uint8, device=weights.device)
    w_out = torch.empty_like(w_init)
    d_trace = torch.full((iters + 1,), float("nan"), dtype=torch.float64, device=weights.device) if trace else None
    done = torch.zeros(1, dtype=torch.int32, device=weights.device)
    _check(load().itc_lattice_literal_fit(ctypes.byref(desc), _ptr(weights), float(omega), int(radius_omega), M,
                                          _ptr(w_init), int(iters), float(theta), _ptr(w_out), _ptr(d_trace),
                                          _ptr(done), _ptr(work), _stream()))
    return w_out, d_trace, done


def fit_literal_density(maps: Maps, w_init: torch.Tensor, omega: float, iters: int, theta: float = -1.0,
                        radius_omega: int = 0, trace: bool = True, work: Optional[torch.Tensor] = None):
    """Algorithm 1 from the density P = plane A of `maps` (precompute or precompute_recursive, any
    width). w_init: (M, 2) int32 lattice points. Returns (W int32 (M, 2), D trace or None, sweeps done)."""
    if maps.real_dtype != torch.float32:
        raise ValueError("Algorithm 1 runs on FP32 maps")
    w_init = w_init.to(torch.int32).contiguous()
    M = int(w_init.shape[0])
    nb = load().itc_lattice_literal_density_work_bytes(ctypes.byref(maps.desc), M, float(omega), int(radius_omega))
    if nb == 0:
        raise ItcError(2, "invalid Algorithm 1 parameters: " + load().itc_last_error().decode())
    if work is None or work.numel() < nb:
        work = torch.empty(nb, dtype=torch.uint8, device=w_init.device)
    w_out = torch.empty_like(w_init)
    d_trace = torch.full((iters + 1,), float("nan"), dtype=torch.float64, device=w_init.device) if trace else None
    done = torch.zeros(1, dtype=torch.int32, device=w_init.device)
    _check(load().itc_lattice_literal_fit_density(ctypes.byref(maps.desc), _ptr(maps.buf), float(omega),
                                                  int(radius_omega), M, _ptr(w_init), int(iters), float(theta),
                                                  _ptr(w_out), _ptr(d_trace), _ptr(done), _ptr(work), _stream()))
    return w_out, d_trace, done


def fit_literal_noalloc(weights: torch.Tensor, w_init: torch.Tensor, xi: float, omega: float, iters: int,
                        theta: float = -1.0, scale: float = 1.0, radius_xi: int = 0, radius_omega: int = 0,
                        trace: bool = True, w_out: Optional[torch.Tensor] = None, d_trace: Optional[torch.Tensor] = None,
                        done: Optional[torch.Tensor] = None):
    """fit_literal through the entry point that allocates nothing (the library's static work array);
    pass w_out, d_trace and done to make the call itself allocation-free."""
    if weights.dim() != 2:
        raise ValueError("weights must be (H, W)")
    if weights.stride(1) != 1:
        weights = weights.contiguous()
    H, W = weights.shape
    desc = make_desc(H, W, xi, weights.dtype, torch.float32, scale, radius_xi, pitch=weights.stride(0))
    w_init = w_init.to(torch.int32).contiguous()
    M = int(w_init.shape[0])
    if w_out is None:
        w_out = torch.empty_like(w_init)
    if trace and d_trace is None:
        d_trace = torch.full((iters + 1,), float("nan"), dtype=torch.float64, device=weights.device)
    if done is None:
        done = torch.zeros(1, dtype=torch.int32, device=weights.device)
    _check(load().itc_lattice_literal_fit_noalloc(ctypes.byref(desc), _ptr(weights), float(omega), int(radius_omega),
                                                  M, _ptr(w_init), int(iters), float(theta), _ptr(w_out),
                                                  _ptr(d_trace if trace else None), _ptr(done), _stream()))
    return w_out, (d_trace if trace else None), done


# ---------------------------------------------------------------------------
# batched form
# ---------------------------------------------------------------------------

class BatchPlan:
    """A batch of images packed in flat device buffers, and its C plan.

    images: sequence of (H, W) uint8/float tensors (host or device); ms: codevectors
    per image; sigmas, scales, iters: per image. The packed weights, maps and
    codebook buffers are allocated once here. `BatchPlan.for_stack` describes a
    contiguous (B, H, W) stack instead, whose weights are passed per call.
    """

    def __init__(self, images: Optional[Sequence[torch.Tensor]], ms: Sequence[int], sigmas: Sequence[float],
                 iters: Sequence[int], scales: Optional[Sequence[float]] = None,
                 radii: Optional[Sequence[int]] = None, device="cuda", _shapes=None, _dtype=None, _woffs=None,
                 _pitches=None):
        shapes = [tuple(im.shape) for im in images] if images is not None else list(_shapes)
        n = len(shapes)
        if n == 0:
            raise ValueError("empty batch")
        scales = [1.0] * n if scales is None else list(scales)
        radii = [0] * n if radii is None else list(radii)
        dt = images[0].dtype if images is not None else _dtype
        esz = torch.tensor([], dtype=dt).element_size()
        self.n = n
        self.dtype = dt
        self.shapes = shapes
        self.sigmas, self.scales, self.radii, self.iters_list = list(sigmas), scales, radii, [int(t) for t in iters]
        self.descs = (Desc * n)()
        # packed images: rows padded to a multiple of 16 elements (8-bit rows
        # start 4-byte aligned, as the matrix-core convolution needs), each
        # image at a 256-byte aligned offset; a stack keeps its own layout
        if _pitches is not None:
            self.pitches = [int(x) for x in _pitches]
        elif images is not None:
            self.pitches = [(W + 15) // 16 * 16 for (_, W) in shapes]
        else:
            self.pitches = [W for (_, W) in shapes]
        wo, mo, wf, mlist, it = [], [], [], [], []
        woff = moff = foff = 0
        for i, (H, W) in enumerate(shapes):
            if images is not None and images[i].dtype != dt:
                raise ValueError("all images of a batch share one storage dtype")
            pitch = self.pitches[i]
            self.descs[i] = make_desc(H, W, sigmas[i], dt, torch.float32, scales[i], radii[i], pitch=pitch)
            wo.append(woff if _woffs is None else int(_woffs[i]))
            woff += H * pitch * esz if images is None else (H * pitch * esz + 255) // 256 * 256
            mo.append(moff)
            moff += maps_bytes(self.descs[i])
            wf.append(foff)
            foff += int(ms[i])
            mlist.append(int(ms[i]))
            it.append(int(iters[i]))
        self.weight_off = (ctypes.c_int64 * n)(*wo)
        self.map_off = (ctypes.c_int64 * n)(*mo)
        self.w_off_arr = (ctypes.c_int64 * n)(*wf)
        self.M = (ctypes.c_int32 * n)(*mlist)
        self.iters = (ctypes.c_int32 * n)(*it)
        self.w_offsets = wf
        self.ms = mlist
        self.total_w = foff
        self.map_bytes_total = max(moff, 256)
        self.map_off_list = mo
        self.weights = None
        if images is not None:
            self.weights = torch.zeros(woff // esz, dtype=dt, device=device)
            for i, img in enumerate(images):
                self.image(self.weights, i).copy_(img.to(device))
        self.maps = torch.empty(self.map_bytes_total, dtype=torch.uint8, device=device)
        b = Batch(n, self.descs, self.weight_off, self.map_off, self.M, self.w_off_arr, self.iters)
        h = ctypes.c_void_p()
        _check(load().itc_lattice_plan_create(ctypes.byref(b), ctypes.byref(h)))
        self.handle = h

    @classmethod
    def for_stack(cls, B: int, H: int, W: int, M: int, sigma: float, iters: int = 0, dtype=torch.float32,
                  scale: float = 1.0, radius: int = 0, device="cuda") -> "BatchPlan":
        """Plan for a contiguous (B, H, W) weight stack and (B * M, 2) codebooks."""
        return cls(None, [M] * B, [sigma] * B, [iters] * B, [scale] * B, [radius] * B, device=device,
                   _shapes=[(H, W)] * B, _dtype=dtype)

    def chamfer(self, a: int = 3, b: int = 4, weights=None, out=None) -> torch.Tensor:
        """Chamfer transform of every (uint8, binary) image: a float32 buffer holding image i at element
        offset weight_off[i], with the images' pitch."""
        w = self._w(weights)
        if out is None:
            out = torch.empty(w.numel(), dtype=torch.float32, device=w.device)
        _check(load().itc_lattice_chamfer_batched(self.handle, _ptr(w), int(a), int(b), _ptr(out), _stream()))
        return out

    def label(self, w: torch.Tensor, weights=None, out=None) -> torch.Tensor:
        """Segments of every image for the packed FP32 codebooks `w`: an int32 buffer holding image i
        at element offset weight_off[i] / element size, at the images' pitch."""
        x = self._w(weights)
        if out is None:
            out = torch.empty(x.numel(), dtype=torch.int32, device=x.device)
        _check(load().itc_lattice_label_batched(self.handle, _ptr(x), _ptr(w), _ptr(out), _stream()))
        return out

    def weighted(self, a: int = 3) -> "BatchPlan":
        """A plan over the same images, codebooks, widths and sweeps whose weights are this plan's
        chamfer transforms (float32, as written by `chamfer`), scaled by 1/a (Section 5)."""
        if self.dtype != torch.uint8:
            raise ValueError("the chamfer weighting starts from uint8 images")
        return BatchPlan(None, self.ms, self.sigmas, self.iters_list, [1.0 / a] * self.n, self.radii,
                         device=self.maps.device, _shapes=self.shapes, _dtype=torch.float32,
                         _woffs=[4 * int(o) for o in self.weight_off], _pitches=self.pitches)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.itc_lattice_plan_destroy(h)
            self.handle = None

    def image(self, flat: torch.Tensor, i: int) -> torch.Tensor:
        """Image i of a flat buffer in the packed layout (the weights, a chamfer transform or labels:
        image i starts at element weight_off[i] / stored element size): an (H, W) view at its pitch."""
        H, W = self.shapes[i]
        off = int(self.weight_off[i]) // torch.tensor([], dtype=self.dtype).element_size()
        pitch = self.pitches[i]
        return flat[off: off + H * pitch].view(H, pitch)[:, :W]

    def pack_codebooks(self, ws: Sequence[torch.Tensor], device="cuda") -> torch.Tensor:
        out = torch.empty((self.total_w, 2), dtype=torch.float32, device=device)
        for i, w in enumerate(ws):
            out[self.w_offsets[i]: self.w_offsets[i] + self.ms[i]].copy_(torch.as_tensor(w).to(device, torch.float32))
        return out

    def unpack(self, flat: torch.Tensor, i: int) -> torch.Tensor:
        return flat[self.w_offsets[i]: self.w_offsets[i] + self.ms[i]]

    def new_maps(self) -> torch.Tensor:
        return torch.empty(self.map_bytes_total, dtype=torch.uint8, device=self.maps.device)

    def maps_of(self, i: int, maps: Optional[torch.Tensor] = None) -> Maps:
        maps = self.maps if maps is None else maps
        d = self.descs[i]
        nb = maps_bytes(d)
        buf = maps[self.map_off_list[i]: self.map_off_list[i] + nb]
        return Maps(d, buf, torch.empty(1, dtype=torch.float64, device=maps.device), torch.float32)

    def _w(self, weights):
        w = self.weights if weights is None else weights
        if w is None:
            raise ValueError("this plan holds no weights: pass them")
        return w

    def conv_classes(self):
        """Convolution classes of the plan: [{key, seg_rows, blocks_per_cu, max_blocks_per_cu}]."""
        lib = load()
        out = []
        for c in range(lib.itc_lattice_plan_conv_classes(self.handle)):
            v = [ctypes.c_int32() for _ in range(4)]
            _check(lib.itc_lattice_plan_conv_class(self.handle, c, *[ctypes.byref(x) for x in v]))
            out.append(dict(zip(("key", "seg_rows", "blocks_per_cu", "max_blocks_per_cu"), (x.value for x in v))))
        return out

    def conv_launches(self) -> int:
        """Kernel launches of one `precompute` (one for all 8-bit images of aligned rows)."""
        return int(load().itc_lattice_plan_conv_launches(self.handle))

    def set_conv_shape(self, key: int, seg_rows: int = 0, blocks_per_cu: int = 0):
        """Tile shape of one convolution class (0 = default); capture graphs after this."""
        torch.cuda.synchronize()
        _check(load().itc_lattice_plan_set_conv_shape(self.handle, int(key), int(seg_rows), int(blocks_per_cu)))

    def precompute(self, weights=None, maps=None):
        _check(load().itc_lattice_precompute_batched(self.handle, _ptr(self._w(weights)),
                                                     _ptr(self.maps if maps is None else maps), _stream()))

    def fit(self, w_init: torch.Tensor, w_out: torch.Tensor, s_x=None, d_out=None, iters_done=None,
            theta: float = -1.0, maps=None, status=None):
        """Fit of every image; `status` (int32 [n]) receives the ITC_FIT_NONFINITE_* bits per image."""
        _check(load().itc_lattice_fit_batched(self.handle, _ptr(self.maps if maps is None else maps), _ptr(w_init),
                                              float(theta), _ptr(w_out), _ptr(s_x), _ptr(d_out), _ptr(iters_done),
                                              _ptr(status), _stream()))

    def run(self, w_init: torch.Tensor, w_out: torch.Tensor, s_x=None, d_out=None, iters_done=None,
            theta: float = -1.0, weights=None, maps=None, status=None):
        _check(load().itc_lattice_run_batched(self.handle, _ptr(self._w(weights)),
                                              _ptr(self.maps if maps is None else maps), _ptr(w_init),
                                              float(theta), _ptr(w_out), _ptr(s_x), _ptr(d_out),
                                              _ptr(iters_done), _ptr(status), _stream()))

    def backward(self, w: torch.Tensor, s_x: torch.Tensor, grad_d: torch.Tensor, grad_w=None, grad_weights=None,
                 maps=None):
        _check(load().itc_lattice_divergence_backward_batched(
            self.handle, _ptr(self.maps if maps is None else maps), _ptr(s_x), _ptr(w),
            _ptr(grad_d.to(torch.float64).contiguous()), _ptr(grad_w), _ptr(grad_weights), _stream()))
