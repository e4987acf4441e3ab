"""Thin ctypes binding of the C ABI in include/rsf.h (same names).

Argument marshalling only: every step of the evolution runs in the HIP
kernels of librsf.so.  PyTorch supplies device memory (tensors) and streams;
the library never sees a torch type.  If librsf.so is missing or cannot be
loaded this module raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librsf.so")

RSF_NOT_READY = 1
RSF_OK = 0
RSF_ERR_INVALID_ARG = -1
RSF_ERR_OUT_OF_MEMORY = -2
RSF_ERR_DEVICE = -3
RSF_ERR_NONFINITE = -4
RSF_ERR_BUDGET = -5
RSF_ERR_INTERNAL = -6

RSF_F32 = 0
RSF_F16 = 1
RSF_BF16 = 2
RSF_U16 = 3

RSF_REG_DOUBLE_WELL = 0
RSF_REG_SINGLE_WELL = 1

RSF_FORCE_RSF = 0
RSF_FORCE_PAPER = 1

EXPORTS = ("rsf_create", "rsf_destroy", "rsf_last_error", "rsf_workspace_bytes",
           "rsf_evolve", "rsf_evolve_ex", "rsf_get_stats", "rsf_gauss3d", "rsf_probe",
           "rsf_profile_enable", "rsf_profile_read", "rsf_batch_workspace_bytes",
           "rsf_evolve_batch", "rsf_get_tile_stats", "rsf_autotune", "rsf_autotune_reset",
           "rsf_set_split_targets", "rsf_evolve_volume", "rsf_workspace_bytes_params",
           "rsf_batch_workspace_bytes_params", "rsf_seeds", "rsf_fast_sweep", "rsf_init_phi", "rsf_set_fusion",
           "rsf_server_create", "rsf_server_submit", "rsf_server_poll", "rsf_server_wait",
           "rsf_server_drain", "rsf_server_get_stats", "rsf_server_last_error",
           "rsf_server_destroy", "rsf_evolve_noalloc", "rsf_set_graphs", "rsf_stream_probe",
           "rsf_volume_workspace_bytes", "rsf_evolve_volume_ex", "rsf_init_workspace_bytes",
           "rsf_init_phi_ex", "rsf_set_fault", "rsf_fault_allocations", "rsf_seeds_ex",
           "rsf_seeds_workspace_bytes", "rsf_autotune_ex", "rsf_autotune_workspace_bytes")

RSF_NOALLOC_MAX_BYTES = 128 << 20

PASS_NAMES = ("setup", "z_heaviside", "xy_fits", "xy_force", "z_update", "reduce",
              "init_smooth", "init_hessian", "init_select", "init_sweep", "init_offset")


class RsfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"rsf status {status}: {msg}")
        self.status = status


class rsf_params(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_float), ("lambda1", ctypes.c_float),
                ("lambda2", ctypes.c_float), ("nu", ctypes.c_float), ("mu", ctypes.c_float),
                ("dt", ctypes.c_float), ("eps", ctypes.c_float), ("eta", ctypes.c_float),
                ("regulariser", ctypes.c_int), ("storage", ctypes.c_int),
                ("force", ctypes.c_int), ("sigma2", ctypes.c_float)]


class rsf_stats(ctypes.Structure):
    _fields_ = [("iters_requested", ctypes.c_int), ("iters_run", ctypes.c_int),
                ("last_sum_abs", ctypes.c_double)]


class rsf_tile(ctypes.Structure):
    _fields_ = [("volume", ctypes.c_void_p), ("phi", ctypes.c_void_p), ("nx", ctypes.c_int64),
                ("ny", ctypes.c_int64), ("nz", ctypes.c_int64)]


class rsf_profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int * len(PASS_NAMES)),
                ("ms", ctypes.c_double * len(PASS_NAMES))]


RSF_ORDER_ARRIVAL = 0
RSF_ORDER_SHORTEST = 1


class rsf_server_config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("budget_bytes", ctypes.c_size_t),
                ("segment_bytes", ctypes.c_size_t), ("chunk_iters", ctypes.c_int),
                ("max_resident", ctypes.c_int), ("batch_voxels", ctypes.c_int64),
                ("order", ctypes.c_int), ("split_targets", ctypes.c_int64 * 3),
                ("separate_passes", ctypes.c_int)]


class rsf_request(ctypes.Structure):
    _fields_ = [("volume", ctypes.c_void_p), ("phi", ctypes.c_void_p), ("nx", ctypes.c_int64),
                ("ny", ctypes.c_int64), ("nz", ctypes.c_int64), ("volume_dtype", ctypes.c_int),
                ("params", rsf_params), ("iters", ctypes.c_int), ("tol", ctypes.c_double)]


class rsf_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters_run", ctypes.c_int),
                ("last_sum_abs", ctypes.c_double), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("workspace_bytes", ctypes.c_size_t)]


class rsf_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("pending", ctypes.c_int), ("resident", ctypes.c_int),
                ("peak_resident", ctypes.c_int), ("bytes_in_use", ctypes.c_size_t),
                ("peak_bytes", ctypes.c_size_t), ("bytes_reserved", ctypes.c_size_t),
                ("chunks", ctypes.c_uint64), ("voxel_iters", ctypes.c_double)]


PROBE_NAMES = ("H", "f1", "f2", "Fd", "kappa", "lap", "R", "E", "phi_next")


class rsf_probe_fields(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in PROBE_NAMES]


_lib = None


def lib() -> ctypes.CDLL:
    """Load librsf.so (once).  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2404_02813_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, f, i = ctypes.c_void_p, ctypes.c_int64, ctypes.c_float, ctypes.c_int
    L.rsf_create.argtypes = [ctypes.POINTER(vp), i]
    L.rsf_create.restype = i
    L.rsf_destroy.argtypes = [vp]
    L.rsf_destroy.restype = None
    L.rsf_last_error.argtypes = [vp]
    L.rsf_last_error.restype = ctypes.c_char_p
    L.rsf_workspace_bytes.argtypes = [i64, i64, i64, i, i]
    L.rsf_workspace_bytes.restype = ctypes.c_size_t
    L.rsf_evolve.argtypes = [vp, vp, i, vp, i64, i64, i64, f, f, f, f, f, f, f, i, vp]
    L.rsf_evolve.restype = i
    L.rsf_evolve_ex.argtypes = [vp, vp, i, vp, i64, i64, i64, ctypes.POINTER(rsf_params), i,
                                ctypes.c_double, vp, ctypes.c_size_t, vp]
    L.rsf_evolve_ex.restype = i
    L.rsf_evolve_noalloc.argtypes = [vp, vp, i, vp, i64, i64, i64, ctypes.POINTER(rsf_params),
                                     i, ctypes.c_double, vp]
    L.rsf_evolve_noalloc.restype = i
    L.rsf_get_stats.argtypes = [vp, ctypes.POINTER(rsf_stats), ctypes.POINTER(ctypes.c_double), i]
    L.rsf_get_stats.restype = i
    L.rsf_gauss3d.argtypes = [vp, vp, vp, i64, i64, i64, f, vp]
    L.rsf_gauss3d.restype = i
    L.rsf_probe.argtypes = [vp, vp, i, vp, i64, i64, i64, ctypes.POINTER(rsf_params),
                            ctypes.POINTER(rsf_probe_fields), vp]
    L.rsf_probe.restype = i
    L.rsf_batch_workspace_bytes.argtypes = [ctypes.POINTER(rsf_tile), i, i, i]
    L.rsf_batch_workspace_bytes.restype = ctypes.c_size_t
    L.rsf_evolve_batch.argtypes = [vp, ctypes.POINTER(rsf_tile), i, i, ctypes.POINTER(rsf_params),
                                   i, ctypes.c_double, vp, ctypes.c_size_t, vp]
    L.rsf_evolve_batch.restype = i
    L.rsf_get_tile_stats.argtypes = [vp, i, ctypes.POINTER(rsf_stats),
                                     ctypes.POINTER(ctypes.c_double), i]
    L.rsf_get_tile_stats.restype = i
    L.rsf_autotune.argtypes = [vp, ctypes.POINTER(rsf_tile), i, i, ctypes.POINTER(rsf_params), i,
                               ctypes.POINTER(ctypes.c_int64), vp]
    L.rsf_autotune.restype = i
    L.rsf_set_fusion.argtypes = [vp, i]
    L.rsf_set_fusion.restype = i
    L.rsf_set_graphs.argtypes = [vp, i]
    L.rsf_set_graphs.restype = i
    L.rsf_stream_probe.argtypes = [vp, i, vp, i, i64, vp]
    L.rsf_stream_probe.restype = i
    i64p = ctypes.POINTER(ctypes.c_int64)
    L.rsf_seeds.argtypes = [vp, vp, i, i64, i64, i64, f, f, vp, i64p, vp]
    L.rsf_seeds.restype = i
    L.rsf_seeds_ex.argtypes = [vp, vp, i, i64, i64, i64, f, f, vp, i64p, vp, ctypes.c_size_t, vp]
    L.rsf_seeds_ex.restype = i
    L.rsf_seeds_workspace_bytes.argtypes = [i64, i64, i64]
    L.rsf_seeds_workspace_bytes.restype = ctypes.c_size_t
    L.rsf_autotune_ex.argtypes = [vp, ctypes.POINTER(rsf_tile), i, i, ctypes.POINTER(rsf_params),
                                  i, ctypes.POINTER(ctypes.c_int64), vp, ctypes.c_size_t, vp]
    L.rsf_autotune_ex.restype = i
    L.rsf_autotune_workspace_bytes.argtypes = [vp, ctypes.POINTER(rsf_tile), i,
                                               ctypes.POINTER(rsf_params), i]
    L.rsf_autotune_workspace_bytes.restype = ctypes.c_size_t
    L.rsf_fast_sweep.argtypes = [vp, vp, i64, i64, i64, i, vp]
    L.rsf_fast_sweep.restype = i
    L.rsf_init_phi.argtypes = [vp, vp, i, vp, i64, i64, i64, f, f, f, i, i64p, vp]
    L.rsf_init_phi.restype = i
    L.rsf_init_phi_ex.argtypes = [vp, vp, i, vp, i64, i64, i64, f, f, f, i, i64p, vp,
                                  ctypes.c_size_t, vp]
    L.rsf_init_phi_ex.restype = i
    L.rsf_init_workspace_bytes.argtypes = [i64, i64, i64]
    L.rsf_init_workspace_bytes.restype = ctypes.c_size_t
    L.rsf_set_fault.argtypes = [ctypes.c_char_p]
    L.rsf_set_fault.restype = i
    L.rsf_fault_allocations.argtypes = []
    L.rsf_fault_allocations.restype = ctypes.c_int64
    L.rsf_workspace_bytes_params.argtypes = [i64, i64, i64, i, ctypes.POINTER(rsf_params)]
    L.rsf_workspace_bytes_params.restype = ctypes.c_size_t
    L.rsf_batch_workspace_bytes_params.argtypes = [ctypes.POINTER(rsf_tile), i, i,
                                                   ctypes.POINTER(rsf_params)]
    L.rsf_batch_workspace_bytes_params.restype = ctypes.c_size_t
    L.rsf_evolve_volume.argtypes = [vp, vp, i, vp, i64, i64, i64, i64, i64,
                                    ctypes.POINTER(rsf_params), i, ctypes.c_size_t, vp]
    L.rsf_evolve_volume.restype = i
    L.rsf_volume_workspace_bytes.argtypes = [vp, i, i64, i64, i64, i64, i64,
                                             ctypes.POINTER(rsf_params), i, ctypes.c_size_t]
    L.rsf_volume_workspace_bytes.restype = ctypes.c_size_t
    L.rsf_evolve_volume_ex.argtypes = [vp, vp, i, vp, i64, i64, i64, i64, i64,
                                       ctypes.POINTER(rsf_params), i, ctypes.c_size_t, vp,
                                       ctypes.c_size_t, vp]
    L.rsf_evolve_volume_ex.restype = i
    L.rsf_set_split_targets.argtypes = [vp, i64, i64, i64]
    L.rsf_set_split_targets.restype = i
    L.rsf_autotune_reset.argtypes = [vp]
    L.rsf_autotune_reset.restype = None
    u64p = ctypes.POINTER(ctypes.c_uint64)
    L.rsf_server_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(rsf_server_config)]
    L.rsf_server_create.restype = i
    L.rsf_server_submit.argtypes = [vp, ctypes.POINTER(rsf_request), u64p]
    L.rsf_server_submit.restype = i
    L.rsf_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(rsf_result)]
    L.rsf_server_poll.restype = i
    L.rsf_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_double,
                                  ctypes.POINTER(rsf_result)]
    L.rsf_server_wait.restype = i
    L.rsf_server_drain.argtypes = [vp]
    L.rsf_server_drain.restype = i
    L.rsf_server_get_stats.argtypes = [vp, ctypes.POINTER(rsf_server_stats)]
    L.rsf_server_get_stats.restype = i
    L.rsf_server_last_error.argtypes = [vp]
    L.rsf_server_last_error.restype = ctypes.c_char_p
    L.rsf_server_destroy.argtypes = [vp]
    L.rsf_server_destroy.restype = None
    L.rsf_profile_enable.argtypes = [vp, i]
    L.rsf_profile_enable.restype = i
    L.rsf_profile_read.argtypes = [vp, ctypes.POINTER(rsf_profile)]
    L.rsf_profile_read.restype = i
    _lib = L
    return L


def _check(ctx, status: int) -> None:
    if status != RSF_OK:
        msg = lib().rsf_last_error(ctx).decode(errors="replace") if ctx else ""
        raise RsfError(status, msg)


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


_IMAGE_DTYPES = {torch.float32: RSF_F32, torch.uint16: RSF_U16}
_STORAGE = {"f32": RSF_F32, "f16": RSF_F16, "bf16": RSF_BF16}


def _field(t: torch.Tensor, name: str, dtype=torch.float32) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if dtype == "image":
        if t.dtype not in _IMAGE_DTYPES:
            raise ValueError(f"{name} must be float32 or uint16")
    elif t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")
    if t.dim() != 3 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous 3D tensor [nz][ny][nx]")
    return t


def make_params(sigma, lambda1, lambda2, nu, mu, dt, eps, eta=1e-10,
                regulariser=RSF_REG_DOUBLE_WELL, storage="f32", force=RSF_FORCE_RSF,
                sigma2=0.0) -> rsf_params:
    st = _STORAGE[storage] if isinstance(storage, str) else int(storage)
    return rsf_params(sigma, lambda1, lambda2, nu, mu, dt, eps, eta, regulariser, st, force,
                      sigma2)


def rsf_create(device: int = 0) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    st = lib().rsf_create(ctypes.byref(ctx), int(device))
    if st != RSF_OK:
        raise RsfError(st, f"rsf_create(device={device}) failed")
    return ctx


def rsf_destroy(ctx) -> None:
    if ctx:
        lib().rsf_destroy(ctx)


def rsf_last_error(ctx) -> str:
    return lib().rsf_last_error(ctx).decode(errors="replace")


def rsf_workspace_bytes(nx: int, ny: int, nz: int, iters: int, storage=RSF_F32) -> int:
    st = _STORAGE[storage] if isinstance(storage, str) else int(storage)
    return int(lib().rsf_workspace_bytes(nx, ny, nz, iters, st))


def rsf_evolve(ctx, volume: torch.Tensor, phi: torch.Tensor, sigma: float, lambda1: float,
               lambda2: float, nu: float, mu: float, dt: float, eps: float, iters: int,
               stream=None) -> None:
    """Evolve `phi` in place (default double-well regulariser)."""
    _field(volume, "volume", "image")
    _field(phi, "phi")
    if volume.shape != phi.shape or volume.device != phi.device:
        raise ValueError("volume and phi must have the same shape and device")
    nz, ny, nx = phi.shape
    _check(ctx, lib().rsf_evolve(ctx, volume.data_ptr(), _IMAGE_DTYPES[volume.dtype],
                                 phi.data_ptr(), nx, ny, nz,
                                 sigma, lambda1, lambda2, nu, mu, dt, eps, int(iters),
                                 _stream(stream)))


def rsf_evolve_ex(ctx, volume: torch.Tensor, phi: torch.Tensor, params: rsf_params, iters: int,
                  tol: float = 0.0, workspace: torch.Tensor | None = None, stream=None) -> None:
    _field(volume, "volume", "image")
    _field(phi, "phi")
    if volume.shape != phi.shape or volume.device != phi.device:
        raise ValueError("volume and phi must have the same shape and device")
    nz, ny, nx = phi.shape
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        if not workspace.is_cuda or not workspace.is_contiguous():
            raise ValueError("workspace must be a contiguous CUDA tensor")
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    _check(ctx, lib().rsf_evolve_ex(ctx, volume.data_ptr(), _IMAGE_DTYPES[volume.dtype],
                                    phi.data_ptr(), nx, ny, nz,
                                    ctypes.byref(params), int(iters), float(tol), ws_ptr,
                                    ws_bytes, _stream(stream)))


def rsf_evolve_noalloc(ctx, volume: torch.Tensor, phi: torch.Tensor, params: rsf_params,
                       iters: int, tol: float = 0.0, stream=None) -> None:
    """As rsf_evolve_ex, with the library's fixed per-GPU workspace (no
    device allocation); volumes up to RSF_NOALLOC_MAX_BYTES of workspace."""
    _field(volume, "volume", "image")
    _field(phi, "phi")
    if volume.shape != phi.shape or volume.device != phi.device:
        raise ValueError("volume and phi must have the same shape and device")
    nz, ny, nx = phi.shape
    _check(ctx, lib().rsf_evolve_noalloc(ctx, volume.data_ptr(), _IMAGE_DTYPES[volume.dtype],
                                         phi.data_ptr(), nx, ny, nz, ctypes.byref(params),
                                         int(iters), float(tol), _stream(stream)))


def rsf_get_stats(ctx, cap: int = 0):
    """Returns (iters_requested, iters_run, last_sum_abs, history list)."""
    return rsf_get_tile_stats(ctx, 0, cap)


def rsf_get_tile_stats(ctx, tile: int, cap: int = 0):
    """Statistics of one tile of the last evolution (see rsf_get_stats)."""
    st = rsf_stats()
    hist = (ctypes.c_double * max(cap, 1))()
    status = lib().rsf_get_tile_stats(ctx, int(tile), ctypes.byref(st),
                                      hist if cap > 0 else None, int(cap))
    _check(ctx, status)
    n = min(cap, st.iters_run)
    return st.iters_requested, st.iters_run, st.last_sum_abs, [hist[i] for i in range(n)]


def _tiles(volumes, phis):
    if len(volumes) != len(phis) or not volumes:
        raise ValueError("need matching, non-empty lists of volumes and phis")
    dt = None
    arr = (rsf_tile * len(volumes))()
    for k, (v, p) in enumerate(zip(volumes, phis)):
        _field(v, "volume", "image")
        _field(p, "phi")
        if v.shape != p.shape:
            raise ValueError("each volume and phi must have the same shape")
        if dt is None:
            dt = v.dtype
        elif v.dtype != dt:
            raise ValueError("all volumes of a batch must share a dtype")
        nz, ny, nx = p.shape
        arr[k] = rsf_tile(v.data_ptr(), p.data_ptr(), nx, ny, nz)
    return arr, _IMAGE_DTYPES[dt]


def rsf_autotune(ctx, volumes, phis, params: rsf_params, trial_iters: int = 3,
                 stream=None) -> tuple:
    """Pick and keep per-shape workgroup splits and the schedule by timing
    (phis untouched); returns the chosen (xy, z, update) workgroup targets and
    1 if the fused update was chosen, else 0."""
    arr, vdt = _tiles(volumes, phis)
    chosen = (ctypes.c_int64 * 4)()
    _check(ctx, lib().rsf_autotune(ctx, arr, len(volumes), vdt, ctypes.byref(params),
                                   int(trial_iters), chosen, _stream(stream)))
    return tuple(chosen)


def rsf_autotune_ex(ctx, volumes, phis, params: rsf_params, trial_iters: int,
                    workspace: torch.Tensor, stream=None) -> tuple:
    """rsf_autotune with the phi copies and trial workspaces in `workspace`."""
    if workspace is None or not workspace.is_cuda or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous device tensor")
    arr, vdt = _tiles(volumes, phis)
    chosen = (ctypes.c_int64 * 4)()
    _check(ctx, lib().rsf_autotune_ex(ctx, arr, len(volumes), vdt, ctypes.byref(params),
                                      int(trial_iters), chosen, workspace.data_ptr(),
                                      workspace.numel() * workspace.element_size(),
                                      _stream(stream)))
    return tuple(chosen)


def rsf_autotune_workspace_bytes(ctx, shapes, params: rsf_params, trial_iters: int = 3) -> int:
    """Device bytes rsf_autotune_ex needs; shapes: list of (nz, ny, nx)."""
    arr = (rsf_tile * len(shapes))()
    for k, (nz, ny, nx) in enumerate(shapes):
        arr[k] = rsf_tile(None, None, nx, ny, nz)
    return int(lib().rsf_autotune_workspace_bytes(ctx, arr, len(shapes), ctypes.byref(params),
                                                  int(trial_iters)))


def rsf_workspace_bytes_params(nx: int, ny: int, nz: int, iters: int, params: rsf_params) -> int:
    return int(lib().rsf_workspace_bytes_params(nx, ny, nz, iters, ctypes.byref(params)))


def rsf_batch_workspace_bytes_params(shapes, iters: int, params: rsf_params) -> int:
    arr = (rsf_tile * len(shapes))()
    for k, (nz, ny, nx) in enumerate(shapes):
        arr[k] = rsf_tile(None, None, nx, ny, nz)
    return int(lib().rsf_batch_workspace_bytes_params(arr, len(shapes), iters,
                                                      ctypes.byref(params)))


def rsf_set_fusion(ctx, on: bool) -> None:
    _check(ctx, lib().rsf_set_fusion(ctx, 1 if on else 0))


def rsf_set_graphs(ctx, on: bool) -> None:
    _check(ctx, lib().rsf_set_graphs(ctx, 1 if on else 0))


def rsf_stream_probe(inp: torch.Tensor, n_read: int, out: torch.Tensor, n_write: int,
                     stream=None) -> None:
    """One launch of the streaming kernel: n_read float fields of inp (flat,
    n_read * n floats) summed into n_write fields of out."""
    for t, k, name in ((inp, n_read, "inp"), (out, n_write, "out")):
        if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
        if t.numel() % k:
            raise ValueError(f"{name} must hold a whole number of fields")
    n = inp.numel() // n_read
    if out.numel() // n_write != n:
        raise ValueError("inp and out fields must have the same length")
    st = lib().rsf_stream_probe(inp.data_ptr(), int(n_read), out.data_ptr(), int(n_write), n,
                                _stream(stream))
    if st != RSF_OK:
        raise RsfError(st, "rsf_stream_probe failed")


def rsf_seeds(ctx, volume: torch.Tensor, sigma_b: float, threshold: float,
              mask: torch.Tensor | None = None, stream=None, workspace: torch.Tensor = None):
    """Seed mask (uint8 tensor) and the seed count.  With `workspace` (a
    device tensor of at least rsf_seeds_workspace_bytes bytes) the scratch is
    the caller's (rsf_seeds_ex)."""
    _field(volume, "volume", "image")
    nz, ny, nx = volume.shape
    if mask is None:
        mask = torch.empty(volume.shape, dtype=torch.uint8, device=volume.device)
    if mask.dtype != torch.uint8 or mask.shape != volume.shape or not mask.is_contiguous():
        raise ValueError("mask must be a contiguous uint8 tensor of the volume's shape")
    n = ctypes.c_int64(0)
    if workspace is None:
        _check(ctx, lib().rsf_seeds(ctx, volume.data_ptr(), _IMAGE_DTYPES[volume.dtype], nx, ny,
                                    nz, float(sigma_b), float(threshold), mask.data_ptr(),
                                    ctypes.byref(n), _stream(stream)))
        return mask, n.value
    if not workspace.is_cuda or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous device tensor")
    _check(ctx, lib().rsf_seeds_ex(ctx, volume.data_ptr(), _IMAGE_DTYPES[volume.dtype], nx, ny, nz,
                                   float(sigma_b), float(threshold), mask.data_ptr(),
                                   ctypes.byref(n), workspace.data_ptr(),
                                   workspace.numel() * workspace.element_size(), _stream(stream)))
    return mask, n.value


def rsf_seeds_ex(ctx, volume: torch.Tensor, sigma_b: float, threshold: float,
                 mask: torch.Tensor | None, workspace: torch.Tensor, stream=None):
    """rsf_seeds with its scratch in `workspace`."""
    if workspace is None:
        raise ValueError("rsf_seeds_ex needs a workspace")
    return rsf_seeds(ctx, volume, sigma_b, threshold, mask, stream, workspace)


def rsf_seeds_workspace_bytes(shape) -> int:
    """Device bytes rsf_seeds_ex needs for a volume of shape (nz, ny, nx)."""
    nz, ny, nx = shape
    return int(lib().rsf_seeds_workspace_bytes(int(nx), int(ny), int(nz)))


def rsf_fast_sweep(ctx, u: torch.Tensor, rounds: int = 2, stream=None) -> None:
    _field(u, "u")
    nz, ny, nx = u.shape
    _check(ctx, lib().rsf_fast_sweep(ctx, u.data_ptr(), nx, ny, nz, int(rounds), _stream(stream)))


def rsf_init_phi(ctx, volume: torch.Tensor, phi: torch.Tensor, sigma_b: float, threshold: float,
                 offset: float = 0.0, rounds: int = 2, stream=None,
                 workspace: torch.Tensor = None) -> int:
    """phi = offset - distance to the nearest seed; returns the seed count.
    With `workspace` (a device tensor of at least rsf_init_workspace_bytes
    bytes) the scratch is the caller's (rsf_init_phi_ex)."""
    _field(volume, "volume", "image")
    _field(phi, "phi")
    if volume.shape != phi.shape:
        raise ValueError("volume and phi must have the same shape")
    nz, ny, nx = phi.shape
    n = ctypes.c_int64(0)
    if workspace is None:
        _check(ctx, lib().rsf_init_phi(ctx, volume.data_ptr(), _IMAGE_DTYPES[volume.dtype],
                                       phi.data_ptr(), nx, ny, nz, float(sigma_b),
                                       float(threshold), float(offset), int(rounds),
                                       ctypes.byref(n), _stream(stream)))
        return n.value
    if not workspace.is_cuda or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous device tensor")
    _check(ctx, lib().rsf_init_phi_ex(ctx, volume.data_ptr(), _IMAGE_DTYPES[volume.dtype],
                                      phi.data_ptr(), nx, ny, nz, float(sigma_b),
                                      float(threshold), float(offset), int(rounds),
                                      ctypes.byref(n), workspace.data_ptr(),
                                      workspace.numel() * workspace.element_size(),
                                      _stream(stream)))
    return n.value


def rsf_init_phi_ex(ctx, volume: torch.Tensor, phi: torch.Tensor, sigma_b: float,
                    threshold: float, offset: float, rounds: int, workspace: torch.Tensor,
                    stream=None) -> int:
    """rsf_init_phi with its scratch in `workspace`."""
    if workspace is None:
        raise ValueError("rsf_init_phi_ex needs a workspace")
    return rsf_init_phi(ctx, volume, phi, sigma_b, threshold, offset, rounds, stream, workspace)


def rsf_set_fault(spec) -> None:
    """Arm ("alloc_fail:N" or "alloc_fail:N:K") or disarm (None, "", "off")
    injected allocation failures, process-wide."""
    st = lib().rsf_set_fault(None if spec is None else str(spec).encode())
    if st != RSF_OK:
        raise RsfError(st, f"malformed fault spec {spec!r}")


def rsf_fault_allocations() -> int:
    """Allocation attempts counted since the fault was armed; -1 if disarmed."""
    return int(lib().rsf_fault_allocations())


def rsf_init_workspace_bytes(shape) -> int:
    """Device bytes rsf_init_phi_ex needs for a volume of shape (nz, ny, nx)."""
    nz, ny, nx = shape
    return int(lib().rsf_init_workspace_bytes(int(nx), int(ny), int(nz)))


def rsf_evolve_volume(ctx, volume: torch.Tensor, phi: torch.Tensor, params: rsf_params,
                      iters: int, block: int, curtain: int = 0, budget_bytes: int = 0,
                      stream=None, workspace: torch.Tensor = None) -> None:
    """Sub-volumes with curtains, evolved independently, merged by linear
    interpolation (phi in place); with `workspace` (a device tensor of at
    least rsf_volume_workspace_bytes bytes) every device buffer is the
    caller's (rsf_evolve_volume_ex)."""
    _field(volume, "volume", "image")
    _field(phi, "phi")
    if volume.shape != phi.shape:
        raise ValueError("volume and phi must have the same shape")
    nz, ny, nx = phi.shape
    if workspace is None:
        _check(ctx, lib().rsf_evolve_volume(ctx, volume.data_ptr(), _IMAGE_DTYPES[volume.dtype],
                                            phi.data_ptr(), nx, ny, nz, int(block), int(curtain),
                                            ctypes.byref(params), int(iters), int(budget_bytes),
                                            _stream(stream)))
        return
    if not workspace.is_cuda or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous device tensor")
    _check(ctx, lib().rsf_evolve_volume_ex(ctx, volume.data_ptr(), _IMAGE_DTYPES[volume.dtype],
                                           phi.data_ptr(), nx, ny, nz, int(block), int(curtain),
                                           ctypes.byref(params), int(iters), int(budget_bytes),
                                           workspace.data_ptr(),
                                           workspace.numel() * workspace.element_size(),
                                           _stream(stream)))


def rsf_evolve_volume_ex(ctx, volume: torch.Tensor, phi: torch.Tensor, params: rsf_params,
                         iters: int, block: int, curtain: int, budget_bytes: int,
                         workspace: torch.Tensor, stream=None) -> None:
    """rsf_evolve_volume with every device buffer in `workspace`."""
    if workspace is None:
        raise ValueError("rsf_evolve_volume_ex needs a workspace")
    rsf_evolve_volume(ctx, volume, phi, params, iters, block, curtain, budget_bytes, stream,
                      workspace)


def rsf_volume_workspace_bytes(ctx, volume_dtype, shape, params: rsf_params, iters: int,
                               block: int, curtain: int = 0, budget_bytes: int = 0) -> int:
    """Device bytes rsf_evolve_volume_ex needs (0 for invalid arguments);
    volume_dtype is a torch dtype of the image, shape (nz, ny, nx)."""
    nz, ny, nx = shape
    return int(lib().rsf_volume_workspace_bytes(ctx, _IMAGE_DTYPES[volume_dtype], nx, ny, nz,
                                                int(block), int(curtain), ctypes.byref(params),
                                                int(iters), int(budget_bytes)))


def rsf_set_split_targets(ctx, xy_waves: int = 0, z_blocks: int = 0, u_blocks: int = 0) -> None:
    _check(ctx, lib().rsf_set_split_targets(ctx, int(xy_waves), int(z_blocks), int(u_blocks)))


def rsf_autotune_reset(ctx) -> None:
    lib().rsf_autotune_reset(ctx)


def rsf_batch_workspace_bytes(shapes, iters: int, storage=RSF_F32) -> int:
    """shapes: list of (nz, ny, nx)."""
    arr = (rsf_tile * len(shapes))()
    for k, (nz, ny, nx) in enumerate(shapes):
        arr[k] = rsf_tile(None, None, nx, ny, nz)
    st = _STORAGE[storage] if isinstance(storage, str) else int(storage)
    return int(lib().rsf_batch_workspace_bytes(arr, len(shapes), int(iters), st))


def rsf_evolve_batch(ctx, volumes, phis, params: rsf_params, iters: int, tol: float = 0.0,
                     workspace: torch.Tensor | None = None, stream=None) -> None:
    """Evolve each phi in place against its volume; one launch per pass for all."""
    arr, vdt = _tiles(volumes, phis)
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    _check(ctx, lib().rsf_evolve_batch(ctx, arr, len(volumes), vdt, ctypes.byref(params),
                                       int(iters), float(tol), ws_ptr, ws_bytes,
                                       _stream(stream)))


def rsf_gauss3d(ctx, inp: torch.Tensor, out: torch.Tensor, sigma: float, stream=None) -> None:
    _field(inp, "in")
    _field(out, "out")
    if inp.shape != out.shape:
        raise ValueError("in and out must have the same shape")
    nz, ny, nx = inp.shape
    _check(ctx, lib().rsf_gauss3d(ctx, inp.data_ptr(), out.data_ptr(), nx, ny, nz, float(sigma),
                                  _stream(stream)))


def rsf_probe(ctx, volume: torch.Tensor, phi: torch.Tensor, params: rsf_params,
              stream=None) -> dict:
    """One iteration's intermediate fields as new tensors (see rsf.h)."""
    _field(volume, "volume", "image")
    _field(phi, "phi")
    nz, ny, nx = phi.shape
    out = {n: torch.empty_like(phi) for n in PROBE_NAMES}
    pf = rsf_probe_fields(*[out[n].data_ptr() for n in PROBE_NAMES])
    _check(ctx, lib().rsf_probe(ctx, volume.data_ptr(), _IMAGE_DTYPES[volume.dtype],
                                phi.data_ptr(), nx, ny, nz,
                                ctypes.byref(params), ctypes.byref(pf), _stream(stream)))
    return out


def rsf_profile_enable(ctx, on: bool) -> None:
    _check(ctx, lib().rsf_profile_enable(ctx, 1 if on else 0))


def rsf_profile_read(ctx) -> dict:
    """{pass name: (launches, total ms)} since profiling was enabled."""
    pr = rsf_profile()
    _check(ctx, lib().rsf_profile_read(ctx, ctypes.byref(pr)))
    return {n: (pr.launches[i], pr.ms[i]) for i, n in enumerate(PASS_NAMES)}


class Context:
    """Owns an rsf_context for one device."""

    def __init__(self, device: int = 0):
        self.device = int(device)
        self.handle = rsf_create(self.device)

    def close(self) -> None:
        if self.handle:
            rsf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def evolve(self, volume, phi, iters, sigma=3.0, lambda1=1.0, lambda2=1.0, nu=0.001, mu=1.0,
               dt=0.1, eps=1.0, stream=None):
        rsf_evolve(self.handle, volume, phi, sigma, lambda1, lambda2, nu, mu, dt, eps, iters,
                   stream)

    def evolve_ex(self, volume, phi, params, iters, tol=0.0, workspace=None, stream=None):
        rsf_evolve_ex(self.handle, volume, phi, params, iters, tol, workspace, stream)

    def evolve_noalloc(self, volume, phi, params, iters, tol=0.0, stream=None):
        rsf_evolve_noalloc(self.handle, volume, phi, params, iters, tol, stream)

    def stats(self, cap=0):
        return rsf_get_stats(self.handle, cap)

    def tile_stats(self, tile, cap=0):
        return rsf_get_tile_stats(self.handle, tile, cap)

    def evolve_batch(self, volumes, phis, params, iters, tol=0.0, workspace=None, stream=None):
        rsf_evolve_batch(self.handle, volumes, phis, params, iters, tol, workspace, stream)

    def autotune(self, volumes, phis, params, trial_iters=3, stream=None):
        return rsf_autotune(self.handle, volumes, phis, params, trial_iters, stream)

    def evolve_volume(self, volume, phi, params, iters, block, curtain=0, budget_bytes=0,
                      stream=None, workspace=None):
        rsf_evolve_volume(self.handle, volume, phi, params, iters, block, curtain, budget_bytes,
                          stream, workspace)

    def volume_workspace_bytes(self, volume_dtype, shape, params, iters, block, curtain=0,
                               budget_bytes=0):
        return rsf_volume_workspace_bytes(self.handle, volume_dtype, shape, params, iters, block,
                                          curtain, budget_bytes)

    def set_graphs(self, on: bool) -> None:
        rsf_set_graphs(self.handle, on)

    def set_fusion(self, on: bool) -> None:
        rsf_set_fusion(self.handle, on)

    def seeds(self, volume, sigma_b, threshold, mask=None, stream=None, workspace=None):
        return rsf_seeds(self.handle, volume, sigma_b, threshold, mask, stream, workspace)

    def fast_sweep(self, u, rounds=2, stream=None):
        rsf_fast_sweep(self.handle, u, rounds, stream)

    def init_phi(self, volume, phi, sigma_b, threshold, offset=0.0, rounds=2, stream=None,
                 workspace=None):
        return rsf_init_phi(self.handle, volume, phi, sigma_b, threshold, offset, rounds, stream,
                            workspace)

    def set_split_targets(self, xy_waves=0, z_blocks=0, u_blocks=0):
        rsf_set_split_targets(self.handle, xy_waves, z_blocks, u_blocks)

    def autotune_reset(self):
        rsf_autotune_reset(self.handle)

    def gauss3d(self, inp, sigma, out=None, stream=None):
        out = torch.empty_like(inp) if out is None else out
        rsf_gauss3d(self.handle, inp, out, sigma, stream)
        return out

    def probe(self, volume, phi, params, stream=None):
        return rsf_probe(self.handle, volume, phi, params, stream)

    def profile(self, on: bool) -> None:
        rsf_profile_enable(self.handle, on)

    def profile_read(self) -> dict:
        return rsf_profile_read(self.handle)


# ---------------------------------------------------------------------------
# Request server
# ---------------------------------------------------------------------------

def _server_check(srv, status: int) -> None:
    if status not in (RSF_OK, RSF_NOT_READY):
        msg = lib().rsf_server_last_error(srv).decode(errors="replace") if srv else ""
        raise RsfError(status, msg)


def rsf_server_create(budget_bytes: int, chunk_iters: int = 0, max_resident: int = 0,
                      segment_bytes: int = 0, device: int = 0, batch_voxels: int = 0,
                      order: int = RSF_ORDER_ARRIVAL, split_targets=(0, 0, 0),
                      separate_passes: bool = False) -> ctypes.c_void_p:
    cfg = rsf_server_config(device, int(budget_bytes), int(segment_bytes), int(chunk_iters),
                            int(max_resident), int(batch_voxels), int(order),
                            (ctypes.c_int64 * 3)(*[int(v) for v in split_targets]),
                            1 if separate_passes else 0)
    h = ctypes.c_void_p()
    st = lib().rsf_server_create(ctypes.byref(h), ctypes.byref(cfg))
    if st != RSF_OK:
        raise RsfError(st, "rsf_server_create failed")
    return h


def rsf_server_submit(srv, volume: torch.Tensor, phi: torch.Tensor, params: rsf_params,
                      iters: int, tol: float = 0.0) -> int:
    _field(volume, "volume", "image")
    _field(phi, "phi")
    if volume.shape != phi.shape:
        raise ValueError("volume and phi must have the same shape")
    nz, ny, nx = phi.shape
    req = rsf_request(volume.data_ptr(), phi.data_ptr(), nx, ny, nz, _IMAGE_DTYPES[volume.dtype],
                      params, int(iters), float(tol))
    t = ctypes.c_uint64()
    _server_check(srv, lib().rsf_server_submit(srv, ctypes.byref(req), ctypes.byref(t)))
    return t.value


def _result_dict(r: rsf_result) -> dict:
    return {k: getattr(r, k) for k, _ in rsf_result._fields_}


def rsf_server_poll(srv, ticket: int):
    r = rsf_result()
    st = lib().rsf_server_poll(srv, ticket, ctypes.byref(r))
    _server_check(srv, st)
    return None if st == RSF_NOT_READY else _result_dict(r)


def rsf_server_wait(srv, ticket: int, timeout_s: float = -1.0):
    r = rsf_result()
    st = lib().rsf_server_wait(srv, ticket, float(timeout_s), ctypes.byref(r))
    _server_check(srv, st)
    return None if st == RSF_NOT_READY else _result_dict(r)


def rsf_server_drain(srv) -> None:
    _server_check(srv, lib().rsf_server_drain(srv))


def rsf_server_get_stats(srv) -> dict:
    s = rsf_server_stats()
    _server_check(srv, lib().rsf_server_get_stats(srv, ctypes.byref(s)))
    return {k: getattr(s, k) for k, _ in rsf_server_stats._fields_}


def rsf_server_last_error(srv) -> str:
    return lib().rsf_server_last_error(srv).decode(errors="replace")


def rsf_server_destroy(srv) -> None:
    lib().rsf_server_destroy(srv)


class Server:
    """Owning wrapper of an rsf_server.  Keeps a reference to each request's
    tensors until its result has been read, so they outlive the device work."""

    def __init__(self, budget_bytes: int, chunk_iters: int = 0, max_resident: int = 0,
                 segment_bytes: int = 0, device: int = 0, batch_voxels: int = 0,
                 order: int = RSF_ORDER_ARRIVAL, split_targets=(0, 0, 0),
                 separate_passes: bool = False):
        self.handle = rsf_server_create(budget_bytes, chunk_iters, max_resident, segment_bytes,
                                        device, batch_voxels, order, split_targets,
                                        separate_passes)
        self._held = {}

    def submit(self, volume, phi, params, iters, tol=0.0) -> int:
        t = rsf_server_submit(self.handle, volume, phi, params, iters, tol)
        self._held[t] = (volume, phi)
        return t

    def poll(self, ticket):
        r = rsf_server_poll(self.handle, ticket)
        if r is not None:
            self._held.pop(ticket, None)
        return r

    def wait(self, ticket, timeout_s=-1.0):
        r = rsf_server_wait(self.handle, ticket, timeout_s)
        if r is not None:
            self._held.pop(ticket, None)
        return r

    def drain(self):
        rsf_server_drain(self.handle)

    def stats(self) -> dict:
        return rsf_server_get_stats(self.handle)

    def close(self):
        if self.handle:
            rsf_server_destroy(self.handle)
            self.handle = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
