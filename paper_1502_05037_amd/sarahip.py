"""ctypes binding of libsarahip.so (the C ABI in include/sarahip.h).

Argument marshalling only: every step of the imaging path runs in the HIP
library.  Device arrays are torch tensors on a ROCm device (float32, or
complex64 / float32 pairs for visibilities); host arrays are numpy arrays.
Each function has the name of the C entry point without the ``sh_`` prefix
and raises :class:`SarahipError` on a non-OK status.  Importing this module
raises if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

# torch ships its own HIP runtime with the same soname (libamdhip64.so.7) as the ROCm one the library
# is linked against; whichever is loaded first serves the whole process.  Importing torch first makes
# that torch's runtime, so the library and torch share one runtime (device pointers and streams).
import torch  # noqa: E402,F401

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsarahip.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is missing: build it with __graft_entry__.build() "
                      "or python paper_1502_05037_amd/csrc/build.py")
lib = C.CDLL(_LIB_PATH)

STATUS = {0: "SH_OK", -1: "SH_EINVAL", -2: "SH_ENOMEM", -3: "SH_EDEVICE", -4: "SH_ENONFINITE", -5: "SH_EUNSUPPORTED"}
SARA_MASK = 0x1FF
PASS_RECORD = 16   # SH_PASS_RECORD
BALL_NOALLOC_MAX_BLOCKS = 65536   # SH_BALL_NOALLOC_MAX_BLOCKS


class SarahipError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib.sh_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")


class SdmmParams(C.Structure):
    _fields_ = [("gamma", C.c_double), ("nu", C.c_double), ("tol_rel", C.c_double), ("eps_slack", C.c_double),
                ("rw_beta", C.c_double), ("rw_delta0", C.c_double), ("max_iter", C.c_int32),
                ("cg_iters", C.c_int32), ("passes", C.c_int32), ("check_every", C.c_int32), ("graph", C.c_int32),
                ("w_from_x0", C.c_int32), ("toeplitz", C.c_int32), ("block_norm", C.c_int32),
                ("tol_dual", C.c_double), ("z_from_x0", C.c_int32), ("block_fraction", C.c_double),
                ("block_seed", C.c_uint64), ("synthesis", C.c_int32)]


class SdmmInfo(C.Structure):
    _fields_ = [("iters_total", C.c_int32), ("passes_done", C.c_int32), ("converged", C.c_int32),
                ("iters_last", C.c_int32), ("rel_change", C.c_double), ("objective", C.c_double),
                ("gamma", C.c_double), ("nu", C.c_double), ("delta", C.c_double), ("seconds", C.c_double),
                ("kkt_primal", C.c_double), ("kkt_dual", C.c_double), ("pass_iters", C.c_int32 * PASS_RECORD)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["pass_iters"] = [int(v) for v in self.pass_iters][:self.passes_done]
        return d


class TuneResult(C.Structure):
    _fields_ = [("accuracy", C.c_double), ("alias_error", C.c_double), ("ms_pair", C.c_double), ("J", C.c_int32),
                ("tile", C.c_int32), ("chunk", C.c_int32), ("candidates", C.c_int32), ("cached", C.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_vp, _i64, _i32, _u32, _f32, _f64 = C.c_void_p, C.c_int64, C.c_int32, C.c_uint32, C.c_float, C.c_double
_P64 = C.POINTER(C.c_double)
_PI64 = C.POINTER(C.c_int64)
_PI32 = C.POINTER(C.c_int32)
_SIGS = {
    "sh_last_error": (C.c_char_p, []),
    "sh_version": (C.c_char_p, []),
    "sh_op_create": (C.c_int, [_P64, _i64, _i32, _i32, _i32, _PI64, _i32, C.POINTER(_vp)]),
    "sh_op_create_tuned": (C.c_int, [_P64, _i64, _i32, _i32, _i32, _PI64, _i32, _i32, _i32, C.POINTER(_vp)]),
    "sh_op_create_batched": (C.c_int, [_P64, _PI64, _i32, _i32, _i32, _i32, _PI64, _PI32, _i32, _i32,
                                       C.POINTER(_vp)]),
    "sh_op_autotune": (C.c_int, [_P64, _PI64, _i32, _i32, _i32, _f64, _PI64, _PI32, _i32, C.POINTER(TuneResult),
                                 C.POINTER(_vp), _vp]),
    "sh_kb_alias_error": (C.c_int, [_i32, _i32, _P64]),
    "sh_op_destroy": (C.c_int, [_vp]),
    "sh_op_query": (C.c_int, [_vp, _PI64]),
    "sh_op_block_offsets": (C.c_int, [_vp, _PI64]),
    "sh_op_permutation": (C.c_int, [_vp, _PI64]),
    "sh_phi_fwd": (C.c_int, [_vp, _vp, _vp, _vp]),
    "sh_phi_adj": (C.c_int, [_vp, _vp, _vp, _vp]),
    "sh_phi_fwd_internal": (C.c_int, [_vp, _vp, _vp, _vp]),
    "sh_phi_adj_internal": (C.c_int, [_vp, _vp, _vp, _vp]),
    "sh_vis_to_internal": (C.c_int, [_vp, _vp, _vp, _vp]),
    "sh_vis_to_user": (C.c_int, [_vp, _vp, _vp, _vp]),
    "sh_op_norm": (C.c_int, [_vp, _vp, _i32, _f64, _P64, _vp]),
    "sh_block_weights": (C.c_int, [_vp, _P64, _vp]),
    "sh_toeplitz_create": (C.c_int, [_vp, _P64, C.POINTER(_vp), _vp]),
    "sh_toeplitz_apply": (C.c_int, [_vp, _vp, _vp, _vp]),
    "sh_toeplitz_destroy": (C.c_int, [_vp]),
    "sh_psi_create": (C.c_int, [_i32, _i32, _u32, C.POINTER(_vp)]),
    "sh_psi_create_batched": (C.c_int, [_i32, _i32, _u32, _i32, C.POINTER(_vp)]),
    "sh_psi_destroy": (C.c_int, [_vp]),
    "sh_psi_planes": (C.c_int, [_vp, C.POINTER(_i32)]),
    "sh_daubechies": (C.c_int, [_i32, _P64]),
    "sh_psi_fwd": (C.c_int, [_vp, _vp, _vp, _vp]),
    "sh_psi_adj": (C.c_int, [_vp, _vp, _vp, _vp]),
    "sh_prox_l1": (C.c_int, [_i64, _vp, _vp, _vp, _f32, _vp, _vp]),
    "sh_prox_pos": (C.c_int, [_i64, _vp, _vp, _vp, _vp]),
    "sh_prox_ball": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "sh_prox_ball_noalloc": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "sh_reweight": (C.c_int, [_i64, _vp, _f64, _vp, _vp]),
    "sh_std": (C.c_int, [_i64, _vp, _P64, _vp]),
    "sh_sdmm_default_params": (None, [C.POINTER(SdmmParams)]),
    "sh_workspace_bytes": (C.c_int, [_vp, _vp, C.POINTER(SdmmParams), C.POINTER(C.c_size_t)]),
    "sh_sdmm_solve_ws": (C.c_int, [_vp, _vp, _vp, _P64, _vp, _vp, C.POINTER(SdmmParams), _vp, _vp, _P64,
                                   C.POINTER(SdmmInfo), _vp, C.c_size_t, _vp]),
    "sh_sdmm_create_ws": (C.c_int, [_vp, _vp, _vp, _P64, _vp, _vp, C.POINTER(SdmmParams), _vp, C.c_size_t,
                                    C.POINTER(_vp), _vp]),
    "sh_psi_workspace_bytes": (C.c_int, [_i32, _i32, _u32, _i32, C.POINTER(C.c_size_t)]),
    "sh_psi_create_ws": (C.c_int, [_i32, _i32, _u32, _i32, _vp, C.c_size_t, C.POINTER(_vp)]),
    "sh_toeplitz_workspace_bytes": (C.c_int, [_vp, C.POINTER(C.c_size_t)]),
    "sh_toeplitz_create_ws": (C.c_int, [_vp, _P64, _vp, C.c_size_t, C.POINTER(_vp), _vp]),
    "sh_sdmm_solve": (C.c_int, [_vp, _vp, _vp, _P64, _vp, _vp, C.POINTER(SdmmParams), _vp, _vp, _P64,
                                C.POINTER(SdmmInfo), _vp]),
    "sh_sdmm_create": (C.c_int, [_vp, _vp, _vp, _P64, _vp, _vp, C.POINTER(SdmmParams), C.POINTER(_vp), _vp]),
    "sh_sdmm_iterate": (C.c_int, [_vp, _i32, _vp]),
    "sh_sdmm_result": (C.c_int, [_vp, _vp, _P64, _P64, _vp]),
    "sh_sdmm_kkt": (C.c_int, [_vp, _P64, _P64, _P64, _vp]),
    "sh_sdmm_state_bytes": (C.c_int, [_vp, C.POINTER(C.c_size_t)]),
    "sh_sdmm_state_export": (C.c_int, [_vp, _vp, C.c_size_t, _vp]),
    "sh_sdmm_state_import": (C.c_int, [_vp, _vp, C.c_size_t, _vp]),
    "sh_sdmm_metrics_enable": (C.c_int, [_vp, _i32, C.POINTER(_i32)]),
    "sh_sdmm_metrics_read": (C.c_int, [_vp, _P64, _i32, C.POINTER(_i32), _PI64, _vp]),
    "sh_op_create_stream": (C.c_int, [_P64, _i64, _i32, _i32, _i32, _PI64, _i32, _i32, _i32, _vp, C.POINTER(_vp)]),
    "sh_device_bytes": (C.c_int, [_PI64, _PI64]),
    "sh_tune_cache_clear": (C.c_int, []),
    "sh_sdmm_destroy": (C.c_int, [_vp]),
    "sh_unet_create": (C.c_int, [_i32, _i32, C.POINTER(_vp)]),
    "sh_unet_destroy": (C.c_int, [_vp]),
    "sh_unet_num_params": (C.c_int, [_vp, _PI64]),
    "sh_unet_set_params": (C.c_int, [_vp, C.POINTER(C.c_float), _i64]),
    "sh_unet_get_params": (C.c_int, [_vp, C.POINTER(C.c_float), _i64]),
    "sh_unet_forward": (C.c_int, [_vp, _vp, _i32, _i32, _i32, _vp, _vp]),
    "sh_unet_loss_grad": (C.c_int, [_vp, _vp, _vp, _i32, _i32, _i32, _P64, C.POINTER(C.c_float), _vp]),
    "sh_unet_train_step": (C.c_int, [_vp, _vp, _vp, _i32, _i32, _i32, _f32, _P64, _vp]),
    "sh_warm_start": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "sh_dirty_normalised": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "sh_scale_images": (C.c_int, [_vp, _vp, _i32, _i64, _i32, _vp]),
    "sh_profile_enable": (C.c_int, [_i32]),
    "sh_profile_read": (C.c_int, [C.c_char_p, _PI64, _P64]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIGS)


def _check(status: int, where: str) -> None:
    if status != 0:
        raise SarahipError(status, where)


def _ptr(t) -> int | None:
    """Device pointer of a torch tensor (None passes NULL)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream(stream):
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def version() -> str:
    return lib.sh_version().decode()


# ---- measurement operator ------------------------------------------------------------------

def op_create(uv: np.ndarray, n: int, oversample: int, kernel_width: int, block_offsets) -> int:
    uv = _f64(uv)
    if uv.ndim != 2 or uv.shape[1] != 2:
        raise ValueError("uv must be (M, 2)")
    off = np.ascontiguousarray(block_offsets, dtype=np.int64)
    h = _vp()
    _check(lib.sh_op_create(uv.ctypes.data_as(_P64), uv.shape[0], n, oversample, kernel_width,
                            off.ctypes.data_as(_PI64), len(off) - 1, C.byref(h)), "op_create")
    return h.value


def op_create_tuned(uv: np.ndarray, n: int, oversample: int, kernel_width: int, block_offsets, tile: int = 0,
                    chunk: int = 0) -> int:
    uv = _f64(uv)
    if uv.ndim != 2 or uv.shape[1] != 2:
        raise ValueError("uv must be (M, 2)")
    off = np.ascontiguousarray(block_offsets, dtype=np.int64)
    h = _vp()
    _check(lib.sh_op_create_tuned(uv.ctypes.data_as(_P64), uv.shape[0], n, oversample, kernel_width,
                                  off.ctypes.data_as(_PI64), len(off) - 1, tile, chunk, C.byref(h)), "op_create_tuned")
    return h.value


def op_create_stream(uv: np.ndarray, n: int, oversample: int, kernel_width: int, block_offsets, tile: int = 0,
                     chunk: int = 0, stream=None) -> int:
    """op_create_tuned with the plan's uploads on `stream` (default: torch's current stream)."""
    uv = _f64(uv)
    if uv.ndim != 2 or uv.shape[1] != 2:
        raise ValueError("uv must be (M, 2)")
    off = np.ascontiguousarray(block_offsets, dtype=np.int64)
    h = _vp()
    _check(lib.sh_op_create_stream(uv.ctypes.data_as(_P64), uv.shape[0], n, oversample, kernel_width,
                                   off.ctypes.data_as(_PI64), len(off) - 1, tile, chunk, _stream(stream), C.byref(h)),
           "op_create_stream")
    return h.value


def device_bytes():
    """(device bytes the library holds, the SH_MAX_DEVICE_BYTES cap or -1)."""
    live, cap = C.c_int64(), C.c_int64()
    _check(lib.sh_device_bytes(C.byref(live), C.byref(cap)), "device_bytes")
    return live.value, cap.value


def op_create_batched(uv: np.ndarray, M_p, n: int, oversample: int, kernel_width: int, block_offsets, R_p,
                      tile: int = 0, chunk: int = 0) -> int:
    """One plan for P problems: uv and block_offsets concatenate the problems (see the C header)."""
    uv = _f64(uv)
    if uv.ndim != 2 or uv.shape[1] != 2:
        raise ValueError("uv must be (M, 2)")
    mp = np.ascontiguousarray(M_p, dtype=np.int64)
    rp = np.ascontiguousarray(R_p, dtype=np.int32)
    if mp.shape != rp.shape or mp.ndim != 1:
        raise ValueError("M_p and R_p must be 1-D of equal length")
    off = np.ascontiguousarray(block_offsets, dtype=np.int64)
    if len(off) != int(rp.sum()) + 1 or uv.shape[0] != int(mp.sum()):
        raise ValueError("block_offsets / uv do not match M_p / R_p")
    h = _vp()
    _check(lib.sh_op_create_batched(uv.ctypes.data_as(_P64), mp.ctypes.data_as(_PI64), len(mp), n, oversample,
                                    kernel_width, off.ctypes.data_as(_PI64), rp.ctypes.data_as(_PI32), tile, chunk,
                                    C.byref(h)), "op_create_batched")
    return h.value


def op_autotune(uv: np.ndarray, M_p, n: int, oversample: int, accuracy: float, block_offsets, R_p, reps: int = 3,
                stream=None):
    """Returns (plan handle, dict of the tuner's choice); arguments as op_create_batched."""
    uv = _f64(uv)
    mp = np.ascontiguousarray(M_p, dtype=np.int64)
    rp = np.ascontiguousarray(R_p, dtype=np.int32)
    off = np.ascontiguousarray(block_offsets, dtype=np.int64)
    if uv.ndim != 2 or uv.shape[1] != 2 or uv.shape[0] != int(mp.sum()) or len(off) != int(rp.sum()) + 1:
        raise ValueError("uv / block_offsets do not match M_p / R_p")
    res = TuneResult()
    h = _vp()
    _check(lib.sh_op_autotune(uv.ctypes.data_as(_P64), mp.ctypes.data_as(_PI64), len(mp), n, oversample, accuracy,
                              off.ctypes.data_as(_PI64), rp.ctypes.data_as(_PI32), reps, C.byref(res), C.byref(h),
                              _stream(stream)), "op_autotune")
    return h.value, res.as_dict()


def tune_cache_clear() -> None:
    """Forgets the process cache of op_autotune (a SH_TUNE_CACHE file stays)."""
    _check(lib.sh_tune_cache_clear(), "tune_cache_clear")


def kb_alias_error(kernel_width: int, oversample: int = 2) -> float:
    e = C.c_double()
    _check(lib.sh_kb_alias_error(kernel_width, oversample, C.byref(e)), "kb_alias_error")
    return e.value


def op_destroy(op: int) -> None:
    _check(lib.sh_op_destroy(op), "op_destroy")


def op_query(op: int) -> dict:
    out = np.zeros(10, dtype=np.int64)
    _check(lib.sh_op_query(op, out.ctypes.data_as(_PI64)), "op_query")
    keys = ("M", "n", "K", "J", "R", "n_items", "tile", "max_items_per_tile", "P", "n_sparse")
    return dict(zip(keys, (int(v) for v in out)))


def op_block_offsets(op: int) -> np.ndarray:
    R = op_query(op)["R"]
    out = np.zeros(R + 1, dtype=np.int64)
    _check(lib.sh_op_block_offsets(op, out.ctypes.data_as(_PI64)), "op_block_offsets")
    return out


def op_permutation(op: int) -> np.ndarray:
    M = op_query(op)["M"]
    out = np.zeros(M, dtype=np.int64)
    _check(lib.sh_op_permutation(op, out.ctypes.data_as(_PI64)), "op_permutation")
    return out


def phi_fwd(op, x, vis, stream=None):
    _check(lib.sh_phi_fwd(op, _ptr(x), _ptr(vis), _stream(stream)), "phi_fwd")


def phi_adj(op, vis, x, stream=None):
    _check(lib.sh_phi_adj(op, _ptr(vis), _ptr(x), _stream(stream)), "phi_adj")


def phi_fwd_internal(op, x, vis, stream=None):
    _check(lib.sh_phi_fwd_internal(op, _ptr(x), _ptr(vis), _stream(stream)), "phi_fwd_internal")


def phi_adj_internal(op, vis, x, stream=None):
    _check(lib.sh_phi_adj_internal(op, _ptr(vis), _ptr(x), _stream(stream)), "phi_adj_internal")


def vis_to_internal(op, user, internal, stream=None):
    _check(lib.sh_vis_to_internal(op, _ptr(user), _ptr(internal), _stream(stream)), "vis_to_internal")


def vis_to_user(op, internal, user, stream=None):
    _check(lib.sh_vis_to_user(op, _ptr(internal), _ptr(user), _stream(stream)), "vis_to_user")


def block_weights(op, stream=None) -> np.ndarray:
    """Density estimate of 1 / ||Phi_b|| per block (float64, R values)."""
    b = np.zeros(op_query(op)["R"], dtype=np.float64)
    _check(lib.sh_block_weights(op, b.ctypes.data_as(_P64), _stream(stream)), "block_weights")
    return b


def toeplitz_create(op, scale=None, stream=None):
    """Toeplitz form of scale_p Re(Phi^H Phi) for every problem of op; scale: P floats or None."""
    h = _vp()
    if scale is None:
        sp = None
    else:
        sc = np.ascontiguousarray(np.atleast_1d(np.asarray(scale, dtype=np.float64)))
        if sc.size != op_query(op)["P"]:
            raise ValueError("scale needs one value per problem")
        sp = sc.ctypes.data_as(_P64)
    _check(lib.sh_toeplitz_create(op, sp, C.byref(h), _stream(stream)), "toeplitz_create")
    return h


def toeplitz_workspace_bytes(op) -> int:
    b = C.c_size_t()
    _check(lib.sh_toeplitz_workspace_bytes(op, C.byref(b)), "toeplitz_workspace_bytes")
    return b.value


def toeplitz_create_ws(op, workspace, scale=None, stream=None):
    h = _vp()
    sp = None
    if scale is not None:
        sc = np.ascontiguousarray(np.atleast_1d(np.asarray(scale, dtype=np.float64)))
        sp = sc.ctypes.data_as(_P64)
    _check(lib.sh_toeplitz_create_ws(op, sp, _ptr(workspace), workspace.numel() * workspace.element_size(),
                                     C.byref(h), _stream(stream)), "toeplitz_create_ws")
    return h


def toeplitz_apply(t, x, out, stream=None):
    _check(lib.sh_toeplitz_apply(t, _ptr(x), _ptr(out), _stream(stream)), "toeplitz_apply")


def toeplitz_destroy(t):
    _check(lib.sh_toeplitz_destroy(t), "toeplitz_destroy")


def op_norm(op, x0, iters: int = 200, tol: float = 1e-12, stream=None):
    """||Phi||: a float for a one-problem plan, a float64 array of P values for a batched one."""
    P = op_query(op)["P"]
    nu = np.zeros(P, dtype=np.float64)
    _check(lib.sh_op_norm(op, _ptr(x0), iters, tol, nu.ctypes.data_as(_P64), _stream(stream)), "op_norm")
    return float(nu[0]) if P == 1 else nu


# ---- SARA dictionary ------------------------------------------------------------------------

def psi_create(n: int, levels: int = 4, basis_mask: int = SARA_MASK) -> int:
    h = _vp()
    _check(lib.sh_psi_create(n, levels, basis_mask, C.byref(h)), "psi_create")
    return h.value


def psi_create_batched(n: int, levels: int, basis_mask: int, batch: int) -> int:
    h = _vp()
    _check(lib.sh_psi_create_batched(n, levels, basis_mask, batch, C.byref(h)), "psi_create_batched")
    return h.value


def psi_workspace_bytes(n: int, levels: int, basis_mask: int, batch: int = 1) -> int:
    b = C.c_size_t()
    _check(lib.sh_psi_workspace_bytes(n, levels, basis_mask, batch, C.byref(b)), "psi_workspace_bytes")
    return b.value


def psi_create_ws(n: int, levels: int, basis_mask: int, batch: int, workspace) -> int:
    h = _vp()
    _check(lib.sh_psi_create_ws(n, levels, basis_mask, batch, _ptr(workspace),
                                workspace.numel() * workspace.element_size(), C.byref(h)), "psi_create_ws")
    return h.value


def psi_destroy(psi: int) -> None:
    _check(lib.sh_psi_destroy(psi), "psi_destroy")


def psi_planes(psi: int) -> int:
    q = C.c_int32()
    _check(lib.sh_psi_planes(psi, C.byref(q)), "psi_planes")
    return q.value


def daubechies(p: int) -> np.ndarray:
    h = np.zeros(2 * p, dtype=np.float64)
    _check(lib.sh_daubechies(p, h.ctypes.data_as(_P64)), "daubechies")
    return h


def psi_fwd(psi, coeffs, x, stream=None):
    _check(lib.sh_psi_fwd(psi, _ptr(coeffs), _ptr(x), _stream(stream)), "psi_fwd")


def psi_adj(psi, x, coeffs, stream=None):
    _check(lib.sh_psi_adj(psi, _ptr(x), _ptr(coeffs), _stream(stream)), "psi_adj")


# ---- proximal steps -------------------------------------------------------------------------

def prox_l1(s, z, W, gamma: float, v_out, stream=None):
    _check(lib.sh_prox_l1(s.numel(), _ptr(s), _ptr(z), _ptr(W), gamma, _ptr(v_out), _stream(stream)), "prox_l1")


def prox_pos(s, z, v_out, stream=None):
    _check(lib.sh_prox_pos(s.numel(), _ptr(s), _ptr(z), _ptr(v_out), _stream(stream)), "prox_pos")


def prox_ball(op, s, z, yhat, eps_dev, v_out, resid_out, stream=None):
    _check(lib.sh_prox_ball(op, _ptr(s), _ptr(z), _ptr(yhat), _ptr(eps_dev), _ptr(v_out), _ptr(resid_out),
                            _stream(stream)), "prox_ball")


def prox_ball_noalloc(op, s, z, yhat, eps_dev, v_out, resid_out, stream=None):
    """sh_prox_ball without device allocation or synchronisation (async)."""
    _check(lib.sh_prox_ball_noalloc(op, _ptr(s), _ptr(z), _ptr(yhat), _ptr(eps_dev), _ptr(v_out), _ptr(resid_out),
                                    _stream(stream)), "prox_ball_noalloc")


def reweight(c, delta: float, W_out, stream=None):
    _check(lib.sh_reweight(c.numel(), _ptr(c), delta, _ptr(W_out), _stream(stream)), "reweight")


def std(c, stream=None) -> float:
    out = C.c_double()
    _check(lib.sh_std(c.numel(), _ptr(c), C.byref(out), _stream(stream)), "std")
    return out.value


# ---- SDMM -----------------------------------------------------------------------------------

def sdmm_default_params() -> SdmmParams:
    p = SdmmParams()
    lib.sh_sdmm_default_params(C.byref(p))
    return p


def sdmm_solve(op, psi, y, eps, W, x0, params: SdmmParams, x_out, W_out=None, stream=None):
    """Returns (info, block residuals ||y_i - Phi_i x|| as float64 numpy); info is a dict for a
    one-problem plan and a list of P dicts for a batched one."""
    eps = _f64(eps)
    R = len(eps)
    P = op_query(op)["P"]
    resid = np.zeros(R, dtype=np.float64)
    info = (SdmmInfo * P)()
    _check(lib.sh_sdmm_solve(op, psi, _ptr(y), eps.ctypes.data_as(_P64), _ptr(W), _ptr(x0), C.byref(params),
                             _ptr(x_out), _ptr(W_out), resid.ctypes.data_as(_P64),
                             C.cast(info, C.POINTER(SdmmInfo)), _stream(stream)), "sdmm_solve")
    dicts = [i.as_dict() for i in info]
    return (dicts[0] if P == 1 else dicts), resid


def workspace_bytes(op, psi, params: SdmmParams) -> int:
    b = C.c_size_t()
    _check(lib.sh_workspace_bytes(op, psi, C.byref(params), C.byref(b)), "workspace_bytes")
    return b.value


def sdmm_solve_ws(op, psi, y, eps, W, x0, params: SdmmParams, x_out, workspace, W_out=None, stream=None):
    """sdmm_solve with the device memory of the solve taken from `workspace` (a uint8 device tensor)."""
    eps = _f64(eps)
    P = op_query(op)["P"]
    resid = np.zeros(len(eps), dtype=np.float64)
    info = (SdmmInfo * P)()
    _check(lib.sh_sdmm_solve_ws(op, psi, _ptr(y), eps.ctypes.data_as(_P64), _ptr(W), _ptr(x0), C.byref(params),
                                _ptr(x_out), _ptr(W_out), resid.ctypes.data_as(_P64), C.cast(info, C.POINTER(SdmmInfo)),
                                _ptr(workspace), workspace.numel() * workspace.element_size(), _stream(stream)),
           "sdmm_solve_ws")
    dicts = [i.as_dict() for i in info]
    return (dicts[0] if P == 1 else dicts), resid


def sdmm_create_ws(op, psi, y, eps, W, x0, params: SdmmParams, workspace, stream=None) -> int:
    eps = _f64(eps)
    h = _vp()
    _check(lib.sh_sdmm_create_ws(op, psi, _ptr(y), eps.ctypes.data_as(_P64), _ptr(W), _ptr(x0), C.byref(params),
                                 _ptr(workspace), workspace.numel() * workspace.element_size(), C.byref(h),
                                 _stream(stream)), "sdmm_create_ws")
    return h.value


def sdmm_create(op, psi, y, eps, W, x0, params: SdmmParams, stream=None) -> int:
    eps = _f64(eps)
    h = _vp()
    _check(lib.sh_sdmm_create(op, psi, _ptr(y), eps.ctypes.data_as(_P64), _ptr(W), _ptr(x0), C.byref(params),
                              C.byref(h), _stream(stream)), "sdmm_create")
    return h.value


def sdmm_iterate(s: int, iters: int, stream=None) -> None:
    _check(lib.sh_sdmm_iterate(s, iters, _stream(stream)), "sdmm_iterate")


def sdmm_result(s: int, x_out=None, R: int = 0, stream=None, P: int = 1):
    """Returns (block residuals as float64 numpy of length R, relative change: a float, or P
    values for a batched session)."""
    resid = np.zeros(max(R, 1), dtype=np.float64)
    rel = np.zeros(P, dtype=np.float64)
    _check(lib.sh_sdmm_result(s, _ptr(x_out), resid.ctypes.data_as(_P64) if R else None, rel.ctypes.data_as(_P64),
                              _stream(stream)), "sdmm_result")
    return resid[:R], (float(rel[0]) if P == 1 else rel)


def sdmm_kkt(s: int, P: int = 1, stream=None):
    """Returns (kkt_primal, kkt_dual, objective) of the session's current state: floats, or arrays of P
    values for a batched session."""
    pr, du, ob = (np.zeros(P, dtype=np.float64) for _ in range(3))
    _check(lib.sh_sdmm_kkt(s, pr.ctypes.data_as(_P64), du.ctypes.data_as(_P64), ob.ctypes.data_as(_P64),
                           _stream(stream)), "sdmm_kkt")
    return (float(pr[0]), float(du[0]), float(ob[0])) if P == 1 else (pr, du, ob)


def sdmm_state_export(s: int, stream=None) -> np.ndarray:
    """The session's state (checkpoint) as a host byte array."""
    nb_ = C.c_size_t()
    _check(lib.sh_sdmm_state_bytes(s, C.byref(nb_)), "sdmm_state_bytes")
    buf = np.empty(nb_.value, dtype=np.uint8)
    _check(lib.sh_sdmm_state_export(s, buf.ctypes.data, nb_.value, _stream(stream)), "sdmm_state_export")
    return buf


def sdmm_state_import(s: int, state: np.ndarray, stream=None) -> None:
    """Overwrites the session's state with one from sdmm_state_export of a like session."""
    buf = np.ascontiguousarray(state, dtype=np.uint8)
    _check(lib.sh_sdmm_state_import(s, buf.ctypes.data, buf.nbytes, _stream(stream)), "sdmm_state_import")


def sdmm_metrics_enable(s: int, rows: int) -> int:
    """Gives the session a ring of `rows` per-iteration metric rows (0: off); returns the row width 2P + R."""
    w = _i32()
    _check(lib.sh_sdmm_metrics_enable(s, int(rows), C.byref(w)), "sdmm_metrics_enable")
    return w.value


def sdmm_metrics_read(s: int, P: int, R: int, max_rows: int, stream=None) -> dict:
    """The metric rows not yet read (oldest first, at most max_rows): relative change and objective per problem
    ((rows, P) arrays), residual over eps per block ((rows, R)), and the iteration count after the first row."""
    buf = np.zeros((max(int(max_rows), 1), 2 * P + R), dtype=np.float64)
    n = _i32()
    first = _i64()
    _check(lib.sh_sdmm_metrics_read(s, buf.ctypes.data_as(_P64), int(max_rows), C.byref(n), C.byref(first),
                                    _stream(stream)), "sdmm_metrics_read")
    rows = buf[:n.value]
    return {"rel_change": rows[:, :P].copy(), "objective": rows[:, P:2 * P].copy(),
            "resid_over_eps": rows[:, 2 * P:].copy(), "first_iter": int(first.value), "rows": n.value}


def sdmm_destroy(s: int) -> None:
    _check(lib.sh_sdmm_destroy(s), "sdmm_destroy")


# ---- learned warm start ---------------------------------------------------------------------

_PF32 = C.POINTER(C.c_float)


def unet_create(base: int = 32, levels: int = 4) -> int:
    h = _vp()
    _check(lib.sh_unet_create(base, levels, C.byref(h)), "unet_create")
    return h.value


def unet_destroy(u: int) -> None:
    _check(lib.sh_unet_destroy(u), "unet_destroy")


def unet_num_params(u: int) -> int:
    n = C.c_int64()
    _check(lib.sh_unet_num_params(u, C.byref(n)), "unet_num_params")
    return n.value


def unet_set_params(u: int, flat: np.ndarray) -> None:
    a = np.ascontiguousarray(flat, dtype=np.float32)
    _check(lib.sh_unet_set_params(u, a.ctypes.data_as(_PF32), a.size), "unet_set_params")


def unet_get_params(u: int) -> np.ndarray:
    a = np.zeros(unet_num_params(u), dtype=np.float32)
    _check(lib.sh_unet_get_params(u, a.ctypes.data_as(_PF32), a.size), "unet_get_params")
    return a


def _bhw(x):
    if x.dim() == 2:
        return 1, x.shape[0], x.shape[1]
    if x.dim() == 3:
        return x.shape[0], x.shape[1], x.shape[2]
    raise ValueError("images must be (H, W) or (B, H, W)")


def unet_forward(u: int, x, y, stream=None) -> None:
    B, H, W = _bhw(x)
    _check(lib.sh_unet_forward(u, _ptr(x), B, H, W, _ptr(y), _stream(stream)), "unet_forward")


def unet_loss_grad(u: int, x, target, want_grads: bool = True, stream=None):
    """Returns (loss, flat float32 gradient or None)."""
    B, H, W = _bhw(x)
    loss = C.c_double()
    g = np.zeros(unet_num_params(u), dtype=np.float32) if want_grads else None
    _check(lib.sh_unet_loss_grad(u, _ptr(x), _ptr(target), B, H, W, C.byref(loss),
                                 g.ctypes.data_as(_PF32) if want_grads else None, _stream(stream)), "unet_loss_grad")
    return loss.value, g


def unet_train_step(u: int, x, target, lr: float, want_loss: bool = True, stream=None):
    B, H, W = _bhw(x)
    loss = C.c_double()
    _check(lib.sh_unet_train_step(u, _ptr(x), _ptr(target), B, H, W, lr, C.byref(loss) if want_loss else None,
                                  _stream(stream)), "unet_train_step")
    return loss.value if want_loss else None


def warm_start(u: int, op: int, y, x0_out, stream=None) -> None:
    _check(lib.sh_warm_start(u, op, _ptr(y), _ptr(x0_out), _stream(stream)), "warm_start")


def dirty_normalised(op: int, y, d_out, scale_out, stream=None) -> None:
    _check(lib.sh_dirty_normalised(op, _ptr(y), _ptr(d_out), _ptr(scale_out), _stream(stream)), "dirty_normalised")


def scale_images(x, scale, invert: bool = False, stream=None) -> None:
    P = scale.numel()
    _check(lib.sh_scale_images(_ptr(x), _ptr(scale), P, x.numel() // P, 1 if invert else 0, _stream(stream)),
           "scale_images")


# ---- timing ---------------------------------------------------------------------------------

def profile_enable(on: bool = True) -> None:
    _check(lib.sh_profile_enable(1 if on else 0), "profile_enable")


def profile_read(name: str):
    cnt = C.c_int64()
    ms = C.c_double()
    _check(lib.sh_profile_read(name.encode(), C.byref(cnt), C.byref(ms)), "profile_read")
    return cnt.value, ms.value
