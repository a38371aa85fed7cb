"""Python binding of the MPR gap-filling library (include/mpr.h).

Argument marshalling only: every step runs in the HIP kernels of
``libmpr.so``.  Device buffers are torch tensors on a ROCm device (torch is
used for memory and streams); host outputs come back as numpy arrays.  If the
shared library is missing or cannot be loaded, importing works but every call
raises ``MprLibraryError``: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpr.so")

MPR_OK, MPR_ERR_ARG, MPR_ERR_DEGENERATE, MPR_ERR_WORKSPACE, MPR_ERR_HIP, MPR_INCOMPLETE = range(6)
FLAG_KEPT, FLAG_ACCEPTED, FLAG_WRAPPED, FLAG_UPDATED, FLAG_FP64 = 1, 2, 4, 8, 16

# Every symbol include/mpr.h declares.
EXPORTS = [
    "mpr_create", "mpr_destroy", "mpr_last_error", "mpr_default_params", "mpr_workspace_size",
    "mpr_map_to_angles", "mpr_estimate_temperature", "mpr_simulate", "mpr_simulate_noalloc",
    "mpr_simulate_noalloc_max_bytes", "mpr_predict", "mpr_spread",
    "mpr_quantiles", "mpr_select_q", "mpr_select_q_workspace_size",
    "mpr_profile_enable", "mpr_profile_read",
    "mpr_cnn_param_count", "mpr_cnn_packed_bytes", "mpr_cnn_workspace_size", "mpr_cnn_pack", "mpr_cnn_encode",
    "mpr_cnn_forward", "mpr_cnn_infer", "mpr_cnn_loss", "mpr_cnn_backward", "mpr_cnn_opt_step", "mpr_cnn_decode",
    "mpr_cnn_diag_conv", "mpr_cnn_diag_wgrad",
    "mpr_diag_philox", "mpr_diag_half_sweep", "mpr_diag_half_sweep_fp64", "mpr_diag_copy", "mpr_diag_energy", "mpr_diag_sg_slope",
]


class MprLibraryError(RuntimeError):
    pass


class MprError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mpr error {code}: {msg}")
        self.code = code


class Image(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("offset", C.c_int64),
                ("id", C.c_uint32), ("reserved", C.c_uint32)]


class Params(C.Structure):
    _fields_ = [
        ("q", C.c_double), ("R", C.c_int32), ("K", C.c_int32), ("n_f", C.c_int32),
        ("n_fit", C.c_int32), ("sg_degree", C.c_int32), ("i_max", C.c_int32),
        ("a_targ", C.c_double), ("k_a", C.c_double), ("fixed_relax", C.c_int32),
        ("eq_a_mode", C.c_int32), ("table_nT", C.c_int32), ("table_burn", C.c_int32),
        ("table_meas", C.c_int32), ("tile_rows", C.c_int32), ("table_T_lo", C.c_double),
        ("table_T_hi", C.c_double), ("seed", C.c_uint64), ("sweeps_per_launch", C.c_int32),
        ("spread", C.c_int32), ("fp64", C.c_int32), ("table_side_cap", C.c_int32),
        ("warm_min_states", C.c_int32), ("sweep_limit", C.c_int32), ("resume", C.c_int32),
        ("barrier_timeout_us", C.c_int32),
    ]


class Profile(C.Structure):
    _fields_ = [("sweep_kernel_ms", C.c_double), ("sweep_launches", C.c_int64),
                ("chain_sweeps", C.c_int64), ("site_updates", C.c_int64), ("useful_bytes", C.c_double),
                ("last_tile", C.c_int32), ("reserved", C.c_int32)]


class ChainStats(C.Structure):
    _fields_ = [("relax_sweeps", C.c_int32), ("not_converged", C.c_int32),
                ("a_final", C.c_double), ("A_last", C.c_double), ("k_last", C.c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libmpr.so (building it first only when it does not exist)."""
    global _lib
    if _lib is not None:
        return _lib
    try:
        # torch ships its own HIP runtime with the same soname as the one the
        # library links; loading torch first makes the process use exactly
        # one runtime (the library then binds to torch's copy).
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(path):
        from . import build as _build
        try:
            _build.build()
        except Exception as e:  # no compiler: no library, no fallback
            raise MprLibraryError(f"{path} is missing and could not be built: {e}") from e
    try:
        lib = C.CDLL(path)
    except OSError as e:
        raise MprLibraryError(f"cannot load {path}: {e}") from e
    _declare(lib)
    _lib = lib
    return lib


TILE_COMPACT = 0x100  # Params.tile_rows flag: the compacted sweep shape
TILE_FUSED = 0x200  # Params.tile_rows flag: the fused tile sweep (rows 8, 12, 16, 24, 32 or 48)
TILE_PERSIST = 0x400  # with TILE_FUSED (rows 8 to 32): many fused sweeps per cooperative launch


def _declare(L):
    P, i32, i64, u32, u64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
    IMG, PRM = C.POINTER(Image), C.POINTER(Params)
    sig = {
        "mpr_create": (i32, [C.POINTER(C.c_void_p), i32]),
        "mpr_destroy": (None, [P]),
        "mpr_last_error": (C.c_char_p, [P]),
        "mpr_default_params": (None, [PRM]),
        "mpr_workspace_size": (i64, [IMG, i32, PRM]),
        "mpr_map_to_angles": (i32, [P, IMG, i32, P, P, P, P, P]),
        "mpr_estimate_temperature": (i32, [P, IMG, i32, P, P, PRM, P, i64, P, P, P, P]),
        "mpr_simulate": (i32, [P, IMG, i32, P, P, P, PRM, P, P, i64, P, P, P, C.POINTER(ChainStats), P]),
        "mpr_simulate_noalloc": (i32, [P, IMG, i32, P, P, P, PRM, P, P, P, P, C.POINTER(ChainStats), P]),
        "mpr_simulate_noalloc_max_bytes": (i64, []),
        "mpr_quantiles": (i32, [P, IMG, i32, P, P, P, i32, P, i32, P, P, P]),
        "mpr_select_q_workspace_size": (i64, [IMG, PRM, P, i32]),
        "mpr_select_q": (i32, [P, IMG, P, P, PRM, P, i32, d, P, i64, P, P, P, P]),
        "mpr_predict": (i32, [P, IMG, i32, P, P, P, P, i32, P, P]),
        "mpr_spread": (i32, [P, IMG, i32, P, P, P, i32, P, P]),
        "mpr_cnn_param_count": (i64, []),
        "mpr_cnn_packed_bytes": (i64, []),
        "mpr_cnn_workspace_size": (i64, [i32, i32, i32, i32]),
        "mpr_cnn_pack": (i32, [P, P, P, P]),
        "mpr_cnn_encode": (i32, [P, i32, i32, i32, P, P, P, P]),
        "mpr_cnn_forward": (i32, [P, i32, i32, i32, P, P, P, P, i64, i32, P, P]),
        "mpr_cnn_infer": (i32, [P, i32, i32, i32, P, P, P, P, P, i64, P, P]),
        "mpr_cnn_loss": (i32, [P, i32, i32, i32, P, P, P, i64, P, P, i64, P, P]),
        "mpr_cnn_backward": (i32, [P, i32, i32, i32, P, P, P, P, P, i64, P, P]),
        "mpr_cnn_opt_step": (i32, [P, P, P, P, P, i64, d, d, d, d, P]),
        "mpr_cnn_decode": (i32, [P, i32, i32, i32, P, P, P, P]),
        "mpr_cnn_diag_conv": (i32, [P, i32, i32, i32, P, P, P, P, P, i32, P, P]),
        "mpr_cnn_diag_wgrad": (i32, [P, i32, i32, i32, P, P, P, P, P, i64, P]),
        "mpr_profile_enable": (i32, [P, i32]),
        "mpr_profile_read": (i32, [P, C.POINTER(Profile)]),
        "mpr_diag_philox": (i32, [P, P, u64, i64, P, P]),
        "mpr_diag_half_sweep": (i32, [P, i32, i32, P, P, i32, d, d, d, u64, u32, u32, u32, i32, i32, P, P, P, P]),
        "mpr_diag_half_sweep_fp64": (i32, [P, i32, i32, P, P, i32, d, d, d, u64, u32, u32, u32, i32, i32, P, P, P,
                                           P]),
        "mpr_diag_copy": (i32, [P, P, P, i64, P]),
        "mpr_diag_energy": (i32, [P, i32, i32, P, d, P, P]),
        "mpr_diag_sg_slope": (i32, [P, P, i32, i32, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


def default_params(**kw) -> Params:
    p = Params()
    load().mpr_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def images(shapes, ids=None):
    """ctypes array of mpr_image for a packed batch of (ny, nx) shapes."""
    arr = (Image * len(shapes))()
    off = 0
    for b, (ny, nx) in enumerate(shapes):
        arr[b].nx, arr[b].ny, arr[b].offset = nx, ny, off
        arr[b].id = b if ids is None else ids[b]
        off += nx * ny
    return arr


def sites_of(imgs) -> int:
    """Length of the packed per-site buffers of a batch: the end of its
    furthest image."""
    return max(int(im.offset) + int(im.nx) * int(im.ny) for im in imgs)


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Context:
    """An mpr_ctx on one device; methods mirror the C calls."""

    def __init__(self, device: int = 0):
        self.lib = load()
        self._h = C.c_void_p()
        rc = self.lib.mpr_create(C.byref(self._h), device)
        if rc != MPR_OK:
            raise MprError(rc, f"mpr_create(device={device}) failed")
        self.device = device

    def close(self):
        if self._h:
            self.lib.mpr_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != MPR_OK:
            raise MprError(rc, self.lib.mpr_last_error(self._h).decode())

    def _t(self, t, name, dtype=None, numel=0, optional=False, nbytes=0):
        """Device pointer of tensor t after checking it: on this context's
        GPU, contiguous, of dtype (None: any, for workspaces) and holding at
        least numel elements (and nbytes bytes), the extent the call reads or
        writes.  A host tensor or a short buffer would otherwise reach a
        kernel."""
        import torch
        if t is None:
            if optional:
                return None
            raise ValueError(f"{name}: a tensor is required")
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.device.index != self.device:
            raise ValueError(f"{name}: must be a tensor on cuda:{self.device}")
        if dtype is not None and t.dtype != dtype:
            raise TypeError(f"{name}: dtype {t.dtype}, expected {dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name}: must be contiguous")
        if t.numel() < numel:
            raise ValueError(f"{name}: {t.numel()} elements, the call needs {numel}")
        if t.numel() * t.element_size() < nbytes:
            raise ValueError(f"{name}: {t.numel() * t.element_size()} bytes, the call needs {nbytes}")
        return C.c_void_p(t.data_ptr())

    def _cnn_sizes(self, n, h, w):
        return n * h * w, int(self.lib.mpr_cnn_param_count()), int(self.lib.mpr_cnn_packed_bytes())

    # -------------------------------------------------------------- calls
    def workspace_size(self, imgs, params) -> int:
        return int(self.lib.mpr_workspace_size(imgs, len(imgs), C.byref(params)))

    def map_to_angles(self, imgs, z, sampled, phi, stream=None) -> np.ndarray:
        import torch
        n = sites_of(imgs)
        zz = np.zeros(2 * len(imgs))
        self._check(self.lib.mpr_map_to_angles(self._h, imgs, len(imgs), self._t(z, "z", torch.float32, n),
                                               self._t(sampled, "sampled", torch.uint8, n),
                                               self._t(phi, "phi", torch.float32, n),
                                               zz.ctypes.data_as(C.c_void_p), _stream(stream)))
        return zz

    def estimate_temperature(self, imgs, phi, sampled, params, ws, stream=None):
        import torch
        n = len(imgs)
        ns = sites_of(imgs)
        e_s, T = np.zeros(n), np.zeros(n)
        cl = np.zeros(n, dtype=np.int32)
        self._check(self.lib.mpr_estimate_temperature(
            self._h, imgs, n, self._t(phi, "phi", torch.float32, ns), self._t(sampled, "sampled", torch.uint8, ns),
            C.byref(params), self._t(ws, "ws"), ws.numel() * ws.element_size(),
            e_s.ctypes.data_as(C.c_void_p), T.ctypes.data_as(C.c_void_p), cl.ctypes.data_as(C.c_void_p),
            _stream(stream)))
        return e_s, T, cl

    def _simulate(self, fn, ws_args, imgs, phi, sampled, T_hat, params, phi_sum, phi_init, stream, phi_m2,
                  phi_states, allow_incomplete):
        import torch
        n = len(imgs)
        ns = sites_of(imgs)
        T = np.ascontiguousarray(T_hat, dtype=np.float64)
        if T.size < n:
            raise ValueError(f"T_hat: {T.size} values for {n} images")
        st = (ChainStats * (n * params.R))()
        f32 = torch.float32
        rc = fn(self._h, imgs, n, self._t(phi, "phi", f32, ns), self._t(sampled, "sampled", torch.uint8, ns),
                T.ctypes.data_as(C.c_void_p), C.byref(params),
                self._t(phi_init, "phi_init", f32, ns, optional=True), *ws_args,
                self._t(phi_sum, "phi_sum", f32, ns), self._t(phi_m2, "phi_m2", f32, ns, optional=True),
                self._t(phi_states, "phi_states", f32, max(0, params.R * params.K) * ns, optional=True), st,
                _stream(stream))
        if not (allow_incomplete and rc == MPR_INCOMPLETE):
            self._check(rc)
        stats = [dict(relax_sweeps=s.relax_sweeps, not_converged=s.not_converged, a_final=s.a_final,
                      A_last=s.A_last, k_last=s.k_last) for s in st]
        return (rc == MPR_OK, stats) if allow_incomplete else stats

    def simulate(self, imgs, phi, sampled, T_hat, params, ws, phi_sum, phi_init=None, stream=None, phi_m2=None,
                 phi_states=None, allow_incomplete=False):
        """Per-chain statistics; with allow_incomplete, (done, statistics),
        done False when params.sweep_limit stopped the run (resume it with
        params.resume = 1 on the same workspace contents)."""
        return self._simulate(self.lib.mpr_simulate, (self._t(ws, "ws"), ws.numel() * ws.element_size()), imgs,
                              phi, sampled, T_hat, params, phi_sum, phi_init, stream, phi_m2, phi_states,
                              allow_incomplete)

    def simulate_noalloc(self, imgs, phi, sampled, T_hat, params, phi_sum, phi_init=None, stream=None, phi_m2=None,
                         phi_states=None, allow_incomplete=False):
        """simulate() on the library's static per-device workspace (no
        workspace argument, nothing allocated by the call)."""
        return self._simulate(self.lib.mpr_simulate_noalloc, (), imgs, phi, sampled, T_hat, params, phi_sum,
                              phi_init, stream, phi_m2, phi_states, allow_incomplete)

    def predict(self, imgs, z, sampled, phi_sum, zmin_zmax, M, z_hat, stream=None):
        import torch
        ns = sites_of(imgs)
        zz = np.ascontiguousarray(zmin_zmax, dtype=np.float64)
        if zz.size < 2 * len(imgs):
            raise ValueError("zmin_zmax: two values per image")
        self._check(self.lib.mpr_predict(self._h, imgs, len(imgs), self._t(z, "z", torch.float32, ns),
                                         self._t(sampled, "sampled", torch.uint8, ns),
                                         self._t(phi_sum, "phi_sum", torch.float32, ns),
                                         zz.ctypes.data_as(C.c_void_p), M, self._t(z_hat, "z_hat", torch.float32, ns),
                                         _stream(stream)))

    def quantiles(self, imgs, z, sampled, phi_states, M, probs, zmin_zmax, z_q, stream=None):
        """Per-site quantiles (probs) of the M recorded states, back-transformed;
        z_q holds len(probs) rows of the packed sites."""
        import torch
        ns = sites_of(imgs)
        pr = np.ascontiguousarray(probs, dtype=np.float64)
        zz = np.ascontiguousarray(zmin_zmax, dtype=np.float64)
        if zz.size < 2 * len(imgs):
            raise ValueError("zmin_zmax: two values per image")
        self._check(self.lib.mpr_quantiles(self._h, imgs, len(imgs), self._t(z, "z", torch.float32, ns),
                                           self._t(sampled, "sampled", torch.uint8, ns),
                                           self._t(phi_states, "phi_states", torch.float32, max(M, 0) * ns), M,
                                           pr.ctypes.data_as(C.c_void_p), pr.size, zz.ctypes.data_as(C.c_void_p),
                                           self._t(z_q, "z_q", torch.float32, pr.size * ns), _stream(stream)))

    def select_q_workspace_size(self, img, params, q_grid) -> int:
        qg = np.ascontiguousarray(q_grid, dtype=np.float64)
        return int(self.lib.mpr_select_q_workspace_size(img, C.byref(params), qg.ctypes.data_as(C.c_void_p),
                                                        qg.size))

    def select_q(self, img, z, sampled, params, q_grid, holdout, ws, stream=None):
        """Hold-out choice of q for one image (img: a one-image array from
        images()); returns (q_best, validation MAE per q, T_hat per q)."""
        import torch
        ns = sites_of(img[:1])
        qg = np.ascontiguousarray(q_grid, dtype=np.float64)
        mae = np.zeros(qg.size)
        T = np.zeros(qg.size)
        qb = C.c_double()
        self._check(self.lib.mpr_select_q(self._h, img, self._t(z, "z", torch.float32, ns),
                                          self._t(sampled, "sampled", torch.uint8, ns), C.byref(params),
                                          qg.ctypes.data_as(C.c_void_p), qg.size, holdout, self._t(ws, "ws"),
                                          ws.numel() * ws.element_size(), mae.ctypes.data_as(C.c_void_p),
                                          T.ctypes.data_as(C.c_void_p), C.byref(qb), _stream(stream)))
        return qb.value, mae, T

    def spread(self, imgs, sampled, phi_m2, zmin_zmax, M, z_std, stream=None):
        import torch
        ns = sites_of(imgs)
        zz = np.ascontiguousarray(zmin_zmax, dtype=np.float64)
        if zz.size < 2 * len(imgs):
            raise ValueError("zmin_zmax: two values per image")
        self._check(self.lib.mpr_spread(self._h, imgs, len(imgs), self._t(sampled, "sampled", torch.uint8, ns),
                                        self._t(phi_m2, "phi_m2", torch.float32, ns),
                                        zz.ctypes.data_as(C.c_void_p), M, self._t(z_std, "z_std", torch.float32, ns),
                                        _stream(stream)))

    # -------------------------------------------------------- warm start
    # Tensors: x, y, dy are (n, h, w, 32) bfloat16; phi, sampled (n, h, w);
    # target (n, h, w, 2) float; params / grads / Adam moments float vectors.
    def cnn_param_count(self) -> int:
        return int(self.lib.mpr_cnn_param_count())

    def cnn_packed_bytes(self) -> int:
        return int(self.lib.mpr_cnn_packed_bytes())

    def cnn_workspace_size(self, n, h, w, training) -> int:
        return int(self.lib.mpr_cnn_workspace_size(n, h, w, 1 if training else 0))

    def cnn_pack(self, params, packed, stream=None):
        import torch
        _, pc, pb = self._cnn_sizes(0, 0, 0)
        self._check(self.lib.mpr_cnn_pack(self._h, self._t(params, "params", torch.float32, pc),
                                          self._t(packed, "packed", nbytes=pb), _stream(stream)))

    def cnn_encode(self, phi, sampled, x, stream=None):
        import torch
        n, h, w = phi.shape
        px, _, _ = self._cnn_sizes(n, h, w)
        self._check(self.lib.mpr_cnn_encode(self._h, n, h, w, self._t(phi, "phi", torch.float32, px),
                                            self._t(sampled, "sampled", torch.uint8, px),
                                            self._t(x, "x", torch.bfloat16, 32 * px), _stream(stream)))

    def cnn_forward(self, params, packed, x, ws, y, training=False, stream=None):
        import torch
        n, h, w, _ = x.shape
        px, pc, pb = self._cnn_sizes(n, h, w)
        self._check(self.lib.mpr_cnn_forward(self._h, n, h, w, self._t(params, "params", torch.float32, pc),
                                             self._t(packed, "packed", nbytes=pb),
                                             self._t(x, "x", torch.bfloat16, 32 * px), self._t(ws, "ws"),
                                             ws.numel() * ws.element_size(), 1 if training else 0,
                                             self._t(y, "y", torch.bfloat16, 32 * px), _stream(stream)))

    def cnn_infer(self, params, packed, phi, sampled, ws, phi_init, stream=None):
        """encode + forward (inference) + decode in one call, phi_init out."""
        import torch
        n, h, w = phi.shape
        px, pc, pb = self._cnn_sizes(n, h, w)
        self._check(self.lib.mpr_cnn_infer(self._h, n, h, w, self._t(params, "params", torch.float32, pc),
                                           self._t(packed, "packed", nbytes=pb),
                                           self._t(phi, "phi", torch.float32, px),
                                           self._t(sampled, "sampled", torch.uint8, px), self._t(ws, "ws"),
                                           ws.numel() * ws.element_size(),
                                           self._t(phi_init, "phi_init", torch.float32, px), _stream(stream)))

    def cnn_loss(self, y, target, sampled, n_gaps, dy, ws, stream=None) -> float:
        import torch
        n, h, w, _ = y.shape
        px, _, _ = self._cnn_sizes(n, h, w)
        out = C.c_double()
        self._check(self.lib.mpr_cnn_loss(self._h, n, h, w, self._t(y, "y", torch.bfloat16, 32 * px),
                                          self._t(target, "target", torch.float32, 2 * px),
                                          self._t(sampled, "sampled", torch.uint8, px), int(n_gaps),
                                          self._t(dy, "dy", torch.bfloat16, 32 * px), self._t(ws, "ws"),
                                          ws.numel() * ws.element_size(), C.byref(out), _stream(stream)))
        return out.value

    def cnn_backward(self, params, packed, x, dy, ws, grads, stream=None):
        import torch
        n, h, w, _ = x.shape
        px, pc, pb = self._cnn_sizes(n, h, w)
        self._check(self.lib.mpr_cnn_backward(self._h, n, h, w, self._t(params, "params", torch.float32, pc),
                                              self._t(packed, "packed", nbytes=pb),
                                              self._t(x, "x", torch.bfloat16, 32 * px),
                                              self._t(dy, "dy", torch.bfloat16, 32 * px), self._t(ws, "ws"),
                                              ws.numel() * ws.element_size(),
                                              self._t(grads, "grads", torch.float32, pc), _stream(stream)))

    def cnn_opt_step(self, params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        import torch
        _, pc, _ = self._cnn_sizes(0, 0, 0)
        f32 = torch.float32
        self._check(self.lib.mpr_cnn_opt_step(self._h, self._t(params, "params", f32, pc),
                                              self._t(grads, "grads", f32, pc), self._t(m, "m", f32, pc),
                                              self._t(v, "v", f32, pc), int(step), lr, beta1, beta2, eps,
                                              _stream(stream)))

    def cnn_decode(self, y, sampled, phi_init, stream=None):
        import torch
        n, h, w, _ = y.shape
        px, _, _ = self._cnn_sizes(n, h, w)
        self._check(self.lib.mpr_cnn_decode(self._h, n, h, w, self._t(y, "y", torch.bfloat16, 32 * px),
                                            self._t(sampled, "sampled", torch.uint8, px),
                                            self._t(phi_init, "phi_init", torch.float32, px), _stream(stream)))

    def cnn_diag_conv(self, x, wpack, bias, out, add=None, ref=None, relu=False, stream=None):
        import torch
        n, h, w, _ = x.shape
        px = n * h * w
        bf = torch.bfloat16
        self._check(self.lib.mpr_cnn_diag_conv(self._h, n, h, w, self._t(x, "x", bf, 32 * px),
                                               self._t(wpack, "wpack", nbytes=9 * 32 * 32 * 2),
                                               self._t(bias, "bias", torch.float32, 32, optional=True),
                                               self._t(add, "add", bf, 32 * px, optional=True),
                                               self._t(ref, "ref", bf, 32 * px, optional=True), 1 if relu else 0,
                                               self._t(out, "out", bf, 32 * px), _stream(stream)))

    def cnn_diag_wgrad(self, x, gout, grads, ws, gref=None, stream=None):
        import torch
        n, h, w, _ = x.shape
        px = n * h * w
        bf = torch.bfloat16
        self._check(self.lib.mpr_cnn_diag_wgrad(self._h, n, h, w, self._t(x, "x", bf, 32 * px),
                                                self._t(gout, "gout", bf, 32 * px),
                                                self._t(gref, "gref", bf, 32 * px, optional=True),
                                                self._t(grads, "grads", torch.float32, 9 * 32 * 32 + 32),
                                                self._t(ws, "ws"), ws.numel() * ws.element_size(), _stream(stream)))

    # ---------------------------------------------------------- profiling
    def profile_enable(self, on=True):
        self._check(self.lib.mpr_profile_enable(self._h, 1 if on else 0))

    def profile_read(self) -> dict:
        p = Profile()
        self._check(self.lib.mpr_profile_read(self._h, C.byref(p)))
        return {k: getattr(p, k) for k, _ in Profile._fields_}

    # -------------------------------------------------------- diagnostics
    def diag_philox(self, ctr, seed, out, stream=None):
        n = ctr.numel() // 4
        self._check(self.lib.mpr_diag_philox(self._h, self._t(ctr, "ctr", nbytes=16 * n), seed, n,
                                             self._t(out, "out", nbytes=16 * n), _stream(stream)))

    def diag_half_sweep(self, phi, sampled, colour, T, a, sweep, chain=0, stream_id=0, seed=3000, q=0.5,
                        mode=0, flags=None, stream=None, with_energy=False, tile=0):
        """One half-sweep in place; returns the accepted count (and the fused
        bond-energy sum H + N_GP when with_energy).  tile: block shape as
        Params.tile_rows (0 = default)."""
        import torch
        ny, nx = phi.shape
        acc = C.c_int64()
        en = C.c_double()
        self._check(self.lib.mpr_diag_half_sweep(self._h, nx, ny, self._t(phi, "phi", torch.float32, nx * ny),
                                                 self._t(sampled, "sampled", torch.uint8, nx * ny), colour, T, a,
                                                 q, seed, sweep, chain, stream_id, mode, int(tile),
                                                 self._t(flags, "flags", torch.uint8, nx * ny, optional=True),
                                                 C.byref(acc), C.byref(en), _stream(stream)))
        return (acc.value, en.value) if with_energy else acc.value

    def diag_half_sweep_fp64(self, phi, sampled, colour, T, a, sweep, chain=0, stream_id=0, seed=3000, q=0.5,
                             mode=0, flags=None, stream=None, with_energy=False, tile=0):
        """diag_half_sweep on a float64 grid through the double-precision sweep."""
        import torch
        if phi.dtype != torch.float64:
            raise TypeError("phi must be float64")
        ny, nx = phi.shape
        acc = C.c_int64()
        en = C.c_double()
        self._check(self.lib.mpr_diag_half_sweep_fp64(self._h, nx, ny, self._t(phi, "phi", torch.float64, nx * ny),
                                                      self._t(sampled, "sampled", torch.uint8, nx * ny), colour, T,
                                                      a, q, seed, sweep, chain, stream_id, mode, int(tile),
                                                      self._t(flags, "flags", torch.uint8, nx * ny, optional=True),
                                                      C.byref(acc), C.byref(en), _stream(stream)))
        return (acc.value, en.value) if with_energy else acc.value

    def diag_copy(self, src, dst, stream=None):
        n = src.numel() * src.element_size()
        self._check(self.lib.mpr_diag_copy(self._h, self._t(src, "src"), self._t(dst, "dst", nbytes=n), n,
                                           _stream(stream)))

    def diag_energy(self, phi, q=0.5, stream=None) -> float:
        import torch
        ny, nx = phi.shape
        out = C.c_double()
        self._check(self.lib.mpr_diag_energy(self._h, nx, ny, self._t(phi, "phi", torch.float32, nx * ny), q,
                                             C.byref(out), _stream(stream)))
        return out.value

    def diag_sg_slope(self, e, degree=1) -> float:
        e = np.ascontiguousarray(e, dtype=np.float64)
        out = C.c_double()
        self._check(self.lib.mpr_diag_sg_slope(self._h, e.ctypes.data_as(C.c_void_p), e.size, degree,
                                               C.byref(out)))
        return out.value
