"""Python binding of the MI355X FBIM library (libfbim.so, C ABI in include/fbim.h).

Argument marshalling only: every step of the method runs in the HIP library.
Device arrays are torch tensors on the GPU (float64, contiguous); torch is used
for device memory and the current stream.  If the built library is missing the
import of this module fails loudly -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

__all__ = ["Params", "Derived", "Info", "Context", "lib", "derive_params", "alpert_rule", "starfish",
           "PART_REAL", "PART_ALPERT", "PART_WAVE", "PART_ALL", "PREC_FP64", "PREC_MIXED", "FbimError",
           "LIB_PATH", "MLP_IN", "MLP_OUT", "MLP_NPARAM", "TuneReport", "TUNE_TILE", "TUNE_SPLIT", "autotune_lookup"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfbim.so")

PART_REAL, PART_ALPERT, PART_WAVE, PART_ALL = 1, 2, 4, 7
(FLAG_SELECTIVE_REORTH, FLAG_BATCH_RFD, FLAG_GRAPH, FLAG_REFINEMENT, FLAG_LIBRARY_FFT, FLAG_BASIS32,
 FLAG_LAGGED_REORTH) = 1, 2, 4, 8, 16, 32, 64
BATCH_GRAPH = 1
PREC_FP64, PREC_MIXED = 0, 1
NOISE_W_R, NOISE_W_GRID, NOISE_W_TILDE = 0, 1, 2
MLP_IN, MLP_HID, MLP_OUT = 32, 128, 6
MLP_NPARAM = 32 * 128 + 128 + 128 * 128 + 128 + 128 * 6 + 6
NOALLOC_MAX_BODIES = 8192
TUNE_TILE = 1
TUNE_SPLIT = 2
STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EOVERLAP", 4: "ENOCONV", 5: "EDEVICE", 6: "ENOTSUP",
          7: "WACCURACY"}


class FbimError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double), ("eta", ctypes.c_double), ("kT", ctypes.c_double),
                ("tol_ewald", ctypes.c_double), ("tol_gmres", ctypes.c_double),
                ("tol_lanczos", ctypes.c_double), ("xi", ctypes.c_double), ("tau_spurious", ctypes.c_double),
                ("alpert_order", ctypes.c_int32), ("n_box", ctypes.c_int32), ("grid_M", ctypes.c_int32),
                ("P", ctypes.c_int32), ("precision", ctypes.c_int32), ("gmres_restart", ctypes.c_int32),
                ("gmres_maxiter", ctypes.c_int32), ("lanczos_maxiter", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("seed", ctypes.c_uint64), ("tol_rfd", ctypes.c_double)]


class Derived(ctypes.Structure):
    _fields_ = [("xi", ctypes.c_double), ("r_c", ctypes.c_double), ("h", ctypes.c_double),
                ("eta_s", ctypes.c_double), ("r_alpert", ctypes.c_double), ("n_box", ctypes.c_int32),
                ("grid_M", ctypes.c_int32), ("P", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("alpert_j", ctypes.c_int32), ("alpert_a", ctypes.c_int32), ("n_bodies", ctypes.c_int32),
                ("n_nodes", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TuneReport(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_int32), ("from_cache", ctypes.c_int32), ("cache_error", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("ms_best", ctypes.c_double), ("ms_default", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class Info(ctypes.Structure):
    _fields_ = [("gmres_iters", ctypes.c_int32), ("gmres_solves", ctypes.c_int32),
                ("lanczos_iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("gmres_residual", ctypes.c_double), ("lanczos_change", ctypes.c_double),
                ("ms_total", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TrainCfg(ctypes.Structure):
    _fields_ = [("n_solves", ctypes.c_int32), ("epochs", ctypes.c_int32), ("lr", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


class TrainInfo(ctypes.Structure):
    _fields_ = [("loss_first", ctypes.c_float), ("loss_last", ctypes.c_float), ("gmres_iters", ctypes.c_int32),
                ("samples", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    # torch first: the process must use the HIP runtime torch was built with;
    # libfbim.so then binds to that already-loaded runtime by soname
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError("libfbim.so is not built; run `python paper_1709_01480_amd/build.py` "
                          "(no CPU fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    p, i32, u32, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "fbim_create": (i32, [P(Params), P(p)]),
        "fbim_destroy": (None, [p]),
        "fbim_last_error": (ctypes.c_char_p, [p]),
        "fbim_status_string": (ctypes.c_char_p, [i32]),
        "fbim_set_stream": (i32, [p, p]),
        "fbim_add_shape": (i32, [p, i32, p, P(i32)]),
        "fbim_starfish": (None, [d, d, i32, i32, p]),
        "fbim_set_bodies": (i32, [p, i32, p, p, p]),
        "fbim_get_derived": (i32, [p, P(Derived)]),
        "fbim_get_nodes": (i32, [p, p]),
        "fbim_apply_M": (i32, [p, p, p, u32]),
        "fbim_random_field": (i32, [p, p, p]),
        "fbim_sqrt_Mr": (i32, [p, p, p, P(Info)]),
        "fbim_mobility": (i32, [p, p, p, p, p, P(Info)]),
        "fbim_apply_precond": (i32, [p, p, p]),
        "fbim_brownian_velocity": (i32, [p, d, p, p, p, p, P(Info)]),
        "fbim_step_em_rfd": (i32, [p, d, d, p, p, p, p, p, i32, P(Info)]),
        "fbim_step_ab2_rfd": (i32, [p, d, d, p, p, p, p, p, i32, p, i32, P(Info)]),
        "fbim_derive_params": (i32, [P(Params), P(Derived)]),
        "fbim_alpert_rule": (i32, [i32, P(i32), P(i32), p, p]),
        "fbim_mlp_init": (i32, [p, ctypes.c_uint64, i32]),
        "fbim_mlp_set_weights": (i32, [p, p, ctypes.c_size_t]),
        "fbim_mlp_get_weights": (i32, [p, p, ctypes.c_size_t]),
        "fbim_mlp_features": (i32, [p, p]),
        "fbim_mlp_forward": (i32, [p, p, i32, p]),
        "fbim_mlp_backward": (i32, [p, p, p, i32, p]),
        "fbim_mlp_forward_noalloc": (i32, [p, p, i32, p]),
        "fbim_mlp_loss": (i32, [p, p, i32, p, p, P(ctypes.c_float), p]),
        "fbim_mlp_train": (i32, [p, P(TrainCfg), P(TrainInfo)]),
        "fbim_mlp_use": (i32, [p, i32]),
        "fbim_batch_create": (i32, [i32, P(Params), P(p)]),
        "fbim_batch_destroy": (None, [p]),
        "fbim_batch_last_error": (ctypes.c_char_p, [p]),
        "fbim_batch_member": (p, [p, i32]),
        "fbim_batch_set_stream": (i32, [p, p]),
        "fbim_batch_set_flags": (i32, [p, u32]),
        "fbim_batch_apply_M": (i32, [p, p, p]),
        "fbim_batch_mobility": (i32, [p, p, p, p, P(Info)]),
        "fbim_batch_step_em_rfd": (i32, [p, d, d, p, p, p, p, p, i32, P(Info)]),
        "fbim_batch_step_ab2_rfd": (i32, [p, d, d, p, p, p, p, p, i32, p, i32, P(Info)]),
        "fbim_noise_normals": (i32, [p, u32, ctypes.c_uint64, ctypes.c_size_t, p]),
        "fbim_noise_words": (i32, [p, u32, ctypes.c_uint64, ctypes.c_size_t, p]),
        "fbim_noise_counter": (i32, [p, P(ctypes.c_uint64)]),
        "fbim_set_noise_counter": (i32, [p, ctypes.c_uint64]),
        "fbim_mobility_second_kind": (i32, [p, p, p, p, p, P(Info)]),
        "fbim_apply_double_layer": (i32, [p, p, p]),
        "fbim_brownian_velocity_mixed": (i32, [p, d, p, p, p, p, P(Info)]),
        "fbim_autotune": (i32, [p, u32, ctypes.c_char_p, P(Params), P(TuneReport)]),
        "fbim_autotune_key": (i32, [p, u32, ctypes.c_char_p, i32]),
        "fbim_autotune_lookup": (i32, [ctypes.c_char_p, ctypes.c_char_p, P(i32), P(i32), P(i32)]),
        "fbim_set_timing": (i32, [p, i32]),
        "fbim_kernel_time": (i32, [p, ctypes.c_char_p, P(d), P(ctypes.c_int64)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


lib = _load()


def autotune_lookup(cache_path, key):
    """fbim_autotune_lookup (host only): (n_box, grid_M, tile) or None."""
    a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    if lib.fbim_autotune_lookup(os.fsencode(cache_path), key.encode(), ctypes.byref(a), ctypes.byref(b),
                                ctypes.byref(c)):
        return a.value, b.value, c.value
    return None


def make_params(**kw) -> Params:
    prm = Params()
    prm.eta = 1.0
    prm.kT = 1.0
    prm.tol_gmres = 1e-6
    prm.tol_lanczos = 1e-6
    prm.tau_spurious = 1e-8
    prm.alpert_order = 4
    for k, v in kw.items():
        setattr(prm, k, v)
    return prm


def derive_params(**kw) -> dict:
    out = Derived()
    st = lib.fbim_derive_params(ctypes.byref(make_params(**kw)), ctypes.byref(out))
    if st != 0:
        raise FbimError(st, "parameter derivation failed")
    return out.as_dict()


def alpert_rule(order: int):
    import numpy as np
    j, a = ctypes.c_int32(), ctypes.c_int32()
    chi = (ctypes.c_double * 8)()
    w = (ctypes.c_double * 8)()
    st = lib.fbim_alpert_rule(order, ctypes.byref(j), ctypes.byref(a), chi, w)
    if st != 0:
        raise FbimError(st, "no Alpert rule")
    return np.array(chi[:j.value]), np.array(w[:j.value]), a.value


def starfish(r_s: float, b: float, n_arm: int, n_p: int):
    import numpy as np
    out = np.zeros(2 * n_p)
    lib.fbim_starfish(r_s, b, n_arm, n_p, out.ctypes.data_as(ctypes.c_void_p))
    return out


def _dptr(t, n=None):
    """Device pointer of a float64 contiguous GPU tensor (checked)."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 GPU tensor")
    if n is not None and t.numel() != n:
        raise ValueError("expected %d elements, got %d" % (n, t.numel()))
    return ctypes.c_void_p(t.data_ptr())


def _optr(t, n=None):
    """_dptr, or a NULL pointer for None."""
    return None if t is None else _dptr(t, n)


def _fptr(t, n=None):
    """Device pointer of a float32 contiguous GPU tensor (checked)."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError("expected a contiguous float32 GPU tensor")
    if n is not None and t.numel() != n:
        raise ValueError("expected %d elements, got %d" % (n, t.numel()))
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """One library context (fbim_ctx) bound to torch's current stream."""

    def __init__(self, _handle=None, **params):
        import torch
        self.n = 0
        self.N = 0
        if _handle is not None:  # a member of a Batch (owned by the batch)
            self._ctx = ctypes.c_void_p(_handle)
            self._owned = False
            return
        self._ctx = ctypes.c_void_p()
        self._owned = True
        self.params = make_params(**params)
        st = lib.fbim_create(ctypes.byref(self.params), ctypes.byref(self._ctx))
        if st != 0:
            raise FbimError(st, "fbim_create failed")
        self._check(lib.fbim_set_stream(self._ctx, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))

    def _check(self, st, allow=()):
        if st != 0 and st not in allow:
            raise FbimError(st, lib.fbim_last_error(self._ctx).decode())
        return st

    def close(self):
        if self._ctx and self._owned:
            lib.fbim_destroy(self._ctx)
        self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- setup
    def add_shape(self, ref_xy):
        import numpy as np
        ref = np.ascontiguousarray(ref_xy, dtype=np.float64)
        sid = ctypes.c_int32()
        st = lib.fbim_add_shape(self._ctx, len(ref) // 2, ref.ctypes.data_as(ctypes.c_void_p), ctypes.byref(sid))
        self._check(st, allow=(7,))
        return sid.value

    def set_bodies(self, shape_id, q, theta):
        import numpy as np
        sid = np.ascontiguousarray(shape_id, dtype=np.int32)
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
        th = np.ascontiguousarray(theta, dtype=np.float64)
        self._check(lib.fbim_set_bodies(self._ctx, len(th), sid.ctypes.data_as(ctypes.c_void_p),
                                        q.ctypes.data_as(ctypes.c_void_p), th.ctypes.data_as(ctypes.c_void_p)))
        d = self.get_derived()
        self.n, self.N = d["n_bodies"], d["n_nodes"]

    # -- completed second-kind formulation
    def mobility_second_kind(self, F, U, slip=None, phi=None):
        info = Info()
        self._check(lib.fbim_mobility_second_kind(self._ctx, _dptr(F, 3 * self.n), _optr(slip, 2 * self.N),
                                                  _dptr(U, 3 * self.n), _optr(phi, 2 * self.N),
                                                  ctypes.byref(info)), allow=(4,))
        return info.as_dict()

    def apply_double_layer(self, phi, out):
        self._check(lib.fbim_apply_double_layer(self._ctx, _dptr(phi, 2 * self.N), _dptr(out, 2 * self.N)))

    def brownian_velocity_mixed(self, dt, F, W_r, W_grid, U):
        M = self.get_derived()["grid_M"]
        info = Info()
        self._check(lib.fbim_brownian_velocity_mixed(self._ctx, dt, _dptr(F, 3 * self.n), _optr(W_r, 2 * self.N),
                                                     _optr(W_grid, 2 * M * M), _dptr(U, 3 * self.n),
                                                     ctypes.byref(info)), allow=(4,))
        return info.as_dict()

    def autotune(self, what, cache_path=None):
        """fbim_autotune: (parameters dict for Context(**...), report dict)."""
        out = Params()
        rep = TuneReport()
        path = None if cache_path is None else os.fsencode(cache_path)
        self._check(lib.fbim_autotune(self._ctx, what, path, ctypes.byref(out), ctypes.byref(rep)))
        return {k: getattr(out, k) for k, _ in Params._fields_}, rep.as_dict()

    def autotune_key(self, what) -> str:
        buf = ctypes.create_string_buffer(1024)
        self._check(lib.fbim_autotune_key(self._ctx, what, buf, len(buf)))
        return buf.value.decode()

    def get_derived(self) -> dict:
        out = Derived()
        self._check(lib.fbim_get_derived(self._ctx, ctypes.byref(out)))
        return out.as_dict()

    # -- hot path
    def get_nodes(self, x):
        self._check(lib.fbim_get_nodes(self._ctx, _dptr(x, 2 * self.N)))

    def apply_M(self, mu, out, parts=PART_ALL):
        self._check(lib.fbim_apply_M(self._ctx, _dptr(mu, 2 * self.N), _dptr(out, 2 * self.N), parts))

    def random_field(self, W_grid, out):
        M = self.get_derived()["grid_M"]
        self._check(lib.fbim_random_field(self._ctx, _dptr(W_grid, 2 * M * M), _dptr(out, 2 * self.N)))

    def sqrt_Mr(self, W_r, out):
        info = Info()
        self._check(lib.fbim_sqrt_Mr(self._ctx, _dptr(W_r, 2 * self.N), _dptr(out, 2 * self.N),
                                     ctypes.byref(info)))
        return info.as_dict()

    def apply_precond(self, z, y):
        n = 2 * self.N + 3 * self.n
        self._check(lib.fbim_apply_precond(self._ctx, _dptr(z, n), _dptr(y, n)))

    def mobility(self, F, U, slip=None, mu_out=None):
        info = Info()
        self._check(lib.fbim_mobility(self._ctx, _dptr(F, 3 * self.n),
                                      None if slip is None else _dptr(slip, 2 * self.N), _dptr(U, 3 * self.n),
                                      None if mu_out is None else _dptr(mu_out, 2 * self.N),
                                      ctypes.byref(info)))
        return info.as_dict()

    def brownian_velocity(self, dt, F, W_r, W_grid, U):
        """W_r / W_grid None: drawn by the context's generator."""
        M = self.get_derived()["grid_M"]
        info = Info()
        self._check(lib.fbim_brownian_velocity(self._ctx, dt, _dptr(F, 3 * self.n), _optr(W_r, 2 * self.N),
                                               _optr(W_grid, 2 * M * M), _dptr(U, 3 * self.n),
                                               ctypes.byref(info)))
        return info.as_dict()

    def step_em_rfd(self, dt, delta, F, W_r, W_grid, W_tilde, dQ, apply=False):
        """Noise arguments that are None are drawn by the context's generator."""
        M = self.get_derived()["grid_M"]
        info = Info()
        self._check(lib.fbim_step_em_rfd(self._ctx, dt, delta, _dptr(F, 3 * self.n), _optr(W_r, 2 * self.N),
                                         _optr(W_grid, 2 * M * M), _optr(W_tilde, 3 * self.n),
                                         _dptr(dQ, 3 * self.n), 1 if apply else 0, ctypes.byref(info)))
        return info.as_dict()

    def step_ab2_rfd(self, dt, delta, F, W_r, W_grid, W_tilde, NF_hist, have_hist, dQ, apply=False):
        """AB2-RFD step; NF_hist (3n, GPU) carries N F from one step to the next."""
        M = self.get_derived()["grid_M"]
        info = Info()
        self._check(lib.fbim_step_ab2_rfd(self._ctx, dt, delta, _dptr(F, 3 * self.n), _optr(W_r, 2 * self.N),
                                          _optr(W_grid, 2 * M * M), _optr(W_tilde, 3 * self.n),
                                          _dptr(NF_hist, 3 * self.n), 1 if have_hist else 0,
                                          _dptr(dQ, 3 * self.n), 1 if apply else 0, ctypes.byref(info)))
        return info.as_dict()

    # -- noise
    def noise_normals(self, stream, counter, out):
        self._check(lib.fbim_noise_normals(self._ctx, stream, counter, out.numel(), _dptr(out)))

    def noise_words(self, stream, counter, out):
        """out: int32 GPU tensor of 4 n_pairs elements (the 32-bit words, reinterpreted)."""
        import torch
        if not isinstance(out, torch.Tensor) or not out.is_cuda or out.dtype != torch.int32 or \
                not out.is_contiguous() or out.numel() % 4:
            raise TypeError("expected a contiguous int32 GPU tensor of 4 n_pairs elements")
        self._check(lib.fbim_noise_words(self._ctx, stream, counter, out.numel() // 4,
                                         ctypes.c_void_p(out.data_ptr())))

    def noise_counter(self):
        v = ctypes.c_uint64()
        self._check(lib.fbim_noise_counter(self._ctx, ctypes.byref(v)))
        return v.value

    def set_noise_counter(self, counter):
        self._check(lib.fbim_set_noise_counter(self._ctx, counter))

    # -- learned preconditioner correction
    def mlp_init(self, seed=0, sym_order=1):
        self._check(lib.fbim_mlp_init(self._ctx, seed, sym_order))

    def mlp_set_weights(self, w):
        import numpy as np
        w = np.ascontiguousarray(w, dtype=np.float32)
        self._check(lib.fbim_mlp_set_weights(self._ctx, w.ctypes.data_as(ctypes.c_void_p), w.size))

    def mlp_get_weights(self):
        import numpy as np
        w = np.zeros(MLP_NPARAM, dtype=np.float32)
        self._check(lib.fbim_mlp_get_weights(self._ctx, w.ctypes.data_as(ctypes.c_void_p), w.size))
        return w

    def mlp_features(self, X):
        self._check(lib.fbim_mlp_features(self._ctx, _fptr(X, self.n * MLP_IN)))

    def mlp_forward(self, X, Y):
        n = X.numel() // MLP_IN
        self._check(lib.fbim_mlp_forward(self._ctx, _fptr(X, n * MLP_IN), n, _fptr(Y, n * MLP_OUT)))

    def mlp_forward_noalloc(self, X, Y):
        n = X.numel() // MLP_IN
        self._check(lib.fbim_mlp_forward_noalloc(self._ctx, _fptr(X, n * MLP_IN), n, _fptr(Y, n * MLP_OUT)))

    def mlp_backward(self, X, dY, grad):
        n = X.numel() // MLP_IN
        self._check(lib.fbim_mlp_backward(self._ctx, _fptr(X, n * MLP_IN), _fptr(dY, n * MLP_OUT), n,
                                          _fptr(grad, MLP_NPARAM)))

    def mlp_loss(self, Y, F, U, dY):
        ns = F.numel() // (3 * self.n)
        loss = ctypes.c_float()
        self._check(lib.fbim_mlp_loss(self._ctx, _fptr(Y, self.n * MLP_OUT), ns, _dptr(F, ns * 3 * self.n),
                                      _dptr(U, ns * 3 * self.n), ctypes.byref(loss), _fptr(dY, self.n * MLP_OUT)))
        return loss.value

    def mlp_train(self, n_solves, epochs, lr=1e-3, seed=0):
        cfg = TrainCfg(n_solves, epochs, lr, seed)
        info = TrainInfo()
        self._check(lib.fbim_mlp_train(self._ctx, ctypes.byref(cfg), ctypes.byref(info)), allow=(4,))
        return info.as_dict()

    def mlp_use(self, on=True):
        self._check(lib.fbim_mlp_use(self._ctx, 1 if on else 0))

    # -- measurement
    def set_timing(self, enable=True):
        self._check(lib.fbim_set_timing(self._ctx, 1 if enable else 0))

    def kernel_time(self, name):
        ms, cnt = ctypes.c_double(), ctypes.c_int64()
        self._check(lib.fbim_kernel_time(self._ctx, name.encode(), ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value


def _ptr_array(tensors, check):
    arr = (ctypes.c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = None if t is None else check(t)
    return arr


class Batch:
    """Several independent systems advanced together (fbim_batch)."""

    def __init__(self, params_list, graph=False):
        import torch
        prm = (Params * len(params_list))(*[make_params(**p) for p in params_list])
        self._b = ctypes.c_void_p()
        st = lib.fbim_batch_create(len(params_list), prm, ctypes.byref(self._b))
        if st != 0:
            raise FbimError(st, "fbim_batch_create failed")
        self._check(lib.fbim_batch_set_stream(self._b, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        self.members = [Context(_handle=lib.fbim_batch_member(self._b, i)) for i in range(len(params_list))]
        if graph:
            self._check(lib.fbim_batch_set_flags(self._b, BATCH_GRAPH))

    def _check(self, st, allow=()):
        if st != 0 and st not in allow:
            raise FbimError(st, lib.fbim_batch_last_error(self._b).decode())
        return st

    def close(self):
        for m in getattr(self, "members", []):
            m._ctx = ctypes.c_void_p()
        if self._b:
            lib.fbim_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_graph(self, on=True):
        self._check(lib.fbim_batch_set_flags(self._b, BATCH_GRAPH if on else 0))

    def apply_M(self, mus, outs):
        m = self.members
        self._check(lib.fbim_batch_apply_M(
            self._b, _ptr_array([_dptr(x, 2 * c.N) for x, c in zip(mus, m)], lambda v: v.value),
            _ptr_array([_dptr(x, 2 * c.N) for x, c in zip(outs, m)], lambda v: v.value)))

    def mobility(self, Fs, Us, slips=None):
        m = self.members
        info = (Info * len(m))()
        F = _ptr_array([_dptr(x, 3 * c.n).value for x, c in zip(Fs, m)], lambda v: v)
        U = _ptr_array([_dptr(x, 3 * c.n).value for x, c in zip(Us, m)], lambda v: v)
        S = None if slips is None else _ptr_array(
            [None if x is None else _dptr(x, 2 * c.N).value for x, c in zip(slips, m)], lambda v: v)
        self._check(lib.fbim_batch_mobility(self._b, F, S, U, info), allow=(4,))
        return [i.as_dict() for i in info]

    def step_em_rfd(self, dt, delta, Fs, W_rs, W_grids, W_tildes, dQs, apply=False):
        m = self.members
        info = (Info * len(m))()
        Ms = [c.get_derived()["grid_M"] for c in m]
        def arr(xs, sizes):  # None (or None entries): drawn by the member's generator
            if xs is None:
                return None
            return _ptr_array([None if x is None else _dptr(x, k).value for x, k in zip(xs, sizes)], lambda v: v)
        self._check(lib.fbim_batch_step_em_rfd(
            self._b, dt, delta, arr(Fs, [3 * c.n for c in m]), arr(W_rs, [2 * c.N for c in m]),
            arr(W_grids, [2 * M * M for M in Ms]), arr(W_tildes, [3 * c.n for c in m]),
            arr(dQs, [3 * c.n for c in m]), 1 if apply else 0, info), allow=(4,))
        return [i.as_dict() for i in info]

    def step_ab2_rfd(self, dt, delta, Fs, W_rs, W_grids, W_tildes, hists, have_hist, dQs, apply=False):
        m = self.members
        info = (Info * len(m))()
        Ms = [c.get_derived()["grid_M"] for c in m]

        def arr(xs, sizes):
            if xs is None:
                return None
            return _ptr_array([None if x is None else _dptr(x, k).value for x, k in zip(xs, sizes)], lambda v: v)
        n3 = [3 * c.n for c in m]
        self._check(lib.fbim_batch_step_ab2_rfd(
            self._b, dt, delta, arr(Fs, n3), arr(W_rs, [2 * c.N for c in m]),
            arr(W_grids, [2 * M * M for M in Ms]), arr(W_tildes, n3), arr(hists, n3), 1 if have_hist else 0,
            arr(dQs, n3), 1 if apply else 0, info), allow=(4,))
        return [i.as_dict() for i in info]
