"""Python binding of the ptlm C ABI (include/ptlm.h): argument marshalling only.

Every computation runs in the HIP kernels of ``libptlm.so``; this module only
checks tensor shapes/dtypes/devices, passes raw device pointers and the current
HIP stream, and converts status codes to exceptions.  Importing it fails
loudly when the compiled library is missing.

Low-level functions carry the C names (``ptlm_forward`` ...) and take a
``Handle``; ``Problem`` bundles a handle with its workspace tensor.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libptlm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libptlm.so is not built (run paper_2103_01767_amd.build.build() or "
                      "__graft_entry__.build()); there is no fallback implementation")
_lib = ctypes.CDLL(LIB_PATH)

PTLM_OK = 0
PTLM_ENOTACCEPTED = 1
PTLM_EINVAL = -1
PTLM_EWORKSPACE = -2
PTLM_EHIP = -3
PTLM_ENUMERIC = -4
GAUSS, POISSON = 0, 1
OBJECT, JOINT = 0, 1
GGN_MAGNITUDE, GGN_INTENSITY = 0, 1
# ptlm_transform values by name (PTLM_TRANSFORM_FFT, _MFMA, _FFT_WIDE)
TRANSFORMS = ("fft", "mfma", "fft_wide")


class ptlm_desc(ctypes.Structure):
    _fields_ = [("ny", ctypes.c_int32), ("nx", ctypes.c_int32), ("my", ctypes.c_int32),
                ("mx", ctypes.c_int32), ("K", ctypes.c_int32), ("metric", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("background", ctypes.c_float), ("ggn", ctypes.c_int32),
                ("seg_len", ctypes.c_int32)]


class ptlm_lm_params(ctypes.Structure):
    _fields_ = [("mu0", ctypes.c_double), ("mu_min", ctypes.c_double), ("kappa", ctypes.c_double),
                ("nu", ctypes.c_double), ("rho_min", ctypes.c_double), ("beta", ctypes.c_double),
                ("diag_floor", ctypes.c_double), ("cg_max", ctypes.c_int32),
                ("retry_max", ctypes.c_int32), ("scaling", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("warm_start", ctypes.c_int32),
                ("surrogate_T", ctypes.c_int32), ("surrogate_s0", ctypes.c_double),
                ("project", ctypes.c_int32), ("ls_max", ctypes.c_int32), ("o_max", ctypes.c_double),
                ("p_max", ctypes.c_double), ("sigma_ls", ctypes.c_double), ("gamma", ctypes.c_double),
                ("tau_s", ctypes.c_double), ("p_s", ctypes.c_double), ("alternate", ctypes.c_int32),
                ("stoch_samples", ctypes.c_int32), ("stoch_seed", ctypes.c_uint64)]


class ptlm_cnn_desc(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("n", "h", "w", "cin", "cmid", "cout", "layers")]


_STATE_DOUBLES = ["f", "f_trial", "mu", "lambda_", "rho", "eta", "gnorm", "resid_norm", "pred",
                  "rz", "rr", "alpha", "beta_cg", "pap", "sigma", "ls_alpha", "mu_alt"]
_STATE_INTS = ["t", "cg_iters", "cg_total", "accepted", "cg_active", "retries", "nonfinite", "products",
               "attempts", "need_lin", "lin_now", "use_warm", "alive", "prev_valid", "t_max", "status", "iter_done", "ls_branch",
               "block", "acc_o", "acc_p", "tile_now", "ls_dir", "ls_neg", "ls_on", "ls_take", "ls_keep", "ls_proj",
               "ls_iter"]


class ptlm_lm_state(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in _STATE_DOUBLES] + [(n, ctypes.c_int32) for n in _STATE_INTS]


STATE_BYTES = ctypes.sizeof(ptlm_lm_state)

_vp = ctypes.c_void_p
_sig = {
    "ptlm_lm_default_params": (None, [ctypes.POINTER(ptlm_lm_params)]),
    "ptlm_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(ptlm_desc), _vp, ctypes.POINTER(ctypes.c_size_t)]),
    "ptlm_create": (ctypes.c_int, [ctypes.POINTER(ptlm_desc), _vp, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
    "ptlm_destroy": (ctypes.c_int, [_vp]),
    "ptlm_forward": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "ptlm_loss": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "ptlm_loss_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "ptlm_linearize": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "ptlm_jvp": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "ptlm_vjp": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "ptlm_ggn_vp": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, _vp, _vp, _vp, _vp, _vp]),
    "ptlm_ggn_vp_stage": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, _vp, _vp, _vp, _vp, ctypes.c_int32,
                                         _vp]),
    "ptlm_set_transform": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "ptlm_diag": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int32, _vp]),
    "ptlm_diag_stochastic": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint64, _vp, _vp, _vp]),
    "ptlm_lm_init": (ctypes.c_int, [_vp, ctypes.POINTER(ptlm_lm_params), _vp, _vp]),
    "ptlm_lm_step": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.POINTER(ptlm_lm_params), _vp, _vp, _vp]),
    "ptlm_lm_solve": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.POINTER(ptlm_lm_params), ctypes.c_int32,
                                     _vp, _vp, _vp]),
    "ptlm_cnn_param_count": (ctypes.c_int, [ctypes.POINTER(ptlm_cnn_desc), ctypes.POINTER(ctypes.c_size_t)]),
    "ptlm_cnn_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(ptlm_cnn_desc), ctypes.POINTER(ctypes.c_size_t)]),
    "ptlm_cnn_forward": (ctypes.c_int, [ctypes.POINTER(ptlm_cnn_desc), _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "ptlm_cnn_loss_grad": (ctypes.c_int, [ctypes.POINTER(ptlm_cnn_desc), _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                          ctypes.c_size_t, _vp]),
    "ptlm_cnn_adam": (ctypes.c_int, [ctypes.c_size_t, _vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_float,
                                     ctypes.c_float, ctypes.c_float, ctypes.c_float, _vp]),
    "ptlm_cnn_features": (ctypes.c_int, [_vp, _vp, _vp]),
    "ptlm_learned_precond": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "ptlm_lm_set_cnn": (ctypes.c_int, [_vp, ctypes.POINTER(ptlm_cnn_desc), _vp, _vp, ctypes.c_size_t]),
    "ptlm_autotune": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32), _vp]),
    "ptlm_batch_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ptlm_desc), _vp,
                                                  ctypes.POINTER(ctypes.c_size_t)]),
    "ptlm_batch_create": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ptlm_desc), _vp, _vp, ctypes.c_size_t, _vp,
                                         ctypes.POINTER(_vp)]),
    "ptlm_batch_problem": (_vp, [_vp, ctypes.c_int32]),
    "ptlm_batch_bind": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, ctypes.POINTER(ptlm_lm_params), ctypes.c_int32,
                                       ctypes.c_int32, _vp]),
    "ptlm_batch_attempt": (ctypes.c_int, [_vp, _vp]),
    "ptlm_batch_cnn_refresh": (ctypes.c_int, [_vp, _vp]),
    "ptlm_batch_solve": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), _vp]),
    "ptlm_batch_destroy": (ctypes.c_int, [_vp]),
    "ptlm_lm_set_cnn_refresh": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "ptlm_last_error": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTS = tuple(_sig)


class PtlmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("ptlm status %d: %s" % (status, msg))
        self.status = status


def _check(st, allow=(PTLM_OK,)):
    if st not in allow:
        raise PtlmError(st, _lib.ptlm_last_error().decode())
    return st


def _stream():
    return _vp(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype, shape=None, name="array"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    return _vp(t.data_ptr())


def default_params(**kw) -> ptlm_lm_params:
    p = ptlm_lm_params()
    _lib.ptlm_lm_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def state_from_tensor(buf: torch.Tensor) -> ptlm_lm_state:
    """Decode a device LM state buffer (copies to the host)."""
    raw = buf.detach().cpu().numpy().tobytes()
    return ptlm_lm_state.from_buffer_copy(raw[:STATE_BYTES])


def _desc(obj_shape, probe_shape, K, metric, mode, background, ggn="magnitude", seg_len=0):
    joint = mode in ("joint", JOINT)
    if ggn not in ("magnitude", "intensity", GGN_MAGNITUDE, GGN_INTENSITY):
        raise ValueError("ggn must be 'magnitude' or 'intensity'")
    return ptlm_desc(int(obj_shape[0]), int(obj_shape[1]), int(probe_shape[0]), int(probe_shape[1]), int(K),
                     POISSON if metric in ("poisson", POISSON) else GAUSS, JOINT if joint else OBJECT,
                     float(background), GGN_INTENSITY if ggn in ("intensity", GGN_INTENSITY) else GGN_MAGNITUDE,
                     int(seg_len))


class Problem:
    """One ptychography problem on one GPU: handle + workspace + positions."""

    def __init__(self, obj_shape, probe_shape, positions, metric="gauss", mode="object",
                 background=1e-8, device="cuda", ggn="magnitude", seg_len=0, _handle=None, _owner=None):
        pos = np.ascontiguousarray(np.asarray(positions, dtype=np.int32).reshape(-1, 2))
        self.obj_shape = tuple(int(v) for v in obj_shape)
        self.probe_shape = tuple(int(v) for v in probe_shape)
        self.K = int(pos.shape[0])
        self.joint = mode in ("joint", JOINT)
        self.desc = _desc(obj_shape, probe_shape, self.K, metric, mode, background, ggn, seg_len)
        self._pos = pos
        self.device = torch.device(device)
        if _handle is not None:  # a problem of a batch: the batch owns handle and workspace
            self.handle = None
            self._borrowed = _handle
            self._owner = _owner
            return
        nbytes = ctypes.c_size_t(0)
        _check(_lib.ptlm_workspace_bytes(ctypes.byref(self.desc), pos.ctypes.data_as(_vp), ctypes.byref(nbytes)))
        self.ws_bytes = int(nbytes.value)
        self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=self.device)
        h = _vp()
        _check(_lib.ptlm_create(ctypes.byref(self.desc), pos.ctypes.data_as(_vp), _vp(self.ws.data_ptr()),
                                self.ws_bytes, _stream(), ctypes.byref(h)))
        self.handle = h

    def __getattribute__(self, name):
        if name == "handle":
            b = object.__getattribute__(self, "__dict__").get("_borrowed")
            if b is not None:
                return b
        return object.__getattribute__(self, name)

    def __del__(self):
        if self.__dict__.get("_borrowed") is not None:
            return
        h = self.__dict__.get("handle")
        if h is not None and h.value and _lib is not None:
            _lib.ptlm_destroy(h)
            self.handle = None

    # -- shapes
    @property
    def meas_shape(self):
        return (self.K,) + self.probe_shape

    def _o(self, t, name="O"):
        return _ptr(t, torch.complex64, self.obj_shape, name)

    def _p(self, t, name="P"):
        return _ptr(t, torch.complex64, self.probe_shape, name)

    def _m(self, t, name):
        return _ptr(t, torch.float32, self.meas_shape, name)

    # -- calls (one C call each)
    def forward(self, O, P):
        out = torch.empty(self.meas_shape, dtype=torch.float32, device=self.device)
        _check(_lib.ptlm_forward(self.handle, self._o(O), self._p(P), self._m(out, "zeta"), _stream()))
        return out

    def loss(self, O, P, y, residual=False):
        f = torch.zeros(1, dtype=torch.float64, device=self.device)
        r = torch.empty(self.meas_shape, dtype=torch.float32, device=self.device) if residual else None
        _check(_lib.ptlm_loss(self.handle, self._o(O), self._p(P), self._m(y, "y"), _ptr(f, torch.float64),
                              self._m(r, "resid") if residual else None, _stream()))
        return (f, r) if residual else f

    def loss_noalloc(self, O, P, y, f=None, r=None):
        """ptlm_loss_noalloc: the loss with its partial sums in the library's static scratch.
        ``f`` (FP64, >= 1 entry) and ``r`` (residual, nullable) are caller-provided outputs."""
        if f is None:
            f = torch.zeros(1, dtype=torch.float64, device=self.device)
        _check(_lib.ptlm_loss_noalloc(self.handle, self._o(O), self._p(P), self._m(y, "y"),
                                      _ptr(f, torch.float64), self._m(r, "resid") if r is not None else None,
                                      _stream()))
        return f

    def linearize(self, O, P, y):
        f = torch.zeros(2, dtype=torch.float64, device=self.device)
        gO = torch.empty(self.obj_shape, dtype=torch.complex64, device=self.device)
        gP = torch.empty(self.probe_shape, dtype=torch.complex64, device=self.device) if self.joint else None
        _check(_lib.ptlm_linearize(self.handle, self._o(O), self._p(P), self._m(y, "y"), _ptr(f, torch.float64),
                                   self._o(gO, "gO"), self._p(gP, "gP") if self.joint else None, _stream()))
        return f, gO, gP

    def jvp(self, vO, vP=None):
        out = torch.empty(self.meas_shape, dtype=torch.float32, device=self.device)
        _check(_lib.ptlm_jvp(self.handle, self._o(vO, "vO"), self._p(vP, "vP") if self.joint else None,
                             self._m(out, "out"), _stream()))
        return out

    def vjp(self, w):
        oO = torch.empty(self.obj_shape, dtype=torch.complex64, device=self.device)
        oP = torch.empty(self.probe_shape, dtype=torch.complex64, device=self.device) if self.joint else None
        _check(_lib.ptlm_vjp(self.handle, self._m(w, "w"), self._o(oO, "outO"),
                             self._p(oP, "outP") if self.joint else None, _stream()))
        return oO, oP

    def ggn_vp(self, vO, vP=None, lam=0.0, dO=None, dP=None, out=None):
        if out is None:
            oO = torch.empty(self.obj_shape, dtype=torch.complex64, device=self.device)
            oP = torch.empty(self.probe_shape, dtype=torch.complex64, device=self.device) if self.joint else None
        else:
            oO, oP = out
        dOp = _ptr(dO, torch.float32, self.obj_shape + (2,), "dO") if dO is not None else None
        dPp = _ptr(dP, torch.float32, self.probe_shape + (2,), "dP") if dP is not None else None
        _check(_lib.ptlm_ggn_vp(self.handle, self._o(vO, "vO"), self._p(vP, "vP") if self.joint else None,
                                float(lam), dOp, dPp, self._o(oO, "outO"),
                                self._p(oP, "outP") if self.joint else None, _stream()))
        return oO, oP

    def set_transform(self, name):
        """ptlm_set_transform: "fft" (radix-16 FFT tile kernels), "mfma" (DFT as matrix products
        on the matrix cores, 16 x 16 and 32 x 32 probes) or "fft_wide" (the FFT with twice the
        tiles per workgroup, probes of at most 4096 pixels) for the GGN-vector product."""
        _check(_lib.ptlm_set_transform(self.handle, TRANSFORMS.index(name)))

    def ggn_vp_stage(self, stage, vO, vP=None, out=None):
        """Run one stage of the GGN-vector product (1: per-position kernel, 2: reductions)."""
        oO, oP = out if out is not None else (None, None)
        _check(_lib.ptlm_ggn_vp_stage(self.handle, self._o(vO, "vO"), self._p(vP, "vP") if self.joint else None,
                                      0.0, None, None, self._o(oO, "outO") if oO is not None else None,
                                      self._p(oP, "outP") if (self.joint and oP is not None) else None,
                                      int(stage), _stream()))

    def diag(self, exact=False):
        dO = torch.empty(self.obj_shape + (2,), dtype=torch.float32, device=self.device)
        dP = torch.empty(self.probe_shape + (2,), dtype=torch.float32, device=self.device) if self.joint else None
        _check(_lib.ptlm_diag(self.handle, _ptr(dO, torch.float32), _ptr(dP, torch.float32) if self.joint else None,
                              1 if exact else 0, _stream()))
        return dO, dP

    def diag_stochastic(self, samples, seed, draw0=0):
        """Unbiased estimate of the GGN diagonal from `samples` sign-field VJPs (ptlm_diag_stochastic)."""
        dO = torch.empty(self.obj_shape + (2,), dtype=torch.float32, device=self.device)
        dP = torch.empty(self.probe_shape + (2,), dtype=torch.float32, device=self.device) if self.joint else None
        _check(_lib.ptlm_diag_stochastic(self.handle, int(samples), int(seed), int(draw0), _ptr(dO, torch.float32),
                                         _ptr(dP, torch.float32) if self.joint else None, _stream()))
        return dO, dP

    def autotune(self, reps=5):
        """Pick the segment count and the transform of the GGN-vector product by timing it.
        Returns (scale, ms, transform): ms[transform * 3 + i] at scale 0.5, 1, 2 (-1: n/a)."""
        ms = (ctypes.c_double * (3 * len(TRANSFORMS)))()
        sc = ctypes.c_double(0)
        xf = ctypes.c_int32(0)
        _check(_lib.ptlm_autotune(self.handle, int(reps), ms, ctypes.byref(sc), ctypes.byref(xf), _stream()))
        return float(sc.value), [float(v) for v in ms], TRANSFORMS[xf.value]

    def new_state(self):
        return torch.zeros(STATE_BYTES, dtype=torch.uint8, device=self.device)

    def lm_init(self, params, state):
        _check(_lib.ptlm_lm_init(self.handle, ctypes.byref(params), _vp(state.data_ptr()), _stream()))

    def lm_step(self, O, P, y, params, state, precond=None):
        pc = _ptr(precond, torch.float32, None, "precond") if precond is not None else None
        return _check(_lib.ptlm_lm_step(self.handle, self._o(O), self._p(P), self._m(y, "y"),
                                        ctypes.byref(params), _vp(state.data_ptr()), pc, _stream()),
                      allow=(PTLM_OK, PTLM_ENOTACCEPTED))

    def lm_solve(self, O, P, y, params, T, state, precond=None):
        pc = _ptr(precond, torch.float32, None, "precond") if precond is not None else None
        return _check(_lib.ptlm_lm_solve(self.handle, self._o(O), self._p(P), self._m(y, "y"),
                                         ctypes.byref(params), int(T), _vp(state.data_ptr()), pc, _stream()),
                      allow=(PTLM_OK, PTLM_ENOTACCEPTED))


class Cnn:
    """Preconditioner network on one GPU: parameters, Adam moments and workspace."""

    def __init__(self, n, h, w, cin=3, cmid=32, cout=2, layers=4, device="cuda", params=None):
        self.desc = ptlm_cnn_desc(n, h, w, cin, cmid, cout, layers)
        cnt = ctypes.c_size_t(0)
        _check(_lib.ptlm_cnn_param_count(ctypes.byref(self.desc), ctypes.byref(cnt)))
        self.count = int(cnt.value)
        nb = ctypes.c_size_t(0)
        _check(_lib.ptlm_cnn_workspace_bytes(ctypes.byref(self.desc), ctypes.byref(nb)))
        self.ws_bytes = int(nb.value)
        self.device = torch.device(device)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.params = (torch.zeros(self.count, dtype=torch.float32, device=self.device) if params is None
                       else params.to(self.device, torch.float32).contiguous())
        assert self.params.numel() == self.count
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0

    @property
    def shape_in(self):
        d = self.desc
        return (d.n, d.cin, d.h, d.w)

    @property
    def shape_out(self):
        d = self.desc
        return (d.n, d.cout, d.h, d.w)

    def forward(self, x):
        out = torch.empty(self.shape_out, dtype=torch.float32, device=self.device)
        _check(_lib.ptlm_cnn_forward(ctypes.byref(self.desc), _ptr(self.params, torch.float32),
                                     _ptr(x, torch.float32, self.shape_in, "x"), _ptr(out, torch.float32),
                                     _vp(self.ws.data_ptr()), self.ws_bytes, _stream()))
        return out

    def loss_grad(self, x, t, mask):
        loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        grad = torch.empty_like(self.params)
        _check(_lib.ptlm_cnn_loss_grad(ctypes.byref(self.desc), _ptr(self.params, torch.float32),
                                       _ptr(x, torch.float32, self.shape_in, "x"),
                                       _ptr(t, torch.float32, self.shape_out, "t"),
                                       _ptr(mask, torch.float32, self.shape_out, "mask"),
                                       _ptr(loss, torch.float64), _ptr(grad, torch.float32),
                                       _vp(self.ws.data_ptr()), self.ws_bytes, _stream()))
        return loss, grad

    def adam(self, grad, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        _check(_lib.ptlm_cnn_adam(self.count, _ptr(self.params, torch.float32), _ptr(grad, torch.float32),
                                  _ptr(self.m, torch.float32), _ptr(self.v, torch.float32), self.step,
                                  lr, b1, b2, eps, _stream()))


def cnn_features(prob: "Problem"):
    out = torch.empty((3,) + prob.obj_shape, dtype=torch.float32, device=prob.device)
    _check(_lib.ptlm_cnn_features(prob.handle, _ptr(out, torch.float32), _stream()))
    return out


def learned_precond(prob: "Problem", r):
    n = prob.obj_shape[0] * prob.obj_shape[1] + (prob.probe_shape[0] * prob.probe_shape[1] if prob.joint else 0)
    out = torch.empty(2 * n, dtype=torch.float32, device=prob.device)
    _check(_lib.ptlm_learned_precond(prob.handle, _ptr(r, torch.float32, (2,) + prob.obj_shape, "r"),
                                     _ptr(out, torch.float32), _stream()))
    return out


def lm_set_cnn(prob: "Problem", cnn: "Cnn | None"):
    if cnn is None:
        _check(_lib.ptlm_lm_set_cnn(prob.handle, None, None, None, 0))
        prob._cnn = None
        return
    _check(_lib.ptlm_lm_set_cnn(prob.handle, ctypes.byref(cnn.desc), _ptr(cnn.params, torch.float32),
                                _vp(cnn.ws.data_ptr()), cnn.ws_bytes))
    prob._cnn = cnn  # keep the network's buffers alive while registered


class Batch:
    """Independent problems solved together (ptlm_batch_*): one workspace, one launch per step
    of an LM attempt for all problems, optionally replayed from a captured HIP graph.

    ``specs``: list of dicts with obj_shape, probe_shape, positions and optional metric, mode,
    background, ggn, seg_len.  ``problem(i)`` is a Problem view on the i-th handle (all single-problem calls)."""

    def __init__(self, specs, device="cuda"):
        self.device = torch.device(device)
        self.n = len(specs)
        self._pos = [np.ascontiguousarray(np.asarray(sp["positions"], dtype=np.int32).reshape(-1, 2))
                     for sp in specs]
        self.specs = specs
        descs = (ptlm_desc * self.n)(*[
            _desc(sp["obj_shape"], sp["probe_shape"], len(p), sp.get("metric", "gauss"), sp.get("mode", "joint"),
                  sp.get("background", 1e-8), sp.get("ggn", "magnitude"), sp.get("seg_len", 0))
            for sp, p in zip(specs, self._pos)])
        self._descs = descs
        self._pos_ptrs = (_vp * self.n)(*[p.ctypes.data_as(_vp) for p in self._pos])
        nb = ctypes.c_size_t(0)
        _check(_lib.ptlm_batch_workspace_bytes(self.n, descs, self._pos_ptrs, ctypes.byref(nb)))
        self.ws_bytes = int(nb.value)
        self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=self.device)
        h = _vp()
        _check(_lib.ptlm_batch_create(self.n, descs, self._pos_ptrs, _vp(self.ws.data_ptr()), self.ws_bytes,
                                      _stream(), ctypes.byref(h)))
        self.handle = h
        self.problems = []
        for i, sp in enumerate(specs):
            ph = _vp(_lib.ptlm_batch_problem(h, i))
            self.problems.append(Problem(sp["obj_shape"], sp["probe_shape"], self._pos[i],
                                         sp.get("metric", "gauss"), sp.get("mode", "joint"),
                                         sp.get("background", 1e-8), device, sp.get("ggn", "magnitude"),
                                         sp.get("seg_len", 0), _handle=ph, _owner=self))
        self.states = torch.zeros(self.n * STATE_BYTES, dtype=torch.uint8, device=self.device)
        self._bound = None

    def problem(self, i):
        return self.problems[i]

    def bind(self, Os, Ps, ys, params, T, use_graph=True):
        pr = self.problems
        oq = [pr[i]._o(Os[i]) for i in range(self.n)]
        pq = [pr[i]._p(Ps[i]) for i in range(self.n)]
        yq = [pr[i]._m(ys[i], "y") for i in range(self.n)]
        self._bound = (list(Os), list(Ps), list(ys), params)  # keep the buffers alive
        arr = lambda v: (_vp * self.n)(*v)
        _check(_lib.ptlm_batch_bind(self.handle, arr(oq), arr(pq), arr(yq), _vp(self.states.data_ptr()),
                                    ctypes.byref(params), int(T), 1 if use_graph else 0, _stream()))

    def attempt(self):
        _check(_lib.ptlm_batch_attempt(self.handle, _stream()))

    def cnn_refresh(self):
        """ptlm_batch_cnn_refresh: re-run every problem's network from its current probe."""
        _check(_lib.ptlm_batch_cnn_refresh(self.handle, _stream()))

    def solve(self, max_attempts, check_every=4):
        done = ctypes.c_int32(0)
        st = _check(_lib.ptlm_batch_solve(self.handle, int(max_attempts), int(check_every), ctypes.byref(done),
                                          _stream()), allow=(PTLM_OK, PTLM_ENOTACCEPTED, PTLM_ENUMERIC))
        return st, int(done.value)

    def state(self, i):
        raw = self.states.detach().cpu().numpy().tobytes()
        return ptlm_lm_state.from_buffer_copy(raw[i * STATE_BYTES:(i + 1) * STATE_BYTES])

    def all_states(self):
        raw = self.states.detach().cpu().numpy().tobytes()
        return [ptlm_lm_state.from_buffer_copy(raw[i * STATE_BYTES:(i + 1) * STATE_BYTES]) for i in range(self.n)]

    def __del__(self):
        h = self.__dict__.get("handle")
        if h is not None and h.value and _lib is not None:
            _lib.ptlm_batch_destroy(h)
            self.handle = None


def lm_set_cnn_refresh(prob: "Problem", every: int):
    _check(_lib.ptlm_lm_set_cnn_refresh(prob.handle, int(every)))


def lib():
    """The loaded ctypes library (for tests of the raw ABI)."""
    return _lib
