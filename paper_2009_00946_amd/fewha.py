"""Python binding of the FEWHA MI355X library (``libfewha.so``, C ABI in include/fewha.h).

Argument marshalling only: every operation runs in the library's HIP kernels.  PyTorch
provides device memory (the plan workspace and all vectors are torch CUDA tensors) and the
stream (``torch.cuda.current_stream()``).  There is no CPU fallback: without the built
library every entry point raises.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfewha.so")

FEWHA_FP32, FEWHA_FP64 = 0, 1
FEWHA_COLD, FEWHA_WARM, FEWHA_REFRESH = 0, 1, 2
STATUS = {0: "FEWHA_OK", -1: "FEWHA_ERR_INVALID_ARG", -2: "FEWHA_ERR_GEOMETRY", -3: "FEWHA_ERR_UNSUPPORTED",
          -4: "FEWHA_ERR_HIP", -5: "FEWHA_ERR_WORKSPACE", -6: "FEWHA_ERR_BREAKDOWN", -7: "FEWHA_ERR_NONFINITE"}

EXPORTS = ["fewha_plan_create", "fewha_workspace_bytes", "fewha_plan_bind", "fewha_plan_destroy", "fewha_sizes",
           "fewha_apply_A", "fewha_apply_At", "fewha_apply_M", "fewha_dwt_forward", "fewha_dwt_inverse",
           "fewha_pcg_solve", "fewha_fit_dm", "fewha_state_get", "fewha_state_set", "fewha_precond_table",
           "fewha_last_status", "fewha_stage_launch", "fewha_strerror", "fewha_solve_M", "fewha_apply_CA",
           "fewha_prior_dot", "fewha_plan_set_batch", "fewha_apply_A_batch", "fewha_apply_At_batch",
           "fewha_apply_M_batch", "fewha_pcg_solve_batch", "fewha_fit_dm_batch", "fewha_last_status_batch",
           "fewha_pol_slopes", "fewha_fit_dm_closed", "fewha_pol_slopes_batch", "fewha_fit_dm_closed_batch",
           "fewha_fit_dm_ls", "fewha_cn2_gradient", "fewha_dwt_forward_noalloc", "fewha_stage_launch_batch",
           "fewha_get_tuning", "fewha_set_tuning", "fewha_autotune", "fewha_reconstruct", "fewha_reconstruct_batch"]


class FewhaError(RuntimeError):
    def __init__(self, status, what=""):
        super().__init__("%s: %s (%d)" % (what, STATUS.get(status, "unknown"), status))
        self.status = status


class _Wfs(ctypes.Structure):
    _fields_ = [("n_sub", ctypes.c_int), ("theta_x", ctypes.c_double), ("theta_y", ctypes.c_double),
                ("gs_height", ctypes.c_double), ("sigma", ctypes.c_double)]


class _Layer(ctypes.Structure):
    _fields_ = [("height", ctypes.c_double), ("cn2_weight", ctypes.c_double), ("spacing", ctypes.c_double),
                ("n", ctypes.c_int)]


class _Dm(ctypes.Structure):
    _fields_ = [("height", ctypes.c_double), ("pitch", ctypes.c_double), ("n_act", ctypes.c_int)]


class _Tuning(ctypes.Structure):
    _fields_ = [("kf", ctypes.c_int), ("tq", ctypes.c_int), ("chunk_wt", ctypes.c_int), ("chunk_proj", ctypes.c_int),
                ("chunk_pt", ctypes.c_int), ("chunk_fwd", ctypes.c_int), ("fold", ctypes.c_int)]


TUNING_FIELDS = [f for f, _ in _Tuning._fields_]


class _Config(ctypes.Structure):
    _fields_ = [("D", ctypes.c_double), ("obstruction", ctypes.c_double), ("n_wfs", ctypes.c_int),
                ("n_layers", ctypes.c_int), ("n_dms", ctypes.c_int), ("J", ctypes.c_int),
                ("wfs", ctypes.POINTER(_Wfs)), ("layers", ctypes.POINTER(_Layer)), ("dms", ctypes.POINTER(_Dm)),
                ("alpha_reg", ctypes.c_double), ("precision", ctypes.c_int)]


_lib = None


def load_library():
    """Load libfewha.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libfewha.so is not built (run python -m paper_2009_00946_amd.build)")
    # torch first: the library then binds to the HIP runtime torch has loaded (same soname), so
    # the process has one runtime.  Loaded first, the library would bring a second runtime that
    # does not see the device torch has opened.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    L.fewha_plan_create.argtypes = [ctypes.POINTER(_Config), ctypes.POINTER(vp)]
    L.fewha_workspace_bytes.argtypes = [vp]
    L.fewha_workspace_bytes.restype = sz
    L.fewha_plan_bind.argtypes = [vp, vp, sz, vp]
    L.fewha_plan_destroy.argtypes = [vp]
    L.fewha_sizes.argtypes = [vp, ctypes.POINTER(sz), ctypes.POINTER(sz), ctypes.POINTER(sz)]
    for name in ("fewha_apply_A", "fewha_apply_At", "fewha_apply_M", "fewha_dwt_forward", "fewha_dwt_inverse",
                 "fewha_state_get", "fewha_state_set", "fewha_apply_CA", "fewha_dwt_forward_noalloc"):
        getattr(L, name).argtypes = [vp, vp, vp, vp]
    L.fewha_solve_M.argtypes = [vp, vp, vp, ctypes.c_int, vp, vp]
    L.fewha_plan_set_batch.argtypes = [vp, ctypes.c_int]
    for name in ("fewha_apply_A_batch", "fewha_apply_At_batch", "fewha_apply_M_batch"):
        getattr(L, name).argtypes = [vp, ctypes.c_int, vp, vp, vp]
    L.fewha_pcg_solve_batch.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_int, ctypes.c_int, vp, vp]
    L.fewha_fit_dm_batch.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_double, vp, vp]
    L.fewha_last_status_batch.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    L.fewha_pol_slopes.argtypes = [vp, vp, vp, vp, vp]
    L.fewha_fit_dm_ls.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_int, ctypes.c_double, vp, vp]
    L.fewha_fit_dm_closed.argtypes = [vp, vp, vp, vp, ctypes.c_double, vp, vp]
    L.fewha_pol_slopes_batch.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
    L.fewha_fit_dm_closed_batch.argtypes = [vp, ctypes.c_int, vp, vp, vp, ctypes.c_double, vp, vp]
    L.fewha_prior_dot.argtypes = [vp, vp, vp, vp, vp]
    L.fewha_cn2_gradient.argtypes = [vp, vp, vp, vp, vp]
    L.fewha_pcg_solve.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int, vp, vp]
    L.fewha_fit_dm.argtypes = [vp, vp, vp, ctypes.c_double, vp, vp]
    L.fewha_reconstruct.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int, vp, vp, ctypes.c_double, vp, vp]
    L.fewha_reconstruct_batch.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_int, ctypes.c_int, vp, vp,
                                          ctypes.c_double, vp, vp]
    L.fewha_precond_table.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.fewha_last_status.argtypes = [vp]
    L.fewha_stage_launch.argtypes = [vp, ctypes.c_int, vp]
    L.fewha_stage_launch_batch.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp]
    L.fewha_get_tuning.argtypes = [vp, ctypes.POINTER(_Tuning)]
    L.fewha_set_tuning.argtypes = [vp, ctypes.POINTER(_Tuning)]
    L.fewha_autotune.argtypes = [vp, ctypes.c_int, ctypes.POINTER(_Tuning), ctypes.POINTER(ctypes.c_double)]
    L.fewha_strerror.argtypes = [ctypes.c_int]
    L.fewha_strerror.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(st, what):
    if st != 0:
        raise FewhaError(st, what)


def make_config(cfg, precision=None):
    """ctypes fewha_config from a configuration dictionary; returns (struct, keepalive)."""
    prec = cfg.get("precision", "fp32") if precision is None else precision
    prec = FEWHA_FP64 if prec in ("fp64", FEWHA_FP64) else FEWHA_FP32
    wfs = (_Wfs * len(cfg["wfs"]))(*[_Wfs(int(w["n_sub"]), float(w["theta_x"]), float(w["theta_y"]),
                                          float(w["gs_height"]), float(w["sigma"])) for w in cfg["wfs"]])
    lay = (_Layer * len(cfg["layers"]))(*[_Layer(float(l["height"]), float(l["cn2_weight"]), float(l["spacing"]),
                                                 int(l["n"])) for l in cfg["layers"]])
    dms = (_Dm * len(cfg["dms"]))(*[_Dm(float(d["height"]), float(d["pitch"]), int(d["n_act"])) for d in cfg["dms"]])
    c = _Config(float(cfg["D"]), float(cfg.get("obstruction", 0.0)), len(cfg["wfs"]), len(cfg["layers"]),
                len(cfg["dms"]), int(cfg["J"]), wfs, lay, dms, float(cfg["alpha_reg"]), prec)
    return c, (wfs, lay, dms)


def create_host_plan(cfg, precision=None):
    """Validate and size a plan without touching a GPU; returns (handle, status)."""
    L = load_library()
    c, keep = make_config(cfg, precision)
    h = ctypes.c_void_p()
    st = L.fewha_plan_create(ctypes.byref(c), ctypes.byref(h))
    return (h if st == 0 else None), st


class Plan:
    """A bound FEWHA plan on the current CUDA (HIP) device.

    ``precision`` overrides the configuration's ("fp32" or "fp64").  All tensors must be
    contiguous CUDA tensors of ``self.dtype`` with the lengths of ``fewha_sizes``.
    """

    def __init__(self, cfg, precision=None, device=None, max_batch=1):
        import torch
        self._torch = torch
        L = load_library()
        self.cfg = cfg
        c, keep = make_config(cfg, precision)
        self.precision = "fp64" if c.precision == FEWHA_FP64 else "fp32"
        self.dtype = torch.float64 if c.precision == FEWHA_FP64 else torch.float32
        h = ctypes.c_void_p()
        _check(L.fewha_plan_create(ctypes.byref(c), ctypes.byref(h)), "fewha_plan_create")
        self._h = h
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        nc, ns, na = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        L.fewha_sizes(h, ctypes.byref(nc), ctypes.byref(ns), ctypes.byref(na))
        self.n_coef, self.n_slopes, self.n_act = nc.value, ns.value, na.value
        self.max_batch = int(max_batch)
        if self.max_batch != 1:
            _check(L.fewha_plan_set_batch(h, self.max_batch), "fewha_plan_set_batch")
        nbytes = L.fewha_workspace_bytes(h)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            self._ws_ptr = (base + 255) & ~255
            _check(L.fewha_plan_bind(h, self._ws_ptr, nbytes, self._stream()), "fewha_plan_bind")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.fewha_plan_destroy(h)
            self._h = None

    # -- helpers -------------------------------------------------------------------------------
    def _stream(self):
        return self._torch.cuda.current_stream(self.device).cuda_stream

    def _arg(self, t, n, name):
        if not t.is_cuda or t.dtype != self.dtype or not t.is_contiguous() or t.numel() != n:
            raise ValueError("%s: expected a contiguous %s CUDA tensor of %d elements, got %s %s %s"
                             % (name, self.dtype, n, tuple(t.shape), t.dtype, t.device))
        return t.data_ptr()

    def _out(self, out, n):
        if out is None:
            return self._torch.empty(n, dtype=self.dtype, device=self.device)
        return out

    def empty(self, n):
        return self._torch.empty(n, dtype=self.dtype, device=self.device)

    def zeros(self, n):
        return self._torch.zeros(n, dtype=self.dtype, device=self.device)

    # -- operators -----------------------------------------------------------------------------
    def apply_A(self, c, out=None):
        s = self._out(out, self.n_slopes)
        _check(_lib.fewha_apply_A(self._h, self._arg(c, self.n_coef, "c"), self._arg(s, self.n_slopes, "s"),
                                  self._stream()), "fewha_apply_A")
        return s

    def apply_At(self, s, out=None):
        c = self._out(out, self.n_coef)
        _check(_lib.fewha_apply_At(self._h, self._arg(s, self.n_slopes, "s"), self._arg(c, self.n_coef, "c"),
                                   self._stream()), "fewha_apply_At")
        return c

    def apply_M(self, c, out=None):
        y = self._out(out, self.n_coef)
        _check(_lib.fewha_apply_M(self._h, self._arg(c, self.n_coef, "c"), self._arg(y, self.n_coef, "y"),
                                  self._stream()), "fewha_apply_M")
        return y

    def dwt_forward(self, layers, out=None):
        c = self._out(out, self.n_coef)
        _check(_lib.fewha_dwt_forward(self._h, self._arg(layers, self.n_coef, "layers"),
                                      self._arg(c, self.n_coef, "c"), self._stream()), "fewha_dwt_forward")
        return c

    def dwt_forward_noalloc(self, layers, out=None):
        """W x through the entry point that allocates nothing (library-owned scratch array)."""
        c = self._out(out, self.n_coef)
        _check(_lib.fewha_dwt_forward_noalloc(self._h, self._arg(layers, self.n_coef, "layers"),
                                              self._arg(c, self.n_coef, "c"), self._stream()),
               "fewha_dwt_forward_noalloc")
        return c

    def dwt_inverse(self, c, out=None):
        x = self._out(out, self.n_coef)
        _check(_lib.fewha_dwt_inverse(self._h, self._arg(c, self.n_coef, "c"),
                                      self._arg(x, self.n_coef, "layers"), self._stream()), "fewha_dwt_inverse")
        return x

    # -- solver --------------------------------------------------------------------------------
    @staticmethod
    def _flags(warm, refresh):
        if refresh and not warm:
            raise ValueError("refresh applies to warm starts")
        return FEWHA_REFRESH if refresh else (FEWHA_WARM if warm else FEWHA_COLD)

    def pcg_solve(self, s, c, n_iter, warm=True, resnorm=None, refresh=False):
        """One frame (RHS, residual update, n_iter PCG passes); c is updated in place and returned.
        ``refresh`` (warm starts): the residual is recomputed as b - M c instead of carried."""
        rp = None
        if resnorm is not None:
            if not resnorm.is_cuda or resnorm.dtype != self._torch.float64 or resnorm.numel() < n_iter:
                raise ValueError("resnorm: float64 CUDA tensor of n_iter elements expected")
            rp = resnorm.data_ptr()
        _check(_lib.fewha_pcg_solve(self._h, self._arg(s, self.n_slopes, "s"), self._arg(c, self.n_coef, "c"),
                                    int(n_iter), self._flags(warm, refresh), rp, self._stream()),
               "fewha_pcg_solve")
        return c

    def reconstruct(self, s, c, n_iter, a_prev=None, gain=1.0, out=None, warm=True, resnorm=None, refresh=False):
        """pcg_solve then fit_dm in one call (the last pass's coarse levels run beside the fit);
        returns the actuator commands."""
        rp = None
        if resnorm is not None:
            if not resnorm.is_cuda or resnorm.dtype != self._torch.float64 or resnorm.numel() < n_iter:
                raise ValueError("resnorm: float64 CUDA tensor of n_iter elements expected")
            rp = resnorm.data_ptr()
        a = self._out(out, self.n_act)
        ap = None if a_prev is None else self._arg(a_prev, self.n_act, "a_prev")
        _check(_lib.fewha_reconstruct(self._h, self._arg(s, self.n_slopes, "s"), self._arg(c, self.n_coef, "c"),
                                      int(n_iter), self._flags(warm, refresh), rp, ap, float(gain),
                                      self._arg(a, self.n_act, "a"), self._stream()), "fewha_reconstruct")
        return a

    def solve_M(self, b, c=None, n_iter=None, resnorm=None):
        """c = M^-1 b (n_iter cold PCG passes) for a wavelet-domain right-hand side; overwrites the
        warm-restart state."""
        n_iter = int(self.cfg["n_iter"] if n_iter is None else n_iter)
        c = self._out(c, self.n_coef)
        rp = None
        if resnorm is not None:
            if not resnorm.is_cuda or resnorm.dtype != self._torch.float64 or resnorm.numel() < n_iter:
                raise ValueError("resnorm: float64 CUDA tensor of n_iter elements expected")
            rp = resnorm.data_ptr()
        _check(_lib.fewha_solve_M(self._h, self._arg(b, self.n_coef, "b"), self._arg(c, self.n_coef, "c"), n_iter,
                                  rp, self._stream()), "fewha_solve_M")
        return c

    def apply_CA(self, c, out=None):
        s = self._out(out, self.n_slopes)
        _check(_lib.fewha_apply_CA(self._h, self._arg(c, self.n_coef, "c"), self._arg(s, self.n_slopes, "s"),
                                   self._stream()), "fewha_apply_CA")
        return s

    def prior_dot(self, x, y):
        """Per layer: sum of x alpha D y over the layer's coefficients (float64 CUDA tensor)."""
        out = self._torch.empty(len(self.cfg["layers"]), dtype=self._torch.float64, device=self.device)
        _check(_lib.fewha_prior_dot(self._h, self._arg(x, self.n_coef, "x"), self._arg(y, self.n_coef, "y"),
                                    out.data_ptr(), self._stream()), "fewha_prior_dot")
        return out

    def cn2_gradient(self, lam, c):
        """Per layer: lambda_l^T (alpha D)_l c_l / gamma_l (float64 CUDA tensor), the implicit
        gradient of a loss of c = M^-1 b with respect to the Cn^2 weights, lambda = M^-1 dL/dc."""
        out = self._torch.empty(len(self.cfg["layers"]), dtype=self._torch.float64, device=self.device)
        _check(_lib.fewha_cn2_gradient(self._h, self._arg(lam, self.n_coef, "lambda"), self._arg(c, self.n_coef, "c"),
                                       out.data_ptr(), self._stream()), "fewha_cn2_gradient")
        return out

    # -- batches of frames (one launch per stage over every frame; tensors [nbatch][length]) ---------
    def _batch(self, t, n, name):
        if t.dim() != 2 or t.shape[1] != n or not (1 <= t.shape[0] <= self.max_batch):
            raise ValueError("%s: expected [nbatch <= %d][%d], got %s" % (name, self.max_batch, n, tuple(t.shape)))
        self._arg(t, t.numel(), name)
        return t.shape[0]

    def apply_A_batch(self, c, out=None):
        nb = self._batch(c, self.n_coef, "c")
        s = out if out is not None else self._torch.empty((nb, self.n_slopes), dtype=self.dtype, device=self.device)
        self._batch(s, self.n_slopes, "s")
        _check(_lib.fewha_apply_A_batch(self._h, nb, c.data_ptr(), s.data_ptr(), self._stream()), "fewha_apply_A_batch")
        return s

    def apply_At_batch(self, s, out=None):
        nb = self._batch(s, self.n_slopes, "s")
        c = out if out is not None else self._torch.empty((nb, self.n_coef), dtype=self.dtype, device=self.device)
        self._batch(c, self.n_coef, "c")
        _check(_lib.fewha_apply_At_batch(self._h, nb, s.data_ptr(), c.data_ptr(), self._stream()), "fewha_apply_At_batch")
        return c

    def apply_M_batch(self, c, out=None):
        nb = self._batch(c, self.n_coef, "c")
        y = out if out is not None else self._torch.empty((nb, self.n_coef), dtype=self.dtype, device=self.device)
        self._batch(y, self.n_coef, "y")
        _check(_lib.fewha_apply_M_batch(self._h, nb, c.data_ptr(), y.data_ptr(), self._stream()), "fewha_apply_M_batch")
        return y

    def pcg_solve_batch(self, s, c, n_iter, warm=True, resnorm=None, refresh=False):
        """Frames f = 0..nbatch-1 (s [nbatch][n_slopes], c [nbatch][n_coef] updated in place), one
        launch per stage; frame f continues its own warm-restart chain."""
        nb = self._batch(s, self.n_slopes, "s")
        if self._batch(c, self.n_coef, "c") != nb:
            raise ValueError("s and c: different batch sizes")
        rp = None
        if resnorm is not None:
            if not resnorm.is_cuda or resnorm.dtype != self._torch.float64 or resnorm.numel() < nb * n_iter:
                raise ValueError("resnorm: float64 CUDA tensor of nbatch * n_iter elements expected")
            rp = resnorm.data_ptr()
        _check(_lib.fewha_pcg_solve_batch(self._h, nb, s.data_ptr(), c.data_ptr(), int(n_iter),
                                          self._flags(warm, refresh), rp, self._stream()),
               "fewha_pcg_solve_batch")
        return c

    def reconstruct_batch(self, s, c, n_iter, a_prev=None, gain=1.0, out=None, warm=True, resnorm=None,
                          refresh=False):
        """pcg_solve_batch then fit_dm_batch in one call; returns the [nbatch][n_act] commands."""
        nb = self._batch(s, self.n_slopes, "s")
        if self._batch(c, self.n_coef, "c") != nb:
            raise ValueError("s and c: different batch sizes")
        rp = None
        if resnorm is not None:
            if not resnorm.is_cuda or resnorm.dtype != self._torch.float64 or resnorm.numel() < nb * n_iter:
                raise ValueError("resnorm: float64 CUDA tensor of nbatch * n_iter elements expected")
            rp = resnorm.data_ptr()
        a = out if out is not None else self._torch.empty((nb, self.n_act), dtype=self.dtype, device=self.device)
        self._batch(a, self.n_act, "a")
        ap = None
        if a_prev is not None:
            self._batch(a_prev, self.n_act, "a_prev")
            ap = a_prev.data_ptr()
        _check(_lib.fewha_reconstruct_batch(self._h, nb, s.data_ptr(), c.data_ptr(), int(n_iter),
                                            self._flags(warm, refresh), rp, ap, float(gain), a.data_ptr(),
                                            self._stream()), "fewha_reconstruct_batch")
        return a

    def fit_dm_batch(self, c, a_prev=None, gain=1.0, out=None):
        nb = self._batch(c, self.n_coef, "c")
        a = out if out is not None else self._torch.empty((nb, self.n_act), dtype=self.dtype, device=self.device)
        self._batch(a, self.n_act, "a")
        ap = None
        if a_prev is not None:
            self._batch(a_prev, self.n_act, "a_prev")
            ap = a_prev.data_ptr()
        _check(_lib.fewha_fit_dm_batch(self._h, nb, c.data_ptr(), ap, float(gain), a.data_ptr(), self._stream()),
               "fewha_fit_dm_batch")
        return a

    def last_status_batch(self, nbatch):
        out = (ctypes.c_int * nbatch)()
        _check(_lib.fewha_last_status_batch(self._h, int(nbatch), out), "fewha_last_status_batch")
        return list(out)

    # -- closed loop (Alg. 1) ----------------------------------------------------------------------
    def pol_slopes(self, s, a_m1, out=None):
        """Pseudo-open-loop slopes mask (s + Gamma P_DM a_m1) (a_m1: the DM shape two frames back)."""
        sp = self._out(out, self.n_slopes)
        _check(_lib.fewha_pol_slopes(self._h, self._arg(s, self.n_slopes, "s"), self._arg(a_m1, self.n_act, "a_m1"),
                                     self._arg(sp, self.n_slopes, "s_pol"), self._stream()), "fewha_pol_slopes")
        return sp

    def fit_dm_closed(self, c, a0, a_m1, gain, out=None):
        """Closed-loop control: a0 + gain (F W^T c - a_m1)."""
        a = self._out(out, self.n_act)
        _check(_lib.fewha_fit_dm_closed(self._h, self._arg(c, self.n_coef, "c"), self._arg(a0, self.n_act, "a0"),
                                        self._arg(a_m1, self.n_act, "a_m1"), float(gain),
                                        self._arg(a, self.n_act, "a"), self._stream()), "fewha_fit_dm_closed")
        return a

    def pol_slopes_batch(self, s, a_m1, out=None):
        nb = self._batch(s, self.n_slopes, "s")
        if self._batch(a_m1, self.n_act, "a_m1") != nb:
            raise ValueError("s and a_m1: different batch sizes")
        sp = out if out is not None else self._torch.empty((nb, self.n_slopes), dtype=self.dtype, device=self.device)
        self._batch(sp, self.n_slopes, "s_pol")
        _check(_lib.fewha_pol_slopes_batch(self._h, nb, s.data_ptr(), a_m1.data_ptr(), sp.data_ptr(), self._stream()),
               "fewha_pol_slopes_batch")
        return sp

    def fit_dm_closed_batch(self, c, a0, a_m1, gain, out=None):
        nb = self._batch(c, self.n_coef, "c")
        for t, nm in ((a0, "a0"), (a_m1, "a_m1")):
            if self._batch(t, self.n_act, nm) != nb:
                raise ValueError("%s: different batch size" % nm)
        a = out if out is not None else self._torch.empty((nb, self.n_act), dtype=self.dtype, device=self.device)
        self._batch(a, self.n_act, "a")
        _check(_lib.fewha_fit_dm_closed_batch(self._h, nb, c.data_ptr(), a0.data_ptr(), a_m1.data_ptr(), float(gain),
                                              a.data_ptr(), self._stream()), "fewha_fit_dm_closed_batch")
        return a

    def fit_dm_ls(self, c, a_prev=None, gain=1.0, n_cg=30, eps=1e-2, out=None):
        """Least-squares fitting over the 25 probe directions (n_cg CG steps), then the gain."""
        a = self._out(out, self.n_act)
        ap = None if a_prev is None else self._arg(a_prev, self.n_act, "a_prev")
        _check(_lib.fewha_fit_dm_ls(self._h, self._arg(c, self.n_coef, "c"), ap, float(gain), int(n_cg), float(eps),
                                    self._arg(a, self.n_act, "a"), self._stream()), "fewha_fit_dm_ls")
        return a

    def fit_dm(self, c, a_prev=None, gain=1.0, out=None):
        a = self._out(out, self.n_act)
        ap = None if a_prev is None else self._arg(a_prev, self.n_act, "a_prev")
        _check(_lib.fewha_fit_dm(self._h, self._arg(c, self.n_coef, "c"), ap, float(gain),
                                 self._arg(a, self.n_act, "a"), self._stream()), "fewha_fit_dm")
        return a

    def state_get(self):
        b, r = self.empty(self.n_coef), self.empty(self.n_coef)
        _check(_lib.fewha_state_get(self._h, b.data_ptr(), r.data_ptr(), self._stream()), "fewha_state_get")
        return b, r

    def state_set(self, b_prev, r_prev):
        _check(_lib.fewha_state_set(self._h, self._arg(b_prev, self.n_coef, "b_prev"),
                                    self._arg(r_prev, self.n_coef, "r_prev"), self._stream()), "fewha_state_set")

    def precond_table(self):
        import numpy as np
        J, nl = int(self.cfg["J"]), len(self.cfg["layers"])
        out = np.zeros(nl * (J + 1) * 4)
        _check(_lib.fewha_precond_table(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               "fewha_precond_table")
        return out.reshape(nl, J + 1, 4)

    STAGES = {"wt": 0, "proj": 1, "pt": 2, "fwd": 3}

    def stage_launch(self, stage):
        """Enqueue one launch of one PCG-pass stage ("wt", "proj", "pt", "fwd") for timing."""
        _check(_lib.fewha_stage_launch(self._h, self.STAGES[stage], self._stream()), "fewha_stage_launch")

    def stage_launch_batch(self, stage, nbatch):
        """Enqueue one launch of one PCG-pass stage over frames 0..nbatch-1 of a batched plan."""
        _check(_lib.fewha_stage_launch_batch(self._h, int(nbatch), self.STAGES[stage], self._stream()),
               "fewha_stage_launch_batch")

    # -- launch shapes ----------------------------------------------------------------------------
    def get_tuning(self):
        t = _Tuning()
        _check(_lib.fewha_get_tuning(self._h, ctypes.byref(t)), "fewha_get_tuning")
        return {f: getattr(t, f) for f in TUNING_FIELDS}

    def set_tuning(self, tuning):
        t = _Tuning(*[int(tuning[f]) for f in TUNING_FIELDS])
        _check(_lib.fewha_set_tuning(self._h, ctypes.byref(t)), "fewha_set_tuning")

    def autotune(self, nbatch=None):
        """Time the stage kernels for every launch shape and keep the fastest (resets the chain
        state); returns (tuning, tuned microseconds per stage launch)."""
        nb = self.max_batch if nbatch is None else int(nbatch)
        t = _Tuning()
        us = (ctypes.c_double * 4)()
        _check(_lib.fewha_autotune(self._h, nb, ctypes.byref(t), us), "fewha_autotune")
        return {f: getattr(t, f) for f in TUNING_FIELDS}, dict(zip(("wt", "proj", "pt", "fwd"), list(us)))

    def last_status(self):
        return _lib.fewha_last_status(self._h)
