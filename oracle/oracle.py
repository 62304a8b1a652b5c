"""ctypes wrapper around the plain-C FP64 oracle (test infrastructure only)."""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fewha_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_long)
_ip = ctypes.POINTER(ctypes.c_int)


class _Wfs(ctypes.Structure):
    _fields_ = [("n_sub", ctypes.c_int), ("theta_x", ctypes.c_double), ("theta_y", ctypes.c_double),
                ("gs_height", ctypes.c_double), ("sigma", ctypes.c_double)]


class _Layer(ctypes.Structure):
    _fields_ = [("height", ctypes.c_double), ("cn2_weight", ctypes.c_double), ("spacing", ctypes.c_double),
                ("n", ctypes.c_int)]


class _Dm(ctypes.Structure):
    _fields_ = [("height", ctypes.c_double), ("pitch", ctypes.c_double), ("n_act", ctypes.c_int)]


def lib_path():
    return LIB


def build(force=False):
    """Compile the oracle with gcc (plain -O2, no vectorisation flags; OpenMP for the outer
    layer / guide-star loops only)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        L.orc_create.restype = ctypes.c_int
        L.orc_create.argtypes = [ctypes.POINTER(_Wfs), ctypes.c_int, ctypes.POINTER(_Layer), ctypes.c_int,
                                 ctypes.POINTER(_Dm), ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_void_p)]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_sizes.argtypes = [ctypes.c_void_p, _lp]
        for name in ("orc_W", "orc_Wt", "orc_P", "orc_Pt", "orc_apply_Ahat", "orc_apply_Ahat_t", "orc_apply_A",
                     "orc_apply_At", "orc_rhs", "orc_apply_M", "orc_fit_interp", "orc_fit_interp_t", "orc_apply_Hdm",
                     "orc_apply_Hdm_t"):
            getattr(L, name).argtypes = [ctypes.c_void_p, _dp, _dp]
        for name in ("orc_slope_mask", "orc_slope_weights", "orc_prior", "orc_precond"):
            getattr(L, name).argtypes = [ctypes.c_void_p, _dp]
        L.orc_gamma.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp]
        L.orc_gamma_t.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp]
        L.orc_active.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_build_precond.argtypes = [ctypes.c_void_p]
        L.orc_pcg.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_int, _dp, _ip]
        L.orc_frame.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, ctypes.c_int, ctypes.c_int, _dp]
        L.orc_fit.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_double, _dp]
        L.orc_pol.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        L.orc_fit_points.argtypes = [ctypes.c_void_p]
        L.orc_fit_points.restype = ctypes.c_long
        L.orc_ls_target.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_ls_H.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_ls_Ht.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_fit_ls.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int, ctypes.c_double, _dp]
        L.orc_fit_closed.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, ctypes.c_double, _dp]
        L.orc_db3.argtypes = [_dp]
        L.orc_dwt1_fwd.argtypes = [_dp, _dp, ctypes.c_int]
        L.orc_dwt1_inv.argtypes = [_dp, _dp, ctypes.c_int]
        L.orc_dwt2_fwd.argtypes = [_dp, _dp, ctypes.c_int, ctypes.c_int]
        L.orc_dwt2_inv.argtypes = [_dp, _dp, ctypes.c_int, ctypes.c_int]
        L.orc_level_of.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _ip, _ip]
        L.orc_dm_of_layer.argtypes = [ctypes.c_void_p, _ip]
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_get_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_dp)


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError("expected %d values, got %d" % (n, a.size))
    return a


def db3():
    h = np.zeros(6)
    _load().orc_db3(_p(h))
    return h


def dwt1(x, inverse=False):
    x = _f64(x)
    out = np.zeros_like(x)
    (_load().orc_dwt1_inv if inverse else _load().orc_dwt1_fwd)(_p(x), _p(out), x.size)
    return out


def dwt2(x, J, inverse=False):
    x = _f64(x)
    n = x.shape[0]
    out = np.zeros_like(x)
    (_load().orc_dwt2_inv if inverse else _load().orc_dwt2_fwd)(_p(x), _p(out), n, J)
    return out


def level_of(n, J, row, col):
    s, o = ctypes.c_int(), ctypes.c_int()
    _load().orc_level_of(n, J, row, col, ctypes.byref(s), ctypes.byref(o))
    return s.value, o.value


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__("oracle status %d" % status)
        self.status = status


class Oracle:
    """FP64 plan over one AO configuration dictionary; every method takes/returns numpy float64."""

    def __init__(self, cfg, precond=True):
        L = _load()
        self.cfg = cfg
        wf = (_Wfs * len(cfg["wfs"]))(*[_Wfs(w["n_sub"], w["theta_x"], w["theta_y"], w["gs_height"], w["sigma"])
                                       for w in cfg["wfs"]])
        ly = (_Layer * len(cfg["layers"]))(*[_Layer(l["height"], l["cn2_weight"], l["spacing"], l["n"])
                                            for l in cfg["layers"]])
        dm = (_Dm * len(cfg["dms"]))(*[_Dm(d["height"], d["pitch"], d["n_act"]) for d in cfg["dms"]])
        h = ctypes.c_void_p()
        st = L.orc_create(wf, len(cfg["wfs"]), ly, len(cfg["layers"]), dm, len(cfg["dms"]), cfg["D"],
                          cfg.get("obstruction", 0.0), cfg["J"], cfg["alpha_reg"], ctypes.byref(h))
        if st != 0:
            raise OracleError(st)
        self._h = h
        sz = (ctypes.c_long * 4)()
        L.orc_sizes(h, sz)
        self.n_coef, self.n_slopes, self.n_nodes, self.n_act = list(sz)
        self._precond = False
        if precond:
            self.build_precond()

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_destroy(self._h)
            self._h = None

    def _call(self, name, x, n_in, n_out):
        x = _f64(x, n_in)
        out = np.zeros(n_out)
        getattr(_lib, name)(self._h, _p(x), _p(out))
        return out

    # operators
    def W(self, layers): return self._call("orc_W", layers, self.n_coef, self.n_coef)
    def Wt(self, c): return self._call("orc_Wt", c, self.n_coef, self.n_coef)
    def P(self, layers): return self._call("orc_P", layers, self.n_coef, self.n_nodes)
    def Pt(self, phi): return self._call("orc_Pt", phi, self.n_nodes, self.n_coef)
    def Ahat(self, layers): return self._call("orc_apply_Ahat", layers, self.n_coef, self.n_slopes)
    def Ahat_t(self, s): return self._call("orc_apply_Ahat_t", s, self.n_slopes, self.n_coef)
    def A(self, c): return self._call("orc_apply_A", c, self.n_coef, self.n_slopes)
    def At(self, s): return self._call("orc_apply_At", s, self.n_slopes, self.n_coef)
    def rhs(self, s): return self._call("orc_rhs", s, self.n_slopes, self.n_coef)
    def M(self, c): return self._call("orc_apply_M", c, self.n_coef, self.n_coef)
    def fit_interp(self, layers): return self._call("orc_fit_interp", layers, self.n_coef, self.n_act)
    def fit_interp_t(self, a): return self._call("orc_fit_interp_t", a, self.n_act, self.n_coef)
    def Hdm(self, a): return self._call("orc_apply_Hdm", a, self.n_act, self.n_slopes)
    def Hdm_t(self, s): return self._call("orc_apply_Hdm_t", s, self.n_slopes, self.n_act)

    # least-squares DM fitting over the probe directions (L > M)
    def fit_points(self): return int(_lib.orc_fit_points(self._h))
    def ls_target(self, layers): return self._call("orc_ls_target", layers, self.n_coef, self.fit_points())
    def ls_H(self, a): return self._call("orc_ls_H", a, self.n_act, self.fit_points())
    def ls_Ht(self, y): return self._call("orc_ls_Ht", y, self.fit_points(), self.n_act)

    def fit_ls(self, c, n_cg, eps):
        """n_cg CG steps on (H^T H + eps I) a = H^T (target of W^T c) from a = 0."""
        a = np.zeros(self.n_act)
        _lib.orc_fit_ls(self._h, _p(_f64(c, self.n_coef)), int(n_cg), float(eps), _p(a))
        return a

    def pol(self, s, a_m1):
        """Pseudo-open-loop slopes of Alg. 1 (closed loop): mask (s + H_dm a^(-1))."""
        out = np.zeros(self.n_slopes)
        _lib.orc_pol(self._h, _p(_f64(s, self.n_slopes)), _p(_f64(a_m1, self.n_act)), _p(out))
        return out

    def fit_closed(self, c, a0, a_m1, gain):
        """Closed-loop control of Alg. 1: a^(1) = a^(0) + gain (F W^T c - a^(-1))."""
        a = np.zeros(self.n_act)
        _lib.orc_fit_closed(self._h, _p(_f64(c, self.n_coef)), _p(_f64(a0, self.n_act)), _p(_f64(a_m1, self.n_act)),
                            gain, _p(a))
        return a

    def gamma(self, g, phi):
        ns = self.cfg["wfs"][g]["n_sub"]
        phi = _f64(phi, (ns + 1) ** 2)
        s = np.zeros(2 * ns * ns)
        _lib.orc_gamma(self._h, g, _p(phi), _p(s))
        return s

    def gamma_t(self, g, s):
        ns = self.cfg["wfs"][g]["n_sub"]
        s = _f64(s, 2 * ns * ns)
        phi = np.zeros((ns + 1) ** 2)
        _lib.orc_gamma_t(self._h, g, _p(s), _p(phi))
        return phi

    def _vec(self, name, n):
        out = np.zeros(n)
        getattr(_lib, name)(self._h, _p(out))
        return out

    def slope_mask(self): return self._vec("orc_slope_mask", self.n_slopes)
    def slope_weights(self): return self._vec("orc_slope_weights", self.n_slopes)
    def prior(self): return self._vec("orc_prior", self.n_coef)

    def dm_of_layer(self):
        out = (ctypes.c_int * len(self.cfg["layers"]))()
        _lib.orc_dm_of_layer(self._h, out)
        return list(out)

    def build_precond(self):
        _lib.orc_build_precond(self._h)
        self._precond = True

    def precond(self):
        if not self._precond:
            self.build_precond()
        return self._vec("orc_precond", self.n_coef)

    # solver
    def pcg(self, c, r, n_iter):
        """Alg. 2 in place on copies; returns (c, r, resnorm, passes, status)."""
        c = _f64(c, self.n_coef).copy()
        r = _f64(r, self.n_coef).copy()
        res = np.zeros(max(n_iter, 1))
        done = ctypes.c_int()
        st = _lib.orc_pcg(self._h, _p(c), _p(r), n_iter, _p(res), ctypes.byref(done))
        return c, r, res[:done.value], done.value, st

    def frame(self, s, c, b_prev, r_prev, n_iter, cold):
        """One Alg. 1 frame (RHS, residual update, PCG); returns (c, b_prev, r_prev, resnorm, status)."""
        s = _f64(s, self.n_slopes)
        c = _f64(c, self.n_coef).copy()
        b_prev = _f64(b_prev, self.n_coef).copy()
        r_prev = _f64(r_prev, self.n_coef).copy()
        res = np.zeros(max(n_iter, 1))
        st = _lib.orc_frame(self._h, _p(s), _p(c), _p(b_prev), _p(r_prev), n_iter, int(bool(cold)), _p(res))
        return c, b_prev, r_prev, res[:n_iter], st

    def fit(self, c, a_prev, gain):
        c = _f64(c, self.n_coef)
        a = np.zeros(self.n_act)
        if a_prev is None:
            _lib.orc_fit(self._h, _p(c), None, gain, _p(a))
        else:
            ap = _f64(a_prev, self.n_act)
            _lib.orc_fit(self._h, _p(c), _p(ap), gain, _p(a))
        return a

    def active(self, g, i, j):
        return bool(_lib.orc_active(self._h, g, i, j))


def set_threads(n):
    """Threads of the oracle's outer layer / guide-star loops (results do not depend on it)."""
    _load().orc_set_threads(int(n))


def get_threads():
    return int(_load().orc_get_threads())
