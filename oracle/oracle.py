"""ctypes front end of the plain FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this module.  It never touches the GPU library.  Every quantity is computed
in FP64 by ``liboracle.so`` (``oracle.c``); this file only marshals arrays and
picks converged parameters for the reference solution.

Reference parameters (paper Sec. 4, eq:error_trunc_velocity; Sec. 5.1 uses
beta = 8 for its reference): with cut-off coefficient beta the truncation
errors decay like exp(-beta^2).  The oracle takes r_c = L (all images within
r_c are summed explicitly), alpha = beta / r_c and keeps every mode with
|m_i| <= K = ceil(beta * alpha * L / pi) (k_max = 2 beta alpha).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C11 + OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", _SO, _SRC, "-lm"])
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_SO)
        L.or_new.restype = C.c_void_p
        L.or_new.argtypes = [C.c_int64, _ip, _dp, _dp, C.c_double, C.c_double, C.c_double, C.c_int,
                             C.c_int, C.c_void_p]
        L.or_free.argtypes = [C.c_void_p]
        L.or_nquad.restype = C.c_int64
        L.or_nquad.argtypes = [C.c_void_p]
        L.or_get_quad.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_get_nodes.argtypes = [C.c_void_p] + [C.c_void_p] * 5
        L.or_spline_eval.argtypes = [C.c_void_p, C.c_int64, C.c_double, C.c_int, _dp]
        L.or_gl_rule.argtypes = [C.c_int, _dp, _dp]
        L.or_gl_rule.restype = C.c_int
        L.or_cyclic_tridiag.argtypes = [C.c_int64, _dp, _dp, _dp, _dp]
        for name in ("or_local",):
            getattr(L, name).argtypes = [C.c_void_p, C.c_int64, _ip, C.c_void_p, C.c_void_p]
        L.or_local_sub.argtypes = [C.c_void_p, C.c_double, C.c_int64, _ip, C.c_void_p,
                                   C.c_void_p]
        L.or_shortrange.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_int64, _ip,
                                    C.c_void_p, C.c_void_p]
        L.or_selfcorr.argtypes = [C.c_void_p, C.c_double, C.c_int64, _ip, C.c_void_p, C.c_void_p]
        L.or_longrange.argtypes = [C.c_void_p, C.c_double, C.c_int, C.c_int64, _ip,
                                   C.c_void_p, C.c_void_p]
        L.or_omega_hat.argtypes = [C.c_void_p, C.c_int, _dp]
        L.or_brute_images.argtypes = [C.c_void_p, C.c_int, C.c_int64, _ip, _dp]
        L.or_energy.restype = C.c_double
        L.or_energy.argtypes = [C.c_void_p, _dp]
        L.or_impulse.argtypes = [C.c_void_p, _dp]
        L.or_length.restype = C.c_double
        L.or_length.argtypes = [C.c_void_p]
        L.or_g_lr.restype = C.c_double
        L.or_g_lr.argtypes = [C.c_double]
        L.or_g_sr.restype = C.c_double
        L.or_g_sr.argtypes = [C.c_double]
        L.or_segment_integral.restype = C.c_int
        L.or_segment_integral.argtypes = [C.c_void_p, C.c_int64, _dp, _dp, C.c_double, _dp]
        L.or_segment_qsum.argtypes = [C.c_void_p, C.c_int64, _dp, _dp, _dp]
        L.or_chord_integral.argtypes = [_dp, _dp, _dp, C.c_double, _dp]
        L.or_ns_correction.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_int64, _ip,
                                       _dp, C.c_void_p]
        L.or_mlp_nparams.restype = C.c_int
        L.or_mlp_loss_grad.restype = C.c_double
        L.or_mlp_loss_grad.argtypes = [_dp, C.c_int64, _dp, C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_num_threads.restype = C.c_int
        L.or_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def gl_rule(Q: int):
    h = np.zeros(8)
    w = np.zeros(8)
    if lib().or_gl_rule(Q, h, w) != 0:
        raise ValueError(Q)
    return h[:Q].copy(), w[:Q].copy()


def cyclic_tridiag(a, b, c, r):
    x = np.array(r, dtype=np.float64, copy=True)
    lib().or_cyclic_tridiag(len(x), np.ascontiguousarray(a, float),
                            np.ascontiguousarray(b, float), np.ascontiguousarray(c, float), x)
    return x


def g_lr(x):
    return lib().or_g_lr(float(x))


def g_sr(x):
    return lib().or_g_sr(float(x))


def chord_integral(A, B, x, gamma=1.0):
    out = np.zeros(3)
    lib().or_chord_integral(np.ascontiguousarray(A, float), np.ascontiguousarray(B, float),
                            np.ascontiguousarray(x, float), float(gamma), out)
    return out


def num_threads() -> int:
    return lib().or_num_threads()


def reference_params(L: float, beta: float = 6.5, rc: float | None = None):
    """Converged Ewald parameters for the reference solution."""
    rc = L if rc is None else rc
    alpha = beta / rc
    K = int(math.ceil(2 * beta * alpha * L / (2 * math.pi)))
    return dict(alpha=alpha, rc=rc, K=K, beta=beta)


class Oracle:
    """FP64 geometry and Ewald components for one filament set."""

    def __init__(self, fs, Q: int = 2, order: int = 4):
        """order 4: periodic cubic spline; 6: periodic quintic spline (App. B)."""
        self.fs = fs
        self.Q = Q
        self.order = order
        self.N = fs.n_nodes
        off = np.ascontiguousarray(fs.offsets, dtype=np.int64)
        xyz = np.ascontiguousarray(fs.xyz, dtype=np.float64)
        gam = np.ascontiguousarray(fs.gamma, dtype=np.float64)
        per = getattr(fs, "periods", None)
        self._per = None if per is None else np.ascontiguousarray(per, dtype=np.int64)
        self._h = lib().or_new(fs.n_fil, off, xyz, gam, fs.L, fs.a, fs.delta, Q,
                               order, _ptr(self._per))
        if not self._h:
            raise ValueError("invalid filament set (N_l < 3, or < 6 for quintic, or "
                             "zero-length segment)")
        self.Nq = lib().or_nquad(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_free(h)
            self._h = None

    # --- geometry -------------------------------------------------------
    def quad(self):
        p = np.zeros((self.Nq, 3)); d = np.zeros((self.Nq, 3)); c = np.zeros((self.Nq, 3))
        lib().or_get_quad(self._h, _ptr(p), _ptr(d), _ptr(c))
        return p, d, c

    def nodes(self):
        N = self.N
        tau = np.zeros(N); dtau = np.zeros(N); sd = np.zeros((N, 3)); sdd = np.zeros((N, 3))
        ell = np.zeros(N)
        lib().or_get_nodes(self._h, _ptr(tau), _ptr(dtau), _ptr(sd), _ptr(sdd), _ptr(ell))
        return dict(tau=tau, dtau=dtau, sdot=sd, sddot=sdd, ell=ell)

    def spline_eval(self, seg: int, u: float, deriv: int = 0):
        out = np.zeros(3)
        lib().or_spline_eval(self._h, int(seg), float(u), int(deriv), out)
        return out

    # --- components --------------------------------------------------------
    def _tg(self, targets):
        if targets is None:
            return np.arange(self.N, dtype=np.int64)
        return np.ascontiguousarray(targets, dtype=np.int64)

    def local(self, targets=None):
        t = self._tg(targets)
        v = np.zeros((len(t), 3)); p = np.zeros((len(t), 3))
        lib().or_local(self._h, len(t), t, _ptr(v), _ptr(p))
        return v, p

    def local_sub(self, eps, targets=None):
        """Local terms with the local segments subdivided (Sec. 5.2)."""
        t = self._tg(targets)
        v = np.zeros((len(t), 3)); p = np.zeros((len(t), 3))
        lib().or_local_sub(self._h, float(eps), len(t), t, _ptr(v), _ptr(p))
        return v, p

    def shortrange(self, alpha, rc, targets=None, psi=True):
        t = self._tg(targets)
        v = np.zeros((len(t), 3)); p = np.zeros((len(t), 3)) if psi else None
        lib().or_shortrange(self._h, float(alpha), float(rc), len(t), t, _ptr(v), _ptr(p))
        return v, p

    def selfcorr(self, alpha, targets=None):
        t = self._tg(targets)
        v = np.zeros((len(t), 3)); p = np.zeros((len(t), 3))
        lib().or_selfcorr(self._h, float(alpha), len(t), t, _ptr(v), _ptr(p))
        return v, p

    def longrange(self, alpha, K, targets=None, psi=True):
        t = self._tg(targets)
        v = np.zeros((len(t), 3)); p = np.zeros((len(t), 3)) if psi else None
        lib().or_longrange(self._h, float(alpha), int(K), len(t), t, _ptr(v), _ptr(p))
        return v, p

    def omega_hat(self, K):
        W = 2 * K + 1
        out = np.zeros(2 * 3 * W * W * (K + 1))
        lib().or_omega_hat(self._h, int(K), out)
        z = out.reshape(K + 1, W, W, 3, 2)
        return z[..., 0] + 1j * z[..., 1]

    def brute_images(self, K, targets=None):
        t = self._tg(targets)
        v = np.zeros((len(t), 3))
        lib().or_brute_images(self._h, int(K), len(t), t, v)
        return v

    def ewald(self, alpha, rc, K, targets=None, psi=True, ns_eta=None, ns_tol=1e-13,
              local_eps=None):
        """Total v (and psi) = local + short + long - self (+ near-singular);
        local_eps subdivides the local segments (Sec. 5.2)."""
        vl, pl = self.local(targets) if local_eps is None else self.local_sub(local_eps, targets)
        vs, ps = self.shortrange(alpha, rc, targets, psi=psi)
        vL, pL = self.longrange(alpha, K, targets, psi=psi)
        vS, pS = self.selfcorr(alpha, targets)
        v = vl + vs + vL - vS
        p = (pl + ps + pL - pS) if psi else None
        if ns_eta is not None:
            v = v + self.ns_correction(ns_eta, targets, ns_tol)[0]
        return v, p

    def reference(self, targets=None, beta=6.5, rc=None, psi=True, ns_eta=None):
        prm = reference_params(self.fs.L, beta, rc)
        return self.ewald(prm["alpha"], prm["rc"], prm["K"], targets, psi=psi, ns_eta=ns_eta)

    # --- diagnostics -----------------------------------------------------
    def energy(self, psi_nodes):
        return lib().or_energy(self._h, np.ascontiguousarray(psi_nodes, dtype=np.float64))

    def impulse(self):
        p = np.zeros(3)
        lib().or_impulse(self._h, p)
        return p

    def length(self):
        return lib().or_length(self._h)

    # --- near-singular ---------------------------------------------------
    def segment_integral(self, seg, x, shift=(0, 0, 0), tol=1e-13):
        out = np.zeros(3)
        n = lib().or_segment_integral(self._h, int(seg), np.ascontiguousarray(x, float),
                                      np.ascontiguousarray(shift, float), float(tol), out)
        return out, n

    def segment_qsum(self, seg, x, shift=(0, 0, 0)):
        out = np.zeros(3)
        lib().or_segment_qsum(self._h, int(seg), np.ascontiguousarray(x, float),
                              np.ascontiguousarray(shift, float), out)
        return out

    def ns_correction(self, eta=1.0, targets=None, tol=1e-13):
        t = self._tg(targets)
        dv = np.zeros((len(t), 3))
        cnt = np.zeros(len(t), dtype=np.int64)
        lib().or_ns_correction(self._h, float(eta), float(tol), len(t), t, dv, _ptr(cnt))
        return dv, cnt


def mlp_nparams() -> int:
    return lib().or_mlp_nparams()


def mlp_forward(params, X):
    X = np.ascontiguousarray(X, dtype=np.float64)
    Y = np.zeros((X.shape[0], 3))
    lib().or_mlp_loss_grad(np.ascontiguousarray(params, float), X.shape[0], X, None, _ptr(Y), None)
    return Y


def mlp_loss_grad(params, X, T):
    X = np.ascontiguousarray(X, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.float64)
    G = np.zeros(mlp_nparams())
    loss = lib().or_mlp_loss_grad(np.ascontiguousarray(params, float), X.shape[0], X,
                                  _ptr(T), None, _ptr(G))
    return loss, G
