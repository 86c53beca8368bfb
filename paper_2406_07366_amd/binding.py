"""Thin ctypes binding of libbs.so (argument marshalling only).

Every step of the velocity / energy evaluation runs in the HIP kernels of
libbs.so; this module only converts torch tensors and numpy arrays into the
pointers and sizes of the C ABI declared in include/bs.h.  PyTorch provides
device memory and the HIP stream.  There is no fallback: if libbs.so is not
built, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbs.so")

BS_OK, BS_EINVAL, BS_EMINIMG, BS_ETOL, BS_EKB, BS_ENOMEM, BS_EDEVICE, BS_ESTATE = \
    0, -1, -2, -3, -4, -5, -6, -7
BS_FP64, BS_FP32_MIXED = 0, 1
BS_NS_OFF, BS_NS_ADAPTIVE, BS_NS_MLP, BS_NS_MAPPED = 0, 1, 2, 3
BS_FFT_AUTO, BS_FFT_LIBRARY, BS_FFT_PRUNED = 0, 1, 2

_CODES = {0: "BS_OK", -1: "BS_EINVAL", -2: "BS_EMINIMG", -3: "BS_ETOL", -4: "BS_EKB",
          -5: "BS_ENOMEM", -6: "BS_EDEVICE", -7: "BS_ESTATE"}

EXPORTED = ["bs_resolve_params", "bs_plan", "bs_set_filaments", "bs_set_periods", "bs_velocity",
            "bs_velocity_terms", "bs_energy", "bs_vorticity_modes", "bs_geometry",
            "bs_status", "bs_set_profiling", "bs_stage_times", "bs_get_params",
            "bs_destroy", "bs_last_error", "bs_mlp_nparams", "bs_mlp_create",
            "bs_mlp_forward", "bs_mlp_loss_grad", "bs_mlp_adam_step", "bs_mlp_get_params",
            "bs_mlp_set_fp32",
            "bs_mlp_destroy", "bs_ns_samples", "bs_ns_error_bins", "bs_ns_error_table",
            "bs_ns_error_table_noalloc",
            "bs_set_mlp", "bs_ns_counts", "bs_rk4_step", "bs_step", "bs_set_graph",
            "bs_graph_active"]

NSTAGES = 11
STAGES = ["geometry", "binning", "local_self", "spread", "fft_fwd", "spectral", "fft_inv",
          "interp", "pairs", "ns", "ns_flag"]


class BsParams(C.Structure):
    _fields_ = [("L", C.c_double), ("a", C.c_double), ("delta", C.c_double),
                ("tol", C.c_double), ("beta", C.c_double), ("alpha", C.c_double),
                ("rcut", C.c_double), ("grid_n", C.c_int), ("sigma", C.c_double),
                ("w", C.c_int), ("Q", C.c_int), ("spline_order", C.c_int),
                ("precision", C.c_int), ("ns_mode", C.c_int), ("ns_eta", C.c_double),
                ("fft_mode", C.c_int),
                ("local_frac", C.c_double), ("K", C.c_int),
                ("ncell", C.c_int),
                ("zeta", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2406_07366_amd.build "
                      "(hipcc --offload-arch=gfx950)")

# torch ships its own HIP runtime (same soname as the system one).  Loading
# torch first makes libbs.so bind to that already-loaded runtime instead of
# pulling in a second copy, which would leave two runtimes fighting over the
# device in one process.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)
_vp = C.c_void_p
_lib.bs_resolve_params.argtypes = [C.POINTER(BsParams), C.POINTER(BsParams)]
_lib.bs_plan.argtypes = [C.POINTER(BsParams), _vp, C.POINTER(_vp)]
_lib.bs_set_filaments.argtypes = [_vp, C.c_int64, C.POINTER(C.c_int64), _vp, _vp]
_lib.bs_set_periods.argtypes = [_vp, C.c_int64, _vp]
_lib.bs_velocity.argtypes = [_vp, _vp]
_lib.bs_velocity_terms.argtypes = [_vp] + [_vp] * 5
_lib.bs_energy.argtypes = [_vp, C.POINTER(C.c_double), _vp]
_lib.bs_vorticity_modes.argtypes = [_vp, _vp]
_lib.bs_geometry.argtypes = [_vp] + [_vp] * 5
_lib.bs_status.argtypes = [_vp]
_lib.bs_get_params.argtypes = [_vp, C.POINTER(BsParams)]
_lib.bs_set_profiling.argtypes = [_vp, C.c_int]
_lib.bs_stage_times.argtypes = [_vp, _vp, _vp, C.c_int]
_lib.bs_destroy.argtypes = [_vp]
_lib.bs_last_error.argtypes = [_vp]
_lib.bs_last_error.restype = C.c_char_p
_lib.bs_mlp_nparams.restype = C.c_int
_lib.bs_mlp_create.argtypes = [_vp, _vp, C.POINTER(_vp)]
_lib.bs_mlp_forward.argtypes = [_vp, C.c_int64, _vp, _vp]
_lib.bs_mlp_loss_grad.argtypes = [_vp, C.c_int64, _vp, _vp, _vp, _vp]
_lib.bs_mlp_adam_step.argtypes = [_vp, C.c_int64, _vp, _vp, C.c_float, C.c_float, C.c_float,
                                  C.c_float, _vp]
_lib.bs_mlp_get_params.argtypes = [_vp, _vp]
_lib.bs_mlp_set_fp32.argtypes = [_vp, C.c_int]
_lib.bs_mlp_destroy.argtypes = [_vp]
_lib.bs_ns_samples.argtypes = [C.c_int64, _vp, _vp, _vp, _vp, _vp]
_lib.bs_ns_error_bins.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int)]
_lib.bs_ns_error_table.argtypes = [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, C.c_int]
_lib.bs_ns_error_table_noalloc.argtypes = [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, C.c_int]
_lib.bs_set_mlp.argtypes = [_vp, _vp, _vp, C.c_int]
_lib.bs_ns_counts.argtypes = [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
_lib.bs_rk4_step.argtypes = [_vp, C.c_int64, C.POINTER(C.c_int64), _vp, _vp, C.c_double]
_lib.bs_step.argtypes = [_vp, C.c_int64, C.POINTER(C.c_int64), _vp, _vp, _vp]
_lib.bs_set_graph.argtypes = [_vp, C.c_int]
_lib.bs_graph_active.argtypes = [_vp]


def lib():
    return _lib


def _check(code, plan=None):
    if code != BS_OK:
        msg = _lib.bs_last_error(plan).decode()
        raise BsError(code, msg)


def make_params(L, a, tol, grid_n, delta=0.25, beta=0.0, alpha=0.0, rcut=0.0, sigma=0.0,
                w=0, Q=0, precision=BS_FP64, ns_mode=BS_NS_OFF, ns_eta=0.0,
                fft_mode=0, spline_order=4, local_frac=0.0) -> BsParams:
    p = BsParams()
    p.L, p.a, p.delta, p.tol = L, a, delta, tol
    p.beta, p.alpha, p.rcut = beta, alpha, rcut
    p.grid_n, p.sigma, p.w, p.Q = grid_n, sigma, w, Q
    p.spline_order = spline_order
    p.precision, p.ns_mode, p.ns_eta = precision, ns_mode, ns_eta
    p.fft_mode = fft_mode
    p.local_frac = local_frac
    return p


def resolve_params(p: BsParams) -> BsParams:
    """Host-only parameter derivation (no device needed)."""
    out = BsParams()
    _check(_lib.bs_resolve_params(C.byref(p), C.byref(out)))
    return out


def params_for(fs, precision=BS_FP64, **kw) -> BsParams:
    """Parameters of a workloads.FilamentSet (box, core, grid and tolerance)."""
    return make_params(L=fs.L, a=fs.a, delta=fs.delta, tol=fs.tol, grid_n=fs.grid_n,
                       precision=precision, **kw)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Plan:
    """One evaluation plan on the current HIP device and torch stream."""

    def __init__(self, params: BsParams, stream=None):
        import torch
        self._torch = torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = _vp()
        _check(_lib.bs_plan(C.byref(params), _vp(stream.cuda_stream), C.byref(h)))
        self._h = h
        self.N = 0
        self.nfil = 0

    def close(self):
        if getattr(self, "_h", None):
            _lib.bs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> BsParams:
        out = BsParams()
        _check(_lib.bs_get_params(self._h, C.byref(out)), self._h)
        return out

    def set_filaments(self, offsets, xyz, gamma):
        torch = self._torch
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        assert xyz.is_cuda and xyz.dtype == torch.float64 and xyz.is_contiguous()
        assert gamma.is_cuda and gamma.dtype == torch.float64 and gamma.is_contiguous()
        assert xyz.shape == (int(off[-1]), 3) and gamma.shape == (len(off) - 1,)
        self._off = off
        _check(_lib.bs_set_filaments(self._h, len(off) - 1,
                                     off.ctypes.data_as(C.POINTER(C.c_int64)),
                                     _ptr(xyz), _ptr(gamma)), self._h)
        self.N = int(off[-1])
        self.nfil = len(off) - 1

    def set_periods(self, periods):
        """Period vectors n [nfil][3] of infinite filaments (None: all closed)."""
        if periods is None:
            _check(_lib.bs_set_periods(self._h, 0, None), self._h)
            return
        per = np.ascontiguousarray(periods, dtype=np.int64)
        assert per.ndim == 2 and per.shape[1] == 3
        self._periods = per
        _check(_lib.bs_set_periods(self._h, len(per), per.ctypes.data_as(_vp)), self._h)

    def _out(self, out):
        if out is None:
            out = self._torch.empty((self.N, 3), dtype=self._torch.float64, device="cuda")
        return out

    def velocity(self, out=None):
        out = self._out(out)
        _check(_lib.bs_velocity(self._h, _ptr(out)), self._h)
        return out

    def velocity_terms(self):
        t = [self._out(None) for _ in range(5)]
        _check(_lib.bs_velocity_terms(self._h, *[_ptr(x) for x in t]), self._h)
        return dict(zip(["local", "short", "long", "self", "ns"], t))

    def energy(self, psi_out=None, want_psi=True):
        E = C.c_double(0.0)
        psi = self._out(psi_out) if (want_psi or psi_out is not None) else None
        _check(_lib.bs_energy(self._h, C.byref(E), _ptr(psi)), self._h)
        return E.value, psi

    def vorticity_modes(self):
        K = self.params().K
        W = 2 * K + 1
        out = self._torch.empty((K + 1, W, W, 3, 2), dtype=self._torch.float64, device="cuda")
        _check(_lib.bs_vorticity_modes(self._h, _ptr(out)), self._h)
        return out

    def geometry(self):
        torch = self._torch
        Nq = self.N * self.params().Q
        qp = torch.empty((Nq, 3), dtype=torch.float64, device="cuda")
        qc = torch.empty_like(qp)
        sd = self._out(None); sdd = self._out(None)
        ell = torch.empty((self.N,), dtype=torch.float64, device="cuda")
        _check(_lib.bs_geometry(self._h, *[_ptr(x) for x in (qp, qc, sd, sdd, ell)]), self._h)
        return dict(qpos=qp, qcharge=qc, sdot=sd, sddot=sdd, ell=ell)

    def status(self):
        _check(_lib.bs_status(self._h), self._h)

    def step(self, offsets, xyz, gamma, out):
        """set_filaments + velocity in one call (graph replay when enabled)."""
        if getattr(self, "_step_off", None) is None or len(self._step_off) != len(offsets) \
                or not np.array_equal(self._step_off, offsets):
            self._step_off = np.ascontiguousarray(offsets, dtype=np.int64)
        off = self._step_off
        _check(_lib.bs_step(self._h, len(off) - 1, off.ctypes.data_as(C.POINTER(C.c_int64)),
                            _ptr(xyz), _ptr(gamma), _ptr(out)), self._h)
        self.N = int(off[-1])
        self.nfil = len(off) - 1
        return out

    def set_graph(self, on: bool):
        _check(_lib.bs_set_graph(self._h, int(bool(on))), self._h)

    def graph_active(self) -> bool:
        return bool(_lib.bs_graph_active(self._h))

    def rk4_step(self, offsets, xyz, gamma, dt):
        """Advance device positions xyz in place by one RK4 step."""
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        _check(_lib.bs_rk4_step(self._h, len(off) - 1, off.ctypes.data_as(C.POINTER(C.c_int64)),
                                _ptr(xyz), _ptr(gamma), float(dt)), self._h)
        self.N = int(off[-1])
        self.nfil = len(off) - 1

    def set_mlp(self, mlp, err_table):
        tab = np.ascontiguousarray(err_table, dtype=np.float32)
        self._mlp = mlp          # keep the network alive while the plan uses it
        _check(_lib.bs_set_mlp(self._h, mlp._h, tab.ctypes.data_as(_vp), len(tab)), self._h)

    def ns_counts(self):
        a, b = C.c_int64(0), C.c_int64(0)
        _check(_lib.bs_ns_counts(self._h, C.byref(a), C.byref(b)), self._h)
        return a.value, b.value

    def set_profiling(self, on: bool):
        _check(_lib.bs_set_profiling(self._h, int(bool(on))), self._h)

    def stage_times(self, reset=False):
        ms = np.zeros(NSTAGES)
        cnt = np.zeros(NSTAGES, dtype=np.int64)
        _check(_lib.bs_stage_times(self._h, ms.ctypes.data_as(C.c_void_p),
                                   cnt.ctypes.data_as(C.c_void_p), int(reset)), self._h)
        return {name: (ms[i], int(cnt[i])) for i, name in enumerate(STAGES)}


def load_workload(fs, device="cuda"):
    """Device tensors (xyz, gamma) of a workloads.FilamentSet."""
    import torch
    xyz = torch.from_numpy(np.ascontiguousarray(fs.xyz)).to(device)
    gamma = torch.from_numpy(np.ascontiguousarray(fs.gamma)).to(device)
    return xyz, gamma


class MLP:
    """Device copy of the 8-64-64-64-3 network (BF16 MFMA kernels)."""

    def __init__(self, params, stream=None):
        import torch
        self._torch = torch
        self.nparams = _lib.bs_mlp_nparams()
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.shape == (self.nparams,)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = _vp()
        _check(_lib.bs_mlp_create(p.ctypes.data_as(_vp), _vp(stream.cuda_stream), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.bs_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _f32(t):
        assert t.is_cuda and t.dtype.is_floating_point
        return t.float().contiguous()

    def forward(self, X):
        torch = self._torch
        X = self._f32(X)
        Y = torch.empty((X.shape[0], 3), dtype=torch.float32, device="cuda")
        _check(_lib.bs_mlp_forward(self._h, X.shape[0], _ptr(X), _ptr(Y)))
        return Y

    def loss_grad(self, X, T):
        torch = self._torch
        X, T = self._f32(X), self._f32(T)
        loss = torch.empty((1,), dtype=torch.float32, device="cuda")
        grad = torch.empty((self.nparams,), dtype=torch.float32, device="cuda")
        _check(_lib.bs_mlp_loss_grad(self._h, X.shape[0], _ptr(X), _ptr(T), _ptr(loss),
                                     _ptr(grad)))
        return loss, grad

    def adam_step(self, X, T, lr, beta1=0.9, beta2=0.999, eps=1e-8, loss=None):
        _check(_lib.bs_mlp_adam_step(self._h, X.shape[0], _ptr(X), _ptr(T), lr, beta1, beta2,
                                     eps, _ptr(loss)))

    def set_fp32(self, on: bool):
        """Debug mode: FP32 weights and activations on FP32 MFMA."""
        _check(_lib.bs_mlp_set_fp32(self._h, int(bool(on))))

    def params(self):
        out = np.zeros(self.nparams, dtype=np.float32)
        _check(_lib.bs_mlp_get_params(self._h, out.ctypes.data_as(_vp)))
        return out


def bf16_round(a):
    """float32 -> nearest-even bfloat16, returned as float32 (host helper for
    comparing against the device's BF16 weights)."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def mlp_init(seed=0):
    """He-style initial parameters of the 8-64-64-64-3 network."""
    rng = np.random.default_rng(seed)
    dims = [8, 64, 64, 64, 3]
    parts = []
    for i in range(4):
        fan_in = dims[i]
        parts.append(rng.standard_normal((dims[i + 1], fan_in)).ravel() * np.sqrt(2.0 / fan_in))
        parts.append(np.zeros(dims[i + 1]))
    return np.concatenate(parts).astype(np.float32)


def ns_error_bins():
    lo, hi, nb = C.c_double(), C.c_double(), C.c_int()
    _check(_lib.bs_ns_error_bins(C.byref(lo), C.byref(hi), C.byref(nb)))
    return lo.value, hi.value, nb.value


def ns_error_table(mlp, X, T, A):
    """Per distance bin, rms and max error of the learned raw segment
    integral on samples (X, T, A) of ns_samples (computed by the library)."""
    _, _, nb = ns_error_bins()
    rms = np.zeros(nb, dtype=np.float32)
    mx = np.zeros(nb, dtype=np.float32)
    X, T = mlp._f32(X), mlp._f32(T)
    assert A.is_cuda and A.dtype == mlp._torch.float64 and A.is_contiguous()
    _check(_lib.bs_ns_error_table(mlp._h, X.shape[0], _ptr(X), _ptr(T), _ptr(A),
                                  rms.ctypes.data_as(_vp), mx.ctypes.data_as(_vp), nb))
    return rms, mx


def ns_error_table_noalloc(mlp, X, T, A, rms_out, max_out):
    """bs_ns_error_table_noalloc: the table into device float32 tensors
    rms_out and max_out (nbins each), asynchronously on the network's stream."""
    _, _, nb = ns_error_bins()
    X, T = mlp._f32(X), mlp._f32(T)
    torch = mlp._torch
    for t in (rms_out, max_out):
        assert t.is_cuda and t.dtype == torch.float32 and t.numel() == nb
    _check(_lib.bs_ns_error_table_noalloc(mlp._h, X.shape[0], _ptr(X), _ptr(T), _ptr(A),
                                          _ptr(rms_out), _ptr(max_out), nb))


def ns_samples(U, aux=True):
    """Features, targets (and aux) for uniforms U (device float64 [n][8])."""
    import torch
    assert U.is_cuda and U.dtype == torch.float64 and U.is_contiguous() and U.shape[1] == 8
    n = U.shape[0]
    X = torch.empty((n, 8), dtype=torch.float32, device="cuda")
    T = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    A = torch.empty((n, 7), dtype=torch.float64, device="cuda") if aux else None
    _check(_lib.bs_ns_samples(n, _ptr(U), _ptr(X), _ptr(T), _ptr(A),
                              _vp(torch.cuda.current_stream().cuda_stream)))
    return X, T, A
