"""ctypes binding of libmsr (argument marshalling only).

Names follow the C ABI in ``include/msr.h``.  Tensors must be float32 (or
float64 for a precision-64 solver),
contiguous and on the context's device; their ``data_ptr()`` and the current
stream's handle are passed through unchanged.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_NAME = "libmsr.so"

OK, ERR_INVALID, ERR_OOM, ERR_HIP, ERR_STATE, ERR_NUMERIC, ERR_UNSUPPORTED = range(7)
# MSR_STATIC_WORKSPACE_BYTES of include/msr.h: the static workspace of msr_set_workspace_static
STATIC_WORKSPACE_BYTES = 32 << 20
_STATUS = {0: "OK", 1: "INVALID", 2: "OOM", 3: "HIP", 4: "STATE", 5: "NUMERIC", 6: "UNSUPPORTED"}


class MsrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"msr error {_STATUS.get(status, status)}: {msg}")
        self.status = status


class Config(C.Structure):
    _fields_ = [
        ("n", C.c_int32),
        ("pad", C.c_int32),
        ("positivity", C.c_int32),
        ("device", C.c_int32),
        ("seed", C.c_uint64),
        ("prune_tol", C.c_double),
        ("precision", C.c_int32),
        ("dictionary", C.c_int32),
        ("iterate_precision", C.c_int32),
    ]


class SolveOptions(C.Structure):
    _fields_ = [
        ("lam", C.c_double),
        ("max_iters", C.c_int32),
        ("check_every", C.c_int32),
        ("tol", C.c_double),
        ("f_ref", C.c_double),
    ]


class Result(C.Structure):
    _fields_ = [
        ("iters", C.c_int32),
        ("converged", C.c_int32),
        ("objective", C.c_double),
        ("data_term", C.c_double),
        ("l1_norm", C.c_double),
        ("theta", C.c_double),
        ("elapsed_ms", C.c_double),
        ("time_to_tol_ms", C.c_double),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class UNetConfig(C.Structure):
    _fields_ = [("in_channels", C.c_int32), ("base_width", C.c_int32), ("levels", C.c_int32), ("device", C.c_int32)]


class Adam(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double)]


# exported symbol -> (restype, argtypes)
_P = C.c_void_p
_ST = C.c_int
SYMBOLS = {
    "msr_abi_version": (C.c_int, []),
    "msr_init": (_ST, [C.POINTER(Config), C.POINTER(_P)]),
    "msr_destroy": (None, [_P]),
    "msr_last_error": (C.c_char_p, [_P]),
    "msr_workspace_bytes": (C.c_size_t, [C.POINTER(Config)]),
    "msr_set_workspace": (_ST, [_P, _P, C.c_size_t]),
    "msr_set_workspace_static": (_ST, [_P]),
    "msr_set_dirty_psf": (_ST, [_P, C.c_int, _P, _P, _P]),
    "msr_set_filters": (_ST, [_P, C.c_double, C.c_double, C.c_double, C.c_double]),
    "msr_lipschitz": (_ST, [_P, C.c_int, C.c_int, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_int), _P]),
    "msr_set_lipschitz": (_ST, [_P, C.c_int, C.c_double]),
    "msr_step1_low_res": (_ST, [_P, C.POINTER(SolveOptions), _P, _P, _P, C.POINTER(Result), _P]),
    "msr_step2_full_res": (_ST, [_P, C.POINTER(SolveOptions), _P, _P, _P, _P, C.POINTER(Result), _P]),
    "msr_major_cycles": (_ST, [_P, C.c_int, C.c_int, C.c_double, C.c_int, _P, _P, _P, C.POINTER(Result), _P]),
    "msr_objective": (_ST, [_P, C.c_int, C.c_double, _P, _P, C.POINTER(C.c_double), _P]),
    "msr_gradient": (_ST, [_P, C.c_int, _P, _P, _P, _P]),
    "msr_apply_psf": (_ST, [_P, C.c_int, _P, _P, _P]),
    "msr_dictionary_synthesis": (_ST, [_P, _P, _P, _P]),
    "msr_upsample": (_ST, [_P, C.c_int, _P, _P, _P]),
    "msr_get_state": (_ST, [_P, C.c_int, _P, _P, C.POINTER(C.c_int), _P]),
    "msr_set_state": (_ST, [_P, C.c_int, _P, _P, C.c_int, _P]),
    "msr_dictionary_analysis": (_ST, [_P, _P, _P, _P]),
    "msr_get_spectrum": (_ST, [_P, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int), _P]),
    "msr_estimate_sigma2": (_ST, [_P, _P, C.POINTER(C.c_double), _P]),
    "msr_default_lambda": (_ST, [_P, C.c_int, C.c_int, C.c_double, C.POINTER(C.c_double), _P]),
    "msr_time_pass": (_ST, [_P, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double),
                            C.POINTER(C.c_double), _P]),
    "msr_autotune": (_ST, [_P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_double), _P]),
    "msr_set_variants": (_ST, [_P, C.c_int, C.c_int, C.c_int, C.c_int]),
    "msr_get_variants": (_ST, [_P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "msr_batch_workspace_bytes": (C.c_size_t, [C.c_int, C.POINTER(Config)]),
    "msr_batch_init": (_ST, [C.c_int, C.POINTER(Config), C.POINTER(_P)]),
    "msr_batch_destroy": (None, [_P]),
    "msr_batch_last_error": (C.c_char_p, [_P]),
    "msr_batch_channels": (C.c_int, [_P]),
    "msr_batch_channel": (_P, [_P, C.c_int]),
    "msr_batch_set_workspace": (_ST, [_P, _P, C.c_size_t]),
    "msr_batch_autotune": (_ST, [_P, C.c_int, _P]),
    "msr_batch_set_mode": (_ST, [_P, C.c_int, C.c_uint]),
    "msr_batch_give_up": (_ST, [_P, C.c_int, _P]),
    "msr_batch_solve": (_ST, [_P, C.c_int, C.POINTER(C.c_double), C.c_int, C.POINTER(_P), C.POINTER(_P),
                              C.POINTER(_P), C.POINTER(_P), C.POINTER(Result), _P]),
    "msr_unet_param_count": (C.c_size_t, [C.POINTER(UNetConfig)]),
    "msr_unet_workspace_bytes": (C.c_size_t, [C.POINTER(UNetConfig), C.c_int, C.c_int, C.c_int]),
    "msr_unet_init": (_ST, [C.POINTER(UNetConfig), C.POINTER(_P)]),
    "msr_unet_destroy": (None, [_P]),
    "msr_unet_last_error": (C.c_char_p, [_P]),
    "msr_unet_set_workspace": (_ST, [_P, _P, C.c_size_t, C.c_int, C.c_int, C.c_int]),
    "msr_unet_set_params": (_ST, [_P, _P, _P]),
    "msr_unet_get_params": (_ST, [_P, _P, _P]),
    "msr_unet_save": (_ST, [_P, C.c_char_p, _P]),
    "msr_unet_load": (_ST, [_P, C.c_char_p, _P]),
    "msr_unet_forward": (_ST, [_P, _P, _P, _P, C.c_int, _P]),
    "msr_unet_loss_grad": (_ST, [_P, _P, _P, _P, C.c_int, C.POINTER(C.c_double), _P, _P]),
    "msr_unet_train_step": (_ST, [_P, _P, _P, _P, C.c_int, C.POINTER(Adam), C.POINTER(C.c_double), _P]),
}

_lib = None


def library_path() -> str:
    return os.environ.get("MSR_LIBRARY", os.path.join(HERE, _LIB_NAME))


def lib() -> C.CDLL:
    """Loads libmsr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        path = library_path()
        if not os.path.exists(path):
            raise ImportError(f"{path} not found: build it with `python -m paper_2406_18356_amd.build`")
        L = C.CDLL(path)
        for name, (res, args) in SYMBOLS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def abi_version() -> int:
    return lib().msr_abi_version()


def _cfg(n, pad=2, positivity=False, device=0, seed=0, prune_tol=1e-6, precision=32, dictionary=0,
         iterate_precision=0) -> Config:
    return Config(int(n), int(pad), int(bool(positivity)), int(device), int(seed), float(prune_tol),
                  int(precision), int(dictionary), int(iterate_precision))


def workspace_bytes(n, pad=2, positivity=False, seed=0, prune_tol=1e-6, precision=32, dictionary=0,
                    iterate_precision=0) -> int:
    c = _cfg(n, pad, positivity, 0, seed, prune_tol, precision, dictionary, iterate_precision)
    return int(lib().msr_workspace_bytes(C.byref(c)))


def _ptr(t, dtype=None) -> Optional[int]:
    if t is None:
        return None
    if (dtype is not None and t.dtype != dtype) or not t.is_contiguous() or not t.is_cuda:
        raise ValueError(f"tensors must be contiguous {dtype} on the GPU (got {t.dtype}, device {t.device})")
    return t.data_ptr()


def _stream(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Solver:
    """One libmsr context with a torch-owned workspace.

    >>> s = Solver(n=256, positivity=True)
    >>> s.set_dirty_psf(1, dirty_L, psf_L); s.set_dirty_psf(2, dirty_H, psf_H)
    >>> beta1, i_L, r1 = s.step1(lam1, iters=200, image=True)
    >>> s.set_filters(ell, delta, sigma2, eta2)
    >>> beta2, r2 = s.step2(lam2, i_L, iters=200)

    ``static_workspace=True`` takes the library's static device array
    (msr_set_workspace_static: no allocation, images up to 512^2 in float32)
    instead of a torch-allocated workspace.
    """

    def __init__(self, n: int, pad: int = 2, positivity: bool = False, device: int = 0, seed: int = 0,
                 prune_tol: float = 1e-6, precision: int = 32, dictionary: int = 0, static_workspace: bool = False,
                 iterate_precision: int = 0, _borrowed=None):
        import torch

        self._lib = lib()
        self._owned = _borrowed is None
        if _borrowed is not None:  # a channel context owned by a Batch
            self.n, self.P, self.precision = n, pad * n, precision
            self.dtype = torch.float32 if precision == 32 else torch.float64
            self.device = torch.device("cuda", device)
            self._h = C.c_void_p(_borrowed)
            return
        self.n = n
        self.P = pad * n
        self.precision = precision
        self.dtype = torch.float32 if precision == 32 else torch.float64
        self.device = torch.device("cuda", device)
        self.dictionary = int(dictionary)
        # float64 iterates with float32 transforms: the state images are float64
        self.state_dtype = torch.float64 if (iterate_precision == 64 or precision == 64) else self.dtype
        cfg = _cfg(n, pad, positivity, device, seed, prune_tol, precision, dictionary, iterate_precision)
        h = C.c_void_p()
        st = self._lib.msr_init(C.byref(cfg), C.byref(h))
        if st != OK:
            raise MsrError(st, "msr_init rejected the configuration")
        self._h = h
        nbytes = int(self._lib.msr_workspace_bytes(C.byref(cfg)))
        self.workspace_bytes = nbytes
        if static_workspace:
            # the library's static array on this device (msr_set_workspace_static)
            self._ws = None
            self._check(self._lib.msr_set_workspace_static(self._h))
            return
        # 256-byte aligned workspace owned by torch
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._check(self._lib.msr_set_workspace(self._h, C.c_void_p(aligned), nbytes))

    def __del__(self):
        h = getattr(self, "_h", None)
        if getattr(self, "_owned", False) and h is not None and h.value:
            self._lib.msr_destroy(h)
            self._h = None

    def _check(self, st):
        if st != OK:
            msg = self._lib.msr_last_error(self._h)
            raise MsrError(st, msg.decode() if msg else "")

    def _img(self):
        import torch

        return torch.empty((self.n, self.n), dtype=self.dtype, device=self.device)

    def _p(self, t):
        return _ptr(t, self.dtype)

    # -- setup ------------------------------------------------------------------
    def set_dirty_psf(self, step: int, dirty, psf, stream=None):
        self._check(self._lib.msr_set_dirty_psf(self._h, step, self._p(dirty), self._p(psf), _stream(stream)))

    def set_filters(self, ell, delta, sigma2, eta2):
        self._check(self._lib.msr_set_filters(self._h, float(ell), float(delta), float(sigma2), float(eta2)))

    def lipschitz(self, step: int, max_iter: int = 200, rtol: float = 1e-6, stream=None):
        th = C.c_double()
        it = C.c_int()
        self._check(self._lib.msr_lipschitz(self._h, step, max_iter, rtol, C.byref(th), C.byref(it), _stream(stream)))
        return th.value, it.value

    def set_lipschitz(self, step: int, theta: float):
        self._check(self._lib.msr_set_lipschitz(self._h, step, float(theta)))

    # -- solves -----------------------------------------------------------------
    def step1(self, lam, iters, x0=None, image=False, check_every=0, tol=0.0, f_ref=0.0, out=None, stream=None):
        opt = SolveOptions(float(lam), int(iters), int(check_every), float(tol), float(f_ref))
        res = Result()
        beta = out if out is not None else self._img()
        img = self._img() if image else None
        self._check(self._lib.msr_step1_low_res(self._h, C.byref(opt), self._p(x0), self._p(beta), self._p(img),
                                                C.byref(res), _stream(stream)))
        return (beta, img, res) if image else (beta, res)

    def step2(self, lam, low_res, iters, x0=None, check_every=0, tol=0.0, f_ref=0.0, out=None, stream=None,
              image=False):
        """(beta_K, res), or (beta_K, image, res) with image = beta_K + (i_H~ - H_H beta_K)."""
        opt = SolveOptions(float(lam), int(iters), int(check_every), float(tol), float(f_ref))
        res = Result()
        beta = out if out is not None else self._img()
        img = self._img() if image else None
        self._check(self._lib.msr_step2_full_res(self._h, C.byref(opt), self._p(low_res), self._p(x0), self._p(beta),
                                                 self._p(img), C.byref(res), _stream(stream)))
        return (beta, img, res) if image else (beta, res)

    def major_cycles(self, step, cycles, iters, c=0.05, low_res=None, stream=None):
        """(image, sum of the cycle images, per-cycle results) of `cycles`
        major cycles of `step` (msr_major_cycles)."""
        img, model = self._img(), self._img()
        res = (Result * int(cycles))()
        self._check(self._lib.msr_major_cycles(self._h, int(step), int(cycles), float(c), int(iters),
                                               self._p(low_res), self._p(model), self._p(img), res,
                                               _stream(stream)))
        return img, model, [res[k] for k in range(int(cycles))]

    # -- single operators ------------------------------------------------------
    def objective(self, step, lam, x, low_res=None, stream=None):
        out = (C.c_double * 3)()
        self._check(self._lib.msr_objective(self._h, step, float(lam), self._p(x), self._p(low_res), out, _stream(stream)))
        return tuple(out)

    def gradient(self, step, x, low_res=None, stream=None):
        g = self._img()
        self._check(self._lib.msr_gradient(self._h, step, self._p(x), self._p(low_res), self._p(g), _stream(stream)))
        return g

    def apply_psf(self, step, x, stream=None):
        y = self._img()
        self._check(self._lib.msr_apply_psf(self._h, step, self._p(x), self._p(y), _stream(stream)))
        return y

    def _state_shape(self):
        return (8, self.n, self.n) if getattr(self, "dictionary", 0) else (self.n, self.n)

    def get_state(self, step, stream=None):
        """(beta_K, beta_{K-1}, K) of the latest solve of `step` (msr_get_state)."""
        import torch

        bk = torch.empty(self._state_shape(), dtype=getattr(self, "state_dtype", self.dtype), device=self.device)
        bp = torch.empty_like(bk)
        k = C.c_int()
        sd = getattr(self, "state_dtype", self.dtype)
        self._check(self._lib.msr_get_state(self._h, int(step), _ptr(bk, sd), _ptr(bp, sd), C.byref(k),
                                            _stream(stream)))
        return bk, bp, k.value

    def set_state(self, step, beta_k, beta_km1, k, stream=None):
        """Loads a state: the next solve of `step` continues from iteration k + 1."""
        sd = getattr(self, "state_dtype", self.dtype)
        self._check(self._lib.msr_set_state(self._h, int(step), _ptr(beta_k, sd), _ptr(beta_km1, sd), int(k),
                                            _stream(stream)))

    def upsample(self, small, factor, stream=None):
        """U small: an (n/factor)^2 low-resolution image up-sampled to n x n
        (msr_upsample), the step-2 low_res for a down-sampled step 1."""
        x = self._img()
        self._check(self._lib.msr_upsample(self._h, int(factor), self._p(small), self._p(x), _stream(stream)))
        return x

    def synthesis(self, coeffs, stream=None):
        """W alpha: (8, n, n) coefficients -> n x n image (dictionary 1)."""
        x = self._img()
        self._check(self._lib.msr_dictionary_synthesis(self._h, self._p(coeffs), self._p(x), _stream(stream)))
        return x

    def analysis(self, x, stream=None):
        """W^T x: n x n image -> (8, n, n) coefficients (dictionary 1)."""
        import torch

        a = torch.empty((8, self.n, self.n), dtype=self.dtype, device=self.device)
        self._check(self._lib.msr_dictionary_analysis(self._h, self._p(x), self._p(a), _stream(stream)))
        return a

    def spectrum(self, step, stream=None):
        import numpy as np

        out = np.zeros((self.P, self.P // 2 + 1), dtype=np.float64)
        kept = C.c_int()
        self._check(self._lib.msr_get_spectrum(self._h, step, out.ctypes.data_as(C.POINTER(C.c_double)),
                                               C.byref(kept), _stream(stream)))
        return out, kept.value

    def estimate_sigma2(self, dirty, stream=None):
        v = C.c_double()
        self._check(self._lib.msr_estimate_sigma2(self._h, self._p(dirty), C.byref(v), _stream(stream)))
        return v.value

    def default_lambda(self, step, cycle=1, c=0.05, stream=None):
        v = C.c_double()
        self._check(self._lib.msr_default_lambda(self._h, step, cycle, float(c), C.byref(v), _stream(stream)))
        return v.value

    def autotune(self, reps=10, stream=None):
        """Returns (row variant, column variant, {variant: (column ms, row ms)})."""
        vr = C.c_int()
        vc = C.c_int()
        t = (C.c_double * 8)()
        self._check(self._lib.msr_autotune(self._h, reps, C.byref(vr), C.byref(vc), t, _stream(stream)))
        times = {v: (t[2 * v], t[2 * v + 1]) for v in range(4) if t[2 * v] >= 0}
        return vr.value, vc.value, times

    def set_variants(self, step, row, col, filt=-1):
        """Selects the kernel variants of a step's passes (msr_set_variants)."""
        self._check(self._lib.msr_set_variants(self._h, int(step), int(row), int(col), int(filt)))

    def get_variants(self, step):
        """(row, column, filter) variants of a step's passes (msr_get_variants)."""
        r, c_, f = C.c_int(), C.c_int(), C.c_int()
        self._check(self._lib.msr_get_variants(self._h, int(step), C.byref(r), C.byref(c_), C.byref(f)))
        return r.value, c_.value, f.value

    def time_pass(self, which, reps=20, step=1, stream=None):
        """(mean ms, algorithmic bytes, algorithmic flops) of one pass launch."""
        ms = C.c_double()
        by = C.c_double()
        fl = C.c_double()
        self._check(self._lib.msr_time_pass(self._h, step, which, reps, C.byref(ms), C.byref(by), C.byref(fl),
                                            _stream(stream)))
        return ms.value, by.value, fl.value


class Batch:
    """Many channels (independent two-step problems, possibly of different
    sizes) solved together: ``msr_batch_*`` of the C ABI.

    >>> b = Batch([2048, 1024, 1024, 512], positivity=True)
    >>> for c, ch in enumerate(b.channels): ch.set_dirty_psf(1, dirty[c], psf[c])
    >>> models, results = b.solve(1, lambdas, iters=500)
    """

    def __init__(self, sizes, pad: int = 2, positivity: bool = False, device: int = 0, seed: int = 0,
                 prune_tol: float = 1e-6, precision: int = 32):
        import torch

        self._lib = lib()
        self.sizes = [int(n) for n in sizes]
        self.precision = precision
        self.dtype = torch.float32 if precision == 32 else torch.float64
        self.device = torch.device("cuda", device)
        cfgs = (Config * len(self.sizes))(*[_cfg(n, pad, positivity, device, seed, prune_tol, precision)
                                            for n in self.sizes])
        h = C.c_void_p()
        st = self._lib.msr_batch_init(len(self.sizes), cfgs, C.byref(h))
        if st != OK:
            raise MsrError(st, "msr_batch_init rejected the configurations")
        self._h = h
        nbytes = int(self._lib.msr_batch_workspace_bytes(len(self.sizes), cfgs))
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        aligned = (self._ws.data_ptr() + 255) // 256 * 256
        self._check(self._lib.msr_batch_set_workspace(self._h, C.c_void_p(aligned), nbytes))
        self.workspace_bytes = nbytes
        self.channels = [Solver(n, pad, positivity, device, seed, prune_tol, precision,
                                _borrowed=self._lib.msr_batch_channel(self._h, c))
                         for c, n in enumerate(self.sizes)]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.channels = []
            self._lib.msr_batch_destroy(h)
            self._h = None

    def _check(self, st):
        if st != OK:
            msg = self._lib.msr_batch_last_error(self._h)
            raise MsrError(st, msg.decode() if msg else "")

    def autotune(self, reps=10, stream=None):
        self._check(self._lib.msr_batch_autotune(self._h, int(reps), _stream(stream)))

    def set_mode(self, mode, spin_limit=0):
        """0: launches per pass, grouped by size; 1: one persistent launch for
        every channel and iteration (msr_batch_set_mode)."""
        self._check(self._lib.msr_batch_set_mode(self._h, int(mode), int(spin_limit)))

    def give_up(self, raise_flag=True, stream=None):
        """Raises or clears the host's give-up flag of the persistent launch."""
        self._check(self._lib.msr_batch_give_up(self._h, 1 if raise_flag else 0, _stream(stream)))

    def solve(self, step, lambdas, iters, low_res=None, x0=None, out=None, image=False, stream=None):
        """Runs `iters` iterations of `step` on every channel; returns (models,
        results), or (models, low-resolution images, results) with image=True (step 1)."""
        import torch

        C_ = len(self.sizes)
        lam = (C.c_double * C_)(*[float(v) for v in lambdas])
        outs = out if out is not None else [torch.empty((n, n), dtype=self.dtype, device=self.device)
                                            for n in self.sizes]

        def arr(ts):
            if ts is None:
                return None
            return (_P * C_)(*[_ptr(t, self.dtype) for t in ts])

        imgs = [torch.empty_like(o) for o in outs] if image else None
        res = (Result * C_)()
        self._check(self._lib.msr_batch_solve(self._h, int(step), lam, int(iters), arr(low_res), arr(x0),
                                              arr(outs), arr(imgs), res, _stream(stream)))
        if image:
            return outs, imgs, [res[c] for c in range(C_)]
        return outs, [res[c] for c in range(C_)]


def unet_layers(base_width=32, levels=4, cin0=8):
    """(cin, cout, kpad) of the 3x3 convolutions in parameter order, as
    include/msr_unet.h lays them out."""
    out, prev = [], cin0
    for j in range(levels):
        w = base_width << j
        out += [(prev, w), (w, w)]
        prev = w
    for j in range(levels - 2, -1, -1):
        w = base_width << j
        out += [(prev + w, w), (w, w)]
        prev = w
    return [(ci, co, (9 * ci + 31) // 32 * 32) for ci, co in out]


def unet_init_params(base_width=32, levels=4, in_channels=2, seed=0):
    """He-normal weights (fan-in of the real input channels), zero biases, as
    a float32 numpy vector in the library's layout."""
    import numpy as np

    rng = np.random.default_rng(seed)
    parts = []
    for i, (ci, co, kpad) in enumerate(unet_layers(base_width, levels)):
        real = in_channels if i == 0 else ci
        w = np.zeros((co, kpad), np.float32)
        blk = rng.normal(0.0, np.sqrt(2.0 / (9 * real)), size=(co, 9, ci)).astype(np.float32)
        if i == 0:
            blk[:, :, real:] = 0.0
        w[:, : 9 * ci] = blk.reshape(co, 9 * ci)
        parts += [w.ravel(), np.zeros(co, np.float32)]
    parts += [rng.normal(0.0, np.sqrt(1.0 / base_width), size=base_width).astype(np.float32),
              np.zeros(1, np.float32)]
    return np.concatenate(parts)


class UNet:
    """The learned warm start (include/msr_unet.h) with a torch-owned workspace
    sized for batches of up to `batch` images of height x width."""

    def __init__(self, batch, height, width=None, base_width=32, levels=4, in_channels=2, device=0):
        import torch

        self._lib = lib()
        width = height if width is None else width
        self.cfg = UNetConfig(in_channels, base_width, levels, device)
        self.batch, self.height, self.width = batch, height, width
        self.device = torch.device("cuda", device)
        self.nparam = int(self._lib.msr_unet_param_count(C.byref(self.cfg)))
        h = C.c_void_p()
        st = self._lib.msr_unet_init(C.byref(self.cfg), C.byref(h))
        if st != OK:
            raise MsrError(st, "msr_unet_init rejected the configuration")
        self._h = h
        nbytes = int(self._lib.msr_unet_workspace_bytes(C.byref(self.cfg), batch, height, width))
        if nbytes == 0:
            self._lib.msr_unet_destroy(h)
            self._h = None
            raise MsrError(ERR_INVALID, f"no workspace for batch {batch} of {height}x{width}")
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        aligned = (self._ws.data_ptr() + 255) // 256 * 256
        self._check(self._lib.msr_unet_set_workspace(self._h, C.c_void_p(aligned), nbytes, batch, height, width))
        self.workspace_bytes = nbytes

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.msr_unet_destroy(h)
            self._h = None

    def _check(self, st):
        if st != OK:
            msg = self._lib.msr_unet_last_error(self._h)
            raise MsrError(st, msg.decode() if msg else "")

    def _p(self, t):
        return _ptr(t, __import__("torch").float32)

    def set_params(self, params, stream=None):
        import torch

        t = params if isinstance(params, torch.Tensor) else torch.from_numpy(params)
        t = t.to(self.device, torch.float32).contiguous()
        if t.numel() != self.nparam:
            raise ValueError(f"expected {self.nparam} parameters, got {t.numel()}")
        self._check(self._lib.msr_unet_set_params(self._h, self._p(t), _stream(stream)))

    def get_params(self, stream=None):
        import torch

        out = torch.empty(self.nparam, dtype=torch.float32, device=self.device)
        self._check(self._lib.msr_unet_get_params(self._h, self._p(out), _stream(stream)))
        return out

    def save(self, path, stream=None):
        """Writes a training checkpoint (msr_unet_save)."""
        self._check(self._lib.msr_unet_save(self._h, str(path).encode(), _stream(stream)))

    def load(self, path, stream=None):
        """Reads a training checkpoint of the same configuration (msr_unet_load)."""
        self._check(self._lib.msr_unet_load(self._h, str(path).encode(), _stream(stream)))

    def forward(self, dirty_h, low_res, out=None, stream=None):
        import torch

        b = dirty_h.shape[0] if dirty_h.dim() == 3 else 1
        x0 = out if out is not None else torch.empty_like(dirty_h)
        self._check(self._lib.msr_unet_forward(self._h, self._p(dirty_h), self._p(low_res), self._p(x0), b,
                                               _stream(stream)))
        return x0

    def loss_grad(self, dirty_h, low_res, target, stream=None):
        import torch

        b = dirty_h.shape[0] if dirty_h.dim() == 3 else 1
        g = torch.empty(self.nparam, dtype=torch.float32, device=self.device)
        loss = C.c_double()
        self._check(self._lib.msr_unet_loss_grad(self._h, self._p(dirty_h), self._p(low_res), self._p(target), b,
                                                 C.byref(loss), self._p(g), _stream(stream)))
        return loss.value, g

    def train_step(self, dirty_h, low_res, target, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        b = dirty_h.shape[0] if dirty_h.dim() == 3 else 1
        opt = Adam(lr, beta1, beta2, eps)
        loss = C.c_double()
        self._check(self._lib.msr_unet_train_step(self._h, self._p(dirty_h), self._p(low_res), self._p(target), b,
                                                  C.byref(opt), C.byref(loss), _stream(stream)))
        return loss.value
