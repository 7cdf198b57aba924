"""FP64 oracle for separable non-local means -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it, and the
two share no code.

The arithmetic lives in ``snlm_oracle.c`` (plain C, double precision, direct
patch sums, ``exp`` from libm).  This module only compiles that file with gcc
and marshals NumPy arrays into it.

What it computes (Ghosh & Chaudhury, "Fast Separable Non-Local Means"):

* ``nlm1d``    -- 1D NLM of eq. 1dNLM with patch distances of eq.
  distanceSquared, computed directly, on the line extended by half-sample
  symmetric reflection.
* ``snlm``     -- the separable RC / CR pipelines of Sec. 3.
* ``pixel``    -- one output pixel of ``snlm``, for sampled checks of large images.
* ``patch_d2`` -- one patch distance (eq. distanceSquared).
* ``nlm1d_div`` -- 1D NLM with its divergence (Sec. 3.1, eq. div, by the
  quotient rule of the Appendix).
* ``sure``     -- the SURE-optimal combination of the two orders (Alg. 4).
* ``snlm3d``   -- the separable NLM of a volume along three axes in turn.
* kernel ``"gauss_iir"`` -- the Gaussian patch kernel by the recursive filter
  of Young & van Vliet (Sec. 2.2's pointer), untruncated; ``yvv`` exposes the
  filter itself.
* ``bilateral``, ``bf_params``, ``full`` -- the bilateral post-processing of
  eq. BF with its parameter rules, and the whole SNLM[f] (Sec. 3.2, 4.1).

Pins (tests that tie it to something other than itself) live in
``tests/test_oracle_pins.py``: hand-derived closed forms, the PatchLift
identity computed a different way (Sec. 2.1-2.2, Alg. 1, eqs. lift and dist),
and invariants; ``tests/test_oracle_mutants.py`` checks that planted mistakes
in this file's C source fail those pins.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "snlm_oracle.c")
_LIB = os.path.join(_HERE, "libsnlm_oracle.so")

BOX, GAUSS, GAUSS_IIR = 0, 1, 2
ROW_COL, COL_ROW = 0, 1
_KERNELS = {"box": BOX, "gauss": GAUSS, "gauss_iir": GAUSS_IIR, BOX: BOX, GAUSS: GAUSS,
            GAUSS_IIR: GAUSS_IIR}
_ORDERS = {"row_col": ROW_COL, "col_row": COL_ROW, ROW_COL: ROW_COL, COL_ROW: COL_ROW}


def build(force: bool = False, src: str = SOURCE, out: str = _LIB) -> str:
    """Compile the C oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
               "-shared", "-fPIC", "-o", tmp, src, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _beta(kernel: int, K: int, beta) -> float:
    # Gaussian width: beta = K/2 unless given (the patch kernel of Sec. 2).
    if beta is None or beta <= 0:
        return K / 2.0
    return float(beta)


class Oracle:
    """The compiled oracle behind a small NumPy interface."""

    def __init__(self, libpath: str):
        lib = ctypes.CDLL(libpath)
        dp = ctypes.POINTER(ctypes.c_double)
        L, I, D = ctypes.c_long, ctypes.c_int, ctypes.c_double
        lib.snlm_oracle_nlm1d.argtypes = [dp, L, L, I, I, D, I, D, dp, L]
        lib.snlm_oracle_nlm1d.restype = I
        lib.snlm_oracle_snlm.argtypes = [dp, L, L, L, I, I, D, I, D, I, dp, I]
        lib.snlm_oracle_snlm.restype = I
        lib.snlm_oracle_pixel.argtypes = [dp, L, L, L, I, I, D, I, D, I, L, L]
        lib.snlm_oracle_pixel.restype = D
        lib.snlm_oracle_patch_d2.argtypes = [dp, L, L, L, I, I, D]
        lib.snlm_oracle_patch_d2.restype = D
        lib.snlm_oracle_nlm1d_div.argtypes = [dp, L, L, I, I, D, I, D, dp, L, dp, L, dp, L]
        lib.snlm_oracle_nlm1d_div.restype = I
        lib.snlm_oracle_sure.argtypes = [dp, L, L, L, I, I, D, I, D, D, dp, dp, dp, dp, dp, dp, dp, I]
        lib.snlm_oracle_sure.restype = I
        lib.snlm_oracle_bilateral.argtypes = [dp, L, L, L, D, D, dp, I]
        lib.snlm_oracle_bilateral.restype = I
        lib.snlm_oracle_bf_params.argtypes = [D, dp, dp]
        lib.snlm_oracle_bf_params.restype = None
        lib.snlm_oracle_snlm3d.argtypes = [dp, L, L, L, I, I, D, I, D, ctypes.POINTER(I), dp, I]
        lib.snlm_oracle_snlm3d.restype = I
        lib.snlm_oracle_yvv.argtypes = [dp, L, D, dp]
        lib.snlm_oracle_yvv.restype = None
        lib.snlm_oracle_iir_d2.argtypes = [dp, L, I, D, dp]
        lib.snlm_oracle_iir_d2.restype = I
        lib.snlm_oracle_max_threads.argtypes = []
        lib.snlm_oracle_max_threads.restype = I
        self._lib = lib
        self.path = libpath

    def nlm1d(self, x, S: int, K: int, h: float, kernel="box", beta=None) -> np.ndarray:
        """1D NLM (eq. 1dNLM) of a line, in float64."""
        k = _KERNELS[kernel]
        xa = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        y = np.empty_like(xa)
        rc = self._lib.snlm_oracle_nlm1d(_ptr(xa), xa.size, 1, S, K, float(h), k,
                                         _beta(k, K, beta), _ptr(y), 1)
        if rc != 0:
            raise ValueError("oracle rejected the arguments")
        return y

    def snlm(self, f, S: int, K: int, h: float, kernel="box", order="row_col", beta=None,
             threads: int = 0) -> np.ndarray:
        """Separable NLM (Sec. 3, RC or CR) of a 2D image, in float64."""
        k = _KERNELS[kernel]
        fa = np.ascontiguousarray(np.asarray(f, dtype=np.float64))
        if fa.ndim != 2:
            raise ValueError("expected a 2D image")
        H, W = fa.shape
        out = np.empty_like(fa)
        nt = threads if threads > 0 else self.max_threads()
        rc = self._lib.snlm_oracle_snlm(_ptr(fa), H, W, W, S, K, float(h), k,
                                        _beta(k, K, beta), _ORDERS[order], _ptr(out), nt)
        if rc != 0:
            raise ValueError("oracle rejected the arguments")
        return out

    def pixel(self, f, r: int, c: int, S: int, K: int, h: float, kernel="box",
              order="row_col", beta=None) -> float:
        """One output pixel of ``snlm`` computed from the input alone."""
        k = _KERNELS[kernel]
        fa = np.ascontiguousarray(np.asarray(f, dtype=np.float64))
        H, W = fa.shape
        v = self._lib.snlm_oracle_pixel(_ptr(fa), H, W, W, S, K, float(h), k,
                                        _beta(k, K, beta), _ORDERS[order], int(r), int(c))
        if np.isnan(v):
            raise ValueError("oracle rejected the arguments")
        return float(v)

    def patch_d2(self, x, i: int, j: int, K: int, kernel="box", beta=None) -> float:
        """Patch distance of eq. distanceSquared on the reflected extension of ``x``."""
        k = _KERNELS[kernel]
        xa = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        return float(self._lib.snlm_oracle_patch_d2(_ptr(xa), xa.size, int(i), int(j), K, k,
                                                    _beta(k, K, beta)))

    def nlm1d_div(self, x, S: int, K: int, h: float, kernel="box", beta=None, din=None):
        """1D NLM of a line and its divergence dy(i)/dx(i) times din(i) (Alg. 3,
        eq. div), in float64.  Returns (y, dout)."""
        k = _KERNELS[kernel]
        xa = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        y = np.empty_like(xa)
        d = np.empty_like(xa)
        if din is not None:
            da = np.ascontiguousarray(np.asarray(din, dtype=np.float64))
            dptr = _ptr(da)
        else:
            dptr = ctypes.POINTER(ctypes.c_double)()
        rc = self._lib.snlm_oracle_nlm1d_div(_ptr(xa), xa.size, 1, S, K, float(h), k,
                                             _beta(k, K, beta), dptr, 1, _ptr(y), 1, _ptr(d), 1)
        if rc != 0:
            raise ValueError("oracle rejected the arguments")
        return y, d

    def sure(self, f, S: int, K: int, h: float, sigma: float, kernel="box", beta=None,
             threads: int = 0) -> dict:
        """SNLM with the SURE-optimal combination of the RC and CR orders
        (Alg. 4), in float64.  Returns a dict with f_rc, f_cr, d_rc, d_cr, out,
        theta (2,) and stats (7,)."""
        k = _KERNELS[kernel]
        fa = np.ascontiguousarray(np.asarray(f, dtype=np.float64))
        if fa.ndim != 2:
            raise ValueError("expected a 2D image")
        H, W = fa.shape
        res = {n: np.empty_like(fa) for n in ("f_rc", "f_cr", "d_rc", "d_cr", "out")}
        theta = np.empty(2)
        stats = np.empty(7)
        nt = threads if threads > 0 else self.max_threads()
        rc = self._lib.snlm_oracle_sure(_ptr(fa), H, W, W, S, K, float(h), k, _beta(k, K, beta),
                                        float(sigma), _ptr(res["f_rc"]), _ptr(res["f_cr"]),
                                        _ptr(res["d_rc"]), _ptr(res["d_cr"]), _ptr(res["out"]),
                                        _ptr(theta), _ptr(stats), nt)
        if rc != 0:
            raise ValueError("oracle rejected the arguments")
        res["theta"] = theta
        res["stats"] = stats
        return res

    def snlm3d(self, f, S: int, K: int, h: float, kernel="box", axes="xyz", beta=None,
               threads: int = 0) -> np.ndarray:
        """Separable NLM of a D x H x W volume along the given axes in order
        (x is the last, contiguous axis), in float64."""
        k = _KERNELS[kernel]
        fa = np.ascontiguousarray(np.asarray(f, dtype=np.float64))
        if fa.ndim != 3:
            raise ValueError("expected a 3D volume")
        D, H, W = fa.shape
        out = np.empty_like(fa)
        ax = (ctypes.c_int * 3)(*["xyz".index(a) for a in axes])
        nt = threads if threads > 0 else self.max_threads()
        rc = self._lib.snlm_oracle_snlm3d(_ptr(fa), D, H, W, S, K, float(h), k, _beta(k, K, beta), ax,
                                          _ptr(out), nt)
        if rc != 0:
            raise ValueError("oracle rejected the arguments")
        return out

    def yvv(self, seq, beta: float) -> np.ndarray:
        """The recursive Gaussian (Young & van Vliet) of a finite sequence, with
        the oracle's steady-state starts; gain 1 (no sqrt(2 pi) beta scale)."""
        a = np.ascontiguousarray(np.asarray(seq, dtype=np.float64))
        out = np.empty_like(a)
        self._lib.snlm_oracle_yvv(_ptr(a), a.size, float(beta), _ptr(out))
        return out

    def iir_d2(self, x, S: int, beta: float) -> np.ndarray:
        """Recursive-Gaussian patch distances of a line: out[s - 1, u + S] is
        the distance between the patches at u and u + s, u in [-S, n)."""
        a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        out = np.empty((S, a.size + S))
        if self._lib.snlm_oracle_iir_d2(_ptr(a), a.size, S, float(beta), _ptr(out)) != 0:
            raise ValueError("bad arguments")
        return out

    def bilateral(self, f, sigma_s: float, sigma_r: float, threads: int = 0) -> np.ndarray:
        """Bilateral filter of eq. BF (Sec. 3.2), in float64."""
        fa = np.ascontiguousarray(np.asarray(f, dtype=np.float64))
        H, W = fa.shape
        out = np.empty_like(fa)
        nt = threads if threads > 0 else self.max_threads()
        rc = self._lib.snlm_oracle_bilateral(_ptr(fa), H, W, W, float(sigma_s), float(sigma_r),
                                             _ptr(out), nt)
        if rc != 0:
            raise ValueError("oracle rejected the arguments")
        return out

    def bf_params(self, sigma: float):
        """(sigma_s, sigma_r) of the bilateral parameter rules (Sec. 4.1)."""
        a, b = ctypes.c_double(), ctypes.c_double()
        self._lib.snlm_oracle_bf_params(float(sigma), ctypes.byref(a), ctypes.byref(b))
        return a.value, b.value

    def full(self, f, S: int, K: int, h: float, sigma: float, kernel="box", beta=None) -> dict:
        """SNLM[f]: the SURE combination followed by the bilateral filter with
        the parameter rules (Sec. 3.2, Sec. 4.1)."""
        r = self.sure(f, S, K, h, sigma, kernel, beta)
        ss, sr = self.bf_params(sigma)
        r["snlm"] = self.bilateral(r["out"], ss, sr)
        r["sigma_s"], r["sigma_r"] = ss, sr
        return r

    def max_threads(self) -> int:
        """Threads an OpenMP region of the oracle uses by default."""
        return int(self._lib.snlm_oracle_max_threads())


_default = None


def load(libpath: str | None = None) -> Oracle:
    """The oracle built from ``snlm_oracle.c`` (or a given compiled copy)."""
    global _default
    if libpath is not None:
        return Oracle(libpath)
    if _default is None:
        _default = Oracle(build())
    return _default


def nlm1d(*a, **k):
    return load().nlm1d(*a, **k)


def snlm(*a, **k):
    return load().snlm(*a, **k)


def pixel(*a, **k):
    return load().pixel(*a, **k)


def patch_d2(*a, **k):
    return load().patch_d2(*a, **k)


def nlm1d_div(*a, **k):
    return load().nlm1d_div(*a, **k)


def sure(*a, **k):
    return load().sure(*a, **k)


def snlm3d(*a, **k):
    return load().snlm3d(*a, **k)


def yvv(*a, **k):
    return load().yvv(*a, **k)


def iir_d2(*a, **k):
    return load().iir_d2(*a, **k)


def bilateral(*a, **k):
    return load().bilateral(*a, **k)


def bf_params(*a, **k):
    return load().bf_params(*a, **k)


def full(*a, **k):
    return load().full(*a, **k)


def max_threads() -> int:
    return load().max_threads()
