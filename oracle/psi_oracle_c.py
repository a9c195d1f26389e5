"""ctypes binding of the C/OpenMP oracle (``psi_oracle_c.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the package's smoke check and
the benchmark's CPU-baseline leg, never by the product path.  The C oracle is
the FP64 Algorithm 2 of ``psi_oracle.power_psi`` written in plain C so that
graphs of 10⁷–10⁸ users fit in host memory and run on every host core: the
operator from the raw edges (Sec. II), the recursion of eq. (power_psi), the
fixed-point residual and ψ = (Bᵀs + d)/N (the last line of Algorithm 2).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "psi_oracle_c.c")
LIB = os.path.join(HERE, "libpsi_oracle.so")

TOL_MODES = {"abs_l1": 0, "bnorm": 1, "rel_l1": 2}
PROGRESS = C.CFUNCTYPE(None, C.c_int64, C.c_double)


def build_library() -> str:
    """Compile the C oracle with gcc (OpenMP, no floating-point contraction)."""
    tmp = LIB + f".tmp{os.getpid()}"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-shared",
                    "-fPIC", "-o", tmp, SRC, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    """The loaded library; compiled first if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build_library()
        L = C.CDLL(LIB)
        p, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        L.po_build.argtypes = [i64, i64, p, p, p, p, C.POINTER(p)]
        L.po_build.restype = C.c_int
        L.po_free.argtypes = [p]
        L.po_stats.argtypes = [p, p]
        L.po_vectors.argtypes = [p, p, p, p]
        L.po_rows.argtypes = [p, p, p]
        L.po_final.argtypes = [p, p, p]
        L.po_residual.argtypes = [p, p, p]
        L.po_residual.restype = dbl
        L.po_row_sum_max.argtypes = [p, C.c_int]
        L.po_row_sum_max.restype = dbl
        L.po_power_psi.argtypes = [p, dbl, C.c_int, i64, i64, p, p, p, p, PROGRESS]
        L.po_power_psi.restype = C.c_int
        L.po_last_error.restype = C.c_char_p
        L.po_set_threads.argtypes = [C.c_int]
        L.po_max_threads.restype = C.c_int
        _lib = L
    return _lib


def set_threads(k: int) -> None:
    lib().po_set_threads(int(k))


def max_threads() -> int:
    return int(lib().po_max_threads())


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class Graph:
    """The operator of one graph in host memory (freed with the object)."""

    def __init__(self, n, follower, leader, lam, mu):
        self._keep = [np.ascontiguousarray(follower, dtype=np.int32),
                      np.ascontiguousarray(leader, dtype=np.int32),
                      np.ascontiguousarray(lam, dtype=np.float64),
                      np.ascontiguousarray(mu, dtype=np.float64)]
        f, l, la, m = self._keep
        if f.shape != l.shape or la.shape != (n,) or m.shape != (n,):
            raise ValueError("edge arrays differ in length or activity is not [n]")
        h = C.c_void_p()
        rc = lib().po_build(int(n), int(f.size), _ptr(f), _ptr(l), _ptr(la), _ptr(m), C.byref(h))
        self._keep = None
        if rc != 0:
            raise ValueError(lib().po_last_error().decode())
        self._h = h
        st = np.zeros(7, dtype=np.int64)
        lib().po_stats(self._h, _ptr(st))
        (self.n, self.m, self.m_in, self.n_self_loops, self.n_duplicates, self.n_no_leaders,
         self.max_followers) = (int(x) for x in st)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.po_free(h)
            self._h = None

    def vectors(self):
        """(c, d, den) as FP64 [n]."""
        c, d, den = (np.empty(self.n) for _ in range(3))
        lib().po_vectors(self._h, _ptr(c), _ptr(d), _ptr(den))
        return c, d, den

    def rows(self):
        """Leader-major CSR: row int64 [n+1], followers int32 [m] ascending."""
        row = np.empty(self.n + 1, dtype=np.int64)
        fol = np.empty(self.m, dtype=np.int32)
        lib().po_rows(self._h, _ptr(row), _ptr(fol))
        return row, fol

    def row_lengths(self):
        """Followers of each user (leader-major row lengths), int64 [n]."""
        row = np.empty(self.n + 1, dtype=np.int64)
        lib().po_rows(self._h, _ptr(row), None)
        return np.diff(row)

    def b_norm(self) -> float:
        return float(lib().po_row_sum_max(self._h, 0))

    def kappa(self) -> float:
        return float(lib().po_row_sum_max(self._h, 1))

    def final(self, s):
        """ψ = (Bᵀ s + d)/N for the given s (the last line of Algorithm 2)."""
        s = np.ascontiguousarray(s, dtype=np.float64)
        if s.shape != (self.n,):
            raise ValueError("s must be [n]")
        psi = np.empty(self.n)
        lib().po_final(self._h, _ptr(s), _ptr(psi))
        return psi

    def residual(self, s):
        """(r, ‖r‖₁) with r = Aᵀ s + c − s, the residual of eq. (power_psi)."""
        s = np.ascontiguousarray(s, dtype=np.float64)
        if s.shape != (self.n,):
            raise ValueError("s must be [n]")
        r = np.empty(self.n)
        l1 = lib().po_residual(self._h, _ptr(s), _ptr(r))
        return r, float(l1)

    def power_psi(self, tol, tol_mode="abs_l1", max_iter=100_000, steps=None, s0=None,
                  want_s=True, progress=None):
        """Algorithm 2 in FP64; returns a dict like ``psi_oracle.power_psi``
        plus the wall seconds of the iteration and of the final pass.  A
        step size that is not finite raises FloatingPointError.
        ``progress(t, gap)`` (optional) is called after every step."""
        s_out = np.empty(self.n) if want_s else None
        psi = np.empty(self.n)
        info = np.zeros(5)
        s0p = None
        if s0 is not None:
            s0 = np.ascontiguousarray(s0, dtype=np.float64)
            if s0.shape != (self.n,):
                raise ValueError("s0 must be [n]")
            s0p = _ptr(s0)
        cb = PROGRESS(progress) if progress is not None else PROGRESS()
        rc = lib().po_power_psi(self._h, float(tol), TOL_MODES[tol_mode], int(max_iter),
                                -1 if steps is None else int(steps), s0p,
                                None if s_out is None else _ptr(s_out), _ptr(psi), _ptr(info), cb)
        if rc == 4:
            raise FloatingPointError(lib().po_last_error().decode())
        if rc == 2:
            raise RuntimeError(lib().po_last_error().decode())
        if rc != 0:
            raise ValueError(lib().po_last_error().decode())
        return dict(psi=psi, s=s_out, iterations=int(info[0]), gap=float(info[1]),
                    l1_step=float(info[2]), seconds=float(info[3]), final_seconds=float(info[4]))
