"""FP64 CPU oracle for supernodal selected inversion (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only users.  The product library neither imports
nor links anything here, and this package imports nothing from the product.

The arithmetic lives in ``selinv_oracle.c`` (plain C, FP64, -O2
-ffp-contract=off): its own symbolic analysis, unpivoted LU and Algorithm 1 of
the paper (steps 2-6), with every already-computed entry of A^{-T} read by a
direct (row, column) lookup.  ``sampled.py`` adds an independent check for
sizes where the supernodal oracle is too slow: single entries of A^{-1} from
linear solves with A itself.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "selinv_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-std=gnu11", "-Wall", "-Wno-unused-function"]

STATUS = {0: "OK", 1: "INVALID_ARG", 2: "BAD_PATTERN", 3: "BAD_PERM", 4: "ZERO_PIVOT",
          5: "NOT_SELECTED", 6: "STATE", 7: "NOMEM", 8: "CLOSURE"}


class OracleError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"oracle error {STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


def build(force: bool = True) -> str:
    """Compile the oracle shared library with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = C.CDLL(_LIB)
    P = C.POINTER
    vp = C.c_void_p
    lib.oracle_analyze.argtypes = [C.c_int64, P(C.c_int64), P(C.c_int32), P(C.c_int32),
                                   C.c_int32, C.c_int32, C.c_int32, C.c_int32, P(vp)]
    lib.oracle_analyze.restype = C.c_int
    lib.oracle_factor.argtypes = [vp, P(C.c_double)]
    lib.oracle_factor.restype = C.c_int
    lib.oracle_selinv.argtypes = [vp]
    lib.oracle_selinv.restype = C.c_int
    lib.oracle_get.argtypes = [vp, C.c_int64, C.c_int64, P(C.c_double)]
    lib.oracle_get.restype = C.c_int
    lib.oracle_get_selected.argtypes = [vp, P(C.c_double)]
    lib.oracle_get_selected.restype = C.c_int
    lib.oracle_superset_nnz.argtypes = [vp]
    lib.oracle_superset_nnz.restype = C.c_int64
    lib.oracle_export.argtypes = [vp, P(C.c_int32), P(C.c_int32), P(C.c_double)]
    lib.oracle_export.restype = C.c_int
    lib.oracle_nsuper.argtypes = [vp]
    lib.oracle_nsuper.restype = C.c_int32
    lib.oracle_rl_total.argtypes = [vp]
    lib.oracle_rl_total.restype = C.c_int64
    lib.oracle_ru_total.argtypes = [vp]
    lib.oracle_ru_total.restype = C.c_int64
    lib.oracle_structure.argtypes = [vp, P(C.c_int32), P(C.c_int32), P(C.c_int64), P(C.c_int32),
                                     P(C.c_int64), P(C.c_int32)]
    lib.oracle_structure.restype = C.c_int
    lib.oracle_diag_alt.argtypes = [vp, P(C.c_double), P(C.c_double)]
    lib.oracle_diag_alt.restype = None
    lib.oracle_from_factors.argtypes = [C.c_int64, C.c_int32, P(C.c_int32), P(C.c_int64),
                                        P(C.c_int32), P(C.c_int64), P(C.c_int32),
                                        P(C.c_double), P(C.c_double), P(vp)]
    lib.oracle_from_factors.restype = C.c_int
    lib.oracle_free.argtypes = [vp]
    lib.oracle_free.restype = None
    lib.oracle_last_error.argtypes = [vp]
    lib.oracle_last_error.restype = C.c_char_p
    lib.oracle_set_threads.argtypes = [C.c_int]
    lib.oracle_set_threads.restype = None
    lib.oracle_get_threads.argtypes = []
    lib.oracle_get_threads.restype = C.c_int
    _lib = lib
    return lib


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def set_threads(t: int) -> None:
    _load().oracle_set_threads(int(t))


def get_threads() -> int:
    return int(_load().oracle_get_threads())


class Oracle:
    """One matrix: analyze -> factor -> selinv -> get / get_selected / export.

    mode 0: symbolic on pattern(PAP^T + (PAP^T)^T) with relaxed, capped
    supernodes (relaxed subtrees of <= relax columns, chains merged while the
    padding estimate stays <= pad_pct percent); mode 1: exact non-symmetric
    structure (small n, no relaxation).
    """

    def __init__(self, n, colptr, rowind, perm=None, max_super=0, relax=0, mode=0, pad_pct=0):
        self._lib = _load()
        self._h = C.c_void_p()
        self.n = int(n)
        self._colptr = np.ascontiguousarray(colptr, dtype=np.int64)
        self._rowind = np.ascontiguousarray(rowind, dtype=np.int32)
        self.nnz = int(self._colptr[-1])
        pp = None
        if perm is not None:
            self._perm = np.ascontiguousarray(perm, dtype=np.int32)
            pp = _ptr(self._perm, C.c_int32)
        rc = self._lib.oracle_analyze(self.n, _ptr(self._colptr, C.c_int64),
                                      _ptr(self._rowind, C.c_int32), pp, int(max_super),
                                      int(relax), int(pad_pct), int(mode), C.byref(self._h))
        if rc:
            raise OracleError(rc, "analyze")

    @classmethod
    def from_factors(cls, n, xsup, rl_ptr, rl, ru_ptr, ru, L, U):
        self = cls.__new__(cls)
        self._lib = _load()
        self._h = C.c_void_p()
        self.n = int(n)
        self.nnz = 0
        xs = np.ascontiguousarray(xsup, dtype=np.int32)
        a = np.ascontiguousarray(rl_ptr, dtype=np.int64)
        b = np.ascontiguousarray(rl, dtype=np.int32)
        c = np.ascontiguousarray(ru_ptr, dtype=np.int64)
        d = np.ascontiguousarray(ru, dtype=np.int32)
        Lf = np.asfortranarray(L, dtype=np.float64)
        Uf = np.asfortranarray(U, dtype=np.float64)
        rc = self._lib.oracle_from_factors(self.n, len(xs) - 1, _ptr(xs, C.c_int32),
                                           _ptr(a, C.c_int64), _ptr(b, C.c_int32),
                                           _ptr(c, C.c_int64), _ptr(d, C.c_int32),
                                           Lf.ctypes.data_as(C.POINTER(C.c_double)),
                                           Uf.ctypes.data_as(C.POINTER(C.c_double)),
                                           C.byref(self._h))
        if rc:
            raise OracleError(rc, "from_factors")
        return self

    def _check(self, rc, what):
        if rc:
            msg = self._lib.oracle_last_error(self._h)
            raise OracleError(rc, f"{what}: {msg.decode() if msg else ''}")

    def factor(self, values):
        v = np.ascontiguousarray(values, dtype=np.float64)
        self._check(self._lib.oracle_factor(self._h, _ptr(v, C.c_double)), "factor")
        return self

    def selinv(self):
        self._check(self._lib.oracle_selinv(self._h), "selinv")
        return self

    def get(self, i, j) -> float:
        out = C.c_double()
        self._check(self._lib.oracle_get(self._h, int(i), int(j), C.byref(out)), "get")
        return out.value

    def get_selected(self) -> np.ndarray:
        out = np.empty(self.nnz, dtype=np.float64)
        self._check(self._lib.oracle_get_selected(self._h, _ptr(out, C.c_double)), "get_selected")
        return out

    def export(self):
        """All computed entries: (row, col, value) with value = A^{-1}(row, col), sorted."""
        m = int(self._lib.oracle_superset_nnz(self._h))
        r = np.empty(m, np.int32)
        c = np.empty(m, np.int32)
        v = np.empty(m, np.float64)
        self._check(self._lib.oracle_export(self._h, _ptr(r, C.c_int32), _ptr(c, C.c_int32),
                                            _ptr(v, C.c_double)), "export")
        # sorted by (column, row); the keys are unique
        order = np.argsort(c.astype(np.int64) * self.n + r)
        return r[order], c[order], v[order]

    def structure(self) -> dict:
        ns = int(self._lib.oracle_nsuper(self._h))
        nl = int(self._lib.oracle_rl_total(self._h))
        nu = int(self._lib.oracle_ru_total(self._h))
        perm = np.empty(self.n, np.int32)
        xsup = np.empty(ns + 1, np.int32)
        rlp = np.empty(ns + 1, np.int64)
        rl = np.empty(max(nl, 1), np.int32)
        rup = np.empty(ns + 1, np.int64)
        ru = np.empty(max(nu, 1), np.int32)
        self._check(self._lib.oracle_structure(self._h, _ptr(perm, C.c_int32), _ptr(xsup, C.c_int32),
                                               _ptr(rlp, C.c_int64), _ptr(rl, C.c_int32),
                                               _ptr(rup, C.c_int64), _ptr(ru, C.c_int32)),
                    "structure")
        return {"perm": perm, "xsup": xsup, "rl_ptr": rlp, "rl": rl[:nl], "ru_ptr": rup,
                "ru": ru[:nu]}

    def diag_alt(self):
        """(max |Z - Z'|, max |Z|) over all diagonal blocks, Z' = the other step-4 formula."""
        a = C.c_double()
        b = C.c_double()
        self._lib.oracle_diag_alt(self._h, C.byref(a), C.byref(b))
        return a.value, b.value

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.oracle_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def selected_inverse(n, colptr, rowind, values, perm=None, max_super=0, relax=0, mode=0, pad_pct=0):
    """Convenience: returns (Oracle, out) with out[p] = A^{-1}(col p, row p)."""
    o = Oracle(n, colptr, rowind, perm, max_super, relax, mode, pad_pct)
    o.factor(values).selinv()
    return o, o.get_selected()
