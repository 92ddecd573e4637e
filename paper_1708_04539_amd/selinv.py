"""ctypes binding of the C ABI in include/selinv.h (argument marshalling only).

Every step of the selected inversion runs in the HIP library
(``libselinv.so``); this module only converts arrays and status codes.  The
library must have been built (``paper_1708_04539_amd.build.build()``); if it is
missing, importing this module raises.

torch is imported first so that the HIP runtime torch ships is the one the
library binds to (both use the soname libamdhip64.so.7); streams passed to
``run`` are torch stream handles.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # noqa: F401  (loads the process-wide HIP runtime first)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libselinv.so")

FP64, MIXED_FP32, MIXED_BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "mixed_fp32": MIXED_FP32, "mixed_bf16x3": MIXED_BF16X3}
STATUS = {0: "OK", 1: "INVALID_ARG", 2: "BAD_PATTERN", 3: "BAD_PERM", 4: "ZERO_PIVOT",
          5: "NOT_SELECTED", 6: "STATE", 7: "NOMEM", 8: "DEVICE"}

EXPORTED = ["selinv_analyze", "selinv_factor", "selinv_factor_device", "selinv_run", "selinv_run_graph", "selinv_batch_create",
            "selinv_batch_run", "selinv_batch_destroy", "selinv_get", "selinv_get_selected",
            "selinv_get_selected_device", "selinv_export", "selinv_structure", "selinv_query",
            "selinv_set_profiling", "selinv_timings", "selinv_level_stats", "selinv_last_error",
            "selinv_status_string", "selinv_destroy", "selinv_check_plan", "selinv_set_sweep_mode",
            "selinv_sweep_is_persistent", "selinv_batch_set_sweep_mode", "selinv_tune", "selinv_get_tuning",
            "selinv_set_tuning", "selinv_set_allocator", "selinv_get_many", "selinv_set_gather_code_budget",
            "selinv_batch_run_graph", "selinv_batch_tune", "selinv_batch_get_tuning", "selinv_batch_set_tuning",
            "selinv_batch_set_profiling", "selinv_batch_timings", "selinv_batch_level_stats", "selinv_batch_query",
            "selinv_batch_last_error", "selinv_get_selected_noalloc", "selinv_set_gather_form",
            "selinv_batch_set_gather_form"]


class SelinvError(RuntimeError):
    def __init__(self, code, msg=""):
        self.code = int(code)
        self.status = STATUS.get(self.code, str(code))
        super().__init__(f"selinv {self.status}: {msg}")


class Info(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz_a", C.c_int64), ("nnz_lu", C.c_int64), ("nsuper", C.c_int32),
                ("nlevels", C.c_int32), ("max_s", C.c_int32), ("max_c", C.c_int32), ("flops", C.c_double),
                ("flops_gemm", C.c_double), ("bytes_min_fp64", C.c_double), ("bytes_min_fp32", C.c_double),
                ("max_gemm_flops", C.c_double), ("max_gemm_m", C.c_int32), ("max_gemm_n", C.c_int32),
                ("max_gemm_k", C.c_int32), ("symbolic", C.c_int32), ("nnz_l", C.c_int64), ("nnz_u", C.c_int64),
                ("complex_values", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Opts(C.Structure):
    _fields_ = [("max_super", C.c_int32), ("relax", C.c_int32), ("pad_pct", C.c_int32), ("symbolic", C.c_int32),
                ("complex_values", C.c_int32)]


# analysis forms: pattern of At + At^T (R_L = R_U), or the exact pattern of L and U
SYMBOLIC = {"symmetrized": 0, "exact": 1}


# device-memory hooks of selinv_set_allocator: (bytes, ctx) -> pointer, (pointer, ctx) -> None
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1708_04539_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    P, vp = C.POINTER, C.c_void_p
    i32, i64, dbl = C.c_int32, C.c_int64, C.c_double
    sig = {
        "selinv_analyze": ([i64, P(i64), P(i32), P(i32), P(Opts), P(vp)], C.c_int),
        "selinv_factor": ([vp, P(dbl)], C.c_int),
        "selinv_factor_device": ([vp, vp, vp], C.c_int),
        "selinv_run": ([vp, C.c_int, vp], C.c_int),
        "selinv_run_graph": ([vp, C.c_int, vp], C.c_int),
        "selinv_batch_create": ([P(vp), i32, P(vp)], C.c_int),
        "selinv_batch_run": ([vp, C.c_int, vp], C.c_int),
        "selinv_batch_destroy": ([vp], None),
        "selinv_get": ([vp, i64, i64, P(dbl)], C.c_int),
        "selinv_get_selected": ([vp, P(dbl)], C.c_int),
        "selinv_get_selected_device": ([vp, vp, vp], C.c_int),
        "selinv_export": ([vp, P(i32), P(i32), P(dbl)], C.c_int),
        "selinv_structure": ([vp, P(i32), P(i32), P(i64), P(i32), P(i64), P(i32), P(i32)], C.c_int),
        "selinv_query": ([vp, P(Info)], C.c_int),
        "selinv_set_profiling": ([vp, i32], C.c_int),
        "selinv_timings": ([vp, P(dbl), i32], C.c_int),
        "selinv_level_stats": ([vp, i32, P(dbl)], C.c_int),
        "selinv_last_error": ([vp], C.c_char_p),
        "selinv_status_string": ([C.c_int], C.c_char_p),
        "selinv_destroy": ([vp], None),
        "selinv_check_plan": ([vp, P(i64)], C.c_int),
        "selinv_set_sweep_mode": ([vp, i32], C.c_int),
        "selinv_sweep_is_persistent": ([vp, C.c_int], i32),
        "selinv_batch_set_sweep_mode": ([vp, i32], C.c_int),
        "selinv_set_gather_form": ([vp, i32], C.c_int),
        "selinv_batch_set_gather_form": ([vp, i32], C.c_int),
        "selinv_tune": ([vp, C.c_int, i32, vp, P(dbl), P(dbl)], C.c_int),
        "selinv_get_tuning": ([vp, C.c_int, P(i32), i32, P(i32)], C.c_int),
        "selinv_set_tuning": ([vp, C.c_int, P(i32), i32], C.c_int),
        "selinv_set_allocator": ([ALLOC_FN, FREE_FN, vp], C.c_int),
        "selinv_get_many": ([vp, i64, P(i64), P(i64), P(dbl)], C.c_int),
        "selinv_set_gather_code_budget": ([vp, i64], C.c_int),
        "selinv_batch_run_graph": ([vp, C.c_int, vp], C.c_int),
        "selinv_batch_tune": ([vp, C.c_int, i32, vp, P(dbl), P(dbl)], C.c_int),
        "selinv_batch_get_tuning": ([vp, C.c_int, P(i32), i32, P(i32)], C.c_int),
        "selinv_batch_set_tuning": ([vp, C.c_int, P(i32), i32], C.c_int),
        "selinv_batch_set_profiling": ([vp, i32], C.c_int),
        "selinv_batch_timings": ([vp, P(dbl), i32], C.c_int),
        "selinv_batch_level_stats": ([vp, i32, P(dbl)], C.c_int),
        "selinv_batch_query": ([vp, P(i32), P(i32), P(dbl)], C.c_int),
        "selinv_batch_last_error": ([vp], C.c_char_p),
        "selinv_get_selected_noalloc": ([vp, P(dbl)], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = _load()


def lib():
    return _lib


def _torch_alloc(nbytes, ctx):
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device())
    except Exception:  # out of memory (or interpreter shutdown): the library reports NOMEM
        return None


def _torch_free(ptr, ctx):
    try:
        torch.cuda.caching_allocator_delete(ptr)
    except Exception:
        pass


_hooks = {"torch": (ALLOC_FN(_torch_alloc), FREE_FN(_torch_free)),
          "hip": (ALLOC_FN(), FREE_FN())}  # NULL hooks: hipMalloc / hipFree
_user_hooks = []  # keeps caller-supplied hooks alive


def set_allocator(kind="torch", alloc=None, free=None):
    """Source of the device memory of handles and batches created from now on:
    "torch" (torch's caching allocator, the default), "hip" (hipMalloc/hipFree),
    or "custom" with Python callables alloc(nbytes) -> int pointer or None and
    free(pointer)."""
    if kind == "custom":
        a = ALLOC_FN(lambda nb, ctx: alloc(int(nb)))
        f = FREE_FN(lambda ptr, ctx: free(ptr))
        _user_hooks.append((a, f))
    else:
        a, f = _hooks[kind]
    rc = _lib.selinv_set_allocator(a, f, None)
    if rc:
        raise SelinvError(rc, "set_allocator")


set_allocator("torch")


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _prec(p):
    return PRECISIONS[p] if isinstance(p, str) else int(p)


class SelInv:
    """One matrix: analyze (construction) -> factor -> run -> get*/export."""

    def __init__(self, n, colptr, rowind, perm=None, max_super=0, relax=0, pad_pct=0, symbolic="symmetrized",
                 complex_values=False):
        self._h = C.c_void_p()
        self.n = int(n)
        self._colptr = np.ascontiguousarray(colptr, dtype=np.int64)
        self._rowind = np.ascontiguousarray(rowind, dtype=np.int32)
        self.nnz = int(self._colptr[-1])
        pp = None
        if perm is not None:
            self._perm = np.ascontiguousarray(perm, dtype=np.int32)
            pp = _p(self._perm, C.c_int32)
        sym = SYMBOLIC[symbolic] if isinstance(symbolic, str) else int(symbolic)
        self.is_complex = bool(complex_values)
        opts = Opts(int(max_super), int(relax), int(pad_pct), sym, 1 if self.is_complex else 0)
        rc = _lib.selinv_analyze(self.n, _p(self._colptr, C.c_int64), _p(self._rowind, C.c_int32), pp,
                                 C.byref(opts), C.byref(self._h))
        if rc:
            msg = _lib.selinv_last_error(None).decode()
            raise SelinvError(rc, "analyze: " + msg)
        self.info = self.query()

    def _check(self, rc, what):
        if rc:
            raise SelinvError(rc, f"{what}: {_lib.selinv_last_error(self._h).decode()}")

    def factor(self, values):
        if self.is_complex:  # (re, im) per entry
            v = np.ascontiguousarray(values, dtype=np.complex128).view(np.float64)
        else:
            v = np.ascontiguousarray(values, dtype=np.float64)
        self._check(_lib.selinv_factor(self._h, _p(v, C.c_double)), "factor")
        return self

    def factor_device(self, values: "torch.Tensor", stream=None):
        """LU on the GPU from values already in device memory (float64, or
        complex128 for a complex handle), aligned with rowind."""
        want = torch.complex128 if self.is_complex else torch.float64
        if not (values.dtype == want and values.is_cuda and values.is_contiguous()
                and values.numel() == self.nnz):
            raise ValueError(f"factor_device wants a contiguous {want} CUDA tensor of {self.nnz} entries")
        self._check(_lib.selinv_factor_device(self._h, C.c_void_p(values.data_ptr()), _stream_ptr(stream)),
                    "factor_device")
        return self

    def run(self, precision="fp64", stream=None, graph=False):
        f = _lib.selinv_run_graph if graph else _lib.selinv_run
        self._check(f(self._h, _prec(precision), _stream_ptr(stream)), "run")
        return self

    def get(self, i, j):
        out = (C.c_double * 2)()
        self._check(_lib.selinv_get(self._h, int(i), int(j), out), "get")
        return complex(out[0], out[1]) if self.is_complex else out[0]

    def get_many(self, i, j) -> np.ndarray:
        """A^{-1}(i[k], j[k]) for every k (one device gather)."""
        ii = np.ascontiguousarray(i, dtype=np.int64)
        jj = np.ascontiguousarray(j, dtype=np.int64)
        if ii.shape != jj.shape:
            raise ValueError("i and j must have the same length")
        out = np.empty(ii.size * (2 if self.is_complex else 1), dtype=np.float64)
        self._check(_lib.selinv_get_many(self._h, ii.size, _p(ii, C.c_int64), _p(jj, C.c_int64),
                                         _p(out, C.c_double)), "get_many")
        return out.view(np.complex128) if self.is_complex else out

    def set_gather_code_budget(self, entries=-1):
        """Precomputed gather source codes: -1 default budget, 0 off (before factor)."""
        self._check(_lib.selinv_set_gather_code_budget(self._h, int(entries)), "set_gather_code_budget")
        return self

    def get_selected(self) -> np.ndarray:
        out = np.empty(self.nnz * (2 if self.is_complex else 1), dtype=np.float64)
        self._check(_lib.selinv_get_selected(self._h, _p(out, C.c_double)), "get_selected")
        return out.view(np.complex128) if self.is_complex else out

    def get_selected_noalloc(self) -> np.ndarray:
        """As get_selected, staged through the library's fixed device array
        (no device allocation)."""
        out = np.empty(self.nnz * (2 if self.is_complex else 1), dtype=np.float64)
        self._check(_lib.selinv_get_selected_noalloc(self._h, _p(out, C.c_double)), "get_selected_noalloc")
        return out.view(np.complex128) if self.is_complex else out

    def get_selected_device(self, out: "torch.Tensor", stream=None):
        want = torch.complex128 if self.is_complex else torch.float64
        assert out.dtype == want and out.is_cuda and out.numel() >= self.nnz and out.is_contiguous()
        self._check(_lib.selinv_get_selected_device(self._h, C.c_void_p(out.data_ptr()), _stream_ptr(stream)),
                    "get_selected_device")
        return out

    def export(self, sort=True):
        """Every computed entry (row, col, A^{-1}(row, col)): sorted by (col, row),
        or in the library's storage order (sort=False; the same order for every
        run of the handle)."""
        m = int(self.info["nnz_lu"])
        r = np.empty(m, np.int32)
        c = np.empty(m, np.int32)
        v = np.empty(m, np.float64)
        self._check(_lib.selinv_export(self._h, _p(r, C.c_int32), _p(c, C.c_int32), _p(v, C.c_double)), "export")
        if not sort:
            return r, c, v
        order = np.argsort(c.astype(np.int64) * int(self.info["n"]) + r)
        return r[order], c[order], v[order]

    def structure(self) -> dict:
        ns = self.info["nsuper"]
        perm = np.empty(self.info["n"], np.int32)  # order of the plan (2 n for a complex handle)
        xsup = np.empty(ns + 1, np.int32)
        rlp = np.empty(ns + 1, np.int64)
        rup = np.empty(ns + 1, np.int64)
        lev = np.empty(ns, np.int32)
        self._check(_lib.selinv_structure(self._h, _p(perm, C.c_int32), _p(xsup, C.c_int32), _p(rlp, C.c_int64),
                                          None, _p(rup, C.c_int64), None, _p(lev, C.c_int32)), "structure")
        rl = np.empty(max(int(rlp[-1]), 1), np.int32)
        ru = np.empty(max(int(rup[-1]), 1), np.int32)
        self._check(_lib.selinv_structure(self._h, None, None, None, _p(rl, C.c_int32), None, _p(ru, C.c_int32),
                                          None), "structure")
        return {"perm": perm, "xsup": xsup, "rl_ptr": rlp, "rl": rl[:int(rlp[-1])], "ru_ptr": rup,
                "ru": ru[:int(rup[-1])], "level": lev}

    def query(self) -> dict:
        info = Info()
        self._check(_lib.selinv_query(self._h, C.byref(info)), "query")
        return info.as_dict()

    def check_plan(self) -> int:
        """Host-side check of every gather/extraction index; returns the mismatch count."""
        out = C.c_int64()
        self._check(_lib.selinv_check_plan(self._h, C.byref(out)), "check_plan")
        return out.value

    SWEEP_MODES = {"auto": 0, "levels": 1, "persistent": 2}

    def set_sweep_mode(self, mode="auto"):
        m = self.SWEEP_MODES[mode] if isinstance(mode, str) else int(mode)
        self._check(_lib.selinv_set_sweep_mode(self._h, m), "set_sweep_mode")
        return self

    # where the level sweep takes G_K from (selinv_set_gather_form)
    GATHER_FORMS = {"auto": 0, "stored": 1, "in_products": 2}

    def set_gather_form(self, form="auto"):
        f = self.GATHER_FORMS[form] if isinstance(form, str) else int(form)
        self._check(_lib.selinv_set_gather_form(self._h, f), "set_gather_form")
        return self

    def sweep_is_persistent(self, precision="fp64") -> int:
        return int(_lib.selinv_sweep_is_persistent(self._h, _prec(precision)))

    def tune(self, precision="fp64", reps=5, stream=None):
        """Measure and keep the fastest launch choices of the sweep (selinv_tune);
        returns (ms with the size policy, ms with the kept choices)."""
        a, b = C.c_double(), C.c_double()
        self._check(_lib.selinv_tune(self._h, _prec(precision), int(reps), _stream_ptr(stream), C.byref(a),
                                     C.byref(b)), "tune")
        return a.value, b.value

    def get_tuning(self, precision="fp64") -> list:
        n = C.c_int32()
        self._check(_lib.selinv_get_tuning(self._h, _prec(precision), None, 0, C.byref(n)), "get_tuning")
        if n.value == 0:
            return []
        out = np.empty(n.value, np.int32)
        self._check(_lib.selinv_get_tuning(self._h, _prec(precision), _p(out, C.c_int32), n.value, C.byref(n)),
                    "get_tuning")
        return out.tolist()

    def set_tuning(self, table, precision="fp64"):
        t = np.ascontiguousarray(table, dtype=np.int32)
        self._check(_lib.selinv_set_tuning(self._h, _prec(precision), _p(t, C.c_int32) if t.size else None,
                                           int(t.size)), "set_tuning")
        return self

    def set_profiling(self, on=True):
        self._check(_lib.selinv_set_profiling(self._h, 1 if on else 0), "set_profiling")

    def timings(self):
        """Per-phase device ms of the last profiled run: tri_inv, normalise, diag init,
        then (small supernodes fused, gather, steps 3+5, step 4) for every level."""
        k = 3 + 4 * self.info["nlevels"]
        out = np.zeros(k, np.float64)
        self._check(_lib.selinv_timings(self._h, _p(out, C.c_double), k), "timings")
        return out

    def level_stats(self, level):
        """Work of one level of the last run's sweep; level = -1: the prologue."""
        out = np.zeros(19, np.float64)
        self._check(_lib.selinv_level_stats(self._h, int(level), _p(out, C.c_double)), "level_stats")
        return self._stats_dict(level, out)

    @staticmethod
    def _stats_dict(level, out):
        if level == -1:
            keys = ["tri_flops", "tri_bytes", "norm_flops", "norm_bytes", "dt_flops", "dt_bytes"]
        else:
            keys = ["nsup", "max_s", "flops35", "flops4", "gather_elems", "gather_tiles", "tiles35", "tiles4",
                    "tile35", "tile4", "small_count", "small_flops", "small_elems", "gather_fused",
                    "bytes35", "bytes4", "bytes_gather", "bytes_small", "max_prod_flops"]
        return dict(zip(keys, out.tolist()))

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.selinv_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """One level sweep over several factored matrices (levels aligned at the roots)."""

    def __init__(self, mats):
        self.mats = list(mats)
        arr = (C.c_void_p * len(self.mats))(*[m.handle.value for m in self.mats])
        self._b = C.c_void_p()
        rc = _lib.selinv_batch_create(arr, len(self.mats), C.byref(self._b))
        if rc:
            raise SelinvError(rc, "batch_create")
        n, L, F = C.c_int32(), C.c_int32(), C.c_double()
        self._check(_lib.selinv_batch_query(self._b, C.byref(n), C.byref(L), C.byref(F)), "batch_query")
        self.info = {"count": n.value, "nlevels": L.value, "flops": F.value}

    def _check(self, rc, what):
        if rc:
            raise SelinvError(rc, f"{what}: {_lib.selinv_batch_last_error(self._b).decode()}")

    def set_sweep_mode(self, mode="auto"):
        m = SelInv.SWEEP_MODES[mode] if isinstance(mode, str) else int(mode)
        self._check(_lib.selinv_batch_set_sweep_mode(self._b, m), "batch_set_sweep_mode")
        return self

    def set_gather_form(self, form="auto"):
        f = SelInv.GATHER_FORMS[form] if isinstance(form, str) else int(form)
        self._check(_lib.selinv_batch_set_gather_form(self._b, f), "batch_set_gather_form")
        return self

    def run(self, precision="fp64", stream=None, graph=False):
        f = _lib.selinv_batch_run_graph if graph else _lib.selinv_batch_run
        self._check(f(self._b, _prec(precision), _stream_ptr(stream)), "batch_run")
        return self

    def tune(self, precision="fp64", reps=5, stream=None):
        a, b = C.c_double(), C.c_double()
        self._check(_lib.selinv_batch_tune(self._b, _prec(precision), int(reps), _stream_ptr(stream), C.byref(a),
                                           C.byref(b)), "batch_tune")
        return a.value, b.value

    def get_tuning(self, precision="fp64") -> list:
        n = C.c_int32()
        self._check(_lib.selinv_batch_get_tuning(self._b, _prec(precision), None, 0, C.byref(n)), "get_tuning")
        if n.value == 0:
            return []
        out = np.empty(n.value, np.int32)
        self._check(_lib.selinv_batch_get_tuning(self._b, _prec(precision), _p(out, C.c_int32), n.value,
                                                 C.byref(n)), "get_tuning")
        return out.tolist()

    def set_tuning(self, table, precision="fp64"):
        t = np.ascontiguousarray(table, dtype=np.int32)
        self._check(_lib.selinv_batch_set_tuning(self._b, _prec(precision), _p(t, C.c_int32) if t.size else None,
                                                 int(t.size)), "set_tuning")
        return self

    def set_profiling(self, on=True):
        self._check(_lib.selinv_batch_set_profiling(self._b, 1 if on else 0), "set_profiling")

    def timings(self):
        k = 3 + 4 * self.info["nlevels"]
        out = np.zeros(k, np.float64)
        self._check(_lib.selinv_batch_timings(self._b, _p(out, C.c_double), k), "timings")
        return out

    def level_stats(self, level):
        out = np.zeros(19, np.float64)
        self._check(_lib.selinv_batch_level_stats(self._b, int(level), _p(out, C.c_double)), "level_stats")
        return SelInv._stats_dict(level, out)

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            _lib.selinv_batch_destroy(self._b)
            self._b = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
