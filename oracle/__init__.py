"""CPU oracle of the beam-search decoder -- test infrastructure only.

A ctypes wrapper around ``bsd_oracle.cpp``: min-sum BP (Appendix A,
eqs. (1)-(4)), masked BP (Algorithm 2) and beam search (Algorithm 3 and
Appendix B), in double precision (the correctness reference) and in single
precision with the natural left-to-right order of operations.

Only the tests, the smoke check and the bench's CPU-baseline leg may import
this package.  It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bsd_oracle.cpp")
# Two builds of the same source: the one the tests use, and one for timing
# the oracle on the host it runs on (-O3 -march=native; both without FMA
# contraction or fast-math, so their results are identical).
_LIB_PATHS = {"tests": os.path.join(_HERE, "liboracle.so"),
              "native": os.path.join(_HERE, "liboracle_native.so")}
_OPT = {"tests": ["-O2"], "native": ["-O3", "-march=native"]}
_LIB_PATH = _LIB_PATHS["tests"]
_libs = {}

LLR_MAX = 1e30


def build(force: bool = True, flavour: str = "tests") -> str:
    """Compile the oracle with the host compiler (no FMA contraction)."""
    path = _LIB_PATHS[flavour]
    if force or not os.path.exists(path):
        tmp = path + ".tmp"
        cmd = ["g++", "-std=c++17", *_OPT[flavour], "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-pthread", _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, path)
    return path


class Pair(C.Structure):
    _fields_ = [("col", C.c_int32), ("val", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("max_rounds", C.c_int32), ("beam_width", C.c_int32),
                ("initial_iters", C.c_int32), ("iters_per_round", C.c_int32),
                ("num_results", C.c_int32), ("alpha", C.c_double), ("llr_max", C.c_double),
                ("alpha_sched", C.POINTER(C.c_double)), ("n_alpha", C.c_int32)]


class ShotDiag(C.Structure):
    _fields_ = [("min_abs_post", C.c_double), ("min_nextpos_gap", C.c_double),
                ("min_score_gap_rel", C.c_double), ("runs", C.c_int64),
                ("iterations", C.c_int64), ("clamp_events", C.c_int64),
                ("rounds", C.c_int32), ("winner_round", C.c_int32),
                ("winner_gen", C.c_int32), ("n_results", C.c_int32)]


DIAG_DTYPE = np.dtype([("min_abs_post", "f8"), ("min_nextpos_gap", "f8"),
                       ("min_score_gap_rel", "f8"), ("runs", "i8"), ("iterations", "i8"),
                       ("clamp_events", "i8"), ("rounds", "i4"), ("winner_round", "i4"),
                       ("winner_gen", "i4"), ("n_results", "i4")])
assert DIAG_DTYPE.itemsize == C.sizeof(ShotDiag)


def _load(flavour: str = "tests"):
    if flavour in _libs:
        return _libs[flavour]
    path = _LIB_PATHS[flavour]
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        build(force=True, flavour=flavour)
    lib = C.CDLL(path)
    P = C.c_void_p
    i32p = C.POINTER(C.c_int32)
    lib.oracle_problem_create.restype = P
    lib.oracle_problem_create.argtypes = [C.c_int32, C.c_int32, C.c_int32, i32p, i32p,
                                          C.POINTER(C.c_double), i32p, i32p]
    lib.oracle_problem_destroy.argtypes = [P]
    for suf, ft in (("f64", C.c_double), ("f32", C.c_float)):
        fp = C.POINTER(ft)
        f = getattr(lib, f"oracle_bp_run_{suf}")
        f.restype = C.c_int
        f.argtypes = [P, fp, C.POINTER(Pair), C.c_int32, C.POINTER(C.c_uint8), C.c_int32, ft, ft,
                      C.c_int32, fp, fp, C.POINTER(C.c_uint8), fp, i32p, i32p]
        f = getattr(lib, f"oracle_score_{suf}")
        f.restype = C.c_int
        f.argtypes = [P, fp, C.POINTER(Pair), C.c_int32, C.c_int32, i32p, fp]
        f = getattr(lib, f"oracle_decode_{suf}")
        f.restype = C.c_int
        f.argtypes = [P, C.POINTER(Params), C.c_int64, C.POINTER(C.c_uint8),
                      C.POINTER(C.c_uint8), C.POINTER(C.c_uint8), C.POINTER(C.c_uint8),
                      C.POINTER(ShotDiag), C.c_int32]
    _libs[flavour] = lib
    return lib


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct)) if a is not None else None


def _pairs(pairs):
    pairs = list(pairs or [])
    arr = (Pair * max(len(pairs), 1))()
    for q, (c, v) in enumerate(pairs):
        arr[q].col, arr[q].val = int(c), int(v)
    return arr, len(pairs)


class OracleProblem:
    """A decoding problem (H, A, p) loaded into the oracle."""

    def __init__(self, m, n, colptr, rowidx, p, L=None, flavour="tests"):
        self._lib = _load(flavour)
        self.m, self.n = int(m), int(n)
        self.colptr = np.ascontiguousarray(colptr, dtype=np.int32)
        self.rowidx = np.ascontiguousarray(rowidx, dtype=np.int32)
        self.p = np.ascontiguousarray(p, dtype=np.float64)
        if L is None:
            L = np.zeros((0, self.n), np.uint8)
        L = np.asarray(L, dtype=np.uint8)
        self.k = int(L.shape[0])
        cols = [np.nonzero(L[:, j])[0] for j in range(self.n)]
        lptr = np.zeros(self.n + 1, np.int32)
        lptr[1:] = np.cumsum([len(c) for c in cols])
        lidx = np.concatenate(cols).astype(np.int32) if lptr[-1] else np.zeros(1, np.int32)
        self._lptr, self._lidx = lptr, lidx
        self._h = self._lib.oracle_problem_create(
            self.m, self.n, self.k, _ptr(self.colptr, C.c_int32), _ptr(self.rowidx, C.c_int32),
            _ptr(self.p, C.c_double), _ptr(lptr, C.c_int32), _ptr(lidx, C.c_int32))
        if not self._h:
            raise ValueError("oracle rejected the problem (malformed CSC or priors)")

    @classmethod
    def from_problem(cls, pr, flavour="tests"):
        return cls(pr.m, pr.n, pr.colptr, pr.rowidx, pr.p, pr.L, flavour=flavour)

    @property
    def nnz(self):
        return int(self.colptr[-1])

    def close(self):
        if getattr(self, "_h", None):
            self._lib.oracle_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def bp_run(self, s, max_iters, alpha=0.625, e_start=None, pairs=(), stop=True,
               dtype=np.float64, llr_max=LLR_MAX):
        """One masked BP run (Algorithm 2); returns a dict of its outputs."""
        dt = np.dtype(dtype)
        ct, suf = (C.c_double, "f64") if dt == np.float64 else (C.c_float, "f32")
        s = np.ascontiguousarray(s, dtype=np.uint8)
        if e_start is not None:
            e_start = np.ascontiguousarray(e_start, dtype=dt)
        e_out = np.zeros(self.nnz, dt)
        sl = np.zeros(self.n, dt)
        eh = np.zeros(self.n, np.uint8)
        post = np.zeros(self.n, dt)
        it = C.c_int32(0)
        cv = C.c_int32(0)
        parr, npairs = _pairs(pairs)
        rc = getattr(self._lib, f"oracle_bp_run_{suf}")(
            self._h, _ptr(e_start, ct), parr, npairs, _ptr(s, C.c_uint8), int(max_iters),
            float(alpha), float(llr_max), 1 if stop else 0, _ptr(e_out, ct), _ptr(sl, ct),
            _ptr(eh, C.c_uint8), _ptr(post, ct), C.byref(it), C.byref(cv))
        if rc != 0:
            raise ValueError("oracle bp_run rejected its arguments")
        return {"e": e_out, "sum_llr": sl, "ehat": eh, "post": post, "iters": it.value,
                "converged": bool(cv.value)}

    def score(self, sum_llr, pairs, iters, dtype=np.float64):
        dt = np.dtype(dtype)
        ct, suf = (C.c_double, "f64") if dt == np.float64 else (C.c_float, "f32")
        sl = np.ascontiguousarray(sum_llr, dtype=dt)
        parr, npairs = _pairs(pairs)
        npos = C.c_int32(0)
        sc = ct(0)
        rc = getattr(self._lib, f"oracle_score_{suf}")(self._h, _ptr(sl, ct), parr, npairs,
                                                       int(iters), C.byref(npos), C.byref(sc))
        if rc != 0:
            raise ValueError("oracle score rejected its arguments")
        return npos.value, sc.value

    def decode(self, syndromes, max_rounds, beam_width, initial_iters, iters_per_round,
               num_results=1, alpha=0.625, dtype=np.float64, threads=0, llr_max=LLR_MAX,
               alpha_sched=None):
        """Beam-search decoding (Algorithm 3) of a batch of syndromes;
        `alpha_sched` (optional) scales iteration t of every BP run by
        alpha_sched[min(t, len) - 1]."""
        syn = np.ascontiguousarray(syndromes, dtype=np.uint8).reshape(-1, self.m)
        shots = syn.shape[0]
        corr = np.zeros((shots, self.n), np.uint8)
        flips = np.zeros((shots, self.k), np.uint8)
        conv = np.zeros(shots, np.uint8)
        diag = np.zeros(shots, DIAG_DTYPE)
        sched = None if alpha_sched is None else np.ascontiguousarray(alpha_sched, dtype=np.float64)
        prm = Params(int(max_rounds), int(beam_width), int(initial_iters), int(iters_per_round),
                     int(num_results), float(alpha), float(llr_max),
                     _ptr(sched, C.c_double) if sched is not None else None,
                     0 if sched is None else len(sched))
        suf = "f64" if np.dtype(dtype) == np.float64 else "f32"
        rc = getattr(self._lib, f"oracle_decode_{suf}")(
            self._h, C.byref(prm), shots, _ptr(syn, C.c_uint8), _ptr(corr, C.c_uint8),
            _ptr(flips, C.c_uint8), _ptr(conv, C.c_uint8),
            diag.ctypes.data_as(C.POINTER(ShotDiag)), int(threads))
        if rc != 0:
            raise ValueError("oracle decode rejected its arguments")
        return {"corrections": corr, "flips": flips, "converged": conv, "diag": diag}

    def decode_params(self, syndromes, params, dtype=np.float64, threads=0, alpha_sched=None):
        return self.decode(syndromes, params.max_rounds, params.beam_width, params.initial_iters,
                           params.iters_per_round, params.num_results, params.alpha,
                           dtype=dtype, threads=threads, alpha_sched=alpha_sched)
