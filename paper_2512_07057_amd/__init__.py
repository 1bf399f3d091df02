"""Python binding of the MI355X beam-search decoder (libbsd.so).

Argument marshalling only: every step of decoding runs in the HIP kernels
behind the C ABI declared in include/bsd.h.  PyTorch supplies device memory
and streams.  The library must have been built (``build.build()``); there is
no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbsd.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "bsd.h")

BSD_OK, BSD_EINVAL, BSD_ENOMEM, BSD_EDEVICE, BSD_EBUSY = 0, -1, -2, -3, -4
MODE_BATCHED, MODE_PLAIN = 0, 1
FLAG_GRAPH = 1
FLAG_DENSE_FIRST = 2
FLAG_ALPHA_SCHEDULE = 4
FLAG_NO_SCREEN = 8
FLAG_NO_SCREEN2 = 16
FLAG_BESIDE = 32
_lib = None


class BsdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"bsd status {status}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("max_rounds", C.c_int32), ("beam_width", C.c_int32),
                ("initial_iters", C.c_int32), ("iters_per_round", C.c_int32),
                ("num_results", C.c_int32), ("alpha", C.c_float), ("mode", C.c_int32),
                ("flags", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("runs", C.c_int64), ("iterations", C.c_int64), ("edge_updates", C.c_int64),
                ("deep_shots", C.c_int64), ("kernel_ms", C.c_double),
                ("screened_shots", C.c_int64), ("screen_ms", C.c_double),
                ("screened2_shots", C.c_int64)]


class ServeReport(C.Structure):
    _fields_ = [("requests", C.c_int64), ("seconds", C.c_double), ("offered_per_s", C.c_double),
                ("served_per_s", C.c_double), ("p50_us", C.c_double), ("p99_us", C.c_double),
                ("p999_us", C.c_double), ("max_us", C.c_double),
                ("code_requests", C.c_int64 * 8), ("code_p50_us", C.c_double * 8),
                ("code_p99_us", C.c_double * 8), ("code_p999_us", C.c_double * 8),
                ("admission_waits", C.c_int64)]


class ServerOpts(C.Structure):
    _fields_ = [("ring_bytes", C.c_int64), ("idle_ms", C.c_int64)]


def exported_symbols_from_header(path: str = HEADER) -> list[str]:
    text = open(path).read()
    return sorted(set(re.findall(r"\b(bsd_[a-z_]+)\s*\(", text)))


def load():
    """Load libbsd.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2512_07057_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    P, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    i32p = C.POINTER(C.c_int32)
    lib.bsd_last_error.restype = C.c_char_p
    lib.bsd_version.restype = C.c_char_p
    lib.bsd_code_create.restype = C.c_int
    lib.bsd_code_create.argtypes = [i32, i32, i32, i32p, i32p, C.POINTER(C.c_double), i32p, i32p,
                                    C.POINTER(P)]
    lib.bsd_code_destroy.restype = C.c_int
    lib.bsd_code_destroy.argtypes = [P]
    lib.bsd_code_set_alpha_schedule.restype = C.c_int
    lib.bsd_code_set_alpha_schedule.argtypes = [P, i32, C.POINTER(C.c_float)]
    lib.bsd_code_info.restype = C.c_int
    lib.bsd_code_info.argtypes = [P, C.POINTER(i64), i32p, i32p, i32p]
    lib.bsd_decode.restype = C.c_int
    lib.bsd_decode.argtypes = [P, C.POINTER(Params), i64, P, P, P, P, P]
    lib.bsd_code_sync.restype = C.c_int
    lib.bsd_code_sync.argtypes = [P, P]
    lib.bsd_decode_ex.restype = C.c_int
    lib.bsd_decode_ex.argtypes = [P, C.POINTER(Params), i64, P, P, P, P, P, C.POINTER(Stats), P]
    lib.bsd_code_autotune.restype = C.c_int
    lib.bsd_code_autotune.argtypes = [P, C.POINTER(Params), i64, P, i32p, i32p,
                                      C.POINTER(C.c_float), P]
    lib.bsd_server_create.restype = C.c_int
    lib.bsd_server_create.argtypes = [i32, C.POINTER(P), C.POINTER(Params), i32p, i64, C.POINTER(P)]
    lib.bsd_server_create_ex.restype = C.c_int
    lib.bsd_server_create_ex.argtypes = [i32, C.POINTER(P), C.POINTER(Params), i32p,
                                         C.POINTER(ServerOpts), C.POINTER(P)]
    lib.bsd_server_info.restype = C.c_int
    lib.bsd_server_info.argtypes = [P, i32, i32p, C.POINTER(i64)]
    lib.bsd_server_submit.restype = C.c_int
    lib.bsd_server_submit.argtypes = [P, i32, P, C.POINTER(i64)]
    lib.bsd_server_poll.restype = C.c_int
    lib.bsd_server_poll.argtypes = [P, i32, i64, P, P, P, C.POINTER(C.c_uint32)]
    lib.bsd_server_destroy.restype = C.c_int
    lib.bsd_server_destroy.argtypes = [P]
    lib.bsd_serve_poisson.restype = C.c_int
    lib.bsd_serve_poisson.argtypes = [P, C.c_double, C.POINTER(C.c_double), i64, C.POINTER(P),
                                      C.POINTER(i64), C.c_uint64, C.POINTER(P), C.POINTER(P),
                                      C.POINTER(P), C.POINTER(C.c_double), i32p,
                                      C.POINTER(ServeReport)]
    lib.bsd_unroll_sizes.restype = C.c_int
    lib.bsd_unroll_sizes.argtypes = [P, i32, i32, i64, C.POINTER(i64), C.POINTER(i64)]
    lib.bsd_unroll_forward.restype = C.c_int
    lib.bsd_unroll_forward.argtypes = [P, i32, i32, i32, i64, P, P, P, P, P, P]
    lib.bsd_unroll_backward.restype = C.c_int
    lib.bsd_unroll_backward.argtypes = [P, i32, i32, i32, i64, P, P, P, P, P, P, P, P, P]
    lib.bsd_unroll_backward_noalloc.restype = C.c_int
    lib.bsd_unroll_backward_noalloc.argtypes = [P, i32, i32, i32, i64, P, P, P, P, P, P, P, P]
    lib.bsd_bp_run.restype = C.c_int
    lib.bsd_bp_run.argtypes = [P, P, i32p, i32, P, i32, C.c_float, i32, P, P, P, i32p, i32p, i32p,
                               C.POINTER(C.c_float), P]
    _lib = lib
    return lib


def _check(rc: int):
    if rc != BSD_OK:
        raise BsdError(rc, load().bsd_last_error().decode())


def version() -> str:
    return load().bsd_version().decode()


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def make_params(max_rounds, beam_width, initial_iters, iters_per_round, num_results=1,
                alpha=0.625, mode=MODE_BATCHED, flags=0) -> Params:
    return Params(int(max_rounds), int(beam_width), int(initial_iters), int(iters_per_round),
                  int(num_results), float(alpha), int(mode), int(flags))


class Code:
    """A decoding problem (H, A, p) resident on the current HIP device."""

    def __init__(self, m, n, colptr, rowidx, p, L=None):
        self._lib = load()
        self.m, self.n = int(m), int(n)
        colptr, rowidx = _i32(colptr), _i32(rowidx)
        p = np.ascontiguousarray(p, dtype=np.float64)
        if L is None:
            L = np.zeros((0, self.n), np.uint8)
        L = np.asarray(L, dtype=np.uint8)
        self.k = int(L.shape[0])
        cols = [np.nonzero(L[:, j])[0] for j in range(self.n)]
        lptr = np.zeros(self.n + 1, np.int32)
        lptr[1:] = np.cumsum([len(c) for c in cols])
        lidx = np.concatenate(cols).astype(np.int32) if lptr[-1] else np.zeros(1, np.int32)
        h = C.c_void_p()
        i32p = C.POINTER(C.c_int32)
        rc = self._lib.bsd_code_create(
            self.m, self.n, self.k, colptr.ctypes.data_as(i32p), rowidx.ctypes.data_as(i32p),
            p.ctypes.data_as(C.POINTER(C.c_double)), lptr.ctypes.data_as(i32p),
            lidx.ctypes.data_as(i32p), C.byref(h))
        _check(rc)
        self._h = h
        self.nnz = int(colptr[-1])

    @classmethod
    def from_problem(cls, pr):
        return cls(pr.m, pr.n, pr.colptr, pr.rowidx, pr.p, pr.L)

    def info(self) -> dict:
        nnz, blk, grid, lds = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(self._lib.bsd_code_info(self._h, C.byref(nnz), C.byref(blk), C.byref(grid), C.byref(lds)))
        return {"nnz": nnz.value, "block": blk.value, "grid": grid.value, "lds_bytes": lds.value}

    def close(self):
        if getattr(self, "_h", None):
            _check(self._lib.bsd_code_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_alpha_schedule(self, alphas):
        """Per-iteration scalings used with FLAG_ALPHA_SCHEDULE (None clears)."""
        a = np.ascontiguousarray([] if alphas is None else alphas, dtype=np.float32)
        _check(self._lib.bsd_code_set_alpha_schedule(self._h, len(a),
                                                     a.ctypes.data_as(C.POINTER(C.c_float))))

    def decode(self, syndromes, params: Params, stream=None, latency=False, out=None, sync=True):
        """Decode a [shots, m] uint8 CUDA tensor; returns a dict of tensors and stats.
        With sync=False (batched mode) the call returns once the work is
        enqueued on `stream` (no stats); input errors are reported by sync()."""
        import torch
        syn = syndromes
        if syn.dtype != torch.uint8 or not syn.is_cuda or not syn.is_contiguous():
            raise ValueError("syndromes must be a contiguous uint8 CUDA tensor")
        shots = syn.shape[0] if syn.dim() == 2 else 0
        if syn.dim() != 2 or syn.shape[1] != self.m:
            raise ValueError(f"syndromes must have shape [shots, {self.m}]")
        dev = syn.device
        if out is None:
            out = {
                "corrections": torch.empty((shots, self.n), dtype=torch.uint8, device=dev),
                "flips": torch.empty((shots, max(self.k, 1)), dtype=torch.uint8, device=dev),
                "converged": torch.empty((shots,), dtype=torch.uint8, device=dev),
            }
        if not sync:
            if latency:
                raise ValueError("latencies need a synchronous call")
            _check(self._lib.bsd_decode(self._h, C.byref(params), shots, _ptr(syn),
                                        _ptr(out["corrections"]), _ptr(out["flips"]),
                                        _ptr(out["converged"]), _stream(stream)))
            res = dict(out)
            if self.k == 0:
                res["flips"] = res["flips"][:, :0]
            return res
        lat = torch.empty((shots,), dtype=torch.int32, device=dev) if latency else None
        st = Stats()
        rc = self._lib.bsd_decode_ex(self._h, C.byref(params), shots, _ptr(syn),
                                     _ptr(out["corrections"]), _ptr(out["flips"]),
                                     _ptr(out["converged"]), _stream(stream), C.byref(st),
                                     _ptr(lat))
        _check(rc)
        res = dict(out)
        if self.k == 0:
            res["flips"] = res["flips"][:, :0]
        res["stats"] = {f: getattr(st, f) for f, _ in Stats._fields_}
        if latency:
            res["latency_ticks"] = lat
        return res

    def sync(self, stream=None):
        """Wait for this code's work on `stream` and raise if an asynchronous
        call on it since the last check met bad input (bsd_code_sync)."""
        _check(self._lib.bsd_code_sync(self._h, _stream(stream)))

    def decode_host(self, syndromes, params: Params) -> dict:
        """Decode a host uint8 [shots, m] array; the library stages it
        through device memory (synchronous).  Returns numpy arrays and stats."""
        syn = np.ascontiguousarray(syndromes, dtype=np.uint8)
        if syn.ndim != 2 or syn.shape[1] != self.m:
            raise ValueError(f"syndromes must have shape [shots, {self.m}]")
        shots = syn.shape[0]
        corr = np.empty((shots, self.n), np.uint8)
        flips = np.empty((shots, max(self.k, 1)), np.uint8)
        conv = np.empty(shots, np.uint8)
        st = Stats()
        vp = lambda a: a.ctypes.data_as(C.c_void_p)
        _check(self._lib.bsd_decode_ex(self._h, C.byref(params), shots, vp(syn), vp(corr), vp(flips),
                                       vp(conv), None, C.byref(st), None))
        return {"corrections": corr, "flips": flips[:, :self.k], "converged": conv,
                "stats": {f: getattr(st, f) for f, _ in Stats._fields_}}

    def autotune(self, syndromes, params: Params, stream=None) -> dict:
        """Time the admissible launch geometries on `syndromes` and keep the fastest."""
        import torch
        if syndromes.dtype != torch.uint8 or not syndromes.is_cuda or syndromes.dim() != 2:
            raise ValueError("syndromes must be a [shots, m] uint8 CUDA tensor")
        blk, grid, ms = C.c_int32(), C.c_int32(), C.c_float()
        _check(self._lib.bsd_code_autotune(self._h, C.byref(params), syndromes.shape[0],
                                           _ptr(syndromes.contiguous()), C.byref(blk),
                                           C.byref(grid), C.byref(ms), _stream(stream)))
        return {"block": blk.value, "grid": grid.value, "ms": ms.value}

    def bp_run(self, syndrome, max_iters, alpha=0.625, e_start=None, pairs=(), stop=True,
               stream=None):
        """One masked BP run (Algorithm 2) on the GPU; messages in CSC edge order."""
        import torch
        if syndrome.dtype != torch.uint8 or not syndrome.is_cuda or syndrome.numel() != self.m:
            raise ValueError("syndrome must be a uint8 CUDA tensor with m entries")
        dev = syndrome.device
        if e_start is not None:
            if e_start.dtype != torch.float32 or not e_start.is_cuda or e_start.numel() != self.nnz:
                raise ValueError("e_start must be a float32 CUDA tensor with nnz entries")
            e_start = e_start.contiguous()
        pairs = list(pairs or [])
        parr = np.array([[int(c), int(v)] for c, v in pairs], dtype=np.int32).reshape(-1)
        e_out = torch.empty(self.nnz, dtype=torch.float32, device=dev)
        sl = torch.empty(self.n, dtype=torch.float32, device=dev)
        eh = torch.empty(self.n, dtype=torch.uint8, device=dev)
        it, cv, npos = C.c_int32(), C.c_int32(), C.c_int32()
        sc = C.c_float()
        pp = parr.ctypes.data_as(C.POINTER(C.c_int32)) if len(pairs) else None
        rc = self._lib.bsd_bp_run(self._h, _ptr(e_start), pp, len(pairs), _ptr(syndrome.contiguous()),
                                  int(max_iters), float(alpha), 1 if stop else 0, _ptr(e_out),
                                  _ptr(sl), _ptr(eh), C.byref(it), C.byref(cv), C.byref(npos),
                                  C.byref(sc), _stream(stream))
        _check(rc)
        return {"e": e_out, "sum_llr": sl, "ehat": eh, "iters": it.value,
                "converged": bool(cv.value), "next_pos": npos.value, "score": sc.value}


class Server:
    """Persistent GPU decoders for several resident codes, fed continuously
    (bsd_server_*).  Codes must outlive the server."""

    def __init__(self, codes, params, grid_blocks=None, ring_bytes=0, idle_ms=0):
        self._lib = load()
        self.codes = list(codes)
        n = len(self.codes)
        hs = (C.c_void_p * n)(*[c._h for c in self.codes])
        prm = (Params * n)(*params)
        grid = (C.c_int32 * n)(*(grid_blocks or [0] * n))
        h = C.c_void_p()
        opts = ServerOpts(int(ring_bytes), int(idle_ms))
        _check(self._lib.bsd_server_create_ex(n, hs, prm, grid, C.byref(opts), C.byref(h)))
        self._h = h

    def info(self, code: int) -> dict:
        """Whether the code's decoder kernel is running, and its launch count."""
        running, launches = C.c_int32(), C.c_int64()
        _check(self._lib.bsd_server_info(self._h, int(code), C.byref(running), C.byref(launches)))
        return {"running": bool(running.value), "launches": launches.value}

    def submit(self, code: int, syndrome) -> int | None:
        """Submit a host uint8 [m] syndrome; returns its ticket, or None when
        the code's ring is full."""
        syn = np.ascontiguousarray(syndrome, dtype=np.uint8)
        t = C.c_int64()
        rc = self._lib.bsd_server_submit(self._h, int(code), syn.ctypes.data_as(C.c_void_p), C.byref(t))
        if rc == BSD_EBUSY:
            return None
        _check(rc)
        return t.value

    def poll(self, code: int, ticket: int):
        """Outputs of a finished request (dict) or None if it is still running."""
        c = self.codes[code]
        corr = np.empty(c.n, np.uint8)
        flips = np.empty(max(c.k, 1), np.uint8)
        conv = np.empty(1, np.uint8)
        ticks = C.c_uint32()
        rc = self._lib.bsd_server_poll(self._h, int(code), int(ticket), corr.ctypes.data_as(C.c_void_p),
                                       flips.ctypes.data_as(C.c_void_p), conv.ctypes.data_as(C.c_void_p),
                                       C.byref(ticks))
        if rc == BSD_EBUSY:
            return None
        _check(rc)
        return {"corrections": corr, "flips": flips[:c.k], "converged": int(conv[0]),
                "device_ticks": ticks.value}

    def serve_poisson(self, rate, mix, requests, syndromes, seed=0):
        """Poisson arrivals over the codes (see bsd_serve_poisson); returns the
        per-syndrome outputs of every code, per-request latencies and the report."""
        n = len(self.codes)
        syns = [np.ascontiguousarray(s_, dtype=np.uint8) for s_ in syndromes]
        corr = [np.zeros((len(s_), c.n), np.uint8) for s_, c in zip(syns, self.codes)]
        flips = [np.zeros((len(s_), max(c.k, 1)), np.uint8) for s_, c in zip(syns, self.codes)]
        conv = [np.zeros(len(s_), np.uint8) for s_ in syns]
        lat = np.zeros(int(requests), np.float64)
        code_of = np.zeros(int(requests), np.int32)
        rep = ServeReport()
        arr = lambda xs: (C.c_void_p * n)(*[x.ctypes.data_as(C.c_void_p) for x in xs])
        _check(self._lib.bsd_serve_poisson(
            self._h, float(rate), (C.c_double * n)(*mix), int(requests), arr(syns),
            (C.c_int64 * n)(*[len(s_) for s_ in syns]), int(seed), arr(corr), arr(flips), arr(conv),
            lat.ctypes.data_as(C.POINTER(C.c_double)), code_of.ctypes.data_as(C.POINTER(C.c_int32)),
            C.byref(rep)))
        report = {f: getattr(rep, f) for f, _ in ServeReport._fields_ if not f.startswith("code_")}
        report["per_code"] = [{"requests": rep.code_requests[i], "p50_us": rep.code_p50_us[i],
                               "p99_us": rep.code_p99_us[i], "p999_us": rep.code_p999_us[i]}
                              for i in range(n)]
        outs = [{"corrections": corr[i], "flips": flips[i][:, :self.codes[i].k], "converged": conv[i]}
                for i in range(n)]
        return outs, lat, code_of, report

    def close(self):
        if getattr(self, "_h", None):
            _check(self._lib.bsd_server_destroy(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _unrolled_function():
    import torch

    class UnrolledMinSum(torch.autograd.Function):
        """post(T) of unrolled min-sum (bsd_unroll_forward) with the
        hand-written adjoint (bsd_unroll_backward) as its backward."""

        @staticmethod
        def forward(ctx, lam, alpha, syndromes, code, K):
            lib = load()
            if lam.dtype not in (torch.float32, torch.float64) or alpha.dtype != lam.dtype:
                raise ValueError("lam and alpha must share a float32 or float64 dtype")
            if not (lam.is_cuda and alpha.is_cuda and syndromes.is_cuda):
                raise ValueError("lam, alpha and syndromes must be CUDA tensors")
            lam, alpha = lam.contiguous(), alpha.contiguous()
            syn = syndromes.contiguous()
            if syn.dtype != torch.uint8 or syn.dim() != 2 or syn.shape[1] != code.m:
                raise ValueError(f"syndromes must be uint8 [shots, {code.m}]")
            shots, T = syn.shape[0], alpha.numel()
            ck_n, ws_n = C.c_int64(), C.c_int64()
            _check(lib.bsd_unroll_sizes(code._h, T, int(K), shots, C.byref(ck_n), C.byref(ws_n)))
            post = torch.empty((shots, code.n), dtype=lam.dtype, device=lam.device)
            ck = torch.empty(max(ck_n.value, 1), dtype=lam.dtype, device=lam.device)
            _check(lib.bsd_unroll_forward(code._h, lam.element_size(), T, int(K), shots, _ptr(syn),
                                          _ptr(lam), _ptr(alpha), _ptr(post), _ptr(ck), _stream(None)))
            ctx.save_for_backward(lam, alpha, syn, ck)
            ctx.code, ctx.K, ctx.ws_n = code, int(K), ws_n.value
            return post

        @staticmethod
        def backward(ctx, grad_post):
            lib = load()
            lam, alpha, syn, ck = ctx.saved_tensors
            code = ctx.code
            g = grad_post.contiguous().to(lam.dtype)
            gl = torch.empty_like(lam)
            ga = torch.empty_like(alpha)
            ws = torch.empty(max(ctx.ws_n, 1), dtype=lam.dtype, device=lam.device)
            _check(lib.bsd_unroll_backward(code._h, lam.element_size(), alpha.numel(), ctx.K,
                                           syn.shape[0], _ptr(syn), _ptr(lam), _ptr(alpha), _ptr(ck),
                                           _ptr(g), _ptr(gl), _ptr(ga), _ptr(ws), _stream(None)))
            return gl, ga, None, None, None

    return UnrolledMinSum


def unrolled_minsum(code: "Code", lam, alpha, syndromes, K: int = 5):
    """Differentiable post(T) [shots, n] of T = len(alpha) flooding min-sum
    iterations with per-iteration scaling alpha and priors lam (CUDA tensors,
    float32 or float64); checkpoints every K iterations."""
    global _UNROLLED
    if _UNROLLED is None:
        _UNROLLED = _unrolled_function()
    return _UNROLLED.apply(lam, alpha, syndromes, code, K)


_UNROLLED = None
