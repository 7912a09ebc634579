"""ctypes binding of libcpr (argument marshalling only).

Names follow the C ABI of include/cpr.h with the `cp_` prefix dropped.
Device buffers are torch CUDA (HIP) tensors; their data pointers are passed
straight through.  Every call checks the returned cp_status and raises
CprError with the library's message.
"""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcpr.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "cpr.h")

SAMPLERS = {"arls": 0, "sts": 1, "exact": 2}
PRECISIONS = {"fp64": 0, "fp32": 1, "mixed": 2}
PHASES = ["pinv", "sample", "merge", "mttkrp", "solve", "gram",
          "sampler_build", "fit"]
STATUS = {0: "CP_OK", -1: "CP_EINVAL", -2: "CP_ENOMEM", -3: "CP_EHIP",
          -4: "CP_ESTATE", -5: "CP_EDEGENERATE", -6: "CP_ENUMERIC",
          -7: "CP_EUNSUPPORTED"}


class CprError(RuntimeError):
    def __init__(self, status, msg):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__(f"{self.name}: {msg}")


class _Tensor(C.Structure):
    _fields_ = [("N", C.c_int32), ("dims", C.POINTER(C.c_int64)),
                ("nnz", C.c_int64), ("idx", C.c_void_p), ("val", C.c_void_p),
                ("val_is_fp64", C.c_int32)]


def _refine_code(refine):
    """cp_solve_refine: None -> automatic (by precision), True / False."""
    return 0 if refine is None else (1 if refine else 2)


class _Config(C.Structure):
    _fields_ = [("R", C.c_int32), ("sampler", C.c_int32),
                ("precision", C.c_int32), ("sts_leaf", C.c_int32),
                ("max_J", C.c_int64), ("bucket_rows", C.c_int32),
                ("solve_gram", C.c_int32), ("solve_refine", C.c_int32)]


_lib = None


def declared_symbols(header=HEADER):
    """Function names declared in include/cpr.h."""
    with open(header) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cp_[a-z_0-9]+)\s*\(", text)))


def load_library(path=None):
    """Load libcpr.so (built by paper_2210_05105_amd.build; another build
    of it if the CPR_LIBRARY environment variable names one); raise if
    absent."""
    global _lib
    if path is None:
        path = os.environ.get("CPR_LIBRARY") or LIB_PATH
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python -m "
            f"paper_2210_05105_amd.build` (there is no CPU fallback)")
    lib = C.CDLL(path)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "cp_init": [C.POINTER(_Tensor), C.POINTER(_Config), P, C.POINTER(P)],
        "cp_set_factor": [P, I32, P],
        "cp_set_sigma": [P, P],
        "cp_sample": [P, I32, I64, P, P, P],
        "cp_set_samples": [P, I32, I64, P, P],
        "cp_sampled_mttkrp": [P, I32, P, C.POINTER(I64)],
        "cp_solve_factor": [P, I32],
        "cp_sweep": [P, I32, I64, P],
        "cp_fit": [P, C.POINTER(D)],
        "cp_sync": [P],
        "cp_get_factor": [P, I32, P],
        "cp_get_sigma": [P, P],
        "cp_get_gram": [P, I32, P],
        "cp_get_unique": [P, P, P, P, P, I64, C.POINTER(I64)],
        "cp_get_extracted": [P, P, P, P, I64, C.POINTER(I64)],
        "cp_profile": [P, I32],
        "cp_profile_phases": [P, C.c_uint32],
        "cp_profile_read": [P, P, P],
        "cp_index_stats": [P, I32, C.POINTER(I64), C.POINTER(I64)],
        "cp_sts_leaf": [P, I32, C.POINTER(I32), C.POINTER(I64)],
        "cp_counters": [P, P, I32],
        "cp_pinv": [P, I32, P, P],
        "cp_batch_init": [C.POINTER(_Tensor), I32, P, C.POINTER(_Config),
                          I32, P, C.POINTER(P)],
        "cp_batch_set_factors": [P, I32, I32, P],
        "cp_batch_sweep": [P, P],
        "cp_batch_fit": [P, P],
        "cp_batch_sync": [P],
        "cp_batch_get_factor": [P, I32, I32, P],
        "cp_batch_get_sigma": [P, I32, P],
        "cp_pinv_noalloc": [P, I32, P, P],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.cp_destroy.argtypes = [P]
    lib.cp_destroy.restype = None
    lib.cp_last_error.argtypes = [P]
    lib.cp_last_error.restype = C.c_char_p
    lib.cp_status_string.argtypes = [C.c_int]
    lib.cp_status_string.restype = C.c_char_p
    lib.cp_phase_name.argtypes = [I32]
    lib.cp_phase_name.restype = C.c_char_p
    lib.cp_batch_destroy.argtypes = [P]
    lib.cp_batch_destroy.restype = None
    lib.cp_batch_last_error.argtypes = [P]
    lib.cp_batch_last_error.restype = C.c_char_p
    lib.cp_batch_stream_of.argtypes = [P, I32]
    lib.cp_batch_stream_of.restype = I32
    _lib = lib
    return lib


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def pinv(G, stream=None):
    """Pseudo-inverse of a symmetric PSD matrix (torch FP64 CUDA tensor)."""
    import torch
    lib = load_library()
    G = G.to(torch.float64).contiguous()
    R = G.shape[0]
    assert G.shape == (R, R) and G.is_cuda
    out = torch.empty_like(G)
    s = stream if stream is not None else torch.cuda.current_stream(G.device)
    st = lib.cp_pinv(_ptr(G), R, _ptr(out), C.c_void_p(s.cuda_stream))
    if st != 0:
        raise CprError(st, "cp_pinv failed")
    return out


def pinv_noalloc(G, out, stream=None):
    """cp_pinv_noalloc: pseudo-inverse into the caller's `out` (same shape,
    FP64 CUDA); the library allocates nothing."""
    import torch
    lib = load_library()
    R = G.shape[0]
    assert G.dtype == torch.float64 and G.is_contiguous() and G.is_cuda
    assert out.dtype == torch.float64 and out.is_contiguous()
    assert G.shape == (R, R) and out.shape == (R, R)
    s = stream if stream is not None else torch.cuda.current_stream(G.device)
    st = lib.cp_pinv_noalloc(_ptr(G), R, _ptr(out), C.c_void_p(s.cuda_stream))
    if st != 0:
        raise CprError(st, "cp_pinv_noalloc failed")
    return out


class Context:
    """One decomposition problem: per-mode indices, factors, sampler state.

    idx: torch.int32 CUDA tensor [nnz, N]; val: float32/float64 CUDA [nnz];
    dims: sequence of N ints.  sampler in SAMPLERS, precision in PRECISIONS.
    """

    def __init__(self, idx, val, dims, R, sampler="arls", precision="fp64",
                 max_J=1, sts_leaf=0, stream=None, bucket_rows=0,
                 sketched=False, refine=None):
        import torch
        self._torch = torch
        lib = load_library()
        self.lib = lib
        self.N = len(dims)
        self.dims = [int(d) for d in dims]
        self.R = int(R)
        self.sampler = sampler
        self.precision = precision
        self.device = idx.device
        assert idx.dtype == torch.int32 and idx.is_contiguous()
        assert idx.shape == (val.shape[0], self.N) and val.is_contiguous()
        assert val.dtype in (torch.float32, torch.float64)
        self.stream = stream if stream is not None else \
            torch.cuda.current_stream(self.device)
        d = (C.c_int64 * self.N)(*self.dims)
        t = _Tensor(self.N, d, int(val.shape[0]), idx.data_ptr(),
                    val.data_ptr(), int(val.dtype == torch.float64))
        cfg = _Config(self.R, SAMPLERS[sampler], PRECISIONS[precision],
                      int(sts_leaf), int(max_J), int(bucket_rows),
                      int(bool(sketched)), _refine_code(refine))
        h = C.c_void_p()
        st = lib.cp_init(C.byref(t), C.byref(cfg),
                         C.c_void_p(self.stream.cuda_stream), C.byref(h))
        self._h = h
        if st != 0:
            msg = lib.cp_last_error(h).decode() if h else "invalid arguments"
            if h:
                lib.cp_destroy(h)
            self._h = None
            raise CprError(st, msg)
        self.fdtype = torch.float64 if precision == "fp64" else torch.float32

    # ------------------------------------------------------------ helpers
    def _check(self, st):
        if st != 0:
            raise CprError(st, self.lib.cp_last_error(self._h).decode())

    def _dev(self, shape, dtype):
        return self._torch.empty(shape, dtype=dtype, device=self.device)

    def close(self):
        if getattr(self, "_h", None):
            self.lib.cp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- API
    def set_factor(self, mode, U):
        U = U.to(device=self.device, dtype=self._torch.float64).contiguous()
        assert U.shape == (self.dims[mode], self.R)
        self._keep = U
        self._check(self.lib.cp_set_factor(self._h, mode, _ptr(U)))

    def set_sigma(self, sigma):
        s = sigma.to(device=self.device, dtype=self._torch.float64).contiguous()
        self._keep = s
        self._check(self.lib.cp_set_sigma(self._h, _ptr(s)))

    def sample(self, mode, uniforms, outputs=True):
        u = uniforms.to(device=self.device, dtype=self._torch.float64).contiguous()
        J = u.shape[0]
        assert u.shape == (J, self.N - 1)
        self._keep = u
        idx = self._dev((J, self.N - 1), self._torch.int32) if outputs else None
        prob = self._dev((J,), self._torch.float64) if outputs else None
        self._check(self.lib.cp_sample(self._h, mode, J, _ptr(u), _ptr(idx),
                                       _ptr(prob)))
        return idx, prob

    def set_samples(self, mode, idx, prob):
        i = idx.to(device=self.device, dtype=self._torch.int32).contiguous()
        p = prob.to(device=self.device, dtype=self._torch.float64).contiguous()
        self._keep = (i, p)
        self._check(self.lib.cp_set_samples(self._h, mode, i.shape[0], _ptr(i),
                                            _ptr(p)))

    def sampled_mttkrp(self, mode, want_M=True, want_nnz=False):
        M = self._dev((self.dims[mode], self.R), self.fdtype) if want_M else None
        n = C.c_int64(0)
        self._check(self.lib.cp_sampled_mttkrp(
            self._h, mode, _ptr(M), C.byref(n) if want_nnz else None))
        return M, (n.value if want_nnz else None)

    def solve_factor(self, mode):
        self._check(self.lib.cp_solve_factor(self._h, mode))

    def sweep(self, nsweeps, J=0, uniforms=None):
        u = None
        if uniforms is not None:
            u = uniforms.to(device=self.device,
                            dtype=self._torch.float64).contiguous()
        self._keep = u
        self._check(self.lib.cp_sweep(self._h, nsweeps, J, _ptr(u)))

    def fit(self):
        f = C.c_double(0)
        self._check(self.lib.cp_fit(self._h, C.byref(f)))
        return f.value

    def sync(self):
        self._check(self.lib.cp_sync(self._h))

    def get_factor(self, mode):
        out = self._dev((self.dims[mode], self.R), self._torch.float64)
        self._check(self.lib.cp_get_factor(self._h, mode, _ptr(out)))
        return out

    def get_sigma(self):
        out = self._dev((self.R,), self._torch.float64)
        self._check(self.lib.cp_get_sigma(self._h, _ptr(out)))
        return out

    def get_gram(self, mode):
        out = self._dev((self.R, self.R), self._torch.float64)
        self._check(self.lib.cp_get_gram(self._h, mode, _ptr(out)))
        return out

    def get_unique(self, cap):
        t = self._torch
        ck = self._dev((cap,), t.int64)
        rep = self._dev((cap,), t.int32)
        cnt = self._dev((cap,), t.int32)
        w = self._dev((cap,), t.float64)
        n = C.c_int64(0)
        self._check(self.lib.cp_get_unique(self._h, _ptr(ck), _ptr(rep),
                                           _ptr(cnt), _ptr(w), cap,
                                           C.byref(n)))
        k = min(n.value, cap)
        return dict(col_key=ck[:k], rep=rep[:k], count=cnt[:k], weight=w[:k],
                    n=n.value)

    def get_extracted(self, cap):
        t = self._torch
        ck = self._dev((max(cap, 1),), t.int64)
        row = self._dev((max(cap, 1),), t.int32)
        rep = self._dev((max(cap, 1),), t.int32)
        n = C.c_int64(0)
        self._check(self.lib.cp_get_extracted(self._h, _ptr(ck), _ptr(row),
                                              _ptr(rep), cap, C.byref(n)))
        k = min(n.value, cap)
        return dict(col_key=ck[:k], row=row[:k], rep=rep[:k], n=n.value)

    def profile(self, enable=True, phases=None):
        """Per-phase HIP-event timing; phases: names to time (default all)."""
        if phases is None or not enable:
            self._check(self.lib.cp_profile(self._h, int(bool(enable))))
        else:
            mask = 0
            for name in phases:
                mask |= 1 << PHASES.index(name)
            self._check(self.lib.cp_profile_phases(self._h, mask))

    def profile_read(self):
        ms = (C.c_double * 8)()
        nl = (C.c_int64 * 8)()
        self._check(self.lib.cp_profile_read(self._h, ms, nl))
        return {PHASES[p]: (ms[p], nl[p]) for p in range(8)}

    def counters(self, reset=False):
        out = (C.c_int64 * 4)()
        self._check(self.lib.cp_counters(self._h, out, int(bool(reset))))
        return dict(solves=out[0], unique=out[1], nnz=out[2], rows=out[3])

    def index_stats(self, mode):
        a, b = C.c_int64(0), C.c_int64(0)
        self._check(self.lib.cp_index_stats(self._h, mode, C.byref(a),
                                            C.byref(b)))
        return a.value, b.value

    def sts_leaf(self, mode):
        """(rows per leaf, leaves) of mode's STS-CP tree; (0, 0) if none."""
        f, n = C.c_int32(0), C.c_int64(0)
        self._check(self.lib.cp_sts_leaf(self._h, mode, C.byref(f),
                                         C.byref(n)))
        return f.value, n.value


class Batch:
    """Batched restarts of one tensor (cp_batch_*): ranks[b] per restart,
    a shared index, one captured HIP graph per sweep."""

    def __init__(self, idx, val, dims, ranks, sampler="arls",
                 precision="fp64", J=1, sts_leaf=0, nstreams=0, stream=None,
                 bucket_rows=0, refine=None):
        import torch
        self._torch = torch
        lib = load_library()
        self.lib = lib
        self.N = len(dims)
        self.dims = [int(d) for d in dims]
        self.ranks = [int(r) for r in ranks]
        self.B = len(self.ranks)
        self.J = int(J)
        self.device = idx.device
        assert idx.dtype == torch.int32 and idx.is_contiguous()
        assert idx.shape == (val.shape[0], self.N) and val.is_contiguous()
        self.stream = stream if stream is not None else \
            torch.cuda.current_stream(self.device)
        d = (C.c_int64 * self.N)(*self.dims)
        t = _Tensor(self.N, d, int(val.shape[0]), idx.data_ptr(),
                    val.data_ptr(), int(val.dtype == torch.float64))
        cfg = _Config(0, SAMPLERS[sampler], PRECISIONS[precision],
                      int(sts_leaf), self.J, int(bucket_rows), 0,
                      _refine_code(refine))
        rk = (C.c_int32 * self.B)(*self.ranks)
        h = C.c_void_p()
        st = lib.cp_batch_init(C.byref(t), self.B, rk, C.byref(cfg),
                               int(nstreams),
                               C.c_void_p(self.stream.cuda_stream),
                               C.byref(h))
        self._h = h
        if st != 0:
            msg = lib.cp_batch_last_error(h).decode() if h else "invalid arguments"
            if h:
                lib.cp_batch_destroy(h)
            self._h = None
            raise CprError(st, msg)
        self._uni = None

    def _check(self, st):
        if st != 0:
            raise CprError(st, self.lib.cp_batch_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self.lib.cp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_factor(self, b, mode, U):
        U = U.to(device=self.device, dtype=self._torch.float64).contiguous()
        assert U.shape == (self.dims[mode], self.ranks[b])
        self._keep = U
        self._check(self.lib.cp_batch_set_factors(self._h, b, mode, _ptr(U)))

    def sweep(self, uniforms):
        """uniforms: [B, N, J, N-1] FP64; kept by the batch (the captured
        graph reads this buffer at every replay)."""
        u = uniforms
        assert u.dtype == self._torch.float64 and u.is_contiguous()
        assert tuple(u.shape) == (self.B, self.N, self.J, self.N - 1)
        self._uni = u
        self._check(self.lib.cp_batch_sweep(self._h, _ptr(u)))

    def fit(self):
        out = (C.c_double * self.B)()
        self._check(self.lib.cp_batch_fit(self._h, out))
        return list(out)

    def sync(self):
        self._check(self.lib.cp_batch_sync(self._h))

    def get_factor(self, b, mode):
        out = self._torch.empty((self.dims[mode], self.ranks[b]),
                                dtype=self._torch.float64, device=self.device)
        self._check(self.lib.cp_batch_get_factor(self._h, b, mode, _ptr(out)))
        return out

    def get_sigma(self, b):
        out = self._torch.empty((self.ranks[b],), dtype=self._torch.float64,
                                device=self.device)
        self._check(self.lib.cp_batch_get_sigma(self._h, b, _ptr(out)))
        return out

    def stream_of(self, b):
        return self.lib.cp_batch_stream_of(self._h, b)
