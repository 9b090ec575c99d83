"""sFFT-DT (arXiv 1407.8315) on MI355X: a thin Python binding over libsft.so.

Every step of the path (downsampling, FFTs, syndrome decoding, CS recovery,
output) runs in the HIP library; this module only marshals arguments.  torch
supplies device memory and the stream.

    plan = Plan(dict(n=1 << 20, k=1000, m=4096, l=4))        # exact mode
    res = plan.exact(x)            # x: complex64 CUDA tensor of length n
    res.loc, res.val               # sorted locations, complex128 values
"""
from __future__ import annotations

import ctypes
import dataclasses

from . import _lib
from ._lib import (  # noqa: F401
    SFT_C64, SFT_C128, SFT_MODE_EXACT, SFT_MODE_GENERAL, SFT_MODE_ITERATIVE,
    SFT_FLAG_LEARNED, SFT_FLAG_SYNC, SFT_FLAG_CHECK_FINITE, SFT_FLAG_AUTOTUNE, SFT_FLAG_FFT64, SFT_FLAG_SP_ALL, SFT_FLAG_UNKNOWN_K,
    SftError,
)

__all__ = ["Plan", "Result", "SftError", "Mlp", "make_params", "library_path", "autotune", "exact_noalloc"]


def library_path() -> str:
    return _lib.LIB_PATH


def autotune(n, k, dtype="c64", target=0.0):
    """(M, L, expected recovery, modelled microseconds) chosen for an exact-mode
    signal of length n with k frequencies (host only; see sft_autotune)."""
    lib = _lib.load()
    m, l = ctypes.c_int64(), ctypes.c_int32()
    rec, us = ctypes.c_double(), ctypes.c_double()
    _lib.check(lib.sft_autotune(int(n), int(k), {"c64": SFT_C64, "c128": SFT_C128}[dtype], float(target),
                                ctypes.byref(m), ctypes.byref(l), ctypes.byref(rec), ctypes.byref(us)),
               "sft_autotune")
    return int(m.value), int(l.value), float(rec.value), float(us.value)


def exact_noalloc(x, params: dict, out: "Result", capacity=None, stream=None) -> "Result":
    """sft_exact_noalloc: exact-mode recovery of one signal without a plan
    (the library's static workspace; no device allocation by the library).
    x: contiguous CUDA tensor of params["n"] elements of params' dtype; out: a
    Result the caller allocated (Plan.new_output or equal tensors).
    Asynchronous on `stream` (default: torch's current stream)."""
    torch = _torch()
    lib = _lib.load()
    p = make_params(**params)
    want = torch.complex128 if p.in_dtype == SFT_C128 else torch.complex64
    if not x.is_cuda or x.dtype != want or x.numel() != p.n or not x.is_contiguous():
        raise ValueError(f"need a contiguous {want} CUDA tensor of {p.n} elements")
    if capacity is None:
        capacity = out.loc.numel()
    if stream is None:
        stream = torch.cuda.current_stream()
    o = Plan._out_struct(out, capacity)
    _lib.check(lib.sft_exact_noalloc(ctypes.byref(p), ctypes.c_void_p(x.data_ptr()), ctypes.byref(o),
                                     ctypes.c_void_p(stream.cuda_stream)), "sft_exact_noalloc")
    return out


def make_params(n, k, m=0, l=0, r=0, dtype="c64", mode="exact", flags=0, seed=0, target_recovery=0.0,
                **taus) -> _lib.Params:
    p = _lib.Params()
    p.n, p.k, p.m, p.l, p.r = int(n), int(k), int(m), int(l), int(r)
    p.in_dtype = {"c64": SFT_C64, "c128": SFT_C128}[dtype]
    p.mode = {"exact": SFT_MODE_EXACT, "general": SFT_MODE_GENERAL, "iterative": SFT_MODE_ITERATIVE}[mode]
    p.flags = int(flags)
    p.reserved = 0
    p.seed = int(seed) & ((1 << 64) - 1)
    p.target_recovery = float(target_recovery)
    for name in ("tau_zero", "tau_rank", "tau_res", "tau_amp", "c_res", "delta_grid", "delta_mag"):
        setattr(p, name, float(taus.pop(name, 0.0)))
    if taus:
        raise TypeError(f"unknown parameters {sorted(taus)}")
    return p


@dataclasses.dataclass
class Result:
    loc: object          # torch int64 [capacity] (device)
    val: object          # torch complex128 [capacity] (device)
    count: object        # torch int64 [1] (device)
    stats: dict | None = None

    def host(self):
        """(locations, values) as numpy arrays, trimmed to the count."""
        n = int(self.count.item())
        n = min(n, self.loc.numel())
        return self.loc[:n].cpu().numpy(), self.val[:n].cpu().numpy()


def _torch():
    import torch
    return torch


class Plan:
    """A plan for one signal (sft_exact / sft_general) or a batch (sft_batch).

    params: a dict (or list of dicts) with keys n, k, m, l, r, dtype ("c64" or
    "c128"), mode ("exact" or "general"), flags, seed and thresholds.  The
    plan is bound to `stream` (default: torch's current stream)."""

    def __init__(self, params, stream=None):
        torch = _torch()
        self._lib = _lib.load()
        plist = params if isinstance(params, (list, tuple)) else [params]
        arr = (_lib.Params * len(plist))(*[make_params(**p) if isinstance(p, dict) else p for p in plist])
        self.n_signals = len(plist)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        handle = ctypes.c_void_p()
        _lib.check(self._lib.sft_plan(ctypes.byref(handle), arr, len(plist), ctypes.c_void_p(stream.cuda_stream)),
                   "sft_plan")
        self._h = handle
        self.infos = [self.info(i) for i in range(self.n_signals)]

    # ------------------------------------------------------------ info
    def info(self, i: int = 0) -> dict:
        inf = _lib.PlanInfo()
        _lib.check(self._lib.sft_plan_get(self._h, i, ctypes.byref(inf)), "sft_plan_get")
        d = {f: getattr(inf, f) for f, _ in _lib.PlanInfo._fields_ if f != "rshifts"}
        d["rshifts"] = [inf.rshifts[j] for j in range(inf.r)]
        return d

    # ------------------------------------------------------------ outputs
    def new_output(self, capacity: int, device=None):
        torch = _torch()
        device = device or torch.device("cuda", torch.cuda.current_device())
        loc = torch.empty(max(capacity, 1), dtype=torch.int64, device=device)
        val = torch.empty(max(capacity, 1), dtype=torch.complex128, device=device)
        cnt = torch.zeros(1, dtype=torch.int64, device=device)
        return Result(loc, val, cnt)

    @staticmethod
    def _out_struct(res: Result, capacity: int) -> _lib.SparseOut:
        o = _lib.SparseOut()
        o.loc_dev = res.loc.data_ptr()
        o.val_dev = res.val.data_ptr()
        o.capacity = int(capacity)
        o.count_dev = res.count.data_ptr()
        return o

    def default_capacity(self, i: int = 0) -> int:
        inf = self.infos[i]
        return int(inf["m"] * inf["l"])

    def _check_input(self, x, i=0):
        torch = _torch()
        inf = self.infos[i]
        want = torch.complex128 if inf["in_dtype"] == SFT_C128 else torch.complex64
        if not x.is_cuda or x.dtype != want or x.numel() != inf["n"] or not x.is_contiguous():
            raise ValueError(f"signal {i}: need a contiguous {want} CUDA tensor of {inf['n']} elements")

    # ------------------------------------------------------------ calls
    def _single(self, fn, x, out, capacity, stats):
        self._check_input(x)
        if capacity is None:
            capacity = self.default_capacity()
        if out is None:
            out = self.new_output(capacity, x.device)
        o = self._out_struct(out, capacity)
        st = _lib.Stats() if stats else None
        status = fn(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.byref(o),
                    ctypes.byref(st) if st is not None else None)
        if st is not None:
            out.stats = st.as_dict()
        if status == _lib.SFT_E_CAPACITY:
            out.stats = (out.stats or {}) | {"capacity_exceeded": True}
            return out
        _lib.check(status, fn.__name__)
        return out

    def exact(self, x, out: Result | None = None, capacity=None, stats=False) -> Result:
        return self._single(self._lib.sft_exact, x, out, capacity, stats)

    def general(self, x, out: Result | None = None, capacity=None, stats=False) -> Result:
        return self._single(self._lib.sft_general, x, out, capacity, stats)

    def iterative(self, x, out: Result | None = None, capacity=None, stats=False) -> Result:
        """Iterative sFFT-DT (Alg. 1) on a single-signal plan in mode "iterative"."""
        return self._single(self._lib.sft_iterative, x, out, capacity, stats)

    def unknown_k(self, x, out: Result | None = None, capacity=None, stats=False):
        """K unknown (Sec. II-G) on a plan made with SFT_FLAG_UNKNOWN_K: returns
        (result, M) of the first rung M = 1, 2, 4 .. that flags no bin."""
        self._check_input(x)
        if capacity is None:
            capacity = self.default_capacity()
        if out is None:
            out = self.new_output(capacity, x.device)
        o = self._out_struct(out, capacity)
        st = _lib.Stats()
        m = ctypes.c_int64(0)
        status = self._lib.sft_unknown_k(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.byref(o), ctypes.byref(st),
                                         ctypes.byref(m))
        if status != _lib.SFT_E_CAPACITY:
            _lib.check(status, "sft_unknown_k")
        out.stats = st.as_dict() if stats else None
        return out, int(m.value)

    def batch(self, xs, outs=None, capacities=None, stats=False):
        if len(xs) != self.n_signals:
            raise ValueError(f"expected {self.n_signals} signals")
        for i, x in enumerate(xs):
            self._check_input(x, i)
        if capacities is None:
            capacities = [self.default_capacity(i) for i in range(self.n_signals)]
        if outs is None:
            outs = [self.new_output(c, xs[0].device) for c in capacities]
        xarr = (ctypes.c_void_p * len(xs))(*[x.data_ptr() for x in xs])
        oarr = (_lib.SparseOut * len(xs))(*[self._out_struct(o, c) for o, c in zip(outs, capacities)])
        st = _lib.Stats() if stats else None
        status = self._lib.sft_batch(self._h, xarr, oarr, ctypes.byref(st) if st is not None else None)
        if status != _lib.SFT_E_CAPACITY:
            _lib.check(status, "sft_batch")
        if st is not None:
            d = st.as_dict()
            for o in outs:
                o.stats = d
        self._keep = (xarr, oarr)      # keep the argument arrays alive until the next call
        return outs

    def prepare_batch(self, xs, outs, capacities=None):
        """Bind fixed inputs and outputs once; returns run(stats=False), which
        calls sft_batch on them (no per-call argument marshalling: for timing
        loops over large batches)."""
        if len(xs) != self.n_signals:
            raise ValueError(f"expected {self.n_signals} signals")
        for i, x in enumerate(xs):
            self._check_input(x, i)
        if capacities is None:
            capacities = [self.default_capacity(i) for i in range(self.n_signals)]
        xarr = (ctypes.c_void_p * len(xs))(*[x.data_ptr() for x in xs])
        oarr = (_lib.SparseOut * len(xs))(*[self._out_struct(o, c) for o, c in zip(outs, capacities)])
        keep = (xs, outs, xarr, oarr)

        def run(stats=False):
            st = _lib.Stats() if stats else None
            status = self._lib.sft_batch(self._h, keep[2], keep[3], ctypes.byref(st) if st is not None else None)
            if status != _lib.SFT_E_CAPACITY:
                _lib.check(status, "sft_batch")
            return st.as_dict() if st is not None else None

        return run

    def syndromes(self, x):
        """Steps 1-2 only: the [S, M] syndromes of a single-signal plan (device
        tensor).  Iterative plans: a list over the iterations l of [2, M_0 / 2^l]
        (shifts 2l and 2l + 1 on that iteration's grid)."""
        torch = _torch()
        self._check_input(x)
        inf = self.infos[0]
        fft64 = inf["in_dtype"] == SFT_C128 or (inf["flags"] & SFT_FLAG_FFT64)
        dt = torch.complex128 if fft64 else torch.complex64
        if inf["mode"] == SFT_MODE_ITERATIVE:
            sizes = [inf["m"] >> l for l in range(inf["l"])]
            out = torch.empty(2 * sum(sizes), dtype=dt, device=x.device)
        else:
            out = torch.empty((2 * inf["l"] + inf["r"], inf["m"]), dtype=dt, device=x.device)
        _lib.check(self._lib.sft_syndromes(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr())),
                   "sft_syndromes")
        if inf["mode"] == SFT_MODE_ITERATIVE:
            return [v.view(2, -1) for v in out.split([2 * m for m in sizes])]
        return out

    def attach(self, mlp):
        """Use a learned order predictor for this plan's SFT_FLAG_LEARNED signals (None detaches)."""
        _lib.check(self._lib.sft_plan_attach_mlp(self._h, mlp._h if mlp is not None else None), "sft_plan_attach_mlp")
        self._mlp = mlp

    def features(self, x, capacity=None):
        """Predictor features of the active bins of x: (features [n, 32], bins [n]) device tensors."""
        torch = _torch()
        self._check_input(x)
        cap = capacity if capacity is not None else self.infos[0]["m"]
        feat = torch.empty((max(cap, 1), _lib.MLP_FEATURES), dtype=torch.float32, device=x.device)
        bins = torch.empty(max(cap, 1), dtype=torch.int64, device=x.device)
        cnt = torch.zeros(1, dtype=torch.int64, device=x.device)
        _lib.check(self._lib.sft_features(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(feat.data_ptr()),
                                          ctypes.c_void_p(bins.data_ptr()), cap, ctypes.c_void_p(cnt.data_ptr())),
                   "sft_features")
        n = min(int(cnt.item()), cap)
        return feat[:n], bins[:n]

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sft_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mlp:
    """The learned order predictor (device weights, FP32 master + BF16 copies)."""

    PARAMS = _lib.MLP_PARAMS

    def __init__(self, seed: int = 0, stream=None):
        torch = _torch()
        self._lib = _lib.load()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _lib.check(self._lib.sft_mlp_create(ctypes.byref(h), int(seed), ctypes.c_void_p(self.stream.cuda_stream)),
                   "sft_mlp_create")
        self._h = h

    def get_params(self):
        import numpy as np
        out = np.empty(self.PARAMS, np.float32)
        _lib.check(self._lib.sft_mlp_get_params(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                self.PARAMS), "sft_mlp_get_params")
        return out

    def set_params(self, theta):
        import numpy as np
        a = np.ascontiguousarray(theta, dtype=np.float32)
        _lib.check(self._lib.sft_mlp_set_params(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size),
                   "sft_mlp_set_params")

    def forward(self, feat):
        torch = _torch()
        feat = feat.contiguous().float()
        logits = torch.empty((feat.shape[0], _lib.MLP_CLASSES), dtype=torch.float32, device=feat.device)
        _lib.check(self._lib.sft_mlp_forward(self._h, ctypes.c_void_p(feat.data_ptr()), feat.shape[0],
                                             ctypes.c_void_p(logits.data_ptr())), "sft_mlp_forward")
        return logits

    def grad(self, feat, labels):
        torch = _torch()
        feat = feat.contiguous().float()
        labels = labels.contiguous().to(torch.int32)
        g = torch.empty(self.PARAMS, dtype=torch.float32, device=feat.device)
        loss = torch.empty(1, dtype=torch.float32, device=feat.device)
        _lib.check(self._lib.sft_mlp_grad(self._h, ctypes.c_void_p(feat.data_ptr()), ctypes.c_void_p(labels.data_ptr()),
                                          feat.shape[0], ctypes.c_void_p(g.data_ptr()),
                                          ctypes.c_void_p(loss.data_ptr())), "sft_mlp_grad")
        return g, loss

    def train_step(self, feat, labels, lr, loss=None):
        _lib.check(self._lib.sft_mlp_train_step(self._h, ctypes.c_void_p(feat.data_ptr()),
                                                ctypes.c_void_p(labels.data_ptr()), feat.shape[0], float(lr),
                                                ctypes.c_void_p(loss.data_ptr()) if loss is not None else None),
                   "sft_mlp_train_step")

    def save(self, path):
        import numpy as np
        np.save(path, self.get_params())

    def load(self, path):
        import numpy as np
        self.set_params(np.load(path, allow_pickle=False))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sft_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
