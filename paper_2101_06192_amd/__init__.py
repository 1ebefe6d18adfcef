"""Forest closeness by uniform spanning trees on AMD MI355X (gfx950).

Thin ctypes binding of ``libfc.so`` (C-ABI in ``include/fc.h``).  Every step
of the computation runs in the library's HIP kernels; this module only
marshals arguments.  PyTorch provides device memory (output tensors) and the
stream the library enqueues on.  If the library has not been built, every
call raises: there is no CPU fallback.

Functions follow the paper's problem statement (Algorithm 1,
ApproxDiagForestMatrix(G, alpha, eps, delta)): ``diag_estimate`` and
``farness`` return the estimated diagonal of Omega = (alpha L + I)^{-1}, the
forest farness and the forest closeness of every vertex; ``sample`` exposes
the tree sampler (Algorithm 3) itself with per-tree outputs.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfc.so")

FC_OK = 0
FC_ERR_ARG = -1
FC_ERR_GRAPH = -2
FC_ERR_NOMEM = -3
FC_ERR_HIP = -4
FC_ERR_UNSUPPORTED = -5
FC_ERR_OVERFLOW = -6
FC_MEM_HOST = 0
FC_MEM_DEVICE = 1
FC_EST_DIRECT = 0
FC_EST_ALG1_LITERAL = 1
FC_FLAG_TRUSTED_GRAPH = 1
FC_FLAG_SAMPLER_LANE = 2
FC_FLAG_SAMPLER_COOP = 4
FC_FLAG_SAMPLER_LDS = 16
FC_FLAG_SAMPLER_HYB = 32
FC_FLAG_SAMPLER_TILE = 64
SAMPLERS = {None: 0, "auto": 0, "lane": FC_FLAG_SAMPLER_LANE, "coop": FC_FLAG_SAMPLER_COOP,
            "lds": FC_FLAG_SAMPLER_LDS, "hyb": FC_FLAG_SAMPLER_HYB, "tile": FC_FLAG_SAMPLER_TILE}


class FCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fc error {code}: {msg}")
        self.code = code


class fc_graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("weights", ctypes.c_void_p), ("mem", ctypes.c_int32)]


class fc_params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("eps", ctypes.c_double),
                ("delta", ctypes.c_double), ("kappa", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("tau", ctypes.c_uint32),
                ("stream_id", ctypes.c_uint32), ("estimator", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


class fc_stats(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_uint32), ("trees_in_flight", ctypes.c_uint32),
                ("walk_steps", ctypes.c_uint64), ("roots", ctypes.c_uint64),
                ("digest_sum", ctypes.c_uint64), ("ms_sample", ctypes.c_double),
                ("ms_total", ctypes.c_double), ("sampler", ctypes.c_char * 16),
                ("phase_ms", ctypes.c_double * 8), ("ms_predraw", ctypes.c_double)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["sampler"] = d["sampler"].decode()
        d["phase_ms"] = list(d["phase_ms"])
        return d


class fc_job(ctypes.Structure):
    _fields_ = [("graph", fc_graph), ("alpha", ctypes.c_double), ("stream_id", ctypes.c_uint32),
                ("tree_begin", ctypes.c_uint32), ("tree_count", ctypes.c_uint32),
                ("pad", ctypes.c_uint32), ("root_counts", ctypes.c_void_p),
                ("tree_digests", ctypes.c_void_p)]


FC_FLAG_AUTOTUNE = 8
FC_PREC_FP64 = 0
FC_PREC_FP32_REFINED = 1

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded product library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, u32, i64, f64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32,
                                  ctypes.c_int64, ctypes.c_double)
        gp, pp, sp = (ctypes.POINTER(fc_graph), ctypes.POINTER(fc_params),
                      ctypes.POINTER(fc_stats))
        sig = {
            "fc_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int, vp]),
            "fc_destroy": (ctypes.c_int, [vp]),
            "fc_set_stream": (ctypes.c_int, [vp, vp]),
            "fc_set_option": (ctypes.c_int, [vp, ctypes.c_char_p, i64]),
            "fc_tau": (ctypes.c_int, [i64, i64, f64, f64, f64, ctypes.POINTER(u32)]),
            "fc_thresholds": (ctypes.c_int, [vp, f64, i32, vp]),
            "fc_sample": (ctypes.c_int, [vp, gp, pp, u32, u32, vp, vp, vp, vp, vp, vp, sp]),
            "fc_sample_noalloc": (ctypes.c_int, [vp, gp, pp, u32, u32, vp, vp, vp, vp, vp, vp, sp]),
            "fc_diag_estimate": (ctypes.c_int, [vp, gp, pp, vp, vp, sp]),
            "fc_farness": (ctypes.c_int, [vp, gp, pp, vp, vp, vp, vp, sp]),
            "fc_solve": (ctypes.c_int, [vp, gp, f64, vp, vp, i32, f64, i32, i32, i32,
                                        ctypes.POINTER(i32), vp]),
            "fc_batch_create": (ctypes.c_int, [vp, ctypes.POINTER(fc_job), i32, ctypes.c_uint64,
                                               i32, ctypes.POINTER(vp)]),
            "fc_batch_run": (ctypes.c_int, [vp, sp]),
            "fc_batch_destroy": (ctypes.c_int, [vp]),
            "fc_probe_random_access": (ctypes.c_int, [vp, ctypes.c_uint64, i32,
                                                      ctypes.POINTER(ctypes.c_double)]),
            "fc_rank": (ctypes.c_int, [vp, vp, i32, i32, vp, vp]),
            "fc_kendall_tau": (ctypes.c_int, [vp, vp, vp, i32, ctypes.POINTER(f64),
                                              ctypes.POINTER(i64)]),
            "fc_group_closeness": (ctypes.c_int, [vp, gp, f64, i32, i32, ctypes.POINTER(i32),
                                                  ctypes.POINTER(f64)]),
            "fc_error_string": (ctypes.c_char_p, [ctypes.c_int]),
            "fc_last_error": (ctypes.c_char_p, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def error_string(code: int) -> str:
    return lib().fc_error_string(code).decode()


def tau(m: int, n: int, eps: float, delta: float, kappa: float = 0.0) -> int:
    """Sample size of Algorithm 1 (see fc_tau in include/fc.h)."""
    out = ctypes.c_uint32(0)
    rc = lib().fc_tau(int(m), int(n), float(eps), float(delta), float(kappa), ctypes.byref(out))
    if rc != FC_OK:
        raise FCError(rc, error_string(rc))
    return int(out.value)


class Context:
    """An ``fc_ctx`` on one GPU; calls run on torch's current stream."""

    def __init__(self, device="cuda:0"):
        import torch
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the library runs on a GPU device only")
        idx = self.device.index if self.device.index is not None else 0
        self.device = torch.device("cuda", idx)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            rc = lib().fc_create(ctypes.byref(h), idx, ctypes.c_void_p(stream))
        if rc != FC_OK:
            raise FCError(rc, error_string(rc))
        self.handle = h

    def check(self, rc: int):
        if rc != FC_OK:
            raise FCError(rc, lib().fc_last_error(self.handle).decode() or error_string(rc))

    def sync_stream(self):
        import torch
        s = torch.cuda.current_stream(self.device).cuda_stream
        self.check(lib().fc_set_stream(self.handle, ctypes.c_void_p(s)))

    def close(self):
        if getattr(self, "handle", None):
            lib().fc_destroy(self.handle)
            self.handle = None


_contexts: dict = {}


def context(device="cuda:0") -> Context:
    import torch
    d = torch.device(device)
    key = (d.type, d.index if d.index is not None else 0)
    if key not in _contexts:
        _contexts[key] = Context(device)
    ctx = _contexts[key]
    ctx.sync_stream()
    return ctx


@dataclass
class DeviceGraph:
    """CSR held in device memory (torch int32 tensors; weights: float64 or None)."""
    n: int
    row_ptr: "object"
    col_idx: "object"
    weights: "object" = None

    @property
    def nnz(self) -> int:
        return int(self.col_idx.numel())

    @property
    def m(self) -> int:
        return self.nnz // 2


def to_device(g, device="cuda:0") -> DeviceGraph:
    import torch
    rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr, dtype=np.int32)).to(device)
    ci = torch.from_numpy(np.ascontiguousarray(g.col_idx, dtype=np.int32)).to(device)
    w = getattr(g, "weights", None)
    if w is not None:
        w = torch.from_numpy(np.ascontiguousarray(w, dtype=np.float64)).to(device)
    return DeviceGraph(int(g.n), rp, ci, w)


def _graph_struct(g) -> fc_graph:
    if isinstance(g, DeviceGraph):
        w = g.weights
        wp = w.data_ptr() if w is not None and g.nnz else 0
        return fc_graph(g.n, g.nnz, ctypes.c_void_p(g.row_ptr.data_ptr()),
                        ctypes.c_void_p(g.col_idx.data_ptr() if g.nnz else 0), ctypes.c_void_p(wp),
                        FC_MEM_DEVICE)
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    w = getattr(g, "weights", None)
    if w is not None:
        w = np.ascontiguousarray(w, dtype=np.float64)
        if w.size != ci.size:
            raise ValueError("weights must have one entry per CSR entry")
    s = fc_graph(int(g.n), int(ci.size), ctypes.c_void_p(rp.ctypes.data),
                 ctypes.c_void_p(ci.ctypes.data if ci.size else 0),
                 ctypes.c_void_p(w.ctypes.data if w is not None and w.size else 0), FC_MEM_HOST)
    s._keep = (rp, ci, w)
    return s


def _params(alpha, eps=0.1, delta=0.1, kappa=0.0, seed=0, tau_=0, stream_id=0,
            literal=False, trusted=False, sampler=None) -> fc_params:
    if sampler not in SAMPLERS:
        raise ValueError(f"sampler must be one of {sorted(k for k in SAMPLERS if k)}")
    flags = (FC_FLAG_TRUSTED_GRAPH if trusted else 0) | SAMPLERS[sampler]
    return fc_params(float(alpha), float(eps), float(delta), float(kappa), int(seed), int(tau_),
                     int(stream_id), FC_EST_ALG1_LITERAL if literal else FC_EST_DIRECT, flags)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _out(t, as_torch):
    if t is None:
        return None
    return t if as_torch else t.cpu().numpy()


def set_option(key: str, value: int, device="cuda:0") -> None:
    """Launch-shape option of the device's context (fc_set_option)."""
    ctx = context(device)
    ctx.check(lib().fc_set_option(ctx.handle, key.encode(), int(value)))


def thresholds(alpha: float, d_max: int, device="cuda:0") -> np.ndarray:
    """thr(d), d = 0..d_max, as computed on the device."""
    ctx = context(device)
    out = np.zeros(d_max + 1, np.uint64)
    ctx.check(lib().fc_thresholds(ctx.handle, float(alpha), int(d_max),
                                  ctypes.c_void_p(out.ctypes.data)))
    return out


def sample(g, alpha: float, seed: int = 0, tree_begin: int = 0, tree_count: int = 1,
           stream_id: int = 0, device="cuda:0", want_visits: bool = False,
           want_digests: bool = False, want_steps: bool = False, want_parents: bool = False,
           want_tree_visits: bool = False, trusted: bool = False, as_torch: bool = False,
           root_counts=None, sampler=None) -> dict:
    """Sample trees [tree_begin, tree_begin + tree_count) (fc_sample)."""
    return _sample("fc_sample", g, alpha, seed, tree_begin, tree_count, stream_id, device,
                   want_visits, want_digests, want_steps, want_parents, want_tree_visits,
                   trusted, as_torch, root_counts, sampler)


def sample_noalloc(g, alpha: float, seed: int = 0, tree_begin: int = 0, tree_count: int = 1,
                   stream_id: int = 0, device="cuda:0", want_visits: bool = False,
                   want_digests: bool = False, want_steps: bool = False,
                   want_parents: bool = False, want_tree_visits: bool = False,
                   trusted: bool = False, as_torch: bool = False, root_counts=None,
                   sampler=None) -> dict:
    """As ``sample``, through fc_sample_noalloc: the library allocates no device
    memory for the call (its scratch is the library's static device array; the
    graph must be device-resident)."""
    return _sample("fc_sample_noalloc", g, alpha, seed, tree_begin, tree_count, stream_id,
                   device, want_visits, want_digests, want_steps, want_parents,
                   want_tree_visits, trusted, as_torch, root_counts, sampler)


def _sample(entry, g, alpha, seed, tree_begin, tree_count, stream_id, device, want_visits,
            want_digests, want_steps, want_parents, want_tree_visits, trusted, as_torch,
            root_counts, sampler) -> dict:
    import torch
    ctx = context(device)
    n = int(g.n)
    dev = ctx.device
    R = root_counts if root_counts is not None else torch.zeros(max(n, 1), dtype=torch.int32, device=dev)
    V = torch.zeros(max(n, 1), dtype=torch.int64, device=dev) if want_visits else None
    D = torch.zeros(max(tree_count, 1), dtype=torch.int64, device=dev) if want_digests else None
    S = torch.zeros(max(tree_count, 1), dtype=torch.int64, device=dev) if want_steps else None
    P = torch.zeros(max(tree_count * n, 1), dtype=torch.int32, device=dev) if want_parents else None
    TV = torch.zeros(max(tree_count * n, 1), dtype=torch.int32, device=dev) if want_tree_visits else None
    gs = _graph_struct(g)
    ps = _params(alpha, seed=seed, stream_id=stream_id, trusted=trusted, sampler=sampler)
    st = fc_stats()
    ctx.check(getattr(lib(), entry)(ctx.handle, ctypes.byref(gs), ctypes.byref(ps),
                                    int(tree_begin), int(tree_count), _ptr(R), _ptr(V), _ptr(D),
                                    _ptr(S), _ptr(P), _ptr(TV), ctypes.byref(st)))
    res = {"stats": st.as_dict()}
    res["root_counts"] = _out(R[:n], as_torch)
    if not as_torch:
        res["root_counts"] = res["root_counts"].view(np.uint32)
    if V is not None:
        res["visit_counts"] = _out(V[:n], as_torch)
        if not as_torch:
            res["visit_counts"] = res["visit_counts"].view(np.uint64)
    if D is not None:
        res["tree_digests"] = _out(D[:tree_count], as_torch)
        if not as_torch:
            res["tree_digests"] = res["tree_digests"].view(np.uint64)
    if S is not None:
        res["tree_steps"] = _out(S[:tree_count], as_torch)
        if not as_torch:
            res["tree_steps"] = res["tree_steps"].view(np.uint64)
    if P is not None:
        p = P[:tree_count * n]
        res["parents"] = p.view(tree_count, n) if as_torch else p.cpu().numpy().reshape(tree_count, n)
    if TV is not None:
        tv = TV[:tree_count * n]
        res["tree_visits"] = (tv.view(tree_count, n) if as_torch
                              else tv.cpu().numpy().reshape(tree_count, n).view(np.uint32))
    return res


def _estimate(entry: str, g, alpha, eps, delta, seed, kappa, tau_, literal, device, trusted,
              as_torch, stream_id=0, sampler=None):
    import torch
    ctx = context(device)
    n = int(g.n)
    dev = ctx.device
    diag = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    R = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    gs = _graph_struct(g)
    ps = _params(alpha, eps, delta, kappa, seed, tau_, stream_id, literal, trusted, sampler)
    st = fc_stats()
    out = {}
    if entry == "diag":
        ctx.check(lib().fc_diag_estimate(ctx.handle, ctypes.byref(gs), ctypes.byref(ps),
                                         _ptr(diag), _ptr(R), ctypes.byref(st)))
    else:
        far = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
        clo = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
        ctx.check(lib().fc_farness(ctx.handle, ctypes.byref(gs), ctypes.byref(ps), _ptr(far),
                                   _ptr(clo), _ptr(diag), _ptr(R), ctypes.byref(st)))
        out["farness"] = _out(far[:n], as_torch)
        out["closeness"] = _out(clo[:n], as_torch)
    out["diag"] = _out(diag[:n], as_torch)
    rc = _out(R[:n], as_torch)
    out["root_counts"] = rc if as_torch else rc.view(np.uint32)
    out["stats"] = st.as_dict()
    out["tau"] = int(st.tau)
    return out


def diag_estimate(g, alpha: float = 1.0, eps: float = 0.1, delta: float = 0.1, seed: int = 0,
                  kappa: float = 0.0, tau: int = 0, literal: bool = False, device="cuda:0",
                  trusted: bool = False, as_torch: bool = False, stream_id: int = 0,
                  sampler=None) -> dict:
    """Algorithm 1: (eps, delta)-estimate of diag(Omega) (fc_diag_estimate)."""
    return _estimate("diag", g, alpha, eps, delta, seed, kappa, tau, literal, device, trusted,
                     as_torch, stream_id, sampler)


def farness(g, alpha: float = 1.0, eps: float = 0.1, delta: float = 0.1, seed: int = 0,
            kappa: float = 0.0, tau: int = 0, literal: bool = False, device="cuda:0",
            trusted: bool = False, as_torch: bool = False, stream_id: int = 0,
            sampler=None) -> dict:
    """Forest farness and closeness of every vertex (fc_farness)."""
    return _estimate("farness", g, alpha, eps, delta, seed, kappa, tau, literal, device, trusted,
                     as_torch, stream_id, sampler)


class Batch:
    """Many (graph, alpha, tree range) jobs sampled by one persistent launch
    (fc_batch_create / fc_batch_run).  ``jobs`` is a list of dicts with keys
    graph (a DeviceGraph), alpha, tree_count, and optionally stream_id,
    tree_begin and digests (bool).  Each job's root counts accumulate in a
    device tensor (``self.root_counts[i]``); ``reset()`` zeroes them."""

    def __init__(self, jobs, seed: int = 0, device="cuda:0", trusted: bool = False,
                 autotune: bool = False):
        import torch
        self.ctx = context(device)
        dev = self.ctx.device
        self.graphs = [j["graph"] for j in jobs]
        for g in self.graphs:
            if not isinstance(g, DeviceGraph):
                raise TypeError("batch jobs need device graphs (to_device)")
        self.root_counts = [torch.zeros(max(j["graph"].n, 1), dtype=torch.int32, device=dev)
                            for j in jobs]
        self.digests = [torch.zeros(max(j["tree_count"], 1), dtype=torch.int64, device=dev)
                        if j.get("digests") else None for j in jobs]
        arr = (fc_job * max(len(jobs), 1))()
        for i, j in enumerate(jobs):
            arr[i] = fc_job(_graph_struct(j["graph"]), float(j["alpha"]), int(j.get("stream_id", 0)),
                            int(j.get("tree_begin", 0)), int(j["tree_count"]), 0,
                            ctypes.c_void_p(self.root_counts[i].data_ptr()),
                            _ptr(self.digests[i]))
        flags = (FC_FLAG_TRUSTED_GRAPH if trusted else 0) | (FC_FLAG_AUTOTUNE if autotune else 0)
        h = ctypes.c_void_p()
        self.ctx.check(lib().fc_batch_create(self.ctx.handle, arr, len(jobs), int(seed), flags,
                                             ctypes.byref(h)))
        self.handle = h
        self.n_jobs = len(jobs)

    def run(self) -> dict:
        self.ctx.sync_stream()
        st = fc_stats()
        self.ctx.check(lib().fc_batch_run(self.handle, ctypes.byref(st)))
        return st.as_dict()

    def reset(self):
        for r in self.root_counts:
            r.zero_()

    def result(self, i: int) -> dict:
        n = self.graphs[i].n
        out = {"root_counts": self.root_counts[i][:n].cpu().numpy().view(np.uint32)}
        if self.digests[i] is not None:
            out["tree_digests"] = self.digests[i].cpu().numpy().view(np.uint64)
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib().fc_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(g, alpha: float, B, X0=None, rtol: float = 1e-9, precision: str = "fp32_refined",
          max_iters: int = 20000, device="cuda:0", trusted: bool = False, as_torch: bool = False) -> dict:
    """(alpha L + I) X = B for up to 64 right-hand sides (fc_solve).  B: (n, k)
    array or tensor; X0: initial guess (zeros if None).  precision "fp64" or
    "fp32_refined"."""
    import torch
    ctx = context(device)
    dev = ctx.device
    Bt = torch.as_tensor(B, dtype=torch.float64).to(dev)
    if Bt.dim() == 1:
        Bt = Bt[:, None]
    Bt = Bt.contiguous()
    n, k = Bt.shape
    X = (torch.zeros_like(Bt) if X0 is None
         else torch.as_tensor(X0, dtype=torch.float64).to(dev).reshape(n, k).contiguous().clone())
    prec = {"fp64": FC_PREC_FP64, "fp32_refined": FC_PREC_FP32_REFINED}[precision]
    gs = _graph_struct(g)
    it = ctypes.c_int32(0)
    rel = np.zeros(max(k, 1), np.float64)
    ctx.check(lib().fc_solve(ctx.handle, ctypes.byref(gs), float(alpha),
                             ctypes.c_void_p(Bt.data_ptr()), ctypes.c_void_p(X.data_ptr()), int(k),
                             float(rtol), prec, int(max_iters),
                             FC_FLAG_TRUSTED_GRAPH if trusted else 0, ctypes.byref(it),
                             ctypes.c_void_p(rel.ctypes.data)))
    return {"X": X if as_torch else X.cpu().numpy(), "iters": int(it.value), "relres": rel[:k]}


def rank(score, descending: bool = False, device="cuda:0", as_torch: bool = False) -> dict:
    """Vertices sorted by score, ties by id (fc_rank): {"order", "rank"}."""
    import torch
    ctx = context(device)
    s = torch.as_tensor(score, dtype=torch.float64).to(ctx.device).reshape(-1).contiguous()
    n = int(s.numel())
    order = torch.empty(max(n, 1), dtype=torch.int32, device=ctx.device)
    rk = torch.empty(max(n, 1), dtype=torch.int32, device=ctx.device)
    ctx.check(lib().fc_rank(ctx.handle, ctypes.c_void_p(s.data_ptr() if n else 0), n,
                            int(bool(descending)), _ptr(order), _ptr(rk)))
    return {"order": _out(order[:n], as_torch), "rank": _out(rk[:n], as_torch)}


def kendall_tau(a, b, device="cuda:0") -> dict:
    """Kendall's tau-b of two score vectors with its exact pair counts
    (fc_kendall_tau): {"tau_b", "counts": (n_c, n_d, n_a, n_b, n_ab)}."""
    import torch
    ctx = context(device)
    ta = torch.as_tensor(a, dtype=torch.float64).to(ctx.device).reshape(-1).contiguous()
    tb = torch.as_tensor(b, dtype=torch.float64).to(ctx.device).reshape(-1).contiguous()
    if ta.numel() != tb.numel():
        raise ValueError("a and b must have the same length")
    n = int(ta.numel())
    tau_b = ctypes.c_double(0.0)
    counts = (ctypes.c_int64 * 5)()
    ctx.check(lib().fc_kendall_tau(ctx.handle, ctypes.c_void_p(ta.data_ptr() if n else 0),
                                   ctypes.c_void_p(tb.data_ptr() if n else 0), n,
                                   ctypes.byref(tau_b), counts))
    return {"tau_b": float(tau_b.value), "counts": tuple(int(x) for x in counts)}


def group_closeness(g, alpha: float, k: int, device="cuda:0", trusted: bool = False) -> dict:
    """Greedy group forest closeness (fc_group_closeness): {"group", "farness"}."""
    ctx = context(device)
    gs = _graph_struct(g)
    grp = (ctypes.c_int32 * max(int(k), 1))()
    far = (ctypes.c_double * max(int(k), 1))()
    ctx.check(lib().fc_group_closeness(ctx.handle, ctypes.byref(gs), float(alpha), int(k),
                                       FC_FLAG_TRUSTED_GRAPH if trusted else 0, grp, far))
    return {"group": [int(x) for x in grp[:k]], "farness": [float(x) for x in far[:k]]}


def probe_random_access(footprint_bytes: int, atomics: bool = False, device="cuda:0") -> float:
    """Random 4-byte accesses per second over a footprint (fc_probe_random_access)."""
    ctx = context(device)
    out = ctypes.c_double(0.0)
    ctx.check(lib().fc_probe_random_access(ctx.handle, int(footprint_bytes), int(bool(atomics)),
                                           ctypes.byref(out)))
    return float(out.value)
