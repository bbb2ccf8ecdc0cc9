"""Thin ctypes binding of the htsvt C-ABI library (argument marshalling only).

Every step of the randomized t-SVT and of the ADMM update runs in the HIP
kernels of libhtsvt.so; this module only converts arguments, allocates the
caller-owned device buffers through PyTorch and passes raw pointers and the
current HIP stream.  Tensors are passed as flat device tensors in Fortran order
(i1 fastest), the library's storage layout; `to_device` / `from_device` convert
from / to numpy arrays indexed (i1, ..., id).

There is no fallback: if the library is missing, importing this module fails.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhtsvt.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libhtsvt.so not found at {LIB_PATH}; build it with paper_2506_09594_amd/build.py")

# PyTorch's HIP runtime must be the one the library binds to: load torch first
# so that the library resolves libamdhip64 to the copy already in the process.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

MAX_ORDER = 8
OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_NONFINITE, ERR_WORKSPACE, ERR_HIP, ERR_ALLOC = 0, -1, -2, -3, -4, -5, -6
TRANSFORMS = {"dct2": 0, "dft": 1, "custom": 2, "dft_unnormalized": 3}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2}
PENALTIES = {"l1": 0, "mcp": 1, "scad": 2, "log": 3, "capped_l1": 4, "firm": 5}
MODELS = {"completion": 0, "rpca": 1, "rpca_tube": 2, "rpca_slice": 3}
REGIONS = {"A": 0, "omega": 1, "Q": 2, "Bt": 3, "K": 4, "QK": 5, "C": 6, "Lnew": 7, "Xin": 8, "state": 9,
           "gram": 10, "gram_q": 11, "widths": 12, "call": 13, "widths_redo": 14, "widths_used": 15,
           "sigma": 16, "kept": 17, "anorm": 18, "features": 19, "learn_state": 20, "status": 21, "rse_part": 22,
           "group_sq": 23, "omega_bf16": 24, "Q_bf16": 25, "Bt_bf16": 26}

# Symbols the header declares (checked by the CPU test suite).
EXPORTS = [
    "ht_version", "ht_last_error", "ht_plan_create", "ht_plan_destroy", "ht_plan_workspace_size",
    "ht_plan_info", "ht_plan_workspace_region", "ht_gnhtsvt", "ht_omega_fp64", "ht_transform",
    "ht_admm_workspace_size", "ht_admm_init", "ht_admm_iterate", "ht_admm_get_stats",
    "ht_profile_enable", "ht_profile_read", "ht_batch_plan_create", "ht_batch_info", "ht_batch_tensor_info",
    "ht_batch_gnhtsvt", "ht_plan_set_tuning", "ht_plan_get_tuning", "ht_plan_autotune", "ht_plan_graph_enable",
    "ht_plan_learned", "ht_plan_learned_reset", "ht_plan_learned_counts", "ht_plan_force_fallback",
    "ht_mlp_param_count", "ht_mlp_workspace_size", "ht_mlp_forward", "ht_mlp_grad", "ht_mlp_train_step",
    "ht_plan_device", "ht_plan_status", "ht_admm_set_truth", "ht_gnhtsvt_noalloc",
]
STAGES = ["transform_fwd", "omega", "sketch_nn", "cholqr", "sketch_tn", "smallsvd", "recon_qk", "recon_nt",
          "transform_inv", "admm_update"]


class HtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"htsvt error {code}: {msg}")
        self.code = code


class _Penalty(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("p0", ctypes.c_double), ("p1", ctypes.c_double)]


class _PlanDesc(ctypes.Structure):
    _fields_ = [
        ("order", ctypes.c_int),
        ("dims", ctypes.c_int64 * MAX_ORDER),
        ("transform", ctypes.c_int * MAX_ORDER),
        ("custom", ctypes.POINTER(ctypes.c_double) * MAX_ORDER),
        ("r", ctypes.c_int), ("p", ctypes.c_int), ("q", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("seed", ctypes.c_uint64),
        ("stream_id", ctypes.c_uint32),
    ]


class _AdmmParams(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_int), ("phi", _Penalty), ("psi", _Penalty),
        ("lam", ctypes.c_double), ("mu0", ctypes.c_double), ("vartheta", ctypes.c_double),
        ("mu_max", ctypes.c_double),
    ]


class _AdmmStats(ctypes.Structure):
    _fields_ = [("iteration", ctypes.c_int32), ("mu", ctypes.c_double), ("dL", ctypes.c_double),
                ("dE", ctypes.c_double), ("resid", ctypes.c_double), ("rse", ctypes.c_double)]


_vp = ctypes.c_void_p
_sig = {
    "ht_version": (ctypes.c_int, []),
    "ht_last_error": (ctypes.c_char_p, []),
    "ht_plan_create": (ctypes.c_int, [ctypes.POINTER(_PlanDesc), ctypes.POINTER(_vp)]),
    "ht_plan_destroy": (ctypes.c_int, [_vp]),
    "ht_plan_workspace_size": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "ht_plan_info": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_int)]),
    "ht_plan_workspace_region": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t),
                                                ctypes.POINTER(ctypes.c_size_t)]),
    "ht_gnhtsvt": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, ctypes.POINTER(_Penalty), ctypes.c_uint32,
                                  _vp, ctypes.c_size_t, _vp, _vp, _vp]),
    "ht_omega_fp64": (ctypes.c_int, [_vp, ctypes.c_uint32, _vp, _vp]),
    "ht_transform": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp]),
    "ht_admm_workspace_size": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "ht_admm_init": (ctypes.c_int, [_vp, ctypes.POINTER(_AdmmParams), _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "ht_admm_iterate": (ctypes.c_int, [_vp, ctypes.POINTER(_AdmmParams), _vp, _vp, _vp, _vp, _vp, ctypes.c_int,
                                       _vp, ctypes.c_size_t, _vp]),
    "ht_admm_get_stats": (ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(_AdmmStats)]),
    "ht_profile_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ht_profile_read": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int),
                                       ctypes.c_int]),
    "ht_batch_plan_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_PlanDesc), ctypes.POINTER(_vp)]),
    "ht_batch_info": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int)]),
    "ht_batch_tensor_info": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                            ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                            ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "ht_batch_gnhtsvt": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.POINTER(_Penalty), ctypes.c_uint32,
                                        _vp, ctypes.c_size_t, _vp, _vp, _vp]),
    "ht_plan_set_tuning": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int]),
    "ht_plan_get_tuning": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "ht_plan_autotune": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_size_t, _vp, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_double)]),
    "ht_plan_graph_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ht_plan_learned": (ctypes.c_int, [_vp, ctypes.c_int, _vp]),
    "ht_plan_learned_reset": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, _vp]),
    "ht_plan_learned_counts": (ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(ctypes.c_int),
                                              ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "ht_plan_force_fallback": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ht_mlp_param_count": (ctypes.c_int, []),
    "ht_mlp_workspace_size": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "ht_mlp_forward": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp]),
    "ht_mlp_grad": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "ht_mlp_train_step": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp, _vp, ctypes.c_int, ctypes.c_float,
                                         ctypes.c_float, ctypes.c_float, ctypes.c_float, _vp, _vp, ctypes.c_size_t,
                                         _vp]),
    "ht_plan_device": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int)]),
    "ht_plan_status": (ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(ctypes.c_int64)]),
    "ht_admm_set_truth": (ctypes.c_int, [_vp, _vp]),
    "ht_gnhtsvt_noalloc": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, ctypes.POINTER(_Penalty), ctypes.c_uint32,
                                          _vp, _vp, _vp]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def _check(rc):
    if rc != OK:
        raise HtError(rc, _lib.ht_last_error().decode(errors="replace"))


def version():
    return _lib.ht_version()


def _penalty(pen):
    kind, params = pen
    params = tuple(params) + (0.0, 0.0)
    return _Penalty(PENALTIES[kind], float(params[0]), float(params[1]))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def check_tensor(t, name, dtype, numel, optional=False):
    """Raise ValueError unless t is a contiguous CUDA tensor of the given dtype
    holding at least numel elements (the library reads and writes exactly the
    plan's element count through the raw pointer)."""
    import torch
    if t is None:
        if optional:
            return
        raise ValueError(f"{name} is required")
    if not torch.is_tensor(t):
        raise ValueError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype} for this plan, not {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous (Fortran-order flat storage)")
    if t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements, the plan needs {numel}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor (the library takes device pointers)")


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def to_device(X, dtype):
    """numpy (n1, ..., nd) -> flat CUDA tensor in Fortran order."""
    import torch
    flat = np.ascontiguousarray(np.asarray(X).ravel(order="F"))
    return torch.from_numpy(flat).to(device="cuda", dtype=dtype)


def from_device(t, dims):
    """flat CUDA tensor in Fortran order -> numpy (n1, ..., nd) float64."""
    return t.detach().double().cpu().numpy().reshape(tuple(dims), order="F")


def _make_desc(dims, transforms, r, p, q, precision, seed, stream_id, custom, keep):
    dims = [int(n) for n in dims]
    if not 2 <= len(dims) <= MAX_ORDER:
        raise ValueError("order must be in [2, 8]")
    transforms = transforms if transforms is not None else ["dct2"] * (len(dims) - 2)
    d = _PlanDesc()
    d.order = len(dims)
    for i, n in enumerate(dims):
        d.dims[i] = n
    for k, kind in enumerate(transforms):
        d.transform[k + 2] = TRANSFORMS[kind]
        if kind == "custom":
            U = np.ascontiguousarray(np.asarray(custom[k], dtype=np.float64))
            keep.append(U)
            d.custom[k + 2] = U.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.r, d.p, d.q = int(r), int(p), int(q)
    d.precision = PRECISIONS[precision]
    d.seed = int(seed)
    d.stream_id = int(stream_id)
    return d


class Plan:
    """One tensor shape + transforms + sketch parameters on the current device."""

    def __init__(self, dims, transforms=None, r=5, p=5, q=1, precision="fp32", seed=0, stream_id=0, custom=None):
        self._custom_keep = []
        d = _make_desc(dims, transforms, r, p, q, precision, seed, stream_id, custom, self._custom_keep)
        h = _vp()
        _check(_lib.ht_plan_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self.dims = tuple(int(n) for n in dims)
        self.transforms = list(transforms) if transforms is not None else ["dct2"] * (len(dims) - 2)
        self.r, self.p, self.q = int(r), int(p), int(q)
        self._finish(precision)

    def _finish(self, precision):
        self.precision = precision
        h = self._h
        n_sl, w, k = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int()
        _check(_lib.ht_plan_info(h, ctypes.byref(n_sl), ctypes.byref(w), ctypes.byref(k)))
        self.n_slices, self.width, self.kept = n_sl.value, w.value, k.value
        nn = ctypes.c_int64()
        _check(_lib.ht_batch_info(h, ctypes.byref(nn), None))
        self.N = nn.value
        sz = ctypes.c_size_t()
        _check(_lib.ht_plan_workspace_size(h, ctypes.byref(sz)))
        self.workspace_bytes = sz.value
        _check(_lib.ht_admm_workspace_size(h, ctypes.byref(sz)))
        self.admm_workspace_bytes = sz.value

    def set_tuning(self, prod_rows=0, transform_lds_kib=0):
        """Tile rows of the sketch products (64 or 128) and LDS budget of a
        transform tile (32, 64 or 128 KiB); 0 keeps the current value."""
        _check(_lib.ht_plan_set_tuning(self._h, int(prod_rows), int(transform_lds_kib)))

    def tuning(self):
        a, b = ctypes.c_int(), ctypes.c_int()
        _check(_lib.ht_plan_get_tuning(self._h, ctypes.byref(a), ctypes.byref(b)))
        return {"prod_rows": a.value, "transform_lds_kib": b.value}

    def autotune(self, X, workspace=None, repeats=3):
        """Time the tile choices on X and keep the fastest; returns (tuning, ms)."""
        import torch
        check_tensor(X, "X", self.torch_dtype, self.N)
        if workspace is None:
            workspace = self.alloc_workspace()
        out = torch.empty_like(X)
        self._check_io(X, out, workspace, self.workspace_bytes)
        wp, wn = self._aligned(workspace)
        ms = ctypes.c_double()
        _check(_lib.ht_plan_autotune(self._h, _ptr(X), _ptr(out), wp, wn, _stream(), int(repeats), ctypes.byref(ms)))
        return self.tuning(), ms.value

    def learned(self, mode, theta=None):
        """0: fixed widths; 1: fixed widths with statistics/features recorded;
        2: widths predicted by the network theta (flat FP32 CUDA tensor)."""
        mode = {"off": 0, "track": 1, "predict": 2}.get(mode, mode)
        self._theta_keep = theta
        _check(_lib.ht_plan_learned(self._h, int(mode), _ptr(theta)))

    def learned_reset(self, workspace):
        wp, wn = self._aligned(workspace)
        _check(_lib.ht_plan_learned_reset(self._h, wp, wn, _stream()))

    def learned_counts(self, workspace):
        wp, _wn = self._aligned(workspace)
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(_lib.ht_plan_learned_counts(self._h, wp, _stream(), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"valid": a.value, "predicted": b.value, "redone": c.value}

    def force_fallback(self, on=True):
        _check(_lib.ht_plan_force_fallback(self._h, 1 if on else 0))

    def device(self):
        d = ctypes.c_int()
        _check(_lib.ht_plan_device(self._h, ctypes.byref(d)))
        return d.value

    def status(self, workspace):
        """Number of slices of the last t-SVT on this workspace whose Gram matrices
        held a NaN or an infinity (raises HtError ERR_NONFINITE when nonzero)."""
        wp, _wn = self._aligned(workspace)
        n = ctypes.c_int64()
        _check(_lib.ht_plan_status(self._h, wp, _stream(), ctypes.byref(n)))
        return n.value

    def graph(self, on=True):
        """Record the launch sequence as a HIP graph on the next call and replay it
        on later calls with the same buffers (the call index is updated in place)."""
        _check(_lib.ht_plan_graph_enable(self._h, 1 if on else 0))

    @property
    def torch_dtype(self):
        import torch
        return torch.float64 if self.precision == "fp64" else torch.float32

    def close(self):
        if getattr(self, "_h", None):
            _lib.ht_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def alloc_workspace(self, admm=False):
        import torch
        n = self.admm_workspace_bytes if admm else self.workspace_bytes
        return torch.empty(n + 256, dtype=torch.uint8, device="cuda")

    @staticmethod
    def _aligned(ws):
        off = (-ws.data_ptr()) % 256
        return ctypes.c_void_p(ws.data_ptr() + off), ws.numel() - off

    def region(self, ws, name, dtype=None):
        """View of a named workspace region as a flat tensor."""
        import torch
        off, nb = ctypes.c_size_t(), ctypes.c_size_t()
        _check(_lib.ht_plan_workspace_region(self._h, REGIONS[name], ctypes.byref(off), ctypes.byref(nb)))
        base = (-ws.data_ptr()) % 256
        dtype = dtype or self.torch_dtype
        raw = ws[base + off.value: base + off.value + nb.value]
        return raw.view(dtype)

    def _check_io(self, X, out, workspace, need):
        import torch
        check_tensor(X, "X", self.torch_dtype, self.N)
        check_tensor(out, "out", self.torch_dtype, self.N)
        check_tensor(workspace, "workspace", torch.uint8, 0)  # its size is checked by the library

    def gnhtsvt(self, X, tau, penalty=("l1", ()), call_index=0, out=None, workspace=None, stats=False):
        import torch
        check_tensor(X, "X", self.torch_dtype, self.N)
        if out is None:
            out = torch.empty_like(X)
        if workspace is None:
            workspace = self.alloc_workspace()
        self._check_io(X, out, workspace, self.workspace_bytes)
        wp, wn = self._aligned(workspace)
        sig = kept = None
        if stats:
            sig = torch.empty(self.n_slices * self.width, dtype=torch.float64, device=X.device)
            kept = torch.empty(self.n_slices, dtype=torch.int32, device=X.device)
        pen = _penalty(penalty)
        _check(_lib.ht_gnhtsvt(self._h, _ptr(X), _ptr(out), float(tau), ctypes.byref(pen), int(call_index),
                               wp, wn, _stream(), _ptr(sig), _ptr(kept)))
        if stats:
            return out, sig.view(self.n_slices, self.width), kept
        return out

    def gnhtsvt_noalloc(self, X, tau, penalty=("l1", ()), call_index=0, out=None, stats=None):
        """ht_gnhtsvt on the library's own device scratch (no workspace argument;
        the call itself allocates nothing).  out and stats = (sigma, kept) are
        caller-allocated; out defaults to a new tensor like X."""
        import torch
        check_tensor(X, "X", self.torch_dtype, self.N)
        if out is None:
            out = torch.empty_like(X)
        check_tensor(out, "out", self.torch_dtype, self.N)
        sig = kept = None
        if stats is not None:
            sig, kept = stats
            check_tensor(sig, "sigma", torch.float64, self.n_slices * self.width)
            check_tensor(kept, "kept", torch.int32, self.n_slices)
        pen = _penalty(penalty)
        _check(_lib.ht_gnhtsvt_noalloc(self._h, _ptr(X), _ptr(out), float(tau), ctypes.byref(pen), int(call_index),
                                       _stream(), _ptr(sig), _ptr(kept)))
        return out

    def omega_fp64(self, call_index=0):
        import torch
        o = torch.empty(self.n_slices * self.dims[1] * self.width, dtype=torch.float64, device="cuda")
        _check(_lib.ht_omega_fp64(self._h, int(call_index), _ptr(o), _stream()))
        return o

    def profile(self, on=True):
        _check(_lib.ht_profile_enable(self._h, 1 if on else 0))

    def profile_read(self):
        """{stage: (total_ms, launches)} for the launches recorded since the last read."""
        n = len(STAGES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int * n)()
        _check(_lib.ht_profile_read(self._h, ms, cnt, n))
        return {STAGES[i]: (ms[i], cnt[i]) for i in range(n)}

    def transform(self, X, inverse=False, out=None):
        import torch
        check_tensor(X, "X", self.torch_dtype, self.N)
        if out is None:
            out = torch.empty_like(X)
        check_tensor(out, "out", self.torch_dtype, self.N)
        _check(_lib.ht_transform(self._h, _ptr(X), _ptr(out), 1 if inverse else 0, _stream()))
        return out


class BatchPlan(Plan):
    """Many tensors of different shapes (orders, sizes, ranks) in one plan: every
    stage of the t-SVT is one launch over all their slices.  The tensors live in
    one packed device buffer, tensor t at element offset offsets[t], each in
    Fortran order."""

    def __init__(self, shapes, transforms=None, r=5, p=5, q=1, precision="fp32", seed=0, stream_id=0):
        n = len(shapes)
        rs = list(r) if np.ndim(r) else [r] * n
        ps = list(p) if np.ndim(p) else [p] * n
        trs = transforms if transforms is not None else [["dct2"] * (len(s) - 2) for s in shapes]
        self._custom_keep = []
        descs = (_PlanDesc * n)()
        for t in range(n):
            descs[t] = _make_desc(shapes[t], trs[t], rs[t], ps[t], q, precision, seed, stream_id, None,
                                  self._custom_keep)
        h = _vp()
        _check(_lib.ht_batch_plan_create(n, descs, ctypes.byref(h)))
        self._h = h
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.transforms = trs
        self.q = int(q)
        self._finish(precision)
        self.offsets, self.numels, self.first_slice, self.widths, self.kepts = [], [], [], [], []
        for t in range(n):
            o, nm, f = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
            w, k = ctypes.c_int(), ctypes.c_int()
            _check(_lib.ht_batch_tensor_info(h, t, ctypes.byref(o), ctypes.byref(nm), ctypes.byref(f),
                                             ctypes.byref(w), ctypes.byref(k)))
            self.offsets.append(o.value)
            self.numels.append(nm.value)
            self.first_slice.append(f.value)
            self.widths.append(w.value)
            self.kepts.append(k.value)

    def pack(self, arrays):
        """list of numpy tensors -> one packed flat CUDA tensor."""
        import torch
        flat = np.zeros(self.N, dtype=np.float64 if self.precision == "fp64" else np.float32)
        for t, X in enumerate(arrays):
            flat[self.offsets[t]: self.offsets[t] + self.numels[t]] = np.asarray(X).ravel(order="F")
        return torch.from_numpy(flat).to(device="cuda")

    def unpack(self, packed):
        host = packed.detach().double().cpu().numpy()
        return [host[o: o + n].reshape(s, order="F") for o, n, s in zip(self.offsets, self.numels, self.shapes)]

    def gnhtsvt(self, X, tau, penalty=("l1", ()), call_index=0, out=None, workspace=None, stats=False):
        """tau: one threshold per tensor (sequence or CUDA float64 tensor)."""
        import torch
        check_tensor(X, "X", self.torch_dtype, self.N)
        if out is None:
            out = torch.empty_like(X)
        if workspace is None:
            workspace = self.alloc_workspace()
        if not torch.is_tensor(tau):
            tau = torch.tensor(np.asarray(tau, dtype=np.float64), device="cuda")
        self._check_io(X, out, workspace, self.workspace_bytes)
        check_tensor(tau, "tau", torch.float64, len(self.shapes))
        wp, wn = self._aligned(workspace)
        sig = kept = None
        if stats:
            sig = torch.empty(self.n_slices * self.width, dtype=torch.float64, device=X.device)
            kept = torch.empty(self.n_slices, dtype=torch.int32, device=X.device)
        pen = _penalty(penalty)
        _check(_lib.ht_batch_gnhtsvt(self._h, _ptr(X), _ptr(out), _ptr(tau), ctypes.byref(pen), int(call_index),
                                     wp, wn, _stream(), _ptr(sig), _ptr(kept)))
        self._tau_keep = tau
        if stats:
            return out, sig.view(self.n_slices, self.width), kept
        return out


class Mlp:
    """The width-predicting network: parameters and Adam moments as flat FP32
    CUDA tensors; forward, gradient and training steps run in the library."""

    def __init__(self, theta):
        import torch
        self.n_params = _lib.ht_mlp_param_count()
        theta = torch.as_tensor(np.asarray(theta, dtype=np.float32)) if not torch.is_tensor(theta) else theta
        assert theta.numel() == self.n_params
        self.theta = theta.to(device="cuda", dtype=torch.float32).contiguous()
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.step = 0
        self._ws = None

    def _workspace(self, n):
        import torch
        sz = ctypes.c_size_t()
        _check(_lib.ht_mlp_workspace_size(int(n), ctypes.byref(sz)))
        if self._ws is None or self._ws.numel() < sz.value + 256:
            self._ws = torch.empty(sz.value + 256, dtype=torch.uint8, device="cuda")
        return Plan._aligned(self._ws)

    def forward(self, X):
        import torch
        z = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
        _check(_lib.ht_mlp_forward(_ptr(self.theta), _ptr(X), _ptr(z), int(X.shape[0]), _stream()))
        return z

    def grad(self, X, y):
        import torch
        g = torch.empty_like(self.theta)
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        wp, wn = self._workspace(X.shape[0])
        _check(_lib.ht_mlp_grad(_ptr(self.theta), _ptr(X), _ptr(y), int(X.shape[0]), _ptr(g), _ptr(loss), wp, wn,
                                _stream()))
        return g, loss

    def train_step(self, X, y, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        import torch
        self.step += 1
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        wp, wn = self._workspace(X.shape[0])
        _check(_lib.ht_mlp_train_step(_ptr(self.theta), _ptr(self.m), _ptr(self.v), self.step, _ptr(X), _ptr(y),
                                      int(X.shape[0]), float(lr), float(beta1), float(beta2), float(eps), _ptr(loss),
                                      wp, wn, _stream()))
        return loss


class Admm:
    """Pure-L ADMM (completion / robust completion) driven through the C-ABI."""

    def __init__(self, plan, model="completion", phi=("l1", ()), psi=("l1", ()), lam=0.0, mu0=1e-3,
                 vartheta=1.15, mu_max=1e10):
        self.plan = plan
        self.prm = _AdmmParams(MODELS[model], _penalty(phi), _penalty(psi), float(lam), float(mu0),
                               float(vartheta), float(mu_max))

    def _check_state(self, L, E, Y, workspace):
        import torch
        dt, N = self.plan.torch_dtype, self.plan.N
        for t, name in ((L, "L"), (E, "E"), (Y, "Y")):
            check_tensor(t, name, dt, N)
        check_tensor(workspace, "workspace", torch.uint8, 0)  # its size is checked by the library

    def init(self, L, E, Y, workspace):
        self._check_state(L, E, Y, workspace)
        wp, wn = Plan._aligned(workspace)
        _check(_lib.ht_admm_init(self.plan._h, ctypes.byref(self.prm), _ptr(L), _ptr(E), _ptr(Y), wp, wn, _stream()))

    def iterate(self, M, mask, L, E, Y, n_iter, workspace):
        import torch
        self._check_state(L, E, Y, workspace)
        check_tensor(M, "M", self.plan.torch_dtype, self.plan.N)
        check_tensor(mask, "mask", torch.uint8, self.plan.N)
        wp, wn = Plan._aligned(workspace)
        _check(_lib.ht_admm_iterate(self.plan._h, ctypes.byref(self.prm), _ptr(M), _ptr(mask), _ptr(L), _ptr(E),
                                    _ptr(Y), int(n_iter), wp, wn, _stream()))

    def set_truth(self, truth):
        """Register the ground truth L* (None clears it): every later iterate()
        call ends with the RSE ||L - L*||_F / ||L*||_F in the solver state."""
        if truth is not None:
            check_tensor(truth, "truth", self.plan.torch_dtype, self.plan.N)
        self._truth_keep = truth
        _check(_lib.ht_admm_set_truth(self.plan._h, _ptr(truth)))

    def stats(self, workspace):
        """Solver scalars; raises HtError ERR_NONFINITE when a stopping term is
        NaN or infinite or a slice met a non-finite value."""
        wp, _wn = Plan._aligned(workspace)
        st = _AdmmStats()
        _check(_lib.ht_admm_get_stats(self.plan._h, wp, _stream(), ctypes.byref(st)))
        return {"iteration": st.iteration, "mu": st.mu, "dL": st.dL, "dE": st.dE, "resid": st.resid, "rse": st.rse}
