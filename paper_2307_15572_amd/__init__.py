"""MI355X randomized truncated SVD (arXiv:2307.15572, section "Randomized
matrix decompositions") behind the C ABI of include/rsvd.h.

This module only marshals arguments: torch supplies device memory and the
current stream, and every step of the decomposition runs in the HIP kernels
of librsvd.so. There is no CPU fallback; importing works without a GPU, but
any call fails loudly when the library or a device is missing.
"""

import ctypes
import os
from dataclasses import dataclass

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG_DIR, "librsvd.so")

RSVD_OK, RSVD_EINVAL, RSVD_ENOMEM, RSVD_EHIP, RSVD_EUNSUPPORTED = range(5)
RANK_MODES = {"fixed": 0, "percent": 1, "rel_threshold": 2, "frob_tail": 3}
PRECISIONS = {"fp64": 0, "mixed_fp32": 1, "mixed_bf16": 2, "mixed_bf16_split": 3,
              "mixed_fp32_sliced": 4}
FORMS = {"svd": 0, "symmetric": 1}
FLAG_FULL_SVD = 1 << 0
FLAG_RANK_CAPPED = 1 << 1
FLAG_QR_FALLBACK = 1 << 2
FLAG_JACOBI_MAXSWEEP = 1 << 3
FLAG_NONFINITE_INPUT = 1 << 4
FLAG_ZERO_SIGMA = 1 << 5
FLAG_ADAPT_LIMIT = 1 << 6
FLAG_SYNC_TIMEOUT = 1 << 7
FLAG_POSTERIOR_FAIL = 1 << 8
FLAG_UNCONVERGED = 1 << 9

EXPORTED = (
    "rsvd_plan", "rsvd_plan_l", "rsvd_run", "rsvd_destroy", "rsvd_strerror",
    "rsvd_gaussian_omega", "rsvd_dgemm_work_bytes", "rsvd_dgemm", "rsvd_gemm",
    "rsvd_sliced_gemm_work_bytes",
    "rsvd_bf16_gemm_work_bytes", "rsvd_bf16_gemm",
    "rsvd_orth_work_bytes", "rsvd_orth", "rsvd_small_svd_work_bytes", "rsvd_small_svd",
    "rsvd_trace_enable", "rsvd_trace_collect",
    "rsvd_batch_plan", "rsvd_batch_run", "rsvd_batch_info", "rsvd_batch_destroy",
    "rsvd_mlp_init", "rsvd_mlp_forward", "rsvd_mlp_grad", "rsvd_mlp_train_step",
    "rsvd_pilot_work_bytes", "rsvd_pilot_features",
    "rsvd_tune", "rsvd_batch_tune", "rsvd_tune_entries", "rsvd_tune_clear", "rsvd_tune_set",
    "rsvd_run_noalloc", "rsvd_noalloc_max_bytes",
    "rsvd_residual_work_bytes", "rsvd_residual",
    "rsvd_factor_transform_work_bytes", "rsvd_factor_transform",
    "rsvd_mlp_targets", "rsvd_mlp_predict", "rsvd_size_label", "rsvd_mlp_save", "rsvd_mlp_load",
)
MLP_PARAMS, MLP_IN, MLP_OUT, MLP_MAX_BATCH, PILOT_COLS = 5443, 16, 3, 128, 32
TRACE_PHASES = ("stream_gemm", "qr", "small_svd", "lift_signs", "residual", "omega", "other",
                "bf16_planes", "bf16_gemm", "fp32_gemm")


class RsvdError(RuntimeError):
    pass


class Problem(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
        ("k_cap", ctypes.c_int64),
        ("symmetric", ctypes.c_int32), ("rank_mode", ctypes.c_int32),
        ("rank_param", ctypes.c_double),
        ("oversample", ctypes.c_int32), ("power_iters", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("trailing_hp", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("channel", ctypes.c_uint64),
        ("want_u", ctypes.c_int32), ("want_v", ctypes.c_int32),
        ("want_residual", ctypes.c_int32), ("max_sweeps", ctypes.c_int32),
        ("adaptive", ctypes.c_int32), ("block", ctypes.c_int32), ("l_max", ctypes.c_int64),
        ("form", ctypes.c_int32), ("posterior", ctypes.c_int32),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("rank", ctypes.c_int64), ("l_used", ctypes.c_int64),
        ("residual", ctypes.c_double), ("rel_percent", ctypes.c_double),
        ("c_eq2", ctypes.c_double), ("c_sym", ctypes.c_double), ("fro2", ctypes.c_double),
        ("sweeps", ctypes.c_int32), ("flags", ctypes.c_uint32),
        ("err_est", ctypes.c_double), ("blocks", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


_lib = None


def lib():
    """Load librsvd.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RsvdError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, u64, dbl, sz = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                  ctypes.c_uint64, ctypes.c_double, ctypes.c_size_t)
    L.rsvd_plan.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(vp), ctypes.POINTER(sz)]
    L.rsvd_plan.restype = ctypes.c_int
    L.rsvd_plan_l.argtypes = [vp]
    L.rsvd_plan_l.restype = i64
    L.rsvd_run.argtypes = [vp, vp, i64, vp, i64, vp, vp, i64, vp, i64, vp, vp, sz, vp]
    L.rsvd_run.restype = ctypes.c_int
    L.rsvd_run_noalloc.argtypes = [vp, vp, i64, vp, i64, vp, vp, i64, vp, i64, vp, vp]
    L.rsvd_run_noalloc.restype = ctypes.c_int
    L.rsvd_noalloc_max_bytes.argtypes = []
    L.rsvd_noalloc_max_bytes.restype = sz
    L.rsvd_residual_work_bytes.argtypes = [i64, i64, i64]
    L.rsvd_residual_work_bytes.restype = sz
    L.rsvd_residual.argtypes = [i64, i64, i64, vp, i64, vp, vp, i64, vp, i64, vp, vp, sz, vp]
    L.rsvd_residual.restype = ctypes.c_int
    L.rsvd_factor_transform_work_bytes.argtypes = [i64, i64, i64, i32]
    L.rsvd_factor_transform_work_bytes.restype = sz
    L.rsvd_factor_transform.argtypes = [i64, i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, vp, i64,
                                        vp, sz, vp]
    L.rsvd_factor_transform.restype = ctypes.c_int
    L.rsvd_destroy.argtypes = [vp]
    L.rsvd_destroy.restype = None
    L.rsvd_strerror.argtypes = [ctypes.c_int]
    L.rsvd_strerror.restype = ctypes.c_char_p
    L.rsvd_gaussian_omega.argtypes = [i64, i64, i64, u64, u64, vp, i64, vp]
    L.rsvd_gaussian_omega.restype = ctypes.c_int
    L.rsvd_dgemm_work_bytes.argtypes = [i64, i64, i64, i32]
    L.rsvd_dgemm_work_bytes.restype = sz
    L.rsvd_sliced_gemm_work_bytes.argtypes = [i64, i64, i64]
    L.rsvd_sliced_gemm_work_bytes.restype = sz
    L.rsvd_dgemm.argtypes = [i32, i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64, vp, sz, vp]
    L.rsvd_dgemm.restype = ctypes.c_int
    L.rsvd_gemm.argtypes = [i32, i32, i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64, vp, sz, vp]
    L.rsvd_gemm.restype = ctypes.c_int
    L.rsvd_bf16_gemm_work_bytes.argtypes = [i64, i64, i64, i32]
    L.rsvd_bf16_gemm_work_bytes.restype = sz
    L.rsvd_bf16_gemm.argtypes = [i32, i32, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp, sz, vp]
    L.rsvd_bf16_gemm.restype = ctypes.c_int
    L.rsvd_orth_work_bytes.argtypes = [i64, i64]
    L.rsvd_orth_work_bytes.restype = sz
    L.rsvd_orth.argtypes = [i64, i64, vp, i64, vp, vp, vp, sz, vp]
    L.rsvd_orth.restype = ctypes.c_int
    L.rsvd_small_svd_work_bytes.argtypes = [i64]
    L.rsvd_small_svd_work_bytes.restype = sz
    L.rsvd_small_svd.argtypes = [i64, vp, vp, vp, vp, i32, vp, vp, vp, sz, vp]
    L.rsvd_small_svd.restype = ctypes.c_int
    L.rsvd_trace_enable.argtypes = [i32]
    L.rsvd_trace_enable.restype = None
    L.rsvd_trace_collect.argtypes = [ctypes.POINTER(dbl), ctypes.POINTER(i64)]
    L.rsvd_trace_collect.restype = ctypes.c_int
    pp = ctypes.POINTER
    L.rsvd_batch_plan.argtypes = [pp(Problem), i64, i32, i32, pp(vp), pp(sz)]
    L.rsvd_batch_plan.restype = ctypes.c_int
    L.rsvd_batch_run.argtypes = [vp, pp(vp), pp(i64), pp(vp), pp(vp), pp(i64), pp(vp), pp(i64),
                                 vp, vp, sz, vp]
    L.rsvd_batch_run.restype = ctypes.c_int
    L.rsvd_tune.argtypes = [vp, vp, i64, vp, i64, vp, vp, i64, vp, i64, vp, vp, sz, i32, pp(i32), vp]
    L.rsvd_tune.restype = ctypes.c_int
    L.rsvd_batch_tune.argtypes = [vp, pp(vp), pp(i64), pp(vp), pp(vp), pp(i64), pp(vp), pp(i64),
                                  vp, vp, sz, i32, pp(i32), vp]
    L.rsvd_batch_tune.restype = ctypes.c_int
    L.rsvd_tune_entries.argtypes = [i64, pp(i32), pp(i64), pp(i32)]
    L.rsvd_tune_entries.restype = i64
    L.rsvd_tune_clear.argtypes = []
    L.rsvd_tune_clear.restype = None
    L.rsvd_tune_set.argtypes = [i32, i32, i32, i64, i64, i64, i32, i32, i32]
    L.rsvd_tune_set.restype = ctypes.c_int
    L.rsvd_batch_info.argtypes = [vp, pp(i32), pp(i32)]
    L.rsvd_batch_info.restype = ctypes.c_int
    L.rsvd_batch_destroy.argtypes = [vp]
    L.rsvd_batch_destroy.restype = None
    fp = ctypes.c_void_p
    L.rsvd_mlp_init.argtypes = [fp, u64, vp]
    L.rsvd_mlp_init.restype = ctypes.c_int
    L.rsvd_mlp_forward.argtypes = [fp, fp, i64, fp, vp]
    L.rsvd_mlp_forward.restype = ctypes.c_int
    L.rsvd_mlp_grad.argtypes = [fp, fp, fp, i64, fp, fp, vp]
    L.rsvd_mlp_grad.restype = ctypes.c_int
    L.rsvd_mlp_train_step.argtypes = [fp, fp, fp, i64, fp, fp, i64, ctypes.c_float, fp, vp]
    L.rsvd_mlp_train_step.restype = ctypes.c_int
    L.rsvd_mlp_targets.argtypes = [vp, i64, fp, fp, vp]
    L.rsvd_mlp_targets.restype = ctypes.c_int
    L.rsvd_mlp_predict.argtypes = [fp, fp, fp, i64, vp, vp, vp]
    L.rsvd_mlp_predict.restype = ctypes.c_int
    L.rsvd_size_label.argtypes = [vp, i64, i64, i64, i64, vp, vp]
    L.rsvd_size_label.restype = ctypes.c_int
    L.rsvd_mlp_save.argtypes = [ctypes.c_char_p, fp, fp, vp]
    L.rsvd_mlp_save.restype = ctypes.c_int
    L.rsvd_mlp_load.argtypes = [ctypes.c_char_p, fp, fp, vp]
    L.rsvd_mlp_load.restype = ctypes.c_int
    L.rsvd_pilot_work_bytes.argtypes = [i64, i64]
    L.rsvd_pilot_work_bytes.restype = sz
    L.rsvd_pilot_features.argtypes = [vp, i64, i64, i64, u64, u64, fp, vp, sz, vp]
    L.rsvd_pilot_features.restype = ctypes.c_int
    _lib = L
    return L


def _check(status, what):
    if status != RSVD_OK:
        msg = lib().rsvd_strerror(status).decode()
        raise RsvdError(f"{what}: {msg} (status {status})")


def check_flags(flags, what):
    """Raise on the result flags that make a result invalid: non-finite input
    and a grid-wide barrier that gave up waiting (SYNC_TIMEOUT)."""
    if flags & FLAG_NONFINITE_INPUT:
        raise RsvdError(f"{what}: A holds NaN or Inf")
    if flags & FLAG_SYNC_TIMEOUT:
        raise RsvdError(f"{what}: a grid-wide barrier timed out (results invalid)")


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RsvdError("no GPU visible: the rSVD library runs only on the device")
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _workspace(torch, nbytes, device):
    """Device workspace with a 256-byte aligned start (kept alive by the caller)."""
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, ctypes.c_void_p(buf.data_ptr() + off), int(nbytes)


def _check_matrix(torch, A, name):
    if not (A.is_cuda and A.dtype == torch.float64 and A.dim() == 2):
        raise RsvdError(f"{name} must be a 2-D float64 CUDA tensor")
    if A.stride(1) != 1:
        raise RsvdError(f"{name} must be row-major (last stride 1)")


@dataclass
class RsvdOutput:
    S: object          # (rank,) decreasing
    U: object          # (m, rank) or None
    V: object          # (n, rank) or None
    rank: int
    l: int
    residual: float
    rel_percent: float
    c_eq2: float
    c_sym: float
    fro2: float
    sweeps: int
    flags: int
    err_est: float = float("nan")   # adaptive: last error estimate of the basis
    blocks: int = 0                 # adaptive: growth steps
    S_all: object = None            # every computed value (min(k_cap, l) of them)


def make_problem(m, n, k, p, q, *, symmetric=False, rank_mode="fixed", rank_param=None,
                 precision="fp64", trailing_hp=1, seed=0, channel=0, want_u=True, want_v=True,
                 want_residual=True, max_sweeps=0, k_cap=0, adaptive=False, block=0, l_max=0,
                 form="svd", posterior=0):
    """Fill an rsvd_problem record."""
    pr = Problem()
    pr.m, pr.n, pr.k, pr.k_cap = int(m), int(n), int(k), int(k_cap)
    pr.symmetric = int(bool(symmetric))
    pr.rank_mode = RANK_MODES[rank_mode]
    pr.rank_param = float(rank_param) if rank_param is not None else float(k)
    pr.oversample, pr.power_iters = int(p), int(q)
    pr.precision = PRECISIONS[precision]
    pr.trailing_hp = int(trailing_hp)
    pr.seed, pr.channel = int(seed) & (2**64 - 1), int(channel) & (2**64 - 1)
    pr.want_u, pr.want_v = int(bool(want_u)), int(bool(want_v))
    pr.want_residual, pr.max_sweeps = int(bool(want_residual)), int(max_sweeps)
    pr.adaptive, pr.block, pr.l_max = int(bool(adaptive)), int(block), int(l_max)
    pr.form = FORMS[form]
    pr.posterior = int(posterior)
    return pr


class Plan:
    """An immutable plan for one problem shape (wraps rsvd_plan).

    adaptive=True grows l by blocks of `block` columns up to l_max (the
    adaptive range finder of the C ABI); k is then ignored and rank_mode must
    be "rel_threshold" or "frob_tail" with rank_param = tau. form="symmetric"
    (with symmetric=True) takes the l x l core Q^T A Q instead of Q^T A.
    """

    def __init__(self, m, n, k, p, q, *, symmetric=False, rank_mode="fixed", rank_param=None,
                 precision="fp64", trailing_hp=1, seed=0, channel=0, want_u=True, want_v=True,
                 want_residual=True, max_sweeps=0, k_cap=0, adaptive=False, block=0, l_max=0,
                 form="svd", posterior=0):
        L = lib()
        pr = make_problem(m, n, k, p, q, symmetric=symmetric, rank_mode=rank_mode,
                          rank_param=rank_param, precision=precision, trailing_hp=trailing_hp,
                          seed=seed, channel=channel, want_u=want_u, want_v=want_v,
                          want_residual=want_residual, max_sweeps=max_sweeps, k_cap=k_cap,
                          adaptive=adaptive, block=block, l_max=l_max, form=form,
                          posterior=posterior)
        self.problem = pr
        h = ctypes.c_void_p()
        ws = ctypes.c_size_t()
        _check(L.rsvd_plan(ctypes.byref(pr), ctypes.byref(h), ctypes.byref(ws)), "rsvd_plan")
        self._h = h
        self.workspace_bytes = ws.value
        self.l = L.rsvd_plan_l(h)
        self.kc = min(int(k_cap) if k_cap else self.l, self.l)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.rsvd_destroy(h)
            self._h = None

    def allocate(self, device="cuda"):
        """Output and workspace buffers for run_into (allocated once, reused)."""
        torch = _torch()
        pr = self.problem
        bufs = {
            "S": torch.empty(self.kc, dtype=torch.float64, device=device),
            "U": torch.empty(pr.m, self.kc, dtype=torch.float64, device=device) if pr.want_u else None,
            "V": torch.empty(pr.n, self.kc, dtype=torch.float64, device=device) if pr.want_v else None,
            "res": torch.zeros(ctypes.sizeof(Result), dtype=torch.uint8, device=device),
        }
        bufs["work_buf"], bufs["work"], bufs["work_bytes"] = _workspace(torch, self.workspace_bytes, device)
        return bufs

    def run_into(self, A, bufs, omega=None):
        """Enqueue one decomposition on the current stream (no synchronization)."""
        torch = _torch()
        _check_matrix(torch, A, "A")
        pr = self.problem
        if tuple(A.shape) != (pr.m, pr.n):
            raise RsvdError(f"A has shape {tuple(A.shape)}, plan expects {(pr.m, pr.n)}")
        ldo = 0
        if omega is not None:
            _check_matrix(torch, omega, "omega")
            if omega.shape[0] != pr.n or omega.shape[1] < self.l:
                raise RsvdError("omega must be n x l")
            ldo = omega.stride(0)
        U, V = bufs["U"], bufs["V"]
        st = lib().rsvd_run(self._h, _ptr(A), A.stride(0), _ptr(omega), ldo, _ptr(bufs["S"]),
                            _ptr(U), U.stride(0) if U is not None else 0,
                            _ptr(V), V.stride(0) if V is not None else 0,
                            _ptr(bufs["res"]), bufs["work"], bufs["work_bytes"],
                            _stream(torch, A.device))
        _check(st, "rsvd_run")

    def run_into_noalloc(self, A, bufs, omega=None):
        """Enqueue one decomposition through rsvd_run_noalloc: the library's
        static workspace instead of bufs' (which needs no "work" entry)."""
        torch = _torch()
        _check_matrix(torch, A, "A")
        pr = self.problem
        if tuple(A.shape) != (pr.m, pr.n):
            raise RsvdError(f"A has shape {tuple(A.shape)}, plan expects {(pr.m, pr.n)}")
        ldo = 0
        if omega is not None:
            _check_matrix(torch, omega, "omega")
            if omega.shape[0] != pr.n or omega.shape[1] < self.l:
                raise RsvdError("omega must be n x l")
            ldo = omega.stride(0)
        U, V = bufs["U"], bufs["V"]
        st = lib().rsvd_run_noalloc(self._h, _ptr(A), A.stride(0), _ptr(omega), ldo,
                                    _ptr(bufs["S"]), _ptr(U), U.stride(0) if U is not None else 0,
                                    _ptr(V), V.stride(0) if V is not None else 0,
                                    _ptr(bufs["res"]), _stream(torch, A.device))
        _check(st, "rsvd_run_noalloc")

    def tune(self, A, bufs, reps=3, omega=None):
        """Autotune the tile shapes of this decomposition's products (see
        rsvd_tune); synchronizes. bufs then hold the tuned run's result.
        Returns the number of shapes added to the process-wide table."""
        torch = _torch()
        _check_matrix(torch, A, "A")
        pr = self.problem
        if tuple(A.shape) != (pr.m, pr.n):
            raise RsvdError(f"A has shape {tuple(A.shape)}, plan expects {(pr.m, pr.n)}")
        ldo = omega.stride(0) if omega is not None else 0
        U, V = bufs["U"], bufs["V"]
        n = ctypes.c_int32(0)
        _check(lib().rsvd_tune(self._h, _ptr(A), A.stride(0), _ptr(omega), ldo, _ptr(bufs["S"]),
                               _ptr(U), U.stride(0) if U is not None else 0,
                               _ptr(V), V.stride(0) if V is not None else 0,
                               _ptr(bufs["res"]), bufs["work"], bufs["work_bytes"], int(reps),
                               ctypes.byref(n), _stream(torch, A.device)), "rsvd_tune")
        return n.value

    def result(self, bufs):
        """Synchronize and read the device result record."""
        torch = _torch()
        torch.cuda.synchronize(bufs["S"].device)
        raw = bytes(bufs["res"].cpu().numpy().tobytes())
        return Result.from_buffer_copy(raw)


class BatchPlan:
    """Independent decompositions run together (wraps rsvd_batch_plan).

    problems: list of dicts with the keyword arguments of make_problem
    (m, n, k, p, q, ...). lanes: concurrent streams (0 = 4). use_graph:
    capture the run into a hipGraph on first use and replay it.
    """

    def __init__(self, problems, lanes=0, use_graph=True):
        L = lib()
        self.count = len(problems)
        arr = (Problem * self.count)()
        for c, kw in enumerate(problems):
            kw = dict(kw)
            m, n, k, p, q = (kw.pop(x) for x in ("m", "n", "k", "p", "q"))
            arr[c] = make_problem(m, n, k, p, q, **kw)
        self.problems = arr
        h = ctypes.c_void_p()
        ws = ctypes.c_size_t()
        _check(L.rsvd_batch_plan(arr, self.count, int(lanes), int(bool(use_graph)),
                                 ctypes.byref(h), ctypes.byref(ws)), "rsvd_batch_plan")
        self._h = h
        self.workspace_bytes = ws.value
        # per-channel sketch width and output columns (same rules as Plan)
        self.l, self.kc = [], []
        for pr in arr:
            one = ctypes.c_void_p()
            _check(L.rsvd_plan(ctypes.byref(pr), ctypes.byref(one), None), "rsvd_plan")
            l = L.rsvd_plan_l(one)
            L.rsvd_destroy(one)
            self.l.append(l)
            self.kc.append(min(pr.k_cap if pr.k_cap else l, l))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.rsvd_batch_destroy(h)
            self._h = None

    def lanes_of(self):
        out = (ctypes.c_int32 * self.count)()
        _check(lib().rsvd_batch_info(self._h, out, None), "rsvd_batch_info")
        return list(out)

    def graph_used(self):
        g = ctypes.c_int32()
        _check(lib().rsvd_batch_info(self._h, None, ctypes.byref(g)), "rsvd_batch_info")
        return bool(g.value)

    def allocate(self, device="cuda"):
        torch = _torch()
        S, U, V = [], [], []
        for pr, kc in zip(self.problems, self.kc):
            S.append(torch.empty(kc, dtype=torch.float64, device=device))
            U.append(torch.empty(pr.m, kc, dtype=torch.float64, device=device) if pr.want_u else None)
            V.append(torch.empty(pr.n, kc, dtype=torch.float64, device=device) if pr.want_v else None)
        bufs = {"S": S, "U": U, "V": V,
                "res": torch.zeros(self.count * ctypes.sizeof(Result), dtype=torch.uint8, device=device)}
        bufs["work_buf"], bufs["work"], bufs["work_bytes"] = _workspace(torch, self.workspace_bytes, device)
        return bufs

    def _pointers(self, torch, As, bufs):
        n = self.count
        if len(As) != n:
            raise RsvdError(f"expected {n} matrices")
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        Ap, lda = (vp * n)(), (i64 * n)()
        Sp, Up, Vp = (vp * n)(), (vp * n)(), (vp * n)()
        ldu, ldv = (i64 * n)(), (i64 * n)()
        for c, (A, pr) in enumerate(zip(As, self.problems)):
            _check_matrix(torch, A, f"A[{c}]")
            if tuple(A.shape) != (pr.m, pr.n):
                raise RsvdError(f"A[{c}] has shape {tuple(A.shape)}, plan expects {(pr.m, pr.n)}")
            Ap[c], lda[c] = A.data_ptr(), A.stride(0)
            Sp[c] = bufs["S"][c].data_ptr()
            U, V = bufs["U"][c], bufs["V"][c]
            Up[c], ldu[c] = (U.data_ptr(), U.stride(0)) if U is not None else (0, 0)
            Vp[c], ldv[c] = (V.data_ptr(), V.stride(0)) if V is not None else (0, 0)
        self._keep = (Ap, lda, Sp, Up, Vp, ldu, ldv)
        return self._keep

    def run_into(self, As, bufs):
        """Enqueue every channel on the current stream (no synchronization)."""
        torch = _torch()
        Ap, lda, Sp, Up, Vp, ldu, ldv = self._pointers(torch, As, bufs)
        _check(lib().rsvd_batch_run(self._h, Ap, lda, Sp, Up, ldu, Vp, ldv, _ptr(bufs["res"]),
                                    bufs["work"], bufs["work_bytes"], _stream(torch, As[0].device)),
               "rsvd_batch_run")

    def tune(self, As, bufs, reps=3):
        """Autotune the tile shapes of every channel's products (see
        rsvd_batch_tune); synchronizes. Returns the number of shapes added."""
        torch = _torch()
        Ap, lda, Sp, Up, Vp, ldu, ldv = self._pointers(torch, As, bufs)
        n = ctypes.c_int32(0)
        _check(lib().rsvd_batch_tune(self._h, Ap, lda, Sp, Up, ldu, Vp, ldv, _ptr(bufs["res"]),
                                     bufs["work"], bufs["work_bytes"], int(reps), ctypes.byref(n),
                                     _stream(torch, As[0].device)), "rsvd_batch_tune")
        return n.value

    def results(self, bufs, check=True):
        """Synchronize and read the count result records. check: raise when a
        channel's flags mark its result invalid (see check_flags)."""
        torch = _torch()
        torch.cuda.synchronize(bufs["res"].device)
        raw = bytes(bufs["res"].cpu().numpy().tobytes())
        sz = ctypes.sizeof(Result)
        out = [Result.from_buffer_copy(raw[c * sz:(c + 1) * sz]) for c in range(self.count)]
        if check:
            for c, r in enumerate(out):
                check_flags(r.flags, f"batch channel {c}")
        return out


def run(A, k, p, q, *, omega=None, **kw):
    """Randomized SVD of the CUDA float64 matrix A (m x n); returns RsvdOutput."""
    torch = _torch()
    _check_matrix(torch, A, "A")
    m, n = A.shape
    plan = Plan(m, n, k, p, q, **kw)
    bufs = plan.allocate(A.device)
    plan.run_into(A, bufs, omega=omega)
    r = plan.result(bufs)
    check_flags(r.flags, "rsvd_run")
    rank = int(r.rank)
    return RsvdOutput(
        S=bufs["S"][:rank], U=bufs["U"][:, :rank] if bufs["U"] is not None else None,
        V=bufs["V"][:, :rank] if bufs["V"] is not None else None, rank=rank, l=int(r.l_used),
        residual=r.residual, rel_percent=r.rel_percent, c_eq2=r.c_eq2, c_sym=r.c_sym,
        fro2=r.fro2, sweeps=int(r.sweeps), flags=int(r.flags), err_est=r.err_est,
        blocks=int(r.blocks), S_all=bufs["S"][: min(plan.kc, int(r.l_used))],
    )


def residual(A, S, U, V, k):
    """Truncate a decomposition (S, U, V) of A at rank k: the Result record
    with the residual ||A - U_k S_k V_k^T||_F / ||A||_F, R% and both
    compression ratios for R_SVD = k (rsvd_residual)."""
    torch = _torch()
    _check_matrix(torch, A, "A")
    _check_matrix(torch, U, "U")
    _check_matrix(torch, V, "V")
    m, n = A.shape
    if U.shape[0] != m or V.shape[0] != n or min(U.shape[1], V.shape[1], S.numel()) < k:
        raise RsvdError("factors do not match A or hold fewer than k columns")
    S = S.contiguous()
    res = torch.zeros(ctypes.sizeof(Result), dtype=torch.uint8, device=A.device)
    L = lib()
    buf, w, wb = _workspace(torch, L.rsvd_residual_work_bytes(m, n, k), A.device)
    _check(L.rsvd_residual(m, n, k, _ptr(A), A.stride(0), _ptr(S), _ptr(U), U.stride(0), _ptr(V),
                           V.stride(0), _ptr(res), w, wb, _stream(torch, A.device)), "rsvd_residual")
    torch.cuda.synchronize(A.device)
    del buf
    return Result.from_buffer_copy(bytes(res.cpu().numpy().tobytes()))


def factor_transform(Ub, L, R=None):
    """Basis change on thin factors: (U^T L, U^T R) with U = Ub (N x Nb)
    streamed once for both (rsvd_factor_transform)."""
    torch = _torch()
    for t, name in ((Ub, "U"), (L, "L")) + (((R, "R"),) if R is not None else ()):
        _check_matrix(torch, t, name)
    N, Nb = Ub.shape
    k = L.shape[1]
    if L.shape[0] != N or (R is not None and tuple(R.shape) != (N, k)):
        raise RsvdError("factors must be N x k with N the rows of U")
    Lo = torch.empty(Nb, k, dtype=torch.float64, device=Ub.device)
    Ro = torch.empty(Nb, k, dtype=torch.float64, device=Ub.device) if R is not None else None
    lb = lib()
    buf, w, wb = _workspace(torch, lb.rsvd_factor_transform_work_bytes(N, Nb, k, int(R is not None)),
                            Ub.device)
    _check(lb.rsvd_factor_transform(N, Nb, k, _ptr(Ub), Ub.stride(0), _ptr(L), L.stride(0), _ptr(R),
                                    R.stride(0) if R is not None else 0, _ptr(Lo), k, _ptr(Ro),
                                    k if R is not None else 0, w, wb, _stream(torch, Ub.device)),
           "rsvd_factor_transform")
    torch.cuda.synchronize(Ub.device)
    del buf
    return Lo, Ro


def gaussian_omega(n, l, seed, channel=0, col0=0, device="cuda"):
    """The projection P (n x l) drawn by the library's Philox/Box-Muller kernel."""
    torch = _torch()
    out = torch.empty(n, l, dtype=torch.float64, device=device)
    _check(lib().rsvd_gaussian_omega(n, l, col0, seed & (2**64 - 1), channel & (2**64 - 1),
                                     _ptr(out), l, _stream(torch, out.device)),
           "rsvd_gaussian_omega")
    return out


def dgemm(A, B, trans_a=False, alpha=1.0, beta=0.0, C=None, precision="fp64"):
    """C = alpha op(A) B + beta C on the matrix cores (FP64 unless a mixed
    precision mode is named: "mixed_fp32" or "mixed_bf16")."""
    torch = _torch()
    _check_matrix(torch, A, "A")
    _check_matrix(torch, B, "B")
    m = A.shape[1] if trans_a else A.shape[0]
    k = A.shape[0] if trans_a else A.shape[1]
    if B.shape[0] != k:
        raise RsvdError("inner dimensions differ")
    n = B.shape[1]
    if C is None:
        C = torch.zeros(m, n, dtype=torch.float64, device=A.device)
    L = lib()
    if precision == "mixed_fp32_sliced":
        wb = L.rsvd_sliced_gemm_work_bytes(m, n, k)
    else:
        wb = L.rsvd_dgemm_work_bytes(m, n, k, int(trans_a))
    work = torch.empty(max(wb // 8, 1), dtype=torch.float64, device=A.device)
    _check(L.rsvd_gemm(PRECISIONS[precision], int(trans_a), m, n, k, alpha, _ptr(A), A.stride(0),
                       _ptr(B), B.stride(0), beta, _ptr(C), C.stride(0), _ptr(work), wb,
                       _stream(torch, A.device)),
           "rsvd_gemm")
    return C


def bf16_gemm(A, B, trans_a=False, split=False):
    """op(A) B from BF16 planes, as the BF16 schedules of run() compute their
    early products (split: hi + lo planes, three products per term)."""
    torch = _torch()
    _check_matrix(torch, A, "A")
    _check_matrix(torch, B, "B")
    m = A.shape[1] if trans_a else A.shape[0]
    k = A.shape[0] if trans_a else A.shape[1]
    if B.shape[0] != k:
        raise RsvdError("inner dimensions differ")
    n = B.shape[1]
    C = torch.empty(m, n, dtype=torch.float64, device=A.device)
    L = lib()
    wb = L.rsvd_bf16_gemm_work_bytes(m, n, k, int(split))
    buf, w, wbytes = _workspace(torch, wb, A.device)
    _check(L.rsvd_bf16_gemm(int(split), int(trans_a), m, n, k, _ptr(A), A.stride(0), _ptr(B),
                            B.stride(0), _ptr(C), C.stride(0), w, wbytes, _stream(torch, A.device)),
           "rsvd_bf16_gemm")
    torch.cuda.synchronize(A.device)
    del buf
    return C


TUNE_KINDS = {0: "fp64_stream", 1: "generic", 2: "residual", 3: "bf16_planes"}


def tune_table():
    """The autotuner's table: list of dicts (kind, arithmetic, transposed,
    M, N, K, and the chosen tiling)."""
    L = lib()
    n = L.rsvd_tune_entries(0, None, None, None)
    if n == 0:
        return []
    kind = (ctypes.c_int32 * n)()
    mnk = (ctypes.c_int64 * (3 * n))()
    cfg = (ctypes.c_int32 * (3 * n))()
    L.rsvd_tune_entries(n, kind, mnk, cfg)
    out = []
    for i in range(n):
        kd = kind[i]
        k0 = TUNE_KINDS.get(kd // 100, str(kd // 100))
        ent = {"kind": k0, "arith": (kd // 10) % 10, "trans": kd % 10,
               "M": mnk[3 * i], "N": mnk[3 * i + 1], "K": mnk[3 * i + 2]}
        a, b, c = cfg[3 * i], cfg[3 * i + 1], cfg[3 * i + 2]
        if k0 == "bf16_planes":
            ent.update(rows_per_wave=16 * a, splits=b, column_groups=c)
        elif k0 == "residual":
            ent.update(waves=a, column_tiles=b, registers=c)
        elif k0 == "generic":
            ent.update(splits=b)
        else:
            ent.update(waves=a, splits=b)
        out.append(ent)
    return out


def tune_clear():
    """Empty the autotuner's table (later products use the heuristics)."""
    lib().rsvd_tune_clear()


def tune_set(kind, M, N, K, arith=0, trans=0, **tiling):
    """Pin the tiling of one product key. kind: "fp64_stream", "generic",
    "residual" or "bf16_planes"; tiling keywords as tune_table() reports them
    (waves, splits, rows_per_wave, column_groups, column_tiles, registers)."""
    kinds = {v: k for k, v in TUNE_KINDS.items()}
    kd = kinds[kind]
    if kind == "bf16_planes":
        a, b, c = tiling["rows_per_wave"] // 16, tiling.get("splits", 1), tiling.get("column_groups", 0)
    elif kind == "generic":
        a, b, c = 0, tiling["splits"], 0
    elif kind == "residual":
        a, b, c = tiling["waves"], tiling.get("column_tiles", 0), tiling.get("registers", 0)
    else:
        a, b, c = tiling["waves"], tiling.get("splits", 1), 0
    _check(lib().rsvd_tune_set(kd, int(arith), int(trans), M, N, K, a, b, c), "rsvd_tune_set")


def orth(Y):
    """Thin QR of a tall panel: returns (Q, X, flags) with Y = Q X."""
    torch = _torch()
    _check_matrix(torch, Y, "Y")
    m, l = Y.shape
    Q = Y.clone().contiguous()
    X = torch.empty(l, l, dtype=torch.float64, device=Y.device)
    flags = torch.zeros(1, dtype=torch.int32, device=Y.device)
    L = lib()
    wb = L.rsvd_orth_work_bytes(m, l)
    buf, w, wbytes = _workspace(torch, wb, Y.device)
    _check(L.rsvd_orth(m, l, _ptr(Q), l, _ptr(X), _ptr(flags), w, wbytes, _stream(torch, Y.device)),
           "rsvd_orth")
    torch.cuda.synchronize(Y.device)
    del buf
    fl = int(flags.item()) & 0xFFFFFFFF
    check_flags(fl, "rsvd_orth")
    return Q, X, fl


def small_svd(R, max_sweeps=0):
    """SVD of an upper-triangular l x l R: R^T = Us diag(s) W^T. Returns (s, Us, W, sweeps, flags)."""
    torch = _torch()
    _check_matrix(torch, R, "R")
    R = R.contiguous()
    l = R.shape[0]
    s = torch.empty(l, dtype=torch.float64, device=R.device)
    Us = torch.empty(l, l, dtype=torch.float64, device=R.device)
    W = torch.empty(l, l, dtype=torch.float64, device=R.device)
    sw = torch.zeros(1, dtype=torch.int32, device=R.device)
    fl = torch.zeros(1, dtype=torch.int32, device=R.device)
    L = lib()
    wb = L.rsvd_small_svd_work_bytes(l)
    buf, w, wbytes = _workspace(torch, wb, R.device)
    _check(L.rsvd_small_svd(l, _ptr(R), _ptr(s), _ptr(Us), _ptr(W), max_sweeps,
                            _ptr(sw), _ptr(fl), w, wbytes, _stream(torch, R.device)),
           "rsvd_small_svd")
    torch.cuda.synchronize(R.device)
    del buf
    flags = int(fl.item()) & 0xFFFFFFFF
    check_flags(flags, "rsvd_small_svd")
    return s, Us, W, int(sw.item()), flags


def pilot_features(A, seed, channel=0, work=None, out=None):
    """16 FP32 features of the pilot sketch of A (see include/rsvd.h), into
    out (a contiguous device FP32 vector of 16, e.g. a row of a batch's
    feature matrix) or a new tensor."""
    torch = _torch()
    _check_matrix(torch, A, "A")
    m, n = A.shape
    if out is None:
        feat = torch.empty(MLP_IN, dtype=torch.float32, device=A.device)
    else:
        if (out.dtype != torch.float32 or out.numel() != MLP_IN or not out.is_contiguous()
                or out.device != A.device):
            raise RsvdError("out: a contiguous FP32 vector of 16 on the device of A")
        feat = out
    L = lib()
    wb = L.rsvd_pilot_work_bytes(m, n)
    if work is None or work[2] < wb:
        work = _workspace(torch, wb, A.device)
    _check(L.rsvd_pilot_features(_ptr(A), A.stride(0), m, n, seed & (2**64 - 1),
                                 channel & (2**64 - 1), _ptr(feat), work[1], work[2],
                                 _stream(torch, A.device)), "rsvd_pilot_features")
    return feat, work


def size_label(S, k, n, l_min=0):
    """(k, p, q) label of a channel from a spectrum the method computed (S:
    device FP64 values, decreasing), its threshold rank k and the width l_min
    the labelling run needed for its posterior estimate (rsvd_size_label);
    p = q = -1 when no grid point qualifies."""
    torch = _torch()
    S = S.contiguous()
    out = torch.empty(3, dtype=torch.int64, device=S.device)
    _check(lib().rsvd_size_label(_ptr(S), S.numel(), int(k), int(n), int(l_min), _ptr(out),
                                 _stream(torch, S.device)), "rsvd_size_label")
    return tuple(int(x) for x in out.cpu().tolist())


class Mlp:
    """The 16-64-64-3 predictor: flat FP32 parameters, Adam moments and the
    target statistics (mean[3], sd[3]) on the device; every computation runs
    in the library's kernels."""

    def __init__(self, seed=0, device="cuda"):
        torch = _torch()
        self.device = torch.device(device)
        self.stats = torch.zeros(6, dtype=torch.float32, device=self.device)
        self.stats[3:] = 1.0
        self.params = torch.empty(MLP_PARAMS, dtype=torch.float32, device=self.device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self._loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        _check(lib().rsvd_mlp_init(_ptr(self.params), seed & (2**64 - 1),
                                   _stream(torch, self.device)), "rsvd_mlp_init")

    @staticmethod
    def _f32(torch, X, cols, name):
        if not (X.is_cuda and X.dtype == torch.float32 and X.dim() == 2 and X.shape[1] == cols
                and X.is_contiguous()):
            raise RsvdError(f"{name} must be a contiguous float32 CUDA tensor with {cols} columns")

    def forward(self, X):
        torch = _torch()
        self._f32(torch, X, MLP_IN, "X")
        Y = torch.empty(X.shape[0], MLP_OUT, dtype=torch.float32, device=X.device)
        _check(lib().rsvd_mlp_forward(_ptr(self.params), _ptr(X), X.shape[0], _ptr(Y),
                                      _stream(torch, X.device)), "rsvd_mlp_forward")
        return Y

    def grad(self, X, T):
        """(loss, gradient) of one batch (B <= 128) without updating."""
        torch = _torch()
        self._f32(torch, X, MLP_IN, "X")
        self._f32(torch, T, MLP_OUT, "T")
        g = torch.empty_like(self.params)
        _check(lib().rsvd_mlp_grad(_ptr(self.params), _ptr(X), _ptr(T), X.shape[0], _ptr(g),
                                   _ptr(self._loss), _stream(torch, X.device)), "rsvd_mlp_grad")
        return float(self._loss.item()), g

    def targets(self, labels):
        """Standardized training targets (device B x 3 FP32) from integer
        (k, p, q) labels (B x 3); sets the target statistics (rsvd_mlp_targets)."""
        torch = _torch()
        lab = torch.as_tensor(labels, dtype=torch.int64).reshape(-1, 3).to(self.device).contiguous()
        T = torch.empty(lab.shape[0], MLP_OUT, dtype=torch.float32, device=self.device)
        _check(lib().rsvd_mlp_targets(_ptr(lab), lab.shape[0], _ptr(self.stats), _ptr(T),
                                      _stream(torch, self.device)), "rsvd_mlp_targets")
        return T

    def predict(self, X, n_cap):
        """Sizing (k, p, q) per sample (rsvd_mlp_predict): X device B x 16
        features, n_cap the min(m, n) of each channel. Returns a host list of
        (k, p, q) tuples (one synchronization)."""
        torch = _torch()
        self._f32(torch, X, MLP_IN, "X")
        nc = torch.as_tensor(list(n_cap), dtype=torch.int64).to(X.device).contiguous()
        if nc.numel() != X.shape[0]:
            raise RsvdError("one n_cap per sample")
        kpq = torch.empty(X.shape[0], 3, dtype=torch.int64, device=X.device)
        _check(lib().rsvd_mlp_predict(_ptr(self.params), _ptr(self.stats), _ptr(X), X.shape[0],
                                      _ptr(nc), _ptr(kpq), _stream(torch, X.device)),
               "rsvd_mlp_predict")
        return [tuple(int(v) for v in row) for row in kpq.cpu().tolist()]

    def save(self, path):
        torch = _torch()
        _check(lib().rsvd_mlp_save(os.fsencode(path), _ptr(self.params), _ptr(self.stats),
                                   _stream(torch, self.device)), "rsvd_mlp_save")

    def load(self, path):
        torch = _torch()
        _check(lib().rsvd_mlp_load(os.fsencode(path), _ptr(self.params), _ptr(self.stats),
                                   _stream(torch, self.device)), "rsvd_mlp_load")

    def train_step(self, X, T, lr=1e-3):
        """One Adam step on a batch (B <= 128); returns a device scalar with the
        batch loss before the step (read it without forcing a sync each step)."""
        torch = _torch()
        self._f32(torch, X, MLP_IN, "X")
        self._f32(torch, T, MLP_OUT, "T")
        self.step += 1
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        _check(lib().rsvd_mlp_train_step(_ptr(self.params), _ptr(self.m), _ptr(self.v), self.step,
                                         _ptr(X), _ptr(T), X.shape[0], float(lr), _ptr(loss),
                                         _stream(torch, X.device)), "rsvd_mlp_train_step")
        return loss


def trace_enable(on=True):
    """Record HIP event pairs around each phase of subsequent runs."""
    lib().rsvd_trace_enable(int(bool(on)))


def trace_collect():
    """Per-phase (total ms, launch groups) since the last collect."""
    n = len(TRACE_PHASES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    _check(lib().rsvd_trace_collect(ms, cnt), "rsvd_trace_collect")
    return {TRACE_PHASES[i]: (ms[i], cnt[i]) for i in range(n)}
