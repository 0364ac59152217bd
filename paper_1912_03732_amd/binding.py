"""Python binding of libsboxwalsh.so (ctypes; argument marshalling only).

Every entry point of ``include/sbox_walsh.h`` has a function of the same
name here that takes plain integers / device pointers, plus a few
torch-tensor conveniences (``walsh_nl``, ``walsh_nl_batched``, ``Plan``)
that allocate outputs with torch and pass torch's current HIP stream.
torch is used for device memory and streams only: all computation runs in
the library's HIP kernels.  There is no CPU fallback: if the library is not
built, or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsboxwalsh.so")

SBOX_OK = 0
SBOX_ERR_INVALID_ARG = 1
SBOX_ERR_UNSUPPORTED = 2
SBOX_ERR_WORKSPACE = 3
SBOX_ERR_HIP = 4

SPECTRUM_NONE = 0
SPECTRUM_B_MAJOR = 1
SPECTRUM_A_MAJOR = 2
SPECTRUM_LAT = 0x10
LAT_B_MAJOR = 0x11
LAT_A_MAJOR = 0x12

_STATUS_NAMES = {0: "SBOX_OK", 1: "SBOX_ERR_INVALID_ARG", 2: "SBOX_ERR_UNSUPPORTED",
                 3: "SBOX_ERR_WORKSPACE", 4: "SBOX_ERR_HIP"}


class SboxError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (_STATUS_NAMES.get(status, str(status)), message))
        self.status = status


class sbox_tuning(ctypes.Structure):
    _fields_ = [("split_p", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("variant", ctypes.c_int32)]


class sbox_job(ctypes.Structure):
    _fields_ = [("S", ctypes.c_void_p), ("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("s_elem_bytes", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("maxabs_per_b", ctypes.c_void_p), ("nl", ctypes.c_void_p),
                ("spectrum", ctypes.c_void_p)]


# Every exported symbol of include/sbox_walsh.h.
EXPORTS = ("sbox_walsh_nl", "sbox_scratch_reserve", "sbox_scratch_release", "sbox_walsh_nl_ex",
           "sbox_walsh_nl_workspace_bytes", "sbox_walsh_nl_static", "sbox_walsh_nl_static_max_bytes",
           "sbox_walsh_nl_batched", "sbox_batched_workspace_bytes", "sbox_plan_create",
           "sbox_plan_launch", "sbox_plan_destroy", "sbox_criteria", "sbox_criteria_ex",
           "sbox_criteria_workspace_bytes", "sbox_walsh_histogram",
           "sbox_walsh_histogram_workspace_bytes", "sbox_avalanche", "sbox_avalanche_workspace_bytes",
           "sbox_last_error", "sbox_version")

_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libsboxwalsh.so is not built (%s); run __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    lib.sbox_walsh_nl.argtypes = [vp, i32, i32, vp, vp, vp]
    lib.sbox_scratch_reserve.argtypes = [i32, i32, vp]
    lib.sbox_scratch_release.argtypes = [vp]
    lib.sbox_walsh_nl_ex.argtypes = [vp, i32, i32, i32, vp, vp, vp, i32, vp, sz,
                                     ctypes.POINTER(sbox_tuning), vp]
    lib.sbox_walsh_nl_static.argtypes = [vp, i32, i32, i32, vp, vp, vp, i32, vp]
    lib.sbox_walsh_nl_static.restype = ctypes.c_int
    lib.sbox_walsh_nl_static_max_bytes.argtypes = []
    lib.sbox_walsh_nl_static_max_bytes.restype = sz
    lib.sbox_walsh_nl_workspace_bytes.argtypes = [i32, i32, i32]
    lib.sbox_walsh_nl_workspace_bytes.restype = sz
    lib.sbox_walsh_nl_batched.argtypes = [ctypes.POINTER(sbox_job), ctypes.c_int32, vp, sz, vp]
    lib.sbox_batched_workspace_bytes.argtypes = [ctypes.POINTER(sbox_job), ctypes.c_int32]
    lib.sbox_batched_workspace_bytes.restype = sz
    lib.sbox_plan_create.argtypes = [ctypes.POINTER(sbox_job), ctypes.c_int32,
                                     ctypes.POINTER(sbox_tuning), ctypes.POINTER(vp)]
    lib.sbox_plan_launch.argtypes = [vp, vp]
    lib.sbox_plan_destroy.argtypes = [vp]
    lib.sbox_plan_destroy.restype = None
    lib.sbox_criteria.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, vp, vp]
    lib.sbox_criteria.restype = ctypes.c_int
    lib.sbox_criteria_ex.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.sbox_criteria_ex.restype = ctypes.c_int
    lib.sbox_criteria_workspace_bytes.argtypes = [i32, i32]
    lib.sbox_criteria_workspace_bytes.restype = sz
    lib.sbox_walsh_histogram.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, sz, vp]
    lib.sbox_walsh_histogram.restype = ctypes.c_int
    lib.sbox_walsh_histogram_workspace_bytes.argtypes = [i32, i32]
    lib.sbox_walsh_histogram_workspace_bytes.restype = sz
    lib.sbox_avalanche.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, sz, vp]
    lib.sbox_avalanche.restype = ctypes.c_int
    lib.sbox_avalanche_workspace_bytes.argtypes = [i32, i32]
    lib.sbox_avalanche_workspace_bytes.restype = sz
    lib.sbox_last_error.restype = ctypes.c_char_p
    lib.sbox_version.restype = ctypes.c_char_p
    for f in ("sbox_walsh_nl", "sbox_scratch_reserve", "sbox_scratch_release", "sbox_walsh_nl_ex",
              "sbox_walsh_nl_batched", "sbox_plan_create", "sbox_plan_launch"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def last_error() -> str:
    return load().sbox_last_error().decode()


def _check(status: int):
    if status != SBOX_OK:
        raise SboxError(status, last_error())


# ------------------------------------------------------ raw C-ABI calls ---

def sbox_walsh_nl(S: int, n: int, m: int, maxabs_per_b: int, nl: int, stream: int) -> int:
    return load().sbox_walsh_nl(S, n, m, maxabs_per_b, nl, stream)


def sbox_scratch_reserve(n: int, m: int, stream: int) -> int:
    return load().sbox_scratch_reserve(n, m, stream)


def sbox_scratch_release(stream: int) -> int:
    return load().sbox_scratch_release(stream)


def sbox_walsh_nl_ex(S: int, n: int, m: int, s_elem_bytes: int, maxabs_per_b: int, nl: int,
                     spectrum: int, layout: int, workspace: int, workspace_bytes: int,
                     tuning: Optional[sbox_tuning], stream: int) -> int:
    tp = ctypes.byref(tuning) if tuning is not None else None
    return load().sbox_walsh_nl_ex(S, n, m, s_elem_bytes, maxabs_per_b, nl, spectrum, layout,
                                   workspace, workspace_bytes, tp, stream)


def sbox_walsh_nl_static(S: int, n: int, m: int, s_elem_bytes: int, maxabs_per_b: int, nl: int,
                         spectrum: int, layout: int, stream: int) -> int:
    return load().sbox_walsh_nl_static(S, n, m, s_elem_bytes, maxabs_per_b, nl, spectrum, layout, stream)


def sbox_walsh_nl_static_max_bytes() -> int:
    return int(load().sbox_walsh_nl_static_max_bytes())


def sbox_walsh_nl_workspace_bytes(n: int, m: int, layout: int) -> int:
    return int(load().sbox_walsh_nl_workspace_bytes(n, m, layout))


def sbox_walsh_nl_batched(jobs, count: int, workspace: int, workspace_bytes: int, stream: int) -> int:
    return load().sbox_walsh_nl_batched(jobs, count, workspace, workspace_bytes, stream)


def sbox_batched_workspace_bytes(jobs, count: int) -> int:
    return int(load().sbox_batched_workspace_bytes(jobs, count))


def sbox_plan_create(jobs, count: int, tuning: Optional[sbox_tuning]):
    out = ctypes.c_void_p()
    tp = ctypes.byref(tuning) if tuning is not None else None
    st = load().sbox_plan_create(jobs, count, tp, ctypes.byref(out))
    return st, out.value


def sbox_plan_launch(plan: int, stream: int) -> int:
    return load().sbox_plan_launch(plan, stream)


def sbox_plan_destroy(plan: int) -> None:
    load().sbox_plan_destroy(plan)


def sbox_criteria(S: int, n: int, m: int, s_elem_bytes: int, summary: int, w0_per_b: int,
                  minwt_per_b: int, acmax_per_b: int, pcwt_per_b: int, stream: int) -> int:
    return load().sbox_criteria(S, n, m, s_elem_bytes, summary, w0_per_b, minwt_per_b, acmax_per_b,
                                pcwt_per_b, stream)


def sbox_criteria_ex(S: int, n: int, m: int, s_elem_bytes: int, summary: int, w0_per_b: int,
                     minwt_per_b: int, acmax_per_b: int, pcwt_per_b: int, workspace: int, workspace_bytes: int,
                     stream: int) -> int:
    return load().sbox_criteria_ex(S, n, m, s_elem_bytes, summary, w0_per_b, minwt_per_b, acmax_per_b,
                                   pcwt_per_b, workspace, workspace_bytes, stream)


def sbox_criteria_workspace_bytes(n: int, m: int) -> int:
    return int(load().sbox_criteria_workspace_bytes(n, m))


def sbox_walsh_histogram(S: int, n: int, m: int, s_elem_bytes: int, hist: int, maxabs_per_b: int, nl: int,
                         workspace: int, workspace_bytes: int, stream: int) -> int:
    return load().sbox_walsh_histogram(S, n, m, s_elem_bytes, hist, maxabs_per_b, nl, workspace,
                                       workspace_bytes, stream)


def sbox_walsh_histogram_workspace_bytes(n: int, m: int) -> int:
    return int(load().sbox_walsh_histogram_workspace_bytes(n, m))


def sbox_avalanche(S: int, n: int, m: int, s_elem_bytes: int, r: int, summary: int, maxabs_per_b: int,
                   workspace: int, workspace_bytes: int, stream: int) -> int:
    return load().sbox_avalanche(S, n, m, s_elem_bytes, r, summary, maxabs_per_b, workspace,
                                 workspace_bytes, stream)


def sbox_avalanche_workspace_bytes(n: int, m: int) -> int:
    return int(load().sbox_avalanche_workspace_bytes(n, m))


def sbox_last_error() -> str:
    return last_error()


def sbox_version() -> str:
    return load().sbox_version().decode()


# ------------------------------------------------- torch conveniences ---

def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device available: the S-box library runs on the GPU only")
    return torch


def _elem_bytes(t) -> int:
    return t.element_size()


def _stream(torch, stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def table_to_device(S, m: int, device="cuda"):
    """Copy a table (numpy or tensor) to the device in the narrowest unsigned width for m."""
    torch = _torch()
    import numpy as np
    dt = {1: torch.uint8, 2: torch.uint16, 4: torch.uint32}[1 if m <= 8 else (2 if m <= 16 else 4)]
    if isinstance(S, torch.Tensor):
        return S.to(device=device, dtype=dt).contiguous()
    npdt = {torch.uint8: np.uint8, torch.uint16: np.uint16, torch.uint32: np.uint32}[dt]
    return torch.from_numpy(np.ascontiguousarray(np.asarray(S).astype(npdt))).to(device)


class Workspace:
    """A 256-byte aligned device scratch buffer (torch-allocated)."""

    def __init__(self, nbytes: int, device="cuda"):
        torch = _torch()
        self.nbytes = int(nbytes)
        self.buf = torch.empty(max(self.nbytes, 1) + 256, dtype=torch.uint8, device=device)
        base = self.buf.data_ptr()
        self.ptr = (base + 255) & ~255

    def ensure(self, nbytes: int):
        if nbytes > self.nbytes:
            self.__init__(nbytes, self.buf.device)
        return self


def walsh_nl(S, n: int, m: int, *, spectrum: Optional[str] = None, maxabs: bool = True,
             tuning: Optional[sbox_tuning] = None, workspace: Optional[Workspace] = None,
             stream=None, sync: bool = True):
    """NL (and per-mask max |W|, and optionally the spectrum) of one S-box.

    ``S`` is a device tensor of 2^n unsigned entries (uint8/16/32).  Returns
    (nl, maxabs_per_b tensor or None, spectrum tensor or None); ``nl`` is a
    Python int when ``sync`` is true, else the 1-element device tensor.
    """
    torch = _torch()
    if not isinstance(S, torch.Tensor) or not S.is_cuda:
        raise TypeError("S must be a device tensor")
    S = S.contiguous()
    layout = {None: SPECTRUM_NONE, "b": SPECTRUM_B_MAJOR, "a": SPECTRUM_A_MAJOR,
              "lat-b": LAT_B_MAJOR, "lat-a": LAT_A_MAJOR}[spectrum]
    dev = S.device
    nl_t = torch.empty(1, dtype=torch.int32, device=dev)
    mx = torch.empty(1 << m, dtype=torch.int32, device=dev) if maxabs else None
    spec = None
    if layout != SPECTRUM_NONE:
        shape = (1 << m, 1 << n) if (layout & 3) == SPECTRUM_B_MAJOR else (1 << n, 1 << m)
        spec = torch.empty(shape, dtype=torch.int32, device=dev)
    if tuning is None and layout == SPECTRUM_NONE:
        from . import autotune
        tuning = autotune.lookup(n, m)
    need = sbox_walsh_nl_workspace_bytes(n, m, layout)
    if need == 0:
        raise SboxError(SBOX_ERR_UNSUPPORTED, "unsupported n=%d m=%d layout=%d" % (n, m, layout))
    ws = (workspace or Workspace(need, dev)).ensure(need)
    st = sbox_walsh_nl_ex(S.data_ptr(), n, m, _elem_bytes(S), mx.data_ptr() if mx is not None else 0,
                          nl_t.data_ptr(), spec.data_ptr() if spec is not None else 0, layout,
                          ws.ptr, ws.nbytes, tuning, _stream(torch, stream))
    _check(st)
    if sync:
        torch.cuda.current_stream(dev).synchronize() if stream is None else stream.synchronize()
        return int(nl_t.item()), mx, spec
    return nl_t, mx, spec


def make_jobs(tables, ns, ms, outs_nl, outs_maxabs, layouts=None, specs=None):
    """Build a ctypes sbox_job array from device tensors."""
    count = len(tables)
    arr = (sbox_job * max(count, 1))()
    for i in range(count):
        S = tables[i]
        arr[i].S = S.data_ptr()
        arr[i].n = ns[i]
        arr[i].m = ms[i]
        arr[i].s_elem_bytes = S.element_size()
        arr[i].layout = layouts[i] if layouts is not None else SPECTRUM_NONE
        arr[i].maxabs_per_b = outs_maxabs[i].data_ptr() if outs_maxabs[i] is not None else None
        arr[i].nl = outs_nl[i].data_ptr()
        arr[i].spectrum = specs[i].data_ptr() if (specs is not None and specs[i] is not None) else None
    return arr


def walsh_nl_batched(tables: Sequence, ns: Sequence[int], ms: Sequence[int], *, maxabs: bool = True,
                     stream=None, sync: bool = True, workspace: Optional[Workspace] = None):
    """Many S-boxes in one batched pass.  Returns (nl tensor [count], list of maxabs tensors)."""
    torch = _torch()
    count = len(tables)
    dev = tables[0].device if count else torch.device("cuda")
    nl_all = torch.empty(max(count, 1), dtype=torch.int32, device=dev)
    outs_nl = [nl_all[i:i + 1] for i in range(count)]
    outs_mx = [torch.empty(1 << ms[i], dtype=torch.int32, device=dev) if maxabs else None
               for i in range(count)]
    jobs = make_jobs(tables, ns, ms, outs_nl, outs_mx)
    need = sbox_batched_workspace_bytes(jobs, count)
    if count and need == 0:
        raise SboxError(SBOX_ERR_UNSUPPORTED, last_error() or "unsupported batch")
    ws = (workspace or Workspace(need, dev)).ensure(need)
    _check(sbox_walsh_nl_batched(jobs, count, ws.ptr, ws.nbytes, _stream(torch, stream)))
    if sync:
        torch.cuda.synchronize(dev)
    return nl_all[:count], outs_mx


class Plan:
    """A batched launch prepared once (descriptors resident on the device) and
    launched many times, e.g. inside a captured HIP graph."""

    def __init__(self, tables, ns, ms, *, maxabs: bool = True, tuning: Optional[sbox_tuning] = None):
        torch = _torch()
        self.count = len(tables)
        dev = tables[0].device
        self.tables = list(tables)
        self.nl = torch.empty(max(self.count, 1), dtype=torch.int32, device=dev)
        self.maxabs = [torch.empty(1 << ms[i], dtype=torch.int32, device=dev) if maxabs else None
                       for i in range(self.count)]
        jobs = make_jobs(self.tables, ns, ms, [self.nl[i:i + 1] for i in range(self.count)], self.maxabs)
        st, handle = sbox_plan_create(jobs, self.count, tuning)
        _check(st)
        self.handle = handle

    def launch(self, stream=None):
        torch = _torch()
        _check(sbox_plan_launch(self.handle, _stream(torch, stream)))

    def close(self):
        if self.handle:
            sbox_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


CRITERIA_FIELDS = ("nl", "unbalanced", "ci_order", "resiliency", "abs_indicator", "pc_order")


def criteria(S, n: int, m: int, *, per_mask: bool = True, workspace: bool = True, stream=None):
    """Balancedness, correlation immunity / resiliency and autocorrelation
    criteria of every nonzero component (n <= 16).  Returns (summary dict,
    dict of per-mask tensors w0, minwt, acmax, pcwt or None).  With
    workspace=False (n <= 14 only) the library runs its LDS kernel instead of
    the register-blocked one that a workspace selects."""
    torch = _torch()
    if not isinstance(S, torch.Tensor) or not S.is_cuda:
        raise TypeError("S must be a device tensor")
    S = S.contiguous()
    dev = S.device
    summ = torch.empty(8, dtype=torch.int32, device=dev)
    arrs = {k: torch.empty(1 << m, dtype=torch.int32, device=dev) for k in ("w0", "minwt", "acmax", "pcwt")} \
        if per_mask else None
    ptr = (lambda k: arrs[k].data_ptr()) if arrs else (lambda k: 0)
    ws = Workspace(sbox_criteria_workspace_bytes(n, m), dev) if (workspace or n >= 15) else None
    _check(sbox_criteria_ex(S.data_ptr(), n, m, S.element_size(), summ.data_ptr(), ptr("w0"), ptr("minwt"),
                            ptr("acmax"), ptr("pcwt"), ws.ptr if ws else 0, ws.nbytes if ws else 0,
                            _stream(torch, stream)))
    torch.cuda.synchronize(dev)
    v = summ.cpu().tolist()
    return {k: int(v[i]) for i, k in enumerate(CRITERIA_FIELDS)}, arrs


def walsh_histogram(S, n: int, m: int, *, maxabs: bool = False, stream=None):
    """|W| histogram over the nonzero masks: hist[k] = #{(a, b): b != 0,
    |W(a, b)| = 2k} as an int64 device tensor of 2^(n-1) + 1 counts, with
    (nl, maxabs tensor or None) from the same pass."""
    torch = _torch()
    if not isinstance(S, torch.Tensor) or not S.is_cuda:
        raise TypeError("S must be a device tensor")
    S = S.contiguous()
    dev = S.device
    hist = torch.empty((1 << (n - 1)) + 1, dtype=torch.int64, device=dev)
    nl = torch.empty(1, dtype=torch.int32, device=dev)
    mx = torch.empty(1 << m, dtype=torch.int32, device=dev) if maxabs else None
    ws = Workspace(sbox_walsh_histogram_workspace_bytes(n, m), dev)
    _check(sbox_walsh_histogram(S.data_ptr(), n, m, S.element_size(), hist.data_ptr(),
                                mx.data_ptr() if mx is not None else 0, nl.data_ptr(), ws.ptr, ws.nbytes,
                                _stream(torch, stream)))
    torch.cuda.synchronize(dev)
    return hist, int(nl.item()), mx


AVALANCHE_FIELDS = ("sac_max", "bic_sac_max", "bic_nl")


def avalanche(S, n: int, m: int, *, maxabs=None, stream=None):
    """Unit-difference autocorrelations r (an (n, 2^m) int32 device tensor)
    and the strict-avalanche / bit-independence summary; pass the maxabs
    tensor of walsh_nl on the same box to get the bit-independence NL."""
    torch = _torch()
    if not isinstance(S, torch.Tensor) or not S.is_cuda:
        raise TypeError("S must be a device tensor")
    S = S.contiguous()
    dev = S.device
    r = torch.empty((n, 1 << m), dtype=torch.int32, device=dev)
    summ = torch.empty(3, dtype=torch.int32, device=dev)
    _check(sbox_avalanche(S.data_ptr(), n, m, S.element_size(), r.data_ptr(), summ.data_ptr(),
                          maxabs.data_ptr() if maxabs is not None else 0, 0, 0, _stream(torch, stream)))
    torch.cuda.synchronize(dev)
    v = summ.cpu().tolist()
    return {k: int(v[i]) for i, k in enumerate(AVALANCHE_FIELDS)}, r
