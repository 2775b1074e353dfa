"""Python binding of libips.so: in-place samplesort (IPS4o) and radix sort
(IPS2Ra) of device arrays on an MI355X.

Argument marshalling only: every step of the sort runs in the HIP library;
PyTorch supplies device memory and the stream.  Importing fails loudly if
the library has not been built (``python -m paper_2009_13569_amd.build``).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# IPS_LIBRARY selects another build of the same sources (a counter build of
# `python -m paper_2009_13569_amd.build --define ... --out ...`).
LIB_PATH = os.environ.get("IPS_LIBRARY") or os.path.join(HERE, "libips.so")

# PyTorch's HIP runtime is loaded first so that libips.so binds to the same
# runtime (its dependency is recorded as plain libamdhip64.so).
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing; build it with `python -m paper_2009_13569_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

IPS_OK = 0
STATUS = {0: "IPS_OK", -1: "IPS_E_INVALID_ARG", -2: "IPS_E_UNSUPPORTED", -3: "IPS_E_WORKSPACE",
          -4: "IPS_E_MISALIGNED", -5: "IPS_E_TOO_LARGE", -6: "IPS_E_HIP", -7: "IPS_E_DEVICE",
          -8: "IPS_E_NO_DEVICE", -9: "IPS_E_SCRATCH"}
TYPES = {"u32": 1, "u64": 2, "f64": 3, "pair": 4, "rec100": 5, "quartet": 6}
ELEM_BYTES = {"u32": 4, "u64": 8, "f64": 8, "pair": 16, "rec100": 100, "quartet": 32}
# Largest task the LDS tier sorts by default (elements), per element kind.
LDS_CAP = {"u32": 16384, "u64": 16384, "f64": 16384, "pair": 8192, "rec100": 1024, "quartet": 2048}
ALGOS = {"samplesort": 0, "radix": 1}
FLAG_NO_SORTED_CHECK = 0x1
FLAG_EQ_ON = 0x2
FLAG_EQ_OFF = 0x4
FLAG_LEVEL1_ONLY = 0x8
FLAG_GLOBAL_BUFFERS = 0x10
FLAG_PROFILE = 0x20
FLAG_GRAPH = 0x40
FLAG_HOST_PLAN = 0x80
FLAG_FUSED = 0x100
FLAG_INSERTION_BASE = 0x200
FLAG_PAPER_ROOT_ALPHA = 0x400
MAX_LEVELS = 16
PHASES = ["sorted_check", "minmax", "sample", "classify", "boundaries", "flags", "permute",
          "cleanup_a", "cleanup_b", "lds_sort", "reverse", "histogram", "fused"]

EXPORTS = ["ips_ctx_create", "ips_ctx_destroy", "ips_workspace_bytes", "ips_sort_keys",
           "ips_sort_pairs", "ips_segments_workspace_bytes", "ips_sort_segments",
           "ips_batch_workspace_bytes", "ips_sort_batch", "ips_serve_workspace_bytes", "ips_serve_trace",
           "ips_get_root_info", "ips_get_stats", "ips_get_profile", "ips_last_hip_error",
           "ips_last_device_error", "ips_status_string", "ips_abi_version", "ips_tuned_params",
           "ips_sort_keys_noalloc", "ips_oop_workspace_bytes", "ips_sort_oop", "ips_probe_memory"]
SERVE_BATCH = 0
SERVE_FIFO = 1


class Params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("block_bytes", ctypes.c_uint32), ("n0", ctypes.c_uint32),
                ("lds_task_max", ctypes.c_uint32), ("piece_blocks", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("seed", ctypes.c_uint64),
                ("perm_groups", ctypes.c_uint32), ("profile_mask", ctypes.c_uint32),
                ("perm_wg", ctypes.c_uint32), ("k_root", ctypes.c_uint32)]


class RootInfo(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint32) for f in
                ("valid", "algo", "alpha", "k_prime", "m", "u", "K", "eq", "nb", "radix_shift",
                 "radix_width", "block_elems", "stripes", "pad")] + [
        ("n", ctypes.c_uint64), ("splitters", (ctypes.c_uint8 * 16) * 256),
        ("bucket_start", ctypes.c_uint64 * 513)]


class Stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_uint32), ("steps", ctypes.c_uint32), ("batches", ctypes.c_uint32),
                ("lds_tasks", ctypes.c_uint32), ("detected", ctypes.c_uint32), ("pad0", ctypes.c_uint32),
                ("partitioned_elems", ctypes.c_uint64), ("lds_elems", ctypes.c_uint64),
                ("max_step_elems", ctypes.c_uint64)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("elem_type", ctypes.c_int32), ("algo", ctypes.c_int32), ("log2n_min", ctypes.c_uint32),
                ("log2n_max", ctypes.c_uint32), ("batched", ctypes.c_uint32), ("k", ctypes.c_uint32),
                ("block_bytes", ctypes.c_uint32), ("n0", ctypes.c_uint32), ("lds_task_max", ctypes.c_uint32),
                ("piece_blocks", ctypes.c_uint32), ("perm_groups", ctypes.c_uint32), ("perm_wg", ctypes.c_uint32),
                ("k_root", ctypes.c_uint32)]


TUNE_FIELDS = ("k", "block_bytes", "n0", "lds_task_max", "piece_blocks", "perm_groups", "perm_wg", "k_root")
# The table written by `python -m paper_2009_13569_amd.tune` (loaded by Sorter).
TUNING_PATH = os.path.join(HERE, "tuning.json")


class Segment(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_uint64), ("n", ctypes.c_uint64)]


class Request(ctypes.Structure):
    _fields_ = [("d_data", ctypes.c_void_p), ("n", ctypes.c_uint64), ("elem_type", ctypes.c_int32),
                ("algo", ctypes.c_int32), ("arrival_s", ctypes.c_double), ("start_s", ctypes.c_double),
                ("done_s", ctypes.c_double), ("status", ctypes.c_int32), ("batch", ctypes.c_uint32),
                ("detail", ctypes.c_int32), ("pad", ctypes.c_int32)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("policy", ctypes.c_uint32), ("max_batch", ctypes.c_uint32)]


class Profile(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("ms", (ctypes.c_double * len(PHASES)) * (MAX_LEVELS + 1)),
                ("elems", (ctypes.c_uint64 * len(PHASES)) * (MAX_LEVELS + 1)),
                ("launches", (ctypes.c_uint32 * len(PHASES)) * (MAX_LEVELS + 1))]


_vp, _u64, _i32, _sz = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_size_t
_lib.ips_ctx_create.argtypes = [ctypes.POINTER(_vp), _i32]
_lib.ips_ctx_destroy.argtypes = [_vp]
_lib.ips_workspace_bytes.argtypes = [_u64, _i32, _i32, ctypes.POINTER(Params), ctypes.POINTER(_sz)]
_lib.ips_sort_keys.argtypes = [_vp, _vp, _u64, _i32, _i32, _vp, _sz, ctypes.POINTER(Params), _vp]
_lib.ips_sort_pairs.argtypes = [_vp, _vp, _u64, _i32, _i32, _vp, _sz, ctypes.POINTER(Params), _vp]
_lib.ips_sort_keys_noalloc.argtypes = [_vp, _vp, _u64, _i32, _i32, ctypes.POINTER(Params), _vp]
_lib.ips_oop_workspace_bytes.argtypes = [_u64, _i32, ctypes.POINTER(Params), ctypes.POINTER(_sz), ctypes.POINTER(_sz)]
_lib.ips_sort_oop.argtypes = [_vp, _vp, _u64, _i32, _vp, _sz, _vp, _sz, ctypes.POINTER(Params), _vp]
_lib.ips_segments_workspace_bytes.argtypes = [_u64, ctypes.POINTER(Segment), ctypes.c_uint32, _i32, _i32,
                                              ctypes.POINTER(Params), ctypes.POINTER(_sz)]
_lib.ips_sort_segments.argtypes = [_vp, _vp, _u64, _i32, _i32, ctypes.POINTER(Segment), ctypes.c_uint32,
                                   _vp, _sz, ctypes.POINTER(Params), _vp]
_lib.ips_batch_workspace_bytes.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(_u64), ctypes.c_uint32, _i32,
                                           _i32, ctypes.POINTER(Params), ctypes.POINTER(_sz)]
_lib.ips_sort_batch.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_u64), ctypes.c_uint32, _i32, _i32,
                                _vp, _sz, ctypes.POINTER(Params), _vp]
_lib.ips_serve_workspace_bytes.argtypes = [ctypes.POINTER(Request), ctypes.c_uint32, ctypes.POINTER(ServeConfig),
                                           ctypes.POINTER(Params), ctypes.POINTER(_sz)]
_lib.ips_serve_trace.argtypes = [_vp, ctypes.POINTER(Request), ctypes.c_uint32, ctypes.POINTER(ServeConfig),
                                 _vp, _sz, ctypes.POINTER(Params), _vp]
_lib.ips_get_root_info.argtypes = [_vp, ctypes.POINTER(RootInfo)]
_lib.ips_tuned_params.argtypes = [ctypes.POINTER(TuneEntry), ctypes.c_uint32, _u64, _i32, _i32, _i32,
                                  ctypes.POINTER(Params), ctypes.POINTER(Params)]
_lib.ips_get_stats.argtypes = [_vp, ctypes.POINTER(Stats)]
_lib.ips_get_profile.argtypes = [_vp, ctypes.POINTER(Profile)]
_lib.ips_last_hip_error.argtypes = [_vp]
_lib.ips_last_device_error.argtypes = [_vp]
_lib.ips_probe_memory.argtypes = [_i32, _vp, _vp, _u64, ctypes.c_uint32, _vp, ctypes.c_uint32, ctypes.c_uint32,
                                  ctypes.c_uint32, _vp, ctypes.POINTER(ctypes.c_float)]
_lib.ips_status_string.argtypes = [_i32]
_lib.ips_status_string.restype = ctypes.c_char_p
for _f in ("ips_ctx_create", "ips_ctx_destroy", "ips_workspace_bytes", "ips_sort_keys",
           "ips_sort_pairs", "ips_segments_workspace_bytes", "ips_sort_segments", "ips_batch_workspace_bytes",
           "ips_sort_batch", "ips_serve_workspace_bytes", "ips_serve_trace", "ips_get_root_info",
           "ips_get_stats", "ips_get_profile", "ips_last_hip_error", "ips_last_device_error",
           "ips_abi_version", "ips_tuned_params", "ips_sort_keys_noalloc", "ips_oop_workspace_bytes",
           "ips_sort_oop", "ips_probe_memory"):
    getattr(_lib, _f).restype = _i32


class IpsError(RuntimeError):
    def __init__(self, code: int, what: str = "", detail: str = ""):
        self.code = code
        msg = _lib.ips_status_string(code).decode()
        super().__init__(f"{what}: {msg}{(' ' + detail) if detail else ''}")


def lib() -> ctypes.CDLL:
    return _lib


PROBES = {"copy": 0, "read": 1, "write": 2, "blocks": 3, "chain": 4}


def probe_memory(mode: str, src, dst, block_bytes: int = 0, table=None, groups: int = 0, reps: int = 10,
                 stream=None) -> float:
    """ips_probe_memory on device tensors (src, dst of equal byte size; table:
    a device int64 tensor for the chain probe): mean ms per launch."""
    ms = ctypes.c_float(0.0)
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst differ in size")
    rc = _lib.ips_probe_memory(PROBES[mode], src.data_ptr(), dst.data_ptr(), nbytes, block_bytes,
                               table.data_ptr() if table is not None else None,
                               table.numel() if table is not None else 0, groups, reps,
                               stream.cuda_stream if stream is not None else None, ctypes.byref(ms))
    if rc != 0:
        raise IpsError(rc, "ips_probe_memory")
    return ms.value


def make_params(k=0, block_bytes=0, n0=0, lds_task_max=0, piece_blocks=0, flags=0, seed=0,
                perm_groups=0, profile_phases=None, perm_wg=0, k_root=0) -> Params:
    """profile_phases: names from PHASES to time with FLAG_PROFILE (None: all)."""
    p = Params()
    p.k, p.block_bytes, p.n0, p.lds_task_max, p.piece_blocks = k, block_bytes, n0, lds_task_max, piece_blocks
    p.flags, p.seed, p.perm_groups, p.perm_wg, p.k_root = flags, seed, perm_groups, perm_wg, k_root
    p.profile_mask = 0 if profile_phases is None else sum(1 << PHASES.index(x) for x in profile_phases)
    return p


def workspace_bytes(n: int, kind: str, algo: str = "samplesort", params: Params | None = None) -> int:
    out = ctypes.c_size_t(0)
    rc = _lib.ips_workspace_bytes(n, TYPES[kind], ALGOS[algo],
                                  ctypes.byref(params) if params is not None else None, ctypes.byref(out))
    if rc != IPS_OK:
        raise IpsError(rc, "ips_workspace_bytes")
    return int(out.value)


def segment_array(offsets, sizes):
    """ctypes array of ips_segment from two equal-length integer sequences."""
    offsets, sizes = list(offsets), list(sizes)
    if len(offsets) != len(sizes):
        raise ValueError("offsets and sizes differ in length")
    arr = (Segment * max(1, len(offsets)))()
    for i, (o, n) in enumerate(zip(offsets, sizes)):
        arr[i].offset, arr[i].n = int(o), int(n)
    return arr, len(offsets)


def segments_workspace_bytes(n_total: int, segs, nseg: int, kind: str, algo: str = "samplesort",
                             params: Params | None = None) -> int:
    out = ctypes.c_size_t(0)
    rc = _lib.ips_segments_workspace_bytes(n_total, segs, nseg, TYPES[kind], ALGOS[algo],
                                           ctypes.byref(params) if params is not None else None,
                                           ctypes.byref(out))
    if rc != IPS_OK:
        raise IpsError(rc, "ips_segments_workspace_bytes")
    return int(out.value)


def tune_table(entries):
    """ctypes array of ips_tune_entry from a list of dicts (keys: kind, algo,
    log2n_min, log2n_max, batched and any of TUNE_FIELDS)."""
    arr = (TuneEntry * max(1, len(entries)))()
    for i, e in enumerate(entries):
        t = arr[i]
        t.elem_type, t.algo = TYPES[e["kind"]], ALGOS[e.get("algo", "samplesort")]
        t.log2n_min, t.log2n_max, t.batched = int(e["log2n_min"]), int(e["log2n_max"]), int(e.get("batched", 0))
        for f in TUNE_FIELDS:
            setattr(t, f, int(e.get(f, 0)))
    return arr, len(entries)


def load_tuning(path: str = TUNING_PATH):
    """Entries of a tuning file, or [] when there is none."""
    import json
    if not os.path.exists(path):
        return []
    with open(path) as f:
        return json.load(f)["entries"]


def tuned_params(table, count: int, n: int, kind: str, algo: str = "samplesort", batched: bool = False,
                 base: Params | None = None) -> Params:
    """ips_tuned_params: `base` with its zero tunable fields filled from the
    first matching entry of the table."""
    out = Params()
    rc = _lib.ips_tuned_params(table, count, n, TYPES[kind], ALGOS[algo], int(bool(batched)),
                               ctypes.byref(base) if base is not None else None, ctypes.byref(out))
    if rc < 0:
        raise IpsError(rc, "ips_tuned_params")
    return out


def kind_of(t) -> str:
    """Element kind of a torch tensor: 1-D uint32/uint64/float64 keys, (n, 2)
    64-bit pairs, (n, 4) 64-bit Quartets, or (n, 100) uint8 records."""
    import torch
    if t.dim() == 1:
        return {torch.uint32: "u32", torch.int32: "u32", torch.uint64: "u64", torch.int64: "u64",
                torch.float64: "f64"}[t.dtype]
    if t.dim() == 2 and t.shape[1] == 2 and t.dtype in (torch.uint64, torch.int64):
        return "pair"
    if t.dim() == 2 and t.shape[1] == 4 and t.dtype in (torch.uint64, torch.int64):
        return "quartet"
    if t.dim() == 2 and t.shape[1] == 100 and t.dtype == torch.uint8:
        return "rec100"
    raise TypeError(f"unsupported tensor {tuple(t.shape)} {t.dtype}")


class Sorter:
    """A context on one device, a cached workspace tensor and a tuning table.

    tuning: "default" loads TUNING_PATH when it exists; None uses no table;
    a list of entry dicts uses those.  Every call fills the zero tunable
    fields of its parameters from the table (ips_tuned_params) and sizes the
    workspace for the same parameters."""

    def __init__(self, device: int = 0, tuning="default"):
        h = ctypes.c_void_p()
        rc = _lib.ips_ctx_create(ctypes.byref(h), device)
        if rc != IPS_OK:
            raise IpsError(rc, "ips_ctx_create")
        self._h = h
        self.device = device
        self._ws = None
        self.tuning = load_tuning() if tuning == "default" else list(tuning or [])
        self._table, self._tcount = tune_table(self.tuning)

    def params_for(self, n: int, kind: str, algo: str = "samplesort", batched: bool = False,
                   params: Params | None = None) -> Params:
        """The parameters a call on n elements in total uses."""
        return tuned_params(self._table, self._tcount, max(int(n), 1), kind, algo, batched, params)

    def _check_ws(self, ws, need: int):
        if ws.numel() < need:
            raise ValueError(f"workspace of {ws.numel()} bytes is smaller than the {need} bytes this call needs "
                             f"(size it with the parameters from Sorter.params_for)")

    def close(self):
        if self._h:
            _lib.ips_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, nbytes: int):
        import torch
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws

    def sort_(self, t, algo: str = "samplesort", params: Params | None = None, kind: str | None = None,
              stream=None, ws=None):
        """Sort tensor `t` in place on its device; returns t."""
        import torch
        if not t.is_cuda:
            raise ValueError("tensor must be on the GPU")
        if not t.is_contiguous():
            raise ValueError("tensor must be contiguous")
        kind = kind or kind_of(t)
        n = t.shape[0]
        params = self.params_for(n, kind, algo, False, params)
        need = workspace_bytes(n, kind, algo, params)
        ws = ws if ws is not None else self.workspace(need)
        self._check_ws(ws, need)
        if stream is None:
            stream = torch.cuda.current_stream(t.device)
        sp = ctypes.c_void_p(stream.cuda_stream)
        pp = ctypes.byref(params)
        fn = _lib.ips_sort_keys if kind in ("u32", "u64", "f64") else _lib.ips_sort_pairs
        rc = fn(self._h, ctypes.c_void_p(t.data_ptr()), n, TYPES[kind], ALGOS[algo],
                ctypes.c_void_p(ws.data_ptr()), ws.numel(), pp, sp)
        if rc != IPS_OK:
            raise IpsError(rc, "ips_sort", f"(hip={_lib.ips_last_hip_error(self._h)}, "
                                           f"device={hex(_lib.ips_last_device_error(self._h))})")
        return t

    def sort_noalloc_(self, t, algo: str = "samplesort", params: Params | None = None, kind: str | None = None,
                      stream=None):
        """Sort keys (u32/u64/f64) in place with ips_sort_keys_noalloc: the
        library's static per-GPU scratch instead of a workspace tensor."""
        import torch
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("tensor must be a contiguous GPU tensor")
        kind = kind or kind_of(t)
        if kind not in ("u32", "u64", "f64"):
            raise ValueError("the allocation-free entry point sorts keys only")
        n = t.shape[0]
        params = self.params_for(n, kind, algo, False, params)
        if stream is None:
            stream = torch.cuda.current_stream(t.device)
        rc = _lib.ips_sort_keys_noalloc(self._h, ctypes.c_void_p(t.data_ptr()), n, TYPES[kind], ALGOS[algo],
                                        ctypes.byref(params), ctypes.c_void_p(stream.cuda_stream))
        if rc != IPS_OK:
            raise IpsError(rc, "ips_sort_keys_noalloc", f"(hip={_lib.ips_last_hip_error(self._h)}, "
                                                        f"device={hex(_lib.ips_last_device_error(self._h))})")
        return t

    def sort_oop_(self, t, params: Params | None = None, kind: str | None = None, stream=None, tmp=None):
        """Sort tensor `t` with the out-of-place partitioning step (the
        ablation ips_sort_oop); the result ends in `t`.  `tmp`: a uint8 device
        tensor of at least the second-array bytes (allocated when None)."""
        import torch
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("tensor must be a contiguous GPU tensor")
        kind = kind or kind_of(t)
        n = t.shape[0]
        if params is None:
            params = Params()
        wsb, tmpb = ctypes.c_size_t(0), ctypes.c_size_t(0)
        rc = _lib.ips_oop_workspace_bytes(n, TYPES[kind], ctypes.byref(params), ctypes.byref(wsb), ctypes.byref(tmpb))
        if rc != IPS_OK:
            raise IpsError(rc, "ips_oop_workspace_bytes")
        ws = self.workspace(wsb.value)
        if tmp is None or tmp.numel() < tmpb.value:
            tmp = torch.empty(max(tmpb.value, 256), dtype=torch.uint8, device=t.device)
        if stream is None:
            stream = torch.cuda.current_stream(t.device)
        rc = _lib.ips_sort_oop(self._h, ctypes.c_void_p(t.data_ptr()), n, TYPES[kind], ctypes.c_void_p(tmp.data_ptr()),
                               tmp.numel(), ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.byref(params),
                               ctypes.c_void_p(stream.cuda_stream))
        if rc != IPS_OK:
            raise IpsError(rc, "ips_sort_oop", f"(hip={_lib.ips_last_hip_error(self._h)}, "
                                               f"device={hex(_lib.ips_last_device_error(self._h))})")
        return t

    def sort_segments_(self, t, offsets, sizes, algo: str = "samplesort", params: Params | None = None,
                       kind: str | None = None, stream=None, ws=None):
        """Sort every segment [offsets[i], offsets[i] + sizes[i]) of tensor `t`
        (element units along dim 0) independently, in place, in one call."""
        import torch
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("tensor must be a contiguous GPU tensor")
        kind = kind or kind_of(t)
        segs, nseg = segment_array(offsets, sizes)
        n = t.shape[0]
        params = self.params_for(sum(int(x) for x in sizes), kind, algo, True, params)
        need = segments_workspace_bytes(n, segs, nseg, kind, algo, params)
        ws = ws if ws is not None else self.workspace(need)
        self._check_ws(ws, need)
        if stream is None:
            stream = torch.cuda.current_stream(t.device)
        pp = ctypes.byref(params)
        rc = _lib.ips_sort_segments(self._h, ctypes.c_void_p(t.data_ptr()), n, TYPES[kind], ALGOS[algo],
                                    segs, nseg, ctypes.c_void_p(ws.data_ptr()), ws.numel(), pp,
                                    ctypes.c_void_p(stream.cuda_stream))
        if rc != IPS_OK:
            raise IpsError(rc, "ips_sort_segments", f"(hip={_lib.ips_last_hip_error(self._h)}, "
                                                    f"device={hex(_lib.ips_last_device_error(self._h))})")
        return t

    def sort_batch_(self, tensors, algo: str = "samplesort", params: Params | None = None, kind: str | None = None,
                    stream=None, ws=None):
        """Sort every tensor of the list (same element kind, separate buffers)
        in place with one batched call."""
        import torch
        if not tensors:
            return tensors
        kind = kind or kind_of(tensors[0])
        for t in tensors:
            if not t.is_cuda or not t.is_contiguous() or kind_of(t) != kind:
                raise ValueError("tensors must be contiguous GPU tensors of one element kind")
        cnt = len(tensors)
        ptrs = (ctypes.c_void_p * cnt)(*[t.data_ptr() for t in tensors])
        ns = (ctypes.c_uint64 * cnt)(*[t.shape[0] for t in tensors])
        params = self.params_for(sum(t.shape[0] for t in tensors), kind, algo, True, params)
        pp = ctypes.byref(params)
        out = ctypes.c_size_t(0)
        rc = _lib.ips_batch_workspace_bytes(ptrs, ns, cnt, TYPES[kind], ALGOS[algo], pp, ctypes.byref(out))
        if rc != IPS_OK:
            raise IpsError(rc, "ips_batch_workspace_bytes")
        ws = ws if ws is not None else self.workspace(out.value)
        self._check_ws(ws, out.value)
        if stream is None:
            stream = torch.cuda.current_stream(tensors[0].device)
        rc = _lib.ips_sort_batch(self._h, ptrs, ns, cnt, TYPES[kind], ALGOS[algo], ctypes.c_void_p(ws.data_ptr()),
                                 ws.numel(), pp, ctypes.c_void_p(stream.cuda_stream))
        if rc != IPS_OK:
            raise IpsError(rc, "ips_sort_batch", f"(hip={_lib.ips_last_hip_error(self._h)}, "
                                                 f"device={hex(_lib.ips_last_device_error(self._h))})")
        return tensors

    def serve_trace(self, tensors, arrivals, algos=None, hbm_budget: int = 64 << 30, policy: int = SERVE_BATCH,
                    max_batch: int = 0, params: Params | None = None, stream=None):
        """Replay an arrival trace: request i is tensor i (sorted in place),
        arriving arrivals[i] seconds after the start.  Returns the list of
        per-request dicts (start_s, done_s, status, batch) and the return code."""
        import torch
        cnt = len(tensors)
        reqs = (Request * max(1, cnt))()
        for i, t in enumerate(tensors):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("tensors must be contiguous GPU tensors")
            r = reqs[i]
            r.d_data, r.n = t.data_ptr(), t.shape[0]
            r.elem_type = TYPES[kind_of(t)]
            r.algo = ALGOS[algos[i] if algos else "samplesort"]
            r.arrival_s = float(arrivals[i])
        cfg = ServeConfig(hbm_budget, policy, max_batch)
        pp = ctypes.byref(params) if params is not None else None
        out = ctypes.c_size_t(0)
        rc = _lib.ips_serve_workspace_bytes(reqs, cnt, ctypes.byref(cfg), pp, ctypes.byref(out))
        if rc != IPS_OK:
            raise IpsError(rc, "ips_serve_workspace_bytes")
        ws = self.workspace(out.value)
        if stream is None:
            stream = torch.cuda.current_stream(tensors[0].device if cnt else None)
        rc = _lib.ips_serve_trace(self._h, reqs, cnt, ctypes.byref(cfg), ctypes.c_void_p(ws.data_ptr()),
                                  ws.numel(), pp, ctypes.c_void_p(stream.cuda_stream))
        res = [{"start_s": reqs[i].start_s, "done_s": reqs[i].done_s, "status": reqs[i].status,
                "batch": reqs[i].batch, "detail": reqs[i].detail} for i in range(cnt)]
        return res, rc

    def root_info(self) -> RootInfo:
        ri = RootInfo()
        _lib.ips_get_root_info(self._h, ctypes.byref(ri))
        return ri

    def stats(self) -> Stats:
        s = Stats()
        _lib.ips_get_stats(self._h, ctypes.byref(s))
        return s

    def profile(self) -> dict:
        """Per-level, per-kernel timing of the last sort run with FLAG_PROFILE:
        {row: {phase: (ms, elems, launches)}}; row "outside" is work outside
        the recursion levels."""
        p = Profile()
        _lib.ips_get_profile(self._h, ctypes.byref(p))
        out = {}
        for row in range(MAX_LEVELS + 1):
            d = {ph: (p.ms[row][i], int(p.elems[row][i]), int(p.launches[row][i]))
                 for i, ph in enumerate(PHASES) if p.launches[row][i]}
            if d:
                out["outside" if row == MAX_LEVELS else row] = d
        return out


_default = {}


def sorter(device: int = 0) -> Sorter:
    if device not in _default:
        _default[device] = Sorter(device)
    return _default[device]


def sort_(t, algo: str = "samplesort", params: Params | None = None, kind: str | None = None):
    """Sort a device tensor in place with the default sorter of its device."""
    return sorter(t.device.index or 0).sort_(t, algo=algo, params=params, kind=kind)
