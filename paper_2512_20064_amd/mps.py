"""ctypes binding of libmps.so: the C-ABI entry points under the same names.

Argument marshalling only.  Every step of the sampling sweep runs in the HIP
kernels of libmps.so; there is no Python or CPU fallback.  If the library is
missing, loading raises instead of degrading.

``Sampler`` is a convenience wrapper that takes torch device tensors (torch
is used for device memory and streams only).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmps.so")

MPS_OK, MPS_EINVAL, MPS_ENOMEM, MPS_ENODEV, MPS_EHIP, MPS_ENUMERIC = 0, -1, -2, -3, -4, -5
MPS_FP32, MPS_BF16X3, MPS_FP16, MPS_FP16X3, MPS_FP16F8, MPS_FP16F6 = 0, 1, 2, 3, 4, 5
PRECISIONS = {"fp32": MPS_FP32, "bf16x3": MPS_BF16X3, "fp16": MPS_FP16, "fp16x3": MPS_FP16X3,
              "fp16f8": MPS_FP16F8, "fp16f6": MPS_FP16F6}
MPS_C64, MPS_CF16, MPS_CF8 = 0, 1, 2
STORAGE = {"c64": MPS_C64, "cf16": MPS_CF16, "cf8": MPS_CF8}

STATUS_NAMES = {0: "MPS_OK", -1: "MPS_EINVAL", -2: "MPS_ENOMEM", -3: "MPS_ENODEV",
                -4: "MPS_EHIP", -5: "MPS_ENUMERIC"}

EXPORTS = ("mps_options_init", "mps_create", "mps_set_options", "mps_sample", "mps_sample_noalloc",
           "mps_sample_batch", "mps_autotune", "mps_autotune_tiles", "mps_set_tiles", "mps_get_stats",
           "mps_last_error", "mps_destroy")
MPS_TILE_WIDE, MPS_TILE_NARROW = 0, 1
NOALLOC_SCRATCH_BYTES = 256 << 20


def stored_bytes(kind: str, chi_l: int, d: int, chi_r: int) -> int:
    """Bytes of one site tensor in a storage form (layouts in include/mps.h)."""
    n = chi_l * d * chi_r
    if kind == "c64":
        return 8 * n
    if kind == "cf16":
        return 4 * n
    if kind == "cf8":
        nb = -(-chi_l // 128) * -(-(d * chi_r) // 128)
        return -(-2 * n // 256) * 256 + 4 * nb
    raise ValueError(kind)


def _bonds(tensors):
    """chi_0 .. chi_M of a list of (chi_k, d_k, chi_{k+1}) site tensors; the
    shapes must chain (the library reads each tensor with these sizes)."""
    for k, t in enumerate(tensors):
        if t.dim() != 3:
            raise ValueError(f"site {k}: expected a 3-d tensor (chi_l, d, chi_r)")
        if k and int(t.shape[0]) != int(tensors[k - 1].shape[2]):
            raise ValueError(f"site {k}: left bond {t.shape[0]} != right bond {tensors[k - 1].shape[2]} of site {k - 1}")
    return [int(tensors[0].shape[0])] + [int(t.shape[2]) for t in tensors]


class mps_options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("n_chunk", ctypes.c_int64),
        ("max_device_bytes", ctypes.c_int64),
        ("stream", ctypes.c_void_p),
        ("mps_id", ctypes.c_uint64),
        ("emit_n", ctypes.c_int64),
        ("emit_dmax", ctypes.c_int32),
        ("tile_group", ctypes.c_int32),
        ("emit_probs", ctypes.c_void_p),
        ("emit_u", ctypes.c_void_p),
        ("graph", ctypes.c_int32),
        ("fused_small", ctypes.c_int32),
        ("displace", ctypes.c_void_p),
    ]


class mps_chain(ctypes.Structure):
    _fields_ = [
        ("tensors", ctypes.POINTER(ctypes.c_void_p)),
        ("chi", ctypes.POINTER(ctypes.c_int32)),
        ("d", ctypes.POINTER(ctypes.c_int32)),
        ("M", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("mps_id", ctypes.c_uint64),
        ("outcomes", ctypes.c_void_p),
        ("logp", ctypes.c_void_p),
    ]


class mps_stats(ctypes.Structure):
    _fields_ = [
        ("contract_launches", ctypes.c_int64),
        ("measure_launches", ctypes.c_int64),
        ("pack_launches", ctypes.c_int64),
        ("contract_ms", ctypes.c_double),
        ("measure_ms", ctypes.c_double),
        ("pack_ms", ctypes.c_double),
        ("contract_flops", ctypes.c_double),
        ("measure_bytes", ctypes.c_double),
        ("n_chunk", ctypes.c_int64),
        ("flagged", ctypes.c_int64),
        ("scratch_bytes", ctypes.c_int64),
        ("h2d_bytes", ctypes.c_double),
        ("h2d_ms", ctypes.c_double),
        ("expand_ms", ctypes.c_double),
        ("staged_sites", ctypes.c_int64),
        ("fused_launches", ctypes.c_int64),
        ("fused_ms", ctypes.c_double),
        ("fused_flops", ctypes.c_double),
    ]


class mps_tune_report(ctypes.Structure):
    _fields_ = [
        ("n_chunk", ctypes.c_int64),
        ("tile_group", ctypes.c_int32),
        ("probe_sites", ctypes.c_int32),
        ("candidates", ctypes.c_int32),
        ("skipped", ctypes.c_int32),
        ("rate", ctypes.c_double),
        ("default_rate", ctypes.c_double),
    ]


class mps_tile_choice(ctypes.Structure):
    _fields_ = [
        ("chi_l", ctypes.c_int32),
        ("d", ctypes.c_int32),
        ("chi_r", ctypes.c_int32),
        ("tile", ctypes.c_int32),
        ("rows", ctypes.c_int64),
        ("ms_wide", ctypes.c_double),
        ("ms_narrow", ctypes.c_double),
    ]


class MPSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmps.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} not built: run __graft_entry__.build() or python -m paper_2512_20064_amd.build")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.mps_options_init.argtypes = [ctypes.POINTER(mps_options)]
    lib.mps_options_init.restype = ctypes.c_int
    lib.mps_create.argtypes = [ctypes.POINTER(P), ctypes.c_int32, ctypes.POINTER(mps_options)]
    lib.mps_create.restype = ctypes.c_int
    lib.mps_set_options.argtypes = [P, ctypes.POINTER(mps_options)]
    lib.mps_set_options.restype = ctypes.c_int
    lib.mps_sample.argtypes = [P, ctypes.POINTER(P), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_int64,
                               ctypes.c_int64, ctypes.c_uint64, P, P]
    lib.mps_sample.restype = ctypes.c_int
    lib.mps_sample_noalloc.argtypes = lib.mps_sample.argtypes
    lib.mps_sample_noalloc.restype = ctypes.c_int
    lib.mps_sample_batch.argtypes = [P, ctypes.c_int32, ctypes.POINTER(mps_chain), ctypes.c_int32, ctypes.c_int64,
                                     ctypes.c_int64, ctypes.c_uint64]
    lib.mps_sample_batch.restype = ctypes.c_int
    lib.mps_autotune.argtypes = [P, ctypes.POINTER(P), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                 ctypes.POINTER(mps_tune_report)]
    lib.mps_autotune.restype = ctypes.c_int
    lib.mps_autotune_tiles.argtypes = [P, ctypes.c_int32, ctypes.POINTER(mps_chain), ctypes.c_int64, ctypes.c_uint64,
                                       ctypes.POINTER(mps_tile_choice), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.mps_autotune_tiles.restype = ctypes.c_int
    lib.mps_set_tiles.argtypes = [P, ctypes.POINTER(mps_tile_choice), ctypes.c_int32]
    lib.mps_set_tiles.restype = ctypes.c_int
    lib.mps_get_stats.argtypes = [P, ctypes.POINTER(mps_stats)]
    lib.mps_get_stats.restype = ctypes.c_int
    lib.mps_last_error.argtypes = []
    lib.mps_last_error.restype = ctypes.c_char_p
    lib.mps_destroy.argtypes = [P]
    lib.mps_destroy.restype = None
    _lib = lib
    return lib


# ---- entry points under their C names --------------------------------------

def mps_last_error() -> str:
    return load().mps_last_error().decode()


def mps_options_init() -> mps_options:
    o = mps_options()
    rc = load().mps_options_init(ctypes.byref(o))
    if rc:
        raise MPSError(rc, mps_last_error())
    return o


def mps_create(device: int = 0, opt: mps_options | None = None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    rc = load().mps_create(ctypes.byref(h), device, ctypes.byref(opt) if opt is not None else None)
    if rc:
        raise MPSError(rc, mps_last_error())
    return h


def mps_set_options(h, opt: mps_options) -> None:
    rc = load().mps_set_options(h, ctypes.byref(opt))
    if rc:
        raise MPSError(rc, mps_last_error())


def mps_sample(h, tensor_ptrs, dtype: int, chi, d, M: int, N: int, n_offset: int, seed: int,
               outcomes_ptr: int, logp_ptr: int | None) -> int:
    """Raw call; returns the status code (MPS_ENUMERIC is not raised)."""
    arr = (ctypes.c_void_p * len(tensor_ptrs))(*[ctypes.c_void_p(int(p)) if p else None for p in tensor_ptrs])
    chi_a = (ctypes.c_int32 * len(chi))(*[int(x) for x in chi])
    d_a = (ctypes.c_int32 * len(d))(*[int(x) for x in d])
    return load().mps_sample(h, arr, dtype, chi_a, d_a, M, N, n_offset, ctypes.c_uint64(seed),
                             ctypes.c_void_p(outcomes_ptr) if outcomes_ptr else None,
                             ctypes.c_void_p(logp_ptr) if logp_ptr else None)


def mps_sample_noalloc(h, tensor_ptrs, dtype: int, chi, d, M: int, N: int, n_offset: int, seed: int,
                       outcomes_ptr: int, logp_ptr: int | None) -> int:
    """Raw call of the allocation-free variant; returns the status code."""
    arr = (ctypes.c_void_p * len(tensor_ptrs))(*[ctypes.c_void_p(int(p)) if p else None for p in tensor_ptrs])
    chi_a = (ctypes.c_int32 * len(chi))(*[int(x) for x in chi])
    d_a = (ctypes.c_int32 * len(d))(*[int(x) for x in d])
    return load().mps_sample_noalloc(h, arr, dtype, chi_a, d_a, M, N, n_offset, ctypes.c_uint64(seed),
                                     ctypes.c_void_p(outcomes_ptr) if outcomes_ptr else None,
                                     ctypes.c_void_p(logp_ptr) if logp_ptr else None)


def mps_autotune(h, tensor_ptrs, dtype: int, chi, d, M: int, N: int, seed: int):
    """Raw call; returns (status, mps_tune_report)."""
    arr = (ctypes.c_void_p * len(tensor_ptrs))(*[ctypes.c_void_p(int(p)) if p else None for p in tensor_ptrs])
    chi_a = (ctypes.c_int32 * len(chi))(*[int(x) for x in chi])
    d_a = (ctypes.c_int32 * len(d))(*[int(x) for x in d])
    rep = mps_tune_report()
    rc = load().mps_autotune(h, arr, dtype, chi_a, d_a, M, N, ctypes.c_uint64(seed), ctypes.byref(rep))
    return rc, rep


def make_chain(tensor_ptrs, chi, d, mps_id: int, outcomes_ptr: int, logp_ptr: int | None):
    """An mps_chain; the returned tuple keeps the ctypes arrays alive."""
    M = len(tensor_ptrs)
    arr = (ctypes.c_void_p * M)(*[ctypes.c_void_p(int(p)) if p else None for p in tensor_ptrs])
    chi_a = (ctypes.c_int32 * len(chi))(*[int(x) for x in chi])
    d_a = (ctypes.c_int32 * len(d))(*[int(x) for x in d])
    c = mps_chain(ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p)), ctypes.cast(chi_a, ctypes.POINTER(ctypes.c_int32)),
                  ctypes.cast(d_a, ctypes.POINTER(ctypes.c_int32)), M, 0, mps_id, outcomes_ptr or None,
                  logp_ptr or None)
    return c, (arr, chi_a, d_a)


def mps_sample_batch(h, chains, dtype: int, N: int, n_offset: int, seed: int) -> int:
    """Raw call over a list of mps_chain; returns the status code."""
    arr = (mps_chain * len(chains))(*chains)
    return load().mps_sample_batch(h, len(chains), arr, dtype, N, n_offset, ctypes.c_uint64(seed))


def mps_autotune_tiles(h, chains, rows: int, seed: int = 0):
    """Raw call over a list of mps_chain; returns (status, [mps_tile_choice])."""
    arr = (mps_chain * len(chains))(*chains)
    n = ctypes.c_int32(0)
    rc = load().mps_autotune_tiles(h, len(chains), arr, rows, ctypes.c_uint64(seed), None, 0, ctypes.byref(n))
    if rc:
        return rc, []
    out = (mps_tile_choice * max(1, n.value))()
    rc = load().mps_autotune_tiles(h, len(chains), arr, rows, ctypes.c_uint64(seed), out, n.value, ctypes.byref(n))
    return rc, list(out[:n.value]) if rc == 0 else []


def mps_set_tiles(h, choices) -> int:
    """Install a list of mps_tile_choice (an empty list clears); returns the status."""
    arr = (mps_tile_choice * max(1, len(choices)))(*choices)
    return load().mps_set_tiles(h, arr if choices else None, len(choices))


def mps_get_stats(h) -> mps_stats:
    st = mps_stats()
    rc = load().mps_get_stats(h, ctypes.byref(st))
    if rc:
        raise MPSError(rc, mps_last_error())
    return st


def mps_destroy(h) -> None:
    load().mps_destroy(h)


# ---- convenience wrapper over torch device tensors --------------------------

class PreparedBatch:
    """Descriptors of a list of chains (site pointers, bonds, physical
    dimensions; chain b has mps_id = b), checked and built once for repeated
    Sampler.sample_batch calls over the same device-resident tensors.  Holds
    references to the tensors, so they stay alive while it does."""

    def __init__(self, chains):
        import torch
        self.chains = [list(c) for c in chains]
        self.descs, self._keep = [], []
        for b, tensors in enumerate(self.chains):
            shapes = []
            for k, t in enumerate(tensors):
                if t.dtype != torch.complex64 or not t.is_cuda or not t.is_contiguous():
                    raise ValueError(f"chain {b} site {k}: site tensors must be contiguous complex64 CUDA tensors")
                shapes.append(tuple(t.shape))
            chi, d = _bonds_of_shapes(shapes, b)
            c, keep = make_chain([t.data_ptr() for t in tensors], chi, d, b, 0, None)
            self.descs.append(c)
            self._keep.append(keep)


def prepare_batch(chains) -> PreparedBatch:
    return PreparedBatch(chains)


def _bonds_of_shapes(shapes, b=0):
    """chi_0 .. chi_M and d_0 .. d_{M-1} from (chi_k, d_k, chi_{k+1}) shapes."""
    if not shapes:
        raise ValueError(f"chain {b}: no sites")
    for k, sh in enumerate(shapes):
        if len(sh) != 3:
            raise ValueError(f"chain {b} site {k}: expected a 3-d tensor (chi_l, d, chi_r)")
        if k and sh[0] != shapes[k - 1][2]:
            raise ValueError(f"chain {b} site {k}: left bond {sh[0]} != right bond {shapes[k - 1][2]} of site {k - 1}")
    return [shapes[0][0]] + [sh[2] for sh in shapes], [sh[1] for sh in shapes]


class Sampler:
    """Owns an mps handle; samples from complex64 torch tensors on the GPU.

    tensors: list of M torch.complex64 CUDA tensors of shape (chi_k, d_k, chi_{k+1}),
    contiguous.  Returns (outcomes int32 [N, M], logp float64 [N]) as CUDA tensors.
    """

    def __init__(self, device: int = 0, n_chunk: int = 0, profile: bool = False,
                 max_device_bytes: int = 0, mps_id: int = 0, precision=MPS_FP32, tile_group: int = 0,
                 graph: bool = False, fused_small: bool = True):
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        self.opt = mps_options_init()
        self.opt.tile_group = tile_group
        self.opt.graph = int(graph)
        self.opt.fused_small = 0 if fused_small else 1
        self.opt.n_chunk = n_chunk
        self.opt.profile = int(profile)
        self.opt.max_device_bytes = max_device_bytes
        self.opt.mps_id = mps_id
        self.opt.precision = precision
        self.device = device
        self.h = mps_create(device, self.opt)

    def close(self):
        if self.h:
            mps_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sample(self, tensors, N: int, seed: int, n_offset: int = 0, emit_n: int = 0,
               emit_dmax: int = 0, want_logp: bool = True, stream=None, raise_numeric: bool = False,
               displace=None):
        """displace: optional complex64 CUDA tensor [N, M] of per-sample displacements."""
        import torch
        dev = torch.device("cuda", self.device)
        M = len(tensors)
        chi = _bonds(tensors)
        d = [int(t.shape[1]) for t in tensors]
        for t in tensors:
            if t.dtype != torch.complex64 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("site tensors must be contiguous complex64 CUDA tensors")
        outcomes = torch.empty((N, M), dtype=torch.int32, device=dev)
        logp = torch.empty((N,), dtype=torch.float64, device=dev) if want_logp else None
        emit_probs = emit_u = None
        opt = mps_options.from_buffer_copy(self.opt)
        if emit_n:
            emit_dmax = emit_dmax or max(d)
            emit_probs = torch.full((emit_n, M, emit_dmax), float("nan"), dtype=torch.float64, device=dev)
            emit_u = torch.zeros((emit_n, M), dtype=torch.float64, device=dev)
            opt.emit_n = emit_n
            opt.emit_dmax = emit_dmax
            opt.emit_probs = emit_probs.data_ptr()
            opt.emit_u = emit_u.data_ptr()
        if displace is not None:
            if displace.dtype != torch.complex64 or not displace.is_cuda or tuple(displace.shape) != (N, M) \
                    or not displace.is_contiguous():
                raise ValueError("displace must be a contiguous complex64 CUDA tensor of shape (N, M)")
            opt.displace = displace.data_ptr()
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        opt.stream = s.cuda_stream
        mps_set_options(self.h, opt)
        rc = mps_sample(self.h, [t.data_ptr() for t in tensors], MPS_C64, chi, d, M, N, n_offset, seed,
                        outcomes.data_ptr(), logp.data_ptr() if logp is not None else None)
        self.status = rc
        if rc and (rc != MPS_ENUMERIC or raise_numeric):
            raise MPSError(rc, mps_last_error())
        self.stats = mps_get_stats(self.h)
        out = {"outcomes": outcomes, "logp": logp, "status": rc}
        if emit_n:
            out["probs"] = emit_probs
            out["u"] = emit_u
        return out

    def autotune(self, tensors, N: int, seed: int = 0, stream=None, cache: str | None = None) -> dict:
        """Pick n_chunk and tile_group for this chain shape (mps_autotune) and
        keep them for later calls.  cache: optional JSON file; an entry for
        the same (precision, N, chi, d) is reused instead of timing again."""
        import hashlib
        import json
        import torch
        M = len(tensors)
        chi = _bonds(tensors)
        d = [int(t.shape[1]) for t in tensors]
        for t in tensors:
            if t.dtype != torch.complex64 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("site tensors must be contiguous complex64 CUDA tensors")
        key = "%d:%d:%s" % (self.opt.precision, N, hashlib.sha256(repr((chi, d)).encode()).hexdigest()[:16])
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
            if key in table:
                self.opt.n_chunk = int(table[key]["n_chunk"])
                self.opt.tile_group = int(table[key]["tile_group"])
                return dict(table[key], cached=True)
        opt = mps_options.from_buffer_copy(self.opt)
        s = stream if stream is not None else torch.cuda.current_stream(torch.device("cuda", self.device))
        opt.stream = s.cuda_stream
        mps_set_options(self.h, opt)
        rc, rep = mps_autotune(self.h, [t.data_ptr() for t in tensors], MPS_C64, chi, d, M, N, seed)
        if rc:
            raise MPSError(rc, mps_last_error())
        self.opt.n_chunk = rep.n_chunk
        self.opt.tile_group = rep.tile_group
        out = {name: getattr(rep, name) for name, _ in mps_tune_report._fields_}
        if cache:
            table[key] = out
            with open(cache, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
        return dict(out, cached=False)

    def autotune_tiles(self, chains, rows: int, seed: int = 0, stream=None, cache: str | None = None) -> list:
        """Choose the contraction tile per site shape for `rows` samples per
        launch (mps_autotune_tiles) and keep the choices in the handle.

        chains: a list of site-tensor lists (one chain), a list of such lists,
        or a PreparedBatch.  cache: optional JSON file of earlier choices,
        keyed by precision, shape and rows; shapes found there are installed
        with mps_set_tiles instead of being timed again.  Returns the choices
        as dicts."""
        import json
        import torch
        if isinstance(chains, PreparedBatch):
            prep = chains
        else:
            lists = [chains] if chains and not isinstance(chains[0], (list, tuple)) else chains
            prep = prepare_batch(lists)
        shapes = set()
        for c in prep.chains:
            for t in c:
                shapes.add((int(t.shape[0]), int(t.shape[1]), int(t.shape[2])))
        key = lambda sh: "%d:%d:%d:%d:%d" % (self.opt.precision, sh[0], sh[1], sh[2], rows)
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        if table and all(key(sh) in table for sh in shapes):
            ch = [mps_tile_choice(*sh, int(table[key(sh)]["tile"]), rows, float(table[key(sh)]["ms_wide"]),
                                  float(table[key(sh)]["ms_narrow"])) for sh in sorted(shapes)]
            rc = mps_set_tiles(self.h, ch)
            if rc:
                raise MPSError(rc, mps_last_error())
            return [dict(table[key(sh)], cached=True) for sh in sorted(shapes)]
        opt = mps_options.from_buffer_copy(self.opt)
        s = stream if stream is not None else torch.cuda.current_stream(torch.device("cuda", self.device))
        opt.stream = s.cuda_stream
        mps_set_options(self.h, opt)
        rc, out = mps_autotune_tiles(self.h, prep.descs, rows, seed)
        if rc:
            raise MPSError(rc, mps_last_error())
        res = []
        for c in out:
            d = {name: getattr(c, name) for name, _ in mps_tile_choice._fields_}
            table[key((c.chi_l, c.d, c.chi_r))] = d
            res.append(dict(d, cached=False))
        if cache:
            with open(cache, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
        return res

    def set_tiles(self, choices) -> None:
        """Install tile choices: dicts with chi_l, d, chi_r, tile, rows ([] clears)."""
        ch = [mps_tile_choice(int(c["chi_l"]), int(c["d"]), int(c["chi_r"]), int(c["tile"]), int(c["rows"]),
                              float(c.get("ms_wide", 0.0)), float(c.get("ms_narrow", 0.0))) for c in choices]
        rc = mps_set_tiles(self.h, ch)
        if rc:
            raise MPSError(rc, mps_last_error())

    def sample_batch(self, chains, N: int, seed: int, n_offset: int = 0, want_logp: bool = True, stream=None,
                     raise_numeric: bool = False):
        """chains: list of lists of complex64 CUDA tensors, or a PreparedBatch
        of them (prepare_batch); chain b uses mps_id = b.

        Returns a list of (outcomes [N, M_b] int32, logp [N] float64) CUDA tensor pairs.
        """
        import torch
        prep = chains if isinstance(chains, PreparedBatch) else prepare_batch(chains)
        dev = torch.device("cuda", self.device)
        outs = []
        descs = (mps_chain * len(prep.descs))()
        for b, c in enumerate(prep.descs):
            o = torch.empty((N, c.M), dtype=torch.int32, device=dev)
            lp = torch.empty((N,), dtype=torch.float64, device=dev) if want_logp else None
            descs[b] = c
            descs[b].outcomes = o.data_ptr() or None
            descs[b].logp = lp.data_ptr() if lp is not None else None
            outs.append((o, lp))
        opt = mps_options.from_buffer_copy(self.opt)
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        opt.stream = s.cuda_stream
        mps_set_options(self.h, opt)
        rc = load().mps_sample_batch(self.h, len(prep.descs), descs, MPS_C64, N, n_offset, ctypes.c_uint64(seed))
        self.status = rc
        if rc and (rc != MPS_ENUMERIC or raise_numeric):
            raise MPSError(rc, mps_last_error())
        self.stats = mps_get_stats(self.h)
        return outs

    def sample_stored(self, stored, shapes, kind: str, N: int, seed: int, n_offset: int = 0, emit_n: int = 0,
                      emit_dmax: int = 0, stream=None, raise_numeric: bool = False, displace=None):
        """Sample from site tensors held in a stored form.

        stored: list of M uint8 torch tensors (CUDA, or pinned CPU memory), one
        per site, holding the bytes of the site in storage `kind` ("c64",
        "cf16" or "cf8"); shapes: the M (chi_l, d, chi_r) site shapes.
        """
        import torch
        dev = torch.device("cuda", self.device)
        M = len(stored)
        chi = [int(shapes[0][0])] + [int(s[2]) for s in shapes]
        d = [int(s[1]) for s in shapes]
        if kind not in STORAGE or len(shapes) != M:
            raise ValueError("kind must be one of %s and shapes must have one entry per site" % sorted(STORAGE))
        for k, t in enumerate(stored):
            if t.dtype != torch.uint8 or not t.is_contiguous() or not (t.is_cuda or t.is_pinned()):
                raise ValueError("stored sites must be contiguous uint8 tensors on the GPU or in pinned memory")
            need = stored_bytes(kind, *[int(x) for x in shapes[k]])
            if t.numel() < need:
                raise ValueError(f"site {k}: {t.numel()} bytes stored, {kind} of shape {tuple(shapes[k])} needs {need}")
            if k + 1 < M and int(shapes[k][2]) != int(shapes[k + 1][0]):
                raise ValueError(f"site {k}: right bond {shapes[k][2]} != left bond of site {k + 1}")
        outcomes = torch.empty((N, M), dtype=torch.int32, device=dev)
        logp = torch.empty((N,), dtype=torch.float64, device=dev)
        emit_probs = emit_u = None
        opt = mps_options.from_buffer_copy(self.opt)
        if emit_n:
            emit_dmax = emit_dmax or max(d)
            emit_probs = torch.full((emit_n, M, emit_dmax), float("nan"), dtype=torch.float64, device=dev)
            emit_u = torch.zeros((emit_n, M), dtype=torch.float64, device=dev)
            opt.emit_n = emit_n
            opt.emit_dmax = emit_dmax
            opt.emit_probs = emit_probs.data_ptr()
            opt.emit_u = emit_u.data_ptr()
        if displace is not None:
            if displace.dtype != torch.complex64 or not displace.is_cuda or tuple(displace.shape) != (N, M) \
                    or not displace.is_contiguous():
                raise ValueError("displace must be a contiguous complex64 CUDA tensor of shape (N, M)")
            opt.displace = displace.data_ptr()
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        opt.stream = s.cuda_stream
        mps_set_options(self.h, opt)
        rc = mps_sample(self.h, [t.data_ptr() for t in stored], STORAGE[kind], chi, d, M, N, n_offset, seed,
                        outcomes.data_ptr(), logp.data_ptr())
        self.status = rc
        if rc and (rc != MPS_ENUMERIC or raise_numeric):
            raise MPSError(rc, mps_last_error())
        self.stats = mps_get_stats(self.h)
        out = {"outcomes": outcomes, "logp": logp, "status": rc}
        if emit_n:
            out["probs"] = emit_probs
            out["u"] = emit_u
        return out
