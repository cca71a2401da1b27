"""Python binding of libdrf (ctypes).  Argument marshalling only: every step
of the check runs in the library's host code and gfx950 kernels.  PyTorch
provides device memory and streams.

    chk = Checker(device=0)
    r = chk.check("(seq (wr tid) (sync) (rd (mod (+ tid 1) 8)))", 8)
    r.racy, r.witness, r.phase_counts, r.num_records

There is no CPU fallback: without libdrf.so or a GPU this module raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple, Union

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdrf.so")

OK = 0
E_ARG, E_BYTECODE, E_UNBOUND, E_SHADOW, E_SYNC_IN_U = -1, -2, -3, -4, -5
E_DIVERGENT, E_RANGE, E_NOMEM, E_HIP, E_LIMIT, E_MULTI, E_ILLTYPED = -6, -7, -8, -9, -10, -11, -12
NONE = 0xFFFFFFFF


class DrfError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__("%s failed with code %d" % (what, code))
        self.code = code


class Plan(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("num_phases", ctypes.c_uint32), ("index_bits", ctypes.c_uint32),
                ("wide", ctypes.c_uint32), ("max_records", ctypes.c_uint64), ("nests", ctypes.c_uint64),
                ("max_phase_records", ctypes.c_uint64), ("scratch_bytes", ctypes.c_uint64)]


class GraphCaps(ctypes.Structure):
    _fields_ = [("max_protocols", ctypes.c_uint32), ("max_nests", ctypes.c_uint32),
                ("max_code_words", ctypes.c_uint32), ("max_fixed", ctypes.c_uint32),
                ("max_phases", ctypes.c_uint64), ("max_units", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


TABLE_OFF = 255


class Tuning(ctypes.Structure):
    _fields_ = [("tile_events", ctypes.c_uint32), ("digit_bits", ctypes.c_uint32),
                ("unit_events", ctypes.c_uint32), ("item_events", ctypes.c_uint32),
                ("table_bits", ctypes.c_uint32)]


class _Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("racy", ctypes.c_uint32), ("phase", ctypes.c_uint32),
                ("index", ctypes.c_uint32), ("tid_i", ctypes.c_uint32), ("tid_j", ctypes.c_uint32),
                ("num_records", ctypes.c_uint64), ("num_phases", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


RESULT_DTYPE = np.dtype([("status", "<i4"), ("racy", "<u4"), ("phase", "<u4"), ("index", "<u4"),
                         ("tid_i", "<u4"), ("tid_j", "<u4"), ("num_records", "<u8"), ("num_phases", "<u4"),
                         ("reserved", "<u4")])
assert RESULT_DTYPE.itemsize == ctypes.sizeof(_Result) == 40

_lib = None


def lib() -> ctypes.CDLL:
    """Load libdrf.so (built in-tree by paper_2203_12878_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libdrf.so is not built (run paper_2203_12878_amd/build.py)")
        # PyTorch ships its own HIP runtime under the same soname: loading it
        # first makes libdrf bind to that one copy, so that device memory,
        # streams and the library's launches share one runtime (a second
        # copy loaded later could not open the device)
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.drf_version.restype = ctypes.c_char_p
        L.drf_compile_text.argtypes = [ctypes.c_char_p, ctypes.c_size_t, u32p, ctypes.c_uint32, u32p]
        L.drf_plan_protocol.argtypes = [u32p, ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(Plan)]
        L.drf_plan_batch.argtypes = [ctypes.c_void_p, u32p, u64p, u32p, ctypes.c_uint32, ctypes.POINTER(Plan), u64p]
        L.drf_ctx_create.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(ctypes.c_void_p)]
        L.drf_ctx_release.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
        L.drf_ctx_destroy.argtypes = [ctypes.c_void_p]
        L.drf_check_protocol.argtypes = [ctypes.c_void_p, u32p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
        L.drf_check_batch.argtypes = [ctypes.c_void_p, u32p, u64p, u32p, ctypes.c_uint32, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
        L.drf_graph_create.argtypes = [ctypes.c_void_p, ctypes.POINTER(GraphCaps), ctypes.c_void_p,
                                       ctypes.POINTER(ctypes.c_void_p)]
        L.drf_graph_check.argtypes = L.drf_check_batch.argtypes
        L.drf_graph_destroy.argtypes = [ctypes.c_void_p]
        for f in ("drf_graph_create", "drf_graph_check", "drf_graph_destroy"):
            getattr(L, f).restype = ctypes.c_int
        L.drf_check_batch_noalloc.argtypes = L.drf_check_batch.argtypes
        L.drf_check_batch_noalloc.restype = ctypes.c_int
        L.drf_prepare_batch.argtypes = [ctypes.c_void_p, u32p, u64p, u32p, ctypes.c_uint32, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_void_p)]
        L.drf_run_prepared.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.drf_prepared_destroy.argtypes = [ctypes.c_void_p]
        L.drf_prepared_launches.argtypes = [ctypes.c_void_p]
        L.drf_prepared_launches.restype = ctypes.c_uint64
        for f in ("drf_prepare_batch", "drf_run_prepared", "drf_prepared_destroy"):
            getattr(L, f).restype = ctypes.c_int
        L.drf_babycuda_infer.argtypes = [ctypes.c_char_p, ctypes.c_size_t, ctypes.c_char_p, ctypes.c_char_p,
                                         ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t),
                                         ctypes.POINTER(ctypes.c_int32)]
        L.drf_babycuda_infer.restype = ctypes.c_int
        L.drf_text_slot.argtypes = [ctypes.c_char_p, ctypes.c_size_t, ctypes.c_char_p, u32p]
        L.drf_bind_param.argtypes = [u32p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, u32p, ctypes.c_uint32,
                                     u32p]
        L.drf_plan_sweep.argtypes = [u32p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                     ctypes.c_uint32, ctypes.POINTER(Plan), u64p]
        L.drf_check_sweep.argtypes = [ctypes.c_void_p, u32p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_uint64, ctypes.c_void_p]
        L.drf_protocol_arrays.argtypes = [u32p, ctypes.c_uint32, u32p]
        L.drf_plan_arrays.argtypes = [u32p, ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(Plan), ctypes.c_uint32,
                                      u64p]
        L.drf_check_arrays.argtypes = [ctypes.c_void_p, u32p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
        for f in ("drf_text_slot", "drf_bind_param", "drf_plan_sweep", "drf_check_sweep", "drf_protocol_arrays",
                  "drf_plan_arrays", "drf_check_arrays"):
            getattr(L, f).restype = ctypes.c_int
        L.drf_ctx_set_tuning.argtypes = [ctypes.c_void_p, ctypes.POINTER(Tuning)]
        L.drf_ctx_get_tuning.argtypes = [ctypes.c_void_p, ctypes.POINTER(Tuning)]
        L.drf_ctx_set_profiling.argtypes = [ctypes.c_void_p, ctypes.c_int]
        for f in ("drf_compile_text", "drf_plan_protocol", "drf_plan_batch", "drf_ctx_create", "drf_ctx_release",
                  "drf_ctx_destroy",
                  "drf_check_protocol", "drf_check_batch", "drf_ctx_set_tuning", "drf_ctx_get_tuning",
                  "drf_ctx_set_profiling"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _u32p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _u64p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def compile_text(text: str) -> np.ndarray:
    """Text form -> bytecode (uint32 array)."""
    L = lib()
    b = text.encode()
    n = ctypes.c_uint32(0)
    cap = max(64, 4 * len(b) + 16)
    out = np.zeros(cap, dtype=np.uint32)
    rc = L.drf_compile_text(b, len(b), _u32p(out), cap, ctypes.byref(n))
    if rc == E_NOMEM:
        out = np.zeros(n.value, dtype=np.uint32)
        rc = L.drf_compile_text(b, len(b), _u32p(out), n.value, ctypes.byref(n))
    if rc != OK:
        raise DrfError(rc, "drf_compile_text")
    return out[:n.value].copy()


def _code(c: Union[str, np.ndarray]) -> np.ndarray:
    return compile_text(c) if isinstance(c, str) else np.ascontiguousarray(c, dtype=np.uint32)


def infer(program: str, params: Sequence[str] = ()) -> Tuple[int, Optional[str]]:
    """BabyCUDA program -> (status, protocol text): drf_babycuda_infer with
    the typing context {tid} + params.  status 0 gives the protocol; else
    E_ILLTYPED / E_UNBOUND / E_SHADOW and None."""
    b = program.encode()
    ps = " ".join(params).encode() if params else None
    need = ctypes.c_size_t(0)
    st = ctypes.c_int32(0)
    cap = 4 * len(b) + 64
    out = ctypes.create_string_buffer(cap)
    rc = lib().drf_babycuda_infer(b, len(b), ps, out, cap, ctypes.byref(need), ctypes.byref(st))
    if rc == E_NOMEM:
        out = ctypes.create_string_buffer(need.value)
        rc = lib().drf_babycuda_infer(b, len(b), ps, out, need.value, ctypes.byref(need), ctypes.byref(st))
    if rc != OK:
        raise DrfError(rc, "drf_babycuda_infer")
    return (st.value, out.value.decode() if st.value == 0 else None)


def text_slot(text: str, name: str) -> int:
    """Variable slot of `name` in the bytecode compile_text(text) gives."""
    b = text.encode()
    s = ctypes.c_uint32(0)
    rc = lib().drf_text_slot(b, len(b), name.encode(), ctypes.byref(s))
    if rc != OK:
        raise DrfError(rc, "drf_text_slot")
    return s.value


def bind_param(code: Union[str, np.ndarray], slot: int, value: int) -> np.ndarray:
    """Bytecode with variable `slot` replaced by the constant `value`."""
    c = _code(code)
    n = ctypes.c_uint32(0)
    out = np.zeros(len(c) + 64, dtype=np.uint32)
    rc = lib().drf_bind_param(_u32p(c), len(c), slot, value, _u32p(out), len(out), ctypes.byref(n))
    if rc == E_NOMEM:
        out = np.zeros(n.value, dtype=np.uint32)
        rc = lib().drf_bind_param(_u32p(c), len(c), slot, value, _u32p(out), len(out), ctypes.byref(n))
    if rc != OK:
        raise DrfError(rc, "drf_bind_param")
    return out[:n.value].copy()


def protocol_arrays(code: Union[str, np.ndarray]) -> int:
    c = _code(code)
    k = ctypes.c_uint32(0)
    rc = lib().drf_protocol_arrays(_u32p(c), len(c), ctypes.byref(k))
    if rc != OK:
        raise DrfError(rc, "drf_protocol_arrays")
    return k.value


def plan(code: Union[str, np.ndarray], n: int) -> Plan:
    code = compile_text(code) if isinstance(code, str) else np.ascontiguousarray(code, dtype=np.uint32)
    p = Plan()
    rc = lib().drf_plan_protocol(_u32p(code), len(code), n, ctypes.byref(p))
    if rc != OK:
        raise DrfError(rc, "drf_plan_protocol")
    return p


def pack(codes: Sequence[np.ndarray]):
    """Concatenated bytecode and the offsets (count + 1) of each protocol."""
    off = np.zeros(len(codes) + 1, dtype=np.uint64)
    if codes:
        off[1:] = np.cumsum([len(c) for c in codes])
    code = np.concatenate(codes).astype(np.uint32) if codes else np.zeros(1, np.uint32)
    return code, off


def plan_batch(items: Sequence[Tuple[Union[str, np.ndarray], int]], checker: "Optional[Checker]" = None):
    """drf_plan_batch: the plan of every protocol and the device scratch one
    batched check of all of them may take (for the checker's tuning)."""
    codes = [compile_text(c) if isinstance(c, str) else np.ascontiguousarray(c, dtype=np.uint32) for c, _ in items]
    code, off = pack(codes)
    nth = np.array([int(n) for _, n in items], dtype=np.uint32)
    plans = (Plan * max(1, len(items)))()
    total = np.zeros(1, dtype=np.uint64)
    ctx = checker._ctx if checker is not None else None
    rc = lib().drf_plan_batch(ctx, _u32p(code), _u64p(off), _u32p(nth), len(items), plans, _u64p(total))
    if rc != OK:
        raise DrfError(rc, "drf_plan_batch")
    return list(plans)[:len(items)], int(total[0])


@dataclass
class CheckResult:
    status: int
    racy: int = 0
    witness: Optional[Tuple[int, int, int, int]] = None
    phase_counts: Sequence[int] = field(default_factory=list)   # uint64 array for device results
    num_records: int = 0

    def key(self):
        return (self.status, self.racy, self.witness, tuple(self.phase_counts), self.num_records)


class Batch:
    """Bytecode of several protocols packed for drf_check_batch, with the
    device result and phase-count buffers it needs."""

    def __init__(self, items: Sequence[Tuple[Union[str, np.ndarray], int]], device: int = 0,
                 plans: Optional[Sequence[Plan]] = None):
        import torch
        codes = [compile_text(c) if isinstance(c, str) else np.ascontiguousarray(c, dtype=np.uint32)
                 for c, _ in items]
        self.count = len(items)
        self.nthreads = np.array([int(n) for _, n in items], dtype=np.uint32)
        self.code, self.code_off = pack(codes)
        self.plans = list(plans) if plans is not None else [plan(c, int(n)) for c, n in zip(codes, self.nthreads)]
        self.phase_off = np.zeros(self.count + 1, dtype=np.uint64)
        nph = [p.num_phases if p.status == 0 else 0 for p in self.plans]
        if nph:
            self.phase_off[1:] = np.cumsum(nph)
        self.total_phases = int(self.phase_off[-1])
        dev = torch.device("cuda", device)
        self.results = torch.zeros(max(1, self.count) * 40, dtype=torch.uint8, device=dev)
        self.counts = torch.zeros(max(1, self.total_phases), dtype=torch.int64, device=dev)

    def collect(self) -> List[CheckResult]:
        """Copy results back (after the stream work has finished)."""
        return _collect(self.results, self.counts, self.phase_off, self.count)


class Outputs:
    """Device result and phase-count buffers for `count` results laid out
    by their plans (as drf_check_batch lays them out)."""

    def __init__(self, plans: Sequence[Plan], device: int = 0):
        import torch
        self.count = len(plans)
        self.phase_off = np.zeros(self.count + 1, dtype=np.uint64)
        nph = [p.num_phases if p.status == 0 else 0 for p in plans]
        if nph:
            self.phase_off[1:] = np.cumsum(nph)
        self.total_phases = int(self.phase_off[-1])
        dev = torch.device("cuda", device)
        self.results = torch.zeros(max(1, self.count) * 40, dtype=torch.uint8, device=dev)
        self.counts = torch.zeros(max(1, self.total_phases), dtype=torch.int64, device=dev)

    def collect(self) -> List[CheckResult]:
        return _collect(self.results, self.counts, self.phase_off, self.count)


def _collect(results, counts_t, phase_off, count) -> List[CheckResult]:
    res = np.frombuffer(results.cpu().numpy().tobytes(), dtype=RESULT_DTYPE)[:count]
    counts = counts_t.cpu().numpy().view(np.uint64)
    out = []
    for i in range(count):
        r = res[i]
        st = int(r["status"])
        if st != 0:
            out.append(CheckResult(st))
            continue
        wit = (int(r["phase"]), int(r["index"]), int(r["tid_i"]), int(r["tid_j"])) if r["racy"] else None
        a = int(phase_off[i])
        pc = counts[a:a + int(r["num_phases"])]   # a view: no per-phase Python objects
        out.append(CheckResult(0, int(r["racy"]), wit, pc, int(r["num_records"])))
    return out


class Prepared:
    """A batch checked once and captured as one hipGraph (drf_prepare_batch);
    run() replays the whole device work into the batch's buffers."""

    def __init__(self, chk: "Checker", b: Batch, stream=None):
        self.batch = b
        self._h = ctypes.c_void_p()
        rc = lib().drf_prepare_batch(chk._ctx, _u32p(b.code), _u64p(b.code_off), _u32p(b.nthreads), b.count,
                                     ctypes.c_void_p(b.results.data_ptr()), ctypes.c_void_p(b.counts.data_ptr()),
                                     b.total_phases, chk._stream(stream), ctypes.byref(self._h))
        if rc != OK:
            raise DrfError(rc, "drf_prepare_batch")
        self._stream = chk._stream

    @property
    def launches(self) -> int:
        return int(lib().drf_prepared_launches(self._h))

    def run(self, stream=None) -> None:
        rc = lib().drf_run_prepared(self._h, self._stream(stream))
        if rc != OK:
            raise DrfError(rc, "drf_run_prepared")

    def close(self):
        if self._h:
            lib().drf_prepared_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GraphClass:
    """A hipGraph captured once for a shape class of statically small
    batches (drf_graph_create); check() replays it for a new batch, or
    returns False when the batch is outside the class (nothing written)."""

    def __init__(self, chk: "Checker", max_protocols: int = 256, max_nests: int = 8192,
                 max_code_words: int = 1 << 18, max_fixed: int = 8192, max_phases: int = 1 << 20,
                 max_units: int = 1 << 16):
        self.caps = GraphCaps(max_protocols, max_nests, max_code_words, max_fixed, max_phases, max_units, 0)
        self._h = ctypes.c_void_p()
        self._stream = chk._stream
        rc = lib().drf_graph_create(chk._ctx, ctypes.byref(self.caps), None, ctypes.byref(self._h))
        if rc != OK:
            raise DrfError(rc, "drf_graph_create")

    def check(self, b: Batch, stream=None) -> bool:
        rc = lib().drf_graph_check(self._h, _u32p(b.code), _u64p(b.code_off), _u32p(b.nthreads), b.count,
                                   ctypes.c_void_p(b.results.data_ptr()), ctypes.c_void_p(b.counts.data_ptr()),
                                   b.total_phases, self._stream(stream))
        if rc == E_LIMIT:
            return False
        if rc != OK:
            raise DrfError(rc, "drf_graph_check")
        return True

    def close(self):
        if self._h:
            lib().drf_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Checker:
    """Owns a libdrf context on one HIP device (one per host thread)."""

    def __init__(self, device: int = 0, scratch_limit: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: libdrf needs an MI355X")
        self.device = device
        self._ctx = ctypes.c_void_p()
        rc = lib().drf_ctx_create(device, int(scratch_limit), ctypes.byref(self._ctx))
        if rc != OK:
            raise DrfError(rc, "drf_ctx_create")

    def close(self):
        if self._ctx:
            lib().drf_ctx_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def release(self, keep_bytes: int = 0) -> None:
        """Hand the context's scratch pools back when they exceed keep_bytes."""
        rc = lib().drf_ctx_release(self._ctx, int(keep_bytes))
        if rc != OK:
            raise DrfError(rc, "drf_ctx_release")

    def set_tuning(self, tile_events=0, digit_bits=0, unit_events=0, item_events=0, table_bits=0):
        """Zero keeps a field; table_bits=TABLE_OFF turns the table path off."""
        t = Tuning(tile_events, digit_bits, unit_events, item_events, table_bits)
        rc = lib().drf_ctx_set_tuning(self._ctx, ctypes.byref(t))
        if rc != OK:
            raise DrfError(rc, "drf_ctx_set_tuning")

    def tuning(self) -> dict:
        t = Tuning()
        lib().drf_ctx_get_tuning(self._ctx, ctypes.byref(t))
        return {f: getattr(t, f) for f, _ in Tuning._fields_}

    def _stream(self, stream):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(s.cuda_stream)

    def run_batch(self, b: Batch, stream=None) -> None:
        """Enqueue drf_check_batch for a prepared batch (results valid after
        the stream is synchronized)."""
        rc = lib().drf_check_batch(self._ctx, _u32p(b.code), _u64p(b.code_off), _u32p(b.nthreads), b.count,
                                   ctypes.c_void_p(b.results.data_ptr()), ctypes.c_void_p(b.counts.data_ptr()),
                                   b.total_phases, self._stream(stream))
        if rc != OK:
            raise DrfError(rc, "drf_check_batch")

    def run_batch_noalloc(self, b: Batch, stream=None) -> None:
        """drf_check_batch_noalloc for a prepared batch: the same check with
        the library's fixed per-device scratch array instead of context
        pools (returns once the work on the stream has completed)."""
        rc = lib().drf_check_batch_noalloc(self._ctx, _u32p(b.code), _u64p(b.code_off), _u32p(b.nthreads), b.count,
                                           ctypes.c_void_p(b.results.data_ptr()),
                                           ctypes.c_void_p(b.counts.data_ptr()), b.total_phases,
                                           self._stream(stream))
        if rc != OK:
            raise DrfError(rc, "drf_check_batch_noalloc")

    def run_plain(self, b: Batch, stream=None) -> None:
        """The plain path: drf_check_protocol once per protocol of the batch."""
        L = lib()
        s = self._stream(stream)
        base_r = b.results.data_ptr()
        base_c = b.counts.data_ptr()
        for i in range(b.count):
            a, e = int(b.code_off[i]), int(b.code_off[i + 1])
            code = b.code[a:e]
            rc = L.drf_check_protocol(self._ctx, _u32p(code), e - a, int(b.nthreads[i]),
                                      ctypes.c_void_p(base_r + 40 * i),
                                      ctypes.c_void_p(base_c + 8 * int(b.phase_off[i])),
                                      int(b.phase_off[i + 1] - b.phase_off[i]), s)
            if rc != OK:
                raise DrfError(rc, "drf_check_protocol")

    def check_sweep(self, proto: Union[str, np.ndarray], n: int, slot: int, first: int, count: int,
                    stream=None) -> List[CheckResult]:
        """drf_check_sweep: result i is that of the protocol with variable
        `slot` bound to first + i (one batch)."""
        import torch
        c = _code(proto)
        plans = (Plan * max(1, count))()
        rc = lib().drf_plan_sweep(_u32p(c), len(c), n, slot, first, count, plans, None)
        if rc != OK:
            raise DrfError(rc, "drf_plan_sweep")
        o = Outputs(list(plans)[:count], self.device)
        rc = lib().drf_check_sweep(self._ctx, _u32p(c), len(c), n, slot, first, count,
                                   ctypes.c_void_p(o.results.data_ptr()), ctypes.c_void_p(o.counts.data_ptr()),
                                   o.total_phases, self._stream(stream))
        if rc != OK:
            raise DrfError(rc, "drf_check_sweep")
        (stream or torch.cuda.current_stream(self.device)).synchronize()
        return o.collect()

    def check_arrays(self, proto: Union[str, np.ndarray], n: int, stream=None) -> List[CheckResult]:
        """drf_check_arrays: one result per shared array the protocol accesses."""
        import torch
        c = _code(proto)
        k = protocol_arrays(c)
        plans = (Plan * k)()
        rc = lib().drf_plan_arrays(_u32p(c), len(c), n, plans, k, None)
        if rc != OK:
            raise DrfError(rc, "drf_plan_arrays")
        o = Outputs(list(plans), self.device)
        rc = lib().drf_check_arrays(self._ctx, _u32p(c), len(c), n, ctypes.c_void_p(o.results.data_ptr()),
                                    ctypes.c_void_p(o.counts.data_ptr()), o.total_phases, self._stream(stream))
        if rc != OK:
            raise DrfError(rc, "drf_check_arrays")
        (stream or torch.cuda.current_stream(self.device)).synchronize()
        return o.collect()

    def graph_class(self, **caps) -> GraphClass:
        """A shape-class graph for statically small batches (drf_graph_create)."""
        return GraphClass(self, **caps)

    def prepare(self, b: Batch, stream=None) -> Prepared:
        """Check `b` once and capture the device work as one hipGraph."""
        return Prepared(self, b, stream)

    def check_batch(self, items: Sequence[Tuple[Union[str, np.ndarray], int]], stream=None) -> List[CheckResult]:
        import torch
        b = Batch(items, self.device)
        self.run_batch(b, stream)
        (stream or torch.cuda.current_stream(self.device)).synchronize()
        return b.collect()

    def check(self, proto: Union[str, np.ndarray], n: int, stream=None) -> CheckResult:
        import torch
        b = Batch([(proto, n)], self.device)
        self.run_plain(b, stream)
        (stream or torch.cuda.current_stream(self.device)).synchronize()
        return b.collect()[0]
