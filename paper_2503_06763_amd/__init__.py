"""Python binding of the SLPF library (libslpf.so, HIP for gfx950).

Argument marshalling only: every step of a parse runs in the library's HIP
kernels.  Device buffers are torch tensors on a ROCm device; their
``data_ptr()`` and the current torch stream are handed to the C ABI
(include/slpf.h).  There is no CPU fallback: if the library is missing the
import of :func:`lib` raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libslpf.so")

SLPF_OK = 0
STATUS = {0: "ok", -1: "invalid argument", -2: "RE syntax error", -3: "infinitely ambiguous RE",
          -4: "automaton too large", -5: "out of memory", -6: "device error",
          -7: "output buffer too small", -8: "internal error"}
E_ARG, E_SYNTAX, E_INF_AMBIG, E_TOO_LARGE, E_NOMEM, E_DEVICE, E_CAPACITY, E_INTERNAL = range(-1, -9, -1)

COMPILE_HOST_ONLY = 1

PARSE_NO_COUNT = 1
PARSE_FORCE_L2 = 2
PARSE_RECOGNIZE = 4
PARSE_COMPACT = 8
PARSE_NEXT_BYTE_ENTRIES = 16
PARSE_EDGE_SHIFT = 32
PARSE_NO_EDGE_SHIFT = 64
PARSE_ALL_DFA_STATES = 128
PARSE_WIDE_COUNT = 256

EXPORTS = ["slpf_compile", "slpf_parser_destroy", "slpf_parser_info_get", "slpf_segment_text",
           "slpf_table_dump", "slpf_forest_bytes", "slpf_parse", "slpf_parse_texts", "slpf_parse_batch", "slpf_tune",
           "slpf_parser_trim",
           "slpf_num_chunks", "slpf_status_str", "slpf_server_create", "slpf_server_destroy",
           "slpf_server_submit", "slpf_server_poll", "slpf_server_result", "slpf_server_release",
           "slpf_server_stats", "slpf_compact_bytes", "slpf_decode_compact", "slpf_get_matches", "slpf_get_children",
           "slpf_parse_noalloc"]


class SlpfError(RuntimeError):
    def __init__(self, status, what="", offset=None):
        super().__init__("%s: %s (%d)%s" % (what, STATUS.get(status, "?"), status,
                                            "" if offset is None else " at offset %d" % offset))
        self.status = status
        self.offset = offset


class CompileOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("max_segments", ctypes.c_uint32), ("max_states", ctypes.c_uint32),
                ("device", ctypes.c_int32)]


class ParserInfo(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint32) for k in (
        "num_segments", "words_per_column", "num_initial", "num_final", "fwd_states", "rev_states",
        "dfa_states", "medfa_states", "rdfa_states", "rmedfa_states", "num_classes", "max_entries",
        "placement", "max_entries_next_byte", "column_unambiguous", "reserved")] + [("table_bytes", ctypes.c_uint64)]


class ParseOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("chunk_bytes", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("trace_dev", ctypes.c_void_p), ("trace_bytes", ctypes.c_uint64),
                ("events", ctypes.POINTER(ctypes.c_void_p)), ("num_events", ctypes.c_uint32),
                ("reserved2", ctypes.c_uint32)]

NUM_PHASE_EVENTS = 6
# scalars of a parse: accepted, trees mod 2^64, count status, trees mod 2^61 - 1
NUM_SCALARS = 4
PHASES = ["reach", "join", "starts", "build", "count"]


class Forest(ctypes.Structure):
    _fields_ = [("columns_dev", ctypes.c_void_p), ("capacity_bytes", ctypes.c_uint64),
                ("scalars_dev", ctypes.c_void_p)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("slots", ctypes.c_uint32),
                ("max_batch_texts", ctypes.c_uint32), ("parse_flags", ctypes.c_uint32),
                ("memory_budget", ctypes.c_uint64), ("device", ctypes.c_int32), ("reserved", ctypes.c_uint32)]


class ServerState(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in ("queued", "in_flight", "busy_slots", "finished_unreleased",
                                               "admitted_bytes", "arena_bytes")]


class Text(ctypes.Structure):
    _fields_ = [("text_dev", ctypes.c_void_p), ("n", ctypes.c_uint64), ("out", Forest)]


class Item(ctypes.Structure):
    _fields_ = [("p", ctypes.c_void_p), ("text_dev", ctypes.c_void_p), ("n", ctypes.c_uint64), ("out", Forest)]


_lib = None


def lib(path: str = LIB_PATH):
    """Load libslpf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libslpf.so not built: run paper_2503_06763_amd/build.py (or __graft_entry__.build())")
    # torch first: its HIP runtime (soname libamdhip64.so.7) is then the one
    # the library binds to, so the process holds a single HIP runtime
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    L.slpf_compile.argtypes = [ctypes.c_char_p, sz, ctypes.POINTER(CompileOpts), ctypes.POINTER(vp),
                               ctypes.POINTER(sz)]
    L.slpf_compile.restype = ctypes.c_int
    L.slpf_parser_destroy.argtypes = [vp]
    L.slpf_parser_destroy.restype = None
    L.slpf_parser_info_get.argtypes = [vp, ctypes.POINTER(ParserInfo)]
    L.slpf_parser_info_get.restype = ctypes.c_int
    L.slpf_segment_text.argtypes = [vp, ctypes.c_uint32, ctypes.c_char_p, sz, ctypes.POINTER(sz)]
    L.slpf_segment_text.restype = ctypes.c_int
    L.slpf_table_dump.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    L.slpf_table_dump.restype = ctypes.c_int
    L.slpf_forest_bytes.argtypes = [vp, ctypes.c_uint64]
    L.slpf_forest_bytes.restype = ctypes.c_uint64
    L.slpf_parse.argtypes = [vp, vp, ctypes.c_uint64, ctypes.POINTER(ParseOpts), ctypes.POINTER(Forest), vp]
    L.slpf_parse.restype = ctypes.c_int
    L.slpf_parse_noalloc.argtypes = [vp, vp, ctypes.c_uint64, ctypes.POINTER(ParseOpts), ctypes.POINTER(Forest), vp]
    L.slpf_parse_noalloc.restype = ctypes.c_int
    L.slpf_parse_texts.argtypes = [vp, ctypes.POINTER(Text), sz, ctypes.POINTER(ParseOpts), vp]
    L.slpf_parse_texts.restype = ctypes.c_int
    L.slpf_parse_batch.argtypes = [ctypes.POINTER(Item), sz, ctypes.POINTER(ParseOpts), vp]
    L.slpf_parse_batch.restype = ctypes.c_int
    L.slpf_tune.argtypes = [vp, ctypes.POINTER(Text), sz, ctypes.c_uint32, ctypes.POINTER(ParseOpts),
                            ctypes.POINTER(ctypes.c_float), vp]
    L.slpf_tune.restype = ctypes.c_int
    L.slpf_parser_trim.argtypes = [vp, vp]
    L.slpf_parser_trim.restype = ctypes.c_int
    L.slpf_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)]
    L.slpf_server_create.restype = ctypes.c_int
    L.slpf_server_destroy.argtypes = [vp]
    L.slpf_server_destroy.restype = None
    L.slpf_server_submit.argtypes = [vp, vp, vp, ctypes.c_uint64, ctypes.c_uint64]
    L.slpf_server_submit.restype = ctypes.c_int
    L.slpf_server_poll.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), sz, ctypes.POINTER(sz)]
    L.slpf_server_poll.restype = ctypes.c_int
    L.slpf_server_result.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(Forest)]
    L.slpf_server_result.restype = ctypes.c_int
    L.slpf_server_release.argtypes = [vp, ctypes.c_uint64]
    L.slpf_server_release.restype = ctypes.c_int
    L.slpf_server_stats.argtypes = [vp, ctypes.POINTER(ServerState)]
    L.slpf_server_stats.restype = ctypes.c_int
    L.slpf_compact_bytes.argtypes = [ctypes.c_uint64]
    L.slpf_compact_bytes.restype = ctypes.c_uint64
    L.slpf_decode_compact.argtypes = [vp, vp, ctypes.c_uint64, vp, vp, vp]
    L.slpf_decode_compact.restype = ctypes.c_int
    L.slpf_get_matches.argtypes = [vp, vp, ctypes.c_uint64, ctypes.c_uint32, vp, ctypes.c_uint64,
                                   ctypes.POINTER(ctypes.c_uint64), vp]
    L.slpf_get_matches.restype = ctypes.c_int
    L.slpf_get_children.argtypes = [vp, vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                                    vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64), vp]
    L.slpf_get_children.restype = ctypes.c_int
    L.slpf_num_chunks.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ParseOpts)]
    L.slpf_num_chunks.restype = ctypes.c_uint64
    L.slpf_status_str.argtypes = [ctypes.c_int]
    L.slpf_status_str.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(st, what, offset=None):
    if st != SLPF_OK:
        raise SlpfError(st, what, offset)


@dataclass
class Info:
    num_segments: int
    words_per_column: int
    num_initial: int
    num_final: int
    fwd_states: int
    rev_states: int
    dfa_states: int
    medfa_states: int
    rdfa_states: int
    rmedfa_states: int
    num_classes: int
    max_entries: int
    placement: int
    max_entries_next_byte: int
    column_unambiguous: int
    reserved: int
    table_bytes: int


class Parser:
    """A compiled RE (slpf_compile); tables live on ``device``."""

    def __init__(self, re, device: int = 0, max_segments: int = 0, max_states: int = 0,
                 host_only: bool = False):
        L = lib()
        b = re.encode("latin1") if isinstance(re, str) else bytes(re)
        o = CompileOpts(ctypes.sizeof(CompileOpts), COMPILE_HOST_ONLY if host_only else 0,
                        max_segments, max_states, device)
        h = ctypes.c_void_p()
        off = ctypes.c_size_t(0)
        st = L.slpf_compile(b, len(b), ctypes.byref(o), ctypes.byref(h), ctypes.byref(off))
        _check(st, "slpf_compile", off.value if st == E_SYNTAX else None)
        self._h = h
        self._L = L
        self.device = device
        self.re = b
        i = ParserInfo()
        _check(L.slpf_parser_info_get(h, ctypes.byref(i)), "slpf_parser_info_get")
        self.info = Info(*[getattr(i, f) for f in Info.__dataclass_fields__])
        self.W = self.info.words_per_column
        self.nseg = self.info.num_segments

    def close(self):
        if getattr(self, "_h", None):
            self._L.slpf_parser_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def segment_text(self, seg: int) -> str:
        need = ctypes.c_size_t(0)
        _check(self._L.slpf_segment_text(self._h, seg, None, 0, ctypes.byref(need)), "slpf_segment_text")
        buf = ctypes.create_string_buffer(need.value + 1)
        _check(self._L.slpf_segment_text(self._h, seg, buf, need.value + 1, None), "slpf_segment_text")
        return buf.value.decode("utf-8")

    @property
    def segments(self):
        return [self.segment_text(i) for i in range(self.nseg)]

    def table(self, direction: int):
        """(sets [states+1, W] uint64, delta [states+1, C] uint32, classmap [256] uint16), host numpy."""
        import numpy as np
        ns = (self.info.fwd_states if direction == 0 else self.info.rev_states) + 1
        sets = np.zeros((ns, self.W), np.uint64)
        delta = np.zeros((ns, self.info.num_classes), np.uint32)
        cm = np.zeros(256, np.uint16)
        _check(self._L.slpf_table_dump(self._h, direction, sets.ctypes.data, delta.ctypes.data, cm.ctypes.data),
               "slpf_table_dump")
        return sets, delta, cm

    def forest_bytes(self, n: int) -> int:
        return int(self._L.slpf_forest_bytes(self._h, n))

    def num_chunks(self, n: int, chunk_bytes: int = 0) -> int:
        o = ParseOpts(ctypes.sizeof(ParseOpts), chunk_bytes, 0, 0, None, 0, None, 0, 0)
        return int(self._L.slpf_num_chunks(self._h, n, ctypes.byref(o)))

    def parse_into(self, text, n: int, columns, scalars, chunk_bytes: int = 0, flags: int = 0,
                   trace=None, stream=None, events=None):
        """Raw slpf_parse on torch device tensors (asynchronous on ``stream``).

        ``events``: optional list of NUM_PHASE_EVENTS torch.cuda.Event(enable_timing=True),
        recorded on the parse stream at the phase boundaries."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(text.device)
        ev = None
        if events is not None:
            for e in events:
                if not e.cuda_event:      # torch creates the HIP event on its first record
                    e.record(stream)
            ev = (ctypes.c_void_p * len(events))(*[e.cuda_event for e in events])
        o = ParseOpts(ctypes.sizeof(ParseOpts), chunk_bytes, flags, 0,
                      trace.data_ptr() if trace is not None else None,
                      trace.numel() * trace.element_size() if trace is not None else 0,
                      ctypes.cast(ev, ctypes.POINTER(ctypes.c_void_p)) if ev is not None else None,
                      len(events) if events is not None else 0, 0)
        f = Forest(columns.data_ptr() if columns is not None else None,
                   columns.numel() * columns.element_size() if columns is not None else 0, scalars.data_ptr())
        st = self._L.slpf_parse(self._h, text.data_ptr() if n else None, n, ctypes.byref(o), ctypes.byref(f),
                                ctypes.c_void_p(stream.cuda_stream))
        _check(st, "slpf_parse")

    def parse_noalloc_into(self, text, n: int, columns, scalars, chunk_bytes: int = 0, flags: int = 0,
                           stream=None):
        """Raw slpf_parse_noalloc (work buffers in the library's device array, no
        allocation) on torch device tensors; asynchronous on ``stream``."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(scalars.device)
        o = ParseOpts(ctypes.sizeof(ParseOpts), chunk_bytes, flags, 0, None, 0, None, 0, 0)
        f = Forest(columns.data_ptr() if columns is not None else None,
                   columns.numel() * columns.element_size() if columns is not None else 0, scalars.data_ptr())
        st = self._L.slpf_parse_noalloc(self._h, text.data_ptr() if n else None, n, ctypes.byref(o),
                                        ctypes.byref(f), ctypes.c_void_p(stream.cuda_stream))
        _check(st, "slpf_parse_noalloc")

    def parse(self, text, chunk_bytes: int = 0, count: bool = True, force_l2: bool = False,
              trace: bool = False, stream=None, events=None, flags: int = 0):
        """Parse a uint8 device tensor; returns (columns [n+1, W] int64 view of uint64 words,
        scalars [4]) on the device, plus the join trace if asked."""
        import torch
        n = text.numel()
        dev = text.device
        cols = torch.empty((n + 1, self.W), dtype=torch.int64, device=dev)
        sc = torch.empty(NUM_SCALARS, dtype=torch.int64, device=dev)
        tr = None
        if trace:
            c = self.num_chunks(n, chunk_bytes)
            tr = torch.zeros((2, c + 1, self.W), dtype=torch.int64, device=dev)
        flags |= (0 if count else PARSE_NO_COUNT) | (PARSE_FORCE_L2 if force_l2 else 0)
        self.parse_into(text, n, cols, sc, chunk_bytes, flags, tr, stream, events)
        return (cols, sc, tr) if trace else (cols, sc)

    def parse_compact(self, text, chunk_bytes: int = 0, count: bool = True, force_l2: bool = False,
                      stream=None, events=None):
        """Parse into the compact SLPF: returns (columns [n+1] int64 view of one uint64 word
        per column over its candidate list, scalars [4]) on the device."""
        import torch
        n = text.numel()
        cols = torch.empty(n + 1, dtype=torch.int64, device=text.device)
        sc = torch.empty(NUM_SCALARS, dtype=torch.int64, device=text.device)
        flags = PARSE_COMPACT | (0 if count else PARSE_NO_COUNT) | (PARSE_FORCE_L2 if force_l2 else 0)
        self.parse_into(text, n, cols, sc, chunk_bytes, flags, None, stream, events)
        return cols, sc

    def matches(self, columns, group: int, capacity: int = 1 << 16, stream=None):
        """Matches of group ``group`` (its number in slpf_segment_text) in the
        plain SLPF ``columns`` [n+1, W] of a parsed text: a host uint64 array
        [k, 2] of (start, end) pairs sorted by (start, end)."""
        import numpy as np
        import torch
        n = columns.shape[0] - 1
        if stream is None:
            stream = torch.cuda.current_stream(columns.device)
        while True:
            out = torch.empty((max(capacity, 1), 2), dtype=torch.int64, device=columns.device)
            cnt = ctypes.c_uint64(0)
            st = self._L.slpf_get_matches(self._h, columns.data_ptr(), n, group, out.data_ptr(), capacity,
                                          ctypes.byref(cnt), ctypes.c_void_p(stream.cuda_stream))
            if st == E_CAPACITY:
                capacity = int(cnt.value)
                continue
            _check(st, "slpf_get_matches")
            return out[:cnt.value].cpu().numpy().view(np.uint64)

    def children(self, columns, group: int, start: int, end: int, capacity: int = 1 << 12, stream=None):
        """Children of the match (start, end) of node ``group`` in the plain
        SLPF ``columns`` [n+1, W]: a host uint64 array [k, 3] of (child, a, b)
        triples sorted by (child, a, b)."""
        import numpy as np
        import torch
        n = columns.shape[0] - 1
        if stream is None:
            stream = torch.cuda.current_stream(columns.device)
        while True:
            out = torch.empty((max(capacity, 1), 3), dtype=torch.int64, device=columns.device)
            cnt = ctypes.c_uint64(0)
            st = self._L.slpf_get_children(self._h, columns.data_ptr(), n, group, start, end, out.data_ptr(),
                                           capacity, ctypes.byref(cnt), ctypes.c_void_p(stream.cuda_stream))
            if st == E_CAPACITY:
                capacity = int(cnt.value)
                continue
            _check(st, "slpf_get_children")
            return out[:cnt.value].cpu().numpy().view(np.uint64)

    def decode_compact(self, text, compact, stream=None):
        """W-word columns [n+1, W] (int64 view) of a compact SLPF of ``text`` (device tensors)."""
        import torch
        n = text.numel()
        out = torch.empty((n + 1, self.W), dtype=torch.int64, device=compact.device)
        if stream is None:
            stream = torch.cuda.current_stream(compact.device)
        st = self._L.slpf_decode_compact(self._h, text.data_ptr() if n else None, n, compact.data_ptr(),
                                         out.data_ptr(), ctypes.c_void_p(stream.cuda_stream))
        _check(st, "slpf_decode_compact")
        return out


    def recognize(self, text, chunk_bytes: int = 0, force_l2: bool = False, stream=None, events=None):
        """Recogniser mode (forward reach and join only): returns the scalars
        tensor [4] on the device (accept, 0, 2, 0); no SLPF is written."""
        import torch
        sc = torch.empty(NUM_SCALARS, dtype=torch.int64, device=text.device)
        flags = PARSE_RECOGNIZE | (PARSE_FORCE_L2 if force_l2 else 0)
        self.parse_into(text, text.numel(), None, sc, chunk_bytes, flags, None, stream, events)
        return sc

    def parse_batch_into(self, items, chunk_bytes: int = 0, flags: int = 0, stream=None, events=None):
        """Raw slpf_parse_texts.  ``items``: list of (text tensor or None, n, columns tensor,
        scalars tensor); asynchronous on ``stream``."""
        import torch
        if stream is None:
            dev = next((t.device for t, _, _, _ in items if t is not None), torch.device("cuda", self.device))
            stream = torch.cuda.current_stream(dev)
        ev = None
        if events is not None:
            for e in events:
                if not e.cuda_event:
                    e.record(stream)
            ev = (ctypes.c_void_p * len(events))(*[e.cuda_event for e in events])
        o = ParseOpts(ctypes.sizeof(ParseOpts), chunk_bytes, flags, 0, None, 0,
                      ctypes.cast(ev, ctypes.POINTER(ctypes.c_void_p)) if ev is not None else None,
                      len(events) if events is not None else 0, 0)
        arr = self._text_array(items)
        st = self._L.slpf_parse_texts(self._h, arr, len(items), ctypes.byref(o), ctypes.c_void_p(stream.cuda_stream))
        _check(st, "slpf_parse_texts")

    def _text_array(self, items):
        arr = (Text * len(items))()
        for k, (t, n, cols, sc) in enumerate(items):
            arr[k].text_dev = t.data_ptr() if (t is not None and n) else None
            arr[k].n = n
            arr[k].out = Forest(cols.data_ptr() if cols is not None else None,
                                cols.numel() * cols.element_size() if cols is not None else 0, sc.data_ptr())
        return arr

    def tune(self, items, count: bool = True, stream=None):
        """slpf_tune over ``items`` (as for parse_batch_into); returns
        (chunk_bytes, flags, ms).  The items' outputs hold a complete parse."""
        import torch
        if stream is None:
            dev = next((t.device for t, _, _, _ in items if t is not None), torch.device("cuda", self.device))
            stream = torch.cuda.current_stream(dev)
        o = ParseOpts(ctypes.sizeof(ParseOpts), 0, 0, 0, None, 0, None, 0, 0)
        ms = ctypes.c_float(0)
        arr = self._text_array(items)
        st = self._L.slpf_tune(self._h, arr, len(items), 0 if count else PARSE_NO_COUNT, ctypes.byref(o),
                               ctypes.byref(ms), ctypes.c_void_p(stream.cuda_stream))
        _check(st, "slpf_tune")
        return int(o.chunk_bytes), int(o.flags), float(ms.value)

    def parse_batch_prepared(self, arr, count: int, chunk_bytes: int, flags: int, stream):
        """slpf_parse_texts on an array made by _text_array (no per-call marshalling)."""
        o = ParseOpts(ctypes.sizeof(ParseOpts), chunk_bytes, flags, 0, None, 0, None, 0, 0)
        st = self._L.slpf_parse_texts(self._h, arr, count, ctypes.byref(o), ctypes.c_void_p(stream.cuda_stream))
        _check(st, "slpf_parse_texts")

    def parse_batch(self, texts, chunk_bytes: int = 0, count: bool = True, force_l2: bool = False,
                    stream=None, events=None):
        """Parse a list of uint8 device tensors in one job; returns a list of
        (columns [n+1, W], scalars [4]) per text.  The columns of all texts are
        views of one allocation, each starting on a 256-byte boundary."""
        import torch
        if not texts:
            return []
        dev = texts[0].device
        W = self.W
        offs, tot = [], 0
        for t in texts:
            offs.append(tot)
            tot += ((t.numel() + 1) * W + 31) // 32 * 32
        big = torch.empty(max(tot, 1), dtype=torch.int64, device=dev)
        sc = torch.empty((len(texts), NUM_SCALARS), dtype=torch.int64, device=dev)
        out, items = [], []
        for k, t in enumerate(texts):
            n = t.numel()
            cols = big[offs[k]:offs[k] + (n + 1) * W].view(n + 1, W)
            out.append((cols, sc[k]))
            items.append((t, n, cols, sc[k]))
        flags = (0 if count else PARSE_NO_COUNT) | (PARSE_FORCE_L2 if force_l2 else 0)
        self.parse_batch_into(items, chunk_bytes, flags, stream, events)
        return out


class Server:
    """slpf_server: continuous batching of parse requests (FIFO admission by
    projected SLPF bytes within ``memory_budget``, ``slots`` jobs in flight).

    The server keeps a reference to every parser submitted to it until it is
    closed (destroying the server releases the parsers' buffers for its
    streams, so they must outlive it), and to each request's text tensor until
    ``poll`` reports the request finished (the GPU reads it until then)."""

    def __init__(self, slots: int = 4, max_batch_texts: int = 256, memory_budget: int = 1 << 30,
                 count: bool = True, device: int = 0, compact: bool = False):
        L = lib()
        flags = (0 if count else PARSE_NO_COUNT) | (PARSE_COMPACT if compact else 0)
        o = ServerOpts(ctypes.sizeof(ServerOpts), slots, max_batch_texts, flags, memory_budget, device, 0)
        self.compact = compact
        h = ctypes.c_void_p()
        _check(L.slpf_server_create(ctypes.byref(o), ctypes.byref(h)), "slpf_server_create")
        self._L, self._h = L, h
        self._buf = (ctypes.c_uint64 * 4096)()
        self._parsers = {}      # handle -> Parser, for the server's lifetime
        self._texts = {}        # tag -> text tensor, until the request finishes

    def close(self):
        if getattr(self, "_h", None):
            self._L.slpf_server_destroy(self._h)
            self._h = None
            self._parsers.clear()
            self._texts.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, parser: Parser, text, n: int, tag: int):
        """Queue a request; ``text`` is a device tensor whose bytes are in place."""
        st = self._L.slpf_server_submit(self._h, parser.handle, text.data_ptr() if n else None, n, tag)
        _check(st, "slpf_server_submit")
        self._parsers[parser.handle.value] = parser
        self._texts[tag] = text

    def poll(self):
        """Advance the server; returns the list of tags finished since the last call."""
        out = []
        while True:
            nd = ctypes.c_size_t(0)
            _check(self._L.slpf_server_poll(self._h, self._buf, len(self._buf), ctypes.byref(nd)),
                   "slpf_server_poll")
            out.extend(self._buf[:nd.value])
            if nd.value < len(self._buf):
                for tag in out:
                    self._texts.pop(tag, None)
                return out

    def result(self, tag: int):
        """(columns_ptr, capacity_bytes, scalars_ptr) of a finished request."""
        f = Forest()
        _check(self._L.slpf_server_result(self._h, tag, ctypes.byref(f)), "slpf_server_result")
        return f.columns_dev, f.capacity_bytes, f.scalars_dev

    def result_tensors(self, tag: int, n: int, W: int, device="cuda:0"):
        """Host copies (columns uint64 [n+1, W], or [n+1] compact words, and
        scalars uint64 [4]) of a finished request."""
        import numpy as np
        import torch
        cp, cap, sp = self.result(tag)
        if self.compact:
            W = 1
        cols = np.empty((n + 1) * W, np.uint64)
        sc = np.empty(NUM_SCALARS, np.uint64)
        torch.cuda.synchronize()
        _hip_copy_to_host(cols.ctypes.data, cp, cols.nbytes)
        _hip_copy_to_host(sc.ctypes.data, sp, sc.nbytes)
        return (cols if self.compact else cols.reshape(n + 1, W)), sc

    def release(self, tag: int):
        _check(self._L.slpf_server_release(self._h, tag), "slpf_server_release")

    def stats(self):
        s = ServerState()
        _check(self._L.slpf_server_stats(self._h, ctypes.byref(s)), "slpf_server_stats")
        return {k: getattr(s, k) for k, _ in ServerState._fields_}


_hip = None


def _hip_copy_to_host(dst, src, nbytes):
    """Synchronous device-to-host copy through the HIP runtime torch loaded."""
    global _hip
    if _hip is None:
        import torch  # noqa: F401  (loads the HIP runtime; the soname resolves to that copy)
        _hip = ctypes.CDLL("libamdhip64.so.7")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    if nbytes:
        st = _hip.hipMemcpy(ctypes.c_void_p(dst), ctypes.c_void_p(src), nbytes, 2)   # device to host
        if st != 0:
            raise SlpfError(E_DEVICE, "hipMemcpy")


def status_str(st: int) -> str:
    return lib().slpf_status_str(st).decode()


def item_array(items):
    """An slpf_item array for parse_items_prepared: ``items`` is a list of
    (Parser, text tensor or None, n, columns tensor, scalars tensor)."""
    arr = (Item * len(items))()
    for k, (p, t, n, cols, sc) in enumerate(items):
        arr[k].p = p.handle.value
        arr[k].text_dev = t.data_ptr() if (t is not None and n) else None
        arr[k].n = n
        arr[k].out = Forest(cols.data_ptr() if cols is not None else None,
                            cols.numel() * cols.element_size() if cols is not None else 0, sc.data_ptr())
    return arr


def parse_items_prepared(arr, count: int, chunk_bytes: int = 0, flags: int = 0, stream=None):
    """slpf_parse_batch (texts of many parsers in one call) on an array from item_array."""
    import torch
    stream = stream or torch.cuda.current_stream()
    o = ParseOpts(ctypes.sizeof(ParseOpts), chunk_bytes, flags, 0, None, 0, None, 0, 0)
    st = lib().slpf_parse_batch(arr, count, ctypes.byref(o), ctypes.c_void_p(stream.cuda_stream))
    _check(st, "slpf_parse_batch")


def parse_items(items, chunk_bytes: int = 0, flags: int = 0, stream=None):
    """slpf_parse_batch: ``items`` as for item_array; asynchronous on ``stream``."""
    parse_items_prepared(item_array(items), len(items), chunk_bytes, flags, stream)
