"""Thin ctypes binding of libbicop.so (include/bicop.h).

Argument marshalling only: every step of the protocols runs in the HIP
kernels behind the C ABI.  Shares are torch tensors on the GPU whose element
size matches the ring (4 bytes for l <= 32, else 8; uint32/int32 or
uint64/int64 storage), contiguous.  Calls enqueue on the current torch
stream unless a stream is given.  If the library is not built, importing
this module raises ImportError: there is no fallback path.
"""

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbicop.so")

BC_OP_DRELU = 0
BC_OP_RELU = 1
BC_OP_RSS_DRELU = 2
BC_OP_RSS_RELU = 3
BC_STATIC_PLAN_BYTES = 65536      # fixed device plan area of bc_batch_run_static
BC_STATIC_MAX_SEGMENTS = 743
BC_RAND_MAGIC = 0x44524342       # bc_rand_desc.magic once bc_rand_expand has filled it
BC_TRUNC_NONE, BC_TRUNC_AFTER, BC_TRUNC_BEFORE = 0, 1, 2
LINKS = ("P0->P2", "P1->P2", "P2->P0", "P2->P1", "P0->P1", "P1->P0")


class BicopError(RuntimeError):
    def __init__(self, code, where, detail):
        super().__init__(f"{where}: error {code} ({detail})")
        self.code = code


class _Params(ctypes.Structure):
    _fields_ = [("ell", ctypes.c_uint32), ("lx", ctypes.c_uint32), ("k_lo", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("p", ctypes.c_uint64)]


class _Seeds(ctypes.Structure):
    _fields_ = [("seed01", ctypes.c_uint64), ("seed02", ctypes.c_uint64), ("seed12", ctypes.c_uint64),
                ("nonce", ctypes.c_uint64)]


class _RssSeeds(ctypes.Structure):
    _fields_ = [("seed01", ctypes.c_uint64), ("seed02", ctypes.c_uint64), ("seed12", ctypes.c_uint64),
                ("nonce", ctypes.c_uint64), ("seed012", ctypes.c_uint64), ("seed2", ctypes.c_uint64)]


class _Acct(ctypes.Structure):
    _fields_ = [("bits", ctypes.c_uint64 * 6), ("stored_bytes", ctypes.c_uint64 * 6), ("rounds", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class _RandDesc(ctypes.Structure):
    _fields_ = [("magic", ctypes.c_uint32), ("op", ctypes.c_uint32), ("prm", _Params), ("n", ctypes.c_uint64),
                ("bytes", ctypes.c_uint64), ("nonce", ctypes.c_uint64), ("elem_base", ctypes.c_uint64)]


class _Segment(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_void_p), ("x1", ctypes.c_void_p), ("y0", ctypes.c_void_p), ("y1", ctypes.c_void_p),
                ("n", ctypes.c_uint64), ("elem_base", ctypes.c_uint64), ("nonce", ctypes.c_uint64),
                ("op", ctypes.c_uint32), ("k_in", ctypes.c_uint32), ("rand", ctypes.c_void_p),
                ("rand_desc", ctypes.POINTER(_RandDesc))]


_P = ctypes.c_void_p
_U64 = ctypes.c_uint64
_U32 = ctypes.c_uint32

_SIGS = {
    "bc_version": ([], ctypes.c_char_p),
    "bc_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "bc_last_error": ([], ctypes.c_char_p),
    "bc_default_prime": ([_U32], _U64),
    "bc_check_params": ([ctypes.POINTER(_Params), ctypes.POINTER(_Params)], ctypes.c_int),
    "bc_msg_account": ([_U32, ctypes.POINTER(_Params), _U64, ctypes.POINTER(_Acct)], ctypes.c_int),
    "bc_keybit_params": ([_U32, _U32, _U32, _U32, ctypes.POINTER(_Params)], ctypes.c_int),
    "bc_zp_mul_add": ([_P, _P, _P, _P, _U64, _U32, _U64, _P], ctypes.c_int),
    "bc_keybit_int_bits": ([_U64, _U32], _U32),
    "bc_prg_blocks": ([_P, _U64, _U32, _U64, _U64, _U32, _U64, _P], ctypes.c_int),
    "bc_trunc_det": ([_P, _P, _P, _P, _U64, _U32, _U32, _U32, _P], ctypes.c_int),
    "bc_trunc_prob": ([_P, _P, _P, _P, _U64, _U32, _U32, _P], ctypes.c_int),
    "bc_mod_switch": ([_P, _P, _P, _P, _U64, _U32, _U64, _P], ctypes.c_int),
    "bc_drelu": ([_P, _P, _P, _P, _U64, ctypes.POINTER(_Params), ctypes.POINTER(_Seeds), _U64, _P,
                  ctypes.POINTER(_Acct), _P], ctypes.c_int),
    "bc_relu": ([_P, _P, _P, _P, _U64, ctypes.POINTER(_Params), ctypes.POINTER(_Seeds), _U64, _P,
                 ctypes.POINTER(_Acct), _P], ctypes.c_int),
    "bc_msg_words": ([_U32], _U32),
    "bc_drelu_send": ([_U32, _P, _P, _U64, ctypes.POINTER(_Params), ctypes.POINTER(_Seeds), _U64, _P], ctypes.c_int),
    "bc_drelu_reply": ([_P, _P, _P, _P, _U64, ctypes.POINTER(_Params), ctypes.POINTER(_Seeds), _U64, _P],
                       ctypes.c_int),
    "bc_drelu_finish": ([_U32, _P, _P, _U64, ctypes.POINTER(_Params), ctypes.POINTER(_Seeds), _U64, _P],
                        ctypes.c_int),
    "bc_mul_trunc": ([_P, _P, _P, _P, _P, _P, _U64, _U32, _U32, _U32, ctypes.POINTER(_Seeds), _U64, _P], ctypes.c_int),
    "bc_rss_drelu": ([_P, _P, _P, _P, _P, _P, _U64, ctypes.POINTER(_Params), ctypes.POINTER(_RssSeeds), _U64, _P,
                      ctypes.POINTER(_Acct), _P], ctypes.c_int),
    "bc_rss_relu": ([_P, _P, _P, _P, _P, _P, _U64, ctypes.POINTER(_Params), ctypes.POINTER(_RssSeeds), _U64, _P,
                     ctypes.POINTER(_Acct), _P], ctypes.c_int),
    "bc_batch_plan_bytes": ([_U32], _U64),
    "bc_batch_plan": ([ctypes.POINTER(_Segment), _U32, ctypes.POINTER(_Params), _U32, _P, _U64], ctypes.c_int),
    "bc_batch_run": ([_P, _P, ctypes.POINTER(_Seeds), _U32, _P], ctypes.c_int),
    "bc_batch_run_static": ([_P, ctypes.POINTER(_Seeds), _U32, _P], ctypes.c_int),
    "bc_rand_bytes": ([_U32, ctypes.POINTER(_Params), _U64], _U64),
    "bc_rand_expand": ([_P, _U64, _U64, _U32, ctypes.POINTER(_Params), ctypes.POINTER(_Seeds), _U64,
                        ctypes.POINTER(_RandDesc), _P], ctypes.c_int),
    "bc_drelu_pre": ([_P, _P, _P, _P, _U64, ctypes.POINTER(_Params), ctypes.POINTER(_Seeds), _U64, _P,
                      ctypes.POINTER(_RandDesc), _P, ctypes.POINTER(_Acct), _P], ctypes.c_int),
    "bc_relu_pre": ([_P, _P, _P, _P, _U64, ctypes.POINTER(_Params), ctypes.POINTER(_Seeds), _U64, _P,
                     ctypes.POINTER(_RandDesc), _P, ctypes.POINTER(_Acct), _P], ctypes.c_int),
    "bc_trunc_drelu": ([_P, _P, _P, _P, _U64, _U32, _U32, ctypes.POINTER(_Params), ctypes.POINTER(_Seeds), _U64, _P,
                        ctypes.POINTER(_Acct), _P], ctypes.c_int),
    "bc_trunc_relu": ([_P, _P, _P, _P, _U64, _U32, _U32, ctypes.POINTER(_Params), ctypes.POINTER(_Seeds), _U64, _P,
                       ctypes.POINTER(_Acct), _P], ctypes.c_int),
    "bc_set_schedule": ([_U32, _U32, _U32, _U32, _U32], ctypes.c_int),
    "bc_get_schedule": ([_U32, _U32, _U32, _U32], _U32),
}

EXPORTED = tuple(_SIGS)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "or python -m paper_2309_04909_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()

SCHED_KINDS = {"fused": 0, "stream": 1, "pre": 2, "expand": 3, "batch": 4, "group": 5, "group_fill": 6}
SCHED_ALL = 0xFFFFFFFF
SCHEDULES_PATH = os.path.join(_HERE, "schedules.json")


def set_schedule(kind: str, npos: int, blocks_per_cu: int, width=None, op=None):
    """Schedule of (kind, npos, storage width 4/8, op BC_OP_DRELU/BC_OP_RELU);
    width or op None sets every width / op."""
    _check(lib.bc_set_schedule(SCHED_KINDS[kind], npos, SCHED_ALL if width is None else width,
                               SCHED_ALL if op is None else op, blocks_per_cu), "set_schedule")


def get_schedule(kind: str, npos: int, width: int = 8, op: int = BC_OP_DRELU) -> int:
    return int(lib.bc_get_schedule(SCHED_KINDS[kind], npos, width, op))


def schedule_key(e):
    """The table key of a schedules.json entry: (kind, npos, width, op)."""
    return (e["kind"], int(e["npos"]), e.get("width"), e.get("op"))


def load_schedules(path=SCHEDULES_PATH):
    """Apply an autotuned schedule table (written by paper_2309_04909_amd.tune).
    Entries are keyed by (kind, npos, width, op); a key that appears twice is
    an error, so two settings can never overwrite each other's schedule."""
    import json
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        table = json.load(f)
    seen = set()
    for e in table.get("grid", []):
        k = schedule_key(e)
        if k in seen:
            raise ValueError(f"{path}: schedule {k} listed twice")
        seen.add(k)
    # wildcard entries first, so that a specific entry of the same kind and npos wins
    for e in sorted(table.get("grid", []), key=lambda e: (e.get("width") is not None) + (e.get("op") is not None)):
        set_schedule(e["kind"], int(e["npos"]), int(e["blocks_per_cu"]), e.get("width"), e.get("op"))
    return table


def _check(rc, where):
    if rc != 0:
        raise BicopError(rc, where, f"{lib.bc_strerror(rc).decode()}: {lib.bc_last_error().decode()}")


# ------------------------------------------------------------------ settings


@dataclass(frozen=True)
class Params:
    """DReLU/ReLU setting: ring bits ell, window width lx, key-bit offset k_lo,
    prime p (0 = largest prime below 2^(lx+1))."""
    ell: int
    lx: int
    k_lo: int = 0
    p: int = 0

    def c(self):
        # the ctypes struct is built once per (immutable) setting
        s = self.__dict__.get("_c")
        if s is None:
            s = self.__dict__["_c"] = _Params(self.ell, self.lx, self.k_lo, 0, self.p)
        return s

    @property
    def npos(self):
        return self.lx + 1

    def resolved(self):
        out = _Params()
        _check(lib.bc_check_params(ctypes.byref(self.c()), ctypes.byref(out)), "check_params")
        return Params(out.ell, out.lx, out.k_lo, out.p)


@dataclass(frozen=True)
class Seeds:
    seed01: int
    seed02: int
    seed12: int
    nonce: int = 0

    def c(self):
        s = self.__dict__.get("_c")
        if s is None:
            m = (1 << 64) - 1
            s = self.__dict__["_c"] = _Seeds(self.seed01 & m, self.seed02 & m, self.seed12 & m, self.nonce & m)
        return s


@dataclass(frozen=True)
class RssSeeds:
    """Seeds of the replicated-sharing calls: those of Seeds, plus seed012
    (all three parties) and seed2 (P2 alone)."""
    seed01: int
    seed02: int
    seed12: int
    seed012: int
    seed2: int
    nonce: int = 0

    def c(self):
        s = self.__dict__.get("_c")
        if s is None:
            m = (1 << 64) - 1
            s = self.__dict__["_c"] = _RssSeeds(self.seed01 & m, self.seed02 & m, self.seed12 & m, self.nonce & m,
                                                self.seed012 & m, self.seed2 & m)
        return s


def version():
    return lib.bc_version().decode()


def default_prime(lx):
    return int(lib.bc_default_prime(lx))


def msg_account(op, params: Params, n):
    a = _Acct()
    _check(lib.bc_msg_account(op, ctypes.byref(params.c()), n, ctypes.byref(a)), "msg_account")
    return {"bits": dict(zip(LINKS, list(a.bits))), "stored_bytes": dict(zip(LINKS, list(a.stored_bytes))),
            "rounds": a.rounds}


def keybit_params(ell, f, int_bits, frac_bits) -> "Params":
    """Key-bit window (Sec. 6.1): k_lo = f - frac_bits, l_x = int_bits + frac_bits, default p."""
    out = _Params()
    _check(lib.bc_keybit_params(ell, f, int_bits, frac_bits, ctypes.byref(out)), "keybit_params")
    return Params(out.ell, out.lx, out.k_lo, out.p)


def keybit_int_bits(bound, f) -> int:
    """Integer bits (guard bit included) of the key-bit window for |x| < bound at f fractional bits."""
    return int(lib.bc_keybit_int_bits(bound, f))


# ------------------------------------------------------------------- helpers


def ring_width(ell):
    return 4 if ell <= 32 else 8


def ring_dtype(ell):
    return torch.uint32 if ell <= 32 else torch.uint64


def field_dtype(p):
    return torch.uint32 if p < (1 << 32) else torch.uint64


_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream(stream, like=None):
    """The HIP stream handle to enqueue on: `stream`, else torch's current
    stream of the device of `like` (or of the current device)."""
    if stream is not None:
        return stream.cuda_stream
    dev = like.get_device() if like is not None else torch.cuda.current_device()
    if _raw_stream is not None:
        return _raw_stream(dev)
    return torch.cuda.current_stream(dev).cuda_stream


def _check_shares(x0, x1, width, what="shares"):
    for t in (x0, x1):
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{what} must be CUDA tensors")
        if t.element_size() != width:
            raise TypeError(f"{what}: expected {width}-byte elements, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{what} must be contiguous")
    if x0.numel() != x1.numel():
        raise ValueError("share arrays differ in length")


def _out(x, like_width, dtype, out):
    if out is not None:
        if out.numel() != x.numel() or out.element_size() != like_width or not out.is_contiguous():
            raise ValueError("bad output tensor")
        return out
    return torch.empty(x.shape, dtype=dtype, device=x.device)


# ------------------------------------------------------------------ protocols


def trunc_det(x0, x1, ell, k1, k2=0, out=None, stream=None):
    """Alg. 4/5: shares of Z_{2^ell} -> shares of Z_{2^(ell-k1-k2)}."""
    _check_shares(x0, x1, ring_width(ell))
    m = ell - k1 - k2
    y0 = _out(x0, ring_width(m), ring_dtype(m), None if out is None else out[0])
    y1 = _out(x1, ring_width(m), ring_dtype(m), None if out is None else out[1])
    _check(lib.bc_trunc_det(x0.data_ptr(), x1.data_ptr(), y0.data_ptr(), y1.data_ptr(), x0.numel(), ell, k1, k2,
                            _stream(stream, x0)), "trunc_det")
    return y0, y1


def trunc_prob(x0, x1, ell, k, out=None, stream=None):
    """Alg. 1: shares of Z_{2^ell} -> shares of Z_{2^ell}."""
    _check_shares(x0, x1, ring_width(ell))
    y0 = _out(x0, ring_width(ell), ring_dtype(ell), None if out is None else out[0])
    y1 = _out(x1, ring_width(ell), ring_dtype(ell), None if out is None else out[1])
    _check(lib.bc_trunc_prob(x0.data_ptr(), x1.data_ptr(), y0.data_ptr(), y1.data_ptr(), x0.numel(), ell, k,
                             _stream(stream, x0)), "trunc_prob")
    return y0, y1


def mod_switch(x0, x1, ell_in, p, out=None, stream=None):
    """Alg. 6: shares of Z_{2^ell_in} -> shares of Z_p."""
    _check_shares(x0, x1, ring_width(ell_in))
    w = 4 if p < (1 << 32) else 8
    y0 = _out(x0, w, field_dtype(p), None if out is None else out[0])
    y1 = _out(x1, w, field_dtype(p), None if out is None else out[1])
    _check(lib.bc_mod_switch(x0.data_ptr(), x1.data_ptr(), y0.data_ptr(), y1.data_ptr(), x0.numel(), ell_in, p,
                             _stream(stream, x0)), "mod_switch")
    return y0, y1


def _drelu_like(fn, name, x0, x1, params, seeds, elem_base, capture, out, stream):
    _check_shares(x0, x1, ring_width(params.ell))
    y0 = _out(x0, ring_width(params.ell), ring_dtype(params.ell), None if out is None else out[0])
    y1 = _out(x1, ring_width(params.ell), ring_dtype(params.ell), None if out is None else out[1])
    cap = None
    if capture:
        p = params.resolved().p
        cap = torch.empty((2, x0.numel(), params.npos), dtype=field_dtype(p), device=x0.device)
    _check(fn(x0.data_ptr(), x1.data_ptr(), y0.data_ptr(), y1.data_ptr(), x0.numel(), ctypes.byref(params.c()),
              ctypes.byref(seeds.c()), elem_base, None if cap is None else cap.data_ptr(), None,
              _stream(stream, x0)), name)
    if capture:
        return y0, y1, cap
    return y0, y1


def drelu(x0, x1, params: Params, seeds: Seeds, elem_base=0, capture=False, out=None, stream=None):
    """Alg. 7.  Returns (y0, y1) or (y0, y1, capture[2, n, lx+1])."""
    return _drelu_like(lib.bc_drelu, "drelu", x0, x1, params, seeds, elem_base, capture, out, stream)


def relu(x0, x1, params: Params, seeds: Seeds, elem_base=0, capture=False, out=None, stream=None):
    """Alg. 8.  Returns (y0, y1) or (y0, y1, capture[2, n, lx+1])."""
    return _drelu_like(lib.bc_relu, "relu", x0, x1, params, seeds, elem_base, capture, out, stream)


def msg_words(npos):
    """32-bit words per element of one party's packed round-1 message."""
    return int(lib.bc_msg_words(npos))


def _check_one(t, width, what):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA tensor")
    if t.element_size() != width or not t.is_contiguous():
        raise TypeError(f"{what}: expected contiguous {width}-byte elements")


def drelu_send(party, x, params: Params, seeds: Seeds, elem_base=0, out=None, stream=None):
    """P0's (party 0) or P1's (party 1) round-1 message, from its own share x,
    bit-packed: an int32 tensor [msg_words(lx + 1), n], word-major."""
    _check_one(x, ring_width(params.ell), "share")
    shape = (msg_words(params.npos), x.numel())
    msg = out if out is not None else torch.empty(shape, dtype=torch.int32, device=x.device)
    if tuple(msg.shape) != shape or msg.element_size() != 4 or not msg.is_contiguous():
        raise ValueError("bad message tensor")
    _check(lib.bc_drelu_send(party, x.data_ptr(), msg.data_ptr(), x.numel(), ctypes.byref(params.c()),
                             ctypes.byref(seeds.c()), elem_base, _stream(stream, x)), "drelu_send")
    return msg


def drelu_reply(msg0, msg1, params: Params, seeds: Seeds, elem_base=0, out=None, stream=None):
    """P2: the zero test on both packed messages; returns its reply shares (d0, d1)."""
    n = msg0.shape[1]
    if msg0.shape != msg1.shape or msg0.shape[0] != msg_words(params.npos):
        raise ValueError("message tensors do not match the setting")
    _check_one(msg0, 4, "message")
    _check_one(msg1, 4, "message")
    d0 = _out(msg0[0], ring_width(params.ell), ring_dtype(params.ell), None if out is None else out[0])
    d1 = _out(msg0[0], ring_width(params.ell), ring_dtype(params.ell), None if out is None else out[1])
    _check(lib.bc_drelu_reply(msg0.data_ptr(), msg1.data_ptr(), d0.data_ptr(), d1.data_ptr(), n,
                              ctypes.byref(params.c()), ctypes.byref(seeds.c()), elem_base, _stream(stream, msg0)),
           "drelu_reply")
    return d0, d1


def drelu_finish(party, d, params: Params, seeds: Seeds, elem_base=0, out=None, stream=None):
    """P0's or P1's unflip of its reply share."""
    _check_one(d, ring_width(params.ell), "reply share")
    y = _out(d, ring_width(params.ell), ring_dtype(params.ell), out)
    _check(lib.bc_drelu_finish(party, d.data_ptr(), y.data_ptr(), d.numel(), ctypes.byref(params.c()),
                               ctypes.byref(seeds.c()), elem_base, _stream(stream, d)), "drelu_finish")
    return y


def mul_trunc(x0, x1, y0, y1, ell, f, order, seeds: Seeds, elem_base=0, out=None, stream=None):
    """Elementwise product of shares with Alg. 1 truncation: order BC_TRUNC_BEFORE
    is Alg. linear (factors by floor(f/2) and ceil(f/2) bits first),
    BC_TRUNC_AFTER truncates the product by f, BC_TRUNC_NONE (f = 0) is the
    plain product.  Returns (z0, z1) in Z_{2^ell}."""
    w = ring_width(ell)
    _check_shares(x0, x1, w)
    _check_shares(y0, y1, w)
    if y0.numel() != x0.numel():
        raise ValueError("x and y differ in length")
    z0 = _out(x0, w, ring_dtype(ell), None if out is None else out[0])
    z1 = _out(x1, w, ring_dtype(ell), None if out is None else out[1])
    _check(lib.bc_mul_trunc(x0.data_ptr(), x1.data_ptr(), y0.data_ptr(), y1.data_ptr(), z0.data_ptr(), z1.data_ptr(),
                            x0.numel(), ell, f, order, ctypes.byref(seeds.c()), elem_base, _stream(stream, x0)),
           "mul_trunc")
    return z0, z1


def _rss_like(fn, name, x, params, seeds, elem_base, capture, out, stream):
    if len(x) != 3:
        raise ValueError("replicated sharing takes three share arrays")
    w = ring_width(params.ell)
    _check_shares(x[0], x[1], w)
    _check_shares(x[1], x[2], w)
    y = [_out(x[j], w, ring_dtype(params.ell), None if out is None else out[j]) for j in range(3)]
    cap = None
    if capture:
        cap = torch.empty((2, x[0].numel(), params.npos), dtype=field_dtype(params.resolved().p), device=x[0].device)
    _check(fn(x[0].data_ptr(), x[1].data_ptr(), x[2].data_ptr(), y[0].data_ptr(), y[1].data_ptr(), y[2].data_ptr(),
              x[0].numel(), ctypes.byref(params.c()), ctypes.byref(seeds.c()), elem_base,
              None if cap is None else cap.data_ptr(), None, _stream(stream, x[0])), name)
    return (tuple(y), cap) if capture else tuple(y)


def rss_drelu(x, params: Params, seeds: RssSeeds, elem_base=0, capture=False, out=None, stream=None):
    """Alg. drelu2 on replicated shares x = (x0, x1, x2).  Returns (y0, y1, y2),
    or ((y0, y1, y2), capture[2, n, lx+1])."""
    return _rss_like(lib.bc_rss_drelu, "rss_drelu", x, params, seeds, elem_base, capture, out, stream)


def rss_relu(x, params: Params, seeds: RssSeeds, elem_base=0, capture=False, out=None, stream=None):
    """RSS ReLU (appendix) on replicated shares x = (x0, x1, x2)."""
    return _rss_like(lib.bc_rss_relu, "rss_relu", x, params, seeds, elem_base, capture, out, stream)


def _trunc_like(fn, name, x0, x1, ell_in, k1, params, seeds, elem_base, capture, out, stream):
    _check_shares(x0, x1, ring_width(ell_in))
    y0 = _out(x0, ring_width(params.ell), ring_dtype(params.ell), None if out is None else out[0])
    y1 = _out(x1, ring_width(params.ell), ring_dtype(params.ell), None if out is None else out[1])
    cap = None
    if capture:
        cap = torch.empty((2, x0.numel(), params.npos), dtype=field_dtype(params.resolved().p), device=x0.device)
    _check(fn(x0.data_ptr(), x1.data_ptr(), y0.data_ptr(), y1.data_ptr(), x0.numel(), ell_in, k1,
              ctypes.byref(params.c()), ctypes.byref(seeds.c()), elem_base, None if cap is None else cap.data_ptr(),
              None, _stream(stream, x0)), name)
    return (y0, y1, cap) if capture else (y0, y1)


def trunc_drelu(x0, x1, ell_in, k1, params: Params, seeds: Seeds, elem_base=0, capture=False, out=None, stream=None):
    """Alg. 5 by k1 bits (Z_{2^ell_in} -> Z_{2^params.ell}) fused with Alg. 7."""
    return _trunc_like(lib.bc_trunc_drelu, "trunc_drelu", x0, x1, ell_in, k1, params, seeds, elem_base, capture,
                       out, stream)


def trunc_relu(x0, x1, ell_in, k1, params: Params, seeds: Seeds, elem_base=0, capture=False, out=None, stream=None):
    """Alg. 5 by k1 bits (Z_{2^ell_in} -> Z_{2^params.ell}) fused with Alg. 8."""
    return _trunc_like(lib.bc_trunc_relu, "trunc_relu", x0, x1, ell_in, k1, params, seeds, elem_base, capture,
                       out, stream)


def prg_blocks(n, nblocks, seed, nonce, tag, elem_base=0, device="cuda", stream=None):
    """Raw Philox4x32-10 words, shape (n, nblocks, 4), uint32."""
    out = torch.empty((n, nblocks, 4), dtype=torch.uint32, device=device)
    m = (1 << 64) - 1
    _check(lib.bc_prg_blocks(out.data_ptr(), n, nblocks, seed & m, nonce & m, tag, elem_base, _stream(stream)),
           "prg_blocks")
    return out


# ------------------------------------------------- precomputed randomness


def zp_mul_add(a, b, d, lx, p=0, out=None, stream=None):
    """(a b + d) mod p elementwise with the kernels' field arithmetic (int64 CUDA tensors)."""
    for t in (a, b, d):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.element_size() != 8 or not t.is_contiguous():
            raise TypeError("a, b, d must be contiguous 8-byte CUDA tensors")
    if not (a.numel() == b.numel() == d.numel()):
        raise ValueError("a, b, d differ in length")
    out = _out(a, 8, torch.int64, out)
    _check(lib.bc_zp_mul_add(a.data_ptr(), b.data_ptr(), d.data_ptr(), out.data_ptr(), a.numel(), lx, p,
                             _stream(stream, a)), "zp_mul_add")
    return out


def rand_bytes(op, params: Params, n):
    return int(lib.bc_rand_bytes(op, ctypes.byref(params.c()), n))


def rand_expand(op, params: Params, seeds: Seeds, n, elem_base=0, out=None, device="cuda", stream=None):
    """Offline phase: the seeds' draws for n elements, as a device byte buffer.
    The record's description (bc_rand_desc) rides on the buffer as
    `bicop_desc`, and the seeds and element offset of the expansion as
    `bicop_seeds` and `bicop_elem_base`; the online calls and batch segments
    pass them to the library, which refuses a record of another op, setting,
    n, nonce or offset."""
    nb = rand_bytes(op, params, n)
    if nb == 0 and n:
        _check(lib.bc_check_params(ctypes.byref(params.c()), None), "rand_expand")
    buf = out if out is not None else torch.empty(max(nb, 1), dtype=torch.uint8, device=device)
    desc = _RandDesc()
    _check(lib.bc_rand_expand(buf.data_ptr(), buf.numel(), n, op, ctypes.byref(params.c()), ctypes.byref(seeds.c()),
                              elem_base, ctypes.byref(desc), _stream(stream, buf)), "rand_expand")
    buf.bicop_desc = desc
    buf.bicop_seeds = seeds
    buf.bicop_elem_base = elem_base
    return buf


def rand_desc(rand):
    """The description bc_rand_expand gave the record `rand`."""
    desc = getattr(rand, "bicop_desc", None)
    if desc is None:
        raise ValueError("the record has no description: make it with rand_expand")
    return desc


def _pre_like(fn, name, x0, x1, params, rand, capture, out, stream, seeds=None, elem_base=None):
    _check_shares(x0, x1, ring_width(params.ell))
    y0 = _out(x0, ring_width(params.ell), ring_dtype(params.ell), None if out is None else out[0])
    y1 = _out(x1, ring_width(params.ell), ring_dtype(params.ell), None if out is None else out[1])
    cap = None
    if capture:
        cap = torch.empty((2, x0.numel(), params.npos), dtype=field_dtype(params.resolved().p), device=x0.device)
    seeds = seeds if seeds is not None else getattr(rand, "bicop_seeds", None)
    if seeds is None:
        raise ValueError("the online call needs the seeds the record was expanded with")
    elem_base = elem_base if elem_base is not None else getattr(rand, "bicop_elem_base", 0)
    _check(fn(x0.data_ptr(), x1.data_ptr(), y0.data_ptr(), y1.data_ptr(), x0.numel(), ctypes.byref(params.c()),
              ctypes.byref(seeds.c()), elem_base, rand.data_ptr(), ctypes.byref(rand_desc(rand)),
              None if cap is None else cap.data_ptr(), None, _stream(stream, x0)), name)
    return (y0, y1, cap) if capture else (y0, y1)


def drelu_pre(x0, x1, params: Params, rand, capture=False, out=None, stream=None, seeds=None, elem_base=None):
    """Online Alg. 7 from a record made by rand_expand(BC_OP_DRELU, ...); the
    seeds and offset default to those of the expansion."""
    return _pre_like(lib.bc_drelu_pre, "drelu_pre", x0, x1, params, rand, capture, out, stream, seeds, elem_base)


def relu_pre(x0, x1, params: Params, rand, capture=False, out=None, stream=None, seeds=None, elem_base=None):
    """Online Alg. 8 from a record made by rand_expand(BC_OP_RELU, ...); the
    seeds and offset default to those of the expansion."""
    return _pre_like(lib.bc_relu_pre, "relu_pre", x0, x1, params, rand, capture, out, stream, seeds, elem_base)


# The autotuned schedule table, applied once the whole binding is defined.
SCHEDULES = load_schedules()
