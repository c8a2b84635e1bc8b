"""The C ABI on the CPU: the library loads, exports every function that
include/bicop.h declares, and its host-only logic (prime choice, parameter
validation, message accounting) agrees with the oracle.  No kernel runs here."""

import ctypes
import os
import re

import numpy as np
import pytest

from oracle import params as OP
from oracle import protocols as OPR

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "bicop.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bc_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2309_04909_amd import bicop as B
    lib = ctypes.CDLL(B.LIB_PATH)
    names = _declared()
    assert "bc_drelu" in names and "bc_relu" in names and "bc_trunc_det" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(B.EXPORTED)


@pytest.mark.parametrize("lx", range(1, 33))
def test_default_prime_matches_oracle(lx):
    from paper_2309_04909_amd import bicop as B
    assert B.default_prime(lx) == OP.default_prime(lx)


def test_default_prime_out_of_range():
    from paper_2309_04909_amd import bicop as B
    assert B.default_prime(0) == 0 and B.default_prime(33) == 0


CASES_OK = [(64, 7, 11, 0), (64, 18, 13, 0), (64, 32, 0, 0), (51, 11, 13, 0), (24, 7, 10, 0), (32, 8, 8, 509),
            (2, 1, 0, 3)]
CASES_BAD = [((65, 7, 0, 0), -2), ((0, 1, 0, 0), -2), ((64, 0, 0, 0), -3), ((64, 33, 0, 0), -3),
             ((64, 18, 29, 0), -3), ((64, 7, 0, 257), -4), ((64, 7, 0, 255), -4), ((64, 7, 0, 509), -4)]


def test_check_params_accepts_and_resolves():
    from paper_2309_04909_amd import bicop as B
    for ell, lx, k, p in CASES_OK:
        r = B.Params(ell, lx, k, p).resolved()
        assert r.p == (p or OP.default_prime(lx))
        OP.check_drelu(ell, lx, k, r.p)          # the oracle accepts the same setting


def test_check_params_rejects_like_oracle():
    from paper_2309_04909_amd import bicop as B
    for (ell, lx, k, p), code in CASES_BAD:
        with pytest.raises(B.BicopError) as ei:
            B.Params(ell, lx, k, p).resolved()
        assert ei.value.code == code
        with pytest.raises(ValueError):
            OP.check_drelu(ell, lx, k, p or (OP.default_prime(lx) if 1 <= lx <= 32 else 3))


@pytest.mark.parametrize("op", ["drelu", "relu", "rss_drelu", "rss_relu"])
@pytest.mark.parametrize("ell,lx,k", [(64, 7, 11), (64, 18, 13), (64, 31, 0), (64, 32, 0), (24, 7, 10)])
def test_msg_account_matches_oracle(op, ell, lx, k):
    from paper_2309_04909_amd import bicop as B
    n = 1000
    code = {"drelu": B.BC_OP_DRELU, "relu": B.BC_OP_RELU, "rss_drelu": B.BC_OP_RSS_DRELU,
            "rss_relu": B.BC_OP_RSS_RELU}[op]
    a = B.msg_account(code, B.Params(ell, lx, k), n)
    bits, rounds = OPR.msg_bits(op, ell, lx, OP.default_prime(lx))
    assert [a["bits"][l] for l in B.LINKS] == [b * n for b in bits]
    assert a["rounds"] == rounds
    wbytes = 4 if OP.default_prime(lx) < (1 << 32) else 8
    assert a["stored_bytes"]["P1->P2"] == (lx + 1) * wbytes * n
    rbytes = 4 if ell <= 32 else 8
    for link in B.LINKS[2:]:
        assert a["stored_bytes"][link] * ell == a["bits"][link] * rbytes


def test_tab1_row_through_the_abi():
    from paper_2309_04909_amd import bicop as B
    a = B.msg_account(B.BC_OP_DRELU, B.Params(64, 7, 11), 1)
    assert a["bits"]["P0->P2"] == 64 and a["rounds"] == 2


def test_error_paths_without_gpu():
    """Invalid arguments are rejected on the host before any GPU work.  Every call
    here fails validation (or has n = 0), so nothing is launched even where a GPU is present."""
    from paper_2309_04909_amd import bicop as B
    L = B.lib
    assert L.bc_trunc_det(None, None, None, None, 10, 65, 1, 0, None) == -2
    assert L.bc_trunc_det(None, None, None, None, 10, 64, 40, 24, None) == -2
    assert L.bc_trunc_det(None, None, None, None, 10, 64, 13, 0, None) == -1
    assert L.bc_trunc_det(None, None, None, None, 0, 64, 13, 0, None) == 0
    assert L.bc_trunc_prob(None, None, None, None, 10, 64, 64, None) == -2
    assert L.bc_mod_switch(None, None, None, None, 10, 7, 256, None) == -4
    assert L.bc_mod_switch(None, None, None, None, 10, 7, 251, None) == -1
    assert L.bc_mod_switch(None, None, None, None, 10, 64, 3, None) == -2
    assert L.bc_prg_blocks(None, 10, 0, 1, 2, 3, 0, None) == -8
    assert L.bc_prg_blocks(None, 10, 1, 1, 2, 256, 0, None) == -8
    prm = B.Params(64, 7, 11).c()
    sd = B.Seeds(1, 2, 3).c()
    assert L.bc_drelu(None, None, None, None, 10, ctypes.byref(prm), None, 0, None, None, None) == -1
    assert L.bc_drelu(None, None, None, None, 10, ctypes.byref(prm), ctypes.byref(sd), 0, None, None, None) == -1
    assert L.bc_drelu(None, None, None, None, 10, ctypes.byref(prm), ctypes.byref(sd), (1 << 48) - 5, None, None,
                      None) == -8
    assert L.bc_relu(None, None, None, None, 0, ctypes.byref(prm), ctypes.byref(sd), 0, None, None, None) == 0
    L.bc_drelu(None, None, None, None, 10, ctypes.byref(prm), ctypes.byref(sd), 1 << 48, None, None, None)
    assert "2^48" in B.lib.bc_last_error().decode()
    bad = B.Params(64, 7, 0, 0).c()
    bad.reserved = 1
    assert L.bc_drelu(None, None, None, None, 1, ctypes.byref(bad), ctypes.byref(sd), 0, None, None, None) == -8
    # the diagnostic field multiply-add validates its setting like the protocol calls
    assert L.bc_zp_mul_add(None, None, None, None, 10, 0, 0, None) == -3            # l_x = 0
    assert L.bc_zp_mul_add(None, None, None, None, 10, 33, 0, None) == -3           # l_x > 32
    assert L.bc_zp_mul_add(None, None, None, None, 10, 7, 255, None) == -4          # not prime
    assert L.bc_zp_mul_add(None, None, None, None, 10, 7, 0, None) == -1            # NULL arrays
    assert L.bc_zp_mul_add(None, None, None, None, 0, 7, 0, None) == 0              # n = 0
    assert L.bc_zp_mul_add(None, None, None, None, (1 << 48) + 1, 7, 0, None) == -8  # n above 2^48


def _record_bytes(npos, relu, width, n):
    """A record's size written out from its layout: one key index byte per
    window position (a whole 32-bit word per four), the 2 npos masks r and
    reshares z of npos bits packed floor(64 / npos) to a 64-bit word, and for
    the ReLU P2's share [c]_1 of the triple's product; each section starts on a
    256-byte boundary."""
    def up(b):
        return (b + 255) // 256 * 256
    per_word = 64 // npos
    words = 2 * npos if npos >= 33 else -(-2 * npos // per_word)
    return up(up(4 * -(-npos // 4) * n) + 8 * words * n) + (width * n if relu else 0)


@pytest.mark.parametrize("op,ell,lx,k_lo", [(0, 64, 7, 11), (1, 64, 7, 11), (0, 64, 18, 13), (1, 64, 18, 13),
                                            (1, 32, 8, 8), (0, 64, 32, 0), (1, 64, 32, 0), (1, 51, 7, 11)])
@pytest.mark.parametrize("n", [0, 1, 1000, 1 << 20])
def test_record_sizes(op, ell, lx, k_lo, n):
    """bc_rand_bytes against the record layout, and the per-element figures the
    precomputed mode is quoted with (ReLU l_x = 7: 32 B, DReLU l_x = 18: 124 B)."""
    from paper_2309_04909_amd import bicop as B
    prm = B.Params(ell, lx, k_lo)
    assert B.rand_bytes(op, prm, n) == _record_bytes(lx + 1, op == B.BC_OP_RELU, B.ring_width(ell), n)
    if n == 1 << 20 and ell == 64 and (op, lx) in ((1, 7), (0, 18)):
        assert B.rand_bytes(op, prm, n) == n * {7: 32, 18: 124}[lx]


def test_batch_plan_validation_on_host():
    """bc_batch_plan is host-only: it validates and fills a host buffer, never launches."""
    from paper_2309_04909_amd import bicop as B
    L = B.lib
    prm = B.Params(64, 7, 11).c()
    seg = (B._Segment * 2)()
    seg[0] = B._Segment(0x1000, 0x2000, 0x3000, 0x4000, 5000, 0, 1, B.BC_OP_RELU, 0)
    seg[1] = B._Segment(0x5000, 0x6000, 0x7000, 0x8000, 0, 99, 2, B.BC_OP_DRELU, 0)
    nbytes = L.bc_batch_plan_bytes(2)
    assert nbytes == 64 + 2 * 80 + 3 * 8
    buf = (ctypes.c_uint8 * nbytes)()
    assert L.bc_batch_plan(seg, 2, ctypes.byref(prm), 1024, buf, nbytes) == 0
    words = np.frombuffer(bytes(buf), dtype=np.uint64)
    tb = words[(64 + 160) // 8:]
    assert list(tb) == [0, 5, 5]                                  # ceil(5000 / 1024) tiles, then the empty one
    assert L.bc_batch_plan(seg, 2, ctypes.byref(prm), 1024, buf, nbytes - 1) == -7
    assert L.bc_batch_plan(seg, 0, ctypes.byref(prm), 1024, buf, nbytes) == -8
    assert L.bc_batch_plan(seg, 2, ctypes.byref(prm), 1 << 20, buf, nbytes) == 0    # the largest tile
    assert L.bc_batch_plan(seg, 2, ctypes.byref(prm), (1 << 20) + 1, buf, nbytes) == -8
    seg[1].op = 5
    assert L.bc_batch_plan(seg, 2, ctypes.byref(prm), 1024, buf, nbytes) == -8
    seg[1].op = B.BC_OP_DRELU
    seg[0].x0 = 0x1004                                              # not 8-byte aligned
    assert L.bc_batch_plan(seg, 2, ctypes.byref(prm), 1024, buf, nbytes) == -5
    seg[0].x0 = None
    assert L.bc_batch_plan(seg, 2, ctypes.byref(prm), 1024, buf, nbytes) == -1
    seg[0].x0 = 0x1000
    seg[0].elem_base = (1 << 48) - 10
    assert L.bc_batch_plan(seg, 2, ctypes.byref(prm), 1024, buf, nbytes) == -8
    bad = B.Params(64, 7, 0, 257).c()
    seg[0].elem_base = 0
    assert L.bc_batch_plan(seg, 2, ctypes.byref(bad), 1024, buf, nbytes) == -4
    # per-segment input truncation: the input ring must keep the storage width
    seg[1].k_in = 1
    assert L.bc_batch_plan(seg, 2, ctypes.byref(prm), 1024, buf, nbytes) == -2      # 64 + 1 bits
    r51 = B.Params(51, 11, 13).c()
    seg[1].k_in = 13
    assert L.bc_batch_plan(seg, 2, ctypes.byref(r51), 1024, buf, nbytes) == 0       # Z_2^64 -> Z_2^51
    r24 = B.Params(24, 7, 10).c()
    seg[1].k_in = 9                                                                  # 33 bits: another width
    assert L.bc_batch_plan(seg, 2, ctypes.byref(r24), 1024, buf, nbytes) == -2
    seg[1].k_in = 0
    # a record segment: a 16-byte aligned record whose description (filled by
    # bc_rand_expand: here an empty expansion, then n set) matches the segment
    desc = B._RandDesc()
    sd0 = B.Seeds(1, 2, 3, 1).c()                                      # the nonce of seg[0]
    assert L.bc_rand_expand(None, 0, 0, B.BC_OP_RELU, ctypes.byref(prm), ctypes.byref(sd0), 0, ctypes.byref(desc),
                            None) == 0
    assert desc.magic == B.BC_RAND_MAGIC and desc.op == B.BC_OP_RELU and desc.prm.p == 251 and desc.n == 0
    assert desc.nonce == 1 and desc.elem_base == 0
    desc.n, desc.bytes = 5000, L.bc_rand_bytes(B.BC_OP_RELU, ctypes.byref(prm), 5000)
    seg[0].rand, seg[0].rand_desc = 0x100000, ctypes.pointer(desc)
    assert L.bc_batch_plan(seg, 2, ctypes.byref(prm), 1024, buf, nbytes) == 0
    desc.bytes -= 1
    assert L.bc_batch_plan(seg, 2, ctypes.byref(prm), 1024, buf, nbytes) == -7
    desc.bytes += 1
    desc.n = 4999                                                      # expanded for another n
    assert L.bc_batch_plan(seg, 2, ctypes.byref(prm), 1024, buf, nbytes) == -8
    assert b"record was expanded for" in L.bc_last_error()
    desc.n, desc.op = 5000, B.BC_OP_DRELU                              # for another op
    assert L.bc_batch_plan(seg, 2, ctypes.byref(prm), 1024, buf, nbytes) == -8
    desc.op, desc.prm.k_lo = B.BC_OP_RELU, 10                          # for another setting
    assert L.bc_batch_plan(seg, 2, ctypes.byref(prm), 1024, buf, nbytes) == -8
    desc.prm.k_lo, desc.nonce = 11, 2                                  # for another nonce
    assert L.bc_batch_plan(seg, 2, ctypes.byref(prm), 1024, buf, nbytes) == -8
    desc.nonce, desc.elem_base = 1, 5                                  # for another element offset
    assert L.bc_batch_plan(seg, 2, ctypes.byref(prm), 1024, buf, nbytes) == -8
    desc.elem_base, desc.magic = 0, 0                                  # not filled by bc_rand_expand
    assert L.bc_batch_plan(seg, 2, ctypes.byref(prm), 1024, buf, nbytes) == -8
    desc.magic = B.BC_RAND_MAGIC
    seg[0].rand_desc = None                                            # missing
    assert L.bc_batch_plan(seg, 2, ctypes.byref(prm), 1024, buf, nbytes) == -1
    seg[0].rand, seg[0].rand_desc = 0x100008, ctypes.pointer(desc)     # misaligned record
    assert L.bc_batch_plan(seg, 2, ctypes.byref(prm), 1024, buf, nbytes) == -5
    seg[0].rand, seg[0].rand_desc = None, None
    # bc_batch_run refuses a buffer that is not a plan (checked before any launch)
    junk = (ctypes.c_uint8 * nbytes)()
    sd = B.Seeds(1, 2, 3).c()
    assert L.bc_batch_run(ctypes.addressof(junk), junk, ctypes.byref(sd), 0, None) == -8


def test_static_batch_run_checks_on_host():
    """bc_batch_run_static refuses, before any HIP call, a NULL plan or seeds,
    a buffer that is not a plan and a plan larger than its fixed device area;
    the area's stated limits agree with bc_batch_plan_bytes."""
    from paper_2309_04909_amd import bicop as B
    L = B.lib
    assert L.bc_batch_plan_bytes(B.BC_STATIC_MAX_SEGMENTS) <= B.BC_STATIC_PLAN_BYTES
    assert L.bc_batch_plan_bytes(B.BC_STATIC_MAX_SEGMENTS + 1) > B.BC_STATIC_PLAN_BYTES
    hdr = open(os.path.join(ROOT, "include", "bicop.h")).read()
    assert re.search(r"#define BC_STATIC_PLAN_BYTES %du" % B.BC_STATIC_PLAN_BYTES, hdr)
    assert re.search(r"#define BC_STATIC_MAX_SEGMENTS %du" % B.BC_STATIC_MAX_SEGMENTS, hdr)
    prm = B.Params(64, 7, 11).c()
    sd = B.Seeds(1, 2, 3).c()
    nseg = B.BC_STATIC_MAX_SEGMENTS + 1
    seg = (B._Segment * nseg)()                    # empty segments: valid, and no pointers needed
    for i in range(nseg):
        seg[i] = B._Segment(None, None, None, None, 0, i, i, B.BC_OP_DRELU, 0)
    nbytes = L.bc_batch_plan_bytes(nseg)
    buf = (ctypes.c_uint8 * nbytes)()
    assert L.bc_batch_plan(seg, nseg, ctypes.byref(prm), 0, buf, nbytes) == 0
    assert L.bc_batch_run_static(buf, ctypes.byref(sd), 0, None) == -7
    assert b"fixed plan area" in L.bc_last_error()
    assert L.bc_batch_run_static(None, ctypes.byref(sd), 0, None) == -1
    assert L.bc_batch_run_static(buf, None, 0, None) == -1
    junk = (ctypes.c_uint8 * 64)()
    assert L.bc_batch_run_static(junk, ctypes.byref(sd), 0, None) == -8


def _snapshot(B, keys):
    return {(k, n, w, o): B.get_schedule(k, n, w, o) for k, n in keys for w in (4, 8) for o in (0, 1)}


def _restore(B, snap):
    for (k, n, w, o), v in snap.items():
        B.set_schedule(k, n, v, w, o)


def test_schedule_table_round_trip(tmp_path):
    """An autotuned schedules.json is applied by load_schedules (host-side table only)."""
    import json
    from paper_2309_04909_amd import bicop as B
    snap = _snapshot(B, (("fused", 19), ("stream", 0), ("batch", 8)))
    table = {"grid": [{"kind": "fused", "npos": 19, "width": 8, "op": 0, "blocks_per_cu": 7},
                      {"kind": "stream", "npos": 0, "width": 8, "blocks_per_cu": 3},
                      {"kind": "batch", "npos": 8, "blocks_per_cu": 5}], "batch_tile": 2048}
    path = tmp_path / "schedules.json"
    path.write_text(json.dumps(table))
    try:
        got = B.load_schedules(str(path))
        assert got["batch_tile"] == 2048
        assert B.get_schedule("fused", 19, 8, B.BC_OP_DRELU) == 7
        assert B.get_schedule("stream", 0, 8, B.BC_OP_DRELU) == B.get_schedule("stream", 0, 8, B.BC_OP_RELU) == 3
        assert all(B.get_schedule("batch", 8, w, o) == 5 for w in (4, 8) for o in (0, 1))
        with pytest.raises(B.BicopError):
            B.set_schedule("fused", 19, 2000)          # above the 1024 limit
        with pytest.raises(B.BicopError):
            B.set_schedule("fused", 19, 4, 2, 0)       # no 2-byte ring
        assert B.get_schedule("fused", 19, 16, 0) == 0 and B.get_schedule("fused", 19, 8, 3) == 0
    finally:
        _restore(B, snap)


def test_schedules_of_one_window_count_stay_apart(tmp_path):
    """Two settings with the same window count but another ring width or op
    run different kernels and keep their own schedules (N = 8: l = 64 and
    l = 24, DReLU and ReLU); a table that lists one key twice is refused."""
    import json
    from paper_2309_04909_amd import bicop as B
    snap = _snapshot(B, (("pre", 8), ("group", 8)))
    table = {"grid": [{"kind": "pre", "npos": 8, "width": 8, "op": 0, "blocks_per_cu": 2},
                      {"kind": "pre", "npos": 8, "width": 4, "op": 0, "blocks_per_cu": 64},
                      {"kind": "pre", "npos": 8, "width": 8, "op": 1, "blocks_per_cu": 16},
                      {"kind": "group", "npos": 8, "blocks_per_cu": 4},
                      {"kind": "group", "npos": 8, "width": 4, "op": 1, "blocks_per_cu": 1}]}
    path = tmp_path / "schedules.json"
    path.write_text(json.dumps(table))
    try:
        B.load_schedules(str(path))
        assert B.get_schedule("pre", 8, 8, B.BC_OP_DRELU) == 2
        assert B.get_schedule("pre", 8, 4, B.BC_OP_DRELU) == 64
        assert B.get_schedule("pre", 8, 8, B.BC_OP_RELU) == 16
        # the wildcard group entry applies where no specific one exists, whatever the order in the file
        assert B.get_schedule("group", 8, 8, B.BC_OP_DRELU) == 4
        assert B.get_schedule("group", 8, 4, B.BC_OP_RELU) == 1
        dup = {"grid": table["grid"] + [{"kind": "pre", "npos": 8, "width": 4, "op": 0, "blocks_per_cu": 8}]}
        path.write_text(json.dumps(dup))
        with pytest.raises(ValueError):
            B.load_schedules(str(path))
    finally:
        _restore(B, snap)


def test_committed_schedule_table_has_unique_keys():
    """schedules.json (the autotuner's output) lists every key once."""
    import json
    from paper_2309_04909_amd import bicop as B
    with open(B.SCHEDULES_PATH) as f:
        grid = json.load(f)["grid"]
    keys = [B.schedule_key(e) for e in grid]
    assert len(keys) == len(set(keys))


@pytest.mark.parametrize("ell,f", [(64, 13), (64, 16), (32, 8), (51, 13)])
def test_keybit_params_match_oracle(ell, f):
    """bc_keybit_params is the oracle's key-bit window (Sec. 6.1) plus its validation and default prime."""
    from paper_2309_04909_amd import bicop as B
    for ib in range(0, 34):
        for fb in range(0, min(f, 4) + 1):
            k_lo, lx = OP.keybit_window(f, ib, fb)
            try:
                OP.check_drelu(ell, lx, k_lo, OP.default_prime(lx) if 1 <= lx <= 32 else 0)
                ok = True
            except ValueError:
                ok = False
            if ok:
                got = B.keybit_params(ell, f, ib, fb)
                assert (got.ell, got.lx, got.k_lo, got.p) == (ell, lx, k_lo, OP.default_prime(lx))
            else:
                with pytest.raises(B.BicopError):
                    B.keybit_params(ell, f, ib, fb)
    with pytest.raises(B.BicopError):
        B.keybit_params(ell, f, 5, f + 1)                # more fractional bits than f


def test_keybit_settings_of_the_workloads():
    """Tab. 5's "5 + 2" at f = 13 and the 2^30-bounded key-bit setting."""
    from paper_2309_04909_amd import bicop as B
    r = B.keybit_params(64, 13, 5, 2)
    assert (r.k_lo, r.lx, r.p) == (11, 7, 251)
    ib = B.keybit_int_bits(1 << 30, 13)
    assert ib == 18
    r = B.keybit_params(64, 13, ib, 0)
    assert (r.k_lo, r.lx, r.p) == (13, 18, (1 << 19) - 1)


@pytest.mark.parametrize("f", [0, 8, 13])
def test_keybit_int_bits_is_the_smallest_guarded_window(f):
    from paper_2309_04909_amd import bicop as B
    for bound in [1, 2, 3, 255, 256, 257, 1 << 20, (1 << 30) - 1, 1 << 30, (1 << 30) + 1, (1 << 62) + 5]:
        i = B.keybit_int_bits(bound, f)
        assert i >= 1
        for fb in range(0, f + 1):
            k_lo, lx = OP.keybit_window(f, i, fb)
            assert OP.guard_bound(k_lo, lx) >= bound                 # |x| < bound is inside the guard domain
            if i > 1:
                assert OP.guard_bound(*OP.keybit_window(f, i - 1, fb)) < bound   # and one bit fewer is not


def test_pseudo_mersenne_table_is_the_default_primes():
    """The kernels' table of 2^K - p (bc_device.h) against the oracle's own
    largest-prime-below-2^K search, for every K = l_x + 1 it covers."""
    src = open(os.path.join(ROOT, "paper_2309_04909_amd", "csrc", "bc_device.h")).read()
    m = re.search(r"kPrimeDelta\[34\]\s*=\s*\{([^}]*)\}", src)
    table = [int(v) for v in m.group(1).replace("\n", " ").split(",")]
    assert len(table) == 34
    for K in range(2, 34):
        assert table[K] == (1 << K) - OP.default_prime(K - 1), K


def test_profile_hash_ignores_comments_only():
    """The counters in profiles/traffic.json stay valid across comment and
    layout edits of a kernel's sources, and not across code edits."""
    from paper_2309_04909_amd.prof_summary import code_text, source_hash
    src = 'int f(int a) { // add one\n  return a + 1; /* "x" */ }\nconst char* s = "a // b";\n'
    assert code_text(src) == 'int f(int a) { return a + 1; } const char* s = "a // b";'
    base = source_hash(["x.h"], read=lambda nm: src)
    assert source_hash(["x.h"], read=lambda nm: src.replace("add one", "increment")) == base
    assert source_hash(["x.h"], read=lambda nm: src.replace("\n  ", "\n    ")) == base
    assert source_hash(["x.h"], read=lambda nm: src.replace("a + 1", "a + 2")) != base
    assert source_hash(["x.h"], read=lambda nm: src.replace('"a // b"', '"a // c"')) != base


def test_profile_last_calls_mean(tmp_path):
    """The timed-step column of the kernel statistics averages each kernel's
    last k dispatches in start-time order, whatever order the trace lists."""
    from paper_2309_04909_amd.prof_summary import last_calls_mean
    rows = [("A", 50, 150), ("B", 0, 10), ("A", 0, 200), ("A", 300, 330), ("B", 20, 24)]   # A: 200, 100, 30
    lines = ['"Kernel_Name","Start_Timestamp","End_Timestamp"'] + [f'"{k}",{s},{e}' for k, s, e in rows]
    (tmp_path / "run").mkdir()
    (tmp_path / "run" / "bench_kernel_trace.csv").write_text("\n".join(lines) + "\n")
    assert last_calls_mean(str(tmp_path), 2) == {"A": 65.0, "B": 7.0}
    assert last_calls_mean(str(tmp_path), 5) == {"A": 110.0, "B": 7.0}


def test_rss_error_paths_without_gpu():
    """The replicated-sharing calls validate on the host like bc_drelu: every
    call below fails validation (or has n = 0), so nothing is launched."""
    from paper_2309_04909_amd import bicop as B
    L = B.lib
    prm, sd = B.Params(64, 7, 11).c(), B.RssSeeds(1, 2, 3, 4, 5, 6).c()
    for fn in (L.bc_rss_drelu, L.bc_rss_relu):
        args = lambda n, prm=prm, sd=sd, base=0: (None, None, None, None, None, None, n, ctypes.byref(prm),
                                                   sd if sd is None else ctypes.byref(sd), base, None, None, None)
        assert fn(*args(10)) == -1                                   # NULL shares
        assert fn(*args(0)) == 0                                      # n = 0
        assert fn(*args(10, sd=None)) == -1                           # NULL seeds
        assert fn(*args(10, prm=B.Params(64, 40, 0).c())) == -3       # window too wide
        assert fn(*args(10, prm=B.Params(64, 7, 0, 255).c())) == -4   # not prime
        assert fn(*args(10, base=(1 << 48) - 5)) == -8                # indices past 2^48
        acct = B._Acct()
        assert fn(None, None, None, None, None, None, 0, ctypes.byref(prm), ctypes.byref(sd), 0, None,
                  ctypes.byref(acct), None) == 0
    assert L.bc_msg_account(4, ctypes.byref(prm), 1, ctypes.byref(B._Acct())) == -8


def test_mul_trunc_error_paths_without_gpu():
    """bc_mul_trunc validates ring, order, f, seeds and indices on the host."""
    from paper_2309_04909_amd import bicop as B
    L = B.lib
    sd = B.Seeds(1, 2, 3, 4).c()
    N = None

    def call(n=10, ell=64, f=26, order=B.BC_TRUNC_BEFORE, seeds=sd, base=0):
        return L.bc_mul_trunc(N, N, N, N, N, N, n, ell, f, order, None if seeds is None else ctypes.byref(seeds),
                              base, N)
    assert call() == -1                                  # NULL shares
    assert call(n=0) == 0
    assert call(ell=0) == -2 and call(ell=65) == -2
    assert call(order=B.BC_TRUNC_NONE) == -8             # f must be 0 without truncation
    assert call(order=B.BC_TRUNC_NONE, f=0) == -1
    assert call(order=B.BC_TRUNC_AFTER, f=64) == -2      # f >= ell
    assert call(order=B.BC_TRUNC_AFTER, ell=8, f=7) == -1
    assert call(order=B.BC_TRUNC_BEFORE, ell=8, f=15) == -2   # ceil(15/2) = 8 >= ell
    assert call(order=B.BC_TRUNC_BEFORE, ell=8, f=14) == -1
    assert call(order=3) == -8
    assert call(seeds=None) == -1
    assert call(base=(1 << 48) - 5) == -8


def test_split_drelu_host_side():
    """Message size per setting matches the oracle's packing, and the
    parties-apart calls validate on the host."""
    from paper_2309_04909_amd import bicop as B
    L = B.lib
    assert [L.bc_msg_words(n) for n in range(2, 34)] == [OPR.msg_words(n) for n in range(2, 34)]
    assert L.bc_msg_words(1) == 0 and L.bc_msg_words(34) == 0
    prm, sd = B.Params(64, 18, 13).c(), B.Seeds(1, 2, 3, 4).c()
    P_, S_ = ctypes.byref(prm), ctypes.byref(sd)
    assert L.bc_drelu_send(2, None, None, 10, P_, S_, 0, None) == -8          # party
    assert L.bc_drelu_send(0, None, None, 10, P_, S_, 0, None) == -1          # NULL
    assert L.bc_drelu_send(1, None, None, 0, P_, S_, 0, None) == 0            # n = 0
    assert L.bc_drelu_send(0, None, None, 10, P_, None, 0, None) == -1        # seeds
    assert L.bc_drelu_reply(None, None, None, None, 10, P_, S_, 0, None) == -1
    assert L.bc_drelu_reply(None, None, None, None, 10, P_, S_, (1 << 48) - 1, None) == -8
    assert L.bc_drelu_finish(3, None, None, 10, P_, S_, 0, None) == -8
    assert L.bc_drelu_finish(1, None, None, 10, ctypes.byref(B.Params(64, 40, 0).c()), S_, 0, None) == -3


def test_boundary_departures_from_the_planned_abi():
    """Where the C ABI's error codes mean something other than the planned
    interface's, each meaning is checked on the host (no launch):
    * BC_ERR_ALIGN asks for element-size alignment, not 16 bytes: an 8-byte
      ring accepts 8-byte-aligned pointers, a 4-byte ring 4-byte-aligned ones;
    * BC_ERR_RING: rings of 1..64 bits (l = 1 only for the identity truncation);
    * BC_ERR_WINDOW: windows of l_x >= 1 (the guard bit is a domain rule of the
      inputs, bc_keybit_int_bits, not a precondition of the arithmetic);
    * streams are opaque pointers, passed through unchanged;
    * BC_ERR_WORKSPACE also covers the static plan area's segment limit."""
    from paper_2309_04909_amd import bicop as B
    L = B.lib
    # alignment: element size, not 16 bytes (host-only plan building)
    for ell, good, bad in ((64, 0x1008, 0x1004), (32, 0x1004, 0x1002)):
        prm = B.Params(ell, 7, 10).c()
        seg = (B._Segment * 1)()
        seg[0] = B._Segment(good, 0x2000, 0x3000, 0x4000, 100, 0, 1, B.BC_OP_DRELU, 0)
        buf = (ctypes.c_uint8 * L.bc_batch_plan_bytes(1))()
        assert L.bc_batch_plan(seg, 1, ctypes.byref(prm), 0, buf, len(buf)) == 0
        seg[0].x0 = bad
        assert L.bc_batch_plan(seg, 1, ctypes.byref(prm), 0, buf, len(buf)) == -5
    # rings: 1..64 bits; the ring check comes before the n = 0 shortcut
    assert L.bc_trunc_det(None, None, None, None, 0, 1, 0, 0, None) == 0
    assert L.bc_trunc_det(None, None, None, None, 0, 0, 0, 0, None) == -2
    assert L.bc_trunc_det(None, None, None, None, 0, 65, 0, 0, None) == -2
    assert L.bc_trunc_prob(None, None, None, None, 0, 1, 0, None) == 0
    assert L.bc_mod_switch(None, None, None, None, 0, 1, 3, None) == 0            # Z_2 -> Z_3
    # windows: l_x = 1 and 2 are settings like any other (N = 2, 3 windows)
    for ell, lx in ((2, 1), (4, 2), (64, 1), (64, 2)):
        assert L.bc_check_params(ctypes.byref(B.Params(ell, lx, 0).c()), None) == 0
    assert L.bc_check_params(ctypes.byref(B.Params(64, 0, 0).c()), None) == -3
    # streams: an opaque handle, not dereferenced by the validation
    assert L.bc_trunc_det(None, None, None, None, 0, 64, 13, 0, ctypes.c_void_p(0xDEAD0)) == 0
