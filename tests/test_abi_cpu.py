"""C-ABI library checks that need no GPU: it loads, exports every function
declared in include/tfft.h, and rejects invalid arguments before any device
work."""
import ctypes
import json
import os
import re

import pytest

from paper_2412_05824_amd import _lib

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "tfft.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tfft_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported_and_bound():
    lib = _lib.load()
    names = declared_functions()
    assert "tfft_c2c" in names and "tfft_c2c_ragged" in names
    for n in names:
        assert hasattr(lib, n), n
        assert n in _lib.SIGNATURES, n


def test_strerror_and_status_codes():
    for st in (_lib.TFFT_OK, _lib.TFFT_EINVAL, _lib.TFFT_EUNSUPPORTED, _lib.TFFT_EALIGN,
               _lib.TFFT_EHIP, _lib.TFFT_ENOMEM, _lib.TFFT_ECAPTURE, _lib.TFFT_ENOTPREPARED,
               _lib.TFFT_ESCRATCH):
        assert _lib.strerror(st) and _lib.strerror(st) != "unknown status"
    assert _lib.strerror(-99) == "unknown status"


def test_invalid_arguments_rejected_on_host():
    lib = _lib.load()
    c2c = lib.tfft_c2c
    dummy = 4096  # never dereferenced: validation fails first
    assert c2c(dummy, dummy, 0, 4, -1, 0, 0, 0.0, None, None) == _lib.TFFT_EINVAL        # N < 1
    assert c2c(dummy, dummy, 64, -1, -1, 0, 0, 0.0, None, None) == _lib.TFFT_EINVAL      # batch < 0
    assert c2c(dummy, dummy, 64, 4, 0, 0, 0, 0.0, None, None) == _lib.TFFT_EINVAL        # dir
    assert c2c(dummy, dummy, 64, 4, -1, 2, 0, 0.0, None, None) == _lib.TFFT_EINVAL       # precision
    assert c2c(dummy, dummy, 64, 4, -1, 0, 3, 0.0, None, None) == _lib.TFFT_EINVAL       # ft mode
    assert c2c(dummy, dummy, 100, 4, -1, 0, 0, 0.0, None, None) == _lib.TFFT_EUNSUPPORTED  # 100 = 4*25
    assert c2c(dummy, dummy, 64, 0, -1, 0, 0, 0.0, None, None) == _lib.TFFT_OK           # empty batch
    assert c2c(None, dummy, 64, 4, -1, 0, 0, 0.0, None, None) == _lib.TFFT_EINVAL        # null x
    assert c2c(dummy, dummy, 64, 4, -1, 0, 2, 0.0, None, None) == _lib.TFFT_EINVAL       # FT without counts
    assert c2c(dummy + 4, dummy + 4, 64, 4, -1, 0, 0, 0.0, None, None) == _lib.TFFT_EALIGN
    assert c2c(dummy, dummy + 8, 64, 4, -1, 0, 0, 0.0, None, None) == _lib.TFFT_EINVAL   # partial overlap
    assert lib.tfft_inject_arm(0, 0, 0, 32, 0) == _lib.TFFT_EINVAL
    assert lib.tfft_inject_arm(0, 0, 2, 3, 0) == _lib.TFFT_EINVAL
    assert lib.tfft_inject_arm(0, 0, 0, 63, 1) == _lib.TFFT_OK
    assert lib.tfft_inject_disarm() == _lib.TFFT_OK
    d = _lib.InjectDesc(signal=0, element=0, part=0, bit=3, precision=0, pass_=3, stage=-1)
    assert lib.tfft_inject_arm_desc(ctypes.byref(d)) == _lib.TFFT_EINVAL      # no fourth pass
    d.pass_ = 2
    assert lib.tfft_inject_arm_desc(ctypes.byref(d)) == _lib.TFFT_OK
    # 2^20 runs as two passes: a flip armed for a third pass does not fit
    assert c2c(dummy, dummy + (1 << 24), 1 << 20, 1, -1, 0, 0, 0.0, None, None) == _lib.TFFT_EINVAL
    d.pass_, d.stage = 0, -2
    assert lib.tfft_inject_arm_desc(ctypes.byref(d)) == _lib.TFFT_EINVAL      # stage below -1
    assert lib.tfft_inject_arm_desc(None) == _lib.TFFT_EINVAL
    d.pass_, d.stage = 1, 0
    assert lib.tfft_inject_arm_desc(ctypes.byref(d)) == _lib.TFFT_OK
    # an armed flip that does not fit the call is refused before any device work:
    # 256 points run as one pass, so pass 1 does not exist
    assert c2c(dummy, dummy + (1 << 20), 256, 4, -1, 0, 0, 0.0, None, None) == _lib.TFFT_EINVAL
    assert lib.tfft_inject_disarm() == _lib.TFFT_OK
    assert lib.tfft_set_tuning(64, 0, 33, 0.0) == _lib.TFFT_EINVAL
    assert lib.tfft_prepare(0, 0, 0, 0, None) == _lib.TFFT_EINVAL
    assert lib.tfft_prepare(256, -1, 0, 0, None) == _lib.TFFT_EINVAL
    assert lib.tfft_prepare(100, 0, 0, 0, None) == _lib.TFFT_EUNSUPPORTED
    # launch-timing filter: fields in range or -1 (any)
    assert lib.tfft_profile_only(2, -1, -1, -1, -1) == _lib.TFFT_EINVAL
    assert lib.tfft_profile_only(-1, 6, -1, -1, -1) == _lib.TFFT_EINVAL
    assert lib.tfft_profile_only(-1, -1, -2, -1, -1) == _lib.TFFT_EINVAL
    assert lib.tfft_profile_only(-1, -1, -1, 4, -1) == _lib.TFFT_EINVAL
    assert lib.tfft_profile_only(-1, -1, -1, -1, -2) == _lib.TFFT_EINVAL
    assert lib.tfft_profile_only(0, 2, 2048, 2, 3) == _lib.TFFT_OK
    assert lib.tfft_profile_only(-1, -1, -1, -1, -1) == _lib.TFFT_OK


def test_supported_sizes_and_tuning_roundtrip():
    lib = _lib.load()
    for N in (64, 256, 1024, 4096):
        assert lib.tfft_supported(N, 0) == 1
        assert lib.tfft_supported(N, 1) == 1
    assert lib.tfft_supported(100, 0) == 0
    T = ctypes.c_int()
    k = ctypes.c_double()
    assert lib.tfft_set_tuning(512, 0, 2, 3.5) == 0
    assert lib.tfft_get_tuning(512, 0, ctypes.byref(T), ctypes.byref(k)) == 0
    assert (T.value, k.value) == (2, 3.5)


def test_ragged_route_menu():
    """Every length of the ragged menu (2^k, 3*2^k, 6 <= k <= 16) has a route,
    lengths outside it do not; ragged batches are fp32 only."""
    lib = _lib.load()
    menu = [1 << k for k in range(6, 18)] + [3 << k for k in range(6, 17)]
    for n in menu:
        assert lib.tfft_ragged_supported(n, _lib.FP32) == 1, n
    for n in (1, 32, 48, 96, 100, 3 << 17, 1 << 18):
        assert lib.tfft_ragged_supported(n, _lib.FP32) == 0, n
    assert lib.tfft_ragged_supported(1024, _lib.FP64) == 0


def test_ragged_invalid_arguments_rejected_on_host():
    lib = _lib.load()
    h = ctypes.c_void_p()
    sizes = (ctypes.c_longlong * 2)(64, 128)
    assert lib.tfft_ragged_plan_create(None, sizes, 2, _lib.FP32) == _lib.TFFT_EINVAL
    assert lib.tfft_ragged_plan_create(ctypes.byref(h), None, 2, _lib.FP32) == _lib.TFFT_EINVAL
    assert lib.tfft_ragged_plan_create(ctypes.byref(h), sizes, -1, _lib.FP32) == _lib.TFFT_EINVAL
    assert lib.tfft_ragged_plan_create(ctypes.byref(h), sizes, 2, 7) == _lib.TFFT_EINVAL
    assert lib.tfft_ragged_plan_create(ctypes.byref(h), sizes, 2, _lib.FP64) == _lib.TFFT_EUNSUPPORTED
    bad = (ctypes.c_longlong * 2)(64, 0)
    assert lib.tfft_ragged_plan_create(ctypes.byref(h), bad, 2, _lib.FP32) == _lib.TFFT_EINVAL
    assert lib.tfft_c2c_ragged(None, None, None, -1, 0, 0, 0, None, None) == _lib.TFFT_EINVAL
    assert lib.tfft_ragged_plan_destroy(None) == _lib.TFFT_EINVAL
    info = (ctypes.c_longlong * 8)()
    assert lib.tfft_ragged_plan_info(None, info, 8) == _lib.TFFT_EINVAL


def test_routes_and_forced_split():
    """Multi-pass decomposition choices (Sec. 3.1): the default route of a
    length, the candidate list (codes n1 | va << 32 | vb << 40), and forcing
    a route."""
    lib = _lib.load()
    FP32 = _lib.FP32

    def routes(n, prec=FP32):
        cnt = lib.tfft_routes(n, prec, 2, None, 0)
        buf = (ctypes.c_longlong * max(1, cnt))()
        assert lib.tfft_routes(n, prec, 2, buf, cnt) == cnt
        return [buf[i] for i in range(cnt)]

    def route(n, prec=FP32):
        v = ctypes.c_longlong()
        assert lib.tfft_get_route(n, prec, 2, ctypes.byref(v)) == _lib.TFFT_OK
        return v.value

    n1 = lambda c: c & 0xFFFFFFFF
    r4096 = routes(4096)
    assert r4096[0] == 1 and len(r4096) > 1          # single pass, and splits
    assert lib.tfft_set_route(1 << 20, FP32, 0) == _lib.TFFT_OK   # the default policy, not the table's
    assert lib.tfft_set_route(4096, FP32, 0) == _lib.TFFT_OK
    assert route(4096) == 1
    big = routes(1 << 20)
    assert all(n1(c) > 1 and (1 << 20) % n1(c) == 0 for c in big)
    assert any(c >> 32 for c in big)                   # tile-width variants exist
    default = route(1 << 20)
    assert default in big and n1(default) ** 2 <= (1 << 20) and default >> 32 == 0
    try:
        alt = [c for c in r4096 if n1(c) > 1][0]
        assert lib.tfft_set_route(4096, FP32, alt) == _lib.TFFT_OK
        assert route(4096) == alt
        assert lib.tfft_set_route(4096, FP32, 3) == _lib.TFFT_EUNSUPPORTED
        assert lib.tfft_set_route(1 << 20, FP32, 1) == _lib.TFFT_EUNSUPPORTED
        assert lib.tfft_set_route(4096, FP32, 1 | (7 << 32)) == _lib.TFFT_EUNSUPPORTED
        wide = [c for c in big if c >> 32][0]
        assert lib.tfft_set_route(1 << 20, FP32, wide) == _lib.TFFT_OK
        assert route(1 << 20) == wide
    finally:
        assert lib.tfft_set_route(4096, FP32, 0) == _lib.TFFT_OK
        assert lib.tfft_set_route(1 << 20, FP32, 0) == _lib.TFFT_OK
        if os.path.exists(_lib.TUNING_PATH):   # back to the package's table
            assert lib.tfft_load_tuning(_lib.TUNING_PATH.encode()) >= 0


def test_load_tuning_table(tmp_path):
    lib = _lib.load()
    T = ctypes.c_int()
    k = ctypes.c_double()
    good = tmp_path / "good.json"
    good.write_text(json.dumps({"format": "x", "entries": [
        {"precision": "fp32", "N": 2048, "T": 1, "kappa": 9.5, "split_n1": 0, "gbs": 1.0},
        {"precision": "fp64", "N": 1024, "T": 4, "chunk_bytes": 1 << 26},
        {"precision": "fp32", "N": 1 << 20, "ft_mode": 0, "split_n1": 512, "variant_a": 1, "variant_b": 1},
    ]}))
    route = ctypes.c_longlong()
    before = ctypes.c_longlong()
    assert lib.tfft_get_route(1 << 20, _lib.FP32, 2, ctypes.byref(before)) == 0
    try:
        assert lib.tfft_load_tuning(str(good).encode()) == 3
        assert lib.tfft_get_route(1 << 20, _lib.FP32, 0, ctypes.byref(route)) == 0
        assert route.value == 512 | (1 << 32) | (1 << 40)
        assert lib.tfft_get_route(1 << 20, _lib.FP32, 2, ctypes.byref(route)) == 0
        assert route.value == before.value              # the other modes keep their route
        assert lib.tfft_get_tuning(2048, _lib.FP32, ctypes.byref(T), ctypes.byref(k)) == 0
        assert (T.value, k.value) == (1, 9.5)
        assert lib.tfft_get_tuning(1024, _lib.FP64, ctypes.byref(T), ctypes.byref(k)) == 0
        assert T.value == 4
        # malformed, out of range, unbuilt route: nothing applied
        for bad in ('{"entries": [', '{"entries": [{"precision": "fp32", "N": 2048, "T": 99}]}',
                    '{"entries": [{"precision": "fp32", "N": 2048, "T": 2}, '
                    '{"precision": "fp32", "N": 4096, "split_n1": 3}]}',
                    '[]', '{"entries": [{"precision": "fp16", "N": 64}]}'):
            p = tmp_path / "bad.json"
            p.write_text(bad)
            assert lib.tfft_load_tuning(str(p).encode()) < 0, bad
        assert lib.tfft_get_tuning(2048, _lib.FP32, ctypes.byref(T), ctypes.byref(k)) == 0
        assert T.value == 1
        assert lib.tfft_load_tuning(str(tmp_path / "missing.json").encode()) == _lib.TFFT_EINVAL
    finally:
        lib.tfft_set_tuning(2048, _lib.FP32, 1, 8.0)
        lib.tfft_set_tuning(1024, _lib.FP64, 8, 16.0)
        lib.tfft_set_chunk(1024, _lib.FP64, 128 << 20)
        lib.tfft_set_route(1 << 20, _lib.FP32, 0)
        if os.path.exists(_lib.TUNING_PATH):
            assert lib.tfft_load_tuning(_lib.TUNING_PATH.encode()) >= 0


def test_shipped_tuning_table_is_complete_and_consistent():
    """The package's tuning table covers every length of the benchmark sweeps
    in both the correcting and the plain mode, gives both modes the same route
    (so switching ABFT on or off never changes an output bit), keeps T within
    the autotuner's accuracy bound for its detection granularity, and is
    accepted by the library."""
    import math
    from paper_2412_05824_amd import autotune
    doc = json.load(open(_lib.TUNING_PATH))
    entries = {(e["precision"], e["N"], e.get("ft_mode", 2)): e for e in doc["entries"]}
    for prec, hi in (("fp32", 22), ("fp64", 20)):
        for lg in range(6, hi + 1):
            N = 1 << lg
            on, off = entries[(prec, N, 2)], entries[(prec, N, 0)]
            route = lambda e: (e.get("split_n1", 1), e.get("variant_a", 0), e.get("variant_b", 0))
            assert route(on) == route(off), (prec, N)
            n1 = on.get("split_n1", 1)
            gran = on.get("gran", 0)
            assert gran in (0, 1), (prec, N, gran)
            # checked per transaction, each signal has its own threshold: T
            # only sets the sums a correction uses (at most 16 per group)
            tmax = 16 if gran else autotune.max_T(prec, autotune.steps(N, n1, on.get("split_n2", 0)), on["kappa"])
            assert 1 <= on["T"] <= tmax, (prec, N, on["T"], gran)
            assert math.isfinite(on["kappa"]) and on["kappa"] > 0
    lib = _lib.load()
    try:
        assert lib.tfft_load_tuning(_lib.TUNING_PATH.encode()) == len(doc["entries"])
    finally:
        lib.tfft_load_tuning(_lib.TUNING_PATH.encode())


def test_route_info_matches_routes():
    lib = _lib.load()
    buf = (ctypes.c_longlong * 6)()
    assert lib.tfft_route_info(256, 0, 2, buf, 6) == 0
    assert buf[0] == 1 and buf[1] == 256 and buf[2] == 1 and buf[3] >= 1 and buf[4] == 0
    assert lib.tfft_route_info(1 << 20, 0, 2, buf, 6) == 0
    assert buf[0] == 2 and buf[1] * buf[2] == 1 << 20 and buf[3] >= 1 and buf[4] >= 1
    assert lib.tfft_route_info(100, 0, 2, buf, 6) == _lib.TFFT_EUNSUPPORTED
    assert lib.tfft_route_info(256, 0, 2, None, 6) == _lib.TFFT_EINVAL


def test_noalloc_validates_on_host():
    """tfft_c2c_noalloc rejects what tfft_c2c rejects, and a signal larger
    than its scratch array, before touching the device."""
    lib = _lib.load()
    f = lib.tfft_c2c_noalloc
    dummy = 4096  # never dereferenced: validation fails first
    assert f(dummy, dummy, 0, 4, -1, 0, 0, 0.0, None, None) == _lib.TFFT_EINVAL
    assert f(dummy, dummy, 64, 4, 0, 0, 0, 0.0, None, None) == _lib.TFFT_EINVAL
    assert f(dummy, dummy, 100, 4, -1, 0, 0, 0.0, None, None) == _lib.TFFT_EUNSUPPORTED
    assert f(dummy, dummy, 64, 0, -1, 0, 0, 0.0, None, None) == _lib.TFFT_OK
    assert f(dummy, dummy, 64, 4, -1, 0, 2, 0.0, None, None) == _lib.TFFT_EINVAL
    assert f(dummy + 4, dummy + 4, 64, 4, -1, 0, 0, 0.0, None, None) == _lib.TFFT_EALIGN
    big = 1 << 40
    # 2^24 complex64 = 128 MiB per signal, 2^23 complex128 = 128 MiB: above 64 MiB
    assert _lib.NOALLOC_SCRATCH_BYTES == 64 << 20
    assert f(dummy, big, 1 << 24, 1, -1, 0, 0, 0.0, None, None) == _lib.TFFT_ESCRATCH
    assert f(dummy, big, 1 << 23, 1, -1, 1, 0, 0.0, None, None) == _lib.TFFT_ESCRATCH


def test_granularity_and_second_target_validated_on_host():
    lib = _lib.load()
    assert lib.tfft_set_granularity(256, 0, 2) == _lib.TFFT_EINVAL
    assert lib.tfft_set_granularity(0, 0, 1) == _lib.TFFT_EINVAL
    assert lib.tfft_set_granularity(256, 3, 1) == _lib.TFFT_EINVAL
    buf = (ctypes.c_longlong * 7)()
    # the granularity of the loaded tuning table; none without ABFT
    table = {(e["precision"], e["N"]): e for e in json.load(open(_lib.TUNING_PATH))["entries"]
             if e.get("ft_mode", 2) == 2}
    for prec, p in (("fp32", 0), ("fp64", 1)):
        assert lib.tfft_route_info(4096, p, 2, buf, 7) == _lib.TFFT_OK
        assert buf[6] == table[(prec, 4096)]["gran"]
        assert lib.tfft_route_info(4096, p, 0, buf, 7) == _lib.TFFT_OK and buf[6] == 0
    # per transaction, T is reduced to what the plan keeps (at most 16)
    T0, k0 = ctypes.c_int(), ctypes.c_double()
    assert lib.tfft_get_tuning(4096, 0, ctypes.byref(T0), ctypes.byref(k0)) == _lib.TFFT_OK
    try:
        assert lib.tfft_set_tuning(4096, 0, 32, 0.0) == _lib.TFFT_OK
        assert lib.tfft_route_info(4096, 0, 2, buf, 7) == _lib.TFFT_OK and 1 <= buf[5] <= 16
        assert lib.tfft_route_info(4096, 0, 0, buf, 7) == _lib.TFFT_OK and buf[5] == 32
        assert lib.tfft_set_granularity(4096, 0, 0) == _lib.TFFT_OK
        assert lib.tfft_route_info(4096, 0, 2, buf, 7) == _lib.TFFT_OK and buf[5] == 32 and buf[6] == 0
    finally:
        # every mode back to the loaded values (set_tuning applies to all modes)
        assert lib.tfft_set_granularity(4096, 0, 1) == _lib.TFFT_OK
        assert lib.tfft_set_tuning(4096, 0, T0.value, k0.value) == _lib.TFFT_OK
    d = _lib.InjectDesc(signal=3, element=0, part=0, bit=3, precision=0, pass_=-1, stage=-1, two=1, signal2=3)
    assert lib.tfft_inject_arm_desc(ctypes.byref(d)) == _lib.TFFT_EINVAL     # same signal twice
    d.two, d.signal2 = 2, 4
    assert lib.tfft_inject_arm_desc(ctypes.byref(d)) == _lib.TFFT_EINVAL
    d.two, d.signal2 = 1, -1
    assert lib.tfft_inject_arm_desc(ctypes.byref(d)) == _lib.TFFT_EINVAL
    d.two, d.signal2 = 1, 4
    assert lib.tfft_inject_arm_desc(ctypes.byref(d)) == _lib.TFFT_OK
    # a second target outside the batch is refused by the call, before device work
    dummy = 4096
    assert lib.tfft_c2c(dummy, dummy + (1 << 20), 256, 4, -1, 0, 0, 0.0, None, None) == _lib.TFFT_EINVAL
    assert lib.tfft_inject_disarm() == _lib.TFFT_OK


def test_three_pass_routes():
    """Lengths beyond the two-pass limit run as three passes (Sec. 3.3 launch
    rule: three launches for 2^23..2^29) in single precision; the route
    code carries the second length; three-pass routes can be forced on a
    two-pass length and read back; tuning tables name them by split_n2."""
    import paper_2412_05824_amd as tff
    lib = _lib.load()
    FP32 = _lib.FP32
    buf = (ctypes.c_longlong * 12)()
    for lg in range(23, 30):
        N = 1 << lg
        assert lib.tfft_supported(N, FP32) == 1, lg
        assert lib.tfft_route_info(N, FP32, 2, buf, 12) == 0
        assert buf[0] == 3 and buf[1] * buf[2] * buf[9] == N, (lg, list(buf))
        assert buf[5] == 1                      # groups of one signal per pass
        assert min(buf[3], buf[4], buf[10]) >= 1 and min(buf[7], buf[8], buf[11]) >= 1
        # the most balanced split: no length beyond the cube root's power of two by more than 2x
        assert max(buf[1], buf[2], buf[9]) <= 2 * (1 << -(-lg // 3)), (lg, list(buf))
    assert lib.tfft_supported(1 << 30, FP32) == 0
    # the two-pass lengths keep two passes by default
    assert lib.tfft_route_info(1 << 22, FP32, 2, buf, 12) == 0 and buf[0] == 2 and buf[9] == 1
    # codes round-trip through the Python helpers
    code = tff.route_code(64, 0, 0, 256)
    assert tff.route_n2(code) == 256 and tff.route_parts(code) == (64, 0, 0)
    three = [c for c in tff.routes(1 << 22) if tff.route_n2(c)]
    assert three, "a three-pass split of 2^22 is built"
    try:
        assert lib.tfft_set_route(1 << 22, FP32, three[0]) == _lib.TFFT_OK
        v = ctypes.c_longlong()
        assert lib.tfft_get_route(1 << 22, FP32, 2, ctypes.byref(v)) == 0 and v.value == three[0]
        assert lib.tfft_route_info(1 << 22, FP32, 2, buf, 12) == 0 and buf[0] == 3
        assert buf[2] == tff.route_n2(three[0])
        # an unbuilt last-pass variant; n2 must divide
        assert lib.tfft_set_route(1 << 22, FP32, three[0] | (7 << 40)) == _lib.TFFT_EUNSUPPORTED
        assert lib.tfft_set_route(1 << 22, FP32, tff.route_code(64, 0, 0, 1 << 17)) == _lib.TFFT_EUNSUPPORTED
        assert lib.tfft_set_route(1 << 22, FP32, 1 << 54) == _lib.TFFT_EUNSUPPORTED
    finally:
        lib.tfft_set_route(1 << 22, FP32, 0)
        if os.path.exists(_lib.TUNING_PATH):
            lib.tfft_load_tuning(_lib.TUNING_PATH.encode())


def test_three_pass_tuning_entries(tmp_path):
    lib = _lib.load()
    FP32 = _lib.FP32
    p = tmp_path / "t3.json"
    p.write_text(json.dumps({"entries": [
        {"precision": "fp32", "N": 1 << 23, "split_n1": 64, "split_n2": 512, "T": 1}]}))
    v = ctypes.c_longlong()
    try:
        assert lib.tfft_load_tuning(str(p).encode()) == 1
        assert lib.tfft_get_route(1 << 23, FP32, 2, ctypes.byref(v)) == 0
        assert v.value == 64 | (9 << 48)
        for bad in ({"split_n1": 64, "split_n2": 300}, {"split_n1": 64, "split_n2": 1 << 20},
                    {"split_n1": 64, "split_n2": -2}):
            p.write_text(json.dumps({"entries": [dict(precision="fp32", N=1 << 23, **bad)]}))
            assert lib.tfft_load_tuning(str(p).encode()) < 0, bad
    finally:
        lib.tfft_set_route(1 << 23, FP32, 0)
        if os.path.exists(_lib.TUNING_PATH):
            lib.tfft_load_tuning(_lib.TUNING_PATH.encode())


def test_stepwise_validates_on_host():
    lib = _lib.load()
    f = lib.tfft_c2c_stepwise
    dummy = 4096   # never dereferenced: validation fails first
    assert f(dummy, dummy + (1 << 20), 256, 4, -1, 4, None) == _lib.TFFT_EINVAL      # level
    assert f(dummy, dummy + (1 << 20), 256, 4, 0, 0, None) == _lib.TFFT_EINVAL       # dir
    assert f(dummy, dummy + (1 << 20), 96, 4, -1, 0, None) == _lib.TFFT_EUNSUPPORTED # not 2^k
    assert f(dummy, dummy + 8, 256, 4, -1, 0, None) == _lib.TFFT_EINVAL              # overlap
    assert f(dummy, dummy, 256, 4, -1, 0, None) == _lib.TFFT_EINVAL                  # in place
    assert f(dummy + 4, dummy + (1 << 20), 256, 4, -1, 0, None) == _lib.TFFT_EALIGN
    assert f(dummy, dummy + (1 << 20), 256, 0, -1, 0, None) == _lib.TFFT_OK          # empty batch


def test_tuning_table_ragged_schedule_validated(tmp_path):
    lib = _lib.load()
    for bad in ({"item_elems": 0}, {"waves": 2}, {"item_elems": "x"}, []):
        p = tmp_path / "r.json"
        p.write_text(json.dumps({"entries": [], "ragged": bad}))
        assert lib.tfft_load_tuning(str(p).encode()) == _lib.TFFT_EINVAL, bad
    p = tmp_path / "r.json"
    p.write_text(json.dumps({"entries": [], "ragged": {"item_elems": 16384, "waves": 3}}))
    try:
        assert lib.tfft_load_tuning(str(p).encode()) == 0
    finally:
        lib.tfft_ragged_set_schedule(0, 32768, 3)
        if os.path.exists(_lib.TUNING_PATH):
            lib.tfft_load_tuning(_lib.TUNING_PATH.encode())
