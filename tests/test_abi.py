"""C ABI on the CPU: the library loads, exports every declared symbol, and its
host-only functions (descriptor validation, partition bounds, flop model,
workspace size) behave.  No compute calls: there is no GPU here.
"""
import ctypes as C
import os
import re

import pytest

from paper_2601_04904_amd import _lib
from paper_2601_04904_amd._lib import make_desc, BT_OK, BT_ERR_INVALID

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in ("bt_si_sq.h", "bt_si_sq_diag.h"):
        txt = open(os.path.join(ROOT, "include", h)).read()
        names |= set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\**\s+\**(bt_si_sq_[a-z_0-9]+)\s*\(", txt, re.M))
    return names


def test_header_parses():
    names = declared_functions()
    assert {"bt_si_sq_create", "bt_si_sq_factor", "bt_si_sq_selected_solve",
            "bt_si_sq_destroy", "bt_si_sq_workspace_bytes"} <= names


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(_lib.EXPORTED) == declared_functions()


def test_struct_layout_matches_header(tmp_path):
    """The ctypes structs have the size and field offsets the C compiler gives
    the header's structs (a small C program built against include/)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    src = tmp_path / "layout.c"
    fields = [f for f, _ in _lib.bt_desc._fields_]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "bt_si_sq.h"', "int main(void) {",
             '  printf("%zu\\n", sizeof(bt_desc));']
    lines += [f'  printf("%zu\\n", offsetof(bt_desc, {f}));' for f in fields]
    lines += ['  printf("%zu\\n", sizeof(bt_blocks));', "  return 0; }"]
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", inc, str(src), "-o", str(exe)], check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                           text=True).stdout.split()]
    assert vals[0] == C.sizeof(_lib.bt_desc)
    assert vals[1:1 + len(fields)] == [getattr(_lib.bt_desc, f).offset for f in fields]
    assert vals[-1] == C.sizeof(_lib.bt_blocks) == 6 * 8


def _bounds(n, b, a, P, bounds=None):
    d = make_desc(n, b, a, P, bounds)
    out = (C.c_int32 * (P + 1))()
    st = _lib.lib().bt_si_sq_partition_bounds(C.byref(d), out)
    return st, list(out)


def test_auto_bounds_balance():
    st, bnd = _bounds(64, 512, 0, 8)
    assert st == BT_OK
    assert bnd == [0, 14, 20, 26, 32, 38, 44, 50, 64]
    st, bnd = _bounds(128, 384, 512, 16)
    assert st == BT_OK and bnd[0] == 0 and bnd[-1] == 128
    sizes = [y - x for x, y in zip(bnd, bnd[1:])]
    assert all(s >= 2 for s in sizes[1:-1]) and sizes[0] >= 1 and sizes[-1] >= 1


@pytest.mark.parametrize("n,b,a,P,bounds", [
    (0, 4, 0, 1, None), (4, 0, 0, 1, None), (4, 4, -1, 1, None), (4, 4, 0, 0, None),
    (6, 4, 0, 3, [0, 2, 3, 6]),      # middle partition of one block
    (6, 4, 0, 2, [0, 3, 5]),         # does not end at n
    (6, 4, 0, 2, [1, 3, 6]),         # does not start at 0
    (4, 2000, 0, 1, None),           # block size above the supported maximum
])
def test_invalid_descriptors(n, b, a, P, bounds):
    d = make_desc(n, b, a, P, bounds)
    assert _lib.lib().bt_si_sq_workspace_bytes(C.byref(d)) == 0
    out = (C.c_int32 * (max(P, 1) + 1))()
    assert _lib.lib().bt_si_sq_partition_bounds(C.byref(d), out) == BT_ERR_INVALID
    h = C.c_void_p()
    assert _lib.lib().bt_si_sq_create(C.byref(d), None, C.byref(h)) == BT_ERR_INVALID
    assert h.value is None
    assert len(_lib.lib().bt_si_sq_last_error(None)) > 0


@pytest.mark.parametrize("n,b,a,P", [(40, 8, 12, 17), (48, 6, 10, 24), (80, 4, 3, 40)])
def test_many_partitions_with_arrow_plan(n, b, a, P):
    """More than 16 partitions with an arrow tip: the tip sum has P + 1 inputs,
    more than one block-sum operation takes, so it is chained; the plan
    compiles (a sum with too many inputs would make the dry run fail)."""
    d = make_desc(n, b, a, P)
    assert _lib.lib().bt_si_sq_workspace_bytes(C.byref(d)) > 0, _lib.lib().bt_si_sq_last_error(None)


def _flops(n, b, a, P, bounds=None):
    d = make_desc(n, b, a, P, bounds)
    ex, us = C.c_double(), C.c_double()
    assert _lib.lib().bt_si_sq_flops(C.byref(d), C.byref(ex), C.byref(us)) == BT_OK
    return ex.value, us.value


def step(dk, Ns):
    D = sum(Ns)
    f = 8 * dk ** 3                              # inverse
    f += 8 * dk * dk * D                         # T_u
    f += 8 * D * D * dk                          # A updates
    f += 16 * dk ** 3                            # S_B
    f += 8 * dk * dk * D                         # W_u
    f += 3 * 8 * D * D * dk                      # B updates
    f += 8 * dk * dk * D + 8 * D * D * dk        # tau, rho
    f += 8 * D * dk * dk + 8 * dk * D * D        # X_uk, X_kv
    f += 8 * D * dk * dk                         # X_kk
    f += 8 * D * D * dk * 2                      # GB, BG
    f += 2 * 8 * D * dk * dk                     # Y21
    f += 2 * 8 * dk * dk * D + 8 * dk * D * D    # L_kv (Y12 + update)
    f += 8 * D * D * dk                          # L_uk
    f += 2 * 8 * dk * dk * D                     # L_kk
    return f


@pytest.mark.parametrize("n,b,a", [(1, 8, 0), (2, 8, 0), (16, 32, 0), (64, 512, 0), (5, 7, 3),
                                   (128, 384, 512)])
def test_flop_model_sequential(n, b, a):
    """Sequential SI+SQ op list: per eliminated block with D = sum of its neighbour sizes,
    inverse 8b^3 + products 8(2b^3 + 11Db^2 + 10D^2 b) (counted independently here)."""
    ex, us = _flops(n, b, a, 1)
    assert ex == us

    ref = 0
    for k in range(n):
        Ns = ([b] if k + 1 < n else []) + ([a] if a else [])
        ref += step(b, Ns)
    if a:
        ref += step(a, [])
    assert ex == pytest.approx(ref, rel=1e-12)
    if a == 0:
        assert ex == pytest.approx(192 * (n - 1) * b ** 3 + 24 * b ** 3, rel=1e-12)


def test_flop_model_partitioned_executes_more():
    ex, us = _flops(64, 512, 0, 8)
    assert us == pytest.approx(192 * 63 * 512 ** 3 + 24 * 512 ** 3)
    assert 1.5 < ex / us < 1.8


def _partitioned_neighbour_counts(n, bounds, Q):
    """Neighbour counts of every elimination of the partitioned scheme on a BT
    matrix (Sec. III-B): first partition top-down and last bottom-up with one
    neighbour, middle ones against their top block with two; the 2(P - 1)
    kept blocks are then solved by the same scheme with Q parts while they
    number at least four (Q < 2: sequentially)."""
    P = len(bounds) - 1
    counts = []
    for p in range(P):
        s, e = bounds[p], bounds[p + 1]
        counts += [1] * (e - s - 1) if p in (0, P - 1) else [2] * (e - s - 2)
    m = 2 * (P - 1)
    while m >= 4 and Q >= 2:
        q = max(2, min(Q, m // 2))
        for p in range(q):
            s, e = p * m // q, (p + 1) * m // q - 1
            counts += [1] * (e - s) if p in (0, q - 1) else [2] * (e - s - 1)
        m = 2 * (q - 1)
    return counts + [1] * (m - 1) + [0]


@pytest.mark.parametrize("n,P,Q", [(64, 16, 0), (64, 16, 1), (64, 16, 3), (64, 16, 4), (64, 16, 9),
                                   (40, 20, 1024), (12, 3, 5), (6, 3, 3), (10, 5, 4), (14, 7, 3)])
def test_flop_model_recursive_reduced_solve(n, P, Q):
    from paper_2601_04904_amd.solver import partition_bounds
    b = 16
    bounds = partition_bounds(n, b, 0, P)
    d = make_desc(n, b, 0, P, bounds, reduced_parts=Q)
    ex, us = C.c_double(), C.c_double()
    assert _lib.lib().bt_si_sq_flops(C.byref(d), C.byref(ex), C.byref(us)) == BT_OK
    counts = _partitioned_neighbour_counts(n, bounds, 2 if Q == 0 else Q)
    assert len(counts) == n
    assert ex.value == pytest.approx(sum(step(b, [b] * c) for c in counts), rel=1e-12)
    assert us.value == pytest.approx(192 * (n - 1) * b ** 3 + 24 * b ** 3, rel=1e-12)


@pytest.mark.parametrize("Q", [-1, 1025])
def test_reduced_parts_out_of_range_rejected(Q):
    d = make_desc(16, 8, 0, 4, reduced_parts=Q)
    assert _lib.lib().bt_si_sq_workspace_bytes(C.byref(d)) == 0
    h = C.c_void_p()
    assert _lib.lib().bt_si_sq_create(C.byref(d), None, C.byref(h)) == BT_ERR_INVALID
    msg = _lib.lib().bt_si_sq_last_error(None)
    assert "reduced_parts" in (msg.decode() if isinstance(msg, bytes) else msg)


def test_workspace_bytes_scales():
    d1 = make_desc(16, 32, 0, 1)
    d2 = make_desc(64, 512, 0, 1)
    w1 = _lib.lib().bt_si_sq_workspace_bytes(C.byref(d1))
    w2 = _lib.lib().bt_si_sq_workspace_bytes(C.byref(d2))
    assert 0 < w1 < w2
    # dominated by O(n b^2) block storage
    assert w2 < 40 * 64 * 512 * 512 * 16


def test_tune_table_roundtrip_and_validation():
    from paper_2601_04904_amd import solver as S, _lib
    saved = S.tune_table()
    assert len(saved) == _lib.BT_TUNE_ENTRIES
    assert all(-1 <= v < _lib.BT_TILE_SHAPES for v in saved)
    try:
        t = [(i % (_lib.BT_TILE_SHAPES + 1)) - 1 for i in range(_lib.BT_TUNE_ENTRIES)]
        S.set_tune_table(t)
        assert S.tune_table() == t
        bad = list(t)
        bad[5] = _lib.BT_TILE_SHAPES
        with pytest.raises(S.BTError):
            S.set_tune_table(bad)
        assert S.tune_table() == t          # a rejected write changes nothing
        with pytest.raises(ValueError):
            S.set_tune_table(t[:-1])
    finally:
        S.set_tune_table(saved)


def test_header_flag_values_match_binding():
    from paper_2601_04904_amd import _lib
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with open(os.path.join(root, "include", "bt_si_sq.h")) as f:
        text = f.read()
    flags = dict(re.findall(r"#define (BT_[A-Z_]+) (0x[0-9a-f]+)u", text))
    assert set(flags) == {"BT_DIAG_ONLY", "BT_PLAIN", "BT_GRAPH", "BT_SIGMA_ANTIHERMITIAN", "BT_FUSED"}
    for name, val in flags.items():
        assert getattr(_lib, name) == int(val, 16), name
    nums = dict(re.findall(r"#define (BT_TILE_SHAPES|BT_TUNE_SIZE_CLASSES|BT_TUNE_WORK_CLASSES) (\d+)", text))
    for name, val in nums.items():
        assert getattr(_lib, name) == int(val), name


@pytest.mark.parametrize("n,b,a", [(1, 8, 0), (16, 32, 0), (64, 512, 0), (5, 7, 3), (128, 384, 512)])
def test_flop_model_antihermitian(n, b, a):
    """With BT_SIGMA_ANTIHERMITIAN the sequential op list drops, per eliminated
    block, the B-update term B_uk T_u^H (diagonal pairs), the three products
    of every second off-diagonal pair and the k-row products BG_v and
    S BG_v - S_B rho_v^H (counted independently here); `useful` stays the
    general count."""
    from paper_2601_04904_amd import solver as S
    ex, us = S.flops(n, b, a, flags=_lib.BT_SIGMA_ANTIHERMITIAN)
    ex0, us0 = S.flops(n, b, a)
    assert us == us0 == ex0

    def saved(dk, Ns):
        D = sum(Ns)
        f = sum(8 * d * d * dk for d in Ns)                                   # diagonal pairs: one term
        f += sum(3 * 8 * Ns[i] * Ns[j] * dk for i in range(len(Ns)) for j in range(i))   # (v, u), v > u
        f += 8 * D * D * dk                                                     # BG
        f += 2 * 8 * dk * dk * D                                                # Y12
        return f

    ref = 0
    for k in range(n):
        Ns = ([b] if k + 1 < n else []) + ([a] if a else [])
        ref += saved(b, Ns)
    assert ex == pytest.approx(ex0 - ref, rel=1e-12)
    if a == 0 and n > 1:
        assert ex == pytest.approx(160 * (n - 1) * b ** 3 + 24 * b ** 3, rel=1e-12)


@pytest.mark.parametrize("opA,opB,big", [(0, 0, "A"), (1, 0, "A"), (0, 1, "B"), (0, 0, "B")])
def test_diag_gemm_rejects_operands_past_32bit_offsets(opA, opB, big):
    """The product kernel addresses each operand with 32-bit byte offsets, so
    the diagnostic entry refuses an operand whose stored extent reaches 2 GiB.
    The check runs before any device call (the pointers are never touched)."""
    L = _lib.lib()
    one = (C.c_double * 2)(1.0, 0.0)
    zero = (C.c_double * 2)(0.0, 0.0)
    m = n = k = 64
    huge = 1 << 25                       # 64 rows x 2^25 elements x 16 B > 2 GiB
    lda = huge if big == "A" else 64
    ldb = huge if big == "B" else 64
    dummy = C.c_void_p(16)
    st = L.bt_si_sq_diag_gemm(m, n, k, one, dummy, lda, opA, dummy, ldb, opB,
                              zero, None, 64, dummy, 64, 0, -1, None)
    assert st == BT_ERR_INVALID
    assert b"2 GiB" in L.bt_si_sq_last_error(None)


def test_noalloc_inverse_rejects_requests_beyond_its_scratch():
    """The allocation-free inverse checks its fixed scratch size on the host,
    before any device call: too many or too large matrices are refused."""
    L = _lib.lib()
    cap = L.bt_si_sq_diag_inverse_noalloc_max_bytes()
    assert cap == 64 << 20
    fake = C.c_void_p(1 << 40)           # never dereferenced: the call returns first
    bad = C.c_int32(0)
    # 1024 x 1024 complex: 16 MiB each, four do not fit with their other scratch
    assert L.bt_si_sq_diag_inverse_noalloc(fake, fake, 1024, 4, C.byref(bad), None) == BT_ERR_INVALID
    assert b"scratch" in L.bt_si_sq_last_error(None)
    assert L.bt_si_sq_diag_inverse_noalloc(fake, fake, 1025, 1, C.byref(bad), None) == BT_ERR_INVALID
    assert L.bt_si_sq_diag_inverse_noalloc(fake, fake, 64, -1, C.byref(bad), None) == BT_ERR_INVALID
    assert L.bt_si_sq_diag_inverse_noalloc(fake, fake, 64, 0, C.byref(bad), None) == BT_OK


def test_diag_only_flop_model_and_mixed_rejection():
    """BT_DIAG_ONLY drops, per sequential BT step, the two products whose
    results nothing reads (X^R_{k,k+1} and X^<_{k+1,k}): 22 instead of 24
    b^3 units per step plus the last step's 3.  With BT_MIXED it is refused."""
    from paper_2601_04904_amd import _lib as LB
    L = _lib.lib()
    for n, b in [(16, 32), (5, 7), (64, 512)]:
        d = LB.make_desc(n, b, 0, 1, None, flags=LB.BT_DIAG_ONLY)
        ex, us = C.c_double(), C.c_double()
        assert L.bt_si_sq_flops(C.byref(d), C.byref(ex), C.byref(us)) == 0
        assert ex.value == pytest.approx(8.0 * b ** 3 * (22 * (n - 1) + 3), rel=1e-12)
        assert us.value == ex.value
    d = LB.make_desc(8, 16, 0, 1, None, precision=LB.BT_MIXED, flags=LB.BT_DIAG_ONLY)
    assert L.bt_si_sq_workspace_bytes(C.byref(d)) == 0
    assert b"BT_DIAG_ONLY" in L.bt_si_sq_last_error(None)


def test_fused_flag_limits():
    """BT_FUSED: every diagonal block and the tip at most 64, FP64, no
    BT_PLAIN."""
    from paper_2601_04904_amd import _lib as LB
    L = _lib.lib()
    ok = [LB.make_desc(16, 32, 0, 1, None, flags=LB.BT_FUSED),
          LB.make_desc(9, 64, 64, 3, None, flags=LB.BT_FUSED | LB.BT_DIAG_ONLY),
          LB.make_desc(5, 0, 16, 1, None, flags=LB.BT_FUSED, sizes=[8, 64, 3, 40, 1])]
    for d in ok:
        assert L.bt_si_sq_workspace_bytes(C.byref(d)) > 0, L.bt_si_sq_last_error(None)
    bad = [LB.make_desc(16, 65, 0, 1, None, flags=LB.BT_FUSED),
           LB.make_desc(16, 32, 65, 1, None, flags=LB.BT_FUSED),
           LB.make_desc(4, 0, 0, 1, None, flags=LB.BT_FUSED, sizes=[8, 65, 3, 4]),
           LB.make_desc(16, 32, 0, 1, None, precision=LB.BT_MIXED, flags=LB.BT_FUSED),
           LB.make_desc(16, 32, 0, 1, None, flags=LB.BT_FUSED | LB.BT_PLAIN)]
    for d in bad:
        assert L.bt_si_sq_workspace_bytes(C.byref(d)) == 0
        assert b"BT_FUSED" in L.bt_si_sq_last_error(None)


def test_block_sizes_descriptor():
    """Per-block sizes (Sec. II-A): the executed flops of the sequential sweep
    equal sum_k 8(3 b_k^3 + 11 D_k b_k^2 + 10 D_k^2 b_k) with D_k the total size
    of block k's remaining neighbours; equal sizes give the uniform results;
    cost-model bounds are admissible; bad sizes are refused."""
    import random
    from paper_2601_04904_amd import _lib as LB
    L = _lib.lib()
    rng = random.Random(11)
    for _ in range(5):
        n = rng.randint(2, 12)
        sizes = [rng.randint(1, 40) for _ in range(n)]
        a = rng.choice([0, 7])
        d = LB.make_desc(n, 0, a, 1, None, sizes=sizes)
        ex, us = C.c_double(), C.c_double()
        assert L.bt_si_sq_flops(C.byref(d), C.byref(ex), C.byref(us)) == BT_OK
        want = 0.0
        for k in range(n):
            Dk = (sizes[k + 1] if k + 1 < n else 0) + a
            b = sizes[k]
            want += 8.0 * (3 * b ** 3 + 11 * Dk * b * b + 10 * Dk * Dk * b)
        want += 8.0 * 3 * a ** 3
        assert ex.value == want
    # equal sizes: same flops, bounds and workspace as the uniform descriptor
    for P in (1, 3):
        du = make_desc(20, 64, 16, P)
        dv = LB.make_desc(20, 0, 16, P, None, sizes=[64] * 20)
        assert L.bt_si_sq_workspace_bytes(C.byref(du)) == L.bt_si_sq_workspace_bytes(C.byref(dv))
        bu, bv = (C.c_int32 * (P + 1))(), (C.c_int32 * (P + 1))()
        assert L.bt_si_sq_partition_bounds(C.byref(du), bu) == BT_OK
        assert L.bt_si_sq_partition_bounds(C.byref(dv), bv) == BT_OK
        assert list(bu) == list(bv)
    # uneven cost-model bounds: first/last partitions >= 1 block, middles >= 2
    from paper_2601_04904_amd.synth import ramp_sizes
    sz = ramp_sizes(48, 256, 512, 4)
    for P in (2, 4, 8, 16):
        d = LB.make_desc(48, 0, 256, P, None, sizes=sz)
        out = (C.c_int32 * (P + 1))()
        assert L.bt_si_sq_partition_bounds(C.byref(d), out) == BT_OK
        bd = list(out)
        assert bd[0] == 0 and bd[-1] == 48
        parts = [bd[p + 1] - bd[p] for p in range(P)]
        assert parts[0] >= 1 and parts[-1] >= 1 and all(x >= 2 for x in parts[1:-1])
    for bad in ([4, 0, 4], [4, 1025, 4]):
        d = LB.make_desc(3, 0, 0, 1, None, sizes=bad)
        assert L.bt_si_sq_workspace_bytes(C.byref(d)) == 0
        assert b"block_sizes" in L.bt_si_sq_last_error(None)


def test_batch_create_in_rejects_bad_workspace_before_any_device_call():
    """bt_si_sq_batch_create_in checks the caller's workspace on the host:
    null, too small or not 256-byte aligned is BT_ERR_INVALID (the fake
    addresses are never dereferenced)."""
    from paper_2601_04904_amd import _lib as LB
    L = _lib.lib()
    d = make_desc(12, 32, 8, 2)
    need = L.bt_si_sq_batch_workspace_bytes(1, C.byref(d))
    assert need > 0 and need == L.bt_si_sq_workspace_bytes(C.byref(d))
    h = C.c_void_p()
    assert L.bt_si_sq_batch_create_in(1, C.byref(d), None, None, need, C.byref(h)) == BT_ERR_INVALID
    assert L.bt_si_sq_batch_create_in(1, C.byref(d), None, C.c_void_p(1 << 40), need - 1,
                                      C.byref(h)) == BT_ERR_INVALID
    assert b"smaller" in L.bt_si_sq_last_error(None)
    assert L.bt_si_sq_batch_create_in(1, C.byref(d), None, C.c_void_p((1 << 40) + 64), need,
                                      C.byref(h)) == BT_ERR_INVALID
    assert b"aligned" in L.bt_si_sq_last_error(None)
    assert not h.value
