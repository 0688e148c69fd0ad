"""CPU tests of the C ABI: the library loads, exports every symbol the header
declares, its host parameter math reproduces the paper's tables, and its
argument checks reject bad plans before touching a device."""
import math
import os
import re

import pytest

import oracle as O
from paper_1911_01377_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "useries.h")


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(useries_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = N.lib()
    declared = header_functions()
    assert declared, "no declarations parsed"
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(N.EXPORTED) == declared


def test_table2_roots():
    b, r0, w0, s0 = N.useries_solve_construction(N.USERIES_C1, 2.0)
    assert abs(r0 - 1.98925368390802627) < 1e-14 and abs(w0 - 0.994446492762232252) < 1e-14
    b, r0, w0, s0 = N.useries_solve_construction(N.USERIES_C0, 2.0)
    assert abs(r0 - 1.84309078551204634) < 1e-14 and w0 == 1.0
    b, r0, w0, s0 = N.useries_solve_construction(N.USERIES_C2_B2, 0.0)
    assert (b, r0, w0, s0) == (2.0, 2.39427106444012661, 0.892857784448501290, 1.02474173246377476)


@pytest.mark.parametrize("row,b,r0,w0,tol_r0,tol_w0", [
    (1, 1.62976708826776469, 2.75200266680234223, 1.00780697934380681, 1e-7, 1e-13),
    (2, 1.32070036405934420, 4.39145547116383425, 1.00188914114811980, 1e-6, 1e-11),
    (3, 1.21812525709410644, 5.63552881512711037, 1.00090146156033341, 1e-5, 1e-8)])
def test_table1_presets_and_tangential_roots(row, b, r0, w0, tol_r0, tol_w0):
    """Table 1 rows are C2 points where eq. 26 has a double root: the presets
    return the printed values; solving C1 at the printed b finds the
    tangential root.  A double root is ill-conditioned in FP64 (its position
    is fixed only to about sqrt(rounding / curvature)), and the curvature
    shrinks with M_b, so the third row is located to 1e-5 only."""
    pb, pr0, pw0, ps0 = N.useries_solve_construction(10 + row, 0.0)
    assert (pb, pr0, pw0, ps0) == (b, r0, w0, 1.0)
    _, sr0, sw0, _ = N.useries_solve_construction(N.USERIES_C1, b)
    assert abs(sr0 - r0) < tol_r0 * r0
    assert abs(sw0 - w0) < tol_w0


def test_solver_matches_oracle_off_table():
    for b in (1.4, 1.7, 1.9):
        _, r0, w0, _ = N.useries_solve_construction(N.USERIES_C1, b)
        orr, ow = O.solve_c1(b)
        assert abs(r0 - orr) < 1e-12 and abs(w0 - ow) < 1e-12


def test_eq33_and_nterms():
    sigma = 8.0 / 1.98925368390802627
    assert 1.5e-5 <= N.useries_eq33_bound(4, 2.0, sigma, 70.0) < 1.6e-5
    s9 = 9.0 / 1.98925368390802627
    assert N.useries_choose_nterms(2.0, s9, 24.0, 1e-8) == 3
    assert N.useries_choose_nterms(2.0, s9, 64.0, 1e-8) == 4
    assert N.useries_choose_nterms(2.0, s9, 100.0, 1e-8) == 5
    assert abs(N.useries_bsa_bound(2.0) - 2.289e-3) < 5e-7


def test_bad_arguments_are_rejected_before_any_device_call():
    box = (30.0, 30.0, 30.0)
    bad = [
        dict(box=box, r_c=15.0, b=2.0, grid=(32, 32, 32)),          # r_c >= L/2
        dict(box=box, r_c=9.0, b=1.0, grid=(32, 32, 32)),           # b <= 1
        dict(box=box, r_c=9.0, b=2.0, grid=(8, 32, 32)),            # grid < 2P
        dict(box=box, r_c=9.0, b=2.0, grid=(32, 32, 200)),          # grid > 128
        dict(box=(30.0, -1.0, 30.0), r_c=9.0, b=2.0, grid=(32, 32, 32)),
    ]
    for kw in bad:
        with pytest.raises(N.UseriesError) as e:
            N.useries_plan(kw["box"], kw["r_c"], kw["b"], 0.0, 0, kw["grid"])
        assert e.value.code == N.USERIES_EINVAL
    o = N.useries_default_opts()
    o.stencil_half = 9
    with pytest.raises(N.UseriesError):
        N.useries_plan(box, 9.0, 2.0, 0.0, 0, (32, 32, 32), o)
    with pytest.raises(N.UseriesError):
        N.useries_solve_construction(N.USERIES_C1, 0.5)
    with pytest.raises(N.UseriesError):
        N.useries_solve_construction(99, 2.0)
    assert N.useries_strerror(N.USERIES_EINVAL) == "invalid argument"


def test_default_opts():
    o = N.useries_default_opts()
    assert o.construction == N.USERIES_C1 and o.precision == N.USERIES_PLAIN_FP32
    assert math.isclose(o.nterms_tol, 1e-8)


# Known-answer vectors of Philox4x32-10 published with the generator
# (Salmon et al., SC 2011, Random123 distribution): counter, key -> output.
PHILOX_KAT = [
    ([0, 0, 0, 0], [0, 0], [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]),
    ([0xffffffff] * 4, [0xffffffff] * 2, [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]),
    ([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344], [0xa4093822, 0x299f31d0],
     [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1]),
]


@pytest.mark.parametrize("ctr,key,want", PHILOX_KAT)
def test_philox_known_answers(ctr, key, want):
    assert N.useries_philox4x32_10(ctr, key) == want


def test_server_arguments_are_rejected_before_any_device_call():
    for slots, prec, budget in ((0, N.USERIES_BF16X3, 1 << 30), (65, N.USERIES_BF16X3, 1 << 30),
                                (4, 7, 1 << 30), (4, N.USERIES_BF16X3, 1000)):
        with pytest.raises(N.UseriesError) as e:
            N.useries_server_create(budget, slots, prec)
        assert e.value.code == N.USERIES_EINVAL
    o = N.useries_server_default_opts()
    assert o.use_graph == 0 and o.inflight == 2 and o.poly_degree == 0 and o.b == 2.0
    o.inflight = 9
    with pytest.raises(N.UseriesError):
        N.useries_server_create(1 << 30, 4, N.USERIES_BF16X3, o)
    with pytest.raises(N.UseriesError) as e:
        N.useries_submit(None, N.useries_request())
    assert e.value.code == N.USERIES_EINVAL
