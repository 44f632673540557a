"""The lane exchanges of the register bitonic sort (lms_device.h,
xor_lanes_i32): each partner distance J = 1, 2, 4, 8 is built from gfx9 DPP
row permutes, whose lane maps are written out here from their definitions
(a quad permute selects within groups of 4 lanes, the row mirror reverses
each row of 16, the half-row mirror each half row of 8). A composition must
give every lane l the value of lane l ^ J, for all 64 lanes, and the header
must use exactly the controls checked here."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_1510_01041_amd", "csrc", "lms_device.h")


def quad_perm(ctrl):
    """Source lane of each lane for a quad_perm control (2 bits per lane of a quad)."""
    sel = [(ctrl >> (2 * i)) & 3 for i in range(4)]
    return [(l & ~3) | sel[l & 3] for l in range(64)]


def row_mirror():
    return [(l & ~15) | (15 - (l & 15)) for l in range(64)]


def row_half_mirror():
    return [(l & ~7) | (7 - (l & 7)) for l in range(64)]


def dpp(ctrl):
    if ctrl < 0x100:
        return quad_perm(ctrl)
    return {0x140: row_mirror(), 0x141: row_half_mirror()}[ctrl]


def apply(src_map, values):
    """The result of a DPP move: lane l takes values[src_map[l]]."""
    return [values[src_map[l]] for l in range(64)]


def controls():
    text = open(HEADER).read()
    names = ["kQuadXor1", "kQuadXor2", "kQuadReverse", "kRowMirror", "kRowHalfMirror"]
    out = {}
    for n in names:
        m = re.search(n + r"\s*=\s*(0x[0-9A-Fa-f]+)", text)
        assert m, n
        out[n] = int(m.group(1), 16)
    return out


def test_controls_give_xor_partners():
    c = controls()
    lanes = list(range(64))
    one = apply(dpp(c["kQuadXor1"]), lanes)
    two = apply(dpp(c["kQuadXor2"]), lanes)
    # J = 4: the half-row mirror first, then the quad reversal
    four = apply(dpp(c["kQuadReverse"]), apply(dpp(c["kRowHalfMirror"]), lanes))
    # J = 8: the row mirror first, then the half-row mirror
    eight = apply(dpp(c["kRowHalfMirror"]), apply(dpp(c["kRowMirror"]), lanes))
    for j, got in ((1, one), (2, two), (4, four), (8, eight)):
        assert got == [l ^ j for l in lanes], j


def test_check_catches_wrong_controls():
    """The lane maps are XOR maps within their groups (a quad reversal is
    l ^ 3, a half-row mirror l ^ 7, a row mirror l ^ 15), so the check above
    fails for a plausible slip: the row mirror in place of the half-row
    mirror gives l ^ 12 for J = 4, a single half-row mirror l ^ 7."""
    c = controls()
    lanes = list(range(64))
    slip4 = apply(dpp(c["kQuadReverse"]), apply(dpp(c["kRowMirror"]), lanes))
    assert slip4 == [l ^ 12 for l in lanes]
    assert apply(dpp(c["kRowHalfMirror"]), lanes) == [l ^ 7 for l in lanes]
    assert apply(dpp(c["kQuadXor2"]), lanes) != [l ^ 1 for l in lanes]
