"""Worked example printed in the paper: the RTCF_2 layout (Sec. 3.5)."""
import os

import numpy as np

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def load_rtcf2():
    rows = []
    with open(os.path.join(HERE, "golden", "rtcf2_dofs.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                a = line.split()
                rows.append((int(a[0]), int(a[1]), int(a[2]), int(a[3]), float(a[4]), float(a[5])))
    return rows


def test_rtcf2_concatenated_numbering():
    """The oracle's concatenation of row-major blocks reproduces the paper's 12 DOF numbers."""
    ext = [[3, 2], [2, 3]]
    rows = load_rtcf2()
    assert len(rows) == 12
    for num, blk, ia, ib, _, _ in rows:
        assert oracle.concat_index(ext, blk, [ia - 1, ib - 1]) + 1 == num


def test_rtcf2_node_sets():
    """P_2 factors sit on the 3 GLL points {0, 0.5, 1}; dP_1 factors on the 2 GL points
    (0.211, 0.789): the node-set reading of Sec. 2.5 matches the figure."""
    gll = oracle.gll_rule(3)[0]
    gl = oracle.gl_rule(2)[0]
    for num, blk, ia, ib, x, y in load_rtcf2():
        if blk == 0:
            got = (gll[ia - 1], gl[ib - 1])
        else:
            got = (gl[ia - 1], gll[ib - 1])
        assert abs(got[0] - x) < 5e-4 and abs(got[1] - y) < 5e-4
