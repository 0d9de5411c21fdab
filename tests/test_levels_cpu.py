"""Rows of one level commute (CPU, FP64 oracle).

The sparse kernel finishes slow frames level by level, running the rows of a level at
once.  This rests on a property of the sequential row order of Sec. IV-C (and of layered
BP, Sec. II-B): a row reads and writes only messages of its own variables, so two rows
with no common variable can be swapped.  Here the oracle decodes each code twice: with its
rows in index order, and with the rows permuted into the level order the library computes
(cbp_code_levels), which keeps every pair of rows with a common variable in order.  Hard
decisions, sweep counts and every message (mapped through the permutation) must be equal
bit for bit in FP64.  A permutation that breaks the order of two rows with a common variable
(the check that the comparison can fail) changes the messages.
"""
import types

import numpy as np
import pytest

import oracle
from paper_2305_05286_amd import cbp
from paper_2305_05286_amd.workload import get_code, make_frames


def permuted(code, rows):
    """The code with its rows in the given order (each row's columns unchanged), and the
    new position of every edge of the original code."""
    rp, ci = code.row_ptr, code.col_idx
    new_rp = [0]
    new_ci = []
    edge_pos = np.empty(code.E, np.int64)
    for i in rows:
        for e in range(rp[i], rp[i + 1]):
            edge_pos[e] = len(new_ci)
            new_ci.append(ci[e])
        new_rp.append(len(new_ci))
    c = types.SimpleNamespace(M=code.M, N=code.N, E=code.E, row_ptr=np.array(new_rp, np.int32),
                              col_idx=np.array(new_ci, np.int32))
    return c, edge_pos


CASES = [("reg36_n96", 1.5, 400), ("qc_t64s", 1.5, 200), ("peg_irr_n2048", 1.4, 24)]


@pytest.mark.parametrize("name,ebn0,frames", CASES)
@pytest.mark.parametrize("algo", ["cbp", "cbp_nms", "lbp", "fbp"])
def test_level_order_equals_index_order(name, ebn0, frames, algo):
    code = get_code(name)
    _, _, rows = cbp.Code.from_workload(code).levels()
    lv, edge_pos = permuted(code, rows)
    llr, _ = make_frames(code, ebn0, frames, key=(43,))
    for stop_rule, max_iter in ((0, 60), (2, 9)):
        a = oracle.decode(code, llr, max_iter, algo, stop_rule=stop_rule, dump_sweep=3, ndump=frames)
        b = oracle.decode(lv, llr, max_iter, algo, stop_rule=stop_rule, dump_sweep=3, ndump=frames)
        assert np.array_equal(a["iters"], b["iters"])
        assert np.array_equal(a["bits"], b["bits"])
        seen = ~np.isnan(a["R"][:, 0])
        assert seen.any()
        assert np.array_equal(a["R"][seen], b["R"][seen][:, edge_pos])
        assert np.array_equal(a["Lam"][seen], b["Lam"][seen])
        if algo.startswith("cbp"):
            assert np.array_equal(a["Q"][seen], b["Q"][seen])
            assert np.array_equal(a["Om"][seen], b["Om"][seen][:, np.argsort(rows)])


def test_breaking_the_order_is_detected():
    code = get_code("reg36_n96")
    _, _, rows = cbp.Code.from_workload(code).levels()
    rows = list(rows)
    # move the last row, which shares a variable with an earlier one, to the front
    last = rows.pop()
    bad, edge_pos = permuted(code, [last] + rows)
    llr, _ = make_frames(code, 1.5, 200, key=(43,))
    a = oracle.decode(code, llr, 9, "cbp", stop_rule=2, dump_sweep=3, ndump=200)
    b = oracle.decode(bad, llr, 9, "cbp", stop_rule=2, dump_sweep=3, ndump=200)
    assert not np.array_equal(a["R"], b["R"][:, edge_pos])
