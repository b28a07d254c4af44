"""The oracle's block loops run on several threads with bit-identical results: every
block's arithmetic is the same whichever thread runs it, and the only quantities
combined across blocks are exact (integer counts, maxima)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2108_12240_amd import inputs as I
from tests import cases


def _run(params, blocks, prim, threads, steps=2):
    O.set_threads(threads)
    try:
        Og = O.OracleGrid(params, blocks)
        U, P = Og.run(prim, steps)
        # a standalone inversion with failing cells, then the centred time step
        Ui = U.copy()
        idx = Og.interior_index()
        sel = idx[::29]
        Ui[4, sel] = -0.5 * Ui[0, sel]
        Pi = P.copy()
        fail = np.zeros(Og.ncp, dtype=np.int8)
        Og.con2prim(Ui, Pi, fail)
        dt = Og.compute_dt(P)
        return U, P, Pi, fail, Og.stats(), dt
    finally:
        O.set_threads(1)


CASES = [
    ("torus_32", lambda: I.case_torus(2, n=32)),
    ("amr_like_24", lambda: I.case4(nblocks=24, n0=48)),
    ("torus_entropy", lambda: I.with_entropy(I.case_torus(2, n=(32, 16, 16)))),
]


@pytest.mark.parametrize("name,make", CASES)
def test_threads_are_bit_identical(name, make):
    c = make()
    one = _run(c.params, c.blocks, c.prim, 1)
    many = _run(c.params, c.blocks, c.prim, 4)
    for a, b in zip(one[:4], many[:4]):
        assert np.array_equal(a, b)
    assert one[4] == many[4]
    assert one[5] == many[5]
    assert one[4]["c2p_fail"] + one[4]["c2p_backup"] > 0


def test_threads_on_a_block_tree_are_bit_identical():
    params, blocks, prim = cases.flat_tree_case(levels=2, ndim=2)
    one = _run(params, blocks, prim, 1)
    many = _run(params, blocks, prim, 3)
    for a, b in zip(one[:4], many[:4]):
        assert np.array_equal(a, b)
    assert one[4] == many[4]


def test_thread_count_is_reported():
    O.set_threads(3)
    try:
        assert O.get_threads() == 3
    finally:
        O.set_threads(1)
    assert O.get_threads() == 1
