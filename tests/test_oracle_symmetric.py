"""Pins of the symmetric-storage oracle (uniform.expand_symmetric, Remark 4.4; no GPU).

The builder runs ACA on one block of each mirrored pair and takes V_sigma = conj(U_sigma),
so the general operator it returns is itself the symmetric one up to rounding.  The
expansion of the symmetric image (one block per mirrored pair) must therefore reproduce
the general operator's product to rounding, list exactly the general operator's blocks,
and give a matrix equal to its own transpose.  Plausible mistakes in the expansion (a
conjugate transpose instead of a transpose, a mirror left out, a diagonal block counted
twice) fail these pins, which the last test checks on planted copies.
"""
import numpy as np
import pytest

from conftest import operator, rel
from oracle import uniform
from paper_2405_15573_amd import builder, inputs

CASES = [("sphere", 2048, 0, 32), ("cube", 1300, 5, 32), ("ellipsoid", 1500, 4, 32), ("sphere", 60, 0, 32)]


def _pairs(rows, cols):
    return sorted(zip(np.asarray(rows).tolist(), np.asarray(cols).tolist()))


@pytest.mark.parametrize("surface,n,seed,leaf", CASES)
def test_expansion_lists_the_general_blocks(surface, n, seed, leaf):
    _, op = operator(surface=surface, n=n, seed=seed, leaf=leaf)
    sym = builder.symmetric_image(op)
    ex = uniform.expand_symmetric(sym)
    assert _pairs(ex["adm_row"], ex["adm_col"]) == _pairs(op.adm_row, op.adm_col)
    assert _pairs(ex["den_row"], ex["den_col"]) == _pairs(op.den_row, op.den_col)
    # one block of each mirrored pair is stored
    assert 2 * sym["adm_row"].size == op.nadm
    assert 2 * sym["den_row"].size - int(np.sum(sym["den_row"] == sym["den_col"])) == op.nden


@pytest.mark.parametrize("surface,n,seed,leaf", CASES)
def test_expansion_reproduces_the_general_product(surface, n, seed, leaf):
    cloud, op = operator(surface=surface, n=n, seed=seed, leaf=leaf)
    ex = uniform.expand_symmetric(builder.symmetric_image(op))
    x = inputs.make_rhs(cloud.n, 3, seed=seed + 40)
    assert rel(uniform.uh_mvp(ex, x), uniform.uh_mvp(vars(op), x)) < 1e-13


def test_expanded_matrix_is_symmetric(small_op):
    _, op = small_op
    a = uniform.assemble_uh(uniform.expand_symmetric(builder.symmetric_image(op)))
    assert np.linalg.norm(a - a.T) <= 1e-14 * np.linalg.norm(a)
    # complex-symmetric, not hermitian
    assert np.linalg.norm(a - a.conj().T) > 1e-3 * np.linalg.norm(a)


def _planted(sym, mistake):
    ex = uniform.expand_symmetric(sym)
    na = sym["adm_row"].size
    if mistake == "adjoint_S":
        S = ex["S"].copy()
        for b in range(na, 2 * na):
            t, s = int(ex["adm_row"][b]), int(ex["adm_col"][b])
            lt, ls = int(ex["rank_row"][t]), int(ex["rank_row"][s])
            o = int(ex["S_off"][b])
            S[o:o + lt * ls] = np.conj(S[o:o + lt * ls])
        ex["S"] = S
    elif mistake == "no_mirror":
        for k in ("adm_row", "adm_col", "S_off"):
            ex[k] = ex[k][:na]
    elif mistake == "adjoint_D":
        D = ex["D"].copy()
        nd = sym["den_row"].size
        for b in range(nd, ex["den_row"].size):
            t, s = int(ex["den_row"][b]), int(ex["den_col"][b])
            o = int(ex["D_off"][b])
            m = int(ex["size"][t]) * int(ex["size"][s])
            D[o:o + m] = np.conj(D[o:o + m])
        ex["D"] = D
    elif mistake == "diagonal_twice":
        d = np.nonzero(sym["den_row"] == sym["den_col"])[0][:1]
        for k in ("den_row", "den_col", "D_off"):
            ex[k] = np.concatenate([ex[k], ex[k][d]])
    elif mistake == "V_is_U":
        ex["V"] = sym["U"]
    return ex


@pytest.mark.parametrize("mistake", ["adjoint_S", "no_mirror", "adjoint_D", "diagonal_twice", "V_is_U"])
def test_pins_reject_planted_mistakes(small_op, mistake):
    cloud, op = small_op
    ex = _planted(builder.symmetric_image(op), mistake)
    x = inputs.make_rhs(cloud.n, 1, seed=77)
    assert rel(uniform.uh_mvp(ex, x), uniform.uh_mvp(vars(op), x)) > 1e-6
