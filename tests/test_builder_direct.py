"""Direct UH construction (builder.build_uniform_direct: Algs. 3-4 of section 4.3 with the
per-block locks of section 4.4, symmetric form of Remark 4.4), against the two-phase builder
(H-matrix first, then Alg. 2) on the same clouds.  No GPU.

* The same blocks are approximated the same way, so the ranks of every cluster and block
  are those of the two-phase builder, and the product agrees to 1e-12.
* The result does not depend on the number of threads or on which thread approximates a
  block (bitwise).
* The pins the two-phase builder meets hold (orthonormal bases, optimal couplings, Thm 5.1,
  Alg. 1's ranks and projection error), checked with the two-phase builder's H factors,
  which the direct construction never holds whole.
* The block factors held at once stay well below the H form's (the point of the direct
  construction): at most half of them on these clouds.
"""
import numpy as np
import pytest

import test_builder as tb
from conftest import rel
from oracle import uniform
from paper_2405_15573_amd import builder, inputs

CASES = [("sphere", 2048, 32), ("ellipsoid", 3500, 64), ("cube", 3000, 32)]


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def pair(request):
    surface, n, leaf = request.param
    cloud = inputs.make_cloud(surface, n, seed=0)
    two = builder.build_operator(cloud, leaf=leaf, eta=1.0, eps_aca=1e-6, eps_comp=1e-6)
    direct = builder.build_uniform_direct(cloud, leaf=leaf, eta=1.0, eps_aca=1e-6, eps_comp=1e-6, threads=4)
    return cloud, two, direct


def test_same_operator_as_two_phase(pair):
    cloud, two, direct = pair
    assert np.array_equal(direct.rank_row, two.rank_row)
    assert np.array_equal(direct.adm_rank, two.adm_rank)
    assert np.array_equal(direct.adm_row, two.adm_row) and np.array_equal(direct.adm_col, two.adm_col)
    assert np.array_equal(direct.D, two.D)
    x = inputs.make_rhs(cloud.n, 2, seed=3)
    assert rel(uniform.uh_mvp(vars(direct), x), uniform.uh_mvp(vars(two), x)) <= 1e-12
    assert rel(uniform.uh_mvp(uniform.assemble_factored(vars(direct), "all"), x),
               uniform.uh_mvp(vars(direct), x)) <= 1e-12


def test_independent_of_threads(pair):
    cloud, two, direct = pair
    one = builder.build_uniform_direct(cloud, leaf=int(direct.leaf), eta=1.0, eps_aca=1e-6, eps_comp=1e-6,
                                       threads=1)
    for k in ("U", "S", "SX", "SY", "rank_row", "adm_rank", "sv_dropped", "sv_tail"):
        assert np.array_equal(getattr(one, k), getattr(direct, k)), k


def test_builder_pins_hold(pair):
    cloud, two, direct = pair
    d = vars(direct).copy()
    for k in ("X", "Y", "X_off", "Y_off"):   # the H factors of the same blocks, for the pins only
        d[k] = getattr(two, k)
    op = builder.HostOperator(**{k: d[k] for k in builder.HostOperator.__dataclass_fields__})
    for fn in (tb.test_orthogonal_bases_and_conjugate_symmetry, tb.test_couplings_are_optimal,
               tb.test_theorem_5_1_and_frobenius_identity, tb.test_algorithm_1_and_2_give_the_same_basis):
        fn((cloud, op))


def test_peak_factor_memory(pair):
    cloud, two, direct = pair
    t = direct.timings
    total_h = 16 * (two.X.size + two.Y.size) / 2   # one block of each mirrored pair is approximated
    assert t["total_factor_bytes"] == pytest.approx(total_h, rel=1e-12)
    assert t["peak_factor_bytes"] <= 0.5 * t["total_factor_bytes"]
