"""Pins of the oracle's storage rounding (oracle/precision.py) against fixed values,
the unit roundoff of each format, and an independent library conversion."""
import numpy as np
import pytest

from oracle import precision


def test_bf16_fixed_values_and_ties_to_even():
    one = 1.0
    cases = [
        (1.0, 1.0),
        (-2.5, -2.5),                       # exactly representable
        (one + 2.0**-8, 1.0),               # halfway between 1 and 1 + 2^-7: the even neighbour is 1
        (one + 3 * 2.0**-8, one + 2.0**-6),  # halfway between 1 + 2^-7 and 1 + 2^-6: even is 1 + 2^-6
        (one + 2.0**-8 + 2.0**-20, one + 2.0**-7),  # just above halfway rounds up
        (-(one + 2.0**-8 + 2.0**-20), -(one + 2.0**-7)),
        (3.140625, 3.140625),               # 8 significant bits: exact
        (0.0, 0.0),
    ]
    x = np.array([c[0] for c in cases])
    want = np.array([c[1] for c in cases])
    got = precision._bf16(x)
    np.testing.assert_array_equal(got, want)


def test_bf16_unit_roundoff_and_library_conversion():
    rng = np.random.default_rng([7, 1])
    x = rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))
    got = precision._bf16(x)
    x32 = x.astype(np.float32).astype(np.float64)
    # round to nearest: at most half a unit in the last place (2^-8 relative) from the float32 value
    assert np.all(np.abs(got - x32) <= 2.0**-8 * np.abs(x32))
    torch = pytest.importorskip("torch")
    lib = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(got, lib)


def test_complex_forms():
    rng = np.random.default_rng([7, 2])
    a = rng.standard_normal(1000) + 1j * rng.standard_normal(1000)
    f = precision.to_f32(a)
    assert np.all(np.abs(f.real - a.real) <= 2.0**-24 * np.abs(a.real))
    assert np.all(np.abs(f.imag - a.imag) <= 2.0**-24 * np.abs(a.imag))
    b = precision.to_bf16_pair(a)
    np.testing.assert_array_equal(b.real, precision._bf16(a.real))
    np.testing.assert_array_equal(b.imag, precision._bf16(a.imag))


def test_round_operator_touches_only_stored_blocks():
    rng = np.random.default_rng([7, 3])
    op = {k: rng.standard_normal(50) + 1j * rng.standard_normal(50) for k in ("U", "V", "S", "D", "X")}
    op["perm"] = np.arange(5)
    out = precision.round_operator(op, "bf16pair")
    for k in ("U", "V", "S", "D"):
        np.testing.assert_array_equal(out[k], precision.to_bf16_pair(op[k]))
    assert out["X"] is op["X"] and out["perm"] is op["perm"]
