"""Pins of the oracle's reduced-precision matrix storage against library conversions."""
import numpy as np
import pytest
import torch

import oracle
from paper_1601_08201_amd import datagen


@pytest.fixture(scope="module")
def system():
    prob = datagen.make_problem(dict(ny=8, nx=8, Q=16, I=2048, nnz_per_col=12, rects=3), seed=4)
    return prob


def quotient(prob):
    sigma = np.zeros(prob.J, np.float32)
    np.maximum.at(sigma, prob.col, prob.val)
    s = sigma[prob.col]
    return sigma, np.where(s > 0, prob.val / np.where(s > 0, s, np.float32(1)), np.float32(0)).astype(np.float32)


def test_bf16_codes_match_torch_rounding(system):
    scale, codes, deq = oracle.quantise(system.col, system.val, system.J, "bf16")
    sigma, t = quotient(system)
    np.testing.assert_array_equal(scale, sigma)
    ref = torch.from_numpy(t).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(codes, ref)
    back = torch.from_numpy(ref.view(np.int16)).view(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(deq, sigma[system.col].astype(np.float64) * back)


def test_f16_codes_match_numpy_rounding(system):
    scale, codes, deq = oracle.quantise(system.col, system.val, system.J, "f16")
    sigma, t = quotient(system)
    ref = t.astype(np.float16)
    np.testing.assert_array_equal(codes, ref.view(np.uint16))
    np.testing.assert_array_equal(deq, sigma[system.col].astype(np.float64) * ref.astype(np.float64))


def test_f16_subnormals_and_ties():
    # values chosen to hit subnormal codes, the normal/subnormal edge and round-half-even ties
    vals = np.array([1.0, 2.0 ** -14, 2.0 ** -15, 2.0 ** -24, 3 * 2.0 ** -25, 2.0 ** -25,
                     0.5 + 2.0 ** -12, 0.5 + 3 * 2.0 ** -12, 0.1, 0.3333333, 0.0], np.float32)
    col = np.zeros(vals.size, np.int32)
    scale, codes, deq = oracle.quantise(col, vals, 1, "f16")
    assert scale[0] == 1.0
    np.testing.assert_array_equal(codes, vals.astype(np.float16).view(np.uint16))
    _, bcodes, _ = oracle.quantise(col, vals, 1, "bf16")
    np.testing.assert_array_equal(bcodes, torch.from_numpy(vals).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16))


def test_relative_error_bounds(system):
    # unit roundoff: 2^-8 for bfloat16 (8-bit significand), 2^-11 for binary16 (11-bit)
    for kind, u in (("bf16", 2.0 ** -8), ("f16", 2.0 ** -11)):
        scale, codes, deq = oracle.quantise(system.col, system.val, system.J, kind)
        v = system.val.astype(np.float64)
        big = v >= scale[system.col] * 2.0 ** -14     # normal range of both formats
        rel = np.abs(deq[big] - v[big]) / v[big]
        assert rel.max() <= u * (1 + 1e-6)
        assert rel.max() > u / 4      # the bound is reached, not loose
