"""The synthetic workloads of Sec. 5 are what the paper describes: an order-6
10 x ... x 10 tensor of exact TT rank 5 plus noise of the stated standard
deviation, and the two 1-D functions sampled at 10^6 points and folded
column-major (the first index fastest, as MATLAB's reshape)."""
import math

import numpy as np

import synth


def test_paper_tt6_has_tt_rank_5_and_the_stated_noise():
    clean, cores = synth.paper_tt6(5, 0.0)
    assert clean.size == 10 ** 6
    assert [c.shape for c in cores] == [(1, 10, 5)] + [(5, 10, 5)] * 4 + [(5, 10, 1)]
    # every unfolding (modes 0..k-1 against the rest) has rank 5 exactly
    T = clean.reshape([10] * 6, order="F")
    for k in range(1, 6):
        M = T.reshape(10 ** k, 10 ** (6 - k), order="F")
        assert np.linalg.matrix_rank(M) == 5, k
    # iid N(0, 1) core entries: a core's mean and spread
    allc = np.concatenate([c.ravel() for c in cores])
    assert abs(allc.mean()) < 0.1 and abs(allc.std() - 1.0) < 0.1
    for sd in (0.1, 0.01):
        noisy, _ = synth.paper_tt6(5, sd)
        e = noisy - clean
        assert abs(e.std() / sd - 1.0) < 0.01 and abs(e.mean()) < 5 * sd / 1000


def test_function_tensors_sample_the_functions_in_column_major_order():
    sinc = synth.function_tensor("sinc")
    osc = synth.function_tensor("osc")
    assert sinc.shape == osc.shape == (10 ** 6,)
    assert np.all(np.isfinite(sinc)) and np.all(np.isfinite(osc))
    for j in (0, 1, 499999, 500000, 123456, 999999):
        x = -5.0 + 10.0 * j / (10 ** 6 - 1)
        want = math.sin(math.pi * x) / (math.pi * x)
        assert abs(sinc[j] - want) < 1e-15, j
        x = (j + 1) / 10 ** 6
        assert abs(osc[j] - math.sin(4.0 / x) * math.cos(x * x)) < 1e-15, j
    # the end points: sinc(+-5) = 0, and the last osc point is x = 1
    assert abs(sinc[0]) < 1e-15 and abs(sinc[-1]) < 1e-15
    assert osc[-1] == math.sin(4.0) * math.cos(1.0)
    # folding: entry (i_0, ..., i_5) is sample i_0 + 10 i_1 + ... + 10^5 i_5
    T = osc.reshape([10] * 6, order="F")
    idx = (3, 1, 4, 1, 5, 9)
    assert T[idx] == osc[sum(i * 10 ** k for k, i in enumerate(idx))]


def test_function_ranks_clip_at_the_boundary_modes():
    assert synth.function_ranks(5) == [1, 5, 5, 5, 5, 5, 1]
    assert synth.function_ranks(13) == [1, 10, 13, 13, 13, 10, 1]
    assert synth.function_ranks(20) == [1, 10, 20, 20, 20, 10, 1]
    assert synth.function_ranks(200) == [1, 10, 100, 200, 100, 10, 1]
