"""The mixed-precision kernel's zero rule, pinned on the oracle (CPU).

The FP32 path ends a path when an operator leaves a squared norm below 1e-10 of
its unit input (a norm below 1e-5), where the FP64 oracle uses 1e-10 of the norm.
Both thresholds are readings of the same exact statement: the operator
annihilates the vector by symmetry and anything left is rounding noise.  On the
7-orbital parity configurations the two thresholds must give bitwise the same
traces, and any retained-state contribution that one of them keeps and the other
drops must lie below the FP64 resolution of the total (|t_i| < 2^-53 |Tr|).  A
larger one would mean the FP32 rule turns a genuine contribution into an exact
zero.  (Two such paths occur in this sample, at e^-57 and e^-98 of their totals.)
"""
import numpy as np

from paper_0908_0681_amd import inputs as I
from oracle import pool as OP


def test_seven_orbital_zero_threshold_equivalence():
    w = I.workload(2)
    b = w.batch()
    idx = np.concatenate([np.arange(12), I.parity_sample(b.n_configs, 64, 19)])
    r10, _ = OP.trace_batch(w.params, w.retain_window, b, configs=idx, zero_tol=1e-10)
    r5, _ = OP.trace_batch(w.params, w.retain_window, b, configs=idx, zero_tol=1e-5)
    assert np.array_equal(r10.sign, r5.sign)
    assert np.array_equal(r10.log_abs, r5.log_abs)
    differ = np.argwhere(r10.contrib_sign != r5.contrib_sign)
    for j, r in differ:
        assert r5.contrib_sign[j, r] == 0, "the larger threshold can only add zeros"
        assert r10.contrib_log[j, r] - r10.log_abs[j] < np.log(2.0 ** -53), (idx[j], r)
    # the sample holds nonzero traces and symmetry zeros of feasible paths
    assert (r10.sign != 0).sum() >= 40
    assert (r10.feasible & (r10.contrib_sign == 0)).sum() >= 1
