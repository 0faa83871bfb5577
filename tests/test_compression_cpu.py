"""Compression-curve reference on the host: the best rank-r error (Eckart-Young)."""
import numpy as np
import pytest


def test_best_rank_reference_is_eckart_young_on_a_diagonal():
    # compression-curve reference: the error of the best rank-r approximation of diag(d) leaves
    # out the n - r entries of smallest magnitude
    from paper_1507_04396_amd.compression import best_rank_error2
    d = np.array([5.0, -4.0, 3.0, 0.5, -0.25])
    lam = d[np.argsort(-np.abs(d), kind="stable")]
    assert best_rank_error2(lam, 2) == pytest.approx(3.0 ** 2 + 0.5 ** 2 + 0.25 ** 2)
    assert best_rank_error2(lam, 5) == 0.0
