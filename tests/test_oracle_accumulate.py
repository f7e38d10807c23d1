"""Pins of the oracle's Krylov subspace accumulation over an image cycle (Experiment 2's
subspace expansion): orthonormality, exact reproduction of the first source, containment of
every appended direction, dependent columns dropped, the per-source and total caps, and the
coordinate-vector case whose answer is known by hand."""
import numpy as np

import oracle


def qr_cols(n, k, seed):
    Q, _ = np.linalg.qr(np.random.default_rng(seed).normal(size=(n, k)))
    return Q


def test_first_source_is_reproduced_and_basis_is_orthonormal(olib):
    A, B = qr_cols(60, 8, 1), qr_cols(60, 8, 2)
    V = oracle.accumulate([A, B], per_source=5, cap=10)
    assert V.shape == (60, 10)
    assert np.abs(V.T @ V - np.eye(10)).max() <= 1e-14
    # source 0's leading columns come through unchanged (they are already orthonormal)
    assert np.abs(V[:, :5] - A[:, :5]).max() <= 1e-14
    # every gathered direction of source 1 lies in the span: B's first 5 columns are
    # reproduced by the projection onto V
    Bq = B[:, :5]
    assert np.abs(Bq - V @ (V.T @ Bq)).max() <= 1e-13


def test_dependent_columns_are_dropped():
    A = qr_cols(40, 6, 3)
    V = oracle.accumulate([A, A], per_source=4, cap=10)
    # the second copy contributes only the two columns the first one did not take
    assert V.shape == (40, 6)
    assert np.abs(V @ V.T - A @ A.T).max() <= 1e-13


def test_caps():
    A, B = qr_cols(50, 9, 4), qr_cols(50, 9, 5)
    assert oracle.accumulate([A, B], per_source=9, cap=12).shape[1] == 12
    assert oracle.accumulate([A, B], per_source=3, cap=12).shape[1] == 6
    assert oracle.accumulate([A], per_source=20, cap=64).shape[1] == 9


def test_coordinate_vectors_by_hand():
    """Sources e_0, e_1 and (e_1 + e_2)/sqrt2, e_0: the second source's first column loses its
    e_1 part and becomes e_2; its second column is dependent."""
    n = 5
    I = np.eye(n)
    s0 = I[:, [0, 1]]
    s1 = np.stack([(I[:, 1] + I[:, 2]) / np.sqrt(2), I[:, 0]], axis=1)
    V = oracle.accumulate([s0, s1], per_source=2, cap=5)
    assert V.shape == (5, 3)
    assert np.abs(V - I[:, :3]).max() <= 1e-15


def test_nearly_dependent_column_needs_the_second_pass():
    """A column 1e-6 away from the span: one Gram-Schmidt pass would leave it non-orthogonal at
    about u / 1e-6; with the second pass the gathered basis stays orthonormal to roundoff."""
    A = qr_cols(80, 6, 6)
    r = np.random.default_rng(7).normal(size=80)
    near = A @ np.random.default_rng(8).normal(size=6) + 1e-6 * r
    V = oracle.accumulate([A, near[:, None] / np.linalg.norm(near)], per_source=6, cap=7)
    assert V.shape == (80, 7)
    assert np.abs(V.T @ V - np.eye(7)).max() <= 1e-14
