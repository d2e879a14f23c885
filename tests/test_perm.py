"""The test helper's minibatch order is a permutation for every row count
(cycle walking over the Feistel bijection), differs between epochs and
seeds, and is not the identity."""
import numpy as np
import pytest

from .perm import epoch_rows, feistel


@pytest.mark.parametrize("n", [1, 2, 3, 5, 16, 17, 1000, 4097])
def test_epoch_order_is_a_permutation(n):
    rows = epoch_rows(n, 7, 0)
    np.testing.assert_array_equal(np.sort(rows), np.arange(n))


def test_feistel_is_a_bijection_on_its_domain():
    vals = [feistel(x, 3, 99, 2) for x in range(64)]
    assert sorted(vals) == list(range(64))


def test_epochs_and_seeds_change_the_order():
    a, b, c = epoch_rows(1000, 1, 0), epoch_rows(1000, 1, 1), epoch_rows(1000, 2, 0)
    assert not np.array_equal(a, np.arange(1000))
    assert not np.array_equal(a, b) and not np.array_equal(a, c)
