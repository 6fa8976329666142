"""Pivot ties on the GPU (Algorithm 1's largest-norm pivot; ties go to the lowest
column index, the rule the oracle is pinned to).

Identical columns of A have bitwise identical sketch columns (every column of a
block runs through the same instructions on the same sketch matrix), so their
residual norms tie exactly at every step until one of them is taken.  The gap
rule cannot check such steps (the gap is zero), so the index is asserted
directly, for each selection kernel: one column per lane, two lanes per column
(tall sketches), part of the sketch in LDS (wide blocks).
"""
import numpy as np
import pytest
import torch

from _harness import gpu_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _tied_block(m, n, seed, first, dup, second, dup2):
    """Columns `dup` = `first` (the largest norm) and `dup2` = `second` (the next
    largest after the first is projected out)."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)) * 0.1
    A[:, first] = rng.standard_normal(m) * 10.0
    A[:, dup] = A[:, first]
    A[:, second] = rng.standard_normal(m) * 5.0
    A[:, dup2] = A[:, second]
    return np.asfortranarray(A)


@pytest.mark.parametrize("l,n,prec", [(24, 64, "f64"), (96, 300, "f64"), (50, 700, "f64"),
                                      (48, 512, "bf16")])
def test_exact_ties_take_the_lowest_index(l, n, prec):
    blocks = [_tied_block(3000, n, 3 + b, first, dup, second, dup2)
              for b, (first, dup, second, dup2) in enumerate(
                  [(5, 2 * n // 3, 9, n - 1), (n // 2, n - 3, 1, n // 4 + 1)])]
    if prec != "f64":
        blocks = [np.asfortranarray(b.astype(np.float32)) for b in blocks]
    print(f"case: ties l={l} n={n} {prec}", flush=True)
    g = gpu_run(blocks, l, 8, 23, prec=prec, lp_terms=2)
    # block 0: first = 5 < dup, then second = 9 < dup2; block 1: the largest pair
    # is (n/2, n-3) -> n/2, the next pair (1, n/4+1) -> 1
    assert g.S[0][0] == 5 and g.S[0][1] == 9, g.S[0][:4]
    assert g.S[1][0] == n // 2 and g.S[1][1] == 1, g.S[1][:4]
    for b in range(2):
        # the duplicates of the taken columns are never chosen before the other columns
        # run out of norm: their residuals are rounding-level
        assert g.k[b] == 8
