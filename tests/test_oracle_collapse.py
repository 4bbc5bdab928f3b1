"""Pins for the oracle's collapse step (oracle.collapse): every maximal
subtree of at most leaf_size primitives becomes one leaf, the rest of the
tree is kept, in preorder.

Inputs are hand-made preorder trees that split every node of count c at
floor(c / 2) (the shape of the balanced trees the binned-SAH pins produce),
so the collapsed tree has a closed form:
  * n = 2^k primitives and leaf size L < n: every leaf holds 2^floor(log2 L)
    primitives, so there are n / 2^floor(log2 L) leaves and one interior node
    fewer;
  * L >= n: the root alone, as a leaf.
For other n the invariants that define the step are checked: leaves hold at
most L primitives, the parent of every leaf holds more than L (maximality),
leaf ranges tile [0, n) in ascending order, each interior row is followed by
its left child and its right child starts where the left subtree ends.
"""
import math

import numpy as np
import pytest


def median_tree(n):
    """Preorder rows (first, count, axis, left count) of the tree that splits
    each node of c > 1 primitives into floor(c/2) and c - floor(c/2)."""
    rows = []

    def rec(first, count):
        nl = count // 2 if count > 1 else 0
        rows.append((first, count, 0, nl))
        if count > 1:
            rec(first, nl)
            rec(first + nl, count - nl)

    rec(0, n)
    return np.array(rows, np.int64)


@pytest.mark.parametrize("k", range(0, 8))
@pytest.mark.parametrize("leaf_size", range(1, 17))
def test_power_of_two_line_closed_form(orc, k, leaf_size):
    n = 1 << k
    out = orc.collapse(median_tree(n), leaf_size)
    leaves = [r for r in out if r[4]]
    if leaf_size >= n:
        assert len(out) == 1 and out[0][4] == 1 and out[0][1] == n
        return
    size = 1 << int(math.floor(math.log2(leaf_size)))
    assert len(leaves) == n // size
    assert all(r[1] == size for r in leaves)
    assert len(out) == 2 * len(leaves) - 1


def _check_invariants(nodes, out, n, leaf_size):
    by_range = {(int(r[0]), int(r[1])): i for i, r in enumerate(nodes)}
    leaves = [r for r in out if r[4]]
    assert all(1 <= r[1] <= leaf_size for r in leaves)
    # leaf ranges tile [0, n) in ascending order
    pos = 0
    for r in leaves:
        assert r[0] == pos
        pos += r[1]
    assert pos == n
    # each row names its source node; the parent of a leaf is too big to be one
    parent = {}
    for i, r in enumerate(nodes):
        if r[1] > 1:
            parent[i + 1] = i
            parent[i + 2 * int(r[3])] = i
    for r in out:
        assert by_range[(r[0], r[1])] == r[5]
        if r[4] and r[5] != 0:
            assert nodes[parent[r[5]]][1] > leaf_size
    # preorder: an interior row is followed by its left child; its right
    # child starts where the left subtree's range ends
    for j, r in enumerate(out):
        if not r[4]:
            left = out[j + 1]
            assert left[0] == r[0] and left[1] == r[3]
    assert len(out) == 2 * len(leaves) - 1


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 100, 1000, 4097])
@pytest.mark.parametrize("leaf_size", [1, 2, 3, 4, 8, 15, 16])
def test_invariants_on_uneven_counts(orc, n, leaf_size):
    nodes = median_tree(n)
    out = orc.collapse(nodes, leaf_size)
    _check_invariants(nodes, out, n, leaf_size)


def test_sah_tree_of_a_scene(orc):
    from paper_2511_15028_amd import workloads as W
    v, t = W.soup_scene(3000, seed=7)
    _, nodes, _ = orc.sah_build(v, t)
    for leaf_size in (1, 4, 16):
        _check_invariants(nodes, orc.collapse(nodes, leaf_size), len(t), leaf_size)
