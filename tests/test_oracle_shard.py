"""Pins for the oracle's tree shards (Sec. VII: a set of CAPTs, each
responsible for one neighbourhood of a large cloud).

- the leaf ranges on hand cases, including more shards than leaves;
- the ranges partition the leaves, and for bits <= D a shard's range is the
  set of leaves whose depth-`bits` ancestor (Eytzinger parent (i - 1) // 2)
  is node 2^bits - 1 + shard;
- Lemma 1 inside a shard: for radii in [r_min, r_max] the shard answers as
  float32 brute force for a sphere whose leaf lies in the shard, and never
  reports a collision for one whose leaf lies elsewhere; so the OR over all
  shards is the brute force answer;
- the shards' sets add up to the whole tree's, leaf by leaf.
"""
import numpy as np
import pytest

import synth


def test_shard_leaves_hand_cases(orc):
    assert list(orc.shard_leaves(8, 0, 0)) == list(range(8))
    assert list(orc.shard_leaves(8, 1, 1)) == [4, 5, 6, 7]
    assert list(orc.shard_leaves(8, 3, 5)) == [5]
    assert list(orc.shard_leaves(8, 4, 10)) == [5]      # 16 shards over 8 leaves: even shards hold one
    assert list(orc.shard_leaves(8, 4, 11)) == []
    assert list(orc.shard_leaves(8, 5, 4)) == [1]
    assert list(orc.shard_leaves(1, 2, 0)) == [0]
    assert list(orc.shard_leaves(1, 2, 3)) == []


@pytest.mark.parametrize("N", [1, 2, 16, 1024])
def test_shards_partition_the_leaves_into_subtrees(orc, N):
    D = N.bit_length() - 1
    for bits in range(0, D + 3):
        owner = np.full(N, -1)
        for s in range(2 ** bits):
            for l in orc.shard_leaves(N, bits, s):
                assert owner[l] == -1
                owner[l] = s
        assert (owner >= 0).all()
        if bits <= D:
            for l in range(N):
                i = l + N - 1                  # the leaf's node index
                for _ in range(D - bits):
                    i = (i - 1) // 2           # parent
                assert i == 2 ** bits - 1 + owner[l]


@pytest.mark.parametrize("prune", [True, False])
def test_lemma1_per_shard_and_or_over_shards(orc, prune):
    pts = synth.tabletop_cloud(3000, 61)
    r_min, r_max = 0.015, 0.08
    tree = orc.build_tree(pts, r_min, r_max, prune)
    sph = synth.uniform_spheres(20000, synth.WORKSPACE, r_min, r_max, 62)
    brute = orc.brute_f32(pts, sph)
    _, leaf, _, _ = orc.query_tree(tree, pts, sph)
    assert brute.sum() > 500
    for bits in (1, 3, tree.D + 1):
        acc = np.zeros(len(sph), np.uint8)
        for s in range(2 ** bits):
            sh = orc.shard_tree(tree, bits, s)
            hit, lf, _, _ = orc.query_tree(sh, pts, sph)
            assert np.array_equal(lf, leaf)    # the splits are the whole tree's
            mine = np.isin(leaf, np.array(orc.shard_leaves(tree.N, bits, s)))
            assert np.array_equal(hit[mine], brute[mine])
            assert not hit[~mine].any()
            acc |= hit
        assert np.array_equal(acc, brute)


def test_shard_sets_add_up_to_the_tree(orc):
    pts = synth.tabletop_cloud(2500, 63)
    tree = orc.build_tree(pts, 0.015, 0.08)
    bits = 2
    total = 0
    pruned = np.zeros(tree.N, np.uint8)
    for s in range(2 ** bits):
        sh = orc.shard_tree(tree, bits, s)
        total += int(sh.off[-1])
        pruned |= sh.pruned
        for l in range(tree.N):
            if l in orc.shard_leaves(tree.N, bits, s):
                assert np.array_equal(sh.set_of(l), tree.set_of(l))
                assert np.array_equal(sh.aabb[l], tree.aabb[l])
            else:
                assert len(sh.set_of(l)) == 0 and sh.pruned[l] == 0
                assert (sh.aabb[l, :3] == np.inf).all() and (sh.aabb[l, 3:] == -np.inf).all()
    assert total == int(tree.off[-1])
    assert np.array_equal(pruned, tree.pruned)
    whole = orc.shard_tree(tree, 0, 0)
    assert np.array_equal(whole.off, tree.off) and np.array_equal(whole.idx, tree.idx)
