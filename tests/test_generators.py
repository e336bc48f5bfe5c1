"""Input generators (svogen) on the host: the C heightfield pool builder is
node-identical to the Python builder (also with far pointers forced), grid
noise equals pointwise noise bit for bit, and the pool-walk helpers agree
with the builder's metadata.  These generators hold no traversal arithmetic;
they feed both the oracle and the device path."""
import numpy as np
import pytest

from svogen import hfbuild, noise
from svogen import octree as ot
from svogen import scenes as S


@pytest.fixture(scope="module", autouse=True)
def _lib():
    hfbuild.build(force=True)


@pytest.mark.parametrize("K,seed", [(5, 1), (7, 3), (9, 2)])
def test_c_builder_equals_python_builder(K, seed):
    H = S.heightfield(K, seed, 0.5 * (1 << K), 0.3 * (1 << K), 5, (1 << K) / 4)
    tree = ot.build_tree(K, ot.heightfield_classifier(H, K), S._colour_fn(K, seed))
    nodes, counts = hfbuild.build_heightfield_pool(H, K, seed)
    assert np.array_equal(nodes, tree.nodes)
    assert counts.sum() == tree.n
    assert np.array_equal(counts[:tree.level.max() + 1], np.bincount(tree.level))
    far, _ = hfbuild.build_heightfield_pool(H, K, seed, far_from=1)
    assert np.array_equal(far, ot.force_far(tree.nodes))


def test_c_builder_edge_cases():
    K = 4
    n = 1 << K
    empty, c = hfbuild.build_heightfield_pool(np.zeros((n, n), np.int32), K, 0)
    assert empty.shape[0] == 0
    full, c = hfbuild.build_heightfield_pool(np.full((n, n), n, np.int32), K, 0)
    assert full.shape[0] == 1 and int(full[0]) & 0xFF == 0          # one solid root leaf
    step = np.zeros((n, n), np.int32)
    step[n // 2:, :] = 3
    tree = ot.build_tree(K, ot.heightfield_classifier(step, K), S._colour_fn(K, 0))
    got, _ = hfbuild.build_heightfield_pool(step, K, 0)
    assert np.array_equal(got, tree.nodes)


def test_grid_noise_equals_pointwise():
    n = 48
    g = np.arange(n) + 0.5
    X, Z = np.meshgrid(g, g, indexing="ij")
    assert np.array_equal(noise.value_noise2_grid(n, 7.0, 2, 5), noise.value_noise2(X, Z, 7.0, 2, 5))
    assert np.array_equal(noise.fbm2_grid(n, 5, 16.0, 9), noise.fbm2(X, Z, 5, 16.0, 9))
    r = noise.ridged2_grid(n, 4, 16.0, 3)
    assert r.shape == (n, n) and r.min() >= -1.0 and r.max() <= 1.0


def test_pool_walk_helpers_match_metadata():
    sc = S.tiny_scene(4, K=6, n_slots=3, nested=False)
    static = ot.clear_transformed(sc.nodes, sc.slot_child)
    idx, lev, crd = ot.top_levels(static, 3)
    sel = sc.tree.level <= 3
    assert np.array_equal(idx, np.nonzero(sel)[0])
    assert np.array_equal(crd, sc.tree.coord[sel]) and np.array_equal(lev, sc.tree.level[sel])
    marked, child, node = ot.mark_transformed_pool(static, list(sc.slot_node))
    assert np.array_equal(marked, sc.nodes) and np.array_equal(child, sc.slot_child)
