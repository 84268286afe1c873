"""The seeded generators: SplitMix64 against its scalar definition and the
published first outputs, masking and sparse sampling."""
import numpy as np

from paper_2201_10473_amd import inputs


def test_splitmix_vector_matches_scalar():
    key = inputs.stream_key(inputs.SEED_BASE + 2, 17, 1)
    v = inputs.splitmix_words(key, 50)
    state = key
    for i in range(50):
        state, z = inputs.splitmix_scalar(state)
        assert int(v[i]) == z


def test_splitmix_published_vector():
    # SplitMix64 seeded with 0: first output 0xE220A8397B1DCDAF (reference
    # implementation by Vigna, splitmix64.c).
    state, z = inputs.splitmix_scalar(0)
    assert z == 0xE220A8397B1DCDAF
    state, z = inputs.splitmix_scalar(state)
    assert z == 0x6E789E6AA1B965F4


def test_dense_masked_and_batch_consistent():
    for n in (1, 63, 64, 65, 17669, 57637):
        B = inputs.dense_batch(n, 4, 123, role=1)
        for p in range(4):
            assert np.array_equal(B[p], inputs.dense(n, 123, p, 1))
        if n % 64:
            assert int(B[:, -1].max()) < (1 << (n % 64))


def test_sparse_positions_distinct_and_in_range():
    for n in inputs.RING_SIZES:
        w = inputs.sparse_weight_for(n)
        pos = inputs.sparse_positions(n, w, 5, 3)
        assert len(pos) == w == len(set(pos))
        assert 0 <= min(pos) and max(pos) < n
        s = inputs.sparse(n, w, 5, 3)
        assert sum(bin(int(x)).count("1") for x in s) == w
