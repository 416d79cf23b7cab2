"""The seeded input generators shared by the tests and the benchmark: the same
seed gives the same text, values stay in the alphabet, shorter texts are
prefixes of longer ones, and the recipes have the stated shapes."""
import numpy as np
import pytest

from paper_1702_07578_amd import inputs


@pytest.mark.parametrize("sigma,b", [(4, 1), (96, 1), (256, 1), (1 << 16, 2), (1 << 20, 4)])
def test_uniform_seeded_in_range_and_prefix(sigma, b):
    a = inputs.uniform(1 << 16, sigma, b, 7)
    assert a.dtype == {1: np.uint8, 2: np.uint16, 4: np.uint32}[b]
    assert int(a.max()) < sigma
    assert np.array_equal(a, inputs.uniform(1 << 16, sigma, b, 7))
    assert not np.array_equal(a, inputs.uniform(1 << 16, sigma, b, 8))
    assert np.array_equal(inputs.uniform(1000, sigma, b, 7), a[:1000])
    # every symbol of a small alphabet turns up
    if sigma <= 256:
        assert len(np.unique(a)) == sigma


def test_markov_seeded_in_range_and_chain_prefix():
    a = inputs.markov2(3 << 12, 96, 2, chain_len=1 << 12)
    assert int(a.max()) < 96
    assert np.array_equal(a, inputs.markov2(3 << 12, 96, 2, chain_len=1 << 12))
    # whole chains are prefixes of the longer text
    assert np.array_equal(inputs.markov2(2 << 12, 96, 2, chain_len=1 << 12), a[:2 << 12])
    # order-2 structure: every context (previous two symbols) has a peaked
    # next-symbol distribution (rows drawn from Dirichlet(0.1)); an i.i.d.
    # text gives each next symbol about 1/96 of a context
    t = inputs.markov2(1 << 20, 96, 2).astype(np.int64)
    c = np.bincount((t[:-2] * 96 + t[1:-1]) * 96 + t[2:], minlength=96 ** 3).reshape(96 * 96, 96)
    seen = c.sum(axis=1) >= 50
    assert (c[seen].max(axis=1) / c[seen].sum(axis=1)).mean() > 0.15


def test_zipf_skew_and_range():
    a = inputs.zipf(1 << 20, 1 << 20, 1.1, 4, 4)
    assert int(a.max()) < (1 << 20)
    counts = np.bincount(a)
    # Zipf(1.1) over 2^20 ranks: the top rank holds about 12 % of the text
    assert 0.08 < counts.max() / a.size < 0.16
    # ids are permuted: the most frequent id is not rank 0's
    assert int(np.argmax(counts)) != 0
    assert np.array_equal(a, inputs.zipf(1 << 20, 1 << 20, 1.1, 4, 4))
    assert np.array_equal(inputs.zipf(5000, 1 << 20, 1.1, 4, 4), a[:5000])


def test_recipes_shapes():
    for name, (n, dtype, L) in {"uniform256": (1 << 20, np.uint8, 8), "markov96": (1 << 30, np.uint8, 7),
                                "markov4": (1 << 31, np.uint8, 2), "zipf20": (1 << 28, np.uint32, 20),
                                "uniform16": (1 << 29, np.uint16, 16)}.items():
        c = inputs.CONFIGS[name]
        assert c["n"] == n and inputs.lg_sigma(c["sigma"]) == L
        t, l = inputs.make(name, 4096)
        assert t.size == 4096 and t.dtype == dtype and l == L


def test_batch_specs():
    specs = inputs.batch_specs(512, seed=6)
    assert len(specs) == 512
    assert specs == inputs.batch_specs(512, seed=6)
    for sp in specs:
        assert (1 << 10) <= sp["n"] < (1 << 22)
        assert sp["sigma"] in (4, 256, 1 << 16)
        assert sp["sym_bytes"] == (1 if sp["sigma"] <= 256 else 2)
        assert sp["dist"] in ("uniform", "zipf")
    # the mix covers every alphabet and both distributions
    assert {sp["sigma"] for sp in specs} == {4, 256, 1 << 16}
    assert {sp["dist"] for sp in specs} == {"uniform", "zipf"}


def test_u64_and_unit_ranges():
    x = inputs.u64(10000, 1000, 3, 1)
    assert x.dtype == np.uint64 and int(x.max()) < 1000
    u = inputs.unit(10000, 3, 1)
    assert 0.0 <= u.min() and u.max() < 1.0
    assert not np.array_equal(inputs.u64(100, 1000, 3, 1), inputs.u64(100, 1000, 3, 2))
