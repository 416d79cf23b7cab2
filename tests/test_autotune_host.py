"""Host-side logic of the batch autotuner: the batch signature and the cache
lookup, which answers without building anything."""
import json

from paper_1702_07578_amd import autotune
from paper_1702_07578_amd import binding as B


def _items(spec):
    # (device text, n, symbol bytes, L, kind, structure): the signature and
    # the cache lookup read only n, b, L and kind
    return [(None, n, b, L, kind, None) for n, b, L, kind in spec]


def test_signature_counts_sizes_and_mix():
    items = _items([(1000, 1, 8, B.WT_TREE), (3000, 2, 16, B.WT_MATRIX), (96, 1, 8, B.WT_TREE)])
    sig = autotune.signature(items)
    assert sig.startswith("count=3;log2sym=12;")  # 4096 symbols
    assert f"1:8:{B.WT_TREE}x2" in sig and f"2:16:{B.WT_MATRIX}x1" in sig


def test_signature_ignores_order_but_not_kind():
    a = _items([(1000, 1, 8, B.WT_TREE), (3000, 2, 16, B.WT_MATRIX)])
    assert autotune.signature(a) == autotune.signature(list(reversed(a)))
    b = _items([(1000, 1, 8, B.WT_MATRIX), (3000, 2, 16, B.WT_MATRIX)])
    assert autotune.signature(a) != autotune.signature(b)


def test_cached_winner_is_returned_without_building(tmp_path):
    items = _items([(1 << 20, 1, 8, B.WT_TREE), (1 << 20, 1, 8, B.WT_MATRIX)])
    table = [[128, 0, 1.5, "ok"], [16, 4096, None, "outputs differ"]]
    cache = tmp_path / "tune.json"
    cache.write_text(json.dumps({autotune.signature(items): {"grid": 128, "persist": 4096, "ms": 1.5,
                                                             "table": table}}))
    tune, got = autotune.tune(items, cache_path=str(cache))
    assert (tune.grid, tune.persist) == (128, 4096)
    assert got == table
