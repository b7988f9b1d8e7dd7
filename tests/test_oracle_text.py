"""Pins for the oracle's n-gram items of symbol sequences (text_items): the
item set of every read and URL string equals the set the workload generator
makes independently (its own packing and MurmurHash3 finalisers, before the
generator deduplicates); window counts follow the definition; 32-bit items
use the 32-bit finaliser of the low words."""
import numpy as np
import pytest

from workloads import synth


def _sets_equal(items, ioff, it, of):
    return all(np.array_equal(np.unique(items[ioff[i]:ioff[i + 1]]), it[of[i]:of[i + 1]])
               for i in range(len(of) - 1))


def test_genome_reads_match_generator(orc):
    it, of, qit, qof, _, ex = synth.genome(n_base=400, nq=60, text=True)
    items, ioff = orc.text_items(*ex["data"], ex["gram"], ex["radix"], ex["key"], 64)
    assert items.dtype == np.uint64 and _sets_equal(items, ioff, it, of)
    q, qo = orc.text_items(*ex["queries"], ex["gram"], ex["radix"], ex["key"], 64)
    assert _sets_equal(q, qo, qit, qof)
    # every 100-base read has 81 windows
    assert np.all(np.diff(ioff.astype(np.int64)) == 81)


def test_url_strings_match_generator(orc):
    it, of, qit, qof, _, _, ex = synth.url(n_templates=300, nq=60, text=True)
    items, ioff = orc.text_items(*ex["data"], ex["gram"], ex["radix"], ex["key"], 32)
    assert items.dtype == np.uint32 and _sets_equal(items, ioff, it, of)
    q, qo = orc.text_items(*ex["queries"], ex["gram"], ex["radix"], ex["key"], 32)
    assert _sets_equal(q, qo, qit, qof)


@pytest.mark.parametrize("gram", [1, 2, 5])
def test_window_counts_and_short_sequences(orc, gram):
    rng = np.random.default_rng(gram)
    lens = np.array([0, 1, gram - 1, gram, gram + 1, 17, 0, 3])
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
    sym = rng.integers(0, 7, int(offs[-1])).astype(np.uint8)
    items, ioff = orc.text_items(sym, offs, gram, 7, 123, 64)
    assert np.array_equal(np.diff(ioff.astype(np.int64)), np.maximum(0, lens - gram + 1))
    # equal windows give equal items, different windows different ones (here)
    win = {}
    for s in range(len(lens)):
        for p in range(max(0, lens[s] - gram + 1)):
            w = tuple(sym[offs[s] + p: offs[s] + p + gram])
            win.setdefault(w, set()).add(int(items[ioff[s] + p]))
    assert all(len(v) == 1 for v in win.values())
    assert len({next(iter(v)) for v in win.values()}) == len(win)
