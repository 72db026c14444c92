"""Host logic of the autotuner: table lookup and the selection rules."""
from __future__ import annotations

import json

from paper_2101_05916_amd import autotune as A


def _table(tmp_path, entries):
    p = tmp_path / "t.json"
    p.write_text(json.dumps({"entries": entries}))
    A._cache = None
    return str(p)


def test_lookup_exact_nearest_and_missing(tmp_path):
    e41 = {"tile_rows": 12, "chunk": 64}
    e61 = {"tile_rows": 8, "chunk": 32}
    e2d = {"tile_rows": 1, "chunk": 64}
    path = _table(tmp_path, {A.key(1, 0, (41,) * 4): e41, A.key(1, 0, (61,) * 4): e61,
                             A.key(0, 0, (101, 101)): e2d})
    assert A.lookup(1, 0, (41,) * 4, path) == e41
    assert A.lookup(1, 0, (57,) * 4, path) == e61       # nearest node count
    assert A.lookup(1, 0, (43,) * 4, path) == e41
    assert A.lookup(0, 0, (151, 151), path) == e2d       # same model and dimension only
    assert A.lookup(1, 1, (41,) * 4, path) is None      # no FP64 entry
    assert A.lookup(2, 0, (9,) * 4, path) is None       # untuned model
    A._cache = None


def test_selection_rules():
    assert A.choose_rows({4: 30.0, 8: 20.0, 12: 20.0}) == 12   # tie: the taller tile
    assert A.choose_chunk({4: 150.0, 16: 145.0, 32: 140.7, 64: 137.6}) == 64
    assert A.choose_chunk({4: 21.0, 16: 17.0, 32: 14.9, 64: 15.1}) == 32  # within 2%: shorter


def test_row_candidates_fit_the_staging_block():
    for n in ((41,) * 4, (61,) * 4, (201, 201), (9, 9, 9, 3)):
        rs = A.row_candidates(n)
        assert rs and all(r * n[-1] <= 512 and (r + 4) * n[-1] <= 1024 for r in rs if r > 1)
