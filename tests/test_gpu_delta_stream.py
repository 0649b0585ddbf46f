"""Triangle maintenance over the full update stream of R-MAT scale 22
(2,000 batches of 1 to 100,000 rows, log-uniform, 10% deletions, seed 1), in
the configuration bench.py times: every batch's count delta, signed output
count, stage counters, no-op counts and edge count against stored oracle
values (tests/golden/delta_stream_rmat22.json, written by
tests/golden/make_golden.py from the oracle's Delta-GJ alone).  On sampled
batches the consolidated rows and signs are compared element by element
with a live oracle that follows the stream up to the last sampled batch."""
import json
import os
import time

import numpy as np
import pytest

import oracle
import synth
from tests import queries as Q

pytestmark = pytest.mark.gpu

GOLDEN_PATH = os.path.join(os.path.dirname(__file__), "golden", "delta_stream_rmat22.json")


@pytest.fixture(scope="module")
def gj():
    import paper_1802_03760_amd as gj
    return gj


def sampled(batches, at=(0, 1, 2, 120, 250, 399), max_rows=20000):
    """The first batch at or after each position with at most max_rows rows."""
    out = []
    for p in at:
        for row in batches[p:]:
            if row[1] <= max_rows:
                out.append(row[0])
                break
    return sorted(set(out))


def test_delta_stream_rmat22(gj):
    GOLD = json.load(open(GOLDEN_PATH))
    s = GOLD["stream"]
    spec = s["graph"]
    n = 1 << spec["scale"]
    cols = GOLD["columns"]
    rows_g = [dict(zip(cols, r)) for r in GOLD["batches"]]
    assert len(rows_g) == s["batches"] == 2000
    src, dst = synth.rmat_draws(spec["scale"], spec["edge_factor"], spec["seed"])
    ctx = gj.Context(0)
    G = gj.Graph(ctx, src, dst, n)
    q = gj.Query(ctx, *Q.TRIANGLE)
    check = set(sampled(GOLD["batches"]))
    O = oracle.Graph(n, src, dst)
    last = max(check)
    del src, dst
    t0 = time.time()
    for k, bs, bd, bg in synth.update_stream(spec["scale"], spec["seed"], s["stream_seed"], s["batches"],
                                             s["size_lo"], s["size_hi"], s["delete_fraction"]):
        g = rows_g[k]
        assert g["batch"] == k and g["rows_in_batch"] == len(bs)
        if k in check:
            ref = oracle.delta(O, bs, bd, bg, Q.TRIANGLE, rows=True, threads=16)
            got = gj.apply_updates(ctx, G, bs, bd, bg, [q], rows=True)[0]
            assert np.array_equal(got["rows"], ref["rows"]), k
            assert np.array_equal(got["signs"], ref["signs"]), k
            assert ref["count_delta"] == g["count_delta"], k
            print("batch %d (%d rows): %d delta rows equal the oracle's" % (k, len(bs), len(ref["rows"])),
                  flush=True)
        else:
            if k < last:
                oracle.delta(O, bs, bd, bg)  # the live oracle follows the stream
            elif k == last + 1:
                del O  # no sampled batch beyond this point
            got = gj.apply_updates(ctx, G, bs, bd, bg, [q])[0]
        st = got["stats"]
        assert got["count_delta"] == g["count_delta"], k
        assert st["raw_emissions"] == g["raw_emissions"], k
        assert st["prefixes"][2] == g["prefixes2"] and st["extensions"][2] == g["extensions2"], k
        assert (st["noop_inserts"], st["noop_deletes"]) == (g["noop_inserts"], g["noop_deletes"]), k
        assert G.info(degrees=False)["edges"] == g["edges_after"], k
        if k % 250 == 249:
            print("delta stream: %d batches equal the oracle's (%.0f s)" % (k + 1, time.time() - t0), flush=True)
    G.close()
    ctx.close()
