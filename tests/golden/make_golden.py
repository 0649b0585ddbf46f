#!/usr/bin/env python3
"""Writes the stored expected values of the full-size parity tests.

Every number comes from the CPU oracle (oracle/) on inputs from the seeded
generators (synth/); nothing here loads the GPU library.  Two files:

* full_counts.json -- whole-graph counts and per-stage Generic Join counters:
  by the oracle's Generic Join (method "gj"), or for the diamond and the
  4-cycle on graphs where that is too slow by the oracle's 2-path counting
  (method "twopath", which the CPU tests pin against Generic Join, brute
  force and dense identities).
* delta_stream_rmat22.json -- triangle maintenance over the update stream of
  R-MAT scale 22 (2,000 batches of 1 to 100,000 rows, log-uniform, 10%
  deletions, seed 1): per batch the signed change of the count, the number of
  signed outputs of the delta queries before consolidation, the stage
  counters, the no-op counts and the edge count after the batch, from the
  oracle's Delta-GJ (count-only mode) applied batch after batch.

Usage: python tests/golden/make_golden.py [--only NAME ...] [--threads T]
Entries already in a file are kept unless named with --only.
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402
from tests import queries as Q  # noqa: E402

FULL = os.path.join(HERE, "full_counts.json")
DELTA = os.path.join(HERE, "delta_stream_rmat22.json")


def rmat(scale, build="directed"):
    return {"generator": "rmat", "scale": scale, "edge_factor": 16, "abc": list(synth.RMAT_ABC), "seed": 0,
            "build": build}


# name -> (graph, query name, method)
ENTRIES = {
    "rmat20_triangle": (rmat(20), "triangle", "gj"),
    "rmat22_triangle": (rmat(22), "triangle", "gj"),
    "rmat20_cyclic_triangle": (rmat(20), "cyclic_triangle", "gj"),
    "rmat14_clique4": (rmat(14), "clique4", "gj"),
    "rmat14_diamond": (rmat(14), "diamond", "gj"),
    "rmat14_cycle4": (rmat(14), "cycle4", "gj"),
    "rmat12_clique5": (rmat(12), "clique5", "gj"),
    "rmat16_clique4": (rmat(16), "clique4", "gj"),
    "rmat18_diamond": (rmat(18), "diamond", "twopath"),
    "rmat18_cycle4": (rmat(18), "cycle4", "twopath"),
    "rmat20_diamond": (rmat(20), "diamond", "twopath"),
    "rmat20_cycle4": (rmat(20), "cycle4", "twopath"),
    "rmat22_diamond": (rmat(22), "diamond", "twopath"),
    "rmat22_cycle4": (rmat(22), "cycle4", "twopath"),
    "rmat18_oriented_clique4": (rmat(18, "degree_order"), "clique4", "gj"),
    "rmat16_oriented_clique5": (rmat(16, "degree_order"), "clique5", "gj"),
}

DELTA_STREAM = {"graph": rmat(22), "query": "triangle", "stream_seed": 1, "batches": 2000, "size_lo": 1,
                "size_hi": 100000, "delete_fraction": 0.1}


def oracle_graph(spec, cache):
    key = (spec["scale"], spec["build"])
    if key not in cache:
        cache.clear()
        n = 1 << spec["scale"]
        src, dst = synth.rmat_draws(spec["scale"], spec["edge_factor"], spec["seed"])
        if spec["build"] == "degree_order":
            src, dst, _ = oracle.relabel_by_degree(n, src, dst)
        cache[key] = oracle.Graph(n, src, dst)
    return cache[key]


def load(path):
    return json.load(open(path)) if os.path.exists(path) else {}


def save(path, obj):
    """Indented JSON, except that a list of lists (the per-batch rows) keeps
    one inner list per line."""
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        f.write("{\n")
        keys = sorted(obj)
        for i, k in enumerate(keys):
            v = obj[k]
            if isinstance(v, list) and v and isinstance(v[0], list):
                body = "[\n" + ",\n".join("  " + json.dumps(r) for r in v) + "\n ]"
            else:
                body = json.dumps(v, indent=1, sort_keys=True).replace("\n", "\n ")
            f.write(" %s: %s%s\n" % (json.dumps(k), body, "," if i + 1 < len(keys) else ""))
        f.write("}\n")
    os.replace(tmp, path)


def make_full(names, threads):
    out = load(FULL)
    out.setdefault("entries", {})
    out["note"] = ("written by tests/golden/make_golden.py from the CPU oracle alone; "
                   "queries as in tests/queries.py")
    cache = {}
    for name in names:
        spec, qname, method = ENTRIES[name]
        G = oracle_graph(spec, cache)
        t = time.time()
        if method == "gj":
            r = oracle.run(G, Q.ALL[qname], threads=threads)
        else:
            r = oracle.twopath(G, qname, threads=threads)
        el = time.time() - t
        out["entries"][name] = {"graph": spec, "query": qname, "method": method, "matches": r["matches"],
                                "prefixes": r["prefixes"], "extensions": r["extensions"],
                                "edges": G.num_edges, "oracle_seconds": round(el, 1), "oracle_threads": threads}
        save(FULL, out)
        print("%s: %d matches (%s, %.1f s)" % (name, r["matches"], method, el), flush=True)


def make_delta(threads):
    spec = DELTA_STREAM["graph"]
    n = 1 << spec["scale"]
    src, dst = synth.rmat_draws(spec["scale"], spec["edge_factor"], spec["seed"])
    G = oracle.Graph(n, src, dst)
    del src, dst
    q = Q.ALL[DELTA_STREAM["query"]]
    rows = []
    t0 = time.time()
    for k, bs, bd, bg in synth.update_stream(spec["scale"], spec["seed"], DELTA_STREAM["stream_seed"],
                                             DELTA_STREAM["batches"], DELTA_STREAM["size_lo"],
                                             DELTA_STREAM["size_hi"], DELTA_STREAM["delete_fraction"]):
        before = G.noops()
        r = oracle.delta(G, bs, bd, bg, q, rows=False, threads=threads)
        after = G.noops()
        rows.append([k, len(bs), r["count_delta"], r["raw_emissions"], r["prefixes"][2], r["extensions"][2],
                     after[0] - before[0], after[1] - before[1], G.num_edges])
        if k % 100 == 99:
            print("delta stream: %d batches, %.0f s" % (k + 1, time.time() - t0), flush=True)
    save(DELTA, {"stream": DELTA_STREAM,
                 "columns": ["batch", "rows_in_batch", "count_delta", "raw_emissions", "prefixes2",
                             "extensions2", "noop_inserts", "noop_deletes", "edges_after"],
                 "batches": rows, "oracle_seconds": round(time.time() - t0, 1), "oracle_threads": threads,
                 "note": "written by tests/golden/make_golden.py from the CPU oracle alone"})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", nargs="*", default=None)
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    names = args.only if args.only is not None else list(ENTRIES) + ["delta_stream"]
    full = [x for x in names if x in ENTRIES]
    if full:
        make_full(full, args.threads)
    if "delta_stream" in names:
        make_delta(args.threads)


if __name__ == "__main__":
    main()
