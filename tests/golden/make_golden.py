"""Write the full-size expected values of the named single-scan workloads.

Every stored value comes from the CPU oracle (``oracle/``) run over the whole
combination space of the workload; nothing here calls the GPU library.

    python tests/golden/make_golden.py [--digest] [workload ...]

Writes ``tests/golden/<workload>.json`` with the spec, the generator's
achieved heritability, and the oracle's best ``top_k`` combinations (best
first), their double-precision MI scores and their 2 x 3^k contingency tables.
With ``--digest`` it writes ``tests/golden/digest_<workload>.json`` instead:
the number of combinations and the oracle's completeness digest of all of
them (each combination hashed with its table, summed modulo 2^64).
"""
from __future__ import annotations

import json
import os
import sys
import time

_ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, _ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from synth import WORKLOADS, make_workload  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main(names):
    o = oracle.default()
    for name in names:
        G, y, spec, info = make_workload(name)
        t0 = time.time()
        res = o.scan(G, y, spec["order"], spec["top_k"], nthreads=0)
        dt = time.time() - t0
        doc = {
            "workload": name,
            "spec": {k: (list(v) if isinstance(v, tuple) else v) for k, v in spec.items()},
            "achieved_h2": info["h2"],
            "n_combinations": o.binomial(spec["M"], spec["order"]),
            "oracle_seconds": round(dt, 2),
            "oracle_threads": res["threads"],
            "combos": res["combos"].tolist(),
            "scores": [float(s) for s in res["scores"]],
            "tables": np.asarray(res["tables"], dtype=np.int64).tolist(),
            "source": "oracle/epi_oracle.c oracle_scan over the full combination space",
        }
        path = os.path.join(HERE, name + ".json")
        with open(path, "w") as f:
            json.dump(doc, f, separators=(",", ":"))
            f.write("\n")
        print(f"{name}: {dt:.1f}s, {res['threads']} threads -> {path}", flush=True)


def main_digest(names):
    o = oracle.default()
    for name in names:
        G, y, spec, _ = make_workload(name)
        t0 = time.time()
        count, digest = o.digest(G, y, spec["order"], nthreads=0)
        dt = time.time() - t0
        doc = {
            "workload": name,
            "spec": {k: (list(v) if isinstance(v, tuple) else v) for k, v in spec.items()},
            "n_combinations": count,
            "digest": digest,
            "oracle_seconds": round(dt, 2),
            "source": "oracle/epi_oracle.c oracle_digest over the full combination space",
        }
        path = os.path.join(HERE, "digest_" + name + ".json")
        with open(path, "w") as f:
            json.dump(doc, f, indent=1)
            f.write("\n")
        print(f"{name}: digest {digest} of {count} combinations, {dt:.1f}s -> {path}", flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    if args and args[0] == "--digest":
        main_digest(args[1:] or list(WORKLOADS))
    else:
        main(args or list(WORKLOADS))
