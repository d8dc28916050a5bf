"""Write the oracle's full-size reference values to tests/golden/.

    python tests/golden/make_goldens.py cfg2 cfg3 [--procs 8]

For each workload (the seeded generators of `synth`, seed 0):
  * the exact neighbor lists of every point, from oracle.neighbors.lag_pruned
    (rows split over worker processes; each row is computed independently),
    stored as the SHA-256 of the whole int32 [n, m] array and of each block of
    `block_rows` rows, so that a test can check every row bit for bit and name
    the blocks that differ;
  * the FP64 VIF negative log-likelihood of oracle.likelihood.vif on those
    lists, with its four terms (sum log D_i, z'z, log det M, q'M^-1 q).

Only `oracle/` and `synth` are called; nothing here comes from the HIP path.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import likelihood as LK  # noqa: E402
from oracle import neighbors as NB  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
BLOCK_ROWS = 65536

_DATA = {}


def _make(name):
    if name == "cfg2":
        return synth.config_cfg2()
    if name == "cfg3":
        return synth.config_cfg3()
    raise ValueError(name)


def _rows_worker(args):
    name, a, b = args
    d = _DATA[name]
    return a, NB.lag_pruned(d["kern"], d["sx"], d["sy"], d["t"], d["m"], rows=np.arange(a, b))


def nbr_hashes(nbr, block_rows=BLOCK_ROWS):
    """SHA-256 of the C-ordered little-endian int32 array, whole and per block of rows."""
    a = np.ascontiguousarray(nbr, dtype="<i4")
    blocks = [hashlib.sha256(a[r:r + block_rows].tobytes()).hexdigest()
              for r in range(0, a.shape[0], block_rows)]
    return hashlib.sha256(a.tobytes()).hexdigest(), blocks


def run(name, procs):
    t0 = time.time()
    d = _make(name)
    _DATA[name] = d
    n, m = d["n"], d["m"]
    print(f"[{name}] {d['name']} generated in {time.time() - t0:.1f} s", flush=True)
    step = 4096
    jobs = [(name, a, min(a + step, n)) for a in range(0, n, step)]
    nbr = np.full((n, m), -1, dtype=np.int32)
    t1 = time.time()
    with mp.get_context("fork").Pool(procs) as pool:
        for a, rows in pool.imap_unordered(_rows_worker, jobs):
            nbr[a:a + rows.shape[0]] = rows
    print(f"[{name}] neighbors in {time.time() - t1:.1f} s", flush=True)
    full, blocks = nbr_hashes(nbr)
    t2 = time.time()
    X = (d["sx"], d["sy"], d["t"])
    Z = (d["zx"], d["zy"], d["zt"])
    o = LK.vif(d["kern"], X, d["y"], nbr, Z)
    print(f"[{name}] VIF NLL {o['nll']!r} in {time.time() - t2:.1f} s", flush=True)
    out = {
        "_source": "tests/golden/make_goldens.py: oracle.neighbors.lag_pruned and "
                   "oracle.likelihood.vif (FP64) on synth.config_" + name + "(seed=0)",
        "workload": d["name"],
        "n": n, "m": m, "k": d["k"],
        "nll": o["nll"],
        "sum_logD": o["sum_logD"],
        "zz": o["zz"],
        "logdetM": o["logdetM"],
        "quadM": o["quadM"],
        "nbr_sha256": full,
        "nbr_block_rows": BLOCK_ROWS,
        "nbr_block_sha256": blocks,
        "numpy": np.__version__,
        "python": platform.python_version(),
    }
    path = os.path.join(HERE, f"oracle_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(f"[{name}] wrote {path} ({time.time() - t0:.1f} s in all)", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("configs", nargs="+", choices=["cfg2", "cfg3"])
    ap.add_argument("--procs", type=int, default=min(8, os.cpu_count() or 1))
    args = ap.parse_args()
    for name in args.configs:
        run(name, args.procs)


if __name__ == "__main__":
    main()
