"""Writes tree_hashes.json: SHA-256 digests and counts of the oracle's elimination trees for the
full-size workloads, so the analyser can be checked bit-exactly against the oracle without
rebuilding these trees in Python on every test run.  Calls only ``oracle`` and ``fixtures``.

    python tests/golden/make_tree_hashes.py [cfg ...]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from fixtures import config_problem  # noqa: E402
from oracle.tree import build_tree, front_flops  # noqa: E402


def digest(tree):
    h = hashlib.sha256()
    for arr, dt in ((tree.parent, np.int32), (tree.level, np.int32), (tree.npiv, np.int32),
                    (tree.front_ptr, np.int64), (tree.front_idx, np.int32),
                    (tree.leaf_elem, np.int64)):
        h.update(np.ascontiguousarray(arr, dtype=dt).tobytes())
    return h.hexdigest()


def main(cfgs):
    path = os.path.join(HERE, "tree_hashes.json")
    out = json.load(open(path)) if os.path.exists(path) else {}
    for cfg in cfgs:
        t0 = time.time()
        p = config_problem(cfg)
        tree = build_tree(p.meshes)
        fac, sol, cb2 = front_flops(tree)
        ms = np.diff(tree.front_ptr)
        out[f"cfg{cfg}"] = {
            "sha256": digest(tree), "n": int(tree.n), "fronts": int(tree.n_fronts),
            "height": int(tree.height), "max_m": int(ms.max()),
            "max_m_per_level": [int(ms[tree.level == l].max()) for l in range(tree.height + 1)],
            "factor_flops": int(fac), "solve_flops_per_rhs": int(sol), "sum_cb2": int(cb2),
        }
        print(f"cfg{cfg}: {out[f'cfg{cfg}']['fronts']} fronts in {time.time() - t0:.1f}s",
              flush=True)
        json.dump(out, open(path, "w"), indent=1)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [1, 2, 3, 5, 4])
