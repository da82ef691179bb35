"""Write full-size expected pair counts computed by the CPU oracle only.

Usage: python tests/golden/make_golden.py [name ...]

Each entry records the workload, the binning, the SHA-256 of the generated
input catalog(s) and the oracle's uint64 counts. The GPU tests regenerate the
same seeded catalogs, check the hashes and compare counts bit for bit.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import catalogs  # noqa: E402
import oracle  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def rmu_binning():
    return (np.arange(41) * 5.0, np.arange(51) / 50.0)


def make_clustered_1e6_dd_rmu():
    d, _ = catalogs.clustered_box_1e6()
    re_, me = rmu_binning()
    t = time.time()
    h = oracle.count_pairs(d, None, oracle.Binning(oracle.RMU, re_, me, los=oracle.LOS_Z),
                           prune=True)
    return {
        "workload": "r-mu DD, 1e6 clustered points (1e4 Gaussian blobs of 100, sigma 5) in an "
                    "open 2000^3 box, r in [0,200) 40 bins, mu in [0,1] 50 bins, line of sight z",
        "generator": "catalogs.clustered_box_1e6() data catalog",
        "sha256": catalogs.sha256_of(d),
        "n": len(d),
        "r_edges": re_.tolist(),
        "mu_edges": me.tolist(),
        "counts": h.reshape(-1).astype(np.uint64).tolist(),
        "oracle_seconds": time.time() - t,
    }


def make_periodic_2e4_dd_mono():
    c = catalogs.periodic_uniform_2e4()
    e = np.arange(31) * 5.0
    t = time.time()
    h = oracle.count_pairs(c, None, oracle.Binning(oracle.MONO, e, periodic=True, L=1000.0))
    return {
        "workload": "monopole DD, 20000 uniform points in a periodic 1000^3 box, r in [0,150) "
                    "30 bins (brute force over all pairs)",
        "generator": "catalogs.periodic_uniform_2e4()",
        "sha256": catalogs.sha256_of(c),
        "n": len(c),
        "r_edges": e.tolist(),
        "counts": h.reshape(-1).astype(np.uint64).tolist(),
        "oracle_seconds": time.time() - t,
    }


MAKERS = {"periodic_2e4_dd_mono": make_periodic_2e4_dd_mono,
          "clustered_1e6_dd_rmu": make_clustered_1e6_dd_rmu}


if __name__ == "__main__":
    names = sys.argv[1:] or list(MAKERS)
    for name in names:
        rec = MAKERS[name]()
        rec["source"] = ("computed by tests/golden/make_golden.py with the CPU oracle "
                         "(oracle/oracle.c); no GPU value was used")
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(rec, f)
        print(name, "done in %.1f s" % rec["oracle_seconds"], flush=True)
