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


def _rmu_box_record(kind, cat_d, cat_r, h, t, note):
    re_, me = rmu_binning()
    return {
        "workload": "r-mu %s, 1e6 clustered points (1e4 Gaussian blobs of 100, sigma 5) and 2e6 "
                    "uniform randoms in an open 2000^3 box, r in [0,200) 40 bins, mu in [0,1] 50 "
                    "bins, line of sight z" % kind,
        "generator": note,
        "sha256_data": catalogs.sha256_of(cat_d),
        "sha256_randoms": catalogs.sha256_of(cat_r),
        "r_edges": re_.tolist(),
        "mu_edges": me.tolist(),
        "counts": h.reshape(-1).astype(np.uint64).tolist(),
        "oracle_seconds": time.time() - t,
    }


def make_clustered_1e6_dr_rmu():
    d, r = catalogs.clustered_box_1e6()
    re_, me = rmu_binning()
    t = time.time()
    h = oracle.count_pairs(d, r, oracle.Binning(oracle.RMU, re_, me, los=oracle.LOS_Z), prune=True)
    return _rmu_box_record("DR", d, r, h, t, "catalogs.clustered_box_1e6() data x randoms")


def make_clustered_1e6_rr_rmu():
    d, r = catalogs.clustered_box_1e6()
    re_, me = rmu_binning()
    t = time.time()
    h = oracle.count_pairs(r, None, oracle.Binning(oracle.RMU, re_, me, los=oracle.LOS_Z),
                           prune=True)
    return _rmu_box_record("RR", d, r, h, t, "catalogs.clustered_box_1e6() randoms")


def _lightcone(kind):
    d, r = catalogs.lightcone_3e6()
    e = np.arange(76) * 2.0
    ob = oracle.Binning(oracle.SIGMAPI, e, e, los=oracle.LOS_MID)
    t = time.time()
    a, b = {"DD": (d, None), "DR": (d, r), "RR": (r, None)}[kind]
    h = oracle.count_pairs(a, b, ob, prune=True)
    return {
        "workload": "sigma-pi %s of the light cone: 3e6 data and 6e6 randoms, RA in [0, 60] deg, "
                    "Dec in [0, 30] deg, Gaussian n(z) (0.6, 0.15), flat LCDM Om=0.3; sigma and pi "
                    "edges 2k Mpc/h (k <= 75), midpoint line of sight" % kind,
        "generator": "catalogs.lightcone_3e6()",
        "sha256_data": catalogs.sha256_of(d),
        "sha256_randoms": catalogs.sha256_of(r),
        "edges": e.tolist(),
        "counts": h.reshape(-1).astype(np.uint64).tolist(),
        "oracle_seconds": time.time() - t,
    }


def make_lightcone_3e6_dd_sigmapi():
    return _lightcone("DD")


def make_lightcone_3e6_dr_sigmapi():
    return _lightcone("DR")


def make_lightcone_3e6_rr_sigmapi():
    return _lightcone("RR")


def mocks_sha256(mocks):
    """One digest over every mock's SHA-256, in mock order."""
    import hashlib
    h = hashlib.sha256()
    for m in mocks:
        h.update(catalogs.sha256_of(m).encode())
    return h.hexdigest()


def make_batched_mocks_256():
    """Monopole and r-mu DD of all 256 mocks, and the 100 leave-one-column-out
    jackknife catalogs of the 1e6-point base (both binnings). The counts go to
    batched_mocks_256.npz beside this record."""
    import hashlib
    L = 1000.0
    mocks, base, region = catalogs.batched_mocks_256()
    e_mono = np.arange(31) * 5.0
    re_, me = rmu_binning()
    mono = oracle.Binning(oracle.MONO, e_mono, periodic=True, L=L)
    rmu = oracle.Binning(oracle.RMU, re_, me, los=oracle.LOS_Z, periodic=True, L=L)
    t = time.time()
    c_mono = np.stack([oracle.count_pairs(m, None, mono, prune=True) for m in mocks])
    print("  mocks monopole %.0f s" % (time.time() - t), flush=True)
    c_rmu = np.stack([oracle.count_pairs(m, None, rmu, prune=True) for m in mocks])
    print("  mocks r-mu %.0f s" % (time.time() - t), flush=True)
    tot_mono, jk_mono = oracle.count_jackknife(base, region, 100, mono)
    tot_rmu, jk_rmu = oracle.count_jackknife(base, region, 100, rmu)
    np.savez_compressed(os.path.join(HERE, "batched_mocks_256.npz"),
                        mono=c_mono.astype(np.uint64), rmu=c_rmu.astype(np.uint64),
                        jk_total_mono=tot_mono.astype(np.uint64), jk_mono=jk_mono.astype(np.uint64),
                        jk_total_rmu=tot_rmu.astype(np.uint64), jk_rmu=jk_rmu.astype(np.uint64))
    with open(os.path.join(HERE, "batched_mocks_256.npz"), "rb") as f:
        npz_sha = hashlib.sha256(f.read()).hexdigest()
    return {
        "workload": "DD of 256 periodic mocks (L = 1000, 2e4..5e5 points, half uniform half "
                    "Gaussian blobs) with the monopole (r < 150, 30 bins) and r-mu (r < 200, 40 "
                    "bins x mu 50 bins, line of sight z) binnings; the 100 jackknife catalogs of "
                    "the 1e6-point base (one 100 x 100 column of (x, y) left out each), both "
                    "binnings",
        "generator": "catalogs.batched_mocks_256()",
        "sha256_mocks": mocks_sha256(mocks),
        "sha256_base": catalogs.sha256_of(base),
        "sha256_region": hashlib.sha256(np.ascontiguousarray(region, dtype="<i4").tobytes()).hexdigest(),
        "mono_edges": e_mono.tolist(),
        "r_edges": re_.tolist(),
        "mu_edges": me.tolist(),
        "counts_file": "batched_mocks_256.npz",
        "counts_file_sha256": npz_sha,
        "arrays": {"mono": "[256, 30]", "rmu": "[256, 40, 50]", "jk_total_mono": "[30]",
                   "jk_mono": "[100, 30] row k = base without region k",
                   "jk_total_rmu": "[40, 50]", "jk_rmu": "[100, 40, 50]"},
        "oracle_seconds": time.time() - t,
    }


def cap_sample(cat, n_random, n_edge, seed):
    """Sample rows of an angular catalog: n_random points drawn without
    replacement (seeded) and the n_edge points farthest from the cap centre
    (RA 180 deg, Dec 0, i.e. the largest x), sorted indices."""
    g = np.random.Generator(np.random.PCG64(seed))
    edge = np.argsort(-cat.x, kind="stable")[:n_edge]
    rest = np.setdiff1d(np.arange(len(cat)), edge)
    pick = g.choice(rest, n_random, replace=False)
    return np.sort(np.concatenate([edge, pick]))


def make_angular_cap_1e7_rows():
    """Sampled rows of the angular workload: 1024 data points (768 random blob
    members, 256 at the cap edge) and 1024 randoms (likewise) against the
    whole data and random catalogs (cross counts, self pairs included)."""
    d, r = catalogs.angular_cap_1e7()
    e = np.deg2rad(0.001 * 10.0 ** (np.arange(31) * 4.0 / 30.0))
    ob = oracle.Binning(oracle.THETA, e)
    sd = cap_sample(d, 768, 256, seed=4101)
    sr = cap_sample(r, 768, 256, seed=4102)
    t = time.time()
    rows = {}
    for sname, cat, idx in (("sd", d, sd), ("sr", r, sr)):
        s = cat.subset(idx)
        for oname, other in (("d", d), ("r", r)):
            rows["%s_x_%s" % (sname, oname)] = oracle.count_pairs(s, other, ob, prune=True)
            print("  %s x %s %.0f s" % (sname, oname, time.time() - t), flush=True)
    return {
        "workload": "theta rows of the angular cap: 1e7 clustered data and 2e7 randoms in a "
                    "5000 sq-deg cap; 30 log bins of theta in [0.001, 10] deg; rows of 1024 "
                    "sampled data points (sd) and 1024 sampled randoms (sr) against the whole "
                    "data (d) and random (r) catalogs, self pairs included",
        "generator": "catalogs.angular_cap_1e7(); sample = cap_sample(cat, 768, 256, seed)",
        "sha256_data": catalogs.sha256_of(d),
        "sha256_randoms": catalogs.sha256_of(r),
        "theta_edges_rad": e.tolist(),
        "sample_data_idx": sd.tolist(),
        "sample_randoms_idx": sr.tolist(),
        "counts": {k: v.reshape(-1).astype(np.uint64).tolist() for k, v in rows.items()},
        "oracle_seconds": time.time() - t,
    }


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


MAKERS = {"periodic_2e4_dd_mono": make_periodic_2e4_dd_mono,
          "clustered_1e6_dd_rmu": make_clustered_1e6_dd_rmu,
          "clustered_1e6_dr_rmu": make_clustered_1e6_dr_rmu,
          "clustered_1e6_rr_rmu": make_clustered_1e6_rr_rmu,
          "angular_cap_1e7_rows": make_angular_cap_1e7_rows,
          "batched_mocks_256": make_batched_mocks_256,
          "lightcone_3e6_dd_sigmapi": make_lightcone_3e6_dd_sigmapi,
          "lightcone_3e6_dr_sigmapi": make_lightcone_3e6_dr_sigmapi,
          "lightcone_3e6_rr_sigmapi": make_lightcone_3e6_rr_sigmapi}


if __name__ == "__main__":
    names = sys.argv[1:] or list(MAKERS)
    for name in names:
        rec = MAKERS[name]()
        rec["source"] = ("computed by tests/golden/make_golden.py with the CPU oracle "
                         "(oracle/oracle.c); no GPU value was used")
        rec["threads"] = os.cpu_count()
        rec["host"] = cpu_model()
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(rec, f)
        print(name, "done in %.1f s" % rec["oracle_seconds"], flush=True)
