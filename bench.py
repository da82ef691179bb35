"""Benchmark of the pair-counting hot path on one MI355X.

Workload (one "step"): the r-mu DD pair count of 1e6 clustered points
(1e4 Gaussian blobs of 100 points, sigma 5, in an open 2000^3 box), r in
[0, 200) with 40 bins and mu in [0, 1] with 50 bins, line of sight z:
  1. build the cell list from device-resident float64 positions,
  2. count the autocorrelation with FP32 separations and the FP64 re-test of
     every pair inside a rounding band of a decision (bit-exact counts),
  3. leave the uint64 counts in device memory.
The metric is candidate pair evaluations per second (the cell-list pairs the
kernel evaluates), counted only when the counts are bit-exact; the FP64
counter is timed the same way for the speedup.

Prints one JSON line. Run with --gpus 1 (the only supported value).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_LANE_OPS = 256 * 64 * 2.4e9     # unpacked VALU lane-instructions/s (256 CUs, 2.4 GHz)
PEAK_FP32_FLOPS = 157.3e12            # FP32 vector peak (packed FMA counted as 4 flops per lane)
I_ALG_RMU_Z = 21                      # algorithmic FP32 lane-ops per r-mu pair evaluation


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_info():
    """Host CPU model and core counts (the oracle's timing context)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except Exception:
        affinity = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cores": affinity,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(d, target_s=15.0):
    """The CPU oracle (brute force, every pair) on a bounded prefix of the
    same data catalog, on every core this process may use (the job's CPU
    share: OMP_NUM_THREADS when set, else the affinity mask), and once on one
    thread; rates in the same unit. The pruned oracle time to solution of
    the whole workload comes from the golden record (measured when the
    expected counts were made)."""
    import oracle
    info = host_info()
    threads = int(info["omp_num_threads"] or 0) or info["affinity_cores"]
    threads = max(1, threads)
    re_, me = np.arange(41) * 5.0, np.arange(51) / 50.0
    ob = oracle.Binning(oracle.RMU, re_, me, los=oracle.LOS_Z)
    n = 20000
    t = time.perf_counter()
    oracle.count_pairs(d.head(n), None, ob, nthreads=threads)
    dt = time.perf_counter() - t
    rate = n * (n - 1) / 2 / max(dt, 1e-9)
    n2 = int(min(len(d), math.sqrt(2 * rate * target_s)))
    t = time.perf_counter()
    oracle.count_pairs(d.head(n2), None, ob, nthreads=threads)
    dt = time.perf_counter() - t
    pairs = n2 * (n2 - 1) / 2
    # one thread, about 4 s of work
    n1 = int(min(len(d), math.sqrt(2 * rate / threads * 4.0)))
    t = time.perf_counter()
    oracle.count_pairs(d.head(n1), None, ob, nthreads=1)
    dt1 = time.perf_counter() - t
    out = {"value": pairs / dt / 1e9, "unit": "Gpair-evals/s", "cores": threads, "kind": "oracle",
           "sample": "brute-force DD (all %d pairs) of the first %d points of the same clustered "
                     "catalog, same r-mu binning, %.1f s" % (pairs, n2, dt),
           "single_thread": {"value": n1 * (n1 - 1) / 2 / dt1 / 1e9, "unit": "Gpair-evals/s",
                             "sample": "first %d points, %.1f s" % (n1, dt1)},
           "host": info}
    golden = os.path.join(ROOT, "tests", "golden", "clustered_1e6_dd_rmu.json")
    if os.path.exists(golden):
        with open(golden) as f:
            g = json.load(f)
        out["pruned_time_to_solution_s"] = {
            "value": round(g["oracle_seconds"], 1),
            "what": "the whole DD of the 1e6-point workload with the exact band-and-window prune",
            "threads": g.get("threads", 8), "where": g.get("host", "the build container")}
    return out


def batched_leg(cute, torch, dev, runs=1):
    """The batched mock workload: 256 periodic mocks (2e4 .. 5e5 points, log-
    uniform, half clustered) and the 100 jackknife catalogs of a 1e6-point base
    (one 100 x 100 Mpc/h column left out each), every catalog counted with the
    monopole (30 bins to 150) and the r-mu (40 x 50 bins to 200) binnings:
    712 autocorrelations, one batch (two persistent launches in one graph)."""
    import catalogs
    t0 = time.perf_counter()
    mocks, base, region = catalogs.batched_mocks_256()
    L = 1000.0
    t_gen = time.perf_counter() - t0
    mono = cute.Binning(cute.BIN_MONO, np.arange(31) * 5.0)
    rmu = cute.Binning(cute.BIN_RMU, np.arange(41) * 5.0, np.arange(51) / 50.0, los=cute.LOS_Z)

    def dxyz(cat):
        return [torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in (cat.x, cat.y, cat.z)]

    # grid layout (cell side, tile size) from the tuner: on the smallest, the
    # median and the largest mock (each mock takes the choice of the nearest
    # size on a log scale) and on the jackknife base
    t0 = time.perf_counter()
    sizes = np.array([len(m) for m in mocks])
    reps = [int(np.argmin(sizes)), int(np.argsort(sizes)[len(sizes) // 2]), int(np.argmax(sizes))]
    tuned = {}
    for k in reps:
        c, t, _ = cute.tune_grid(dxyz(mocks[k]), cute.GEOM_BOX_PERIODIC, rmu, box_size=L, r_max=200.0)
        tuned[k] = (c, t)
    cb, tb, _ = cute.tune_grid(dxyz(base), cute.GEOM_BOX_PERIODIC, rmu, box_size=L, r_max=200.0)
    t_tune = time.perf_counter() - t0

    def layout(n):
        k = min(reps, key=lambda r: abs(np.log(sizes[r]) - np.log(n)))
        return tuned[k]

    t0 = time.perf_counter()
    gm = []
    for m in mocks:
        c, t = layout(len(m))
        gm.append(cute.build_grid(dxyz(m), cute.GEOM_BOX_PERIODIC, box_size=L, r_max=200.0,
                                  cell_size=c, tile_points=t))
    gb = cute.build_grid(dxyz(base), cute.GEOM_BOX_PERIODIC, box_size=L, r_max=200.0,
                         cell_size=cb, tile_points=tb)
    torch.cuda.synchronize()
    t_grid = time.perf_counter() - t0
    reg = torch.from_numpy(region).to(dev)
    items = []
    for g in gm:
        items += [cute.BatchItem(g, None, mono), cute.BatchItem(g, None, rmu)]
    for k in range(100):
        m = (reg == k).to(torch.uint8)
        items += [cute.BatchItem(gb, None, mono, mask_a=m), cute.BatchItem(gb, None, rmu, mask_a=m)]
    t0 = time.perf_counter()
    b = cute.Batch(items, cute.PREC_FP32_EDGE)
    t_plan = time.perf_counter() - t0
    log("bench: batched workload, %d items, planned in %.2f s" % (len(items), t_plan))
    b.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(runs):
        b.run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / runs
    st = b.stats()
    # spot checks: two mocks and one jackknife catalog against the single-count path
    allc = b.counts()
    ok = True
    for k in (0, len(items) // 2 - 1, len(items) - 1):
        it = items[k]
        w, o = b.layout(k)
        if it.mask_a is None:
            ref = cute.count_pairs(it.a, None, it.binning, cute.PREC_FP64).reshape(-1)
        else:
            keep = torch.nonzero(it.mask_a == 0).flatten()
            sub = [torch.from_numpy(np.ascontiguousarray(v)).to(dev)[keep] for v in (base.x, base.y, base.z)]
            gs = cute.build_grid(sub, cute.GEOM_BOX_PERIODIC, box_size=L, r_max=200.0)
            ref = cute.count_pairs(gs, None, it.binning, cute.PREC_FP64).reshape(-1)
            gs.close()
        ok = ok and bool(np.array_equal(allc[o:o + w], ref))
    # the same 100 jackknife catalogs by region decomposition (two passes over
    # the base whatever the number of regions), checked row by row against
    # the masked catalogs of the batch
    jk = {}
    reg_h = np.ascontiguousarray(region, dtype=np.int32)
    jk_ok = True
    for name, bn_, first in (("monopole", mono, 2 * len(gm)), ("r_mu", rmu, 2 * len(gm) + 1)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        total, jack, jst = cute.count_jackknife(gb, reg_h, 100, bn_, cute.PREC_FP32_EDGE,
                                                with_stats=True)
        dt = time.perf_counter() - t0
        for k in range(100):
            w, o = b.layout(first + 2 * k)
            jk_ok = jk_ok and bool(np.array_equal(jack[k].reshape(-1), allc[o:o + w]))
        jk[name] = {"wall_ms": round(dt * 1e3, 2), "kernel_ms": round(jst["ms_count"], 2),
                    "pair_evals": int(jst["pair_evals"])}
    # the DR jackknife of the same base against 1e6 uniform randoms with the
    # same column regions (three passes whatever the number of regions)
    rnd = catalogs.uniform_box(1_000_000, L, seed=5600)
    rreg = (np.minimum((rnd.y * (10.0 / L)).astype(np.int64), 9) * 10
            + np.minimum((rnd.x * (10.0 / L)).astype(np.int64), 9)).astype(np.int32)
    grn = cute.build_grid([torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in (rnd.x, rnd.y, rnd.z)],
                          cute.GEOM_BOX_PERIODIC, box_size=L, r_max=200.0, cell_size=cb, tile_points=tb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, jst = cute.count_jackknife_cross(gb, reg_h, grn, rreg, 100, rmu, cute.PREC_FP32_EDGE,
                                           with_stats=True)
    dt = time.perf_counter() - t0
    jk["r_mu_dr_vs_1e6_randoms"] = {"wall_ms": round(dt * 1e3, 2), "kernel_ms": round(jst["ms_count"], 2),
                                    "pair_evals": int(jst["pair_evals"])}
    grn.close()
    b.close()
    return {"jackknife_by_regions": dict(jk, bit_exact_vs_masked_batch=jk_ok,
                                         note="all 100 jackknife catalogs of the base, per binning"),
            "workload": "256 periodic mocks (2e4..5e5 points) + 100 jackknife catalogs of a 1e6 base, "
                        "each with monopole (30 bins, r<150) and r-mu (40x50, r<200) DD; 712 items",
            "items": len(items), "ms_per_run": round(ms, 3), "runs": runs,
            "pair_evals": int(st["pair_evals"]), "pairs_in_range": int(st["pairs_in_range"]),
            "gpair_evals_per_s": round(st["pair_evals"] / (ms * 1e-3) / 1e9, 3),
            "retests": int(st["retests"]), "spot_checks_bit_exact_vs_fp64_single": ok,
            "tuned_layout": {"mocks": {str(int(sizes[k])): {"cell": round(c, 3), "tile": t}
                                       for k, (c, t) in tuned.items()},
                             "jackknife_base": {"cell": round(cb, 3), "tile": tb}},
            "host_s": {"generate": round(t_gen, 2), "tune": round(t_tune, 2),
                       "grids": round(t_grid, 2), "plan": round(t_plan, 2)}}


# the paper's Table 2 (Server-GPU column: Tesla C2070, DR brute force, double
# precision, seconds), quoted as context
TABLE2_SERVER_GPU_S = {"xi_lin": 13.0, "xi_log": 20.0, "w_theta": 22.0, "w_pix": 0.46,
                       "xi_sigma_pi": 27.0}
# 2048 rings x 4028 sectors: pixels of 5.0e-3 sq-deg, the Table 2 resolution
TABLE2_PIX = (2048, 4028)


def table2_leg(cute, torch, dev, reps=3):
    """The correlation functions of the paper's Table 2 on a synthetic
    light-cone subset of its shape (RA, Dec in [0, 18] deg, z in [0.5, 0.6],
    3e5 data and 3e5 randoms, uniform in volume): the DR histogram, brute
    force (one cell holds every point) and with the cell list, FP32_EDGE and
    FP64. Brute force and cell list must give the same counts."""
    import catalogs
    d, r = catalogs.table2()
    du, ru = catalogs.unit_vectors(d), catalogs.unit_vectors(r)
    funcs = {
        "xi_lin": (cute.Binning(cute.BIN_MONO, np.linspace(0.0, 100.0, 257)), False),
        "xi_log": (cute.Binning(cute.BIN_MONO, 100.0 * 10.0 ** ((np.arange(257) - 256) / 50.0)), False),
        "w_theta": (cute.Binning(cute.BIN_THETA, np.deg2rad(np.linspace(0.0, 30.0, 257))), True),
        "xi_sigma_pi": (cute.Binning(cute.BIN_SIGMAPI, np.linspace(0.0, 100.0, 65),
                                     np.linspace(0.0, 100.0, 65), los=cute.LOS_MIDPOINT), False),
    }

    def dxyz(cat):
        return [torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in (cat.x, cat.y, cat.z)]

    out = {}
    for name, (bn, sphere) in funcs.items():
        geom = cute.GEOM_SPHERE if sphere else cute.GEOM_BOX_OPEN
        reach = bn.edges1[-1] if sphere else float(np.hypot(bn.edges1[-1], bn.edges2[-1])
                                                   if bn.edges2 is not None else bn.edges1[-1])
        a, b = (dxyz(du), dxyz(ru)) if sphere else (dxyz(d), dxyz(r))
        res = {}
        for label, cell in (("brute", 1e9), ("cells", 0.0)):
            ga = cute.build_grid(a, geom, r_max=reach, cell_size=cell)
            gb = cute.build_grid(b, geom, r_max=reach, cell_size=cell)
            for prec in ((cute.PREC_FP32_EDGE, cute.PREC_FP64) if label == "brute"
                         else (cute.PREC_FP32_EDGE,)):
                best, cnt, st = None, None, None
                for _ in range(reps):
                    cnt, st = cute.count_pairs(ga, gb, bn, prec, with_stats=True)
                    best = st["ms_count"] if best is None else min(best, st["ms_count"])
                res[(label, prec)] = (best, cnt, st)
            ga.close()
            gb.close()
        c_ref = res[("brute", cute.PREC_FP64)][1]
        exact = all(np.array_equal(v[1], c_ref) for v in res.values())
        tb, _, sb = res[("brute", cute.PREC_FP32_EDGE)]
        tc, _, sc = res[("cells", cute.PREC_FP32_EDGE)]
        out[name] = {"bins": bn.nbins, "dr_pairs": len(d) * len(r),
                     "brute_fp32_edge_s": round(tb / 1e3, 5),
                     "brute_fp64_s": round(res[("brute", cute.PREC_FP64)][0] / 1e3, 5),
                     "cell_list_fp32_edge_s": round(tc / 1e3, 5),
                     "brute_gpair_per_s": round(sb["pair_evals"] / (tb * 1e-3) / 1e9, 1),
                     "cell_list_pair_evals": int(sc["pair_evals"]),
                     "pairs_in_range": int(sb["pairs_in_range"]), "bit_exact": exact,
                     "paper_server_gpu_s": TABLE2_SERVER_GPU_S[name]}
    out["w_pix"] = wpix_leg(cute, torch, dev, du, ru, reps)
    out["radial"] = radial_leg(cute, torch, dev, du, ru, reps)
    return out


def radial_leg(cute, torch, dev, du, ru, reps):
    """The radial correlation on the same catalogs (not a Table 2 row):
    redshifts drawn uniform in [0.5, 0.6] (seeded), pairs within a 1 deg
    aperture, 100 bins of dz in [0, 0.1]; DD, DR and RR, FP64, inputs
    resident on the device."""
    rng = np.random.default_rng(6003)
    zd = torch.from_numpy(rng.uniform(0.5, 0.6, len(du))).to(dev)
    zr = torch.from_numpy(rng.uniform(0.5, 0.6, len(ru))).to(dev)
    ap, e = float(np.deg2rad(1.0)), np.linspace(0.0, 0.1, 101)
    a = [torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in (du.x, du.y, du.z)]
    b = [torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in (ru.x, ru.y, ru.z)]
    gd = cute.build_grid(a, cute.GEOM_SPHERE, r_max=ap)
    gr = cute.build_grid(b, cute.GEOM_SPHERE, r_max=ap)
    out = {"aperture_deg": 1.0, "bins": len(e) - 1}
    for name, (g1, z1, g2, z2) in (("dd", (gd, zd, None, None)), ("dr", (gd, zd, gr, zr)),
                                   ("rr", (gr, zr, None, None))):
        best = None
        for _ in range(reps):
            _, st = cute.count_radial(g1, z1, g2, z2, ap, e, with_stats=True)
            if best is None or st["ms_count"] < best["ms_count"]:
                best = st
        out[name] = {"ms": round(best["ms_count"], 3), "pair_evals": int(best["pair_evals"]),
                     "pairs_in_range": int(best["pairs_in_range"]),
                     "gpair_evals_per_s": round(best["pair_evals"] / (best["ms_count"] * 1e-3) / 1e9, 1)}
    return out


def wpix_leg(cute, torch, dev, du, ru, reps):
    """w_pix of Table 2: both catalogs binned into 5e-3 sq-deg pixel maps
    (inputs resident on the device), then the occupancy-weighted DR count of
    the pixel centres, 256 linear theta bins to 30 deg. The time is map
    building plus counting, FP32_EDGE; FP64 must give the same counts."""
    bn = cute.Binning(cute.BIN_THETA, np.deg2rad(np.linspace(0.0, 30.0, 257)))
    a = [torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in (du.x, du.y, du.z)]
    b = [torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in (ru.x, ru.y, ru.z)]
    best, res = None, {}
    for _ in range(reps):
        gd = cute.build_pixel_map(a, *TABLE2_PIX, r_max=bn.edges1[-1])
        gr = cute.build_pixel_map(b, *TABLE2_PIX, r_max=bn.edges1[-1])
        cnt, st = cute.count_pairs(gd, gr, bn, cute.PREC_FP32_EDGE, with_stats=True)
        ms = gd.info().ms_build + gr.info().ms_build + st["ms_count"]
        if best is None or ms < best:
            best = ms
            res = {"map_ms": round(gd.info().ms_build + gr.info().ms_build, 3),
                   "count_ms": round(st["ms_count"], 3), "pixels": [gd.n, gr.n],
                   "pixel_pair_evals": int(st["pair_evals"]), "counts": cnt}
    c64 = cute.count_pairs(gd, gr, bn, cute.PREC_FP64)
    exact = bool(np.array_equal(res.pop("counts"), c64))
    return dict(res, bins=bn.nbins, dr_object_pairs=len(du) * len(ru),
                pixel_sq_deg=round(4 * np.pi * np.rad2deg(1.0) ** 2 / (TABLE2_PIX[0] * TABLE2_PIX[1]), 5),
                total_s=round(best / 1e3, 5), bit_exact_vs_fp64=exact,
                paper_server_gpu_s=TABLE2_SERVER_GPU_S["w_pix"])


def committed_traffic():
    """HBM bytes per count launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source; None otherwise."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_count_rmu_clustered_1e6_dd.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        prof = json.load(f)
    if "kernel_sources_sha256" not in prof:
        return None
    for src, sha in prof["kernel_sources_sha256"].items():
        with open(os.path.join(ROOT, src), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != sha:
                return None
    return prof["fp32_edge"]["hbm_bytes_per_launch"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched mock/jackknife workload")
    ap.add_argument("--no-tune", action="store_true", help="skip the cell-size tuner leg")
    ap.add_argument("--no-xi", action="store_true",
                    help="skip the full xi(r, mu) time-to-solution leg (DD + DR + RR)")
    ap.add_argument("--no-table2", action="store_true",
                    help="skip the correlation functions of the paper's Table 2")
    ap.add_argument("--cell-size", type=float, default=0.0,
                    help="cell side of the grid (0 = the library's choice)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--no-modes", action="store_true",
                    help="skip the sigma-pi and theta DD legs")
    ap.add_argument("--only", choices=("sigmapi", "theta"), default=None,
                    help="run only that DD leg and print its result (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import catalogs
    import paper_1210_1833_amd as cute

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(0)
    if args.only:
        print(json.dumps({args.only: mode_leg(cute, torch, dev, args.only)}), flush=True)
        return
    d, _ = catalogs.clustered_box_1e6()
    n = len(d)
    xyz = [torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in (d.x, d.y, d.z)]
    bn = cute.Binning(cute.BIN_RMU, np.arange(41) * 5.0, np.arange(51) / 50.0, los=cute.LOS_Z)
    counts = torch.zeros(bn.nbins, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()

    def step(prec):
        g = cute.build_grid(xyz, cute.GEOM_BOX_OPEN, r_max=200.0, cell_size=args.cell_size)
        _, st = cute.count_pairs(g, None, bn, prec, out=counts, with_stats=True)
        g.close()
        return st

    def run(prec, steps, warmup):
        for _ in range(warmup):
            step(prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sts = [step(prec) for _ in range(steps)]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return dt, sts

    if args.copy_probe_mib:
        # a plain streaming kernel of known traffic (reads and writes copy_probe_mib
        # MiB each), for scaling the FETCH_SIZE / WRITE_SIZE counters
        src = torch.ones(args.copy_probe_mib * (1 << 20) // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        log("bench: copy probe of %d MiB done" % args.copy_probe_mib)
        del src, dst
    log("bench: r-mu DD, n=%d, FP32_EDGE %d steps" % (n, args.steps))
    dt32, st32 = run(cute.PREC_FP32_EDGE, args.steps, args.warmup)
    c32 = counts.cpu().numpy().astype(np.uint64)
    log("bench: FP64 %d steps" % args.fp64_steps)
    dt64, st64 = run(cute.PREC_FP64, args.fp64_steps, 1)
    c64 = counts.cpu().numpy().astype(np.uint64)

    # the grid build alone: host time of the call (it returns once the build
    # is enqueued), the wall time of builds in a row, and the GPU time of one
    # build from its events
    nb_ = 10
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    host_ms, gpu_ms = [], []
    for _ in range(nb_):
        t1 = time.perf_counter()
        g = cute.build_grid(xyz, cute.GEOM_BOX_OPEN, r_max=200.0, cell_size=args.cell_size)
        host_ms.append((time.perf_counter() - t1) * 1e3)
        gpu_ms.append(g.info().ms_build)
        g.close()
    torch.cuda.synchronize()
    build = {"calls": nb_, "ms_wall_per_build": round((time.perf_counter() - t0) / nb_ * 1e3, 4),
             "ms_host_call": round(float(np.median(host_ms)), 4),
             "ms_gpu_build": round(float(np.median(gpu_ms)), 4)}

    exact = bool(np.array_equal(c32, c64))
    golden = os.path.join(ROOT, "tests", "golden", "clustered_1e6_dd_rmu.json")
    oracle_checked = False
    if os.path.exists(golden):
        with open(golden) as f:
            g = json.load(f)
        if g["sha256"] == catalogs.sha256_of(d):
            exact = exact and bool(np.array_equal(c32, np.array(g["counts"], dtype=np.uint64)))
            oracle_checked = True

    evals = st32[-1]["pair_evals"]
    in_range = int(c32.sum())
    ms32 = dt32 / args.steps * 1e3
    ms64 = dt64 / args.fp64_steps * 1e3
    value = evals / (ms32 * 1e-3) / 1e9 if exact else 0.0
    kern_ms = float(np.mean([s["ms_count"] for s in st32]))
    kern64_ms = float(np.mean([s["ms_count"] for s in st64]))
    achieved = evals * I_ALG_RMU_Z / (kern_ms * 1e-3) / 1e12
    peak = PEAK_LANE_OPS / 1e12

    out = {
        "metric": "Gpair-evals/s (bit-exact counts), DD r-mu N=1e6; FP32+edge vs FP64 speedup",
        "value": round(value, 3),
        "unit": "Gpair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms32, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (+f64 edge re-test)",
        "data": "synthetic",
        "config": {
            "workload": "r-mu DD of 1e6 clustered points (1e4 Gaussian blobs x 100, sigma 5) in an "
                        "open 2000^3 box; r<200 in 40 bins x mu in [0,1] in 50 bins; LOS z; "
                        "cell list + FP32 separations with FP64 edge re-test",
            "n_points": n,
            "step": "cute_build_grid + cute_count_pairs (auto), inputs resident in HBM",
            "precision": "FP32_EDGE",
            "cell_size": args.cell_size or "auto",
        },
        "bit_exact": exact,
        "checked_against": "oracle golden counts" if oracle_checked else "GPU FP64 path",
        "pair_evals_per_step": int(evals),
        "tiles_per_step": int(st32[-1]["tiles"]),
        "pairs_in_range_per_step": in_range,
        "retests_per_step": int(st32[-1]["retests"]),
        "flips_per_step": int(st32[-1]["flips"]),
        "pairs_in_range_per_s": in_range / (ms32 * 1e-3),
        "brute_force_equiv_pairs_per_s": n * (n - 1) / 2 / (ms32 * 1e-3),
        "step_overhead_ms": round(ms32 - kern_ms, 4),
        "grid_build": build,
        "fp64": {"ms_per_step": round(ms64, 4), "kernel_ms": round(kern64_ms, 4),
                 "gpair_evals_per_s": round(st64[-1]["pair_evals"] / (ms64 * 1e-3) / 1e9, 3)},
        "speedup_fp32edge_vs_fp64": round(ms64 / ms32, 3),
        "kernel_speedup_fp32edge_vs_fp64": round(kern64_ms / kern_ms, 3),
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3),
                     "unit": "Tlane-op/s", "frac": round(achieved / peak, 4),
                     "traffic": committed_traffic(),
                     "traffic_source": "rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE of this kernel "
                                       "source (profiles/k_count_rmu_clustered_1e6_dd.json), "
                                       "not measured in this run; null when the source changed",
                     "kernel_ms": round(kern_ms, 4), "i_alg": I_ALG_RMU_Z,
                     "flop_convention_frac": round(evals * I_ALG_RMU_Z / (kern_ms * 1e-3)
                                                   / PEAK_FP32_FLOPS, 4),
                     "flop_convention_peak_tflops": PEAK_FP32_FLOPS / 1e12},
        "fp32_only": fp32_only_leg(cute, xyz, bn, counts, c64, st32[-1]),
    }
    if not args.no_xi:
        log("bench: full xi(r, mu): DD, DR, RR, Landy-Szalay, multipoles")
        out["xi_rmu_full"] = xi_leg(cute, torch, dev, xyz, bn, c32)
    # the cell-size tuner on the same data: its choice and the count time with it
    if not args.no_tune:
        out["tuned_cell"] = tuned_leg(cute, xyz, bn, counts, c32)
    if not args.no_modes:
        out["sigmapi_dd"] = mode_leg(cute, torch, dev, "sigmapi")
        out["theta_dd"] = mode_leg(cute, torch, dev, "theta")
    if not args.no_batched:
        out["batched"] = batched_leg(cute, torch, dev)
    if not args.no_table2:
        log("bench: the paper's Table 2 functions")
        out["paper_table2"] = table2_leg(cute, torch, dev)
    if not args.no_cpu_baseline:
        log("bench: cpu baseline")
        out["cpu_baseline"] = cpu_baseline(d)
    print(json.dumps(out), flush=True)


I_ALG_SIGMAPI = 40                    # algorithmic FP32 lane-ops per sigma-pi (midpoint) pair evaluation
I_ALG_THETA = 16                      # algorithmic FP32 lane-ops per theta pair evaluation


def mode_leg(cute, torch, dev, kind, reps=2):
    """The DD count of one more workload at full size, FP32_EDGE, FP64 and
    FP32_ONLY kernels: 'sigmapi', the light cone (3e6 points, sigma and pi in
    [0, 150) with 75 x 75 bins, midpoint line of sight), or 'theta', the
    angular cap (1e7 clustered unit vectors, 30 log bins of theta in
    [0.001, 10] deg). FP32_EDGE must equal FP64 (and the oracle's golden
    counts where they exist); the VALU fraction is taken at the mode's
    algorithmic lane-ops per pair."""
    import catalogs
    t0 = time.perf_counter()
    if kind == "sigmapi":
        cat, _ = catalogs.lightcone_3e6()
        e = np.arange(76) * 2.0
        bn = cute.Binning(cute.BIN_SIGMAPI, e, e, los=cute.LOS_MIDPOINT)
        geom, reach, i_alg = cute.GEOM_BOX_OPEN, float(np.hypot(e[-1], e[-1])) * (1 + 1e-12), I_ALG_SIGMAPI
        golden, workload = "lightcone_3e6_dd_sigmapi.json", (
            "sigma-pi DD of the light cone: 3e6 points, RA 0-60 deg, Dec 0-30 deg, Gaussian n(z), "
            "sigma and pi in [0, 150) Mpc/h, 75 x 75 bins, midpoint line of sight")
    else:
        cat, _ = catalogs.angular_cap_1e7()
        e = np.deg2rad(0.001 * 10.0 ** (np.arange(31) * 4.0 / 30.0))
        bn = cute.Binning(cute.BIN_THETA, e)
        geom, reach, i_alg = cute.GEOM_SPHERE, float(e[-1]), I_ALG_THETA
        golden, workload = None, ("theta DD of the angular cap: 1e7 clustered unit vectors in "
                                  "5000 sq-deg, 30 log bins of theta in [0.001, 10] deg")
    xyz = [torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in (cat.x, cat.y, cat.z)]
    g = cute.build_grid(xyz, geom, r_max=reach)
    t_gen = time.perf_counter() - t0
    res = {}
    for name, prec in (("fp32_edge", cute.PREC_FP32_EDGE), ("fp64", cute.PREC_FP64),
                       ("fp32_only", cute.PREC_FP32_ONLY)):
        best = None
        for _ in range(reps if name != "fp64" else 1):
            c, st = cute.count_pairs(g, None, bn, prec, with_stats=True)
            if best is None or st["ms_count"] < best[1]["ms_count"]:
                best = (c, st)
        res[name] = best
        log("bench: %s DD %s %.1f ms" % (kind, name, best[1]["ms_count"]))
    g.close()
    c32, st = res["fp32_edge"]
    exact = bool(np.array_equal(c32, res["fp64"][0]))
    checked = "GPU FP64 path"
    if golden is not None and os.path.exists(os.path.join(ROOT, "tests", "golden", golden)):
        with open(os.path.join(ROOT, "tests", "golden", golden)) as f:
            gr = json.load(f)
        if gr["sha256_data"] == catalogs.sha256_of(cat):
            exact = exact and bool(np.array_equal(c32.reshape(-1), np.array(gr["counts"], dtype=np.uint64)))
            checked = "oracle golden counts"
    ms = st["ms_count"]
    pir = int(st["pairs_in_range"])
    l1 = int(np.abs(res["fp32_only"][0].astype(np.int64) - c32.astype(np.int64)).sum())
    return {"workload": workload, "bit_exact": exact, "checked_against": checked,
            "kernel_ms": {k: round(v[1]["ms_count"], 3) for k, v in res.items()},
            "pair_evals": int(st["pair_evals"]), "pairs_in_range": pir,
            "retests": int(st["retests"]), "retests_per_pair_in_range": st["retests"] / max(pir, 1),
            "fp32_only_hist_l1": l1, "flips": int(st["flips"]),
            "gpair_evals_per_s": round(st["pair_evals"] / (ms * 1e-3) / 1e9, 1),
            "speedup_fp32edge_vs_fp64": round(res["fp64"][1]["ms_count"] / ms, 3),
            "lane_op_frac_at_i_alg": round(st["pair_evals"] * i_alg / (ms * 1e-3) / PEAK_LANE_OPS, 4),
            "i_alg": i_alg,
            "lane_op_note": "i_alg lane-ops counted for every candidate pair, also those of steps "
                            "dropped after the top-edge vote (a few operations each), so the "
                            "fraction can pass 1; the VALU instructions actually issued per pair "
                            "and the issue share are in the rocprofv3 counter summaries",
            "host_s": round(t_gen, 1)}


def fp32_only_leg(cute, xyz, bn, counts, c_exact, st_edge, reps=3):
    """The FP32 fast path alone (no FP64 re-test) on the benchmark workload:
    its kernel time and how far its counts are from the exact ones (the L1
    distance of the histograms), beside the flips of the exact path (re-tested
    pairs whose FP32-only decision was wrong)."""
    g = cute.build_grid(xyz, cute.GEOM_BOX_OPEN, r_max=200.0)
    best = None
    for _ in range(reps):
        _, st = cute.count_pairs(g, None, bn, cute.PREC_FP32_ONLY, out=counts, with_stats=True)
        best = st["ms_count"] if best is None else min(best, st["ms_count"])
    c = counts.cpu().numpy().astype(np.int64)
    g.close()
    l1 = int(np.abs(c - c_exact.astype(np.int64)).sum())
    pir = int(c_exact.sum())
    return {"kernel_ms": round(best, 4), "hist_l1_vs_exact": l1,
            "hist_l1_per_pair_in_range": l1 / max(pir, 1),
            "flips": int(st_edge["flips"]), "flips_per_pair_in_range": int(st_edge["flips"]) / max(pir, 1),
            "note": "flips: re-tested pairs whose FP32-only decision differed from FP64 (FP32_EDGE "
                    "run); hist_l1: sum over bins of |FP32_ONLY count - exact count|"}


def xi_leg(cute, torch, dev, xyz, bn, c_dd, reps=3):
    """Time to solution of the whole r-mu correlation function of the
    benchmark workload: grids of the 1e6 data and 2e6 randoms, DD, DR and RR
    (FP32_EDGE, counts in device memory), then the Landy-Szalay estimator
    and the multipoles l = 0, 2, 4 on the host. Inputs resident in HBM."""
    import catalogs
    _, r = catalogs.clustered_box_1e6()
    rxyz = [torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in (r.x, r.y, r.z)]
    outs = [torch.zeros(bn.nbins, dtype=torch.int64, device=dev) for _ in range(3)]
    best, parts = None, None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gd = cute.build_grid(xyz, cute.GEOM_BOX_OPEN, r_max=200.0)
        gr = cute.build_grid(rxyz, cute.GEOM_BOX_OPEN, r_max=200.0)
        sts = [cute.count_pairs(a, b, bn, cute.PREC_FP32_EDGE, out=o, with_stats=True)[1]
               for (a, b), o in zip(((gd, None), (gd, gr), (gr, None)), outs)]
        dd, dr, rr = (o.cpu().numpy().astype(np.uint64).reshape(bn.shape) for o in outs)
        xi = cute.xi_estimate(cute.EST_LS, dd, dr, rr, len(xyz[0]), len(rxyz[0]), bn)
        mp = cute.xi_multipoles(np.nan_to_num(xi), bn, (0, 2, 4))
        dt = (time.perf_counter() - t0) * 1e3
        gd.close()
        gr.close()
        if best is None or dt < best:
            best, parts = dt, sts
    assert np.all(np.isfinite(mp))
    evals = sum(int(s["pair_evals"]) for s in parts)
    return {"ms": round(best, 3), "kernel_ms": {k: round(s["ms_count"], 3) for k, s in
                                                zip(("dd", "dr", "rr"), parts)},
            "pair_evals": evals, "gpair_evals_per_s": round(evals / (best * 1e-3) / 1e9, 1),
            "dd_equals_headline": bool(np.array_equal(dd.reshape(-1), c_dd)),
            "n_data": len(xyz[0]), "n_randoms": len(rxyz[0])}


def tuned_leg(cute, xyz, bn, counts, c32):
    """cute_tune_grid on the benchmark data, then the count with its choice."""
    cell, tile, cand = cute.tune_grid(xyz, cute.GEOM_BOX_OPEN, bn, r_max=200.0)
    gt = cute.build_grid(xyz, cute.GEOM_BOX_OPEN, r_max=200.0, cell_size=cell, tile_points=tile)
    tt = []
    for _ in range(5):
        _, stt = cute.count_pairs(gt, None, bn, cute.PREC_FP32_EDGE, out=counts, with_stats=True)
        tt.append(stt["ms_count"])
    gt.close()
    tuned_ok = bool(np.array_equal(counts.cpu().numpy().astype(np.uint64), c32))
    return {"cell_size": cell if cell > 0 else "auto", "tile_points": tile,
            "kernel_ms": round(min(tt), 4), "pair_evals": int(stt["pair_evals"]),
            "bit_exact": tuned_ok,
            "candidates_ms": {"%s/%d" % ("auto" if c == 0 else round(c, 3), t): round(v, 4)
                              for (c, t), v in cand.items()}}


if __name__ == "__main__":
    main()
