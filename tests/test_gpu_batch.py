"""GPU parity of the batched counts (cute_batch_* / cute_count_pairs_batched).

Every item of a batch must equal the oracle's count of the same catalog pair
with the masked points removed (bit-exact for FP64 and FP32_EDGE), and the
single-count path on the same grids (bit-exact for all three precisions: the
FP32-only decision does not depend on the rounding bands, which a batch
widens to the largest error bound of its items). Inputs follow the batched
mock workload: periodic boxes of side 1000 with half uniform, half clustered
points, log-uniform sizes, and jackknife catalogs that leave out one (x, y)
column of a 10 x 10 grid of regions."""
import sys

import numpy as np
import pytest

import catalogs
import oracle
import paper_1210_1833_amd as cute

pytestmark = pytest.mark.gpu

L = 1000.0
MONO_E = np.arange(31) * 5.0
RMU_E1, RMU_E2 = np.arange(41) * 5.0, np.arange(51) / 50.0
EXACT = [cute.PREC_FP64, cute.PREC_FP32_EDGE]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    cute.load()
    yield


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def bins():
    return (cute.Binning(cute.BIN_MONO, MONO_E),
            cute.Binning(cute.BIN_RMU, RMU_E1, RMU_E2, los=cute.LOS_Z))


def obins():
    return (oracle.Binning(oracle.MONO, MONO_E, periodic=True, L=L),
            oracle.Binning(oracle.RMU, RMU_E1, RMU_E2, los=oracle.LOS_Z, periodic=True, L=L))


def grid(cat):
    return cute.build_grid(cat, cute.GEOM_BOX_PERIODIC, box_size=L, r_max=200.0)


@pytest.fixture(scope="module")
def small():
    """6 mocks (500 .. 4000 points), a 6000-point jackknife base, its regions."""
    mocks, base, region = catalogs.batched_mocks_256(n_mocks=6, n_lo=500, n_hi=4000, jk_base=6000, box=L)
    return mocks, base, region


def small_items(mocks, base, region, gm, gb, gb2, regions):
    """(item, oracle catalogs (a, b or None)) for mocks, jackknife catalogs
    and masked cross counts, on both binnings."""
    mono, rmu = bins()
    out = []
    for k, m in enumerate(mocks):
        for bn in (mono, rmu):
            out.append((cute.BatchItem(gm[k], None, bn), (m, None)))
    # DR between two mocks
    out.append((cute.BatchItem(gm[0], gm[1], mono), (mocks[0], mocks[1])))
    for r in regions:
        inside = (region == r).astype(np.uint8)
        rest = base.subset(np.nonzero(region != r)[0])
        reg = base.subset(np.nonzero(region == r)[0])
        for bn in (mono, rmu):
            # jackknife catalog: every point outside region r
            out.append((cute.BatchItem(gb, None, bn, mask_a=inside), (rest, None)))
        # cross count of the rest with the region (two handles of the same catalog)
        out.append((cute.BatchItem(gb, gb2, rmu, mask_a=inside, mask_b=1 - inside), (rest, reg)))
    return out


def oracle_count(cats, bn):
    ob = obins()[0 if bn.edges2 is None else 1]
    a, b = cats
    return oracle.count_pairs(a, b, ob).reshape(-1)


def test_batch_matches_oracle(small):
    mocks, base, region = small
    gm = [grid(m) for m in mocks]
    gb, gb2 = grid(base), grid(base)
    items = small_items(mocks, base, region, gm, gb, gb2, regions=[0, 37, 99])
    expect = [oracle_count(c, it.binning) for it, c in items]
    for prec in EXACT:
        say("batch vs oracle: %d items, prec %d" % (len(items), prec))
        got, st = cute.count_pairs_batched([it for it, _ in items], prec, with_stats=True)
        for k, ((it, _), g, e) in enumerate(zip(items, got, expect)):
            assert np.array_equal(g.reshape(-1), e), "item %d prec %d" % (k, prec)
        assert st["pairs_in_range"] == sum(int(e.sum()) for e in expect)
        assert st["pair_evals"] >= st["pairs_in_range"]


def test_batch_matches_single_all_precisions(small):
    mocks, base, region = small
    gm = [grid(m) for m in mocks]
    gb, gb2 = grid(base), grid(base)
    items = small_items(mocks, base, region, gm, gb, gb2, regions=[5])
    for prec in (cute.PREC_FP64, cute.PREC_FP32_EDGE, cute.PREC_FP32_ONLY):
        say("batch vs single: prec %d" % prec)
        got = cute.count_pairs_batched([it for it, _ in items], prec)
        for k, (it, _) in enumerate(items):
            if it.mask_a is not None:
                continue  # the single path has no masks; the oracle test covers them
            single = cute.count_pairs(it.a, it.b, it.binning, prec)
            assert np.array_equal(got[k], single), "item %d prec %d" % (k, prec)


def test_graph_replays_match_eager(small):
    """The captured graph, replayed several times with other device work and
    synchronisations in between, gives the eager run's counts every time."""
    import torch
    mocks, base, region = small
    gm = [grid(m) for m in mocks]
    gb, gb2 = grid(base), grid(base)
    items = [it for it, _ in small_items(mocks, base, region, gm, gb, gb2, regions=[12, 13])]
    b = cute.Batch(items, cute.PREC_FP32_EDGE)
    b.run(eager=True)
    ref = b.counts()
    ref_stats = b.stats()
    assert ref.sum() > 0
    mono, _ = bins()
    for rep in range(4):
        say("graph replay %d" % rep)
        b.run()
        got = b.counts()
        assert np.array_equal(got, ref), "replay %d" % rep
        assert b.stats()["tiles"] == ref_stats["tiles"]
        # unrelated eager work between replays
        cute.count_pairs(gm[0], None, mono, cute.PREC_FP32_EDGE)
        torch.cuda.synchronize()
    # per-item views of the concatenation
    for k in range(len(items)):
        w, o = b.layout(k)
        assert np.array_equal(b.counts(k).reshape(-1), ref[o:o + w])
    # device-side copy
    out = torch.zeros(b.layout()[0], dtype=torch.int64, device="cuda")
    b.counts(out=out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().astype(np.uint64), ref)
    b.close()


def test_empty_items_and_full_mask(small):
    mocks, base, region = small
    mono, rmu = bins()
    e = catalogs.Catalog.from_xyz(np.zeros((0, 3)))
    ge, g0 = grid(e), grid(mocks[0])
    all_masked = np.ones(len(mocks[0]), dtype=np.uint8)
    items = [cute.BatchItem(ge, None, mono), cute.BatchItem(g0, ge, rmu),
             cute.BatchItem(g0, None, mono, mask_a=all_masked),
             cute.BatchItem(g0, None, mono)]
    got = cute.count_pairs_batched(items, cute.PREC_FP32_EDGE)
    assert got[0].sum() == 0 and got[1].sum() == 0 and got[2].sum() == 0
    assert np.array_equal(got[3].reshape(-1), oracle_count((mocks[0], None), mono))


def test_batch_rejects_bad_items(small):
    mocks, _, _ = small
    g0 = grid(mocks[0])
    mono, _ = bins()
    with pytest.raises(cute.CuteError) as ei:
        cute.count_pairs_batched([cute.BatchItem(g0, None, mono),
                                  cute.BatchItem(g0, None, cute.Binning(cute.BIN_MONO, [0.0, 600.0]))])
    assert ei.value.status == cute.E_INVALID_ARG
    assert "item 1" in str(ei.value)
    with pytest.raises(ValueError):
        cute.count_pairs_batched([cute.BatchItem(g0, None, mono, mask_a=np.zeros(3, np.uint8))])


def test_c5_shaped_batch_matches_single_and_jackknife_identity():
    """Batched-mock shapes at reduced count: 24 mocks of 2e4 .. 1e5 points and
    a 3e5-point jackknife base, both binnings, FP32_EDGE. Every mock equals
    its single count; the smallest mock equals the oracle; each jackknife
    catalog satisfies DD(base) = DD(rest) + DD(region) + DR(rest, region)."""
    import torch
    mocks, base, region = catalogs.batched_mocks_256(n_mocks=24, n_lo=2e4, n_hi=1e5, jk_base=300_000, box=L)
    mono, rmu = bins()
    gm = [grid(m) for m in mocks]
    gb, gb2 = grid(base), grid(base)
    items = []
    for g in gm:
        items += [cute.BatchItem(g, None, mono), cute.BatchItem(g, None, rmu)]
    regs = [0, 44, 99]
    masks = {r: torch.from_numpy((region == r).astype(np.uint8)).cuda() for r in regs}
    for r in regs:
        items += [cute.BatchItem(gb, None, rmu, mask_a=masks[r]),                    # rest
                  cute.BatchItem(gb, None, rmu, mask_a=1 - masks[r]),                # region
                  cute.BatchItem(gb, gb2, rmu, mask_a=masks[r], mask_b=1 - masks[r])]  # cross
    say("C5-shaped batch: %d items" % len(items))
    got, st = cute.count_pairs_batched(items, cute.PREC_FP32_EDGE, with_stats=True)
    say("C5-shaped batch: %.1f ms, %d pair evals" % (st["ms_count"], st["pair_evals"]))
    for k, g in enumerate(gm):
        for j, bn in enumerate((mono, rmu)):
            single = cute.count_pairs(g, None, bn, cute.PREC_FP32_EDGE)
            assert np.array_equal(got[2 * k + j], single), "mock %d binning %d" % (k, j)
    small_k = int(np.argmin([len(m) for m in mocks]))
    assert np.array_equal(got[2 * small_k].reshape(-1),
                          oracle.count_pairs(mocks[small_k], None, obins()[0], prune=True))
    dd_base = cute.count_pairs(gb, None, rmu, cute.PREC_FP32_EDGE)
    for q, r in enumerate(regs):
        rest, reg, cross = got[2 * len(gm) + 3 * q: 2 * len(gm) + 3 * q + 3]
        assert np.array_equal(rest + reg + cross, dd_base), "region %d" % r
        assert cross.sum() > 0 and reg.sum() > 0


def test_batch_lattice_ties_match_oracle():
    """Dyadic lattices in a periodic box of side 12: many pairs lie exactly on
    the r and mu edges and go through the FP64 re-test, whose queue a wave
    empties whenever it moves to another item; every item must equal the
    oracle for FP64 and FP32_EDGE."""
    Ll = 12.0
    e1, e2 = np.arange(0, 9) * 0.5, np.array([0.0, 0.25, 0.5, 0.75, 1.0])
    mono = cute.Binning(cute.BIN_MONO, e1)
    rmu = cute.Binning(cute.BIN_RMU, e1, e2, los=cute.LOS_Z)
    omono = oracle.Binning(oracle.MONO, e1, periodic=True, L=Ll)
    ormu = oracle.Binning(oracle.RMU, e1, e2, los=oracle.LOS_Z, periodic=True, L=Ll)
    g = np.random.Generator(np.random.PCG64(23))
    cats = [g.integers(0, 24, size=(n, 3)).astype(np.float64) * 0.5 for n in (700, 1500, 2600)]
    grids = [cute.build_grid(c, cute.GEOM_BOX_PERIODIC, box_size=Ll, r_max=4.0) for c in cats]
    mask = (g.random(len(cats[2])) < 0.3).astype(np.uint8)
    items, expect = [], []
    for c, gr in zip(cats, grids):
        for bn, ob in ((mono, omono), (rmu, ormu)):
            items.append(cute.BatchItem(gr, None, bn))
            expect.append(oracle.count_pairs(c, None, ob).reshape(-1))
    items.append(cute.BatchItem(grids[2], None, rmu, mask_a=mask))
    expect.append(oracle.count_pairs(cats[2][mask == 0], None, ormu).reshape(-1))
    items.append(cute.BatchItem(grids[0], grids[1], rmu))
    expect.append(oracle.count_pairs(cats[0], cats[1], ormu).reshape(-1))
    for prec in EXACT:
        say("batch lattice: %d items, prec %d" % (len(items), prec))
        got, st = cute.count_pairs_batched(items, prec, with_stats=True)
        for k, (gk, ek) in enumerate(zip(got, expect)):
            assert np.array_equal(gk.reshape(-1), ek), "item %d prec %d" % (k, prec)
        if prec == cute.PREC_FP32_EDGE:
            assert st["retests"] > 0
