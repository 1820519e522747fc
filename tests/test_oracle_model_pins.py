"""Pins of the oracle's chunk-count model (Section 3.5, Eqs. 2-7), reorder
(Section 3.2, Algorithm 3) and ideal volume (Section 4.3) to numbers the
paper prints and to library routines.

CPU constants: a 64-byte cache line and four-byte histogram and prefix types
give s_chunkFine = 4 + 4 + 2*64 = 136 bytes (Section 3.5); the value type of
the microbenchmarks is four bytes (Section 4.1), so s_denseAccum = 5 in the
numeric phase and 1 in the symbolic phase."""
import numpy as np

import oracle
from oracle import chunk_model as cm

MiB = 1 << 20


def test_s_chunk_fine_cpu():
    assert cm.s_chunk_fine(64) == 136


def test_reorder_breaking_point_2e13():
    # Section 4.1.2: reordering slows past 2^13 chunks on SPR (2 MB L2), where
    # the per-chunk reorder storage no longer fits
    assert cm.pow2_floor(2 * MiB / 136) == 1 << 13


def test_dense_fits_l2_at_stream_length_2e18():
    # Section 4.1.1: at stream length 2^18 the dense accumulation arrays fit
    # the 2 MB L2 (4-byte value + 1-byte bitmap entry per column), 2^19 not
    assert (1 << 18) * 5 < 2 * MiB < (1 << 19) * 5


def test_coarse_crossover_skx_spr():
    # Section 4.3: coarse level starts at m_C = 2^30 on SKX (1 MB L2) and 2^32
    # on SPR/EMR (2 MB L2).  Eq. 5 reproduces both with s_denseAccum = 1 (the
    # symbolic-phase value) and flooring.
    assert cm.paper_mcmax(1 * MiB, 1, 136) == 1 << 30
    assert cm.paper_mcmax(2 * MiB, 1, 136) == 1 << 32
    # the numeric-phase value (5) would give 2^28 and 2^30 instead
    assert cm.paper_mcmax(1 * MiB, 5, 136) == 1 << 28
    assert cm.paper_mcmax(2 * MiB, 5, 136) == 1 << 30


def test_fine_level_breaking_point_2e31_reading():
    # Section 4.1.2 places the fine-level breaking point at stream length 2^31
    # on SPR.  Eq. 5 with s_denseAccum = 5 gives 1.62e9, which is 2^31 only
    # when rounded to the nearest power of two (the floored reading gives
    # 2^30): an inconsistency in the paper, recorded here.
    x = (2 * MiB) ** 2 / (4 * 5 * 136)
    assert 1.6e9 < x < 1.65e9
    assert cm.pow2_nearest(x) == 1 << 31
    assert cm.pow2_floor(x) == 1 << 30


def test_optimal_fine_chunks_at_2e29():
    # Section 4.1.2 (Fig. 5's middle line): Eq. 3 with the stream length 2^29
    # in place of m_C: sqrt(2^29 * 5 / 136) = 4443 -> 2^12
    assert cm.paper_fine_nchunks(1 << 29, 5, 136) == 1 << 12


def test_eq2_minimiser_and_eq4():
    # Eq. 3 minimises the convex Eq. 2 over powers of two (up to the rounding
    # reading) and Eq. 4 is its value at the unrounded optimum
    for mc in (1 << 10, 1 << 18, 1 << 24, 1 << 29):
        for sd, sc in ((5, 136), (1, 136), (9, 264)):
            best = min((cm.fine_storage(mc, 1 << k, sd, sc), 1 << k) for k in range(0, 30))
            n = cm.paper_fine_nchunks(mc, sd, sc)
            assert cm.fine_storage(mc, n, sd, sc) <= 1.07 * best[0]
            nstar = np.sqrt(mc * sd / sc)
            assert np.isclose(cm.fine_storage(mc, nstar, sd, sc), cm.fine_storage_opt(mc, sd, sc))


def test_two_level_split():
    # Eq. 7: once coarse is on, fine chunk count stops growing and coarse grows
    a = cm.paper_model(1 << 33, 2 * MiB, 64, 4, phase="symbolic")
    b = cm.paper_model(1 << 35, 2 * MiB, 64, 4, phase="symbolic")
    assert a["use_coarse"] and b["use_coarse"]
    assert a["n_chunks_fine"] == b["n_chunks_fine"]
    assert b["n_chunks_coarse"] == 4 * a["n_chunks_coarse"]
    assert a["chunk_len_coarse"] == a["m_cmax"] == 1 << 32
    c = cm.paper_model(1 << 20, 2 * MiB, 64, 4)
    assert not c["use_coarse"] and c["n_chunks_coarse"] == 1
    assert c["chunk_len_fine"] * c["n_chunks_fine"] == 1 << 20


def test_reorder_is_stable_counting_sort():
    # sequential reorder = a stable sort by chunk id (numpy's stable argsort)
    rng = np.random.default_rng(5)
    cols = rng.integers(1000, 1000 + (1 << 12), size=3000)
    vals = rng.standard_normal(3000)
    off, cf, vf = oracle.reorder_row(cols, vals, 8, 1000, 16)
    ch = (cols - 1000) >> 8
    order = np.argsort(ch, kind="stable")
    assert np.array_equal(vf, vals[order])
    assert np.array_equal(cf, (cols - 1000)[order] - (ch[order] << 8))
    assert np.array_equal(off, np.concatenate([[0], np.cumsum(np.bincount(ch, minlength=16))]))
    assert (cf >= 0).all() and (cf < 256).all()


def test_ideal_volume_config3_magnitude():
    # the size quoted for C = A*B on 2^24 x 2^24 ER, 16 per row, f32, int64
    # row pointers, int32 columns: about 98 GB (the ideal read+write volume)
    n, nnz_a, ip = 1 << 24, 1 << 28, 1 << 32
    nnz_c = ip - 30720
    r, w = oracle.ideal_volume(n, nnz_a, ip, n, nnz_c, s_rp_a=8, s_rp_b=8, s_col_a=4, s_col_b=4,
                               s_val=4, s_rp_c=8, s_col_c=4)
    assert 97e9 < r + w < 99e9


def test_golden_numbers_match_model():
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))
    assert cm.pow2_floor(2 * MiB / 136) == g["reorder_breaking_point_chunks"]["value"]
    L = g["dense_fits_l2_stream_length"]["value"]
    assert L * 5 < 2 * MiB < 2 * L * 5
    assert cm.pow2_nearest((2 * MiB) ** 2 / (4 * 5 * 136)) == \
        g["fine_level_breaking_point_stream_length"]["value"]
    # derived (not printed): Eq. 3 at stream length 2^29, see the golden file
    assert cm.paper_fine_nchunks(1 << 29, 5, 136) == g["_derived"]["optimal_fine_chunks_at_2e29"]["value"]
    cx = g["coarse_crossover_mC"]
    assert cm.paper_mcmax(1 * MiB, 1, 136) == cx["SKX"]
    assert cm.paper_mcmax(2 * MiB, 1, 136) == cx["SPR"] == cx["EMR"]
    for row in g["rmat16_table3"]["rows"]:
        assert row["n"] == 1 << row["scale"] and row["nnz_A"] == 16 * row["n"]
