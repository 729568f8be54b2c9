"""Host checks of the banded SpMM work schedule (no GPU needed).

The schedule must cover every entry exactly once, keep each piece inside one
band of the gathered index, give split rows consecutive partial slots, and
place band r on XCD r % 8 in increasing band order.
"""

import numpy as np
import pytest

import synth

WAVES, XCDS = 4, 8


def split_len(cap):
    # shortest row the banded form splits at the band boundaries
    return max(256, 4 * cap)


@pytest.fixture(scope="module")
def K():
    from paper_1810_06860_amd import kernels
    return kernels


def _structure(rows, gathered, cap, seed):
    rng = np.random.default_rng(seed)
    lens = np.where(rng.random(rows) < 0.25, rng.integers(0, 12 * cap, rows),
                    rng.integers(0, 300, rows))
    lens[rng.random(rows) < 0.1] = 0
    edge = [split_len(cap) - 1, split_len(cap), split_len(cap) + 1]   # around the threshold
    lens[:3] = edge[:min(rows, 3)]
    lens = np.minimum(lens, gathered)
    idx = [np.sort(rng.choice(gathered, size=int(k), replace=False)) for k in lens]
    ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    return ptr, (np.concatenate(idx) if idx else np.zeros(0)).astype(np.int32)


def _check(ptr, idx, gathered, cap, bands, segs, fix, nslot):
    rows = ptr.size - 1
    assert segs.shape[0] % (WAVES * XCDS) == 0
    cover = np.zeros(idx.size, np.int64)
    direct = np.zeros(rows, np.int64)
    pieces = np.zeros(rows, np.int64)
    slot_owner = np.full(nslot, -1)
    last_band = np.full(XCDS, -1)
    bound = np.array([r * gathered // bands for r in range(bands + 1)])
    for s, (row, b, e, slot) in enumerate(segs):
        if row < 0:
            continue
        xcd = (s // WAVES) % XCDS
        assert ptr[row] <= b <= e <= ptr[row + 1] and e - b <= cap
        cover[b:e] += 1
        pieces[row] += 1
        if slot < 0:
            direct[row] += 1
        else:
            assert slot_owner[slot] == -1
            slot_owner[slot] = row
        if ptr[row + 1] - ptr[row] >= split_len(cap) and e > b:
            band = np.searchsorted(bound, idx[b], side="right") - 1
            # the whole piece lies in one band, and that band is this XCD's
            assert bound[band] <= idx[b] and idx[e - 1] < bound[band + 1]
            assert band % XCDS == xcd
            assert band >= last_band[xcd]            # bands in increasing order
            last_band[xcd] = band
    assert np.all(cover == 1)
    assert np.all(slot_owner >= 0)
    fixed = np.zeros(rows, np.int64)
    for row, first, count, _ in fix:
        fixed[row] += 1
        assert np.all(slot_owner[first:first + count] == row)
        assert pieces[row] == count and direct[row] == 0
    assert np.all(direct + fixed == 1)
    assert np.all(pieces[direct == 1] == 1)
    # a split row has at most len / cap + bands <= (1 + bands / 4) len / cap
    # pieces (it is split only from 4 cap entries on): with the 8 bands of
    # the library, the 3 len / cap the footprint reserves partial rows for
    assert nslot <= (1 + bands // 4) * -(-idx.size // cap)


@pytest.mark.parametrize("rows,gathered,cap,bands,seed", [
    (2, 20000, 64, 8, 1), (37, 16384, 64, 8, 2), (500, 50021, 611, 8, 3),
    (300, 9000, 128, 16, 4), (800, 70001, 1024, 32, 5)])
def test_band_schedule_invariants(K, rows, gathered, cap, bands, seed):
    ptr, idx = _structure(rows, gathered, cap, seed)
    segs, fix, nslot = K.band_schedule(ptr, idx, gathered, cap, bands)
    _check(ptr, idx, gathered, cap, bands, segs, fix, nslot)


def test_band_schedule_power_law_balance(K):
    # columns of a Zipf rating matrix (the transposed product's structure):
    # the eight XCDs get nearly the same number of workgroups' worth of work
    m, n = 20000, 600
    p = synth.ratings(m, n, 200_000, 3, seed_data=9)
    order = np.lexsort((p.rows, p.cols))
    idx = p.rows[order].astype(np.int32)
    ptr = np.concatenate([[0], np.cumsum(np.bincount(p.cols, minlength=n))]).astype(np.int32)
    segs, fix, nslot = K.band_schedule(ptr, idx, m, 64, 8)
    _check(ptr, idx, m, 64, 8, segs, fix, nslot)
    live = segs[:, 0] >= 0
    per_xcd = np.bincount((np.flatnonzero(live) // WAVES) % XCDS, minlength=XCDS)
    assert per_xcd.max() - per_xcd.min() <= 0.1 * per_xcd.mean()
    assert (~live).sum() < 0.1 * live.sum()


def test_band_schedule_rejects_bad_input(K):
    from paper_1810_06860_amd import MCError
    ptr = np.array([0, 2, 3], np.int32)
    for idx, gathered, bands in ((np.array([5, 3, 1], np.int32), 10, 8),   # not increasing
                                 (np.array([1, 10, 1], np.int32), 10, 8),  # out of range
                                 (np.array([1, 3, 1], np.int32), 10, 12)):  # bands % 8
        with pytest.raises(MCError):
            K.band_schedule(ptr, idx, gathered, 64, bands)
    # a NULL idx with non-empty rows is an error, not a crash
    import ctypes as C
    from paper_1810_06860_amd import lib
    nseg, nfix, nslot = C.c_int64(0), C.c_int64(0), C.c_int64(0)
    st = lib().mc_k_band_schedule(2, ptr.ctypes.data_as(C.POINTER(C.c_int32)), None,
                                  10, 64, 8, None, C.byref(nseg), None, C.byref(nfix),
                                  C.byref(nslot))
    assert st == 1                                  # MC_EINVAL
